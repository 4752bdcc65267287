// Memory-bound kernels of the code: encoding, erasure (failure simulation),
// decoding / re-encoding along a code line, post-orthogonalization.
// One thread per element position inside a block; consecutive threads take
// consecutive rows of a column-major matrix, so every wavefront load and store
// covers whole 128-byte lines.
#include "cqr_kernels.hpp"

#include <algorithm>
#include <cmath>

namespace cqr {

constexpr int kThreads = 256;

static unsigned grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b < 1 ? 1 : b);
}

// --------------------------------------------------------------------------
// Checksum rows alone, C_(k,J) = sum_t g~_v[k][t] A_(t,J) for all n columns
// (R's vertical code when the plan has no horizontal code).  Thread = (row r
// in a block, column c).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void encode_rows_kernel(EncodeArgs a) {
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= a.bs * a.n) return;
  int64_t r = e % a.bs, c = e / a.bs;
  double* col = a.At + c * a.ld;
  double acc[kMaxGen];
#pragma unroll
  for (int k = 0; k < kMaxGen; ++k) acc[k] = 0.0;
  for (int t = 0; t < a.pr; ++t) {
    double v = col[t * a.bs + r];
#pragma unroll
    for (int k = 0; k < kMaxGen; ++k)
      if (k < a.kv) acc[k] += a.g[k * a.pr + t] * v;
  }
#pragma unroll
  for (int k = 0; k < kMaxGen; ++k)
    if (k < a.kv) col[a.m + k * a.bs + r] = acc[k];
}

// --------------------------------------------------------------------------
// Encode in one pass (the whole encoding equation): checksum rows, checksum
// columns and corner from a single read of A.  A workgroup takes R = 512 / T
// consecutive rows r of a block row at one column position s of a block
// column, and walks the p_r block rows u; thread (rho, t) loads the element
// at row u bs + r, column t bw + s for every u up front (all its loads in
// flight at once), and
//   - as a row-code thread (t < p_c) sums C_k += g~_v[k][u] A_(u,t)[r, s]
//     over u (checksum block row k, block column t);
//   - as a column-code thread (t = l < K_h) forms, for each u, the checksum
//     column entry sum_t' g~_h[t'][l] A_(u,t')[r, s] from the workgroup's
//     LDS copy of that row of blocks, and after the walk the corner entries
//     sum_t' g~_h[t'][l] C_k(t') from the row-code threads' sums.
// Threads (rho, t) with the same t read R consecutive rows of one column:
// whole cache-line segments per wave and column.  Every element of A is read
// once and every checksum element written once: 8 (mn + cn + md + cd) bytes.
// 512 threads: at p_c = 16, 32-row (256-byte) segments per column; alone, on
// the n = 32768 workload's encode (18 GB), 3.97 TB/s against 3.66 with 256
// threads (16-row segments) and 3.25 with 1024.
// --------------------------------------------------------------------------
constexpr int kEncThreads = 512;

template <int T>
__global__ __launch_bounds__(kEncThreads) void encode_fused_kernel(EncodeArgs a) {
  constexpr int R = kEncThreads / T;
  __shared__ double X[2][T][R + 1];
  __shared__ double Cl[kMaxGen][T][R + 1];
  __shared__ double Gc[kMaxGen][kMaxGrid];
  const int tid = threadIdx.x, rho = tid % R, t = tid / R;
  const int64_t nseg = (a.bs + R - 1) / R;
  const int64_t s = blockIdx.x / nseg;
  const int64_t r = (blockIdx.x % nseg) * R + rho;
  const bool rok = r < a.bs;
  const bool rowt = t < a.pc, colt = t < a.kh;
  for (int e = tid; e < kMaxGen * kMaxGrid; e += kEncThreads) Gc[e / kMaxGrid][e % kMaxGrid] = a.gc[e];
  double x[kMaxGrid];
  const double* src = a.At + r + (t * a.bw + s) * a.ld;
#pragma unroll
  for (int u = 0; u < kMaxGrid; ++u) x[u] = (u < a.pr && rok && rowt) ? src[u * a.bs] : 0.0;
  double c[kMaxGen];
#pragma unroll
  for (int k = 0; k < kMaxGen; ++k) c[k] = 0.0;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kMaxGrid; ++u) {
    if (u >= a.pr) break;
    X[u & 1][t][rho] = x[u];
#pragma unroll
    for (int k = 0; k < kMaxGen; ++k)
      if (k < a.kv) c[k] += a.g[k * a.pr + u] * x[u];
    __syncthreads();
    if (colt && rok) {
      double d = 0.0;
      for (int tt = 0; tt < a.pc; ++tt) d += Gc[t][tt] * X[u & 1][tt][rho];
      a.At[u * a.bs + r + (a.n + t * a.bw + s) * a.ld] = d;
    }
  }
  if (a.kv == 0) return;
  if (rowt) {
#pragma unroll
    for (int k = 0; k < kMaxGen; ++k)
      if (k < a.kv) {
        Cl[k][t][rho] = c[k];
        if (rok) a.At[a.m + k * a.bs + r + (t * a.bw + s) * a.ld] = c[k];
      }
  }
  __syncthreads();
  if (colt && rok) {
    for (int k = 0; k < a.kv; ++k) {
      double e = 0.0;
      for (int tt = 0; tt < a.pc; ++tt) e += Gc[t][tt] * Cl[k][tt][rho];
      a.At[a.m + k * a.bs + r + (a.n + t * a.bw + s) * a.ld] = e;
    }
  }
}

void launch_encode_fused(const EncodeArgs& a, hipStream_t st) {
  const int T = std::max(a.pc, a.kh) <= 8 ? 8 : (std::max(a.pc, a.kh) <= 16 ? 16 : 32);
  const int R = kEncThreads / T;
  const unsigned grid = (unsigned)(((a.bs + R - 1) / R) * a.bw);
  if (T == 8)
    hipLaunchKernelGGL(encode_fused_kernel<8>, dim3(grid), dim3(kEncThreads), 0, st, a);
  else if (T == 16)
    hipLaunchKernelGGL(encode_fused_kernel<16>, dim3(grid), dim3(kEncThreads), 0, st, a);
  else
    hipLaunchKernelGGL(encode_fused_kernel<32>, dim3(grid), dim3(kEncThreads), 0, st, a);
}

void launch_encode_rows(const EncodeArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(encode_rows_kernel, dim3(grid_for(a.bs * a.n)), dim3(kThreads), 0, st, a);
}

// --------------------------------------------------------------------------
// One code line: every output block is a fixed linear combination of the
// surviving blocks of the line (coefficients solved on the host).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void line_kernel(LineArgs a) {
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= (int64_t)a.rows * a.cols) return;
  int64_t r = e % a.rows, c = e / a.rows;
  int64_t pos = r + c * a.ld;
  double acc[kMaxOut];
#pragma unroll
  for (int o = 0; o < kMaxOut; ++o) acc[o] = 0.0;
  for (int s = 0; s < a.nsrc; ++s) {
    double v = a.base[a.src[s] + pos];
#pragma unroll
    for (int o = 0; o < kMaxOut; ++o)
      if (o < a.nout) acc[o] += a.coef[o][s] * v;
  }
#pragma unroll
  for (int o = 0; o < kMaxOut; ++o)
    if (o < a.nout) a.base[a.dst[o] + pos] = acc[o];
}

void launch_line(const LineArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(line_kernel, dim3(grid_for((int64_t)a.rows * a.cols)), dim3(kThreads), 0, st, a);
}

__global__ __launch_bounds__(kThreads) void erase_kernel(EraseArgs a) {
  int64_t per = (int64_t)a.rows * a.cols;
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= per * a.nblk) return;
  int blk = (int)(e / per);
  int64_t w = e % per;
  int64_t r = w % a.rows, c = w / a.rows;
  a.base[a.off[blk] + r + c * a.ld] = __builtin_nan("");
}

void launch_erase(const EraseArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(erase_kernel, dim3(grid_for((int64_t)a.rows * a.cols * a.nblk)), dim3(kThreads), 0,
                     st, a);
}

// --------------------------------------------------------------------------
// Post-orthogonalization  W = (G^_0 (x) I_bs) Z  (G^_0 built from G~_v) with
//   G^_0 = [[I_K + G~_1, V~], [V~^T, -I]]:
//   block row i <  K: sum_l G^_0[i][l] Z_l   (all p_r blocks)
//   block row i >= K: sum_{l<K} V~[l][i-K] Z_l - Z_i
// Thread = (row r in a block, column c); reads the p_r blocks once.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void postorth_kernel(PostArgs a) {
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= a.bs * a.cols) return;
  int64_t r = e % a.bs, c = e / a.bs;
  const double* src = a.src + c * a.lds + r;
  double* dst = a.dst + c * a.ldd + r;
  double z[kMaxGrid];
#pragma unroll
  for (int l = 0; l < kMaxGrid; ++l) z[l] = (l < a.pr) ? src[l * a.bs] : 0.0;
  // G^_0[i][l]: i, l < K: delta_il + G~_1[i][l];  i < K <= l: V~[i][l-K] = g~_v[i][l];
  //            i >= K > l: V~[l][i-K] = g~_v[l][i];  i, l >= K: -delta_il.
  double head[kMaxGen];
#pragma unroll
  for (int i = 0; i < kMaxGen; ++i) {
    double v = 0.0;
    if (i < a.kv) {
      v = z[i];
#pragma unroll
      for (int l = 0; l < kMaxGrid; ++l)
        if (l < a.pr) v += a.gv[i * a.pr + l] * z[l];
    }
    head[i] = v;
  }
#pragma unroll
  for (int i = 0; i < kMaxGrid; ++i) {
    if (i >= a.kv && i < a.pr) {
      double v = -z[i];
#pragma unroll
      for (int l = 0; l < kMaxGen; ++l)
        if (l < a.kv) v += a.gv[l * a.pr + i] * z[l];
      dst[i * a.bs] = v;
    }
  }
#pragma unroll
  for (int i = 0; i < kMaxGen; ++i)
    if (i < a.kv) dst[i * a.bs] = head[i];
}

void launch_postorth(const PostArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(postorth_kernel, dim3(grid_for(a.bs * a.cols)), dim3(kThreads), 0, st, a);
}

__global__ void zero_ints_kernel(int* p, int n) {
  int e = blockIdx.x * kThreads + threadIdx.x;
  if (e < n) p[e] = 0;
}

void launch_zero_ints(int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, p, n);
}

__global__ __launch_bounds__(kThreads) void fill_zero_kernel(double* p, int64_t ld, int64_t rows, int64_t cols) {
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= rows * cols) return;
  p[(e % rows) + (e / rows) * ld] = 0.0;
}

void launch_fill_zero(double* p, int64_t ld, int64_t rows, int64_t cols, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(rows * cols)), dim3(kThreads), 0, st, p, ld, rows, cols);
}

}  // namespace cqr
