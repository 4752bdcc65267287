// Memory-bound kernels of the code: encoding, erasure (failure simulation),
// decoding / re-encoding along a code line, post-orthogonalization.
// One thread per element position inside a block; consecutive threads take
// consecutive rows of a column-major matrix, so every wavefront load and store
// covers whole 128-byte lines.
#include "cqr_kernels.hpp"

#include <cmath>

namespace cqr {

constexpr int kThreads = 256;

static unsigned grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b < 1 ? 1 : b);
}

// --------------------------------------------------------------------------
// Encode, column pass: checksum rows  C_(k,J) = sum_t g~_v[k][t] A_(t,J)
// for all n systematic columns.  Thread = (row r in a block, column c).
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

// Encode, row pass: checksum columns  C_(I,k) = sum_t g~_h[t][k] A~_(I,t) for
// every row of A~ (systematic and checksum rows; the corner follows).
__global__ __launch_bounds__(kThreads) void encode_cols_kernel(EncodeArgs a) {
  const int64_t mp = a.m + a.kv * a.bs;
  int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= mp * a.bw) return;
  int64_t row = e % mp, s = e / mp;
  double acc[kMaxGen];
#pragma unroll
  for (int k = 0; k < kMaxGen; ++k) acc[k] = 0.0;
  for (int t = 0; t < a.pc; ++t) {
    double v = a.At[row + (t * a.bw + s) * a.ld];
#pragma unroll
    for (int k = 0; k < kMaxGen; ++k)
      if (k < a.kh) acc[k] += a.g[k * a.pc + t] * v;
  }
#pragma unroll
  for (int k = 0; k < kMaxGen; ++k)
    if (k < a.kh) a.At[row + (a.n + k * a.bw + s) * a.ld] = acc[k];
}

void launch_encode_rows(const EncodeArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(encode_rows_kernel, dim3(grid_for(a.bs * a.n)), dim3(kThreads), 0, st, a);
}

void launch_encode_cols(const EncodeArgs& a, hipStream_t st) {
  int64_t mp = a.m + a.kv * a.bs;
  hipLaunchKernelGGL(encode_cols_kernel, dim3(grid_for(mp * a.bw)), dim3(kThreads), 0, st, a);
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
