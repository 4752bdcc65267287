// Coded linear solve (the linear-solve equations that follow the
// post-orthogonalization theorem):  X = R_1^{-1} (Qpost^T Bpost).
//   1. trinv_kernel: every 64 x 64 diagonal block of R_1 is inverted at once
//      (one workgroup per block, column-oriented substitution in LDS).
//   2. gemv_t_kernel: Y = Qpost^T Bpost, one wave per column of Qpost (its m
//      entries are contiguous), partial sums reduced across the wave.
//   3. Block back substitution, bottom-up, one launch per 64-row block k
//      (right-hand sides in groups of 4 along the grid's y dimension): every
//      workgroup forms x_k = T_kk y_k (T_kk = R_kk^{-1}) in LDS, the first
//      column of workgroups stores it, and each thread subtracts
//      R_1[i, block k] x_k from its row i < k0 of Y (loads of a column of R
//      coalesced across the wave).
#include "cqr_kernels.hpp"

#include <mutex>

namespace cqr {

constexpr int kSolveThreads = 256;
constexpr int kSolveBlock = 64;      // diagonal block of the back substitution
constexpr int kRhsChunk = 4;         // right-hand sides per pass

__global__ __launch_bounds__(kSolveThreads) void gemv_t_kernel(const double* Q, int64_t ldq, int64_t m, int n,
                                                               const double* B, int64_t ldb, int nrhs, double* Y,
                                                               int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * (kSolveThreads / 64) + (threadIdx.x >> 6);
  if (col >= n) return;
  const double* q = Q + (int64_t)col * ldq;
  constexpr int kBatch = 8;   // rows per lane whose loads are issued together
  for (int r0 = 0; r0 < nrhs; r0 += kRhsChunk) {
    const int nr = nrhs - r0 < kRhsChunk ? nrhs - r0 : kRhsChunk;
    double acc[kRhsChunk] = {0.0, 0.0, 0.0, 0.0};
    int64_t i = lane;
    for (; i + (kBatch - 1) * 64 < m; i += kBatch * 64) {
      double qv[kBatch], bv[kBatch][kRhsChunk];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        qv[j] = q[i + j * 64];
#pragma unroll
        for (int t = 0; t < kRhsChunk; ++t)
          bv[j][t] = t < nr ? B[i + j * 64 + (int64_t)(r0 + t) * ldb] : 0.0;
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
#pragma unroll
        for (int t = 0; t < kRhsChunk; ++t) acc[t] += qv[j] * bv[j][t];
    }
    for (; i < m; i += 64) {
      const double v = q[i];
#pragma unroll
      for (int t = 0; t < kRhsChunk; ++t)
        if (t < nr) acc[t] += v * B[i + (int64_t)(r0 + t) * ldb];
    }
#pragma unroll
    for (int t = 0; t < kRhsChunk; ++t) {
      double v = acc[t];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0 && r0 + t < nrhs) Y[col + (int64_t)(r0 + t) * ldy] = v;
    }
  }
}

// T_kk = R_kk^{-1} for block k = blockIdx.x (w = min(64, n - 64k) rows; the
// 64 x 64 output is padded with the identity).  T is column-major, 64 x 64
// per block.  Thread (row, q) owns Tl[row][16q .. 16q+15]; pivot i divides
// row i, then rows above subtract R[row][i] times it (one barrier per pivot).
__global__ __launch_bounds__(kSolveThreads) void trinv_kernel(const double* R, int64_t ldr, int64_t n, double* T) {
  __shared__ double Rl[kSolveBlock][kSolveBlock + 1];
  __shared__ double Tl[kSolveBlock][kSolveBlock + 1];
  const int tid = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * kSolveBlock;
  const int w = (int)((n - k0) < kSolveBlock ? (n - k0) : kSolveBlock);
  for (int e = tid; e < kSolveBlock * kSolveBlock; e += kSolveThreads) {
    const int r = e % kSolveBlock, c = e / kSolveBlock;
    Rl[r][c] = (r < w && c < w) ? R[(k0 + r) + (k0 + c) * ldr] : (r == c ? 1.0 : 0.0);
    Tl[r][c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  const int row = tid & 63, c0 = (tid >> 6) * 16;
  for (int i = kSolveBlock - 1; i >= 0; --i) {
    if (row == i) {
      const double d = Rl[i][i];
#pragma unroll
      for (int c = 0; c < 16; ++c) Tl[i][c0 + c] /= d;
    }
    __syncthreads();
    if (row < i) {
      const double f = Rl[row][i];
#pragma unroll
      for (int c = 0; c < 16; ++c) Tl[row][c0 + c] -= f * Tl[i][c0 + c];
    }
  }
  __syncthreads();
  double* out = T + (int64_t)blockIdx.x * kSolveBlock * kSolveBlock;
  for (int e = tid; e < kSolveBlock * kSolveBlock; e += kSolveThreads)
    out[e] = Tl[e % kSolveBlock][e / kSolveBlock];
}

// Block k0 of the back substitution for right-hand sides r0 .. r0+3
// (r0 = 4 blockIdx.y): x = T_kk Y[k0:k0+w] -> X[k0:k0+w] (workgroups with
// blockIdx.x == 0), Y[0:k0] -= R_1[0:k0, k0:k0+w] x (one thread per row).
__global__ __launch_bounds__(kSolveThreads) void trsv_step_kernel(const double* R, int64_t ldr, const double* T,
                                                                  double* Y, int64_t ldy, double* X, int64_t ldx,
                                                                  int nrhs, int64_t k0, int w) {
  __shared__ double Tl[kSolveBlock][kSolveBlock + 1];
  __shared__ double yk[kSolveBlock][kRhsChunk];
  __shared__ double xk[kSolveBlock][kRhsChunk];
  const int tid = threadIdx.x;
  const double* Tk = T + (k0 / kSolveBlock) * kSolveBlock * kSolveBlock;
  for (int e = tid; e < kSolveBlock * kSolveBlock; e += kSolveThreads)
    Tl[e % kSolveBlock][e / kSolveBlock] = Tk[e];
  const int row = tid & 63, u = tid >> 6;
  const int r0 = blockIdx.y * kRhsChunk;
  const bool mine = row < w && r0 + u < nrhs;
  yk[row][u] = mine ? Y[k0 + row + (int64_t)(r0 + u) * ldy] : 0.0;
  __syncthreads();
  double x = 0.0;
#pragma unroll 16
  for (int t = 0; t < kSolveBlock; ++t) x += Tl[row][t] * yk[t][u];
  xk[row][u] = x;
  if (blockIdx.x == 0 && mine) X[k0 + row + (int64_t)(r0 + u) * ldx] = x;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kSolveThreads + tid;
  if (i >= k0) return;
  const double* ri = R + i + k0 * ldr;
  double acc[kRhsChunk] = {0.0, 0.0, 0.0, 0.0};
  if (w == kSolveBlock) {
    // every load of the row's 64 coefficients in flight before the sums
    double v[kSolveBlock];
#pragma unroll
    for (int t = 0; t < kSolveBlock; ++t) v[t] = ri[t * ldr];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < kSolveBlock; ++t)
#pragma unroll
      for (int q = 0; q < kRhsChunk; ++q) acc[q] += v[t] * xk[t][q];
  } else {
    for (int t = 0; t < w; ++t) {
      const double v = ri[t * ldr];
#pragma unroll
      for (int q = 0; q < kRhsChunk; ++q) acc[q] += v * xk[t][q];
    }
  }
#pragma unroll
  for (int q = 0; q < kRhsChunk; ++q)
    if (r0 + q < nrhs) Y[i + (int64_t)(r0 + q) * ldy] -= acc[q];
}

void launch_gemv_t(const double* Q, int64_t ldq, int64_t m, int n, const double* B, int64_t ldb, int nrhs,
                   double* Y, int64_t ldy, hipStream_t st) {
  const int per = kSolveThreads / 64;
  hipLaunchKernelGGL(gemv_t_kernel, dim3((n + per - 1) / per), dim3(kSolveThreads), 0, st, Q, ldq, m, n, B, ldb,
                     nrhs, Y, ldy);
}

void launch_trinv(const double* R, int64_t ldr, int64_t n, double* T, hipStream_t st) {
  hipLaunchKernelGGL(trinv_kernel, dim3((unsigned)((n + kSolveBlock - 1) / kSolveBlock)), dim3(kSolveThreads), 0,
                     st, R, ldr, n, T);
}

void launch_trsv_step(const double* R, int64_t ldr, const double* T, double* Y, int64_t ldy, double* X,
                      int64_t ldx, int nrhs, int64_t k0, int w, hipStream_t st) {
  const unsigned grid = k0 > 0 ? (unsigned)((k0 + kSolveThreads - 1) / kSolveThreads) : 1u;
  const unsigned chunks = (unsigned)((nrhs + kRhsChunk - 1) / kRhsChunk);
  hipLaunchKernelGGL(trsv_step_kernel, dim3(grid, chunks), dim3(kSolveThreads), 0, st, R, ldr, T, Y, ldy, X, ldx,
                     nrhs, k0, w);
}

// Scratch memory of the allocation-free solve (coded_qr_solve_noalloc): the
// inverted diagonal blocks of R_1 and Y = Qpost^T Bpost live in this
// file-scope array, one copy per device, held until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): its device address is looked up once per device,
// with that device current, and that address is what the kernels receive.
// Every kernel writes the parts of it that later kernels read (trinv_kernel
// all 64 x 64 entries of each block, gemv_t_kernel all n x nrhs entries of
// Y), so no call depends on what a previous call left there.
static __device__ __align__(256) char scratch[kSolveScratchBytes];

hipError_t solve_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = a;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace cqr
