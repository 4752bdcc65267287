// Memory-bound kernels of the adjoint (reverse-mode derivative) of the coded
// QR and of the coded solve.  The dense products of the adjoint (Q~^T dQ~,
// R dR^T, Q~ copyltu(M), D R^{-T}) run on the MFMA product kernels; these
// kernels transpose, symmetrize, form outer products and matrix-vector
// products, and fold the checksum rows back onto A.
#include "cqr_kernels.hpp"

namespace cqr {

constexpr int kAdjThreads = 256;

static unsigned blocks_for(int64_t n) {
  int64_t b = (n + kAdjThreads - 1) / kAdjThreads;
  return (unsigned)(b < 1 ? 1 : b);
}

// dst (cols x rows) = scale * src^T (src rows x cols), through a 64 x 64 LDS
// tile so both the loads and the stores cover contiguous columns.  upper:
// entries of src below its diagonal are taken as zero.
__global__ __launch_bounds__(kAdjThreads) void transpose_kernel(const double* src, int64_t lds, double* dst,
                                                                int64_t ldd, int64_t rows, int64_t cols, double scale,
                                                                int upper) {
  __shared__ double t[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int c = ty; c < 64; c += 4) {
    const int64_t i = i0 + tx, j = j0 + c;
    double v = 0.0;
    if (i < rows && j < cols && (!upper || i <= j)) v = src[i + j * lds];
    t[tx][c] = v;
  }
  __syncthreads();
  for (int c = ty; c < 64; c += 4) {
    const int64_t j = j0 + tx, i = i0 + c;
    if (j < cols && i < rows) dst[j + i * ldd] = scale * t[c][tx];
  }
}

// C <- copyltu(C) (n x n): every entry above the diagonal takes the value of
// its mirror below it.  Reads only the lower triangle, writes only the upper.
__global__ __launch_bounds__(kAdjThreads) void copyltu_kernel(double* C, int64_t ldc, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  if (i < j) C[i + j * ldc] = C[j + i * ldc];
}

// C[i][j] = scale * sum_{r < k} U[i][r] V[j][r]  (rows x cols); with upper,
// entries below the diagonal are zero.
__global__ __launch_bounds__(kAdjThreads) void outer_kernel(const double* U, int64_t ldu, const double* V,
                                                            int64_t ldv, int64_t rows, int64_t cols, int k,
                                                            double scale, int upper, double* C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e % rows, j = e / rows;
  double acc = 0.0;
  if (!upper || i <= j)
    for (int r = 0; r < k; ++r) acc += U[i + r * ldu] * V[j + r * ldv];
  C[i + j * ldc] = scale * acc;
}

// y[i][r] = sum_j A[i][j] x[j][r]  (A m x n, x n x nrhs); one thread per row,
// eight columns of A in flight per batch.
__global__ __launch_bounds__(kAdjThreads) void gemv_n_kernel(const double* A, int64_t lda, int64_t m, int n,
                                                             const double* x, int64_t ldx, int nrhs, double* y,
                                                             int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
  if (i >= m) return;
  constexpr int kB = 8;
  for (int r = 0; r < nrhs; ++r) {
    const double* xr = x + (int64_t)r * ldx;
    double acc = 0.0;
    int j = 0;
    for (; j + kB <= n; j += kB) {
      double a[kB];
#pragma unroll
      for (int t = 0; t < kB; ++t) a[t] = A[i + (int64_t)(j + t) * lda];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < kB; ++t) acc += a[t] * xr[j + t];
    }
    for (; j < n; ++j) acc += A[i + (int64_t)j * lda] * xr[j];
    y[i + (int64_t)r * ldy] = acc;
  }
}

// dA = X_top + G_v^T X_bottom:  block t of dA (rows t bs .. t bs + bs) is
// X_t + sum_k g~_v[k][t] X_{p_r + k}.  Thread = (row r in a block, column c);
// the K_v checksum values are read once and reused for every block t.
__global__ __launch_bounds__(kAdjThreads) void fold_kernel(FoldArgs a) {
  const int64_t e = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
  if (e >= a.bs * a.cols) return;
  const int64_t r = e % a.bs, c = e / a.bs;
  const double* x = a.X + c * a.ldx + r;
  double* d = a.dA + c * a.ldd + r;
  double chk[kMaxGen];
#pragma unroll
  for (int k = 0; k < kMaxGen; ++k) chk[k] = k < a.kv ? x[a.m + k * a.bs] : 0.0;
  for (int t = 0; t < a.pr; ++t) {
    double v = x[t * a.bs];
#pragma unroll
    for (int k = 0; k < kMaxGen; ++k)
      if (k < a.kv) v += a.gv[k * a.pr + t] * chk[k];
    d[t * a.bs] = v;
  }
}

// Y (n x n) = the block diagonal of the 64 x 64 tiles in T (tile k at
// T + 4096 k, column-major), zeros elsewhere: the inverted diagonal blocks of
// an upper-triangular matrix laid out as the start of its inverse.
__global__ __launch_bounds__(kAdjThreads) void blockdiag_kernel(const double* T, double* Y, int64_t ldy, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  Y[i + j * ldy] = (i >> 6) == (j >> 6) ? T[(i >> 6) * 4096 + (i & 63) + (j & 63) * 64] : 0.0;
}

// C *= s (rows x cols, ld ldc)
__global__ __launch_bounds__(kAdjThreads) void scale_kernel(double* C, int64_t ldc, int64_t rows, int64_t cols,
                                                            double s) {
  const int64_t e = (int64_t)blockIdx.x * kAdjThreads + threadIdx.x;
  if (e >= rows * cols) return;
  C[e % rows + (e / rows) * ldc] *= s;
}

void launch_blockdiag(const double* T, double* Y, int64_t ldy, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(blockdiag_kernel, dim3(blocks_for(n * n)), dim3(kAdjThreads), 0, st, T, Y, ldy, n);
}

void launch_scale(double* C, int64_t ldc, int64_t rows, int64_t cols, double s, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(rows * cols)), dim3(kAdjThreads), 0, st, C, ldc, rows, cols, s);
}

void launch_transpose(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows, int64_t cols,
                      double scale, bool upper, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  const dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(kAdjThreads), 0, st, src, lds, dst, ldd, rows, cols, scale,
                     upper ? 1 : 0);
}

void launch_copyltu(double* C, int64_t ldc, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(copyltu_kernel, dim3(blocks_for(n * n)), dim3(kAdjThreads), 0, st, C, ldc, n);
}

void launch_outer(const double* U, int64_t ldu, const double* V, int64_t ldv, int64_t rows, int64_t cols, int k,
                  double scale, bool upper, double* C, int64_t ldc, hipStream_t st) {
  hipLaunchKernelGGL(outer_kernel, dim3(blocks_for(rows * cols)), dim3(kAdjThreads), 0, st, U, ldu, V, ldv, rows,
                     cols, k, scale, upper ? 1 : 0, C, ldc);
}

void launch_gemv_n(const double* A, int64_t lda, int64_t m, int n, const double* x, int64_t ldx, int nrhs,
                   double* y, int64_t ldy, hipStream_t st) {
  hipLaunchKernelGGL(gemv_n_kernel, dim3(blocks_for(m)), dim3(kAdjThreads), 0, st, A, lda, m, n, x, ldx, nrhs, y,
                     ldy);
}

void launch_fold(const FoldArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(fold_kernel, dim3(blocks_for(a.bs * a.cols)), dim3(kAdjThreads), 0, st, a);
}


}  // namespace cqr
