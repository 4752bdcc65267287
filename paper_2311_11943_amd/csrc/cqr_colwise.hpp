// Column-wise Gram-Schmidt helpers.
//
// colwise_panel: the classical Gram-Schmidt with reorthogonalisation (CGS2:
// every column projected twice against the finished columns) on one panel of
// w <= 64 columns, in place, by one workgroup; the second Cholesky-QR pass
// falls back to it when a Cholesky factorization breaks down.  Norms,
// coefficients and R are FP64.  The panel stays in global memory (L2); thread
// t owns rows t, t + NT, ... of every column, so each pass over the panel
// reads whole 512-byte row segments per wave and column.  Inner products
// against many columns run in chunks of 16 columns (16 accumulators per
// thread) with one workgroup reduction per chunk.  Normalisation of column j
// is folded into the first pass of column j + 1.
//
// colwise_wave_sum16 / colwise_block_sum: the reductions -- a transposing
// butterfly inside each wavefront (after four exchange steps lane l holds its
// lane group's sum for column l mod 16), two more exchanges across the lane
// groups, and (for the workgroup sum) a fixed-order sum over the waves in
// LDS, so results do not depend on scheduling.  colgrid_kernel, the
// multi-workgroup CGS2 / ICGS / MGS panel modes, uses the wavefront part.
#pragma once
#include "cqr_kernels.hpp"

namespace cqr {

constexpr int kColChunk = 16;

// LDS a workgroup of NT threads needs: per-wave partial sums and the reduced
// vectors (slot kLeaf of s1 / s2 holds a norm).
template <int NT>
struct ColwiseLds {
  double red[NT / 64][kColChunk + 1];
  double s1[kLeaf + 1];      // first projection's coefficients
  double s2[kLeaf + 1];      // second projection's coefficients
};

// Wavefront sums of v[0..16): afterwards every lane l holds the sum over the
// wavefront of v[l mod 16] (v is overwritten).
__device__ __forceinline__ double colwise_wave_sum16(double (&v)[kColChunk]) {
  const int lane = threadIdx.x & 63;
  // transposing butterfly over lane bits 3..0: a lane keeps the half of its
  // slots whose index bit matches its lane bit and adds the partner's copy,
  // in place (slot c of the kept half moves to slot c of the lower half)
#pragma unroll
  for (int h = kColChunk / 2; h >= 1; h >>= 1) {
    const bool hi = lane & h;
#pragma unroll
    for (int c = 0; c < h; ++c) {
      const double a = v[c], b = v[c + h];
      v[c] = (hi ? b : a) + __shfl_xor(hi ? a : b, h, 64);
    }
  }
  // lane l holds the sum over its lane group for column l mod 16
  double x = v[0];
  x += __shfl_xor(x, 16, 64);
  x += __shfl_xor(x, 32, 64);
  return x;
}

// Workgroup sums of v[0..16) into out[0..nv) and of `extra` into *xout (when
// xout != nullptr).  Every thread calls it.
template <int NT>
__device__ __forceinline__ void colwise_block_sum(double (&v)[kColChunk], double extra, int nv, double* out,
                                                  double* xout, double (*red)[kColChunk + 1]) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const double x = colwise_wave_sum16(v);
  double e = extra;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if (lane < kColChunk) red[wave][lane] = x;
  if (lane == 0) red[wave][kColChunk] = e;
  __syncthreads();
  if (tid < nv || (tid == kColChunk && xout)) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NT / 64; ++q) s += red[q][tid];
    if (tid < nv) out[tid] = s; else *xout = s;
  }
  __syncthreads();
}

// out[c] = sum over rows of P[r, c] y[r] for c in [c0, c1) (c1 - c0 <= 16),
// and the sum of y[r]^2 into *nrm when nrm != nullptr.  If scale_col is in
// [c0, c1), that column is first multiplied by `scale` in place.
template <int NT>
__device__ __forceinline__ void colwise_dots(double* P, int64_t ldp, int64_t mrows, int c0, int c1,
                                             const double* y, double* out, double* nrm, int scale_col,
                                             double scale, ColwiseLds<NT>& L) {
  const int tid = threadIdx.x;
  double acc[kColChunk];
#pragma unroll
  for (int c = 0; c < kColChunk; ++c) acc[c] = 0.0;
  double n2 = 0.0;
  for (int64_t r = tid; r < mrows; r += NT) {
    const double yr = y[r];
    n2 += yr * yr;
#pragma unroll
    for (int c = 0; c < kColChunk; ++c)
      if (c0 + c < c1) {
        double x = P[r + (c0 + c) * ldp];
        if (c0 + c == scale_col) {
          x *= scale;
          P[r + (c0 + c) * ldp] = x;
        }
        acc[c] += x * yr;
      }
  }
  colwise_block_sum<NT>(acc, n2, c1 - c0, out + c0, nrm, L.red);
}

// Orthonormalise P (mrows x w, ld ldp, w <= 64) in place by CGS2; the
// triangular factor goes to Rl (row-major, zero below the diagonal,
// zero-padded to 64 x 64).  Returns false if a column has zero (or
// non-finite) norm after projection: the panel is exactly rank-deficient, and
// that column is left unnormalised.
template <int NT>
__device__ bool colwise_panel(double* P, int64_t ldp, int64_t mrows, int w, double (*Rl)[kLeaf + 1],
                              ColwiseLds<NT>& L) {
  const int tid = threadIdx.x;
  bool ok = true;
  for (int e = tid; e < kLeaf * kLeaf; e += NT) Rl[e >> 6][e & 63] = 0.0;
  __syncthreads();
  double none[kColChunk];
  double prev_inv = 1.0;    // 1 / r_{j-1, j-1}, applied to column j-1 in column j's first pass
  for (int j = 0; j < w; ++j) {
    double* pj = P + (int64_t)j * ldp;
    // pass 1: s1 = P[:, <j]^T p_j (chunk by chunk), column j-1 normalised on the way
    for (int c0 = 0; c0 < max(j, 1); c0 += kColChunk)
      colwise_dots<NT>(P, ldp, mrows, c0, min(j, c0 + kColChunk), pj, L.s1, nullptr, j - 1, prev_inv, L);
    // pass 2: p_j -= P s1
    for (int64_t r = tid; r < mrows; r += NT) {
      double x = pj[r];
      for (int c = 0; c < j; ++c) x -= P[r + c * ldp] * L.s1[c];
      pj[r] = x;
    }
    __syncthreads();
    // pass 3: s2 = P[:, <j]^T p_j; pass 4: p_j -= P s2, ||p_j||^2
    if (j > 0)
      for (int c0 = 0; c0 < j; c0 += kColChunk)
        colwise_dots<NT>(P, ldp, mrows, c0, min(j, c0 + kColChunk), pj, L.s2, nullptr, -1, 1.0, L);
    double n2 = 0.0;
    for (int64_t r = tid; r < mrows; r += NT) {
      double x = pj[r];
      for (int c = 0; c < j; ++c) x -= P[r + c * ldp] * L.s2[c];
      pj[r] = x;
      n2 += x * x;
    }
#pragma unroll
    for (int c = 0; c < kColChunk; ++c) none[c] = 0.0;
    colwise_block_sum<NT>(none, n2, 0, L.s2, &L.s2[kLeaf], L.red);
    double rjj2 = L.s2[kLeaf];
    if (!(rjj2 > 0.0) || !isfinite(rjj2)) { ok = false; rjj2 = 1.0; }
    const double rjj = sqrt(rjj2);
    if (tid < j) Rl[tid][j] = L.s1[tid] + L.s2[tid];
    if (tid == 0) Rl[j][j] = rjj;
    prev_inv = 1.0 / rjj;
    __syncthreads();
  }
  // normalise the last column
  for (int64_t r = tid; r < mrows; r += NT) P[r + (int64_t)(w - 1) * ldp] *= prev_inv;
  __syncthreads();
  return ok;
}

}  // namespace cqr
