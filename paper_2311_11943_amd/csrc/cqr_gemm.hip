// FP64 MFMA kernels of the blocked Gram-Schmidt: the split-K projection
// product (R_bar = Qbar^T Q_t, S = Q_prev^T P, Gram matrices), the rank-K
// update (Q_t -= Qbar R_bar, P -= Q_prev S), the panel's Cholesky step and the
// in-place triangular transform of the panel (P <- P R^{-1}).
//
// MFMA layout used throughout (v_mfma_f64_16x16x4, one wavefront of 64 lanes):
// D = X Y + D with X 16x4, Y 4x16; lane l supplies X[l%16][l/16] and
// Y[l/16][l%16] and holds D[4r + l/16][l%16] in accumulator element r.  Every
// product is issued as the transposed product (D = C^T), so lane l holds
// C[i0 + l%16][j0 + 4r + l/16]: sixteen consecutive rows of a column-major C
// per lane group, i.e. whole 128-byte lines on load and store.  Within a group
// of 16 k-values lane l contributes k = k0 + 4*(l/16) + s in MFMA step s (one
// fixed permutation of the reduction index, shared by both operands).
//
// Reductions over long K are split across blocks; partial tiles go to the
// workspace and a second small kernel sums them in split order, so results do
// not depend on scheduling and no device-wide fence is needed.
#include "cqr_colwise.hpp"
#include "cqr_kernels.hpp"

#include <algorithm>
#include <cmath>

namespace cqr {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v4d mfma(double x, double y, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

// FP32 product of FP64 operands rounded to FP32 (the mixed-precision
// coefficient product R_bar = Qbar^T Q_t).  Operand lanes as in the FP64 form.
// The product kernels accumulate it in FP32 over 16 k-values only (four MFMA
// steps) and add each group's sums into FP64 accumulators, so the rounding of
// the reduction does not grow with K.
__device__ __forceinline__ v4f mfma(double x, double y, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32((float)x, (float)y, c, 0, 0, 0);
}

__device__ __forceinline__ v4f mfma(float x, float y, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
}

// Operand type of the product kernels' MFMA steps.
template <bool F32> struct OpT { typedef double type; };
template <> struct OpT<true> { typedef float type; };

// acc += t, element by element in FP64 (one slab's FP32 sums into the FP64
// accumulators of the mixed-precision product).
__device__ __forceinline__ void widen_add(v4d& acc, const v4f& t) {
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] += (double)t[r];
}

// Result layout of the transposed-issue 16x16x4 products: lane (li, g),
// register r holds C[i0 + li][j0 + colsub(r, g)] -- the FP64 form spreads a
// lane's four values over columns g, g+4, g+8, g+12, the FP32 form over the
// consecutive columns 4g .. 4g+3.
__device__ __forceinline__ int colsub(int r, int g, bool f32) { return f32 ? 4 * g + r : 4 * r + g; }


// Partial-tile layout shared by the product and reduction kernels: tile
// `tile` of split `sp`, wave w, accumulator element q (16 per lane), lane l at
// part[((sp * ntiles + tile) * 4 + w) * 1024 + q * 64 + l].
__device__ __forceinline__ int64_t part_off(int sp, int ntiles, int tile, int wave) {
  return (((int64_t)sp * ntiles + tile) * 4 + wave) * 1024;
}

// Sum over splits of four element slots q = 4 qg + u (u < 4) of one wave's
// partial tiles, lane `lane`, in split order.  Batches of 16 splits have all
// their loads issued before the first addition.
__device__ __forceinline__ void sum_partials4(const double* part, int nsplit, int ntiles, int tile, int wave,
                                              int qg, int lane, double (&v)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = 0.0;
  const double* base = part + part_off(0, ntiles, tile, wave) + 4 * qg * 64 + lane;
  const int64_t sstride = (int64_t)ntiles * 4 * 1024;
  for (int sp0 = 0; sp0 < nsplit; sp0 += 16) {
    double t[16][4];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int sp = std::min(sp0 + k, nsplit - 1);       // clamped: extra loads are discarded
#pragma unroll
      for (int u = 0; u < 4; ++u) t[k][u] = base[sp * sstride + u * 64];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] += (sp0 + k < nsplit) ? t[k][u] : 0.0;
  }
}

// --------------------------------------------------------------------------
// Split-K product  C = A^T B  (A: K x M, B: K x N, both K-contiguous).
// Tile 64x64 per block, 4 waves each a 32x32 quadrant.  Operand slabs of
// KC = 32 k-values are staged through LDS (double-buffered): each global load
// instruction covers 4 columns x 256 contiguous bytes.  Requires 16-byte
// aligned operands with even leading dimensions (else tn_direct_kernel).
// --------------------------------------------------------------------------

constexpr int KC = 32;           // k-values per LDS slab
constexpr int LDP = KC + 2;      // padded LDS column (doubles)

// Store a wave's 32 x 32 quadrant (16 values per lane, element (x, y, r) at
// row i0 + 16x + li, column j0 + 16y + 4r + g) to C, and add it into C2 if
// given; the C2 loads are all issued before any store.
__device__ __forceinline__ void store_quadrant(double* C, int64_t ldc, double* C2, int64_t ldc2, int M, int M2,
                                               int N, int i0, int j0, int li, int g, bool f32,
                                               const double (&v)[16]) {
  double old[16];
  if (C2) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int x = e >> 3, y = (e >> 2) & 1, r = e & 3;
      const int i = i0 + 16 * x + li, j = j0 + 16 * y + colsub(r, g, f32);
      old[e] = (i < M2 && j < N) ? C2[i + (int64_t)j * ldc2] : 0.0;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int x = e >> 3, y = (e >> 2) & 1, r = e & 3;
    const int i = i0 + 16 * x + li, j = j0 + 16 * y + colsub(r, g, f32);
    if (i < M && j < N) {
      C[i + (int64_t)j * ldc] = v[e];
      if (C2 && i < M2) C2[i + (int64_t)j * ldc2] = old[e] + v[e];
    }
  }
}

template <class Acc>
__device__ __forceinline__ void tn_store(const TnArgs& a, const Acc (&acc)[2][2], int tile, int split, int wave,
                                         int lane, int i0, int j0, bool f32_layout) {
  const int li = lane & 15, g = lane >> 4;
  if (a.nsplit > 1) {
    double* mine = a.part + part_off(split, a.ntiles, tile, wave);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) mine[((x * 2 + y) * 4 + r) * 64 + lane] = acc[x][y][r];
    return;
  }
  double v[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) v[e] = acc[e >> 3][(e >> 2) & 1][e & 3];
  store_quadrant(a.C, a.ldc, a.C2, a.ldc2, a.M, a.M2, a.N, i0, j0, li, g, f32_layout, v);
}

template <int TAG, bool F32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void tn_lds_kernel(TnArgs a) {
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  typedef v4d Acc;    // FP64 accumulators (FP32 products are widened per slab)
  typedef typename OpT<F32>::type Op;
  __shared__ double sA[2][64 * LDP];
  __shared__ double sB[2][64 * LDP];
  const int tile = blockIdx.x, split = blockIdx.y;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int64_t kb = (int64_t)split * a.kchunk;
  const int64_t ke = std::min<int64_t>(a.K, kb + a.kchunk);
  // staging: thread loads one v2d (k pair lq) of columns lc + 16r, r < 4
  const int lc = tid >> 4, lq = tid & 15;
  const double* ga[4];
  const double* gb[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int ia = tm * 64 + lc + 16 * r, jb = tn * 64 + lc + 16 * r;
    // columns outside the matrix read column 0 and feed only unstored outputs
    ga[r] = a.A + (int64_t)(ia < a.M ? ia : 0) * a.lda + 2 * lq;
    gb[r] = a.B + (int64_t)(jb < a.N ? jb : 0) * a.ldb + 2 * lq;
  }
  Acc acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Acc{0, 0, 0, 0};
  const int ia0 = (wave & 1) * 32, jb0 = (wave >> 1) * 32;
  const int nfull = (int)((ke - kb) / KC);

  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 16) {
      [[maybe_unused]] v4f t32[2][2];
      if constexpr (F32)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) t32[x][y] = v4f{0, 0, 0, 0};
      Op xa[2][4], xb[2][4];   // FP32 operands are rounded as they leave LDS
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double* pa = &sA[buf][(ia0 + 16 * t + li) * LDP + kk + 4 * g];
        const double* pb = &sB[buf][(jb0 + 16 * t + li) * LDP + kk + 4 * g];
        v2d a0 = *reinterpret_cast<const v2d*>(pa), a1 = *reinterpret_cast<const v2d*>(pa + 2);
        v2d b0 = *reinterpret_cast<const v2d*>(pb), b1 = *reinterpret_cast<const v2d*>(pb + 2);
        xa[t][0] = a0.x; xa[t][1] = a0.y; xa[t][2] = a1.x; xa[t][3] = a1.y;
        xb[t][0] = b0.x; xb[t][1] = b0.y; xb[t][2] = b1.x; xb[t][3] = b1.y;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            if constexpr (F32)
              t32[x][y] = mfma(xb[y][s], xa[x][s], t32[x][y]);
            else
              acc[x][y] = mfma(xb[y][s], xa[x][s], acc[x][y]);
          }
      if constexpr (F32)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) widen_add(acc[x][y], t32[x][y]);
    }
  };
  // slab sl's first k (clamped to the last full slab: prefetches past the end
  // reload cached data that is never used)
  auto koff = [&](int sl) { return kb + (int64_t)std::min(sl, nfull - 1) * KC; };

  if (nfull > 0) {
    // three-stage pipeline: slab sl in LDS is multiplied while the register
    // set of slab sl+1 (issued one slab earlier) lands and slab sl+2 is
    // requested into the other set; the two sets alternate explicitly
    v2d ra0[4], rb0[4], ra1[4], rb1[4];
#define CQR_TN_LOAD(RA, RB, K) {                                        \
    RA[0] = *reinterpret_cast<const v2d*>(ga[0] + (K));              \
    RB[0] = *reinterpret_cast<const v2d*>(gb[0] + (K));              \
    RA[1] = *reinterpret_cast<const v2d*>(ga[1] + (K));              \
    RB[1] = *reinterpret_cast<const v2d*>(gb[1] + (K));              \
    RA[2] = *reinterpret_cast<const v2d*>(ga[2] + (K));              \
    RB[2] = *reinterpret_cast<const v2d*>(gb[2] + (K));              \
    RA[3] = *reinterpret_cast<const v2d*>(ga[3] + (K));              \
    RB[3] = *reinterpret_cast<const v2d*>(gb[3] + (K));              \
  }
#define CQR_TN_PUT(BUF, RA, RB) {                                       \
    *reinterpret_cast<v2d*>(&sA[BUF][(lc + 0) * LDP + 2 * lq]) = RA[0];      \
    *reinterpret_cast<v2d*>(&sB[BUF][(lc + 0) * LDP + 2 * lq]) = RB[0];      \
    *reinterpret_cast<v2d*>(&sA[BUF][(lc + 16) * LDP + 2 * lq]) = RA[1];      \
    *reinterpret_cast<v2d*>(&sB[BUF][(lc + 16) * LDP + 2 * lq]) = RB[1];      \
    *reinterpret_cast<v2d*>(&sA[BUF][(lc + 32) * LDP + 2 * lq]) = RA[2];      \
    *reinterpret_cast<v2d*>(&sB[BUF][(lc + 32) * LDP + 2 * lq]) = RB[2];      \
    *reinterpret_cast<v2d*>(&sA[BUF][(lc + 48) * LDP + 2 * lq]) = RA[3];      \
    *reinterpret_cast<v2d*>(&sB[BUF][(lc + 48) * LDP + 2 * lq]) = RB[3];      \
  }
    CQR_TN_LOAD(ra0, rb0, koff(0))
    CQR_TN_LOAD(ra1, rb1, koff(1))
    CQR_TN_PUT(0, ra0, rb0)
    __syncthreads();
    int sl = 0;
    for (; sl + 2 <= nfull; sl += 2) {
      CQR_TN_LOAD(ra0, rb0, koff(sl + 2))
      __builtin_amdgcn_sched_barrier(0);
      compute(0);
      __builtin_amdgcn_sched_barrier(0);
      CQR_TN_PUT(1, ra1, rb1)
      __syncthreads();
      CQR_TN_LOAD(ra1, rb1, koff(sl + 3))
      __builtin_amdgcn_sched_barrier(0);
      compute(1);
      __builtin_amdgcn_sched_barrier(0);
      CQR_TN_PUT(0, ra0, rb0)
      __syncthreads();
    }
    if (sl < nfull) compute(0);
#undef CQR_TN_LOAD
#undef CQR_TN_PUT
  }
  const int64_t kt = kb + (int64_t)nfull * KC;
  if (kt < ke) {
    // partial last slab: masked scalar loads, zero beyond ke
    const int buf = nfull & 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t k = kt + 2 * lq;
      const double* pa = ga[r] - 2 * lq;
      const double* pb = gb[r] - 2 * lq;
      v2d va, vb;
      va.x = (k < ke) ? pa[k] : 0.0;
      va.y = (k + 1 < ke) ? pa[k + 1] : 0.0;
      vb.x = (k < ke) ? pb[k] : 0.0;
      vb.y = (k + 1 < ke) ? pb[k + 1] : 0.0;
      *reinterpret_cast<v2d*>(&sA[buf][(lc + 16 * r) * LDP + 2 * lq]) = va;
      *reinterpret_cast<v2d*>(&sB[buf][(lc + 16 * r) * LDP + 2 * lq]) = vb;
    }
    __syncthreads();
    compute(buf);
  }
  tn_store(a, acc, tile, split, wave, lane, tm * 64 + ia0, tn * 64 + jb0, F32);
}

// The same product with 16-deep slabs (36 KB of LDS, three waves per SIMD),
// taken by FP32 products with at least two tile rows and two or three tile
// columns whose depth is not a multiple of 32 (tnf_kernel takes the others;
// with four or more tile columns, such products take tn2_kernel).  An FP32 MFMA
// takes fewer cycles than the FP64 one, so the FP32 product waits more on its
// loads and the third wave hides them (the n = 16384 factorization with FP32
// updates runs 5% faster); in FP64 the twice as many barriers of the shorter
// slabs cost more than the extra wave returns (about 1% slower at n = 16384
// and n = 32768), and FP64 products keep tn_lds_kernel.
// Thread (lc, lq) stages one v2d (k pair lq) of columns lc + 32 q, q < 2, of
// each operand per slab; the pipeline, the tile order and the output contract
// (partials or C, C2) are those of tn_lds_kernel.
template <int TAG, bool F32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void tn16_kernel(TnArgs a) {
  constexpr int SK = 16, LW = SK + 2, NQ = 2, TPC = SK / 2, CPP = 256 / TPC;
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  typedef v4d Acc;    // FP64 accumulators (FP32 products are widened per slab)
  typedef typename OpT<F32>::type Op;
  __shared__ double sA[2][64 * LW];
  __shared__ double sB[2][64 * LW];
  const int tile = blockIdx.x, split = blockIdx.y;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int64_t kb = (int64_t)split * a.kchunk;
  const int64_t ke = std::min<int64_t>(a.K, kb + a.kchunk);
  const int lc = tid / TPC, lq = tid % TPC;
  const double* ga[NQ];
  const double* gb[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int ia = tm * 64 + lc + CPP * q, jb = tn * 64 + lc + CPP * q;
    // columns outside the matrix read column 0 and feed only unstored outputs
    ga[q] = a.A + (int64_t)(ia < a.M ? ia : 0) * a.lda + 2 * lq;
    gb[q] = a.B + (int64_t)(jb < a.N ? jb : 0) * a.ldb + 2 * lq;
  }
  Acc acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Acc{0, 0, 0, 0};
  const int ia0 = (wave & 1) * 32, jb0 = (wave >> 1) * 32;
  const int nfull = (int)((ke - kb) / SK);
  auto compute = [&](int buf) {
    Op xa[2][4], xb[2][4];   // FP32 operands are rounded as they leave LDS
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const double* pa = &sA[buf][(ia0 + 16 * t + li) * LW + 4 * g];
      const double* pb = &sB[buf][(jb0 + 16 * t + li) * LW + 4 * g];
      v2d a0 = *reinterpret_cast<const v2d*>(pa), a1 = *reinterpret_cast<const v2d*>(pa + 2);
      v2d b0 = *reinterpret_cast<const v2d*>(pb), b1 = *reinterpret_cast<const v2d*>(pb + 2);
      xa[t][0] = a0.x; xa[t][1] = a0.y; xa[t][2] = a1.x; xa[t][3] = a1.y;
      xb[t][0] = b0.x; xb[t][1] = b0.y; xb[t][2] = b1.x; xb[t][3] = b1.y;
    }
    [[maybe_unused]] v4f t32[2][2];
    if constexpr (F32)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) t32[x][y] = v4f{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          if constexpr (F32)
            t32[x][y] = mfma(xb[y][s], xa[x][s], t32[x][y]);
          else
            acc[x][y] = mfma(xb[y][s], xa[x][s], acc[x][y]);
        }
    if constexpr (F32)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) widen_add(acc[x][y], t32[x][y]);
  };
  auto koff = [&](int sl) { return kb + (int64_t)std::min(sl, nfull - 1) * SK; };
  v2d ra0[NQ], rb0[NQ], ra1[NQ], rb1[NQ];
  auto load = [&](v2d (&ra)[NQ], v2d (&rb)[NQ], int64_t k) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      ra[q] = *reinterpret_cast<const v2d*>(ga[q] + k);
      rb[q] = *reinterpret_cast<const v2d*>(gb[q] + k);
    }
  };
  auto put = [&](int buf, const v2d (&ra)[NQ], const v2d (&rb)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      *reinterpret_cast<v2d*>(&sA[buf][(lc + CPP * q) * LW + 2 * lq]) = ra[q];
      *reinterpret_cast<v2d*>(&sB[buf][(lc + CPP * q) * LW + 2 * lq]) = rb[q];
    }
  };
  if (nfull > 0) {
    load(ra0, rb0, koff(0));
    load(ra1, rb1, koff(1));
    put(0, ra0, rb0);
    __syncthreads();
    int sl = 0;
    for (; sl + 2 <= nfull; sl += 2) {
      load(ra0, rb0, koff(sl + 2));
      __builtin_amdgcn_sched_barrier(0);
      compute(0);
      __builtin_amdgcn_sched_barrier(0);
      put(1, ra1, rb1);
      __syncthreads();
      load(ra1, rb1, koff(sl + 3));
      __builtin_amdgcn_sched_barrier(0);
      compute(1);
      __builtin_amdgcn_sched_barrier(0);
      put(0, ra0, rb0);
      __syncthreads();
    }
    if (sl < nfull) compute(0);
  }
  const int64_t kt = kb + (int64_t)nfull * SK;
  if (kt < ke) {
    // partial last slab: masked scalar loads, zero beyond ke
    const int buf = nfull & 1;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int64_t k = kt + 2 * lq;
      const double* pa = ga[q] - 2 * lq;
      const double* pb = gb[q] - 2 * lq;
      v2d va, vb;
      va.x = (k < ke) ? pa[k] : 0.0;
      va.y = (k + 1 < ke) ? pa[k + 1] : 0.0;
      vb.x = (k < ke) ? pb[k] : 0.0;
      vb.y = (k + 1 < ke) ? pb[k + 1] : 0.0;
      *reinterpret_cast<v2d*>(&sA[buf][(lc + CPP * q) * LW + 2 * lq]) = va;
      *reinterpret_cast<v2d*>(&sB[buf][(lc + CPP * q) * LW + 2 * lq]) = vb;
    }
    __syncthreads();
    compute(buf);
  }
  tn_store(a, acc, tile, split, wave, lane, tm * 64 + ia0, tn * 64 + jb0, F32);
}

// Two tile rows per workgroup (512 threads): waves 0-3 compute tile row
// 2 tp, waves 4-7 tile row 2 tp + 1, both over the same staged slab of B, so
// B's columns are read once per pair of tile rows.  16-deep slabs (55 KB of
// LDS).  Thread (lc, lq) stages k pair lq of A's columns lc and lc + 64 and
// of B's column lc.  Each wave stores its 32 x 32 quadrant of its own 64 x 64
// tile with the contract of tn_lds_kernel (a missing second tile row of an
// odd tilesM stages and computes but stores nothing).
// Taken by the products with at least two tile rows and four tile columns
// that the 128 x 128 kernels do not take: FP32 ones whose depth is not a
// multiple of 32 (tnf_kernel) and FP64 ones whose depth is not a multiple of
// 16 (tnq_kernel).  Alone, the K = 49152, 256 x 32768 FP64 product
// ran at 63 TFLOP/s on it against 55 for tn_lds_kernel (tnq_kernel: 65-67).
template <int TAG, bool F32>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4))) void tn2_kernel(TnArgs a) {
  constexpr int SK = 16, LW = SK + 2;
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  typedef v4d Acc;    // FP64 accumulators (FP32 products are widened per slab)
  typedef typename OpT<F32>::type Op;
  __shared__ double sA[2][128 * LW];
  __shared__ double sB[2][64 * LW];
  const int tp = blockIdx.x / a.tilesN, tn = blockIdx.x % a.tilesN, split = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int h = wave >> 2, w4 = wave & 3;
  const int tm = 2 * tp + h;
  const int64_t kb = (int64_t)split * a.kchunk;
  const int64_t ke = std::min<int64_t>(a.K, kb + a.kchunk);
  const int lc = tid >> 3, lq = tid & 7;
  const double* ga[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int ia = tp * 128 + lc + 64 * q;
    // columns outside the matrix read column 0 and feed only unstored outputs
    ga[q] = a.A + (int64_t)(ia < a.M ? ia : 0) * a.lda + 2 * lq;
  }
  const int jb = tn * 64 + lc;
  const double* gb = a.B + (int64_t)(jb < a.N ? jb : 0) * a.ldb + 2 * lq;
  Acc acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Acc{0, 0, 0, 0};
  const int ia0 = h * 64 + (w4 & 1) * 32, jb0 = (w4 >> 1) * 32;
  const int nfull = (int)((ke - kb) / SK);
  auto compute = [&](int buf) {
    Op xa[2][4], xb[2][4];   // FP32 operands are rounded as they leave LDS
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const double* pa = &sA[buf][(ia0 + 16 * t + li) * LW + 4 * g];
      const double* pb = &sB[buf][(jb0 + 16 * t + li) * LW + 4 * g];
      v2d a0 = *reinterpret_cast<const v2d*>(pa), a1 = *reinterpret_cast<const v2d*>(pa + 2);
      v2d b0 = *reinterpret_cast<const v2d*>(pb), b1 = *reinterpret_cast<const v2d*>(pb + 2);
      xa[t][0] = a0.x; xa[t][1] = a0.y; xa[t][2] = a1.x; xa[t][3] = a1.y;
      xb[t][0] = b0.x; xb[t][1] = b0.y; xb[t][2] = b1.x; xb[t][3] = b1.y;
    }
    [[maybe_unused]] v4f t32[2][2];
    if constexpr (F32)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) t32[x][y] = v4f{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          if constexpr (F32)
            t32[x][y] = mfma(xb[y][s], xa[x][s], t32[x][y]);
          else
            acc[x][y] = mfma(xb[y][s], xa[x][s], acc[x][y]);
        }
    if constexpr (F32)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) widen_add(acc[x][y], t32[x][y]);
  };
  auto koff = [&](int sl) { return kb + (int64_t)std::min(sl, nfull - 1) * SK; };
  v2d ra0[2], rb0, ra1[2], rb1;
  auto load = [&](v2d (&ra)[2], v2d& rb, int64_t k) {
    ra[0] = *reinterpret_cast<const v2d*>(ga[0] + k);
    ra[1] = *reinterpret_cast<const v2d*>(ga[1] + k);
    rb = *reinterpret_cast<const v2d*>(gb + k);
  };
  auto put = [&](int buf, const v2d (&ra)[2], const v2d& rb) {
    *reinterpret_cast<v2d*>(&sA[buf][lc * LW + 2 * lq]) = ra[0];
    *reinterpret_cast<v2d*>(&sA[buf][(lc + 64) * LW + 2 * lq]) = ra[1];
    *reinterpret_cast<v2d*>(&sB[buf][lc * LW + 2 * lq]) = rb;
  };
  if (nfull > 0) {
    load(ra0, rb0, koff(0));
    load(ra1, rb1, koff(1));
    put(0, ra0, rb0);
    __syncthreads();
    int sl = 0;
    for (; sl + 2 <= nfull; sl += 2) {
      load(ra0, rb0, koff(sl + 2));
      __builtin_amdgcn_sched_barrier(0);
      compute(0);
      __builtin_amdgcn_sched_barrier(0);
      put(1, ra1, rb1);
      __syncthreads();
      load(ra1, rb1, koff(sl + 3));
      __builtin_amdgcn_sched_barrier(0);
      compute(1);
      __builtin_amdgcn_sched_barrier(0);
      put(0, ra0, rb0);
      __syncthreads();
    }
    if (sl < nfull) compute(0);
  }
  const int64_t kt = kb + (int64_t)nfull * SK;
  if (kt < ke) {
    // partial last slab: masked scalar loads, zero beyond ke
    const int buf = nfull & 1;
    const int64_t k = kt + 2 * lq;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double* p = (q < 2 ? ga[q] : gb) - 2 * lq;
      v2d v;
      v.x = (k < ke) ? p[k] : 0.0;
      v.y = (k + 1 < ke) ? p[k + 1] : 0.0;
      double* d = q < 2 ? &sA[buf][(lc + 64 * q) * LW + 2 * lq] : &sB[buf][lc * LW + 2 * lq];
      *reinterpret_cast<v2d*>(d) = v;
    }
    __syncthreads();
    compute(buf);
  }
  if (tm < a.ntiles / a.tilesN)
    tn_store(a, acc, tm * a.tilesN + tn, split, w4, lane, tm * 64 + (w4 & 1) * 32, tn * 64 + jb0, F32);
}

// 128 x 128 output per workgroup (512 threads, 2 x 4 waves, each wave 64
// rows x 32 columns: a 4 x 2 grid of 16 x 16 MFMA blocks), FP64, 16-deep
// slabs (72 KB of LDS) with one register set of staged loads (slab s + 1 is
// requested while slab s is multiplied), two workgroups per CU.  K a
// multiple of 16 (a masked last slab would not fit the 128 registers).  Each
// operand column staged is reused by 128 output columns (tn2_kernel: 64 or
// 128), which halves the L2 requests per flop.  Alone, the K = 49152
// products with 256 rows run at 67 TFLOP/s against 62 for tn2_kernel (the
// clock under FP64 MFMA load is ~2.2 GHz, not 2.4, and the MFMA pipes are
// busy ~80% of those cycles).  The output contract is tn_lds_kernel's on the
// 64 x 64 tiles the workgroup covers: wave (wi, wj) holds rows 64 wi .. +64
// and columns 32 wj .. +32, i.e. quadrants (0, wj % 2) and (1, wj % 2) of
// tile (2 tp + wi, 2 tq + wj / 2).  Tiles are taken with the row index
// fastest, so the workgroups that read the same columns of B are adjacent.
template <int TAG>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4))) void tnq_kernel(TnArgs a) {
  constexpr int SK = 16, LW = SK + 2, TPC = SK / 2, CPP = 512 / TPC;   // 8 threads per column, 64 columns a pass
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  __shared__ double sA[2][128 * LW];
  __shared__ double sB[2][128 * LW];
  const int tilesM = a.ntiles / a.tilesN;
  const int qm = (tilesM + 1) / 2;
  const int tp = blockIdx.x % qm, tq = blockIdx.x / qm, split = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int wi = wave & 1, wj = wave >> 1;
  const int ia0 = 64 * wi, jb0 = 32 * wj;
  const int64_t kb = (int64_t)split * a.kchunk;
  const int64_t ke = std::min<int64_t>(a.K, kb + a.kchunk);
  const int lc = tid / TPC, lq = tid % TPC;
  const double* ga[2];
  const double* gb[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int i = tp * 128 + lc + CPP * q, j = tq * 128 + lc + CPP * q;
    // columns outside the matrix read column 0 and feed only unstored outputs
    ga[q] = a.A + (int64_t)(i < a.M ? i : 0) * a.lda + 2 * lq;
    gb[q] = a.B + (int64_t)(j < a.N ? j : 0) * a.ldb + 2 * lq;
  }
  v4d acc[4][2];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0, 0, 0, 0};
  auto compute = [&](int buf) {
#pragma unroll
    for (int s0 = 0; s0 < 4; s0 += 2) {
      double xa[4][2], xb[2][2];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const v2d v = *reinterpret_cast<const v2d*>(&sA[buf][(ia0 + 16 * t + li) * LW + 4 * g + s0]);
        xa[t][0] = v.x; xa[t][1] = v.y;
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const v2d v = *reinterpret_cast<const v2d*>(&sB[buf][(jb0 + 16 * t + li) * LW + 4 * g + s0]);
        xb[t][0] = v.x; xb[t][1] = v.y;
      }
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma(xb[y][s], xa[x][s], acc[x][y]);
    }
  };
  const int nfull = (int)((ke - kb) / SK);
  v2d ra[2], rb[2];
  auto load = [&](int64_t k) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ra[q] = *reinterpret_cast<const v2d*>(ga[q] + k);
      rb[q] = *reinterpret_cast<const v2d*>(gb[q] + k);
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      *reinterpret_cast<v2d*>(&sA[buf][(lc + CPP * q) * LW + 2 * lq]) = ra[q];
      *reinterpret_cast<v2d*>(&sB[buf][(lc + CPP * q) * LW + 2 * lq]) = rb[q];
    }
  };
  if (nfull > 0) {
    load(kb);
    put(0);
    __syncthreads();
    for (int sl = 0; sl < nfull; ++sl) {
      if (sl + 1 < nfull) load(kb + (int64_t)(sl + 1) * SK);
      __builtin_amdgcn_sched_barrier(0);
      compute(sl & 1);
      __builtin_amdgcn_sched_barrier(0);
      if (sl + 1 < nfull) put((sl + 1) & 1);
      __syncthreads();
    }
  }
  // the wave's two quadrants of tile (tm, tn), in tn_lds_kernel's layout
  const int tm = 2 * tp + wi, tn = 2 * tq + (wj >> 1), ch = wj & 1;
  if (tm >= tilesM || tn >= a.tilesN) return;
  const int tile = tm * a.tilesN + tn;
#pragma unroll
  for (int xh = 0; xh < 2; ++xh) {
    const int quadrant = xh + 2 * ch;
    if (a.nsplit > 1) {
      double* mine = a.part + part_off(split, a.ntiles, tile, quadrant);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) mine[((x * 2 + y) * 4 + r) * 64 + lane] = acc[2 * xh + x][y][r];
    } else {
      // one 16 x 16 block at a time (its C2 loads issued before its stores)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int i = tm * 64 + 32 * xh + 16 * x + li;
          const int j0 = tn * 64 + 32 * ch + 16 * y;
          double old[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = j0 + colsub(r, g, false);
            old[r] = (a.C2 && i < a.M2 && j < a.N) ? a.C2[i + (int64_t)j * a.ldc2] : 0.0;
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = j0 + colsub(r, g, false);
            const double v = acc[2 * xh + x][y][r];
            if (i < a.M && j < a.N) {
              a.C[i + (int64_t)j * a.ldc] = v;
              if (a.C2 && i < a.M2) a.C2[i + (int64_t)j * a.ldc2] = old[r] + v;
            }
          }
        }
    }
  }
}

// FP32 form of tnq_kernel (the mixed-precision coefficient product
// R_bar = Qbar^T Q_t): 128 x 128 output per 512-thread workgroup, each wave a
// 64 x 32 block.  The operands are rounded to FP32 once, as they are staged,
// and LDS holds FP32 slabs of 32 k-values (72 KB; SK / 2 threads stage one
// column's slab, one 16-byte pair each).  Each 16 k-values are summed in FP32
// on v_mfma_f32_16x16x4_f32 and then added into the FP64 accumulators.  The
// accumulators of both precisions take more than 128 registers: one
// workgroup per CU.  Alone, at K = 49152 with 256 rows and 32768 columns:
// ~93 TFLOP/s, against ~69 when every wave rounded the FP64 operands it read
// from LDS.  K a multiple of 32; output contract of tnq_kernel in the FP32
// result layout.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void tnf_kernel(TnArgs a) {
  constexpr int SK = 32, LW = SK + 4, TPC = SK / 2, CPP = 512 / TPC, NQ = 128 / CPP;
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  __shared__ float sA[2][128 * LW];
  __shared__ float sB[2][128 * LW];
  const int tilesM = a.ntiles / a.tilesN;
  const int qm = (tilesM + 1) / 2;
  const int tp = blockIdx.x % qm, tq = blockIdx.x / qm, split = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int wi = wave & 1, wj = wave >> 1;
  const int ia0 = 64 * wi, jb0 = 32 * wj;
  const int64_t kb = (int64_t)split * a.kchunk;
  const int64_t ke = std::min<int64_t>(a.K, kb + a.kchunk);
  const int lc = tid / TPC, lq = tid % TPC;
  const double* ga[NQ];
  const double* gb[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int i = tp * 128 + lc + CPP * q, j = tq * 128 + lc + CPP * q;
    // columns outside the matrix read column 0 and feed only unstored outputs
    ga[q] = a.A + (int64_t)(i < a.M ? i : 0) * a.lda + 2 * lq;
    gb[q] = a.B + (int64_t)(j < a.N ? j : 0) * a.ldb + 2 * lq;
  }
  v4d acc[4][2];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0, 0, 0, 0};
  auto compute = [&](int buf) {
    // per 16 k-values: lane group g supplies k-values kk + 4 g .. + 4
#pragma unroll
    for (int kk = 0; kk < SK; kk += 16) {
      v4f t[4][2];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) t[x][y] = v4f{0, 0, 0, 0};
#pragma unroll
      for (int s0 = 0; s0 < 4; s0 += 2) {
        float fa[4][2], fb[2][2];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const v2f v = *reinterpret_cast<const v2f*>(&sA[buf][(ia0 + 16 * x + li) * LW + kk + 4 * g + s0]);
          fa[x][0] = v.x; fa[x][1] = v.y;
        }
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const v2f v = *reinterpret_cast<const v2f*>(&sB[buf][(jb0 + 16 * y + li) * LW + kk + 4 * g + s0]);
          fb[y][0] = v.x; fb[y][1] = v.y;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) t[x][y] = mfma(fb[y][s], fa[x][s], t[x][y]);
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) widen_add(acc[x][y], t[x][y]);
    }
  };
  v2d ra[NQ], rb[NQ];
  auto load = [&](int64_t k) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) ra[q] = *reinterpret_cast<const v2d*>(ga[q] + k);
#pragma unroll
    for (int q = 0; q < NQ; ++q) rb[q] = *reinterpret_cast<const v2d*>(gb[q] + k);
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      *reinterpret_cast<v2f*>(&sA[buf][(lc + CPP * q) * LW + 2 * lq]) = v2f{(float)ra[q].x, (float)ra[q].y};
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      *reinterpret_cast<v2f*>(&sB[buf][(lc + CPP * q) * LW + 2 * lq]) = v2f{(float)rb[q].x, (float)rb[q].y};
  };
  const int nfull = (int)((ke - kb) / SK);
  if (nfull > 0) {
    load(kb);
    put(0);
    __syncthreads();
    for (int sl = 0; sl < nfull; ++sl) {
      if (sl + 1 < nfull) load(kb + (int64_t)(sl + 1) * SK);
      __builtin_amdgcn_sched_barrier(0);
      compute(sl & 1);
      __builtin_amdgcn_sched_barrier(0);
      if (sl + 1 < nfull) put((sl + 1) & 1);
      __syncthreads();
    }
  }
  // the wave's two quadrants of tile (tm, tn), in tn_lds_kernel's layout
  const int tm = 2 * tp + wi, tn = 2 * tq + (wj >> 1), ch = wj & 1;
  if (tm >= tilesM || tn >= a.tilesN) return;
  const int tile = tm * a.tilesN + tn;
#pragma unroll
  for (int xh = 0; xh < 2; ++xh) {
    const int quadrant = xh + 2 * ch;
    if (a.nsplit > 1) {
      double* mine = a.part + part_off(split, a.ntiles, tile, quadrant);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) mine[((x * 2 + y) * 4 + r) * 64 + lane] = acc[2 * xh + x][y][r];
    } else {
      // one 16 x 16 block at a time (its C2 loads issued before its stores)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int i = tm * 64 + 32 * xh + 16 * x + li;
          const int j0 = tn * 64 + 32 * ch + 16 * y;
          double old[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = j0 + colsub(r, g, true);
            old[r] = (a.C2 && i < a.M2 && j < a.N) ? a.C2[i + (int64_t)j * a.ldc2] : 0.0;
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = j0 + colsub(r, g, true);
            const double v = acc[2 * xh + x][y][r];
            if (i < a.M && j < a.N) {
              a.C[i + (int64_t)j * a.ldc] = v;
              if (a.C2 && i < a.M2) a.C2[i + (int64_t)j * a.ldc2] = old[r] + v;
            }
          }
        }
    }
  }
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// x = hi + mid + lo + e with BF16 parts, each the rounding of what the parts
// before it leave (through FP32), |e| <= 2^-26 |x|: the differences x - hi
// and x - hi - mid are exact in FP64 (each part is within a factor 2^-8 of
// what it approximates).
__device__ __forceinline__ void split3(double x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)(float)x;
  const double r1 = x - (double)(float)h;
  m = (__bf16)(float)r1;
  const double r2 = r1 - (double)(float)m;
  l = (__bf16)(float)r2;
}

// D += X Y on BF16 MFMA, 16 x 16 x 32 (lane l supplies 8 k-values of row l % 16
// of X and of column l % 16 of Y; FP32 result in the f32 layout)
__device__ __forceinline__ v4f mfma_bf(const bf16x8& x, const bf16x8& y, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
}

// Split-BF16 form of tnq_kernel (the mixed-precision coefficient product
// R_bar = Qbar^T Q_t): 128 x 128 output per 512-thread workgroup, each wave a
// 64 x 32 block.  Slabs are 32 deep.  Every staged FP64 element is split
// into three BF16 parts (split3) as it is stored to LDS, into three planes
// per operand (k contiguous, 80-byte column pitch: conflict-free 16-byte
// reads); the product of two elements is taken as the six part products
// whose size is at least 2^-16 of the whole (hi hi, hi mid, mid hi, hi lo,
// lo hi, mid mid; the three dropped ones are below 2^-25 of it), issued
// smallest first into one FP32 accumulator per 32-k slab, which is then
// added into the FP64 accumulators.  Two LDS buffers (120 KB): one
// workgroup per CU, two waves per SIMD.  K a multiple of 32.
template <int TAG>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void tnb_kernel(TnArgs a) {
  constexpr int SK = 32, LW = SK + 8, TPC = SK / 2, CPP = 512 / TPC;   // 16 threads per column, 32 columns a pass
  constexpr int PL = 128 * LW;                                         // one plane of one operand
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  __shared__ __bf16 sA[2][3 * PL];
  __shared__ __bf16 sB[2][3 * PL];
  const int tilesM = a.ntiles / a.tilesN;
  const int qm = (tilesM + 1) / 2;
  const int tp = blockIdx.x % qm, tq = blockIdx.x / qm, split = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int wi = wave & 1, wj = wave >> 1;
  const int ia0 = 64 * wi, jb0 = 32 * wj;
  const int64_t kb = (int64_t)split * a.kchunk;
  const int64_t ke = std::min<int64_t>(a.K, kb + a.kchunk);
  const int lc = tid / TPC, lq = tid % TPC;
  const double* ga[4];
  const double* gb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = tp * 128 + lc + CPP * q, j = tq * 128 + lc + CPP * q;
    // columns outside the matrix read column 0 and feed only unstored outputs
    ga[q] = a.A + (int64_t)(i < a.M ? i : 0) * a.lda + 2 * lq;
    gb[q] = a.B + (int64_t)(j < a.N ? j : 0) * a.ldb + 2 * lq;
  }
  v4d acc[4][2];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0, 0, 0, 0};
  auto compute = [&](int buf) {
    bf16x8 fb[2][3];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int pl = 0; pl < 3; ++pl)
        fb[y][pl] = *reinterpret_cast<const bf16x8*>(&sB[buf][pl * PL + (jb0 + 16 * y + li) * LW + 8 * g]);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      bf16x8 fa[3];
#pragma unroll
      for (int pl = 0; pl < 3; ++pl)
        fa[pl] = *reinterpret_cast<const bf16x8*>(&sA[buf][pl * PL + (ia0 + 16 * x + li) * LW + 8 * g]);
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        // issued transposed (B's part first), smallest part products first
        v4f t = v4f{0, 0, 0, 0};
        t = mfma_bf(fb[y][2], fa[0], t);
        t = mfma_bf(fb[y][0], fa[2], t);
        t = mfma_bf(fb[y][1], fa[1], t);
        t = mfma_bf(fb[y][1], fa[0], t);
        t = mfma_bf(fb[y][0], fa[1], t);
        t = mfma_bf(fb[y][0], fa[0], t);
        widen_add(acc[x][y], t);
      }
    }
  };
  const int nsl = (int)((ke - kb) / SK);
  v2d ra[4], rb[4];
  auto load = [&](int64_t k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ra[q] = *reinterpret_cast<const v2d*>(ga[q] + k);
      rb[q] = *reinterpret_cast<const v2d*>(gb[q] + k);
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      __bf16 h0, m0, l0, h1, m1, l1;
      const int off = (lc + CPP * q) * LW + 2 * lq;
      split3(ra[q].x, h0, m0, l0);
      split3(ra[q].y, h1, m1, l1);
      *reinterpret_cast<bf16x2*>(&sA[buf][off]) = bf16x2{h0, h1};
      *reinterpret_cast<bf16x2*>(&sA[buf][PL + off]) = bf16x2{m0, m1};
      *reinterpret_cast<bf16x2*>(&sA[buf][2 * PL + off]) = bf16x2{l0, l1};
      split3(rb[q].x, h0, m0, l0);
      split3(rb[q].y, h1, m1, l1);
      *reinterpret_cast<bf16x2*>(&sB[buf][off]) = bf16x2{h0, h1};
      *reinterpret_cast<bf16x2*>(&sB[buf][PL + off]) = bf16x2{m0, m1};
      *reinterpret_cast<bf16x2*>(&sB[buf][2 * PL + off]) = bf16x2{l0, l1};
    }
  };
  if (nsl > 0) {
    load(kb);
    put(0);
    __syncthreads();
    for (int sl = 0; sl < nsl; ++sl) {
      if (sl + 1 < nsl) load(kb + (int64_t)(sl + 1) * SK);
      __builtin_amdgcn_sched_barrier(0);
      compute(sl & 1);
      __builtin_amdgcn_sched_barrier(0);
      if (sl + 1 < nsl) put((sl + 1) & 1);
      __syncthreads();
    }
  }
  // the wave's two quadrants of tile (tm, tn), in tn_lds_kernel's layout (f32 form)
  const int tm = 2 * tp + wi, tn = 2 * tq + (wj >> 1), ch = wj & 1;
  if (tm >= tilesM || tn >= a.tilesN) return;
  const int tile = tm * a.tilesN + tn;
#pragma unroll
  for (int xh = 0; xh < 2; ++xh) {
    const int quadrant = xh + 2 * ch;
    if (a.nsplit > 1) {
      double* mine = a.part + part_off(split, a.ntiles, tile, quadrant);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) mine[((x * 2 + y) * 4 + r) * 64 + lane] = acc[2 * xh + x][y][r];
    } else {
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int i = tm * 64 + 32 * xh + 16 * x + li;
          const int j0 = tn * 64 + 32 * ch + 16 * y;
          double old[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = j0 + colsub(r, g, true);
            old[r] = (a.C2 && i < a.M2 && j < a.N) ? a.C2[i + (int64_t)j * a.ldc2] : 0.0;
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j = j0 + colsub(r, g, true);
            const double v = acc[2 * xh + x][y][r];
            if (i < a.M && j < a.N) {
              a.C[i + (int64_t)j * a.ldc] = v;
              if (a.C2 && i < a.M2) a.C2[i + (int64_t)j * a.ldc2] = old[r] + v;
            }
          }
        }
    }
  }
}

// Fallback for operands that are not 16-byte aligned or have odd leading
// dimensions: direct scalar loads, same tiling and output contract.
__global__ __launch_bounds__(256) void tn_direct_kernel(TnArgs a) {
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  const int tile = blockIdx.x, split = blockIdx.y;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int i0 = tm * 64 + (wave & 1) * 32, j0 = tn * 64 + (wave >> 1) * 32;
  const int64_t kb = (int64_t)split * a.kchunk;
  const int64_t ke = std::min<int64_t>(a.K, kb + a.kchunk);
  const double* ap[2];
  const double* bp[2];
  bool aok[2], bok[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    int i = i0 + 16 * t + li, j = j0 + 16 * t + li;
    aok[t] = i < a.M;
    bok[t] = j < a.N;
    ap[t] = a.A + (int64_t)(aok[t] ? i : 0) * a.lda;
    bp[t] = a.B + (int64_t)(bok[t] ? j : 0) * a.ldb;
  }
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0, 0, 0, 0};
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
    double xa[2][4], xb[2][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = k0 + 4 * g + s;
      const bool kok = k < ke;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        xa[t][s] = (aok[t] && kok) ? ap[t][k] : 0.0;
        xb[t][s] = (bok[t] && kok) ? bp[t][k] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma(xb[y][s], xa[x][s], acc[x][y]);
  }
  tn_store(a, acc, tile, split, wave, lane, i0, j0, false);
}

// Sum the split partials in split order; write C (and C2 +=).  One block per
// wave quadrant of a tile, thread (qg, lane) owns 4 of the lane's 16 values.
__global__ __launch_bounds__(256) void tn_reduce_kernel(TnArgs a) {
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  const int tile = blockIdx.x >> 2, wave = blockIdx.x & 3;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int qg = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int i = tm * 64 + (wave & 1) * 32 + 16 * (qg >> 1) + li;
  const int jq = tn * 64 + (wave >> 1) * 32 + 16 * (qg & 1);         // + colsub(u, g)
  double old[4];
  if (a.C2) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = jq + colsub(u, g, a.f32);
      old[u] = (i < a.M2 && j < a.N) ? a.C2[i + (int64_t)j * a.ldc2] : 0.0;
    }
  }
  double v[4];
  sum_partials4(a.part, a.nsplit, a.ntiles, tile, wave, qg, lane, v);
  if (i >= a.M) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = jq + colsub(u, g, a.f32);
    if (j < a.N) {
      a.C[i + (int64_t)j * a.ldc] = v[u];
      if (a.C2 && i < a.M2) a.C2[i + (int64_t)j * a.ldc2] = old[u] + v[u];
    }
  }
}

static bool aligned16(const void* p, int64_t ld) {
  return (reinterpret_cast<uintptr_t>(p) % 16 == 0) && (ld % 2 == 0);
}

static int pick_split(int tiles, int64_t K, int64_t cap) {
  // Below 256 workgroups: at most 512 (two resident per CU, so one wave of
  // workgroups; a few over that run as a second wave and cost ~16% at 79
  // tiles).  From 256 on, splits up to ~1280 workgroups: the shorter
  // workgroups even out the last wave (alone, the 128 x 20480 product with
  // depth 24576 runs at 51.6 TFLOP/s with two splits against 44.3 with one).
  // Each split keeps at least 256 rows (8 slabs).
  int want = tiles >= 256 ? (1280 + tiles - 1) / tiles : std::max(1, 512 / std::max(1, tiles));
  int64_t maxs = std::max<int64_t>(1, K / 256);
  int ns = (int)std::min<int64_t>(want, maxs);
  while (ns > 1 && (int64_t)ns * tiles > cap) --ns;
  return ns;
}

// The 512-thread products (128 x 128 or two-tile-row; two workgroups per CU,
// 512 slots): about 1280 workgroups whatever the tile count, so that the last
// wave of workgroups is short, each split keeping at least 256 rows.  Alone, the 128 x 20480
// product of depth 24576 (160 tiles) runs at 60.8 TFLOP/s with 8 splits
// against 51.5 with the 3 that filling one wave of slots gives.
static int pick_split_quad(int blocks, int64_t K, int64_t cap, int tiles) {
  const int64_t maxs = std::max<int64_t>(1, K / 256);
  int ns = (int)std::min<int64_t>((1280 + blocks - 1) / blocks, maxs);
  while (ns > 1 && (int64_t)ns * tiles > cap) --ns;
  return std::max(ns, 1);
}

TnArgs tn_setup(const double* A, int64_t lda, const double* B, int64_t ldb, int M, int N, int64_t K, double* C,
                int64_t ldc, double* C2, int64_t ldc2, const Scratch& s, int force_split, int lowp) {
  const bool f32 = lowp != 0;
  TnArgs a{};
  a.A = A; a.lda = lda; a.B = B; a.ldb = ldb;
  a.C = C; a.ldc = ldc; a.C2 = C2; a.ldc2 = ldc2; a.M2 = M;
  const int tilesM = (M + kTile - 1) / kTile, tilesN = (N + kTile - 1) / kTile;
  const int tiles = tilesM * tilesN;
  const bool vec = aligned16(A, lda) && aligned16(B, ldb);
  // two tile rows per workgroup from two tile rows and four tile columns on
  // (with fewer tile columns the re-projections on the panel chain slow down)
  const bool pair = vec && tilesM >= 2 && tilesN >= 4;
  // products of at least two tile rows and columns: 128 x 128 per workgroup
  // and a depth that is a multiple of 16 (whole slabs in every split)
  // (32 for FP32 products, whose slabs are 32 deep)
  const bool quad = vec && tilesM >= 2 && tilesN >= 2 && K % (f32 ? 32 : 16) == 0;
  // the split-BF16 product on the same 128 x 128 tiles
  const bool bf3 = vec && lowp == 2 && tilesM >= 2 && tilesN >= 2 && K % 32 == 0;
  // the split count fills the grid of workgroups the product launches
  const int blocks = quad || bf3 ? (tilesM + 1) / 2 * ((tilesN + 1) / 2) : pair ? (tilesM + 1) / 2 * tilesN : tiles;
  int ns = force_split > 0 ? force_split
           : quad || bf3 || pair ? pick_split_quad(blocks, K, s.npart, tiles)
                           : pick_split(blocks, K, s.npart);
  while (ns > 1 && (int64_t)ns * tiles > s.npart) --ns;
  int64_t kchunk = (K + ns - 1) / ns;
  kchunk = (kchunk + KC - 1) / KC * KC;
  ns = (int)((K + kchunk - 1) / kchunk);
  a.M = M; a.N = N; a.K = K; a.kchunk = kchunk; a.nsplit = ns; a.tilesN = tilesN; a.ntiles = tiles;
  a.part = s.part;
  a.vec = vec;
  a.f32 = f32 && a.vec;     // the FP32 form exists for the LDS-staged kernel
  a.pair = pair && !quad && !bf3;
  a.quad = quad;
  a.bf3 = bf3;
  return a;
}

void launch_tn_product(const TnArgs& a, int tag, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0) return;
  const dim3 grid(a.ntiles, a.nsplit);
  if (!a.vec) {
    hipLaunchKernelGGL(tn_direct_kernel, grid, dim3(256), 0, st, a);
    return;
  }
  if (a.bf3) {
    const dim3 gridb((unsigned)((a.ntiles / a.tilesN + 1) / 2 * ((a.tilesN + 1) / 2)), a.nsplit);
    hipLaunchKernelGGL((tnb_kernel<TAG_TRAIL>), gridb, dim3(512), 0, st, a);
    return;
  }
  if (a.quad) {
    const dim3 gridq((unsigned)((a.ntiles / a.tilesN + 1) / 2 * ((a.tilesN + 1) / 2)), a.nsplit);
    if (a.f32) {
      hipLaunchKernelGGL(tnf_kernel, gridq, dim3(512), 0, st, a);
      return;
    }
    switch (tag) {
      case TAG_TRAIL: hipLaunchKernelGGL((tnq_kernel<TAG_TRAIL>), gridq, dim3(512), 0, st, a); break;
      case TAG_REPROJ: hipLaunchKernelGGL((tnq_kernel<TAG_REPROJ>), gridq, dim3(512), 0, st, a); break;
      default: hipLaunchKernelGGL((tnq_kernel<TAG_PANEL>), gridq, dim3(512), 0, st, a); break;
    }
    return;
  }
  if (a.pair) {
    const dim3 grid2((unsigned)((a.ntiles / a.tilesN + 1) / 2 * a.tilesN), a.nsplit);
    if (a.f32) {
      hipLaunchKernelGGL((tn2_kernel<TAG_TRAIL, true>), grid2, dim3(512), 0, st, a);
      return;
    }
    switch (tag) {
      case TAG_TRAIL: hipLaunchKernelGGL((tn2_kernel<TAG_TRAIL, false>), grid2, dim3(512), 0, st, a); break;
      case TAG_REPROJ: hipLaunchKernelGGL((tn2_kernel<TAG_REPROJ, false>), grid2, dim3(512), 0, st, a); break;
      default: hipLaunchKernelGGL((tn2_kernel<TAG_PANEL, false>), grid2, dim3(512), 0, st, a); break;
    }
    return;
  }
  if (a.f32 && a.ntiles / a.tilesN >= 2 && a.tilesN >= 2) {
    hipLaunchKernelGGL((tn16_kernel<TAG_TRAIL, true>), grid, dim3(256), 0, st, a);
    return;
  }
  if (a.f32) {
    hipLaunchKernelGGL((tn_lds_kernel<TAG_TRAIL, true>), grid, dim3(256), 0, st, a);
    return;
  }
  switch (tag) {
    case TAG_TRAIL: hipLaunchKernelGGL((tn_lds_kernel<TAG_TRAIL, false>), grid, dim3(256), 0, st, a); break;
    case TAG_REPROJ: hipLaunchKernelGGL((tn_lds_kernel<TAG_REPROJ, false>), grid, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((tn_lds_kernel<TAG_PANEL, false>), grid, dim3(256), 0, st, a); break;
  }
}

void launch_tn_reduce(const TnArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0 || a.nsplit <= 1) return;
  hipLaunchKernelGGL(tn_reduce_kernel, dim3(a.ntiles * 4), dim3(256), 0, st, a);
}

// --------------------------------------------------------------------------
// Upper Cholesky factor of a panel leaf's Gram matrix W (w <= kLeaf), its
// inverse, and on the second pass R2 R1 and the lookahead coefficients T^T X.
// One block of four waves (see chol_blocked for the factorization).  A
// pivot at most kCholBreak times its column's diagonal entry is a breakdown,
// handled by the column-wise fallback described at chol_body.
// --------------------------------------------------------------------------

// Smallest pivot / diagonal ratio a Cholesky-QR pass accepts: below it a
// column lies within 1e-7 rad of the span of the columns before it, the
// panel's condition number exceeds ~1e7, and one Cholesky-QR pass could no
// longer bring the panel close enough to orthonormal for the second to finish.
constexpr double kCholBreak = 1e-14;


// 1/sqrt(x) to full double precision: hardware estimate plus one Newton step.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * y;
  const double r = fma(-h, y, 0.5);
  return fma(y, r, y);
}

// 16 x 16 block product on MFMA: acc += sum over k < 16 nk of A(i, k) B(k, j)
// for the block's i, j < 16.  Lane (li, g) feeds A(li, k) and B(k, li) for
// k = k0 + 4g + s, and holds C[li][4r + g] in acc[r] (the layout used
// throughout this file).
template <class FA, class FB>
__device__ __forceinline__ void mma16(v4d& acc, int lane, int nk, FA A, FB B) {
  const int li = lane & 15, g = lane >> 4;
  for (int k0 = 0; k0 < 16 * nk; k0 += 16) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      acc = mfma(B(k, li), A(li, k), acc);
    }
  }
}

// One wave factors the 16 x 16 diagonal block at offset o of Rl (its upper
// triangle, already updated, read symmetrically): Gauss elimination of the
// augmented [D | I] with each final row scaled by 1/sqrt(pivot), so D = R^T R
// gives R (into Rl's block, zero below the diagonal) and T = R^{-1} (into
// Tl's block).  Lanes 0..15 hold column tx of D, lanes 16..31 column tx of
// the identity half, 16 rows in registers.  Step j: the D lanes publish row j
// (by symmetry also column j) through LDS, every lane reads the pivot and the
// column-j factors, and subtracts.  Only the wave's own LDS traffic orders the
// steps (in-order LDS within a wave), so there is no block barrier.
__device__ __forceinline__ void chol_diag16(int lane, int o, double (*Rl)[kLeaf + 1], double (*Tl)[kLeaf + 1],
                                            double* prow, const double* dg, bool& bad) {
  const int tx = lane & 15;
  const bool dl = lane < 16, zl = lane >= 16 && lane < 32;
  double c[16];
#pragma unroll
  for (int i = 0; i < 16; ++i)
    c[i] = dl ? ((i <= tx) ? Rl[o + i][o + tx] : Rl[o + tx][o + i]) : (zl && i == tx ? 1.0 : 0.0);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (dl) prow[tx] = c[j];
    __builtin_amdgcn_wave_barrier();
    double piv = prow[j];
    double fac[16];
#pragma unroll
    for (int i = j + 1; i < 16; ++i) fac[i] = prow[i];
    __builtin_amdgcn_wave_barrier();
    // breakdown: a pivot that is not positive, or below kCholBreak times the
    // column's diagonal entry in the Gram matrix (the column lies within an
    // angle of 1e-7 of the span of the columns before it)
    if (!(piv > kCholBreak * dg[o + j]) || !isfinite(piv)) {
      bad = true;
      piv = 1.0;
    }
    const double inv = rsqrt_nr(piv);
    const double f = c[j] * inv * inv;
#pragma unroll
    for (int i = j + 1; i < 16; ++i) c[i] -= fac[i] * f;
    if (dl) Rl[o + j][o + tx] = (tx >= j) ? c[j] * inv : 0.0;
    if (zl) Tl[o + tx][o + j] = c[j] * inv;
  }
}

// Exact path: blocked right-looking Cholesky of the 64 x 64 W in Rl (16 x 16
// blocks) and the inverse T = R^{-1} in Tl.  Block step b: wave 0 factors the
// diagonal block (R_bb, T_bb); the row panel R_bc = T_bb^T W_bc (c > b) and
// the trailing update W_cd -= R_bc^T R_bd (b < c <= d) run on MFMA, one
// 16 x 16 block per wave.  Then T's off-diagonal blocks, one block column per
// wave: T_ab = -T_aa sum_{c=a+1..b} R_ac T_cb for a = b-1 down to 0.  About a
// dozen block barriers instead of one per pivot.
__device__ __forceinline__ void chol_blocked(int tid, double (*Rl)[kLeaf + 1], double (*Tl)[kLeaf + 1],
                                             double* prow, const double* dg, bool& bad) {
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
#pragma unroll 1
  for (int b = 0; b < 4; ++b) {
    const int o = 16 * b;
    if (wave == 0) chol_diag16(lane, o, Rl, Tl, prow, dg, bad);
    __syncthreads();
    // row panel R_bc = T_bb^T W_bc, in place
    const int c = b + 1 + wave;
    if (c < 4) {
      v4d acc = v4d{0, 0, 0, 0};
      mma16(acc, lane, 1, [&](int i, int k) { return Tl[o + k][o + i]; },
            [&](int k, int j) { return Rl[o + k][16 * c + j]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) Rl[o + li][16 * c + 4 * r + g] = acc[r];
    }
    __syncthreads();
    // trailing update W_cd -= R_bc^T R_bd over the upper blocks b < c <= d
    int p = 0;
#pragma unroll 1
    for (int cc = b + 1; cc < 4; ++cc)
#pragma unroll 1
      for (int dd = cc; dd < 4; ++dd, ++p) {
        if ((p & 3) != wave) continue;
        v4d acc = v4d{0, 0, 0, 0};
        mma16(acc, lane, 1, [&](int i, int k) { return Rl[o + k][16 * cc + i]; },
              [&](int k, int j) { return Rl[o + k][16 * dd + j]; });
#pragma unroll
        for (int r = 0; r < 4; ++r) Rl[16 * cc + li][16 * dd + 4 * r + g] -= acc[r];
      }
    __syncthreads();
  }
  if (wave < 3) {
    // block column bc = wave + 1 of T
    const int bc = wave + 1;
#pragma unroll 1
    for (int a = bc - 1; a >= 0; --a) {
      v4d acc = v4d{0, 0, 0, 0};
#pragma unroll 1
      for (int cb = a + 1; cb <= bc; ++cb)
        mma16(acc, lane, 1, [&](int i, int k) { return Rl[16 * a + i][16 * cb + k]; },
              [&](int k, int j) { return Tl[16 * cb + k][16 * bc + j]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) Tl[16 * a + li][16 * bc + 4 * r + g] = acc[r];
      __builtin_amdgcn_wave_barrier();
      v4d t = v4d{0, 0, 0, 0};
      mma16(t, lane, 1, [&](int i, int k) { return Tl[16 * a + i][16 * a + k]; },
            [&](int k, int j) { return Tl[16 * a + k][16 * bc + j]; });
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int r = 0; r < 4; ++r) Tl[16 * a + li][16 * bc + 4 * r + g] = -t[r];
    }
  } else {
    // the blocks below the diagonal of R and T are zero
    for (int e = lane; e < 6 * 256; e += 64) {
      const int blk = e >> 8, q = e & 255;
      const int cb = blk < 3 ? 1 + blk : (blk < 5 ? 2 + (blk - 3) : 3);   // (1,0) (2,0) (3,0) (2,1) (3,1) (3,2)
      const int db = blk < 3 ? 0 : (blk < 5 ? 1 : 2);
      Rl[16 * cb + (q & 15)][16 * db + (q >> 4)] = 0.0;
      Tl[16 * cb + (q & 15)][16 * db + (q >> 4)] = 0.0;
    }
  }
  __syncthreads();
}

// C = op(A) B for 64 x 64 LDS matrices (row-major, padded): op(A) = A, or
// A^T when TRANS_A.  UPPER: A and B upper triangular (C[i][j] needs only
// k in [i, j]; k blocks left of the row block are skipped).  Wave v computes
// rows 16v..16v+15 and stores C[i][j] (i < w, j < wc) into the column-major
// global matrix out (ld ldo).
template <bool TRANS_A, bool UPPER>
__device__ __forceinline__ void lds_mm_store(int tid, const double (*Al)[kLeaf + 1], const double (*Bl)[kLeaf + 1],
                                             int w, int wc, double* out, int64_t ldo) {
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  v4d acc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) acc[y] = v4d{0, 0, 0, 0};
  for (int k0 = UPPER ? 16 * wave : 0; k0 < kLeaf; k0 += 16) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      const double xa = TRANS_A ? Al[k][16 * wave + li] : Al[16 * wave + li][k];
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[y] = mfma(Bl[k][16 * y + li], xa, acc[y]);
    }
  }
  const int i = 16 * wave + li;
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * y + 4 * r + g;
      if (i < w && j < wc) out[i + (int64_t)j * ldo] = acc[y][r];
    }
}

// The split reduction of a trailing-update product W = P1^T Q_t formed from
// a panel after its first Cholesky pass, with the second pass's transform
// folded in: out = T^T W (T = R2^{-1}, w x w upper triangular) equals
// (P1 T)^T Q_t, the coefficients against the finished panel P = P1 T.  M = w
// <= 64, so the product has a single tile row; four blocks share a 64-column
// tile, block cg taking the 16 columns that two wave quadrants of the product
// hold in their accumulator registers (quadrant column half cg >> 1, lane
// column group cg & 1).  The 64 x 16 strip of W is summed in split order into
// LDS (or read from a.C, where a product without a split stored it) and
// multiplied by T^T on MFMA, wave v forming rows 16v .. 16v + 15.
// When the panel's second pass took the column-wise fallback (*fb set), the
// finished panel is no longer P1 T, and the strip's coefficients are formed
// directly as P^T Q_t over the a.K rows (P: ld ldp, Q_t = a.B), on MFMA with
// operands read straight from memory (a rare path; its speed does not
// matter).
__global__ __launch_bounds__(256) void tn_reduce_tmul_kernel(TnArgs a, const double* T, int w, double* out,
                                                             int64_t ldo, const int* fb, const double* P,
                                                             int64_t ldp) {
  __shared__ double Wl[kLeaf][16 + 1];
  __shared__ double Tl[kLeaf][kLeaf + 1];
  const int tile = blockIdx.x >> 2, cg = blockIdx.x & 3, tid = threadIdx.x;
  const int lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int64_t jc = (int64_t)tile * kTile + (cg >> 1) * 32 + 16 * (cg & 1);   // first column of the strip
  const int wc = (int)std::max<int64_t>(0, std::min<int64_t>(16, a.N - jc));
  if (fb && *fb) {
    const int wave = tid >> 6;
    const int i = 16 * wave + li, j = li;
    const double* pa = P + (int64_t)(i < w ? i : 0) * ldp;
    const double* pb = a.B + (jc + (j < wc ? j : 0)) * a.ldb;
    v4d acc = v4d{0, 0, 0, 0};
    for (int64_t k0 = 0; k0 < a.K; k0 += 16) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t k = k0 + 4 * g + s;
        const double xa = (k < a.K && i < w) ? pa[k] : 0.0;
        const double xb = (k < a.K && j < wc) ? pb[k] : 0.0;
        acc = mfma(xb, xa, acc);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jj = 4 * r + g;
      if (i < w && jj < wc) out[i + (jc + jj) * ldo] = acc[r];
    }
    return;
  }
  double tv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, k = e & 63, i = e >> 6;
    tv[q] = (k < w && i < w) ? T[k + (int64_t)i * w] : 0.0;
  }
  if (a.nsplit > 1) {
    // thread (row half wr, row group qh, lane) sums 4 values of quadrant
    // wr + 2 (cg >> 1), lane group 2 qh + (cg & 1)
    const int wr = tid >> 7, qh = (tid >> 6) & 1;
    double v[4];
    sum_partials4(a.part, a.nsplit, a.ntiles, tile, wr | ((cg >> 1) << 1), (qh << 1) | (cg & 1), lane, v);
    const int i = wr * 32 + 16 * qh + li;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = colsub(u, g, a.f32);
      Wl[i][j] = (i < w && j < wc) ? v[u] : 0.0;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, i = e & 63, j = e >> 6;
      Wl[i][j] = (i < w && j < wc) ? a.C[i + (jc + j) * a.ldc] : 0.0;
    }
  }
  // Tl[k][i] = T[k][i]: the transposed operand of the product
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    Tl[e & 63][e >> 6] = tv[q];
  }
  __syncthreads();
  const int wave = tid >> 6;
  v4d acc = v4d{0, 0, 0, 0};
#pragma unroll
  for (int k0 = 0; k0 < kLeaf; k0 += 16)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      acc = mfma(Wl[k][li], Tl[k][16 * wave + li], acc);
    }
  const int i = 16 * wave + li;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j = 4 * r + g;
    if (i < w && j < wc) out[i + (jc + j) * ldo] = acc[r];
  }
}

void launch_tn_reduce_tmul(const TnArgs& a, const double* T, int w, double* out, int64_t ldo, hipStream_t st,
                           const int* fb, const double* P, int64_t ldp) {
  if (a.M <= 0 || a.N <= 0) return;
  hipLaunchKernelGGL(tn_reduce_tmul_kernel, dim3(a.ntiles * 4), dim3(256), 0, st, a, T, w, out, ldo, fb, P, ldp);
}

// C = T^T X with T (64 x 64, upper triangular, row-major LDS) and X (w x w,
// column-major global, ld ldx, read straight from L2); C[i][j] (i, j < w) to
// the column-major global matrix out (ld ldo).  Wave v computes rows
// 16v..16v+15; (T^T)[i][k] = T[k][i] vanishes for k > i.
__device__ __forceinline__ void tmul_global_store(int tid, const double (*Tl)[kLeaf + 1], const double* X,
                                                  int64_t ldx, int w, double* out, int64_t ldo) {
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  v4d acc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) acc[y] = v4d{0, 0, 0, 0};
  // every k block the wave needs (k0 <= 16 wave) is requested before the
  // first product, so the L2 round trips overlap
  double xb[4][4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 16 * c + 4 * g + s, j = 16 * y + li;
        xb[c][y][s] = (c <= wave && k < w && j < w) ? X[k + (int64_t)j * ldx] : 0.0;
      }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c > wave) break;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 16 * c + 4 * g + s;
      const double xa = Tl[k][16 * wave + li];
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[y] = mfma(xb[c][y][s], xa, acc[y]);
    }
  }
  const int i = 16 * wave + li;
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * y + 4 * r + g;
      if (i < w && j < w) out[i + (int64_t)j * ldo] = acc[y][r];
    }
}

// Breakdown fallback of the second pass: the column-wise CGS2 product
// out (w x wn, ld ldo) = P^T Qn over mrows rows, one column of Qn per
// workgroup pass (the coefficients of the next panel against the panel the
// fallback orthogonalised).
template <int NT>
__device__ void colwise_product_store(double* P, int64_t ldp, int64_t mrows, int w, const double* Qn,
                                      int64_t ldqn, int wn, double* out, int64_t ldo, ColwiseLds<NT>& L) {
  const int tid = threadIdx.x;
  for (int jn = 0; jn < wn; ++jn) {
    for (int c0 = 0; c0 < w; c0 += kColChunk)
      colwise_dots<NT>(P, ldp, mrows, c0, min(w, c0 + kColChunk), Qn + (int64_t)jn * ldqn, L.s1, nullptr, -1,
                       1.0, L);
    if (tid < w) out[tid + jn * ldo] = L.s1[tid];
    __syncthreads();
  }
}

// The second pass's breakdown fallback, kept out of line so that its loops
// do not add to the registers of the Cholesky path: CGS2 of the panel into
// Rl, and the next panel's coefficients P^T Q_next when Rbar is given.
// Returns false for a zero column (exact rank deficiency).
__device__ __attribute__((noinline)) bool chol_fallback(const CholArgs& a, double (*Rl)[kLeaf + 1],
                                                        ColwiseLds<256>* L) {
  const bool ok = colwise_panel<256>(a.P, a.ldp, a.mrows, a.w, Rl, *L);
  if (a.X)
    colwise_product_store<256>(a.P, a.ldp, a.mrows, a.w, a.P + (int64_t)a.w * a.ldp, a.ldp, a.w, a.Rbar, a.ldr,
                               *L);
  return ok;
}

// The kernel body on caller-provided LDS (Rl, Tl: 64 x 65 each; prow: 16;
// dg: 64; flags: 3 ints; L: the column-wise routine's reduction space, pass 2
// only).  PASS1_ONLY drops the second-pass code.
//
// Breakdown (a Cholesky pivot at most kCholBreak times its diagonal entry):
// on the first pass R1 = T1 = I are returned, so the transform leaves the
// panel as it is, and the breakdown is flagged in info[1]; on the second pass
// (flagged, or breaking down itself) the panel is orthogonalised column by
// column by CGS2 in this workgroup, T = I is returned, R_panel = R_cgs2 R1,
// the next panel's coefficients are computed from the finished panel
// directly, the panel is marked in a.fb for the update that started from its
// first pass, and info[2] counts the fallback.  Only a panel that is exactly
// rank-deficient (a zero column after projection) sets info[0].
template <bool PASS1_ONLY>
__device__ __forceinline__ void chol_body(const CholArgs& a, double (*Rl)[kLeaf + 1], double (*Tl)[kLeaf + 1],
                                          double* prow, double* dg, int* flags, ColwiseLds<256>* L) {
  const int pass = PASS1_ONLY ? 1 : a.pass;
  int& s_exact = flags[0];
  int& s_bad = flags[1];
  int& s_fb = flags[2];
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6, w = a.w;
  if (tid == 0) {
    s_exact = (pass == 1);
    s_bad = 0;
    s_fb = pass == 2 ? a.info[1] : 0;
  }
  // W (w x w) into Rl, identity-padded: all loads issued first
  {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = ty + 4 * q;   // column
      v[q] = (tx < w && k < w) ? a.W[tx + (int64_t)k * a.ldw] : (tx == k ? 1.0 : 0.0);
    }
    bool far = false;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = ty + 4 * q;
      Rl[tx][k] = v[q];
      if (k == tx) dg[tx] = v[q];
      far |= !(fabs(v[q] - (tx == k ? 1.0 : 0.0)) <= 1e-8);
    }
    __syncthreads();
    if (pass == 2 && far) s_exact = 1;
  }
  __syncthreads();
  if (s_fb) {
    // the first pass broke down: nothing to factor here
  } else if (s_exact) {
    bool bad = false;
    chol_blocked(tid, Rl, Tl, prow, dg, bad);
    if (bad) s_bad = 1;
  } else {
    // W = I + E with |E| <= 1e-8: R = I + F, F = strict upper part of E plus
    // half its diagonal; R^{-1} = I - F up to O(|E|^2), below rounding.
    double f[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = ty + 4 * q;
      f[q] = (i < tx) ? Rl[i][tx] : (i == tx ? 0.5 * (Rl[i][i] - 1.0) : 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = ty + 4 * q;
      const double id = (i == tx) ? 1.0 : 0.0;
      Rl[i][tx] = id + f[q];
      Tl[i][tx] = id - f[q];
    }
  }
  __syncthreads();
  bool rank_deficient = false;
  if (pass == 1 && s_bad) {
    // leave the panel as it is: R1 = T1 = I; the second pass takes over
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = ty + 4 * q;
      Rl[tx][k] = Tl[tx][k] = (tx == k) ? 1.0 : 0.0;
    }
    if (tid == 0) a.info[1] = 1;
    __syncthreads();
  }
  if constexpr (!PASS1_ONLY) {
    if (pass == 2 && (s_fb || s_bad)) {
      // column-wise CGS2 of the panel in place: R_cgs2 into Rl, T = I, and
      // the next panel's coefficients from the finished panel
      rank_deficient = !chol_fallback(a, Rl, L);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = ty + 4 * q;
        Tl[tx][k] = (tx == k) ? 1.0 : 0.0;
      }
      if (tid == 0) {
        a.info[1] = 0;
        a.info[2] += 1;
        if (a.fb) *a.fb = 1;
      }
      __syncthreads();
    }
  }
  // T (and R1 on the first pass) to global, column-major w x w
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = ty + 4 * q;
    if (tx < w && k < w) {
      a.T[tx + k * w] = Tl[tx][k];
      if (pass == 1) a.R1[tx + k * w] = Rl[tx][k];
      if (pass == 2 && a.Tcopy) a.Tcopy[tx + k * w] = Tl[tx][k];
    }
  }
  if constexpr (!PASS1_ONLY) {
    if (pass == 2) {
      // R1 for R_panel = R2 R1, requested before T^T X so both loads overlap
      double r1v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = ty + 4 * q;
        r1v[q] = (tx < w && k < w) ? a.R1[tx + k * w] : (tx == k ? 1.0 : 0.0);
      }
      // the next panel's update coefficients: (P1 T)^T Q_next = T^T X (after a
      // fallback they were formed from the finished panel itself)
      if (a.X && !(s_fb || s_bad)) tmul_global_store(tid, Tl, a.X, a.ldx, w, a.Rbar, a.ldr);
      // R_panel = R2 R1 with R1 staged in Tl (T is stored)
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = ty + 4 * q;
        Tl[tx][k] = r1v[q];
      }
      __syncthreads();
      lds_mm_store<false, true>(tid, Rl, Tl, w, w, a.Rout, a.ldr);
    }
  }
  if (tid == 0 && rank_deficient && a.info[0] == 0) a.info[0] = 1 + a.panel;
}

__global__ __launch_bounds__(256) void chol_kernel(CholArgs a) {
  __builtin_amdgcn_s_setprio(2);   // the panel chain sets the pace of the factorization
  __shared__ double Rl[kLeaf][kLeaf + 1];
  __shared__ double Tl[kLeaf][kLeaf + 1];
  __shared__ double prow[16];
  __shared__ double dg[kLeaf];
  __shared__ int flags[3];
  __shared__ ColwiseLds<256> L;
  chol_body<false>(a, Rl, Tl, prow, dg, flags, &L);
}

// A panel leaf orthogonalised column by column (the CGS2, ICGS and MGS panel
// modes) by a grid of workgroups, each owning one slab of rows.  A column
// needs a sum over all rows before every update, so each step of the method
// is one launch: it first reduces the partial sums every workgroup of the
// previous launch left (all workgroups sum them redundantly, in the same
// fixed order, so they take identical decisions), then works on its own
// slab and leaves its partial sums for the next launch.  Kernel boundaries
// order the steps; nothing waits inside a launch.
//
// CGS2 / ICGS, column j:
//   PROJECT(j)  s1 = the reduced P[:, <j]^T p_j; column j-1 normalised by its
//               r (known now); p_j -= P[:, <j] s1; partials of ||p_j||^2 and,
//               speculatively, of P[:, <j]^T p_j for a second projection.
//   REORTH(j)   second projection when CGS2, or when ICGS finds
//               ||p_j||^2 < eta^2 ||p_j before||^2 (the DGKS test); partials
//               of ||p_j||^2, of ||p_{j+1}||^2 and of P[:, <=j]^T p_{j+1}
//               (column j not yet normalised: that product is divided by
//               r_jj in PROJECT(j+1)).
// MGS, column i (the paper's sequential MGS):
//   MGS(i)      r_{i-1,i-1} and r_{i-1,c} = u_{i-1}^T u_c / r_{i-1,i-1} from
//               the reduced sums; q_{i-1} = u_{i-1} / r_{i-1,i-1};
//               u_c -= r_{i-1,c} q_{i-1} for c >= i; partials of ||u_i||^2 and
//               of u_i^T u_c for c > i.
// FINISH normalises the last column.  Workgroup 0 writes R.
//
// A thread loads the columns a step touches in its row into registers at
// once (the first row block before the reduction of the previous partial
// sums, so that the two memory latencies overlap), computes the update and
// the step's inner products from them, and stores what changed; one row per
// thread up to 65536 rows.  The wavefront sums of every 16-slot chunk are
// formed first and exchanged through LDS once per row block.  Partial sums:
// slots [0, 64) inner products (whole 16-slot chunks are written), 64-66 the
// squared norms (all three written by every launch).
enum : int { CG_START = 0, CG_PROJECT = 1, CG_REORTH = 2, CG_FINISH = 3, CG_MGS = 4 };
constexpr int kColThreads = 256;
constexpr int kSlotNA = 64, kSlotNB = 65, kSlotNC = 66;

// Row r's columns [lo, hi) into v (zeros elsewhere) and its columns e0 and
// e1 (e1 < 0: none) into x0, x1, addressed as a uniform column base plus the
// row's 32-bit byte offset in the slab that starts at row r0.
__device__ __forceinline__ void colgrid_load_row(double (&v)[kLeaf], double& x0, double& x1, const double* P,
                                                 int64_t r0, int64_t ld, int64_t r, bool act, int lo, int hi, int e0,
                                                 int e1) {
  const char* const slab = reinterpret_cast<const char*>(P + r0);
  const uint32_t off = act ? (uint32_t)(r - r0) * 8u : 0u;
#pragma unroll
  for (int c = 0; c < kLeaf; ++c)
    v[c] = (act && c >= lo && c < hi) ? *reinterpret_cast<const double*>(slab + c * ld * 8 + off) : 0.0;
  x0 = act ? P[r + e0 * ld] : 0.0;
  x1 = act && e1 >= 0 ? P[r + e1 * ld] : 0.0;
}

template <int kind>
__global__ __launch_bounds__(kColThreads) void colgrid_kernel(ColArgs a, int G, int64_t rb, int j, int par) {
  __builtin_amdgcn_s_setprio(2);   // panel chain
  __shared__ double red[kColSlots];
  __shared__ double tmp[kColThreads];
  __shared__ double wsum[kColThreads / 64][kLeaf + kColChunk];   // per-wavefront sums of every slot
  __shared__ double coef[kLeaf + kColChunk];                     // zero beyond the step's coefficients
  const int tid = threadIdx.x, g = blockIdx.x, w = a.w;
  const int64_t ld = a.ldp;
  double* const P = a.P;
  const int64_t r0 = (int64_t)g * rb, r1 = min(a.mrows, r0 + rb);
  const int64_t bufsz = (int64_t)kColGridMax * kColSlots;
  const double* in = a.work + (par ^ 1) * bufsz;
  double* out = a.work + par * bufsz + (int64_t)g * kColSlots;
  double* state = a.work + 2 * bufsz;   // [0] ||p_j||^2 before its first projection, [1] after it, [2] second taken
  const bool lead = g == 0 && tid == 0;

  // inner-product slots this launch reads [rlo, rhi) and writes [wlo, whi);
  // columns a row holds in registers [lo, hi); single columns e0 and e1
  int rlo = 0, rhi = 0, wlo = 0, whi = 0, lo = 0, hi = 0, e0 = 0, e1 = -1;
  if constexpr (kind == CG_PROJECT) {   // e0 = p_j, e1 = column j-1
    rhi = j; whi = j; hi = j; e0 = j; e1 = j - 1;
  }
  if constexpr (kind == CG_REORTH) {    // e0 = p_j, e1 = p_{j+1}
    rhi = j; whi = j + 1 < w ? j + 1 : 0; hi = j; e0 = j; e1 = j + 1 < w ? j + 1 : -1;
  }
  if constexpr (kind == CG_MGS) {       // e0 = u_j, e1 = u_{j-1}
    if (j > 0) { rlo = j; rhi = w; }
    wlo = j + 1; whi = w; lo = j; hi = w; e0 = j; e1 = j - 1;
  }
  if constexpr (kind == CG_FINISH) e0 = w - 1;

  double v[kLeaf], x0 = 0.0, x1 = 0.0;
  // the first row block is loaded before the reduction below, which it does
  // not depend on, so the two memory latencies overlap
  const int nit = (int)((rb + kColThreads - 1) / kColThreads);
  colgrid_load_row(v, x0, x1, P, r0, ld, r0 + tid, r0 + tid < r1, lo, hi, e0, e1);
  // the state words a step uses, read before the reduction below (workgroup 0
  // of the same launch writes only words the step does not read: PROJECT
  // writes [0] and reads [1], [2]; REORTH writes [1], [2] and reads [0])
  double st0 = 0.0, st1 = 0.0, st2 = 0.0;
  if constexpr (kind == CG_REORTH) st0 = state[0];
  if constexpr (kind == CG_PROJECT || kind == CG_FINISH) {
    st1 = state[1];
    st2 = state[2];
  }

  for (int c = tid; c < kLeaf + kColChunk; c += kColThreads) coef[c] = 0.0;
  // reduce the previous launch's partials: its inner products in [rlo, rhi)
  // and the three norms; thread (si, q) sums workgroups q, q + Q, ... in order
  if (!(kind == CG_START || (kind == CG_MGS && j == 0))) {
    const int nd = rhi - rlo, ns = nd + 3, Q = kColThreads / ns;
    const int si = tid % ns, q = tid / ns;
    const int slot = si < nd ? rlo + si : kSlotNA + (si - nd);
    if (q < Q) {
      double acc = 0.0;
      int h = q;
      for (; h + 3 * Q < G; h += 4 * Q) {
        const double y0 = in[(int64_t)h * kColSlots + slot], y1 = in[(int64_t)(h + Q) * kColSlots + slot];
        const double y2 = in[(int64_t)(h + 2 * Q) * kColSlots + slot], y3 = in[(int64_t)(h + 3 * Q) * kColSlots + slot];
        acc += y0;
        acc += y1;
        acc += y2;
        acc += y3;
      }
      for (; h < G; h += Q) acc += in[(int64_t)h * kColSlots + slot];
      tmp[q * ns + si] = acc;
    }
    __syncthreads();
    if (tid < ns) {
      double s = 0.0;
      for (int k = 0; k < Q; ++k) s += tmp[k * ns + tid];
      red[tid < nd ? rlo + tid : kSlotNA + (tid - nd)] = s;
    }
  }
  __syncthreads();
  // r from a squared norm; a zero or non-finite norm flags the panel as
  // exactly rank-deficient and leaves the column unnormalised
  auto diag = [&](double r2) {
    if (!(r2 > 0.0) || !isfinite(r2)) {
      if (lead && a.info[0] == 0) a.info[0] = 1 + a.panel;
      r2 = 1.0;
    }
    return sqrt(r2);
  };

  if constexpr (kind == CG_FINISH) {
    // r of the last column, which is normalised; zeros below R's diagonal
    const double r = diag(a.mode == COLWISE_MGS ? red[kSlotNA] : (st2 != 0.0 ? red[kSlotNC] : st1));
    const double inv = 1.0 / r;
    if (lead) a.Rout[(w - 1) + (int64_t)(w - 1) * a.ldr] = r;
    if (g == 0)
      for (int e = tid; e < w * w; e += kColThreads) {
        const int i = e % w, c = e / w;
        if (i > c) a.Rout[i + (int64_t)c * a.ldr] = 0.0;
      }
    for (int it = 0; it < nit; ++it) {
      const int64_t r = r0 + (int64_t)it * kColThreads + tid;
      if (it > 0) colgrid_load_row(v, x0, x1, P, r0, ld, r, r < r1, lo, hi, e0, e1);
      if (r < r1) P[r + (w - 1) * ld] = x0 * inv;
    }
  } else {
    // this step's coefficients, decision and R entries
    double inv = 1.0;
    bool second = false;
    if constexpr (kind == CG_PROJECT) {
      if (j > 0) {
        const double r = diag(st2 != 0.0 ? red[kSlotNC] : st1);
        inv = 1.0 / r;
        if (lead) a.Rout[(j - 1) + (int64_t)(j - 1) * a.ldr] = r;
      }
      if (tid < j) coef[tid] = tid == j - 1 ? red[tid] * inv : red[tid];
      __syncthreads();
      if (g == 0) {
        if (tid < j) a.Rout[tid + (int64_t)j * a.ldr] = coef[tid];
        if (tid == 0) state[0] = red[kSlotNA];
      }
    } else if constexpr (kind == CG_REORTH) {
      const double n1 = red[kSlotNB];
      second = j > 0 && (a.mode == COLWISE_CGS2 || n1 < a.eta * a.eta * st0);
      if (second && tid < j) coef[tid] = red[tid];
      __syncthreads();
      if (g == 0) {
        if (second && tid < j) a.Rout[tid + (int64_t)j * a.ldr] += coef[tid];
        if (tid == 0) {
          state[1] = n1;
          state[2] = second ? 1.0 : 0.0;
        }
      }
    } else if constexpr (kind == CG_MGS) {
      if (j > 0) {
        const double r = diag(red[kSlotNA]);
        inv = 1.0 / r;
        if (tid >= j && tid < w) coef[tid] = red[tid] * inv;
        if (lead) a.Rout[(j - 1) + (int64_t)(j - 1) * a.ldr] = r;
      }
      __syncthreads();
      if (g == 0 && j > 0 && tid >= j && tid < w) a.Rout[(j - 1) + (int64_t)tid * a.ldr] = coef[tid];
    }

    double total = 0.0;   // threads < kColSlots: this workgroup's sum for slot tid
    for (int it = 0; it < nit; ++it) {
      const int64_t r = r0 + (int64_t)it * kColThreads + tid;
      const bool act = r < r1;
      if (it > 0) colgrid_load_row(v, x0, x1, P, r0, ld, r, act, lo, hi, e0, e1);
      double na = 0.0, nb = 0.0, nc = 0.0;
      if constexpr (kind == CG_START) {
        na = x0 * x0;
      } else if constexpr (kind == CG_PROJECT) {
        // column j-1 normalised; p_j -= P[:, <j] s1; ||p_j||^2; P[:, <j]^T p_j
        double x = x0;
        if (j > 0) {
          const double qp = x1 * inv;
          if (act) P[r + (j - 1) * ld] = qp;
#pragma unroll
          for (int c = 0; c < kLeaf; ++c)
            if (c + 1 == j) v[c] = qp;
        }
#pragma unroll
        for (int c = 0; c < kLeaf; ++c) x -= v[c] * coef[c];
        if (act) P[r + j * ld] = x;
        nb = x * x;
#pragma unroll
        for (int c = 0; c < kLeaf; ++c) v[c] *= x;
      } else if constexpr (kind == CG_REORTH) {
        double x = x0;
        const double y = x1;
        if (second) {
#pragma unroll
          for (int c = 0; c < kLeaf; ++c) x -= v[c] * coef[c];
          if (act) P[r + j * ld] = x;
          nc = x * x;
        }
        // the next column's first projection: P[:, <=j]^T p_{j+1}, ||p_{j+1}||^2
        na = y * y;
#pragma unroll
        for (int c = 0; c < kLeaf; ++c) v[c] = c == j ? x * y : v[c] * y;
      } else {   // CG_MGS
        // q_{j-1} = u_{j-1} / r; u_c -= r_{j-1,c} q_{j-1} for c >= j;
        // ||u_j||^2 and u_j^T u_c for c > j
        double u = x0;
        if (j > 0) {
          const double q = x1 * inv;
          if (act) P[r + (j - 1) * ld] = q;
          u -= coef[j] * q;
          const uint32_t off = act ? (uint32_t)(r - r0) * 8u : 0u;
          char* const wslab = reinterpret_cast<char*>(P + r0);
#pragma unroll
          for (int c = 0; c < kLeaf; ++c) {
            v[c] -= coef[c] * q;
            if (act && c >= j && c < w) *reinterpret_cast<double*>(wslab + c * ld * 8 + off) = v[c];
          }
        }
        na = u * u;
#pragma unroll
        for (int c = 0; c < kLeaf; ++c) v[c] *= u;
      }
      // workgroup sums of this row block (the chunks covering [wlo, whi),
      // then the norms): every wavefront butterfly first, independent of one
      // another, then one exchange through LDS; each slot's total adds the
      // wavefronts in order, then the row blocks in order
      double xs[kLeaf / kColChunk + 1];
#pragma unroll
      for (int k = 0; k < kLeaf / kColChunk; ++k) {
        xs[k] = 0.0;
        if (whi > wlo && (k + 1) * kColChunk > wlo && k * kColChunk < whi) {
          double v16[kColChunk];
#pragma unroll
          for (int c = 0; c < kColChunk; ++c) v16[c] = v[k * kColChunk + c];
          xs[k] = colwise_wave_sum16(v16);
        }
      }
      {
        double n16[kColChunk];
#pragma unroll
        for (int c = 0; c < kColChunk; ++c) n16[c] = 0.0;
        n16[0] = na;
        n16[1] = nb;
        n16[2] = nc;
        xs[kLeaf / kColChunk] = colwise_wave_sum16(n16);
      }
      const int wave = tid >> 6, lane = tid & 63;
      if (lane < kColChunk) {
#pragma unroll
        for (int k = 0; k <= kLeaf / kColChunk; ++k) wsum[wave][k * kColChunk + lane] = xs[k];
      }
      __syncthreads();
      if (tid < kColSlots) {
        double sacc = 0.0;
#pragma unroll
        for (int q = 0; q < kColThreads / 64; ++q) sacc += wsum[q][tid];
        total += sacc;
      }
      __syncthreads();
    }
    const int k = tid / kColChunk;
    const bool chunk = whi > wlo && (k + 1) * kColChunk > wlo && k * kColChunk < whi && tid < kLeaf;
    if (chunk || (tid >= kSlotNA && tid <= kSlotNC)) out[tid] = total;
  }
}

// The launches of one leaf: 2w + 2 for CGS2 / ICGS, w + 1 for MGS.  One row
// per thread while the rows fit kColGridMax workgroups, more beyond.
void launch_colpanel(const ColArgs& a, hipStream_t st) {
  const int G = (int)std::min<int64_t>(kColGridMax, std::max<int64_t>(1, (a.mrows + kColThreads - 1) / kColThreads));
  const int64_t rb = (a.mrows + G - 1) / G;
  int par = 0;
  auto go = [&](auto kern, int j) {
    hipLaunchKernelGGL(kern, dim3(G), dim3(kColThreads), 0, st, a, G, rb, j, par);
    par ^= 1;
  };
  if (a.mode == COLWISE_MGS) {
    for (int i = 0; i < a.w; ++i) go(colgrid_kernel<CG_MGS>, i);
  } else {
    go(colgrid_kernel<CG_START>, 0);
    for (int j = 0; j < a.w; ++j) {
      go(colgrid_kernel<CG_PROJECT>, j);
      go(colgrid_kernel<CG_REORTH>, j);
    }
  }
  go(colgrid_kernel<CG_FINISH>, a.w - 1);
}

CholArgs chol_args(const double* W, int64_t ldw, int w, int pass, double* Rout, int64_t ldr, const double* X,
                   int64_t ldx, double* Rbar, int panel, const Scratch& s) {
  CholArgs c{};
  c.W = W; c.ldw = ldw;
  c.w = w; c.pass = pass; c.panel = panel;
  c.T = s.T; c.R1 = s.R1; c.Rout = Rout; c.ldr = ldr; c.info = s.info;
  c.X = X; c.ldx = ldx; c.Rbar = Rbar;
  c.Tcopy = nullptr;
  c.P = nullptr; c.ldp = 0; c.mrows = 0;
  c.fb = nullptr;
  return c;
}

void launch_chol(const double* W, int64_t ldw, int w, int pass, double* Rout, int64_t ldr, const double* X,
                 int64_t ldx, double* Rbar, int panel, const Scratch& s, hipStream_t st, double* Tcopy, double* P,
                 int64_t ldp, int64_t mrows, int* fb) {
  CholArgs c = chol_args(W, ldw, w, pass, Rout, ldr, X, ldx, Rbar, panel, s);
  c.Tcopy = Tcopy;
  c.P = P; c.ldp = ldp; c.mrows = mrows;
  c.fb = fb;
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(256), 0, st, c);
}

// --------------------------------------------------------------------------
// In-place panel transform P <- P T (T upper triangular, w <= 64 columns).
// Each block stages 64 rows of P in LDS, then 4 waves (16 rows each) form
// the product with MFMA.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void apply_kernel(double* P, int64_t ldp, int64_t mrows, int w,
                                                    const double* T) {
  __builtin_amdgcn_s_setprio(2);   // panel chain
  __shared__ double tileP[kLeaf][64 + 1];   // [col][row]
  __shared__ double tileT[kLeaf][kLeaf + 1];   // [k][j]
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  {
    // every load of the block in flight at once: 16 of P and 16 of T per thread
    const int64_t row = r0 + tx;
    const bool rok = row < mrows;
    double vp[16], vt[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = ty + 4 * q;
      vp[q] = (rok && c < w) ? P[row + (int64_t)c * ldp] : 0.0;
      vt[q] = (tx < w && c < w) ? T[tx + c * w] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = ty + 4 * q;
      tileP[c][tx] = vp[q];
      tileT[tx][c] = vt[q];
    }
  }
  __syncthreads();
  const int wave = ty, lane = tx, li = lane & 15, g = lane >> 4;
  const int rl = wave * 16 + li;
  v4d acc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) acc[y] = v4d{0, 0, 0, 0};
#pragma unroll 4
  for (int k0 = 0; k0 < kLeaf; k0 += 16) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      const double xa = tileP[k][rl];
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[y] = mfma(tileT[k][16 * y + li], xa, acc[y]);
    }
  }
  const int64_t row = r0 + rl;
  if (row >= mrows) return;
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * y + 4 * r + g;
      if (j < w) P[row + (int64_t)j * ldp] = acc[y][r];
    }
}

void launch_apply(double* P, int64_t ldp, int64_t mrows, int w, const Scratch& s, hipStream_t st) {
  const int blocks = (int)((mrows + 63) / 64);
  hipLaunchKernelGGL(apply_kernel, dim3(blocks), dim3(256), 0, st, P, ldp, mrows, w, (const double*)s.T);
}

// --------------------------------------------------------------------------
// Rank-K update  C -= A B  (A: M x K, B: K x N, C: M x N, column-major).
// Tile 64 x 64 per block; wave w takes rows 16w..16w+15 and all 64 columns
// (4 accumulator blocks).  K advances in slabs of 64: the B slab (64 x 64) is
// staged in LDS and shared by the four waves, each lane keeps its 16 A values
// of a slab in registers, and the next slab's A and B loads are in flight
// while the current slab is multiplied (two A register sets alternate
// explicitly).  Short K (the trailing update, K = b): C is loaded at the start
// so all of a tile's loads are in flight together.  Long K with few tiles
// (re-projection): the K range is split over blocks and nn_reduce_kernel
// subtracts the partial tiles from C in split order.
// --------------------------------------------------------------------------

constexpr int NK = 64;   // k per slab of the rank-K update
// Fewest columns for which the update takes the 128 x 128 kernel.
constexpr int kQuadMinN = 256;

// Shared pieces of the rank-K update kernels.  B staging: thread t moves
// B[k0 + 16(t & 3) + e][jb + (t >> 2)], e < 16 (8 vector loads from one
// column); columns past N read column 0 and feed only unstored outputs.
struct NnTile {
  int tm, tn, wave, lane, li, g, tid;
  int64_t i, ic;
  int jb;
  bool aok;
  const double* ar;   // A[ic][g]: lane (li, g) supplies A[i][k0 + 4m + g] to product m
  const double* bp;   // B[16(t & 3)][jb + (t >> 2)]
};

__device__ __forceinline__ NnTile nn_tile_at(const NnArgs& a, int tm, int tn) {
  NnTile t;
  t.tm = tm;
  t.tn = tn;
  t.tid = threadIdx.x;
  t.wave = t.tid >> 6;
  t.lane = t.tid & 63;
  t.li = t.lane & 15;
  t.g = t.lane >> 4;
  t.i = (int64_t)t.tm * 64 + t.wave * 16 + t.li;
  t.jb = t.tn * 64;
  t.aok = t.i < a.M;
  t.ic = t.aok ? t.i : 0;            // clamped row: valid address, result unused
  t.ar = a.A + t.ic + (int64_t)t.g * a.lda;
  const int jc = t.jb + (t.tid >> 2);
  t.bp = a.B + 16 * (t.tid & 3) + (int64_t)(jc < a.N ? jc : 0) * a.ldb;
  return t;
}

__device__ __forceinline__ NnTile nn_tile(const NnArgs& a, int tile) {
  return nn_tile_at(a, tile / a.tilesN, tile % a.tilesN);
}

// XCD-aware tile order for one-pass updates.  Workgroups are dealt to the
// eight XCDs round-robin (block b runs on XCD b mod 8), and each XCD has its
// own L2.  Block b takes position start(x) + b / 8 of an order in which the
// tiles come in four bands of row tiles, each band walked column slab by
// column slab; XCD x's positions form one contiguous range of that order,
// i.e. about half of one band.  Each XCD thus reads a quarter of the A rows
// and half of the B columns instead of all of both.
__device__ __forceinline__ void xcd_tile(int b, int ntiles, int tilesM, int tilesN, int& tm, int& tn) {
  const int x = b & 7, j = b >> 3;
  const int q = ntiles >> 3, r = ntiles & 7;
  const int pos = x * q + (x < r ? x : r) + j;
  const int bm = (tilesM + 3) >> 2;                 // row tiles per band
  const int band = pos / (bm * tilesN);
  const int rows = min(bm, tilesM - band * bm);     // rows in this band (the last may be short)
  const int in = pos - band * bm * tilesN;
  tn = in / rows;
  tm = band * bm + in % rows;
}

__device__ __forceinline__ void nn_load_a(const NnArgs& a, const NnTile& t, int k0, double (&xa)[16]) {
#pragma unroll
  for (int m = 0; m < 16; ++m) xa[m] = t.ar[(int64_t)(k0 + 4 * m) * a.lda];
}

__device__ __forceinline__ void nn_load_b(const NnTile& t, int k0, v2d (&rb)[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) rb[e] = *reinterpret_cast<const v2d*>(t.bp + k0 + 2 * e);
}

__device__ __forceinline__ void nn_put_b(double (*sBb)[64 + 1], const NnTile& t, const v2d (&rb)[8]) {
  const int kq = 16 * (t.tid & 3), j = t.tid >> 2;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    sBb[kq + 2 * e][j] = rb[e].x;
    sBb[kq + 2 * e + 1][j] = rb[e].y;
  }
}

// Partial slab [k0, ke): zero beyond ke on both operands (scalar loads).
__device__ __forceinline__ void nn_load_tail(const NnArgs& a, const NnTile& t, int k0, int ke, double (&xa)[16],
                                             double (*sBb)[64 + 1]) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int k = k0 + 4 * m + t.g;
    xa[m] = (k < ke) ? t.ar[(int64_t)(k0 + 4 * m) * a.lda] : 0.0;
  }
  const int kq = 16 * (t.tid & 3), j = t.tid >> 2;
#pragma unroll
  for (int e = 0; e < 16; ++e) sBb[kq + e][j] = (k0 + kq + e < ke) ? t.bp[k0 + e] : 0.0;
}

template <class Acc>
__device__ __forceinline__ void nn_mma(Acc (&acc)[4], const double (*sBb)[64 + 1], const NnTile& t,
                                       const double (&xa)[16]) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int k = 4 * m + t.g;
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[y] = mfma(sBb[k][16 * y + t.li], xa[m], acc[y]);
  }
}

// C -= A B for K <= 64 (K < 64, or operands nnw_kernel does not take):
// every load of the tile (C, A, the B slab) is issued before the first
// product.  The tile loop is
// grid-strided; launched with one block per tile it runs once.  This form
// compiles to more registers than the straight-line one (three waves per SIMD
// instead of four), and measured faster in the factorization: the update's
// blocks leave more room for the panel chain's kernels that run beside them.
template <int TAG>
__global__ __launch_bounds__(256) void nn1_kernel(NnArgs a) {
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  typedef v4d Acc;
  __shared__ double sB[NK][64 + 1];
  for (int blk = blockIdx.x; blk < a.ntiles; blk += gridDim.x) {
    int tm, tn;
    xcd_tile(blk, a.ntiles, a.ntiles / a.tilesN, a.tilesN, tm, tn);
    const NnTile t = nn_tile_at(a, tm, tn);
    double cval[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int j = t.jb + 16 * (e >> 2) + colsub(e & 3, t.g, false);
      cval[e] = a.C[t.ic + (int64_t)(j < a.N ? j : 0) * a.ldc];
    }
    double xa[16];
    if (blk != (int)blockIdx.x) __syncthreads();   // the previous tile's reads of sB are done
    if (a.K == NK && a.vec) {
      v2d rb[8];
      nn_load_a(a, t, 0, xa);
      nn_load_b(t, 0, rb);
      __builtin_amdgcn_sched_barrier(0);
      nn_put_b(sB, t, rb);
    } else {
      nn_load_tail(a, t, 0, a.K, xa, sB);
    }
    __syncthreads();
    Acc acc[4];
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[y] = Acc{0, 0, 0, 0};
    nn_mma(acc, sB, t, xa);
    if (t.aok) {
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = t.jb + 16 * y + colsub(r, t.g, false);
          if (j < a.N) a.C[t.i + (int64_t)j * a.ldc] = cval[y * 4 + r] - acc[y][r];
        }
    }
  }
}

// The second pass's panel transform and the lookahead update in one launch:
// P <- P1 T (T: w x w upper triangular, w = K <= 64), then C -= P B.  Each
// block owns 64 rows of P and of C.  A lane's accumulators of the first
// product hold P[i][4m + g] for m = 4y + r, which is exactly the operand the
// lane supplies to the second product, so the transformed strip never leaves
// the registers; it is also stored to P (the panel's final columns).
__global__ __launch_bounds__(256) void nn1_apply_kernel(NnArgs a, const double* T, int w) {
  __builtin_amdgcn_s_setprio(2);   // panel chain
  __shared__ double sT[NK][64 + 1];
  __shared__ double sB[NK][64 + 1];
  const NnTile t = nn_tile(a, blockIdx.x);
  double cval[16], xa[16], tv[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int j = t.jb + 16 * (e >> 2) + colsub(e & 3, t.g, false);
    cval[e] = a.C[t.ic + (int64_t)(j < a.N ? j : 0) * a.ldc];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t.tid + 256 * q, k = e & 63, j = e >> 6;
    tv[q] = (k < w && j < w) ? T[k + j * w] : 0.0;
  }
  // A = P1 (zero past K) in registers, the B slab into LDS
  if (a.K == NK && a.vec) {
    v2d rb[8];
    nn_load_a(a, t, 0, xa);
    nn_load_b(t, 0, rb);
    __builtin_amdgcn_sched_barrier(0);
    nn_put_b(sB, t, rb);
  } else {
    nn_load_tail(a, t, 0, a.K, xa, sB);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = t.tid + 256 * q;
    sT[e & 63][e >> 6] = tv[q];
  }
  __syncthreads();
  v4d pf[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) pf[y] = v4d{0, 0, 0, 0};
  nn_mma(pf, sT, t, xa);
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) xa[4 * y + r] = pf[y][r];
  v4d acc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) acc[y] = v4d{0, 0, 0, 0};
  nn_mma(acc, sB, t, xa);
  if (!t.aok) return;
  double* P = const_cast<double*>(a.A);
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * y + 4 * r + t.g;
      if (j < w) P[t.i + (int64_t)j * a.lda] = pf[y][r];
      if (j < a.N) a.C[t.i + (int64_t)j * a.ldc] = cval[y * 4 + r] - acc[y][r];
    }
}

bool launch_nn1_apply(const NnArgs& a, const double* T, int w, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0 || a.K != w || w > NK || a.tilesN != 1) return false;
  hipLaunchKernelGGL(nn1_apply_kernel, dim3(a.ntiles), dim3(256), 0, st, a, T, w);
  return true;
}

// Long K: slabs of 64 with the next slab's A and B loads in flight while the
// current slab is multiplied (A register sets alternate explicitly).  SPLIT:
// the block's K range is one split and its partial tile is stored for
// nn_reduce_kernel; otherwise C is updated in place (the path for operands
// nnw_kernel does not take).
template <bool SPLIT, int TAG>
__device__ __forceinline__ void nn_body(const NnArgs& a, double (*sB)[NK][64 + 1], int bx, int split) {
  typedef v4d Acc;
  int tm = bx / a.tilesN, tn = bx % a.tilesN;
  if (!SPLIT) xcd_tile(bx, a.ntiles, a.ntiles / a.tilesN, a.tilesN, tm, tn);
  const NnTile t = nn_tile_at(a, tm, tn);
  const int kb = split * a.kchunk;
  const int ke = std::min(a.K, kb + a.kchunk);
  const int nfull = a.vec ? (ke - kb) / NK : 0;
  // in-place update: C's loads go out before the products, so their latency
  // overlaps the K loop instead of following it
  double cval[16];
  if (!SPLIT) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int j = t.jb + 16 * (e >> 2) + colsub(e & 3, t.g, false);
      cval[e] = a.C[t.ic + (int64_t)(j < a.N ? j : 0) * a.ldc];
    }
  }
  Acc acc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) acc[y] = Acc{0, 0, 0, 0};
  auto koff = [&](int sl) { return kb + std::min(sl, nfull - 1) * NK; };
  if (nfull > 0) {
    double xa0[16], xa1[16];
    v2d rb[8];
    nn_load_a(a, t, koff(0), xa0);
    nn_load_b(t, koff(0), rb);
    __builtin_amdgcn_sched_barrier(0);
    nn_put_b(sB[0], t, rb);
    __syncthreads();
    int sl = 0;
    for (; sl + 2 <= nfull; sl += 2) {
      nn_load_a(a, t, koff(sl + 1), xa1);
      nn_load_b(t, koff(sl + 1), rb);
      __builtin_amdgcn_sched_barrier(0);
      nn_mma(acc, sB[0], t, xa0);
      __builtin_amdgcn_sched_barrier(0);
      nn_put_b(sB[1], t, rb);
      __syncthreads();
      nn_load_a(a, t, koff(sl + 2), xa0);
      nn_load_b(t, koff(sl + 2), rb);
      __builtin_amdgcn_sched_barrier(0);
      nn_mma(acc, sB[1], t, xa1);
      __builtin_amdgcn_sched_barrier(0);
      nn_put_b(sB[0], t, rb);
      __syncthreads();
    }
    if (sl < nfull) nn_mma(acc, sB[0], t, xa0);
  }
  const int kt = kb + nfull * NK;
  for (int k0 = kt; k0 < ke; k0 += NK) {
    // partial (or unaligned) slabs; the buffer not read by the last full slab
    const int buf = ((k0 - kb) / NK) & 1;
    double xa[16];
    nn_load_tail(a, t, k0, ke, xa, sB[buf]);
    __syncthreads();
    nn_mma(acc, sB[buf], t, xa);
    __syncthreads();
  }
  if (SPLIT) {
    double* mine = a.part + part_off(split, a.ntiles, bx, t.wave);
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) mine[(y * 4 + r) * 64 + t.lane] = acc[y][r];
    return;
  }
  if (!t.aok) return;
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = t.jb + 16 * y + colsub(r, t.g, false);
      if (j < a.N) a.C[t.i + (int64_t)j * a.ldc] = cval[y * 4 + r] - acc[y][r];
    }
}

template <bool SPLIT, int TAG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void nn_kernel(NnArgs a) {
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  __shared__ double sB[2][NK][64 + 1];
  nn_body<SPLIT, TAG>(a, sB, blockIdx.x, blockIdx.y);
}

// The re-projection update P -= Q S, split over K, with one extra block that
// runs the panel's first Cholesky-QR pass: the factorization reads only the
// Gram rows of the preceding product and the update only its coefficient
// rows, so the single-block Cholesky runs alongside the update's blocks
// instead of after them on the panel chain.  Block column x = ntiles holds the
// Cholesky (its y > 0 blocks exit at once); both uses share the LDS layout
// size (two 64 x 65 double arrays).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void nn_chol_kernel(NnArgs a,
                                                                                               CholArgs c) {
  __builtin_amdgcn_s_setprio(2);
  __shared__ double smem[2 * NK * (64 + 1)];
  __shared__ double prow[16];
  __shared__ double dg[kLeaf];
  __shared__ int flags[3];
  if ((int)blockIdx.x == a.ntiles) {
    if (blockIdx.y == 0)
      chol_body<true>(c, reinterpret_cast<double (*)[kLeaf + 1]>(smem),
                      reinterpret_cast<double (*)[kLeaf + 1]>(smem + kLeaf * (kLeaf + 1)), prow, dg, flags,
                      nullptr);
    return;
  }
  nn_body<true, TAG_REPROJ>(a, reinterpret_cast<double (*)[NK][64 + 1]>(smem), blockIdx.x, blockIdx.y);
}

// C -= sum of the split partials (split order).  One block per wave of a
// tile, thread (qg, lane) owns the lane's 4 values of column block qg.
__global__ __launch_bounds__(256) void nn_reduce_kernel(NnArgs a) {
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  const int tile = blockIdx.x >> 2, wave = blockIdx.x & 3;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int qg = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int64_t i = (int64_t)tm * 64 + wave * 16 + li;
  const int jq = tn * 64 + 16 * qg;            // + colsub(u, g)
  const bool aok = i < a.M;
  const int64_t ic = aok ? i : 0;
  double old[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = jq + colsub(u, g, false);
    old[u] = a.C[ic + (int64_t)(j < a.N ? j : 0) * a.ldc];
  }
  double v[4];
  sum_partials4(a.part, a.nsplit, a.ntiles, tile, wave, qg, lane, v);
  if (!aok) return;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = jq + colsub(u, g, false);
    if (j < a.N) a.C[i + (int64_t)j * a.ldc] = old[u] - v[u];
  }
}

// The split reduction of a panel update (N = w <= 64 columns) followed by
// the panel transform P <- P T (T: w x w, upper triangular): each block's 16 x
// 64 strip of C - sum(partials) is staged in LDS and multiplied by T on MFMA
// (wave q forms output columns 16q .. 16q + 15) before it is stored, so the
// transform needs no launch or pass over P of its own.
__global__ __launch_bounds__(256) void nn_reduce_apply_kernel(NnArgs a, const double* T, int w, double* X,
                                                              int64_t ldx) {
  __builtin_amdgcn_s_setprio(2);   // panel chain
  __shared__ double sP[16][64 + 1];
  __shared__ double sT[64][64 + 1];
  const int tile = blockIdx.x >> 2, wave = blockIdx.x & 3;
  const int qg = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int64_t i = (int64_t)tile * 64 + wave * 16 + li;
  const bool aok = i < a.M;
  const int64_t ic = aok ? i : 0;
  double old[4], tv[16];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = 16 * qg + colsub(u, g, false);
    old[u] = a.C[ic + (int64_t)(j < a.N ? j : 0) * a.ldc];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q, k = e & 63, j = e >> 6;
    tv[q] = (k < w && j < w) ? T[k + j * w] : 0.0;
  }
  double v[4];
  sum_partials4(a.part, a.nsplit, a.ntiles, tile, wave, qg, lane, v);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = 16 * qg + colsub(u, g, false);
    sP[li][j] = j < w ? old[u] - v[u] : 0.0;   // columns past w hold clamped loads
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q;
    sT[e & 63][e >> 6] = tv[q];
  }
  __syncthreads();
  v4d acc = v4d{0, 0, 0, 0};
#pragma unroll
  for (int k0 = 0; k0 < 64; k0 += 16)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      acc = mfma(sT[k][16 * qg + li], sP[li][k], acc);
    }
  if (!aok) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j = 16 * qg + 4 * r + g;
    if (j < w) {
      a.C[i + (int64_t)j * a.ldc] = acc[r];
      if (X) X[i + (int64_t)j * ldx] = acc[r];
    }
  }
}

bool launch_nn_reduce_apply(const NnArgs& a, const double* T, int w, double* X, int64_t ldx, hipStream_t st) {
  if (a.M <= 0 || a.nsplit <= 1 || a.tilesN != 1 || a.N != w || w > kLeaf) return false;
  hipLaunchKernelGGL(nn_reduce_apply_kernel, dim3(a.ntiles * 4), dim3(256), 0, st, a, T, w, X, ldx);
  return true;
}

NnArgs nn_setup(double* C, int64_t ldc, const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M,
                int N, int K, const Scratch& s) {
  NnArgs a{};
  a.C = C; a.ldc = ldc; a.A = A; a.lda = lda; a.B = B; a.ldb = ldb;
  a.M = M; a.N = N; a.K = K;
  a.tilesN = (N + 63) / 64;
  a.ntiles = (int)((M + 63) / 64) * a.tilesN;
  a.part = s.part;
  a.vec = aligned16(B, ldb);
  // few tiles and a long reduction: split K so at most 512 blocks (two per
  // CU, one wave of blocks) run, each over at least 2 slabs
  int ns = 1;
  if (K > NK && a.ntiles < 512 && K >= 4 * NK) {
    ns = (int)std::min<int64_t>(std::max(1, 512 / a.ntiles), K / (2 * NK));
    while (ns > 1 && (int64_t)ns * a.ntiles > s.npart) --ns;
  }
  int kchunk = (K + ns - 1) / ns;
  kchunk = (kchunk + NK - 1) / NK * NK;
  ns = (K + kchunk - 1) / kchunk;
  a.kchunk = kchunk;
  a.nsplit = ns;
  return a;
}

// In-place rank-K update C (M x N) -= A (M x K) B (K x N) for K >= 64 (the
// trailing update, long unsplit re-projections), with
// the product kernel's pipeline: 64 x 64 output tile per block, 4 waves each
// a 32 x 32 quadrant, both operands staged through LDS in slabs of KC
// k-values (slab s multiplied while slab s+1 lands in one register set and
// slab s+2 is requested into the other).  A (i contiguous) is transposed into
// the product kernel's [i][k] LDS layout as it is staged; B (k contiguous)
// is staged as there.  C's loads are issued before the K loop.  Requires K a
// multiple of KC, 16-byte aligned A and B with even leading dimensions, and
// an even M; tiles take the XCD-aware order.
// The body for slabs of SK k-values (32 or 16; LDS row pitch SK + 2).
template <int TAG, int SK>
__device__ __forceinline__ void nnw_body(const NnArgs& a, double (*sA)[64 * (SK + 2)], double (*sB)[64 * (SK + 2)]) {
  typedef v4d Acc;
  constexpr int LW = SK + 2;         // padded LDS row (doubles)
  constexpr int NQ = SK / 8;         // v2d loads per thread and operand per slab
  constexpr int TPC = SK / 2;        // B staging: threads per column (one k pair each)
  constexpr int CPP = 256 / TPC;     // B staging: columns per pass
  int tm, tn;
  xcd_tile(blockIdx.x, a.ntiles, a.ntiles / a.tilesN, a.tilesN, tm, tn);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int ia0 = (wave & 1) * 32, jb0 = (wave >> 1) * 32;
  const int64_t ib = (int64_t)tm * 64, jb = (int64_t)tn * 64;
  // C's 16 values of this lane (quadrant element (x, y, r)); rows and
  // columns outside C read row or column 0 and are not stored
  double cval[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int x = e >> 3, y = (e >> 2) & 1, r = e & 3;
    const int64_t i = ib + ia0 + 16 * x + li, j = jb + jb0 + 16 * y + colsub(r, g, false);
    cval[e] = a.C[(i < a.M ? i : 0) + (j < a.N ? j : 0) * a.ldc];
  }
  // staging of A: thread loads one v2d (rows 2 ip, 2 ip + 1) of k rows kr + 8 q
  const int ip = tid & 31, kr = tid >> 5;
  const int64_t ia = ib + 2 * ip;
  const double* ga = a.A + (ia + 1 < a.M ? ia : 0) + (int64_t)kr * a.lda;
  // staging of B: thread loads one v2d (k pair lq) of columns lc + CPP q
  const int lc = tid / TPC, lq = tid % TPC;
  const double* gb[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int64_t j = jb + lc + CPP * q;
    gb[q] = a.B + (j < a.N ? j : 0) * a.ldb + 2 * lq;
  }
  Acc acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = Acc{0, 0, 0, 0};
  const int nsl = a.K / SK;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < SK; kk += 16) {
      double xa[2][4], xb[2][4];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double* pa = &sA[buf][(ia0 + 16 * t + li) * LW + kk + 4 * g];
        const double* pb = &sB[buf][(jb0 + 16 * t + li) * LW + kk + 4 * g];
        v2d a0 = *reinterpret_cast<const v2d*>(pa), a1 = *reinterpret_cast<const v2d*>(pa + 2);
        v2d b0 = *reinterpret_cast<const v2d*>(pb), b1 = *reinterpret_cast<const v2d*>(pb + 2);
        xa[t][0] = a0.x; xa[t][1] = a0.y; xa[t][2] = a1.x; xa[t][3] = a1.y;
        xb[t][0] = b0.x; xb[t][1] = b0.y; xb[t][2] = b1.x; xb[t][3] = b1.y;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma(xb[y][s], xa[x][s], acc[x][y]);
    }
  };
  // slab sl's first k (clamped to the last slab: prefetches past the end
  // reload cached data that is never used)
  auto koff = [&](int sl) { return (int64_t)std::min(sl, nsl - 1) * SK; };
  v2d ra0[NQ], rb0[NQ], ra1[NQ], rb1[NQ];
  auto load = [&](v2d (&ra)[NQ], v2d (&rb)[NQ], int64_t k) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      ra[q] = *reinterpret_cast<const v2d*>(ga + (k + 8 * q) * a.lda);
      rb[q] = *reinterpret_cast<const v2d*>(gb[q] + k);
    }
  };
  auto put = [&](int buf, const v2d (&ra)[NQ], const v2d (&rb)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      sA[buf][(2 * ip) * LW + kr + 8 * q] = ra[q].x;
      sA[buf][(2 * ip + 1) * LW + kr + 8 * q] = ra[q].y;
      *reinterpret_cast<v2d*>(&sB[buf][(lc + CPP * q) * LW + 2 * lq]) = rb[q];
    }
  };
  load(ra0, rb0, koff(0));
  load(ra1, rb1, koff(1));
  put(0, ra0, rb0);
  __syncthreads();
  int sl = 0;
  for (; sl + 2 <= nsl; sl += 2) {
    load(ra0, rb0, koff(sl + 2));
    __builtin_amdgcn_sched_barrier(0);
    compute(0);
    __builtin_amdgcn_sched_barrier(0);
    put(1, ra1, rb1);
    __syncthreads();
    load(ra1, rb1, koff(sl + 3));
    __builtin_amdgcn_sched_barrier(0);
    compute(1);
    __builtin_amdgcn_sched_barrier(0);
    put(0, ra0, rb0);
    __syncthreads();
  }
  if (sl < nsl) compute(0);
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int x = e >> 3, y = (e >> 2) & 1, r = e & 3;
    const int64_t i = ib + ia0 + 16 * x + li, j = jb + jb0 + 16 * y + colsub(r, g, false);
    if (i < a.M && j < a.N) a.C[i + j * a.ldc] = cval[e] - acc[x][y][r];
  }
}

// 32-deep slabs, two waves per SIMD: the rank-64 trailing update, which runs
// beside the panel chain (with 16-deep slabs and three waves per SIMD it is
// faster alone but the step at n = 4096 was 3.8% slower).
template <int TAG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void nnw_kernel(NnArgs a) {
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  __shared__ double sA[2][64 * (32 + 2)];
  __shared__ double sB[2][64 * (32 + 2)];
  nnw_body<TAG, 32>(a, sA, sB);
}

// 16-deep slabs (37 KB of LDS, 148-164 VGPRs), three waves per SIMD: K >= 128,
// where the update is MFMA-bound in FP64.  Against the 32-deep form, 9% faster
// alone at K = 128 and 8% at K = 256, and 4% off the n = 16384 step.
template <int TAG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void nnw16_kernel(NnArgs a) {
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  __shared__ double sA[2][64 * (16 + 2)];
  __shared__ double sB[2][64 * (16 + 2)];
  nnw_body<TAG, 16>(a, sA, sB);
}

// 128 x 128 output tile per workgroup (512 threads, 2 x 4 waves, each wave
// 64 rows x 32 columns), 16-deep slabs double-buffered in LDS (72 KB) with
// one register set of staged loads, two workgroups per CU: K >= 128.  Each
// staged column of A and row of B feeds 128 outputs instead of 64, which
// halves the L2 requests per flop against nnw16_kernel.  Alone, the
// K = 256 update of a 49152 x 32768 C runs at 58.7 TFLOP/s against 51.3
// (K = 128, 32768 x 20480: 48.1 against 41.1).  A (i contiguous) is
// transposed into the [i][k] LDS layout as it is staged; C is read after
// the K loop, one 16-row block at a time, and written back in place.
// Requires K a multiple of 16, 16-byte aligned A and B with even leading
// dimensions, and an even M; tiles take the XCD-aware order.
template <int TAG>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4))) void nnq_kernel(NnArgs a) {
  constexpr int SK = 16, LW = SK + 2;
  constexpr int AKR = 8;               // A staging: k rows per pass (64 row pairs x 8)
  constexpr int TPC = SK / 2, CPP = 512 / TPC;   // B staging: 8 threads per column, 64 columns a pass
  if (a.prio) __builtin_amdgcn_s_setprio(2);
  __shared__ double sA[2][128 * LW];
  __shared__ double sB[2][128 * LW];
  const int tilesM = (int)((a.M + 127) / 128), tilesN = (a.N + 127) / 128;
  int tm, tn;
  xcd_tile(blockIdx.x, tilesM * tilesN, tilesM, tilesN, tm, tn);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int ia0 = 64 * (wave & 1), jb0 = 32 * (wave >> 1);
  const int64_t ib = (int64_t)tm * 128, jb = (int64_t)tn * 128;
  const int ip = tid & 63, kr = tid >> 6;
  const int64_t ia = ib + 2 * ip;
  const double* ga = a.A + (ia + 1 < a.M ? ia : 0) + (int64_t)kr * a.lda;
  const int lc = tid / TPC, lq = tid % TPC;
  const double* gb[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int64_t j = jb + lc + CPP * q;
    gb[q] = a.B + (j < a.N ? j : 0) * a.ldb + 2 * lq;
  }
  v4d acc[4][2];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0, 0, 0, 0};
  auto compute = [&](int buf) {
#pragma unroll
    for (int s0 = 0; s0 < 4; s0 += 2) {
      double xa[4][2], xb[2][2];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const v2d v = *reinterpret_cast<const v2d*>(&sA[buf][(ia0 + 16 * t + li) * LW + 4 * g + s0]);
        xa[t][0] = v.x; xa[t][1] = v.y;
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const v2d v = *reinterpret_cast<const v2d*>(&sB[buf][(jb0 + 16 * t + li) * LW + 4 * g + s0]);
        xb[t][0] = v.x; xb[t][1] = v.y;
      }
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma(xb[y][s], xa[x][s], acc[x][y]);
    }
  };
  const int nsl = a.K / SK;
  v2d ra[2], rb[2];
  auto load = [&](int64_t k) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ra[q] = *reinterpret_cast<const v2d*>(ga + (k + AKR * q) * a.lda);
      rb[q] = *reinterpret_cast<const v2d*>(gb[q] + k);
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      sA[buf][(2 * ip) * LW + kr + AKR * q] = ra[q].x;
      sA[buf][(2 * ip + 1) * LW + kr + AKR * q] = ra[q].y;
      *reinterpret_cast<v2d*>(&sB[buf][(lc + CPP * q) * LW + 2 * lq]) = rb[q];
    }
  };
  load(0);
  put(0);
  __syncthreads();
  for (int sl = 0; sl < nsl; ++sl) {
    if (sl + 1 < nsl) load((int64_t)(sl + 1) * SK);
    __builtin_amdgcn_sched_barrier(0);
    compute(sl & 1);
    __builtin_amdgcn_sched_barrier(0);
    if (sl + 1 < nsl) put((sl + 1) & 1);
    __syncthreads();
  }
  // C -= acc, one 16-row block of the wave's 64 rows at a time; rows and
  // columns outside C read row or column 0 and are not stored
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int64_t i = ib + ia0 + 16 * x + li;
    double cv[2][4];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = jb + jb0 + 16 * y + colsub(r, g, false);
        cv[y][r] = a.C[(i < a.M ? i : 0) + (j < a.N ? j : 0) * a.ldc];
      }
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = jb + jb0 + 16 * y + colsub(r, g, false);
        if (i < a.M && j < a.N) a.C[i + j * a.ldc] = cv[y][r] - acc[x][y][r];
      }
  }
}

// Operands the LDS-staged update takes, K >= 64 (else the register-staged
// kernels): 18-22% faster standalone than the register-staged long-K kernel
// at K = 128 and 256.  At K = 64 it is ~8% slower alone than nn1_kernel but
// 1% faster in the factorization, beside the panel chain's kernels.
static bool nnw_ok(const NnArgs& a) {
  return a.K >= NK && a.K % KC == 0 && a.M % 2 == 0 && aligned16(a.A, a.lda) && aligned16(a.B, a.ldb);
}

// The 128 x 128 update: K >= 128 and at least two 128-wide tiles each way
// (see kQuadMinN for the column count).
static bool nnq_ok(const NnArgs& a) {
  return nnw_ok(a) && a.K >= 2 * NK && a.M >= 256 && a.N >= kQuadMinN;
}

template <int TAG>
static void nn_launch_tag(const NnArgs& a, hipStream_t st) {
  if (a.K <= NK && !nnw_ok(a))
    hipLaunchKernelGGL((nn1_kernel<TAG>), dim3(a.ntiles), dim3(256), 0, st, a);
  else if (a.nsplit > 1)
    hipLaunchKernelGGL((nn_kernel<true, TAG>), dim3(a.ntiles, a.nsplit), dim3(256), 0, st, a);
  else if (nnq_ok(a))
    hipLaunchKernelGGL((nnq_kernel<TAG>), dim3((unsigned)(((a.M + 127) / 128) * ((a.N + 127) / 128))), dim3(512), 0,
                       st, a);
  else if (nnw_ok(a) && a.K >= 2 * NK)
    hipLaunchKernelGGL((nnw16_kernel<TAG>), dim3(a.ntiles), dim3(256), 0, st, a);
  else if (nnw_ok(a))
    hipLaunchKernelGGL((nnw_kernel<TAG>), dim3(a.ntiles), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((nn_kernel<false, TAG>), dim3(a.ntiles, 1), dim3(256), 0, st, a);
}

void launch_nn_product(const NnArgs& a, int tag, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0 || a.K <= 0) return;
  switch (tag) {
    case TAG_TRAIL: nn_launch_tag<TAG_TRAIL>(a, st); break;
    case TAG_REPROJ: nn_launch_tag<TAG_REPROJ>(a, st); break;
    default: nn_launch_tag<TAG_PANEL>(a, st); break;
  }
}

bool launch_nn_chol(const NnArgs& a, const CholArgs& c, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0 || a.K <= NK || a.nsplit <= 1 || c.w > kLeaf) return false;
  hipLaunchKernelGGL(nn_chol_kernel, dim3(a.ntiles + 1, a.nsplit), dim3(256), 0, st, a, c);
  return true;
}

void launch_nn_reduce(const NnArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0 || a.K <= NK || a.nsplit <= 1) return;
  hipLaunchKernelGGL(nn_reduce_kernel, dim3(a.ntiles * 4), dim3(256), 0, st, a);
}

}  // namespace cqr
