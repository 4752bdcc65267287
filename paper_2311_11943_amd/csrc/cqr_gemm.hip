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
#include "cqr_kernels.hpp"

#include <algorithm>
#include <cmath>

namespace cqr {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double x, double y, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

// Partial-tile layout shared by the product and reduction kernels: tile
// `tile` of split `sp`, wave w, accumulator element q (16 per lane), lane l at
// part[((sp * ntiles + tile) * 4 + w) * 1024 + q * 64 + l].
__device__ __forceinline__ int64_t part_off(int sp, int ntiles, int tile, int wave) {
  return (((int64_t)sp * ntiles + tile) * 4 + wave) * 1024;
}

// Sum the 16 per-lane values of `nsplit` partial tiles in split order.  The
// loads of four splits are issued before they are added, so the single pass
// is bandwidth- rather than latency-bound; the addition order stays 0, 1, 2...
__device__ __forceinline__ void sum_partials(const double* part, int nsplit, int ntiles, int tile, int wave,
                                             int lane, double (&v)[16]) {
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = 0.0;
  int sp = 0;
  for (; sp + 4 <= nsplit; sp += 4) {
    double t[4][16];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double* p = part + part_off(sp + u, ntiles, tile, wave);
#pragma unroll
      for (int q = 0; q < 16; ++q) t[u][q] = p[q * 64 + lane];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] += t[u][q];
  }
  for (; sp < nsplit; ++sp) {
    const double* p = part + part_off(sp, ntiles, tile, wave);
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] += p[q * 64 + lane];
  }
}

// --------------------------------------------------------------------------
// Split-K product  C = A^T B  (A: K x M, B: K x N, both K-contiguous).
// Tile 64x64 per block, 4 waves each a 32x32 quadrant.  Operand slabs of
// KC = 32 k-values are staged through LDS (double-buffered): each global load
// instruction covers 4 columns x 256 contiguous bytes.  Requires 16-byte
// aligned operands with even leading dimensions (else tn_direct_kernel).
// --------------------------------------------------------------------------
struct TnArgs {
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  int M, N; int64_t K;
  int64_t kchunk; int nsplit; int tilesN; int ntiles;
  double* C; int64_t ldc;
  double* C2; int64_t ldc2;
  double* part;
};

constexpr int KC = 32;           // k-values per LDS slab
constexpr int LDP = KC + 2;      // padded LDS column (doubles)

__device__ __forceinline__ void tn_store(const TnArgs& a, const v4d (&acc)[2][2], int tile, int split, int wave,
                                         int lane, int i0, int j0) {
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
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = i0 + 16 * x + li, j = j0 + 16 * y + 4 * r + g;
        if (i < a.M && j < a.N) {
          double v = acc[x][y][r];
          a.C[i + (int64_t)j * a.ldc] = v;
          if (a.C2) a.C2[i + (int64_t)j * a.ldc2] += v;
        }
      }
}

__global__ __launch_bounds__(256) void tn_lds_kernel(TnArgs a) {
  __shared__ double sA[2][64 * LDP];
  __shared__ double sB[2][64 * LDP];
  const int tile = blockIdx.x, split = blockIdx.y;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int64_t kb = (int64_t)split * a.kchunk;
  const int64_t ke = std::min<int64_t>(a.K, kb + a.kchunk);
  // staging: thread loads one double2 (k pair lq) of columns lc + 16r, r < 4
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
  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0, 0, 0, 0};
  const int ia0 = (wave & 1) * 32, jb0 = (wave >> 1) * 32;
  const int nfull = (int)((ke - kb) / KC);
  double2 ra[4], rb[4];

  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 16) {
      double xa[2][4], xb[2][4];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double* pa = &sA[buf][(ia0 + 16 * t + li) * LDP + kk + 4 * g];
        const double* pb = &sB[buf][(jb0 + 16 * t + li) * LDP + kk + 4 * g];
        double2 a0 = *reinterpret_cast<const double2*>(pa), a1 = *reinterpret_cast<const double2*>(pa + 2);
        double2 b0 = *reinterpret_cast<const double2*>(pb), b1 = *reinterpret_cast<const double2*>(pb + 2);
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

  if (nfull > 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ra[r] = *reinterpret_cast<const double2*>(ga[r] + kb);
      rb[r] = *reinterpret_cast<const double2*>(gb[r] + kb);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      *reinterpret_cast<double2*>(&sA[0][(lc + 16 * r) * LDP + 2 * lq]) = ra[r];
      *reinterpret_cast<double2*>(&sB[0][(lc + 16 * r) * LDP + 2 * lq]) = rb[r];
    }
    __syncthreads();
    for (int sl = 0; sl < nfull; ++sl) {
      const int buf = sl & 1;
      // prefetch the next slab into registers (clamped: the last iteration
      // reloads the current slab, which is cached and not used)
      const int64_t kn = kb + (int64_t)((sl + 1 < nfull) ? sl + 1 : sl) * KC;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        ra[r] = *reinterpret_cast<const double2*>(ga[r] + kn);
        rb[r] = *reinterpret_cast<const double2*>(gb[r] + kn);
      }
      compute(buf);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        *reinterpret_cast<double2*>(&sA[buf ^ 1][(lc + 16 * r) * LDP + 2 * lq]) = ra[r];
        *reinterpret_cast<double2*>(&sB[buf ^ 1][(lc + 16 * r) * LDP + 2 * lq]) = rb[r];
      }
      __syncthreads();
    }
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
      double2 va, vb;
      va.x = (k < ke) ? pa[k] : 0.0;
      va.y = (k + 1 < ke) ? pa[k + 1] : 0.0;
      vb.x = (k < ke) ? pb[k] : 0.0;
      vb.y = (k + 1 < ke) ? pb[k + 1] : 0.0;
      *reinterpret_cast<double2*>(&sA[buf][(lc + 16 * r) * LDP + 2 * lq]) = va;
      *reinterpret_cast<double2*>(&sB[buf][(lc + 16 * r) * LDP + 2 * lq]) = vb;
    }
    __syncthreads();
    compute(buf);
  }
  tn_store(a, acc, tile, split, wave, lane, tm * 64 + ia0, tn * 64 + jb0);
}

// Fallback for operands that are not 16-byte aligned or have odd leading
// dimensions: direct scalar loads, same tiling and output contract.
__global__ __launch_bounds__(256) void tn_direct_kernel(TnArgs a) {
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
  tn_store(a, acc, tile, split, wave, lane, i0, j0);
}

// Sum the split partials of every tile in split order; write C (and C2 +=).
__global__ __launch_bounds__(256) void tn_reduce_kernel(TnArgs a) {
  const int tile = blockIdx.x;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int i0 = tm * 64 + (wave & 1) * 32, j0 = tn * 64 + (wave >> 1) * 32;
  double v[16];
  sum_partials(a.part, a.nsplit, a.ntiles, tile, wave, lane, v);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = i0 + 16 * x + li, j = j0 + 16 * y + 4 * r + g;
        if (i < a.M && j < a.N) {
          double val = v[(x * 2 + y) * 4 + r];
          a.C[i + (int64_t)j * a.ldc] = val;
          if (a.C2) a.C2[i + (int64_t)j * a.ldc2] += val;
        }
      }
}

static bool aligned16(const void* p, int64_t ld) {
  return (reinterpret_cast<uintptr_t>(p) % 16 == 0) && (ld % 2 == 0);
}

static int pick_split(int tiles, int64_t K, int64_t cap) {
  // ~768 blocks in flight; each split keeps at least 512 rows of the reduction
  int want = std::max(1, 768 / std::max(1, tiles));
  int64_t maxs = std::max<int64_t>(1, K / 512);
  int ns = (int)std::min<int64_t>(want, maxs);
  while (ns > 1 && (int64_t)ns * tiles > cap) --ns;
  return ns;
}

// Launch the split-K product; returns the number of splits (partials left in
// s.part when > 1).  With reduce_here the tiles are summed into C right away.
static int tn_partials(TnArgs& a, int M, int N, int64_t K, const Scratch& s, hipStream_t st, bool reduce_here,
                       int force_split = 0) {
  const int tilesM = (M + kTile - 1) / kTile, tilesN = (N + kTile - 1) / kTile;
  const int tiles = tilesM * tilesN;
  int ns = force_split > 0 ? force_split : pick_split(tiles, K, s.npart);
  while (ns > 1 && (int64_t)ns * tiles > s.npart) --ns;
  int64_t kchunk = (K + ns - 1) / ns;
  kchunk = (kchunk + KC - 1) / KC * KC;
  ns = (int)((K + kchunk - 1) / kchunk);
  a.M = M; a.N = N; a.K = K; a.kchunk = kchunk; a.nsplit = ns; a.tilesN = tilesN; a.ntiles = tiles;
  a.part = s.part;
  const bool vec = aligned16(a.A, a.lda) && aligned16(a.B, a.ldb);
  if (vec)
    hipLaunchKernelGGL(tn_lds_kernel, dim3(tiles, ns), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(tn_direct_kernel, dim3(tiles, ns), dim3(256), 0, st, a);
  if (ns > 1 && reduce_here) hipLaunchKernelGGL(tn_reduce_kernel, dim3(tiles), dim3(256), 0, st, a);
  return ns;
}

void launch_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int M, int N, int64_t K,
               double* C, int64_t ldc, double* C2, int64_t ldc2, const Scratch& s, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  TnArgs a{};
  a.A = A; a.lda = lda; a.B = B; a.ldb = ldb;
  a.C = C; a.ldc = ldc; a.C2 = C2; a.ldc2 = ldc2;
  tn_partials(a, M, N, K, s, st, true);
}

// --------------------------------------------------------------------------
// Gram matrix of a panel leaf (w <= kLeaf columns) and its upper Cholesky
// factor.  The split-K partial tiles are first summed by gram_sum_kernel
// (16 blocks, one 256-entry slice each, split order), then one wavefront
// factors W: lane t keeps column t of W in registers and the rows of R are
// exchanged through LDS, so the 64 sequential steps need no block barrier.
// pass 1: R1 <- chol(W), T <- R1^{-1}.  pass 2: T <- R2^{-1}, Rout <- R2 R1.
// A non-positive pivot sets info[0] = 1 + panel (first occurrence kept) and
// the factorization continues with pivot 1.
// --------------------------------------------------------------------------
struct CholArgs {
  const double* part; int nsplit;
  double* W;               // w x w Gram matrix (ld w): written by the sum kernel or the product kernel
  int w, pass, panel;
  double* T; double* R1; double* Rout; int64_t ldr; int* info;
};

// W entry e = i + j*w  <-  sum over splits of the partial element mapped to (i, j)
__global__ __launch_bounds__(256) void gram_sum_kernel(CholArgs a) {
  const int e = blockIdx.x * 256 + threadIdx.x;      // 0 .. 4095 over the 64 x 64 tile
  const int i = e & 63, j = e >> 6;
  // inverse of the (wave, q, lane) -> (i, j) map of the product kernel
  const int wave = (i >> 5) | ((j >> 5) << 1);
  const int x = (i >> 4) & 1, y = (j >> 4) & 1, li = i & 15, r = (j & 15) >> 2, g = j & 3;
  const int q = (x * 2 + y) * 4 + r, lane = g * 16 + li;
  const double* p = a.part + part_off(0, 1, 0, wave) + q * 64 + lane;
  double v = 0.0;
  int sp = 0;
  for (; sp + 8 <= a.nsplit; sp += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = p[(int64_t)(sp + u) * 4096];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
  }
  for (; sp < a.nsplit; ++sp) v += p[(int64_t)sp * 4096];
  if (i < a.w && j < a.w) a.W[i + j * a.w] = v;
}

// Exact path: upper Cholesky factor R of W (64 x 64, identity-padded in Rl)
// by four wavefronts.  Thread (tx, ty) holds column tx, rows ty + 4q (q < 16)
// in registers; row j of R is exchanged through LDS buffers alternating with
// the step parity (two block barriers per step).  Entries below the diagonal
// are updated too but never read.  On exit Rl holds R (zero below).
__device__ __forceinline__ void chol4(int tid, double (*rowP)[kLeaf], double (*rowR)[kLeaf], double (*Rl)[kLeaf + 1],
                                      bool& bad) {
  const int tx = tid & 63, ty = tid >> 6;
  double c[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) c[q] = Rl[ty + 4 * q][tx];
#pragma unroll
  for (int j = 0; j < kLeaf; ++j) {
    const int jq = j >> 2, jt = j & 3, par = j & 1;
    if (ty == jt) rowP[par][tx] = c[jq];
    __syncthreads();
    double piv = rowP[par][j];
    if (!(piv > 0.0) || !isfinite(piv)) {
      bad = true;
      piv = 1.0;
    }
    const double rjj = sqrt(piv);
    const double inv = 1.0 / rjj;
    const double rk = (tx > j) ? rowP[par][tx] * inv : (tx == j ? rjj : 0.0);   // R[j][tx]
    if (ty == jt) {
      c[jq] = rk;
      rowR[par][tx] = rk;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (ty + 4 * q > j) c[q] -= rowR[par][ty + 4 * q] * rk;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) Rl[ty + 4 * q][tx] = (ty + 4 * q <= tx) ? c[q] : 0.0;
}

__global__ __launch_bounds__(256) void chol_kernel(CholArgs a) {
  __shared__ double Rl[kLeaf][kLeaf + 1];
  __shared__ double Tl[kLeaf][kLeaf + 1];
  __shared__ double rowP[2][kLeaf];
  __shared__ double rowR[2][kLeaf];
  __shared__ int s_exact, s_bad;
  const int tid = threadIdx.x, wave = tid >> 6, w = a.w;
  if (tid == 0) { s_exact = (a.pass == 1); s_bad = 0; }
  __syncthreads();
  // W, identity-padded, into LDS; the second pass checks W = I + E, |E| small
  for (int e = tid; e < kLeaf * kLeaf; e += 256) {
    const int i = e % kLeaf, k = e / kLeaf;
    const double val = (i < w && k < w) ? a.W[i + k * w] : (i == k ? 1.0 : 0.0);
    Rl[i][k] = val;
    if (a.pass == 2 && !(fabs(val - (i == k ? 1.0 : 0.0)) <= 1e-8)) s_exact = 1;
  }
  __syncthreads();
  if (s_exact) {
    bool bad = false;
    chol4(tid, rowP, rowR, Rl, bad);
    if (bad && tid == 0) s_bad = 1;
    __syncthreads();
    // T = R^{-1}: wave 0, lane t solves column t by back substitution
    if (wave == 0) {
      const int t = tid;
      double tc[kLeaf];
#pragma unroll
      for (int i = kLeaf - 1; i >= 0; --i) {
        double acc = (t == i) ? 1.0 : 0.0;
#pragma unroll
        for (int k = i + 1; k < kLeaf; ++k) acc -= Rl[i][k] * tc[k];
        tc[i] = acc / Rl[i][i];
      }
#pragma unroll
      for (int i = 0; i < kLeaf; ++i) Tl[i][t] = tc[i];
    }
  } else {
    // W = I + E, |E| <= 1e-8:  R = I + F with F the strict upper part of E
    // plus half its diagonal; R^{-1} = I - F up to O(|E|^2), below rounding.
    for (int e = tid; e < kLeaf * kLeaf; e += 256) {
      const int i = e % kLeaf, k = e / kLeaf;
      const double f = (i < k) ? Rl[i][k] : (i == k ? 0.5 * (Rl[i][k] - 1.0) : 0.0);
      Tl[i][k] = ((i == k) ? 1.0 : 0.0) - f;
    }
    __syncthreads();
    for (int e = tid; e < kLeaf * kLeaf; e += 256) {
      const int i = e % kLeaf, k = e / kLeaf;
      Rl[i][k] = (i <= k) ? 2.0 * ((i == k) ? 1.0 : 0.0) - Tl[i][k] : 0.0;   // I + F
    }
  }
  __syncthreads();
  for (int e = tid; e < w * w; e += 256) a.T[e] = Tl[e % w][e / w];
  if (a.pass == 1) {
    for (int e = tid; e < w * w; e += 256) a.R1[e] = Rl[e % w][e / w];
  } else {
    // R_panel = R2 R1, R1 staged in LDS (Tl is free once T is stored)
    __syncthreads();
    for (int e = tid; e < kLeaf * kLeaf; e += 256) {
      const int i = e % kLeaf, k = e / kLeaf;
      Tl[i][k] = (i < w && k < w) ? a.R1[i + k * w] : 0.0;
    }
    __syncthreads();
    const int t = tid & 63, v = tid >> 6;
    for (int q = 0; q < 16; ++q) {
      const int i = v + 4 * q;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int p = i & ~3; p < kLeaf; p += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (p + u >= i) acc[u] += Rl[i][p + u] * Tl[p + u][t];
      }
      if (i < w && t < w) a.Rout[i + (int64_t)t * a.ldr] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
  }
  if (tid == 0 && s_bad && *a.info == 0) *a.info = 1 + a.panel;
}

void launch_gram_chol(const double* P, int64_t ldp, int64_t mrows, int w, int pass, double* Rout,
                      int64_t ldr, int panel, const Scratch& s, hipStream_t st) {
  TnArgs a{};
  a.A = P; a.lda = ldp; a.B = P; a.ldb = ldp;
  a.C = s.W; a.ldc = w; a.C2 = nullptr; a.ldc2 = 0;
  // one output tile: split the rows finely (>= 128 per block, at most 64 blocks)
  const int ns = tn_partials(a, w, w, mrows, s, st, false,
                             (int)std::max<int64_t>(1, std::min<int64_t>(64, mrows / 128)));
  CholArgs c{};
  c.part = s.part; c.nsplit = ns; c.W = s.W;
  c.w = w; c.pass = pass; c.panel = panel;
  c.T = s.T; c.R1 = s.R1; c.Rout = Rout; c.ldr = ldr; c.info = s.info;
  if (ns > 1) hipLaunchKernelGGL(gram_sum_kernel, dim3(16), dim3(256), 0, st, c);
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(256), 0, st, c);
}

// --------------------------------------------------------------------------
// In-place panel transform P <- P T (T upper triangular, w <= 64 columns).
// Each block stages 64 rows of P in LDS, then 4 waves (16 rows each) form
// the product with MFMA.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void apply_kernel(double* P, int64_t ldp, int64_t mrows, int w,
                                                    const double* T) {
  __shared__ double tileP[kLeaf][64 + 1];   // [col][row]
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * w; e += 256) {
    const int rr = e % 64, c = e / 64;
    const int64_t row = r0 + rr;
    tileP[c][rr] = (row < mrows) ? P[row + (int64_t)c * ldp] : 0.0;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int rl = wave * 16 + li;
  v4d acc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) acc[y] = v4d{0, 0, 0, 0};
  for (int k0 = 0; k0 < w; k0 += 16) {
    double xb[4][4];
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int j = 16 * y + li;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = k0 + 4 * g + s;
        xb[y][s] = (k < w && j < w) ? T[k + (int64_t)j * w] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      const double xa = (k < w) ? tileP[k][rl] : 0.0;
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[y] = mfma(xb[y][s], xa, acc[y]);
    }
  }
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * y + 4 * r + g;
      const int64_t row = r0 + wave * 16 + li;
      if (j < w && row < mrows) P[row + (int64_t)j * ldp] = acc[y][r];
    }
}

void launch_apply(double* P, int64_t ldp, int64_t mrows, int w, const Scratch& s, hipStream_t st) {
  const int blocks = (int)((mrows + 63) / 64);
  hipLaunchKernelGGL(apply_kernel, dim3(blocks), dim3(256), 0, st, P, ldp, mrows, w, (const double*)s.T);
}

// --------------------------------------------------------------------------
// Rank-K update  C -= A B  (A: M x K, B: K x N, C: M x N, column-major).
// Tile 64 x 64 per block; wave w takes rows 16w..16w+15 and all 64 columns
// (4 accumulator blocks).  Short K (the trailing update, K = b): C is loaded
// at the start so its latency overlaps the products.  Long K with few tiles
// (re-projection): the K range is split over blocks and nn_reduce_kernel
// subtracts the partial tiles from C in split order.
// --------------------------------------------------------------------------
struct NnArgs {
  double* C; int64_t ldc;
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  int64_t M; int N; int K;
  int kchunk; int nsplit; int tilesN; int ntiles; int vec;
  double* part;
};

template <bool SPLIT>
__global__ __launch_bounds__(256) void nn_kernel(NnArgs a) {
  const int tile = blockIdx.x, split = blockIdx.y;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int64_t i = (int64_t)tm * 64 + wave * 16 + li;
  const int jb = tn * 64;
  const bool aok = i < a.M;
  const int64_t ic = aok ? i : 0;                 // clamped row: valid address, result unused
  const int kb = split * a.kchunk;
  const int ke = std::min(a.K, kb + a.kchunk);
  double cval[4][4];
  if (!SPLIT) {
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jb + 16 * y + 4 * r + g;
        cval[y][r] = a.C[ic + (int64_t)(j < a.N ? j : 0) * a.ldc];
      }
  }
  const double* ar = a.A + ic;
  const double* bc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    const int j = jb + 16 * y + li;
    bc[y] = a.B + (int64_t)(j < a.N ? j : 0) * a.ldb;
  }
  v4d acc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) acc[y] = v4d{0, 0, 0, 0};
  double xa[4], xb[4][4], na[4], nb[4][4];
  auto load_full = [&](int k0, double (&ya)[4], double (&yb)[4][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) ya[s] = ar[(int64_t)(k0 + 4 * g + s) * a.lda];
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const double2* pb = reinterpret_cast<const double2*>(bc[y] + k0 + 4 * g);
      const double2 b0 = pb[0], b1 = pb[1];
      yb[y][0] = b0.x; yb[y][1] = b0.y; yb[y][2] = b1.x; yb[y][3] = b1.y;
    }
  };
  auto mma = [&](const double (&ya)[4], const double (&yb)[4][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[y] = mfma(yb[y][s], ya[s], acc[y]);
  };
  const int kfull = a.vec ? kb + (ke - kb) / 16 * 16 : kb;
  if (kfull > kb) {
    load_full(kb, xa, xb);
    int k0 = kb;
    for (; k0 + 16 < kfull; k0 += 32) {
      load_full(k0 + 16, na, nb);
      mma(xa, xb);
      load_full((k0 + 32 < kfull) ? k0 + 32 : k0 + 16, xa, xb);
      mma(na, nb);
    }
    if (k0 < kfull) mma(xa, xb);
  }
  for (int k0 = kfull; k0 < ke; k0 += 16) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      const bool kok = k < ke;
      xa[s] = kok ? ar[(int64_t)k * a.lda] : 0.0;
#pragma unroll
      for (int y = 0; y < 4; ++y) xb[y][s] = kok ? bc[y][k] : 0.0;
    }
    mma(xa, xb);
  }
  if (SPLIT) {
    double* mine = a.part + part_off(split, a.ntiles, tile, wave);
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) mine[(y * 4 + r) * 64 + lane] = acc[y][r];
    return;
  }
  if (!aok) return;
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = jb + 16 * y + 4 * r + g;
      if (j < a.N) a.C[i + (int64_t)j * a.ldc] = cval[y][r] - acc[y][r];
    }
}

__global__ __launch_bounds__(256) void nn_reduce_kernel(NnArgs a) {
  const int tile = blockIdx.x;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int64_t i = (int64_t)tm * 64 + wave * 16 + li;
  const int jb = tn * 64;
  double v[16];
  sum_partials(a.part, a.nsplit, a.ntiles, tile, wave, lane, v);
  if (i >= a.M) return;
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = jb + 16 * y + 4 * r + g;
      if (j < a.N) a.C[i + (int64_t)j * a.ldc] -= v[y * 4 + r];
    }
}

void launch_nn_sub(double* C, int64_t ldc, const double* A, int64_t lda, const double* B, int64_t ldb,
                   int64_t M, int N, int K, const Scratch& s, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  NnArgs a{};
  a.C = C; a.ldc = ldc; a.A = A; a.lda = lda; a.B = B; a.ldb = ldb;
  a.M = M; a.N = N; a.K = K;
  a.tilesN = (N + 63) / 64;
  a.ntiles = (int)((M + 63) / 64) * a.tilesN;
  a.vec = aligned16(B, ldb);
  a.part = s.part;
  int ns = 1;
  if (a.ntiles < 512 && K >= 1024) {
    ns = (int)std::min<int64_t>((768 + a.ntiles - 1) / a.ntiles, K / 512);
    while (ns > 1 && (int64_t)ns * a.ntiles > s.npart) --ns;
  }
  int kchunk = (K + ns - 1) / ns;
  kchunk = (kchunk + 15) / 16 * 16;
  ns = (K + kchunk - 1) / kchunk;
  a.kchunk = kchunk;
  a.nsplit = ns;
  if (ns > 1) {
    hipLaunchKernelGGL(nn_kernel<true>, dim3(a.ntiles, ns), dim3(256), 0, st, a);
    hipLaunchKernelGGL(nn_reduce_kernel, dim3(a.ntiles), dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL(nn_kernel<false>, dim3(a.ntiles, 1), dim3(256), 0, st, a);
  }
}

}  // namespace cqr
