// FP64 MFMA kernels of the blocked Gram-Schmidt: the split-K projection
// product (R_bar = Qbar^T Q_t, S = Q_prev^T P, Gram matrices), the rank-b
// update (Q_t -= Qbar R_bar, P -= Q_prev S), the panel's Cholesky step and the
// in-place triangular transform of the panel (P <- P R^{-1}).
//
// MFMA layout used throughout (v_mfma_f64_16x16x4, one wavefront of 64 lanes):
// D = X Y + D with X 16x4, Y 4x16; lane l supplies X[l%16][l/16] and
// Y[l/16][l%16] and holds D[4r + l/16][l%16] in accumulator element r.  Every
// product here is issued as the transposed product (D = C^T), so lane l holds
// C[i0 + l%16][j0 + 4r + l/16]: sixteen consecutive rows of a column-major C per
// lane group, i.e. full 128-byte lines on store.  Within a group of 16 k-values
// lane l contributes k = k0 + 4*(l/16) + s in MFMA step s (a fixed permutation
// of the reduction index shared by both operands).
#include "cqr_kernels.hpp"

#include <algorithm>
#include <cmath>

namespace cqr {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double x, double y, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
}

// --------------------------------------------------------------------------
// Split-K product  C = A^T B  (A: K x M, B: K x N, both K-contiguous).
// Grid (tilesM * tilesN, nsplit); 4 waves, each a 32x32 quadrant of the
// 64x64 tile over the block's K range.  With nsplit > 1 every block writes
// its partial tile, and the last block to arrive (per-tile counter) sums the
// partials in split order, so the result does not depend on scheduling.
// --------------------------------------------------------------------------
struct TnArgs {
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  int M, N; int64_t K;
  int64_t kchunk; int nsplit; int tilesN;
  double* C; int64_t ldc;
  double* C2; int64_t ldc2;
  double* part; int* cnt;
  // Gram/Cholesky epilogue (gram != 0)
  int gram; int pass; int panel;
  double* Rout; int64_t ldr;
  double* W; double* T; double* R1; int* info; int* cnt_all;
};

__device__ void chol_block(const TnArgs& a, int w);

template <bool GRAM>
__global__ __launch_bounds__(256) void tn_kernel(TnArgs a) {
  const int tile = blockIdx.x, split = blockIdx.y;
  const int ntiles = gridDim.x;
  const int tm = tile / a.tilesN, tn = tile % a.tilesN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, g = lane >> 4;
  const int i0 = tm * kTile + (wave & 1) * 32;
  const int j0 = tn * kTile + (wave >> 1) * 32;
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

  double xa[2][4], xb[2][4];
  auto load = [&](int64_t k0, double (&ya)[2][4], double (&yb)[2][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int64_t k = k0 + 4 * g + s;
      bool kok = k < ke;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ya[t][s] = (aok[t] && kok) ? ap[t][k] : 0.0;
        yb[t][s] = (bok[t] && kok) ? bp[t][k] : 0.0;
      }
    }
  };
  if (kb < ke) load(kb, xa, xb);
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
    double na[2][4], nb[2][4];
    if (k0 + 16 < ke) load(k0 + 16, na, nb);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma(xb[y][s], xa[x][s], acc[x][y]);
    if (k0 + 16 < ke) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int s = 0; s < 4; ++s) { xa[t][s] = na[t][s]; xb[t][s] = nb[t][s]; }
    }
  }

  __shared__ int s_flag;
  if (a.nsplit > 1) {
    double* mine = a.part + ((int64_t)split * ntiles + tile) * (kTile * kTile) + wave * 1024;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) mine[((x * 2 + y) * 4 + r) * 64 + lane] = acc[x][y][r];
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_flag = (atomicAdd(&a.cnt[tile], 1) == a.nsplit - 1);
    __syncthreads();
    if (!s_flag) return;
    __threadfence();
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0, 0, 0, 0};
    for (int sp = 0; sp < a.nsplit; ++sp) {
      const double* p = a.part + ((int64_t)sp * ntiles + tile) * (kTile * kTile) + wave * 1024;
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[x][y][r] += p[((x * 2 + y) * 4 + r) * 64 + lane];
    }
    if (threadIdx.x == 0) a.cnt[tile] = 0;
  }

#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = i0 + 16 * x + li;
        int j = j0 + 16 * y + 4 * r + g;
        if (i < a.M && j < a.N) {
          double v = acc[x][y][r];
          a.C[i + (int64_t)j * a.ldc] = v;
          if (a.C2) a.C2[i + (int64_t)j * a.ldc2] += v;
        }
      }

  if constexpr (GRAM) {
    // All tiles of the Gram matrix stored: the last tile to finish factors it.
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_flag = (atomicAdd(a.cnt_all, 1) == ntiles - 1);
    __syncthreads();
    if (!s_flag) return;
    __threadfence();
    if (threadIdx.x == 0) *a.cnt_all = 0;
    chol_block(a, a.M);
  }
}

// Upper Cholesky factor of the w x w Gram matrix W (w <= kLeaf) in one block,
// then T = R^{-1}; pass 2 also forms R2 * R1 into the panel's diagonal block.
__device__ void chol_block(const TnArgs& a, int w) {
  __shared__ double L[kLeaf][kLeaf + 1];
  __shared__ double Ti[kLeaf][kLeaf + 1];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (tid == 0) s_bad = 0;
  for (int e = tid; e < w * w; e += blockDim.x) {
    int i = e % w, k = e / w;
    L[i][k] = a.W[i + (int64_t)k * w];
  }
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    double piv = L[j][j];
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (tid == 0) s_bad = 1;
      piv = 1.0;
    }
    double rjj = sqrt(piv);
    __syncthreads();
    for (int k = j + tid; k < w; k += blockDim.x) L[j][k] = (k == j) ? rjj : L[j][k] / rjj;
    __syncthreads();
    int rem = w - j - 1;
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      int i = j + 1 + e % rem, k = j + 1 + e / rem;
      if (k >= i) L[i][k] -= L[j][i] * L[j][k];
    }
    __syncthreads();
  }
  // T = R^{-1}: column c solved by back substitution, 4 threads per column.
  {
    const int c = tid >> 2, q = tid & 3;
    for (int i = w - 1; i >= 0; --i) {
      double sum = 0.0;
      if (c < w && c >= i) {
        for (int k = i + 1 + q; k <= c; k += 4) sum += L[i][k] * Ti[k][c];
      }
      sum += __shfl_xor(sum, 1);
      sum += __shfl_xor(sum, 2);
      if (c < w && q == 0) {
        if (c == i) Ti[i][c] = 1.0 / L[i][i];
        else if (c > i) Ti[i][c] = -sum / L[i][i];
        else Ti[i][c] = 0.0;
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < w * w; e += blockDim.x) {
    int i = e % w, k = e / w;
    a.T[i + (int64_t)k * w] = (k >= i) ? Ti[i][k] : 0.0;
  }
  if (a.pass == 1) {
    for (int e = tid; e < w * w; e += blockDim.x) {
      int i = e % w, k = e / w;
      a.R1[i + (int64_t)k * w] = (k >= i) ? L[i][k] : 0.0;
    }
  } else {
    // R_panel = R2 R1 (both upper triangular)
    for (int e = tid; e < w * w; e += blockDim.x) {
      int i = e % w, k = e / w;
      double v = 0.0;
      if (k >= i)
        for (int p = i; p <= k; ++p) v += L[i][p] * a.R1[p + (int64_t)k * w];
      a.Rout[i + (int64_t)k * a.ldr] = v;
    }
  }
  if (tid == 0 && s_bad && *a.info == 0) *a.info = 1 + a.panel;
}

static int pick_split(int tiles, int64_t K) {
  // Aim for ~1024 blocks; each split keeps >= 256 rows of the reduction.
  int want = std::max(1, 1024 / std::max(1, tiles));
  int64_t maxs = std::max<int64_t>(1, K / 256);
  return (int)std::min<int64_t>(want, maxs);
}

static void tn_common(TnArgs& a, int M, int N, int64_t K, const Scratch& s, hipStream_t st) {
  int tilesM = (M + kTile - 1) / kTile, tilesN = (N + kTile - 1) / kTile;
  int tiles = tilesM * tilesN;
  int ns = pick_split(tiles, K);
  while (ns > 1 && (int64_t)ns * tiles > s.npart) --ns;
  // tiles must fit the per-tile counters (the last counter is the Gram counter)
  int64_t kchunk = (K + ns - 1) / ns;
  kchunk = (kchunk + 15) / 16 * 16;
  ns = (int)((K + kchunk - 1) / kchunk);
  if (ns < 1) ns = 1;
  a.M = M; a.N = N; a.K = K; a.kchunk = kchunk; a.nsplit = ns; a.tilesN = tilesN;
  a.part = s.part; a.cnt = s.counters;
  if (a.gram)
    hipLaunchKernelGGL(tn_kernel<true>, dim3(tiles, ns), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(tn_kernel<false>, dim3(tiles, ns), dim3(256), 0, st, a);
}

void launch_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int M, int N, int64_t K,
               double* C, int64_t ldc, double* C2, int64_t ldc2, const Scratch& s, hipStream_t st) {
  TnArgs a{};
  a.A = A; a.lda = lda; a.B = B; a.ldb = ldb;
  a.C = C; a.ldc = ldc; a.C2 = C2; a.ldc2 = ldc2;
  a.gram = 0;
  tn_common(a, M, N, K, s, st);
}

void launch_gram_chol(const double* P, int64_t ldp, int64_t mrows, int w, int pass, double* Rout,
                      int64_t ldr, int panel, const Scratch& s, hipStream_t st) {
  TnArgs a{};
  a.A = P; a.lda = ldp; a.B = P; a.ldb = ldp;
  a.C = s.W; a.ldc = w; a.C2 = nullptr; a.ldc2 = 0;
  a.gram = 1; a.pass = pass; a.panel = panel;
  a.Rout = Rout; a.ldr = ldr;
  a.W = s.W; a.T = s.T; a.R1 = s.R1; a.info = s.info; a.cnt_all = s.counters + (s.ncounters - 1);
  tn_common(a, w, w, mrows, s, st);
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
    int rr = e % 64, c = e / 64;
    int64_t row = r0 + rr;
    tileP[c][rr] = (row < mrows) ? P[row + (int64_t)c * ldp] : 0.0;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int rl = wave * 16 + li;   // local row supplied by this lane
  v4d acc[4];
#pragma unroll
  for (int y = 0; y < 4; ++y) acc[y] = v4d{0, 0, 0, 0};
  for (int k0 = 0; k0 < w; k0 += 16) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int k = k0 + 4 * g + s;
      double xa = (k < w) ? tileP[k][rl] : 0.0;
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        int j = 16 * y + li;
        double xb = (k < w && j < w) ? T[k + (int64_t)j * w] : 0.0;
        acc[y] = mfma(xb, xa, acc[y]);
      }
    }
  }
#pragma unroll
  for (int y = 0; y < 4; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int j = 16 * y + 4 * r + g;
      int64_t row = r0 + wave * 16 + li;
      if (j < w && row < mrows) P[row + (int64_t)j * ldp] = acc[y][r];
    }
}

void launch_apply(double* P, int64_t ldp, int64_t mrows, int w, const Scratch& s, hipStream_t st) {
  int blocks = (int)((mrows + 63) / 64);
  hipLaunchKernelGGL(apply_kernel, dim3(blocks), dim3(256), 0, st, P, ldp, mrows, w, (const double*)s.T);
}

// --------------------------------------------------------------------------
// Rank-K update  C -= A B  (A: M x K, B: K x N, C: M x N, column-major).
// Tile TM x 64 per block; waves arranged WM x WN, each 16 rows x 16*BN cols.
// --------------------------------------------------------------------------
template <int TM>
__global__ __launch_bounds__(256) void nn_kernel(double* C, int64_t ldc, const double* A, int64_t lda,
                                                 const double* B, int64_t ldb, int64_t M, int N, int K,
                                                 int tilesN) {
  constexpr int WM = TM / 16, WN = 4 / WM, BN = 4 / WN;
  const int tm = blockIdx.x / tilesN, tn = blockIdx.x % tilesN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
  const int wm = wave % WM, wn = wave / WM;
  const int64_t i = (int64_t)tm * TM + wm * 16 + li;
  const int jb = tn * 64 + wn * 16 * BN;
  const bool aok = i < M;
  const double* ar = A + (aok ? i : 0);
  const double* bc[BN];
  bool bok[BN];
#pragma unroll
  for (int y = 0; y < BN; ++y) {
    int j = jb + 16 * y + li;
    bok[y] = j < N;
    bc[y] = B + (int64_t)(bok[y] ? j : 0) * ldb;
  }
  v4d acc[BN];
#pragma unroll
  for (int y = 0; y < BN; ++y) acc[y] = v4d{0, 0, 0, 0};
  double xa[4], xb[BN][4];
  auto load = [&](int k0, double (&ya)[4], double (&yb)[BN][4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int k = k0 + 4 * g + s;
      bool kok = k < K;
      ya[s] = (aok && kok) ? ar[(int64_t)k * lda] : 0.0;
#pragma unroll
      for (int y = 0; y < BN; ++y) yb[y][s] = (bok[y] && kok) ? bc[y][k] : 0.0;
    }
  };
  if (K > 0) load(0, xa, xb);
  for (int k0 = 0; k0 < K; k0 += 16) {
    double na[4], nb[BN][4];
    if (k0 + 16 < K) load(k0 + 16, na, nb);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int y = 0; y < BN; ++y) acc[y] = mfma(xb[y][s], xa[s], acc[y]);
    if (k0 + 16 < K) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        xa[s] = na[s];
#pragma unroll
        for (int y = 0; y < BN; ++y) xb[y][s] = nb[y][s];
      }
    }
  }
  if (!aok) return;
#pragma unroll
  for (int y = 0; y < BN; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int j = jb + 16 * y + 4 * r + g;
      if (j < N) C[i + (int64_t)j * ldc] -= acc[y][r];
    }
}

void launch_nn_sub(double* C, int64_t ldc, const double* A, int64_t lda, const double* B, int64_t ldb,
                   int64_t M, int N, int K, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  int tilesN = (N + 63) / 64;
  int64_t t64 = (M + 63) / 64 * tilesN, t32 = (M + 31) / 32 * tilesN;
  if (t64 >= 512) {
    hipLaunchKernelGGL(nn_kernel<64>, dim3((unsigned)t64), dim3(256), 0, st, C, ldc, A, lda, B, ldb, M, N, K, tilesN);
  } else if (t32 >= 512) {
    hipLaunchKernelGGL(nn_kernel<32>, dim3((unsigned)t32), dim3(256), 0, st, C, ldc, A, lda, B, ldb, M, N, K, tilesN);
  } else {
    int64_t t16 = (M + 15) / 16 * tilesN;
    hipLaunchKernelGGL(nn_kernel<16>, dim3((unsigned)t16), dim3(256), 0, st, C, ldc, A, lda, B, ldb, M, N, K, tilesN);
  }
}

}  // namespace cqr
