// Internal interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace cqr {

constexpr int kMaxLine = 32;     // blocks in one code line (data + checksums)
constexpr int kMaxOut = 8;       // blocks written by one decode launch
constexpr int kMaxGen = 8;       // checksum blocks per code (K_v, K_h)
constexpr int kMaxGrid = 32;     // p_r, p_c upper bound
constexpr int kLeaf = 64;        // widest panel leaf factored by Cholesky QR
constexpr int kTile = 64;        // output tile of the split-K product kernel

// Linear combination of blocks along one code line: out_o = sum_s coef[o][s] * src_s.
struct LineArgs {
  double* base;
  int64_t ld;
  int rows, cols;
  int nsrc, nout;
  int64_t src[kMaxLine];
  int64_t dst[kMaxOut];
  double coef[kMaxOut][kMaxLine];
};

struct EraseArgs {
  double* base;
  int64_t ld;
  int rows, cols;
  int nblk;
  int64_t off[64];
};

struct EncodeArgs {
  double* At;
  int64_t ld;
  int64_t m, n, bs, bw;
  int pr, pc, kv, kh;
  double g[kMaxGen * kMaxGrid];    // row code: g[k * pr + t] = g~_v[k][t]
  double gc[kMaxGen * kMaxGrid];   // column code: gc[l * kMaxGrid + t] = g~_h[t][l]
};

struct PostArgs {
  const double* src;
  int64_t lds;
  double* dst;
  int64_t ldd;
  int64_t bs, cols;
  int pr, kv;
  double gv[kMaxGen * kMaxGrid];   // G~_v = [G~_1  V~], K_v x p_r row-major
};

// dA = X_top + G_v^T X_bottom (encoding adjoint), X with m + K_v bs rows.
struct FoldArgs {
  const double* X;
  int64_t ldx;
  double* dA;
  int64_t ldd;
  int64_t m, bs, cols;
  int pr, kv;
  double gv[kMaxGen * kMaxGrid];   // G~_v, K_v x p_r row-major
};

// Scratch regions inside the caller's workspace (all device pointers).
struct Scratch {
  int* info;          // [0]: 0, or 1 + the first panel that is exactly rank-deficient;
                      // [1]: first Cholesky pass of the current leaf broke down;
                      // [2]: leaves orthogonalised by the column-wise fallback
  int* fb;            // per panel: 1 if its second pass took the column-wise fallback
  double* part;       // split-K partial tiles
  int64_t npart;      // capacity in tiles (of kTile*kTile doubles)
  double* S;          // projection coefficients (and the fused first-pass Gram)
  double* G;          // second-pass Gram and lookahead product (kLeaf x 2 kLeaf)
  double* T;          // inverse Cholesky factor (kLeaf x kLeaf)
  double* R1;         // first-pass Cholesky factor (kLeaf x kLeaf)
  double* X;          // two first-pass panel copies (ldx x b each, xstride doubles apart)
  int64_t ldx, xstride;
  double* T2;         // the second pass's inverse factor, kept for the update stream
  double* colw;       // column-wise panel partial sums (kColWorkDoubles)
};

// Kernel-instance tags: each use of a product kernel gets its own symbol, so
// per-kernel profiles map onto the steps of the factorization.
enum : int { TAG_TRAIL = 0, TAG_REPROJ = 1, TAG_PANEL = 2 };

// C (M x N) [= or +=] A^T B, A: K x M (lda), B: K x N (ldb), split over K.
struct TnArgs {
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  int M, N; int64_t K;
  int64_t kchunk; int nsplit; int tilesN; int ntiles;
  double* C; int64_t ldc;
  double* C2; int64_t ldc2;
  int M2;             // only rows i < M2 are added into C2
  double* part;
  int vec;            // both operands 16-byte aligned with even leading dimensions
  int f32;            // FP32 products (operands rounded), FP32 sums over 16
                      // k-values, FP64 sums across those groups
  int prio;           // raise the waves' issue priority (panel-chain products)
  int pair;           // two tile rows per 512-thread workgroup (tn2_kernel)
  int quad;           // 128 x 128 output per 512-thread workgroup (tnq_kernel, FP64)
  int bf3;            // split-BF16 product (tnb_kernel): each FP64 operand as hi + mid + lo
                      // BF16 parts, six part products on BF16 MFMA with FP32 sums over
                      // 32 k-values, FP64 sums across them (output layout as f32)
};

// Choose the split of C = A^T B (stored to C; rows below M2 -- all rows
// unless changed -- also added into C2 if C2 != nullptr).
// force_split > 0 fixes the split count (capped by the partial capacity).
// lowp: 1 = the product on FP32 MFMA (operands rounded to FP32, FP32 sums over
// 16 k-values, FP64 sums across them); 2 = split BF16 (tnb_kernel) where the
// shape allows it (at least two tile rows and columns, depth a multiple of
// 32, aligned operands), else FP32; for the mixed-precision coefficient
// product R_bar = Qbar^T Q_t.
TnArgs tn_setup(const double* A, int64_t lda, const double* B, int64_t ldb, int M, int N, int64_t K, double* C,
                int64_t ldc, double* C2, int64_t ldc2, const Scratch& s, int force_split = 0, int lowp = 0);
// The product; with nsplit == 1 it stores C (and C2) itself, else partials.
void launch_tn_product(const TnArgs& a, int tag, hipStream_t st);
// Sum the partials into C (and C2) in split order (nsplit > 1 only).
void launch_tn_reduce(const TnArgs& a, hipStream_t st);
// out (w x N, ldo) = T^T W for the product W = A^T B of a (a.M = w <= 64 rows,
// one tile row): W is summed from the split partials (nsplit > 1) or read from
// a.C (nsplit == 1, where the product stored it); T is w x w (ld w).
// fb, P, ldp: when *fb is set (the panel's second pass took the column-wise
// fallback) out = P^T B is formed directly from the finished panel P instead.
void launch_tn_reduce_tmul(const TnArgs& a, const double* T, int w, double* out, int64_t ldo, hipStream_t st,
                           const int* fb = nullptr, const double* P = nullptr, int64_t ldp = 0);

// C (M x N) -= A (M x K) B (K x N).
struct NnArgs {
  double* C; int64_t ldc;
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  int64_t M; int N; int K;
  int kchunk; int nsplit; int tilesN; int ntiles;
  int vec;            // B 16-byte aligned with even ldb (vector B loads)
  double* part;
  int prio;           // raise the waves' issue priority (panel-chain products)
};
// The update is FP64 in every precision mode: it is a column operation on the
// encoded matrix and must keep the checksum relations to FP64 rounding.
NnArgs nn_setup(double* C, int64_t ldc, const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M,
                int N, int K, const Scratch& s);
void launch_nn_product(const NnArgs& a, int tag, hipStream_t st);
void launch_nn_reduce(const NnArgs& a, hipStream_t st);   // nsplit > 1 only

// Arguments of the panel Cholesky kernel (Gram matrix W in, T = R^{-1} and R1
// to scratch, on the second pass R2 R1 to Rout and T^T X to Rbar).
struct CholArgs {
  const double* W; int64_t ldw;     // w x w Gram matrix
  int w, pass, panel;
  double* T; double* R1; double* Rout; int64_t ldr; int* info;
  const double* X; int64_t ldx;     // pass 2, optional: w x w product P1^T Q_next
  double* Rbar;                     // T^T X (ld ldr)
  double* Tcopy;                    // pass 2, optional: second destination of T (w x w, ld w)
  double* P; int64_t ldp; int64_t mrows;   // pass 2: the panel (for the column-wise fallback)
  int* fb;                          // pass 2, optional: set to 1 when the fallback ran
};

// One panel leaf orthogonalised column by column (colgrid_kernel): the rows
// are split over up to kColGridMax workgroups, and each launch takes one step
// of the method on every slab, leaving per-workgroup partial sums (kColSlots
// each) that every workgroup of the next launch reduces in the same order.
enum : int { COLWISE_CGS2 = 0, COLWISE_ICGS = 1, COLWISE_MGS = 2 };
constexpr int kColGridMax = 256;
constexpr int kColSlots = 68;       // 64 inner products, three squared norms, one spare
// partial sums (two buffers, alternating by launch) and four state words
constexpr int64_t kColWorkDoubles = 2 * (int64_t)kColGridMax * kColSlots + 4;
struct ColArgs {
  double* P; int64_t ldp; int64_t mrows;
  int w, mode;                      // w <= kLeaf; mode: COLWISE_CGS2 / _ICGS / _MGS
  double eta;                       // ICGS: reorthogonalise when ||p after|| < eta ||p before||
  double* Rout; int64_t ldr;        // the panel's R block (w x w, zeros below the diagonal)
  int* info; int panel;             // a zero column sets info[0] = 1 + panel
  double* work;                     // kColWorkDoubles of scratch
};
void launch_colpanel(const ColArgs& a, hipStream_t st);

CholArgs chol_args(const double* W, int64_t ldw, int w, int pass, double* Rout, int64_t ldr, const double* X,
                   int64_t ldx, double* Rbar, int panel, const Scratch& s);

// Upper Cholesky factor of the panel Gram matrix W (w x w, ld ldw, w <= kLeaf).
// pass 1: R1 <- chol(W), T <- R1^{-1}.  pass 2: R2 <- chol(W), T <- R2^{-1},
// Rout (ldr) <- R2 R1, and, if X != nullptr, Rbar (ldr) <- T^T X (X: w x w,
// ld ldx).  On the second pass T is also stored to Tcopy when it is not
// nullptr.
// Breakdown (a pivot at most 1e-14 times its diagonal entry): pass 1 returns
// R1 = T = I and flags info[1]; pass 2 (flagged or breaking down) then
// orthogonalises the panel P (mrows x w, ld ldp) column by column with CGS2,
// returns T = I, Rout = R_cgs2 R1, Rbar = P^T Q_next from the finished panel
// (Q_next: the w columns after P), sets *fb (if given) and counts the
// fallback in info[2]; a zero column after projection sets info[0].
void launch_chol(const double* W, int64_t ldw, int w, int pass, double* Rout, int64_t ldr, const double* X,
                 int64_t ldx, double* Rbar, int panel, const Scratch& s, hipStream_t st, double* Tcopy = nullptr,
                 double* P = nullptr, int64_t ldp = 0, int64_t mrows = 0, int* fb = nullptr);

// The split re-projection update (launch_nn_product with nsplit > 1) with the
// first Cholesky pass described by c run by one extra block of the same
// launch; returns false, launching nothing, when the update does not split.
bool launch_nn_chol(const NnArgs& a, const CholArgs& c, hipStream_t st);
// The split reduction of a panel update (a.N = w <= 64 columns, one column
// tile) fused with the panel transform C <- C T (T: w x w, ld w); the result
// is also stored to X (ld ldx) when X != nullptr.  False, launching nothing,
// for any other shape.
bool launch_nn_reduce_apply(const NnArgs& a, const double* T, int w, double* X, int64_t ldx, hipStream_t st);
// The panel transform A <- A T (A: M x w, the update's left operand; T: w x w,
// ld w) and the rank-w update C -= A B in one launch (K = w <= 64, one column
// tile, FP64); false, launching nothing, for any other shape.
bool launch_nn1_apply(const NnArgs& a, const double* T, int w, hipStream_t st);

// P <- P T in place (T = s.T, w x w upper triangular), P is mrows x w.
void launch_apply(double* P, int64_t ldp, int64_t mrows, int w, const Scratch& s, hipStream_t st);

void launch_zero_ints(int* p, int n, hipStream_t st);
void launch_fill_zero(double* p, int64_t ld, int64_t rows, int64_t cols, hipStream_t st);
// checksum rows only (a.kv rows of the code g over a.n columns)
void launch_encode_rows(const EncodeArgs& a, hipStream_t st);
// the whole encoding in one pass: checksum rows (g), columns (gc) and corner
void launch_encode_fused(const EncodeArgs& a, hipStream_t st);
void launch_line(const LineArgs& a, hipStream_t st);
void launch_erase(const EraseArgs& a, hipStream_t st);
void launch_postorth(const PostArgs& a, hipStream_t st);
// coded solve: Y = Q^T B (Q m x n), then blocked back substitution with R_1
void launch_gemv_t(const double* Q, int64_t ldq, int64_t m, int n, const double* B, int64_t ldb, int nrhs,
                   double* Y, int64_t ldy, hipStream_t st);
void launch_trinv(const double* R, int64_t ldr, int64_t n, double* T, hipStream_t st);
// adjoint helpers
void launch_transpose(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows, int64_t cols,
                      double scale, bool upper, hipStream_t st);
void launch_copyltu(double* C, int64_t ldc, int64_t n, hipStream_t st);
void launch_outer(const double* U, int64_t ldu, const double* V, int64_t ldv, int64_t rows, int64_t cols, int k,
                  double scale, bool upper, double* C, int64_t ldc, hipStream_t st);
void launch_gemv_n(const double* A, int64_t lda, int64_t m, int n, const double* x, int64_t ldx, int nrhs,
                   double* y, int64_t ldy, hipStream_t st);
void launch_fold(const FoldArgs& a, hipStream_t st);
// Y (n x n) = block diagonal of the 64 x 64 tiles of T (tile k at T + 4096 k)
void launch_blockdiag(const double* T, double* Y, int64_t ldy, int64_t n, hipStream_t st);
// C *= s (rows x cols)
void launch_scale(double* C, int64_t ldc, int64_t rows, int64_t cols, double s, hipStream_t st);
void launch_trsv_step(const double* R, int64_t ldr, const double* T, double* Y, int64_t ldy, double* X,
                      int64_t ldx, int nrhs, int64_t k0, int w, hipStream_t st);
// The allocation-free solve's scratch: a file-scope device array of
// kSolveScratchBytes, one copy per device.  *ptr receives the current
// device's copy's address (looked up on the first call on each device).
constexpr size_t kSolveScratchBytes = size_t(32) << 20;
hipError_t solve_scratch(void** ptr);

}  // namespace cqr
