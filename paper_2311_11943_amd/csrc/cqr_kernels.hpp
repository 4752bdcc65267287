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
  // rows pass: g[k * pr + t] = g~_v[k][t];  columns pass: g[k * pc + t] = g~_h[t][k]
  double g[kMaxGen * kMaxGrid];
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

// Scratch regions inside the caller's workspace (all device pointers).
struct Scratch {
  int* info;          // [0]: breakdown flag (0 or 1 + panel)
  double* part;       // split-K partial tiles
  int64_t npart;      // capacity in tiles (of kTile*kTile doubles)
  double* S;          // projection coefficients
  double* W;          // Gram matrix (kLeaf x kLeaf)
  double* T;          // inverse Cholesky factor (kLeaf x kLeaf)
  double* R1;         // first-pass Cholesky factor (kLeaf x kLeaf)
};

// C (M x N) [= or +=] A^T B, A: K x M (lda), B: K x N (ldb).  The result is
// stored to C (ldc); if C2 != nullptr it is also added into C2 (ldc2).
void launch_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int M, int N, int64_t K,
               double* C, int64_t ldc, double* C2, int64_t ldc2, const Scratch& s, hipStream_t st);

// Gram matrix W = P^T P of the w-column panel P (m' x w), then its upper
// Cholesky factor.  pass 1: R1 <- chol, T <- R1^{-1}.  pass 2: R2 <- chol,
// T <- R2^{-1}, Rout (ldr) <- R2 R1.  Breakdown sets info[0] = 1 + panel.
void launch_gram_chol(const double* P, int64_t ldp, int64_t mrows, int w, int pass, double* Rout,
                      int64_t ldr, int panel, const Scratch& s, hipStream_t st);

// P <- P T in place (T = s.T, w x w upper triangular), P is mrows x w.
void launch_apply(double* P, int64_t ldp, int64_t mrows, int w, const Scratch& s, hipStream_t st);

// C (M x N) -= A (M x K) B (K x N).
void launch_nn_sub(double* C, int64_t ldc, const double* A, int64_t lda, const double* B, int64_t ldb,
                   int64_t M, int N, int K, const Scratch& s, hipStream_t st);

void launch_zero_ints(int* p, int n, hipStream_t st);
void launch_fill_zero(double* p, int64_t ld, int64_t rows, int64_t cols, hipStream_t st);
void launch_encode_rows(const EncodeArgs& a, hipStream_t st);
void launch_encode_cols(const EncodeArgs& a, hipStream_t st);
void launch_line(const LineArgs& a, hipStream_t st);
void launch_erase(const EraseArgs& a, hipStream_t st);
void launch_postorth(const PostArgs& a, hipStream_t st);

}  // namespace cqr
