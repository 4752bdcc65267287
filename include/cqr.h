/*
 * cqr.h - C ABI of the MI355X coded-QR library.
 *
 * Coded QR after Nguyen, Weissburg & Jeong, "Coded Computing for
 * Fault-Tolerant Parallel QR Decomposition" (arXiv 2311.11943).  The nodes of
 * the paper's p_r x p_c processor grid are the blocks of one matrix held in the
 * HBM of one GPU; a node failure is an erasure of the blocks it holds.
 *
 * Conventions (every entry point):
 *   - Matrices are column-major FP64 with an explicit leading dimension.
 *   - Matrix pointers are DEVICE pointers owned by the caller; the library never
 *     allocates, frees or retains them.  Host pointers are marked "host".
 *   - Calls that take a hipStream_t enqueue their work on that stream and return
 *     without waiting for it (no host-device synchronisation, no allocation).
 *   - Errors are returned as cqr_status; nothing is thrown or aborted.  When an
 *     argument check fails (CQR_EINVAL, CQR_ENOTRECOVERABLE) nothing has been
 *     enqueued and every buffer is untouched.
 *   - A plan is immutable after creation (apart from the opt-in profiling
 *     record) and may be shared by streams, but calls that touch the same
 *     matrices or workspace must be ordered by the caller (one stream, or events).
 *
 * Shapes: A is m x n (m >= n), p_r | m, p_c | n, p_r | n.  Block height
 * bs = m/p_r, block width bw = n/p_c, R block height hr = n/p_r.  The encoded
 * matrix A~ has m' = m + K_v*bs rows and N = n + K_h*bw columns; R is
 * r_rows x N (coded_qr_plan_r_rows): n rows, plus, when the plan has no
 * horizontal code (K_h = 0, K_v > 0, e.g. a p_r x 1 grid), K_v*hr checksum rows
 * that protect R's block rows with the vertical code (below R_1's n rows).
 */
#ifndef CQR_H
#define CQR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CQR_OK = 0,
  CQR_EINVAL = 1,          /* bad shape, pointer, leading dimension or option */
  CQR_ENOTRECOVERABLE = 2, /* more erased blocks in a block row/column than surviving checksums */
  CQR_ESINGULAR = 3,       /* the small generator submatrix to invert is numerically singular */
  CQR_EHIP = 4,            /* a HIP runtime call failed (launch, copy) */
  CQR_ENOMEM = 5,          /* workspace too small / host allocation failed */
  CQR_EBREAKDOWN = 6       /* a panel column is zero after projection (rank-deficient input) */
} cqr_status;

typedef enum { CQR_OUT_OF_NODE = 0, CQR_IN_NODE = 1 } cqr_storage;

/* Arithmetic of the trailing update's coefficient product R_bar = Qbar^T Q_t
 * (not in the paper: a growth direction).  CQR_FP64: everything in FP64.
 * CQR_TRAIL_FP32: R_bar (and the early update's Qbar1^T Q_t) on FP32 MFMA,
 * operands rounded to FP32, FP32 sums over 16 k-values and FP64 sums across
 * them.  CQR_TRAIL_BF16X3: the same products split into BF16 parts (each FP64
 * operand x = hi + mid + lo to 2^-26 |x|; the six part products of size at
 * least 2^-16 of the whole on BF16 MFMA, FP32 sums over 32 k-values, FP64
 * sums across them) where the product has at least two 64-row and two
 * 64-column tiles and a depth that is a multiple of 32 (the trailing products
 * of panels wider than 64 columns), FP32 otherwise.  In every mode the column operations
 * on A~ -- the rank-b update Q_t -= Qbar R_bar, the re-projection and the
 * panel factorization -- run in FP64 with the coefficients R records, so the
 * checksum rows are carried (Q_2 = G_v Q_1 to FP64 rounding, nothing is
 * re-encoded) and A~ = Q~ R holds to FP64 rounding; the FP64 re-projection of
 * the next panels removes what the reduced-precision R_bar leaves behind.  The
 * R-side relation R_2 = R_1 G_h holds for finished columns to FP64 rounding
 * and for unfinished columns to the accuracy of R_bar, which bounds the error
 * of R blocks decoded mid-factorization. */
typedef enum { CQR_FP64 = 0, CQR_TRAIL_FP32 = 1, CQR_TRAIL_BF16X3 = 2 } cqr_precision;

/* How each panel is orthogonalised (appendix algorithms PBMGS, CGS,
 * sequential MGS; ICGS in the PBMGS listing).  Every mode is a column
 * operation on the panel, so the checksum rows are carried through it.
 *   CQR_PANEL_CHOLQR2 (default): two Cholesky-QR passes, the block form of
 *     CGS2 (a Gram product and a 64 x 64 Cholesky per pass).  A pass whose
 *     Cholesky pivot falls to 1e-14 of its diagonal entry (a column within
 *     1e-7 rad of the span of the others) hands the panel to the column-wise
 *     CGS2 below; coded_qr_ws_panel_fallbacks counts such panels.
 *   CQR_PANEL_CGS2: column-wise classical Gram-Schmidt, every column
 *     projected twice against the finished columns of its panel.
 *   CQR_PANEL_ICGS: the same with the second projection only when the first
 *     left less than icgs_eta of the column's norm (the Daniel-Gragg-
 *     Kaufman-Stewart test, a reading of the paper's unstated criterion).
 *   CQR_PANEL_MGS: the paper's sequential modified Gram-Schmidt within the
 *     panel (its experiments' choice; with reproject = 0 the paper's method).
 * The column-wise modes run one workgroup per panel leaf of up to 64 columns
 * with FP64 norms and wavefront reductions; wider panels are split in halves,
 * the right half projected twice against the left one. */
typedef enum { CQR_PANEL_CHOLQR2 = 0, CQR_PANEL_CGS2 = 1, CQR_PANEL_ICGS = 2, CQR_PANEL_MGS = 3 } cqr_panel;

typedef struct {
  int64_t m, n;        /* A is m x n; the paper's problem is square (m == n) */
  int32_t pr, pc;      /* simulated node grid */
  int32_t kv, kh;      /* checksum block-rows (protect Q) / block-columns (protect R) */
  int32_t storage;     /* cqr_storage: which blocks a node failure erases */
  int32_t b;           /* panel width of the blocked Gram-Schmidt; b | n */
  int32_t reproject;   /* 1: re-project each panel against all earlier Q columns
                          before factoring it (default); 0: the paper's PBMGS */
  int32_t precision;   /* cqr_precision */
  int32_t lookahead;   /* 1: the panel chain runs on a plan-owned stream while a
                          second plan-owned stream applies each panel's update to
                          the columns right of the next panel; both fork from and
                          join back to the caller's stream within each call.  The
                          update starts from the panel after its first Cholesky
                          pass, its coefficients taken as R2^{-T} (P1^T Q_t), equal
                          to P^T Q_t up to rounding (split products may also sum in
                          another order).  Two plans with lookahead alive at once
                          hold four streams, as many as a device has hardware
                          queues by default, so their streams may share queues and
                          lose the overlap.  0: everything on the caller's stream */
  int32_t panel;       /* cqr_panel */
  double icgs_eta;     /* CQR_PANEL_ICGS threshold in (0, 1]; 0 selects 1/sqrt(2) */
} cqr_config;

typedef struct cqr_plan_s* cqr_plan;

/*
 * Create a plan (host only, no device work).
 *   v_tilde (host, K_v x (p_r - K_v), row-major): the Unif(0,1) entries that the
 *     Q-side generator construction draws; the plan forms
 *     G~_v = [G~_1  V~] with G~_1 = -1/2 V~ V~^T  (construction of the Q-factor
 *     checksum generator, out-of-node and in-node forms).  Ignored if K_v = 0.
 *   gh (host, p_c x K_h, row-major): R-side generator (any MDS code, System
 *     Model / R-factor protection); for in-node storage the plan zeroes entry
 *     (k mod p_c, k) so checksum k excludes its storing column (In-Node
 *     Systematic MDS construction).  Ignored if K_h = 0.
 *   Requires: K_v <= p_r/2 when K_v > 0 (post-orthogonalization construction);
 *   m % p_r == n % p_c == n % p_r == 0; b | n; p_r, p_c <= 32; K_v, K_h <= 8;
 *   p_r + K_v <= 32 and p_c + K_h <= 32; precision is CQR_FP64 or
 *   CQR_TRAIL_FP32; panel is a cqr_panel; 0 <= icgs_eta <= 1.
 * Returns CQR_EINVAL on any violated condition; *out is then NULL.
 */
cqr_status coded_qr_plan_create(const cqr_config* cfg, const double* v_tilde, const double* gh,
                                cqr_plan* out);
void coded_qr_plan_destroy(cqr_plan plan);

/* Copy the plan's generators to host buffers: gv (K_v x p_r, row-major),
 * gh (p_c x K_h, row-major, exclusion zeros applied).  Either may be NULL. */
cqr_status coded_qr_plan_generators(cqr_plan plan, double* gv, double* gh);

/* Placement of the checksum blocks (host outputs; either may be NULL).
 * qrow (K_v entries): the grid row whose nodes store Q-checksum block row k,
 * the same in every block column; rcol (K_h entries): the grid column whose
 * nodes store R-checksum block column k, the same in every block row.
 * In-node storage (load-balanced distribution: of the p_r nodes of a grid
 * column, K_v - p_r floor(K_v/p_r) hold ceil(K_v/p_r) checksum blocks and the
 * rest floor(K_v/p_r)): qrow[k] = k mod p_r, rcol[k] = k mod p_c, and the R
 * code excludes the storer, G~_h[rcol[k], k] = 0.  Out-of-node storage:
 * checksum nodes of their own, qrow[k] = p_r + k and rcol[k] = p_c + k on the
 * extended grid. */
cqr_status coded_qr_plan_placement(cqr_plan plan, int32_t* qrow, int32_t* rcol);

/* Failures per grid row / column the plan's code tolerates (out-of-node: K;
 * in-node: largest f with f + f*ceil(f/(p_r-f)) <= K, the theorem on the
 * minimum in-node checksum count). */
int32_t coded_qr_plan_ftol(cqr_plan plan);

/* Rows of R: n, or n + K_v*hr when K_h = 0 and K_v > 0.  Without R-checksum
 * columns, a failed node's R blocks would have no code; R's p_r block rows
 * then carry K_v checksum block rows R_chk = (G~_v (x) I_hr) R[0:n], written
 * by coded_qr_factor at the end of every call (the panel boundaries where
 * failures strike; R's entries become final only column block by column
 * block, since each panel's re-projection adds into earlier rows) and decoded
 * along block columns by coded_qr_recover. */
int64_t coded_qr_plan_r_rows(cqr_plan plan);

/* Bytes of device workspace coded_qr_factor needs (caller allocates). */
size_t coded_qr_workspace_bytes(cqr_plan plan);

/*
 * Encode (System Model, encoding equation):
 *   A~ = [[A, A G_h], [G_v A, G_v A G_h]],  G = G~ (x) I.
 * At (device, m' x N, ld ldat >= m'): on entry A sits in At[0:m, 0:n]; on exit
 * the checksum rows, checksum columns and corner are written.  A is not read
 * outside At[0:m, 0:n].
 */
cqr_status coded_qr_encode(cqr_plan plan, double* At, int64_t ldat, hipStream_t stream);

/*
 * Factor panels [panel_begin, panel_end) of the blocked Gram-Schmidt (the
 * paper's PBMGS run on A~, appendix algorithm PBMGS / BMGS): for panel k with
 * columns [kb, (k+1)b):
 *   optional re-projection  S = Q[:, :kb]^T P,  P -= Q[:, :kb] S,  R[:kb, panel] += S;
 *   panel orthogonalisation with reorthogonalisation (two Cholesky-QR passes,
 *     the block form of CGS2; each a column operation P <- P T);
 *   trailing update over every column right of the panel, checksum columns
 *     included:  R_bar = Qbar^T Q_t,  R[panel, right] = R_bar,  Q_t -= Qbar R_bar.
 * At (device, m' x N, ldat): the iteration state Q^(t) (A~ on the first call);
 * R (device, r_rows x N, ldr >= r_rows): rows [0, n) zeroed by this call when
 * panel_begin == 0; R's checksum rows (if any) re-encoded before it returns.
 * ws (device, >= coded_qr_workspace_bytes bytes, 256-byte aligned).
 * Calls may be split at any panel boundary (failures are injected between).
 * Numerical breakdown (rank deficiency) is recorded in the workspace and read
 * with coded_qr_ws_info.
 */
cqr_status coded_qr_factor(cqr_plan plan, double* At, int64_t ldat, double* R, int64_t ldr,
                           int32_t panel_begin, int32_t panel_end, void* ws, size_t ws_bytes,
                           hipStream_t stream);

/* Blocking: wait for `stream`, then return the breakdown flag stored in ws
 * (0 = none, else 1 + the index of the first panel with a zero column after
 * projection, i.e. exactly rank-deficient input) in *info (host); returns
 * CQR_EBREAKDOWN when it is set. */
cqr_status coded_qr_ws_info(cqr_plan plan, const void* ws, hipStream_t stream, int32_t* info);

/* Blocking: wait for `stream`, then return in *count (host) how many panel
 * leaves since the last call with panel_begin == 0 were orthogonalised by
 * the column-wise CGS2 fallback after a Cholesky-QR breakdown. */
cqr_status coded_qr_ws_panel_fallbacks(cqr_plan plan, const void* ws, hipStream_t stream, int32_t* count);

/*
 * Fail-stop failure simulation: set every block held by the listed nodes to NaN
 * (System Model, failure model; a node loses its inputs and results).
 * failed_ij (host, 2*nfailed int32): node coordinates (i, j).  Out-of-node
 * storage: 0 <= i < p_r + K_v, 0 <= j < p_c + K_h (i >= p_r or j >= p_c name
 * checksum nodes).  In-node: 0 <= i < p_r, 0 <= j < p_c; a node also holds the
 * checksum blocks placed on it (Q-checksum row k on grid row k mod p_r,
 * R-checksum column k on grid column k mod p_c).  With R checksum rows
 * (coded_qr_plan_r_rows > n) R-checksum block row k sits with Q-checksum row k.
 * ldq >= m', ldr >= r_rows.
 */
cqr_status coded_qr_erase(cqr_plan plan, double* Q, int64_t ldq, double* R, int64_t ldr,
                          const int32_t* failed_ij, int32_t nfailed, hipStream_t stream);

/*
 * Recover every block held by the listed nodes from surviving blocks and
 * checksums (recovery-overhead lemma, decoding equation): per affected block
 * column of Q (vertical code, Q_2 = G_v Q_1 holds for all N columns) and per
 * block row of R (horizontal code, R_2 = R_1 G_h; without one, per block
 * column of R with its checksum rows and G_v), with F the erased data blocks
 * and S the |F| lowest-index surviving checksums,
 *   X_F = G_hat^{-1} (C_S - sum_{t not in F} g~_{S,t} X_t),   G_hat = G~[S, F],
 * then lost checksum blocks are re-encoded.  The small solve runs on the host
 * in FP64 (no device read-back); every output block is one linear combination
 * of surviving blocks, written by one HIP pass.
 * Returns CQR_ENOTRECOVERABLE (nothing enqueued) if a line has more erased
 * data blocks than surviving checksums, CQR_ESINGULAR if G_hat is singular.
 * No panel index is taken: between panels both relations hold for every
 * column, finished or not, so the decode is the same at any panel boundary;
 * no workspace either: the decode coefficients travel in the kernel
 * arguments.
 */
cqr_status coded_qr_recover(cqr_plan plan, double* Q, int64_t ldq, double* R, int64_t ldr,
                            const int32_t* failed_ij, int32_t nfailed, hipStream_t stream);

/*
 * Post-orthogonalization (theorem on low-cost post-orthogonalization):
 *   Qpost = G_0 Q_1,  Bpost = G_0 B,  G_0 = [[I + G_1, V], [V^T, -I]] = G^_0 (x) I_bs,
 * with Q_1 = Q[0:m, 0:n].  Q (device, ldq >= m), Qpost (device, m x n, ldqp >= m),
 * B / Bpost (device, m x nrhs, ldb / ldbp >= m; may be NULL when nrhs == 0).
 * Qpost may alias Q and Bpost may alias B (in-place).  Requires K_v > 0.
 */
cqr_status coded_qr_postorth(cqr_plan plan, const double* Q, int64_t ldq, double* Qpost, int64_t ldqp,
                             const double* B, int64_t ldb, double* Bpost, int64_t ldbp, int32_t nrhs,
                             hipStream_t stream);

/*
 * Coded linear solve (the linear-solve equations that follow the theorem on
 * low-cost post-orthogonalization):  R_1 X = Qpost^T Bpost, i.e.
 *   X = R_1^{-1} (G_0 Q_1)^T (G_0 B),
 * with Qpost = G_0 Q_1 and Bpost = G_0 B from coded_qr_postorth and R_1 =
 * R[0:n, 0:n] from coded_qr_factor.  For square A this is the solution of
 * A X = B.  For tall A (m > n) it minimises (AX - B)^T W (AX - B) with
 * W = I + G_v^T G_v (ordinary least squares only when the residual is zero).
 * Qpost (device, m x n, ldqp >= m), R (device, ldr >= n; only its upper
 * triangle R[0:n, 0:n] is read), Bpost (device, m x nrhs, ldbp >= m),
 * X (device, n x nrhs, ldx >= n, written; must not alias the inputs).
 * nrhs >= 1.  ws: caller-owned device workspace, 256-byte aligned, of at least
 * coded_qr_solve_workspace_bytes(plan, nrhs) bytes (the inverted 64 x 64
 * diagonal blocks of R_1 and Y = Qpost^T Bpost); CQR_ENOMEM if smaller or
 * misaligned.  No pivoting and no singularity check: R_1 from coded_qr_factor
 * has a positive diagonal whenever its info is 0, and a zero pivot gives
 * non-finite entries of X.
 */
size_t coded_qr_solve_workspace_bytes(cqr_plan plan, int32_t nrhs);
cqr_status coded_qr_solve(cqr_plan plan, const double* Qpost, int64_t ldqp, const double* R, int64_t ldr,
                          const double* Bpost, int64_t ldbp, int32_t nrhs, double* X, int64_t ldx, void* ws,
                          size_t ws_bytes, hipStream_t stream);

/*
 * coded_qr_solve without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, serving loops that
 * forbid allocation).  Same arguments, kernels and result as coded_qr_solve
 * (X bit-identical); its scratch (the inverted diagonal blocks of R_1 and
 * Y = Qpost^T Bpost) is a file-scope device array of
 * CQR_SOLVE_NOALLOC_MAX_BYTES, one copy per device, held until the process
 * ends.  Returns CQR_ENOMEM, enqueueing nothing, when
 * coded_qr_solve_workspace_bytes(plan, nrhs) exceeds that size.  Allocates
 * nothing.  Every call on one device shares that device's array: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller.
 */
#define CQR_SOLVE_NOALLOC_MAX_BYTES ((size_t)32 << 20)
cqr_status coded_qr_solve_noalloc(cqr_plan plan, const double* Qpost, int64_t ldqp, const double* R, int64_t ldr,
                                  const double* Bpost, int64_t ldbp, int32_t nrhs, double* X, int64_t ldx,
                                  hipStream_t stream);

/*
 * Adjoint (reverse-mode derivative) of the coded QR.  Not in the paper: a
 * growth direction built on its definitions.  The coded QR maps A to the
 * factors of the encoded systematic columns, A~ = [A; G_v A] = Q~ R_1 (System
 * Model, encoding equation).  Given the cotangents dQ~ (m' x n) and dR_1
 * (n x n; only its upper triangle is read), this computes the standard
 * reverse-mode rule of the thin QR followed by the encoding's transpose:
 *   M = R_1 dR_1^T - dQ~^T Q~,   dA~ = (dQ~ + Q~ copyltu(M)) R_1^{-T},
 *   dA = dA~_top + G_v^T dA~_bottom,
 * where copyltu(M) is the symmetric matrix that holds M's lower triangle.
 * Q (device, m' x n, ldq >= m': Q~ from coded_qr_factor), R (device,
 * ldr >= n: R_1 = R[0:n, 0:n], zero below the diagonal as coded_qr_factor
 * leaves it), dQ (device, m' x n, lddq >= m'), dR (device, n x n,
 * lddr >= n), dA (device, m x n, ldda >= m, written; must not alias inputs).
 * ws: caller-owned device workspace of at least
 * coded_qr_backward_workspace_bytes(plan) bytes, 256-byte aligned, else
 * CQR_ENOMEM (split-product partials, R_1^{-1}, three n x n and two m' x n
 * buffers).  Asynchronous on `stream`; allocates nothing.
 */
size_t coded_qr_backward_workspace_bytes(cqr_plan plan);
cqr_status coded_qr_backward(cqr_plan plan, const double* Q, int64_t ldq, const double* R, int64_t ldr,
                             const double* dQ, int64_t lddq, const double* dR, int64_t lddr, double* dA,
                             int64_t ldda, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Adjoint of the coded solve X = R_1^{-1} (G_0 Q_1)^T (G_0 B) (coded_qr_solve).
 * With dY = R_1^{-T} dX:
 *   dR_1 = -triu(dY X^T),   dQ~[0:m] = G_0 (Bpost dY^T),   dQ~[m:m'] = 0,
 *   dB = G_0 (Qpost dY)     (G_0 is symmetric, so it is its own transpose);
 * dQ~ and dR_1 feed coded_qr_backward.  Qpost, Bpost from coded_qr_postorth
 * (device, m x n and m x nrhs), R from coded_qr_factor, X from coded_qr_solve
 * (device, n x nrhs, ldx >= n), dX (device, n x nrhs, lddx >= n).  Written:
 * dQ (device, m' x n, lddq >= m'), dR (device, n x n upper, zero below,
 * lddr >= n), dB (device, m x nrhs, lddb >= m).  Requires K_v > 0.  ws: at
 * least coded_qr_solve_backward_workspace_bytes(plan, nrhs) bytes, 256-byte
 * aligned, else CQR_ENOMEM.
 */
size_t coded_qr_solve_backward_workspace_bytes(cqr_plan plan, int32_t nrhs);
cqr_status coded_qr_solve_backward(cqr_plan plan, const double* Qpost, int64_t ldqp, const double* R, int64_t ldr,
                                   const double* Bpost, int64_t ldbp, const double* X, int64_t ldx,
                                   const double* dX, int64_t lddx, int32_t nrhs, double* dQ, int64_t lddq,
                                   double* dR, int64_t lddr, double* dB, int64_t lddb, void* ws, size_t ws_bytes,
                                   hipStream_t stream);

/*
 * Per-phase timing (diagnostics).  While enabled, the plan records a HIP event
 * pair around every kernel launch, on the stream that launch runs on, and
 * remembers the phase, the algorithmic flops and the minimum HBM bytes of that
 * launch; each record covers exactly one kernel.  Enabling or disabling clears
 * the record.  Reading waits for the recorded events (host-blocking).
 * Profiling makes the plan stateful: do not profile one plan from several host
 * threads at once.
 * Phases: 0 encode, 1 re-projection product (S = Q^T P), 2 re-projection update
 * (P -= Q S), 3 panel Gram product (P^T P), 4 panel Cholesky factor and
 * inverse, 5 panel transform (P <- P R^{-1}), 6 in-panel projection (split
 * panels), 7 trailing product (R_bar = Qbar^T Q_t), 8 trailing update
 * (Q_t -= Qbar R_bar), 9 reduction of split-product partial tiles, 10 recovery,
 * 11 post-orthogonalization, 12 erase, 13 other (workspace/R initialisation),
 * 14 column-wise panel (CQR_PANEL_CGS2 / ICGS / MGS), 15 coded solve,
 * 16 adjoint (coded_qr_backward, coded_qr_solve_backward).
 * coded_qr_profile_read returns, for `phase`, the summed event time (ms), the
 * number of launches and the summed flops / bytes (host outputs; may be NULL).
 */
#define CQR_NPHASES 17
cqr_status coded_qr_profile_enable(cqr_plan plan, int32_t enable);
cqr_status coded_qr_profile_read(cqr_plan plan, int32_t phase, double* total_ms, int64_t* launches,
                                 double* flops, double* bytes);

const char* coded_qr_status_string(cqr_status status);

/* Name of the HIP error behind the calling thread's most recent CQR_EHIP
 * ("hipSuccess" if there was none).  Entry points that launch work first
 * discard an error that other code left pending on the thread, so a CQR_EHIP
 * always stems from the library's own HIP calls. */
const char* coded_qr_hip_error_name(void);

#ifdef __cplusplus
}
#endif
#endif /* CQR_H */
