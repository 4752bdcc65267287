// C-ABI entry points of the coded-QR library (declared in include/cqr.h).
// Host side: argument checks, the code construction, the failure bookkeeping
// and the small FP64 solves of the decoder; all matrix work is enqueued as HIP
// kernels on the caller's stream.
#include "cqr.h"
#include "cqr_kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <set>
#include <utility>
#include <vector>

using cqr::kLeaf;
using cqr::kMaxGen;
using cqr::kMaxGrid;
using cqr::kMaxLine;
using cqr::kMaxOut;
using cqr::kTile;

struct cqr_plan_s {
  cqr_config cfg;
  int64_t bs, bw, hr, mp, N;
  // no horizontal code (K_h = 0, K_v > 0): R carries K_v checksum block rows
  // of the vertical code below its n rows, so R has rrows rows
  bool rcode = false;
  int64_t rrows = 0;
  int ftol;
  std::vector<double> gv;   // K_v x p_r row-major:  [G~_1  V~]
  std::vector<double> gh;   // p_c x K_h row-major
  int64_t npart = 0, nS = 0;
  int64_t ldx = 0, xstride = 0;   // first-pass panel copies for the early update (0: none)
  size_t off_part = 0, off_part2 = 0, off_S = 0, off_G = 0, off_T = 0, off_R1 = 0, off_X = 0, off_T2 = 0,
         off_colw = 0, ws_bytes = 0;
  int ninfo = 0;           // ints of the info area: 64 status words, then one fallback flag per panel
  double eta = 0.0;        // ICGS threshold in use
  // lookahead: the panel chain's stream, the update stream and four events,
  // created on first use on the device current at that time
  hipStream_t chain = nullptr, side = nullptr;
  hipEvent_t ev_main = nullptr, ev_side = nullptr, ev_chain = nullptr, ev_apply = nullptr;
  int side_dev = -1;
  // opt-in per-launch timing
  struct Rec { int phase; hipEvent_t a, b; double flops, bytes; };
  bool prof = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
};

enum Phase { PH_ENCODE = 0, PH_REPROJ_TN, PH_REPROJ_NN, PH_GRAM, PH_CHOL, PH_APPLY, PH_INPANEL, PH_TRAIL_TN,
             PH_TRAIL_NN, PH_REDUCE, PH_RECOVER, PH_POST, PH_ERASE, PH_OTHER, PH_COLPANEL, PH_SOLVE,
             PH_ADJOINT };
static_assert(PH_ADJOINT + 1 == CQR_NPHASES, "phase list and header disagree");
static_assert(cqr::kSolveScratchBytes == CQR_SOLVE_NOALLOC_MAX_BYTES, "scratch size and header disagree");

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Minimum in-node checksum count for f failures with L = P data blocks
// (theorem on the in-node lower bound): K = f + f * ceil(f / (P - f)).
int k_min_in_node(int f, int P) { return f + f * ((f + (P - f) - 1) / (P - f)); }

int tolerated_code(int K, int P, int storage) {
  if (K == 0) return 0;
  if (storage == CQR_OUT_OF_NODE) return K;
  int best = 0;
  for (int f = 1; f < P; ++f)
    if (k_min_in_node(f, P) <= K) best = f;
  return best;
}

// Failures per grid row/column both codes tolerate.
int tolerated(const cqr_plan_s& p) {
  int f = tolerated_code(p.cfg.kv, p.cfg.pr, p.cfg.storage);
  if (p.cfg.kh > 0) f = std::min(f, tolerated_code(p.cfg.kh, p.cfg.pc, p.cfg.storage));
  return f;
}

// Gauss-Jordan inverse with partial pivoting (n <= kMaxOut); false if singular.
bool invert(std::vector<double> a, int n, std::vector<double>& inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  double scale = 0.0;
  for (double v : a) scale = std::max(scale, std::fabs(v));
  if (!(scale > 0.0)) return false;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
    if (!(std::fabs(a[piv * n + c]) > 1e-13 * scale)) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(a[c * n + k], a[piv * n + k]);
        std::swap(inv[c * n + k], inv[piv * n + k]);
      }
    double d = a[c * n + c];
    for (int k = 0; k < n; ++k) { a[c * n + k] /= d; inv[c * n + k] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { a[r * n + k] -= f * a[c * n + k]; inv[r * n + k] -= f * inv[c * n + k]; }
    }
  }
  return true;
}

// Blocks a failed node holds.  Q blocks are (I, J) on the (p_r+K_v) x (p_c+K_h)
// block grid of A~; R blocks are (i, J) with i < p_r.
// Blocks a node holds: Q blocks (I, J) of bs x bw, R blocks (i, J) of hr x bw
// (block rows i >= p_r are R's checksum rows when the plan has the R row code).
void node_blocks(const cqr_plan_s& p, int i, int j, std::vector<std::pair<int, int>>& q,
                 std::vector<std::pair<int, int>>& r) {
  const int pr = p.cfg.pr, pc = p.cfg.pc, kv = p.cfg.kv, kh = p.cfg.kh;
  if (p.cfg.storage == CQR_OUT_OF_NODE) {
    q.push_back({i, j});
    if (i < pr || p.rcode) r.push_back({i, j});
    return;
  }
  std::vector<int> rows{i}, cols{j};
  for (int k = 0; k < kv; ++k) if (k % pr == i) rows.push_back(pr + k);
  for (int k = 0; k < kh; ++k) if (k % pc == j) cols.push_back(pc + k);
  for (int I : rows) for (int J : cols) q.push_back({I, J});
  if (p.rcode) {
    for (int I : rows) for (int J : cols) r.push_back({I, J});
  } else {
    for (int J : cols) r.push_back({i, J});
  }
}

cqr_status check_nodes(const cqr_plan_s& p, const int32_t* ij, int32_t nf) {
  if (nf < 0 || (nf > 0 && !ij)) return CQR_EINVAL;
  for (int f = 0; f < nf; ++f) {
    int i = ij[2 * f], j = ij[2 * f + 1];
    if (p.cfg.storage == CQR_OUT_OF_NODE) {
      if (i < 0 || j < 0 || i >= p.cfg.pr + p.cfg.kv || j >= p.cfg.pc + p.cfg.kh) return CQR_EINVAL;
    } else if (i < 0 || j < 0 || i >= p.cfg.pr || j >= p.cfg.pc) {
      return CQR_EINVAL;
    }
  }
  return CQR_OK;
}

// One decode job: a code line with `ndata` data blocks and `nchk` checksum
// blocks, chk_k = sum_t gen[k][t] data_t.  Produces the launch descriptors.
struct LineJob {
  std::vector<int> lost_d, lost_c;
};

cqr_status plan_line(const std::vector<double>& gen, int ndata, int nchk, const LineJob& job,
                     std::vector<int>& srcs, std::vector<int>& outs, std::vector<double>& coef) {
  // Block index convention: data t -> t, checksum k -> ndata + k.
  const auto& F = job.lost_d;
  const auto& CF = job.lost_c;
  std::vector<int> surv;
  for (int k = 0; k < nchk; ++k)
    if (std::find(CF.begin(), CF.end(), k) == CF.end()) surv.push_back(k);
  const int f = (int)F.size();
  if ((int)surv.size() < f) return CQR_ENOTRECOVERABLE;
  std::vector<int> S(surv.begin(), surv.begin() + f);
  std::vector<int> keep;
  for (int t = 0; t < ndata; ++t)
    if (std::find(F.begin(), F.end(), t) == F.end()) keep.push_back(t);
  // sources: surviving data blocks, then the used checksums
  srcs = keep;
  for (int k : S) srcs.push_back(ndata + k);
  const int ns = (int)srcs.size();
  // coefficient rows of the recovered data blocks over all ndata+nchk slots
  std::vector<std::vector<double>> xrow(ndata, std::vector<double>(ndata + nchk, 0.0));
  for (int t : keep) xrow[t][t] = 1.0;
  if (f > 0) {
    std::vector<double> gh((size_t)f * f), ginv;
    for (int a = 0; a < f; ++a)
      for (int b = 0; b < f; ++b) gh[a * f + b] = gen[(size_t)S[a] * ndata + F[b]];
    if (!invert(gh, f, ginv)) return CQR_ESINGULAR;
    // X_F = Ginv (C_S - sum_{t in keep} gen[S, t] X_t)
    for (int a = 0; a < f; ++a) {
      auto& row = xrow[F[a]];
      for (int b = 0; b < f; ++b) {
        double gi = ginv[a * f + b];
        row[ndata + S[b]] += gi;
        for (int t : keep) row[t] -= gi * gen[(size_t)S[b] * ndata + t];
      }
    }
  }
  outs.clear();
  coef.clear();
  auto push = [&](int slot, const std::vector<double>& full) {
    outs.push_back(slot);
    for (int s = 0; s < ns; ++s) coef.push_back(full[srcs[s]]);
  };
  for (int t : F) push(t, xrow[t]);
  for (int k : CF) {
    std::vector<double> full(ndata + nchk, 0.0);
    for (int t = 0; t < ndata; ++t) {
      double g = gen[(size_t)k * ndata + t];
      for (int s = 0; s < ndata + nchk; ++s) full[s] += g * xrow[t][s];
    }
    push(ndata + k, full);
  }
  return CQR_OK;
}

// Workspace views: `second` selects the split-product partials of the
// lookahead stream (the two streams never share a scratch region).
cqr::Scratch scratch_of(const cqr_plan_s& p, void* ws, bool second = false) {
  char* b = static_cast<char*>(ws);
  cqr::Scratch s;
  s.info = reinterpret_cast<int*>(b);
  s.fb = s.info + 64;
  s.part = reinterpret_cast<double*>(b + (second ? p.off_part2 : p.off_part));
  s.npart = p.npart;
  s.S = reinterpret_cast<double*>(b + p.off_S);
  s.G = reinterpret_cast<double*>(b + p.off_G);
  s.T = reinterpret_cast<double*>(b + p.off_T);
  s.R1 = reinterpret_cast<double*>(b + p.off_R1);
  s.X = p.xstride ? reinterpret_cast<double*>(b + p.off_X) : nullptr;
  s.ldx = p.ldx;
  s.xstride = p.xstride;
  s.T2 = reinterpret_cast<double*>(b + p.off_T2);
  s.colw = reinterpret_cast<double*>(b + p.off_colw);
  return s;
}

// HIP error behind the calling thread's last CQR_EHIP.
thread_local hipError_t t_hip_error = hipSuccess;

cqr_status hip_fail(hipError_t e) {
  t_hip_error = e;
  return CQR_EHIP;
}

// Entry points that launch work first drop an error another library left
// pending on this thread, so that hip_status() reports only their own.
void drop_pending_error() { (void)hipGetLastError(); }

cqr_status hip_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CQR_OK : hip_fail(e);
}

hipEvent_t take_event(cqr_plan_s& p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  // timing events with a device-scope release: a system-scope one (the
  // default) stalls the stream at every record and changes the schedule
  // being measured
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventReleaseToDevice) != hipSuccess) return nullptr;
  return e;
}

// Run `launch` (one kernel) and, while profiling is on, bracket it with events.
template <class F>
void prof(cqr_plan_s& p, int phase, double flops, double bytes, hipStream_t st, F&& launch) {
  if (!p.prof) {
    launch();
    return;
  }
  cqr_plan_s::Rec r{phase, take_event(p), take_event(p), flops, bytes};
  if (r.a) (void)hipEventRecord(r.a, st);
  launch();
  if (r.b) (void)hipEventRecord(r.b, st);
  p.recs.push_back(r);
}

void side_release(cqr_plan_s& p) {
  if (p.ev_main) (void)hipEventDestroy(p.ev_main);
  if (p.ev_side) (void)hipEventDestroy(p.ev_side);
  if (p.ev_chain) (void)hipEventDestroy(p.ev_chain);
  if (p.ev_apply) (void)hipEventDestroy(p.ev_apply);
  if (p.side) (void)hipStreamDestroy(p.side);
  if (p.chain) (void)hipStreamDestroy(p.chain);
  p.side = p.chain = nullptr;
  p.ev_main = p.ev_side = p.ev_chain = p.ev_apply = nullptr;
  p.side_dev = -1;
}

// The lookahead streams (default priority, no implicit synchronization with
// the null stream) and their events on the current device.  The per-panel fork
// and join events order work between two streams of one device only, so they
// skip the system-scope fence (a writeback for host visibility that would
// stall each stream at every panel); the event the caller's stream waits on
// keeps it.
constexpr unsigned kStreamEvent = hipEventDisableTiming | hipEventDisableSystemFence;
bool side_ready(cqr_plan_s& p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (p.side && p.side_dev == dev) return true;
  side_release(p);
  const bool ok = hipStreamCreateWithFlags(&p.chain, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&p.ev_main, kStreamEvent) == hipSuccess &&
                  hipEventCreateWithFlags(&p.ev_side, kStreamEvent) == hipSuccess &&
                  hipEventCreateWithFlags(&p.ev_apply, kStreamEvent) == hipSuccess &&
                  hipEventCreateWithFlags(&p.ev_chain, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    side_release(p);
    (void)hipGetLastError();
    return false;
  }
  p.side_dev = dev;
  return true;
}

void prof_clear(cqr_plan_s& p) {
  for (auto& r : p.recs) {
    if (r.a) p.pool.push_back(r.a);
    if (r.b) p.pool.push_back(r.b);
  }
  p.recs.clear();
}

// Typed wrappers: flops and minimum bytes of each launch.  A split product
// is recorded as two launches: the product (its phase) and the reduction of
// its partial tiles (PH_REDUCE).
int tag_of(int phase) {
  if (phase == PH_TRAIL_TN || phase == PH_TRAIL_NN) return cqr::TAG_TRAIL;
  if (phase == PH_REPROJ_TN || phase == PH_REPROJ_NN) return cqr::TAG_REPROJ;
  return cqr::TAG_PANEL;
}

// Products of the panel chain (everything but the bulk trailing update) run
// their waves at raised issue priority: while they share compute units with
// the update stream's kernels, the chain sets the pace of the factorization.
int chain_phase(int phase) { return phase != PH_TRAIL_TN && phase != PH_TRAIL_NN; }

double partial_bytes(int nsplit, int ntiles) { return 8.0 * nsplit * ntiles * cqr::kTile * cqr::kTile; }

void tn(cqr_plan_s& p, int phase, const double* A, int64_t lda, const double* B, int64_t ldb, int M, int N,
        int64_t K, double* C, int64_t ldc, double* C2, int64_t ldc2, const cqr::Scratch& s, hipStream_t st,
        int M2 = -1, int lowp = 0) {
  if (M <= 0 || N <= 0) return;
  cqr::TnArgs a = cqr::tn_setup(A, lda, B, ldb, M, N, K, C, ldc, C2, ldc2, s, 0, lowp);
  if (M2 >= 0) a.M2 = M2;
  a.prio = chain_phase(phase);
  const double fl = 2.0 * M * N * (double)K, by = 8.0 * ((double)K * M + (double)K * N);
  const double out = 8.0 * (double)M * N * (C2 ? 3.0 : 1.0);
  const int tag = tag_of(phase);
  if (a.nsplit > 1) {
    prof(p, phase, fl, by + partial_bytes(a.nsplit, a.ntiles), st, [&] { cqr::launch_tn_product(a, tag, st); });
    prof(p, PH_REDUCE, (a.nsplit - 1.0) * M * N, partial_bytes(a.nsplit, a.ntiles) + out, st,
         [&] { cqr::launch_tn_reduce(a, st); });
  } else {
    prof(p, phase, fl, by + out, st, [&] { cqr::launch_tn_product(a, tag, st); });
  }
}

void nn(cqr_plan_s& p, int phase, double* C, int64_t ldc, const double* A, int64_t lda, const double* B,
        int64_t ldb, int64_t M, int N, int K, const cqr::Scratch& s, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  cqr::NnArgs a = cqr::nn_setup(C, ldc, A, lda, B, ldb, M, N, K, s);
  a.prio = chain_phase(phase);
  const double fl = 2.0 * M * N * (double)K, by = 8.0 * ((double)M * K + (double)K * N);
  const double upd = 16.0 * (double)M * N;
  const int tag = tag_of(phase);
  if (a.nsplit > 1) {
    prof(p, phase, fl, by + partial_bytes(a.nsplit, a.ntiles), st, [&] { cqr::launch_nn_product(a, tag, st); });
    prof(p, PH_REDUCE, (double)a.nsplit * M * N, partial_bytes(a.nsplit, a.ntiles) + upd, st,
         [&] { cqr::launch_nn_reduce(a, st); });
  } else {
    prof(p, phase, fl, by + upd, st, [&] { cqr::launch_nn_product(a, tag, st); });
  }
}

// The second pass (pass 2) gets the panel P (for its column-wise breakdown
// fallback) and, when an update already started from the panel's first
// pass, that panel's fallback flag.
void chol(cqr_plan_s& p, const double* W, int64_t ldw, int w, int pass, double* Rout, int64_t ldr, const double* X,
          int64_t ldx, double* Rbar, int panel, const cqr::Scratch& s, hipStream_t st, double* Tcopy = nullptr,
          double* P = nullptr, int64_t ldp = 0, int* fb = nullptr) {
  prof(p, PH_CHOL, 2.0 * w * w * w * (X ? 2.0 : 1.0),
       8.0 * w * w * (pass == 1 ? 3.0 : (X ? 6.0 : 4.0) + (Tcopy ? 1.0 : 0.0)), st,
       [&] { cqr::launch_chol(W, ldw, w, pass, Rout, ldr, X, ldx, Rbar, panel, s, st, Tcopy, P, ldp, p.mp, fb); });
}

// Column-wise panel modes (CGS2, ICGS, MGS): a grid of workgroups
// orthogonalises the leaf P (m' x w) column by column, one launch per step,
// and stores R[leaf, leaf].  Flops: 4 m' w^2 for CGS2 (two projections, each
// a product and an update), 2 m' w^2 for MGS; bytes: the panel read and
// written once (the minimum).
void colpanel(cqr_plan_s& p, double* P, int64_t ldq, int w, double* Rout, int64_t ldr, int panel,
              const cqr::Scratch& s, hipStream_t st) {
  cqr::ColArgs a{};
  a.P = P; a.ldp = ldq; a.mrows = p.mp; a.w = w;
  a.mode = p.cfg.panel == CQR_PANEL_MGS ? cqr::COLWISE_MGS
                                         : (p.cfg.panel == CQR_PANEL_ICGS ? cqr::COLWISE_ICGS : cqr::COLWISE_CGS2);
  a.eta = p.eta;
  a.Rout = Rout; a.ldr = ldr; a.info = s.info; a.panel = panel;
  a.work = s.colw;
  const double mult = a.mode == cqr::COLWISE_MGS ? 2.0 : 4.0;
  prof(p, PH_COLPANEL, mult * (double)p.mp * w * w, 16.0 * (double)p.mp * w, st,
       [&] { cqr::launch_colpanel(a, st); });
}

// The product W = X^T B of an update that starts before its panel is
// finished (X: the panel after its first Cholesky pass, mp x w; B: the
// trailing columns), on the update stream.  It leaves the split partials, or
// W itself (ld w) in the partial buffer when the product does not split, for
// tn_tmul's reduction.  Its split keeps the launch to about kEarlyBlocks
// workgroups, below the 512 that two per CU would hold: its workgroups live
// for the whole product, and the chain's kernels, which run beside it, need
// free slots (measured: 448 beats 512 by 2% on the n = 4096 step).
constexpr int kEarlyBlocks = 448;
cqr::TnArgs tn_early(cqr_plan_s& p, const double* X, int64_t ldx, const double* B, int64_t ldb, int w, int N,
                     const cqr::Scratch& s, hipStream_t st, int lowp) {
  const int tiles = (N + kTile - 1) / kTile;
  const int ns = (int)std::max<int64_t>(1, std::min<int64_t>(kEarlyBlocks / tiles, p.mp / 256));
  cqr::TnArgs a = cqr::tn_setup(X, ldx, B, ldb, w, N, p.mp, s.part, w, nullptr, 0, s, ns, lowp);
  a.prio = chain_phase(PH_TRAIL_TN);
  const double fl = 2.0 * w * N * (double)p.mp, by = 8.0 * (double)p.mp * ((double)w + N);
  const double out = a.nsplit > 1 ? partial_bytes(a.nsplit, a.ntiles) : 8.0 * (double)w * N;
  prof(p, PH_TRAIL_TN, fl, by + out, st, [&] { cqr::launch_tn_product(a, cqr::TAG_TRAIL, st); });
  return a;
}

// out = T^T W for the W that tn_early left (T: w x w, the second pass's
// R^{-1}): the update's coefficients against the finished panel.
// (fb, P, ldp: the panel's fallback flag and the finished panel, from which
// the coefficients are formed directly if its second pass fell back.)
void tn_tmul(cqr_plan_s& p, const cqr::TnArgs& a, const double* T, int w, double* out, int64_t ldo,
             hipStream_t st, const int* fb, const double* P, int64_t ldp) {
  const double in = a.nsplit > 1 ? partial_bytes(a.nsplit, a.ntiles) : 8.0 * (double)w * a.N;
  prof(p, PH_REDUCE, (a.nsplit - 1.0) * w * a.N + 2.0 * w * w * (double)a.N, in + 8.0 * (w * w + (double)w * a.N),
       st, [&] { cqr::launch_tn_reduce_tmul(a, T, w, out, ldo, st, fb, P, ldp); });
}

// The split re-projection update C -= A B with the panel's first Cholesky
// pass (c) run by one extra block of the same launch, then the split
// reduction fused with the pass's transform C <- C T (the result also stored
// to X when X != nullptr).  Returns false, launching nothing, when the update
// would not split over K; the caller then runs the update, the Cholesky and
// the transform separately.
bool nn_chol(cqr_plan_s& p, double* C, int64_t ldc, const double* A, int64_t lda, const double* B, int64_t ldb,
             int64_t M, int N, int K, const cqr::CholArgs& c, const cqr::Scratch& s, hipStream_t st,
             double* X = nullptr, int64_t ldx = 0) {
  if (M <= 0 || N <= 0 || K <= cqr::kLeaf || c.w > cqr::kLeaf) return false;
  cqr::NnArgs a = cqr::nn_setup(C, ldc, A, lda, B, ldb, M, N, K, s);
  a.prio = 1;
  if (a.nsplit <= 1 || a.tilesN != 1 || N != c.w) return false;
  const double fl = 2.0 * M * N * (double)K + 2.0 * c.w * c.w * c.w;
  const double by = 8.0 * ((double)M * K + (double)K * N) + 24.0 * c.w * c.w;
  bool launched = false;
  prof(p, PH_REPROJ_NN, fl, by + partial_bytes(a.nsplit, a.ntiles), st,
       [&] { launched = cqr::launch_nn_chol(a, c, st); });
  if (!launched) return false;
  prof(p, PH_REDUCE, (double)a.nsplit * M * N + 2.0 * M * N * N,
       partial_bytes(a.nsplit, a.ntiles) + (X ? 24.0 : 16.0) * (double)M * N, st,
       [&] { cqr::launch_nn_reduce_apply(a, c.T, c.w, X, ldx, st); });
  return true;
}

// The second pass's transform P <- P T (T = the pass's R^{-1} in scratch) and
// the lookahead update C -= P B (B: w x w) in one launch; false, launching
// nothing, when the shapes do not allow it.
bool apply_update(cqr_plan_s& p, double* C, int64_t ldc, double* P, int64_t ldq, const double* B, int64_t ldb,
                  int w, const cqr::Scratch& s, hipStream_t st) {
  const int64_t mp = p.mp;
  const cqr::NnArgs a = cqr::nn_setup(C, ldc, P, ldq, B, ldb, mp, w, w, s);
  if (a.tilesN != 1 || a.K != w || w > cqr::kLeaf) return false;
  bool launched = false;
  prof(p, PH_APPLY, 4.0 * mp * w * w, 8.0 * (4.0 * mp * w + 2.0 * w * w), st,
       [&] { launched = cqr::launch_nn1_apply(a, s.T, w, st); });
  return launched;
}

void apply(cqr_plan_s& p, double* P, int64_t ldq, int w, const cqr::Scratch& s, hipStream_t st) {
  const int64_t mp = p.mp;
  prof(p, PH_APPLY, 2.0 * mp * w * w, 16.0 * mp * w, st, [&] { cqr::launch_apply(P, ldq, mp, w, s, st); });
}

// One Cholesky-QR pass on the panel P (m' x w): Gram product (+ reduction),
// Cholesky factor and inverse, then P <- P R^{-1}.
void cholqr_pass(cqr_plan_s& p, double* P, int64_t ldq, int w, int pass, double* Rout, int64_t ldr, int panel,
                 const cqr::Scratch& s, hipStream_t st) {
  tn(p, PH_GRAM, P, ldq, P, ldq, w, w, p.mp, s.G, w, nullptr, 0, s, st);
  chol(p, s.G, w, w, pass, Rout, ldr, nullptr, 0, nullptr, panel, s, st, nullptr, P, ldq);
  apply(p, P, ldq, w, s, st);
}

// Panel of w columns starting at column c: leaves of <= kLeaf columns are
// orthogonalised by two Cholesky-QR passes (or column by column in the CGS2,
// ICGS and MGS panel modes); wider panels are split, the right part projected
// (twice) against the left part before being factored.
void factor_panel(cqr_plan_s& p, double* Q, int64_t ldq, double* R, int64_t ldr, int64_t c, int w,
                  int panel, const cqr::Scratch& s, hipStream_t st) {
  const int64_t mp = p.mp;
  if (w <= kLeaf) {
    double* P = Q + c * ldq;
    if (p.cfg.panel != CQR_PANEL_CHOLQR2) {
      colpanel(p, P, ldq, w, R + c + c * ldr, ldr, panel, s, st);
      return;
    }
    cholqr_pass(p, P, ldq, w, 1, nullptr, 0, panel, s, st);
    cholqr_pass(p, P, ldq, w, 2, R + c + c * ldr, ldr, panel, s, st);
    return;
  }
  int h = (w / 2 + 15) / 16 * 16;
  if (h >= w) h = w / 2;
  factor_panel(p, Q, ldq, R, ldr, c, h, panel, s, st);
  for (int pass = 0; pass < 2; ++pass) {
    tn(p, PH_INPANEL, Q + c * ldq, ldq, Q + (c + h) * ldq, ldq, h, w - h, mp, s.S, h, R + c + (c + h) * ldr,
       ldr, s, st);
    nn(p, PH_INPANEL, Q + (c + h) * ldq, ldq, Q + c * ldq, ldq, s.S, h, mp, w - h, h, s, st);
  }
  factor_panel(p, Q, ldq, R, ldr, c + h, w - h, panel, s, st);
}

}  // namespace

extern "C" {

const char* coded_qr_hip_error_name(void) { return hipGetErrorName(t_hip_error); }

const char* coded_qr_status_string(cqr_status s) {
  switch (s) {
    case CQR_OK: return "ok";
    case CQR_EINVAL: return "invalid argument";
    case CQR_ENOTRECOVERABLE: return "not recoverable: more erased blocks than surviving checksums";
    case CQR_ESINGULAR: return "singular generator submatrix";
    case CQR_EHIP: return "HIP runtime error";
    case CQR_ENOMEM: return "out of memory / workspace too small";
    case CQR_EBREAKDOWN: return "panel breakdown: a panel column is zero after projection (rank-deficient input)";
  }
  return "unknown status";
}

cqr_status coded_qr_plan_create(const cqr_config* cfg, const double* v_tilde, const double* gh, cqr_plan* out) {
  if (!out) return CQR_EINVAL;
  *out = nullptr;
  if (!cfg) return CQR_EINVAL;
  const cqr_config& c = *cfg;
  if (c.m <= 0 || c.n <= 0 || c.m < c.n || c.pr <= 0 || c.pc <= 0 || c.b <= 0) return CQR_EINVAL;
  if (c.pr > kMaxGrid || c.pc > kMaxGrid || c.kv < 0 || c.kh < 0 || c.kv > kMaxGen || c.kh > kMaxGen)
    return CQR_EINVAL;
  if (c.pr + c.kv > kMaxLine || c.pc + c.kh > kMaxLine) return CQR_EINVAL;
  if (c.m % c.pr || c.n % c.pc || c.n % c.pr || c.n % c.b) return CQR_EINVAL;
  if (c.kv > 0 && 2 * c.kv > c.pr) return CQR_EINVAL;        // post-orthogonalization needs K_v <= p_r/2
  if (c.kh > c.pc && c.storage == CQR_IN_NODE) return CQR_EINVAL;
  if (c.storage != CQR_OUT_OF_NODE && c.storage != CQR_IN_NODE) return CQR_EINVAL;
  if (c.precision != CQR_FP64 && c.precision != CQR_TRAIL_FP32 && c.precision != CQR_TRAIL_BF16X3) return CQR_EINVAL;
  if (c.panel < CQR_PANEL_CHOLQR2 || c.panel > CQR_PANEL_MGS) return CQR_EINVAL;
  if (!(c.icgs_eta >= 0.0 && c.icgs_eta <= 1.0)) return CQR_EINVAL;   // also rejects NaN
  if (c.lookahead != 0 && c.lookahead != 1) return CQR_EINVAL;
  if (c.kv > 0 && !v_tilde) return CQR_EINVAL;
  if (c.kh > 0 && !gh) return CQR_EINVAL;
  if (c.m > (int64_t)1 << 31 || c.n > (int64_t)1 << 30) return CQR_EINVAL;

  cqr_plan_s* p = new (std::nothrow) cqr_plan_s();
  if (!p) return CQR_ENOMEM;
  p->cfg = c;
  p->eta = c.icgs_eta > 0.0 ? c.icgs_eta : 1.0 / std::sqrt(2.0);
  p->bs = c.m / c.pr;
  p->bw = c.n / c.pc;
  p->hr = c.n / c.pr;
  p->mp = c.m + c.kv * p->bs;
  p->rcode = c.kh == 0 && c.kv > 0;
  p->rrows = c.n + (p->rcode ? (int64_t)c.kv * p->hr : 0);
  p->N = c.n + c.kh * p->bw;

  // Q-side generator: G~_v = [G~_1  V~],  G~_1 = -1/2 V~ V~^T.
  const int pr = c.pr, kv = c.kv, pc = c.pc, kh = c.kh;
  p->gv.assign((size_t)kv * pr, 0.0);
  for (int a = 0; a < kv; ++a) {
    for (int t = 0; t < pr - kv; ++t) p->gv[a * pr + kv + t] = v_tilde[a * (pr - kv) + t];
    for (int b2 = 0; b2 < kv; ++b2) {
      double s = 0.0;
      for (int t = 0; t < pr - kv; ++t) s += v_tilde[a * (pr - kv) + t] * v_tilde[b2 * (pr - kv) + t];
      p->gv[a * pr + b2] = -0.5 * s;
    }
  }
  // R-side generator; in-node storage excludes the storing column.
  p->gh.assign((size_t)pc * kh, 0.0);
  for (int t = 0; t < pc; ++t)
    for (int k = 0; k < kh; ++k) p->gh[t * kh + k] = gh[t * kh + k];
  if (c.storage == CQR_IN_NODE)
    for (int k = 0; k < kh; ++k) p->gh[(k % pc) * kh + k] = 0.0;
  p->ftol = tolerated(*p);

  // Workspace layout.
  const int64_t n = c.n, b = c.b, N = p->N;
  int64_t maxTiles = 1;
  auto tiles = [](int64_t M, int64_t Nc) { return ((M + kTile - 1) / kTile) * ((Nc + kTile - 1) / kTile); };
  maxTiles = std::max(maxTiles, tiles(b, N - b));          // trailing update
  maxTiles = std::max(maxTiles, tiles(n - b, b));          // re-projection
  maxTiles = std::max(maxTiles, tiles(b, b));              // within-panel projection, Gram
  // four partial tiles per output tile: large products split up to ~1280
  // workgroups (32 KB per partial tile)
  p->npart = std::max<int64_t>(1024, 4 * maxTiles);
  p->nS = std::max<int64_t>(n * b, (int64_t)kLeaf * kLeaf);   // S with the fused Gram rows: c1 x b, c1 <= n
  p->ninfo = 64 + (int)(n / b);
  size_t off = align256(sizeof(int) * (size_t)p->ninfo);
  p->off_part = off;  off = align256(off + sizeof(double) * (size_t)p->npart * kTile * kTile);
  p->off_part2 = off; off = align256(off + sizeof(double) * (size_t)p->npart * kTile * kTile);
  p->off_S = off;    off = align256(off + sizeof(double) * (size_t)p->nS);
  p->off_G = off;    off = align256(off + sizeof(double) * 2 * kLeaf * kLeaf);
  p->off_T = off;    off = align256(off + sizeof(double) * kLeaf * kLeaf);
  p->off_R1 = off;   off = align256(off + sizeof(double) * kLeaf * kLeaf);
  p->off_T2 = off;   off = align256(off + sizeof(double) * kLeaf * kLeaf);
  p->off_colw = off; off = align256(off + sizeof(double) * (size_t)cqr::kColWorkDoubles);
  if (b <= kLeaf) {
    // two copies of a first-pass panel (even leading dimension, 256-byte
    // aligned each) for the update that starts before the second pass
    p->ldx = (p->mp + 1) / 2 * 2;
    p->xstride = (int64_t)(align256(sizeof(double) * (size_t)(p->ldx * b)) / sizeof(double));
    p->off_X = off;  off = align256(off + sizeof(double) * 2 * (size_t)p->xstride);
  }
  p->ws_bytes = off;

  *out = p;
  return CQR_OK;
}

void coded_qr_plan_destroy(cqr_plan p) {
  if (!p) return;
  prof_clear(*p);
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  side_release(*p);
  delete p;
}

cqr_status coded_qr_profile_enable(cqr_plan p, int32_t enable) {
  if (!p) return CQR_EINVAL;
  prof_clear(*p);
  p->prof = enable != 0;
  return CQR_OK;
}

cqr_status coded_qr_profile_read(cqr_plan p, int32_t phase, double* total_ms, int64_t* launches, double* flops,
                                 double* bytes) {
  if (!p || phase < 0 || phase >= CQR_NPHASES) return CQR_EINVAL;
  double ms = 0.0, fl = 0.0, by = 0.0;
  int64_t cnt = 0;
  for (auto& r : p->recs) {
    if (r.phase != phase) continue;
    if (!r.a || !r.b) return hip_fail(hipErrorInvalidResourceHandle);
    hipError_t he = hipEventSynchronize(r.b);
    if (he != hipSuccess) return hip_fail(he);
    float e = 0.f;
    he = hipEventElapsedTime(&e, r.a, r.b);
    if (he != hipSuccess) return hip_fail(he);
    ms += e;
    fl += r.flops;
    by += r.bytes;
    ++cnt;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = cnt;
  if (flops) *flops = fl;
  if (bytes) *bytes = by;
  return CQR_OK;
}

cqr_status coded_qr_plan_generators(cqr_plan p, double* gv, double* gh) {
  if (!p) return CQR_EINVAL;
  if (gv) std::memcpy(gv, p->gv.data(), p->gv.size() * sizeof(double));
  if (gh) std::memcpy(gh, p->gh.data(), p->gh.size() * sizeof(double));
  return CQR_OK;
}

int32_t coded_qr_plan_ftol(cqr_plan p) { return p ? p->ftol : -1; }

cqr_status coded_qr_plan_placement(cqr_plan p, int32_t* qrow, int32_t* rcol) {
  if (!p) return CQR_EINVAL;
  const bool in = p->cfg.storage == CQR_IN_NODE;
  if (qrow)
    for (int k = 0; k < p->cfg.kv; ++k) qrow[k] = in ? k % p->cfg.pr : p->cfg.pr + k;
  if (rcol)
    for (int k = 0; k < p->cfg.kh; ++k) rcol[k] = in ? k % p->cfg.pc : p->cfg.pc + k;
  return CQR_OK;
}

int64_t coded_qr_plan_r_rows(cqr_plan p) { return p ? p->rrows : 0; }

size_t coded_qr_workspace_bytes(cqr_plan p) { return p ? p->ws_bytes : 0; }

cqr_status coded_qr_encode(cqr_plan p, double* At, int64_t ldat, hipStream_t st) {
  drop_pending_error();
  if (!p || !At || ldat < p->mp) return CQR_EINVAL;
  if (p->cfg.kv == 0 && p->cfg.kh == 0) return CQR_OK;
  cqr::EncodeArgs a{};
  a.At = At; a.ld = ldat;
  a.m = p->cfg.m; a.n = p->cfg.n; a.bs = p->bs; a.bw = p->bw;
  a.pr = p->cfg.pr; a.pc = p->cfg.pc; a.kv = p->cfg.kv; a.kh = p->cfg.kh;
  for (size_t e = 0; e < p->gv.size(); ++e) a.g[e] = p->gv[e];
  for (int l = 0; l < a.kh; ++l)
    for (int t = 0; t < a.pc; ++t) a.gc[l * cqr::kMaxGrid + t] = p->gh[t * a.kh + l];
  // one pass: A read once, every checksum element written once (without a
  // column code, e.g. a p_r x 1 grid, the checksum rows alone)
  const double m = (double)a.m, n = (double)a.n, c = (double)a.kv * a.bs, d = (double)a.kh * a.bw;
  prof(*p, PH_ENCODE, 2.0 * (c * a.pr * n + (m + c) * a.pc * d), 8.0 * (m * n + c * n + m * d + c * d), st, [&] {
    if (a.kh > 0)
      cqr::launch_encode_fused(a, st);
    else
      cqr::launch_encode_rows(a, st);
  });
  return hip_status();
}

cqr_status coded_qr_factor(cqr_plan p, double* Q, int64_t ldq, double* R, int64_t ldr, int32_t pb, int32_t pe,
                           void* ws, size_t ws_bytes, hipStream_t st) {
  drop_pending_error();
  if (!p || !Q || !R || !ws) return CQR_EINVAL;
  const int64_t n = p->cfg.n, b = p->cfg.b, N = p->N, mp = p->mp;
  const int npan = (int)(n / b);
  if (ldq < mp || ldr < p->rrows || pb < 0 || pe > npan || pb > pe) return CQR_EINVAL;
  if (ws_bytes < p->ws_bytes || (reinterpret_cast<uintptr_t>(ws) & 255)) return CQR_ENOMEM;
  cqr::Scratch s = scratch_of(*p, ws);
  const cqr::Scratch s2 = scratch_of(*p, ws, true);
  if (pb == 0) {
    prof(*p, PH_OTHER, 0.0, 4.0 * p->ninfo, st, [&] { cqr::launch_zero_ints(s.info, p->ninfo, st); });
    prof(*p, PH_OTHER, 0.0, 8.0 * n * N, st, [&] { cqr::launch_fill_zero(R, ldr, n, N, st); });
  }
  const bool la = p->cfg.lookahead && pe - pb > 1 && side_ready(*p);
  const hipStream_t caller = st;
  if (la) {
    // both lookahead streams start after everything already queued on the
    // caller's stream; the chain runs on its own stream from here on
    hipError_t e = hipEventRecord(p->ev_main, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->chain, p->ev_main, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev_main, 0);
    if (e != hipSuccess) return hip_fail(e);
    st = p->chain;
  }
  // Mixed precision: the coefficient products R_bar = Qbar^T Q_t of the
  // trailing update (and of the early update) run on FP32 MFMA, or as
  // split-BF16 products on BF16 MFMA (FP32 where the product's shape does
  // not suit the split kernel).  Every column
  // operation on the encoded matrix -- the rank-b update Q_t -= Qbar R_bar, the
  // re-projection, the panel transforms -- stays FP64: a column operation
  // applied with the same coefficients to every row keeps Q_2 = G_v Q_1 to
  // FP64 rounding whatever the coefficients are, and R records exactly the
  // coefficients applied, so A~ = Q~ R holds to FP64 rounding as well.  The
  // FP32 error of R_bar leaves components of Qbar in the trailing columns;
  // the next panels' FP64 re-projection removes them and adds their
  // coefficients into R.
  const int lowp = p->cfg.precision == CQR_TRAIL_FP32 ? 1 : p->cfg.precision == CQR_TRAIL_BF16X3 ? 2 : 0;
  // Panel k's update of columns [from, to):  R_bar = Qbar^T Q_t -> R[panel, from:];  Q_t -= Qbar R_bar
  auto trail = [&](int64_t c0, int64_t from, int64_t to, const cqr::Scratch& sc, hipStream_t ss) {
    double* Rb = R + c0 + from * ldr;
    const double* P = Q + c0 * ldq;
    tn(*p, PH_TRAIL_TN, P, ldq, Q + from * ldq, ldq, (int)b, (int)(to - from), mp, Rb, ldr, nullptr, 0, sc, ss, -1,
       lowp);
    nn(*p, PH_TRAIL_NN, Q + from * ldq, ldq, P, ldq, Rb, ldr, mp, (int)(to - from), (int)b, sc, ss);
  };
  bool deferred = false;       // a wide panel's update of the columns after the next panel, not yet forked
  int64_t def_c0 = 0, def_from = 0;
  bool side_pending = false;   // ev_side marks side-stream work the chain has not waited for
  bool side_tail = false;      // side-stream work queued after the last ev_side record
  // the chain waits for the side stream's update of the next panel's columns
  auto join_side = [&]() -> hipError_t {
    if (!side_pending) return hipSuccess;
    side_pending = false;
    return hipStreamWaitEvent(st, p->ev_side, 0);
  };
  // the chain waits for everything queued on the side stream
  auto join_side_all = [&]() -> hipError_t {
    if (side_tail) {
      if (hipError_t e = hipEventRecord(p->ev_side, p->side); e != hipSuccess) return e;
      side_pending = true;
      side_tail = false;
    }
    return join_side();
  };
  // panel k's update of columns [c1 + b, N) on the side stream
  auto fork_side = [&](int64_t c0, int64_t from) -> hipError_t {
    hipError_t e = hipEventRecord(p->ev_main, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev_main, 0);
    if (e != hipSuccess) return e;
    trail(c0, from, N, s2, p->side);
    e = hipEventRecord(p->ev_side, p->side);
    if (e == hipSuccess) {
      side_pending = true;
      side_tail = false;
    }
    return e;
  };
  for (int k = pb; k < pe; ++k) {
    const int64_t c0 = (int64_t)k * b, c1 = c0 + b;
    double* P = Q + c0 * ldq;
    const bool next = la && k + 1 < pe;     // panel k+1 is factored in this call
    if (b <= kLeaf && p->cfg.panel == CQR_PANEL_CHOLQR2) {
      // First Cholesky-QR pass.  With re-projection its Gram matrix comes from
      // the same product as the coefficients, [Q[:, :c0] | P]^T P: since the
      // re-projection coefficients S are at rounding level, P^T P equals the
      // Gram matrix of the re-projected panel up to rounding, and any residual
      // difference is removed by the second pass.
      const double* W1 = s.G;
      int64_t ldw1 = b;
      bool chol1 = false;   // first Cholesky pass already launched
      // Early update (with the first pass inside the re-projection's
      // launches): panel k's update of the columns [c1 + b, N) starts on the
      // side stream from the first-pass panel P1, which the first pass's
      // transform also stores to X, while the chain runs the second pass.  Its
      // reduction folds in the second pass's R2^{-1} (R_t = R2^{-T} P1^T Q_t =
      // P^T Q_t), and the update Q_t -= P R_t waits for the finished panel P.
      // X alternates between two buffers: the chain writes panel k+1's copy
      // before it waits for panel k's update.
      double* X = (next && c1 + b < N && s.X) ? s.X + (k & 1) * s.xstride : nullptr;
      if (p->cfg.reproject && k > 0) {
        // S = Q[:, :c0]^T P (rows < c0, also added into R[:c0, panel]);  P -= Q[:, :c0] S.
        // The first Cholesky pass needs only the Gram rows and the update only
        // S, so when the update splits over K the Cholesky runs in its launch
        // and the transform P <- P R1^{-1} in its split reduction.
        tn(*p, PH_REPROJ_TN, Q, ldq, P, ldq, (int)c1, (int)b, mp, s.S, c1, R + c0 * ldr, ldr, s, st, (int)c0);
        W1 = s.S + c0;
        ldw1 = c1;
        chol1 = nn_chol(*p, P, ldq, Q, ldq, s.S, c1, mp, (int)b, (int)c0,
                        cqr::chol_args(W1, ldw1, (int)b, 1, nullptr, 0, nullptr, 0, nullptr, k, s), s, st, X, s.ldx);
        if (!chol1) nn(*p, PH_REPROJ_NN, P, ldq, Q, ldq, s.S, c1, mp, (int)b, (int)c0, s, st);
      } else {
        tn(*p, PH_GRAM, P, ldq, P, ldq, (int)b, (int)b, mp, s.G, b, nullptr, 0, s, st);
      }
      if (!chol1) {
        chol(*p, W1, ldw1, (int)b, 1, nullptr, 0, nullptr, 0, nullptr, k, s, st);
        apply(*p, P, ldq, (int)b, s, st);
      }
      const bool early = chol1 && X;
      // (recorded before the chain's wait below, so the side stream's product
      // does not wait for the chain to pass it)
      if (early)
        if (hipError_t e = hipEventRecord(p->ev_main, st); e != hipSuccess) return hip_fail(e);
      // Second pass.  With lookahead the same product also gives
      // X = P1^T Q_next, and the Cholesky kernel forms the next panel's
      // coefficients R[panel, next] = (P1 R2^{-1})^T Q_next = R2^{-T} X.
      // Q_next must first carry panel k-1's update from the side stream.  (The
      // wait is queued before panel k's early update records its own event.)
      if (hipError_t e = join_side(); e != hipSuccess) return hip_fail(e);
      cqr::TnArgs ea{};
      if (early) {
        if (hipError_t e = hipStreamWaitEvent(p->side, p->ev_main, 0); e != hipSuccess) return hip_fail(e);
        ea = tn_early(*p, X, s.ldx, Q + (c1 + b) * ldq, ldq, (int)b, (int)(N - c1 - b), s2, p->side, lowp);
      }
      tn(*p, PH_GRAM, P, ldq, P, ldq, (int)b, next ? 2 * (int)b : (int)b, mp, s.G, b, nullptr, 0, s, st);
      chol(*p, s.G, b, (int)b, 2, R + c0 + c0 * ldr, ldr, next ? s.G + b * b : nullptr, b,
           next ? R + c0 + c1 * ldr : nullptr, k, s, st, early ? s.T2 : nullptr, P, ldq, early ? s.fb + k : nullptr);
      // P <- P1 R2^{-1}, and with lookahead Q_next -= P R[panel, next] (one
      // launch)
      const bool fused = next &&
                         apply_update(*p, Q + c1 * ldq, ldq, P, ldq, R + c0 + c1 * ldr, ldr, (int)b, s, st);
      if (!fused) apply(*p, P, ldq, (int)b, s, st);
      if (next) {
        if (!fused)
          nn(*p, PH_TRAIL_NN, Q + c1 * ldq, ldq, P, ldq, R + c0 + c1 * ldr, ldr, mp, (int)b, (int)b, s, st);
        if (early) {
          // the early update's reduction and rank-b update, after the panel
          hipError_t e = hipEventRecord(p->ev_apply, st);
          if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev_apply, 0);
          if (e != hipSuccess) return hip_fail(e);
          // The next panel's chain needs only panel k+2's columns from this
          // update: they are updated first and marked by ev_side, and the
          // columns after them are updated while the chain moves on (the
          // chain touches them only after join_side_all).
          double* Rb = R + c0 + (c1 + b) * ldr;
          tn_tmul(*p, ea, s.T2, (int)b, Rb, ldr, p->side, s.fb + k, P, ldq);
          const int64_t near = std::min<int64_t>(b, N - c1 - b);
          nn(*p, PH_TRAIL_NN, Q + (c1 + b) * ldq, ldq, P, ldq, Rb, ldr, mp, (int)near, (int)b, s2, p->side);
          e = hipEventRecord(p->ev_side, p->side);
          if (e != hipSuccess) return hip_fail(e);
          side_pending = true;
          if (c1 + b + near < N) {
            nn(*p, PH_TRAIL_NN, Q + (c1 + b + near) * ldq, ldq, P, ldq, Rb + near * ldr, ldr, mp,
               (int)(N - c1 - b - near), (int)b, s2, p->side);
            side_tail = true;
          }
        } else if (c1 + b < N) {
          // the remaining columns on the side stream
          if (hipError_t e = fork_side(c0, c1 + b); e != hipSuccess) return hip_fail(e);
        }
      } else if (c1 < N) {
        if (hipError_t e = join_side_all(); e != hipSuccess) return hip_fail(e);
        trail(c0, c1, N, s, st);
      }
      continue;
    }
    // Panels wider than a Cholesky-QR leaf, and every panel of the
    // column-wise modes: re-projection, recursive panel, then the update (the
    // next panel's columns first with lookahead).
    if (p->cfg.reproject && k > 0) {
      tn(*p, PH_REPROJ_TN, Q, ldq, P, ldq, (int)c0, (int)b, mp, s.S, c0, R + c0 * ldr, ldr, s, st);
      nn(*p, PH_REPROJ_NN, P, ldq, Q, ldq, s.S, c0, mp, (int)b, (int)c0, s, st);
    }
    // With lookahead the previous panel's update of the columns after this
    // panel starts only here, behind this panel's re-projection: the two
    // large products run one after the other instead of sharing the GPU, and
    // the update overlaps this panel's factorization, whose kernels are small.
    if (deferred) {
      if (hipError_t e = fork_side(def_c0, def_from); e != hipSuccess) return hip_fail(e);
      deferred = false;
    }
    factor_panel(*p, Q, ldq, R, ldr, c0, (int)b, k, s, st);
    if (c1 >= N) continue;
    if (hipError_t e = join_side_all(); e != hipSuccess) return hip_fail(e);
    if (next && c1 + b < N) {
      trail(c0, c1, c1 + b, s, st);
      deferred = true;
      def_c0 = c0;
      def_from = c1 + b;
    } else {
      trail(c0, c1, N, s, st);
    }
  }
  if (deferred)
    if (hipError_t e = fork_side(def_c0, def_from); e != hipSuccess) return hip_fail(e);
  if (hipError_t e = join_side_all(); e != hipSuccess) return hip_fail(e);
  if (la) {
    // the caller's stream waits for the chain (which has joined the updates)
    hipError_t e = hipEventRecord(p->ev_chain, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(caller, p->ev_chain, 0);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (p->rcode) {
    // R's checksum rows: the vertical code of its block rows, encoded at the
    // panel boundary where this call ends (where failures are injected); R's
    // entries become final only column block by column block, because each
    // panel's re-projection adds into earlier rows
    cqr::EncodeArgs a{};
    a.At = R; a.ld = ldr;
    a.m = n; a.n = N; a.bs = p->hr; a.bw = p->bw;
    a.pr = p->cfg.pr; a.pc = p->cfg.pc; a.kv = p->cfg.kv; a.kh = 0;
    for (size_t e = 0; e < p->gv.size(); ++e) a.g[e] = p->gv[e];
    const double c = (double)a.kv * a.bs;
    prof(*p, PH_ENCODE, 2.0 * c * a.pr * N, 8.0 * (n + c) * N, caller, [&] { cqr::launch_encode_rows(a, caller); });
  }
  return hip_status();
}

cqr_status coded_qr_ws_info(cqr_plan p, const void* ws, hipStream_t st, int32_t* info) {
  if (!p || !ws || !info) return CQR_EINVAL;
  hipError_t he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(he);
  int32_t v = 0;
  he = hipMemcpy(&v, ws, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return hip_fail(he);
  *info = v;
  return v ? CQR_EBREAKDOWN : CQR_OK;
}

cqr_status coded_qr_ws_panel_fallbacks(cqr_plan p, const void* ws, hipStream_t st, int32_t* count) {
  if (!p || !ws || !count) return CQR_EINVAL;
  hipError_t he = hipStreamSynchronize(st);
  if (he != hipSuccess) return hip_fail(he);
  int32_t v = 0;
  he = hipMemcpy(&v, static_cast<const int32_t*>(ws) + 2, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return hip_fail(he);
  *count = v;
  return CQR_OK;
}

cqr_status coded_qr_erase(cqr_plan p, double* Q, int64_t ldq, double* R, int64_t ldr, const int32_t* ij,
                          int32_t nf, hipStream_t st) {
  drop_pending_error();
  if (!p || !Q || !R || ldq < p->mp || ldr < p->rrows) return CQR_EINVAL;
  cqr_status cs = check_nodes(*p, ij, nf);
  if (cs != CQR_OK) return cs;
  std::set<std::pair<int, int>> qs, rs;
  for (int f = 0; f < nf; ++f) {
    std::vector<std::pair<int, int>> q, r;
    node_blocks(*p, ij[2 * f], ij[2 * f + 1], q, r);
    qs.insert(q.begin(), q.end());
    rs.insert(r.begin(), r.end());
  }
  auto flush = [&](double* base, int64_t ld, int rows, int cols, std::vector<int64_t>& offs) {
    for (size_t i = 0; i < offs.size(); i += 64) {
      cqr::EraseArgs a{};
      a.base = base; a.ld = ld; a.rows = rows; a.cols = cols;
      a.nblk = (int)std::min<size_t>(64, offs.size() - i);
      for (int k = 0; k < a.nblk; ++k) a.off[k] = offs[i + k];
      prof(*p, PH_ERASE, 0.0, 8.0 * rows * cols * a.nblk, st, [&] { cqr::launch_erase(a, st); });
    }
  };
  std::vector<int64_t> qo, ro;
  for (auto& q : qs) qo.push_back(q.first * p->bs + (int64_t)q.second * p->bw * ldq);
  for (auto& r : rs) ro.push_back(r.first * p->hr + (int64_t)r.second * p->bw * ldr);
  flush(Q, ldq, (int)p->bs, (int)p->bw, qo);
  flush(R, ldr, (int)p->hr, (int)p->bw, ro);
  return hip_status();
}

cqr_status coded_qr_recover(cqr_plan p, double* Q, int64_t ldq, double* R, int64_t ldr, const int32_t* ij,
                            int32_t nf, hipStream_t st) {
  drop_pending_error();
  if (!p || !Q || !R || ldq < p->mp || ldr < p->rrows) return CQR_EINVAL;
  cqr_status cs = check_nodes(*p, ij, nf);
  if (cs != CQR_OK) return cs;
  const int pr = p->cfg.pr, pc = p->cfg.pc, kv = p->cfg.kv, kh = p->cfg.kh;
  std::set<std::pair<int, int>> qs, rs;
  for (int f = 0; f < nf; ++f) {
    std::vector<std::pair<int, int>> q, r;
    node_blocks(*p, ij[2 * f], ij[2 * f + 1], q, r);
    qs.insert(q.begin(), q.end());
    rs.insert(r.begin(), r.end());
  }
  std::vector<cqr::LineArgs> launches;
  // Q: every block column J, vertical code  chk_k = sum_t g~_v[k][t] data_t.
  for (int J = 0; J < pc + kh; ++J) {
    LineJob job;
    for (int I = 0; I < pr; ++I) if (qs.count({I, J})) job.lost_d.push_back(I);
    for (int k = 0; k < kv; ++k) if (qs.count({pr + k, J})) job.lost_c.push_back(k);
    if (job.lost_d.empty() && job.lost_c.empty()) continue;
    std::vector<int> srcs, outs;
    std::vector<double> coef;
    cs = plan_line(p->gv, pr, kv, job, srcs, outs, coef);
    if (cs != CQR_OK) return cs;
    auto off = [&](int slot) { return (int64_t)slot * p->bs + (int64_t)J * p->bw * ldq; };
    const int ns = (int)srcs.size();
    for (size_t o0 = 0; o0 < outs.size(); o0 += kMaxOut) {
      cqr::LineArgs a{};
      a.base = Q; a.ld = ldq; a.rows = (int)p->bs; a.cols = (int)p->bw;
      a.nsrc = ns;
      a.nout = (int)std::min<size_t>(kMaxOut, outs.size() - o0);
      for (int s = 0; s < ns; ++s) a.src[s] = off(srcs[s]);
      for (int o = 0; o < a.nout; ++o) {
        a.dst[o] = off(outs[o0 + o]);
        for (int s = 0; s < ns; ++s) a.coef[o][s] = coef[(o0 + o) * ns + s];
      }
      launches.push_back(a);
    }
  }
  // R without a horizontal code: every block column J, the vertical code of
  // R's block rows (the same generator as Q's).
  if (p->rcode && !rs.empty()) {
    for (int J = 0; J < pc; ++J) {
      LineJob job;
      for (int I = 0; I < pr; ++I) if (rs.count({I, J})) job.lost_d.push_back(I);
      for (int k = 0; k < kv; ++k) if (rs.count({pr + k, J})) job.lost_c.push_back(k);
      if (job.lost_d.empty() && job.lost_c.empty()) continue;
      std::vector<int> srcs, outs;
      std::vector<double> coef;
      cs = plan_line(p->gv, pr, kv, job, srcs, outs, coef);
      if (cs != CQR_OK) return cs;
      auto off = [&](int slot) { return (int64_t)slot * p->hr + (int64_t)J * p->bw * ldr; };
      const int ns = (int)srcs.size();
      for (size_t o0 = 0; o0 < outs.size(); o0 += kMaxOut) {
        cqr::LineArgs a{};
        a.base = R; a.ld = ldr; a.rows = (int)p->hr; a.cols = (int)p->bw;
        a.nsrc = ns;
        a.nout = (int)std::min<size_t>(kMaxOut, outs.size() - o0);
        for (int s = 0; s < ns; ++s) a.src[s] = off(srcs[s]);
        for (int o = 0; o < a.nout; ++o) {
          a.dst[o] = off(outs[o0 + o]);
          for (int s = 0; s < ns; ++s) a.coef[o][s] = coef[(o0 + o) * ns + s];
        }
        launches.push_back(a);
      }
    }
  }
  // R: every block row i, horizontal code  chk_k = sum_t g~_h[t][k] data_t.
  if (!rs.empty() && !p->rcode) {
    std::vector<double> genT((size_t)kh * pc);
    for (int k = 0; k < kh; ++k)
      for (int t = 0; t < pc; ++t) genT[(size_t)k * pc + t] = p->gh[t * kh + k];
    for (int i = 0; i < pr; ++i) {
      LineJob job;
      for (int J = 0; J < pc; ++J) if (rs.count({i, J})) job.lost_d.push_back(J);
      for (int k = 0; k < kh; ++k) if (rs.count({i, pc + k})) job.lost_c.push_back(k);
      if (job.lost_d.empty() && job.lost_c.empty()) continue;
      std::vector<int> srcs, outs;
      std::vector<double> coef;
      cs = plan_line(genT, pc, kh, job, srcs, outs, coef);
      if (cs != CQR_OK) return cs;
      auto off = [&](int slot) { return (int64_t)i * p->hr + (int64_t)slot * p->bw * ldr; };
      const int ns = (int)srcs.size();
      for (size_t o0 = 0; o0 < outs.size(); o0 += kMaxOut) {
        cqr::LineArgs a{};
        a.base = R; a.ld = ldr; a.rows = (int)p->hr; a.cols = (int)p->bw;
        a.nsrc = ns;
        a.nout = (int)std::min<size_t>(kMaxOut, outs.size() - o0);
        for (int s = 0; s < ns; ++s) a.src[s] = off(srcs[s]);
        for (int o = 0; o < a.nout; ++o) {
          a.dst[o] = off(outs[o0 + o]);
          for (int s = 0; s < ns; ++s) a.coef[o][s] = coef[(o0 + o) * ns + s];
        }
        launches.push_back(a);
      }
    }
  }
  for (const auto& a : launches) {
    const double el = (double)a.rows * a.cols;
    prof(*p, PH_RECOVER, 2.0 * el * a.nsrc * a.nout, 8.0 * el * (a.nsrc + a.nout), st,
         [&] { cqr::launch_line(a, st); });
  }
  return hip_status();
}

cqr_status coded_qr_postorth(cqr_plan p, const double* Q, int64_t ldq, double* Qpost, int64_t ldqp,
                             const double* B, int64_t ldb, double* Bpost, int64_t ldbp, int32_t nrhs,
                             hipStream_t st) {
  drop_pending_error();
  if (!p || !Q || !Qpost || p->cfg.kv == 0 || nrhs < 0) return CQR_EINVAL;
  const int64_t m = p->cfg.m;
  if (ldq < m || ldqp < m) return CQR_EINVAL;
  if (nrhs > 0 && (!B || !Bpost || ldb < m || ldbp < m)) return CQR_EINVAL;
  cqr::PostArgs a{};
  a.pr = p->cfg.pr; a.kv = p->cfg.kv; a.bs = p->bs;
  for (size_t e = 0; e < p->gv.size(); ++e) a.gv[e] = p->gv[e];
  const double pr = p->cfg.pr, kv = p->cfg.kv;
  const double fl_el = 2.0 * (kv * pr + (pr - kv) * (kv + 1)) / pr;   // flops per element
  a.src = Q; a.lds = ldq; a.dst = Qpost; a.ldd = ldqp; a.cols = p->cfg.n;
  prof(*p, PH_POST, fl_el * m * a.cols, 16.0 * m * a.cols, st, [&] { cqr::launch_postorth(a, st); });
  if (nrhs > 0) {
    a.src = B; a.lds = ldb; a.dst = Bpost; a.ldd = ldbp; a.cols = nrhs;
    prof(*p, PH_POST, fl_el * m * nrhs, 16.0 * m * nrhs, st, [&] { cqr::launch_postorth(a, st); });
  }
  return hip_status();
}

size_t coded_qr_solve_workspace_bytes(cqr_plan p, int32_t nrhs) {
  if (!p || nrhs < 1) return 0;
  const int64_t n = p->cfg.n, nb = (n + 63) / 64;
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  return up(8 * (size_t)nb * 64 * 64) + up(8 * (size_t)n * nrhs);
}

cqr_status coded_qr_solve(cqr_plan p, const double* Qpost, int64_t ldqp, const double* R, int64_t ldr,
                          const double* Bpost, int64_t ldbp, int32_t nrhs, double* X, int64_t ldx, void* ws,
                          size_t ws_bytes, hipStream_t st) {
  drop_pending_error();
  if (!p || !Qpost || !R || !Bpost || !X || !ws || nrhs < 1) return CQR_EINVAL;
  const int64_t m = p->cfg.m, n = p->cfg.n, nb = (n + 63) / 64;
  if (ldqp < m || ldr < n || ldbp < m || ldx < n) return CQR_EINVAL;
  if (ws_bytes < coded_qr_solve_workspace_bytes(p, nrhs) || (reinterpret_cast<uintptr_t>(ws) & 255))
    return CQR_ENOMEM;
  double* T = static_cast<double*>(ws);
  double* Y = T + ((8 * (size_t)nb * 64 * 64 + 255) & ~size_t(255)) / 8;
  // inverses of the 64 x 64 diagonal blocks of R_1, all at once
  prof(*p, PH_SOLVE, nb * 64.0 * 64 * 64 / 3, 8.0 * (n * 64.0 + nb * 64.0 * 64), st,
       [&] { cqr::launch_trinv(R, ldr, n, T, st); });
  // Y = Qpost^T Bpost
  prof(*p, PH_SOLVE, 2.0 * m * n * nrhs, 8.0 * (m * n + m * nrhs + n * nrhs), st,
       [&] { cqr::launch_gemv_t(Qpost, ldqp, m, (int)n, Bpost, ldbp, nrhs, Y, n, st); });
  // R_1 X = Y, 64-row blocks from the bottom
  for (int64_t k0 = (nb - 1) * 64; k0 >= 0; k0 -= 64) {
    const int w = (int)std::min<int64_t>(64, n - k0);
    prof(*p, PH_SOLVE, 2.0 * (64.0 * w + k0 * w) * nrhs, 8.0 * (k0 * w + 64.0 * 64 + 2.0 * (k0 + w) * nrhs), st,
         [&] { cqr::launch_trsv_step(R, ldr, T, Y, n, X, ldx, nrhs, k0, w, st); });
  }
  return hip_status();
}

cqr_status coded_qr_solve_noalloc(cqr_plan p, const double* Qpost, int64_t ldqp, const double* R, int64_t ldr,
                                  const double* Bpost, int64_t ldbp, int32_t nrhs, double* X, int64_t ldx,
                                  hipStream_t st) {
  drop_pending_error();
  if (!p || !Qpost || !R || !Bpost || !X || nrhs < 1) return CQR_EINVAL;
  const size_t need = coded_qr_solve_workspace_bytes(p, nrhs);
  if (need > cqr::kSolveScratchBytes) return CQR_ENOMEM;
  void* ws = nullptr;
  if (hipError_t e = cqr::solve_scratch(&ws); e != hipSuccess) return hip_fail(e);
  return coded_qr_solve(p, Qpost, ldqp, R, ldr, Bpost, ldbp, nrhs, X, ldx, ws, cqr::kSolveScratchBytes, st);
}

}  // extern "C"

namespace {

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Rinv = R_1^{-1} (n x n, ld n) by recursive doubling: the 64 x 64 diagonal
// blocks are inverted at once and laid out as a block-diagonal Rinv; then,
// for h = 64, 128, 256, ..., every pair of adjacent h-blocks [i, i+h) and
// [i+h, i+2h) gets its off-diagonal block T12 = -T11 R12 T22 from the two
// inverted diagonal blocks (W = R12 T22 into Wtmp, then T12 -= T11 W), on the
// MFMA update kernels: n^3/3 flops in products (s: the split partials).
void upper_inverse(cqr_plan_s& p, const double* R, int64_t ldr, double* Rinv, double* Wtmp, double* T,
                   const cqr::Scratch& s, hipStream_t st) {
  const int64_t n = p.cfg.n, nb = (n + 63) / 64;
  prof(p, PH_ADJOINT, nb * 64.0 * 64 * 64 / 3, 8.0 * (n * 64.0 + nb * 64.0 * 64), st,
       [&] { cqr::launch_trinv(R, ldr, n, T, st); });
  prof(p, PH_ADJOINT, 0.0, 8.0 * n * n, st, [&] { cqr::launch_blockdiag(T, Rinv, n, n, st); });
  for (int64_t h = 64; h < n; h *= 2) {
    for (int64_t i = 0; i + h < n; i += 2 * h) {
      const int64_t h2 = std::min(h, n - i - h);
      const double* R12 = R + i + (i + h) * ldr;
      const double* T11 = Rinv + i + i * n;
      const double* T22 = Rinv + (i + h) + (i + h) * n;
      double* T12 = Rinv + i + (i + h) * n;
      // Wtmp = -R12 T22, negated to R12 T22; T12 (zero) -= T11 Wtmp
      prof(p, PH_ADJOINT, 0.0, 8.0 * h * h2, st, [&] { cqr::launch_fill_zero(Wtmp, h, h, h2, st); });
      nn(p, PH_ADJOINT, Wtmp, h, R12, ldr, T22, n, h, (int)h2, (int)h2, s, st);
      prof(p, PH_ADJOINT, 0.0, 16.0 * h * h2, st, [&] { cqr::launch_scale(Wtmp, h, h, h2, -1.0, st); });
      nn(p, PH_ADJOINT, T12, n, T11, n, Wtmp, h, h, (int)h2, (int)h, s, st);
    }
  }
}

}  // namespace

extern "C" {

size_t coded_qr_backward_workspace_bytes(cqr_plan p) {
  if (!p) return 0;
  const size_t n = (size_t)p->cfg.n, mp = (size_t)p->mp, nb = (n + 63) / 64;
  return up256(p->ws_bytes) + 3 * up256(8 * n * n) + up256(8 * nb * 64 * 64) + 2 * up256(8 * mp * n);
}

cqr_status coded_qr_backward(cqr_plan p, const double* Q, int64_t ldq, const double* R, int64_t ldr,
                             const double* dQ, int64_t lddq, const double* dR, int64_t lddr, double* dA,
                             int64_t ldda, void* ws, size_t ws_bytes, hipStream_t st) {
  drop_pending_error();
  if (!p || !Q || !R || !dQ || !dR || !dA || !ws) return CQR_EINVAL;
  const int64_t m = p->cfg.m, n = p->cfg.n, mp = p->mp, nb = (n + 63) / 64;
  if (ldq < mp || ldr < n || lddq < mp || lddr < n || ldda < m) return CQR_EINVAL;
  if (ws_bytes < coded_qr_backward_workspace_bytes(p) || (reinterpret_cast<uintptr_t>(ws) & 255))
    return CQR_ENOMEM;
  const cqr::Scratch s = scratch_of(*p, ws);
  char* w = static_cast<char*>(ws) + up256(p->ws_bytes);
  auto take = [&](size_t bytes) { double* q = reinterpret_cast<double*>(w); w += up256(bytes); return q; };
  double* Rinv = take(8 * (size_t)n * n);
  double* W1 = take(8 * (size_t)n * n);
  double* W2 = take(8 * (size_t)n * n);
  double* T = take(8 * (size_t)nb * 64 * 64);
  double* D = take(8 * (size_t)mp * n);
  double* X = take(8 * (size_t)mp * n);
  const double nn2 = 8.0 * n * n;
  upper_inverse(*p, R, ldr, Rinv, W1, T, s, st);
  // W2 = M1 = Q~^T dQ~
  tn(*p, PH_ADJOINT, Q, ldq, dQ, lddq, (int)n, (int)n, mp, W2, n, nullptr, 0, s, st);
  // W1 = M1^T;  W2 = triu(dR)^T;  W1 -= R W2, so W1 = dQ~^T Q~ - R dR^T = -M
  prof(*p, PH_ADJOINT, 0.0, 2 * nn2, st, [&] { cqr::launch_transpose(W2, n, W1, n, n, n, 1.0, false, st); });
  prof(*p, PH_ADJOINT, 0.0, 2 * nn2, st, [&] { cqr::launch_transpose(dR, lddr, W2, n, n, n, 1.0, true, st); });
  nn(*p, PH_ADJOINT, W1, n, R, ldr, W2, n, n, (int)n, (int)n, s, st);
  // W1 <- copyltu(W1) = -copyltu(M)
  prof(*p, PH_ADJOINT, 0.0, nn2, st, [&] { cqr::launch_copyltu(W1, n, n, st); });
  // D = dQ~ - Q~ W1 = dQ~ + Q~ copyltu(M)
  {
    hipError_t e = hipMemcpy2DAsync(D, 8 * mp, dQ, 8 * lddq, 8 * mp, n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e);
  }
  nn(*p, PH_ADJOINT, D, mp, Q, ldq, W1, n, mp, (int)n, (int)n, s, st);
  // W2 = -R^{-T};  X = 0;  X -= D W2, so X = D R^{-T} = dA~
  prof(*p, PH_ADJOINT, 0.0, 2 * nn2, st, [&] { cqr::launch_transpose(Rinv, n, W2, n, n, n, -1.0, false, st); });
  prof(*p, PH_ADJOINT, 0.0, 8.0 * mp * n, st, [&] { cqr::launch_fill_zero(X, mp, mp, n, st); });
  nn(*p, PH_ADJOINT, X, mp, D, mp, W2, n, mp, (int)n, (int)n, s, st);
  // dA = dA~_top + G_v^T dA~_bottom
  cqr::FoldArgs f{};
  f.X = X; f.ldx = mp; f.dA = dA; f.ldd = ldda;
  f.m = m; f.bs = p->bs; f.cols = n; f.pr = p->cfg.pr; f.kv = p->cfg.kv;
  for (size_t e = 0; e < p->gv.size(); ++e) f.gv[e] = p->gv[e];
  prof(*p, PH_ADJOINT, 2.0 * f.kv * m * n, 8.0 * (mp + m) * n, st, [&] { cqr::launch_fold(f, st); });
  return hip_status();
}

// Split partials of the triangular inverse's products (the update kernels
// split K over at most 512 workgroups).
constexpr int64_t kSolvePartTiles = 1024;

size_t coded_qr_solve_backward_workspace_bytes(cqr_plan p, int32_t nrhs) {
  if (!p || nrhs < 1) return 0;
  const size_t n = (size_t)p->cfg.n, nb = (n + 63) / 64;
  return 2 * up256(8 * n * n) + up256(8 * nb * 64 * 64) + up256(8 * n * (size_t)nrhs) +
         up256(8 * (size_t)kSolvePartTiles * kTile * kTile);
}

cqr_status coded_qr_solve_backward(cqr_plan p, const double* Qpost, int64_t ldqp, const double* R, int64_t ldr,
                                   const double* Bpost, int64_t ldbp, const double* X, int64_t ldx,
                                   const double* dX, int64_t lddx, int32_t nrhs, double* dQ, int64_t lddq,
                                   double* dR, int64_t lddr, double* dB, int64_t lddb, void* ws, size_t ws_bytes,
                                   hipStream_t st) {
  drop_pending_error();
  if (!p || !Qpost || !R || !Bpost || !X || !dX || !dQ || !dR || !dB || !ws || nrhs < 1 || p->cfg.kv == 0)
    return CQR_EINVAL;
  const int64_t m = p->cfg.m, n = p->cfg.n, mp = p->mp, nb = (n + 63) / 64;
  if (ldqp < m || ldr < n || ldbp < m || ldx < n || lddx < n || lddq < mp || lddr < n || lddb < m)
    return CQR_EINVAL;
  if (ws_bytes < coded_qr_solve_backward_workspace_bytes(p, nrhs) || (reinterpret_cast<uintptr_t>(ws) & 255))
    return CQR_ENOMEM;
  char* w = static_cast<char*>(ws);
  auto take = [&](size_t bytes) { double* q = reinterpret_cast<double*>(w); w += up256(bytes); return q; };
  double* Rinv = take(8 * (size_t)n * n);
  double* Ytmp = take(8 * (size_t)n * n);
  double* T = take(8 * (size_t)nb * 64 * 64);
  double* DY = take(8 * (size_t)n * nrhs);
  cqr::Scratch s{};
  s.part = take(8 * (size_t)kSolvePartTiles * kTile * kTile);
  s.npart = kSolvePartTiles;
  upper_inverse(*p, R, ldr, Rinv, Ytmp, T, s, st);
  // dy = R_1^{-T} dX = Rinv^T dX
  prof(*p, PH_ADJOINT, 2.0 * n * n * nrhs, 8.0 * (n * n + 2.0 * n * nrhs), st,
       [&] { cqr::launch_gemv_t(Rinv, n, n, (int)n, dX, lddx, nrhs, DY, n, st); });
  // dR_1 = -triu(dy x^T)
  prof(*p, PH_ADJOINT, 2.0 * n * n * nrhs, 8.0 * n * n, st,
       [&] { cqr::launch_outer(DY, n, X, ldx, n, n, nrhs, -1.0, true, dR, lddr, st); });
  // dQ~[:m] = G_0 (Bpost dy^T), dQ~[m:] = 0
  prof(*p, PH_ADJOINT, 2.0 * m * n * nrhs, 8.0 * m * n, st,
       [&] { cqr::launch_outer(Bpost, ldbp, DY, n, m, n, nrhs, 1.0, false, dQ, lddq, st); });
  cqr::PostArgs a{};
  a.pr = p->cfg.pr; a.kv = p->cfg.kv; a.bs = p->bs;
  for (size_t e = 0; e < p->gv.size(); ++e) a.gv[e] = p->gv[e];
  a.src = dQ; a.lds = lddq; a.dst = dQ; a.ldd = lddq; a.cols = n;
  prof(*p, PH_ADJOINT, 0.0, 16.0 * m * n, st, [&] { cqr::launch_postorth(a, st); });
  prof(*p, PH_ADJOINT, 0.0, 8.0 * (mp - m) * n, st, [&] { cqr::launch_fill_zero(dQ + m, lddq, mp - m, n, st); });
  // dB = G_0 (Qpost dy)
  prof(*p, PH_ADJOINT, 2.0 * m * n * nrhs, 8.0 * (m * n + m * nrhs), st,
       [&] { cqr::launch_gemv_n(Qpost, ldqp, m, (int)n, DY, n, nrhs, dB, lddb, st); });
  a.src = dB; a.lds = lddb; a.dst = dB; a.ldd = lddb; a.cols = nrhs;
  prof(*p, PH_ADJOINT, 0.0, 16.0 * m * nrhs, st, [&] { cqr::launch_postorth(a, st); });
  return hip_status();
}


}  // extern "C"
