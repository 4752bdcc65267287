"""Plain FP64 CPU oracle for coded QR (Nguyen, Weissburg, Jeong: "Coded Computing
for Fault-Tolerant Parallel QR Decomposition", arXiv 2311.11943).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct reference
that the HIP library is checked against.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path never
does.  It shares no code with the HIP library.

Everything is numpy float64 and follows the paper's steps in its notation:

  encode        A -> A~ = [[A, A G_h], [G_v A, G_v A G_h]]      (System Model,
                encoding equation), G = G~ (x) I, checksum blocks formed as the
                linear combination C_ij = sum_t g~_it A_tj   (Sec. Q-factor
                protection, out-of-node construction)
  generators    G~_v = [G~_1  V~], G~_1 = -1/2 V~ V~^T   (Construction of the
                Q-factor checksum generator; in-node variant with K rows);
                R side: any MDS generator, with the storing column excluded for
                in-node storage (Construction "In-Node Systematic MDS Coding")
  factor        blocked Gram-Schmidt (algorithms PBMGS / BMGS): per panel of
                width b, an orthonormal basis of the panel (ICGS/CGS2/MGS), then
                every column right of the panel projected onto the orthogonal
                complement of that basis, the coefficients recorded in R
  recover       erased blocks decoded from surviving blocks and checksums by
                solving the small G_hat system (proof of the recovery-overhead
                lemma), then lost checksum blocks re-encoded
  postorth      G_0 Q_1 and G_0 b with G_0 = [[I + G_1, V], [V^T, -I]]
                (Theorem on low-cost post-orthogonalization)

Readings where the paper is silent or its printed algorithms are garbled (all
listed with reasons in the design notes of the repository):
  * PBMGS stores R_bar into the off-diagonal block R[panel, right of panel]
    (the sequential BMGS statement does so); the update runs whenever any
    column (systematic or carried checksum) lies right of the panel.
  * The CGS listing's update must use the normalised row v^T / sqrt(v_1); the
    panel here is the standard column-wise CGS2 / ICGS.
  * ICGS reorthogonalises a column once when its norm drops below eta times its
    norm before projection (Daniel-Gragg-Kaufman-Stewart test, eta = 1/sqrt 2);
    the paper cites but does not state its criterion.
  * Only the n systematic columns are orthogonalised; the d checksum columns are
    carried as trailing columns, so R is n x (n + d).
  * Optional left re-projection of each panel against all earlier Q columns
    (a column operation, so checksums are preserved); on by default.
  * 2D block (not cyclic) distribution; node (i, j) owns block (i, j).
  * In-node placement: Q-checksum row k lives on grid row k mod p_r, R-checksum
    column k on grid column k mod p_c, corner blocks at their intersection.
  * Recovery uses the lowest-index surviving checksums.
  * Without a horizontal code (K_h = 0, e.g. a p_r x 1 grid) R would be
    unprotected; its p_r block rows then carry K_v checksum block rows of the
    vertical code with G~_v, encoded at every panel boundary where failures
    strike, and lost R blocks are decoded along block columns.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from itertools import combinations

import numpy as np

OUT_OF_NODE = "out"
IN_NODE = "in"


class NotRecoverable(Exception):
    """More erased blocks in a block row/column than surviving checksums."""


# --------------------------------------------------------------------------
# Code construction
# --------------------------------------------------------------------------

def q_generator(v_tilde: np.ndarray) -> np.ndarray:
    """G~_v = [G~_1  V~] with G~_1 = -1/2 V~ V~^T (K x p_r).

    Construction of the Q-factor checksum generator (out-of-node: K = f rows;
    in-node: K rows as in the in-node Q construction)."""
    v_tilde = np.asarray(v_tilde, dtype=np.float64)
    g1 = -0.5 * (v_tilde @ v_tilde.T)
    return np.hstack([g1, v_tilde])


def r_generator(gh_raw: np.ndarray, storage: str) -> np.ndarray:
    """R-side generator G~_h (p_c x K_h).

    Out-of-node: any MDS generator, used as given.  In-node: the systematic
    MDS construction excludes the storing node's own data from checksum k, i.e.
    G~_h[s_k, k] = 0 for the storing block column s_k = k mod p_c."""
    g = np.array(gh_raw, dtype=np.float64, copy=True)
    if storage == IN_NODE:
        pc = g.shape[0]
        for k in range(g.shape[1]):
            g[k % pc, k] = 0.0
    return g


def k_min_in_node(f: int, L: int, P: int) -> int:
    """Minimum checksum-block count for in-node storage (Theorem on the lower
    bound of K, attained with equality): K = fL/P + f * ceil(fL / ((P-f)P))."""
    assert L % P == 0 and 0 < f < P
    return f * L // P + f * (-(-(f * L) // ((P - f) * P)))


def k_lower_bound_bruteforce(f: int, L: int, P: int) -> int:
    """Smallest K satisfying the necessary condition of the lemma behind that
    theorem, by enumeration: with load-balanced placement (a_bar nodes hold
    ceil(K/P) checksum blocks, b_bar hold floor(K/P)), every choice of P - f
    surviving nodes (a from the first kind, b from the second) must hold at
    least f L / P checksum blocks."""
    need = f * L / P
    K = 0
    while True:
        K += 1
        hi, lo = -(-K // P), K // P
        a_bar = K - P * (K // P)
        b_bar = P - a_bar
        ok = True
        for a in range(0, P - f + 1):
            b = P - f - a
            if a <= a_bar and b <= b_bar and a * hi + b * lo < need:
                ok = False
                break
        if ok:
            return K


def f_tolerated(K: int, P: int, storage: str) -> int:
    """Failures per grid row/column a code with K checksum blocks tolerates."""
    if K == 0:
        return 0
    if storage == OUT_OF_NODE:
        return K
    best = 0
    for f in range(1, P):
        if k_min_in_node(f, P, P) <= K:
            best = f
    return best


def kron_generator(g_tilde: np.ndarray, block: int) -> np.ndarray:
    """G = G~ (x) I_block (System Model; used only to check block formulas)."""
    return np.kron(g_tilde, np.eye(block))


# --------------------------------------------------------------------------
# Layout
# --------------------------------------------------------------------------

@dataclass
class Layout:
    """Block geometry of the encoded problem.

    A is m x n on a p_r x p_c grid (blocks bs x bw).  The encoded matrix has
    K_v checksum block-rows and K_h checksum block-columns:  m' = m + K_v bs,
    N = n + K_h bw.  R is n x N with block rows of height hr = n / p_r."""
    m: int
    n: int
    pr: int
    pc: int
    kv: int
    kh: int
    storage: str = OUT_OF_NODE

    def __post_init__(self):
        assert self.m % self.pr == 0 and self.n % self.pc == 0 and self.n % self.pr == 0
        self.bs = self.m // self.pr
        self.bw = self.n // self.pc
        self.hr = self.n // self.pr
        self.mp = self.m + self.kv * self.bs
        self.N = self.n + self.kh * self.bw
        # Without a horizontal code (K_h = 0, e.g. p_c = 1) R is protected by a
        # vertical code over its p_r block rows with the Q side's generator:
        # K_v checksum block rows of height hr below R's n rows.
        self.rcode = self.kh == 0 and self.kv > 0
        self.rrows = self.n + (self.kv * self.hr if self.rcode else 0)

    def qblock(self, I: int, J: int):
        return (slice(I * self.bs, (I + 1) * self.bs), slice(J * self.bw, (J + 1) * self.bw))

    def rblock(self, i: int, J: int):
        return (slice(i * self.hr, (i + 1) * self.hr), slice(J * self.bw, (J + 1) * self.bw))

    def node_blocks(self, node):
        """Q blocks (I, J) and R blocks (i, J) held by a node.

        Out-of-node: the extended grid has a node per block position; checksum
        nodes sit at I >= p_r or J >= p_c and hold no R data in checksum rows.
        In-node: node (i, j) holds its data block plus the checksum blocks the
        placement assigns to it."""
        i, j = node
        pr, pc = self.pr, self.pc
        if self.storage == OUT_OF_NODE:
            assert 0 <= i < pr + self.kv and 0 <= j < pc + self.kh
            q = [(i, j)]
            r = [(i, j)] if (i < pr or self.rcode) else []
            return q, r
        assert 0 <= i < pr and 0 <= j < pc
        rows = [i] + [pr + k for k in range(self.kv) if k % pr == i]
        cols = [j] + [pc + k for k in range(self.kh) if k % pc == j]
        q = [(I, J) for I in rows for J in cols]
        r = [(I, J) for I in (rows if self.rcode else [i]) for J in cols]
        return q, r


# --------------------------------------------------------------------------
# Encode
# --------------------------------------------------------------------------

def encode(A: np.ndarray, gv: np.ndarray, gh: np.ndarray, lay: Layout) -> np.ndarray:
    """A~ = [[A, A G_h], [G_v A, G_v A G_h]] with G = G~ (x) I.

    Checksum rows: block (p_r + k, J) = sum_t g~_v[k, t] A_(t, J);
    checksum columns: block (I, p_c + k) = sum_t g~_h[t, k] A_(I, t);
    the corner applies the column code to the checksum rows."""
    At = np.zeros((lay.mp, lay.N))
    At[:lay.m, :lay.n] = A
    for k in range(lay.kv):
        for J in range(lay.pc):
            acc = np.zeros((lay.bs, lay.bw))
            for t in range(lay.pr):
                acc += gv[k, t] * At[lay.qblock(t, J)]
            At[lay.qblock(lay.pr + k, J)] = acc
    for k in range(lay.kh):
        for I in range(lay.pr + lay.kv):
            acc = np.zeros((lay.bs, lay.bw))
            for t in range(lay.pc):
                acc += gh[t, k] * At[lay.qblock(I, t)]
            At[lay.qblock(I, lay.pc + k)] = acc
    return At


# --------------------------------------------------------------------------
# Panel factorizations (columns of one panel, in place)
# --------------------------------------------------------------------------

ETA_DGKS = 1.0 / math.sqrt(2.0)


def panel_cgs2(P: np.ndarray, Rpp: np.ndarray, reorth: str = "always", eta: float = ETA_DGKS) -> int:
    """Column-wise classical Gram-Schmidt with reorthogonalisation on a panel.

    For column j: s1 = P[:, :j]^T p_j, p_j -= P[:, :j] s1; a second projection
    (always for CGS2, or when ||p_j|| < eta ||p_j before|| for ICGS); then
    r_jj = ||p_j|| and p_j /= r_jj.  Writes the panel's diagonal block of R.
    Returns how many columns were reorthogonalised."""
    b = P.shape[1]
    nre = 0
    for j in range(b):
        p = P[:, j].copy()
        Qj = P[:, :j]
        norm0 = np.linalg.norm(p)
        s = Qj.T @ p
        p = p - Qj @ s
        if reorth == "always" or (reorth == "dgks" and np.linalg.norm(p) < eta * norm0):
            s2 = Qj.T @ p
            p = p - Qj @ s2
            s = s + s2
            nre += 1
        r = np.linalg.norm(p)
        Rpp[:j, j] = s
        Rpp[j, j] = r
        P[:, j] = p / r
    return nre


def panel_mgs(P: np.ndarray, Rpp: np.ndarray) -> int:
    """Modified Gram-Schmidt restricted to the panel (the paper's sequential MGS,
    which its experiments used in place of ICGS).

    Each new basis vector q_i = u_i / ||u_i|| is removed at once from every
    column to its right by the rank-one projection I - q_i q_i^T, so a column
    has been projected against q_0 .. q_{j-1} one vector at a time by the time
    it is normalised.  The coefficients q_i^T u_j form row i of the panel's R."""
    b = P.shape[1]
    for i in range(b):
        Rpp[i, i] = np.linalg.norm(P[:, i])
        P[:, i] /= Rpp[i, i]
        if i + 1 < b:
            coef, P[:, i + 1:] = _project_out(P[:, i:i + 1], P[:, i + 1:])
            Rpp[i, i + 1:] = coef[0]
    return 0


# --------------------------------------------------------------------------
# Blocked factorization (PBMGS on one address space)
# --------------------------------------------------------------------------

@dataclass
class FactorOptions:
    b: int
    panel: str = "cgs2"          # "cgs2" | "icgs" | "mgs"
    reproject: bool = True
    eta: float = ETA_DGKS


def _project_out(basis: np.ndarray, X: np.ndarray):
    """Split X into its part in the span of an orthonormal basis and the rest:
    X = basis C + X_perp with C = basis^T X.  Returns (C, X_perp)."""
    C = basis.T @ X
    return C, X - basis @ C


def panel_factor(P: np.ndarray, opt: "FactorOptions"):
    """Orthonormal basis of the panel's columns and the upper-triangular
    factor with P = basis R_pp (positive diagonal), by the panel method chosen.
    Returns (basis, R_pp, number of reorthogonalised columns)."""
    P = P.copy()
    Rpp = np.zeros((P.shape[1], P.shape[1]))
    if opt.panel == "mgs":
        nre = panel_mgs(P, Rpp)
    else:
        nre = panel_cgs2(P, Rpp, "always" if opt.panel == "cgs2" else "dgks", opt.eta)
    return P, Rpp, nre


def factor_panels(Q: np.ndarray, R: np.ndarray, n: int, k0: int, k1: int, opt: FactorOptions) -> dict:
    """Panels k0 .. k1-1 of the blocked Gram-Schmidt (algorithms BMGS / PBMGS)
    on the iteration state Q (m' x N, in place; A~ at the start), accumulating
    the coefficients in R (n x N).

    Panel k holds columns [kb, (k+1)b).  Its columns are first made orthogonal
    to every earlier basis vector (the optional left re-projection: the part of
    the panel in the span of Q[:, :kb] is removed and its coefficients are
    added to R[:kb, panel]); the panel method then gives an orthonormal basis
    of the panel and its triangular factor R[panel, panel]; finally every
    column to the right -- systematic or carried checksum column -- is replaced
    by its component orthogonal to the new basis, the coefficients of the
    removed part going to R[panel, right].  Every step is a column operation
    on the encoded matrix, which is what keeps its checksum rows valid."""
    b = opt.b
    N = Q.shape[1]
    nre = 0
    for k in range(k0, k1):
        panel, right = slice(k * b, (k + 1) * b), slice((k + 1) * b, N)
        if opt.reproject and k > 0:
            S, Q[:, panel] = _project_out(Q[:, :k * b], Q[:, panel])
            R[:k * b, panel] += S
        Q[:, panel], R[panel, panel], nr = panel_factor(Q[:, panel], opt)
        nre += nr
        if (k + 1) * b < N:
            R[panel, right], Q[:, right] = _project_out(Q[:, panel], Q[:, right])
    return {"reorth_columns": nre}


# --------------------------------------------------------------------------
# Failures: erasure and recovery
# --------------------------------------------------------------------------

def erase(Q: np.ndarray, R: np.ndarray, nodes, lay: Layout):
    """Fail-stop failure: every block a failed node holds is lost (NaN)."""
    for node in nodes:
        qb, rb = lay.node_blocks(node)
        for I, J in qb:
            Q[lay.qblock(I, J)] = np.nan
        for i, J in rb:
            R[lay.rblock(i, J)] = np.nan


def _erased_sets(nodes, lay: Layout):
    qset, rset = set(), set()
    for node in nodes:
        qb, rb = lay.node_blocks(node)
        qset.update(qb)
        rset.update(rb)
    return qset, rset


def decode_line(blocks: list, checks: list, gen: np.ndarray, lost_data: list, lost_chk: list):
    """Decode one block column (or row) of a systematic linear code.

    blocks[t] (t < p) are data blocks, checks[k] are checksum blocks with
    checks[k] = sum_t gen[k, t] blocks[t].  Lost data blocks F are recovered
    from the lowest-index surviving checksums S (|S| = |F|):
        G_hat = gen[S, F],  X_F = G_hat^{-1} (C_S - sum_{t not in F} gen[S, t] X_t),
    then lost checksum blocks are re-encoded from the (now complete) data.
    Blocks are modified in place; returns the G_hat used (or None)."""
    F = sorted(lost_data)
    ghat = None
    if F:
        surv = [k for k in range(len(checks)) if k not in lost_chk]
        if len(surv) < len(F):
            raise NotRecoverable(f"{len(F)} erased data blocks, {len(surv)} surviving checksums")
        S = surv[:len(F)]
        ghat = gen[np.ix_(S, F)]
        keep = [t for t in range(len(blocks)) if t not in F]
        rhs = []
        for k in S:
            acc = checks[k].copy()
            for t in keep:
                acc -= gen[k, t] * blocks[t]
            rhs.append(acc)
        # solve G_hat X = rhs blockwise (all block entries at once)
        shape = blocks[keep[0] if keep else F[0]].shape
        rhs_mat = np.stack([r.reshape(-1) for r in rhs])
        X = np.linalg.solve(ghat, rhs_mat)
        for idx, t in enumerate(F):
            blocks[t][...] = X[idx].reshape(shape)
    for k in sorted(lost_chk):
        acc = np.zeros_like(blocks[0])
        for t in range(len(blocks)):
            acc += gen[k, t] * blocks[t]
        checks[k][...] = acc
    return ghat


def encode_r_rows(R: np.ndarray, gv: np.ndarray, lay: Layout):
    """Without a horizontal code: R's checksum block rows (below its n rows)
    are the vertical code of its p_r block rows, R_chk = (G~_v (x) I_hr) R[:n].
    R entries become final only column block by column block (each panel's
    re-projection adds into earlier rows), so the code is applied where
    failures strike: at panel boundaries."""
    if lay.rcode:
        R[lay.n:] = kron_generator(gv, lay.hr) @ R[:lay.n]


def recover(Q: np.ndarray, R: np.ndarray, nodes, lay: Layout, gv: np.ndarray, gh: np.ndarray):
    """Recover every block lost by `nodes` (erasure decoding, recovery lemma).

    Q is protected along each block column by the vertical code (Q_2 = G_v Q_1
    for every column, systematic and checksum); R along each block row by the
    horizontal code (R_2 = R_1 G_h), or, without a horizontal code, along each
    block column by the vertical code of encode_r_rows."""
    qset, rset = _erased_sets(nodes, lay)
    pr, pc = lay.pr, lay.pc
    for J in range(pc + lay.kh):
        lost_d = [I for I in range(pr) if (I, J) in qset]
        lost_c = [k for k in range(lay.kv) if (pr + k, J) in qset]
        if not lost_d and not lost_c:
            continue
        data = [Q[lay.qblock(I, J)] for I in range(pr)]
        chks = [Q[lay.qblock(pr + k, J)] for k in range(lay.kv)]
        decode_line(data, chks, gv, lost_d, lost_c)
    if lay.rcode:
        for J in range(pc):
            lost_d = [I for I in range(pr) if (I, J) in rset]
            lost_c = [k for k in range(lay.kv) if (pr + k, J) in rset]
            if not lost_d and not lost_c:
                continue
            data = [R[lay.rblock(I, J)] for I in range(pr)]
            chks = [R[lay.rblock(pr + k, J)] for k in range(lay.kv)]
            decode_line(data, chks, gv, lost_d, lost_c)
        rset = set()
    for i in range(pr):
        lost_d = [J for J in range(pc) if (i, J) in rset]
        lost_c = [k for k in range(lay.kh) if (i, pc + k) in rset]
        if not lost_d and not lost_c:
            continue
        # R_2 = R_1 G_h: transposed blocks satisfy check_k^T = sum_t gh[t, k] data_t^T
        data = [R[lay.rblock(i, J)].T for J in range(pc)]
        chks = [R[lay.rblock(i, pc + k)].T for k in range(lay.kh)]
        decode_line(data, chks, gh.T, lost_d, lost_c)
    if np.isnan(Q).any() or np.isnan(R).any():
        raise NotRecoverable("NaN left after recovery")


# --------------------------------------------------------------------------
# Post-orthogonalization and coded solve
# --------------------------------------------------------------------------

def g0_tilde(gv: np.ndarray) -> np.ndarray:
    """G^_0 = [[I_K + G~_1, V~], [V~^T, -I_{p_r-K}]]  (p_r x p_r); G_0 = G^_0 (x) I."""
    K, pr = gv.shape
    g1, v = gv[:, :K], gv[:, K:]
    top = np.hstack([np.eye(K) + g1, v])
    bot = np.hstack([v.T, -np.eye(pr - K)])
    return np.vstack([top, bot])


def postorth(Q1: np.ndarray, rhs: np.ndarray | None, gv: np.ndarray, pr: int):
    """Q_post = G_0 Q_1 and b_post = G_0 b, block row i = sum_l G^_0[i, l] Z_l
    (Theorem on low-cost post-orthogonalization; block form of its proof)."""
    g0 = g0_tilde(gv)
    m = Q1.shape[0]
    bs = m // pr

    def apply(Z):
        out = np.zeros_like(Z)
        for i in range(pr):
            acc = np.zeros_like(Z[:bs])
            for l in range(pr):
                if g0[i, l] != 0.0:
                    acc += g0[i, l] * Z[l * bs:(l + 1) * bs]
            out[i * bs:(i + 1) * bs] = acc
        return out

    qp = apply(Q1)
    bp = apply(rhs) if rhs is not None else None
    return qp, bp


def coded_solve(Qpost: np.ndarray, R1: np.ndarray, bpost: np.ndarray) -> np.ndarray:
    """x from R x = (G_0 Q_1)^T (G_0 b) by back substitution (linear-solve
    equations after the post-orthogonalization theorem)."""
    y = Qpost.T @ bpost
    n = R1.shape[0]
    x = np.zeros_like(y)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - R1[i, i + 1:] @ x[i + 1:]) / R1[i, i]
    return x


# --------------------------------------------------------------------------
# Plain definition (used to pin the step-by-step algorithm)
# --------------------------------------------------------------------------

def qr_plain(At: np.ndarray, n: int):
    """The coded factors by definition: the thin QR of A~[:, :n] with positive
    diag(R_1) (unique for full column rank), and R_2 = Q~^T A~[:, n:]."""
    q, r = np.linalg.qr(At[:, :n])
    s = np.sign(np.diag(r))
    q = q * s
    r = (r.T * s).T
    R = np.hstack([r, q.T @ At[:, n:]])
    return q, R


# --------------------------------------------------------------------------
# Whole pipeline
# --------------------------------------------------------------------------

@dataclass
class Problem:
    A: np.ndarray
    lay: Layout
    v_tilde: np.ndarray
    gh_raw: np.ndarray
    opt: FactorOptions
    schedule: list = field(default_factory=list)   # [(panel, [nodes])]
    rhs: np.ndarray | None = None


def run(prob: Problem, snapshots: bool = False) -> dict:
    """encode -> factor with scheduled failures (erase at the start of the
    panel, recover, continue) -> retrieve Q_1, R -> post-orthogonalize."""
    lay, opt = prob.lay, prob.opt
    gv = q_generator(prob.v_tilde) if lay.kv else np.zeros((0, lay.pr))
    gh = r_generator(prob.gh_raw, lay.storage) if lay.kh else np.zeros((lay.pc, 0))
    At = encode(prob.A, gv, gh, lay)
    Q = At.copy()
    R = np.zeros((lay.rrows, lay.N))     # n rows, then R's checksum rows when lay.rcode
    npan = lay.n // opt.b
    events = dict((t, nodes) for t, nodes in prob.schedule)
    k = 0
    snaps = []
    for t in sorted(events) + [npan]:
        factor_panels(Q, R[:lay.n], lay.n, k, t, opt)
        k = t
        if t == npan:
            break
        encode_r_rows(R, gv, lay)
        before = (Q.copy(), R.copy()) if snapshots else None
        erase(Q, R, events[t], lay)
        recover(Q, R, events[t], lay, gv, gh)
        if snapshots:
            snaps.append((t, before[0], before[1], Q.copy(), R.copy()))
    out = {"At": At, "Q": Q, "R": R[:lay.n], "gv": gv, "gh": gh, "snapshots": snaps}
    if lay.kv:
        qp, bp = postorth(Q[:lay.m, :lay.n], prob.rhs, gv, lay.pr)
        out["Qpost"], out["bpost"] = qp, bp
    return out


def metrics(A: np.ndarray, out: dict, lay: Layout) -> dict:
    """Error norms used throughout the tests and the bench."""
    Q, R = out["Q"], out["R"]
    n, m = lay.n, lay.m
    Qt = Q[:, :n]
    res = np.linalg.norm(A - Q[:m, :n] @ R[:, :n]) / np.linalg.norm(A)
    orth = np.linalg.norm(np.eye(n) - Qt.T @ Qt)
    d = {"residual": res, "orth_coded": orth}
    if "Qpost" in out:
        qp = out["Qpost"]
        d["orth_post"] = np.linalg.norm(np.eye(n) - qp.T @ qp)
    return d
