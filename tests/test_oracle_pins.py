"""Pins of the FP64 oracle against things other than itself: the paper's worked
example, exact closed forms (sympy), the uniquely defined QR (Householder via
LAPACK), the paper's theorems and brute force over failure sets."""
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest
import sympy as sp

import synth
from oracle import coded_qr as oc
from tests.golden import fixtures

F = np.float64


def _f(x):
    return float(x)


def _mat(rows):
    return np.array([[_f(x) for x in r] for r in rows])


# ---------------------------------------------------------------- P-1 / P-2
def _exact_coded_qr(A_rows, gv_rows, gh_cols):
    """Exact coded factors: Q~, R_1 from the Cholesky factor of A~_sys^T A~_sys
    (the QR with positive diagonal is unique), R_2 = Q~^T A~_chk."""
    A = sp.Matrix(A_rows)
    Gv = sp.Matrix(gv_rows)
    Gh = sp.Matrix(gh_cols)
    top = A.row_join(A * Gh)
    At = top.col_join((Gv * A).row_join(Gv * A * Gh))
    n = A.shape[1]
    S = At[:, :n]
    L = (S.T * S).cholesky(hermitian=False)
    R1 = L.T
    Q = S * R1.inv()
    R2 = Q.T * At[:, n:]
    return At, Q, R1.row_join(R2)


@pytest.mark.parametrize("name,pr", [("paper_example_2x2.txt", 2), ("paper_example_3x3.txt", 3)])
def test_paper_example_closed_form(name, pr):
    fx = fixtures.load(name)
    v = fx["v"] if isinstance(fx["v"], list) else [fx["v"]]
    v_tilde = np.array([[_f(x) for x in v]])
    gv = oc.q_generator(v_tilde)
    # generator: G~ = [g1 V~], g1 = -1/2 V~V~^T, as printed in the example
    assert gv[0, 0] == pytest.approx(_f(fx["g1"][0] if isinstance(fx["g1"], list) else fx["g1"]), abs=0)
    np.testing.assert_array_equal(gv[0, 1:], v_tilde[0])
    # G_0 of the example
    np.testing.assert_allclose(oc.g0_tilde(gv), _mat(fx["G0"]), rtol=0, atol=1e-16)
    A = _mat(fx["A"])
    lay = oc.Layout(pr, pr, pr, pr, 1, 1, oc.OUT_OF_NODE)
    gh = oc.r_generator(np.array([[_f(x)] for x in fx["Gh"]]), oc.OUT_OF_NODE)
    At = oc.encode(A, gv, gh, lay)
    if "At" in fx:
        np.testing.assert_allclose(At, _mat(fx["At"]), rtol=0, atol=1e-15)
    # exact factors
    gv_exact = [[Fraction(-1, 2) * sum(x * x for x in v)] + list(v)]
    At_x, Qx, Rx = _exact_coded_qr([list(r) for r in fx["A"]], gv_exact, [[x] for x in fx["Gh"]])
    np.testing.assert_allclose(At, np.array(At_x.evalf(30), dtype=F), atol=1e-15)
    Qx = np.array(Qx.evalf(30), dtype=F)
    Rx = np.array(Rx.evalf(30), dtype=F)
    for panel in ("cgs2", "icgs", "mgs"):
        for reproject in (True, False):
            Q = At.copy()
            R = np.zeros((pr, pr + 1))
            oc.factor_panels(Q, R, pr, 0, pr, oc.FactorOptions(1, panel, reproject))
            np.testing.assert_allclose(Q[:, :pr], Qx, atol=2e-15)
            np.testing.assert_allclose(R, Rx, atol=4e-15 * np.abs(Rx).max())
    # post-orthogonalization makes G_0 Q_1 exactly orthogonal
    G0 = sp.Matrix([[sp.Rational(x) for x in r] for r in fx["G0"]])
    _, Qs, _ = _exact_coded_qr([list(r) for r in fx["A"]], gv_exact, [[x] for x in fx["Gh"]])
    Q1 = Qs[:pr, :]
    W = sp.simplify((G0 * Q1).T * (G0 * Q1))
    assert W == sp.eye(pr)
    qp, _ = oc.postorth(Qx[:pr], None, gv, pr)
    np.testing.assert_allclose(qp, np.array((G0 * Q1).evalf(30), dtype=F), atol=1e-15)


def test_paper_example_recovery_formula():
    """After the first iteration the example recovers node (1,1) (0-based (0,0))
    by Q11 = (Q31 - v Q21)/g1 and R11 = R13 - R12 (corrected index)."""
    fx = fixtures.load("paper_example_2x2.txt")
    v = _f(fx["v"][0])
    g1 = _f(fx["g1"][0])
    A = _mat(fx["A"])
    lay = oc.Layout(2, 2, 2, 2, 1, 1, oc.OUT_OF_NODE)
    gv = oc.q_generator(np.array([[v]]))
    gh = oc.r_generator(np.ones((2, 1)), oc.OUT_OF_NODE)
    Q = oc.encode(A, gv, gh, lay)
    R = np.zeros((2, 3))
    oc.factor_panels(Q, R, 2, 0, 1, oc.FactorOptions(1, "cgs2"))
    Q0, R0 = Q.copy(), R.copy()
    oc.erase(Q, R, [(0, 0)], lay)
    assert np.isnan(Q[0, 0]) and np.isnan(R[0, 0])
    oc.recover(Q, R, [(0, 0)], lay, gv, gh)
    assert Q[0, 0] == pytest.approx((Q0[2, 0] - v * Q0[1, 0]) / g1, rel=1e-14)
    assert R[0, 0] == pytest.approx(R0[0, 2] - R0[0, 1], rel=1e-14)
    np.testing.assert_allclose(Q, Q0, rtol=1e-13)
    np.testing.assert_allclose(R, R0, rtol=1e-13)


# ---------------------------------------------------------------- P-3, P-4
CASES = [
    # n, pr, K, b, storage, panel, reproject
    (64, 4, 1, 8, oc.OUT_OF_NODE, "cgs2", True),
    (64, 4, 2, 4, oc.OUT_OF_NODE, "icgs", True),
    (96, 6, 3, 8, oc.OUT_OF_NODE, "cgs2", False),
    (128, 8, 2, 16, oc.IN_NODE, "icgs", True),
    (128, 8, 4, 8, oc.IN_NODE, "mgs", True),
    (48, 3, 1, 16, oc.OUT_OF_NODE, "cgs2", True),
]


def _setup(n, pr, K, storage, seed=0, A=None):
    lay = oc.Layout(n, n, pr, pr, K, K, storage)
    gv = oc.q_generator(synth.q_generator_draws(K, pr, seed))
    gh = oc.r_generator(synth.r_generator_draws(pr, K, seed), storage)
    if A is None:
        A = synth.gaussian(n, n, seed)
    return lay, gv, gh, A


@pytest.mark.parametrize("n,pr,K,b,storage,panel,reproject", CASES)
def test_factor_matches_householder_and_invariants(n, pr, K, b, storage, panel, reproject):
    lay, gv, gh, A = _setup(n, pr, K, storage)
    At = oc.encode(A, gv, gh, lay)
    Gv = oc.kron_generator(gv, lay.bs)
    Gh = oc.kron_generator(gh, lay.bw)
    # encoding equals its Kronecker definition
    np.testing.assert_allclose(At, np.block([[A, A @ Gh], [Gv @ A, Gv @ A @ Gh]]), atol=1e-13)
    Qh, Rh = oc.qr_plain(At, n)
    Q = At.copy()
    R = np.zeros((n, lay.N))
    opt = oc.FactorOptions(b, panel, reproject)
    for k in range(n // b):
        oc.factor_panels(Q, R, n, k, k + 1, opt)
        t = (k + 1) * b
        # checksum preservation after every iteration (Lemma on two-way checksums)
        assert np.abs(Q[lay.m:] - Gv @ Q[:lay.m]).max() < 1e-12
        assert np.abs(R[:, n:] - R[:, :n] @ Gh).max() < 1e-11 * np.abs(R).max()
        # intermediate state: Q^(t) = [Q~_<t | (I - Q~_<t Q~_<t^T) A~_>=t], R^(t) = [R_<t ; 0]
        Qt = Qh[:, :t]
        np.testing.assert_allclose(Q[:, :t], Qt, atol=1e-12)
        np.testing.assert_allclose(Q[:, t:], At[:, t:] - Qt @ (Qt.T @ At[:, t:]), atol=1e-11)
        np.testing.assert_allclose(R[:t], Rh[:t], atol=1e-11 * np.abs(Rh).max())
        assert not R[t:].any()
    # final form: unique thin QR with positive diagonal (Corollary on the final form)
    np.testing.assert_allclose(Q[:, :n], Qh, atol=1e-12)
    np.testing.assert_allclose(R, Rh, atol=1e-12 * np.abs(Rh).max())
    assert np.all(np.diag(R[:, :n]) > 0)
    assert np.allclose(np.tril(R[:, :n], -1), 0)
    assert np.linalg.norm(np.eye(n) - Q[:, :n].T @ Q[:, :n]) < 1e-12
    assert np.linalg.norm(A - Q[:n, :n] @ R[:, :n]) / np.linalg.norm(A) < 1e-14
    # carried checksum columns end with a residual at rounding level
    assert np.abs(Q[:, n:]).max() < 1e-12 * np.abs(At).max()
    # R_1 = chol(A^T (I + G_v^T G_v) A)
    Rc = np.linalg.cholesky(A.T @ (np.eye(n) + Gv.T @ Gv) @ A).T
    np.testing.assert_allclose(R[:, :n], Rc, atol=1e-11 * np.abs(Rc).max())


def test_pbmgs_project_step_matches_theorem():
    """R^(t)[panel rows, :] = Qbar^T A~ (the parallel-MGS preservation lemma)."""
    lay, gv, gh, A = _setup(64, 4, 1, oc.OUT_OF_NODE, seed=3)
    At = oc.encode(A, gv, gh, lay)
    Q = At.copy()
    R = np.zeros((64, lay.N))
    for k in range(8):
        oc.factor_panels(Q, R, 64, k, k + 1, oc.FactorOptions(8, "cgs2", False))
        qb = Q[:, 8 * k:8 * k + 8]
        np.testing.assert_allclose(R[8 * k:8 * k + 8, 8 * k + 8:], (qb.T @ At)[:, 8 * k + 8:], atol=1e-12)


def test_paper_cgs_listing_literal_is_not_orthogonal():
    """Reading check: the CGS listing run literally (v not normalised before
    the rank-1 update) does not orthogonalise; the oracle's CGS2 does."""
    rng = np.random.default_rng(0)
    P = rng.standard_normal((200, 16)) / np.sqrt(200.0) * 3.0
    Q = P.copy()
    for i in range(16):
        v = Q[:, i:].T @ Q[:, i]
        q = Q[:, i] / np.sqrt(v[0])
        Q[:, i] = q
        Q[:, i + 1:] -= np.outer(q, v[1:])
    loss = np.linalg.norm(np.eye(16) - Q.T @ Q)
    assert not np.isfinite(loss) or loss > 0.1
    P2 = P.copy()
    oc.panel_cgs2(P2, np.zeros((16, 16)))
    assert np.linalg.norm(np.eye(16) - P2.T @ P2) < 1e-14


# ---------------------------------------------------------------- THM G_0
@pytest.mark.parametrize("K,pr,bs", [(1, 2, 3), (2, 4, 2), (3, 8, 2), (4, 8, 1)])
def test_g0_theorem(K, pr, bs):
    gv = oc.q_generator(synth.q_generator_draws(K, pr, 5))
    G = oc.kron_generator(gv, bs)
    G0 = oc.kron_generator(oc.g0_tilde(gv), bs)
    n, c = pr * bs, K * bs
    # G_0 written from its definition with G = [G_1 V]
    G1, V = G[:, :c], G[:, c:]
    G0_def = np.block([[np.eye(c) + G1, V], [V.T, -np.eye(n - c)]])
    np.testing.assert_allclose(G0, G0_def, atol=1e-15)
    np.testing.assert_allclose(G0, G0.T, atol=0)
    np.testing.assert_allclose(G0.T @ G0, np.eye(n) + G.T @ G, atol=1e-14)
    det = np.linalg.det(G0)
    expect = (-1) ** (n - c) * np.linalg.det(np.eye(c) + 0.5 * V @ V.T)
    assert det == pytest.approx(expect, rel=1e-12) and abs(det) >= 1 - 1e-12
    # orthogonality of G_0 Q_1 for any Q with orthonormal [Q_1; G Q_1]
    rng = np.random.default_rng(1)
    A = rng.standard_normal((n, n))
    q, _ = np.linalg.qr(np.vstack([A, G @ A]))
    W = G0 @ q[:n]
    assert np.linalg.norm(W.T @ W - np.eye(n)) < 1e-13


# ---------------------------------------------------------------- P-7, P-8
@pytest.mark.parametrize("K,pr", [(1, 2), (1, 4), (2, 4), (2, 8), (3, 6), (4, 8)])
def test_generator_mds_bruteforce(K, pr):
    """Every square submatrix of G~_v is nonsingular (MDS property, Theorem on
    probability-one full rank)."""
    for seed in range(3):
        gv = oc.q_generator(synth.q_generator_draws(K, pr, seed))
        for s in range(1, K + 1):
            for rows in combinations(range(K), s):
                for cols in combinations(range(pr), s):
                    sub = gv[np.ix_(rows, cols)]
                    assert abs(np.linalg.det(sub)) > 1e-12
                    assert np.linalg.cond(sub) < 1e12


def test_generator_structured_vs_random_condition():
    """The structured generator's worst square-submatrix condition number stays
    within a small factor of a fully random one (paper reports at most ~3x on
    average); checked loosely on small sizes."""
    ratios = []
    for seed in range(20):
        rng = np.random.default_rng(seed)
        v = rng.uniform(size=(2, 14))
        gs = oc.q_generator(v)
        gr = np.hstack([rng.uniform(size=(2, 2)), v])

        def worst(g):
            w = 1.0
            for s in (1, 2):
                for rows in combinations(range(2), s):
                    for cols in combinations(range(16), s):
                        w = max(w, np.linalg.cond(g[np.ix_(rows, cols)]))
            return w
        ratios.append(np.log10(worst(gs)) - np.log10(worst(gr)))
    assert np.mean(ratios) < np.log10(10.0)


def test_k_bound_matches_bruteforce():
    for P in range(2, 13):
        for mult in (1, 2, 3):
            L = mult * P
            for f in range(1, P // 2 + 1):
                assert oc.k_min_in_node(f, L, P) == oc.k_lower_bound_bruteforce(f, L, P), (f, L, P)


def test_k_bound_values():
    assert oc.k_min_in_node(1, 8, 8) == 2
    assert oc.k_min_in_node(4, 16, 16) == 8
    assert oc.f_tolerated(2, 8, oc.IN_NODE) == 1
    assert oc.f_tolerated(8, 16, oc.IN_NODE) == 4
    assert oc.f_tolerated(4, 8, oc.OUT_OF_NODE) == 4


# ---------------------------------------------------------------- P-6 decode brute force
def _mid_state(n, pr, K, b, storage, seed, t):
    lay, gv, gh, A = _setup(n, pr, K, storage, seed)
    Q = oc.encode(A, gv, gh, lay)
    R = np.zeros((n, lay.N))
    oc.factor_panels(Q, R, n, 0, t, oc.FactorOptions(b, "cgs2"))
    return lay, gv, gh, Q, R


@pytest.mark.parametrize("pr,K", [(2, 1), (3, 1), (4, 2), (6, 3), (8, 4)])
def test_recover_every_subset_in_a_block_column(pr, K):
    """Out-of-node: in one block column any set of erased blocks (data and
    checksum) of size <= K is recovered exactly; K+1 erased data blocks is
    not recoverable."""
    n = 8 * pr
    lay, gv, gh, Q0, R0 = _mid_state(n, pr, K, 4, oc.OUT_OF_NODE, 11, (n // 4) // 2)
    J = 1
    positions = [(I, J) for I in range(pr + K)]
    for s in range(1, K + 1):
        for sub in combinations(positions, s):
            Q, R = Q0.copy(), R0.copy()
            oc.erase(Q, R, list(sub), lay)
            oc.recover(Q, R, list(sub), lay, gv, gh)
            err = np.abs(Q - Q0).max() / np.abs(Q0).max()
            assert err < 1e-10, (sub, err)
            assert np.abs(R - R0).max() <= 1e-10 * np.abs(R0).max()
    Q, R = Q0.copy(), R0.copy()
    bad = [(I, J) for I in range(K + 1)]
    oc.erase(Q, R, bad, lay)
    with pytest.raises(oc.NotRecoverable):
        oc.recover(Q, R, bad, lay, gv, gh)


@pytest.mark.parametrize("pr,K", [(4, 2), (6, 2), (8, 2), (8, 4)])
def test_in_node_tolerates_f_failures(pr, K):
    """In-node storage with K = K_min(f) tolerates any f failed nodes of a grid
    column (Theorem on in-node systematic MDS coding) - both the Q code (full
    sum) and the R code (storing column excluded)."""
    f = oc.f_tolerated(K, pr, oc.IN_NODE)
    assert f >= 1
    n = 8 * pr
    lay, gv, gh, Q0, R0 = _mid_state(n, pr, K, 4, oc.IN_NODE, 12, (n // 4) // 2)
    for j in (0, pr - 1):
        for rows in combinations(range(pr), f):
            nodes = [(i, j) for i in rows]
            Q, R = Q0.copy(), R0.copy()
            oc.erase(Q, R, nodes, lay)
            oc.recover(Q, R, nodes, lay, gv, gh)
            assert np.abs(Q - Q0).max() < 1e-10 * np.abs(Q0).max()
            assert np.abs(R - R0).max() < 1e-10 * np.abs(R0).max()
    # the same along a grid row (R is decoded along block rows)
    for cols in combinations(range(pr), f):
        nodes = [(1, j) for j in cols]
        Q, R = Q0.copy(), R0.copy()
        oc.erase(Q, R, nodes, lay)
        oc.recover(Q, R, nodes, lay, gv, gh)
        assert np.abs(R - R0).max() < 1e-10 * np.abs(R0).max()


def _storers(lay):
    """From the oracle's node_blocks alone: the grid row of the node that holds
    Q-checksum block row k in each block column, and the grid column of the
    node that holds R-checksum block column k in each block row."""
    qrow, rcol = {}, {}
    for i in range(lay.pr):
        for j in range(lay.pc):
            qb, rb = lay.node_blocks((i, j))
            for I, J in qb:
                if I >= lay.pr and J == j:
                    qrow.setdefault(I - lay.pr, set()).add(i)
            for I, J in rb:
                if J >= lay.pc and I == i:
                    rcol.setdefault(J - lay.pc, set()).add(j)
    return qrow, rcol


@pytest.mark.parametrize("P,K", [(8, 2), (8, 3), (16, 8), (4, 4), (6, 9), (5, 7), (3, 1)])
def test_in_node_placement_is_load_balanced(P, K):
    """Definition of the load-balanced in-node distribution: of the P nodes of a
    code line, a_bar = K - P floor(K/P) hold ceil(K/P) checksum blocks and the
    other P - a_bar hold floor(K/P); every checksum block sits on exactly one
    node of the line, and in the same position in every line (so one
    generator describes the code of every block row and column)."""
    lay = oc.Layout(4 * P, 4 * P, P, P, K, K, oc.IN_NODE)
    qrow, rcol = _storers(lay)
    for where in (qrow, rcol):
        assert sorted(where) == list(range(K))
        assert all(len(nodes) == 1 for nodes in where.values())      # one storer, same in every line
        count = [0] * P
        for nodes in where.values():
            count[next(iter(nodes))] += 1
        a_bar = K - P * (K // P)
        assert sorted(count, reverse=True) == [-(-K // P)] * a_bar + [K // P] * (P - a_bar)


@pytest.mark.parametrize("P,K", [(8, 2), (16, 8), (4, 2), (6, 3)])
def test_in_node_r_code_excludes_its_storer(P, K):
    """In-node systematic MDS construction: the checksum stored on node s sums
    the data of every other node of its line and not s's own,
    C_k = sum_{t != s_k} g~[t, k] D_t; the storer s_k is found from the
    placement alone.  The Q side keeps the full sum (its generator has no zero:
    G~_1 = -1/2 V~ V~^T and V~ are dense), the alternative that the paper's
    remark on in-node storage allows."""
    lay = oc.Layout(4 * P, 4 * P, P, P, K, K, oc.IN_NODE)
    _, rcol = _storers(lay)
    raw = synth.r_generator_draws(P, K, 3) + 0.5          # strictly positive raw entries
    g = oc.r_generator(raw, oc.IN_NODE)
    for k in range(K):
        s_k = next(iter(rcol[k]))
        assert g[s_k, k] == 0.0
        assert all(g[t, k] == raw[t, k] for t in range(P) if t != s_k)
    gv = oc.q_generator(synth.q_generator_draws(K, P, 3) + 0.5)
    assert (gv != 0.0).all()
    # out of node nothing is excluded
    assert (oc.r_generator(raw, oc.OUT_OF_NODE) == raw).all()


def test_reverse_diagonal_storm_recovers():
    pr, K = 8, 4
    n = 64
    lay, gv, gh, Q0, R0 = _mid_state(n, pr, K, 4, oc.OUT_OF_NODE, 13, 9)
    nodes = synth.reverse_diagonal(pr, K)
    Q, R = Q0.copy(), R0.copy()
    oc.erase(Q, R, nodes, lay)
    oc.recover(Q, R, nodes, lay, gv, gh)
    assert np.abs(Q - Q0).max() < 1e-10 * np.abs(Q0).max()
    assert np.abs(R - R0).max() < 1e-10 * np.abs(R0).max()


# ---------------------------------------------------------------- whole pipeline / solve
@pytest.mark.parametrize("storage,K", [(oc.OUT_OF_NODE, 1), (oc.IN_NODE, 2)])
def test_pipeline_with_failures_equals_failure_free(storage, K):
    n, pr, b = 128, 8 if storage == oc.IN_NODE else 4, 16
    lay, gv, gh, A = _setup(n, pr, K, storage, seed=21)
    rhs = synth.gaussian(n, 2, 99)
    sched = synth.draw_schedule("random", n // b, pr, pr, 21, nfail=2)
    assert sched
    base = oc.run(oc.Problem(A, lay, synth.q_generator_draws(K, pr, 21), synth.r_generator_draws(pr, K, 21),
                             oc.FactorOptions(b, "icgs"), [], rhs))
    fail = oc.run(oc.Problem(A, lay, synth.q_generator_draws(K, pr, 21), synth.r_generator_draws(pr, K, 21),
                             oc.FactorOptions(b, "icgs"), sched, rhs))
    np.testing.assert_allclose(fail["Q"], base["Q"], atol=1e-13)
    np.testing.assert_allclose(fail["R"], base["R"], atol=1e-13 * np.abs(base["R"]).max())
    m = oc.metrics(A, fail, lay)
    assert m["residual"] < 1e-14 and m["orth_coded"] < 1e-12 and m["orth_post"] < 1e-12
    # coded solve: R x = (G_0 Q_1)^T (G_0 b) equals the direct solution of A x = b
    x = oc.coded_solve(fail["Qpost"], fail["R"][:, :n], fail["bpost"])
    np.testing.assert_allclose(x, np.linalg.solve(A, rhs), rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("storage", [oc.OUT_OF_NODE, oc.IN_NODE])
def test_r_row_code_recovers_without_horizontal_code(storage):
    """p_c = 1 leaves R without a horizontal code; its block rows are then
    protected by the vertical code with the Q side's generator.  Every set of
    tolerated node failures (all pairs, checksum nodes included, out of node;
    every single node in node, where f_tol = 1) at a mid panel must give the
    failure-free factors."""
    import itertools
    m, n, pr, K, b = 256, 32, 8, 2, 8
    lay = oc.Layout(m, n, pr, 1, K, 0, storage)
    assert lay.rcode and lay.rrows == n + K * n // pr
    A = synth.gaussian(m, n, 51)
    v = synth.q_generator_draws(K, pr, 51)
    opt = oc.FactorOptions(b, "cgs2")
    base = oc.run(oc.Problem(A, lay, v, None, opt, []))
    if storage == oc.OUT_OF_NODE:
        nodes = [(i, 0) for i in range(pr + K)]
        sets = list(itertools.combinations(nodes, 2))
    else:
        assert oc.f_tolerated(K, pr, storage) == 1
        sets = [((i, 0),) for i in range(pr)]
    for fail in sets:
        out = oc.run(oc.Problem(A, lay, v, None, opt, [(2, list(fail))]))
        assert np.abs(out["Q"] - base["Q"]).max() < 1e-12, fail
        assert np.abs(out["R"] - base["R"]).max() < 1e-12 * np.abs(base["R"]).max(), fail
    # one more than tolerated on the code line cannot be decoded
    with pytest.raises(oc.NotRecoverable):
        over = [(i, 0) for i in range(K + 1)] if storage == oc.OUT_OF_NODE else [(0, 0), (1, 0)]
        oc.run(oc.Problem(A, lay, v, None, opt, [(2, over)]))


def test_tall_coded_solve_is_weighted_least_squares():
    """For tall A the post-orthogonalized solve x = R_1^{-1} (G_0 Q_1)^T (G_0 b)
    minimises (Ax - b)^T W (Ax - b) with W = I + G_v^T G_v: closed form
    (A^T W A)^{-1} A^T W b.  With a nonzero residual this differs from
    ordinary least squares."""
    m, n, pr, K, b = 512, 64, 8, 2, 16
    lay = oc.Layout(m, n, pr, 1, K, 0, oc.OUT_OF_NODE)
    A = synth.gaussian(m, n, 5)
    v = synth.q_generator_draws(K, pr, 5)
    rhs = synth.gaussian(m, 3, 6)
    out = oc.run(oc.Problem(A, lay, v, None, oc.FactorOptions(b, "cgs2"), [], rhs))
    x = oc.coded_solve(out["Qpost"], out["R"][:, :n], out["bpost"])
    Gv = np.kron(oc.q_generator(v), np.eye(lay.bs))
    W = np.eye(m) + Gv.T @ Gv
    xw = np.linalg.solve(A.T @ W @ A, A.T @ W @ rhs)
    np.testing.assert_allclose(x, xw, rtol=1e-11, atol=1e-12)
    xo = np.linalg.lstsq(A, rhs, rcond=None)[0]
    assert np.abs(x - xo).max() > 1e-6


# ---------------------------------------------------------------- ICGS criterion
def test_icgs_criterion_reduces_to_cgs_and_cgs2_at_its_limits():
    """The re-orthogonalization test ||p_j|| < eta ||p_j before|| (reading 4)
    at its limits and at the default eta = 1/sqrt 2:
    - eta = 0 never fires: plain classical Gram-Schmidt, which loses
      orthogonality on a column 1e-9 from another (u kappa);
    - eta > 1 always fires: bitwise the CGS2 panel;
    - the default fires on no column of a well-conditioned Gaussian panel and
      on exactly the nearly dependent column of the other, restoring
      orthogonality to CGS2's level."""
    rng = np.random.default_rng(7)
    gauss = rng.standard_normal((200, 24))
    dep = gauss.copy()
    dep[:, 10] = dep[:, 3] + 1e-9 * rng.standard_normal(200)

    def panel(P, reorth, eta):
        Q, R = P.copy(), np.zeros((24, 24))
        n = oc.panel_cgs2(Q, R, reorth, eta)
        return Q, R, n

    def orth(Q):
        return np.linalg.norm(np.eye(Q.shape[1]) - Q.T @ Q)

    Q, R, n = panel(dep, "dgks", 0.0)
    assert n == 0 and orth(Q) > 1e-9
    Qc, Rc, nc = panel(dep, "always", 0.0)
    assert orth(Qc) < 1e-14
    for P in (gauss, dep):
        Q1, R1, n1 = panel(P, "dgks", 1.1)
        Q2, R2, n2 = panel(P, "always", 0.0)
        assert n1 == n2 == 24 and np.array_equal(Q1, Q2) and np.array_equal(R1, R2)
    Q, R, n = panel(gauss, "dgks", oc.ETA_DGKS)
    assert n == 0
    Q, R, n = panel(dep, "dgks", oc.ETA_DGKS)
    assert n == 1 and orth(Q) < 1e-14
    assert np.linalg.norm(dep - Q @ R) <= 1e-15 * np.linalg.norm(dep)


# ---------------------------------------------------------------- planted mistakes
def test_pins_catch_planted_mistakes(monkeypatch):
    """A wrong sign in the generator construction breaks the post-orth
    theorem check; a transposed recovery generator breaks recovery."""
    real = oc.q_generator
    monkeypatch.setattr(oc, "q_generator", lambda v: np.hstack([+0.5 * v @ v.T, v]))
    gv = oc.q_generator(synth.q_generator_draws(2, 4, 5))
    G = oc.kron_generator(gv, 2)
    G0 = oc.kron_generator(oc.g0_tilde(gv), 2)
    assert np.abs(G0.T @ G0 - (np.eye(8) + G.T @ G)).max() > 1e-3
    monkeypatch.setattr(oc, "q_generator", real)

    lay, gv, gh, Q0, R0 = _mid_state(32, 4, 2, 4, oc.OUT_OF_NODE, 11, 3)
    Q, R = Q0.copy(), R0.copy()
    oc.erase(Q, R, [(1, 2)], lay)
    real_decode = oc.decode_line

    def swapped(blocks, checks, gen, ld, lc):
        return real_decode(blocks, checks, gen[::-1].copy(), ld, lc)
    monkeypatch.setattr(oc, "decode_line", swapped)
    oc.recover(Q, R, [(1, 2)], lay, gv, gh)
    assert np.abs(Q - Q0).max() > 1e-6
