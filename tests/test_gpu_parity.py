"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
identical seeded inputs.  Bounds: ||A - Q_1 R_1||_F/||A||_F <= 1e-12,
||I - Q~^T Q~||_F <= 1e-12, elementwise |R - R_oracle| <= 1e-11 max|R_oracle|,
recovered blocks within 1e-10 (relative) of their values before erasure."""
import numpy as np
import pytest

import synth
from oracle import coded_qr as oc
from tests.gpu_helpers import gpu_config, host, make_inputs, oracle_state, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cqr():
    from paper_2311_11943_amd import cqr as mod
    return mod


def _dev(cqr, a):
    return cqr.to_device_colmajor(a, "cuda:0")


SHAPES = [
    # id, n, pr, K, b, storage, extra
    ("c1", 256, 4, 1, 16, "out", {}),
    ("ragged", 240, 4, 1, 16, "out", {}),           # m' = 300: partial tiles everywhere
    ("tall", 192, 4, 2, 16, "out", {"m": 384}),      # m > n
    ("innode", 512, 8, 2, 64, "in", {}),
    ("wide_panel", 512, 4, 2, 128, "out", {}),       # recursive panel 64 + 64
    ("odd_panel", 384, 4, 1, 96, "out", {}),         # recursive panel 48 + 48
    ("k4", 256, 8, 4, 32, "out", {}),
    # panels of four tile rows: the two-tile-row product for the trailing
    # products and re-projections, also with a 48-row last tile (b = 240)
    ("panel256", 1024, 4, 1, 256, "out", {}),
    ("ragged_panel240", 960, 4, 1, 240, "out", {}),
    # three tile rows (odd): the last workgroup of the two-tile-row product
    # computes an empty second half; its trailing products split over K
    ("odd_tile_rows192", 768, 4, 1, 192, "out", {}),
]


@pytest.mark.parametrize("sid,n,pr,K,b,storage,extra", SHAPES, ids=[s[0] for s in SHAPES])
def test_encode_and_factor_match_oracle(cqr, sid, n, pr, K, b, storage, extra):
    print(f"[case] {sid} n={n} pr={pr} K={K} b={b} {storage} {extra}", flush=True)
    A, v, gh, lay = make_inputs(n, pr, K, b, storage, seed=1, **extra)
    cfg = gpu_config(cqr, lay, b)
    q = cqr.CodedQR(cfg, v, gh)
    At, R = q.alloc()
    At[:lay.m, :lay.n].copy_(_dev(cqr, A))
    q.encode(At)
    At0, Qo, Ro, gv, ghm = oracle_state(A, v, gh, lay, b, 0)
    assert rel(host(At), At0) < 1e-14, "encode"
    npan = n // b
    # panel by panel: intermediate states equal the oracle's
    checkpoints = sorted({1, npan // 2, npan})
    k = 0
    for t in checkpoints:
        q.factor(At, R, k, t)
        k = t
        _, Qo, Ro, _, _ = oracle_state(A, v, gh, lay, b, t)
        torch.cuda.synchronize()
        Qg, Rg = host(At), host(R)
        assert not np.isnan(Qg).any() and not np.isnan(Rg).any()
        assert rel(Rg, Ro) < 1e-11, f"R after {t} panels"
        assert np.abs(Qg - Qo).max() < 1e-11 * np.abs(Qo).max(), f"Q after {t} panels"
    assert q.info() == 0
    Qg, Rg = host(At), host(R)
    Qt = Qg[:, :n]
    res = np.linalg.norm(A - Qg[:lay.m, :n] @ Rg[:, :n]) / np.linalg.norm(A)
    orth = np.linalg.norm(np.eye(n) - Qt.T @ Qt)
    assert res < 1e-12 and orth < 1e-12, (res, orth)
    # the unique factor, independently of either Gram-Schmidt variant
    Qh, Rh = oc.qr_plain(At0, n)
    assert rel(Rg, Rh) < 1e-11
    # checksum relations of the final form
    Gv = oc.kron_generator(gv, lay.bs)
    assert np.abs(Qg[lay.m:, :n] - Gv @ Qg[:lay.m, :n]).max() < 1e-12
    if lay.kh:
        Gh = oc.kron_generator(ghm, lay.bw)
        assert np.abs(Rg[:, n:] - Rg[:, :n] @ Gh).max() < 1e-11 * np.abs(Rg).max()
    q.close()


@pytest.mark.parametrize("sid,n,pr,K,b,storage,kind", [
    ("c1_random", 256, 4, 1, 16, "out", "random"),
    ("innode_random", 512, 8, 2, 64, "in", "random"),
    ("revdiag", 256, 8, 4, 32, "out", "revdiag"),
    ("burst", 384, 4, 2, 32, "out", "burst"),
])
def test_failures_recover_to_snapshot_and_final_matches(cqr, sid, n, pr, K, b, storage, kind):
    print(f"[case] {sid}", flush=True)
    A, v, gh, lay = make_inputs(n, pr, K, b, storage, seed=2)
    cfg = gpu_config(cqr, lay, b)
    q = cqr.CodedQR(cfg, v, gh)
    f = q.ftol
    sched = synth.draw_schedule(kind, n // b, pr, pr, 2, nfail=max(1, min(2, f)), every=3, f=min(f, 2))
    assert sched
    At, R = q.alloc()
    At[:lay.m, :lay.n].copy_(_dev(cqr, A))
    q.encode(At)
    k = 0
    for t, nodes in sched:
        q.factor(At, R, k, t)
        k = t
        before_Q, before_R = host(At), host(R)
        q.erase(At, R, nodes)
        torch.cuda.synchronize()
        erased_Q = np.isnan(host(At))
        assert erased_Q.any()
        q.recover(At, R, nodes)
        torch.cuda.synchronize()
        Qg, Rg = host(At), host(R)
        assert not np.isnan(Qg).any() and not np.isnan(Rg).any()
        assert rel(Qg[erased_Q], before_Q[erased_Q]) < 1e-10
        assert np.abs(Rg - before_R).max() <= 1e-10 * np.abs(before_R).max()
    q.factor(At, R, k, cfg.npanels)
    # the oracle with the same schedule
    prob = oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "icgs"), sched)
    out = oc.run(prob)
    Qg, Rg = host(At), host(R)
    assert rel(Rg, out["R"]) < 1e-11
    assert np.abs(Qg - out["Q"]).max() < 1e-11
    q.close()


@pytest.mark.parametrize("storage", ["out", "in"])
def test_failures_without_horizontal_code(cqr, storage):
    """An 8 x 1 grid has no R-checksum columns: R's checksum rows (the vertical
    code of its block rows) decode a failed node's R block row.  Out of node:
    two nodes at once, then a data and a checksum node; in node (f_tol = 1):
    one node per event."""
    n, pr, K, b, m = 128, 8, 2, 32, 1024
    A, v, gh, lay = make_inputs(n, pr, K, b, storage, seed=4, m=m, pc=1, kh=0)
    print(f"[case] no horizontal code, {storage} of node", flush=True)
    q = cqr.CodedQR(gpu_config(cqr, lay, b), v, gh)
    assert lay.rcode and q.r_rows == lay.rrows
    sched = [(1, [(1, 0), (5, 0)]), (3, [(2, 0), (pr + 1, 0)])] if storage == "out" else \
            [(1, [(3, 0)]), (3, [(1, 0)])]
    At, R = q.alloc()
    At[:lay.m, :lay.n].copy_(_dev(cqr, A))
    q.encode(At)
    k = 0
    for t, nodes in sched:
        q.factor(At, R, k, t)
        k = t
        before_Q, before_R = host(At), host(R)
        q.erase(At, R, nodes)
        torch.cuda.synchronize()
        erased_R = np.isnan(host(R))
        assert erased_R.any()
        q.recover(At, R, nodes)
        torch.cuda.synchronize()
        Qg, Rg = host(At), host(R)
        assert not np.isnan(Qg).any() and not np.isnan(Rg).any()
        assert rel(Qg, before_Q) < 1e-10
        assert np.abs(Rg - before_R).max() <= 1e-10 * np.abs(before_R).max()
    q.factor(At, R, k, n // b)
    out = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "icgs"), sched))
    Qg, Rg = host(At), host(R)
    q.close()
    assert rel(Rg[:n], out["R"]) < 1e-11
    assert np.abs(Qg - out["Q"]).max() < 1e-11


@pytest.mark.parametrize("sid,n,pr,K,b", [("innode", 512, 8, 2, 64), ("ragged", 240, 4, 1, 16),
                                          ("b32_5x5", 480, 5, 1, 32)])
def test_lookahead_matches_single_stream(cqr, sid, n, pr, K, b):
    """The second-stream schedule computes each panel's update coefficients as
    R2^{-T} (P1^T Q_t) from the first-pass panel instead of P^T Q_t, and splits
    products differently: equal up to rounding.  Both agree with the oracle.
    (b = 32 on a 5 x 5 grid: the early update's column counts end in half
    tiles, and its near launch is narrower than a tile.)"""
    print(f"[case] lookahead {sid}", flush=True)
    A, v, gh, lay = make_inputs(n, pr, K, b, "in" if sid == "innode" else "out", seed=7)
    sched = synth.draw_schedule("random", n // b, pr, pr, 7, nfail=1)
    out = {}
    for la in (0, 1):
        q = cqr.CodedQR(gpu_config(cqr, lay, b, lookahead=la), v, gh)
        At, R, _, _ = q.run(_dev(cqr, A), sched)
        torch.cuda.synchronize()
        out[la] = (host(At), host(R))
        assert q.info() == 0
        q.close()
    assert rel(out[1][1], out[0][1]) < 1e-13
    assert np.abs(out[1][0] - out[0][0]).max() < 1e-13
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "icgs"), sched))
    for la in (0, 1):
        assert rel(out[la][1], ref["R"]) < 1e-11
        assert np.abs(out[la][0] - ref["Q"]).max() < 1e-11


def test_postorth_matches_oracle(cqr):
    n, pr, K, b = 256, 8, 4, 32
    A, v, gh, lay = make_inputs(n, pr, K, b, "out", seed=3)
    rhs = synth.gaussian(n, 3, 33)
    q = cqr.CodedQR(gpu_config(cqr, lay, b), v, gh)
    At, R, Qp, Bp = q.run(_dev(cqr, A), [], _dev(cqr, rhs))
    out = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "cgs2"), [], rhs))
    Qpg, Bpg = host(Qp), host(Bp)
    assert rel(Qpg, out["Qpost"]) < 1e-11
    assert rel(Bpg, out["bpost"]) < 1e-14
    orth_or = np.linalg.norm(np.eye(n) - out["Qpost"].T @ out["Qpost"])
    orth = np.linalg.norm(np.eye(n) - Qpg.T @ Qpg)
    assert orth <= max(1e-12, 4 * orth_or)
    # in place
    Q1 = At[:lay.m, :n].clone()
    q.postorth(Q1, Q1)
    assert rel(host(Q1), Qpg) == 0.0
    x = oc.coded_solve(Qpg, host(R)[:, :n], Bpg)
    np.testing.assert_allclose(x, np.linalg.solve(A, rhs), rtol=1e-9, atol=1e-10)
    q.close()


def test_not_recoverable_and_invalid(cqr):
    n, pr, K, b = 256, 4, 1, 16
    A, v, gh, lay = make_inputs(n, pr, K, b, "out", seed=4)
    q = cqr.CodedQR(gpu_config(cqr, lay, b), v, gh)
    At, R = q.alloc()
    At[:n, :n].copy_(_dev(cqr, A))
    q.encode(At)
    q.factor(At, R, 0, 5)
    nodes = [(0, 1), (2, 1)]            # two erased data blocks in one block column, K = 1
    q.erase(At, R, nodes)
    torch.cuda.synchronize()
    snap = host(At)
    with pytest.raises(cqr.CqrError) as e:
        q.recover(At, R, nodes)
    assert e.value.status == cqr.CQR_ENOTRECOVERABLE
    torch.cuda.synchronize()
    np.testing.assert_array_equal(np.isnan(host(At)), np.isnan(snap))   # untouched
    assert cqr.coded_qr_recover(q.plan, At, R, [(9, 9)]) == cqr.CQR_EINVAL
    assert cqr.coded_qr_factor(q.plan, At, R, 3, 99, q.ws) == cqr.CQR_EINVAL
    small = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    assert cqr.coded_qr_factor(q.plan, At, R, 0, 1, small) == cqr.CQR_ENOMEM
    assert cqr.coded_qr_factor(q.plan, At, R, 5, 5, q.ws) == cqr.CQR_OK     # empty range
    q.close()


def test_uncoded_and_deterministic(cqr):
    n, pr, b = 256, 4, 32
    A = synth.gaussian(n, n, 5)
    lay = oc.Layout(n, n, pr, pr, 0, 0)
    q = cqr.CodedQR(gpu_config(cqr, lay, b), None, None)
    runs = []
    for _ in range(2):
        At, R = q.alloc()
        At.copy_(_dev(cqr, A))
        q.factor(At, R)
        torch.cuda.synchronize()
        runs.append((host(At), host(R)))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    Qh, Rh = np.linalg.qr(A)
    s = np.sign(np.diag(Rh))
    assert rel(runs[0][1], (Rh.T * s).T) < 1e-11
    q.close()


def test_paper_mode_without_reprojection(cqr):
    n, pr, K, b = 512, 8, 2, 64
    A, v, gh, lay = make_inputs(n, pr, K, b, "out", seed=6)
    q = cqr.CodedQR(gpu_config(cqr, lay, b, reproject=0), v, gh)
    At, R, _, _ = q.run(_dev(cqr, A))
    _, Qo, Ro, _, _ = oracle_state(A, v, gh, lay, b, n // b, reproject=False)
    assert rel(host(R), Ro) < 1e-11
    q.close()
