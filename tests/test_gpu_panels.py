"""The panel modes on the GPU against the FP64 oracle, through the C ABI.

- Column-wise CGS2, ICGS (DGKS test, eta = 1/sqrt 2) and MGS panels
  (CQR_PANEL_CGS2 / ICGS / MGS) against the oracle's panel of the same name:
  R and Q~ element by element (1e-11 of the largest entry), FP64 residual and
  orthogonality (1e-12), with and without failures, on a tall panel whose
  leaves take the kernel's widest grid (a ragged last slab), and the paper's
  method (MGS panel, no re-projection) at the n = 4096 workload's shape.
- The ICGS test taken both ways: at eta = 0.97 (most columns, not all,
  re-orthogonalised by the oracle) element by element, and with a nearly
  dependent pair in one panel, bounded against the oracle's orthogonality.
- A panel with two nearly dependent columns (one 1e-9 from another,
  cond(A) ~ 1e11): the Cholesky-QR panel breaks down and the column-wise
  CGS2 fallback takes the panel; the result is bounded by backward error
  against the oracle (FP64 residual; orthogonality within 4x the oracle's,
  which reaches 1e-13 when the pair sits in the first panel and ~5e-7 when it
  sits in a later one, where the intra-panel projection re-introduces
  components along the earlier basis after the re-projection; G_0 Q_1 within
  4x the oracle's, whose checksum drift grows like u kappa(A)), both
  where the panel is the first (no re-projection, no early update) and where
  its update already started from the first pass (the early update then
  forms its coefficients from the finished panel).  With a node failure
  mid-factorization, a decode carries that drift into the recovered blocks
  (the FP64 oracle itself then ends near residual 1e-8 and orthogonality
  4e-7), so residual and orthogonality are bounded against the oracle's.
"""
import numpy as np
import pytest

import synth
from oracle import coded_qr as oc
from tests.gpu_helpers import gpu_config, host, make_inputs, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cqr():
    from paper_2311_11943_amd import cqr as mod
    return mod


MODES = {"cgs2": 1, "icgs": 2, "mgs": 3}
SHAPES = [
    # id, n, pr, K, b, storage
    ("c1", 256, 4, 1, 16, "out"),
    ("innode", 512, 8, 2, 64, "in"),
    ("ragged", 240, 4, 1, 16, "out"),
    ("wide_panel", 512, 4, 2, 128, "out"),     # leaves of 64 columns, block projections between them
    ("odd_panel", 384, 4, 1, 48, "out"),
]


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("sid,n,pr,K,b,storage", SHAPES, ids=[s[0] for s in SHAPES])
def test_columnwise_panels_match_oracle(cqr, mode, sid, n, pr, K, b, storage):
    print(f"[case] panel {mode} {sid}", flush=True)
    A, v, gh, lay = make_inputs(n, pr, K, b, storage, seed=11)
    sched = synth.draw_schedule("random", n // b, pr, pr, 11, nfail=1)
    q = cqr.CodedQR(gpu_config(cqr, lay, b, panel=MODES[mode]), v, gh)
    At, R, _, _ = q.run(cqr.to_device_colmajor(A, "cuda:0"), sched)
    torch.cuda.synchronize()
    assert q.info() == 0 and q.panel_fallbacks() == 0
    Qg, Rg = host(At), host(R)
    q.close()
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, mode), sched))
    m = oc.metrics(A, {"Q": Qg, "R": Rg}, lay)
    print(f"    R {rel(Rg, ref['R']):.2e} Q {rel(Qg, ref['Q']):.2e} {m}", flush=True)
    assert rel(Rg, ref["R"]) <= 1e-11 and rel(Qg, ref["Q"]) <= 1e-11
    assert m["residual"] <= 1e-12 and m["orth_coded"] <= 1e-12


@pytest.mark.parametrize("m", [40000, 60000], ids=["one_row_per_thread", "two_rows_per_thread"])
@pytest.mark.parametrize("mode", sorted(MODES))
def test_columnwise_panels_on_the_widest_grid(cqr, mode, m):
    """Tall panels (16 x 1 grid, K_v = 4 out-of-node, no horizontal code,
    n = 192, b = 64, one failure) whose leaves take the column-wise kernel's
    widest grids: m' = 50000 rows (196 workgroups, one row per thread, a
    short last slab) and m' = 75000 (the 256-workgroup cap, two row blocks
    per thread, the second one partly empty), against the oracle's panel of
    the same name."""
    n, pr, K, b = 192, 16, 4, 64
    A, v, _, lay = make_inputs(n, pr, K, b, "out", seed=3, m=m, pc=1, kh=0)
    sched = synth.draw_schedule("random", n // b, pr, 1, 3, nfail=1)
    print(f"[case] panel {mode} m'={lay.mp} n={n}, schedule {sched}", flush=True)
    q = cqr.CodedQR(gpu_config(cqr, lay, b, panel=MODES[mode]), v, None)
    At, R, _, _ = q.run(cqr.to_device_colmajor(A, "cuda:0"), sched)
    torch.cuda.synchronize()
    assert q.info() == 0
    Qg, Rg = host(At), host(R)
    q.close()
    ref = oc.run(oc.Problem(A, lay, v, None, oc.FactorOptions(b, mode), sched))
    # R's own checksum rows follow its n rows (the oracle returns R_1's rows)
    Rg = Rg[:n]
    res = np.linalg.norm(A - Qg[:m, :n] @ Rg[:n, :n]) / np.linalg.norm(A)
    orth = np.linalg.norm(np.eye(n) - Qg[:, :n].T @ Qg[:, :n])
    print(f"    R {rel(Rg, ref['R']):.2e} Q {rel(Qg, ref['Q']):.2e} residual {res:.2e} orth {orth:.2e}", flush=True)
    assert rel(Rg, ref["R"]) <= 1e-11 and rel(Qg, ref["Q"]) <= 1e-11
    assert res <= 1e-12 and orth <= 1e-12


@pytest.mark.parametrize("eta,pair", [(0.97, None), (2 ** -0.5, (140, 170))], ids=["eta0.97", "dependent_pair"])
def test_icgs_reorthogonalises_where_the_oracle_does(cqr, eta, pair):
    """The ICGS test (second projection when ||p_j|| < eta ||p_j before||)
    taken both ways: at eta = 0.97 the oracle re-orthogonalises some columns
    of every panel and not others, and the GPU's R and Q~ must match it
    element by element; with the default eta and a column 1e-9 from another of
    its panel, the second projection is what keeps Q~ orthogonal, so residual
    and orthogonality are bounded against the oracle's (backward error)."""
    n, pr, K, b = 512, 8, 2, 64
    A, v, gh, lay = make_inputs(n, pr, K, b, "in", seed=21)
    A = A.copy()
    if pair:
        A[:, pair[1]] = A[:, pair[0]] + 1e-9 * np.random.default_rng(2).standard_normal(n)
    print(f"[case] icgs eta {eta:.3f} pair {pair}", flush=True)
    q = cqr.CodedQR(gpu_config(cqr, lay, b, panel=MODES["icgs"], icgs_eta=eta), v, gh)
    At, R, _, _ = q.run(cqr.to_device_colmajor(A, "cuda:0"), [])
    torch.cuda.synchronize()
    assert q.info() == 0
    Qg, Rg = host(At), host(R)
    q.close()
    opt = oc.FactorOptions(b, "icgs", eta=eta)
    gv, ghm = oc.q_generator(v), oc.r_generator(gh, lay.storage)
    Q = oc.encode(A, gv, ghm, lay)
    Ro = np.zeros((lay.n, lay.N))
    nre = oc.factor_panels(Q, Ro, lay.n, 0, n // b, opt)["reorth_columns"]
    mg = oc.metrics(A, {"Q": Qg, "R": Rg}, lay)
    mo = oc.metrics(A, {"Q": Q, "R": Ro}, lay)
    print(f"    oracle re-orthogonalised {nre} of {lay.n} columns; R {rel(Rg, Ro):.2e} Q {rel(Qg, Q):.2e}\n"
          f"    GPU {mg}\n    oracle {mo}", flush=True)
    assert 0 < nre < lay.n
    if pair is None:
        assert rel(Rg, Ro) <= 1e-11 and rel(Qg, Q) <= 1e-11
        assert mg["residual"] <= 1e-12 and mg["orth_coded"] <= 1e-12
    else:
        assert mg["residual"] <= 1e-12
        assert mg["orth_coded"] <= max(1e-12, 4 * mo["orth_coded"])


def test_paper_method_mgs_without_reprojection(cqr):
    """The paper's method: MGS panels, no re-projection (n = 4096, 8 x 8 grid,
    b = 64, K = 2 in-node, two random failures)."""
    import bench
    w = bench.WORKLOADS["c2"]
    n, pr, K, b = w["n"], w["pr"], w["K"], w["b"]
    inp = bench.workload_inputs("c2", oc.f_tolerated(K, pr, oc.IN_NODE), 0)
    lay = oc.Layout(n, n, pr, pr, K, K, oc.IN_NODE)
    print(f"[case] paper method at n={n}, schedule {inp['schedule']}", flush=True)
    q = cqr.CodedQR(gpu_config(cqr, lay, b, reproject=0, panel=cqr.CQR_PANEL_MGS), inp["v"], inp["gh"])
    At, R, _, _ = q.run(cqr.to_device_colmajor(inp["A"], "cuda:0"), inp["schedule"])
    torch.cuda.synchronize()
    assert q.info() == 0
    Qg, Rg = host(At), host(R)
    q.close()
    ref = oc.run(oc.Problem(inp["A"], lay, inp["v"], inp["gh"], oc.FactorOptions(b, "mgs", reproject=False),
                            inp["schedule"]))
    mg, mo = oc.metrics(inp["A"], {"Q": Qg, "R": Rg}, lay), oc.metrics(inp["A"], ref, lay)
    print(f"    R {rel(Rg, ref['R']):.2e} Q {rel(Qg, ref['Q']):.2e}\n    GPU {mg}\n    oracle {mo}", flush=True)
    assert rel(Rg, ref["R"]) <= 1e-11 and rel(Qg, ref["Q"]) <= 1e-10
    assert mg["residual"] <= 1e-12
    assert mg["orth_coded"] <= max(1e-12, 4 * mo["orth_coded"])


@pytest.mark.parametrize("cols,lookahead,fail", [((12, 37), 1, False), ((140, 170), 1, False),
                                                 ((140, 170), 0, False), ((140, 170), 1, True)],
                         ids=["first_panel", "later_panel", "later_panel_one_stream", "later_panel_with_failure"])
def test_nearly_dependent_columns_fall_back(cqr, cols, lookahead, fail):
    n, pr, K, b = 512, 8, 2, 64
    A, v, gh, lay = make_inputs(n, pr, K, b, "in", seed=5)
    A = A.copy()
    A[:, cols[1]] = A[:, cols[0]] + 1e-9 * np.random.default_rng(1).standard_normal(n)
    rhs = synth.gaussian(n, 1, 6)
    sched = [(6, [(3, 5)])] if fail else []
    print(f"[case] columns {cols} 1e-9 apart, cond {np.linalg.cond(A):.1e}, lookahead {lookahead}, "
          f"failures {sched}", flush=True)
    q = cqr.CodedQR(gpu_config(cqr, lay, b, lookahead=lookahead), v, gh)
    At, R, Qp, _ = q.run(cqr.to_device_colmajor(A, "cuda:0"), sched, cqr.to_device_colmajor(rhs, "cuda:0"))
    torch.cuda.synchronize()
    info, fallbacks = q.info(), q.panel_fallbacks()
    Qg, Rg, Qpg = host(At), host(R), host(Qp)
    q.close()
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "cgs2"), sched, rhs))
    mg = oc.metrics(A, {"Q": Qg, "R": Rg, "Qpost": Qpg}, lay)
    mo = oc.metrics(A, ref, lay)
    print(f"    info {info} fallbacks {fallbacks}\n    GPU {mg}\n    oracle {mo}", flush=True)
    assert info == 0 and fallbacks >= 1
    if not fail:
        assert mg["residual"] <= 1e-12
    else:
        # a decode mid-factorization carries the checksum drift (u kappa(A) on
        # both sides) into the recovered blocks: bounded against the oracle
        assert mg["residual"] <= max(1e-12, 4 * mo["residual"])
    # in a panel after the first, projecting the nearly dependent column
    # against its partner re-introduces components along the earlier basis of
    # size u kappa(panel) after the re-projection has removed them, in the
    # oracle as on the GPU: orthogonality is bounded against the oracle's
    assert mg["orth_coded"] <= max(1e-12, 4 * mo["orth_coded"])
    assert mg["orth_post"] <= max(1e-12, 4 * mo["orth_post"])
