"""GPU parity on the codes, grids and failure patterns of the large workloads
and of the paper's overhead sweep, at sizes the FP64 oracle finishes in
seconds, through the C ABI in the launch configuration bench.py times
(lookahead on):

- the n = 32768 workload's code at n = 8192: 16 x 16 grid of 512 x 512
  blocks, b = 256, K = 8 in-node checksums (f_tol = 4; a decode uses 4 of the
  8), a reverse-diagonal storm of 4 nodes per grid row and column at panel 16.
  Its trailing products launch more than 256 workgroups, so the split rule
  for large grids runs.  Element by element against the oracle (R, Q~ and the
  post-orthogonalized factor to 1e-11 / 1e-10 of their largest entries), every
  recovered block against its value before the erasure (1e-10);
- the n = 16384 workload's grid and code at n = 2048 with cond(A) = 1e10:
  8 x 8 grid, b = 128, K = 4 out-of-node, reverse-diagonal storms of 4 nodes
  every 4 panels.  An ill-conditioned A moves the factors by up to
  kappa(A) u, so the comparison with the oracle is by backward error: both
  reach the FP64 residual and orthogonality bounds, and G_0 Q_1 matches the
  oracle's orthogonality within a factor of 4 (its drift grows with
  kappa(A) u on both sides);
- one point of the paper's sweep at reduced n: p = 6, f = 3 out-of-node
  checksums, one panel per grid block column (n = 1536, b = 256, factored
  recursively), a reverse-diagonal failure of 3 nodes per grid line at every
  panel boundary; element by element against the oracle.
"""
import numpy as np
import pytest

import synth
from oracle import coded_qr as oc
from tests.gpu_helpers import host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cqr():
    from paper_2311_11943_amd import cqr as mod
    return mod


def _run_with_snapshots(cqr, q, A, sched, rhs):
    """The bench's step with a snapshot before each erasure; returns the
    factors, the post-orthogonalized outputs and the worst recovery error
    (relative to the snapshot's largest entry)."""
    c = q.cfg
    At, R = q.alloc()
    At[:c.m, :c.n].copy_(cqr.to_device_colmajor(A, "cuda:0"))
    q.encode(At)
    worst = 0.0
    k = 0
    for t, nodes in list(sched) + [(c.npanels, None)]:
        q.factor(At, R, k, t)
        k = t
        if nodes is None:
            break
        Q0, R0 = At.clone(), R.clone()
        q.erase(At, R, nodes)
        q.recover(At, R, nodes)
        eq = ((At - Q0).abs().max() / Q0.abs().max()).item()
        er = ((R - R0).abs().max() / R0.abs().max()).item()
        print(f"    event at panel {t}: {len(nodes)} nodes, recovery Q~ {eq:.2e} R {er:.2e}", flush=True)
        worst = max(worst, eq, er, float("inf") if np.isnan(eq + er) else 0.0)
        del Q0, R0
    Qp = cqr.col_major(c.m, c.n, "cuda:0")
    Bp = cqr.col_major(c.m, 1, "cuda:0")
    B = cqr.to_device_colmajor(rhs, "cuda:0")
    q.postorth(At, Qp, B, Bp)
    torch.cuda.synchronize()
    return host(At), host(R), host(Qp), host(Bp), worst


def test_large_workload_code_matches_oracle(cqr):
    import bench
    w = bench.WORKLOADS["c5"]
    n, pr, K, b = 8192, w["pr"], w["K"], w["b"]
    inp = bench.workload_inputs_at(w, n, 0)
    sched = inp["schedule"]
    print(f"[case] c5 code at n={n}: {len(sched)} event(s), {len(sched[0][1])} nodes at panel {sched[0][0]}",
          flush=True)
    assert sched and sched[0][0] == 16 and len(sched[0][1]) == 4 * pr
    lay = oc.Layout(n, n, pr, pr, K, K, oc.IN_NODE)
    q = cqr.CodedQR(cqr.Config(n, n, pr, pr, K, K, b, cqr.CQR_IN_NODE, lookahead=1), inp["v"], inp["gh"])
    assert q.ftol == 4
    Qg, Rg, Qpg, Bpg, worst = _run_with_snapshots(cqr, q, inp["A"], sched, inp["rhs"])
    assert q.info() == 0
    q.close()
    assert worst <= 1e-10
    ref = oc.run(oc.Problem(inp["A"], lay, inp["v"], inp["gh"], oc.FactorOptions(b, "cgs2"), sched, inp["rhs"]))
    eR, eQ, eP = rel(Rg, ref["R"]), rel(Qg, ref["Q"]), rel(Qpg, ref["Qpost"])
    print(f"    vs oracle: R {eR:.2e} Q~ {eQ:.2e} G0 Q1 {eP:.2e} G0 b {rel(Bpg, ref['bpost']):.2e}", flush=True)
    assert eR <= 1e-11 and eQ <= 1e-11
    assert eP <= 1e-10 and rel(Bpg, ref["bpost"]) <= 1e-10
    A = inp["A"]
    res = np.linalg.norm(A - Qg[:n, :n] @ Rg[:, :n]) / np.linalg.norm(A)
    Qt = Qg[:, :n]
    orth = np.linalg.norm(np.eye(n) - Qt.T @ Qt)
    print(f"    residual {res:.2e} orth {orth:.2e}", flush=True)
    assert res <= 1e-12 and orth <= 1e-12


def test_conditioned_grid_code_backward_error(cqr):
    n, pr, K, b, cond = 2048, 8, 4, 128, 1e10
    A = synth.conditioned(n, cond, 3)
    v = synth.q_generator_draws(K, pr, 3)
    gh = synth.r_generator_draws(pr, K, 3)
    rhs = synth.gaussian(n, 1, 4)
    sched = synth.draw_schedule("revdiag", n // b, pr, pr, 3, every=4, f=K)
    print(f"[case] c3 code at n={n}, cond {cond:g}: storms at {[t for t, _ in sched]}", flush=True)
    lay = oc.Layout(n, n, pr, pr, K, K, oc.OUT_OF_NODE)
    q = cqr.CodedQR(cqr.Config(n, n, pr, pr, K, K, b, cqr.CQR_OUT_OF_NODE, lookahead=1), v, gh)
    Qg, Rg, Qpg, _, worst = _run_with_snapshots(cqr, q, A, sched, rhs)
    assert q.info() == 0
    q.close()
    assert worst <= 1e-10
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "cgs2"), sched, rhs))
    mg, mo = oc.metrics(A, {"Q": Qg, "R": Rg, "Qpost": Qpg}, lay), oc.metrics(A, ref, lay)
    print(f"    GPU {mg}\n    oracle {mo}\n    R vs oracle {rel(Rg, ref['R']):.2e}", flush=True)
    assert mg["residual"] <= 1e-12 and mo["residual"] <= 1e-12
    assert mg["orth_coded"] <= 1e-12 and mo["orth_coded"] <= 1e-12
    assert mg["orth_post"] <= max(1e-12, 4 * mo["orth_post"])


def test_sweep_point_matches_oracle(cqr):
    p, f, n = 6, 3, 1536
    b = n // p
    A = synth.gaussian(n, n, 5)
    v = synth.q_generator_draws(f, p, 5)
    gh = synth.r_generator_draws(p, f, 5)
    rhs = synth.gaussian(n, 1, 6)
    sched = synth.draw_schedule("revdiag", p, p, p, 5, every=1, f=f)
    print(f"[case] sweep point p={p} f={f} n={n} b={b}: failures at panels {[t for t, _ in sched]}", flush=True)
    assert len(sched) == p - 1
    lay = oc.Layout(n, n, p, p, f, f, oc.OUT_OF_NODE)
    q = cqr.CodedQR(cqr.Config(n, n, p, p, f, f, b, cqr.CQR_OUT_OF_NODE, lookahead=1), v, gh)
    Qg, Rg, Qpg, Bpg, worst = _run_with_snapshots(cqr, q, A, sched, rhs)
    assert q.info() == 0
    q.close()
    assert worst <= 1e-10
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "cgs2"), sched, rhs))
    eR, eQ = rel(Rg, ref["R"]), rel(Qg, ref["Q"])
    print(f"    vs oracle: R {eR:.2e} Q~ {eQ:.2e} G0 Q1 {rel(Qpg, ref['Qpost']):.2e}", flush=True)
    assert eR <= 1e-11 and eQ <= 1e-11 and rel(Qpg, ref["Qpost"]) <= 1e-10
    mg = oc.metrics(A, {"Q": Qg, "R": Rg}, lay)
    assert mg["residual"] <= 1e-12 and mg["orth_coded"] <= 1e-12
