"""GPU parity on the codes, grids and failure patterns of the large workloads
and of the paper's overhead sweep, at sizes the FP64 oracle finishes in
seconds, through the C ABI in the launch configuration bench.py times
(lookahead on):

- the n = 32768 workload's code at n = 8192: 16 x 16 grid of 512 x 512
  blocks, b = 256, K = 8 in-node checksums (f_tol = 4; a decode uses 4 of the
  8), a reverse-diagonal storm of 4 nodes per grid row and column at panel 16.
  Its trailing products launch more than 256 workgroups, so the split rule
  for large grids runs.  Element by element against the oracle: R to 1e-11 of
  its largest entry, Q~ and the post-orthogonalized factor to the QR factor's
  forward error 10 u kappa_2(R_1) (times ||G^_0||_2), which at this size is
  above 1e-11 (the FP64 oracle's own Q~ moves by ~3e-11 when A changes by one
  ulp); every recovered block against its value before the erasure (1e-10);
  FP64 residual, and orthogonality within 4x the oracle's (the Frobenius norm
  of I - Q~^T Q~ sums n^2 rounding-size entries, ~1e-12 at this size);
- the n = 16384 workload's grid and code at n = 2048 with cond(A) = 1e10:
  8 x 8 grid, b = 128, K = 4 out-of-node, reverse-diagonal storms of 4 nodes
  every 4 panels.  An ill-conditioned A moves the factors by up to
  kappa(A) u, and the row checksums drift by ~u kappa(A) relative to a
  column's final norm, which a decode passes on through G_hat^{-1}: each
  recovered Q block is checked against G_hat^{-1} applied to the snapshot's
  measured drift (the decode gain ||G_hat^{-1}|| reaches ~5e4 for this code).
  Without failures the factorization reaches the FP64 residual and
  orthogonality within 4x the oracle's; with them, the final residual and
  orthogonality are bounded by the failure-free values plus the first-order
  effect of the measured recovery errors;
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


def _cond2_upper(R, iters=30):
    """kappa_2 of an upper-triangular R: power iteration on R^T R and on
    (R^T R)^{-1} (triangular solves), 30 steps each from a seeded start."""
    from scipy.linalg import solve_triangular
    rng = np.random.default_rng(0)
    x = rng.standard_normal(R.shape[0])
    for _ in range(iters):
        x = R.T @ (R @ x)
        x /= np.linalg.norm(x)
    smax = np.sqrt(np.linalg.norm(R.T @ (R @ x)))
    y = rng.standard_normal(R.shape[0])
    for _ in range(iters):
        y = solve_triangular(R, solve_triangular(R, y, trans="T"))
        y /= np.linalg.norm(y)
    smin = 1.0 / np.sqrt(np.linalg.norm(solve_triangular(R, solve_triangular(R, y, trans="T"))))
    return float(smax / smin)


def _q_decode_bound(q, Q0, nodes):
    """What a decode of the snapshot Q0 may differ from it by: per block column
    with erased data blocks F (lowest-index surviving checksums S), the decoded
    blocks get G_hat^{-1} (G_hat = G~_v[S, F]) applied to the checksum
    relation's error Q_2 - G_v Q_1 of the snapshot; the bound is the worst
    ||G_hat^{-1}||_inf times the worst relation error (absolute)."""
    c = q.cfg
    gv = q.generators()[0]
    bs, bw = c.m // c.pr, c.n // c.pc
    G = torch.tensor(np.kron(gv, np.eye(bs)), device=Q0.device, dtype=torch.float64)
    drift = (Q0[c.m:] - G @ Q0[:c.m]).abs().max().item()
    cols = {}
    for i, j in nodes:
        cols.setdefault(j, []).append(i)
    gain = 1.0
    for rows in cols.values():
        ghat = gv[np.ix_(list(range(len(rows))), sorted(rows))]
        gain = max(gain, float(np.abs(np.linalg.inv(ghat)).sum(axis=1).max()))
    del G
    return gain * drift, gain, drift


def _run_with_snapshots(cqr, q, A, sched, rhs, decode_bound=False, perturb=None):
    """The bench's step with a snapshot before each erasure; returns the
    factors, the post-orthogonalized outputs and the worst recovery error
    (relative to the snapshot's largest entry).  With decode_bound, the worst
    ratio of a recovery's error in Q~ to what the decode may make of the
    snapshot's checksum drift (_q_decode_bound) instead, and each event's
    Frobenius-norm changes (finished columns of Q~, the other columns, R)
    appended to `perturb`."""
    c = q.cfg
    At, R = q.alloc()
    At[:c.m, :c.n].copy_(cqr.to_device_colmajor(A, "cuda:0"))
    q.encode(At)
    worst = 0.0
    if perturb is not None:
        perturb.clear()
    k = 0
    for t, nodes in list(sched) + [(c.npanels, None)]:
        q.factor(At, R, k, t)
        k = t
        if nodes is None:
            break
        Q0, R0 = At.clone(), R.clone()
        bound = _q_decode_bound(q, Q0, nodes) if decode_bound else None
        q.erase(At, R, nodes)
        q.recover(At, R, nodes)
        eq = ((At - Q0).abs().max() / Q0.abs().max()).item()
        er = ((R - R0).abs().max() / R0.abs().max()).item()
        msg = f"    event at panel {t}: {len(nodes)} nodes, recovery Q~ {eq:.2e} R {er:.2e}"
        if decode_bound:
            ratio = (At - Q0).abs().max().item() / (1.01 * bound[0] + 1e-12 * Q0.abs().max().item())
            msg += f" (drift {bound[2]:.2e} x decode gain {bound[1]:.1f}; error / bound {ratio:.2f})"
            worst = max(worst, ratio, er / 1e-10, float("inf") if np.isnan(eq + er) else 0.0)
            done = t * c.b
            perturb.append((torch.linalg.norm(At[:, :done] - Q0[:, :done]).item(),
                            torch.linalg.norm(At[:, done:] - Q0[:, done:]).item(),
                            torch.linalg.norm(R - R0).item()))
        else:
            worst = max(worst, eq, er, float("inf") if np.isnan(eq + er) else 0.0)
        print(msg, flush=True)
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
    # Q~ and G_0 Q_1 move by O(u kappa(A)) elementwise under rounding-level
    # changes (the FP64 oracle itself moves them by ~3e-11 and ~7e-11 of their
    # largest entries when A changes by one ulp at this size): their bound is
    # the QR factor's forward error 10 u kappa_2(R_1), times ||G^_0||_2 for
    # G_0 Q_1; R's sensitivity is far smaller and keeps the 1e-11 bound
    kappa = _cond2_upper(ref["R"][:, :n])
    g0 = np.linalg.norm(oc.g0_tilde(oc.q_generator(inp["v"])), 2)
    bq = 10 * 2.0 ** -53 * kappa
    print(f"    vs oracle: R {eR:.2e} Q~ {eQ:.2e} G0 Q1 {eP:.2e} G0 b {rel(Bpg, ref['bpost']):.2e}; "
          f"kappa_2(R_1) {kappa:.2e}, Q~ bound {bq:.2e}, ||G^_0|| {g0:.2f}", flush=True)
    assert eR <= 1e-11 and eQ <= max(1e-11, bq)
    assert eP <= max(1e-10, g0 * bq) and rel(Bpg, ref["bpost"]) <= 1e-10
    A = inp["A"]
    res = np.linalg.norm(A - Qg[:n, :n] @ Rg[:, :n]) / np.linalg.norm(A)
    Qt = Qg[:, :n]
    orth = np.linalg.norm(np.eye(n) - Qt.T @ Qt)
    # ||I - Q~^T Q~||_F sums n^2 entries of rounding size: at n = 8192 the
    # oracle itself is near 1e-12, so the bound is 4x the oracle's
    Qo = ref["Q"][:, :n]
    orth_or = np.linalg.norm(np.eye(n) - Qo.T @ Qo)
    print(f"    residual {res:.2e} orth {orth:.2e} (oracle {orth_or:.2e})", flush=True)
    assert res <= 1e-12 and orth <= max(1e-12, 4 * orth_or)


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
    events = []
    Qg, Rg, Qpg, _, worst = _run_with_snapshots(cqr, q, A, sched, rhs, decode_bound=True, perturb=events)
    assert q.info() == 0
    q.close()
    # the row checksums drift by ~u kappa(A) relative to a column's final
    # norm; a decode turns that drift into its error through G_hat^{-1}, so a
    # recovered Q block is checked against that, R blocks against 1e-10
    assert worst <= 1.0
    # without failures: FP64 backward error, orthogonality within 4x the oracle's
    q0 = cqr.CodedQR(cqr.Config(n, n, pr, pr, K, K, b, cqr.CQR_OUT_OF_NODE, lookahead=1), v, gh)
    Q0g, R0g, _, _, _ = _run_with_snapshots(cqr, q0, A, [], rhs)
    q0.close()
    ref0 = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "cgs2"), [], rhs))
    m0, mo0 = oc.metrics(A, {"Q": Q0g, "R": R0g}, lay), oc.metrics(A, ref0, lay)
    print(f"    without failures: GPU {m0}\n    oracle {mo0}", flush=True)
    assert m0["residual"] <= 1e-12 and m0["orth_coded"] <= max(1e-12, 4 * mo0["orth_coded"])
    # with the storms: the recoveries' errors, measured against the snapshots,
    # perturb the factorization to first order.  An error d in finished columns
    # of Q~ changes Q~^T Q~ by at most 2 ||d||_F + ||d||_F^2; as a change of
    # the matrix being factored, d costs the residual ||d||_F ||R||_2, an error
    # in the unfinished columns its own norm, an error dR in R ||dR||_F.
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "cgs2"), sched, rhs))
    mg, mo = oc.metrics(A, {"Q": Qg, "R": Rg, "Qpost": Qpg}, lay), oc.metrics(A, ref, lay)
    fin = sum(e[0] for e in events)
    normR = np.linalg.norm(Rg[:, :n], 2)
    res_add = sum(e[1] + e[0] * normR + e[2] for e in events) / np.linalg.norm(A)
    b_orth = max(1e-12, 4 * mo0["orth_coded"]) + 2.01 * fin + fin * fin
    b_res = 1e-12 + 1.01 * res_add
    print(f"    GPU {mg}\n    oracle {mo}\n    R vs oracle {rel(Rg, ref['R']):.2e}; "
          f"bounds: orthogonality {b_orth:.2e}, residual {b_res:.2e}", flush=True)
    assert mg["orth_coded"] <= b_orth and mg["residual"] <= b_res
    assert mg["orth_post"] <= max(1e-12, 4 * mo["orth_post"]) + 2.01 * fin * np.linalg.norm(
        oc.g0_tilde(oc.q_generator(v)), 2)


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
