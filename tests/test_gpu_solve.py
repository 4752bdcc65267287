"""Coded linear solve on the GPU (coded_qr_solve): X = R_1^{-1} (G_0 Q_1)^T (G_0 B).

Each case checks:
- the solve kernels alone, on the oracle's own factors: X from the same
  Qpost, R, Bpost as the oracle's back substitution, up to rounding order
  (1e-11 relative);
- the whole GPU pipeline (encode, factor with failures, recover, post-orth,
  solve) against the oracle's pipeline (1e-9 relative);
- the closed form: A X = B for square A; for tall A the W-weighted least
  squares (A^T W A)^{-1} A^T W B with W = I + G_v^T G_v, within
  1e-13 cond(A) relative.
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


CASES = [
    # id, n, pr, K, b, storage, layout extras, nrhs, failures
    ("square_innode_failures", 512, 8, 2, 64, "in", {}, 1, 2),
    ("ragged_multi_rhs", 240, 4, 1, 16, "out", {}, 5, 1),
    ("tall_weighted_ls", 256, 8, 2, 64, "out", {"m": 1024, "pc": 1, "kh": 0}, 3, 0),
    ("one_block", 64, 4, 1, 16, "out", {}, 4, 0),
]


@pytest.mark.parametrize("sid,n,pr,K,b,storage,extra,nrhs,nfail", CASES, ids=[c[0] for c in CASES])
def test_solve_matches_oracle_and_closed_form(cqr, sid, n, pr, K, b, storage, extra, nrhs, nfail):
    print(f"[case] solve {sid}", flush=True)
    A, v, gh, lay = make_inputs(n, pr, K, b, storage, seed=21, **extra)
    B = synth.gaussian(lay.m, nrhs, 22)
    sched = synth.draw_schedule("random", n // b, pr, lay.pc, 21, nfail=nfail) if nfail else []
    dev = lambda x: cqr.to_device_colmajor(np.ascontiguousarray(x), "cuda:0")
    q = cqr.CodedQR(gpu_config(cqr, lay, b), v, gh if lay.kh else None)
    At, R, Qp, Bp = q.run(dev(A), sched, dev(B))
    X = host(q.solve(Qp, R, Bp))
    ref = oc.run(oc.Problem(A, lay, v, gh if lay.kh else None, oc.FactorOptions(b, "icgs"), sched, B))
    Xo = oc.coded_solve(ref["Qpost"], ref["R"][:, :n], ref["bpost"])
    X2 = host(q.solve(dev(ref["Qpost"]), dev(ref["R"]), dev(ref["bpost"])))
    torch.cuda.synchronize()
    q.close()
    assert X.shape == (n, nrhs) and np.isfinite(X).all()
    print(f"    kernels {rel(X2, Xo):.2e}  pipeline {rel(X, Xo):.2e}", flush=True)
    assert rel(X2, Xo) <= 1e-11
    assert rel(X, Xo) <= 1e-9
    if lay.m == n:
        Xc = np.linalg.solve(A, B)
    else:
        Gv = np.kron(oc.q_generator(v), np.eye(lay.bs))
        W = np.eye(lay.m) + Gv.T @ Gv
        Xc = np.linalg.solve(A.T @ W @ A, A.T @ W @ B)
    assert rel(X, Xc) <= 1e-13 * np.linalg.cond(A)


def test_solve_rejects_bad_arguments(cqr):
    A, v, gh, lay = make_inputs(64, 4, 1, 16, "out", seed=3)
    q = cqr.CodedQR(gpu_config(cqr, lay, 16), v, gh)
    Qp = cqr.col_major(lay.m, lay.n, q.device)
    R = cqr.col_major(lay.n, lay.N, q.device)
    Bp = cqr.col_major(lay.m, 2, q.device)
    X = cqr.col_major(lay.n - 1, 2, q.device)        # too few rows for X
    ws = q.solve_workspace(2)
    assert cqr.coded_qr_solve(q.plan, Qp, R, Bp, X, ws) == cqr.CQR_EINVAL
    X = cqr.col_major(lay.n, 2, q.device)
    small = ws[: ws.numel() // 2]                      # workspace too small
    assert cqr.coded_qr_solve(q.plan, Qp, R, Bp, X, small) == cqr.CQR_ENOMEM
    q.close()
