"""Mixed precision (trailing-update products in FP32 on MFMA, everything else
FP64) against the FP64 oracle.

Bounds for this form, at every conditioning and also after failures:
||I - Q~^T Q~||_F <= 1e-5 (the stated mixed-precision target) and
||A - Q_1 R_1||_F / ||A||_F <= 1e-6, or 1e-5 after failures (a decoded block of
unfinished columns carries the FP32 checksum drift of the updates so far,
amplified by the decode solve, and enters A as a perturbation of that size:
about 1e-6 here against 1e-7 without failures).  The FP32 updates act as a backward
perturbation of about u32 ||A|| (u32 = 6e-8), so the deviation from the FP64
oracle moves with u32 kappa(A): it is bounded for the Gaussian inputs
(kappa ~ 1e3: R within 1e-5, Q~ within 1e-3 of the oracle, relative to the
largest entry) and printed for the conditioned ones.  Each panel's checksum
rows are re-derived in FP64 before the panel is factored, so the finished
columns keep Q_2 = G_v Q_1 to FP64 rounding (1e-10 relative) and blocks of
finished columns decode to FP64 accuracy; unfinished columns and the R
checksum columns hold their relations to FP32 rounding of the updates
(1e-4 relative).
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
    # id, n, pr, K, b, storage, kind, cond
    ("innode_gauss", 512, 8, 2, 64, "in", "gauss", 1.0),
    ("innode_cond1e6", 512, 8, 2, 64, "in", "cond", 1e6),
    ("wide_panel_cond1e10", 512, 4, 2, 128, "out", "cond", 1e10),
    # panels of two tile rows: the 16-deep FP32 product, also with a ragged
    # second tile row (b = 120) and a partial last slab (600 coded rows)
    ("wide_panel_gauss", 512, 4, 2, 128, "out", "gauss", 1.0),
    ("ragged_wide_panel", 480, 4, 1, 120, "out", "gauss", 1.0),
    # four tile rows: the FP32 form of the two-tile-row product
    ("panel256", 1024, 4, 1, 256, "out", "gauss", 1.0),
    ("ragged", 240, 4, 1, 16, "out", "gauss", 1.0),
]


@pytest.mark.parametrize("sid,n,pr,K,b,storage,kind,cond", CASES, ids=[c[0] for c in CASES])
def test_fp32_trailing_matches_fp64_oracle(cqr, sid, n, pr, K, b, storage, kind, cond):
    print(f"[case] mixed {sid}", flush=True)
    A, v, gh, lay = make_inputs(n, pr, K, b, storage, seed=8, kind=kind, cond=cond)
    cfg = gpu_config(cqr, lay, b, precision=cqr.CQR_TRAIL_FP32)
    q = cqr.CodedQR(cfg, v, gh)
    At, R, _, _ = q.run(cqr.to_device_colmajor(A, "cuda:0"))
    torch.cuda.synchronize()
    assert q.info() == 0
    Qg, Rg = host(At), host(R)
    q.close()
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "cgs2"), []))
    Qt = Qg[:, :n]
    orth = np.linalg.norm(np.eye(n) - Qt.T @ Qt)
    res = np.linalg.norm(A - Qg[:lay.m, :n] @ Rg[:, :n]) / np.linalg.norm(A)
    print(f"    orth {orth:.2e} res {res:.2e} R {rel(Rg, ref['R']):.2e} Q {rel(Qg, ref['Q']):.2e}", flush=True)
    assert orth <= 1e-5 and res <= 1e-6
    gv = oc.q_generator(v)
    Gv = oc.kron_generator(gv, lay.bs)
    drift_q = np.abs(Qg[lay.m:, :n] - Gv @ Qg[:lay.m, :n]).max() / np.abs(Qg).max()
    drift_r = 0.0
    if lay.kh:
        Gh = oc.kron_generator(oc.r_generator(gh, lay.storage), lay.bw)
        drift_r = np.abs(Rg[:, n:] - Rg[:, :n] @ Gh).max() / np.abs(Rg).max()
    carried = np.abs(Qg[:, n:]).max() / np.abs(Qg).max()
    print(f"    checksum drift Q {drift_q:.2e} R {drift_r:.2e}, carried residual {carried:.2e}", flush=True)
    assert drift_q <= 1e-10 and drift_r <= 1e-4
    if kind == "gauss":
        assert rel(Rg, ref["R"]) <= 1e-5
        assert rel(Qg[:, :n], ref["Q"][:, :n]) <= 1e-3
        assert carried <= 1e-4


def test_fp32_trailing_recovers_failures(cqr):
    n, pr, K, b = 512, 8, 2, 64
    A, v, gh, lay = make_inputs(n, pr, K, b, "in", seed=9)
    q = cqr.CodedQR(gpu_config(cqr, lay, b, precision=cqr.CQR_TRAIL_FP32), v, gh)
    sched = synth.draw_schedule("random", n // b, pr, pr, 9, nfail=2)
    At, R = q.alloc()
    At[:lay.m, :lay.n].copy_(cqr.to_device_colmajor(A, "cuda:0"))
    q.encode(At)
    k = 0
    for t, nodes in sched:
        q.factor(At, R, k, t)
        k = t
        before_Q, before_R = host(At), host(R)
        q.erase(At, R, nodes)
        q.recover(At, R, nodes)
        torch.cuda.synchronize()
        Qg, Rg = host(At), host(R)
        done = t * b
        fin = rel(Qg[:, :done], before_Q[:, :done])
        print(f"    failure at panel {t}: finished columns {fin:.2e}, all {rel(Qg, before_Q):.2e}, "
              f"R {np.abs(Rg - before_R).max() / np.abs(before_R).max():.2e}", flush=True)
        assert fin <= 1e-10
        assert rel(Qg, before_Q) <= 1e-5 and np.abs(Rg - before_R).max() <= 1e-5 * np.abs(before_R).max()
    q.factor(At, R, k, n // b)
    torch.cuda.synchronize()
    Qg, Rg = host(At), host(R)
    q.close()
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "icgs"), sched))
    assert rel(Rg, ref["R"]) <= 1e-5
    Qt = Qg[:, :n]
    orth = np.linalg.norm(np.eye(n) - Qt.T @ Qt)
    res = np.linalg.norm(A - Qg[:lay.m, :n] @ Rg[:, :n]) / np.linalg.norm(A)
    print(f"    after failures: orth {orth:.2e} res {res:.2e}", flush=True)
    assert orth <= 1e-5 and res <= 1e-5
