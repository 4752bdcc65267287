"""The largest code line the library takes (p_r + K_v = p_c + K_h = 32
blocks: a 24 x 24 grid with K = 8 out-of-node checksums each way) through the
C ABI against the FP64 oracle: encode and factor, then a storm of eight node
failures in one grid column at a panel boundary (eight erased data blocks in
one block column of Q, decoded from all eight checksum rows; one block in
each of eight block rows of R), recovery, the rest of the factorization and
post-orthogonalization.

Bounds: a decoded block's error is the rounding of the decode's right-hand
side (about u times the blocks it sums) amplified by ||G_hat^{-1}||_inf, the
decode gain, so recovered blocks are checked against the snapshot taken
before the erasure within 1e-13 x gain of the matrix's largest entry, and
the final factors against the oracle (which decodes with the same G_hat)
within 1e-11 x gain."""
import numpy as np
import pytest

from oracle import coded_qr as oc
from tests.gpu_helpers import gpu_config, host, make_inputs, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gain(gen: np.ndarray, lost: list) -> float:
    """||G_hat^{-1}||_inf with G_hat the generator's columns `lost` over its
    lowest-index rows (all checksums survive)."""
    ghat = gen[np.ix_(range(len(lost)), lost)]
    return float(np.abs(np.linalg.inv(ghat)).sum(axis=1).max())


def test_largest_code_line_recovers_and_matches_oracle():
    from paper_2311_11943_amd import cqr
    n, pr, K, b = 384, 24, 8, 16
    A, v, gh, lay = make_inputs(n, pr, K, b, "out", seed=3)
    col = 3
    nodes = [(i, col) for i in range(K)]
    sched = [(12, nodes)]
    print(f"[case] max line: {pr} x {pr} grid, K = {K}, storm {sched}", flush=True)
    q = cqr.CodedQR(gpu_config(cqr, lay, b), v, gh)
    assert q.ftol == K
    gain = max(_gain(oc.q_generator(v), list(range(K))), 1.0)
    At, R = q.alloc()
    At[:lay.m, :lay.n].copy_(cqr.to_device_colmajor(A, "cuda:0"))
    q.encode(At)
    q.factor(At, R, 0, 12)
    before_Q, before_R = host(At), host(R)
    q.erase(At, R, nodes)
    torch.cuda.synchronize()
    erased = np.isnan(host(At))
    assert erased.any()
    q.recover(At, R, nodes)
    torch.cuda.synchronize()
    Qg, Rg = host(At), host(R)
    err_q = np.abs(Qg - before_Q).max() / np.abs(before_Q).max()
    err_r = np.abs(Rg - before_R).max() / np.abs(before_R).max()
    print(f"    recovery: Q {err_q:.2e}, R {err_r:.2e} (decode gain {gain:.1f})", flush=True)
    assert err_q <= 1e-13 * gain and err_r <= 1e-13 * gain
    q.factor(At, R, 12, n // b)
    Qp = cqr.col_major(lay.m, lay.n, "cuda:0")
    q.postorth(At, Qp)
    torch.cuda.synchronize()
    Qg, Rg, Qpg = host(At), host(R), host(Qp)
    q.close()
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "icgs"), sched))
    errs = (rel(Rg, ref["R"]), np.abs(Qg - ref["Q"]).max(), rel(Qpg, ref["Qpost"]))
    print("    vs oracle: R {:.2e}  Q~ (abs) {:.2e}  Qpost {:.2e}".format(*errs), flush=True)
    assert errs[0] <= 1e-11 * gain and errs[1] <= 1e-11 * gain and errs[2] <= 1e-10 * gain
    res = np.linalg.norm(A - Qg[:n, :n] @ Rg[:, :n]) / np.linalg.norm(A)
    orth = np.linalg.norm(np.eye(n) - Qg[:, :n].T @ Qg[:, :n])
    print(f"    residual {res:.2e}  orth {orth:.2e}", flush=True)
    assert res <= 1e-12 and orth <= 1e-12


@pytest.mark.parametrize("sid,n,pr,b", [("uncoded_4x4", 256, 4, 16), ("single_node", 128, 1, 16),
                                        ("uncoded_wide_panels", 512, 2, 128)])
def test_uncoded_grids_match_oracle(sid, n, pr, b):
    """Degenerate codes: no checksums at all (K = 0; the uncoded runs the
    overhead figures compare against), also on a 1 x 1 grid, and with
    128-column panels on the 128 x 128-tile kernels."""
    from paper_2311_11943_amd import cqr
    A, v, gh, lay = make_inputs(n, pr, 0, b, "out", seed=5)
    print(f"[case] {sid}", flush=True)
    q = cqr.CodedQR(gpu_config(cqr, lay, b), None, None)
    At, R, _, _ = q.run(cqr.to_device_colmajor(A, "cuda:0"))
    torch.cuda.synchronize()
    assert q.info() == 0
    Qg, Rg = host(At), host(R)
    q.close()
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "cgs2"), []))
    print(f"    R {rel(Rg, ref['R']):.2e}  Q {np.abs(Qg - ref['Q']).max():.2e}", flush=True)
    assert rel(Rg, ref["R"]) < 1e-11 and np.abs(Qg - ref["Q"]).max() < 1e-11
