"""Full-size parity on the tall-skinny least-squares workload (m = 65536,
n = 512 Gaussian A and b, 16 x 1 grid of 4096-row blocks, b = 64, K_v = 2
out-of-node checksum block rows, no horizontal code, so R carries its own
checksum rows; two nodes failing at once at a random panel), the shape that
bench.py --adjoint times:
  - encode, factor with the erasure and recovery, post-orthogonalization and
    the coded solve through the C ABI against the FP64 oracle, element by
    element;
  - the adjoint kernels (coded_qr_backward, coded_qr_solve_backward) on the
    oracle's factors against the adjoint oracle.
The oracle takes a few seconds per pass on the host cores at this size."""
import numpy as np
import pytest

import synth
from oracle import adjoint as oa
from oracle import coded_qr as oc
from tests.gpu_helpers import gpu_config, host, make_inputs, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

M, N, PR, K, B = 65536, 512, 16, 2, 64


@pytest.fixture(scope="module")
def tall():
    from paper_2311_11943_amd import cqr
    A, v, _, lay = make_inputs(N, PR, K, B, "out", seed=0, m=M, pc=1, kh=0)
    rhs = synth.gaussian(M, 1, 1)
    sched = synth.draw_schedule("burst", N // B, PR, 1, 0, nfail=2)
    ref = oc.run(oc.Problem(A, lay, v, None, oc.FactorOptions(B, "cgs2"), sched, rhs))
    return cqr, A, v, lay, rhs, sched, ref


def _dev(cqr, x):
    return cqr.to_device_colmajor(np.ascontiguousarray(x), "cuda:0")


def test_tall_workload_matches_oracle(tall):
    cqr, A, v, lay, rhs, sched, ref = tall
    print(f"[case] tall full size m={M} n={N}, schedule {sched}", flush=True)
    assert len(sched) == 1 and len(sched[0][1]) == 2
    q = cqr.CodedQR(gpu_config(cqr, lay, B), v, None)
    At, R, Qp, Bp = q.run(_dev(cqr, A), sched, _dev(cqr, rhs))
    X = host(q.solve(Qp, R, Bp))
    torch.cuda.synchronize()
    assert q.info() == 0
    Qg, Rg, Qpg, Bpg = host(At), host(R), host(Qp), host(Bp)
    q.close()
    # R's own checksum rows follow its n rows (the oracle returns R_1's rows)
    assert Rg.shape[0] == lay.rrows and not np.isnan(Qg).any() and not np.isnan(Rg).any()
    errs = (rel(Rg[:N], ref["R"]), np.abs(Qg - ref["Q"]).max(), rel(Qpg, ref["Qpost"]), rel(Bpg, ref["bpost"]))
    print("    R {:.2e}  Q~ (abs) {:.2e}  Qpost {:.2e}  bpost {:.2e}".format(*errs), flush=True)
    assert errs[0] < 1e-11 and errs[1] < 1e-11 and errs[2] < 1e-10 and errs[3] < 1e-10
    res = np.linalg.norm(A - Qg[:M, :N] @ Rg[:N, :N]) / np.linalg.norm(A)
    Qt = Qg[:, :N]
    orth = np.linalg.norm(np.eye(N) - Qt.T @ Qt)
    print(f"    residual {res:.2e}  orth {orth:.2e}", flush=True)
    assert res < 1e-12 and orth < 1e-12
    xo = oc.coded_solve(ref["Qpost"], ref["R"][:N, :N], ref["bpost"])
    print(f"    solve {rel(X, xo):.2e}", flush=True)
    assert rel(X, xo) < 1e-9


def test_tall_backward_matches_oracle(tall):
    cqr, A, v, lay, rhs, sched, ref = tall
    print(f"[case] tall full-size adjoint m={M} n={N}", flush=True)
    Q, R1 = ref["Q"][:, :N], ref["R"][:N, :N]
    gv = oc.q_generator(v)
    rng = np.random.default_rng(5)
    dQ = rng.standard_normal((lay.mp, N))
    dR = np.triu(rng.standard_normal((N, N)))
    q = cqr.CodedQR(gpu_config(cqr, lay, B), v, None)
    dA = host(q.backward(_dev(cqr, Q), _dev(cqr, R1), _dev(cqr, dQ), _dev(cqr, dR)))
    x = oc.coded_solve(ref["Qpost"], R1, ref["bpost"])
    dx = rng.standard_normal(x.shape)
    dQs, dRs, dBs = q.solve_backward(_dev(cqr, ref["Qpost"]), _dev(cqr, R1), _dev(cqr, ref["bpost"]),
                                     _dev(cqr, x), _dev(cqr, dx))
    torch.cuda.synchronize()
    q.close()
    dA_ref = oa.coded_qr_backward(Q, R1, dQ, dR, gv, lay)
    dQs_ref, dRs_ref, dBs_ref = oa.coded_solve_backward(ref["Qpost"], R1, ref["bpost"], x, dx, gv, lay)
    errs = (rel(dA, dA_ref), rel(host(dQs), dQs_ref), rel(host(dRs), dRs_ref), rel(host(dBs), dBs_ref))
    print("    dA {:.2e}  solve: dQ {:.2e} dR {:.2e} dB {:.2e}".format(*errs), flush=True)
    assert max(errs) <= 1e-10
