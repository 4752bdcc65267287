"""Full-size parity: the benchmark's workload (n = 4096 Gaussian, 8 x 8 grid,
b = 64, K = 2 in-node checksums, two random single-node failures at random
panels) run through the C ABI exactly as bench.py times it (lookahead on,
same seeds, same schedule), then the coded solve, against the FP64 oracle
element by element.
The oracle takes ~10 s on the host cores at this size."""
import numpy as np
import pytest

from oracle import coded_qr as oc
from tests.gpu_helpers import host, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_bench_workload_matches_oracle():
    import bench
    from paper_2311_11943_amd import cqr

    w = bench.WORKLOADS["c2"]
    n, pr, K, b = w["n"], w["pr"], w["K"], w["b"]
    lay = oc.Layout(n, n, pr, pr, K, K, oc.IN_NODE)
    ftol = oc.f_tolerated(K, pr, oc.IN_NODE)
    inp = bench.workload_inputs("c2", ftol, 0)
    sched = inp["schedule"]
    print(f"[case] c2 full size, schedule {sched}", flush=True)
    assert len(sched) == 2

    cfg = cqr.Config(n, n, pr, pr, K, K, b, cqr.CQR_IN_NODE, lookahead=1)
    q = cqr.CodedQR(cfg, inp["v"], inp["gh"])
    assert q.ftol == ftol
    At, R, Qp, Bp = q.run(cqr.to_device_colmajor(inp["A"], "cuda:0"), sched,
                          cqr.to_device_colmajor(inp["rhs"], "cuda:0"))
    torch.cuda.synchronize()
    assert q.info() == 0
    Xg = host(q.solve(Qp, R, Bp))
    Qg, Rg, Qpg, Bpg = host(At), host(R), host(Qp), host(Bp)
    q.close()

    ref = oc.run(oc.Problem(inp["A"], lay, inp["v"], inp["gh"], oc.FactorOptions(b, "icgs"), sched, inp["rhs"]))
    assert not np.isnan(Qg).any() and not np.isnan(Rg).any()
    assert rel(Rg, ref["R"]) < 1e-11
    assert np.abs(Qg - ref["Q"]).max() < 1e-11
    assert rel(Qpg, ref["Qpost"]) < 1e-10
    assert rel(Bpg, ref["bpost"]) < 1e-10
    A = inp["A"]
    res = np.linalg.norm(A - Qg[:n, :n] @ Rg[:, :n]) / np.linalg.norm(A)
    Qt = Qg[:, :n]
    orth = np.linalg.norm(np.eye(n) - Qt.T @ Qt)
    assert res < 1e-12 and orth < 1e-12, (res, orth)
    # coded solve on the GPU against the oracle's and the direct solution
    xo = oc.coded_solve(ref["Qpost"], ref["R"][:, :n], ref["bpost"])
    assert rel(Xg, xo) < 1e-9
    np.testing.assert_allclose(Xg, np.linalg.solve(A, inp["rhs"]), rtol=1e-8, atol=1e-9)
