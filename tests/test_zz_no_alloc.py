"""The allocation-free coded solve (coded_qr_solve_noalloc, for callers that
cannot allocate device memory) against the coded solve with a caller-owned
workspace (coded_qr_solve), through the C ABI: two calls in a row on one
device, the second with a smaller problem, each bit-identical to the
workspace form (the same kernels on the same inputs, whatever the shared
scratch held before); a request beyond the scratch maximum is refused with
CQR_ENOMEM before anything is enqueued."""
import numpy as np
import pytest

import synth
from tests.gpu_helpers import host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_solve_matches_workspace_solve():
    from paper_2311_11943_amd import cqr
    for n, pr, nrhs in ((512, 8, 3), (256, 4, 1)):
        print(f"[case] noalloc solve n={n} pr={pr} nrhs={nrhs}", flush=True)
        K, b = 1, 16
        A = synth.gaussian(n, n, 21)
        Bh = synth.gaussian(n, nrhs, 22)
        q = cqr.CodedQR(cqr.Config(n, n, pr, pr, K, K, b), synth.q_generator_draws(K, pr, 21),
                        synth.r_generator_draws(pr, K, 21))
        At, R, Qp, Bp = q.run(cqr.to_device_colmajor(A, "cuda:0"), (), cqr.to_device_colmajor(Bh, "cuda:0"))
        X_ws = cqr.col_major(n, nrhs, "cuda:0")
        q.solve(Qp, R, Bp, X_ws, q.solve_workspace(nrhs))
        X_na = cqr.col_major(n, nrhs, "cuda:0")
        X_na.fill_(np.nan)
        st = cqr.coded_qr_solve_noalloc(q.plan, Qp, R, Bp, X_na)
        torch.cuda.synchronize()
        assert st == cqr.CQR_OK, cqr.status_string(st)
        a, w = host(X_na), host(X_ws)
        assert not np.isnan(a).any()
        assert np.array_equal(a, w), np.abs(a - w).max()
        np.testing.assert_allclose(a, np.linalg.solve(A, Bh), rtol=1e-8, atol=1e-9)
        q.close()


def test_noalloc_solve_refuses_beyond_its_scratch():
    from paper_2311_11943_amd import cqr
    n, pr = 4096, 8
    q = cqr.CodedQR(cqr.Config(n, n, pr, pr, 1, 1, 64), synth.q_generator_draws(1, pr, 0),
                    synth.r_generator_draws(pr, 1, 0))
    nrhs = 2048          # 8 n nrhs = 64 MiB of Y alone, beyond the 32 MiB scratch
    assert cqr.coded_qr_solve_workspace_bytes(q.plan, nrhs) > cqr.CQR_SOLVE_NOALLOC_MAX_BYTES
    Qp = cqr.col_major(n, n, "cuda:0")
    R = cqr.col_major(n, n, "cuda:0")
    Bp = cqr.col_major(n, nrhs, "cuda:0")
    X = cqr.col_major(n, nrhs, "cuda:0")
    X.fill_(7.0)
    assert cqr.coded_qr_solve_noalloc(q.plan, Qp, R, Bp, X) == cqr.CQR_ENOMEM
    torch.cuda.synchronize()
    assert bool((X == 7.0).all())
    q.close()
