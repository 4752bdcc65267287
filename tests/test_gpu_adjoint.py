"""Adjoint of the coded QR and of the coded solve on the GPU.

- coded_qr_backward and coded_qr_solve_backward against the adjoint oracle on
  the same factors and cotangents (1e-10 relative to the largest entry);
- the torch.autograd functions end to end (forward with a failure schedule,
  backward through the solve and the QR) against the closed-form gradient of
  the W-weighted least-squares solution (1e-8 relative);
- torch.autograd.gradcheck (central differences through the GPU forward) on a
  small problem.
"""
import numpy as np
import pytest

import synth
from oracle import adjoint as oa
from oracle import coded_qr as oc
from tests.gpu_helpers import gpu_config, host, make_inputs, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    from paper_2311_11943_amd import autograd, cqr
    return cqr, autograd


CASES = [
    # id, n, pr, K, b, storage, layout extras
    ("square_innode", 256, 8, 2, 64, "in", {}),
    ("tall", 128, 8, 2, 64, "out", {"m": 1024, "pc": 1, "kh": 0}),
    ("ragged", 240, 4, 1, 16, "out", {}),
    ("wide_n", 512, 4, 2, 128, "out", {}),
    # R_1^{-1} by recursive doubling over 64-wide diagonal blocks: five levels,
    # the last off-diagonal block of each level ragged (1152 = 1024 + 128)
    ("five_levels_ragged", 1152, 4, 1, 96, "out", {}),
]


def _dev(cqr, x):
    return cqr.to_device_colmajor(np.ascontiguousarray(x), "cuda:0")


@pytest.mark.parametrize("sid,n,pr,K,b,storage,extra", CASES, ids=[c[0] for c in CASES])
def test_backward_kernels_match_oracle(mods, sid, n, pr, K, b, storage, extra):
    cqr, _ = mods
    print(f"[case] adjoint {sid}", flush=True)
    A, v, gh, lay = make_inputs(n, pr, K, b, storage, seed=31, **extra)
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "cgs2"), [], synth.gaussian(lay.m, 2, 32)))
    Q, R1 = ref["Q"][:, :n], ref["R"][:, :n]
    gv = oc.q_generator(v)
    rng = np.random.default_rng(33)
    dQ = rng.standard_normal((lay.mp, n))
    dR = np.triu(rng.standard_normal((n, n)))
    q = cqr.CodedQR(gpu_config(cqr, lay, b), v, gh)
    dA = host(q.backward(_dev(cqr, Q), _dev(cqr, R1), _dev(cqr, dQ), _dev(cqr, dR)))
    dA_ref = oa.coded_qr_backward(Q, R1, dQ, dR, gv, lay)
    # the solve's adjoint on the oracle's post-orthogonalized factors
    x = oc.coded_solve(ref["Qpost"], R1, ref["bpost"])
    dx = rng.standard_normal(x.shape)
    dQs, dRs, dBs = q.solve_backward(_dev(cqr, ref["Qpost"]), _dev(cqr, R1), _dev(cqr, ref["bpost"]),
                                     _dev(cqr, x), _dev(cqr, dx))
    torch.cuda.synchronize()
    q.close()
    dQs_ref, dRs_ref, dBs_ref = oa.coded_solve_backward(ref["Qpost"], R1, ref["bpost"], x, dx, gv, lay)
    errs = (rel(dA, dA_ref), rel(host(dQs), dQs_ref), rel(host(dRs), dRs_ref), rel(host(dBs), dBs_ref))
    print("    dA {:.2e}  solve: dQ {:.2e} dR {:.2e} dB {:.2e}".format(*errs), flush=True)
    assert max(errs) <= 1e-10


@pytest.mark.parametrize("kind", ["square", "tall"])
def test_autograd_matches_weighted_least_squares_gradient(mods, kind):
    cqr, ag = mods
    if kind == "square":
        A, v, gh, lay = make_inputs(256, 8, 2, 32, "in", seed=34)
        b = 32
        sched = synth.draw_schedule("random", lay.n // b, lay.pr, lay.pc, 34, nfail=2)
    else:
        # p_c = 1: no horizontal code, R's checksum rows protect it; two nodes at once
        A, v, gh, lay = make_inputs(128, 8, 2, 32, "out", seed=34, m=1024, pc=1, kh=0)
        b = 32
        sched = [(2, [(1, 0), (6, 0)])]
    print(f"[case] autograd {kind}, schedule {sched}", flush=True)
    Bh = synth.gaussian(lay.m, 1, 35)
    xt = synth.gaussian(lay.n, 1, 36)
    engine = cqr.CodedQR(gpu_config(cqr, lay, b), v, gh)
    At = torch.tensor(A, device="cuda:0", requires_grad=True)
    Bt = torch.tensor(Bh, device="cuda:0", requires_grad=True)
    Q, R1 = ag.coded_qr(At, engine, sched)
    x = ag.coded_solve(Q, R1, Bt, engine)
    loss = ((x - torch.tensor(xt, device="cuda:0")) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    gA, gB, xg = host(At.grad), host(Bt.grad), host(x)
    engine.close()
    Gv = np.kron(oc.q_generator(v), np.eye(lay.bs))
    W = np.eye(lay.m) + Gv.T @ Gv
    H = A.T @ W @ A
    xw = np.linalg.solve(H, A.T @ W @ Bh)
    z = np.linalg.solve(H, 2 * (xw - xt))
    cA = W @ (Bh - A @ xw) @ z.T - W @ A @ z @ xw.T
    cB = W @ A @ z
    print(f"    x {rel(xg, xw):.2e}  dA {rel(gA, cA):.2e}  db {rel(gB, cB):.2e}", flush=True)
    assert rel(xg, xw) <= 1e-9
    assert rel(gA, cA) <= 1e-8 and rel(gB, cB) <= 1e-8


def test_gradcheck_small(mods):
    cqr, ag = mods
    A, v, gh, lay = make_inputs(32, 4, 1, 8, "out", seed=37, m=64, pc=4)
    engine = cqr.CodedQR(gpu_config(cqr, lay, 8), v, gh)
    Bt = torch.tensor(synth.gaussian(lay.m, 1, 38), device="cuda:0", requires_grad=True)
    At = torch.tensor(A, device="cuda:0", requires_grad=True)

    def f(Ain, Bin):
        Q, R1 = ag.coded_qr(Ain, engine)
        return ag.coded_solve(Q, R1, Bin, engine)

    assert torch.autograd.gradcheck(f, (At, Bt), eps=1e-6, atol=1e-6, rtol=1e-4)
    engine.close()


def test_recomputed_factorization_gives_the_same_gradient(mods):
    """coded_qr(..., recompute=True) keeps only A and factors again in the
    backward; the factorization is deterministic, so the gradients are
    bitwise those of the stored-factor path."""
    cqr, ag = mods
    A, v, gh, lay = make_inputs(256, 8, 2, 32, "in", seed=37)
    b = 32
    sched = synth.draw_schedule("random", lay.n // b, lay.pr, lay.pc, 37, nfail=2)
    print(f"[case] recompute, schedule {sched}", flush=True)
    Bh = synth.gaussian(lay.m, 1, 38)
    xt = torch.tensor(synth.gaussian(lay.n, 1, 39), device="cuda:0")
    engine = cqr.CodedQR(gpu_config(cqr, lay, b), v, gh)
    grads = []
    for recompute in (False, True):
        At = torch.tensor(A, device="cuda:0", requires_grad=True)
        Bt = torch.tensor(Bh, device="cuda:0", requires_grad=True)
        Q, R1 = ag.coded_qr(At, engine, sched, recompute=recompute)
        x = ag.coded_solve(Q, R1, Bt, engine)
        del Q
        ((x - xt) ** 2).sum().backward()
        torch.cuda.synchronize()
        grads.append((host(At.grad), host(Bt.grad)))
    engine.close()
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
