"""Pins of the adjoint oracle (oracle/adjoint.py) against quantities it does
not compute itself:
- central finite differences (h = 1e-6) of the oracle's forward coded QR,
  along 8 random directions, for a loss that weights every entry of Q~ and R_1;
- the closed-form gradient of the W-weighted least-squares solution that the
  coded solve computes (W = I + G_v^T G_v):
      x = (A^T W A)^{-1} A^T W b,  L = ||x - x_t||^2,  z = (A^T W A)^{-1} 2 (x - x_t),
      dL/dA = W r z^T - W A z x^T  (r = b - A x),   dL/db = W A z;
- planted mistakes (copyltu replaced by M itself, a dropped G_v^T term) fail them.
"""
import numpy as np
import pytest

import synth
from oracle import adjoint as oa
from oracle import coded_qr as oc


def _geometry(kind):
    # (m, n, pr, pc, kv, kh, b)
    return {"square": (32, 32, 4, 4, 1, 1, 8), "tall": (128, 32, 8, 1, 2, 0, 8)}[kind]


def _loss_and_grad(A, v, lay, b, WQ, WR):
    Q, R = oa.coded_qr_forward(A, v, lay, b)
    L = float(np.sum(WQ * Q) + np.sum(WR * np.triu(R)))
    gv = oc.q_generator(v)
    return L, oa.coded_qr_backward(Q, R, WQ, np.triu(WR), gv, lay)


@pytest.mark.parametrize("kind", ["square", "tall"])
def test_qr_adjoint_matches_central_differences(kind):
    m, n, pr, pc, kv, kh, b = _geometry(kind)
    lay = oc.Layout(m, n, pr, pc, kv, kh, oc.OUT_OF_NODE)
    A = synth.gaussian(m, n, 41)
    v = synth.q_generator_draws(kv, pr, 41)
    rng = np.random.default_rng(42)
    WQ = rng.standard_normal((lay.mp, n))
    WR = rng.standard_normal((n, n))
    _, dA = _loss_and_grad(A, v, lay, b, WQ, WR)
    h = 1e-6
    for _ in range(8):
        E = rng.standard_normal((m, n))
        Lp, _ = _loss_and_grad(A + h * E, v, lay, b, WQ, WR)
        Lm, _ = _loss_and_grad(A - h * E, v, lay, b, WQ, WR)
        fd = (Lp - Lm) / (2 * h)
        an = float(np.sum(dA * E))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)


def _solve_chain(A, B, v, lay, b, xt):
    """x from the coded QR and coded solve, and (dL/dA, dL/db) by the adjoint chain."""
    Q, R = oa.coded_qr_forward(A, v, lay, b)
    gv = oc.q_generator(v)
    Qp, Bp = oc.postorth(Q[:lay.m], B, gv, lay.pr)
    x = oc.coded_solve(Qp, R, Bp)
    dx = 2 * (x - xt)
    dQ, dR, dB = oa.coded_solve_backward(Qp, R, Bp, x, dx, gv, lay)
    dA = oa.coded_qr_backward(Q, R, dQ, dR, gv, lay)
    return x, dA, dB


@pytest.mark.parametrize("kind", ["square", "tall"])
def test_solve_chain_gradient_matches_weighted_least_squares(kind):
    m, n, pr, pc, kv, kh, b = _geometry(kind)
    lay = oc.Layout(m, n, pr, pc, kv, kh, oc.OUT_OF_NODE)
    A = synth.gaussian(m, n, 43)
    B = synth.gaussian(m, 1, 44)
    xt = synth.gaussian(n, 1, 45)
    v = synth.q_generator_draws(kv, pr, 43)
    x, dA, dB = _solve_chain(A, B, v, lay, b, xt)
    Gv = np.kron(oc.q_generator(v), np.eye(lay.bs))
    W = np.eye(m) + Gv.T @ Gv
    H = A.T @ W @ A
    xw = np.linalg.solve(H, A.T @ W @ B)
    np.testing.assert_allclose(x, xw, rtol=1e-11, atol=1e-12)
    z = np.linalg.solve(H, 2 * (xw - xt))
    r = B - A @ xw
    gA = W @ r @ z.T - W @ A @ z @ xw.T
    gB = W @ A @ z
    assert np.abs(dA - gA).max() <= 1e-10 * np.abs(gA).max()
    assert np.abs(dB - gB).max() <= 1e-10 * np.abs(gB).max()


def test_pins_catch_planted_adjoint_mistakes(monkeypatch):
    m, n, pr, pc, kv, kh, b = _geometry("tall")
    lay = oc.Layout(m, n, pr, pc, kv, kh, oc.OUT_OF_NODE)
    A = synth.gaussian(m, n, 43)
    B = synth.gaussian(m, 1, 44)
    xt = synth.gaussian(n, 1, 45)
    v = synth.q_generator_draws(kv, pr, 43)
    Gv = np.kron(oc.q_generator(v), np.eye(lay.bs))
    W = np.eye(m) + Gv.T @ Gv
    H = A.T @ W @ A
    xw = np.linalg.solve(H, A.T @ W @ B)
    z = np.linalg.solve(H, 2 * (xw - xt))
    gA = W @ (B - A @ xw) @ z.T - W @ A @ z @ xw.T

    def off(dA):
        return np.abs(dA - gA).max() / np.abs(gA).max()

    with monkeypatch.context() as mp:
        mp.setattr(oa, "copyltu", lambda M: M)
        assert off(_solve_chain(A, B, v, lay, b, xt)[1]) > 1e-3
    with monkeypatch.context() as mp:
        mp.setattr(oa, "encode_adjoint", lambda dAt, gv, lay: dAt[:lay.m].copy())
        assert off(_solve_chain(A, B, v, lay, b, xt)[1]) > 1e-3
