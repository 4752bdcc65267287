"""Plain FP64 CPU oracle for the reverse-mode derivative (adjoint) of the coded
QR and of the coded solve.  The paper does not differentiate its method; this
is a growth direction built on its definitions.

TEST INFRASTRUCTURE ONLY: like the rest of `oracle/`, only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It shares
no code with the HIP library.

The coded QR as a function of A: the n systematic columns of the encoded
matrix are A~ = [A; G_v A] (System Model, encoding equation), and the
factorization gives A~ = Q~ R_1 with Q~^T Q~ = I and R_1 upper triangular with a
positive diagonal (unique for full column rank).

QR adjoint.  This is the standard reverse-mode rule for the thin QR of a
full-column-rank matrix. Given the cotangents dQ (m' x n) and dR (n x n,
upper triangular):
    M = R dR^T - dQ^T Q,
    copyltu(M)_ij = M_{max(i,j), min(i,j)}  (the symmetric matrix holding M's lower triangle),
    dA~ = (dQ + Q copyltu(M)) R^{-T}.
Encoding adjoint:  A~ = [I; G_v] A, so  dA = dA~_top + G_v^T dA~_bottom.

Coded-solve adjoint.  The solve is x = R_1^{-1} (G_0 Q_1)^T (G_0 b) (the
linear-solve equations after the post-orthogonalization theorem). With
Qp = G_0 Q_1, bp = G_0 b, y = Qp^T bp and x = R_1^{-1} y:
    dy = R_1^{-T} dx,   dR_1 = -triu(dy x^T),   dQp = bp dy^T,   dbp = Qp dy,
    dQ_1 = G_0^T dQp,   db = G_0^T dbp,
and dQ~ = [dQ_1; 0], because the checksum rows do not enter the solve.

Pins (tests/test_oracle_pins.py): central finite differences of the oracle's
own forward map along random directions, and the closed-form gradient of the
W-weighted least-squares solution that the coded solve computes.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from oracle import coded_qr as oc


def copyltu(M: np.ndarray) -> np.ndarray:
    """Symmetric matrix with the lower triangle (diagonal included) of M."""
    return np.tril(M) + np.tril(M, -1).T


def qr_adjoint(Q: np.ndarray, R: np.ndarray, dQ: np.ndarray, dR: np.ndarray) -> np.ndarray:
    """dA~ from the cotangents of the thin QR A~ = Q R (only the upper triangle of dR is used)."""
    dR = np.triu(dR)
    M = R @ dR.T - dQ.T @ Q
    B = dQ + Q @ copyltu(M)
    # B R^{-T}: the rows of X solve X R^T = B, i.e. R X^T = B^T
    return solve_triangular(R, B.T, lower=False).T


def encode_adjoint(dAt: np.ndarray, gv: np.ndarray, lay: oc.Layout) -> np.ndarray:
    """dA = dA~_top + G_v^T dA~_bottom for A~ = [A; G_v A]."""
    dA = dAt[:lay.m].copy()
    if lay.kv:
        Gv = oc.kron_generator(gv, lay.bs)
        dA += Gv.T @ dAt[lay.m:]
    return dA


def coded_qr_backward(Q: np.ndarray, R1: np.ndarray, dQ: np.ndarray, dR1: np.ndarray, gv: np.ndarray,
                      lay: oc.Layout) -> np.ndarray:
    """dA from the cotangents of (Q~[:, :n], R_1) of the coded QR of A."""
    return encode_adjoint(qr_adjoint(Q, R1, dQ, dR1), gv, lay)


def coded_solve_backward(Qpost: np.ndarray, R1: np.ndarray, bpost: np.ndarray, x: np.ndarray, dx: np.ndarray,
                         gv: np.ndarray, lay: oc.Layout):
    """Cotangents (dQ~ (m' x n), dR_1 (n x n, upper), db (m x nrhs)) of the
    coded solve x = R_1^{-1} (G_0 Q_1)^T (G_0 b), given dx."""
    dy = solve_triangular(R1, dx, trans="T", lower=False)
    dR = -np.triu(dy @ x.T)
    dQp = bpost @ dy.T
    dbp = Qpost @ dy
    G0 = oc.kron_generator(oc.g0_tilde(gv), lay.bs)
    dQ = np.zeros((lay.mp, lay.n))
    dQ[:lay.m] = G0.T @ dQp
    return dQ, dR, G0.T @ dbp


def coded_qr_forward(A: np.ndarray, v_tilde: np.ndarray, lay: oc.Layout, b: int):
    """(Q~[:, :n], R_1) of the coded QR of A, failure free (the factors do not
    depend on failures, which recovery undoes)."""
    out = oc.run(oc.Problem(A, lay, v_tilde, None if not lay.kh else _ones_gh(lay),
                            oc.FactorOptions(b, "cgs2"), []))
    return out["Q"][:, :lay.n], out["R"][:, :lay.n]


def _ones_gh(lay: oc.Layout) -> np.ndarray:
    # the R-side generator does not affect Q~[:, :n] or R_1
    return np.full((lay.pc, lay.kh), 0.5)
