"""Shared set-up for the GPU parity tests: seeded inputs for both sides, the
oracle run, and conversions.  The oracle and the HIP library only meet here,
through arrays."""
from __future__ import annotations

import numpy as np

import synth
from oracle import coded_qr as oc


def make_inputs(n, pr, K, b, storage="out", seed=0, m=None, pc=None, kh=None, kind="gauss", cond=1.0):
    m = n if m is None else m
    pc = pr if pc is None else pc
    kh = K if kh is None else kh
    if kind == "gauss":
        A = synth.gaussian(m, n, seed)
    else:
        A = synth.conditioned(n, cond, seed)
    v = synth.q_generator_draws(K, pr, seed)
    gh = synth.r_generator_draws(pc, kh, seed)
    lay = oc.Layout(m, n, pr, pc, K, kh, oc.IN_NODE if storage == "in" else oc.OUT_OF_NODE)
    return A, v, gh, lay


def gpu_config(cqr, lay, b, reproject=1, precision=0, lookahead=1, panel=0, icgs_eta=0.0):
    return cqr.Config(lay.m, lay.n, lay.pr, lay.pc, lay.kv, lay.kh, b,
                      cqr.CQR_IN_NODE if lay.storage == "in" else cqr.CQR_OUT_OF_NODE, reproject, precision,
                      lookahead, panel, icgs_eta)


def oracle_state(A, v, gh, lay, b, k, panel="cgs2", reproject=True):
    gv = oc.q_generator(v) if lay.kv else np.zeros((0, lay.pr))
    ghm = oc.r_generator(gh, lay.storage) if lay.kh else np.zeros((lay.pc, 0))
    At = oc.encode(A, gv, ghm, lay)
    Q = At.copy()
    R = np.zeros((lay.n, lay.N))
    oc.factor_panels(Q, R, lay.n, 0, k, oc.FactorOptions(b, panel, reproject))
    return At, Q, R, gv, ghm


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy().copy()


def rel(a, b) -> float:
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
