"""Seeded synthetic inputs shared by the tests, the bench and the oracle's callers.

This module holds no arithmetic of the coded-QR method itself: it only draws
random numbers (matrices, the uniform entries the generator construction asks
for, failure schedules).  Every consumer receives the same arrays, so the HIP
path and the oracle are compared on identical data without sharing code.

Workload shapes follow the paper's experiments (square Gaussian systems on a
p x p grid, failures injected at the start of panel iterations, reverse-diagonal
failure pattern); the paper does not state the input distribution, so i.i.d.
N(0,1) entries are used, plus U diag(s) V^T matrices with log-spaced singular
values for the conditioning study.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian",
    "conditioned",
    "q_generator_draws",
    "r_generator_draws",
    "random_failures",
    "reverse_diagonal",
    "draw_schedule",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def gaussian(m: int, n: int, seed: int) -> np.ndarray:
    """m x n matrix of i.i.d. N(0,1) entries, float64, column-major (Fortran order)."""
    return np.asfortranarray(_rng(seed).standard_normal((m, n)))


def _haar(n: int, rng: np.random.Generator) -> np.ndarray:
    # Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    # signs of R's diagonal folded into Q (Mezzadri 2007).
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))


def conditioned(n: int, cond: float, seed: int) -> np.ndarray:
    """A = U diag(s) V^T with Haar U, V and s_i = cond^(-i/(n-1)) (log-spaced)."""
    rng = _rng(seed)
    u = _haar(n, rng)
    v = _haar(n, rng)
    s = cond ** (-np.arange(n) / max(n - 1, 1))
    return np.asfortranarray((u * s) @ v.T)


def q_generator_draws(kv: int, pr: int, seed: int) -> np.ndarray:
    """The Kv x (pr - Kv) matrix of i.i.d. Unif(0,1) entries that the Q-side
    generator construction draws (its V-tilde block)."""
    if kv == 0:
        return np.zeros((0, pr))
    return _rng(seed + 7919).uniform(0.0, 1.0, size=(kv, pr - kv))


def r_generator_draws(pc: int, kh: int, seed: int) -> np.ndarray:
    """pc x Kh R-side generator entries.  Any MDS code is admissible for R; one
    checksum uses the all-ones column of the paper's worked example, more use
    i.i.d. Unif(0,1) entries (MDS with probability one)."""
    if kh == 0:
        return np.zeros((pc, 0))
    if kh == 1:
        return np.ones((pc, 1))
    return _rng(seed + 104729).uniform(0.0, 1.0, size=(pc, kh))


def reverse_diagonal(p: int, f: int) -> list[tuple[int, int]]:
    """Reverse-diagonal failure pattern on a p x p grid: nodes (i, (p-1-i-k) mod p)
    for k < f, i.e. f failures in every grid row and every grid column."""
    return [(i, (p - 1 - i - k) % p) for i in range(p) for k in range(f)]


def random_failures(pr: int, pc: int, count: int, rng: np.random.Generator,
                    distinct_lines: bool = True) -> list[tuple[int, int]]:
    """`count` distinct systematic nodes; with `distinct_lines` no two share a
    grid row or a grid column (at most one failure per row and column)."""
    out: list[tuple[int, int]] = []
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > 10000:
            raise RuntimeError("cannot draw failure set")
        i = int(rng.integers(pr))
        j = int(rng.integers(pc))
        if (i, j) in out:
            continue
        if distinct_lines and any(i == a or j == b for a, b in out):
            continue
        out.append((i, j))
    return out


def draw_schedule(kind: str, npanels: int, pr: int, pc: int, seed: int,
                  nfail: int = 1, every: int = 16, f: int = 1) -> list[tuple[int, list[tuple[int, int]]]]:
    """Failure schedule as a list of (panel index, [failed nodes]) sorted by panel.

    kind = "random":  `nfail` events, each one random systematic node at an
                      independent random panel in [1, npanels-1]; events that
                      share a panel are merged (their nodes differ in row and col).
    kind = "burst":   `nfail` nodes at one random panel.
    kind = "revdiag": the reverse-diagonal pattern with f per row/column at
                      panels every, 2*every, ... (< npanels).
    """
    rng = _rng(seed + 31337)
    events: dict[int, list[tuple[int, int]]] = {}
    if kind == "none":
        return []
    if kind == "random":
        for _ in range(nfail):
            t = int(rng.integers(1, max(npanels, 2)))
            cur = events.setdefault(t, [])
            nodes = random_failures(pr, pc, 1, rng)
            while any(nodes[0][0] == a or nodes[0][1] == b for a, b in cur):
                nodes = random_failures(pr, pc, 1, rng)
            cur.extend(nodes)
    elif kind == "burst":
        t = int(rng.integers(1, max(npanels, 2)))
        events[t] = random_failures(pr, pc, nfail, rng,
                                    distinct_lines=min(pr, pc) >= nfail)
    elif kind == "revdiag":
        assert pr == pc
        for t in range(every, npanels, every):
            events[t] = reverse_diagonal(pr, f)
    else:
        raise ValueError(kind)
    return sorted(events.items())
