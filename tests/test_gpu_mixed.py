"""Mixed precision (the coefficient product R_bar = Qbar^T Q_t on FP32 MFMA,
or as split-BF16 products on BF16 MFMA, every column operation in FP64)
against the FP64 oracle.

What the arithmetic fixes, and so what is asserted:
  * The rank-b update, the re-projection and the panel transforms are FP64
    column operations with the coefficients that R records, so A~ = Q~ R and
    the carried row checksums Q_2 = G_v Q_1 hold to FP64 rounding, and the
    FP64 re-projection of later panels removes what the FP32 coefficients
    leave behind: residual at the FP64 bound (1e-12), ||I - Q~^T Q~|| at the
    FP64 bound or within 4x the FP64 oracle's where that exceeds it, plus
    n u64 u32 kappa(A) for the re-projection's cancellation on ill-conditioned
    inputs,
    Q~ and R_1 equal to the FP64 oracle's to its elementwise bound (1e-11 on
    Gaussian inputs), decoded Q blocks exact to 1e-10, and the row-checksum
    drift (u kappa(A) in the FP64 method itself) within 4x the FP64 oracle's.
  * The carried R-checksum columns take their coefficients from the FP32
    product and are never re-projected.  One coefficient's error is at most
    (s + 2) u32 ||q|| ||x|| (operands rounded, relative 2 u32 per product; FP32
    sums over s = 16 terms, FP64 across), and a checksum column collects one
    per row of R, so ||R_2 - R_1 G_h||_F <= (s + 2) u32 sqrt(n) ||R_2||_F.  The
    same bound holds for the carried residual Q~ (R_1 G_h - R_2).
  * The split-BF16 form: each FP64 operand is hi + mid + lo to 2^-26 of
    itself, and the three part products it drops are below 2^-25 of the
    whole, so the parts represent each product to about u32; the five small
    part products are summed first, so the FP32 rounding is that of the
    hi hi sum over s = 32 k-values: (s + 3) u32 per coefficient.
  * An R block decoded mid-factorization inherits that relation's error
    through the decode solve: its error is G_hat^{-1} applied to the relation
    error of the surviving checksums, checked against the snapshot taken
    before the erasure.
"""
import numpy as np
import pytest

import synth
from oracle import coded_qr as oc
from tests.gpu_helpers import gpu_config, host, make_inputs, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24          # unit roundoff of FP32
# k-values summed in FP32 before the FP64 sum, and the u32 terms per
# coefficient beyond them (operand rounding; for the split form the split)
TERMS = {"fp32": (16, 2), "bf16x3": (32, 3)}


def r_relation_bound(n: int, precision: str = "fp32") -> float:
    s, extra = TERMS[precision]
    return (s + extra) * U32 * np.sqrt(n)


def _code(cqr, precision):
    return cqr.CQR_TRAIL_FP32 if precision == "fp32" else cqr.CQR_TRAIL_BF16X3


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
    # three tile rows (odd): the pair kernel's second half of the last pair is empty
    ("odd_tile_rows", 768, 4, 1, 192, "out", "gauss", 1.0),
    ("ragged", 240, 4, 1, 16, "out", "gauss", 1.0),
    # depth 320 < 512: one split, so the 128 x 128 products store C directly
    ("one_split", 256, 4, 1, 128, "out", "gauss", 1.0),
]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("sid,n,pr,K,b,storage,kind,cond", CASES, ids=[c[0] for c in CASES])
def test_reduced_precision_coefficients_match_fp64_oracle(cqr, sid, n, pr, K, b, storage, kind, cond, precision):
    # the split-BF16 product needs two tile rows and a depth that is a multiple
    # of 32; the other cases run its FP32 fallback, checked here all the same
    print(f"[case] mixed {precision} {sid}", flush=True)
    A, v, gh, lay = make_inputs(n, pr, K, b, storage, seed=8, kind=kind, cond=cond)
    cfg = gpu_config(cqr, lay, b, precision=_code(cqr, precision))
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
    print(f"    orth {orth:.2e} res {res:.2e} R1 {rel(Rg[:, :n], ref['R'][:, :n]):.2e} "
          f"Q {rel(Qt, ref['Q'][:, :n]):.2e} R2 {rel(Rg[:, n:], ref['R'][:, n:]) if lay.kh else 0:.2e}", flush=True)
    # FP64 orthogonality up to what the FP32 first projection costs an
    # ill-conditioned input: it leaves components of size ~u32 ||x|| along the
    # finished basis, which the FP64 re-projection removes with relative
    # rounding u64 (u32 kappa(A)), i.e. about n u64 u32 kappa(A) in the
    # Frobenius norm; the FP64 oracle itself passes 1e-12 near kappa 1e10
    orth_or = oc.metrics(A, ref, lay)["orth_coded"]
    kappa = np.linalg.cond(A)
    bound = max(1e-12, 4 * orth_or) + n * 2.0 ** -53 * U32 * kappa
    print(f"    orthogonality bound {bound:.2e} (oracle {orth_or:.2e}, kappa {kappa:.1e})", flush=True)
    assert orth <= bound and res <= 1e-12
    gv = oc.q_generator(v)
    Gv = oc.kron_generator(gv, lay.bs)
    # the carried row checksums drift by the FP64 rounding of the updates,
    # which grows like u kappa(A) in the FP64 method itself: bounded by the
    # FP64 oracle's own drift on the same input
    drift_q = np.abs(Qg[lay.m:, :n] - Gv @ Qg[:lay.m, :n]).max() / np.abs(Qg[:, :n]).max()
    Qo = ref["Q"]
    drift_o = np.abs(Qo[lay.m:, :n] - Gv @ Qo[:lay.m, :n]).max() / np.abs(Qo[:, :n]).max()
    print(f"    row-checksum drift {drift_q:.2e} (FP64 oracle {drift_o:.2e})", flush=True)
    assert drift_q <= max(1e-12, 4 * drift_o)
    if lay.kh:
        Gh = oc.kron_generator(oc.r_generator(gh, lay.storage), lay.bw)
        d_r = np.linalg.norm(Rg[:, n:] - Rg[:, :n] @ Gh) / np.linalg.norm(Rg[:, n:])
        carried = np.linalg.norm(Qg[:, n:]) / np.linalg.norm(Rg[:, n:])
        bound = r_relation_bound(n, precision)
        print(f"    R-checksum relation {d_r:.2e}, carried residual {carried:.2e}, bound {bound:.2e}", flush=True)
        assert d_r <= bound and carried <= bound
    if kind == "gauss":
        assert rel(Rg[:, :n], ref["R"][:, :n]) <= 1e-11
        assert rel(Qt, ref["Q"][:, :n]) <= 1e-11


def _decode_gain(gen: np.ndarray, lost: list[int], chk_lost: list[int]) -> float:
    """Factor by which an error in the checksum relation of one code line
    reaches its blocks after a decode (lowest-index surviving checksums): the
    decoded data blocks get G_hat^{-1} of the used checksums' relation error
    (||G_hat^{-1}||_inf), a re-encoded lost checksum its own relation error
    plus its generator row applied to the decoded blocks' errors."""
    surv = [k for k in range(gen.shape[0]) if k not in chk_lost][:len(lost)]
    ginv = np.abs(np.linalg.inv(gen[np.ix_(surv, lost)])).sum(axis=1).max()
    reenc = max((1.0 + np.abs(gen[k, lost]).sum() * ginv for k in chk_lost), default=0.0)
    return float(max(ginv, reenc))


@pytest.mark.parametrize("precision,n,pr,K,b", [("fp32", 512, 8, 2, 64), ("bf16x3", 512, 4, 2, 128)])
def test_reduced_precision_coefficients_recover_failures(cqr, precision, n, pr, K, b):
    print(f"[case] mixed {precision} recovery n={n} pr={pr} K={K} b={b}", flush=True)
    A, v, gh, lay = make_inputs(n, pr, K, b, "in", seed=9)
    q = cqr.CodedQR(gpu_config(cqr, lay, b, precision=_code(cqr, precision)), v, gh)
    sched = synth.draw_schedule("random", n // b, pr, pr, 9, nfail=2)
    ghm = oc.r_generator(gh, lay.storage)
    Gh = oc.kron_generator(ghm, lay.bw)
    # the encoded checksum columns: their norms bound the trailing columns' at every step
    enc = oc.encode(A, oc.q_generator(v), ghm, lay)
    chk_norm = np.linalg.norm(enc[:, n:])
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
        # the snapshot's R-checksum relation error, and what the decode makes of it
        # (in-node: R-checksum column k is stored on grid column k mod p_c)
        d_rel = np.abs(before_R[:, n:] - before_R[:, :n] @ Gh).max()
        gain = max(_decode_gain(ghm.T, [j], [kk for kk in range(lay.kh) if kk % lay.pc == j]) for (_, j) in nodes)
        err_r = np.abs(Rg - before_R).max()
        print(f"    failure at panel {t}: Q {rel(Qg, before_Q):.2e}, R abs {err_r:.2e} "
              f"(relation error {d_rel:.2e} x decode gain {gain:.2f})", flush=True)
        assert rel(Qg, before_Q) <= 1e-10
        assert err_r <= 1.01 * gain * d_rel + 1e-12 * np.abs(before_R).max()
        assert d_rel <= r_relation_bound(n, precision) * chk_norm
    q.factor(At, R, k, n // b)
    torch.cuda.synchronize()
    Qg, Rg = host(At), host(R)
    q.close()
    ref = oc.run(oc.Problem(A, lay, v, gh, oc.FactorOptions(b, "icgs"), sched))
    Qt = Qg[:, :n]
    orth = np.linalg.norm(np.eye(n) - Qt.T @ Qt)
    res = np.linalg.norm(A - Qg[:lay.m, :n] @ Rg[:, :n]) / np.linalg.norm(A)
    print(f"    after failures: orth {orth:.2e} res {res:.2e} R vs oracle {rel(Rg, ref['R']):.2e}", flush=True)
    assert orth <= 1e-12 and res <= 1e-6
