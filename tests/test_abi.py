"""C-ABI checks that need no GPU: every function that include/cqr.h declares
is exported by libcqr.so and wrapped by the binding, and the host-only entry
points (plan creation and validation, generators, tolerance, workspace size,
status strings) agree with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import coded_qr as oc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cqr.h")

cqr = pytest.importorskip("paper_2311_11943_amd.cqr", reason="libcqr.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return sorted(set(re.findall(r"\b(coded_qr_\w+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("coded_qr_encode", "coded_qr_factor", "coded_qr_recover", "coded_qr_postorth",
                     "coded_qr_erase", "coded_qr_plan_create"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(cqr.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    assert sorted(cqr.EXPORTS) == declared_functions()
    for name in cqr.EXPORTS:
        if name not in ("coded_qr_status_string", "coded_qr_hip_error_name"):
            assert callable(getattr(cqr, name))
    assert cqr.hip_error_name() == "hipSuccess"


def test_status_strings():
    for st in range(7):
        s = cqr.status_string(st)
        assert isinstance(s, str) and s
    assert cqr.status_string(cqr.CQR_OK) != cqr.status_string(cqr.CQR_ENOTRECOVERABLE)


@pytest.mark.parametrize("pr,pc,kv,kh,storage", [
    (4, 4, 1, 1, "out"), (8, 8, 2, 2, "in"), (8, 8, 2, 2, "out"), (4, 6, 2, 2, "in"), (6, 4, 3, 1, "out"), (8, 8, 4, 4, "in"),
])
def test_plan_generators_and_tolerance_match_oracle(pr, pc, kv, kh, storage):
    b = 16
    n = 16 * np.lcm(pr, pc)
    m = max(n, 32 * pr)
    st = cqr.CQR_IN_NODE if storage == "in" else cqr.CQR_OUT_OF_NODE
    cfg = cqr.Config(m=m, n=n, pr=pr, pc=pc, kv=kv, kh=kh, b=b, storage=st)
    vt = synth.q_generator_draws(kv, pr, 11)
    gr = synth.r_generator_draws(pc, kh, 11)
    p = cqr.coded_qr_plan_create(cfg, vt, gr)
    try:
        gv, gh = cqr.coded_qr_plan_generators(p, cfg)
        # -V V^T/2 is summed in a different order on each side
        np.testing.assert_allclose(gv, oc.q_generator(vt), rtol=1e-14, atol=1e-15)
        sname = oc.IN_NODE if storage == "in" else oc.OUT_OF_NODE
        np.testing.assert_array_equal(gh, oc.r_generator(gr, sname))
        # both codes must survive: the smaller of the two per-line tolerances
        f = min(oc.f_tolerated(kv, pr, sname), oc.f_tolerated(kh, pc, sname))
        assert cqr.coded_qr_plan_ftol(p) == f
        ws = cqr.coded_qr_workspace_bytes(p)
        assert ws > 0 and ws % 8 == 0
        # placement: the storers the oracle's node map gives (whose load balance
        # and exclusion are pinned to their definitions in the oracle tests),
        # and the R code excludes the storer's own block column
        qrow, rcol = cqr.coded_qr_plan_placement(p, cfg)
        lay = oc.Layout(m, n, pr, pc, kv, kh, sname)
        if storage == "in":
            for k in range(kv):
                holders = {i for i in range(pr) if (pr + k, 0) in lay.node_blocks((i, 0))[0]}
                assert holders == {int(qrow[k])}
            for k in range(kh):
                holders = {j for j in range(pc) if (0, pc + k) in lay.node_blocks((0, j))[1]}
                assert holders == {int(rcol[k])}
                assert gh[rcol[k], k] == 0.0
        else:
            assert list(qrow) == [pr + k for k in range(kv)] and list(rcol) == [pc + k for k in range(kh)]
    finally:
        cqr.coded_qr_plan_destroy(p)


@pytest.mark.parametrize("bad", [
    dict(m=100),                    # m not a multiple of pr
    dict(n=100),                    # n not a multiple of pc
    dict(b=24),                     # panel width does not divide the block width
    dict(pr=33, m=33 * 8),          # grid too large
    dict(kv=9),                     # too many checksums
    dict(kv=3),                     # post-orthogonalization needs K_v <= p_r / 2
    dict(precision=7),              # unknown precision
    dict(storage=5),                # unknown storage
    dict(panel=4),                  # unknown panel mode
    dict(icgs_eta=1.5),             # ICGS threshold above 1
    dict(icgs_eta=-0.1),            # negative ICGS threshold
    dict(icgs_eta=float("nan")),
])
def test_plan_create_rejects_invalid_configs(bad):
    base = dict(m=256, n=256, pr=4, pc=4, kv=1, kh=1, b=16)
    base.update(bad)
    cfg = cqr.Config(**base)
    with pytest.raises(cqr.CqrError) as e:
        cqr.coded_qr_plan_create(cfg, synth.q_generator_draws(cfg.kv, cfg.pr, 1)
                                 if cfg.kv <= 8 and cfg.pr > cfg.kv else None,
                                 synth.r_generator_draws(cfg.pc, cfg.kh, 1))
    assert e.value.status == cqr.CQR_EINVAL


@pytest.mark.parametrize("precision", ["CQR_TRAIL_FP32", "CQR_TRAIL_BF16X3"])
def test_plan_accepts_reduced_precision_products(precision):
    cfg = cqr.Config(m=256, n=256, pr=4, pc=4, kv=1, kh=1, b=16, precision=getattr(cqr, precision))
    p = cqr.coded_qr_plan_create(cfg, synth.q_generator_draws(1, 4, 1), synth.r_generator_draws(4, 1, 1))
    cqr.coded_qr_plan_destroy(p)


def test_r_rows_with_and_without_horizontal_code():
    cfg = cqr.Config(m=1024, n=128, pr=8, pc=1, kv=2, kh=0, b=32)
    p = cqr.coded_qr_plan_create(cfg, synth.q_generator_draws(2, 8, 1), None)
    try:
        assert cqr.coded_qr_plan_r_rows(p) == 128 + 2 * 128 // 8
    finally:
        cqr.coded_qr_plan_destroy(p)
    cfg = cqr.Config(m=256, n=256, pr=4, pc=4, kv=1, kh=1, b=16)
    p = cqr.coded_qr_plan_create(cfg, synth.q_generator_draws(1, 4, 1), synth.r_generator_draws(4, 1, 1))
    try:
        assert cqr.coded_qr_plan_r_rows(p) == 256
    finally:
        cqr.coded_qr_plan_destroy(p)


def test_solve_workspace_size():
    cfg = cqr.Config(m=240, n=240, pr=4, pc=4, kv=1, kh=1, b=16)
    p = cqr.coded_qr_plan_create(cfg, synth.q_generator_draws(1, 4, 1), synth.r_generator_draws(4, 1, 1))
    try:
        # four inverted 64 x 64 diagonal blocks, then Y (240 x nrhs), each 256-byte aligned
        assert cqr.coded_qr_solve_workspace_bytes(p, 3) == 4 * 64 * 64 * 8 + 5888
        assert cqr.coded_qr_solve_workspace_bytes(p, 0) == 0
    finally:
        cqr.coded_qr_plan_destroy(p)


def test_new_entry_points_reject_null_arguments_before_any_launch():
    """The solve and adjoint entry points validate their arguments on the host
    and return CQR_EINVAL without touching the device."""
    import ctypes as C
    cfg = cqr.Config(m=256, n=256, pr=4, pc=4, kv=1, kh=1, b=16)
    p = cqr.coded_qr_plan_create(cfg, synth.q_generator_draws(1, 4, 1), synth.r_generator_draws(4, 1, 1))
    P = C.c_void_p(p)
    try:
        assert cqr.LIB.coded_qr_solve(P, None, 256, None, 256, None, 256, 1, None, 256, None, 0, None) == cqr.CQR_EINVAL
        assert cqr.LIB.coded_qr_backward(P, None, 320, None, 256, None, 320, None, 256, None, 256, None, 0,
                                         None) == cqr.CQR_EINVAL
        assert cqr.LIB.coded_qr_solve_backward(P, None, 256, None, 256, None, 256, None, 256, None, 256, 1, None, 320,
                                               None, 256, None, 256, None, 0, None) == cqr.CQR_EINVAL
        assert cqr.coded_qr_backward_workspace_bytes(p) > cqr.coded_qr_workspace_bytes(p)
        assert cqr.coded_qr_solve_backward_workspace_bytes(p, 0) == 0
    finally:
        cqr.coded_qr_plan_destroy(p)


def test_oracle_not_imported_by_product_package():
    pkg = os.path.join(ROOT, "paper_2311_11943_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", text, re.M), f
                assert "oracle/" not in text, f


def test_binding_shares_torchs_hip_runtime():
    """Importing the binding first must not load a second HIP runtime next to
    torch's (two HSA runtimes in one process leave the library without a
    device)."""
    import subprocess
    import sys
    code = ("from paper_2311_11943_amd import cqr\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
            "print(len(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
