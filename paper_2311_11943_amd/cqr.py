"""ctypes binding of libcqr.so (the C ABI in include/cqr.h).

Argument marshalling only: every step of the coded QR runs in the library's
HIP kernels.  Device buffers are torch tensors (float64, column-major views
are passed by pointer and leading dimension); streams are torch's current HIP
stream.  If the library has not been built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcqr.so")

CQR_OK, CQR_EINVAL, CQR_ENOTRECOVERABLE, CQR_ESINGULAR, CQR_EHIP, CQR_ENOMEM, CQR_EBREAKDOWN = range(7)
CQR_OUT_OF_NODE, CQR_IN_NODE = 0, 1
CQR_FP64, CQR_TRAIL_FP32, CQR_TRAIL_BF16X3 = 0, 1, 2
CQR_PANEL_CHOLQR2, CQR_PANEL_CGS2, CQR_PANEL_ICGS, CQR_PANEL_MGS = 0, 1, 2, 3

EXPORTS = [
    "coded_qr_plan_create", "coded_qr_plan_destroy", "coded_qr_plan_generators", "coded_qr_plan_ftol",
    "coded_qr_workspace_bytes", "coded_qr_encode", "coded_qr_factor", "coded_qr_ws_info",
    "coded_qr_erase", "coded_qr_recover", "coded_qr_postorth", "coded_qr_status_string",
    "coded_qr_profile_enable", "coded_qr_profile_read", "coded_qr_hip_error_name", "coded_qr_solve",
    "coded_qr_solve_workspace_bytes", "coded_qr_solve_noalloc", "coded_qr_backward", "coded_qr_backward_workspace_bytes",
    "coded_qr_solve_backward", "coded_qr_solve_backward_workspace_bytes", "coded_qr_plan_r_rows",
    "coded_qr_plan_placement", "coded_qr_ws_panel_fallbacks",
]

PHASES = ["encode", "reproj_product", "reproj_update", "panel_gram", "panel_chol", "panel_transform",
          "inpanel_projection", "trailing_product", "trailing_update", "split_reduce", "recover", "postorth",
          "erase", "other", "panel_colwise", "solve", "adjoint"]


class CqrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = f", {hip_error_name()}" if status == CQR_EHIP else ""
        super().__init__(f"{where}: {status_string(status)} (status {status}{detail})")


class cqr_config(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("pr", ctypes.c_int32), ("pc", ctypes.c_int32),
                ("kv", ctypes.c_int32), ("kh", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("b", ctypes.c_int32),
                ("reproject", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("lookahead", ctypes.c_int32), ("panel", ctypes.c_int32), ("icgs_eta", ctypes.c_double)]


def _load() -> ctypes.CDLL:
    # torch first: libcqr.so then binds to the HIP runtime torch has loaded.
    # Loaded the other way round, the process would hold two HIP/HSA runtimes
    # and the library's would find no device.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_11943_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ, D, V = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t,
                             ctypes.c_void_p, ctypes.c_void_p)
    sig = {
        "coded_qr_plan_create": (I32, [ctypes.POINTER(cqr_config), P, P, ctypes.POINTER(ctypes.c_void_p)]),
        "coded_qr_plan_destroy": (None, [P]),
        "coded_qr_plan_generators": (I32, [P, P, P]),
        "coded_qr_plan_ftol": (I32, [P]),
        "coded_qr_plan_placement": (I32, [P, P, P]),
        "coded_qr_workspace_bytes": (SZ, [P]),
        "coded_qr_encode": (I32, [P, D, I64, V]),
        "coded_qr_factor": (I32, [P, D, I64, D, I64, I32, I32, D, SZ, V]),
        "coded_qr_ws_info": (I32, [P, D, V, ctypes.POINTER(ctypes.c_int32)]),
        "coded_qr_ws_panel_fallbacks": (I32, [P, D, V, ctypes.POINTER(ctypes.c_int32)]),
        "coded_qr_erase": (I32, [P, D, I64, D, I64, P, I32, V]),
        "coded_qr_recover": (I32, [P, D, I64, D, I64, P, I32, V]),
        "coded_qr_postorth": (I32, [P, D, I64, D, I64, D, I64, D, I64, I32, V]),
        "coded_qr_solve": (I32, [P, D, I64, D, I64, D, I64, I32, D, I64, V, ctypes.c_size_t, V]),
        "coded_qr_solve_workspace_bytes": (ctypes.c_size_t, [P, I32]),
        "coded_qr_solve_noalloc": (I32, [P, D, I64, D, I64, D, I64, I32, D, I64, V]),
        "coded_qr_backward_workspace_bytes": (ctypes.c_size_t, [P]),
        "coded_qr_plan_r_rows": (I64, [P]),
        "coded_qr_backward": (I32, [P, D, I64, D, I64, D, I64, D, I64, D, I64, V, ctypes.c_size_t, V]),
        "coded_qr_solve_backward_workspace_bytes": (ctypes.c_size_t, [P, I32]),
        "coded_qr_solve_backward": (I32, [P, D, I64, D, I64, D, I64, D, I64, D, I64, I32, D, I64, D, I64, D, I64,
                                          V, ctypes.c_size_t, V]),
        "coded_qr_status_string": (ctypes.c_char_p, [I32]),
        "coded_qr_hip_error_name": (ctypes.c_char_p, []),
        "coded_qr_profile_enable": (I32, [P, I32]),
        "coded_qr_profile_read": (I32, [P, I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()


def status_string(status: int) -> str:
    return LIB.coded_qr_status_string(status).decode()


def hip_error_name() -> str:
    """HIP error behind this thread's most recent CQR_EHIP."""
    return LIB.coded_qr_hip_error_name().decode()


def _check(status: int, where: str):
    if status != CQR_OK:
        raise CqrError(status, where)


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _ld(t) -> int:
    """Leading dimension of a column-major (Fortran-ordered) 2-D tensor view.
    Single-column tensors may carry any column stride; their ld is the row count."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    rows, cols = t.shape
    if cols <= 1:
        if rows > 1 and t.stride(0) != 1:
            raise ValueError("expected a column-major 2-D tensor (stride(0) == 1)")
        return max(rows, 1)
    if rows > 1 and t.stride(0) != 1:
        raise ValueError("expected a column-major 2-D tensor (stride(0) == 1)")
    return max(t.stride(1), 1)


def col_major(rows: int, cols: int, device, dtype=None):
    """Zero tensor of shape (rows, cols) in column-major layout."""
    import torch
    dt = dtype or torch.float64
    return torch.zeros((cols, rows), dtype=dt, device=device).t()


def to_device_colmajor(a: np.ndarray, device):
    """Copy a numpy matrix to the device in column-major layout."""
    import torch
    a = np.asarray(a, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(device).t()


@dataclass
class Config:
    m: int
    n: int
    pr: int
    pc: int
    kv: int
    kh: int
    b: int
    storage: int = CQR_OUT_OF_NODE
    reproject: int = 1
    precision: int = CQR_FP64
    lookahead: int = 1
    panel: int = CQR_PANEL_CHOLQR2
    icgs_eta: float = 0.0

    def c(self) -> cqr_config:
        return cqr_config(self.m, self.n, self.pr, self.pc, self.kv, self.kh, self.storage, self.b,
                          self.reproject, self.precision, self.lookahead, self.panel, self.icgs_eta)

    @property
    def bs(self):
        return self.m // self.pr

    @property
    def bw(self):
        return self.n // self.pc

    @property
    def mp(self):
        return self.m + self.kv * self.bs

    @property
    def N(self):
        return self.n + self.kh * self.bw

    @property
    def npanels(self):
        return self.n // self.b


# ---------------------------------------------------------------- raw entry points
def coded_qr_plan_create(cfg: Config, v_tilde: np.ndarray | None, gh: np.ndarray | None) -> int:
    c = cfg.c()
    v = np.ascontiguousarray(v_tilde, dtype=np.float64) if v_tilde is not None and cfg.kv else None
    g = np.ascontiguousarray(gh, dtype=np.float64) if gh is not None and cfg.kh else None
    out = ctypes.c_void_p()
    st = LIB.coded_qr_plan_create(ctypes.byref(c), None if v is None else v.ctypes.data_as(ctypes.c_void_p),
                                  None if g is None else g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out))
    _check(st, "coded_qr_plan_create")
    return out.value


def coded_qr_plan_destroy(plan: int):
    LIB.coded_qr_plan_destroy(ctypes.c_void_p(plan))


def coded_qr_plan_generators(plan: int, cfg: Config):
    gv = np.zeros((cfg.kv, cfg.pr))
    gh = np.zeros((cfg.pc, cfg.kh))
    _check(LIB.coded_qr_plan_generators(ctypes.c_void_p(plan), gv.ctypes.data_as(ctypes.c_void_p),
                                        gh.ctypes.data_as(ctypes.c_void_p)), "coded_qr_plan_generators")
    return gv, gh


def coded_qr_plan_placement(plan: int, cfg: Config):
    """(qrow, rcol): the grid row storing each Q-checksum block row and the grid
    column storing each R-checksum block column (extended-grid indices for
    out-of-node storage)."""
    qrow = np.zeros(max(cfg.kv, 1), dtype=np.int32)
    rcol = np.zeros(max(cfg.kh, 1), dtype=np.int32)
    _check(LIB.coded_qr_plan_placement(ctypes.c_void_p(plan), qrow.ctypes.data_as(ctypes.c_void_p),
                                       rcol.ctypes.data_as(ctypes.c_void_p)), "coded_qr_plan_placement")
    return qrow[:cfg.kv].copy(), rcol[:cfg.kh].copy()


def coded_qr_plan_ftol(plan: int) -> int:
    return LIB.coded_qr_plan_ftol(ctypes.c_void_p(plan))


def coded_qr_workspace_bytes(plan: int) -> int:
    return LIB.coded_qr_workspace_bytes(ctypes.c_void_p(plan))


def coded_qr_encode(plan: int, At, stream=None) -> int:
    return LIB.coded_qr_encode(ctypes.c_void_p(plan), _ptr(At), _ld(At), ctypes.c_void_p(_stream(stream)))


def coded_qr_factor(plan: int, At, R, pb: int, pe: int, ws, stream=None) -> int:
    return LIB.coded_qr_factor(ctypes.c_void_p(plan), _ptr(At), _ld(At), _ptr(R), _ld(R), pb, pe, _ptr(ws),
                               ws.numel() * ws.element_size(), ctypes.c_void_p(_stream(stream)))


def coded_qr_ws_info(plan: int, ws, stream=None) -> tuple[int, int]:
    info = ctypes.c_int32(0)
    st = LIB.coded_qr_ws_info(ctypes.c_void_p(plan), _ptr(ws), ctypes.c_void_p(_stream(stream)),
                              ctypes.byref(info))
    return st, info.value


def _nodes(nodes):
    arr = np.ascontiguousarray(np.array(nodes, dtype=np.int32).reshape(-1))
    return arr, len(arr) // 2


def coded_qr_ws_panel_fallbacks(plan: int, ws, stream=None) -> int:
    """Blocking: panel leaves orthogonalised by the column-wise fallback."""
    v = ctypes.c_int32(0)
    _check(LIB.coded_qr_ws_panel_fallbacks(ctypes.c_void_p(plan), _ptr(ws), ctypes.c_void_p(_stream(stream)),
                                           ctypes.byref(v)), "coded_qr_ws_panel_fallbacks")
    return v.value


def coded_qr_erase(plan: int, Q, R, nodes, stream=None) -> int:
    arr, nf = _nodes(nodes)
    return LIB.coded_qr_erase(ctypes.c_void_p(plan), _ptr(Q), _ld(Q), _ptr(R), _ld(R),
                              arr.ctypes.data_as(ctypes.c_void_p), nf, ctypes.c_void_p(_stream(stream)))


def coded_qr_recover(plan: int, Q, R, nodes, stream=None) -> int:
    arr, nf = _nodes(nodes)
    return LIB.coded_qr_recover(ctypes.c_void_p(plan), _ptr(Q), _ld(Q), _ptr(R), _ld(R),
                                arr.ctypes.data_as(ctypes.c_void_p), nf, ctypes.c_void_p(_stream(stream)))


def coded_qr_postorth(plan: int, Q, Qpost, B=None, Bpost=None, stream=None) -> int:
    nrhs = 0 if B is None else B.shape[1]
    return LIB.coded_qr_postorth(ctypes.c_void_p(plan), _ptr(Q), _ld(Q), _ptr(Qpost), _ld(Qpost),
                                 _ptr(B), _ld(B) if B is not None else 0, _ptr(Bpost),
                                 _ld(Bpost) if Bpost is not None else 0, nrhs,
                                 ctypes.c_void_p(_stream(stream)))


def coded_qr_solve_workspace_bytes(plan: int, nrhs: int) -> int:
    return LIB.coded_qr_solve_workspace_bytes(ctypes.c_void_p(plan), nrhs)


def coded_qr_solve(plan: int, Qpost, R, Bpost, X, ws, stream=None) -> int:
    """ws: device tensor of at least coded_qr_solve_workspace_bytes(plan, nrhs) bytes."""
    return LIB.coded_qr_solve(ctypes.c_void_p(plan), _ptr(Qpost), _ld(Qpost), _ptr(R), _ld(R), _ptr(Bpost),
                              _ld(Bpost), Bpost.shape[1], _ptr(X), _ld(X), _ptr(ws),
                              ws.numel() * ws.element_size(), ctypes.c_void_p(_stream(stream)))


# size of coded_qr_solve_noalloc's per-device scratch array
CQR_SOLVE_NOALLOC_MAX_BYTES = 32 << 20


def coded_qr_solve_noalloc(plan: int, Qpost, R, Bpost, X, stream=None) -> int:
    """coded_qr_solve with the library's per-device scratch array instead of a
    workspace (allocates nothing; overlapping calls on one device race)."""
    return LIB.coded_qr_solve_noalloc(ctypes.c_void_p(plan), _ptr(Qpost), _ld(Qpost), _ptr(R), _ld(R), _ptr(Bpost),
                                      _ld(Bpost), Bpost.shape[1], _ptr(X), _ld(X), ctypes.c_void_p(_stream(stream)))


def coded_qr_plan_r_rows(plan: int) -> int:
    return LIB.coded_qr_plan_r_rows(ctypes.c_void_p(plan))


def coded_qr_backward_workspace_bytes(plan: int) -> int:
    return LIB.coded_qr_backward_workspace_bytes(ctypes.c_void_p(plan))


def coded_qr_backward(plan: int, Q, R, dQ, dR, dA, ws, stream=None) -> int:
    return LIB.coded_qr_backward(ctypes.c_void_p(plan), _ptr(Q), _ld(Q), _ptr(R), _ld(R), _ptr(dQ), _ld(dQ),
                                 _ptr(dR), _ld(dR), _ptr(dA), _ld(dA), _ptr(ws), ws.numel() * ws.element_size(),
                                 ctypes.c_void_p(_stream(stream)))


def coded_qr_solve_backward_workspace_bytes(plan: int, nrhs: int) -> int:
    return LIB.coded_qr_solve_backward_workspace_bytes(ctypes.c_void_p(plan), nrhs)


def coded_qr_solve_backward(plan: int, Qpost, R, Bpost, X, dX, dQ, dR, dB, ws, stream=None) -> int:
    return LIB.coded_qr_solve_backward(ctypes.c_void_p(plan), _ptr(Qpost), _ld(Qpost), _ptr(R), _ld(R),
                                       _ptr(Bpost), _ld(Bpost), _ptr(X), _ld(X), _ptr(dX), _ld(dX), X.shape[1],
                                       _ptr(dQ), _ld(dQ), _ptr(dR), _ld(dR), _ptr(dB), _ld(dB), _ptr(ws),
                                       ws.numel() * ws.element_size(), ctypes.c_void_p(_stream(stream)))


def coded_qr_profile_enable(plan: int, enable: bool) -> int:
    return LIB.coded_qr_profile_enable(ctypes.c_void_p(plan), int(bool(enable)))


def coded_qr_profile_read(plan: int, phase: int) -> dict:
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(LIB.coded_qr_profile_read(ctypes.c_void_p(plan), phase, ctypes.byref(ms), ctypes.byref(cnt),
                                     ctypes.byref(fl), ctypes.byref(by)), "coded_qr_profile_read")
    return {"ms": ms.value, "launches": cnt.value, "flops": fl.value, "bytes": by.value}


# ---------------------------------------------------------------- convenience wrapper
class CodedQR:
    """Plan + workspace on one device; methods raise CqrError on a bad status."""

    def __init__(self, cfg: Config, v_tilde=None, gh=None, device="cuda:0"):
        import torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.plan = coded_qr_plan_create(cfg, v_tilde, gh)
        nbytes = coded_qr_workspace_bytes(self.plan)
        self.ws = torch.empty(((nbytes + 7) // 8,), dtype=torch.float64, device=self.device)

    def close(self):
        if self.plan:
            coded_qr_plan_destroy(self.plan)
            self.plan = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ftol(self) -> int:
        return coded_qr_plan_ftol(self.plan)

    def profile(self, enable: bool):
        _check(coded_qr_profile_enable(self.plan, enable), "coded_qr_profile_enable")

    def profile_report(self) -> dict:
        return {name: coded_qr_profile_read(self.plan, i) for i, name in enumerate(PHASES)}

    def generators(self):
        return coded_qr_plan_generators(self.plan, self.cfg)

    @property
    def r_rows(self) -> int:
        return coded_qr_plan_r_rows(self.plan)

    def alloc(self):
        """Column-major A~ (m' x N) and R (r_rows x N) buffers; R_1 is R[:n, :n]."""
        c = self.cfg
        return col_major(c.mp, c.N, self.device), col_major(self.r_rows, c.N, self.device)

    def encode(self, At):
        _check(coded_qr_encode(self.plan, At), "coded_qr_encode")

    def factor(self, At, R, pb=0, pe=None):
        pe = self.cfg.npanels if pe is None else pe
        _check(coded_qr_factor(self.plan, At, R, pb, pe, self.ws), "coded_qr_factor")

    def info(self) -> int:
        st, info = coded_qr_ws_info(self.plan, self.ws)
        if st not in (CQR_OK, CQR_EBREAKDOWN):
            _check(st, "coded_qr_ws_info")
        return info

    def panel_fallbacks(self) -> int:
        """Panel leaves the last factorization handed to the column-wise CGS2
        fallback after a Cholesky-QR breakdown (blocking)."""
        return coded_qr_ws_panel_fallbacks(self.plan, self.ws)

    def erase(self, At, R, nodes):
        _check(coded_qr_erase(self.plan, At, R, nodes), "coded_qr_erase")

    def recover(self, At, R, nodes):
        _check(coded_qr_recover(self.plan, At, R, nodes), "coded_qr_recover")

    def postorth(self, Q, Qpost, B=None, Bpost=None):
        _check(coded_qr_postorth(self.plan, Q, Qpost, B, Bpost), "coded_qr_postorth")

    def solve_workspace(self, nrhs: int):
        import torch
        nbytes = coded_qr_solve_workspace_bytes(self.plan, nrhs)
        return torch.empty(((nbytes + 7) // 8,), dtype=torch.float64, device=self.device)

    def solve(self, Qpost, R, Bpost, X=None, ws=None):
        """X = R_1^{-1} Qpost^T Bpost (n x nrhs, column-major, on the device)."""
        nrhs = Bpost.shape[1]
        X = col_major(self.cfg.n, nrhs, self.device) if X is None else X
        ws = self.solve_workspace(nrhs) if ws is None else ws
        _check(coded_qr_solve(self.plan, Qpost, R, Bpost, X, ws), "coded_qr_solve")
        return X

    def _bytes_buffer(self, nbytes: int):
        import torch
        return torch.empty(((nbytes + 7) // 8,), dtype=torch.float64, device=self.device)

    def backward(self, Q, R, dQ, dR, dA=None):
        """dA (m x n) from the cotangents of Q~[:, :n] and R_1 (coded_qr_backward)."""
        dA = col_major(self.cfg.m, self.cfg.n, self.device) if dA is None else dA
        ws = self._bytes_buffer(coded_qr_backward_workspace_bytes(self.plan))
        _check(coded_qr_backward(self.plan, Q, R, dQ, dR, dA, ws), "coded_qr_backward")
        return dA

    def solve_backward(self, Qpost, R, Bpost, X, dX):
        """(dQ~ (m' x n), dR_1 (n x n), dB (m x nrhs)) from dX (coded_qr_solve_backward)."""
        c = self.cfg
        dQ = col_major(c.mp, c.n, self.device)
        dR = col_major(c.n, c.n, self.device)
        dB = col_major(c.m, X.shape[1], self.device)
        ws = self._bytes_buffer(coded_qr_solve_backward_workspace_bytes(self.plan, X.shape[1]))
        _check(coded_qr_solve_backward(self.plan, Qpost, R, Bpost, X, dX, dQ, dR, dB, ws),
               "coded_qr_solve_backward")
        return dQ, dR, dB

    def run(self, A_dev, schedule=(), B=None):
        """encode -> factor with scheduled erasures/recoveries -> post-orth.
        A_dev: m x n column-major device tensor.  Returns (At, R, Qpost, Bpost)."""
        c = self.cfg
        At, R = self.alloc()
        At[:c.m, :c.n].copy_(A_dev)
        self.encode(At)
        k = 0
        for t, nodes in list(schedule) + [(c.npanels, None)]:
            self.factor(At, R, k, t)
            k = t
            if nodes is None:
                break
            self.erase(At, R, nodes)
            self.recover(At, R, nodes)
        Qpost = Bpost = None
        if c.kv > 0:
            Qpost = col_major(c.m, c.n, self.device)
            if B is not None:
                Bpost = col_major(c.m, B.shape[1], self.device)
            self.postorth(At, Qpost, B, Bpost)
        return At, R, Qpost, Bpost
