"""Blocked randomized QR with column pivoting on an AMD Instinct MI355X.

Thin Python binding of librqrcp (include/rqrcp.h): argument marshalling
only.  Every step of the factorization runs in the library's HIP kernels;
torch supplies device memory and the current stream.  The library must be
built (``python -m paper_1505_08115_amd.build_lib``); importing works without
it, but every call raises if it is missing.

Matrices are passed as torch tensors of shape (rows, cols) in column-major
layout (``stride(0) == 1``), the layout of the C ABI.  ``colmajor(t)`` makes
such a copy.
"""
import atexit
import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librqrcp.so")

(RQRCP_OK, RQRCP_ERR_ARG, RQRCP_ERR_WORKSPACE, RQRCP_ERR_HIP, RQRCP_ERR_UNSUPPORTED, RQRCP_ERR_NONFINITE,
 RQRCP_ERR_TIMEOUT) = range(7)
F64, F32 = 0, 1
PIVOT = {"perm": 0, "ortho": 1}
PRECISION = {"plain": 0, "mixed": 1}
TAIL = {"classical": 0, "sampled": 1}

#: every function that include/rqrcp.h declares
EXPORTS = [
    "rqrcp_default_opts", "rqrcp_create", "rqrcp_set_stream", "rqrcp_destroy", "rqrcp_status_string",
    "rqrcp_check", "rqrcp_last_error", "rqrcp_factor_sizes", "rqrcp_factor", "rqrcp_factor_noalloc",
    "rqrcp_apply_q_work_bytes", "rqrcp_apply_q", "rqrcp_diag_offset",
    "rqrcp_apply_p_work_bytes", "rqrcp_apply_p", "rqrcp_lowrank_work_bytes", "rqrcp_lowrank",
    "rqrcp_lowrank_backward_work_bytes", "rqrcp_lowrank_backward", "rqrcp_sketch", "rqrcp_timing_enable",
    "rqrcp_timing_read", "rqrcp_timing_classes",
]

#: kernel classes of rqrcp_timing_read
KERNEL_CLASSES = ["sketch", "sample_gemm", "qrcp", "moves", "panel", "tfactor", "vt_gemm", "w_gemm",
                  "update_gemm", "ortho", "other"]


class RqrcpError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"status {status}: {message}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int64), ("oversample", ctypes.c_int64), ("rank", ctypes.c_int64),
        ("pivot", ctypes.c_int32), ("precision", ctypes.c_int32), ("tail", ctypes.c_int32),
        ("fixed_pivots", ctypes.c_int32), ("seed", ctypes.c_uint64), ("G", ctypes.c_void_p),
        ("info", ctypes.c_void_p), ("power", ctypes.c_int32), ("panel_pivot", ctypes.c_int32),
        ("diagonalize", ctypes.c_int32),
    ]


_lib = None
_handles = {}
_i64, _u64, _i32, _vp, _sz = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t


def load_library():
    """Load librqrcp.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1505_08115_amd.build_lib`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "rqrcp_default_opts": (None, [_vp]),
        "rqrcp_create": (_i32, [ctypes.POINTER(_vp), _vp]),
        "rqrcp_set_stream": (_i32, [_vp, _vp]),
        "rqrcp_destroy": (_i32, [_vp]),
        "rqrcp_status_string": (ctypes.c_char_p, [_i32]),
        "rqrcp_check": (_i32, [_vp, _vp]),
        "rqrcp_last_error": (ctypes.c_char_p, [_vp]),
        "rqrcp_factor_sizes": (_i32, [_i32, _i64, _i64, _vp, ctypes.POINTER(_sz), ctypes.POINTER(_sz),
                                      ctypes.POINTER(_sz), ctypes.POINTER(_sz)]),
        "rqrcp_factor": (_i32, [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _sz]),
        "rqrcp_factor_noalloc": (_i32, [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
        "rqrcp_apply_q_work_bytes": (_sz, [_i32, _i64, _i64, _i64, _i64]),
        "rqrcp_apply_q": (_i32, [_vp, _i32, _i32, _i64, _i64, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _vp,
                                 _sz]),
        "rqrcp_diag_offset": (_sz, [_i64, _i64, _i64]),
        "rqrcp_apply_p_work_bytes": (_sz, [_i32, _i64, _i64, _i64, _i64]),
        "rqrcp_apply_p": (_i32, [_vp, _i32, _i32, _i64, _i64, _i64, _i64, _vp, _vp, _i32, _vp, _i64, _vp, _sz]),
        "rqrcp_lowrank_work_bytes": (_sz, [_i32, _i64, _i64, _i64, _i64]),
        "rqrcp_lowrank": (_i32, [_vp, _i32, _i64, _i64, _i64, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _i32, _vp,
                                 _i64, _vp, _sz]),
        "rqrcp_lowrank_backward_work_bytes": (_sz, [_i32, _i64, _i64, _i64, _i64]),
        "rqrcp_lowrank_backward": (_i32, [_vp, _i32, _i64, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp,
                                          _vp, _i64, _vp, _i64, _vp, _sz]),
        "rqrcp_sketch": (_i32, [_vp, _u64, _i64, _i64, _i64, _i64, _vp, _i64]),
        "rqrcp_timing_enable": (_i32, [_vp, _i32]),
        "rqrcp_timing_classes": (_i32, [_vp, ctypes.c_uint32]),
        "rqrcp_timing_read": (_i32, [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(st, h=None):
    if st != RQRCP_OK:
        msg = load_library().rqrcp_last_error(h).decode()
        raise RqrcpError(st, msg)


def handle(device=None):
    """Library handle bound to torch's current stream on `device`."""
    L = load_library()
    dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, stream)
    h = _handles.get(key)
    if h is None:
        with torch.cuda.device(dev):
            hp = _vp()
            _check(L.rqrcp_create(ctypes.byref(hp), _vp(stream)))
        h = hp
        _handles[key] = h
    return h


def _destroy_handles():
    """Synchronise and destroy every handle before the HIP runtime is torn
    down at exit (their streams and events must not outlive it)."""
    if _lib is None:
        return
    for key, h in list(_handles.items()):
        try:
            torch.cuda.synchronize(key[0])
        except Exception:  # pragma: no cover - the runtime may already be gone
            pass
        _lib.rqrcp_destroy(h)
        del _handles[key]


atexit.register(_destroy_handles)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def colmajor(t):
    """A column-major (stride(0) == 1) copy of a 2-D tensor (always a new tensor)."""
    m, n = t.shape
    out = torch.empty_strided((m, n), (1, max(1, m)), dtype=t.dtype, device=t.device)
    out.copy_(t)
    return out


def _ld(t):
    assert t.dim() == 2 and t.stride(0) == 1, "expected a column-major 2-D tensor (stride(0) == 1)"
    return max(1, t.stride(1)) if t.shape[1] > 1 else max(1, t.shape[0])


def _dt(t):
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def make_opts(block=128, oversample=10, rank=0, pivot="perm", precision="plain", tail="classical",
              fixed_pivots=False, seed=0, G=None, info=None, power=0, panel_pivot=False, diagonalize=False):
    o = Opts()
    o.block, o.oversample, o.rank = int(block), int(oversample), int(rank)
    o.pivot, o.precision, o.tail = PIVOT[pivot], PRECISION[precision], TAIL[tail]
    o.fixed_pivots = 1 if fixed_pivots else 0
    o.seed = int(seed) & (2 ** 64 - 1)
    o.G = G.data_ptr() if G is not None else None
    o.info = info.data_ptr() if info is not None else None
    o.power = int(power)
    o.panel_pivot = 1 if panel_pivot else 0
    o.diagonalize = 1 if diagonalize else 0
    return o


def factor_sizes(m, n, dtype=torch.float64, **kw):
    """(tau_elems, T_elems, S_elems, work_bytes) of rqrcp_factor (host only)."""
    L = load_library()
    o = make_opts(**kw)
    a, b, c, d = _sz(), _sz(), _sz(), _sz()
    dt = F64 if dtype == torch.float64 else F32
    _check(L.rqrcp_factor_sizes(dt, m, n, ctypes.byref(o), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


@dataclass
class Factorization:
    F: torch.Tensor               # R on/above the diagonal, Householder vectors below (column-major)
    jpvt: torch.Tensor            # int32[n]
    tau: torch.Tensor             # float64[k]
    T: torch.Tensor               # float64[nblocks * b * b]
    S: Optional[torch.Tensor]     # orthonormal pivoting blocks, or None
    block: int
    rank: int
    pivot: str
    diagonalized: bool = False    # Section 6.2: U'_i, V'_i stored in S after the T_S blocks
    info: Optional[torch.Tensor] = None   # device int32[4], the factorization's info word

    def check(self):
        """Synchronise and read the info word: raise RqrcpError if a grid-wide
        wait gave up (the results are invalid); otherwise return the four
        flags ([0] = 1 if a non-finite norm was met, [1] = its block + 1)."""
        if self.info is None:
            return [0, 0, 0, 0]
        torch.cuda.current_stream(self.info.device).synchronize()
        iv = self.info.cpu().tolist()
        if iv[2]:
            raise RqrcpError(RQRCP_ERR_TIMEOUT, "a grid-wide wait gave up: the factorization is invalid")
        return iv


class Workspace:
    """Reusable device workspace for rqrcp_factor (grows on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes, device):
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


def factor_into(F, jpvt, tau, T, S, work, *, block=128, oversample=10, rank=0, pivot="perm", precision="plain",
                tail="classical", fixed_pivots=False, seed=0, G=None, info=None, power=0, panel_pivot=False,
                diagonalize=False):
    """rqrcp_factor on caller-owned buffers (F is factored in place)."""
    L = load_library()
    m, n = F.shape
    o = make_opts(block, oversample, rank, pivot, precision, tail, fixed_pivots, seed, G, info, power, panel_pivot,
                  diagonalize)
    h = handle(F.device)
    _check(L.rqrcp_factor(h, _dt(F), m, n, _ptr(F), _ld(F), _ptr(jpvt), _ptr(tau), _ptr(T), _ptr(S),
                          ctypes.byref(o), _ptr(work), work.numel()), h)


def factor(A, block=128, oversample=10, seed=0, pivot="perm", precision="plain", rank=0, tail="classical",
           G=None, jpvt=None, info=None, workspace=None, power=0, panel_pivot=False,
           diagonalize=False) -> Factorization:
    """A P = Q R by blocked randomized QRCP.  A is not modified.

    jpvt: optional int32[n] of fixed pivots (factor A(:, jpvt) without any
    sketch; permutation form only).  power: q steps of the power iteration
    of Section 6.3 on every sketch.  panel_pivot: Fig. 3's in-block pivot
    P-hat (permutation form).  diagonalize:
    Section 6.2's diagonal blocks (with pivot="ortho": blockRRQR)."""
    m, n = A.shape
    F = colmajor(A)
    kk = n if rank in (0, None) else int(rank)
    sizes = factor_sizes(m, n, A.dtype, block=block, oversample=oversample, rank=kk, pivot=pivot,
                         precision=precision, tail=tail, fixed_pivots=jpvt is not None, seed=seed, power=power,
                         panel_pivot=panel_pivot, diagonalize=diagonalize)
    dev = A.device
    tau = torch.empty(max(1, sizes[0]), dtype=torch.float64, device=dev)
    T = torch.empty(max(1, sizes[1]), dtype=torch.float64, device=dev)
    S = torch.empty(sizes[2], dtype=torch.float64, device=dev) if pivot == "ortho" else None
    jp = jpvt.to(device=dev, dtype=torch.int32).clone() if jpvt is not None else torch.empty(n, dtype=torch.int32, device=dev)
    if info is None:
        info = torch.zeros(4, dtype=torch.int32, device=dev)
    ws = workspace or Workspace()
    work = ws.get(sizes[3], dev)
    factor_into(F, jp, tau, T, S, work, block=block, oversample=oversample, rank=kk, pivot=pivot,
                precision=precision, tail=tail, fixed_pivots=jpvt is not None, seed=seed, G=G, info=info,
                power=power, panel_pivot=panel_pivot, diagonalize=diagonalize)
    return Factorization(F, jp, tau, T, S, int(block), kk, pivot, bool(diagonalize), info)


#: workspace bytes of rqrcp_factor_noalloc (RQRCP_NOALLOC_WORK_BYTES)
NOALLOC_WORK_BYTES = 64 << 20


def factor_noalloc(A, block=128, oversample=10, seed=0, pivot="perm", precision="plain", rank=0,
                   tail="classical", G=None, jpvt=None, info=None, power=0, panel_pivot=False,
                   diagonalize=False) -> Factorization:
    """factor() through rqrcp_factor_noalloc: the library's own device array
    serves as the workspace (the outputs are still allocated here, by torch)."""
    L = load_library()
    m, n = A.shape
    F = colmajor(A)
    kk = n if rank in (0, None) else int(rank)
    sizes = factor_sizes(m, n, A.dtype, block=block, oversample=oversample, rank=kk, pivot=pivot,
                         precision=precision, tail=tail, fixed_pivots=jpvt is not None, seed=seed, power=power,
                         panel_pivot=panel_pivot, diagonalize=diagonalize)
    dev = A.device
    tau = torch.empty(max(1, sizes[0]), dtype=torch.float64, device=dev)
    T = torch.empty(max(1, sizes[1]), dtype=torch.float64, device=dev)
    S = torch.empty(sizes[2], dtype=torch.float64, device=dev) if pivot == "ortho" else None
    jp = jpvt.to(device=dev, dtype=torch.int32).clone() if jpvt is not None else torch.empty(n, dtype=torch.int32, device=dev)
    if info is None:
        info = torch.zeros(4, dtype=torch.int32, device=dev)
    o = make_opts(block, oversample, kk, pivot, precision, tail, jpvt is not None, seed, G, info, power, panel_pivot,
                  diagonalize)
    h = handle(dev)
    with torch.cuda.device(dev):
        _check(L.rqrcp_factor_noalloc(h, _dt(F), m, n, _ptr(F), _ld(F), _ptr(jp), _ptr(tau), _ptr(T), _ptr(S),
                                      ctypes.byref(o)), h)
    return Factorization(F, jp, tau, T, S, int(block), kk, pivot, bool(diagonalize), info)


def _uv_ptr(Fz):
    """Device address of the U'/V' blocks of a diagonalised factorization, or None."""
    if not Fz.diagonalized:
        return None
    off = load_library().rqrcp_diag_offset(Fz.F.shape[1], Fz.rank, Fz.block)
    return Fz.S.data_ptr() + 8 * off


def apply_q(Fz: Factorization, C, trans=False):
    """Q C or Q^T C in place on a column-major C; returns C."""
    L = load_library()
    m, k = Fz.F.shape[0], Fz.rank
    dt = _dt(C)
    wb = L.rqrcp_apply_q_work_bytes(dt, m, k, Fz.block, C.shape[1])
    work = torch.empty(max(wb, 256), dtype=torch.uint8, device=C.device)
    h = handle(C.device)
    _check(L.rqrcp_apply_q(h, dt, 1 if trans else 0, m, k, Fz.block, _ptr(Fz.F), _ld(Fz.F), _ptr(Fz.T),
                           _uv_ptr(Fz), C.shape[1], _ptr(C), _ld(C), _ptr(work), work.numel()), h)
    return C


def apply_p(Fz: Factorization, C, trans=False):
    """C P or C P^T in place on a column-major C (nrow x n); returns C."""
    L = load_library()
    n, k = Fz.F.shape[1], Fz.rank
    dt = _dt(C)
    wb = L.rqrcp_apply_p_work_bytes(dt, C.shape[0], n, k, Fz.block)
    work = torch.empty(max(wb, 256), dtype=torch.uint8, device=C.device)
    h = handle(C.device)
    _check(L.rqrcp_apply_p(h, dt, 1 if trans else 0, C.shape[0], n, k, Fz.block, _ptr(Fz.jpvt), _ptr(Fz.S),
                           1 if Fz.diagonalized else 0, _ptr(C), _ld(C), _ptr(work), work.numel()), h)
    return C


def lowrank(Fz: Factorization, k=None):
    """A_k = Q(:, 0:k) R(0:k, :) P^* as a new column-major tensor."""
    L = load_library()
    m, n = Fz.F.shape
    k = Fz.rank if k is None else int(k)
    dt = _dt(Fz.F)
    Ak = colmajor(torch.empty(m, n, dtype=Fz.F.dtype, device=Fz.F.device))
    wb = L.rqrcp_lowrank_work_bytes(dt, m, n, k, Fz.block)
    work = torch.empty(max(wb, 256), dtype=torch.uint8, device=Ak.device)
    h = handle(Ak.device)
    _check(L.rqrcp_lowrank(h, dt, m, n, k, Fz.rank, Fz.block, _ptr(Fz.F), _ld(Fz.F), _ptr(Fz.jpvt), _ptr(Fz.T),
                           _ptr(Fz.S), 1 if Fz.diagonalized else 0, _ptr(Ak), _ld(Ak), _ptr(work), work.numel()),
           h)
    return Ak


def lowrank_backward(A, Fz: Factorization, dAk, k=None):
    """Gradient w.r.t. A of a loss of A_k, pivots held fixed (column-major in/out).
    Permutation form only (the library's backward reads jpvt, not S)."""
    if Fz.pivot != "perm":
        raise RqrcpError(RQRCP_ERR_UNSUPPORTED, "lowrank_backward covers the permutation form only")
    L = load_library()
    m, n = A.shape
    k = Fz.rank if k is None else int(k)
    dt = _dt(A)
    dA = colmajor(torch.empty(m, n, dtype=A.dtype, device=A.device))
    wb = L.rqrcp_lowrank_backward_work_bytes(dt, m, n, k, Fz.block)
    work = torch.empty(max(wb, 256), dtype=torch.uint8, device=A.device)
    h = handle(A.device)
    _check(L.rqrcp_lowrank_backward(h, dt, m, n, k, Fz.block, _ptr(A), _ld(A), _ptr(Fz.F), _ld(Fz.F),
                                    _ptr(Fz.jpvt), _ptr(Fz.T), _ptr(dAk), _ld(dAk), _ptr(dA), _ld(dA),
                                    _ptr(work), work.numel()), h)
    return dA


def sketch(seed, block, nsample, row0, nrows, device="cuda"):
    """The Gaussian sketch G_i (nsample x nrows, column-major FP64) drawn on the GPU."""
    L = load_library()
    G = colmajor(torch.empty(nsample, nrows, dtype=torch.float64, device=device))
    h = handle(G.device)
    _check(L.rqrcp_sketch(h, int(seed) & (2 ** 64 - 1), block, nsample, row0, nrows, _ptr(G), max(1, nsample)), h)
    return G


def timing_enable(enable=True, device=None):
    """Bracket every kernel class's launches with HIP events (no host sync)."""
    h = handle(device)
    _check(load_library().rqrcp_timing_enable(h, 1 if enable else 0), h)


def timing_classes(classes=None, device=None):
    """Bracket only the named kernel classes while timing is on (None: all)."""
    h = handle(device)
    mask = 0xFFFFFFFF if classes is None else sum(1 << KERNEL_CLASSES.index(c) for c in classes)
    _check(load_library().rqrcp_timing_classes(h, mask), h)


def timing_read(device=None):
    """{class: (launches, ms, flops, bytes)} since the last read; sync first."""
    L = load_library()
    h = handle(device)
    out = {}
    for kc, name in enumerate(KERNEL_CLASSES):
        n, ms, fl, by = _i64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(L.rqrcp_timing_read(h, kc, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)), h)
        if n.value:
            out[name] = (n.value, ms.value, fl.value, by.value)
    return out


class LowRankQRCP(torch.autograd.Function):
    """A -> A_k = Q_k R_k P_k^T (truncated randomized QRCP), differentiable
    with the pivots held fixed.  recompute=True keeps only A and the pivots
    and refactors in the backward pass instead of storing the WY blocks."""

    @staticmethod
    def forward(ctx, A, k, block=128, oversample=10, seed=0, recompute=False):
        Ac = colmajor(A.detach())
        Fz = factor(Ac, block=block, oversample=oversample, seed=seed, rank=k)
        Fz.check()
        Ak = lowrank(Fz, k)
        ctx.k, ctx.block, ctx.recompute = int(k), int(block), bool(recompute)
        ctx.jpvt = Fz.jpvt
        ctx.save_for_backward(Ac)
        ctx.fz = None if recompute else Fz
        return Ak

    @staticmethod
    def backward(ctx, gAk):
        (Ac,) = ctx.saved_tensors
        Fz = ctx.fz
        if Fz is None:
            Fz = factor(Ac, block=ctx.block, oversample=0, rank=ctx.k, jpvt=ctx.jpvt)
            Fz.check()
        dA = lowrank_backward(Ac, Fz, colmajor(gAk.to(Ac.dtype)), ctx.k)
        return dA, None, None, None, None, None
