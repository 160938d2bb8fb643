"""Python binding of libsr (include/sr.h): argument marshalling only.

Every function here takes torch tensors that already live on the GPU,
checks dtype/shape/contiguity, and passes raw device pointers to the C ABI
of the same name.  All computation happens in the HIP kernels of libsr.so;
there is no fallback of any kind: if the library is missing or fails to
load, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsr.so")

SR_OK, SR_EDEVICE, SR_ENOMEM, SR_EBUSY, SR_EINVAL, SR_ERANGE = 0, -5, -12, -16, -22, -34
_NAMES = {0: "SR_OK", -5: "SR_EDEVICE", -12: "SR_ENOMEM", -16: "SR_EBUSY", -22: "SR_EINVAL",
          -34: "SR_ERANGE"}


class SRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


class Tuning(ctypes.Structure):
    """sr_tuning: pair-loop tiling knobs."""

    _fields_ = [("xsplit", ctypes.c_int32), ("_reserved", ctypes.c_int32 * 3)]


class Box(ctypes.Structure):
    """sr_box: [0, len)^3, periodic or open with a passive skin."""

    _fields_ = [("len", ctypes.c_double * 3), ("periodic", ctypes.c_int32),
                ("_pad", ctypes.c_int32), ("skin", ctypes.c_double)]

    @staticmethod
    def make(L, periodic: bool = True, skin: float = 0.0) -> "Box":
        if isinstance(L, (int, float)):
            L = (float(L),) * 3
        b = Box()
        for d in range(3):
            b.len[d] = float(L[d])
        b.periodic = 1 if periodic else 0
        b.skin = float(skin)
        return b


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsr.so not built at %s (run __graft_entry__.build())" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f32, f64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                 ctypes.c_double, ctypes.c_size_t)
    BP = ctypes.POINTER(Box)
    sig = {
        "sr_ctx_create": (ctypes.c_int, [ctypes.c_int, P, sz, ctypes.POINTER(P)]),
        "sr_ctx_destroy": (ctypes.c_int, [P]),
        "sr_last_error": (ctypes.c_char_p, [P]),
        "sr_set_stream": (ctypes.c_int, [P, P]),
        "sr_arena_info": (ctypes.c_int, [P, ctypes.POINTER(sz), ctypes.POINTER(sz)]),
        "sr_sync": (ctypes.c_int, [P]),
        "sr_grid_dims": (ctypes.c_int, [BP, f64, ctypes.POINTER(i32), ctypes.POINTER(i64)]),
        "sr_scratch_bytes": (ctypes.c_int, [BP, f64, i64, ctypes.c_int, ctypes.POINTER(sz)]),
        "sr_bin": (ctypes.c_int, [P, P, P, P, i64, BP, f64, P, P]),
        "sr_force": (ctypes.c_int, [P, P, P, P, P, i64, BP, f64, f32, f32, P, P, P, P, P]),
        "sr_pair_stats": (ctypes.c_int, [P, P, P, P, i64, BP, f64, f32, P,
                                         ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "sr_timing_enable": (ctypes.c_int, [P, ctypes.c_int]),
        "sr_set_tuning": (ctypes.c_int, [P, ctypes.POINTER(Tuning)]),
        "sr_get_tuning": (ctypes.c_int, [P, ctypes.POINTER(Tuning)]),
        "sr_timing_collect": (ctypes.c_int, [P, ctypes.POINTER(f64), ctypes.POINTER(f64),
                                             ctypes.POINTER(i64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def exported_symbols() -> list[str]:
    return ["sr_ctx_create", "sr_ctx_destroy", "sr_last_error", "sr_set_stream", "sr_arena_info",
            "sr_sync", "sr_grid_dims", "sr_scratch_bytes", "sr_bin", "sr_force", "sr_pair_stats",
            "sr_timing_enable", "sr_timing_collect", "sr_set_tuning", "sr_get_tuning"]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _f32(t, n, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous() and t.dim() == 1 and t.shape[0] == n):
        raise ValueError("%s must be a contiguous 1-D float32 CUDA tensor of length %d" % (name, n))
    return _ptr(t)


def sr_grid_dims(box: Box, cell: float):
    dims = (ctypes.c_int32 * 3)()
    nc = ctypes.c_int64()
    rc = lib.sr_grid_dims(ctypes.byref(box), float(cell), dims, ctypes.byref(nc))
    if rc:
        raise SRError(rc, "bad geometry")
    return tuple(dims), int(nc.value)


def sr_scratch_bytes(box: Box, cell: float, n: int, with_force: bool = True) -> int:
    out = ctypes.c_size_t()
    rc = lib.sr_scratch_bytes(ctypes.byref(box), float(cell), int(n), int(bool(with_force)),
                              ctypes.byref(out))
    if rc:
        raise SRError(rc, "bad geometry")
    return int(out.value)


class Context:
    """sr_ctx: device, stream and scratch arena.  Each call enqueues on the
    torch stream that is current at call time."""

    def __init__(self, device: int = 0, arena_bytes: int = 0):
        self.device = int(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream().cuda_stream
        rc = lib.sr_ctx_create(self.device, ctypes.c_void_p(stream), int(arena_bytes),
                               ctypes.byref(h))
        if rc:
            raise SRError(rc, "sr_ctx_create failed")
        self._h = h

    def _check(self, rc):
        if rc:
            raise SRError(rc, lib.sr_last_error(self._h).decode())

    def _bind_stream(self):
        self._check(lib.sr_set_stream(self._h, ctypes.c_void_p(
            torch.cuda.current_stream(self.device).cuda_stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib.sr_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def arena_info(self):
        a, h = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(lib.sr_arena_info(self._h, ctypes.byref(a), ctypes.byref(h)))
        return int(a.value), int(h.value)

    def sync(self):
        self._check(lib.sr_sync(self._h))

    def set_tuning(self, xsplit: int):
        t = Tuning()
        t.xsplit = int(xsplit)
        self._check(lib.sr_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(lib.sr_get_tuning(self._h, ctypes.byref(t)))
        return {"xsplit": int(t.xsplit)}

    def timing_enable(self, on: bool = True):
        self._check(lib.sr_timing_enable(self._h, int(bool(on))))

    def timing_collect(self):
        """(prep_ms_total, force_ms_total, calls) since the last collect."""
        p, f, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        self._check(lib.sr_timing_collect(self._h, ctypes.byref(p), ctypes.byref(f),
                                          ctypes.byref(c)))
        return float(p.value), float(f.value), int(c.value)


def sr_sync(ctx: Context) -> None:
    ctx.sync()


def sr_bin(ctx: Context, x, y, z, box: Box, cell: float, cell_offsets=None, perm=None):
    """Returns (cell_offsets int32[n_cells+1], perm int32[n]) on the device."""
    n = int(x.shape[0])
    _, nc = sr_grid_dims(box, cell)
    dev = x.device
    if cell_offsets is None:
        cell_offsets = torch.empty(nc + 1, dtype=torch.int32, device=dev)
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)[:n]
    ctx._bind_stream()
    ctx._check(lib.sr_bin(ctx._h, _f32(x, n, "x"), _f32(y, n, "y"), _f32(z, n, "z"), n,
                          ctypes.byref(box), float(cell), _ptr(cell_offsets), _ptr(perm)))
    return cell_offsets, perm


def sr_force(ctx: Context, x, y, z, m, box: Box, cell: float, r_max: float, eps: float, poly,
             out=None, momentum: bool = False):
    """Returns (ax, ay, az, momentum3 or None) on the device."""
    n = int(x.shape[0])
    dev = x.device
    if out is None:
        out = tuple(torch.empty(max(n, 1), dtype=torch.float32, device=dev)[:n] for _ in range(3))
    ax, ay, az = out
    if isinstance(momentum, torch.Tensor):
        if not (momentum.is_cuda and momentum.dtype == torch.float64 and momentum.numel() == 3
                and momentum.is_contiguous()):
            raise ValueError("momentum must be a contiguous float64[3] CUDA tensor")
        mom = momentum
    else:
        mom = torch.zeros(3, dtype=torch.float64, device=dev) if momentum else None
    c = (ctypes.c_float * 6)(*[float(v) for v in poly])
    ctx._bind_stream()
    ctx._check(lib.sr_force(ctx._h, _f32(x, n, "x"), _f32(y, n, "y"), _f32(z, n, "z"),
                            _f32(m, n, "mass"), n, ctypes.byref(box), float(cell), float(r_max),
                            float(eps), c, _f32(ax, n, "ax"), _f32(ay, n, "ay"),
                            _f32(az, n, "az"), _ptr(mom)))
    return ax, ay, az, mom


def sr_pair_stats(ctx: Context, x, y, z, box: Box, cell: float, r_max: float,
                  per_target: bool = False):
    """Returns (useful, candidates, per_target int32[n] or None); waits."""
    n = int(x.shape[0])
    pt = torch.zeros(max(n, 1), dtype=torch.int32, device=x.device)[:n] if per_target else None
    u, c = ctypes.c_int64(), ctypes.c_int64()
    ctx._bind_stream()
    ctx._check(lib.sr_pair_stats(ctx._h, _f32(x, n, "x"), _f32(y, n, "y"), _f32(z, n, "z"), n,
                                 ctypes.byref(box), float(cell), float(r_max), _ptr(pt),
                                 ctypes.byref(u), ctypes.byref(c)))
    return int(u.value), int(c.value), pt
