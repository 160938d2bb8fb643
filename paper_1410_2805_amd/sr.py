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

    _fields_ = [("xsplit", ctypes.c_int32), ("order", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("cell_scale", ctypes.c_float)]


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


class BatchBox(ctypes.Structure):
    """sr_batch_box: one box of a plan (device pointers)."""

    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("mass", ctypes.c_void_p), ("n", ctypes.c_int64), ("box", Box),
                ("cell", ctypes.c_double), ("ax", ctypes.c_void_p), ("ay", ctypes.c_void_p),
                ("az", ctypes.c_void_p), ("cell3", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("len", ctypes.c_double), ("steps", ctypes.c_int32),
                ("dt", ctypes.c_float),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("vx", ctypes.c_void_p), ("vy", ctypes.c_void_p), ("vz", ctypes.c_void_p),
                ("mass", ctypes.c_void_p),
                ("out_x", ctypes.c_void_p), ("out_y", ctypes.c_void_p), ("out_z", ctypes.c_void_p),
                ("out_vx", ctypes.c_void_p), ("out_vy", ctypes.c_void_p),
                ("out_vz", ctypes.c_void_p), ("out_kinetic", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("r_max", ctypes.c_float), ("eps", ctypes.c_float), ("poly", ctypes.c_float * 6),
                ("cell", ctypes.c_double), ("tuning", Tuning)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("active", ctypes.c_int64),
                ("draining", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("state_bytes_in_use", ctypes.c_size_t),
                ("state_bytes_high_water", ctypes.c_size_t),
                ("state_bytes_capacity", ctypes.c_size_t),
                ("scratch_bytes_capacity", ctypes.c_size_t), ("ticks", ctypes.c_int64)]


class StepParams(ctypes.Structure):
    """sr_step_params: one full step of Eq. (tstep)."""

    _fields_ = [("r_max", ctypes.c_float), ("eps", ctypes.c_float), ("poly", ctypes.c_float * 6),
                ("cell", ctypes.c_double), ("dt", ctypes.c_float), ("n_sub", ctypes.c_int32),
                ("ml_d", ctypes.c_int32), ("ml_min", ctypes.c_int32), ("ml_max", ctypes.c_int32)]

    @staticmethod
    def make(r_max, eps, poly, cell, dt, n_sub, ml=None) -> "StepParams":
        """ml = (d, l_min, l_max) switches on multilevel subcycles."""
        p = StepParams()
        p.r_max, p.eps, p.cell, p.dt, p.n_sub = float(r_max), float(eps), float(cell), float(dt), \
            int(n_sub)
        if ml is not None:
            p.ml_d, p.ml_min, p.ml_max = (int(v) for v in ml)
        for k in range(6):
            p.poly[k] = float(poly[k])
        return p


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
        "sr_force_static": (ctypes.c_int, [P, P, P, P, P, i64, BP, f64, f32, f32, P, P, P, P,
                                           P]),
        "sr_force_static_capacity": (sz, []),
        "sr_pair_stats": (ctypes.c_int, [P, P, P, P, i64, BP, f64, f32, P,
                                         ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "sr_timing_enable": (ctypes.c_int, [P, ctypes.c_int]),
        "sr_set_tuning": (ctypes.c_int, [P, ctypes.POINTER(Tuning)]),
        "sr_split_from_f64": (ctypes.c_int, [P, P, P, P, i64, BP, f64, P, P, P, P]),
        "sr_split_to_f64": (ctypes.c_int, [P, P, P, P, P, i64, BP, f64, P, P, P]),
        "sr_force_split": (ctypes.c_int, [P, P, P, P, P, P, i64, BP, f64, f32, f32, P, P, P, P,
                                          P]),
        "sr_sks_split": (ctypes.c_int, [P, P, P, P, P, P, P, P, P, i64, BP, f64, f32, f32, P,
                                        f32, P, P, P]),
        "sr_plan_create": (ctypes.c_int, [P, ctypes.POINTER(BatchBox), ctypes.c_int, f32, f32, P,
                                          P, ctypes.POINTER(P)]),
        "sr_plan_set_tuning": (ctypes.c_int, [P, ctypes.POINTER(Tuning)]),
        "sr_plan_get_tuning": (ctypes.c_int, [P, ctypes.POINTER(Tuning)]),
        "sr_plan_run": (ctypes.c_int, [P]),
        "sr_plan_capture": (ctypes.c_int, [P]),
        "sr_plan_launch": (ctypes.c_int, [P]),
        "sr_plan_autotune": (ctypes.c_int, [P, ctypes.c_int, ctypes.POINTER(Tuning),
                                            ctypes.POINTER(f64)]),
        "sr_plan_destroy": (ctypes.c_int, [P]),
        "sr_server_create": (ctypes.c_int, [P, ctypes.POINTER(ServerConfig), ctypes.POINTER(P)]),
        "sr_server_submit": (ctypes.c_int, [P, ctypes.POINTER(Request), ctypes.POINTER(i64)]),
        "sr_server_tick": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int)]),
        "sr_server_poll": (ctypes.c_int, [P, ctypes.POINTER(i64), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int)]),
        "sr_server_cancel": (ctypes.c_int, [P, i64]),
        "sr_server_info_get": (ctypes.c_int, [P, ctypes.POINTER(ServerInfo)]),
        "sr_server_destroy": (ctypes.c_int, [P]),
        "sr_get_tuning": (ctypes.c_int, [P, ctypes.POINTER(Tuning)]),
        "sr_timing_collect": (ctypes.c_int, [P, ctypes.POINTER(f64), ctypes.POINTER(f64),
                                             ctypes.POINTER(i64)]),
        "sr_kinetic": (ctypes.c_int, [P, P, P, P, P, i64, P]),
        "sr_permute": (ctypes.c_int, [P, P, i64, i32, P, P]),
        "sr_force_tree": (ctypes.c_int, [P, P, P, P, P, i64, BP, f64, f32, f32, P, i32, P, P, P,
                                         P]),
        "sr_tree_leaves": (ctypes.c_int, [P, P, P, P, P, i64, BP, f64, i32, P,
                                          ctypes.POINTER(i64)]),
        "sr_pm_create": (ctypes.c_int, [P, i32, f64, f32, i32, ctypes.POINTER(P)]),
        "sr_pm_destroy": (ctypes.c_int, [P]),
        "sr_pm_bytes": (ctypes.c_int, [i32, ctypes.POINTER(sz)]),
        "sr_pm_deposit": (ctypes.c_int, [P, P, P, P, P, i64, P]),
        "sr_pm_fft": (ctypes.c_int, [P, P, i32]),
        "sr_pm_force": (ctypes.c_int, [P, P, P, P, P, i64, P, P, P]),
        "sr_pm_force_split": (ctypes.c_int, [P, P, P, P, P, P, i64, f64, P, P, P]),
        "sr_ksk_step": (ctypes.c_int, [P, P, P, P, P, P, P, P, P, P, i64, BP,
                                       ctypes.POINTER(StepParams), P, P, P, i32, P, P, P]),
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
            "sr_timing_enable", "sr_timing_collect", "sr_set_tuning", "sr_get_tuning",
            "sr_split_from_f64", "sr_split_to_f64", "sr_force_split", "sr_sks_split",
            "sr_plan_create", "sr_plan_set_tuning", "sr_plan_get_tuning", "sr_plan_run",
            "sr_plan_capture", "sr_plan_launch", "sr_plan_autotune", "sr_plan_destroy",
            "sr_server_create", "sr_server_submit", "sr_server_tick", "sr_server_poll",
            "sr_server_cancel", "sr_server_info_get", "sr_server_destroy",
            "sr_pm_create", "sr_pm_destroy", "sr_pm_bytes", "sr_pm_deposit", "sr_pm_fft",
            "sr_pm_force", "sr_pm_force_split", "sr_ksk_step", "sr_force_tree",
            "sr_tree_leaves", "sr_kinetic", "sr_force_static", "sr_force_static_capacity",
            "sr_permute"]


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


def sr_scratch_bytes(box: Box, cell: float, n: int, with_force=True) -> int:
    """with_force: True / 1 sr_force, False / 0 sr_bin, 2 a multilevel
    sr_ksk_step."""
    out = ctypes.c_size_t()
    mode = 2 if with_force == 2 and not isinstance(with_force, bool) else int(bool(with_force))
    rc = lib.sr_scratch_bytes(ctypes.byref(box), float(cell), int(n), mode, ctypes.byref(out))
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

    def set_tuning(self, xsplit: int | None = None, order: int | None = None,
                   persistent: int | None = None):
        cur = self.get_tuning()
        t = Tuning()
        t.xsplit = int(cur["xsplit"] if xsplit is None else xsplit)
        t.order = int(cur["order"] if order is None else order)
        t.persistent = int(cur["persistent"] if persistent is None else persistent)
        t.cell_scale = 1.0
        self._check(lib.sr_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(lib.sr_get_tuning(self._h, ctypes.byref(t)))
        return {"xsplit": int(t.xsplit), "order": int(t.order), "persistent": int(t.persistent)}

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


def sr_permute(ctx: Context, perm, a, out=None):
    """out[k] = a[perm[k]] (a contiguous 1-D CUDA tensor of 4-, 8- or 16-byte
    elements; perm int32); returns out."""
    n = int(perm.shape[0])
    if not (isinstance(perm, torch.Tensor) and perm.is_cuda and perm.dtype == torch.int32
            and perm.is_contiguous() and perm.dim() == 1):
        raise ValueError("perm must be a contiguous 1-D int32 CUDA tensor")
    if not (isinstance(a, torch.Tensor) and a.is_cuda and a.is_contiguous() and a.dim() == 1
            and a.shape[0] == n):
        raise ValueError("a must be a contiguous 1-D CUDA tensor of length %d" % n)
    if out is None:
        out = torch.empty_like(a)
    if not (out.dtype == a.dtype and out.is_cuda and out.is_contiguous() and out.shape == a.shape):
        raise ValueError("out must match a")
    ctx._bind_stream()
    ctx._check(lib.sr_permute(ctx._h, _ptr(perm), n, a.element_size(), _ptr(a), _ptr(out)))
    return out


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


def sr_force_static(ctx: Context, x, y, z, m, box: Box, cell: float, r_max: float, eps: float,
                    poly, out, momentum=None):
    """sr_force with the library's fixed scratch array: the outputs (ax, ay,
    az) and the optional float64[3] momentum are caller-allocated tensors,
    and the call allocates nothing.  Returns (ax, ay, az, momentum)."""
    n = int(x.shape[0])
    ax, ay, az = out
    if momentum is not None and not (momentum.is_cuda and momentum.dtype == torch.float64
                                     and momentum.numel() == 3 and momentum.is_contiguous()):
        raise ValueError("momentum must be a contiguous float64[3] CUDA tensor")
    c = (ctypes.c_float * 6)(*[float(v) for v in poly])
    ctx._bind_stream()
    ctx._check(lib.sr_force_static(ctx._h, _f32(x, n, "x"), _f32(y, n, "y"), _f32(z, n, "z"),
                                   _f32(m, n, "mass"), n, ctypes.byref(box), float(cell),
                                   float(r_max), float(eps), c, _f32(ax, n, "ax"),
                                   _f32(ay, n, "ay"), _f32(az, n, "az"), _ptr(momentum)))
    return ax, ay, az, momentum


def sr_force_static_capacity() -> int:
    """Bytes of the fixed scratch array sr_force_static uses (per GPU)."""
    return int(lib.sr_force_static_capacity())


def _typed(t, n, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
            and t.dim() == 1 and t.shape[0] == n):
        raise ValueError("%s must be a contiguous 1-D %s CUDA tensor of length %d" % (name, dtype, n))
    return _ptr(t)


def sr_split_from_f64(ctx: Context, x, y, z, box: Box, cell: float):
    """float64 positions -> (cell3 int32, ox, oy, oz float32) on the device."""
    n = int(x.shape[0])
    dev = x.device
    cell3 = torch.empty(max(n, 1), dtype=torch.int32, device=dev)[:n]
    o = tuple(torch.empty(max(n, 1), dtype=torch.float32, device=dev)[:n] for _ in range(3))
    ctx._bind_stream()
    ctx._check(lib.sr_split_from_f64(ctx._h, _typed(x, n, torch.float64, "x"),
                                     _typed(y, n, torch.float64, "y"),
                                     _typed(z, n, torch.float64, "z"), n, ctypes.byref(box),
                                     float(cell), _ptr(cell3), _ptr(o[0]), _ptr(o[1]),
                                     _ptr(o[2])))
    return cell3, o[0], o[1], o[2]


def sr_split_to_f64(ctx: Context, cell3, ox, oy, oz, box: Box, cell: float):
    n = int(cell3.shape[0])
    dev = cell3.device
    out = tuple(torch.empty(max(n, 1), dtype=torch.float64, device=dev)[:n] for _ in range(3))
    ctx._bind_stream()
    ctx._check(lib.sr_split_to_f64(ctx._h, _typed(cell3, n, torch.int32, "cell3"),
                                   _f32(ox, n, "ox"), _f32(oy, n, "oy"), _f32(oz, n, "oz"), n,
                                   ctypes.byref(box), float(cell), _ptr(out[0]), _ptr(out[1]),
                                   _ptr(out[2])))
    return out


def sr_force_split(ctx: Context, cell3, ox, oy, oz, m, box: Box, cell: float, r_max: float,
                   eps: float, poly, out=None, momentum: bool = False):
    """sr_force on split coordinates; returns (ax, ay, az, momentum3 or None)."""
    n = int(cell3.shape[0])
    dev = cell3.device
    if out is None:
        out = tuple(torch.empty(max(n, 1), dtype=torch.float32, device=dev)[:n] for _ in range(3))
    ax, ay, az = out
    mom = torch.zeros(3, dtype=torch.float64, device=dev) if momentum else None
    c = (ctypes.c_float * 6)(*[float(v) for v in poly])
    ctx._bind_stream()
    ctx._check(lib.sr_force_split(ctx._h, _typed(cell3, n, torch.int32, "cell3"),
                                  _f32(ox, n, "ox"), _f32(oy, n, "oy"), _f32(oz, n, "oz"),
                                  _f32(m, n, "mass"), n, ctypes.byref(box), float(cell),
                                  float(r_max), float(eps), c, _f32(ax, n, "ax"),
                                  _f32(ay, n, "ay"), _f32(az, n, "az"), _ptr(mom)))
    return ax, ay, az, mom


def sr_sks_split(ctx: Context, state: dict, box: Box, cell: float, r_max: float, eps: float,
                 poly, dt: float, out=None):
    """One stream-kick-stream step of one box of split state (the serving
    maps), in place on state's cell3, ox, oy, oz, vx, vy, vz (mass m);
    returns the step's accelerations (ax, ay, az)."""
    n = int(state["cell3"].shape[0])
    dev = state["cell3"].device
    if out is None:
        out = tuple(torch.empty(max(n, 1), dtype=torch.float32, device=dev)[:n] for _ in range(3))
    c = (ctypes.c_float * 6)(*[float(v) for v in poly])
    ctx._bind_stream()
    ctx._check(lib.sr_sks_split(ctx._h, _typed(state["cell3"], n, torch.int32, "cell3"),
                                *(_f32(state[k], n, k) for k in ("ox", "oy", "oz", "vx", "vy",
                                                                  "vz", "m")),
                                n, ctypes.byref(box), float(cell), float(r_max), float(eps), c,
                                float(dt), *(_f32(a, n, "a") for a in out)))
    return out


def sr_force_tree(ctx: Context, x, y, z, m, box: Box, cell: float, r_max: float, eps: float,
                  poly, leaf_max: int = 128, out=None, momentum: bool = False):
    """sr_force through RCB trees in the chaining cells (include/sr.h)."""
    n = int(x.shape[0])
    dev = x.device
    if out is None:
        out = tuple(torch.empty(max(n, 1), dtype=torch.float32, device=dev)[:n] for _ in range(3))
    ax, ay, az = out
    mom = torch.zeros(3, dtype=torch.float64, device=dev) if momentum else None
    c = (ctypes.c_float * 6)(*[float(v) for v in poly])
    ctx._bind_stream()
    ctx._check(lib.sr_force_tree(ctx._h, _f32(x, n, "x"), _f32(y, n, "y"), _f32(z, n, "z"),
                                 _f32(m, n, "mass"), n, ctypes.byref(box), float(cell),
                                 float(r_max), float(eps), c, int(leaf_max), _f32(ax, n, "ax"),
                                 _f32(ay, n, "ay"), _f32(az, n, "az"), _ptr(mom)))
    return ax, ay, az, mom


def sr_kinetic(ctx: Context, vx, vy, vz, m):
    """FP64 sum m |v|^2 / 2 as a one-element float64 device tensor."""
    n = int(vx.shape[0])
    out = torch.zeros(1, dtype=torch.float64, device=vx.device)
    ctx._bind_stream()
    ctx._check(lib.sr_kinetic(ctx._h, _f32(vx, n, "vx"), _f32(vy, n, "vy"), _f32(vz, n, "vz"),
                              _f32(m, n, "mass"), n, _ptr(out)))
    return out


def sr_tree_leaves(ctx: Context, x, y, z, m, box: Box, cell: float, leaf_max: int = 128):
    """(leaf index of every particle as an int32 device tensor, leaf count);
    waits."""
    n = int(x.shape[0])
    leaf_of = torch.empty(max(n, 1), dtype=torch.int32, device=x.device)[:n]
    cnt = ctypes.c_int64()
    ctx._bind_stream()
    ctx._check(lib.sr_tree_leaves(ctx._h, _f32(x, n, "x"), _f32(y, n, "y"), _f32(z, n, "z"),
                                  _f32(m, n, "mass"), n, ctypes.byref(box), float(cell),
                                  int(leaf_max), _ptr(leaf_of), ctypes.byref(cnt)))
    return leaf_of, int(cnt.value)


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


def _tuning_dict(t: Tuning) -> dict:
    return {"xsplit": int(t.xsplit), "order": int(t.order), "persistent": int(t.persistent),
            "cell_scale": float(t.cell_scale)}


class Plan:
    """sr_plan: a batch of independent boxes evaluated in one pass.

    boxes: list of dicts with device tensors x, y, z, m, outputs ax, ay, az,
    and box (Box), cell (float); a box with an int32 tensor "cell3" is in
    split coordinates (x, y, z are then the offsets).  The tensors must
    outlive the plan."""

    def __init__(self, ctx: Context, boxes, r_max: float, eps: float, poly, momentum=None):
        self.ctx = ctx
        arr = (BatchBox * len(boxes))()
        self._keep = []
        for i, b in enumerate(boxes):
            n = int(b["x"].shape[0])
            for k in ("x", "y", "z", "m", "ax", "ay", "az"):
                _f32(b[k], n, k)
                self._keep.append(b[k])
            arr[i].x, arr[i].y, arr[i].z = (b[k].data_ptr() for k in "xyz")
            arr[i].mass = b["m"].data_ptr()
            arr[i].n = n
            arr[i].box = b["box"]
            arr[i].cell = float(b["cell"])
            arr[i].ax, arr[i].ay, arr[i].az = (b[k].data_ptr() for k in ("ax", "ay", "az"))
            if b.get("cell3") is not None:
                arr[i].cell3 = _typed(b["cell3"], n, torch.int32, "cell3")
                self._keep.append(b["cell3"])
        if momentum is not None:
            if not (momentum.is_cuda and momentum.dtype == torch.float64
                    and momentum.numel() == 3 * len(boxes) and momentum.is_contiguous()):
                raise ValueError("momentum must be a contiguous float64[3 * nboxes] CUDA tensor")
            self._keep.append(momentum)
        c = (ctypes.c_float * 6)(*[float(v) for v in poly])
        h = ctypes.c_void_p()
        ctx._bind_stream()
        ctx._check(lib.sr_plan_create(ctx._h, arr, len(boxes), float(r_max), float(eps), c,
                                      _ptr(momentum), ctypes.byref(h)))
        self._h = h

    def run(self):
        self.ctx._check(lib.sr_plan_run(self._h))

    def capture(self):
        self.ctx._check(lib.sr_plan_capture(self._h))

    def launch(self):
        self.ctx._check(lib.sr_plan_launch(self._h))

    def set_tuning(self, xsplit: int, order: int, persistent: int, cell_scale: float = 1.0):
        t = Tuning()
        t.xsplit, t.order, t.persistent, t.cell_scale = int(xsplit), int(order), \
            int(persistent), float(cell_scale)
        self.ctx._check(lib.sr_plan_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        self.ctx._check(lib.sr_plan_get_tuning(self._h, ctypes.byref(t)))
        return _tuning_dict(t)

    def autotune(self, reps: int = 3):
        t = Tuning()
        ms = ctypes.c_double()
        self.ctx._check(lib.sr_plan_autotune(self._h, int(reps), ctypes.byref(t),
                                             ctypes.byref(ms)))
        return _tuning_dict(t), float(ms.value)

    def close(self):
        if getattr(self, "_h", None):
            lib.sr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """sr_server: continuous batching of stream-kick-stream requests.

    submit() takes numpy host arrays, positions and velocities either as
    (n, 3) arrays (copied) or as tuples of three contiguous 1-D arrays (used
    in place); the caller keeps them alive until the request completes.
    Pinned arrays (pinned_empty) keep the input and result copies
    asynchronous; pageable ones make each admission wait for its copy."""

    def __init__(self, ctx: Context, hbm_budget: int, max_slots: int, r_max: float, eps: float,
                 poly, cell: float, xsplit: int = 2, order: int = 1, persistent: int = 0):
        self.ctx = ctx
        cfg = ServerConfig()
        cfg.hbm_budget = int(hbm_budget)
        cfg.max_slots = int(max_slots)
        cfg.r_max, cfg.eps = float(r_max), float(eps)
        for k in range(6):
            cfg.poly[k] = float(poly[k])
        cfg.cell = float(cell)
        cfg.tuning.xsplit, cfg.tuning.order = int(xsplit), int(order)
        cfg.tuning.persistent, cfg.tuning.cell_scale = int(persistent), 1.0
        h = ctypes.c_void_p()
        ctx._bind_stream()
        ctx._check(lib.sr_server_create(ctx._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, L: float, steps: int, dt: float, pos64, vel, mass, out_pos, out_vel,
               out_kinetic=None) -> int:
        """out_kinetic: optional float64 numpy array of one element that
        receives the final state's FP64 kinetic energy."""
        import numpy as np
        n = int(mass.shape[0])
        if isinstance(pos64, (tuple, list)):
            # structure of arrays, used in place (pinned arrays keep the
            # admission copies asynchronous)
            arrs = list(pos64) + list(vel) + [mass]
            for a, dt_ in zip(arrs, [np.float64] * 3 + [np.float32] * 4):
                assert a.dtype == dt_ and a.flags["C_CONTIGUOUS"] and a.shape == (n,)
        else:
            arrs = [np.ascontiguousarray(pos64[:, d], dtype=np.float64) for d in range(3)]
            arrs += [np.ascontiguousarray(vel[:, d], dtype=np.float32) for d in range(3)]
            arrs += [np.ascontiguousarray(mass, dtype=np.float32)]
        for a in list(out_pos) + list(out_vel):
            assert a.flags["C_CONTIGUOUS"] and a.shape[0] == n
        r = Request()
        r.n, r.len, r.steps, r.dt = n, float(L), int(steps), float(dt)
        r.x, r.y, r.z, r.vx, r.vy, r.vz, r.mass = (a.ctypes.data for a in arrs)
        r.out_x, r.out_y, r.out_z = (a.ctypes.data for a in out_pos)
        r.out_vx, r.out_vy, r.out_vz = (a.ctypes.data for a in out_vel)
        if out_kinetic is not None:
            assert out_kinetic.dtype == np.float64 and out_kinetic.size >= 1
            r.out_kinetic = out_kinetic.ctypes.data
        rid = ctypes.c_int64()
        self.ctx._bind_stream()
        self.ctx._check(lib.sr_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._keep[int(rid.value)] = (arrs, out_pos, out_vel, out_kinetic)
        return int(rid.value)

    def tick(self) -> int:
        a = ctypes.c_int()
        self.ctx._bind_stream()
        self.ctx._check(lib.sr_server_tick(self._h, ctypes.byref(a)))
        return int(a.value)

    def poll(self) -> list[int]:
        ids = (ctypes.c_int64 * 256)()
        n = ctypes.c_int()
        out = []
        while True:
            self.ctx._check(lib.sr_server_poll(self._h, ids, 256, ctypes.byref(n)))
            out += [int(ids[k]) for k in range(n.value)]
            if n.value < 256:
                break
        for rid in out:
            self._keep.pop(rid, None)
        return out

    def cancel(self, rid: int):
        self.ctx._check(lib.sr_server_cancel(self._h, int(rid)))

    def info(self) -> dict:
        i = ServerInfo()
        self.ctx._check(lib.sr_server_info_get(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib.sr_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_PINNED = {}


def pinned_empty(shape, dtype):
    """Page-locked host numpy array backed by a pinned torch tensor (kept
    alive for the process; use for serving result buffers)."""
    import numpy as np
    tdt = {np.float64: torch.float64, np.float32: torch.float32}[np.dtype(dtype).type]
    t = torch.empty(shape, dtype=tdt, pin_memory=True)
    a = t.numpy()
    _PINNED[a.ctypes.data] = t
    return a


def pinned_release(a) -> None:
    _PINNED.pop(a.ctypes.data, None)


# ---- long-range PM force and the full step (include/sr_pm.h) -------------

def sr_pm_bytes(ng: int) -> int:
    out = ctypes.c_size_t()
    rc = lib.sr_pm_bytes(int(ng), ctypes.byref(out))
    if rc:
        raise SRError(rc, "bad grid size")
    return int(out.value)


class PM:
    """sr_pm: the long-range solver of one periodic cube (ng^3 grid)."""

    def __init__(self, ctx: Context, ng: int, L: float, sigma: float = 0.8, ns: int = 3):
        self.ctx, self.ng, self.L = ctx, int(ng), float(L)
        h = ctypes.c_void_p()
        ctx._bind_stream()
        ctx._check(lib.sr_pm_create(ctx._h, self.ng, self.L, float(sigma), int(ns),
                                    ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib.sr_pm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _out3(self, n, dev, out):
        if out is None:
            out = tuple(torch.empty(max(n, 1), dtype=torch.float32, device=dev)[:n]
                        for _ in range(3))
        return out

    def deposit(self, x, y, z, m, rho=None):
        """CIC density (ng, ng, ng) float32 (mass per cell volume)."""
        n = int(x.shape[0])
        g = self.ng
        if rho is None:
            rho = torch.empty((g, g, g), dtype=torch.float32, device=x.device)
        if not (rho.is_cuda and rho.dtype == torch.float32 and rho.is_contiguous()
                and rho.numel() == g ** 3):
            raise ValueError("rho must be a contiguous float32 CUDA tensor of ng^3 values")
        self.ctx._bind_stream()
        self.ctx._check(lib.sr_pm_deposit(self._h, _f32(x, n, "x"), _f32(y, n, "y"),
                                          _f32(z, n, "z"), _f32(m, n, "mass"), n, _ptr(rho)))
        return rho

    def fft(self, data, inverse: bool = False):
        """In-place unnormalised 3-D DFT of a complex64 (ng, ng, ng) tensor."""
        g = self.ng
        if not (isinstance(data, torch.Tensor) and data.is_cuda and data.dtype == torch.complex64
                and data.is_contiguous() and data.numel() == g ** 3):
            raise ValueError("data must be a contiguous complex64 CUDA tensor of ng^3 values")
        self.ctx._bind_stream()
        self.ctx._check(lib.sr_pm_fft(self._h, _ptr(data), 1 if inverse else 0))
        return data

    def force(self, x, y, z, m, out=None):
        n = int(x.shape[0])
        ax, ay, az = self._out3(n, x.device, out)
        self.ctx._bind_stream()
        self.ctx._check(lib.sr_pm_force(self._h, _f32(x, n, "x"), _f32(y, n, "y"),
                                        _f32(z, n, "z"), _f32(m, n, "mass"), n,
                                        _f32(ax, n, "ax"), _f32(ay, n, "ay"), _f32(az, n, "az")))
        return ax, ay, az

    def force_split(self, cell3, ox, oy, oz, m, cell: float, out=None):
        n = int(cell3.shape[0])
        ax, ay, az = self._out3(n, cell3.device, out)
        self.ctx._bind_stream()
        self.ctx._check(lib.sr_pm_force_split(
            self._h, _typed(cell3, n, torch.int32, "cell3"), _f32(ox, n, "ox"), _f32(oy, n, "oy"),
            _f32(oz, n, "oz"), _f32(m, n, "mass"), n, float(cell), _f32(ax, n, "ax"),
            _f32(ay, n, "ay"), _f32(az, n, "az")))
        return ax, ay, az


def sr_ksk_step(ctx: Context, pm: PM, state: dict, box: Box, params: StepParams, lr, lr_valid,
                sr_out):
    """One full step on split state {cell3, ox, oy, oz, vx, vy, vz, m} (updated
    in place); lr = (ax, ay, az) PM acceleration (in/out), sr_out receives the
    last subcycle's short-range acceleration."""
    n = int(state["cell3"].shape[0])
    ctx._bind_stream()
    ctx._check(lib.sr_ksk_step(
        ctx._h, pm._h, _typed(state["cell3"], n, torch.int32, "cell3"),
        _f32(state["ox"], n, "ox"), _f32(state["oy"], n, "oy"), _f32(state["oz"], n, "oz"),
        _f32(state["vx"], n, "vx"), _f32(state["vy"], n, "vy"), _f32(state["vz"], n, "vz"),
        _f32(state["m"], n, "mass"), n, ctypes.byref(box), ctypes.byref(params),
        _f32(lr[0], n, "lr_ax"), _f32(lr[1], n, "lr_ay"), _f32(lr[2], n, "lr_az"),
        1 if lr_valid else 0, _f32(sr_out[0], n, "sr_ax"), _f32(sr_out[1], n, "sr_ay"),
        _f32(sr_out[2], n, "sr_az")))
