"""Python binding of libse2n (argument marshalling only).

Every call hands device pointers of torch tensors and the current HIP stream
to the C ABI declared in include/se2n.h; all arithmetic runs in the library's
gfx950 kernels.  Importing this module fails when libse2n.so has not been
built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SE2N_LIB names another build of the library (e.g. one compiled with other
# tuning constants); by default the in-tree build next to this file.
LIB_PATH = os.environ.get("SE2N_LIB") or os.path.join(_HERE, "libse2n.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1304_2062_amd.build` "
        "(the HIP library is required; there is no CPU fallback)"
    )

_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double

_lib.se2n_plan_create.argtypes = [ctypes.POINTER(_vp), _i, _i, _i]
_lib.se2n_plan_destroy.argtypes = [_vp]
_lib.se2n_workspace_bytes.argtypes = [_vp]
_lib.se2n_workspace_bytes.restype = ctypes.c_size_t
_lib.se2n_precompute.argtypes = [_vp, _d, _d, _i, _i, _vp]
_lib.se2n_orient.argtypes = [_vp, _vp, _vp, _d, _vp, _vp, _vp]
_lib.se2n_orient_method.argtypes = [_vp, _d, ctypes.POINTER(_i)]
_lib.se2n_propagator_flags.argtypes = [_vp, _d, _d, _i, _i, _vp, _vp, ctypes.c_long, ctypes.POINTER(_i)]
_lib.se2n_lift.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_lib.se2n_diffuse.argtypes = [_vp, _vp, _d, _d, _i, _i, _vp, _vp]
_lib.se2n_project.argtypes = [_vp, _vp, _i, _vp, _vp]
_lib.se2n_inpaint.argtypes = [_vp, _vp, _vp, _d, _d, _d, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]
_lib.se2n_inpaint_noalloc.argtypes = [_vp, _vp, _vp, _d, _d, _d, _i, _i, _i, _vp, _vp, _vp, _vp]
_lib.se2n_debug_fail_allocations.argtypes = [ctypes.c_long]
_lib.se2n_debug_fail_allocations.restype = _i
_lib.se2n_set_schedule.argtypes = [_vp, _i]
_lib.se2n_last_schedule.argtypes = [_vp, ctypes.POINTER(_i)]
_lib.se2n_restore_workspace_bytes.argtypes = [_vp]
_lib.se2n_restore_workspace_bytes.restype = ctypes.c_size_t
_lib.se2n_restore.argtypes = [_vp, _vp, _vp, _d, _d, _d, _i, _i, _i, _d, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double)]


_lib.se2n_profile.argtypes = [_vp, _i]
_lib.se2n_profile.restype = _i
_lib.se2n_profile_stats.argtypes = [_vp, ctypes.POINTER(KernelStat), _i, ctypes.POINTER(_i)]
_lib.se2n_profile_stats.restype = _i
_lib.se2n_last_error.restype = ctypes.c_char_p
_lib.se2n_version.restype = ctypes.c_char_p
for _name in ("se2n_plan_create", "se2n_plan_destroy", "se2n_precompute", "se2n_orient", "se2n_orient_method", "se2n_propagator_flags", "se2n_lift",
              "se2n_diffuse", "se2n_project", "se2n_inpaint", "se2n_inpaint_noalloc", "se2n_restore",
              "se2n_set_schedule", "se2n_last_schedule"):
    getattr(_lib, _name).restype = _i

F32, F64 = 0, 1
NOALLOC_MAX_BYTES = 64 << 20  # SE2N_NOALLOC_MAX_BYTES
CN, EXACT = 0, 1
PROJ_MAX, PROJ_MEAN = 0, 1

_SCHEMES = {"cn": CN, "exact": EXACT}
_SCHEDULES = {"auto": 0, "propagator": 1, "iterated": 2}
_PROJ = {"max": PROJ_MAX, "mean": PROJ_MEAN}


class Se2nError(RuntimeError):
    """A negative status returned by the library, with its message."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"se2n error {code}: {msg}")
        self.code = code


def _check(rc: int) -> None:
    if rc != 0:
        raise Se2nError(rc, _lib.se2n_last_error().decode())


def debug_fail_allocations(after: int) -> None:
    """Make the library's allocations fail after `after` more successes (-1 resets)."""
    _check(_lib.se2n_debug_fail_allocations(int(after)))


def version() -> str:
    return _lib.se2n_version().decode()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None):
    return None if t is None else _vp(t.data_ptr())


class Plan:
    """A plan for M x M images and N orientations in float32 or float64."""

    def __init__(self, M: int, N: int, dtype: torch.dtype = torch.float32, device: int | str | None = None):
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.M, self.N, self.dtype = int(M), int(N), dtype
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else int(device))
        h = _vp()
        with torch.cuda.device(self.device):
            _check(_lib.se2n_plan_create(ctypes.byref(h), self.M, self.N, F32 if dtype == torch.float32 else F64))
        self._h = h
        self._ws = None

    # -- helpers -----------------------------------------------------------
    def _image(self, t: torch.Tensor, name: str, dtype=None) -> torch.Tensor:
        dtype = self.dtype if dtype is None else dtype
        if t.device != self.device or t.dtype != dtype or tuple(t.shape) != (self.M, self.M) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape ({self.M}, {self.M}) on {self.device}")
        return t

    def _volume(self, t: torch.Tensor, name: str) -> torch.Tensor:
        if (t.device != self.device or t.dtype != self.dtype or tuple(t.shape) != (self.N, self.M, self.M)
                or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape "
                             f"({self.N}, {self.M}, {self.M}) on {self.device}")
        return t

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.se2n_workspace_bytes(self._h))

    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        return self._ws

    # -- the C ABI ---------------------------------------------------------
    def precompute(self, T: float, beta: float, n_steps: int, scheme: str = "cn") -> None:
        _check(_lib.se2n_precompute(self._h, float(T), float(beta), int(n_steps), _SCHEMES[scheme], _vp(_stream())))

    def orient(self, f: torch.Tensor, mask: torch.Tensor, sigma: float = 2.0) -> torch.Tensor:
        self._image(f, "f")
        self._image(mask, "mask", torch.uint8)
        rmap = torch.empty((self.M, self.M), dtype=torch.uint8, device=self.device)
        _check(_lib.se2n_orient(self._h, _ptr(f), _ptr(mask), float(sigma), _ptr(rmap), _ptr(self.workspace()),
                                _vp(_stream())))
        return rmap

    def propagator_flags(self, T: float, beta: float, n_steps: int, scheme: str = "cn"):
        """[Q][Q] uint8 host array, Q = M/4 + 1: 1 where the class's propagator is negligible."""
        import numpy as np
        q = _i(0)
        _check(_lib.se2n_propagator_flags(self._h, float(T), float(beta), int(n_steps), _SCHEMES[scheme],
                                          _vp(_stream()), None, 0, ctypes.byref(q)))
        out = np.zeros((q.value, q.value), dtype=np.uint8)
        _check(_lib.se2n_propagator_flags(self._h, float(T), float(beta), int(n_steps), _SCHEMES[scheme],
                                          _vp(_stream()), out.ctypes.data, out.size, ctypes.byref(q)))
        return out

    def orient_radius(self, sigma: float = 2.0) -> int:
        """Compiled radius of the orientation stencil for sigma, 0 for the FFT route."""
        r = _i(0)
        _check(_lib.se2n_orient_method(self._h, float(sigma), ctypes.byref(r)))
        return r.value

    def lift(self, f: torch.Tensor, mask: torch.Tensor, rmap: torch.Tensor) -> torch.Tensor:
        self._image(f, "f")
        self._image(mask, "mask", torch.uint8)
        self._image(rmap, "rmap", torch.uint8)
        psi = torch.empty((self.N, self.M, self.M), dtype=self.dtype, device=self.device)
        _check(_lib.se2n_lift(self._h, _ptr(f), _ptr(mask), _ptr(rmap), _ptr(psi), _vp(_stream())))
        return psi

    def diffuse(self, psi: torch.Tensor, T: float, beta: float, n_steps: int, scheme: str = "cn") -> torch.Tensor:
        """In place; returns psi."""
        self._volume(psi, "psi")
        _check(_lib.se2n_diffuse(self._h, _ptr(psi), float(T), float(beta), int(n_steps), _SCHEMES[scheme],
                                 _ptr(self.workspace()), _vp(_stream())))
        return psi

    def project(self, psi: torch.Tensor, mode: str = "max") -> torch.Tensor:
        self._volume(psi, "psi")
        out = torch.empty((self.M, self.M), dtype=self.dtype, device=self.device)
        _check(_lib.se2n_project(self._h, _ptr(psi), _PROJ[mode], _ptr(out), _vp(_stream())))
        return out

    def inpaint(self, f: torch.Tensor, mask: torch.Tensor, T: float, beta: float, n_steps: int,
                sigma: float = 2.0, scheme: str = "cn", proj: str = "max", rmap_in: torch.Tensor | None = None,
                out: torch.Tensor | None = None, rmap_out: torch.Tensor | None = None):
        """Fused orient -> lift -> diffuse -> project.  Returns (out, rmap)."""
        self._image(f, "f")
        self._image(mask, "mask", torch.uint8)
        if rmap_in is not None:
            self._image(rmap_in, "rmap_in", torch.uint8)
        if out is None:
            out = torch.empty((self.M, self.M), dtype=self.dtype, device=self.device)
        self._image(out, "out")
        if rmap_out is None:
            rmap_out = torch.empty((self.M, self.M), dtype=torch.uint8, device=self.device)
        self._image(rmap_out, "rmap_out", torch.uint8)
        _check(_lib.se2n_inpaint(self._h, _ptr(f), _ptr(mask), float(sigma), float(T), float(beta), int(n_steps),
                                 _SCHEMES[scheme], _PROJ[proj], _ptr(rmap_in), _ptr(rmap_out), _ptr(out),
                                 _ptr(self.workspace()), _vp(_stream())))
        return out, rmap_out

    def inpaint_noalloc(self, f: torch.Tensor, mask: torch.Tensor, T: float, beta: float, n_steps: int,
                        out: torch.Tensor, rmap_out: torch.Tensor | None = None, sigma: float = 2.0,
                        scheme: str = "cn", proj: str = "max", rmap_in: torch.Tensor | None = None):
        """se2n_inpaint_noalloc: the fused path on the library's static scratch.  The
        caller passes every output; the propagators (precompute) and, for FP32
        without rmap_in, the orientation taps (orient_radius) must be prepared."""
        self._image(f, "f")
        self._image(mask, "mask", torch.uint8)
        self._image(out, "out")
        if rmap_in is not None:
            self._image(rmap_in, "rmap_in", torch.uint8)
        if rmap_out is not None:
            self._image(rmap_out, "rmap_out", torch.uint8)
        _check(_lib.se2n_inpaint_noalloc(self._h, _ptr(f), _ptr(mask), float(sigma), float(T), float(beta),
                                         int(n_steps), _SCHEMES[scheme], _PROJ[proj], _ptr(rmap_in),
                                         _ptr(rmap_out), _ptr(out), _vp(_stream())))
        return out

    def set_schedule(self, schedule: str) -> None:
        """'auto' (default), 'propagator' (collapsed, cached per key) or 'iterated' (n CN steps per mode)."""
        _check(_lib.se2n_set_schedule(self._h, _SCHEDULES[schedule]))

    def last_schedule(self) -> str:
        v = _i(0)
        _check(_lib.se2n_last_schedule(self._h, ctypes.byref(v)))
        return {k: n for n, k in _SCHEDULES.items()}[v.value]

    def restore_workspace(self) -> torch.Tensor:
        n = int(_lib.se2n_restore_workspace_bytes(self._h))
        if getattr(self, "_rws", None) is None or self._rws.numel() < n:
            self._rws = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self._rws

    def restore(self, f: torch.Tensor, mask: torch.Tensor, T: float, beta: float, n_intervals: int, eps: float,
                dynamic: bool = False, substeps: int = 1, sigma: float = 2.0, scheme: str = "cn",
                proj: str = "max", rmap_in: torch.Tensor | None = None, out: torch.Tensor | None = None,
                rmap_out: torch.Tensor | None = None, join_out: torch.Tensor | None = None):
        """Static (dynamic=False) or dynamic restoration.  Returns (out, rmap, join)."""
        self._image(f, "f")
        self._image(mask, "mask", torch.uint8)
        if rmap_in is not None:
            self._image(rmap_in, "rmap_in", torch.uint8)
        if out is None:
            out = torch.empty((self.M, self.M), dtype=self.dtype, device=self.device)
        self._image(out, "out")
        if rmap_out is None:
            rmap_out = torch.empty((self.M, self.M), dtype=torch.uint8, device=self.device)
        self._image(rmap_out, "rmap_out", torch.uint8)
        if join_out is None:
            join_out = torch.empty((self.M, self.M), dtype=torch.int16, device=self.device)
        self._image(join_out, "join_out", torch.int16)
        _check(_lib.se2n_restore(self._h, _ptr(f), _ptr(mask), float(sigma), float(T), float(beta),
                                 int(n_intervals), int(substeps), _SCHEMES[scheme], float(eps), 1 if dynamic else 0,
                                 _PROJ[proj], _ptr(rmap_in), _ptr(rmap_out), _ptr(join_out), _ptr(out),
                                 _ptr(self.restore_workspace()), _vp(_stream())))
        return out, rmap_out, join_out

    def profile(self, enable: bool = True) -> None:
        """Enable/disable per-kernel event timing (clears the statistics)."""
        _check(_lib.se2n_profile(self._h, 1 if enable else 0))

    def profile_stats(self) -> dict:
        """{kernel name: (launches, total ms)} of the launches timed so far (synchronises)."""
        n = _i(0)
        _check(_lib.se2n_profile_stats(self._h, None, 0, ctypes.byref(n)))
        arr = (KernelStat * max(n.value, 1))()
        _check(_lib.se2n_profile_stats(self._h, arr, n.value, ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _check(_lib.se2n_plan_destroy(self._h))
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Batched inpainting (FP32)
# ---------------------------------------------------------------------------
class _Item(ctypes.Structure):
    _fields_ = [("M", _i), ("N", _i), ("n_steps", _i), ("scheme", _i), ("proj", _i), ("reserved", _i),
                ("T", _d), ("beta", _d), ("sigma", _d),
                ("f", _vp), ("mask", _vp), ("rmap_out", _vp), ("out", _vp)]


class _Tune(ctypes.Structure):
    _fields_ = [("wg_per_cu", _i), ("order", _i), ("row_groups", _i), ("reserved", _i)]


_IP = ctypes.POINTER(_Item)
_TP = ctypes.POINTER(_Tune)
_lib.se2n_batch_workspace_bytes.argtypes = [_IP, _i]
_lib.se2n_batch_workspace_bytes.restype = ctypes.c_size_t
_lib.se2n_inpaint_batched.argtypes = [_IP, _i, _vp, _vp]
_lib.se2n_batch_autotune.argtypes = [_IP, _i, _vp, _vp, _i, ctypes.c_char_p, _TP, ctypes.POINTER(_d)]
_lib.se2n_batch_load_tune_table.argtypes = [ctypes.c_char_p]
_lib.se2n_batch_set_tune.argtypes = [_IP, _i, _TP]
_lib.se2n_batch_get_tune.argtypes = [_IP, _i, _TP]
_lib.se2n_batch_tiles.argtypes = [_IP, _i, _TP, _i, ctypes.POINTER(_i), _i, ctypes.POINTER(_i)]
_lib.se2n_batch_profile.argtypes = [_i]
_lib.se2n_batch_profile_stats.argtypes = [ctypes.POINTER(KernelStat), _i, ctypes.POINTER(_i)]
for _name in ("se2n_inpaint_batched", "se2n_batch_autotune", "se2n_batch_load_tune_table", "se2n_batch_set_tune",
              "se2n_batch_get_tune", "se2n_batch_tiles", "se2n_batch_profile", "se2n_batch_profile_stats",
              "se2n_batch_clear"):
    getattr(_lib, _name).restype = _i


class BatchItem:
    """One image of a batched inpaint: float32 f and uint8 mask of shape (M, M) on one device.

    out / rmap_out are allocated when not given."""

    def __init__(self, f: torch.Tensor, mask: torch.Tensor, N: int, T: float, beta: float, n_steps: int,
                 sigma: float = 2.0, scheme: str = "cn", proj: str = "max", out: torch.Tensor | None = None,
                 rmap_out: torch.Tensor | None = None):
        M = f.shape[0]
        for name, t, dt in (("f", f, torch.float32), ("mask", mask, torch.uint8)):
            if t.dtype != dt or tuple(t.shape) != (M, M) or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError(f"{name} must be a contiguous {dt} CUDA tensor of shape ({M}, {M})")
        self.f, self.mask = f, mask
        self.M, self.N, self.T, self.beta, self.n_steps = int(M), int(N), float(T), float(beta), int(n_steps)
        self.sigma, self.scheme, self.proj = float(sigma), scheme, proj
        self.out = out if out is not None else torch.empty((M, M), dtype=torch.float32, device=f.device)
        self.rmap_out = rmap_out if rmap_out is not None else torch.empty((M, M), dtype=torch.uint8, device=f.device)
        for name, t, dt in (("out", self.out, torch.float32), ("rmap_out", self.rmap_out, torch.uint8)):
            if t.dtype != dt or tuple(t.shape) != (M, M) or not t.is_contiguous() or t.device != f.device:
                raise ValueError(f"{name} must be a contiguous {dt} tensor of shape ({M}, {M}) on {f.device}")

    def _c(self) -> _Item:
        return _Item(self.M, self.N, self.n_steps, _SCHEMES[self.scheme], _PROJ[self.proj], 0,
                     self.T, self.beta, self.sigma, _ptr(self.f), _ptr(self.mask), _ptr(self.rmap_out),
                     _ptr(self.out))


def _items(items) -> tuple:
    arr = (_Item * len(items))(*[it._c() for it in items])
    return arr, len(items)


def _tune_dict(t: _Tune) -> dict:
    return {"wg_per_cu": t.wg_per_cu, "order": t.order, "row_groups": t.row_groups}


def batch_workspace_bytes(items) -> int:
    arr, n = _items(items)
    b = int(_lib.se2n_batch_workspace_bytes(arr, n))
    if b == 0:
        raise Se2nError(-1, _lib.se2n_last_error().decode())
    return b


def batch_workspace(items) -> torch.Tensor:
    return torch.empty(batch_workspace_bytes(items), dtype=torch.uint8, device=items[0].f.device)


def inpaint_batched(items, workspace: torch.Tensor | None = None) -> list:
    """Inpaint every item with one graph launch; returns [item.out]."""
    arr, n = _items(items)
    ws = workspace if workspace is not None else batch_workspace(items)
    _check(_lib.se2n_inpaint_batched(arr, n, _ptr(ws), _vp(_stream())))
    return [it.out for it in items]


def batch_autotune(items, workspace: torch.Tensor | None = None, reps: int = 3,
                   table_path: str | None = None) -> tuple:
    """Time the candidate schedules, keep the fastest; returns (tune dict, ms per batch)."""
    arr, n = _items(items)
    ws = workspace if workspace is not None else batch_workspace(items)
    t, ms = _Tune(), _d()
    _check(_lib.se2n_batch_autotune(arr, n, _ptr(ws), _vp(_stream()), int(reps),
                                    None if table_path is None else table_path.encode(), ctypes.byref(t),
                                    ctypes.byref(ms)))
    return _tune_dict(t), ms.value


def batch_set_tune(items, wg_per_cu: int, order: int, row_groups: int) -> None:
    arr, n = _items(items)
    t = _Tune(int(wg_per_cu), int(order), int(row_groups), 0)
    _check(_lib.se2n_batch_set_tune(arr, n, ctypes.byref(t)))


def batch_get_tune(items) -> dict:
    arr, n = _items(items)
    t = _Tune()
    _check(_lib.se2n_batch_get_tune(arr, n, ctypes.byref(t)))
    return _tune_dict(t)


def batch_load_tune_table(path: str) -> None:
    _check(_lib.se2n_batch_load_tune_table(path.encode()))


def batch_profile(enable: bool = True) -> None:
    _check(_lib.se2n_batch_profile(1 if enable else 0))


def batch_profile_stats() -> dict:
    n = _i(0)
    _check(_lib.se2n_batch_profile_stats(None, 0, ctypes.byref(n)))
    arr = (KernelStat * max(n.value, 1))()
    _check(_lib.se2n_batch_profile_stats(arr, n.value, ctypes.byref(n)))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}


def batch_clear() -> None:
    _check(_lib.se2n_batch_clear())


# ---------------------------------------------------------------------------
# Learned corrector (BF16 MFMA network)
# ---------------------------------------------------------------------------
_FP = ctypes.POINTER(ctypes.c_float)
_lib.se2n_plan_info.argtypes = [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]
_lib.se2n_cnn_create.argtypes = [ctypes.POINTER(_vp), _i, ctypes.c_uint64]
_lib.se2n_cnn_destroy.argtypes = [_vp]
_lib.se2n_cnn_get_params.argtypes = [_vp, _FP, _i, ctypes.POINTER(_i)]
_lib.se2n_cnn_set_params.argtypes = [_vp, _FP, _i]
_lib.se2n_cnn_workspace_bytes.argtypes = [_vp, _i, _i, _i]
_lib.se2n_cnn_workspace_bytes.restype = ctypes.c_size_t
_lib.se2n_cnn_forward.argtypes = [_vp, _vp, _vp, _i, _i, _vp, _vp]
_lib.se2n_cnn_gradients.argtypes = [_vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _vp]
_lib.se2n_cnn_adam_step.argtypes = [_vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp]
_lib.se2n_cnn_train_step.argtypes = [_vp, _vp, _vp, _i, _i, ctypes.c_float, _vp, _vp, _vp]
_lib.se2n_cnn_profile.argtypes = [_vp, _i]
_lib.se2n_cnn_profile_stats.argtypes = [_vp, ctypes.POINTER(KernelStat), _i, ctypes.POINTER(_i)]
_lib.se2n_corrected_workspace_bytes.argtypes = [_vp, _vp]
_lib.se2n_corrected_workspace_bytes.restype = ctypes.c_size_t
_lib.se2n_inpaint_corrected.argtypes = [_vp, _vp, _vp, _vp, _d, _d, _d, _i, _i, _i, _i, _d, _vp, _vp,
                                        ctypes.POINTER(_i), _vp, _vp]
_lib.se2n_cnn_set_validation.argtypes = [_vp, _i, _d, _d, _i, _i, _i, _d]
_lib.se2n_cnn_get_adam.argtypes = [_vp, _FP, _FP, _i, ctypes.POINTER(_i)]
_lib.se2n_cnn_set_adam.argtypes = [_vp, _FP, _FP, _i, _i]
_lib.se2n_cnn_get_validation.argtypes = [_vp, _i, _d, _d, _i, _i, _i, ctypes.POINTER(_d)]
for _name in ("se2n_plan_info", "se2n_cnn_create", "se2n_cnn_destroy", "se2n_cnn_get_params", "se2n_cnn_set_params",
              "se2n_cnn_forward", "se2n_cnn_gradients", "se2n_cnn_adam_step", "se2n_cnn_train_step",
              "se2n_cnn_profile", "se2n_cnn_profile_stats", "se2n_inpaint_corrected", "se2n_cnn_set_validation",
              "se2n_cnn_get_validation", "se2n_cnn_get_adam", "se2n_cnn_set_adam"):
    getattr(_lib, _name).restype = _i

CNN_PARAMS = 3 * (32 * 32 * 9 + 32)


class Corrector:
    """The learned corrector for N orientations: psi -> psi + r(psi) on FP32
    volumes [N][M][M] or batches [B][N][M][M] (M a multiple of 16)."""

    def __init__(self, N: int, seed: int = 0, device: int | None = None):
        self.N = int(N)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else int(device))
        h = _vp()
        with torch.cuda.device(self.device):
            _check(_lib.se2n_cnn_create(ctypes.byref(h), self.N, int(seed)))
        self._h = h
        self._ws = {}
        self._validation = {}

    def _vol(self, t: torch.Tensor, name: str) -> tuple:
        if t.dim() == 3:
            t = t.unsqueeze(0)
        if (t.dim() != 4 or t.shape[1] != self.N or t.shape[2] != t.shape[3] or t.dtype != torch.float32
                or t.device != self.device or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float32 [B][{self.N}][M][M] (or [{self.N}][M][M]) "
                             f"tensor on {self.device}")
        return t, int(t.shape[0]), int(t.shape[2])

    def workspace(self, M: int, batch: int, training: bool) -> torch.Tensor:
        key = (int(M), int(batch), bool(training))
        if key not in self._ws:
            n = int(_lib.se2n_cnn_workspace_bytes(self._h, key[0], key[1], int(key[2])))
            if n == 0:
                raise Se2nError(-1, _lib.se2n_last_error().decode())
            self._ws[key] = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self._ws[key]

    def params(self):
        import numpy as np
        n = _i(0)
        _check(_lib.se2n_cnn_get_params(self._h, None, 0, ctypes.byref(n)))
        a = np.empty(n.value, dtype=np.float32)
        _check(_lib.se2n_cnn_get_params(self._h, a.ctypes.data_as(_FP), n.value, ctypes.byref(n)))
        return a

    def set_params(self, a) -> None:
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float32)
        _check(_lib.se2n_cnn_set_params(self._h, a.ctypes.data_as(_FP), int(a.size)))

    def forward(self, psi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        v, B, M = self._vol(psi, "psi")
        if out is None:
            out = torch.empty_like(psi)
        o, _, _ = self._vol(out, "out")
        _check(_lib.se2n_cnn_forward(self._h, _ptr(v), _ptr(o), M, B, _ptr(self.workspace(M, B, False)),
                                     _vp(_stream())))
        return out

    def gradients(self, coarse: torch.Tensor, fine: torch.Tensor) -> tuple:
        c, B, M = self._vol(coarse, "coarse")
        f, _, _ = self._vol(fine, "fine")
        grads = torch.empty(CNN_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(_lib.se2n_cnn_gradients(self._h, _ptr(c), _ptr(f), M, B, _ptr(grads), _ptr(loss),
                                       _ptr(self.workspace(M, B, True)), _vp(_stream())))
        return grads, loss

    def adam_step(self, grads: torch.Tensor, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8) -> None:
        if grads.dtype != torch.float32 or grads.numel() != CNN_PARAMS or grads.device != self.device:
            raise ValueError("grads must be a float32 device tensor of the parameter count")
        _check(_lib.se2n_cnn_adam_step(self._h, _ptr(grads), float(lr), float(beta1), float(beta2), float(eps),
                                       _vp(_stream())))

    def train_step(self, coarse: torch.Tensor, fine: torch.Tensor, lr: float,
                   loss: torch.Tensor | None = None) -> torch.Tensor:
        c, B, M = self._vol(coarse, "coarse")
        f, _, _ = self._vol(fine, "fine")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(_lib.se2n_cnn_train_step(self._h, _ptr(c), _ptr(f), M, B, float(lr), _ptr(loss),
                                        _ptr(self.workspace(M, B, True)), _vp(_stream())))
        return loss

    def profile(self, enable: bool = True) -> None:
        _check(_lib.se2n_cnn_profile(self._h, 1 if enable else 0))

    def profile_stats(self) -> dict:
        n = _i(0)
        _check(_lib.se2n_cnn_profile_stats(self._h, None, 0, ctypes.byref(n)))
        arr = (KernelStat * max(n.value, 1))()
        _check(_lib.se2n_cnn_profile_stats(self._h, arr, n.value, ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}

    def set_validation(self, M: int, T: float, beta: float, n_coarse: int, n_fine: int, rel_l2: float,
                       scheme: str = "cn") -> None:
        """Record the measured volume rel-L2 against the n_fine-step FP64 solve in a regime."""
        _check(_lib.se2n_cnn_set_validation(self._h, int(M), float(T), float(beta), int(n_coarse), int(n_fine),
                                            _SCHEMES[scheme], float(rel_l2)))
        self._validation[(int(M), float(T), float(beta), int(n_coarse), int(n_fine), scheme)] = float(rel_l2)

    def validation(self, M: int, T: float, beta: float, n_coarse: int, n_fine: int, scheme: str = "cn"):
        """The recorded rel-L2 of a regime, or None."""
        r = _d()
        _check(_lib.se2n_cnn_get_validation(self._h, int(M), float(T), float(beta), int(n_coarse), int(n_fine),
                                            _SCHEMES[scheme], ctypes.byref(r)))
        return None if r.value < 0 else r.value

    def adam_state(self):
        """(m, v, step) of the Adam optimiser, host copies."""
        import numpy as np
        t = _i(0)
        m = np.empty(CNN_PARAMS, dtype=np.float32)
        v = np.empty(CNN_PARAMS, dtype=np.float32)
        _check(_lib.se2n_cnn_get_adam(self._h, m.ctypes.data_as(_FP), v.ctypes.data_as(_FP), CNN_PARAMS,
                                      ctypes.byref(t)))
        return m, v, t.value

    def set_adam_state(self, m, v, step: int) -> None:
        import numpy as np
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        _check(_lib.se2n_cnn_set_adam(self._h, m.ctypes.data_as(_FP), v.ctypes.data_as(_FP), int(m.size), int(step)))

    def save(self, path: str, with_optimizer: bool = False) -> None:
        """Parameters and validation records (and, for a training checkpoint,
        the Adam state) to a NumPy .npz (no pickled objects)."""
        import numpy as np
        rec = np.array([[k[0], k[1], k[2], k[3], k[4], _SCHEMES[k[5]], v] for k, v in self._validation.items()],
                       dtype=np.float64).reshape(-1, 7)
        extra = {}
        if with_optimizer:
            m, v, t = self.adam_state()
            extra = dict(adam_m=m, adam_v=v, adam_step=np.int64(t))
        np.savez(path, params=self.params(), N=np.int64(self.N), validation=rec, **extra)

    def load(self, path: str) -> None:
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            if int(z["N"]) != self.N:
                raise ValueError(f"{path} holds a network for N={int(z['N'])}, not {self.N}")
            self.set_params(z["params"])
            if "adam_m" in z.files:
                self.set_adam_state(z["adam_m"], z["adam_v"], int(z["adam_step"]))
            rec = z["validation"] if "validation" in z.files else np.zeros((0, 7))
        names = {v: k for k, v in _SCHEMES.items()}
        for M, T, beta, nc, nf, sch, err in rec:
            self.set_validation(int(M), T, beta, int(nc), int(nf), err, names[int(sch)])

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _check(_lib.se2n_cnn_destroy(self._h))
            self._h = None
            self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def inpaint_corrected(plan: Plan, cnn: Corrector, f: torch.Tensor, mask: torch.Tensor, T: float, beta: float,
                      n_steps: int, n_fine: int | None = None, sigma: float = 2.0, scheme: str = "cn",
                      proj: str = "max", max_rel_l2: float = 1e-3, out: torch.Tensor | None = None,
                      rmap_out: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Corrected inpainting (coarse n_steps + network) where the network's recorded
    error against the n_fine-step solve (default 8 n_steps) is within max_rel_l2,
    else the plain fused path with n_fine steps.  Returns (out, rmap, used_fallback)."""
    plan._image(f, "f")
    plan._image(mask, "mask", torch.uint8)
    n_fine = 8 * int(n_steps) if n_fine is None else int(n_fine)
    if out is None:
        out = torch.empty((plan.M, plan.M), dtype=torch.float32, device=plan.device)
    if rmap_out is None:
        rmap_out = torch.empty((plan.M, plan.M), dtype=torch.uint8, device=plan.device)
    if workspace is None:
        n = int(_lib.se2n_corrected_workspace_bytes(plan._h, cnn._h))
        if n == 0:
            raise Se2nError(-1, _lib.se2n_last_error().decode() or "plan and network do not match")
        workspace = torch.empty(n, dtype=torch.uint8, device=plan.device)
    used = _i(0)
    _check(_lib.se2n_inpaint_corrected(plan._h, cnn._h, _ptr(f), _ptr(mask), float(sigma), float(T), float(beta),
                                       int(n_steps), n_fine, _SCHEMES[scheme], _PROJ[proj], float(max_rel_l2),
                                       _ptr(rmap_out), _ptr(out), ctypes.byref(used), _ptr(workspace),
                                       _vp(_stream())))
    return out, rmap_out, bool(used.value)
