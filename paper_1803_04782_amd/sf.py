"""Python binding of libsf (include/sf.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
and torch device tensors into the pointers and sizes the C ABI takes.  It
raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsf.so")

SF_OK = 0
SF_EINVAL = -1
SF_ENOMEM = -2
SF_EDEVICE = -3
SF_EUNREACHABLE = -4
SF_MAX_RADIUS = 48
SF_MAX_PEDS = 2147483647 - 1023

SF_FLAG_MOVER = 1
SF_FLAG_WON = 2
SF_FLAG_TIED = 4

SF_KERNEL_SUPERPOSE = 0
SF_KERNEL_DECIDE = 1
SF_KERNEL_COMMIT = 2

# every symbol include/sf.h declares
EXPORTS = ("sf_create_scene", "sf_step", "sf_field", "sf_positions", "sf_last_moves",
           "sf_static_field", "sf_set_state", "sf_stats", "sf_sync", "sf_set_timing",
           "sf_kernel_time", "sf_refresh_field", "sf_set_field_update", "sf_set_field_sect",
           "sf_sect_image", "sf_destroy_scene", "sf_batch_create", "sf_batch_tune",
           "sf_batch_get_tiling", "sf_batch_step", "sf_batch_refresh_field", "sf_batch_stats",
           "sf_batch_sync",
           "sf_batch_destroy", "sf_superpose", "sf_superpose_noalloc",
           "sf_device_count",
           "sf_last_error")
_VOID = ("sf_destroy_scene", "sf_batch_destroy", "sf_last_error")


class SceneDesc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("obstacle", ctypes.c_void_p), ("exit", ctypes.c_void_p),
                ("n_peds", ctypes.c_int32), ("pos", ctypes.c_void_p),
                ("radius", ctypes.c_int32), ("k", ctypes.c_double), ("alpha", ctypes.c_double),
                ("k_obs", ctypes.c_double), ("alpha_obs", ctypes.c_double),
                ("radius_obs", ctypes.c_int32), ("w_dest", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("start_step", ctypes.c_int64),
                ("periodic", ctypes.c_int32), ("heading", ctypes.c_void_p),
                ("w_heading", ctypes.c_double), ("walk_period", ctypes.c_void_p),
                ("body_w", ctypes.c_int32), ("body_h", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("live", ctypes.c_int64), ("evacuated", ctypes.c_int64),
                ("ped_steps", ctypes.c_int64), ("movers", ctypes.c_int64),
                ("moved", ctypes.c_int64), ("tied", ctypes.c_int64),
                ("max_claimants", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class GroupTiling(ctypes.Structure):
    """sf_group_tiling: field tile shape and schedule of one batch group."""
    _fields_ = [("tw", ctypes.c_int32), ("hl", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("nw", ctypes.c_int32), ("list_cap", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("items_per_block", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


MAX_GROUPS = 4  # SF_MAX_GROUPS


class Tiling(ctypes.Structure):
    """sf_batch_tiling: split of a batch into groups by radius and each
    group's tiling (zero fields = library defaults)."""
    _fields_ = [("groups", ctypes.c_int32), ("split_radius", ctypes.c_int32 * (MAX_GROUPS - 1)),
                ("group", GroupTiling * MAX_GROUPS)]

    @classmethod
    def from_dict(cls, d: dict) -> "Tiling":
        """{"groups", "split_radius": int or list, "group": [dict, ...]} or a
        flat dict of group fields applied to every group."""
        t = cls()
        group_keys = {k for k, _ in GroupTiling._fields_}
        flat = {k: v for k, v in d.items() if k in group_keys}
        per_group = list(d.get("group", []))
        if len(per_group) > MAX_GROUPS:
            raise ValueError(f"at most {MAX_GROUPS} groups")
        for gi in range(MAX_GROUPS):
            g = dict(flat)
            if gi < len(per_group):
                g.update(per_group[gi])
            for k, v in g.items():
                setattr(t.group[gi], k, int(v))
        t.groups = int(d.get("groups", 0))
        split = d.get("split_radius", 0)
        split = [split] if isinstance(split, int) else list(split)
        if len(split) > MAX_GROUPS - 1:
            raise ValueError(f"at most {MAX_GROUPS - 1} split radii")
        for gi, r in enumerate(split):
            t.split_radius[gi] = int(r)
        return t

    def as_dict(self):
        n = max(1, int(self.groups))
        return {"groups": int(self.groups),
                "split_radius": [int(r) for r in self.split_radius][: max(0, n - 1)],
                "group": [self.group[gi].as_dict() for gi in range(n)]}


class SfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsf error {code}: {msg}")
        self.code = code


_lib = None


def _hip_runtimes():
    """Distinct HIP runtime files mapped into this process (Linux)."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({line.split()[-1] for line in f if "libamdhip64" in line})
    except OSError:
        return []


def load():
    """Load libsf.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime.  Imported first, it is the one the
    # library binds to; loaded the other way round, the process maps two HIP
    # (and HSA) runtimes and whichever starts second finds no device.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError("two HIP runtimes are loaded in this process "
                           f"({', '.join(runtimes)}): import torch before anything "
                           "that links the system HIP runtime")
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.sf_create_scene.argtypes = [ctypes.POINTER(SceneDesc), P, ctypes.POINTER(P)]
    lib.sf_step.argtypes = [P, i32]
    lib.sf_field.argtypes = [P, P, ctypes.c_int]
    lib.sf_positions.argtypes = [P, P, P, ctypes.c_int]
    lib.sf_last_moves.argtypes = [P, P, P, ctypes.c_int]
    lib.sf_static_field.argtypes = [P, P, P, ctypes.c_int]
    lib.sf_set_state.argtypes = [P, P, i64]
    lib.sf_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.sf_sync.argtypes = [P]
    lib.sf_set_timing.argtypes = [P, ctypes.c_int]
    lib.sf_kernel_time.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(i64)]
    lib.sf_set_field_update.argtypes = [P, i32]
    lib.sf_refresh_field.argtypes = [P, i32]
    lib.sf_set_field_sect.argtypes = [P, i32, i32]
    lib.sf_sect_image.argtypes = [P, P, ctypes.c_int]
    lib.sf_destroy_scene.argtypes = [P]
    lib.sf_destroy_scene.restype = None
    lib.sf_batch_create.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(Tiling), P,
                                    ctypes.POINTER(P)]
    lib.sf_batch_tune.argtypes = [P, i32, ctypes.POINTER(Tiling)]
    lib.sf_batch_get_tiling.argtypes = [P, ctypes.POINTER(Tiling)]
    lib.sf_batch_step.argtypes = [P, i32]
    lib.sf_batch_refresh_field.argtypes = [P, i32]
    lib.sf_batch_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.sf_batch_sync.argtypes = [P]
    lib.sf_batch_destroy.argtypes = [P]
    lib.sf_batch_destroy.restype = None
    lib.sf_superpose.argtypes = [i32, i32, i32, i32, ctypes.c_double, ctypes.c_double, P, P, i32,
                                 P, P]
    lib.sf_superpose_noalloc.argtypes = lib.sf_superpose.argtypes
    lib.sf_last_error.restype = ctypes.c_char_p
    lib.sf_last_error.argtypes = []
    lib.sf_device_count.argtypes = []
    for name in EXPORTS:
        if name not in _VOID:
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def device_count() -> int:
    """HIP devices the library sees (0 without one)."""
    return int(load().sf_device_count())


def _device_tensor(t, dtype, numel: int, what: str):
    """Pointer of a contiguous CUDA tensor of `dtype` with at least `numel` elements."""
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{what} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{what} must be a contiguous {dtype} tensor of at least {numel} "
                         f"elements (got {t.dtype}, {tuple(t.shape)}, contiguous="
                         f"{t.is_contiguous()})")
    return ctypes.c_void_p(t.data_ptr())


def superpose(S, pos, width: int, height: int, radius: int, k: float = 1.0,
              alpha: float = -0.5, periodic: bool = False, out=None, stream=None,
              noalloc: bool = False):
    """sf_superpose: P = fl32(S + sum of the strengths of the sources at `pos`)
    for device tensors S (float64, width*height) and pos (int32; entries
    outside the grid are skipped).  Returns `out` (float32, width*height, made
    on S's device when None).  Enqueued on `stream` (default: torch's current
    stream of S's device); does not block.  noalloc: sf_superpose_noalloc (no
    device allocation; scratch in a static device array shared by every call on
    the device)."""
    import torch

    n_su = width * height
    if out is None:
        out = torch.empty(n_su, dtype=torch.float32, device=S.device)
    s_ptr = _device_tensor(S, torch.float64, n_su, "S")
    p_ptr = _device_tensor(out, torch.float32, n_su, "out")
    n = int(pos.numel())
    pos_ptr = _device_tensor(pos, torch.int32, n, "pos") if n else None
    for t in (pos, out):
        if t.device != S.device:
            raise ValueError("S, pos and out must be on one device")
    with torch.cuda.device(S.device):
        st = stream if stream is not None else torch.cuda.current_stream(S.device)
        fn = load().sf_superpose_noalloc if noalloc else load().sf_superpose
        _check(fn(width, height, int(bool(periodic)), radius, float(k), float(alpha), s_ptr,
                  pos_ptr, n, p_ptr, ctypes.c_void_p(st.cuda_stream)))
    return out


def _check(rc: int):
    if rc != SF_OK:
        raise SfError(rc, load().sf_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_desc(scene, start_step: Optional[int] = None):
    """Descriptor plus the numpy arrays it points to (keep both alive)."""
    ob = np.ascontiguousarray(scene.obstacle, dtype=np.uint8)
    ex = np.ascontiguousarray(scene.exit, dtype=np.uint8)
    pos = np.ascontiguousarray(scene.pos, dtype=np.int32)
    per_ped = []
    for name in ("heading", "walk_period"):
        a = getattr(scene, name, None)
        if a is not None:
            a = np.ascontiguousarray(a, dtype=np.uint8)
            if a.shape != pos.shape:
                raise ValueError(f"{name} has {a.shape[0]} entries for {pos.shape[0]} pedestrians")
        per_ped.append(a)
    hd, wk = per_ped
    d = SceneDesc(width=int(scene.width), height=int(scene.height), obstacle=_ptr(ob).value,
                  exit=_ptr(ex).value, n_peds=int(pos.shape[0]),
                  pos=_ptr(pos).value if pos.size else None, radius=int(scene.radius),
                  k=float(scene.k), alpha=float(scene.alpha), k_obs=float(scene.k_obs),
                  alpha_obs=float(scene.alpha_obs), radius_obs=int(scene.radius_obs),
                  w_dest=float(scene.w_dest), seed=int(scene.seed) & (2**64 - 1),
                  start_step=int(scene.start_step if start_step is None else start_step),
                  periodic=int(bool(getattr(scene, "periodic", False))),
                  heading=_ptr(hd).value if hd is not None and hd.size else None,
                  w_heading=float(getattr(scene, "w_heading", 1.0)),
                  walk_period=_ptr(wk).value if wk is not None and wk.size else None,
                  body_w=int(getattr(scene, "body_w", 1)), body_h=int(getattr(scene, "body_h", 1)))
    return d, (ob, ex, pos, hd, wk)


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream) or None
    return int(stream) or None


class GpuScene:
    """One scene resident on the current HIP device."""

    def __init__(self, scene, stream=None):
        lib = load()
        self.width, self.height = int(scene.width), int(scene.height)
        self.n_peds = int(np.asarray(scene.pos).shape[0])
        desc, keep = make_desc(scene)
        h = ctypes.c_void_p()
        _check(lib.sf_create_scene(ctypes.byref(desc), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        del keep
        import torch

        # the library creates the scene on the device current at the call
        self.device = torch.cuda.current_device()

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().sf_destroy_scene(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n: int = 1):
        _check(load().sf_step(self._h, int(n)))

    def sync(self):
        _check(load().sf_sync(self._h))

    def field(self, out=None):
        """Host copy (numpy float32 [H*W]) or, with a torch tensor `out`, a
        device-to-device copy enqueued on the scene's stream.  `out` must be a
        contiguous float32 tensor of at least H*W elements on the scene's
        device; a reader on another stream must wait for the scene's stream
        (for instance with an event) before it uses `out`."""
        if out is not None:
            import torch

            n = self.width * self.height
            if not isinstance(out, torch.Tensor):
                raise TypeError("out must be a torch tensor")
            if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() < n:
                raise ValueError(f"out must be a contiguous float32 tensor of at least {n} "
                                 f"elements (got {out.dtype}, {tuple(out.shape)}, "
                                 f"contiguous={out.is_contiguous()})")
            if out.device.type != "cuda" or out.device.index != self.device:
                raise ValueError(f"out is on {out.device}, the scene on cuda:{self.device}")
            _check(load().sf_field(self._h, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        a = np.empty(self.width * self.height, dtype=np.float32)
        _check(load().sf_field(self._h, _ptr(a), 0))
        return a

    def static_field(self):
        """(S float64 [H*W] = w_dest*D + O, +inf on obstacles; D int32 [H*W])."""
        S = np.empty(self.width * self.height, dtype=np.float64)
        D = np.empty(self.width * self.height, dtype=np.int32)
        _check(load().sf_static_field(self._h, _ptr(S), _ptr(D), 0))
        return S, D

    def positions(self):
        pos = np.empty(self.n_peds, dtype=np.int32)
        _check(load().sf_positions(self._h, _ptr(pos), None, 0))
        return pos

    def last_moves(self):
        t = np.empty(self.n_peds, dtype=np.int32)
        f = np.empty(self.n_peds, dtype=np.uint8)
        _check(load().sf_last_moves(self._h, _ptr(t), _ptr(f), 0))
        return t, f

    def set_state(self, pos, step: int):
        p = np.ascontiguousarray(pos, dtype=np.int32)
        _check(load().sf_set_state(self._h, _ptr(p) if p.size else None, int(step)))

    def stats(self) -> dict:
        st = Stats()
        _check(load().sf_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def set_field_update(self, refresh_ticks: int):
        """0/1: full superposition every tick; K >= 2: incremental update with
        a full superposition every K ticks."""
        _check(load().sf_set_field_update(self._h, int(refresh_ticks)))

    def set_field_sect(self, K: int, image: bool = False):
        """The paper's sect path with K in {2, 4, 8, 16} FP32 slots (0: the
        exact gather); image: keep the 8 sect planes."""
        _check(load().sf_set_field_sect(self._h, int(K), 1 if image else 0))

    def sect_image(self):
        """The 8 sect planes (float32 [8, H*W]) of the sect path."""
        a = np.empty((8, self.width * self.height), dtype=np.float32)
        _check(load().sf_sect_image(self._h, _ptr(a), 0))
        return a

    def refresh_field(self, n_times: int = 1):
        """Superpose the field of the current positions again, n_times times
        (enqueued on the scene stream)."""
        _check(load().sf_refresh_field(self._h, int(n_times)))

    def set_timing(self, on: bool):
        _check(load().sf_set_timing(self._h, 1 if on else 0))

    def kernel_time(self, kernel: int):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(load().sf_kernel_time(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)


class Batch:
    """Scenes advanced together: one decide, commit and field launch per tick
    for all members, replayed from captured HIP graphs (sf_batch_*)."""

    def __init__(self, scenes, tiling: Optional[dict] = None, stream=None):
        lib = load()
        self.scenes = list(scenes)
        arr = (ctypes.c_void_p * len(self.scenes))(*[s.handle.value for s in self.scenes])
        t = Tiling.from_dict(tiling) if tiling else None
        h = ctypes.c_void_p()
        _check(lib.sf_batch_create(arr, len(self.scenes), ctypes.byref(t) if t else None,
                                   _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().sf_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n: int = 1):
        _check(load().sf_batch_step(self._h, int(n)))

    def refresh_field(self, n: int = 1):
        """n field passes over every member (no tick; the fields keep their bits)."""
        _check(load().sf_batch_refresh_field(self._h, int(n)))

    def sync(self):
        _check(load().sf_batch_sync(self._h))

    def stats(self) -> list:
        """Running totals of every member (one launch, one copy)."""
        arr = (Stats * len(self.scenes))()
        _check(load().sf_batch_stats(self._h, arr))
        return [a.as_dict() for a in arr]

    def tune(self, reps: int = 3) -> dict:
        t = Tiling()
        _check(load().sf_batch_tune(self._h, int(reps), ctypes.byref(t)))
        return t.as_dict()

    def tiling(self) -> dict:
        t = Tiling()
        _check(load().sf_batch_get_tiling(self._h, ctypes.byref(t)))
        return t.as_dict()


def create_error(scene) -> tuple:
    """(code, message) of sf_create_scene for a descriptor; destroys the scene
    if creation succeeded.  Used to exercise validation."""
    lib = load()
    desc, keep = make_desc(scene)
    h = ctypes.c_void_p()
    rc = lib.sf_create_scene(ctypes.byref(desc), None, ctypes.byref(h))
    msg = lib.sf_last_error().decode()
    if rc == SF_OK:
        lib.sf_destroy_scene(h)
    del keep
    return rc, msg
