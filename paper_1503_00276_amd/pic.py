"""Python binding of libpic.so: the C ABI of include/pic.h, argument marshalling only.

Every step of the PIC loop runs in the HIP library; this module converts numpy
arrays (or torch tensors, passed as device pointers) into the plain pointers
and sizes the C functions take.  Importing it without a built library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK = 0
PIC_E_INVALID = -1
PIC_E_NOMEM = -2
PIC_E_HIP = -3
PIC_E_STATE = -4
PIC_E_RANGE = -5
PIC_E_UNSUPPORTED = -6

PIC_ACC_FP32 = 0
PIC_ACC_COMPENSATED = 1
PIC_ACC_FIXED64 = 2

PIC_DEPOSIT_ISIS = 0
PIC_DEPOSIT_TRISTAN = 1

PIC_GEOM_CARTESIAN = 0
PIC_GEOM_RZ = 1

PIC_DEVICE_PTRS = 1

PIC_DIAG_ENERGY = 0
PIC_DIAG_MOMENTUM = 1
PIC_DIAG_RHO = 2
PIC_DIAG_GAUSS_RESIDUAL = 3
PIC_DIAG_GAUSS_NORM = 4
PIC_DIAG_RHO_SNAPSHOT = 5
PIC_DIAG_CHARGE_RESIDUAL = 6
PIC_DIAG_EXPORT_STATE = 7
PIC_DIAG_EXPORT_FIELDS = 8
PIC_DIAG_EXPORT_CURRENT = 9
PIC_DIAG_COUNTS = 10
PIC_DIAG_KERNEL_TIMES = 11

EXPORTED = [
    "pic_create", "pic_destroy", "pic_load_particles", "pic_load_fields", "pic_step", "pic_sync",
    "pic_diag", "pic_diag_noalloc", "pic_get_info", "pic_last_error", "pic_profile", "pic_batch_profile", "pic_batch_create", "pic_batch_destroy",
    "pic_batch_load_particles", "pic_batch_load_fields", "pic_batch_step", "pic_batch_diag",
    "pic_batch_sync", "pic_batch_last_error", "pic_autotune", "pic_batch_autotune", "pic_batch_get_info",
]

PIC_TUNE_TILE = 1
PIC_TUNE_SORT = 2
PIC_TUNE_CHUNK = 4


class pic_config(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("nx", C.c_int32 * 3),
        ("dx", C.c_double * 3),
        ("xmin", C.c_double * 3),
        ("dt", C.c_double),
        ("shape_order", C.c_int32),
        ("e0", C.c_double * 3),
        ("b0", C.c_double * 3),
        ("ion_density", C.c_double),
        ("capacity", C.c_int64),
        ("tile", C.c_int32 * 3),
        ("sort_interval", C.c_int32),
        ("chunk", C.c_int32),
        ("accumulator", C.c_int32),
        ("deposit", C.c_int32),
        ("smooth_level", C.c_int32 * 3),
        ("smooth_weights", C.c_double * 72),
        ("move_window", C.c_int32),
        ("inject_ppc", C.c_int32 * 3),
        ("inject_w", C.c_double),
        ("geometry", C.c_int32),
        ("inject_uth", C.c_double),
        ("inject_seed", C.c_uint64),
    ]


class pic_info(C.Structure):
    _fields_ = [
        ("tile", C.c_int32 * 3),
        ("sort_interval", C.c_int32),
        ("chunk", C.c_int32),
        ("slack", C.c_int32),
        ("accumulator", C.c_int32),
        ("nspecies", C.c_int32),
        ("nparticles", C.c_int64 * 8),
        ("rqm", C.c_double * 8),
        ("lds_bytes", C.c_int64),
    ]


class pic_tune(C.Structure):
    _fields_ = [
        ("trial_steps", C.c_int32),
        ("what", C.c_int32),
        ("candidates", C.c_int32),
        ("particles_per_tile", C.c_int32),
        ("sort_interval", C.c_int32),
        ("chunk", C.c_int32),
        ("ms_before", C.c_double),
        ("ms_after", C.c_double),
    ]


def _tune_dict(t: pic_tune) -> dict:
    return {k: getattr(t, k) for k, _ in pic_tune._fields_}


_lib = None


def lib():
    """Load libpic.so; raise if it was not built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1503_00276_amd.build`")
        # torch first when it is installed: its HIP runtime (the same soname
        # the library needs) is then the only one in the process; loading the
        # library first would bring in the system's copy beside torch's, and
        # torch's device initialisation then fails
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, V, I64, I32, U32, D, SZ = (C.POINTER(C.c_double), C.c_void_p, C.c_int64, C.c_int32,
                                      C.c_uint32, C.c_double, C.c_size_t)
        L.pic_create.argtypes = [C.POINTER(pic_config), V, C.POINTER(V)]
        L.pic_destroy.argtypes = [V]
        L.pic_load_particles.argtypes = [V, I32, D, I64, V, V, V, U32]
        L.pic_load_fields.argtypes = [V, V, V, U32]
        L.pic_step.argtypes = [V, I64]
        L.pic_sync.argtypes = [V]
        L.pic_diag.argtypes = [V, C.c_int, V, SZ, C.POINTER(SZ)]
        L.pic_diag_noalloc.argtypes = [V, C.c_int, V, SZ, C.POINTER(SZ)]
        L.pic_get_info.argtypes = [V, C.POINTER(pic_info)]
        L.pic_profile.argtypes = [V, I32]
        L.pic_batch_profile.argtypes = [V, I32]
        L.pic_last_error.argtypes = [V]
        L.pic_last_error.restype = C.c_char_p
        L.pic_batch_create.argtypes = [C.POINTER(pic_config), I32, V, C.POINTER(V)]
        L.pic_batch_destroy.argtypes = [V]
        L.pic_batch_load_particles.argtypes = [V, I32, I32, D, I64, V, V, V, U32]
        L.pic_batch_load_fields.argtypes = [V, I32, V, V, U32]
        L.pic_batch_step.argtypes = [V, I64]
        L.pic_batch_diag.argtypes = [V, I32, C.c_int, V, SZ, C.POINTER(SZ)]
        L.pic_batch_sync.argtypes = [V]
        L.pic_batch_last_error.argtypes = [V]
        L.pic_batch_last_error.restype = C.c_char_p
        L.pic_autotune.argtypes = [V, C.POINTER(pic_tune)]
        L.pic_batch_autotune.argtypes = [V, C.POINTER(pic_tune)]
        L.pic_batch_get_info.argtypes = [V, I32, C.POINTER(pic_info)]
        for name in EXPORTED:
            fn = getattr(L, name)
            if fn.restype is None or fn.restype is C.c_int:
                fn.restype = C.c_int
        _lib = L
    return _lib


class PicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pic error {code}: {msg}")
        self.code = code


@dataclass
class Config:
    """Python view of pic_config (see include/pic.h)."""

    ndim: int
    nx: Sequence[int]
    dx: Sequence[float]
    dt: float
    shape_order: int = 1
    xmin: Sequence[float] = (0.0, 0.0, 0.0)
    e0: Sequence[float] = (0.0, 0.0, 0.0)
    b0: Sequence[float] = (0.0, 0.0, 0.0)
    ion_density: float = 0.0
    capacity: int = 0
    tile: Sequence[int] = (0, 0, 0)
    sort_interval: int = 0
    chunk: int = 0
    accumulator: int = PIC_ACC_FP32
    deposit: int = PIC_DEPOSIT_ISIS
    smooth: Sequence = ()  # per axis: a list of (a, b, c) weights, one per smoothing pass
    move_window: int = 0   # 1: the window moves along +x1 at c
    inject_ppc: Sequence[int] = (1, 1, 1)  # moving window: injected particles per cell per axis
    inject_w: float = 0.0  # moving window: weight of an injected particle
    geometry: int = 0      # PIC_GEOM_CARTESIAN, or PIC_GEOM_RZ (x1 = z, x2 = r)
    inject_uth: float = 0.0  # moving window: thermal spread of the injected momenta (0: cold)
    inject_seed: int = 0     # moving window: seed of the injected momenta's generator

    def c(self) -> pic_config:
        c = pic_config()
        c.ndim = self.ndim
        for i in range(3):
            c.nx[i] = int(self.nx[i]) if i < len(self.nx) else 1
            c.dx[i] = float(self.dx[i]) if i < len(self.dx) else 1.0
            c.xmin[i] = float(self.xmin[i]) if i < len(self.xmin) else 0.0
            c.e0[i] = float(self.e0[i])
            c.b0[i] = float(self.b0[i])
            c.tile[i] = int(self.tile[i]) if i < len(self.tile) else 0
        c.dt = float(self.dt)
        c.shape_order = int(self.shape_order)
        c.ion_density = float(self.ion_density)
        c.capacity = int(self.capacity)
        c.sort_interval = int(self.sort_interval)
        c.chunk = int(self.chunk)
        c.accumulator = int(self.accumulator)
        c.deposit = int(self.deposit)
        c.move_window = int(self.move_window)
        for i in range(3):
            c.inject_ppc[i] = int(self.inject_ppc[i]) if i < len(self.inject_ppc) else 1
        c.inject_w = float(self.inject_w)
        c.geometry = int(self.geometry)
        c.inject_uth = float(self.inject_uth)
        c.inject_seed = int(self.inject_seed) & 0xFFFFFFFFFFFFFFFF
        for ax, passes in enumerate(self.smooth):
            c.smooth_level[ax] = len(passes)
            for p, wts in enumerate(passes[:8]):
                for k in range(3):
                    c.smooth_weights[(ax * 8 + p) * 3 + k] = float(wts[k])
        return c

    @property
    def ncell(self) -> int:
        n = 1
        for i in range(self.ndim):
            n *= int(self.nx[i])
        return n


def _ptr(a, want_device: bool = False):
    """(pointer, flags, keepalive) for a numpy array or a torch tensor."""
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        import torch

        t = a.detach().to(torch.float64).contiguous()
        if t.is_cuda:
            return C.c_void_p(t.data_ptr()), PIC_DEVICE_PTRS, t
        arr = t.numpy()
    else:
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return C.c_void_p(arr.ctypes.data), 0, arr


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


class _Base:
    _h: C.c_void_p

    def _check(self, rc: int):
        if rc != PIC_OK:
            raise PicError(rc, self.last_error())

    def last_error(self) -> str:
        raise NotImplementedError


class Pic(_Base):
    """One simulation instance (a pic_ctx)."""

    def __init__(self, cfg: Config, stream=None):
        self.cfg = cfg
        self._L = lib()
        self._h = C.c_void_p()
        self._cc = cfg.c()
        rc = self._L.pic_create(C.byref(self._cc), _stream_handle(stream), C.byref(self._h))
        if rc != PIC_OK:
            raise PicError(rc, "pic_create failed (see stderr)")

    def last_error(self) -> str:
        return self._L.pic_last_error(self._h).decode()

    def close(self):
        if self._h:
            self._L.pic_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_particles(self, x, u, w, rqm: float = -1.0, species: int = 0):
        n = len(w)
        px, fx, kx = _ptr(x)
        pu, fu, ku = _ptr(u)
        pw, fw, kw = _ptr(w)
        if len({fx, fu, fw}) != 1:
            raise ValueError("x, u, w must all be host or all be device data")
        self._check(self._L.pic_load_particles(self._h, species, float(rqm), n, px, pu, pw, fx))

    def load_fields(self, E, B):
        pe, fe, ke = _ptr(E)
        pb, fb, kb = _ptr(B)
        if fe != fb:
            raise ValueError("E and B must both be host or both be device data")
        self._check(self._L.pic_load_fields(self._h, pe, pb, fe))

    def step(self, n: int = 1):
        self._check(self._L.pic_step(self._h, int(n)))

    def sync(self):
        self._check(self._L.pic_sync(self._h))

    def diag(self, kind: int, count: int) -> np.ndarray:
        out = np.zeros(max(count, 1), dtype=np.float64)
        wr = C.c_size_t(0)
        self._check(self._L.pic_diag(self._h, kind, C.c_void_p(out.ctypes.data), out.nbytes, C.byref(wr)))
        return out[:count]

    def diag_noalloc(self, kind: int, out) -> int:
        """pic_diag_noalloc into a caller-owned device tensor (float64, at
        least ncell elements); returns the bytes written."""
        wr = C.c_size_t(0)
        nbytes = out.numel() * out.element_size()
        self._check(self._L.pic_diag_noalloc(self._h, kind, C.c_void_p(out.data_ptr()), nbytes, C.byref(wr)))
        return wr.value

    def info(self) -> pic_info:
        i = pic_info()
        self._check(self._L.pic_get_info(self._h, C.byref(i)))
        return i

    # convenience views ----------------------------------------------------
    def nparticles(self) -> int:
        return int(sum(self.info().nparticles))

    def state(self):
        """(x [n, ndim], u [n, 3], w [n]) of all species in load order."""
        if self.cfg.move_window or self.cfg.geometry == PIC_GEOM_RZ:
            self.sync()  # the window removes and injects particles, the r-z wall removes some
        n = self.nparticles()
        d = self.cfg.ndim
        a = self.diag(PIC_DIAG_EXPORT_STATE, n * (d + 4)).reshape(n, d + 4)
        return a[:, :d].copy(), a[:, d:d + 3].copy(), a[:, d + 3].copy()

    def fields(self):
        a = self.diag(PIC_DIAG_EXPORT_FIELDS, 6 * self.cfg.ncell).reshape(6, self.cfg.ncell)
        return a[:3].copy(), a[3:].copy()

    def current(self):
        return self.diag(PIC_DIAG_EXPORT_CURRENT, 3 * self.cfg.ncell).reshape(3, self.cfg.ncell)

    def rho(self):
        return self.diag(PIC_DIAG_RHO, self.cfg.ncell)

    def gauss_residual(self):
        return self.diag(PIC_DIAG_GAUSS_RESIDUAL, self.cfg.ncell)

    def rho_snapshot(self):
        wr = C.c_size_t(0)
        self._check(self._L.pic_diag(self._h, PIC_DIAG_RHO_SNAPSHOT, None, 0, C.byref(wr)))

    def charge_residual(self):
        return self.diag(PIC_DIAG_CHARGE_RESIDUAL, self.cfg.ncell)

    def energy(self):
        return self.diag(PIC_DIAG_ENERGY, 4)

    def momentum(self):
        return self.diag(PIC_DIAG_MOMENTUM, 3)

    def counts(self):
        return self.diag(PIC_DIAG_COUNTS, 4)

    def profile(self, enable: int):
        self._check(self._L.pic_profile(self._h, int(enable)))

    def autotune(self, trial_steps: int = 20, what: int = 0) -> dict:
        """Measured search of tile, sort interval and chunk (pic_autotune)."""
        t = pic_tune(trial_steps=int(trial_steps), what=int(what))
        self._check(self._L.pic_autotune(self._h, C.byref(t)))
        return _tune_dict(t)

    def kernel_times(self):
        """{family: (ms, launches)} for 'particle', 'field', 'rebin'."""
        a = self.diag(PIC_DIAG_KERNEL_TIMES, 6)
        return {"particle": (a[0], a[1]), "field": (a[2], a[3]), "rebin": (a[4], a[5])}


class PicBatch(_Base):
    """Many independent instances advanced together (a pic_batch)."""

    def __init__(self, cfgs: Sequence[Config], stream=None):
        self.cfgs = list(cfgs)
        self._L = lib()
        arr = (pic_config * len(self.cfgs))(*[c.c() for c in self.cfgs])
        self._arr = arr
        self._h = C.c_void_p()
        rc = self._L.pic_batch_create(arr, len(self.cfgs), _stream_handle(stream), C.byref(self._h))
        if rc != PIC_OK:
            raise PicError(rc, "pic_batch_create failed (see stderr)")
        self._np = [0] * len(self.cfgs)

    def last_error(self) -> str:
        return self._L.pic_batch_last_error(self._h).decode()

    def close(self):
        if self._h:
            self._L.pic_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_particles(self, inst: int, x, u, w, rqm: float = -1.0, species: int = 0):
        n = len(w)
        px, fx, kx = _ptr(x)
        pu, fu, ku = _ptr(u)
        pw, fw, kw = _ptr(w)
        self._check(self._L.pic_batch_load_particles(self._h, inst, species, float(rqm), n, px, pu, pw, fx))
        self._np[inst] += n

    def load_fields(self, inst: int, E, B):
        pe, fe, ke = _ptr(E)
        pb, fb, kb = _ptr(B)
        self._check(self._L.pic_batch_load_fields(self._h, inst, pe, pb, fe))

    def step(self, n: int = 1):
        self._check(self._L.pic_batch_step(self._h, int(n)))

    def sync(self):
        self._check(self._L.pic_batch_sync(self._h))

    def diag(self, inst: int, kind: int, count: int) -> np.ndarray:
        out = np.zeros(max(count, 1), dtype=np.float64)
        wr = C.c_size_t(0)
        self._check(self._L.pic_batch_diag(self._h, inst, kind, C.c_void_p(out.ctypes.data), out.nbytes,
                                           C.byref(wr)))
        return out[:count]

    def state(self, inst: int):
        cfg = self.cfgs[inst]
        if cfg.move_window or cfg.geometry == PIC_GEOM_RZ:
            self.sync()  # the window or the r-z wall changed the count
            n = int(sum(self.info(inst).nparticles))
        else:
            n = self._np[inst]
        d = cfg.ndim
        a = self.diag(inst, PIC_DIAG_EXPORT_STATE, n * (d + 4)).reshape(n, d + 4)
        return a[:, :d].copy(), a[:, d:d + 3].copy(), a[:, d + 3].copy()

    def profile(self, enable: int):
        self._check(self._L.pic_batch_profile(self._h, int(enable)))

    def autotune(self, trial_steps: int = 20, what: int = 0) -> dict:
        t = pic_tune(trial_steps=int(trial_steps), what=int(what))
        self._check(self._L.pic_batch_autotune(self._h, C.byref(t)))
        return _tune_dict(t)

    def info(self, inst: int) -> pic_info:
        i = pic_info()
        self._check(self._L.pic_batch_get_info(self._h, inst, C.byref(i)))
        return i

    def kernel_times(self):
        a = self.diag(0, PIC_DIAG_KERNEL_TIMES, 6)
        return {"particle": (a[0], a[1]), "field": (a[2], a[3]), "rebin": (a[4], a[5])}

    def counts(self, inst: int):
        return self.diag(inst, PIC_DIAG_COUNTS, 4)

    def fields(self, inst: int):
        nc = self.cfgs[inst].ncell
        a = self.diag(inst, PIC_DIAG_EXPORT_FIELDS, 6 * nc).reshape(6, nc)
        return a[:3].copy(), a[3:].copy()

    def current(self, inst: int):
        nc = self.cfgs[inst].ncell
        return self.diag(inst, PIC_DIAG_EXPORT_CURRENT, 3 * nc).reshape(3, nc)
