"""Python binding of the cmlb C ABI (include/cmlb.h): argument marshalling only.

Every step of the update runs in the HIP library ``libcmlb.so``; this module
converts numpy arrays and torch streams/tensors to plain pointers and status
codes to exceptions.  There is no fallback: if the library is missing the
import of :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmlb.so")

LATTICES = {"D2Q9": 0, "D3Q27": 1, "D2Q37": 2, "E9B": 3, "E9C": 4, "E9D": 5, "E7A": 6, "E7B": 7, "E7C": 8,
            "E7D": 9}
LATTICES["E9A"] = LATTICES["D2Q37"]   # the ninth-degree 37-velocity rule on |e|^2 <= 10
STORAGES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
STORAGE_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}
MODELS = {"cm": 0, "raw_mrt": 1, "reg_bgk": 2}

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSTABLE = 0, -1, -2, -3, -4, -5
MAX_BATCH = 16   # CMLB_MAX_BATCH
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ESTATE: "ESTATE", EUNSTABLE: "EUNSTABLE"}


class CmlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("storage", ctypes.c_int32), ("model", ctypes.c_int32),
                ("thermal", ctypes.c_int32), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("rho0", ctypes.c_double), ("theta0", ctypes.c_double),
                ("tau", ctypes.c_double * 8), ("scale", ctypes.c_double * 37),
                ("device", ctypes.c_int32), ("reserved", ctypes.c_int32), ("hip_stream", ctypes.c_void_p)]


class Globals(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3), ("energy", ctypes.c_double),
                ("kinetic_energy", ctypes.c_double), ("enstrophy", ctypes.c_double),
                ("n_nonfinite", ctypes.c_int64), ("rho_min", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("u_max", ctypes.c_double)]


class Batch(ctypes.Structure):
    _fields_ = [("state", ctypes.c_void_p), ("target", ctypes.c_void_p), ("n_pairs", ctypes.c_int64)]


CLOSURE_NPARAM = 2084

_lib = None


def lib():
    """Load libcmlb.so (built by ``python -m paper_1808_04406_amd.build``)."""
    global _lib
    if _lib is None:
        try:
            # libcmlb needs libamdhip64.so.7; if torch is present its copy is
            # loaded first so that one HIP runtime serves both
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1808_04406_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, c_int, c_i64, vp = ctypes.POINTER, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        dp = P(ctypes.c_double)
        L.cmlb_lattice_info.argtypes = [c_int, P(c_int), P(c_int), P(c_int), dp, dp]
        L.cmlb_create.argtypes = [P(Params), P(vp)]
        L.cmlb_create_external.argtypes = [P(Params), vp, vp, P(vp)]
        L.cmlb_create_error.restype = ctypes.c_char_p
        L.cmlb_destroy.argtypes = [vp]
        L.cmlb_destroy.restype = None
        L.cmlb_last_error.argtypes = [vp]
        L.cmlb_last_error.restype = ctypes.c_char_p
        L.cmlb_set_tau.argtypes = [vp, dp, c_int]
        L.cmlb_init_fields.argtypes = [vp, dp, dp, dp]
        L.cmlb_init_fields_device.argtypes = [vp, vp, vp, vp]
        L.cmlb_step.argtypes = [vp, c_i64]
        L.cmlb_set_step_fusion.argtypes = [vp, c_int]
        L.cmlb_set_graph_steps.argtypes = [vp, c_int]
        L.cmlb_step_batch.argtypes = [P(vp), c_int, c_i64]
        L.cmlb_copy_bandwidth.argtypes = [c_int, ctypes.c_uint64, c_int, c_int, dp]
        L.cmlb_state_bytes.argtypes = [P(Params), P(ctypes.c_size_t)]
        L.cmlb_state_layout.argtypes = [P(Params), P(ctypes.c_uint64), P(ctypes.c_uint64)]
        L.cmlb_sync.argtypes = [vp]
        L.cmlb_get_moments.argtypes = [vp, dp, dp, dp]
        L.cmlb_get_moments_device.argtypes = [vp, vp, vp, vp]
        L.cmlb_get_populations.argtypes = [vp, dp]
        L.cmlb_set_populations.argtypes = [vp, dp]
        L.cmlb_reduce.argtypes = [vp, P(Globals)]
        L.cmlb_reduce_noalloc.argtypes = [vp, P(Globals)]
        L.cmlb_state.argtypes = [vp, P(vp), P(ctypes.c_size_t), P(vp)]
        L.cmlb_step_count.argtypes = [vp]
        L.cmlb_step_count.restype = c_i64
        L.cmlb_set_step_count.argtypes = [vp, c_i64]
        L.cmlb_get_tau.argtypes = [vp, dp]
        L.cmlb_get_scale.argtypes = [vp, dp]
        fp = P(ctypes.c_float)
        L.cmlb_store_state_device.argtypes = [vp, vp]
        L.cmlb_load_state_device.argtypes = [vp, vp]
        L.cmlb_load_deviations_device.argtypes = [vp, vp]
        L.cmlb_box_filter.argtypes = [vp, c_int, vp]
        L.cmlb_closure_load.argtypes = [vp, fp, fp]
        L.cmlb_closure_enable.argtypes = [vp, c_int]
        L.cmlb_closure_tie_even.argtypes = [vp, c_int]
        L.cmlb_closure_get.argtypes = [vp, fp]
        L.cmlb_closure_objective.argtypes = [vp, P(Batch), fp, fp]
        L.cmlb_closure_train_step.argtypes = [vp, P(Batch), ctypes.c_float, fp]
        L.cmlb_closure_set_objective.argtypes = [vp, c_int]
        L.cmlb_closure_set_adam.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.cmlb_closure_freeze.argtypes = [vp, c_int]
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice_info(kind: str) -> dict:
    """cmlb_lattice_info: D, Q, e (Q,3), w (Q,), r."""
    D, Q = ctypes.c_int(), ctypes.c_int()
    e = np.zeros(37 * 3, np.int32)
    w = np.zeros(37)
    r = ctypes.c_double()
    rc = lib().cmlb_lattice_info(LATTICES[kind], ctypes.byref(D), ctypes.byref(Q),
                                 e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w), ctypes.byref(r))
    if rc:
        raise CmlbError(rc, "lattice_info failed")
    q = Q.value
    return dict(D=D.value, Q=q, e=e[:3 * q].reshape(q, 3).astype(np.int64), w=w[:q].copy(), r=r.value)


def make_params(lattice, shape, storage="f32", model="cm", thermal=False, rho0=1.0, theta0=1.0,
                tau=None, scale=None, device=0, stream=None) -> Params:
    p = Params()
    p.lattice = LATTICES[lattice]
    p.storage = STORAGES[storage]
    p.model = MODELS[model]
    p.thermal = 1 if thermal else 0
    if len(shape) == 2:
        shape = (1,) + tuple(shape)
    p.nz, p.ny, p.nx = (int(s) for s in shape)
    p.rho0, p.theta0 = rho0, theta0
    for n, t in (tau or {}).items():
        p.tau[n] = t
    if scale is not None:
        for i, s in enumerate(scale):
            p.scale[i] = s
    p.device = device
    p.reserved = 0
    p.hip_stream = _stream_handle(stream)
    return p


def _stream_handle(stream):
    """hipStream_t of a torch stream (or a raw handle).  The legacy default
    stream (handle 0) cannot be named through the C ABI, where NULL asks for
    a library-owned stream that does not order with it; it is refused."""
    if stream is None:
        return None
    h = stream if isinstance(stream, int) else int(stream.cuda_stream)
    if h == 0:
        raise ValueError("pass a non-default stream (e.g. torch.cuda.Stream()); the default stream "
                         "does not order with the library's own stream")
    return h


def state_bytes(lattice, shape, storage="f32", **kw):
    """cmlb_state_bytes: bytes of one population buffer (rows and planes
    padded); the size of each external buffer."""
    p = make_params(lattice, shape, storage, **kw)
    n = ctypes.c_size_t()
    rc = lib().cmlb_state_bytes(ctypes.byref(p), ctypes.byref(n))
    if rc:
        raise CmlbError(rc, lib().cmlb_create_error().decode())
    return n.value


def state_layout(lattice, shape, storage="f32", **kw):
    """cmlb_state_layout: (pitch, plane) in elements; population i of node
    (x, y, z) sits at i * plane + (z * ny + y) * pitch + x."""
    p = make_params(lattice, shape, storage, **kw)
    pitch, plane = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().cmlb_state_layout(ctypes.byref(p), ctypes.byref(pitch), ctypes.byref(plane))
    if rc:
        raise CmlbError(rc, lib().cmlb_create_error().decode())
    return pitch.value, plane.value


def copy_bandwidth(nbytes=4 << 30, planes=27, reps=10, device=0):
    """cmlb_copy_bandwidth: GB/s of a streaming copy of `planes` FP32 planes."""
    g = ctypes.c_double()
    rc = lib().cmlb_copy_bandwidth(int(device), int(nbytes), int(planes), int(reps), ctypes.byref(g))
    if rc:
        raise CmlbError(rc, "copy bandwidth measurement failed")
    return g.value


def step_batch(ctxs, n=1):
    """cmlb_step_batch: n steps of each context, one launch per step for all of
    them (at most MAX_BATCH contexts of one configuration)."""
    ctxs = list(ctxs)
    if not ctxs:
        return
    arr = (ctypes.c_void_p * len(ctxs))(*[c.h for c in ctxs])
    rc = lib().cmlb_step_batch(arr, len(ctxs), int(n))
    if rc:
        raise CmlbError(rc, lib().cmlb_last_error(ctxs[0].h).decode() if ctxs[0].h else "invalid batch")


def _device_ptr(t, what, device, dtype=None, numel=None, min_bytes=None):
    """Device address of a contiguous CUDA tensor on `device`, after checking
    its dtype and size: the kernels trust the sizes the header states, so a
    short or mistyped tensor is refused here rather than read or written past
    its end on the GPU."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous CUDA tensor")
    if t.device.index != device:
        raise ValueError(f"{what}: tensor on cuda:{t.device.index}, context on cuda:{device}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what}: expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {t.numel()}")
    if min_bytes is not None and t.numel() * t.element_size() < min_bytes:
        raise ValueError(f"{what}: expected at least {min_bytes} bytes, got {t.numel() * t.element_size()}")
    return t.data_ptr()


class Context:
    """One simulation context (cmlb_ctx*).  Methods mirror the C entry points."""

    def __init__(self, lattice="D3Q27", shape=(32, 32, 32), storage="f32", model="cm", thermal=False,
                 rho0=1.0, theta0=1.0, tau=None, scale=None, device=0, stream=None, external=None):
        self.lattice, self.storage = lattice, storage
        self.shape = tuple(shape)
        self.info = lattice_info(lattice)
        self.Q, self.D = self.info["Q"], self.info["D"]
        self.nodes = int(np.prod(shape))
        self.params = make_params(lattice, shape, storage, model, thermal, rho0, theta0, tau, scale,
                                  device, stream)
        self._external = external  # keep caller tensors alive
        self._closure = None         # closure inputs (kept for checkpoints)
        h = ctypes.c_void_p()
        if external is None:
            rc = lib().cmlb_create(ctypes.byref(self.params), ctypes.byref(h))
        else:
            # tensors are checked against the state size; plain integers are
            # device addresses the caller vouches for (cmlb_create_external)
            need = state_bytes(lattice, shape, storage)
            fa, fb = (_device_ptr(t, "external buffer", device, min_bytes=need) if hasattr(t, "data_ptr")
                      else int(t) for t in external)
            rc = lib().cmlb_create_external(ctypes.byref(self.params), fa, fb, ctypes.byref(h))
        if rc:
            raise CmlbError(rc, lib().cmlb_create_error().decode())
        self.h = h

    # -- helpers -----------------------------------------------------------
    def _check(self, rc):
        if rc:
            raise CmlbError(rc, lib().cmlb_last_error(self.h).decode())

    def _field(self, a, comps=1):
        a = np.ascontiguousarray(a, np.float64)
        if a.size != comps * self.nodes:
            raise ValueError(f"expected {comps}x{self.nodes} values, got {a.size}")
        return a

    # -- entry points ------------------------------------------------------
    def destroy(self):
        if getattr(self, "h", None):
            lib().cmlb_destroy(self.h)
            self.h = None

    close = destroy

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def set_tau(self, tau_by_order):
        t = np.ascontiguousarray(tau_by_order, np.float64)
        self._check(lib().cmlb_set_tau(self.h, _dp(t), len(t)))

    def init_fields(self, rho, u, theta=None):
        rho = self._field(rho)
        u = self._field(u, self.D)
        th = None if theta is None else self._field(theta)
        self._check(lib().cmlb_init_fields(self.h, _dp(rho), _dp(u), _dp(th)))

    def init_fields_device(self, rho, u, theta=None):
        """Fields as float64 device tensors (torch) of nodes / D*nodes elements."""
        import torch
        dev = self.params.device

        def ptr(t, what, n):
            return None if t is None else _device_ptr(t, what, dev, torch.float64, n)
        self._check(lib().cmlb_init_fields_device(self.h, ptr(rho, "rho", self.nodes), ptr(u, "u", self.D * self.nodes),
                                                  ptr(theta, "theta", self.nodes)))

    def step(self, n=1):
        self._check(lib().cmlb_step(self.h, int(n)))

    def set_graph_steps(self, steps):
        """Replay steps from a HIP graph of `steps` steps (multiple of 4; 0 = direct launches)."""
        self._check(lib().cmlb_set_graph_steps(self.h, int(steps)))

    def set_step_fusion(self, steps_per_launch):
        """0 (default): automatic; 1: one launch per step; 2: pairs of steps in one launch (D3Q27 FP32/FP64, D2Q37 FP32)."""
        self._check(lib().cmlb_set_step_fusion(self.h, int(steps_per_launch)))

    def sync(self):
        self._check(lib().cmlb_sync(self.h))

    def get_moments(self):
        shape = self.shape
        rho = np.zeros(shape)
        u = np.zeros((self.D,) + shape)
        th = np.zeros(shape)
        self._check(lib().cmlb_get_moments(self.h, _dp(rho), _dp(u), _dp(th)))
        return rho, u, th

    def get_moments_device(self, rho=None, u=None, theta=None):
        """Write rho, u (lattice units), theta into FP64 device tensors (any may
        be None), ordered on the context stream."""
        import torch

        def ptr(t, what, n):
            return None if t is None else _device_ptr(t, what, self.params.device, torch.float64, n)
        nodes = self.nodes
        self._check(lib().cmlb_get_moments_device(self.h, ptr(rho, "rho", nodes), ptr(u, "u", self.D * nodes),
                                                  ptr(theta, "theta", nodes)))

    def get_populations(self):
        f = np.zeros((self.Q,) + self.shape)
        self._check(lib().cmlb_get_populations(self.h, _dp(f)))
        return f

    def set_populations(self, f):
        f = self._field(f, self.Q)
        self._check(lib().cmlb_set_populations(self.h, _dp(f)))

    def reduce(self, allow_unstable=False, noalloc=False):
        """FP64 global diagnostics (cmlb_reduce; with noalloc=True
        cmlb_reduce_noalloc, whose scratch is a fixed device array)."""
        g = Globals()
        fn = lib().cmlb_reduce_noalloc if noalloc else lib().cmlb_reduce
        rc = fn(self.h, ctypes.byref(g))
        if rc and not (allow_unstable and rc == EUNSTABLE):
            self._check(rc)
        return dict(mass=g.mass, momentum=np.array(list(g.momentum)), energy=g.energy,
                    ke=g.kinetic_energy, enstrophy=g.enstrophy, nonfinite=g.n_nonfinite,
                    rho_min=g.rho_min, rho_max=g.rho_max, u_max=g.u_max)

    def state(self):
        p, n, s = ctypes.c_void_p(), ctypes.c_size_t(), ctypes.c_void_p()
        self._check(lib().cmlb_state(self.h, ctypes.byref(p), ctypes.byref(n), ctypes.byref(s)))
        return p.value, n.value, s.value

    def step_count(self):
        return lib().cmlb_step_count(self.h)

    def set_step_count(self, n):
        self._check(lib().cmlb_set_step_count(self.h, int(n)))

    def get_tau(self):
        """Relaxation times by order (8 values; entries 0 and 1 unused)."""
        t = np.zeros(8)
        self._check(lib().cmlb_get_tau(self.h, _dp(t)))
        return t

    def get_scale(self):
        s = np.zeros(37)
        self._check(lib().cmlb_get_scale(self.h, _dp(s)))
        return s[:self.Q]

    # -- device-side state transfer and coarse-graining ---------------------
    def store_state_device(self, dst):
        """Copy the current populations into a device tensor (storage layout,
        at least state_bytes(...) bytes)."""
        need = self.state()[1]
        self._check(lib().cmlb_store_state_device(self.h, _device_ptr(dst, "dst", self.params.device,
                                                                      min_bytes=need)))

    def load_state_device(self, src):
        need = self.state()[1]
        self._check(lib().cmlb_load_state_device(self.h, _device_ptr(src, "src", self.params.device,
                                                                     min_bytes=need)))

    def load_deviations_device(self, src):
        """Load the state from unpadded FP32 deviations [Q][z][y][x] on the
        device (a box filter's output or a training batch entry)."""
        need = 4 * self.Q * int(np.prod(self.shape))
        self._check(lib().cmlb_load_deviations_device(self.h, _device_ptr(src, "src", self.params.device,
                                                                          min_bytes=need)))

    def box_filter(self, factor, dst):
        """Mean over factor^3 blocks into an FP32 device tensor (coarse layout)."""
        import torch
        f = int(factor)
        if f < 1 or any(n % f for n in self.shape):
            raise ValueError("the filter factor must divide every grid size")
        coarse = self.Q * int(np.prod([n // f for n in self.shape]))
        self._check(lib().cmlb_box_filter(self.h, f, _device_ptr(dst, "dst", self.params.device, torch.float32,
                                                                 coarse)))

    # -- learned closure -----------------------------------------------------
    def closure_load(self, params, sigma):
        p = np.ascontiguousarray(params, np.float32)
        s = np.ascontiguousarray(sigma, np.float32)
        if p.size != CLOSURE_NPARAM or s.size != 27:
            raise ValueError("closure needs 2084 parameters and 27 scales")
        fp = ctypes.POINTER(ctypes.c_float)
        self._check(lib().cmlb_closure_load(self.h, p.ctypes.data_as(fp), s.ctypes.data_as(fp)))
        self._closure = {"sigma": s.copy(), "enabled": False, "tie_even": False}

    def closure_enable(self, on=True):
        self._check(lib().cmlb_closure_enable(self.h, 1 if on else 0))
        if getattr(self, "_closure", None) is not None:
            self._closure["enabled"] = bool(on)

    def closure_tie_even(self, on=True):
        self._check(lib().cmlb_closure_tie_even(self.h, 1 if on else 0))
        if getattr(self, "_closure", None) is not None:
            self._closure["tie_even"] = bool(on)

    CLOSURE_OBJECTIVES = {"populations": 0, "momentum": 1}

    def closure_set_objective(self, kind):
        """Objective of closure_objective / closure_train_step: "populations"
        (target one coarse step later) or "momentum" (target two coarse steps
        later; see cmlb_closure_set_objective)."""
        self._check(lib().cmlb_closure_set_objective(self.h, self.CLOSURE_OBJECTIVES[kind]))

    def closure_set_adam(self, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam's constants for closure_train_step (cmlb_closure_set_adam);
        eps must lie well below the gradient's size."""
        self._check(lib().cmlb_closure_set_adam(self.h, float(beta1), float(beta2), float(eps)))

    def closure_freeze(self, orders=()):
        """Orders (3..6) whose rate weights closure_train_step leaves
        unchanged (cmlb_closure_freeze)."""
        mask = 0
        for n in orders:
            if n not in (3, 4, 5, 6):
                raise ValueError(f"order {n} is not set by the network")
            mask |= 1 << (n - 3)
        self._check(lib().cmlb_closure_freeze(self.h, mask))

    def closure_get(self):
        p = np.zeros(CLOSURE_NPARAM, np.float32)
        self._check(lib().cmlb_closure_get(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    def _batch(self, state, target, n_pairs):
        import torch
        n = int(n_pairs) * 27 * self.nodes
        dev = self.params.device
        return Batch(_device_ptr(state, "state", dev, torch.float32, n),
                     _device_ptr(target, "target", dev, torch.float32, n), int(n_pairs))

    def closure_objective(self, state, target, n_pairs=1, grad=True):
        fp = ctypes.POINTER(ctypes.c_float)
        b = self._batch(state, target, n_pairs)
        obj = ctypes.c_float()
        g = np.zeros(CLOSURE_NPARAM, np.float32) if grad else None
        self._check(lib().cmlb_closure_objective(self.h, ctypes.byref(b), ctypes.byref(obj),
                                                 None if g is None else g.ctypes.data_as(fp)))
        return (obj.value, g) if grad else obj.value

    def closure_train_step(self, state, target, lr, n_pairs=1):
        b = self._batch(state, target, n_pairs)
        obj = ctypes.c_float()
        self._check(lib().cmlb_closure_train_step(self.h, ctypes.byref(b), float(lr), ctypes.byref(obj)))
        return obj.value
