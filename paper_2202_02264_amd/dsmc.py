"""Thin ctypes binding of libdsmc.so (include/dsmc.h).

Functions carry the C names and only marshal arguments: models are uploaded
from numpy fp64 arrays, outputs are torch tensors on the GPU whose device
pointers are passed through.  Every step of the smoother runs in the HIP
kernels of libdsmc.so; there is no CPU fallback.  If the library is missing
the import fails.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdsmc.so")

DSMC_OK, DSMC_EINVAL, DSMC_ENOMEM, DSMC_EUNSUPPORTED = 0, -1, -2, -3
DSMC_EAGAIN, DSMC_EDEGENERATE, DSMC_ENUMERIC, DSMC_EDEVICE, DSMC_ECANCELLED = -4, -5, -6, -8, -9
DSMC_ECALLBACK = -7
DSMC_EDEADLINE = -10
DSMC_FLAG_DEGENERATE, DSMC_FLAG_NUMERIC, DSMC_FLAG_LAZY_CAP = 1, 2, 4
DSMC_RESAMPLE_EXACT, DSMC_RESAMPLE_MH, DSMC_RESAMPLE_RS = 0, 1, 2
DSMC_MH_STEPS_DEFAULT, DSMC_RS_CAP_DEFAULT = 32, 1 << 20
DSMC_OBS_NONE, DSMC_OBS_LINEAR_GAUSSIAN, DSMC_OBS_STOCH_VOL, DSMC_OBS_BOX = -1, 0, 1, 2
DSMC_PROPOSAL_GAUSSIAN, DSMC_PROPOSAL_UNIFORM = 0, 1
DSMC_WEIGHT_LEAF_OBS, DSMC_WEIGHT_BOUNDARY_OBS = 0, 1
DSMC_FP32, DSMC_FP64, DSMC_BF16 = 0, 1, 2
DSMC_PLAN_PROFILE = 1
DSMC_PLAN_AUTOTUNE = 2
DSMC_PLAN_GRAPH = 4
DSMC_PLAN_RESCUE_ALL = 8
DSMC_MAX_DX, DSMC_MAX_N = 32, 4096
DSMC_NUM_KERNEL_CLASSES = 4
KERNEL_CLASSES = ("leaves", "rows", "sample", "output")

_dp = C.POINTER(C.c_double)


LOG_PRIOR_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, _dp, _dp)
LOG_TRANSITION_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int, _dp, _dp, _dp)
LOG_OBSERVATION_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int, _dp, _dp)
PROPOSAL_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int, _dp, _dp, _dp)


class dsmc_model_callbacks(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("log_prior", LOG_PRIOR_FN),
                ("log_transition", LOG_TRANSITION_FN), ("log_observation", LOG_OBSERVATION_FN),
                ("proposal", PROPOSAL_FN)]


class dsmc_model_desc(C.Structure):
    _fields_ = [("K", C.c_int), ("d_x", C.c_int), ("d_y", C.c_int),
                ("m0", _dp), ("P0_chol", _dp), ("F", _dp), ("f", _dp), ("Q_chol", _dp),
                ("obs_kind", C.c_int), ("H", _dp), ("h", _dp), ("R_chol", _dp), ("y", _dp),
                ("q_mean", _dp), ("q_chol", _dp), ("weighting", C.c_int),
                ("proposal_kind", C.c_int), ("callbacks", C.POINTER(dsmc_model_callbacks))]


class dsmc_plan_desc(C.Structure):
    _fields_ = [("N", C.c_int), ("d_x", C.c_int), ("max_K", C.c_int), ("max_total_K", C.c_int),
                ("precision", C.c_int), ("flags", C.c_int), ("stream", C.c_void_p),
                ("resampling", C.c_int), ("lazy_param", C.c_int)]


class dsmc_output(C.Structure):
    _fields_ = [("traj", C.c_void_p), ("logw", C.c_void_p), ("log_Z", C.c_void_p),
                ("status", C.c_void_p), ("leaf_x", C.c_void_p), ("leaf_logw", C.c_void_p),
                ("leaf_logL", C.c_void_p), ("ancestry", C.c_void_p), ("logZ_inc", C.c_void_p),
                ("row_lse", C.c_void_p), ("index", C.c_void_p)]


class dsmc_server_desc(C.Structure):
    _fields_ = [("mem_budget", C.c_size_t), ("max_jobs", C.c_int), ("max_classes", C.c_int),
                ("precision", C.c_int), ("flags", C.c_int)]


class dsmc_job(C.Structure):
    _fields_ = [("model", C.c_void_p), ("N", C.c_int), ("seed", C.c_uint64), ("out", dsmc_output),
                ("admit_deadline", C.c_double)]


DSMC_JOB_QUEUED, DSMC_JOB_RUNNING, DSMC_JOB_DONE, DSMC_JOB_FAILED = 0, 1, 2, 3


class dsmc_profile(C.Structure):
    _fields_ = [("launches", C.c_int * DSMC_NUM_KERNEL_CLASSES),
                ("ms", C.c_double * DSMC_NUM_KERNEL_CLASSES), ("pairs", C.c_double),
                ("rescued_rows", C.c_double)]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # PyTorch ships its own copy of the HIP runtime; it must be loaded before
    # this library's (the system one), or one of the two sees no GPU.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, i, u64 = C.c_void_p, C.c_int, C.c_uint64
    sig = {
        "dsmc_model_create": (i, [C.POINTER(dsmc_model_desc), C.POINTER(vp)]),
        "dsmc_model_check": (i, [C.POINTER(dsmc_model_desc)]),
        "dsmc_model_gaussian_proposals": (i, [vp, vp]),
        "dsmc_model_read_proposals": (i, [vp, _dp, _dp]),
        "dsmc_model_destroy": (None, [vp]),
        "dsmc_model_K": (i, [vp]),
        "dsmc_plan": (i, [C.POINTER(dsmc_plan_desc), C.POINTER(vp)]),
        "dsmc_plan_destroy": (None, [vp]),
        "dsmc_smooth": (i, [vp, vp, u64, C.POINTER(dsmc_output)]),
        "dsmc_smooth_batch": (i, [vp, i, C.POINTER(vp), C.POINTER(u64), C.POINTER(dsmc_output)]),
        "dsmc_smooth_conditional": (i, [vp, vp, u64, vp, C.POINTER(dsmc_output)]),
        "dsmc_smooth_batch_conditional": (i, [vp, i, C.POINTER(vp), C.POINTER(u64),
                                              C.POINTER(vp), C.POINTER(dsmc_output)]),
        "dsmc_plan_profile": (i, [vp, C.POINTER(dsmc_profile)]),
        "dsmc_smooth_static": (i, [vp, i, i, u64, C.POINTER(dsmc_output), vp]),
        "dsmc_server_create": (i, [C.POINTER(dsmc_server_desc), C.POINTER(vp)]),
        "dsmc_server_destroy": (None, [vp]),
        "dsmc_submit": (i, [vp, C.POINTER(dsmc_job), C.POINTER(u64)]),
        "dsmc_poll": (i, [vp, u64, C.POINTER(i)]),
        "dsmc_cancel": (i, [vp, u64]),
        "dsmc_job_release": (i, [vp, u64]),
        "dsmc_job_times": (i, [vp, u64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]),
        "dsmc_schedule": (i, [i, i, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "dsmc_last_error": (C.c_char_p, []),
        "dsmc_debug_fail_allocation": (i, [i]),
        "dsmc_device_count": (i, [C.POINTER(i)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


class DsmcError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.dsmc_last_error().decode()
        super().__init__(f"{where} failed with {code}: {msg}")
        self.code = code


def _check(code: int, where: str) -> None:
    if code != DSMC_OK:
        raise DsmcError(code, where)


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def model_desc(spec, callbacks: Optional[dsmc_model_callbacks] = None):
    """(dsmc_model_desc, arrays it points into) for a model spec; the arrays
    must outlive every use of the description."""
    K, dx, dy = spec.K, spec.d_x, spec.d_y
    keep = {
        "m0": _f64(spec.m0).reshape(dx), "P0_chol": _f64(spec.P0_chol).reshape(dx, dx),
        "F": _f64(spec.F).reshape(dx, dx), "f": _f64(spec.f).reshape(dx),
        "Q_chol": _f64(spec.Q_chol).reshape(dx, dx), "y": _f64(spec.y).reshape(K, dy),
        "q_mean": _f64(spec.q_mean).reshape(K, dx), "q_chol": _f64(spec.q_chol).reshape(K, dx, dx),
    }
    if spec.obs == "lg":
        keep["H"] = _f64(spec.H).reshape(dy, dx)
        keep["h"] = _f64(spec.h).reshape(dy)
        keep["R_chol"] = _f64(spec.R_chol).reshape(dy, dy)
    d = dsmc_model_desc()
    d.K, d.d_x, d.d_y = K, dx, dy
    for k, v in keep.items():
        setattr(d, k, _ptr(v))
    d.obs_kind = {"lg": DSMC_OBS_LINEAR_GAUSSIAN, "sv": DSMC_OBS_STOCH_VOL,
                  "box": DSMC_OBS_BOX, "none": DSMC_OBS_NONE}[spec.obs]
    d.proposal_kind = {"gaussian": DSMC_PROPOSAL_GAUSSIAN, "uniform": DSMC_PROPOSAL_UNIFORM}[
        getattr(spec, "proposal", "gaussian")]
    d.weighting = {"leaf_obs": DSMC_WEIGHT_LEAF_OBS,
                   "boundary_obs": DSMC_WEIGHT_BOUNDARY_OBS}[spec.weighting]
    if callbacks is not None:
        d.callbacks = C.pointer(callbacks)
        keep["callbacks"] = callbacks
    return d, keep


def dsmc_model_check(spec, callbacks: Optional[dsmc_model_callbacks] = None) -> int:
    """Host-only validation (and callback self-check); returns the status code."""
    d, keep = model_desc(spec, callbacks)
    rc = _lib.dsmc_model_check(C.byref(d))
    del keep
    return rc


def last_error() -> str:
    return _lib.dsmc_last_error().decode()


def dsmc_debug_fail_allocation(k: int) -> None:
    """Make the k-th device allocation of the next dsmc_plan fail (k < 0: off)."""
    _check(_lib.dsmc_debug_fail_allocation(int(k)), "dsmc_debug_fail_allocation")


class Model:
    """Device-resident model (dsmc_model_create), optionally with host callbacks
    that dsmc_model_create checks the device form against."""

    def __init__(self, spec, callbacks: Optional[dsmc_model_callbacks] = None):
        K, dx = spec.K, spec.d_x
        d, keep = model_desc(spec, callbacks)
        h = C.c_void_p()
        _check(_lib.dsmc_model_create(C.byref(d), C.byref(h)), "dsmc_model_create")
        del keep
        self.handle = h
        self.K, self.d_x = K, dx

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dsmc_model_destroy(self.handle)
            self.handle = None


def dsmc_model_gaussian_proposals(model: Model, stream=None) -> None:
    """Algorithm 5 on the device for a linear-Gaussian model: the parallel-in-time
    Kalman filter and RTS smoother set q_t to the smoothing marginals."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(_lib.dsmc_model_gaussian_proposals(model.handle, C.c_void_p(stream.cuda_stream)),
           "dsmc_model_gaussian_proposals")


def dsmc_model_read_proposals(model: Model):
    """(q_mean (K, d_x), q_chol (K, d_x, d_x)) of the device model, as numpy fp64."""
    qm = np.zeros((model.K, model.d_x))
    qc = np.zeros((model.K, model.d_x, model.d_x))
    _check(_lib.dsmc_model_read_proposals(model.handle, _ptr(qm), _ptr(qc)),
           "dsmc_model_read_proposals")
    return qm, qc


def dsmc_model_create(spec, callbacks: Optional[dsmc_model_callbacks] = None) -> Model:
    return Model(spec, callbacks)


class Plan:
    """dsmc_plan: workspace for series of up to max_K points (sum max_total_K)."""

    def __init__(self, N: int, d_x: int, max_K: int, max_total_K: int = 0,
                 precision: int = DSMC_FP32, profile: bool = False, autotune: bool = False,
                 graph: bool = False, rescue_all: bool = False, stream=None,
                 resampling: int = 0, lazy_param: int = 0):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        d = dsmc_plan_desc()
        d.N, d.d_x, d.max_K, d.max_total_K = N, d_x, max_K, max_total_K
        d.precision = precision
        d.flags = ((DSMC_PLAN_PROFILE if profile else 0) | (DSMC_PLAN_AUTOTUNE if autotune else 0)
                   | (DSMC_PLAN_GRAPH if graph else 0) | (DSMC_PLAN_RESCUE_ALL if rescue_all else 0))
        d.stream = C.c_void_p(stream.cuda_stream)
        d.resampling, d.lazy_param = resampling, lazy_param
        h = C.c_void_p()
        _check(_lib.dsmc_plan(C.byref(d), C.byref(h)), "dsmc_plan")
        self.handle = h
        self.N, self.d_x, self.precision = N, d_x, precision
        self.max_K = max_K
        self.max_total_K = max(max_total_K, max_K)
        self.stream = stream
        self.dtype = torch.float64 if precision == DSMC_FP64 else torch.float32

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dsmc_plan_destroy(self.handle)
            self.handle = None


def dsmc_plan(N: int, d_x: int, max_K: int, **kw) -> Plan:
    return Plan(N, d_x, max_K, **kw)


@dataclass
class Output:
    """Caller-owned device buffers of one series (torch tensors)."""
    traj: "object"
    logw: "object"
    log_Z: "object"
    status: "object"
    leaf_x: "object" = None
    leaf_logw: "object" = None
    leaf_logL: "object" = None
    ancestry: "object" = None
    logZ_inc: "object" = None
    row_lse: "object" = None
    index: "object" = None

    def c_struct(self) -> dsmc_output:
        o = dsmc_output()
        for f in dsmc_output._fields_:
            t = getattr(self, f[0])
            setattr(o, f[0], None if t is None else t.data_ptr())
        return o


def alloc_output(plan: Plan, K: int, diagnostics: bool = False, device="cuda") -> Output:
    import torch
    N, dx, dt = plan.N, plan.d_x, plan.dtype
    kw = dict(device=device)
    o = Output(traj=torch.empty((dx, K, N), dtype=dt, **kw), logw=torch.empty(N, dtype=dt, **kw),
               log_Z=torch.empty(1, dtype=torch.float64, **kw),
               status=torch.zeros(1, dtype=torch.int32, **kw))
    if diagnostics:
        o.leaf_x = torch.empty((dx, K, N), dtype=dt, **kw)
        o.leaf_logw = torch.empty((K, N), dtype=dt, **kw)
        o.leaf_logL = torch.empty(K, dtype=torch.float64, **kw)
        o.ancestry = torch.empty((max(K - 1, 0), 2, N), dtype=torch.int32, **kw)
        o.logZ_inc = torch.empty(max(K - 1, 0), dtype=torch.float64, **kw)
        o.row_lse = torch.empty((max(K - 1, 0), N), dtype=torch.float64, **kw)
        o.index = torch.empty((K, N), dtype=torch.int32, **kw)
    return o


def dsmc_smooth(plan: Plan, model: Model, seed: int, out: Output) -> None:
    o = out.c_struct()
    _check(_lib.dsmc_smooth(plan.handle, model.handle, C.c_uint64(seed & (2**64 - 1)),
                            C.byref(o)), "dsmc_smooth")


DSMC_STATIC_SCRATCH_BYTES = 256 << 20


def dsmc_smooth_static(model: Model, N: int, seed: int, out: Output, precision: int = DSMC_FP32,
                       stream=None) -> None:
    """dsmc_smooth without a plan or any device allocation (the library's fixed
    per-GPU workspace); ``out`` as from alloc_output for (N, d_x, K, precision)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    o = out.c_struct()
    _check(_lib.dsmc_smooth_static(model.handle, N, precision, C.c_uint64(seed & (2**64 - 1)),
                                   C.byref(o), C.c_void_p(stream.cuda_stream)),
           "dsmc_smooth_static")


def dsmc_smooth_conditional(plan: Plan, model: Model, seed: int, star, out: Output) -> None:
    """Conditional dSMC with the star trajectory ``star``: a contiguous device
    tensor [d_x][K] of the plan's real type, kept in slot 0 of the output."""
    if (not star.is_cuda or star.dtype != plan.dtype or not star.is_contiguous()
            or tuple(star.shape) != (plan.d_x, model.K)):
        raise ValueError(f"star must be a contiguous {plan.dtype} device tensor of shape "
                         f"({plan.d_x}, {model.K})")
    o = out.c_struct()
    _check(_lib.dsmc_smooth_conditional(plan.handle, model.handle,
                                        C.c_uint64(seed & (2**64 - 1)),
                                        C.c_void_p(star.data_ptr()), C.byref(o)),
           "dsmc_smooth_conditional")


def dsmc_smooth_batch_conditional(plan: Plan, models: Sequence[Model], seeds: Sequence[int],
                                  stars: Sequence, outs: Sequence[Output]) -> None:
    """B conditional runs in packed launches; stars[s] is a contiguous device
    tensor [d_x][K_s] of the plan's real type, or None (unconditional)."""
    B = len(models)
    for st, m in zip(stars, models):
        if st is not None and (not st.is_cuda or st.dtype != plan.dtype or not st.is_contiguous()
                               or tuple(st.shape) != (plan.d_x, m.K)):
            raise ValueError(f"each star must be a contiguous {plan.dtype} device tensor of "
                             f"shape ({plan.d_x}, K)")
    hs = (C.c_void_p * B)(*[m.handle.value for m in models])
    ss = (C.c_uint64 * B)(*[int(s) & (2**64 - 1) for s in seeds])
    ps = (C.c_void_p * B)(*[None if st is None else st.data_ptr() for st in stars])
    os_ = (dsmc_output * B)(*[o.c_struct() for o in outs])
    _check(_lib.dsmc_smooth_batch_conditional(plan.handle, B, hs, ss, ps, os_),
           "dsmc_smooth_batch_conditional")


def dsmc_smooth_batch(plan: Plan, models: Sequence[Model], seeds: Sequence[int],
                      outs: Sequence[Output]) -> None:
    B = len(models)
    hs = (C.c_void_p * B)(*[m.handle.value for m in models])
    ss = (C.c_uint64 * B)(*[int(s) & (2**64 - 1) for s in seeds])
    os_ = (dsmc_output * B)(*[o.c_struct() for o in outs])
    _check(_lib.dsmc_smooth_batch(plan.handle, B, hs, ss, os_), "dsmc_smooth_batch")


def dsmc_plan_profile(plan: Plan) -> dict:
    p = dsmc_profile()
    _check(_lib.dsmc_plan_profile(plan.handle, C.byref(p)), "dsmc_plan_profile")
    return {"launches": dict(zip(KERNEL_CLASSES, list(p.launches))),
            "ms": dict(zip(KERNEL_CLASSES, list(p.ms))), "pairs": p.pairs,
            "rescued_rows": p.rescued_rows}


def check_status(out: Output) -> int:
    """Synchronise and return the device status bits of an output."""
    import torch
    torch.cuda.synchronize()
    return int(out.status.item())


def smooth(spec, N: int, seed: int, precision: int = DSMC_FP32, diagnostics: bool = False,
           plan: Optional[Plan] = None, model: Optional[Model] = None) -> Output:
    """Convenience wrapper: upload, plan, run, synchronise, raise on device flags."""
    import torch
    model = model or Model(spec)
    plan = plan or Plan(N, spec.d_x, spec.K, precision=precision)
    out = alloc_output(plan, spec.K, diagnostics)
    dsmc_smooth(plan, model, seed, out)
    torch.cuda.synchronize()
    st = int(out.status.item())
    if st & DSMC_FLAG_NUMERIC:
        raise DsmcError(DSMC_ENUMERIC, "dsmc_smooth (device)")
    return out


class Server:
    """dsmc_server_create: continuous-batching serving engine.  Keeps a reference
    to every submitted job's model and output buffers until it is polled done."""

    def __init__(self, mem_budget: int = 16 << 30, max_jobs: int = 1024, max_classes: int = 4,
                 precision: int = DSMC_FP32):
        d = dsmc_server_desc()
        d.mem_budget, d.max_jobs, d.max_classes, d.precision = mem_budget, max_jobs, max_classes, precision
        h = C.c_void_p()
        _check(_lib.dsmc_server_create(C.byref(d), C.byref(h)), "dsmc_server_create")
        self.handle = h
        self.dtype_is_fp64 = precision == DSMC_FP64
        self._keep = {}

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.dsmc_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        self.close()


def dsmc_server_create(**kw) -> Server:
    return Server(**kw)


def alloc_job_output(N: int, d_x: int, K: int, fp64: bool = False, diagnostics: bool = False):
    class _P:
        pass
    p = _P()
    import torch
    p.N, p.d_x, p.dtype = N, d_x, (torch.float64 if fp64 else torch.float32)
    return alloc_output(p, K, diagnostics)


def dsmc_submit(server: Server, model: Model, N: int, seed: int, out: Output,
                admit_deadline: float = 0.0) -> int:
    j = dsmc_job()
    j.model = model.handle.value
    j.N = N
    j.seed = seed & (2**64 - 1)
    j.out = out.c_struct()
    j.admit_deadline = admit_deadline
    jid = C.c_uint64()
    _check(_lib.dsmc_submit(server.handle, C.byref(j), C.byref(jid)), "dsmc_submit")
    server._keep[jid.value] = (model, out)
    return jid.value


def dsmc_cancel(server: Server, job_id: int) -> int:
    """DSMC_OK if the queued job will be cancelled, DSMC_EAGAIN if it already runs."""
    rc = _lib.dsmc_cancel(server.handle, C.c_uint64(job_id))
    if rc not in (DSMC_OK, DSMC_EAGAIN):
        _check(rc, "dsmc_cancel")
    return rc


def dsmc_poll(server: Server, job_id: int):
    """(return code, state); code 0 = done, DSMC_EAGAIN = not yet, else failed."""
    st = C.c_int()
    rc = _lib.dsmc_poll(server.handle, C.c_uint64(job_id), C.byref(st))
    if rc != DSMC_EAGAIN:
        server._keep.pop(job_id, None)
    return rc, st.value


def dsmc_job_release(server: Server, job_id: int) -> int:
    """Forget a finished job; DSMC_OK, or DSMC_EAGAIN while it is queued or running."""
    rc = _lib.dsmc_job_release(server.handle, C.c_uint64(job_id))
    if rc not in (DSMC_OK, DSMC_EAGAIN):
        _check(rc, "dsmc_job_release")
    if rc == DSMC_OK:
        server._keep.pop(job_id, None)
    return rc


def dsmc_job_times(server: Server, job_id: int):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(_lib.dsmc_job_times(server.handle, C.c_uint64(job_id), C.byref(a), C.byref(b),
                               C.byref(c)), "dsmc_job_times")
    return a.value, b.value, c.value


def dsmc_schedule(K: int):
    """Algorithm 6's combines for K points as the library runs them: a list of
    levels, each a list of (a, c, b)."""
    n = max(K - 1, 1)
    arrs = [np.zeros(n, dtype=np.int32) for _ in range(4)]
    ptrs = [x.ctypes.data_as(C.POINTER(C.c_int32)) for x in arrs]
    cnt = _lib.dsmc_schedule(K, n, *ptrs)
    if cnt < 0:
        _check(cnt, "dsmc_schedule")
    a, c, b, lv = (x[:cnt] for x in arrs)
    levels = [[] for _ in range(int(lv.max()) + 1)] if cnt else []
    for i in range(cnt):
        levels[lv[i]].append((int(a[i]), int(c[i]), int(b[i])))
    return levels
