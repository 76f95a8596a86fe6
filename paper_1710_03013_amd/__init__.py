"""Python binding of libkkm (mini-batch kernel k-means with landmark centroids on MI355X).

The functions carry the names of the C ABI in include/kkm.h and only marshal
arguments: torch tensors supply device memory and the current HIP stream, and
every step of the computation runs in the library's HIP kernels.  Importing the
package loads libkkm.so and raises if it has not been built
(``python -m paper_1710_03013_amd.build`` or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import atexit
import ctypes as ct
import os
import sys
import weakref

import numpy as np

__all__ = [
    "KKM_OK", "KKM_KERNEL_LINEAR", "KKM_KERNEL_RBF", "KKM_KERNEL_RMSD", "KKM_F32", "KKM_F64",
    "KKM_PREC_FP64", "KKM_PREC_FP32", "KKM_PREC_BF16", "KKM_PREC_BF16X3", "KKM_SAMPLE_STRIDE", "KKM_SAMPLE_BLOCK",
    "KKM_INIT_KMEANSPP", "KKM_INIT_RANDOM_LABELS", "KKM_INIT_MEDOIDS", "KkmError", "Model", "lib",
    "kkm_model_create", "kkm_model_load", "kkm_model_export", "kkm_model_shape", "kkm_fit",
    "kkm_fit_workspace_bytes", "kkm_fit_min_batches", "kkm_fit_restarts", "kkm_assign", "kkm_assign_workspace_bytes", "kkm_cost",
    "kkm_kernel_block", "kkm_kernel_block_workspace_bytes", "kkm_assign_noalloc",
    "kkm_landmark_count", "kkm_draw_landmarks", "kkm_draw_kmpp_uniforms", "kkm_draw_init_labels",
    "kkm_version", "EXPORTED_SYMBOLS", "release_models",
]

KKM_OK = 0
KKM_KERNEL_LINEAR, KKM_KERNEL_RBF, KKM_KERNEL_RMSD = 0, 1, 2
KKM_F32, KKM_F64 = 0, 1
KKM_PREC_FP64, KKM_PREC_FP32, KKM_PREC_BF16, KKM_PREC_BF16X3 = 0, 1, 2, 3
KKM_SAMPLE_STRIDE, KKM_SAMPLE_BLOCK = 0, 1
KKM_INIT_KMEANSPP, KKM_INIT_RANDOM_LABELS, KKM_INIT_MEDOIDS = 0, 1, 2
KKM_FIT_COOPERATIVE = 1
KKM_FIT_GLOBAL_COST = 2

_KERNELS = {"linear": KKM_KERNEL_LINEAR, "rbf": KKM_KERNEL_RBF, "rmsd": KKM_KERNEL_RMSD}
_PRECISIONS = {"fp64": KKM_PREC_FP64, "fp32": KKM_PREC_FP32, "bf16": KKM_PREC_BF16, "bf16x3": KKM_PREC_BF16X3}
_SAMPLING = {"stride": KKM_SAMPLE_STRIDE, "block": KKM_SAMPLE_BLOCK}
_INITS = {"kmeans++": KKM_INIT_KMEANSPP, "random": KKM_INIT_RANDOM_LABELS, "medoids": KKM_INIT_MEDOIDS}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkkm.so")


class KkmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libkkm status {status}: {msg}")
        self.status = status


class _Kernel(ct.Structure):
    _fields_ = [("type", ct.c_int32), ("n_atoms", ct.c_int32), ("sigma", ct.c_double)]


class _Params(ct.Structure):
    _fields_ = [("C", ct.c_int32), ("B", ct.c_int32), ("s", ct.c_double), ("max_iter", ct.c_int32),
                ("sampling", ct.c_int32), ("init", ct.c_int32), ("precision", ct.c_int32),
                ("flags", ct.c_int32), ("seed", ct.c_uint64),
                ("landmarks", ct.POINTER(ct.c_int64)), ("kmpp_uniforms", ct.POINTER(ct.c_double)),
                ("init_labels", ct.POINTER(ct.c_int32)), ("init_medoids", ct.POINTER(ct.c_int64))]


class _FitInfo(ct.Structure):
    _fields_ = [("updates_per_batch", ct.POINTER(ct.c_int32)), ("batch_medoids", ct.POINTER(ct.c_int64)),
                ("batch_counts", ct.POINTER(ct.c_int64)), ("global_medoids", ct.POINTER(ct.c_int64)),
                ("evals_algorithmic", ct.c_int64), ("evals_performed", ct.c_int64),
                ("rows_refined", ct.c_int64), ("medoid_candidates", ct.c_int64),
                ("time_phases", ct.c_int32), ("reserved", ct.c_int32), ("ms_init", ct.c_double),
                ("ms_landmark", ct.c_double), ("ms_dist", ct.c_double), ("ms_refine", ct.c_double),
                ("ms_select", ct.c_double), ("ms_landmark_loop", ct.c_double),
                ("landmark_trace", ct.POINTER(ct.c_int64)), ("medoid_displacement", ct.POINTER(ct.c_double)),
                ("partial_cost", ct.POINTER(ct.c_double)), ("global_cost", ct.POINTER(ct.c_double))]


# name -> (restype, argtypes): every symbol include/kkm.h declares
_SIGS = {
    "kkm_model_create": (ct.c_int, [ct.POINTER(_Kernel), ct.c_int64, ct.c_int32, ct.c_int64, ct.c_int32,
                                    ct.POINTER(ct.c_void_p)]),
    "kkm_model_load": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.POINTER(ct.c_int64),
                                  ct.POINTER(ct.c_double)]),
    "kkm_model_export": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double),
                                    ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64)]),
    "kkm_model_shape": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32),
                                   ct.POINTER(ct.c_int64)]),
    "kkm_model_free": (None, [ct.c_void_p]),
    "kkm_fit_workspace_bytes": (ct.c_size_t, [ct.c_int64, ct.c_int64, ct.c_int32, ct.POINTER(_Kernel),
                                              ct.POINTER(_Params)]),
    "kkm_fit_min_batches": (ct.c_int64, [ct.c_int64, ct.c_int64, ct.c_int32, ct.POINTER(_Kernel),
                                         ct.POINTER(_Params), ct.c_size_t]),
    "kkm_fit": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_int32, ct.POINTER(_Kernel),
                           ct.POINTER(_Params), ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_void_p,
                           ct.c_void_p, ct.POINTER(_FitInfo)]),
    "kkm_fit_restarts_workspace_bytes": (ct.c_size_t, [ct.c_int64, ct.c_int64, ct.c_int32, ct.POINTER(_Kernel),
                                                       ct.POINTER(_Params), ct.c_int32]),
    "kkm_fit_restarts": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_int32, ct.POINTER(_Kernel),
                                    ct.POINTER(_Params), ct.c_int32, ct.c_void_p, ct.c_size_t, ct.c_void_p,
                                    ct.c_void_p, ct.c_void_p, ct.POINTER(_FitInfo), ct.POINTER(ct.c_double),
                                    ct.POINTER(ct.c_int32)]),
    "kkm_assign_workspace_bytes": (ct.c_size_t, [ct.c_void_p, ct.c_int64, ct.c_int32]),
    "kkm_assign": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_void_p,
                              ct.c_size_t, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "kkm_cost": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_void_p,
                            ct.c_size_t, ct.c_void_p, ct.POINTER(ct.c_double)]),
    "kkm_assign_noalloc": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_void_p,
                                      ct.c_void_p, ct.c_void_p]),
    "kkm_kernel_block_workspace_bytes": (ct.c_size_t, [ct.POINTER(_Kernel), ct.c_int64, ct.c_int64, ct.c_int64,
                                                       ct.c_int32]),
    "kkm_kernel_block": (ct.c_int, [ct.POINTER(_Kernel), ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int64,
                                    ct.c_int64, ct.c_int32, ct.c_void_p, ct.c_size_t, ct.c_void_p, ct.c_void_p]),
    "kkm_landmark_count": (ct.c_int64, [ct.c_int64, ct.c_double]),
    "kkm_draw_landmarks": (ct.c_int, [ct.c_uint64, ct.c_int32, ct.c_int64, ct.c_double, ct.POINTER(ct.c_int64)]),
    "kkm_draw_kmpp_uniforms": (ct.c_int, [ct.c_uint64, ct.c_int32, ct.POINTER(ct.c_double)]),
    "kkm_draw_init_labels": (ct.c_int, [ct.c_uint64, ct.c_int64, ct.c_int32, ct.POINTER(ct.c_int32)]),
    "kkm_last_error": (ct.c_char_p, []),
    "kkm_version": (ct.c_char_p, []),
}
EXPORTED_SYMBOLS = tuple(_SIGS)

_lib = None


def lib() -> ct.CDLL:
    """The loaded libkkm (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1710_03013_amd.build.build()")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


lib()


def _check(status: int) -> None:
    if status != KKM_OK:
        raise KkmError(status, lib().kkm_last_error().decode())


def _i64p(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_int64)) if a is not None else None


def _f64p(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double)) if a is not None else None


def _i32p(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_int32)) if a is not None else None


def _kernel(kind, sigma=1.0, n_atoms=0) -> _Kernel:
    t = _KERNELS[kind] if isinstance(kind, str) else int(kind)
    return _Kernel(t, int(n_atoms), float(sigma))


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return KKM_F32
    if t.dtype == torch.float64:
        return KKM_F64
    raise TypeError("samples must be float32 or float64")


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class _OnStream:
    """Runs a library call on `stream` (default: the current stream) in the order of the caller's
    current stream: the library stream first waits for the current stream (which produced X), the
    call's temporaries (contiguous copy, workspace, outputs) are allocated on the library stream, and
    caller tensors read there are recorded on it, so the caching allocator does not hand their
    memory out again before the library stream has finished with them."""

    def __init__(self, stream):
        import torch
        self.torch = torch
        self.cur = torch.cuda.current_stream()
        self.s = stream if stream is not None else self.cur
        self.other = self.s != self.cur

    def __enter__(self):
        if self.other:
            self.s.wait_stream(self.cur)
            self.ctx = self.torch.cuda.stream(self.s)
            self.ctx.__enter__()
        return self

    def use(self, *tensors):
        if self.other:
            for t in tensors:
                if t is not None:
                    t.record_stream(self.s)

    def __exit__(self, *exc):
        if self.other:
            self.ctx.__exit__(*exc)
        return False


def _workspace(nbytes: int, device):
    import torch
    return torch.empty(max(256, int(nbytes)), dtype=torch.uint8, device=device)


_LIVE_MODELS = weakref.WeakSet()


class Model:
    """Owner of a kkm_model handle (device-resident sparse centroids).

    The device memory is released when the object is collected, or at interpreter exit by
    ``release_models`` (registered with atexit), which runs while the HIP runtime is still fully up;
    a model still alive once the interpreter is finalising is left to the process exit instead of
    calling into the runtime during teardown."""

    def __init__(self, ptr: int, kernel: _Kernel, d: int, C: int, dtype: int):
        self.ptr = ct.c_void_p(ptr)
        self.kernel = kernel
        self.d, self.C, self.dtype = d, C, dtype
        _LIVE_MODELS.add(self)

    def free(self) -> None:
        """Release the model's device memory now (the handle becomes empty)."""
        ptr = getattr(self, "ptr", None)
        if ptr is not None and ptr.value:
            lib().kkm_model_free(ptr)
            self.ptr = ct.c_void_p(0)

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def release_models() -> None:
    """Free every live model after the device has finished the work queued on it (called at exit,
    before interpreter teardown; safe to call at any time: models freed here become empty)."""
    live = [m for m in list(_LIVE_MODELS) if getattr(m, "ptr", None) is not None and m.ptr.value]
    if not live:
        return
    try:
        import torch
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for m in live:
        try:
            m.free()
        except Exception:
            pass


atexit.register(release_models)


def kkm_model_create(kernel="rbf", d=1, C=1, max_support=None, dtype="f32", sigma=1.0, n_atoms=0) -> Model:
    k = kernel if isinstance(kernel, _Kernel) else _kernel(kernel, sigma, n_atoms)
    dt = dtype if isinstance(dtype, int) else (KKM_F64 if dtype in ("f64", "float64") else KKM_F32)
    out = ct.c_void_p()
    _check(lib().kkm_model_create(ct.byref(k), int(d), int(C), int(max_support or C), dt, ct.byref(out)))
    return Model(out.value, k, int(d), int(C), dt)


def kkm_model_load(model: Model, support: np.ndarray, offsets, coef) -> None:
    dt = np.float64 if model.dtype == KKM_F64 else np.float32
    sup = np.ascontiguousarray(support, dtype=dt).reshape(-1, model.d)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    cf = np.ascontiguousarray(coef, dtype=np.float64)
    _check(lib().kkm_model_load(model.ptr, sup.ctypes.data_as(ct.c_void_p), sup.shape[0], _i64p(off), _f64p(cf)))


def kkm_model_shape(model: Model):
    d, C, n = ct.c_int64(), ct.c_int32(), ct.c_int64()
    _check(lib().kkm_model_shape(model.ptr, ct.byref(d), ct.byref(C), ct.byref(n)))
    return d.value, C.value, n.value


def kkm_model_export(model: Model) -> dict:
    d, C, n = kkm_model_shape(model)
    dt = np.float64 if model.dtype == KKM_F64 else np.float32
    sup = np.zeros((max(n, 1), d), dtype=dt)
    off = np.zeros(C + 1, dtype=np.int64)
    coef = np.zeros(max(n, 1), dtype=np.float64)
    selfterm = np.zeros(C, dtype=np.float64)
    counts = np.zeros(C, dtype=np.int64)
    med = np.zeros(C, dtype=np.int64)
    _check(lib().kkm_model_export(model.ptr, sup.ctypes.data_as(ct.c_void_p), _i64p(off), _f64p(coef),
                                  _f64p(selfterm), _i64p(counts), _i64p(med)))
    return dict(support=sup[:n], offsets=off, coef=coef[:n], self=selfterm, counts=counts, medoid_index=med)


def _params(C, B, s, max_iter, sampling, init, precision, seed, landmarks, kmpp_uniforms, init_labels,
            init_medoids, keep, cooperative=False, global_cost=False):
    p = _Params()
    p.flags = (KKM_FIT_COOPERATIVE if cooperative else 0) | (KKM_FIT_GLOBAL_COST if global_cost else 0)
    p.C, p.B, p.s, p.max_iter = int(C), int(B), float(s), int(max_iter)
    p.sampling = _SAMPLING[sampling] if isinstance(sampling, str) else int(sampling)
    p.init = _INITS[init] if isinstance(init, str) else int(init)
    p.precision = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.seed = int(seed) & ((1 << 64) - 1)
    if landmarks is not None:
        lm = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.int64) for x in landmarks])
                                  if isinstance(landmarks, (list, tuple)) else landmarks, dtype=np.int64)
        keep.append(lm)
        p.landmarks = _i64p(lm)
    if kmpp_uniforms is not None:
        u = np.ascontiguousarray(kmpp_uniforms, dtype=np.float64)
        keep.append(u)
        p.kmpp_uniforms = _f64p(u)
    if init_labels is not None:
        lab = np.ascontiguousarray(init_labels, dtype=np.int32)
        keep.append(lab)
        p.init_labels = _i32p(lab)
    if init_medoids is not None:
        med = np.ascontiguousarray(init_medoids, dtype=np.int64)
        keep.append(med)
        p.init_medoids = _i64p(med)
    return p


def kkm_fit_workspace_bytes(N, d, dtype, kernel, **params) -> int:
    keep = []
    p = _params(**params, keep=keep)
    return int(lib().kkm_fit_workspace_bytes(int(N), int(d), int(dtype), ct.byref(kernel), ct.byref(p)))


def kkm_fit_min_batches(N, d, dtype, kernel, budget_bytes, **params) -> int:
    """Smallest number of mini-batches whose fit workspace fits budget_bytes (params as for
    kkm_fit_workspace_bytes; their B is not read).  Raises KkmError when none fits."""
    keep = []
    p = _params(**{"B": 1, **params}, keep=keep)
    B = int(lib().kkm_fit_min_batches(int(N), int(d), int(dtype), ct.byref(kernel), ct.byref(p), int(budget_bytes)))
    if B == 0:
        raise KkmError(-1, lib().kkm_last_error().decode())
    return B


def kkm_fit(X, kernel="rbf", sigma=1.0, n_atoms=0, C=2, B=1, s=1.0, max_iter=20, sampling="stride",
            init="kmeans++", precision="fp32", seed=0, landmarks=None, kmpp_uniforms=None, init_labels=None,
            init_medoids=None, model=None, workspace=None, stream=None, want_labels=True, time_phases=False,
            landmark_trace=False, cooperative=False, cost_trace=False, global_cost=False):
    """Fit on X (a CUDA tensor, N x d).  Returns (model, labels tensor or None, info dict).

    time_phases: False / 0 no timing; True / 1 HIP events around every phase; 2 only around the
    landmark loop kernel and the batch-wide distance kernel (info["ms"] holds 0 for the others).
    cooperative: launch the kernels whose workgroups wait for each other cooperatively (for callers
    that keep other streams busy on the same GPU meanwhile).
    cost_trace: also return the per-batch observables of Sec. 4.1: info["partial_cost"] (the partial
    cost of every batch, one more reduction per batch) and info["medoid_displacement"] (B x C).
    global_cost: also return info["global_cost"], the global cost after every batch (an assign pass
    over all N samples per batch)."""
    import torch
    if not X.is_cuda:
        raise ValueError("X must be a device tensor")
    with _OnStream(stream) as os_:
        os_.use(X, workspace)
        return _kkm_fit(X.contiguous(), kernel, sigma, n_atoms, C, B, s, max_iter, sampling, init, precision, seed,
                        landmarks, kmpp_uniforms, init_labels, init_medoids, model, workspace, os_.s, want_labels,
                        time_phases, landmark_trace, cooperative, cost_trace, global_cost)


def _kkm_fit(X, kernel, sigma, n_atoms, C, B, s, max_iter, sampling, init, precision, seed, landmarks, kmpp_uniforms,
             init_labels, init_medoids, model, workspace, stream, want_labels, time_phases, landmark_trace, cooperative,
             cost_trace, global_cost):
    import torch
    N, d = X.shape
    k = _kernel(kernel, sigma, n_atoms)
    dt = _dtype_code(X)
    keep = []
    p = _params(C, B, s, max_iter, sampling, init, precision, seed, landmarks, kmpp_uniforms, init_labels,
                init_medoids, keep, cooperative, global_cost)
    need = int(lib().kkm_fit_workspace_bytes(N, d, dt, ct.byref(k), ct.byref(p)))
    if need == 0:
        _check(lib().kkm_fit(None, N, d, dt, ct.byref(k), ct.byref(p), None, 0, None, None, None, None))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
    if model is None:
        model = kkm_model_create(k, d, C, C, dt)
    labels = torch.empty(N, dtype=torch.int32, device=X.device) if want_labels else None
    upd = np.zeros(B, dtype=np.int32)
    bmed = np.zeros(B * C, dtype=np.int64)
    bcnt = np.zeros(B * C, dtype=np.int64)
    gmed = np.zeros(B * C, dtype=np.int64)
    trace = np.zeros(64, dtype=np.int64) if landmark_trace else None
    disp = np.zeros(B * C, dtype=np.float64) if cost_trace else None
    pc = np.zeros(B, dtype=np.float64) if cost_trace else None
    gc = np.zeros(B, dtype=np.float64) if global_cost else None
    info = _FitInfo(_i32p(upd), _i64p(bmed), _i64p(bcnt), _i64p(gmed), 0, 0, 0, 0, int(time_phases))
    if trace is not None:
        info.landmark_trace = _i64p(trace)
    if cost_trace:
        info.medoid_displacement = _f64p(disp)
        info.partial_cost = _f64p(pc)
    if global_cost:
        info.global_cost = _f64p(gc)
    _check(lib().kkm_fit(ct.c_void_p(X.data_ptr()), N, d, dt, ct.byref(k), ct.byref(p),
                         ct.c_void_p(ws.data_ptr()), ws.numel(), ct.c_void_p(_stream_ptr(stream)), model.ptr,
                         ct.c_void_p(labels.data_ptr()) if labels is not None else None, ct.byref(info)))
    out = dict(updates_per_batch=upd, batch_medoids=bmed.reshape(B, C), batch_counts=bcnt.reshape(B, C),
               global_medoids=gmed.reshape(B, C),
               medoid_displacement=disp.reshape(B, C) if disp is not None else None, partial_cost=pc, global_cost=gc,
               evals_algorithmic=info.evals_algorithmic,
               evals_performed=info.evals_performed, rows_refined=info.rows_refined,
               medoid_candidates=info.medoid_candidates, workspace_bytes=need,
               ms=dict(init=info.ms_init, landmark=info.ms_landmark, landmark_loop=info.ms_landmark_loop,
                       dist=info.ms_dist, refine=info.ms_refine, select=info.ms_select) if time_phases else None,
               landmark_trace=trace[1:1 + int(trace[0])] if trace is not None else None)
    return model, labels, out


def kkm_fit_restarts(X, restarts=5, kernel="rbf", sigma=1.0, n_atoms=0, C=2, B=1, s=1.0, max_iter=20,
                     sampling="stride", init="kmeans++", precision="fp32", seed=0, init_medoids=None, model=None,
                     workspace=None, stream=None, want_labels=True):
    """Best of `restarts` fits with seeds seed .. seed + restarts - 1, the lowest FP64 cost over all of X
    winning (the lowest restart on equal costs), all run by the library back to back on one stream.
    Returns (model, labels tensor or None, info dict with "restart" and "restart_costs" added)."""
    import torch
    if not X.is_cuda:
        raise ValueError("X must be a device tensor")
    with _OnStream(stream) as os_:
        os_.use(X, workspace)
        X = X.contiguous()
        N, d = X.shape
        k = _kernel(kernel, sigma, n_atoms)
        dt = _dtype_code(X)
        keep = []
        p = _params(C, B, s, max_iter, sampling, init, precision, seed, None, None, None, init_medoids, keep)
        need = int(lib().kkm_fit_restarts_workspace_bytes(N, d, dt, ct.byref(k), ct.byref(p), int(restarts)))
        if need == 0:
            _check(lib().kkm_fit_restarts(None, N, d, dt, ct.byref(k), ct.byref(p), int(restarts), None, 0, None,
                                          None, None, None, None, None))
        ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
        if model is None:
            model = kkm_model_create(k, d, C, C, dt)
        labels = torch.empty(N, dtype=torch.int32, device=X.device) if want_labels else None
        upd = np.zeros(B, dtype=np.int32)
        bmed, bcnt, gmed = (np.zeros(B * C, dtype=np.int64) for _ in range(3))
        info = _FitInfo(_i32p(upd), _i64p(bmed), _i64p(bcnt), _i64p(gmed), 0, 0, 0, 0, 0)
        costs = np.zeros(int(restarts), dtype=np.float64)
        best = ct.c_int32(-1)
        _check(lib().kkm_fit_restarts(ct.c_void_p(X.data_ptr()), N, d, dt, ct.byref(k), ct.byref(p), int(restarts),
                                      ct.c_void_p(ws.data_ptr()), ws.numel(), ct.c_void_p(_stream_ptr(os_.s)),
                                      model.ptr, ct.c_void_p(labels.data_ptr()) if labels is not None else None,
                                      ct.byref(info), _f64p(costs), ct.byref(best)))
    out = dict(updates_per_batch=upd, batch_medoids=bmed.reshape(B, C), batch_counts=bcnt.reshape(B, C),
               global_medoids=gmed.reshape(B, C), evals_algorithmic=info.evals_algorithmic,
               evals_performed=info.evals_performed, rows_refined=info.rows_refined,
               medoid_candidates=info.medoid_candidates, workspace_bytes=need, restart=int(best.value),
               restart_costs=costs)
    return model, labels, out


def kkm_assign_workspace_bytes(model: Model, n: int, precision="fp32") -> int:
    pr = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return int(lib().kkm_assign_workspace_bytes(model.ptr, int(n), pr))


def kkm_assign(model: Model, X, precision="fp32", want_gap=False, workspace=None, labels=None, gap=None,
               stream=None):
    """Labels (int32 CUDA tensor) of the rows of X, and the relative margins if asked."""
    import torch
    with _OnStream(stream) as os_:
        os_.use(X, workspace, labels, gap)
        X = X.contiguous()
        n = X.shape[0]
        pr = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        need = kkm_assign_workspace_bytes(model, n, pr)
        ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
        if labels is None:
            labels = torch.empty(n, dtype=torch.int32, device=X.device)
        if want_gap and gap is None:
            gap = torch.empty(n, dtype=torch.float32, device=X.device)
        _check(lib().kkm_assign(model.ptr, ct.c_void_p(X.data_ptr()), n, _dtype_code(X), pr,
                                ct.c_void_p(ws.data_ptr()), ws.numel(), ct.c_void_p(_stream_ptr(os_.s)),
                                ct.c_void_p(labels.data_ptr()),
                                ct.c_void_p(gap.data_ptr()) if gap is not None else None))
    return (labels, gap) if want_gap else labels


def kkm_assign_noalloc(model: Model, X, labels, gap=None, precision="fp32", stream=None):
    """kkm_assign into caller-given outputs (int32 labels, optional float32 gaps) with the library's fixed
    scratch: the call allocates nothing (X must already be contiguous).  Calls overlapping on one GPU
    race on that scratch."""
    if not X.is_contiguous():
        raise ValueError("X must be contiguous (the call allocates nothing, not even a contiguous copy)")
    pr = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    with _OnStream(stream) as os_:
        os_.use(X, labels, gap)
        _check(lib().kkm_assign_noalloc(model.ptr, ct.c_void_p(X.data_ptr()), X.shape[0], _dtype_code(X), pr,
                                        ct.c_void_p(_stream_ptr(os_.s)), ct.c_void_p(labels.data_ptr()),
                                        ct.c_void_p(gap.data_ptr()) if gap is not None else None))
    return labels


def kkm_cost(model: Model, X, precision="fp32", workspace=None, stream=None) -> float:
    """Eq. 1 on the rows of X (FP64 sum in a fixed order)."""
    with _OnStream(stream) as os_:
        os_.use(X, workspace)
        X = X.contiguous()
        n = X.shape[0]
        pr = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        need = kkm_assign_workspace_bytes(model, n, pr)
        ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
        out = ct.c_double()
        _check(lib().kkm_cost(model.ptr, ct.c_void_p(X.data_ptr()), n, _dtype_code(X), pr,
                              ct.c_void_p(ws.data_ptr()), ws.numel(), ct.c_void_p(_stream_ptr(os_.s)), ct.byref(out)))
    return out.value


def kkm_kernel_block(X, Y, kernel="rbf", sigma=1.0, n_atoms=0, workspace=None, stream=None):
    """K(x_i, y_j) in FP64 for the rows of X and Y (device tensors of one dtype): an nx x ny tensor."""
    import torch
    if X.dtype != Y.dtype or X.shape[1] != Y.shape[1]:
        raise ValueError("X and Y need the same dtype and row length")
    k = _kernel(kernel, sigma, n_atoms)
    with _OnStream(stream) as os_:
        os_.use(X, Y, workspace)
        X, Y = X.contiguous(), Y.contiguous()
        nx, d = X.shape
        ny = Y.shape[0]
        dt = _dtype_code(X)
        need = int(lib().kkm_kernel_block_workspace_bytes(ct.byref(k), nx, ny, d, dt))
        ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
        K = torch.empty((nx, ny), dtype=torch.float64, device=X.device)
        _check(lib().kkm_kernel_block(ct.byref(k), ct.c_void_p(X.data_ptr()), nx, ct.c_void_p(Y.data_ptr()), ny, d, dt,
                                      ct.c_void_p(ws.data_ptr()), ws.numel(), ct.c_void_p(_stream_ptr(os_.s)),
                                      ct.c_void_p(K.data_ptr())))
    return K


def kkm_landmark_count(n: int, s: float) -> int:
    return int(lib().kkm_landmark_count(int(n), float(s)))


def kkm_draw_landmarks(seed: int, batch: int, n: int, s: float) -> np.ndarray:
    out = np.zeros(max(1, kkm_landmark_count(n, s)), dtype=np.int64)
    _check(lib().kkm_draw_landmarks(int(seed), int(batch), int(n), float(s), _i64p(out)))
    return out


def kkm_draw_kmpp_uniforms(seed: int, C: int) -> np.ndarray:
    out = np.zeros(C, dtype=np.float64)
    _check(lib().kkm_draw_kmpp_uniforms(int(seed), int(C), _f64p(out)))
    return out


def kkm_draw_init_labels(seed: int, n: int, C: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int32)
    _check(lib().kkm_draw_init_labels(int(seed), int(n), int(C), _i32p(out)))
    return out


def kkm_version() -> str:
    return lib().kkm_version().decode()
