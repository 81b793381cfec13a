"""Thin ctypes binding of the C-ABI in ``include/skel.h``.

Argument marshalling only: every stage of every skeleton runs in the HIP
library ``libskel.so``.  PyTorch supplies device memory and streams.  If the
library is missing, every entry point raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libskel.so")

# --------------------------------------------------------------- constants
OK, EINVAL, ESHAPE, ETYPE, ENOMEM, EDEVICE, EUNSUPPORTED = range(7)
U8, U32, U64, F32, F64 = range(5)
OP_NOISE, OP_SOLARISE, OP_MIRROR, OP_BLUR5, OP_SAXPY, OP_NBODY_FORCE, OP_LEAPFROG, OP_FFT, OP_IFFT, OP_SEGMENT = range(10)
FFT_POINTS = 65536
RED_HIST256_SUM, RED_SUM = 0, 1
FUSE_AUTO, FUSE_OFF, FUSE_ON, FUSE_MASK = -1, 0, 1, 2
IMMUTABLE, COPY = 1, 2
CMP_GT, CMP_GE, CMP_LT, CMP_LE = range(4)
CMP_BY_NAME = {">": CMP_GT, ">=": CMP_GE, "<": CMP_LT, "<=": CMP_LE}
COND_VALUE, COND_DELTA = 0, 1
COND_BY_NAME = {"value": COND_VALUE, "delta": COND_DELTA}

OP_BY_NAME = {"noise": OP_NOISE, "solarise": OP_SOLARISE, "mirror": OP_MIRROR, "blur5": OP_BLUR5,
              "saxpy": OP_SAXPY, "nbody_force": OP_NBODY_FORCE, "leapfrog": OP_LEAPFROG, "fft": OP_FFT,
              "ifft": OP_IFFT, "segment": OP_SEGMENT}
STATUS_NAMES = {OK: "SKEL_OK", EINVAL: "SKEL_EINVAL", ESHAPE: "SKEL_ESHAPE", ETYPE: "SKEL_ETYPE",
                ENOMEM: "SKEL_ENOMEM", EDEVICE: "SKEL_EDEVICE", EUNSUPPORTED: "SKEL_EUNSUPPORTED"}


class SkelError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Buffer(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("ndim", ctypes.c_int32),
                ("shape", ctypes.c_int64 * 4), ("stride_bytes", ctypes.c_int64 * 4),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Params(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint32), ("a", ctypes.c_float), ("eps", ctypes.c_float),
                ("G", ctypes.c_float), ("dt", ctypes.c_float), ("lo", ctypes.c_uint32), ("hi", ctypes.c_uint32)]


class LoopState(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("carried_mask", ctypes.c_uint32),
                ("global_sync", ctypes.c_int32)]


class LoopCond(ctypes.Structure):
    _fields_ = [("channel", ctypes.c_int32), ("cmp", ctypes.c_int32), ("threshold", ctypes.c_uint64),
                ("check_every", ctypes.c_int32), ("kind", ctypes.c_int32)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("fusion", ctypes.c_int32), ("split_mask", ctypes.c_uint32), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("wg", ctypes.c_int32), ("ept", ctypes.c_int32),
                ("select", ctypes.c_int32), ("variant", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_node_p = ctypes.c_void_p
_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "skel_plan_opts_default": (None, [ctypes.POINTER(PlanOpts)]),
    "skel_init": (ctypes.c_int32, [ctypes.c_int32]),
    "skel_map": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(Params), ctypes.POINTER(_node_p)]),
    "skel_pipeline": (ctypes.c_int32, [ctypes.POINTER(_node_p), ctypes.c_int32, ctypes.POINTER(_node_p)]),
    "skel_mapreduce": (ctypes.c_int32, [_node_p, ctypes.c_int32, ctypes.POINTER(_node_p)]),
    "skel_loop": (ctypes.c_int32, [_node_p, ctypes.POINTER(LoopState), ctypes.POINTER(_node_p)]),
    "skel_loop_while": (ctypes.c_int32, [_node_p, ctypes.POINTER(LoopState), ctypes.POINTER(LoopCond),
                                         ctypes.POINTER(_node_p)]),
    "skel_node_release": (ctypes.c_int32, [_node_p]),
    "skel_plan_compile": (ctypes.c_int32, [_node_p, ctypes.POINTER(Buffer), ctypes.c_int32,
                                           ctypes.POINTER(PlanOpts), ctypes.POINTER(_vp)]),
    "skel_plan_run": (ctypes.c_int32, [_vp, ctypes.POINTER(Buffer), ctypes.c_int32, _vp]),
    "skel_plan_run_event": (ctypes.c_int32, [_vp, ctypes.POINTER(Buffer), ctypes.c_int32, _vp, _vp]),
    "skel_plan_run_noalloc": (ctypes.c_int32, [_vp, ctypes.POINTER(Buffer), ctypes.c_int32, _vp]),
    "skel_batch_run": (ctypes.c_int32, [_vp, ctypes.POINTER(Buffer), ctypes.c_int32, ctypes.c_int32, _vp]),
    "skel_plan_describe": (ctypes.c_int32, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "skel_plan_destroy": (ctypes.c_int32, [_vp]),
    "skel_plan_kernel_events": (ctypes.c_int32, [_vp, ctypes.c_int32, _vp, _vp]),
    "skel_sync": (ctypes.c_int32, [_vp]),
    "skel_last_error": (ctypes.c_char_p, []),
    "skel_tune": (ctypes.c_int32, [_node_p, ctypes.POINTER(Buffer), ctypes.c_int32, ctypes.c_char_p,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(PlanOpts),
                                   ctypes.POINTER(ctypes.c_double)]),
    "skel_tune_pruned": (ctypes.c_int32, [_node_p, ctypes.POINTER(Buffer), ctypes.c_int32, ctypes.c_char_p,
                                          ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(PlanOpts), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int32)]),
    "skel_time_config": (ctypes.c_int32, [_node_p, ctypes.POINTER(Buffer), ctypes.c_int32, ctypes.POINTER(PlanOpts),
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]),
    "skel_tune_batch": (ctypes.c_int32, [_node_p, ctypes.POINTER(Buffer), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_char_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                         ctypes.POINTER(PlanOpts), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int32)]),
    "skel_config_count": (ctypes.c_int32, [_node_p, ctypes.POINTER(Buffer), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32)]),
    "skel_feature_count": (ctypes.c_int32, []),
    "skel_features": (ctypes.c_int32, [_node_p, ctypes.POINTER(Buffer), ctypes.c_int32,
                                       ctypes.POINTER(PlanOpts), ctypes.POINTER(ctypes.c_float)]),
    "skel_mlp_param_count": (ctypes.c_int32, []),
    "skel_mlp_forward": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, _vp]),
    "skel_mlp_grad": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "skel_mlp_adam": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, _vp]),
    "skel_cost_train": (ctypes.c_int32, [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "skel_cost_select": (ctypes.c_int32, [_node_p, ctypes.POINTER(Buffer), ctypes.c_int32, ctypes.c_char_p,
                                          ctypes.POINTER(PlanOpts)]),
    "skel_cost_rank": (ctypes.c_int32, [_node_p, ctypes.POINTER(Buffer), ctypes.c_int32, ctypes.c_char_p,
                                        ctypes.c_int32, ctypes.POINTER(PlanOpts), ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_int32)]),
}
EXPORTS = tuple(_SIGS)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1510_06585_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != OK:
        raise SkelError(st, lib().skel_last_error().decode(errors="replace"))


# ------------------------------------------------------------------ buffers
def _torch_dtype_code(t):
    import torch
    m = {torch.uint8: U8, torch.float32: F32, torch.float64: F64, torch.int32: U32, torch.int64: U64}
    for name, code in (("uint32", U32), ("uint64", U64)):
        if hasattr(torch, name):
            m[getattr(torch, name)] = code
    if t.dtype not in m:
        raise TypeError(f"unsupported tensor dtype {t.dtype}")
    return m[t.dtype]


def buffer(t, flags: int = 0) -> Buffer:
    """skel_buffer describing a dense torch tensor (int32/int64 tensors stand for
    uint32/uint64 data)."""
    if t.dim() < 1 or t.dim() > 4:
        raise ValueError("buffers have 1..4 dims")
    if not t.is_contiguous():
        raise ValueError("buffers must be contiguous")
    b = Buffer()
    b.data = t.data_ptr() if t.numel() else None
    b.dtype = _torch_dtype_code(t)
    b.ndim = t.dim()
    for d in range(t.dim()):
        b.shape[d] = t.shape[d]
        b.stride_bytes[d] = t.stride(d) * t.element_size()
    b.flags = flags
    return b


def proto(shape, dtype: int) -> Buffer:
    """Shape-only prototype buffer for plan compilation."""
    b = Buffer()
    b.data = None
    b.dtype = dtype
    b.ndim = len(shape)
    for d, s in enumerate(shape):
        b.shape[d] = s
    return b


class Bound:
    """Pre-marshalled argument list (skips per-call conversion in hot loops).
    Holds references to the tensors so they outlive the bound arguments."""

    def __init__(self, bufs):
        self.tensors = list(bufs)
        self.arr, self.n = _buf_array(self.tensors)


def bind(bufs) -> Bound:
    return Bound(bufs)


class BoundBatch:
    """Pre-marshalled request list for Plan.batch_run (one argument list per
    request, flattened request by request)."""

    def __init__(self, reqs):
        reqs = list(reqs)
        self.per = len(reqs[0]) if reqs else 0
        self.nreq = len(reqs)
        self.tensors = [a for r in reqs for a in r]
        self.arr, _ = _buf_array(self.tensors)


def bind_batch(reqs) -> BoundBatch:
    return BoundBatch(reqs)


def _buf_array(bufs):
    if isinstance(bufs, Bound):
        return bufs.arr, bufs.n
    arr = (Buffer * max(1, len(bufs)))()
    for i, b in enumerate(bufs):
        arr[i] = b if isinstance(b, Buffer) else buffer(b)
    return arr, len(bufs)


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# -------------------------------------------------------------------- nodes
class Node:
    """Owning handle of an SCT node."""

    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.skel_node_release(h)


def Map(op, seed: int = 0, a: float = 0.0, eps: float = 0.0, G: float = 0.0, dt: float = 0.0, lo: int = 0,
        hi: int = 0) -> Node:
    if isinstance(op, str):
        op = OP_BY_NAME[op]
    p = Params(seed & 0xFFFFFFFF, a, eps, G, dt, lo, hi)
    h = _node_p()
    _check(lib().skel_map(op, ctypes.byref(p), ctypes.byref(h)))
    return Node(h.value)


def Pipeline(*stages: Node) -> Node:
    arr = (_node_p * len(stages))(*[s.handle for s in stages])
    h = _node_p()
    _check(lib().skel_pipeline(arr, len(stages), ctypes.byref(h)))
    return Node(h.value)


def MapReduce(m: Node, red: int = RED_HIST256_SUM) -> Node:
    h = _node_p()
    _check(lib().skel_mapreduce(m.handle, red, ctypes.byref(h)))
    return Node(h.value)


def Loop(body: Node, iterations: int, carried_mask: int = 0, global_sync: int = 0) -> Node:
    st = LoopState(iterations, carried_mask, global_sync)
    h = _node_p()
    _check(lib().skel_loop(body.handle, ctypes.byref(st), ctypes.byref(h)))
    return Node(h.value)


def LoopWhile(body: Node, max_iterations: int, channel: int, cmp, threshold: int, check_every: int = 0,
              carried_mask: int = 0, global_sync: int = 0, kind="value") -> Node:
    """While Loop over an image MapReduce body: repeat while sum[channel] <cmp>
    threshold (kind "value") or |sum[channel] - previous sum[channel]| <cmp>
    threshold (kind "delta"), cmp: CMP_* or one of ">", ">=", "<", "<=", at
    most max_iterations times; the condition is evaluated on the device.
    check_every < 0 makes runs fully asynchronous; carried_mask bits on the
    reduce outputs merge them by addition across iterations."""
    st = LoopState(max_iterations, carried_mask, global_sync)
    k = COND_BY_NAME.get(kind, kind)
    c = LoopCond(channel, CMP_BY_NAME.get(cmp, cmp), threshold, check_every, k)
    h = _node_p()
    _check(lib().skel_loop_while(body.handle, ctypes.byref(st), ctypes.byref(c), ctypes.byref(h)))
    return Node(h.value)


def opts(**kw) -> PlanOpts:
    o = PlanOpts()
    lib().skel_plan_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _opts(o):
    if o is None:
        return None
    if isinstance(o, dict):
        o = opts(**o)
    return ctypes.byref(o)


# -------------------------------------------------------------------- plans
class Plan:
    """A compiled, shape-specialised plan (skel_plan)."""

    def __init__(self, root: Node, protos, options=None):
        arr, n = _buf_array(protos)
        h = _vp()
        _check(lib().skel_plan_compile(root.handle, arr, n, _opts(options), ctypes.byref(h)))
        self._h = h.value
        self.root = root

    @property
    def handle(self):
        return self._h

    def run(self, args, stream=None):
        arr, n = _buf_array(args)
        _check(lib().skel_plan_run(self._h, arr, n, _stream_handle(stream)))

    def run_noalloc(self, args, stream=None):
        """skel_plan_run with the plan's scratch in the library's static
        per-GPU array (no allocation by the call)."""
        arr, n = _buf_array(args)
        _check(lib().skel_plan_run_noalloc(self._h, arr, n, _stream_handle(stream)))

    def run_event(self, args, event, stream=None):
        arr, n = _buf_array(args)
        ev = ctypes.c_void_p(event.cuda_event) if event is not None else None
        _check(lib().skel_plan_run_event(self._h, arr, n, _stream_handle(stream), ev))

    def batch_run(self, reqs, stream=None):
        """reqs: a list of per-request argument lists, or a BoundBatch."""
        if not isinstance(reqs, BoundBatch):
            reqs = BoundBatch(reqs)
        _check(lib().skel_batch_run(self._h, reqs.arr, reqs.per, reqs.nreq, _stream_handle(stream)))

    def describe(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().skel_plan_describe(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def kernel_events(self, kernel: int, start=None, end=None):
        """Record hipEvent_t `start`/`end` (raw handles, or objects with a
        `cuda_event` handle) around kernel `kernel` of every subsequent run;
        None clears the hook."""
        def h(e):
            if e is None:
                return None
            return ctypes.c_void_p(e if isinstance(e, int) else e.cuda_event)
        _check(lib().skel_plan_kernel_events(self._h, kernel if start is not None else -1, h(start), h(end)))

    def destroy(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.skel_plan_destroy(h)

    def __del__(self):
        self.destroy()


def sync(stream=None):
    _check(lib().skel_sync(_stream_handle(stream)))


def init(device: int = 0):
    _check(lib().skel_init(device))


# ------------------------------------------------------- tuning / cost model
def tune(root: Node, args, db_path: str | None = None, reps: int = 10, max_configs: int = 0,
         sample_seed: int = 0):
    arr, n = _buf_array(args)
    best = PlanOpts()
    us = ctypes.c_double()
    _check(lib().skel_tune(root.handle, arr, n, db_path.encode() if db_path else None, reps, max_configs,
                           sample_seed, ctypes.byref(best), ctypes.byref(us)))
    return best.as_dict(), us.value


def time_config(root: Node, args, options=None, reps: int = 10):
    """Median and minimum microseconds of one configuration (None: the default
    plan) under the tuner's timing protocol (skel_time_config)."""
    arr, n = _buf_array(args)
    med = ctypes.c_double()
    mn = ctypes.c_double()
    _check(lib().skel_time_config(root.handle, arr, n, _opts(options), reps, ctypes.byref(med), ctypes.byref(mn)))
    return med.value, mn.value


def tune_batch(root: Node, reqs, db_path: str | None = None, reps: int = 10, pruned: bool = False,
               precision_us: float = 0.0):
    """Tunes tile height and work-group size of a batched run of `reqs` (a list
    of per-request argument lists, or a BoundBatch) with skel_tune_batch;
    returns (options, median us, number of points timed)."""
    if not isinstance(reqs, BoundBatch):
        reqs = BoundBatch(reqs)
    best = PlanOpts()
    us = ctypes.c_double()
    timed = ctypes.c_int32()
    _check(lib().skel_tune_batch(root.handle, reqs.arr, reqs.per, reqs.nreq,
                                 db_path.encode() if db_path else None, reps, 1 if pruned else 0, precision_us,
                                 ctypes.byref(best), ctypes.byref(us), ctypes.byref(timed)))
    return best.as_dict(), us.value, timed.value


def tune_pruned(root: Node, args, db_path: str | None = None, reps: int = 10, precision_us: float = 0.0,
                occ_threshold: float = 0.0):
    """Algorithm-1 style search (skel_tune_pruned); returns (options, median us,
    number of configurations timed)."""
    arr, n = _buf_array(args)
    best = PlanOpts()
    us = ctypes.c_double()
    timed = ctypes.c_int32()
    _check(lib().skel_tune_pruned(root.handle, arr, n, db_path.encode() if db_path else None, reps,
                                  precision_us, occ_threshold, ctypes.byref(best), ctypes.byref(us),
                                  ctypes.byref(timed)))
    return best.as_dict(), us.value, timed.value


def config_count(root: Node, protos) -> int:
    arr, n = _buf_array(protos)
    c = ctypes.c_int32()
    _check(lib().skel_config_count(root.handle, arr, n, ctypes.byref(c)))
    return c.value


def features(root: Node, protos, options=None) -> np.ndarray:
    arr, n = _buf_array(protos)
    f = (ctypes.c_float * lib().skel_feature_count())()
    _check(lib().skel_features(root.handle, arr, n, _opts(options), f))
    return np.array(f, dtype=np.float32)


def mlp_param_count() -> int:
    return int(lib().skel_mlp_param_count())


def mlp_forward(params, X, y, stream=None):
    _check(lib().skel_mlp_forward(params.data_ptr(), X.data_ptr(), X.shape[0], y.data_ptr(),
                                  _stream_handle(stream)))


def mlp_grad(params, X, t, grad, loss, stream=None):
    _check(lib().skel_mlp_grad(params.data_ptr(), X.data_ptr(), t.data_ptr(), X.shape[0], grad.data_ptr(),
                               loss.data_ptr(), _stream_handle(stream)))


def mlp_adam(params, grad, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().skel_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), step, lr, beta1,
                               beta2, eps, _stream_handle(stream)))


def cost_train(db_path: str, weights_out: str, epochs: int, seed: int = 0, init=None) -> float:
    loss = ctypes.c_float()
    ip = None
    if init is not None:
        a = np.ascontiguousarray(init, dtype=np.float32)
        ip = a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    _check(lib().skel_cost_train(db_path.encode(), weights_out.encode(), epochs, seed, ip, ctypes.byref(loss)))
    return loss.value


def cost_select(root: Node, protos, weights: str) -> dict:
    arr, n = _buf_array(protos)
    o = PlanOpts()
    _check(lib().skel_cost_select(root.handle, arr, n, weights.encode(), ctypes.byref(o)))
    return o.as_dict()


def cost_rank(root: Node, protos, weights: str, k: int):
    """The k configurations with the lowest predicted runtime (skel_cost_rank):
    a list of (options, predicted microseconds), best first."""
    arr, n = _buf_array(protos)
    out = (PlanOpts * max(1, k))()
    pred = (ctypes.c_float * max(1, k))()
    cnt = ctypes.c_int32()
    _check(lib().skel_cost_rank(root.handle, arr, n, weights.encode(), k, out, pred, ctypes.byref(cnt)))
    return [(out[i].as_dict(), float(pred[i])) for i in range(cnt.value)]


# --------------------------------------------------------------- helpers
def image_chain(stages, reduce=None) -> Node:
    """SCT for a list of (name, params) image/vector stages, optionally wrapped in
    a MapReduce (reduce = "hist_sum" or "sum")."""
    nodes = []
    for name, prm in stages:
        prm = prm or {}
        nodes.append(Map(OP_BY_NAME[name], seed=prm.get("seed", 0), a=prm.get("a", 0.0), lo=prm.get("lo", 0),
                         hi=prm.get("hi", 0)))
    root = Pipeline(*nodes) if len(nodes) != 1 else nodes[0]
    if reduce is not None:
        root = MapReduce(root, RED_HIST256_SUM if reduce == "hist_sum" else RED_SUM)
    return root


def nbody_loop(iterations: int, eps: float = 1e-2, G: float = 1.0, dt: float = 1e-3) -> Node:
    body = Pipeline(Map(OP_NBODY_FORCE, eps=eps, G=G), Map(OP_LEAPFROG, dt=dt))
    return Loop(body, iterations, carried_mask=0b011, global_sync=1)
