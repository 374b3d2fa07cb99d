"""ctypes binding of ``libslrcount.so`` (declared in ``include/slrcount.h``).

Argument marshalling only: every step of the computation runs in the library's HIP kernels.
PyTorch provides device memory and the current stream.  The library is loaded on first use;
if it is missing or cannot be loaded the call raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslrcount.so")

SLR_OK, SLR_BUDGET = 0, 1
UNDECIDED, UNSAFE, SAFE = 0, 1, 2

# every entry point declared in include/slrcount.h
EXPORTS = ("load_net", "free_net", "load_property", "free_property", "bound_boxes",
           "workspace_size", "count_exact", "count_approx", "sample_violations", "last_error",
           "bound_kernel_variant", "alpha_size", "alpha_tape_size", "bound_boxes_alpha",
           "bound_boxes_backward", "alpha_workspace_size", "alpha_optimize", "batch_create",
           "batch_run", "batch_free", "count_exact_batch", "bound_tile_shape",
           "alpha_state_variant", "count_exact_noalloc", "count_exact_noalloc_max_bytes",
           "stack_workspace_size", "count_exact_stack", "alpha_kernel_variant",
           "batch_create_opts", "load_net_act", "workspace_size_exact", "bound_boxes_relax",
           "bound_tape_size")


class SlrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"slrcount error {code}: {msg}")
        self.code = code


class ExactOpts(C.Structure):
    _fields_ = [("max_depth", C.c_int32), ("max_leaves", C.c_int64), ("chunk", C.c_int32),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stream", C.c_void_p), ("trace_capacity", C.c_int64),
                ("trace_depth", C.POINTER(C.c_int32)), ("trace_path", C.POINTER(C.c_uint64)),
                ("trace_cls", C.POINTER(C.c_int8)), ("timing", C.c_int32),
                ("alpha_steps", C.c_int32), ("alpha_lr", C.c_float),
                ("alpha_min_depth", C.c_int32), ("alpha_chunk", C.c_int32),
                ("alpha_select", C.c_float), ("split_layers", C.c_int32),
                ("trace_dim", C.POINTER(C.c_int8)), ("relax", C.c_int32)]


RELAX = {"one": 0, "two": 1}


def _relax(relax) -> int:
    if relax not in RELAX:
        raise ValueError(f"relax must be one of {sorted(RELAX)}, not {relax!r}")
    return RELAX[relax]


class CountResult(C.Structure):
    _fields_ = [("unsafe", C.c_double), ("safe", C.c_double), ("undecided", C.c_double),
                ("n_unsafe", C.c_int64), ("n_safe", C.c_int64), ("n_undecided", C.c_int64),
                ("n_boxes_bounded", C.c_int64), ("n_recheck64", C.c_int64),
                ("depth_reached", C.c_int32), ("status", C.c_int32), ("seconds", C.c_double),
                ("trace_count", C.c_int64), ("bound_ms", C.c_double),
                ("bound_launches", C.c_int64), ("n_alpha_boxes", C.c_int64),
                ("n_alpha_decided", C.c_int64), ("alpha_ms", C.c_double),
                ("split_ms", C.c_double), ("split_bytes", C.c_int64)]


class StackOpts(C.Structure):
    _fields_ = [("max_depth", C.c_int32), ("chunk", C.c_int32), ("max_boxes", C.c_int64),
                ("device_boxes", C.c_int64), ("host_spill", C.c_void_p),
                ("host_spill_bytes", C.c_size_t), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("stream", C.c_void_p),
                ("trace_capacity", C.c_int64), ("trace_depth", C.POINTER(C.c_int32)),
                ("trace_path", C.POINTER(C.c_uint64)), ("trace_cls", C.POINTER(C.c_int8))]


class BatchOpts(C.Structure):
    _fields_ = [("use_graph", C.c_int32), ("alpha_steps", C.c_int32), ("alpha_lr", C.c_float),
                ("alpha_min_depth", C.c_int32), ("alpha_select", C.c_float),
                ("alpha_chunk", C.c_int32)]


class AlphaOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("raw", C.c_int32)]


class ApproxOpts(C.Structure):
    _fields_ = [("trials", C.c_int32), ("samples", C.c_int32), ("confidence", C.c_double),
                ("seed", C.c_uint64), ("max_splits", C.c_int32), ("grid_bits", C.c_int32),
                ("resolve_tol", C.c_double), ("concurrency", C.c_int32), ("leaf", ExactOpts)]


class ApproxResult(C.Structure):
    _fields_ = [("lower_bound", C.c_double), ("estimate", C.c_double * 64),
                ("splits", C.c_int32 * 64), ("trials", C.c_int32), ("seconds", C.c_double)]


_LIB = None


def lib() -> C.CDLL:
    """Load the HIP library (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        # torch first: it brings its own HIP runtime, and the library must bind to that same
        # runtime (loaded the other way round, torch later finds no GPU)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2312_05890_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.load_net.argtypes = [i32, C.POINTER(C.c_int32), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
        L.load_net.restype = C.c_int
        L.load_net_act.argtypes = [i32, C.POINTER(C.c_int32), C.POINTER(vp), C.POINTER(vp), i32,
                                   C.POINTER(vp)]
        L.load_net_act.restype = C.c_int
        L.free_net.argtypes = [vp]
        L.free_net.restype = None
        L.load_property.argtypes = [vp, i32, vp, vp, C.POINTER(vp)]
        L.load_property.restype = C.c_int
        L.free_property.argtypes = [vp]
        L.free_property.restype = None
        L.bound_boxes.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, i32, vp]
        L.bound_boxes.restype = C.c_int
        L.workspace_size.argtypes = [vp, vp, i64, i32, i32, C.POINTER(C.c_size_t)]
        L.workspace_size.restype = C.c_int
        L.workspace_size_exact.argtypes = [vp, vp, C.POINTER(ExactOpts), C.POINTER(C.c_size_t)]
        L.workspace_size_exact.restype = C.c_int
        L.count_exact.argtypes = [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(ExactOpts), C.POINTER(CountResult)]
        L.count_exact.restype = C.c_int
        L.count_exact_noalloc.argtypes = [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.POINTER(ExactOpts), C.POINTER(CountResult)]
        L.count_exact_noalloc.restype = C.c_int
        L.count_exact_noalloc_max_bytes.argtypes = []
        L.count_exact_noalloc_max_bytes.restype = C.c_size_t
        L.stack_workspace_size.argtypes = [vp, vp, C.POINTER(StackOpts), C.POINTER(C.c_size_t)]
        L.stack_workspace_size.restype = C.c_int
        L.count_exact_stack.argtypes = [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(StackOpts), C.POINTER(CountResult)]
        L.count_exact_stack.restype = C.c_int
        L.count_approx.argtypes = [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(ApproxOpts), C.POINTER(ApproxResult)]
        L.count_approx.restype = C.c_int
        L.sample_violations.argtypes = [vp, vp, i64, vp, vp, vp]
        L.sample_violations.restype = C.c_int
        L.bound_kernel_variant.argtypes = [i32]
        L.bound_kernel_variant.restype = C.c_int
        sz = C.POINTER(C.c_size_t)
        L.alpha_size.argtypes = [vp, C.POINTER(C.c_int64)]
        L.alpha_size.restype = C.c_int
        L.alpha_tape_size.argtypes = [vp, vp, i64, sz]
        L.alpha_tape_size.restype = C.c_int
        L.alpha_workspace_size.argtypes = [vp, vp, i64, sz]
        L.alpha_workspace_size.restype = C.c_int
        L.bound_boxes_alpha.argtypes = [vp, vp, i64, vp, vp, vp, i32, vp, vp, vp, i32, vp,
                                        C.c_size_t, vp]
        L.bound_boxes_alpha.restype = C.c_int
        L.bound_boxes_relax.argtypes = [vp, vp, i64, vp, vp, i32, vp, vp, vp, i32, vp,
                                        C.c_size_t, vp]
        L.bound_boxes_relax.restype = C.c_int
        L.bound_tape_size.argtypes = [vp, vp, i64, sz]
        L.bound_tape_size.restype = C.c_int
        L.bound_boxes_backward.argtypes = [vp, vp, i64, vp, vp, C.c_size_t, vp, vp, vp, i32, vp]
        L.bound_boxes_backward.restype = C.c_int
        L.alpha_optimize.argtypes = [vp, vp, i64, vp, vp, C.POINTER(AlphaOpts), vp, vp, vp, vp,
                                     vp, C.c_size_t, vp]
        L.alpha_optimize.restype = C.c_int
        L.batch_create.argtypes = [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                   C.POINTER(vp), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                   i32, C.POINTER(vp)]
        L.batch_create.restype = C.c_int
        L.batch_create_opts.argtypes = [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                        C.POINTER(vp), C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                        C.POINTER(BatchOpts), C.POINTER(vp)]
        L.batch_create_opts.restype = C.c_int
        L.batch_run.argtypes = [vp, vp, C.POINTER(CountResult)]
        L.batch_run.restype = C.c_int
        L.batch_free.argtypes = [vp]
        L.batch_free.restype = None
        L.count_exact_batch.argtypes = [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                        C.POINTER(vp), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int64), vp, C.POINTER(CountResult)]
        L.count_exact_batch.restype = C.c_int
        L.alpha_kernel_variant.argtypes = [i32]
        L.alpha_kernel_variant.restype = C.c_int
        L.alpha_state_variant.argtypes = [i32]
        L.alpha_state_variant.restype = C.c_int
        L.bound_tile_shape.argtypes = [i32, i32, i32, i32, i32]
        L.bound_tile_shape.restype = C.c_int
        L.last_error.argtypes = []
        L.last_error.restype = C.c_char_p
        _LIB = L
    return _LIB


def last_error() -> str:
    return lib().last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise SlrError(rc, last_error())
    return rc


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


ACTIVATIONS = {"relu": 0, "tanh": 1, "sigmoid": 2}


class Net:
    """A network resident on the device (``load_net_act``): ReLU hidden layers, or tanh /
    sigmoid when ``act`` (or the ``act`` attribute of ``layers``) says so."""

    def __init__(self, layers: Sequence[Tuple[np.ndarray, np.ndarray]], act: Optional[str] = None):
        if act is None:
            act = getattr(layers, "act", "relu")
        if act not in ACTIVATIONS:
            raise ValueError(f"unknown activation {act!r}")
        self.act = act
        L = lib()
        self._keep = [(np.ascontiguousarray(W, np.float32), np.ascontiguousarray(b, np.float32))
                      for W, b in layers]
        sizes = [self._keep[0][0].shape[1]] + [W.shape[0] for W, _ in self._keep]
        for (W, b), n_in, n_out in zip(self._keep, sizes[:-1], sizes[1:]):
            if W.shape != (n_out, n_in) or b.shape != (n_out,):
                raise ValueError("layer shapes do not chain")
        self.sizes = sizes
        self.d = sizes[0]
        n = len(self._keep)
        arr_s = (C.c_int32 * (n + 1))(*sizes)
        arr_w = (C.c_void_p * n)(*[W.ctypes.data for W, _ in self._keep])
        arr_b = (C.c_void_p * n)(*[b.ctypes.data for _, b in self._keep])
        h = C.c_void_p()
        _check(L.load_net_act(n, arr_s, arr_w, arr_b, ACTIVATIONS[act], C.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.free_net(self.handle)
            self.handle = None


class Property:
    """Unsafe set {y : C y + d > 0 on every row} bound to a network (``load_property``)."""

    def __init__(self, net: Net, Cm, dv):
        self.net = net
        self.C = np.ascontiguousarray(np.atleast_2d(Cm), np.float32)
        self.dv = np.ascontiguousarray(np.ravel(dv), np.float32)
        self.rows = self.C.shape[0]
        if self.C.shape[1] != net.sizes[-1] or self.dv.shape[0] != self.rows:
            raise ValueError("property shape does not match the network output")
        h = C.c_void_p()
        _check(lib().load_property(net.handle, self.rows, self.C.ctypes.data,
                                   self.dv.ctypes.data, C.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.free_property(self.handle)
            self.handle = None


def load_net(layers) -> Net:
    return Net(layers)


def load_property(net: Net, Cm, dv) -> Property:
    return Property(net, Cm, dv)


def bound_boxes(net: Net, prop: Property, lo, hi, g_lo=None, g_hi=None, cls=None,
                raw: bool = False, stream=None, want_cls: bool = True):
    """Bounds of every property row over each box; ``lo``/``hi`` are device float32 [n, d]."""
    import torch
    n = lo.shape[0]
    assert lo.is_cuda and hi.is_cuda and lo.dtype == torch.float32 and hi.dtype == torch.float32
    assert lo.is_contiguous() and hi.is_contiguous() and tuple(lo.shape) == (n, net.d)
    assert tuple(hi.shape) == (n, net.d)
    if g_lo is None:
        g_lo = torch.empty((n, prop.rows), dtype=torch.float32, device=lo.device)
    if g_hi is None:
        g_hi = torch.empty((n, prop.rows), dtype=torch.float32, device=lo.device)
    if cls is None and want_cls:
        cls = torch.empty((n,), dtype=torch.int8, device=lo.device)
    _check(lib().bound_boxes(net.handle, prop.handle, n, lo.data_ptr(), hi.data_ptr(),
                             g_lo.data_ptr(), g_hi.data_ptr(),
                             cls.data_ptr() if cls is not None else None, int(bool(raw)),
                             _stream(stream)))
    return g_lo, g_hi, cls


def bound_kernel_variant(variant: int) -> None:
    """0 automatic, 1 LDS-staged, 2 register-resident, 3 tape-state (see include/slrcount.h)."""
    _check(lib().bound_kernel_variant(int(variant)))


def bound_tile_shape(d: int, mt_max: int, nt: int, uw: int, nw: int) -> None:
    """Tile shape of the LDS-staged bound kernel for a (d class, mt_max); nt = 0 = default."""
    _check(lib().bound_tile_shape(int(d), int(mt_max), int(nt), int(uw), int(nw)))
    if nt == 0:
        _SHAPES.pop((int(d), int(mt_max)), None)
    else:
        _SHAPES[(int(d), int(mt_max))] = (int(nt), int(uw), int(nw))


_SHAPES = {}


def current_tile_shape(sizes):
    """(nt, uw, nw) last installed with bound_tile_shape for this network shape, else the
    library default for its hidden tiles."""
    mt = max((w + 15) // 16 for w in sizes[1:-1])
    got = _SHAPES.get((sizes[0], mt))
    if got:
        return got
    return (4, 1, 4) if mt <= 1 else (2, 1, 4) if mt == 2 else (1, 1, 4) if mt <= 4 else \
        (1, 2, 4) if mt <= 8 else (1, 4, 4)


def workspace_size(net: Net, prop: Property, max_leaves: int, samples: int = 0,
                   alpha_chunk: int = 0) -> int:
    out = C.c_size_t()
    _check(lib().workspace_size(net.handle, prop.handle, int(max_leaves), int(samples),
                                int(alpha_chunk), C.byref(out)))
    return out.value


def _exact_opts(net, prop, max_depth, max_leaves, chunk, workspace, stream, samples,
                trace_capacity=0, timing=False, alpha_steps=0, alpha_lr=0.0, alpha_min_depth=0,
                alpha_chunk=0, alpha_select=0.0, split_layers=0, relax="one"):
    import torch
    if alpha_steps > 0 and alpha_chunk <= 0:
        alpha_chunk = 16384
    o = ExactOpts()
    o.max_depth = int(max_depth)
    o.max_leaves = int(max_leaves)
    o.chunk = int(chunk)
    o.alpha_steps = int(alpha_steps)
    o.alpha_chunk = int(alpha_chunk)
    o.relax = _relax(relax)
    need = workspace_size(net, prop, max_leaves, samples, alpha_chunk if alpha_steps > 0 else 0)
    if o.relax:
        out = C.c_size_t()
        _check(lib().workspace_size_exact(net.handle, prop.handle, C.byref(o), C.byref(out)))
        need = max(need, out.value)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    assert workspace.is_cuda
    o.workspace = workspace.data_ptr()
    o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.stream = _stream(stream)
    o.trace_capacity = int(trace_capacity)
    o.timing = int(timing)
    o.alpha_steps = int(alpha_steps)
    o.alpha_lr = float(alpha_lr)
    o.alpha_min_depth = int(alpha_min_depth)
    o.alpha_chunk = int(alpha_chunk)
    o.alpha_select = float(alpha_select)
    o.split_layers = int(split_layers)
    return o, workspace


def count_exact(net: Net, prop: Property, lo, hi, max_depth: int, max_leaves: int,
                chunk: int = 0, workspace=None, stream=None, trace: bool = False,
                trace_capacity: Optional[int] = None, timing: int = 0,
                alpha_steps: int = 0, alpha_lr: float = 0.1, alpha_min_depth: int = 0,
                alpha_chunk: int = 0, alpha_select: float = 0.0, split_layers: int = 0,
                relax: str = "one") -> dict:
    """Alg. 1 on the device; returns the bracket, counts and (optionally) a per-box trace
    (with the side bisected per box in ``trace_dim``).  ``relax``: "one" (Eq. 1) or "two" (one
    ratio per equation, ``slr_exact_opts.relax``).

    ``timing``: bit 0 times the bound-kernel launches (``bound_ms``), bit 1 the split launches
    (``split_ms``, with their algorithmic ``split_bytes``); bit 2 keeps the level-by-level driver
    for the top of the tree as well (same results); True means 1.
    With ``alpha_steps`` > 0 the boxes the plain bounds leave undecided (from depth
    ``alpha_min_depth`` on) are re-bounded with optimized lower slopes before they are split;
    ``alpha_select`` > 0 limits that to boxes whose plain bounds are within that fraction of
    their width from a decision (see ``slr_exact_opts.alpha_select``)."""
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    cap = 0
    if trace:
        cap = int(trace_capacity if trace_capacity is not None else 4 * max_leaves + 64)
    o, ws = _exact_opts(net, prop, max_depth, max_leaves, chunk, workspace, stream, 0, cap, timing,
                        alpha_steps, alpha_lr, alpha_min_depth, alpha_chunk, alpha_select,
                        split_layers, relax)
    if trace:
        t_depth = np.zeros(cap, np.int32)
        t_path = np.zeros(cap, np.uint64)
        t_cls = np.zeros(cap, np.int8)
        t_dim = np.zeros(cap, np.int8)
        o.trace_depth = t_depth.ctypes.data_as(C.POINTER(C.c_int32))
        o.trace_path = t_path.ctypes.data_as(C.POINTER(C.c_uint64))
        o.trace_cls = t_cls.ctypes.data_as(C.POINTER(C.c_int8))
        o.trace_dim = t_dim.ctypes.data_as(C.POINTER(C.c_int8))
    r = CountResult()
    rc = _check(lib().count_exact(net.handle, prop.handle,
                                  lo.ctypes.data_as(C.POINTER(C.c_double)),
                                  hi.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o),
                                  C.byref(r)))
    out = {f: getattr(r, f) for f, _ in CountResult._fields_}
    out["rc"] = rc
    if trace:
        k = r.trace_count
        out["trace_depth"] = t_depth[:k].copy()
        out["trace_path"] = t_path[:k].copy()
        out["trace_cls"] = t_cls[:k].copy()
        out["trace_dim"] = t_dim[:k].copy()
    return out


def count_exact_noalloc(net: Net, prop: Property, lo, hi, max_depth: int, max_leaves: int,
                        chunk: int = 0, stream=None, alpha_steps: int = 0, alpha_lr: float = 0.1,
                        alpha_min_depth: int = 0, alpha_chunk: int = 0,
                        alpha_select: float = 0.0, relax: str = "one") -> dict:
    """``count_exact`` on the library's static workspace (no allocation by the library or here:
    only the host option and result structs)."""
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    if alpha_steps > 0 and alpha_chunk <= 0:
        alpha_chunk = 16384
    o = ExactOpts()
    o.max_depth = int(max_depth)
    o.max_leaves = int(max_leaves)
    o.chunk = int(chunk)
    o.stream = _stream(stream)
    o.alpha_steps = int(alpha_steps)
    o.alpha_lr = float(alpha_lr)
    o.alpha_min_depth = int(alpha_min_depth)
    o.alpha_chunk = int(alpha_chunk)
    o.alpha_select = float(alpha_select)
    o.relax = _relax(relax)
    r = CountResult()
    rc = _check(lib().count_exact_noalloc(net.handle, prop.handle,
                                          lo.ctypes.data_as(C.POINTER(C.c_double)),
                                          hi.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o),
                                          C.byref(r)))
    out = {f: getattr(r, f) for f, _ in CountResult._fields_}
    out["rc"] = rc
    return out


def count_exact_noalloc_max_bytes() -> int:
    return int(lib().count_exact_noalloc_max_bytes())


def _stack_opts(max_depth, chunk, max_boxes, device_boxes, host_spill, stream):
    o = StackOpts()
    o.max_depth = int(max_depth)
    o.chunk = int(chunk)
    o.max_boxes = int(max_boxes)
    o.device_boxes = int(device_boxes)
    if host_spill is not None:
        o.host_spill = host_spill.data_ptr()
        o.host_spill_bytes = host_spill.numel() * host_spill.element_size()
    o.stream = _stream(stream)
    return o


def stack_workspace_size(net: Net, prop: Property, max_depth: int, chunk: int = 0,
                         device_boxes: int = 0) -> int:
    o = _stack_opts(max_depth, chunk, 0, device_boxes, None, None)
    out = C.c_size_t()
    _check(lib().stack_workspace_size(net.handle, prop.handle, C.byref(o), C.byref(out)))
    return out.value


def count_exact_stack(net: Net, prop: Property, lo, hi, max_depth: int, chunk: int = 0,
                      max_boxes: int = 0, device_boxes: int = 0, host_spill=None, workspace=None,
                      stream=None, trace: bool = False, trace_capacity: int = 0) -> dict:
    """Alg. 1 without a leaf budget in bounded memory (depth-first over chunks of the frontier,
    optional spill of the stack's bottom to ``host_spill``, a pinned uint8 tensor); results
    equal ``count_exact`` with the same depth and an unlimited leaf budget."""
    import torch
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    o = _stack_opts(max_depth, chunk, max_boxes, device_boxes, host_spill, stream)
    need = stack_workspace_size(net, prop, max_depth, chunk, device_boxes)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    o.workspace = workspace.data_ptr()
    o.workspace_bytes = workspace.numel() * workspace.element_size()
    if trace:
        cap = int(trace_capacity)
        t_depth = np.zeros(cap, np.int32)
        t_path = np.zeros(cap, np.uint64)
        t_cls = np.zeros(cap, np.int8)
        o.trace_capacity = cap
        o.trace_depth = t_depth.ctypes.data_as(C.POINTER(C.c_int32))
        o.trace_path = t_path.ctypes.data_as(C.POINTER(C.c_uint64))
        o.trace_cls = t_cls.ctypes.data_as(C.POINTER(C.c_int8))
    r = CountResult()
    rc = _check(lib().count_exact_stack(net.handle, prop.handle,
                                        lo.ctypes.data_as(C.POINTER(C.c_double)),
                                        hi.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o),
                                        C.byref(r)))
    out = {f: getattr(r, f) for f, _ in CountResult._fields_}
    out["rc"] = rc
    if trace:
        k = r.trace_count
        out["trace_depth"] = t_depth[:k].copy()
        out["trace_path"] = t_path[:k].copy()
        out["trace_cls"] = t_cls[:k].copy()
    return out


def count_approx(net: Net, prop: Property, lo, hi, trials: int = 20, samples: int = 1000,
                 confidence: float = 0.99, seed: int = 0, max_splits: int = 300,
                 grid_bits: int = 16, resolve_tol: float = 0.01, leaf_depth: int = 48,
                 leaf_leaves: int = 1 << 16, chunk: int = 0, workspace=None,
                 stream=None, concurrency: int = 1) -> dict:
    """CountingProVe with count_exact as the leaf count.  ``concurrency`` must be 0 or 1 (the
    trials run one after another; larger values are rejected, see ``slr_approx_opts``)."""
    lo = np.ascontiguousarray(lo, np.float64)
    hi = np.ascontiguousarray(hi, np.float64)
    leaf, ws = _exact_opts(net, prop, leaf_depth, leaf_leaves, chunk, workspace, stream, samples)
    o = ApproxOpts()
    o.concurrency = int(concurrency)
    o.trials = int(trials)
    o.samples = int(samples)
    o.confidence = float(confidence)
    o.seed = int(seed)
    o.max_splits = int(max_splits)
    o.grid_bits = int(grid_bits)
    o.resolve_tol = float(resolve_tol)
    o.leaf = leaf
    r = ApproxResult()
    _check(lib().count_approx(net.handle, prop.handle, lo.ctypes.data_as(C.POINTER(C.c_double)),
                              hi.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o), C.byref(r)))
    t = r.trials
    return dict(lower_bound=r.lower_bound, estimates=list(r.estimate[:t]),
                splits=list(r.splits[:t]), seconds=r.seconds)


def sample_violations(net: Net, prop: Property, x, viol=None, stream=None):
    import torch
    assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
    n = x.shape[0]
    if viol is None:
        viol = torch.empty((n,), dtype=torch.int8, device=x.device)
    _check(lib().sample_violations(net.handle, prop.handle, n, x.data_ptr(), viol.data_ptr(),
                                   _stream(stream)))
    return viol


# ---------------------------------------------------------------------------------------------
# alpha mode
# ---------------------------------------------------------------------------------------------
def alpha_state_variant(variant: int) -> None:
    """0 automatic, 1 LDS where it fits, 2 global (see include/slrcount.h)."""
    _check(lib().alpha_state_variant(int(variant)))


def alpha_kernel_variant(variant: int) -> None:
    """0: one launch per alpha pass (default); 1: one fused launch per optimization."""
    _check(lib().alpha_kernel_variant(int(variant)))


def alpha_size(net: Net) -> int:
    """Slopes per box: the sum of the hidden widths."""
    out = C.c_int64()
    _check(lib().alpha_size(net.handle, C.byref(out)))
    return out.value


def alpha_tape_size(net: Net, prop: Property, n: int) -> int:
    out = C.c_size_t()
    _check(lib().alpha_tape_size(net.handle, prop.handle, int(n), C.byref(out)))
    return out.value


def alpha_workspace_size(net: Net, prop: Property, n: int) -> int:
    out = C.c_size_t()
    _check(lib().alpha_workspace_size(net.handle, prop.handle, int(n), C.byref(out)))
    return out.value


def _check_boxes(net, lo, hi):
    import torch
    n = lo.shape[0]
    assert lo.is_cuda and hi.is_cuda and lo.dtype == torch.float32 and hi.dtype == torch.float32
    assert lo.is_contiguous() and hi.is_contiguous() and tuple(lo.shape) == (n, net.d)
    assert tuple(hi.shape) == (n, net.d)
    return n


def _ptr(t):
    return t.data_ptr() if t is not None else None


def bound_boxes_alpha(net: Net, prop: Property, lo, hi, alpha=None, init: bool = False,
                      raw: bool = False, tape=None, want_cls: bool = False, stream=None):
    """Bounds with per-box slopes ``alpha`` (device [n, nh]); returns (g_lo, g_hi, cls, tape)."""
    import torch
    n = _check_boxes(net, lo, hi)
    if alpha is not None:
        assert alpha.is_cuda and alpha.dtype == torch.float32 and alpha.is_contiguous()
        assert tuple(alpha.shape) == (n, alpha_size(net))
    need = alpha_tape_size(net, prop, n)
    if tape is None:
        tape = torch.empty(max(need, 1), dtype=torch.uint8, device=lo.device)
    g_lo = torch.empty((n, prop.rows), dtype=torch.float32, device=lo.device)
    g_hi = torch.empty((n, prop.rows), dtype=torch.float32, device=lo.device)
    cls = torch.empty((n,), dtype=torch.int8, device=lo.device) if want_cls else None
    _check(lib().bound_boxes_alpha(net.handle, prop.handle, n, lo.data_ptr(), hi.data_ptr(),
                                   _ptr(alpha), int(bool(init)), g_lo.data_ptr(), g_hi.data_ptr(),
                                   _ptr(cls), int(bool(raw)), tape.data_ptr(),
                                   tape.numel() * tape.element_size(), _stream(stream)))
    return g_lo, g_hi, cls, tape


def bound_tape_size(net: Net, prop: Property, n: int) -> int:
    out = C.c_size_t()
    _check(lib().bound_tape_size(net.handle, prop.handle, int(n), C.byref(out)))
    return out.value


def bound_boxes_relax(net: Net, prop: Property, lo, hi, relax: str = "two", raw: bool = False,
                      tape=None, want_cls: bool = False, stream=None):
    """Bounds from the tape-state kernel with the plain slopes of ``relax`` ("one": Eq. 1,
    "two": one ratio per equation); returns (g_lo, g_hi, cls)."""
    import torch
    n = _check_boxes(net, lo, hi)
    need = bound_tape_size(net, prop, n)
    if tape is None:
        tape = torch.empty(max(need, 1), dtype=torch.uint8, device=lo.device)
    g_lo = torch.empty((n, prop.rows), dtype=torch.float32, device=lo.device)
    g_hi = torch.empty((n, prop.rows), dtype=torch.float32, device=lo.device)
    cls = torch.empty((n,), dtype=torch.int8, device=lo.device) if want_cls else None
    _check(lib().bound_boxes_relax(net.handle, prop.handle, n, lo.data_ptr(), hi.data_ptr(),
                                   _relax(relax), g_lo.data_ptr(), g_hi.data_ptr(), _ptr(cls),
                                   int(bool(raw)), tape.data_ptr(),
                                   tape.numel() * tape.element_size(), _stream(stream)))
    return g_lo, g_hi, cls


def bound_boxes_backward(net: Net, prop: Property, tape, alpha, dg_lo=None, dg_hi=None,
                         raw: bool = False, stream=None):
    """dJ/dalpha from seeds dJ/dg_lo and dJ/dg_hi (device [n, rows]) and a forward tape."""
    import torch
    n = alpha.shape[0]
    dalpha = torch.empty_like(alpha)
    for t in (dg_lo, dg_hi):
        if t is not None:
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
            assert tuple(t.shape) == (n, prop.rows)
    _check(lib().bound_boxes_backward(net.handle, prop.handle, n, alpha.data_ptr(),
                                      tape.data_ptr(), tape.numel() * tape.element_size(),
                                      _ptr(dg_lo), _ptr(dg_hi), dalpha.data_ptr(),
                                      int(bool(raw)), _stream(stream)))
    return dalpha


def alpha_optimize(net: Net, prop: Property, lo, hi, steps: int = 20, lr: float = 0.1,
                   betas=(0.9, 0.999), eps: float = 1e-8, raw: bool = False, workspace=None,
                   stream=None) -> dict:
    """Projected Adam on per-box slopes; returns the last slopes, the intersected bounds and
    their classes (device tensors)."""
    import torch
    n = _check_boxes(net, lo, hi)
    need = alpha_workspace_size(net, prop, n)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=lo.device)
    alpha = torch.empty((n, alpha_size(net)), dtype=torch.float32, device=lo.device)
    best_lo = torch.empty((n, prop.rows), dtype=torch.float32, device=lo.device)
    best_hi = torch.empty((n, prop.rows), dtype=torch.float32, device=lo.device)
    cls = torch.empty((n,), dtype=torch.int8, device=lo.device)
    o = AlphaOpts(int(steps), float(lr), float(betas[0]), float(betas[1]), float(eps),
                  int(bool(raw)))
    _check(lib().alpha_optimize(net.handle, prop.handle, n, lo.data_ptr(), hi.data_ptr(),
                                C.byref(o), alpha.data_ptr(), best_lo.data_ptr(),
                                best_hi.data_ptr(), cls.data_ptr(), workspace.data_ptr(),
                                workspace.numel() * workspace.element_size(), _stream(stream)))
    return dict(alpha=alpha, best_lo=best_lo, best_hi=best_hi, cls=cls)


def _make_slr_bound():
    import torch

    class SLRBound(torch.autograd.Function):
        """(g_lo, g_hi) = SLRBound.apply(alpha, lo, hi, net, prop, raw): the bounds of every
        property row over each box with per-box slopes; the backward pass is the library's
        hand-written adjoint kernel (bound_boxes_backward)."""

        @staticmethod
        def forward(ctx, alpha, lo, hi, net, prop, raw=False):
            a = alpha.detach().contiguous()
            g_lo, g_hi, _, tape = bound_boxes_alpha(net, prop, lo, hi, a, raw=raw)
            ctx.net, ctx.prop, ctx.raw = net, prop, raw
            ctx.save_for_backward(a, tape)
            return g_lo, g_hi

        @staticmethod
        def backward(ctx, dg_lo, dg_hi):
            a, tape = ctx.saved_tensors
            dlo = dg_lo.contiguous() if dg_lo is not None else None
            dhi = dg_hi.contiguous() if dg_hi is not None else None
            da = bound_boxes_backward(ctx.net, ctx.prop, tape, a, dlo, dhi, raw=ctx.raw)
            return da, None, None, None, None, None

    return SLRBound


_SLRBOUND = None


def __getattr__(name):
    global _SLRBOUND
    if name == "SLRBound":
        if _SLRBOUND is None:
            _SLRBOUND = _make_slr_bound()
        return _SLRBOUND
    raise AttributeError(name)


# ---------------------------------------------------------------------------------------------
# batches of independent exact counts
# ---------------------------------------------------------------------------------------------
def _batch_arrays(items):
    """items: sequence of (net, prop, lo, hi, max_depth, max_leaves)."""
    n = len(items)
    keep = []
    nets = (C.c_void_p * n)(*[it[0].handle.value for it in items])
    props = (C.c_void_p * n)(*[it[1].handle.value for it in items])
    los, his = [], []
    for it in items:
        lo = np.ascontiguousarray(it[2], np.float64)
        hi = np.ascontiguousarray(it[3], np.float64)
        keep += [lo, hi]
        los.append(lo.ctypes.data)
        his.append(hi.ctypes.data)
    lo_a = (C.c_void_p * n)(*los)
    hi_a = (C.c_void_p * n)(*his)
    depth = (C.c_int32 * n)(*[int(it[4]) for it in items])
    leaves = (C.c_int64 * n)(*[int(it[5]) for it in items])
    return nets, props, lo_a, hi_a, depth, leaves, keep


def _results(res, rc):
    out = []
    for r in res:
        d = {f: getattr(r, f) for f, _ in CountResult._fields_}
        d["rc"] = rc
        out.append(d)
    return out


class Batch:
    """Many exact counts advanced together on the device (``batch_create``); ``run()`` replays
    the captured graph (or issues the same launches) and returns one result dict per instance."""

    def __init__(self, items, use_graph: bool = True, alpha_steps: int = 0,
                 alpha_lr: float = 0.1, alpha_min_depth: int = 0, alpha_select: float = 0.0,
                 alpha_chunk: int = 0):
        self.items = list(items)   # keeps nets and properties alive
        self.n = len(self.items)
        nets, props, lo, hi, depth, leaves, self._keep = _batch_arrays(self.items)
        h = C.c_void_p()
        o = BatchOpts(int(bool(use_graph)), int(alpha_steps), float(alpha_lr),
                      int(alpha_min_depth), float(alpha_select), int(alpha_chunk))
        _check(lib().batch_create_opts(self.n, nets, props, lo, hi, depth, leaves, C.byref(o),
                                       C.byref(h)))
        self.handle = h

    def run(self, stream=None):
        res = (CountResult * self.n)()
        rc = _check(lib().batch_run(self.handle, _stream(stream), res))
        return _results(res, rc)

    def __del__(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.batch_free(self.handle)
            self.handle = None


def count_exact_batch(items, stream=None):
    """One-shot batch (no graph): items are (net, prop, lo, hi, max_depth, max_leaves)."""
    items = list(items)
    n = len(items)
    nets, props, lo, hi, depth, leaves, keep = _batch_arrays(items)
    res = (CountResult * n)()
    rc = _check(lib().count_exact_batch(n, nets, props, lo, hi, depth, leaves, _stream(stream),
                                        res))
    return _results(res, rc)
