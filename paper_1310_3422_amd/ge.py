"""Thin ctypes binding of libge (include/ge.h).

The C functions keep their names (``ge_plan``, ``ge_step_n``, ...); the
classes below only marshal torch tensors (device memory) and torch streams
into plain pointers.  Every level of the sweep runs in the HIP kernels of
libge.so; there is no fallback path, and a missing library raises.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libge.so")

(GE_OK, GE_ERR_INVALID, GE_ERR_NOMEM, GE_ERR_HIP, GE_ERR_UNSUPPORTED, GE_ERR_NONFINITE,
 GE_ERR_SYNC) = range(7)
GE_FP64, GE_FP32, GE_FP32_COMP = 0, 1, 2
PRECISIONS = {"fp64": GE_FP64, "fp32": GE_FP32, "fp32c": GE_FP32_COMP}

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double


class GeDesc(ctypes.Structure):
    _fields_ = [("n", _i64), ("r", _dbl), ("precision", _i32), ("tile", _i32),
                ("depth", _i32), ("waves", _i32), ("g_left", _dbl),
                ("g_right", _dbl), ("src_b", _vp), ("schedule", _i32), ("k", _i32)]


class GeBatchDesc(ctypes.Structure):
    _fields_ = [("nrods", _i64), ("n", _vp), ("offsets", _vp), ("r", _vp),
                ("g_left", _vp), ("g_right", _vp), ("precision", _i32),
                ("tune", _i32), ("sync", _i32)]


class Ge2dDesc(ctypes.Structure):
    _fields_ = [("nx", _i64), ("ny", _i64), ("rx", _dbl), ("ry", _dbl), ("precision", _i32),
                ("g_west", _dbl), ("g_east", _dbl), ("g_south", _dbl), ("g_north", _dbl),
                ("depth", _i32)]


class GEError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_str(status)}: {message}")
        self.status = status


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "ge_version": (ctypes.c_char_p, []),
    "ge_last_error": (ctypes.c_char_p, []),
    "ge_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "ge_comp_offset": (_i64, [_i64]),
    "ge_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(GeDesc)]),
    "ge_plan": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(GeDesc)]),
    "ge_destroy": (None, [_vp]),
    "ge_plan_check": (ctypes.c_int, [_vp, _vp]),
    "ge_step_n": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp]),
    "ge_plan_config": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                      ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "ge_comp_to_fp64": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "ge_comp_from_fp64": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "ge_batch_plan": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(GeBatchDesc)]),
    "ge_batch_destroy": (None, [_vp]),
    "ge_batch_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "ge_batch_state_elems": (_i64, [_vp]),
    "ge_batch_info": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                     ctypes.POINTER(_dbl), _vp]),
    "ge_solve_batch": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _vp]),
    "ge_batch_set_wait_polls": (ctypes.c_int, [_vp, _i64]),
    "ge_solve_batch_static": (ctypes.c_int, [_vp, _vp, _i64, _i64, _vp]),
    "ge_batch_check": (ctypes.c_int, [_vp, _vp]),
    "ge_plan_schedule": (_i32, [_vp]),
    "ge_nn_param_count": (_i64, []),
    "ge_nn_create": (ctypes.c_int, [ctypes.POINTER(_vp), _i32, _i32, ctypes.c_uint64]),
    "ge_nn_destroy": (None, [_vp]),
    "ge_nn_set_params": (ctypes.c_int, [_vp, _vp, _i64]),
    "ge_nn_get_params": (ctypes.c_int, [_vp, _vp, _i64]),
    "ge_nn_forward": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    "ge_nn_jump": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "ge_nn_grads": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _vp, _vp]),
    "ge_nn_gradient": (ctypes.c_int, [_vp, _vp, _vp]),
    "ge_nn_train_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, ctypes.c_float, _vp, _vp]),
    "ge_nn_advance": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i32, _i64, _i32, _i32, _dbl,
                                     _vp, _vp, _vp, ctypes.POINTER(_i64), _vp]),
    "ge_nn_layer_shape": (ctypes.c_int, [_i32] + [ctypes.POINTER(_i32)] * 6),
    "ge_nn_layer_probe": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _i32, _vp, _vp]),
    "ge_2d_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Ge2dDesc)]),
    "ge_2d_step_n": (ctypes.c_int, [ctypes.POINTER(Ge2dDesc), _vp, _vp, _i64, _i64, _vp]),
    "ge_f32_to_f64": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "ge_f64_to_f32": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
}


def lib():
    """Load libge.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1310_3422_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def status_str(status):
    return lib().ge_status_str(status).decode()


def last_error():
    return lib().ge_last_error().decode()


def check(status):
    if status != GE_OK:
        raise GEError(status, last_error())


_check_status = check


def comp_offset(n):
    return int(lib().ge_comp_offset(n))


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def state_dtype(precision):
    torch = _torch()
    return torch.float64 if _prec(precision) == GE_FP64 else torch.float32


def state_numel(n, precision):
    return 2 * comp_offset(n) if _prec(precision) == GE_FP32_COMP else n


class Plan:
    """A ge_plan for one rod; ``step_n`` advances a device state tensor."""

    def __init__(self, n, r, precision="fp64", g_left=0.0, g_right=0.0, src_b=None,
                 tile=0, depth=0, waves=0, schedule=0, k=0):
        self.n, self.r = int(n), float(r)
        self.precision = _prec(precision)
        self._src_b = src_b   # keep the profile alive
        if src_b is not None:
            self._check_tensor(src_b, self.n, "src_b", state_dtype(self.precision))
        self.desc = GeDesc(n=self.n, r=self.r, precision=self.precision, tile=tile,
                           depth=depth, waves=waves, g_left=float(g_left),
                           g_right=float(g_right), src_b=_ptr(src_b), schedule=int(schedule),
                           k=int(k))
        self.k = int(k)
        h = _vp()
        check(lib().ge_plan(ctypes.byref(h), ctypes.byref(self.desc)))
        self.handle = h
        self.workspace_bytes = int(lib().ge_workspace_bytes(ctypes.byref(self.desc)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.ge_destroy(h)
            self.handle = None

    def config(self):
        t, d, w, h = _i32(), _i32(), _i32(), _i32()
        check(lib().ge_plan_config(self.handle, ctypes.byref(t), ctypes.byref(d),
                                   ctypes.byref(w), ctypes.byref(h)))
        out = {"tile": t.value, "depth": d.value, "waves": w.value, "halo": h.value,
               "schedule": int(lib().ge_plan_schedule(self.handle))}
        if self.k >= 2:
            out["k"] = self.k
        return out

    @staticmethod
    def _check_tensor(t, numel, name, dtype):
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of {numel} values")

    def new_state(self):
        torch = _torch()
        return torch.zeros(state_numel(self.n, self.precision),
                           dtype=state_dtype(self.precision), device="cuda")

    def new_workspace(self):
        torch = _torch()
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device="cuda")

    def step_n(self, u, step0, nsteps, workspace=None, g_left_t=None, g_right_t=None,
               src_a_t=None, flux=None, stream=None):
        torch = _torch()
        self._check_tensor(u, state_numel(self.n, self.precision), "u",
                           state_dtype(self.precision))
        if workspace is None:
            workspace = self.new_workspace()
        for name, t, k in (("g_left_t", g_left_t, nsteps + 1), ("g_right_t", g_right_t, nsteps + 1),
                           ("src_a_t", src_a_t, nsteps), ("flux", flux, 2)):
            if t is not None:
                self._check_tensor(t, k, name, torch.float64)
        check(lib().ge_step_n(self.handle, _ptr(u), _ptr(workspace), int(step0), int(nsteps),
                              _ptr(g_left_t), _ptr(g_right_t), _ptr(src_a_t), _ptr(flux),
                              _stream_ptr(stream)))
        return u

    def check(self, stream=None):
        """ge_plan_check: wait for the stream; raise GEError(GE_ERR_NONFINITE)
        if a launch of this plan stored a NaN or infinite value."""
        check(lib().ge_plan_check(self.handle, _stream_ptr(stream)))


def comp_to_fp64(pair, n, stream=None):
    torch = _torch()
    x = torch.empty(n, dtype=torch.float64, device=pair.device)
    check(lib().ge_comp_to_fp64(_ptr(pair), _ptr(x), int(n), _stream_ptr(stream)))
    return x


def comp_from_fp64(x, stream=None):
    torch = _torch()
    n = x.numel()
    pair = torch.zeros(2 * comp_offset(n), dtype=torch.float32, device=x.device)
    check(lib().ge_comp_from_fp64(_ptr(x), _ptr(pair), int(n), _stream_ptr(stream)))
    return pair


def pack_state(u0, precision, device="cuda"):
    """Host FP64 values -> device state tensor in the precision's layout
    (FP32 forms round the same FP64 values; the compensated pair starts with
    e = fl32(u0 - s))."""
    torch = _torch()
    p = _prec(precision)
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    if p == GE_FP64:
        return torch.from_numpy(u0.copy()).to(device)
    if p == GE_FP32:
        return torch.from_numpy(u0.astype(np.float32)).to(device)
    n = u0.size
    off = comp_offset(n)
    s = u0.astype(np.float32)
    e = (u0 - s.astype(np.float64)).astype(np.float32)
    buf = np.zeros(2 * off, dtype=np.float32)
    buf[:n], buf[off:off + n] = s, e
    return torch.from_numpy(buf).to(device)


def unpack_state(u, n, precision):
    """Device state tensor -> host FP64 values (s + e for the pair)."""
    p = _prec(precision)
    a = u.detach().cpu().numpy()
    if p == GE_FP32_COMP:
        off = comp_offset(n)
        return a[:n].astype(np.float64) + a[off:off + n].astype(np.float64)
    return a[:n].astype(np.float64)


class Batch:
    """A ge_batch plan: independent rods advanced together in one persistent,
    graph-captured launch.  Host arrays describe the rods; the packed state
    lives in a device tensor (see ``pack_batch_state``)."""

    def __init__(self, n, offsets, r, g_left, g_right, precision="fp32", tune=False, sync=0):
        self.n = np.ascontiguousarray(n, dtype=np.int64)
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.r = np.ascontiguousarray(r, dtype=np.float64)
        self.g_left = np.ascontiguousarray(g_left, dtype=np.float64)
        self.g_right = np.ascontiguousarray(g_right, dtype=np.float64)
        self.precision = _prec(precision)
        nr = self.n.size
        if self.offsets.size != nr + 1 or any(a.size != nr for a in (self.r, self.g_left, self.g_right)):
            raise ValueError("rod table arrays have inconsistent lengths")
        c = lambda a: ctypes.c_void_p(a.ctypes.data)
        self.desc = GeBatchDesc(nrods=nr, n=c(self.n), offsets=c(self.offsets), r=c(self.r),
                                g_left=c(self.g_left), g_right=c(self.g_right),
                                precision=self.precision, tune=1 if tune else 0,
                                sync=int(sync))
        h = _vp()
        check(lib().ge_batch_plan(ctypes.byref(h), ctypes.byref(self.desc)))
        self.handle = h
        self.state_elems = int(lib().ge_batch_state_elems(h))
        self.workspace_bytes = int(lib().ge_batch_workspace_bytes(h))

    @classmethod
    def from_inputs(cls, rb, precision="fp32", tune=False, sync=0):
        """From an ``inputs.RodBatch``."""
        return cls(rb.n, rb.offsets, rb.r, rb.g_left, rb.g_right, precision, tune, sync)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.ge_batch_destroy(h)
            self.handle = None

    def info(self):
        nt, gr, est = _i32(), _i32(), _dbl()
        ks = np.zeros(self.n.size, dtype=np.int32)
        check(lib().ge_batch_info(self.handle, ctypes.byref(nt), ctypes.byref(gr),
                                  ctypes.byref(est), ctypes.c_void_p(ks.ctypes.data)))
        return {"ntasks": nt.value, "grid": gr.value, "est_us_per_level": est.value,
                "rod_k": ks}

    def new_workspace(self):
        torch = _torch()
        return torch.zeros(max(self.workspace_bytes, 256), dtype=torch.uint8, device="cuda")

    def solve(self, u, step0, nsteps, workspace, stream=None):
        torch = _torch()
        Plan._check_tensor(u, self.state_elems, "u", state_dtype(self.precision))
        if not workspace.is_cuda or workspace.numel() < self.workspace_bytes:
            raise ValueError("workspace too small")
        check(lib().ge_solve_batch(self.handle, _ptr(u), _ptr(workspace), int(step0),
                                   int(nsteps), _stream_ptr(stream)))
        return u

    def solve_static(self, u, step0, nsteps, stream=None):
        """ge_solve_batch_static: the same run with the library's static
        scratch (allocates nothing, no graph)."""
        Plan._check_tensor(u, self.state_elems, "u", state_dtype(self.precision))
        check(lib().ge_solve_batch_static(self.handle, _ptr(u), int(step0), int(nsteps),
                                          _stream_ptr(stream)))
        return u

    def set_wait_polls(self, polls):
        check(lib().ge_batch_set_wait_polls(self.handle, int(polls)))

    def check(self, stream=None):
        """ge_batch_check: wait for the stream; raise GEError with GE_ERR_SYNC
        or GE_ERR_NONFINITE if a run raised one."""
        check(lib().ge_batch_check(self.handle, _stream_ptr(stream)))


def pack_batch_state(rb_u0, offsets, n, precision, device="cuda"):
    """Host FP64 packed values (rods at ``offsets``) -> device state tensor in
    the batch layout of the precision."""
    torch = _torch()
    p = _prec(precision)
    u0 = np.ascontiguousarray(rb_u0, dtype=np.float64)
    total = int(offsets[-1])
    if p == GE_FP64:
        return torch.from_numpy(u0[:total].copy()).to(device)
    if p == GE_FP32:
        return torch.from_numpy(u0[:total].astype(np.float32)).to(device)
    off = comp_offset(total)
    s = u0[:total].astype(np.float32)
    e = (u0[:total] - s.astype(np.float64)).astype(np.float32)
    buf = np.zeros(2 * off, dtype=np.float32)
    buf[:total], buf[off:off + total] = s, e
    return torch.from_numpy(buf).to(device)


def unpack_batch_rod(u_host, offsets, n, i, precision):
    """FP64 values of rod i from a host copy (numpy) of a batch state."""
    p = _prec(precision)
    a, b = int(offsets[i]), int(offsets[i]) + int(n[i])
    if p == GE_FP32_COMP:
        off = comp_offset(int(offsets[-1]))
        return u_host[a:b].astype(np.float64) + u_host[off + a:off + b].astype(np.float64)
    return u_host[a:b].astype(np.float64)


class Net:
    """The learned 64-level propagator (ge_nn_*): parameters and buffers live
    on the device; tensors passed in are float32 CUDA tensors, rods back to
    back (batch x width)."""

    def __init__(self, width=4096, max_batch=512, seed=4):
        self.width, self.max_batch = int(width), int(max_batch)
        h = _vp()
        check(lib().ge_nn_create(ctypes.byref(h), self.width, self.max_batch, int(seed)))
        self.handle = h
        self.nparam = int(lib().ge_nn_param_count())

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.ge_nn_destroy(h)
            self.handle = None

    def _check(self, t, numel, name):
        torch = _torch()
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of {numel} values")

    def params(self):
        out = np.zeros(self.nparam, dtype=np.float32)
        check(lib().ge_nn_get_params(self.handle, ctypes.c_void_p(out.ctypes.data), self.nparam))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        check(lib().ge_nn_set_params(self.handle, ctypes.c_void_p(p.ctypes.data), p.size))

    def forward(self, u, r, stream=None):
        torch = _torch()
        b = r.numel()
        self._check(u, b * self.width, "u")
        self._check(r, b, "r")
        out = torch.empty(b * self.width, dtype=torch.float32, device=u.device)
        scale = torch.empty(b, dtype=torch.float32, device=u.device)
        check(lib().ge_nn_forward(self.handle, _ptr(u), _ptr(r), b, _ptr(out), _ptr(scale),
                                  _stream_ptr(stream)))
        return out, scale

    def jump(self, u, r, out=None, stream=None):
        torch = _torch()
        b = r.numel()
        self._check(u, b * self.width, "u")
        self._check(r, b, "r")
        if out is None:
            out = torch.empty_like(u)
        check(lib().ge_nn_jump(self.handle, _ptr(u), _ptr(r), b, _ptr(out), _stream_ptr(stream)))
        return out

    def grads(self, u, u64, r, stream=None):
        """(loss, flat gradient) for one batch, without an update."""
        torch = _torch()
        b = r.numel()
        for t, name in ((u, "u"), (u64, "u64")):
            self._check(t, b * self.width, name)
        loss = torch.zeros(1, dtype=torch.float32, device=u.device)
        g = torch.empty(self.nparam, dtype=torch.float32, device=u.device)
        check(lib().ge_nn_grads(self.handle, _ptr(u), _ptr(u64), _ptr(r), b, _ptr(loss),
                                _stream_ptr(stream)))
        check(lib().ge_nn_gradient(self.handle, _ptr(g), _stream_ptr(stream)))
        return loss, g

    def advance(self, ge_batch, ge_ws, u, r, njumps, step0=0, check=8, tol=1e-4,
                accepted=None, fallbacks=None, last_err=None, stream=None):
        """Re-checked surrogate stepping (ge_nn_advance); returns the number
        of rod-windows that fell back to the GE sweep."""
        b = r.numel()
        self._check(u, b * self.width, "u")
        self._check(r, b, "r")
        nfb = _i64(0)
        _check_status(lib().ge_nn_advance(
            self.handle, ge_batch.handle, _ptr(ge_ws), _ptr(u), _ptr(r), b, int(step0),
            int(njumps), int(check), float(tol), _ptr(accepted), _ptr(fallbacks),
            _ptr(last_err), ctypes.byref(nfb), _stream_ptr(stream)))
        return int(nfb.value)

    @staticmethod
    def layer_shape(layer):
        """(ci, co, cip, cop, cod, dil) of layer 1..6 (ge_nn_layer_shape)."""
        v = [_i32() for _ in range(6)]
        check(lib().ge_nn_layer_shape(int(layer), *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def layer_probe(self, layer, op, batch, x=None, g=None, stream=None):
        """ge_nn_layer_probe: one product of one layer on bfloat16 operands
        (torch.bfloat16 CUDA tensors, channels last, padded channels zero),
        returned in FP32: op 0 forward [batch, width, cop], op 1 input
        gradient [batch, width, cip], op 2 weight gradient (flat dW, db)."""
        torch = _torch()
        ci, co, cip, cop, cod, dil = self.layer_shape(layer)
        for t, c, name in ((x, cip, "x"), (g, cod, "g")):
            if t is not None and (not t.is_cuda or t.dtype != torch.bfloat16 or
                                  not t.is_contiguous() or t.numel() != batch * self.width * c):
                raise ValueError(f"{name} must be a contiguous bfloat16 CUDA tensor "
                                 f"[{batch}, {self.width}, {c}]")
        shape = {0: (batch, self.width, cop), 1: (batch, self.width, cip),
                 2: (5 * co * ci + co,)}[int(op)]
        out = torch.empty(shape, dtype=torch.float32, device="cuda")
        check(lib().ge_nn_layer_probe(self.handle, int(layer), int(op), _ptr(x), _ptr(g),
                                      int(batch), _ptr(out), _stream_ptr(stream)))
        return out

    def train_step(self, u, u64, r, lr, loss=None, stream=None):
        b = r.numel()
        for t, name in ((u, "u"), (u64, "u64")):
            self._check(t, b * self.width, name)
        check(lib().ge_nn_train_step(self.handle, _ptr(u), _ptr(u64), _ptr(r), b, float(lr),
                                     _ptr(loss), _stream_ptr(stream)))


def f32_to_f64(x, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(x.numel(), dtype=torch.float64, device=x.device)
    check(lib().ge_f32_to_f64(_ptr(x), _ptr(out), x.numel(), _stream_ptr(stream)))
    return out


def f64_to_f32(x, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(x.numel(), dtype=torch.float32, device=x.device)
    check(lib().ge_f64_to_f32(_ptr(x), _ptr(out), x.numel(), _stream_ptr(stream)))
    return out


def ge_2d_desc(nx, ny, rx, ry, precision="fp64", walls=(0.0, 0.0, 0.0, 0.0), depth=0):
    gw, ge_, gs, gn = (float(w) for w in walls)
    return Ge2dDesc(nx=int(nx), ny=int(ny), rx=float(rx), ry=float(ry),
                    precision=_prec(precision), g_west=gw, g_east=ge_, g_south=gs, g_north=gn,
                    depth=int(depth))


def step2d_n(u, nx, ny, rx, ry, step0, nsteps, precision="fp64", walls=(0.0, 0.0, 0.0, 0.0),
             workspace=None, stream=None, depth=0):
    """Advance the ny x nx grid ``u`` (contiguous CUDA tensor, row-major,
    float64 for fp64, float32 for fp32) in place by ``nsteps`` levels of the
    two-dimensional extension (ge_2d_step_n); walls = (west, east, south,
    north)."""
    torch = _torch()
    d = ge_2d_desc(nx, ny, rx, ry, precision, walls, depth)
    dtype = torch.float64 if d.precision == GE_FP64 else torch.float32
    if not u.is_cuda or u.dtype != dtype or not u.is_contiguous() or u.numel() != nx * ny:
        raise ValueError(f"u must be a contiguous {dtype} CUDA tensor of {nx * ny} values")
    if workspace is None:
        workspace = torch.empty(int(lib().ge_2d_workspace_bytes(ctypes.byref(d))),
                                dtype=torch.uint8, device=u.device)
    check(lib().ge_2d_step_n(ctypes.byref(d), _ptr(u), _ptr(workspace), int(step0), int(nsteps),
                            _stream_ptr(stream)))
    return u
