"""Python binding of libmatcha (include/matcha.h): argument marshalling only.

Every step of the alignment path runs in the HIP kernels of libmatcha.so; torch is used
for device memory and the current stream.  There is no CPU fallback: importing this
module on a machine without the built library raises.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses
import os
from typing import Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmatcha.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_WORKSPACE = 0, -1, -2, -3, -4
FP32, BF16_FP32ACC = 0, 1
ST_NONFINITE, ST_INDEFINITE, ST_SINGULAR, ST_NEAR_POLE, ST_FEW_MAXIMA, ST_EARLY_STOP = 1, 2, 4, 8, 16, 32
MAX_L, MAX_KC, MAX_LEVELS = 64, 64, 16

EXPORTED = ["matcha_create", "matcha_destroy", "matcha_prepare", "matcha_status_string", "matcha_set_tuning",
            "matcha_get_tuning", "matcha_c_elems", "matcha_f_elems", "matcha_workspace_size", "matcha_lpt_order",
            "matcha_coeff_assemble", "matcha_soft_search", "matcha_march_newton", "matcha_evaluate",
            "matcha_grad_template", "matcha_align_graph_create", "matcha_graph_launch", "matcha_graph_destroy",
            "matcha_autotune"]


class MatchaError(RuntimeError):
    pass


class _Batch(ct.Structure):
    _fields_ = [("n_particles", ct.c_int32), ("L_max", ct.c_int32),
                ("L_host", ct.POINTER(ct.c_int32)), ("R_host", ct.POINTER(ct.c_int32)),
                ("L_dev", ct.c_void_p), ("R_dev", ct.c_void_p), ("f_offset", ct.c_void_p), ("C_offset", ct.c_void_p),
                ("L_h", ct.c_int32), ("R_h", ct.c_int32), ("order", ct.c_void_p)]


class _Tuning(ct.Structure):
    _fields_ = [("march_nc", ct.c_int32), ("soft_threads", ct.c_int32)]


class _SoftCfg(ct.Structure):
    _fields_ = [("B", ct.c_int32), ("n_grid", ct.c_int32), ("Kc", ct.c_int32)]


class _MarchCfg(ct.Structure):
    _fields_ = [("levels", ct.POINTER(ct.c_int32)), ("n_levels", ct.c_int32), ("steps", ct.c_int32),
                ("max_step", ct.c_double), ("early_stop", ct.c_int32),
                ("tol_grad", ct.c_double), ("tol_step", ct.c_double), ("tol_rel", ct.c_double),
                ("fp64_above", ct.c_int32)]


_lib = None


def lib():
    """The loaded libmatcha.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MatchaError(f"libmatcha.so not found at {LIB_PATH}; run __graft_entry__.build()")
        L = ct.CDLL(LIB_PATH)
        vp, i32, i64, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
        bp = ct.POINTER(_Batch)
        L.matcha_create.argtypes = [ct.c_int, ct.POINTER(vp)]
        L.matcha_destroy.argtypes = [vp]
        L.matcha_prepare.argtypes = [vp, i32, i32, i32]
        L.matcha_status_string.argtypes = [ct.c_int]
        L.matcha_status_string.restype = ct.c_char_p
        L.matcha_set_tuning.argtypes = [vp, ct.POINTER(_Tuning)]
        L.matcha_get_tuning.argtypes = [vp, ct.POINTER(_Tuning)]
        L.matcha_c_elems.argtypes = [i32]
        L.matcha_c_elems.restype = i64
        L.matcha_f_elems.argtypes = [i32, i32]
        L.matcha_f_elems.restype = i64
        L.matcha_workspace_size.argtypes = [bp, i32]
        L.matcha_workspace_size.restype = sz
        L.matcha_coeff_assemble.argtypes = [vp, bp, vp, vp, vp, vp, ct.c_int, vp]
        L.matcha_soft_search.argtypes = [vp, bp, vp, ct.POINTER(_SoftCfg), vp, vp, vp]
        L.matcha_march_newton.argtypes = [vp, bp, vp, ct.POINTER(_MarchCfg), i32, vp, vp, vp, vp, vp]
        L.matcha_evaluate.argtypes = [vp, bp, vp, i32, i32, vp, vp, vp]
        L.matcha_grad_template.argtypes = [vp, bp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.matcha_lpt_order.argtypes = [bp, ct.POINTER(_MarchCfg), ct.POINTER(ct.c_int32)]
        L.matcha_align_graph_create.argtypes = [vp, bp, vp, vp, vp, vp, ct.c_int, ct.POINTER(_SoftCfg),
                                                ct.POINTER(_MarchCfg), vp, vp, vp, vp, ct.POINTER(vp)]
        L.matcha_graph_launch.argtypes = [vp, vp]
        L.matcha_graph_destroy.argtypes = [vp]
        L.matcha_autotune.argtypes = [vp, bp, vp, ct.POINTER(_SoftCfg), ct.POINTER(_MarchCfg), vp, vp, vp, vp, i32,
                                      ct.POINTER(_Tuning)]
        for name in ["matcha_create", "matcha_destroy", "matcha_prepare", "matcha_set_tuning", "matcha_get_tuning",
                     "matcha_lpt_order", "matcha_coeff_assemble", "matcha_soft_search", "matcha_march_newton",
                     "matcha_evaluate", "matcha_grad_template", "matcha_align_graph_create", "matcha_graph_launch",
                     "matcha_graph_destroy", "matcha_autotune"]:
            getattr(L, name).restype = ct.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != OK:
        msg = lib().matcha_status_string(rc).decode()
        raise MatchaError(f"{what} failed: {msg} ({rc})")


def c_elems(L: int) -> int:
    return int(lib().matcha_c_elems(L))


def f_elems(L: int, R: int) -> int:
    return int(lib().matcha_f_elems(L, R))


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, name: str):
    if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype:
        raise MatchaError(f"{name} must be a contiguous CUDA tensor of dtype {dtype}")


class Context:
    """A libmatcha context on one device (owns the read-only recurrence tables)."""

    def __init__(self, device: int | None = None):
        dev = torch.cuda.current_device() if device is None else int(device)
        h = ct.c_void_p()
        _check(lib().matcha_create(dev, ct.byref(h)), "matcha_create")
        self.handle = h
        self.device = dev

    def prepare(self, L_max: int, B: int = 0, n_grid: int = 0):
        _check(lib().matcha_prepare(self.handle, L_max, B, n_grid), "matcha_prepare")

    def set_tuning(self, march_nc: int = 0, soft_threads: int = 0):
        t = _Tuning(int(march_nc), int(soft_threads))
        _check(lib().matcha_set_tuning(self.handle, ct.byref(t)), "matcha_set_tuning")

    def get_tuning(self) -> dict:
        t = _Tuning()
        _check(lib().matcha_get_tuning(self.handle, ct.byref(t)), "matcha_get_tuning")
        return {"march_nc": int(t.march_nc), "soft_threads": int(t.soft_threads)}

    def close(self):
        if self.handle:
            lib().matcha_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class Batch:
    """Host and device descriptions of a batch (keeps every buffer alive)."""

    L: np.ndarray
    R: np.ndarray
    L_h: int
    R_h: int
    f_offset: np.ndarray
    C_offset: np.ndarray
    L_dev: torch.Tensor
    R_dev: torch.Tensor
    f_off_dev: torch.Tensor
    C_off_dev: torch.Tensor
    c_total: int
    f_total: int
    order_dev: torch.Tensor | None = None

    @staticmethod
    def make(L: Sequence[int], R: Sequence[int], L_h: int, R_h: int, device="cuda", f_offset=None) -> "Batch":
        L = np.ascontiguousarray(L, dtype=np.int32)
        R = np.ascontiguousarray(R, dtype=np.int32)
        csz = np.array([c_elems(int(x)) for x in L], dtype=np.int64)
        C_offset = np.concatenate([[0], np.cumsum(csz)[:-1]]).astype(np.int64)
        fsz = R.astype(np.int64) * (L.astype(np.int64) + 1) ** 2
        if f_offset is None:
            f_offset = np.concatenate([[0], np.cumsum(fsz)[:-1]]).astype(np.int64)
        f_offset = np.ascontiguousarray(f_offset, dtype=np.int64)
        t = lambda a: torch.from_numpy(a).to(device)  # noqa: E731
        return Batch(L, R, int(L_h), int(R_h), f_offset, C_offset, t(L), t(R), t(f_offset), t(C_offset),
                     int(csz.sum()), int(fsz.sum()))

    @property
    def n(self) -> int:
        return int(self.L.shape[0])

    def c_struct(self) -> _Batch:
        b = _Batch()
        b.n_particles = self.n
        b.L_max = int(self.L.max()) if self.n else 0
        b.L_host = self.L.ctypes.data_as(ct.POINTER(ct.c_int32))
        b.R_host = self.R.ctypes.data_as(ct.POINTER(ct.c_int32))
        b.L_dev = self.L_dev.data_ptr()
        b.R_dev = self.R_dev.data_ptr()
        b.f_offset = self.f_off_dev.data_ptr()
        b.C_offset = self.C_off_dev.data_ptr()
        b.L_h = self.L_h
        b.R_h = self.R_h
        b.order = self.order_dev.data_ptr() if self.order_dev is not None else None
        return b

    def set_lpt_order(self, levels: Sequence[int], steps: int):
        """Process particles longest-first in the march (uneven L_p)."""
        cfg = _march_cfg(levels, steps)
        order = np.zeros(self.n, dtype=np.int32)
        bs = self.c_struct()
        _check(lib().matcha_lpt_order(ct.byref(bs), ct.byref(cfg), order.ctypes.data_as(ct.POINTER(ct.c_int32))),
               "matcha_lpt_order")
        self.order_dev = torch.from_numpy(order).to(self.L_dev.device)
        return order


def _march_cfg(levels, steps, max_step=0.0, early_stop=False, tol_grad=1e-6, tol_step=1e-7, tol_rel=1e-7,
               fp64_above=0):
    lv = np.ascontiguousarray(levels, dtype=np.int32)
    cfg = _MarchCfg(lv.ctypes.data_as(ct.POINTER(ct.c_int32)), len(lv), int(steps), float(max_step),
                    int(early_stop), float(tol_grad), float(tol_step), float(tol_rel), int(fp64_above))
    cfg._keep = lv  # the levels array must outlive the struct
    return cfg


def coeff_assemble(ctx: Context, batch: Batch, f: torch.Tensor, h: torch.Tensor, w: torch.Tensor,
                   C: torch.Tensor | None = None, prec: int = FP32, stream=None) -> torch.Tensor:
    """C (wedge layout, float32 view of complex pairs) = assembly of f against h (eq. sigmalmm)."""
    _need(w, torch.float32, "w")
    if C is None:
        C = torch.empty(2 * batch.c_total, dtype=torch.float32, device=f.device)
    _need(C, torch.float32, "C")
    bs = batch.c_struct()
    _check(lib().matcha_coeff_assemble(ctx.handle, ct.byref(bs), _ptr(f), _ptr(h), _ptr(w), _ptr(C), prec,
                                       ct.c_void_p(_stream(stream))), "matcha_coeff_assemble")
    return C


def soft_search(ctx: Context, batch: Batch, C: torch.Tensor, B: int, n_grid: int, Kc: int,
                cand: torch.Tensor | None = None, status: torch.Tensor | None = None, stream=None):
    if cand is None:
        cand = torch.empty((batch.n, Kc, 4), dtype=torch.float32, device=C.device)
    if status is None:
        status = torch.empty(batch.n, dtype=torch.int32, device=C.device)
    _need(cand, torch.float32, "cand")
    bs = batch.c_struct()
    cfg = _SoftCfg(B, n_grid, Kc)
    _check(lib().matcha_soft_search(ctx.handle, ct.byref(bs), _ptr(C), ct.byref(cfg), _ptr(cand), _ptr(status),
                                    ct.c_void_p(_stream(stream))), "matcha_soft_search")
    return cand, status


def march_newton(ctx: Context, batch: Batch, C: torch.Tensor, levels: Sequence[int], steps: int,
                 cand: torch.Tensor, status: torch.Tensor, best: torch.Tensor | None = None,
                 best_idx: torch.Tensor | None = None, max_step: float = 0.0, early_stop: bool = False,
                 tol_grad: float = 1e-6, tol_step: float = 1e-7, tol_rel: float = 1e-7, fp64_above: int = 0,
                 stream=None):
    Kc = int(cand.shape[1])
    if best is None:
        best = torch.empty((batch.n, 4), dtype=torch.float32, device=C.device)
    if best_idx is None:
        best_idx = torch.empty(batch.n, dtype=torch.int32, device=C.device)
    cfg = _march_cfg(levels, steps, max_step, early_stop, tol_grad, tol_step, tol_rel, fp64_above)
    bs = batch.c_struct()
    _check(lib().matcha_march_newton(ctx.handle, ct.byref(bs), _ptr(C), ct.byref(cfg), Kc, _ptr(cand), _ptr(best),
                                     _ptr(best_idx), _ptr(status), ct.c_void_p(_stream(stream))),
           "matcha_march_newton")
    return best, best_idx, status


def evaluate(ctx: Context, batch: Batch, C: torch.Tensor, L_eval: int, theta: torch.Tensor, fp64_above: int = 0,
             stream=None):
    """Objective, gradient and Hessian (10 values) at one rotation per particle (L_eval = 0: each L_p)."""
    _need(theta, torch.float32, "theta")
    out = torch.empty((batch.n, 10), dtype=torch.float32, device=C.device)
    bs = batch.c_struct()
    _check(lib().matcha_evaluate(ctx.handle, ct.byref(bs), _ptr(C), int(L_eval), int(fp64_above), _ptr(theta), _ptr(out),
                                 ct.c_void_p(_stream(stream))), "matcha_evaluate")
    return out


def workspace_bytes(batch: Batch, Kc: int = 0) -> int:
    bs = batch.c_struct()
    return int(lib().matcha_workspace_size(ct.byref(bs), int(Kc)))


def grad_template(ctx: Context, batch: Batch, f: torch.Tensor, h: torch.Tensor, w: torch.Tensor,
                  best: torch.Tensor, g: torch.Tensor, want_h: bool = True, want_f: bool = True, stream=None):
    """Adjoint of sum_p g_p C_{L_p}(R_p*) at fixed rotations: (grad_h, grad_f), each None if not wanted.
    Gradients are d/dRe + i d/dIm of the full complex arrays, as float32 views of complex pairs."""
    _need(best, torch.float32, "best")
    _need(g, torch.float32, "g")
    gh = torch.empty_like(h) if want_h else None
    gf = torch.empty_like(f) if want_f else None
    ws = None
    nbytes = 0
    if want_h:
        nbytes = workspace_bytes(batch)
        ws = torch.empty(max(nbytes // 4, 1), dtype=torch.float32, device=f.device)
    bs = batch.c_struct()
    _check(lib().matcha_grad_template(ctx.handle, ct.byref(bs), _ptr(f), _ptr(h), _ptr(w), _ptr(best), _ptr(g),
                                      _ptr(gh), _ptr(gf), _ptr(ws), nbytes, ct.c_void_p(_stream(stream))),
           "matcha_grad_template")
    return gh, gf


class Objective(torch.autograd.Function):
    """F_p = C_{L_p}(R_p*) for fixed rotations best[p]; backward through the hand-written adjoint.

    forward(ctx_, batch, f, h, w, best) -> F [P]; f and h are float32 views of complex coefficients."""

    @staticmethod
    def forward(fctx, mctx: Context, batch: Batch, f, h, w, best):
        C = coeff_assemble(mctx, batch, f.detach(), h.detach(), w)
        out = evaluate(mctx, batch, C, 0, best.detach().contiguous())
        fctx.save_for_backward(f.detach(), h.detach(), w, best.detach().contiguous())
        fctx.mctx, fctx.batch = mctx, batch
        return out[:, 0].clone()

    @staticmethod
    def backward(fctx, gF):
        f, h, w, best = fctx.saved_tensors
        gh, gf = grad_template(fctx.mctx, fctx.batch, f, h, w, best, gF.contiguous().float(),
                               want_h=fctx.needs_input_grad[3], want_f=fctx.needs_input_grad[2])
        return None, None, gf, gh, None, None


def align(ctx: Context, batch: Batch, f: torch.Tensor, h: torch.Tensor, w: torch.Tensor, B: int, n_grid: int,
          Kc: int, levels: Sequence[int], steps: int, max_step: float = 0.0, fp64_above: int = 0,
          bufs: dict | None = None, stream=None):
    """The whole path: assembly, SOFFT search, march and selection.  Returns (best, best_idx, status)."""
    b = {} if bufs is None else bufs
    C = coeff_assemble(ctx, batch, f, h, w, C=b.get("C"), stream=stream)
    cand, status = soft_search(ctx, batch, C, B, n_grid, Kc, cand=b.get("cand"), status=b.get("status"),
                               stream=stream)
    best, best_idx, status = march_newton(ctx, batch, C, levels, steps, cand, status, best=b.get("best"),
                                          best_idx=b.get("best_idx"), max_step=max_step, fp64_above=fp64_above,
                                          stream=stream)
    if bufs is not None:
        bufs.update(C=C, cand=cand, status=status, best=best, best_idx=best_idx)
    return best, best_idx, status


class AlignGraph:
    """The whole path (assembly, SOFFT search, march) for fixed buffers, captured once into a HIP
    graph and replayed with one launch."""

    def __init__(self, ctx: Context, batch: Batch, f, h, w, B: int, n_grid: int, Kc: int, levels, steps: int,
                 prec: int = FP32, fp64_above: int = 0):
        dev = f.device
        self.bufs = dict(C=torch.empty(2 * batch.c_total, dtype=torch.float32, device=dev),
                         cand=torch.empty((batch.n, Kc, 4), dtype=torch.float32, device=dev),
                         status=torch.empty(batch.n, dtype=torch.int32, device=dev),
                         best=torch.empty((batch.n, 4), dtype=torch.float32, device=dev),
                         best_idx=torch.empty(batch.n, dtype=torch.int32, device=dev))
        self._keep = (ctx, batch, f, h, w)
        self._bs = batch.c_struct()
        self._soft = _SoftCfg(B, n_grid, Kc)
        self._march = _march_cfg(levels, steps, fp64_above=fp64_above)
        g = ct.c_void_p()
        b = self.bufs
        _check(lib().matcha_align_graph_create(ctx.handle, ct.byref(self._bs), _ptr(f), _ptr(h), _ptr(w), _ptr(b["C"]),
                                               prec, ct.byref(self._soft), ct.byref(self._march), _ptr(b["cand"]),
                                               _ptr(b["best"]), _ptr(b["best_idx"]), _ptr(b["status"]), ct.byref(g)),
               "matcha_align_graph_create")
        self.handle = g

    def launch(self, stream=None):
        _check(lib().matcha_graph_launch(self.handle, ct.c_void_p(_stream(stream))), "matcha_graph_launch")
        return self.bufs["best"], self.bufs["best_idx"], self.bufs["status"]

    def close(self):
        if self.handle:
            lib().matcha_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ctx: Context, batch: Batch, C: torch.Tensor, B: int, n_grid: int, Kc: int, levels, steps: int,
             reps: int = 2, fp64_above: int = 0) -> dict:
    """Times the supported launch shapes on this batch and keeps the fastest in the context."""
    dev = C.device
    cand = torch.empty((batch.n, Kc, 4), dtype=torch.float32, device=dev)
    status = torch.empty(batch.n, dtype=torch.int32, device=dev)
    best = torch.empty((batch.n, 4), dtype=torch.float32, device=dev)
    best_idx = torch.empty(batch.n, dtype=torch.int32, device=dev)
    soft = _SoftCfg(B, n_grid, Kc)
    march = _march_cfg(levels, steps, fp64_above=fp64_above)
    t = _Tuning()
    bs = batch.c_struct()
    _check(lib().matcha_autotune(ctx.handle, ct.byref(bs), _ptr(C), ct.byref(soft), ct.byref(march), _ptr(cand),
                                 _ptr(best), _ptr(best_idx), _ptr(status), int(reps), ct.byref(t)), "matcha_autotune")
    return {"march_nc": int(t.march_nc), "soft_threads": int(t.soft_threads)}


# ------------------------------------------------------------ layout helpers
def wedge_index(L: int):
    """For the wedge layout of band L: arrays (l, m, n, partner_m, partner_n) per stored float4."""
    ls, ms, ns = [], [], []
    for l in range(L + 1):
        for m in range(l + 1):
            for n in range(-m, m + 1):
                ls.append(l)
                ms.append(m)
                ns.append(n)
    l, m, n = (np.array(x, dtype=np.int64) for x in (ls, ms, ns))
    pm = np.where(n >= 0, n, -n)
    pn = np.where(n >= 0, m, -m)
    return l, m, n, pm, pn


def canonical_at(l, m, n):
    """Offset of C^l_mn in the packed-by-l canonical layout (block l at l(4l^2-1)/3)."""
    return l * (4 * l * l - 1) // 3 + (m + l) * (2 * l + 1) + (n + l)
