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

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_WORKSPACE, ERR_NOT_PREPARED = 0, -1, -2, -3, -4, -5
FP32, BF16_FP32ACC = 0, 1
ST_NONFINITE, ST_INDEFINITE, ST_SINGULAR, ST_NEAR_POLE, ST_FEW_MAXIMA, ST_EARLY_STOP = 1, 2, 4, 8, 16, 32
MAX_L, MAX_KC, MAX_LEVELS = 64, 64, 16

EXPORTED = ["matcha_create", "matcha_destroy", "matcha_prepare", "matcha_status_string", "matcha_set_tuning",
            "matcha_get_tuning", "matcha_c_elems", "matcha_f_elems", "matcha_workspace_size", "matcha_lpt_order",
            "matcha_coeff_assemble", "matcha_soft_search", "matcha_march_newton", "matcha_evaluate",
            "matcha_grad_template", "matcha_align_graph_create", "matcha_graph_launch", "matcha_graph_destroy",
            "matcha_autotune", "matcha_c_unpack", "matcha_soft_search_noalloc", "matcha_grad_workspace_size",
            "matcha_ball_index", "matcha_ball_prepare", "matcha_ball_workspace_size", "matcha_ball_transform",
            "matcha_lowrank_spectrum", "matcha_fft_prepare", "matcha_translate_workspace_size",
            "matcha_volume_spectrum", "matcha_shift_volumes", "matcha_translation_search"]
NOALLOC_SCRATCH_BYTES = 128 << 20
BALL_MAX_L, BALL_MAX_LAMBDA, BALL_MAX_N = 63, 71.0, 256


class MatchaError(RuntimeError):
    pass


class _Batch(ct.Structure):
    _fields_ = [("n_particles", ct.c_int32), ("L_max", ct.c_int32),
                ("L_host", ct.POINTER(ct.c_int32)), ("R_host", ct.POINTER(ct.c_int32)),
                ("L_dev", ct.c_void_p), ("R_dev", ct.c_void_p), ("f_offset", ct.c_void_p), ("C_offset", ct.c_void_p),
                ("L_h", ct.c_int32), ("R_h", ct.c_int32), ("order", ct.c_void_p)]


TUNING_FIELDS = ("march_nc", "soft_threads", "asm_tiles", "grid_nodes", "march_persistent")


class _Tuning(ct.Structure):
    _fields_ = [(name, ct.c_int32) for name in TUNING_FIELDS]


class _SoftCfg(ct.Structure):
    _fields_ = [("B", ct.c_int32), ("n_grid", ct.c_int32), ("Kc", ct.c_int32)]


class _MarchCfg(ct.Structure):
    _fields_ = [("levels", ct.POINTER(ct.c_int32)), ("n_levels", ct.c_int32), ("steps", ct.c_int32),
                ("max_step", ct.c_double), ("early_stop", ct.c_int32),
                ("tol_grad", ct.c_double), ("tol_step", ct.c_double), ("tol_rel", ct.c_double),
                ("fp64_above", ct.c_int32), ("C_final", ct.c_void_p), ("gd_rate", ct.c_double)]


class _AlignBufs(ct.Structure):
    _fields_ = [("f", ct.c_void_p), ("h", ct.c_void_p), ("w", ct.c_void_p), ("prec", ct.c_int),
                ("f32", ct.c_void_p), ("h32", ct.c_void_p), ("C", ct.c_void_p), ("C32", ct.c_void_p),
                ("cand", ct.c_void_p), ("best", ct.c_void_p), ("best_idx", ct.c_void_p), ("status", ct.c_void_p)]


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
        L.matcha_create.argtypes = [ct.c_int, ct.c_char_p, ct.POINTER(vp)]
        L.matcha_destroy.argtypes = [vp]
        L.matcha_prepare.argtypes = [vp, i32, i32]
        L.matcha_status_string.argtypes = [ct.c_int]
        L.matcha_status_string.restype = ct.c_char_p
        L.matcha_set_tuning.argtypes = [vp, ct.POINTER(_Tuning)]
        L.matcha_get_tuning.argtypes = [vp, ct.POINTER(_Tuning)]
        L.matcha_c_elems.argtypes = [i32]
        L.matcha_c_elems.restype = i64
        L.matcha_f_elems.argtypes = [i32, i32]
        L.matcha_f_elems.restype = i64
        L.matcha_workspace_size.argtypes = [vp, bp, ct.POINTER(_SoftCfg), ct.POINTER(_MarchCfg)]
        L.matcha_workspace_size.restype = sz
        L.matcha_grad_workspace_size.argtypes = [bp]
        L.matcha_grad_workspace_size.restype = sz
        L.matcha_coeff_assemble.argtypes = [vp, bp, vp, vp, vp, vp, ct.c_int, vp, sz, vp]
        L.matcha_soft_search.argtypes = [vp, bp, vp, ct.POINTER(_SoftCfg), vp, vp, vp, sz, vp]
        L.matcha_march_newton.argtypes = [vp, bp, vp, ct.POINTER(_MarchCfg), i32, vp, vp, vp, vp, vp, sz, vp]
        L.matcha_evaluate.argtypes = [vp, bp, vp, i32, i32, vp, vp, vp]
        L.matcha_grad_template.argtypes = [vp, bp, vp, vp, vp, vp, vp, vp, vp, ct.c_int, vp, sz, vp]
        L.matcha_lpt_order.argtypes = [bp, ct.POINTER(_MarchCfg), ct.POINTER(ct.c_int32)]
        L.matcha_c_unpack.argtypes = [i32, vp, vp]
        L.matcha_soft_search_noalloc.argtypes = [vp, bp, vp, ct.POINTER(_SoftCfg), vp, vp, vp]
        L.matcha_align_graph_create.argtypes = [vp, bp, ct.POINTER(_AlignBufs), ct.POINTER(_SoftCfg),
                                                ct.POINTER(_MarchCfg), vp, sz, ct.POINTER(vp)]
        L.matcha_graph_launch.argtypes = [vp, vp]
        L.matcha_graph_destroy.argtypes = [vp]
        L.matcha_autotune.argtypes = [vp, bp, ct.POINTER(_AlignBufs), ct.POINTER(_SoftCfg), ct.POINTER(_MarchCfg), i32,
                                      vp, sz, ct.POINTER(_Tuning)]
        L.matcha_ball_index.argtypes = [ct.c_double, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), vp, vp]
        L.matcha_ball_prepare.argtypes = [vp, i32, ct.c_double]
        L.matcha_lowrank_spectrum.argtypes = [vp, bp, vp, vp, vp, ct.c_double, i32, vp, vp, vp]
        L.matcha_fft_prepare.argtypes = [vp, i32, i32]
        L.matcha_translate_workspace_size.argtypes = [vp, i32, i32, i32]
        L.matcha_translate_workspace_size.restype = sz
        L.matcha_volume_spectrum.argtypes = [vp, i32, i32, vp, vp, vp, sz, vp]
        L.matcha_shift_volumes.argtypes = [vp, i32, i32, vp, vp, vp, vp, sz, vp]
        L.matcha_translation_search.argtypes = [vp, i32, i32, vp, vp, vp, i32, i32, vp, vp, sz, vp]
        L.matcha_ball_workspace_size.argtypes = [vp, i32, ct.c_double, i32]
        L.matcha_ball_workspace_size.restype = sz
        L.matcha_ball_transform.argtypes = [vp, i32, ct.c_double, i32, vp, vp, vp, sz, vp]
        for name in ["matcha_create", "matcha_destroy", "matcha_prepare", "matcha_set_tuning", "matcha_get_tuning",
                     "matcha_lpt_order", "matcha_coeff_assemble", "matcha_soft_search", "matcha_march_newton",
                     "matcha_evaluate", "matcha_grad_template", "matcha_align_graph_create", "matcha_graph_launch",
                     "matcha_graph_destroy", "matcha_autotune", "matcha_c_unpack", "matcha_soft_search_noalloc",
                     "matcha_ball_index", "matcha_ball_prepare", "matcha_ball_transform", "matcha_lowrank_spectrum",
                     "matcha_fft_prepare", "matcha_volume_spectrum", "matcha_shift_volumes",
                     "matcha_translation_search"]:
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
    """A libmatcha context on one device (owns the read-only tables and the tuning).

    As the caller of the C ABI, this object also owns a workspace tensor that the eager calls
    share (grown on demand; torch orders its reuse on the current stream)."""

    def __init__(self, device: int | None = None, tune_cache: str | None = None):
        dev = torch.cuda.current_device() if device is None else int(device)
        h = ct.c_void_p()
        _check(lib().matcha_create(dev, tune_cache.encode() if tune_cache else None, ct.byref(h)), "matcha_create")
        self.handle = h
        self.device = dev
        self._prepared = set()
        self._balls = {}
        self._ws = None

    def prepare(self, B: int, n_grid: int):
        """SOFFT node tables for band B on an n_grid^3 grid (synchronous; needed before capture)."""
        if (B, n_grid) not in self._prepared:
            _check(lib().matcha_prepare(self.handle, int(B), int(n_grid)), "matcha_prepare")
            self._prepared.add((B, n_grid))

    def workspace(self, nbytes: int) -> torch.Tensor | None:
        """A device buffer of at least nbytes (None for 0), reused by later eager calls."""
        if nbytes <= 0:
            return None
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def set_tuning(self, march_nc: int = 0, soft_threads: int = 0, asm_tiles: int = 0, grid_nodes: int = 0,
                   march_persistent: int = 0):
        t = _Tuning(int(march_nc), int(soft_threads), int(asm_tiles), int(grid_nodes), int(march_persistent))
        _check(lib().matcha_set_tuning(self.handle, ct.byref(t)), "matcha_set_tuning")

    def get_tuning(self) -> dict:
        t = _Tuning()
        _check(lib().matcha_get_tuning(self.handle, ct.byref(t)), "matcha_get_tuning")
        return {name: int(getattr(t, name)) for name in TUNING_FIELDS}

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


# Early-stopping tolerances (Sec. 2.4): the oracle's defaults, so that both sides stop at the same
# tests unless a caller chooses otherwise.
TOL_GRAD, TOL_STEP, TOL_REL = 1e-9, 1e-10, 1e-13


def _march_cfg(levels, steps, max_step=0.0, early_stop=False, tol_grad=TOL_GRAD, tol_step=TOL_STEP, tol_rel=TOL_REL,
               fp64_above=0, C_final=None, gd_rate=0.0):
    lv = np.ascontiguousarray(levels, dtype=np.int32)
    cfg = _MarchCfg(lv.ctypes.data_as(ct.POINTER(ct.c_int32)), len(lv), int(steps), float(max_step),
                    int(early_stop), float(tol_grad), float(tol_step), float(tol_rel), int(fp64_above),
                    None if C_final is None else C_final.data_ptr(), float(gd_rate))
    cfg._keep = lv  # the levels array must outlive the struct
    return cfg


def grad_workspace_bytes(batch: "Batch") -> int:
    """matcha_grad_workspace_size: the adjoint's workspace for this batch."""
    bs = batch.c_struct()
    return int(lib().matcha_grad_workspace_size(ct.byref(bs)))


def workspace_bytes(batch: "Batch", B: int = 0, n_grid: int = 0, ctx: "Context | None" = None) -> int:
    """matcha_workspace_size: bytes with which the forward calls on this batch run in one pass (the
    SOFFT share only when B and n_grid are given)."""
    bs = batch.c_struct()
    soft = _SoftCfg(int(B), int(n_grid), 1) if B and n_grid else None
    return int(lib().matcha_workspace_size(ctx.handle if ctx else None, ct.byref(bs),
                                           ct.byref(soft) if soft is not None else None, None))


def coeff_assemble(ctx: Context, batch: Batch, f: torch.Tensor, h: torch.Tensor, w: torch.Tensor,
                   C: torch.Tensor | None = None, prec: int = FP32, stream=None) -> torch.Tensor:
    """C (wedge layout, float32 view of complex pairs) = assembly of f against h (eq. sigmalmm)."""
    _need(w, torch.float32, "w")
    if C is None:
        C = torch.empty(2 * batch.c_total, dtype=torch.float32, device=f.device)
    _need(C, torch.float32, "C")
    bs = batch.c_struct()
    nb = workspace_bytes(batch) if int(batch.L.min(initial=0)) != int(batch.L.max(initial=0)) else 0
    ws = ctx.workspace(nb)
    _check(lib().matcha_coeff_assemble(ctx.handle, ct.byref(bs), _ptr(f), _ptr(h), _ptr(w), _ptr(C), prec, _ptr(ws), nb,
                                       ct.c_void_p(_stream(stream))), "matcha_coeff_assemble")
    return C


def soft_search(ctx: Context, batch: Batch, C: torch.Tensor, B: int, n_grid: int, Kc: int,
                cand: torch.Tensor | None = None, status: torch.Tensor | None = None, stream=None):
    if cand is None:
        cand = torch.empty((batch.n, Kc, 4), dtype=torch.float32, device=C.device)
    if status is None:
        status = torch.empty(batch.n, dtype=torch.int32, device=C.device)
    _need(cand, torch.float32, "cand")
    ctx.prepare(B, n_grid)
    bs = batch.c_struct()
    cfg = _SoftCfg(B, n_grid, Kc)
    nb = workspace_bytes(batch, B, n_grid)
    ws = ctx.workspace(nb)
    _check(lib().matcha_soft_search(ctx.handle, ct.byref(bs), _ptr(C), ct.byref(cfg), _ptr(cand), _ptr(status),
                                    _ptr(ws), nb, ct.c_void_p(_stream(stream))), "matcha_soft_search")
    return cand, status


def soft_search_noalloc(ctx: Context, batch: Batch, C: torch.Tensor, B: int, n_grid: int, Kc: int,
                        cand: torch.Tensor, status: torch.Tensor, stream=None):
    """matcha_soft_search_noalloc: the search with the library's static device scratch as workspace
    ((B, n_grid) must be prepared; nothing is allocated)."""
    _need(cand, torch.float32, "cand")
    bs = batch.c_struct()
    cfg = _SoftCfg(B, n_grid, Kc)
    _check(lib().matcha_soft_search_noalloc(ctx.handle, ct.byref(bs), _ptr(C), ct.byref(cfg), _ptr(cand),
                                            _ptr(status), ct.c_void_p(_stream(stream))), "matcha_soft_search_noalloc")
    return cand, status


def march_newton(ctx: Context, batch: Batch, C: torch.Tensor, levels: Sequence[int], steps: int,
                 cand: torch.Tensor, status: torch.Tensor, best: torch.Tensor | None = None,
                 best_idx: torch.Tensor | None = None, max_step: float = 0.0, early_stop: bool = False,
                 tol_grad: float = TOL_GRAD, tol_step: float = TOL_STEP, tol_rel: float = TOL_REL, fp64_above: int = 0,
                 C_final: torch.Tensor | None = None, gd_rate: float = 0.0, stream=None):
    """C_final (same layout as C): coefficients for each particle's final level (None: C).
    gd_rate > 0: gradient ascent steps instead of Newton steps (the first-order comparator)."""
    Kc = int(cand.shape[1])
    if best is None:
        best = torch.empty((batch.n, 4), dtype=torch.float32, device=C.device)
    if best_idx is None:
        best_idx = torch.empty(batch.n, dtype=torch.int32, device=C.device)
    if C_final is not None:
        _need(C_final, torch.float32, "C_final")
    cfg = _march_cfg(levels, steps, max_step, early_stop, tol_grad, tol_step, tol_rel, fp64_above, C_final, gd_rate)
    bs = batch.c_struct()
    nb = workspace_bytes(batch)
    ws = ctx.workspace(nb)
    _check(lib().matcha_march_newton(ctx.handle, ct.byref(bs), _ptr(C), ct.byref(cfg), Kc, _ptr(cand), _ptr(best),
                                     _ptr(best_idx), _ptr(status), _ptr(ws), nb, ct.c_void_p(_stream(stream))),
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


def grad_template(ctx: Context, batch: Batch, f: torch.Tensor, h: torch.Tensor, w: torch.Tensor,
                  best: torch.Tensor, g: torch.Tensor, want_h: bool = True, want_f: bool = True, stream=None):
    """Adjoint of sum_p g_p C_{L_p}(R_p*) at fixed rotations: (grad_h, grad_f), each None if not wanted.
    Gradients are d/dRe + i d/dIm of the full complex arrays, as float32 views of complex pairs."""
    _need(best, torch.float32, "best")
    _need(g, torch.float32, "g")
    gh = torch.empty_like(h) if want_h else None
    gf = torch.empty_like(f) if want_f else None
    nbytes = grad_workspace_bytes(batch) if want_h else 0
    ws = ctx.workspace(nbytes)
    bs = batch.c_struct()
    _check(lib().matcha_grad_template(ctx.handle, ct.byref(bs), _ptr(f), _ptr(h), _ptr(w), _ptr(best), _ptr(g),
                                      _ptr(gh), _ptr(gf), FP32, _ptr(ws), nbytes, ct.c_void_p(_stream(stream))),
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
          prec: int = FP32, f32: torch.Tensor | None = None, h32: torch.Tensor | None = None,
          early_stop: bool = False, tol_grad: float = TOL_GRAD, tol_step: float = TOL_STEP, tol_rel: float = TOL_REL,
          bufs: dict | None = None, gd_rate: float = 0.0, stream=None):
    """The whole path: assembly, SOFFT search, march and selection.  Returns (best, best_idx, status).

    prec = BF16_FP32ACC with f32 / h32 given: the final level marches on FP32-assembled coefficients."""
    b = {} if bufs is None else bufs
    C = coeff_assemble(ctx, batch, f, h, w, C=b.get("C"), prec=prec, stream=stream)
    C32 = None
    if f32 is not None or h32 is not None:
        C32 = coeff_assemble(ctx, batch, f32, h32, w, C=b.get("C32"), prec=FP32, stream=stream)
    cand, status = soft_search(ctx, batch, C, B, n_grid, Kc, cand=b.get("cand"), status=b.get("status"),
                               stream=stream)
    best, best_idx, status = march_newton(ctx, batch, C, levels, steps, cand, status, best=b.get("best"),
                                          best_idx=b.get("best_idx"), max_step=max_step, early_stop=early_stop,
                                          tol_grad=tol_grad, tol_step=tol_step, tol_rel=tol_rel,
                                          fp64_above=fp64_above, C_final=C32, gd_rate=gd_rate, stream=stream)
    if bufs is not None:
        bufs.update(C=C, cand=cand, status=status, best=best, best_idx=best_idx)
        if C32 is not None:
            bufs.update(C32=C32)
    return best, best_idx, status


class AlignGraph:
    """The whole path (assembly, SOFFT search, march) for fixed buffers and a workspace of its own,
    captured once into a HIP graph (matcha_align_graph_create) and replayed with one launch.

    prec = BF16_FP32ACC with f32 / h32: the graph also assembles FP32 coefficients from f32 / h32
    and marches each particle's final level on them."""

    def __init__(self, ctx: Context, batch: Batch, f, h, w, B: int, n_grid: int, Kc: int, levels, steps: int,
                 prec: int = FP32, fp64_above: int = 0, f32=None, h32=None):
        dev = f.device
        ctx.prepare(B, n_grid)
        fin = f32 is not None
        self.bufs = dict(C=torch.empty(2 * batch.c_total, dtype=torch.float32, device=dev),
                         C32=torch.empty(2 * batch.c_total, dtype=torch.float32, device=dev) if fin else None,
                         cand=torch.empty((batch.n, Kc, 4), dtype=torch.float32, device=dev),
                         status=torch.empty(batch.n, dtype=torch.int32, device=dev),
                         best=torch.empty((batch.n, 4), dtype=torch.float32, device=dev),
                         best_idx=torch.empty(batch.n, dtype=torch.int32, device=dev))
        nb = workspace_bytes(batch, B, n_grid)
        self.ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        self._keep = (ctx, batch, f, h, w, f32, h32)
        self._bs = batch.c_struct()
        self._soft = _SoftCfg(B, n_grid, Kc)
        self._march = _march_cfg(levels, steps, fp64_above=fp64_above)
        b = self.bufs
        self._io = _AlignBufs(f.data_ptr(), h.data_ptr(), w.data_ptr(), int(prec),
                              f32.data_ptr() if fin else None, h32.data_ptr() if fin else None,
                              b["C"].data_ptr(), b["C32"].data_ptr() if fin else None, b["cand"].data_ptr(),
                              b["best"].data_ptr(), b["best_idx"].data_ptr(), b["status"].data_ptr())
        g = ct.c_void_p()
        _check(lib().matcha_align_graph_create(ctx.handle, ct.byref(self._bs), ct.byref(self._io), ct.byref(self._soft),
                                               ct.byref(self._march), _ptr(self.ws), nb, ct.byref(g)),
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


def autotune(ctx: Context, batch: Batch, f: torch.Tensor, h: torch.Tensor, w: torch.Tensor, B: int, n_grid: int,
             Kc: int, levels, steps: int, reps: int = 2, fp64_above: int = 0, prec: int = FP32) -> dict:
    """Times the supported launch and tile shapes on this batch (assembly of f, h, w; search; march)
    and keeps the fastest in the context, or applies the context's tune cache entry for this batch
    and configuration."""
    dev = f.device
    ctx.prepare(B, n_grid)
    C = torch.empty(2 * batch.c_total, dtype=torch.float32, device=dev)
    cand = torch.empty((batch.n, Kc, 4), dtype=torch.float32, device=dev)
    status = torch.empty(batch.n, dtype=torch.int32, device=dev)
    best = torch.empty((batch.n, 4), dtype=torch.float32, device=dev)
    best_idx = torch.empty(batch.n, dtype=torch.int32, device=dev)
    io = _AlignBufs(f.data_ptr(), h.data_ptr(), w.data_ptr(), int(prec), None, None, C.data_ptr(), None,
                    cand.data_ptr(), best.data_ptr(), best_idx.data_ptr(), status.data_ptr())
    soft = _SoftCfg(B, n_grid, Kc)
    march = _march_cfg(levels, steps, fp64_above=fp64_above)
    nb = workspace_bytes(batch, B, n_grid)
    ws = ctx.workspace(nb)
    t = _Tuning()
    bs = batch.c_struct()
    _check(lib().matcha_autotune(ctx.handle, ct.byref(bs), ct.byref(io), ct.byref(soft), ct.byref(march), int(reps),
                                 _ptr(ws), nb, ct.byref(t)), "matcha_autotune")
    return {name: int(getattr(t, name)) for name in TUNING_FIELDS}


def c_unpack(L: int, C_wedge: np.ndarray) -> np.ndarray:
    """One particle's wedge-layout C (host complex64 [matcha_c_elems(L)]) in the packed-by-l
    layout (complex64 [sum_{l<=L} (2l+1)^2]), through matcha_c_unpack."""
    cw = np.ascontiguousarray(C_wedge, dtype=np.complex64)
    if cw.size != c_elems(L):
        raise MatchaError(f"C_wedge has {cw.size} values, band {L} needs {c_elems(L)}")
    out = np.zeros((L + 1) * (2 * L + 1) * (2 * L + 3) // 3, dtype=np.complex64)
    _check(lib().matcha_c_unpack(int(L), cw.ctypes.data, out.ctypes.data), "matcha_c_unpack")
    return out


# ------------------------------------------------------------ low-rank structure
LOWRANK_MAX_SHELLS = 48


def lowrank_spectrum(ctx: Context, batch: Batch, f: torch.Tensor, h: torch.Tensor, w: torch.Tensor,
                     rho: float = 0.2, n_sv: int | None = None, stream=None):
    """matcha_lowrank_spectrum: singular values of every C^l (float64 [P, L_max+1, n_sv], descending)
    and the effective ranks at rho (int32 [P, L_max+1])."""
    _need(f, torch.float32, "f")
    _need(h, torch.float32, "h")
    L_max = int(batch.L.max()) if batch.n else 0
    if n_sv is None:
        n_sv = int(min(64, max(1, int(batch.R.max()) if batch.n else 1)))
    sv = torch.zeros((batch.n, L_max + 1, n_sv), dtype=torch.float64, device=f.device)
    r_eff = torch.zeros((batch.n, L_max + 1), dtype=torch.int32, device=f.device)
    bs = batch.c_struct()
    _check(lib().matcha_lowrank_spectrum(ctx.handle, ct.byref(bs), _ptr(f), _ptr(h), _ptr(w), float(rho), int(n_sv),
                                         _ptr(sv), _ptr(r_eff), ct.c_void_p(_stream(stream))),
           "matcha_lowrank_spectrum")
    return sv, r_eff


# ------------------------------------------------------------ translations (App. C)
def fft_prepare(ctx: Context, N: int, n: int):
    """matcha_fft_prepare: hipFFT plans for n volumes of N^3 (synchronous, once per shape)."""
    key = ("fft", int(N), int(n))
    if key not in ctx._prepared:
        _check(lib().matcha_fft_prepare(ctx.handle, int(N), int(n)), "matcha_fft_prepare")
        ctx._prepared.add(key)


def _trans_ws(ctx: Context, N: int, n: int, upsample: int = 1):
    fft_prepare(ctx, N, n)
    nb = int(lib().matcha_translate_workspace_size(ctx.handle, int(N), int(n), int(upsample)))
    return ctx.workspace(nb), nb


def _vols(u: torch.Tensor, name: str):
    _need(u, torch.float32, name)
    if u.dim() != 4 or not (u.shape[1] == u.shape[2] == u.shape[3]):
        raise MatchaError(f"{name} must be [n, N, N, N]")
    return int(u.shape[0]), int(u.shape[1])


def volume_spectrum(ctx: Context, vols: torch.Tensor, stream=None) -> torch.Tensor:
    """matcha_volume_spectrum: complex64 [n, N, N, N/2+1], the unnormalised forward transforms."""
    n, N = _vols(vols, "vols")
    spec = torch.empty((n, N, N, N // 2 + 1), dtype=torch.complex64, device=vols.device)
    ws, nb = _trans_ws(ctx, N, n)
    _check(lib().matcha_volume_spectrum(ctx.handle, N, n, _ptr(vols), _ptr(spec), _ptr(ws), nb,
                                        ct.c_void_p(_stream(stream))), "matcha_volume_spectrum")
    return spec


def shift_volumes(ctx: Context, spec: torch.Tensor, shifts: torch.Tensor, stream=None) -> torch.Tensor:
    """matcha_shift_volumes: f_p(x + s_p) from the spectra; shifts float32 [n, 4] (x, y, z, .) voxels."""
    _need(spec, torch.complex64, "spec")
    _need(shifts, torch.float32, "shifts")
    n, N = int(spec.shape[0]), int(spec.shape[1])
    out = torch.empty((n, N, N, N), dtype=torch.float32, device=spec.device)
    ws, nb = _trans_ws(ctx, N, n)
    _check(lib().matcha_shift_volumes(ctx.handle, N, n, _ptr(spec), _ptr(shifts), _ptr(out), _ptr(ws), nb,
                                      ct.c_void_p(_stream(stream))), "matcha_shift_volumes")
    return out


def translation_search(ctx: Context, spec_f: torch.Tensor, h: torch.Tensor, euler: torch.Tensor, window: int,
                       upsample: int = 10, stream=None) -> torch.Tensor:
    """matcha_translation_search: float32 [n, 4] (s_x, s_y, s_z, c(s)), the shift maximising
    sum_x f_p(x) h(R_p^T (x - s)); euler float32 [n, 4] (a, b, c, .)."""
    _need(spec_f, torch.complex64, "spec_f")
    _need(h, torch.float32, "h")
    _need(euler, torch.float32, "euler")
    n, N = int(spec_f.shape[0]), int(spec_f.shape[1])
    out = torch.empty((n, 4), dtype=torch.float32, device=spec_f.device)
    ws, nb = _trans_ws(ctx, N, n, upsample)
    _check(lib().matcha_translation_search(ctx.handle, N, n, _ptr(spec_f), _ptr(h), _ptr(euler), int(window),
                                           int(upsample), _ptr(out), _ptr(ws), nb, ct.c_void_p(_stream(stream))),
           "matcha_translation_search")
    return out


def align6d(ctx: Context, f_vols: torch.Tensor, h_vol: torch.Tensor, lam: float, B: int, n_grid: int, Kc: int,
            levels: Sequence[int], steps: int, T: int = 3, window: int | None = None, upsample: int = 10,
            fp64_above: int = 0):
    """Rotation-translation alternation (App. C), T rounds from zero shift: the ball transform of the
    shifted particles f_p(x + s_p) and the path against the template's coefficients (rotations),
    then the translation search at those rotations (shifts).  Returns (best [n, 4] rotations as the
    march writes them, shifts [n, 4] (s, c(s)), status): f_p ~ S_s (g o h), tau = R_g^T s."""
    n, N = _vols(f_vols, "f_vols")
    window = N // 4 if window is None else int(window)
    spec = volume_spectrum(ctx, f_vols)
    hc = ball_transform(ctx, h_vol, lam)
    K, nlm = int(hc.shape[0]), int(hc.shape[1])
    L = int(round(nlm ** 0.5)) - 1
    batch = Batch.make([L] * n, [K] * n, L, K)
    h_flat = hc.contiguous().view(torch.float32).reshape(-1)
    w = torch.ones(K, dtype=torch.float32, device=f_vols.device)
    shifts = torch.zeros((n, 4), dtype=torch.float32, device=f_vols.device)
    best = status = None
    for t in range(T):
        fs = f_vols if t == 0 else shift_volumes(ctx, spec, shifts)
        fc = ball_transform(ctx, fs, lam)
        best, _, status = align(ctx, batch, fc.contiguous().view(torch.float32).reshape(-1), h_flat, w, B, n_grid,
                                Kc, levels, steps, fp64_above=fp64_above)
        shifts = translation_search(ctx, spec, h_vol, best, window, upsample)
    return best, shifts, status


# ------------------------------------------------------------ ball-harmonic front end
def ball_index(lam: float):
    """matcha_ball_index: (L, zeros) with zeros[l] the kept lam_lk of degree l (float64 arrays)."""
    L, K = ct.c_int32(), ct.c_int32()
    _check(lib().matcha_ball_index(float(lam), ct.byref(L), ct.byref(K), None, None), "matcha_ball_index")
    nk = np.zeros(L.value + 1, dtype=np.int32)
    z = np.zeros((L.value + 1, K.value), dtype=np.float64)
    _check(lib().matcha_ball_index(float(lam), ct.byref(L), ct.byref(K), nk.ctypes.data, z.ctypes.data),
           "matcha_ball_index")
    return L.value, [z[l, :nk[l]].copy() for l in range(L.value + 1)]


def ball_prepare(ctx: Context, N: int, lam: float):
    """matcha_ball_prepare: the transform's tables for an N^3 grid and Lambda (synchronous)."""
    _check(lib().matcha_ball_prepare(ctx.handle, int(N), float(lam)), "matcha_ball_prepare")


def ball_transform(ctx: Context, u: torch.Tensor, lam: float, out: torch.Tensor | None = None, stream=None):
    """matcha_ball_transform of real volumes u (float32 CUDA [P, N, N, N] or [N, N, N], index
    (z, y, x)); returns complex64 [P, Kmax, (L+1)^2] (or [Kmax, (L+1)^2]).  The tables for
    (N, lam) are built on first use."""
    _need(u, torch.float32, "u")
    single = u.dim() == 3
    uu = u.unsqueeze(0) if single else u
    if uu.dim() != 4 or not (uu.shape[1] == uu.shape[2] == uu.shape[3]):
        raise MatchaError("u must be [P, N, N, N] or [N, N, N]")
    P, N = int(uu.shape[0]), int(uu.shape[1])
    key = (N, float(lam))
    if key not in ctx._balls:  # the index set and tables are built once per (N, lam)
        L, K = ct.c_int32(), ct.c_int32()
        _check(lib().matcha_ball_index(float(lam), ct.byref(L), ct.byref(K), None, None), "matcha_ball_index")
        ball_prepare(ctx, N, lam)
        ctx._balls[key] = (L.value, K.value)
    L, K = ctx._balls[key]
    nb = int(lib().matcha_ball_workspace_size(ctx.handle, N, float(lam), P))
    ws = ctx.workspace(nb)
    shape = (P, K, (L + 1) ** 2)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=u.device)
    elif tuple(out.shape) != shape:
        raise MatchaError(f"out must have shape {shape}")
    _need(out, torch.complex64, "out")
    _check(lib().matcha_ball_transform(ctx.handle, N, float(lam), P, _ptr(uu), _ptr(out), _ptr(ws), nb,
                                       ct.c_void_p(_stream(stream))), "matcha_ball_transform")
    return out[0] if single else out


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
