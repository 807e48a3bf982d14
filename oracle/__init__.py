"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and bench.py's cpu_baseline leg import this package.
Every array crossing this boundary is a contiguous numpy float64 / complex128 array.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libmatcha_oracle.so")
_lib = None

NONFINITE, INDEFINITE, SINGULAR, NEAR_POLE, FEW_MAXIMA, EARLY_STOP = 1, 2, 4, 8, 16, 32

_dp = ct.POINTER(ct.c_double)
_ip = ct.POINTER(ct.c_int)
_i64p = ct.POINTER(ct.c_int64)
_up = ct.POINTER(ct.c_uint)


def use_native():
    """Rebuilds the oracle with -march=native on this host and loads that build (for CPU timing)."""
    global _lib, _LIB_PATH
    from . import build as _b
    _LIB_PATH = _b.build(native=True)
    _lib = None
    return lib()


def set_num_threads(n: int):
    lib().mo_set_num_threads(int(n))


def max_threads() -> int:
    return int(lib().mo_max_threads())


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ct.CDLL(_LIB_PATH)
        L.mo_set_num_threads.argtypes = [ct.c_int]
        L.mo_max_threads.restype = ct.c_int
        L.mo_term_count.restype = ct.c_long
        L.mo_term_count.argtypes = [ct.c_int]
        L.mo_wigner_d.argtypes = [ct.c_int, ct.c_double, _dp, _dp, _dp]
        L.mo_coeff_assemble.argtypes = [ct.c_int, ct.c_int, _dp, ct.c_int, _dp, ct.c_int, _dp, _dp]
        L.mo_eval.argtypes = [ct.c_int, _dp, ct.c_double, ct.c_double, ct.c_double, _dp]
        L.mo_eval_F.argtypes = [ct.c_int, _dp, ct.c_double, ct.c_double, ct.c_double]
        L.mo_eval_F.restype = ct.c_double
        L.mo_soft_grid.argtypes = [ct.c_int, _dp, ct.c_int, _dp]
        L.mo_soft_select.argtypes = [ct.c_int, _dp, ct.c_int, _i64p, _dp]
        L.mo_soft_select.restype = ct.c_int
        L.mo_newton_step.argtypes = [_dp, ct.c_double, _dp, _dp]
        L.mo_newton_step.restype = ct.c_uint
        L.mo_schedule.argtypes = [ct.c_int, _ip, ct.c_int, _ip]
        L.mo_schedule.restype = ct.c_int
        L.mo_march.argtypes = [ct.c_int, _dp, ct.c_int, _ip, ct.c_int, ct.c_double, ct.c_int, ct.c_double,
                               ct.c_double, ct.c_double, ct.c_double, ct.c_int, _dp, _up]
        L.mo_gradient_step.argtypes = [_dp, ct.c_double, ct.c_int, ct.c_double, _dp, _dp]
        L.mo_gradient_step.restype = ct.c_uint
        L.mo_march.restype = ct.c_int
        L.mo_align_one.argtypes = [ct.c_int, ct.c_int, _dp, _dp, ct.c_int, _dp, ct.c_int, ct.c_int, ct.c_int,
                                   ct.c_int, _ip, ct.c_int, ct.c_double, _dp, _dp, _ip]
        L.mo_align_one.restype = ct.c_uint
        L.mo_grad_one.argtypes = [ct.c_int, ct.c_int, _dp, _dp, ct.c_int, _dp, _dp, ct.c_double, _dp, _dp]
        L.mo_align_batch.argtypes = [ct.c_int, _ip, _ip, _i64p, _dp, _dp, ct.c_int, _dp, ct.c_int, ct.c_int,
                                     ct.c_int, ct.c_int, _ip, ct.c_int, ct.c_double, _dp, _dp, _ip, _up]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def n_terms(L: int) -> int:
    """sum_{l<=L} (2l+1)^2."""
    return int(lib().mo_term_count(L))


def blk(l: int) -> int:
    return l * (4 * l * l - 1) // 3


def at(l: int, m: int, n: int) -> int:
    return blk(l) + (m + l) * (2 * l + 1) + (n + l)


def wigner_d(L: int, beta: float, derivs: bool = True):
    N = n_terms(L)
    d = np.zeros(N)
    d1 = np.zeros(N) if derivs else None
    d2 = np.zeros(N) if derivs else None
    lib().mo_wigner_d(L, float(beta), _d(d), _d(d1) if derivs else None, _d(d2) if derivs else None)
    return (d, d1, d2) if derivs else d


def coeff_assemble(L: int, R: int, f, Lf: int, h, Lh: int, w):
    f, h, w = _c128(f), _c128(h), _f64(w)
    C = np.zeros(n_terms(L), dtype=np.complex128)
    lib().mo_coeff_assemble(L, R, _d(f), Lf, _d(h), Lh, _d(w), _d(C))
    return C


def evaluate(L: int, C, theta):
    C = _c128(C)
    out = np.zeros(10)
    lib().mo_eval(L, _d(C), float(theta[0]), float(theta[1]), float(theta[2]), _d(out))
    return out


def evaluate_F(L: int, C, theta) -> float:
    C = _c128(C)
    return float(lib().mo_eval_F(L, _d(C), float(theta[0]), float(theta[1]), float(theta[2])))


def soft_grid(B: int, C, n: int):
    C = _c128(C)
    g = np.zeros(n * n * n)
    lib().mo_soft_grid(B, _d(C), n, _d(g))
    return g.reshape(n, n, n)


def soft_select(grid, Kc: int):
    grid = _f64(grid)
    n = grid.shape[0]
    idx = np.zeros(Kc, dtype=np.int64)
    val = np.zeros(Kc)
    nmx = lib().mo_soft_select(n, _d(grid), Kc, idx.ctypes.data_as(_i64p), _d(val))
    return idx, val, int(nmx)


def grid_euler(idx, n: int):
    idx = np.asarray(idx, dtype=np.int64)
    i, j, k = idx // (n * n), (idx // n) % n, idx % n
    return np.stack([2 * np.pi * j / n, np.pi * (2 * i + 1) / (2 * n), 2 * np.pi * k / n], -1)


def newton_step(e, theta, max_step: float = 0.0):
    e = _f64(e)
    th = _f64(np.array(theta, dtype=np.float64).copy())
    sinf = np.zeros(1)
    st = lib().mo_newton_step(_d(e), float(max_step), _d(th), _d(sinf))
    return th, int(st), float(sinf[0])


def gradient_step(e, theta, rate: float, L: int, max_step: float = 0.0):
    """One gradient ascent step (the first-order comparator); returns (theta, status, step_inf)."""
    e = _f64(e)
    th = _f64(np.array(theta, dtype=np.float64).copy())
    sinf = np.zeros(1)
    st = lib().mo_gradient_step(_d(e), float(rate), int(L), float(max_step), _d(th), _d(sinf))
    return th, int(st), float(sinf[0])


def schedule(Lp: int, levels):
    lv = _i32(levels)
    out = np.zeros(len(levels) + 1, dtype=np.int32)
    k = lib().mo_schedule(Lp, lv.ctypes.data_as(_ip), len(levels), out.ctypes.data_as(_ip))
    return [int(x) for x in out[:k]]


def march(Lp: int, C, levels, steps: int, cand, max_step: float = 0.0, early_stop: bool = False,
          tol_grad: float = 1e-9, tol_step: float = 1e-10, tol_rel: float = 1e-13, gd_rate: float = 0.0):
    C = _c128(C)
    lv = _i32(levels)
    cand = _f64(np.array(cand, dtype=np.float64).copy())
    Kc = cand.shape[0]
    cst = np.zeros(Kc, dtype=np.uint32)
    best = lib().mo_march(Lp, _d(C), len(levels), lv.ctypes.data_as(_ip), steps, float(max_step), int(early_stop),
                          tol_grad, tol_step, tol_rel, float(gd_rate), Kc, _d(cand), cst.ctypes.data_as(_up))
    return cand, int(best), cst


def align_one(f, Lp: int, Rp: int, h, Lh: int, w, B: int, n: int, Kc: int, levels, steps: int, max_step: float = 0.0):
    f, h, w = _c128(f), _c128(h), _f64(w)
    lv = _i32(levels)
    cand = np.zeros((Kc, 4))
    best = np.zeros(4)
    bi = np.zeros(1, dtype=np.int32)
    st = lib().mo_align_one(Lp, Rp, _d(f), _d(h), Lh, _d(w), B, n, Kc, len(levels), lv.ctypes.data_as(_ip), steps,
                            float(max_step), _d(cand), _d(best), bi.ctypes.data_as(_ip))
    return best, int(bi[0]), int(st), cand


def align_batch(batch, B: int, n: int, Kc: int, levels, steps: int, particles=None, max_step: float = 0.0):
    """Whole path for the listed particles of a synth.Batch (OpenMP over particles)."""
    idx = np.arange(batch.n_particles) if particles is None else np.asarray(particles)
    P = idx.size
    Lp = _i32(batch.L[idx])
    Rp = _i32(batch.R[idx])
    # repack the selected ragged particles
    parts = [batch.f(int(p)).reshape(-1) for p in idx]
    sizes = np.array([x.size for x in parts], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    flat = _c128(np.concatenate(parts))
    h, w = _c128(batch.h), _f64(batch.w)
    lv = _i32(levels)
    cand = np.zeros((P, Kc, 4))
    best = np.zeros((P, 4))
    bi = np.zeros(P, dtype=np.int32)
    st = np.zeros(P, dtype=np.uint32)
    lib().mo_align_batch(P, Lp.ctypes.data_as(_ip), Rp.ctypes.data_as(_ip), off.ctypes.data_as(_i64p), _d(flat),
                         _d(h), batch.L_h, _d(w), B, n, Kc, len(levels), lv.ctypes.data_as(_ip), steps,
                         float(max_step), _d(cand), _d(best), bi.ctypes.data_as(_ip), st.ctypes.data_as(_up))
    return best, bi, st, cand


def grad_one(L: int, R: int, f, h, Lh: int, w, euler, g: float, grad_h=None, want_f: bool = True):
    f, h, w = _c128(f), _c128(h), _f64(w)
    e = _f64(euler)
    gh = grad_h if grad_h is not None else np.zeros_like(h)
    gf = np.zeros_like(f) if want_f else None
    lib().mo_grad_one(L, R, _d(f), _d(h), Lh, _d(w), _d(e), float(g), _d(gh), _d(gf) if want_f else None)
    return gh, gf
