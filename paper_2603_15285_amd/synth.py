"""Seeded synthetic inputs shaped like the paper's rotational-alignment workloads.

This module only *makes inputs*: a template h, a batch of rotated noisy copies f,
the radial weights w, the ground-truth rotations and the SNRs.  It holds none of
the alignment method's arithmetic (no correlation coefficients, no SOFFT, no
Wigner-d recurrence, no Newton step) and is shared as input by the FP64 oracle and
by the HIP path.

Data model (paper Sec. 2.1 and App. A.1): a volume is represented per radial shell r
by complex spherical-harmonic coefficients c_lm(r), l <= L, stored in the packed
order lm = l*l + l + m.  Real volumes (paper Sec. 1, problem statement) give
Hermitian-symmetric coefficients c_{l,-m} = (-1)^m conj(c_lm); the generator
enforces this exactly.

Rotating the template (paper App. A.4: under a rotation the spherical-harmonic
coefficients of degree l mix through the degree-l Wigner-D matrix):
(g o h)_l(r) = D^l(g) h_l(r) with D^l_mn(a,b,c) = e^{-ima} d^l_mn(b) e^{-inc}
(eq. wigner-D) and the ZYZ chart g = r_z(a) r_y(b) r_z(c) (eq. Euler).  Here
d^l(b) = exp(-i b J_y) is formed from the eigen-decomposition of the angular
momentum operator J_y -- a route unrelated to the l-recurrences used by the
oracle and by the GPU kernels, so a convention slip in either of those cannot be
masked by the generator.

Noise: white in the weighted (orthonormal) norm, eta_lm(r) ~ CN(0, s2 / w_r),
with s2 chosen so that sum_r w_r |D h|^2 / E sum_r w_r |eta|^2 equals the linear
SNR (the paper's 0 dB is "equal energy", Sec. 4.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np

SEED_BASE = 2603152850


def n_lm(L: int) -> int:
    """Number of packed (l, m) entries for l <= L."""
    return (L + 1) * (L + 1)


def lm_index(l: int, m: int) -> int:
    return l * l + l + m


# ---------------------------------------------------------------- rotations
def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    """Unit quaternion(s) (w, x, y, z) -> rotation matrices [..., 3, 3]."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - z * w)
    R[..., 0, 2] = 2 * (x * z + y * w)
    R[..., 1, 0] = 2 * (x * y + z * w)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - x * w)
    R[..., 2, 0] = 2 * (x * z - y * w)
    R[..., 2, 1] = 2 * (y * z + x * w)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def euler_zyz_to_matrix(a, b, c) -> np.ndarray:
    """g = r_z(a) r_y(b) r_z(c) with the explicit matrices of eq. Euler."""
    a, b, c = (np.asarray(v, dtype=np.float64) for v in (a, b, c))

    def rz(t):
        R = np.zeros(t.shape + (3, 3))
        R[..., 0, 0] = np.cos(t)
        R[..., 0, 1] = -np.sin(t)
        R[..., 1, 0] = np.sin(t)
        R[..., 1, 1] = np.cos(t)
        R[..., 2, 2] = 1.0
        return R

    def ry(t):
        R = np.zeros(t.shape + (3, 3))
        R[..., 0, 0] = np.cos(t)
        R[..., 0, 2] = np.sin(t)
        R[..., 1, 1] = 1.0
        R[..., 2, 0] = -np.sin(t)
        R[..., 2, 2] = np.cos(t)
        return R

    return rz(a) @ ry(b) @ rz(c)


def matrix_to_euler_zyz(R: np.ndarray) -> np.ndarray:
    """Inverse of euler_zyz_to_matrix away from b in {0, pi}; returns [..., 3]."""
    R = np.asarray(R, dtype=np.float64)
    b = np.arccos(np.clip(R[..., 2, 2], -1.0, 1.0))
    a = np.arctan2(R[..., 1, 2], R[..., 0, 2])
    c = np.arctan2(R[..., 2, 1], -R[..., 2, 0])
    two_pi = 2.0 * math.pi
    return np.stack([np.mod(a, two_pi), b, np.mod(c, two_pi)], axis=-1)


def geodesic_deg(R1: np.ndarray, R2: np.ndarray) -> np.ndarray:
    """Bi-invariant angle between rotations, stable at tiny angles (degrees)."""
    M = np.swapaxes(R1, -1, -2) @ R2
    v = np.stack([M[..., 2, 1] - M[..., 1, 2], M[..., 0, 2] - M[..., 2, 0], M[..., 1, 0] - M[..., 0, 1]], -1)
    tr = M[..., 0, 0] + M[..., 1, 1] + M[..., 2, 2]
    return np.degrees(np.arctan2(np.linalg.norm(v, axis=-1), tr - 1.0))


# ------------------------------------------------- rotation of coefficients
_JY_EIG: dict[int, tuple[np.ndarray, np.ndarray]] = {}


def _jy_eig(l: int):
    """Eigen-decomposition of J_y in the |l m>, m = -l..l basis (cached)."""
    if l not in _JY_EIG:
        m = np.arange(-l, l + 1, dtype=np.float64)
        jp = np.zeros((2 * l + 1, 2 * l + 1), dtype=np.complex128)
        # <m+1| J+ |m> = sqrt((l-m)(l+m+1))
        for i in range(2 * l):
            jp[i + 1, i] = math.sqrt((l - m[i]) * (l + m[i] + 1))
        jy = (jp - jp.conj().T) / 2j
        lam, V = np.linalg.eigh(jy)
        _JY_EIG[l] = (lam, V)
    return _JY_EIG[l]


def wigner_d_expm(l: int, beta: np.ndarray) -> np.ndarray:
    """d^l(beta) = exp(-i beta J_y) for a batch of beta; returns real [..., 2l+1, 2l+1]."""
    lam, V = _jy_eig(l)
    beta = np.asarray(beta, dtype=np.float64)
    ph = np.exp(-1j * beta[..., None] * lam)  # [..., k]
    d = (V[None, :, :] * ph.reshape(-1, 1, lam.size)) @ V.conj().T[None]
    return d.real.reshape(beta.shape + (2 * l + 1, 2 * l + 1))


def rotate_coeffs(h: np.ndarray, L: int, euler: np.ndarray, hermitian: bool = False) -> np.ndarray:
    """(g o h)_l = D^l(g) h_l for a batch of rotations.

    h: [R, (L+1)^2] complex; euler: [P, 3].  Returns [P, R, (L+1)^2] complex128.

    d^l(b) = V e^{-i b Lambda} V^H with J_y = V Lambda V^H, applied to the vectors rather than
    formed: for all particles and shells at once, X = (e^{-inc} h_l) conj(V) and
    Z = (e^{-i b lambda_k} X) V^T are two GEMMs per degree with the shared V; then e^{-ima}.
    hermitian: h is Hermitian-symmetric, c_{l,-m} = (-1)^m conj(c_lm), which D^l of a real rotation
    preserves; the m < 0 half is then written from the m > 0 half so that the output is
    Hermitian-symmetric exactly."""
    euler = np.atleast_2d(np.asarray(euler, dtype=np.float64))
    P, R = euler.shape[0], h.shape[0]
    out = np.empty((P, R, n_lm(L)), dtype=np.complex128)
    a, b, c = euler[:, 0], euler[:, 1], euler[:, 2]
    for l in range(L + 1):
        lam, V = _jy_eig(l)
        m = np.arange(-l, l + 1)
        hl = h[:, l * l: (l + 1) * (l + 1)]  # [R, 2l+1]
        U = np.exp(-1j * c[:, None, None] * m[None, None, :]) * hl[None]  # [P, R, 2l+1]
        X = (U.reshape(P * R, 2 * l + 1) @ V.conj()).reshape(P, R, 2 * l + 1)
        X *= np.exp(-1j * b[:, None, None] * lam[None, None, :])
        Z = (X.reshape(P * R, 2 * l + 1) @ V.T).reshape(P, R, 2 * l + 1)
        Z *= np.exp(-1j * a[:, None, None] * m[None, None, :])
        if not hermitian:
            out[:, :, l * l: (l + 1) * (l + 1)] = Z
            continue
        c0 = l * l + l
        out[:, :, c0] = Z[:, :, l].real
        if l > 0:
            mpos = np.arange(1, l + 1)
            out[:, :, c0 + mpos] = Z[:, :, l + mpos]
            out[:, :, c0 - mpos] = ((-1.0) ** mpos) * np.conj(Z[:, :, l + mpos])
    return out


# ------------------------------------------------------------ random fields
def hermitian_gaussian(rng: np.random.Generator, shape_r: int, L: int, var_l: np.ndarray, scale_r=None) -> np.ndarray:
    """Random coefficients with c_{l,-m} = (-1)^m conj(c_lm) exactly.

    var_l[l]: variance of each coefficient (complex CN for m > 0, real for m = 0);
    scale_r[r]: optional per-shell multiplier of the variance.  The normals are drawn in one call
    and used degree by degree: for each l, R values for m = 0, then R*l real and R*l imaginary
    parts (shell-major) for m = 1..l.
    """
    out = np.zeros((shape_r, n_lm(L)), dtype=np.complex128)
    sr = np.ones(shape_r) if scale_r is None else np.asarray(scale_r, dtype=np.float64)
    z = rng.standard_normal(shape_r * n_lm(L))
    k = 0
    for l in range(L + 1):
        sd = np.sqrt(var_l[l] * sr)  # [R]
        c0 = l * l + l
        out[:, c0] = z[k: k + shape_r] * sd
        k += shape_r
        if l > 0:
            n = shape_r * l
            zc = (z[k: k + n] + 1j * z[k + n: k + 2 * n]).reshape(shape_r, l) * (sd[:, None] / math.sqrt(2.0))
            k += 2 * n
            mpos = np.arange(1, l + 1)
            out[:, c0 + mpos] = zc
            out[:, c0 - mpos] = ((-1.0) ** mpos) * np.conj(zc)
    return out


def haar_euler(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    return matrix_to_euler_zyz(quat_to_matrix(q))


@dataclasses.dataclass
class Batch:
    """A synthetic batch.  f is ragged: particle p occupies f_flat[f_offset[p]:...]
    as an [R_p, (L_p+1)^2] row-major complex array (shell-major, packed lm)."""

    L_h: int
    R_h: int
    h: np.ndarray  # [R_h, (L_h+1)^2] complex128
    w: np.ndarray  # [R_h] float64, w_r = r^2
    L: np.ndarray  # [P] int32
    R: np.ndarray  # [P] int32
    f_offset: np.ndarray  # [P] int64, element offsets into f_flat
    f_flat: np.ndarray  # complex128
    euler_true: np.ndarray  # [P, 3]
    snr: np.ndarray  # [P]

    @property
    def n_particles(self) -> int:
        return int(self.L.shape[0])

    def f(self, p: int) -> np.ndarray:
        Lp, Rp = int(self.L[p]), int(self.R[p])
        o = int(self.f_offset[p])
        return self.f_flat[o: o + Rp * n_lm(Lp)].reshape(Rp, n_lm(Lp))

    def R_true(self) -> np.ndarray:
        e = self.euler_true
        return euler_zyz_to_matrix(e[:, 0], e[:, 1], e[:, 2])


def make_template(L: int, R: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    rng = np.random.default_rng(seed)
    var = (1.0 + np.arange(L + 1)) ** -2.0
    h = hermitian_gaussian(rng, R, L, var)
    w = (np.arange(1, R + 1, dtype=np.float64)) ** 2
    return h, w


_WORKER_TEMPLATE: dict = {}


def _worker_init(h, w):
    _WORKER_TEMPLATE.update(h=h, w=w)


def _particles_chunk(task):
    """Rotated noisy copies of the template for one chunk of particles with equal (L_p, R_p):
    [chunk, R_p (L_p+1)^2] in f_dtype."""
    Lp, Rp, chunk, eul, snrs, rngs, noiseless, f_dtype = task
    h, w = _WORKER_TEMPLATE["h"], _WORKER_TEMPLATE["w"]
    rot = rotate_coeffs(h[:Rp, : n_lm(Lp)], Lp, eul, hermitian=True)
    if not noiseless:
        e_sig = np.einsum("prk,r->p", rot.real ** 2 + rot.imag ** 2, w[:Rp])
        for j in range(len(chunk)):
            s2 = float(e_sig[j]) / (snrs[j] * Rp * n_lm(Lp))
            rot[j] += hermitian_gaussian(rngs[j], Rp, Lp, np.full(Lp + 1, s2), scale_r=1.0 / w[:Rp])
    return rot.reshape(len(chunk), -1).astype(f_dtype)


def _place(f_flat, f_offset, chunk, block):
    for j, p in enumerate(chunk):
        o = f_offset[p]
        f_flat[o: o + block.shape[1]] = block[j]


def _workers(n_values: int, n_tasks: int, workers) -> int:
    """Processes for generating a batch: one unless the caller asks for more (the processes are
    started with the spawn method, which re-imports the caller's main module: only a main module
    guarded by `if __name__ == "__main__"` may ask)."""
    if workers is None or n_values < (1 << 22):
        return 1
    return max(1, min(int(workers), n_tasks))


def make_batch(L_h: int, R_h: int, n_particles: int, *, seed: int, snr=(0.05, 0.2),
               L_per: Sequence[int] | None = None, R_per: Sequence[int] | None = None,
               noiseless: bool = False, euler: np.ndarray | None = None, f_dtype=np.complex128,
               workers: int | None = None) -> Batch:
    """Template h (l <= L_h, R_h shells) and n_particles rotated noisy copies.

    snr: a float (fixed linear SNR) or a (lo, hi) pair drawn uniformly per particle.
    L_per / R_per: per-particle band limit and shell count (default L_h / R_h); a
    particle uses template shells 1..R_p and degrees l <= L_p.
    f_dtype: storage of f (complex64 halves the host memory of the large workloads; both the oracle
    and the GPU then read the same rounded values).
    workers: processes sharing the chunks of particles (default one; see _workers); the result does
    not depend on it.
    """
    h, w = make_template(L_h, R_h, seed)
    ss = np.random.SeedSequence(seed + 1)
    kids = ss.spawn(n_particles)
    L = np.full(n_particles, L_h, dtype=np.int32) if L_per is None else np.asarray(L_per, dtype=np.int32)
    R = np.full(n_particles, R_h, dtype=np.int32) if R_per is None else np.asarray(R_per, dtype=np.int32)
    assert L.max() <= L_h and R.max() <= R_h
    sizes = R.astype(np.int64) * (L.astype(np.int64) + 1) ** 2
    f_offset = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    f_flat = np.empty(int(sizes.sum()), dtype=f_dtype)
    eul = np.empty((n_particles, 3))
    snrs = np.empty(n_particles)
    rngs = [np.random.default_rng(k) for k in kids]
    for p in range(n_particles):
        if euler is None:
            eul[p] = haar_euler(rngs[p], 1)[0]
        else:
            eul[p] = euler[p]
        snrs[p] = snr if np.isscalar(snr) else rngs[p].uniform(snr[0], snr[1])
    # Rotate grouped by (L_p, R_p), in chunks of particles whose size depends only on (L_p, R_p), so
    # that the GEMMs stay large, the temporaries bounded and the result independent of how many
    # processes share the chunks; each particle's noise comes from its own generator.
    keys = np.stack([L, R], 1)
    tasks = []
    for (Lp, Rp) in sorted({tuple(k) for k in keys.tolist()}):
        idx = np.nonzero((L == Lp) & (R == Rp))[0]
        step = max(1, (1 << 22) // (Rp * n_lm(Lp)))
        for s in range(0, idx.size, step):
            chunk = idx[s: s + step]
            tasks.append((int(Lp), int(Rp), chunk, eul[chunk], snrs[chunk], [rngs[p] for p in chunk], noiseless,
                          f_dtype))
    nproc = _workers(int(sizes.sum()), len(tasks), workers)
    if nproc <= 1:
        _WORKER_TEMPLATE.update(h=h, w=w)
        for t, block in zip(tasks, map(_particles_chunk, tasks)):
            _place(f_flat, f_offset, t[2], block)
    else:
        import concurrent.futures as cf
        import multiprocessing as mp
        import os
        # one BLAS thread per worker: the workers start at the first submission and read this then
        saved = os.environ.get("OPENBLAS_NUM_THREADS")
        os.environ["OPENBLAS_NUM_THREADS"] = "1"
        try:
            with cf.ProcessPoolExecutor(nproc, mp_context=mp.get_context("spawn"), initializer=_worker_init,
                                        initargs=(h, w)) as ex:
                for t, block in zip(tasks, ex.map(_particles_chunk, tasks)):
                    _place(f_flat, f_offset, t[2], block)
        finally:
            if saved is None:
                del os.environ["OPENBLAS_NUM_THREADS"]
            else:
                os.environ["OPENBLAS_NUM_THREADS"] = saved
    return Batch(L_h=L_h, R_h=R_h, h=h, w=w, L=L, R=R, f_offset=f_offset, f_flat=f_flat,
                 euler_true=eul, snr=snrs)


# ----------------------------------------------------- workload definitions
@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_particles: int
    L: int
    R: int
    B: int
    Kc: int
    levels: tuple
    steps: int
    snr: object
    uneven: bool = False

    @property
    def n_grid(self) -> int:
        return 4 * self.B


WORKLOADS = {
    "smoke_L16": Workload("smoke_L16", 1, 16, 16, 8, 8, (8, 12, 16), 3, 0.1),
    "L32_R32_B12_K16": Workload("L32_R32_B12_K16", 4096, 32, 32, 12, 16, (12, 16, 24, 32), 3, (0.05, 0.2)),
    "uneven_L24to48": Workload("uneven_L24to48", 8192, 48, 48, 12, 16, (12, 16, 24, 32, 40, 48), 3, (0.05, 0.2), True),
    "adjoint_L32": Workload("adjoint_L32", 1024, 32, 32, 12, 16, (12, 16, 24, 32), 3, (0.05, 0.2)),
    "L64_R64_B16_K32": Workload("L64_R64_B16_K32", 16384, 64, 64, 16, 32, (16, 24, 32, 48, 64), 2, (0.05, 0.2)),
}
WORKLOAD_INDEX = {k: i for i, k in enumerate(WORKLOADS)}


def make_workload(name: str, n_particles: int | None = None, seed_offset: int = 0, f_dtype=np.complex128,
                  workers: int | None = None) -> Batch:
    wl = WORKLOADS[name]
    n = wl.n_particles if n_particles is None else n_particles
    seed = SEED_BASE + WORKLOAD_INDEX[name] + 1000 * seed_offset
    if wl.uneven:
        rng = np.random.default_rng(seed + 7)
        Lp = rng.integers(24, 49, size=n)
        return make_batch(wl.L, wl.R, n, seed=seed, snr=wl.snr, L_per=Lp, R_per=Lp, f_dtype=f_dtype,
                          workers=workers)
    return make_batch(wl.L, wl.R, n, seed=seed, snr=wl.snr, f_dtype=f_dtype, workers=workers)
