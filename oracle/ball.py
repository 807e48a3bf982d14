"""FP64 ball-harmonic (Fourier-Bessel) transform of volumes on a Cartesian grid (test
infrastructure only; the HIP library never imports this module).

App. A.1: on the unit ball B3, psi_{k,l,m}(x) = c_lk j_l(lam_lk |x|) Y_lm(x/|x|), with lam_lk the
k-th positive zero of the spherical Bessel function j_l (Dirichlet Laplacian eigenfunctions),
orthonormal on L2(B3): c_lk = sqrt(2) / |j_{l+1}(lam_lk)|, since the integral of j_l(lam r)^2 r^2
over [0, 1] is j_{l+1}(lam)^2 / 2 when j_l(lam) = 0.  The expansion keeps the index set
I_Lam = {(k, l, m): lam_lk <= Lam}, i.e. radial sets K_l = {k: lam_lk <= Lam} whose size falls
with l.

A volume given on an N^3 grid is read as samples at the voxel centres x_v = -1 + (2/N)(v + 1/2)
per axis (the grid spans [-1, 1]^3, the ball is inscribed), and its coefficients are the
voxel-sum inner product
    u_klm = (2/N)^3 sum_{v: |x_v| < 1} u(x_v) conj(psi_klm(x_v)).
Layout of the result: [K_max][(L+1)^2] complex, k-major ("shell" k, packed lm = l*l + l + m),
zero where k >= |K_l|: the same layout as the per-shell coefficients of the alignment path, with
unit weights.  Library primitives used as steps: scipy's spherical Bessel function and spherical
harmonics (Condon-Shortley phase), and a bracketing root finder.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq
from scipy.special import sph_harm_y, spherical_jn


def sph_jn_zeros(l: int, lam_max: float) -> np.ndarray:
    """Positive zeros of j_l that are <= lam_max, ascending (scan for sign changes, then bisection
    refined by Brent's method).  The first zero of j_l lies above l, so the scan starts there."""
    if lam_max <= l:
        return np.zeros(0)
    xs = np.arange(max(l, 1e-3), lam_max + 0.5, 0.05)
    v = spherical_jn(l, xs)
    out = []
    for i in range(len(xs) - 1):
        if v[i] == 0.0:
            out.append(xs[i])
        elif v[i] * v[i + 1] < 0.0:
            out.append(brentq(lambda x: spherical_jn(l, x), xs[i], xs[i + 1], xtol=1e-15, rtol=1e-15, maxiter=200))
    z = np.array([x for x in out if x <= lam_max])
    return z


def ball_index(lam: float):
    """(L_max, zeros): zeros[l] = the kept lam_lk of degree l (|K_l| of them), for l <= L_max, the
    largest degree with a zero <= lam."""
    zeros = []
    l = 0
    while True:
        z = sph_jn_zeros(l, lam)
        if z.size == 0:
            break
        zeros.append(z)
        l += 1
    return len(zeros) - 1, zeros


def psi(l: int, m: int, lam_lk: float, x: np.ndarray) -> np.ndarray:
    """psi_{k,l,m} at points x [..., 3] (|x| <= 1)."""
    r = np.linalg.norm(x, axis=-1)
    theta = np.arccos(np.clip(np.where(r > 0, x[..., 2] / np.where(r > 0, r, 1.0), 1.0), -1.0, 1.0))
    phi = np.arctan2(x[..., 1], x[..., 0])
    c = np.sqrt(2.0) / abs(spherical_jn(l + 1, lam_lk))
    return c * spherical_jn(l, lam_lk * r) * sph_harm_y(l, m, theta, phi)


def voxel_centres(N: int):
    """Voxel centres of an N^3 grid spanning [-1, 1]^3 ([N, N, N, 3], index order (z, y, x)
    slowest to fastest... as (i, j, k) -> (x_k, y_j, z_i)), and the mask of those inside the ball."""
    t = -1.0 + (2.0 / N) * (np.arange(N) + 0.5)
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    pts = np.stack([x, y, z], axis=-1)
    return pts, np.linalg.norm(pts, axis=-1) < 1.0


def ball_transform(u: np.ndarray, lam: float) -> np.ndarray:
    """The voxel-sum ball-harmonic coefficients of a real volume u [N, N, N] (index (z, y, x)),
    in the [K_max][(L+1)^2] layout of the module docstring."""
    N = u.shape[0]
    L, zeros = ball_index(lam)
    K = zeros[0].size
    pts, inside = voxel_centres(N)
    xv = pts[inside]
    uv = u[inside].astype(np.float64)
    out = np.zeros((K, (L + 1) ** 2), dtype=np.complex128)
    dv = (2.0 / N) ** 3
    for l in range(L + 1):
        for k, lk in enumerate(zeros[l]):
            for m in range(-l, l + 1):
                out[k, l * l + l + m] = dv * np.sum(uv * np.conj(psi(l, m, lk, xv)))
    return out


def ball_coefficient(u: np.ndarray, lam: float, k: int, l: int, m: int) -> complex:
    """One coefficient u_klm of the voxel sum (zero when k >= |K_l|), for sampling large volumes."""
    N = u.shape[0]
    L, zeros = ball_index(lam)
    if l > L or k >= zeros[l].size:
        return 0j
    pts, inside = voxel_centres(N)
    return complex((2.0 / N) ** 3 * np.sum(u[inside].astype(np.float64) * np.conj(psi(l, m, zeros[l][k], pts[inside]))))


def ball_synthesize(coef: np.ndarray, lam: float, pts: np.ndarray) -> np.ndarray:
    """u(x) = sum over I_Lam of coef psi at the points pts [..., 3] (real part: coef is assumed
    Hermitian-symmetric, coef_{k,l,-m} = (-1)^m conj(coef_klm))."""
    L, zeros = ball_index(lam)
    u = np.zeros(pts.shape[:-1], dtype=np.complex128)
    for l in range(L + 1):
        for k, lk in enumerate(zeros[l]):
            for m in range(-l, l + 1):
                u += coef[k, l * l + l + m] * psi(l, m, lk, pts)
    return u.real
