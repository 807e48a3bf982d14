"""Pins for the FP64 ball-harmonic transform of the oracle (oracle/ball.py, App. A.1), each against
something other than itself: closed forms of the spherical Bessel zeros, orthonormality by
product quadrature, exact recovery of synthesised coefficients under that quadrature, exact
covariance of the voxel sum under the rotations that map the grid onto itself (checked with the
generator's J_y-exponential Wigner matrices), and convergence of the voxel sum to the exact
coefficients as the grid is refined."""
import math

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

from oracle import ball as B
from paper_2603_15285_amd import synth as S


def test_bessel_zeros_closed_forms():
    z0 = B.sph_jn_zeros(0, 30.0)
    assert np.allclose(z0, np.pi * np.arange(1, z0.size + 1), rtol=0, atol=1e-12)  # j_0 = sin x / x
    assert z0.size == int(30.0 // np.pi)
    z1 = B.sph_jn_zeros(1, 30.0)
    assert np.all(np.abs(np.tan(z1) - z1) < 1e-9 * z1 ** 2)  # j_1 = 0  <=>  tan x = x
    # interlacing lam_{l,k} < lam_{l+1,k} < lam_{l,k+1}
    for l in range(6):
        a, b = B.sph_jn_zeros(l, 40.0), B.sph_jn_zeros(l + 1, 40.0)
        for k in range(b.size):
            assert a[k] < b[k] and (k + 1 >= a.size or b[k] < a[k + 1])


def product_quadrature(n_r=48, n_t=None, L=8):
    """Nodes and weights exact (to rounding) for band-L angular products; Gauss-Legendre in r with
    the r^2 weight for the analytic radial factors."""
    n_t = n_t or L + 2
    xr, wr = leggauss(n_r)
    r = 0.5 * (xr + 1.0)
    wr = 0.5 * wr * r ** 2
    ct, wt = leggauss(n_t)
    n_p = 2 * L + 3
    ph = 2 * np.pi * np.arange(n_p) / n_p
    R, CT, PH = np.meshgrid(r, ct, ph, indexing="ij")
    st = np.sqrt(1 - CT ** 2)
    pts = np.stack([R * st * np.cos(PH), R * st * np.sin(PH), R * CT], -1)
    w = (wr[:, None, None] * wt[None, :, None] * np.full(n_p, 2 * np.pi / n_p)[None, None, :])
    return pts, w


def test_basis_is_orthonormal():
    lam = 12.0
    L, zeros = B.ball_index(lam)
    pts, w = product_quadrature(L=L)
    funcs = [(l, m, lk) for l in range(L + 1) for lk in zeros[l] for m in range(-l, l + 1)]
    vals = np.array([B.psi(l, m, lk, pts).ravel() for l, m, lk in funcs])
    G = (vals * w.ravel()) @ vals.conj().T
    assert np.abs(G - np.eye(len(funcs))).max() < 1e-11


def random_coef(lam, seed):
    L, zeros = B.ball_index(lam)
    rng = np.random.default_rng(seed)
    K = zeros[0].size
    c = np.zeros((K, (L + 1) ** 2), dtype=np.complex128)
    for l in range(L + 1):
        g = S.hermitian_gaussian(rng, len(zeros[l]), l, np.full(l + 1, 1.0 / (1 + l) ** 2))
        c[: len(zeros[l]), l * l:(l + 1) ** 2] = g[:, l * l:(l + 1) ** 2]
    return c


def test_exact_quadrature_recovers_coefficients():
    lam = 10.0
    L, zeros = B.ball_index(lam)
    c = random_coef(lam, 3)
    pts, w = product_quadrature(L=L)
    u = B.ball_synthesize(c, lam, pts)
    got = np.zeros_like(c)
    for l in range(L + 1):
        for k, lk in enumerate(zeros[l]):
            for m in range(-l, l + 1):
                got[k, l * l + l + m] = np.sum(w * u * np.conj(B.psi(l, m, lk, pts)))
    assert np.abs(got - c).max() < 1e-11 * np.abs(c).max()


def grid_rotation(u, g):
    """u'(x) = u(g^{-1} x) on the voxel grid, for a rotation g that maps voxel centres onto voxel
    centres (a permutation of the samples, no interpolation)."""
    N = u.shape[0]
    pts, _ = B.voxel_centres(N)
    src = pts @ g  # rows: g^{-1} x = g^T x
    idx = np.rint((src + 1.0) * N / 2.0 - 0.5).astype(int)
    assert np.allclose(-1.0 + (2.0 / N) * (idx + 0.5), src, atol=1e-12)
    return u[idx[..., 2], idx[..., 1], idx[..., 0]]


@pytest.mark.parametrize("euler", [(np.pi / 2, 0.0, 0.0), (0.0, np.pi / 2, 0.0), (np.pi / 2, np.pi / 2, np.pi),
                                   (np.pi, np.pi / 2, np.pi / 2)])
def test_voxel_sum_is_exactly_covariant_under_grid_rotations(euler):
    """Rotations of the cube group permute the voxel centres inside the ball, so the voxel sum
    obeys T(u o g^{-1})_l = D^l(g) T(u)_l exactly (up to rounding), for any volume."""
    N, lam = 12, 9.0
    rng = np.random.default_rng(1)
    u = rng.standard_normal((N, N, N))
    g = S.euler_zyz_to_matrix(*euler)
    assert np.allclose(np.abs(g), np.rint(np.abs(g)))
    a = B.ball_transform(u, lam)
    b = B.ball_transform(grid_rotation(u, g), lam)
    L = int(math.isqrt(a.shape[1])) - 1
    rot = S.rotate_coeffs(a, L, np.array([euler]))[0]
    assert np.abs(rot - b).max() < 1e-12 * np.abs(a).max()
    # real volume: Hermitian symmetry of the coefficients
    for l in range(L + 1):
        for m in range(1, l + 1):
            assert np.allclose(a[:, l * l + l - m], (-1) ** m * np.conj(a[:, l * l + l + m]), atol=1e-14)


def test_voxel_sum_converges_to_the_coefficients():
    """For a smooth volume synthesised from known coefficients (the Dirichlet basis vanishes at
    the sphere), the voxel sum approaches the coefficients as the grid is refined."""
    lam = 8.0
    c = random_coef(lam, 5)
    errs = []
    for N in (16, 32, 64):
        pts, inside = B.voxel_centres(N)
        u = np.zeros((N, N, N))
        u[inside] = B.ball_synthesize(c, lam, pts[inside])
        errs.append(np.abs(B.ball_transform(u, lam) - c).max() / np.abs(c).max())
    # measured: 1.6e-4, 9.2e-6, 3.4e-7 (faster than N^-4: the integrand is smooth and vanishes at the
    # sphere, so the midpoint sums converge quickly)
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-6, errs
    assert errs[1] / errs[2] > 8, errs


def test_single_coefficient_agrees_with_the_full_transform():
    N, lam = 10, 11.0
    u = np.random.default_rng(4).standard_normal((N, N, N))
    a = B.ball_transform(u, lam)
    L, zeros = B.ball_index(lam)
    for k, l, m in [(0, 0, 0), (1, 3, -2), (0, L, L), (len(zeros[2]) - 1, 2, 1), (len(zeros[L]), L, 0)]:
        assert abs(B.ball_coefficient(u, lam, k, l, m) - a[k, l * l + l + m]) <= 1e-15 * np.abs(a).max()
