"""Pins for the FP64 translation oracle (oracle/translate.py, App. C), each against something other
than itself: a brute-force cyclic correlation, np.roll for integer shifts, exact recovery of known
sub-voxel shifts of band-limited volumes, exact cube rotations against the ball-harmonic rotation
route, and the Euler matrix against the generator's."""
import math

import numpy as np

from oracle import ball as OB
from oracle import translate as OT
from paper_2603_15285_amd import synth as S


def bandlimited(N, seed, kmax=None):
    """A real volume whose spectrum is zero at |k_i| > kmax on every axis (Nyquist planes included)."""
    rng = np.random.default_rng(seed)
    kmax = N // 4 if kmax is None else kmax
    F = np.fft.rfftn(rng.standard_normal((N, N, N)))
    k = np.where(np.arange(N) <= N // 2, np.arange(N), np.arange(N) - N)
    kx = np.arange(N // 2 + 1)
    keep = (np.abs(k)[:, None, None] <= kmax) & (np.abs(k)[None, :, None] <= kmax) & (kx[None, None, :] <= kmax)
    return np.fft.irfftn(F * keep, s=(N, N, N), axes=(0, 1, 2))


def test_correlation_against_brute_force():
    rng = np.random.default_rng(0)
    N = 6
    f, u = rng.standard_normal((N, N, N)), rng.standard_normal((N, N, N))
    c = OT.correlation(f, u)
    for sz in range(N):
        for sy in range(N):
            for sx in range(N):
                ref = np.sum(f * np.roll(u, (sz, sy, sx), axis=(0, 1, 2)))  # u(x - s)
                assert abs(c[sz, sy, sx] - ref) < 1e-11 * np.abs(f).sum()


def test_interpolant_at_integer_shifts_is_the_correlation():
    rng = np.random.default_rng(1)
    N = 8
    f, u = rng.standard_normal((N, N, N)), rng.standard_normal((N, N, N))
    c = OT.correlation(f, u)
    for s in [(0, 0, 0), (1, -2, 3), (-3, 3, -1), (2, 2, 2)]:
        assert abs(OT.correlation_at(f, u, s) - c[s[2] % N, s[1] % N, s[0] % N]) < 1e-10 * np.abs(c).max()


def test_shift_volume_integer_is_roll_and_subvoxel_is_recovered():
    N = 16
    f = bandlimited(N, 2)
    g = OT.shift_volume(f, (2.0, -1.0, 3.0))  # f(x + s)
    assert np.abs(g - np.roll(f, (-3, 1, -2), axis=(0, 1, 2))).max() < 1e-12 * np.abs(f).max()
    s_true = np.array([1.3, -0.6, 2.45])
    part = OT.shift_volume(f, -s_true)  # f(x - s): f shifted by +s
    s, val = OT.search(part, f, (0.0, 0.0, 0.0), window=4, kappa=20)
    assert np.abs(s - s_true).max() <= 0.5 / 20 + 1e-9, s
    assert val > 0.99 * np.sum(f * f)


def test_cube_rotation_matches_the_ball_harmonic_rotation_route():
    """rotate_volume by a cube rotation is an exact permutation of the voxels; its ball-harmonic
    coefficients are D(g) times the original's (the convention the path's rotations use)."""
    N, lam = 12, 9.0
    h = np.random.default_rng(3).standard_normal((N, N, N))
    for euler in ((np.pi / 2, 0.0, 0.0), (0.0, np.pi / 2, 0.0)):
        u = OT.rotate_volume(h, euler)
        a, b = OB.ball_transform(h, lam), OB.ball_transform(u, lam)
        L = int(math.isqrt(a.shape[1])) - 1
        rot = S.rotate_coeffs(a, L, np.array([euler]))[0]
        assert np.abs(rot - b).max() < 1e-12 * np.abs(a).max()
    rng = np.random.default_rng(4)
    for _ in range(5):
        e = rng.uniform(0, 2 * np.pi, 3)
        assert np.allclose(OT.euler_matrix(*e), S.euler_zyz_to_matrix(*e), atol=1e-14)
    assert np.abs(OT.rotate_volume(h, (0.0, 0.0, 0.0)) - h).max() < 1e-13 * np.abs(h).max()
