"""Pins for the FP64 oracle: each test checks it against something other than itself.

Sources of truth: Wigner's explicit finite sum evaluated in 40-digit mpmath, the
Legendre special case, the matrix exponential of J_y (the generator's route),
real-space rotation with exact sphere quadrature, Haar-measure quadrature on
SO(3), finite differences, numpy's FFT, brute-force numpy scans and closed forms.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import eval_legendre, roots_legendre, sph_harm_y

import oracle as O
from paper_2603_15285_amd import synth as S


def D_matrix(L, l, theta):
    """D^l(theta) assembled from the oracle's d table (m rows, n columns)."""
    d = O.wigner_d(L, theta[1], derivs=False)
    dl = d[O.blk(l):O.blk(l + 1)].reshape(2 * l + 1, 2 * l + 1)
    m = np.arange(-l, l + 1)
    return np.exp(-1j * m[:, None] * theta[0]) * dl * np.exp(-1j * m[None, :] * theta[2])


# ------------------------------------------------------------------ Wigner d
def wigner_explicit(l, m, n, beta):
    """Wigner's explicit finite sum for <l m|exp(-i beta J_y)|l n>, in mpmath."""
    mpmath.mp.dps = 40
    c, s = mpmath.cos(mpmath.mpf(beta) / 2), mpmath.sin(mpmath.mpf(beta) / 2)
    f = mpmath.factorial
    pre = mpmath.sqrt(f(l + n) * f(l - n) * f(l + m) * f(l - m))
    tot = mpmath.mpf(0)
    for k in range(0, 2 * l + 1):
        a1, a2, a3 = l + n - k, l - k - m, k - n + m
        if a1 < 0 or a2 < 0 or a3 < 0:
            continue
        tot += (-1) ** (k - n + m) * pre / (f(a1) * f(k) * f(a2) * f(a3)) * c ** (2 * l - 2 * k + n - m) * s ** (2 * k - n + m)
    return float(tot)


@pytest.mark.parametrize("beta", [0.05, 0.9, 2.0, 3.1])
def test_wigner_d_matches_explicit_sum(beta):
    L = 20
    d = O.wigner_d(L, beta, derivs=False)
    rng = np.random.default_rng(5)
    for l in [0, 1, 2, 5, 11, 20]:
        pairs = [(l, l), (-l, l), (0, 0)] + [tuple(rng.integers(-l, l + 1, 2)) for _ in range(12)]
        for m, n in pairs:
            assert abs(d[O.at(l, m, n)] - wigner_explicit(l, int(m), int(n), beta)) < 1e-12


def test_wigner_d00_is_legendre():
    for beta in [0.01, 0.7, 1.9, 3.0]:
        d = O.wigner_d(64, beta, derivs=False)
        for l in range(65):
            assert abs(d[O.at(l, 0, 0)] - eval_legendre(l, math.cos(beta))) < 1e-12


def test_wigner_d_special_angles():
    L = 16
    d0 = O.wigner_d(L, 0.0, derivs=False)
    dpi = O.wigner_d(L, math.pi, derivs=False)
    for l in range(L + 1):
        b0 = d0[O.blk(l):O.blk(l + 1)].reshape(2 * l + 1, 2 * l + 1)
        bp = dpi[O.blk(l):O.blk(l + 1)].reshape(2 * l + 1, 2 * l + 1)
        assert np.abs(b0 - np.eye(2 * l + 1)).max() < 1e-13
        m = np.arange(-l, l + 1)
        ref = np.fliplr(np.diag((-1.0) ** (l + m)))  # (-1)^{l+m} delta_{m,-n}
        assert np.abs(bp - ref).max() < 1e-12


def test_wigner_d_matches_Jy_exponential_and_is_orthogonal():
    for beta in [0.3, 1.4, 2.8]:
        d = O.wigner_d(64, beta, derivs=False)
        for l in [3, 17, 33, 48, 64]:
            blk = d[O.blk(l):O.blk(l + 1)].reshape(2 * l + 1, 2 * l + 1)
            assert np.abs(blk - S.wigner_d_expm(l, np.array([beta]))[0]).max() < 1e-11
            assert np.abs(blk @ blk.T - np.eye(2 * l + 1)).max() < 1e-11


def test_wigner_D_homomorphism():
    rng = np.random.default_rng(11)
    for _ in range(4):
        e1, e2 = S.haar_euler(rng, 2)
        R = S.euler_zyz_to_matrix(*e1) @ S.euler_zyz_to_matrix(*e2)
        e12 = S.matrix_to_euler_zyz(R)
        for l in [1, 4, 9]:
            lhs = D_matrix(9, l, e12)
            rhs = D_matrix(9, l, e1) @ D_matrix(9, l, e2)
            assert np.abs(lhs - rhs).max() < 1e-11


def test_wigner_D_orthogonality_quadrature():
    """App. A.4, eq. wigner-orthogonality: int D^l_mn conj(D^l'_m'n') dg = delta / (2l+1)."""
    L = 4
    nb = L + 2
    x, wx = roots_legendre(nb)
    betas = np.arccos(x)
    na = 2 * L + 2
    alphas = 2 * np.pi * np.arange(na) / na
    # D for all (l, m, n) at all quadrature nodes: index list
    idx = [(l, m, n) for l in range(L + 1) for m in range(-l, l + 1) for n in range(-l, l + 1)]
    vals = np.zeros((len(idx), nb, na, na), dtype=complex)
    for ib, b in enumerate(betas):
        d = O.wigner_d(L, b, derivs=False)
        for t, (l, m, n) in enumerate(idx):
            vals[t, ib] = np.exp(-1j * m * alphas)[:, None] * d[O.at(l, m, n)] * np.exp(-1j * n * alphas)[None, :]
    wq = (wx[:, None, None] / 2.0) / (na * na)  # normalised Haar measure
    G = np.einsum("tbac,sbac->ts", vals * wq, vals.conj())
    ref = np.diag([1.0 / (2 * l + 1) for (l, m, n) in idx])
    assert np.abs(G - ref).max() < 1e-13


def test_wigner_derivatives_finite_difference():
    L = 24
    for beta in [0.4, 1.3, 2.5]:
        d, d1, d2 = O.wigner_d(L, beta)
        h = 1e-5
        dp, dm = O.wigner_d(L, beta + h, derivs=False), O.wigner_d(L, beta - h, derivs=False)
        assert np.abs((dp - dm) / (2 * h) - d1).max() < 1e-7 * L
        _, d1p, _ = O.wigner_d(L, beta + h)
        _, d1m, _ = O.wigner_d(L, beta - h)
        assert np.abs((d1p - d1m) / (2 * h) - d2).max() < 1e-6 * L * L


def test_term_count_closed_form():
    """App. A.5: sum_{l<=L} (2l+1)^2 = (L+1)(2L+1)(2L+3)/3."""
    for L in [0, 1, 8, 12, 16, 32, 48, 64]:
        assert O.n_terms(L) == (L + 1) * (2 * L + 1) * (2 * L + 3) // 3 == sum((2 * l + 1) ** 2 for l in range(L + 1))
    assert [O.n_terms(L) for L in (12, 16, 24, 32, 40, 64)] == [2925, 6545, 20825, 47905, 91881, 366145]


# --------------------------------------------------------- conventions / objective
def sh_matrix(L, theta, phi):
    """Y_lm(theta, phi) for all packed lm at the given points: [npts, (L+1)^2]."""
    cols = []
    for l in range(L + 1):
        for m in range(-l, l + 1):
            cols.append(sph_harm_y(l, m, theta, phi))
    return np.stack(cols, -1)


def sphere_quadrature(L):
    x, wx = roots_legendre(L + 2)
    nphi = 2 * L + 2
    th = np.arccos(x)
    ph = 2 * np.pi * np.arange(nphi) / nphi
    T, P = np.meshgrid(th, ph, indexing="ij")
    W = np.repeat(wx, nphi) * (2 * np.pi / nphi)
    return T.ravel(), P.ravel(), W


def cart(theta, phi):
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], -1)


def sph(xyz):
    return np.arccos(np.clip(xyz[..., 2], -1, 1)), np.arctan2(xyz[..., 1], xyz[..., 0])


def test_objective_is_real_space_correlation():
    """Eq. maxcc_rot: C(g) = <f, g o h> with (g o h)(x) = h(g^-1 x), integrated by
    exact product quadrature on each shell and summed with the shell weights."""
    rng = np.random.default_rng(3)
    for L in [2, 4]:
        R = 3
        var = 1.0 / (1.0 + np.arange(L + 1)) ** 2
        f = S.hermitian_gaussian(rng, R, L, var)
        h = S.hermitian_gaussian(rng, R, L, var)
        w = np.arange(1, R + 1) ** 2.0
        C = O.coeff_assemble(L, R, f, L, h, L, w)
        T, P, Wq = sphere_quadrature(L)
        Y = sh_matrix(L, T, P)
        x = cart(T, P)
        for _ in range(3):
            th = S.haar_euler(rng, 1)[0]
            g = S.euler_zyz_to_matrix(*th)
            Tr, Pr = sph(x @ g)  # rows x_i^T g = (g^T x_i)^T = (g^-1 x_i)^T
            Yr = sh_matrix(L, Tr, Pr)
            tot = 0.0
            for r in range(R):
                fx = Y @ f[r]
                hx = Yr @ h[r]
                assert np.abs(fx.imag).max() < 1e-12 and np.abs(hx.imag).max() < 1e-12
                tot += w[r] * np.sum(Wq * fx.real * hx.real)
            F = O.evaluate(L, C, th)[0]
            assert abs(F - tot) < 1e-12 * max(1.0, abs(tot))


def test_generator_rotation_matches_real_space():
    """The generator's (g o h)_l = D^l(g) h_l against projecting h(g^-1 x) on Y_lm."""
    rng = np.random.default_rng(8)
    L = 5
    h = S.hermitian_gaussian(rng, 2, L, np.ones(L + 1))
    T, P, Wq = sphere_quadrature(L)
    Y = sh_matrix(L, T, P)
    x = cart(T, P)
    th = S.haar_euler(rng, 1)[0]
    g = S.euler_zyz_to_matrix(*th)
    Tr, Pr = sph(x @ g)
    Yr = sh_matrix(L, Tr, Pr)
    rot = S.rotate_coeffs(h, L, th[None])[0]
    for r in range(2):
        proj = (Y.conj() * Wq[:, None]).T @ (Yr @ h[r])
        assert np.abs(proj - rot[r]).max() < 1e-12


def test_gradient_and_hessian_finite_difference():
    rng = np.random.default_rng(21)
    L, R = 10, 6
    var = 1.0 / (1.0 + np.arange(L + 1)) ** 2
    f = S.hermitian_gaussian(rng, R, L, var)
    h = S.hermitian_gaussian(rng, R, L, var)
    C = O.coeff_assemble(L, R, f, L, h, L, np.arange(1, R + 1) ** 2.0)
    for th in [np.array([0.3, 1.1, 4.0]), np.array([5.5, 2.6, 0.2])]:
        e = O.evaluate(L, C, th)
        scale = np.abs(C).sum()
        hs = 1e-5
        grad = np.zeros(3)
        Hfd = np.zeros((3, 3))
        for i in range(3):
            dp, dm = th.copy(), th.copy()
            dp[i] += hs
            dm[i] -= hs
            ep, em = O.evaluate(L, C, dp), O.evaluate(L, C, dm)
            grad[i] = (ep[0] - em[0]) / (2 * hs)
            Hfd[i] = (ep[1:4] - em[1:4]) / (2 * hs)
        H = np.array([[e[4], e[5], e[6]], [e[5], e[7], e[8]], [e[6], e[8], e[9]]])
        assert np.abs(grad - e[1:4]).max() < 1e-8 * scale
        assert np.abs(Hfd - H).max() < 1e-7 * scale


def test_noiseless_maximum_at_truth_every_band():
    """Cauchy-Schwarz: with f = g* o h, C_L peaks at g* with value |h_{<=L}|^2_w."""
    b = S.make_batch(16, 8, 2, seed=4, noiseless=True)
    for p in range(2):
        C = O.coeff_assemble(16, 8, b.f(p), 16, b.h, 16, b.w)
        for L in [4, 8, 12, 16]:
            e = O.evaluate(L, C, b.euler_true[p])
            ref = np.sum(b.w[:, None] * np.abs(b.h[:, : (L + 1) ** 2]) ** 2)
            assert abs(e[0] - ref) < 1e-12 * ref
            assert np.abs(e[1:4]).max() < 1e-10 * ref
            H = np.array([[e[4], e[5], e[6]], [e[5], e[7], e[8]], [e[6], e[8], e[9]]])
            assert np.linalg.eigvalsh(H).max() < 0 or abs(math.sin(b.euler_true[p][1])) < 1e-2


def test_newton_converges_quadratically_noiseless():
    b = S.make_batch(12, 6, 1, seed=9, noiseless=True)
    C = O.coeff_assemble(12, 6, b.f(0), 12, b.h, 12, b.w)
    Rt = b.R_true()[0]
    rng = np.random.default_rng(0)
    ax = rng.standard_normal(3)
    ax /= np.linalg.norm(ax)
    ang = math.radians(3.0)
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    Rp = (np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K) @ Rt
    th = S.matrix_to_euler_zyz(Rp)
    errs = [math.radians(float(S.geodesic_deg(Rt, Rp)))]
    for _ in range(4):
        e = O.evaluate(12, C, th)
        th, st, _ = O.newton_step(e, th)
        errs.append(math.radians(float(S.geodesic_deg(Rt, S.euler_zyz_to_matrix(*th)))))
    for a, c in zip(errs[:-1], errs[1:]):
        if a > 1e-7:
            assert c < 20.0 * a * a  # quadratic contraction
    assert errs[-1] < 1e-12


# --------------------------------------------------------------- Newton step
def test_newton_step_solves_the_3x3_system_and_wraps():
    rng = np.random.default_rng(2)
    for _ in range(20):
        A = rng.standard_normal((3, 3))
        H = -(A @ A.T + 0.5 * np.eye(3))
        g = rng.standard_normal(3) * 0.01
        e = np.array([1.0, g[0], g[1], g[2], H[0, 0], H[0, 1], H[0, 2], H[1, 1], H[1, 2], H[2, 2]])
        th0 = np.array([1.0, 1.5, 2.0])
        th, st, sinf = O.newton_step(e, th0)
        assert st == 0
        ref = th0 - np.linalg.solve(H, g)
        assert np.abs(th - ref).max() < 1e-13
        assert abs(sinf - np.abs(np.linalg.solve(H, g)).max()) < 1e-13
    # indefinite Hessian: still a pure Newton step, flagged
    e = np.array([1.0, 0.1, 0.0, 0.0, 1.0, 0, 0, -1.0, 0, -1.0])
    th, st, _ = O.newton_step(e, [1.0, 1.0, 1.0])
    assert st & O.INDEFINITE and abs(th[0] - 0.9) < 1e-14
    # singular Hessian: no step
    e = np.zeros(10)
    th, st, _ = O.newton_step(e, [1.0, 1.0, 1.0])
    assert st & O.SINGULAR and np.allclose(th, 1.0)
    # non-finite value: no step
    e = np.full(10, np.nan)
    th, st, _ = O.newton_step(e, [1.0, 1.0, 1.0])
    assert st & O.NONFINITE and np.allclose(th, 1.0)
    # a step through the pole b = 0 lands on the same rotation, re-charted
    th0 = np.array([0.5, 0.1, 0.7])
    target = np.array([0.5, -0.3, 0.7])
    H = -np.eye(3)
    g = -(target - th0)  # dth = -H^-1 g = g... choose g so that dth = target - th0
    g = H @ (-(target - th0))
    e = np.array([1.0, g[0], g[1], g[2], -1, 0, 0, -1, 0, -1])
    th, st, _ = O.newton_step(e, th0)
    assert 0 <= th[1] <= math.pi and 0 <= th[0] < 2 * math.pi and 0 <= th[2] < 2 * math.pi
    Ra = S.euler_zyz_to_matrix(*target)
    Rb = S.euler_zyz_to_matrix(*th)
    assert np.abs(Ra - Rb).max() < 1e-14
    # clipping
    e = np.array([1.0, 1.0, 0.0, 0.0, -1.0, 0, 0, -1.0, 0, -1.0])
    th, st, sinf = O.newton_step(e, [1.0, 1.0, 1.0], max_step=0.1)
    assert abs(th[0] - 1.1) < 1e-14 and abs(sinf - 0.1) < 1e-15


# ----------------------------------------------------------- coefficient assembly
def test_assembly_definition_rank_and_rotation_covariance():
    rng = np.random.default_rng(6)
    L, R = 9, 4
    var = np.ones(L + 1)
    f = S.hermitian_gaussian(rng, R, L, var)
    h = S.hermitian_gaussian(rng, R, L, var)
    w = np.arange(1, R + 1) ** 2.0
    C = O.coeff_assemble(L, R, f, L, h, L, w)
    th = S.haar_euler(rng, 1)[0]
    hr = S.rotate_coeffs(h, L, th[None])[0]
    Cr = O.coeff_assemble(L, R, f, L, hr, L, w)
    for l in range(L + 1):
        sl = slice(l * l, (l + 1) ** 2)
        ref = np.einsum("r,rm,rn->mn", w, f[:, sl], h[:, sl].conj())
        blk = C[O.blk(l):O.blk(l + 1)].reshape(2 * l + 1, 2 * l + 1)
        assert np.abs(blk - ref).max() < 1e-12 * np.abs(ref).max()
        sv = np.linalg.svd(blk, compute_uv=False)
        assert np.sum(sv > 1e-10 * sv[0]) <= min(R, 2 * l + 1)  # App. A.6, eq. rank_bound
        D = S.rotate_coeffs(np.eye((L + 1) ** 2, dtype=complex)[sl.start:sl.stop], L, th[None])[0][:, sl].T
        blkr = Cr[O.blk(l):O.blk(l + 1)].reshape(2 * l + 1, 2 * l + 1)
        assert np.abs(blkr - blk @ D.conj().T).max() < 1e-11 * np.abs(blk).max()  # A^(g) = A D(g)^*
        svr = np.linalg.svd(blkr, compute_uv=False)
        assert np.abs(svr - sv).max() < 1e-10 * sv[0]
        # Hermitian-symmetric inputs give C^l_{-m,-n} = (-1)^{m-n} conj(C^l_mn)
        m = np.arange(-l, l + 1)
        sgn = (-1.0) ** (m[:, None] - m[None, :])
        assert np.abs(blk[::-1, ::-1] - sgn * blk.conj()).max() < 1e-12 * np.abs(blk).max()


# ------------------------------------------------------------------ SOFFT grid
def test_soft_grid_matches_wigner_transform_plus_fft():
    """Grid values through an independent route: d from exp(-i beta J_y), the
    Wigner transform S_i[m,n], then numpy's inverse 2-D FFT over (alpha, gamma)."""
    rng = np.random.default_rng(12)
    B, R = 5, 3
    n = 4 * B
    var = 1.0 / (1.0 + np.arange(B + 1)) ** 2
    f = S.hermitian_gaussian(rng, R, B, var)
    h = S.hermitian_gaussian(rng, R, B, var)
    C = O.coeff_assemble(B, R, f, B, h, B, np.ones(R))
    grid = O.soft_grid(B, C, n)
    betas = np.pi * (2 * np.arange(n) + 1) / (2 * n)
    ref = np.zeros((n, n, n))
    for i, b in enumerate(betas):
        X = np.zeros((n, n), dtype=complex)
        for l in range(B + 1):
            dl = S.wigner_d_expm(l, np.array([b]))[0]
            blk = C[O.blk(l):O.blk(l + 1)].reshape(2 * l + 1, 2 * l + 1)
            m = np.arange(-l, l + 1)
            X[np.ix_(m % n, m % n)] += blk * dl
        ref[i] = (np.fft.ifft2(X) * n * n).real
    assert np.abs(grid - ref).max() < 1e-12 * np.abs(ref).max()


def brute_local_max(grid):
    n = grid.shape[0]
    idx = np.arange(n ** 3).reshape(n, n, n)
    is_max = np.ones(grid.shape, bool)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for dk in (-1, 0, 1):
                if di == dj == dk == 0:
                    continue
                u = np.roll(np.roll(grid, -dj, 1), -dk, 2)
                ui = np.roll(np.roll(idx, -dj, 1), -dk, 2)
                if di:
                    u = np.roll(u, -di, 0)
                    ui = np.roll(ui, -di, 0)
                beats = (grid > u) | ((grid == u) & (idx < ui))
                if di == -1:
                    beats[0] = True
                if di == 1:
                    beats[-1] = True
                is_max &= beats
    return is_max


def ranked(grid, mask):
    v = grid.ravel()[mask.ravel()]
    i = np.nonzero(mask.ravel())[0]
    o = np.lexsort((i, -v))
    return i[o], v[o]


@pytest.mark.parametrize("kind", ["random", "ties", "unimodal"])
def test_soft_select_brute_force(kind):
    rng = np.random.default_rng(1)
    n, Kc = 12, 10
    if kind == "random":
        grid = rng.standard_normal((n, n, n))
    elif kind == "ties":
        grid = np.round(rng.standard_normal((n, n, n)) * 2) / 2
    else:
        t = 2 * np.pi * np.arange(n) / n
        b = np.pi * (2 * np.arange(n) + 1) / (2 * n)
        grid = np.cos(b)[:, None, None] + 0.5 * np.cos(t)[None, :, None] + 0.25 * np.cos(t)[None, None, :]
    idx, val, nmx = O.soft_select(grid, Kc)
    mask = brute_local_max(grid)
    mi, mv = ranked(grid, mask)
    ri, rv = ranked(grid, ~mask)
    allidx = np.concatenate([mi, ri])[:Kc]
    assert nmx == mask.sum()
    assert np.array_equal(idx, allidx)
    assert np.array_equal(val, grid.ravel()[allidx])
    if kind == "unimodal":
        assert nmx == 1


# ----------------------------------------------------------------- march / align
def test_schedule_rule():
    assert O.schedule(32, [12, 16, 24, 32]) == [12, 16, 24, 32]
    assert O.schedule(30, [12, 16, 24, 32, 40, 48]) == [12, 16, 24, 30]
    assert O.schedule(24, [12, 16, 24, 32]) == [12, 16, 24]
    assert O.schedule(48, [12, 16, 24, 32, 40, 48]) == [12, 16, 24, 32, 40, 48]


def test_align_recovers_noiseless_rotation():
    b = S.make_batch(16, 8, 3, seed=31, noiseless=True)
    best, bi, st, cand = O.align_batch(b, 8, 32, 8, [8, 12, 16], 3)
    Rb = S.euler_zyz_to_matrix(best[:, 0], best[:, 1], best[:, 2])
    err = S.geodesic_deg(b.R_true(), Rb)
    assert np.all(err < 1e-9), err
    hn = np.sum(b.w[:, None] * np.abs(b.h) ** 2)
    assert np.allclose(best[:, 3], hn, rtol=1e-12)


def test_align_smoke_workload_noisy():
    b = S.make_workload("smoke_L16")
    best, bi, st, cand = O.align_batch(b, 8, 32, 8, [8, 12, 16], 3)
    err = S.geodesic_deg(b.R_true(), S.euler_zyz_to_matrix(best[:, 0], best[:, 1], best[:, 2]))
    assert err[0] < 2.0


def test_tiny_band_march_finds_the_global_maximum():
    """Theorem / Corollary (Sec. 3): when the best basin wins by a clear gap the
    march selects it.  The reference global maximum comes from a dense grid of
    C_L itself, every grid maximum polished by Newton to convergence."""
    L, R = 3, 4
    for seed in range(3):
        b = S.make_batch(L, R, 1, seed=100 + seed, snr=2.0)
        C = O.coeff_assemble(L, R, b.f(0), L, b.h, L, b.w)
        n = 24
        grid = O.soft_grid(L, C, n)
        idx, val, nmx = O.soft_select(grid, min(40, n ** 3))
        tops = []
        for e0 in O.grid_euler(idx[: max(nmx, 1)], n):
            th = e0.copy()
            for _ in range(30):
                th, st, _ = O.newton_step(O.evaluate(L, C, th), th)
            tops.append((O.evaluate_F(L, C, th), th))
        tops.sort(key=lambda t: -t[0])
        G, thG = tops[0]
        best, bi, st, cand = O.align_one(b.f(0), L, R, b.h, L, b.w, 2, 8, 4, [2, 3], 6)
        assert best[3] > G - 1e-9 * abs(G)
        assert S.geodesic_deg(S.euler_zyz_to_matrix(*thG), S.euler_zyz_to_matrix(*best[:3])) < 1e-6


# -------------------------------------------------------------------- adjoint
def test_adjoint_matches_central_differences():
    """F is bilinear in (f, h) at fixed R*, so central differences are exact up to rounding."""
    rng = np.random.default_rng(14)
    L, R, P = 6, 3, 3
    var = 1.0 / (1.0 + np.arange(L + 1)) ** 2
    h = S.hermitian_gaussian(rng, R, L, var)
    fs = [S.hermitian_gaussian(rng, R, L, var) for _ in range(P)]
    w = np.arange(1, R + 1) ** 2.0
    eul = S.haar_euler(rng, P)
    g = rng.standard_normal(P)

    def loss(fs_, h_):
        tot = 0.0
        for p in range(P):
            C = O.coeff_assemble(L, R, fs_[p], L, h_, L, w)
            tot += g[p] * O.evaluate_F(L, C, eul[p])
        return tot

    gh = np.zeros_like(h)
    gfs = []
    for p in range(P):
        gh, gf = O.grad_one(L, R, fs[p], h, L, w, eul[p], g[p], grad_h=gh)
        gfs.append(gf)
    eps = 1e-3
    for _ in range(10):
        r, j = rng.integers(R), rng.integers((L + 1) ** 2)
        for unit, part in ((1.0, "re"), (1j, "im")):
            hp, hm = h.copy(), h.copy()
            hp[r, j] += eps * unit
            hm[r, j] -= eps * unit
            fd = (loss(fs, hp) - loss(fs, hm)) / (2 * eps)
            an = gh[r, j].real if part == "re" else gh[r, j].imag
            assert abs(fd - an) < 1e-9 * max(1.0, abs(an))
            p = rng.integers(P)
            fp = [x.copy() for x in fs]
            fm = [x.copy() for x in fs]
            fp[p][r, j] += eps * unit
            fm[p][r, j] -= eps * unit
            fd = (loss(fp, h) - loss(fm, h)) / (2 * eps)
            an = gfs[p][r, j].real if part == "re" else gfs[p][r, j].imag
            assert abs(fd - an) < 1e-9 * max(1.0, abs(an))


def test_oracle_matches_its_golden_fixture():
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_smallcase.json")))
    b = S.make_batch(6, 4, 2, seed=fx["seed"], snr=0.5)
    for p, ref in enumerate(fx["particles"]):
        C = O.coeff_assemble(6, 4, b.f(p), 6, b.h, 6, b.w)
        c2 = np.array([complex(*z) for z in ref["C_l2"]])
        assert np.abs(C[O.blk(2):O.blk(3)] - c2).max() < 1e-12
        assert np.allclose(O.evaluate(6, C, [0.4, 1.2, 2.2]), ref["eval_at_0.4_1.2_2.2"], rtol=1e-12, atol=1e-12)
        best, bi, st, _ = O.align_one(b.f(p), 6, 4, b.h, 6, b.w, fx["B"], fx["n"], fx["Kc"], fx["levels"], fx["steps"])
        assert bi == ref["best_idx"] and st == ref["status"]
        assert np.allclose(best, ref["best"], rtol=1e-10, atol=1e-12)


# ------------------------------------------------------------- early stopping
def _perturbed(Rt, deg, seed):
    """Euler angles of Rt turned by `deg` degrees about a random axis."""
    rng = np.random.default_rng(seed)
    ax = rng.standard_normal(3)
    ax /= np.linalg.norm(ax)
    ang = math.radians(deg)
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    return S.matrix_to_euler_zyz((np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K) @ Rt)


def _expected_level(Lj, C, th0, steps, tol_grad, tol_step, tol_rel):
    """One level of the march with the Sec. 2.4 stopping rules, taken from the fixed-step
    trajectory: before step t the level stops if |grad F(th_t)| <= tol_grad |F(th_t)| or (t > 0)
    |F(th_t) - F(th_{t-1})| <= tol_rel |F(th_t)|; after step t it stops if the step's largest
    component is <= tol_step.  The trajectory comes from the oracle's Newton step (pinned above)
    and the fixed-step march; the stopping decisions are made here.  Returns (theta, stopped)."""
    th = np.array(th0[:3], dtype=np.float64)
    Fprev = None
    for t in range(steps):
        e = O.evaluate(Lj, C, th)
        gn = float(np.linalg.norm(e[1:4]))
        if gn <= tol_grad * abs(e[0]) or (t > 0 and abs(e[0] - Fprev) <= tol_rel * abs(e[0])):
            return th, True
        Fprev = e[0]
        th, _, sinf = O.newton_step(e, th)
        # the same point as the oracle's own fixed-step march after t + 1 steps
        cf, _, _ = O.march(Lj, C, [], t + 1, np.r_[th0[:3], 0.0][None])
        assert np.array_equal(cf[0, :3], th)
        if sinf <= tol_step:
            return th, True
    return th, False


def _trajectory(Lj, C, th0, steps):
    """(|grad|/|F|, |dF|/|F|, step) along the fixed-step trajectory at band Lj."""
    th = np.array(th0[:3], dtype=np.float64)
    g, r, s = [], [], []
    Fprev = None
    for t in range(steps):
        e = O.evaluate(Lj, C, th)
        g.append(float(np.linalg.norm(e[1:4])) / abs(e[0]))
        r.append(abs(e[0] - Fprev) / abs(e[0]) if t > 0 else np.inf)
        Fprev = e[0]
        th, _, sinf = O.newton_step(e, th)
        s.append(sinf)
    return np.array(g), np.array(r), np.array(s)


@pytest.mark.parametrize("which", ["grad", "rel", "step"])
def test_early_stop_each_criterion_truncates_the_fixed_march(which):
    """Each Sec. 2.4 criterion alone (the other tolerances 0, which never fire on a moving
    candidate) stops a level exactly where the criterion first holds on the fixed-step
    trajectory, with the EARLY_STOP flag; the thresholds sit in the middle of a gap of the
    trajectory's sequence, so the expected stopping step is unambiguous."""
    L, R, steps = 10, 6, 6
    b = S.make_batch(L, R, 1, seed=61, noiseless=True)
    C = O.coeff_assemble(L, R, b.f(0), L, b.h, L, b.w)
    th0 = _perturbed(b.R_true()[0], 4.0, 3)
    g, r, s = _trajectory(L, C, th0, steps)
    seq = {"grad": g, "rel": r, "step": s}[which]
    # threshold between the 2nd and 3rd entries of the sequence (geometric mean), so the level
    # stops at the third check; the sequence must fall by at least 100x there
    k = 2 if which != "rel" else 3
    assert seq[k - 1] > 100 * seq[k], seq
    tol = math.sqrt(seq[k - 1] * seq[k])
    tols = dict(tol_grad=0.0, tol_step=0.0, tol_rel=0.0)
    tols["tol_" + which] = tol
    start = np.r_[th0, 0.0][None]
    got, _, cst = O.march(L, C, [], steps, start, early_stop=True, **tols)
    exp, stopped = _expected_level(L, C, th0, steps, **tols)
    assert stopped
    assert bool(cst[0] & O.EARLY_STOP)
    assert np.array_equal(got[0, :3], exp)
    # with zero tolerances a level can only stop once the candidate no longer moves at all (an
    # exactly zero step or change of F), so the result is the fixed-step one; before convergence
    # (two steps) it is not flagged
    full, _, _ = O.march(L, C, [], steps, start, early_stop=True, tol_grad=0.0, tol_step=0.0, tol_rel=0.0)
    ref, _, _ = O.march(L, C, [], steps, start)
    assert np.array_equal(full[0, :3], ref[0, :3])
    _, _, cst2 = O.march(L, C, [], 2, start, early_stop=True, tol_grad=0.0, tol_step=0.0, tol_rel=0.0)
    assert not cst2[0] & O.EARLY_STOP


def test_early_stop_restarts_at_every_level():
    """Two levels: the second level's stepping starts afresh (no relative-change test at its first
    step) from where the first stopped."""
    L, R, steps = 10, 6, 5
    b = S.make_batch(L, R, 1, seed=62, noiseless=True)
    C = O.coeff_assemble(L, R, b.f(0), L, b.h, L, b.w)
    th0 = _perturbed(b.R_true()[0], 3.0, 4)
    tols = dict(tol_grad=1e-6, tol_step=1e-9, tol_rel=1e-12)
    th_a, s_a = _expected_level(6, C, th0, steps, **tols)
    th_b, s_b = _expected_level(L, C, th_a, steps, **tols)
    got, _, cst = O.march(L, C, [6], steps, np.r_[th0, 0.0][None], early_stop=True, **tols)
    assert s_a or s_b
    assert bool(cst[0] & O.EARLY_STOP) == (s_a or s_b)
    assert np.array_equal(got[0, :3], th_b)


def test_early_stop_noiseless_agrees_with_fixed_steps():
    """With the default FP64 tolerances a noiseless particle stops early, and its rotation is the
    fixed-step result (the true rotation) to 1e-8 degrees: a level stops once |grad F| <= 1e-9 |F|
    or |dF| <= 1e-13 |F|, which leaves at most about 1e-9 degrees to the quadratically converging
    steps it skips (measured: up to 1.2e-9 degrees from a 4-degree start)."""
    wl_levels, steps = [8, 12, 16], 6
    b = S.make_batch(16, 8, 3, seed=63, noiseless=True)
    for p in range(3):
        C = O.coeff_assemble(16, 8, b.f(p), 16, b.h, 16, b.w)
        start = np.array([np.r_[_perturbed(b.R_true()[p], d, 10 + p), 0.0] for d in (1.0, 2.5, 4.0)])
        es, bi_e, cst = O.march(16, C, wl_levels, steps, start, early_stop=True)
        fx, bi_f, _ = O.march(16, C, wl_levels, steps, start)
        assert np.all(cst & O.EARLY_STOP)
        # all three reach the same maximum, so the selection is a near-tie: only its value is unique
        assert abs(es[bi_e, 3] - fx[bi_f, 3]) <= 1e-12 * abs(fx[bi_f, 3])
        err = S.geodesic_deg(S.euler_zyz_to_matrix(es[:, 0], es[:, 1], es[:, 2]),
                             S.euler_zyz_to_matrix(fx[:, 0], fx[:, 1], fx[:, 2]))
        assert np.all(err < 1e-8), err
        assert np.all(S.geodesic_deg(b.R_true()[p], S.euler_zyz_to_matrix(es[:, 0], es[:, 1], es[:, 2])) < 1e-8)


# --------------------------------------------------------------- gradient ascent comparator
def test_gradient_step_is_a_first_order_ascent_step():
    """theta + t grad F with t = rate / ((1+L)^2 |F|): for a small step the objective rises by
    t |grad F|^2 to first order (the gradient itself is pinned by central differences above)."""
    b = S.make_batch(12, 6, 1, seed=31, snr=0.5)
    C = O.coeff_assemble(12, 6, b.f(0), 12, b.h, 12, b.w)
    rng = np.random.default_rng(3)
    for _ in range(5):
        th = np.array([rng.uniform(0, 2 * np.pi), rng.uniform(0.3, 2.8), rng.uniform(0, 2 * np.pi)])
        e = O.evaluate(12, C, th)
        rate = 1e-4
        t = rate / (13.0 ** 2 * abs(e[0]))
        new, st, sinf = O.gradient_step(e, th, rate, 12)
        assert st == 0
        assert np.allclose(new, th + t * np.asarray(e[1:4]), rtol=0, atol=1e-15)
        rise = O.evaluate_F(12, C, new) - e[0]
        g2 = float(np.sum(np.asarray(e[1:4]) ** 2))
        assert abs(rise - t * g2) <= 1e-3 * t * g2
        assert sinf == pytest.approx(t * np.abs(e[1:4]).max(), rel=1e-14)


def test_gradient_ascent_converges_linearly_where_newton_is_quadratic():
    """Noiseless particle, 3 degrees off: gradient ascent (rate 10) raises F at every step and
    closes in linearly (a roughly constant factor per step), while Newton from the same start is at
    the maximum within four steps (Fig. newton_v_gd's contrast)."""
    b = S.make_batch(16, 8, 1, seed=9, noiseless=True)
    C = O.coeff_assemble(16, 8, b.f(0), 16, b.h, 16, b.w)
    Rt = b.R_true()[0]
    th = _perturbed(Rt, 3.0, 1)
    F, errs = [], []
    for _ in range(60):
        e = O.evaluate(16, C, th)
        F.append(e[0])
        th, st, _ = O.gradient_step(e, th, 10.0, 16)
        assert st == 0
        errs.append(float(S.geodesic_deg(Rt, S.euler_zyz_to_matrix(*th))))
    assert all(F[i + 1] >= F[i] - 1e-12 * abs(F[i]) for i in range(len(F) - 1))
    assert errs[-1] < 1e-3
    ratios = [errs[i + 1] / errs[i] for i in range(20, 59)]
    assert 0.5 < min(ratios) and max(ratios) < 0.9  # linear, not quadratic
    # the march with gd_rate takes exactly these steps at one level
    cand = np.array([np.r_[_perturbed(Rt, 3.0, 1), 0.0]])
    out, _, cst = O.march(16, C, [16], 60, cand, gd_rate=10.0)
    assert np.allclose(out[0, :3], th, rtol=0, atol=1e-12)
    assert cst[0] == 0
    thn = _perturbed(Rt, 3.0, 1)
    for _ in range(4):
        thn, _, _ = O.newton_step(O.evaluate(16, C, thn), thn)
    assert S.geodesic_deg(Rt, S.euler_zyz_to_matrix(*thn)) < 1e-9


# --------------------------------------------------------------- low-rank structure (App. A.6, B.1)
def test_effective_rank_definition_on_known_spectra():
    from oracle import lowrank as LR
    assert LR.effective_rank([1.0, 0.5, 0.05, 0.01]) == 2        # 0.05 / 0.5 = 0.1 < 0.2
    assert LR.effective_rank([1.0, 0.1, 0.09]) == 1
    assert LR.effective_rank([1.0, 0.9, 0.8]) == 3               # no gap: all of them
    assert LR.effective_rank([1.0, 0.0, 0.0]) == 1               # exact rank 1
    assert LR.effective_rank([0.0, 0.0]) == 0
    assert LR.effective_rank([2.0, 0.39]) == 1 and LR.effective_rank([2.0, 0.4]) == 2  # strict inequality
    assert LR.effective_rank([1.0, 0.5, 0.05], rho=0.05) == 3


def test_block_singular_values_of_a_constructed_factorisation():
    """f and h built so that C^l = U diag(s) V^H with orthonormal U, V (shell weights w_r = 1):
    f_l(r) = s_r u_r, h_l(r) = v_r for r < R, so the singular values are s exactly."""
    from oracle import lowrank as LR
    rng = np.random.default_rng(17)
    L, R = 6, 4
    f = np.zeros((R, (L + 1) ** 2), dtype=complex)
    h = np.zeros((R, (L + 1) ** 2), dtype=complex)
    want = {}
    for l in range(L + 1):
        n = 2 * l + 1
        k = min(n, R)
        U, _ = np.linalg.qr(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
        V, _ = np.linalg.qr(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
        s = np.sort(rng.uniform(0.1, 2.0, k))[::-1]
        for r in range(k):
            f[r, l * l:(l + 1) ** 2] = s[r] * U[:, r]
            h[r, l * l:(l + 1) ** 2] = V[:, r]
        want[l] = s
    got = LR.block_singular_values(L, R, f, L, h, L, np.ones(R))
    for l in range(L + 1):
        assert np.allclose(got[l], want[l], rtol=0, atol=1e-13)
