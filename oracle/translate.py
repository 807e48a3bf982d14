"""FP64 translation search of the rotation-translation alternation (App. C); test infrastructure only
(the HIP library never imports this module).

Conventions (shared by definition, not by code, with the kernels): volumes [N][N][N] indexed (z, y, x)
with voxel centres -1 + (2/N)(i + 1/2); shifts in voxels along (x, y, z); the pose is f = S_s (g o h)
with (S_s u)(x) = u(x - s) and (g o h)(x) = h(R^T x), R = Rz(a) Ry(b) Rz(c).
- The rotated template is the trilinear interpolation of h at R^T x (zero outside the grid).
- The correlation c(s) = sum_x f(x) u(x - s) is cyclic; on integer shifts it is the inverse DFT of
  F conj(U) (numpy's FFT as a library step).  At a real shift it is the trigonometric interpolant
  c(s) = (1/N^3) Re sum over kx = 0..N/2, all ky, kz of w_kx F conj(U)(k) e^{2 pi i k.s / N}, with
  w = 1 at kx = 0 and N/2 and 2 otherwise, and signed frequencies k <= N/2 (the Nyquist index +N/2).
- The search: the best integer shift with |s_i| <= window (ties: the smaller linear index), then the
  best point of the grid s0 + (j - (m-1)/2) / kappa, j = 0..m-1 per axis, m = 2 ceil(3 kappa / 4) + 1
  (ties: the smaller offset index, x fastest).
- A shifted volume f(x + s) is the inverse DFT of F e^{2 pi i k.s / N} with the Nyquist planes zeroed.
Readings where the paper is silent (it cites the upsampled correlation of Guizar-Sicairos et al.):
the window, the +-0.75 voxel refinement range, trilinear resampling, cyclic boundaries.
"""
from __future__ import annotations

import math

import numpy as np


def euler_matrix(a: float, b: float, c: float) -> np.ndarray:
    def rz(t):
        return np.array([[math.cos(t), -math.sin(t), 0.0], [math.sin(t), math.cos(t), 0.0], [0.0, 0.0, 1.0]])

    ry = np.array([[math.cos(b), 0.0, math.sin(b)], [0.0, 1.0, 0.0], [-math.sin(b), 0.0, math.cos(b)]])
    return rz(a) @ ry @ rz(c)


def rotate_volume(h: np.ndarray, euler) -> np.ndarray:
    """u(x) = h(R^T x) by trilinear interpolation on the voxel grid."""
    N = h.shape[0]
    R = euler_matrix(*euler[:3])
    t = -1.0 + (2.0 / N) * (np.arange(N) + 0.5)
    z, y, x = np.meshgrid(t, t, t, indexing="ij")
    pts = np.stack([x, y, z], -1) @ R  # rows: R^T x
    f = (pts + 1.0) * (N / 2.0) - 0.5
    i0 = np.floor(f).astype(np.int64)
    fr = f - i0
    out = np.zeros((N, N, N))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                ix, iy, iz = i0[..., 0] + dx, i0[..., 1] + dy, i0[..., 2] + dz
                ok = (ix >= 0) & (iy >= 0) & (iz >= 0) & (ix < N) & (iy < N) & (iz < N)
                wgt = ((fr[..., 0] if dx else 1 - fr[..., 0]) * (fr[..., 1] if dy else 1 - fr[..., 1]) *
                       (fr[..., 2] if dz else 1 - fr[..., 2]))
                val = np.zeros((N, N, N))
                val[ok] = h[iz[ok], iy[ok], ix[ok]]
                out += wgt * val
    return out


def correlation(f: np.ndarray, u: np.ndarray) -> np.ndarray:
    """c[sz, sy, sx] = sum_x f(x) u(x - s), cyclic, on the integer shifts (index i = s mod N)."""
    return np.fft.irfftn(np.fft.rfftn(f) * np.conj(np.fft.rfftn(u)), s=f.shape, axes=(0, 1, 2))


def _signed(k, N):
    return np.where(k <= N // 2, k, k - N)


def correlation_at(f: np.ndarray, u: np.ndarray, s) -> float:
    """The trigonometric interpolant of the correlation at a real shift s = (sx, sy, sz)."""
    N = f.shape[0]
    X = np.fft.rfftn(f) * np.conj(np.fft.rfftn(u))  # [kz][ky][kx], kx = 0..N/2
    kx = np.arange(N // 2 + 1)
    k = _signed(np.arange(N), N)
    w = np.where((kx == 0) | (2 * kx == N), 1.0, 2.0)
    ph = (np.exp(2j * np.pi * k * s[2] / N)[:, None, None] * np.exp(2j * np.pi * k * s[1] / N)[None, :, None] *
          (w * np.exp(2j * np.pi * kx * s[0] / N))[None, None, :])
    return float(np.real(np.sum(X * ph))) / N ** 3


def refine_points(kappa: int) -> int:
    return 2 * math.ceil(3 * kappa / 4) + 1


def search(f: np.ndarray, h: np.ndarray, euler, window: int, kappa: int):
    """((sx, sy, sz), c(s)) for one particle, as described in the module note."""
    N = f.shape[0]
    u = rotate_volume(h, euler)
    c = correlation(f, u)
    k = _signed(np.arange(N), N)
    ok = (np.abs(k)[:, None, None] <= window) & (np.abs(k)[None, :, None] <= window) & (np.abs(k)[None, None, :] <= window)
    flat = np.where(ok, c, -np.inf).ravel()
    v = int(np.flatnonzero(flat == flat.max())[0])
    iz, iy, ix = v // (N * N), (v // N) % N, v % N
    s0 = np.array([k[ix], k[iy], k[iz]], dtype=np.float64)
    m = refine_points(kappa)
    d = (np.arange(m) - 0.5 * (m - 1)) / kappa
    X = np.fft.rfftn(f) * np.conj(np.fft.rfftn(u))
    kx = np.arange(N // 2 + 1)
    w = np.where((kx == 0) | (2 * kx == N), 1.0, 2.0)
    Ex = w[:, None] * np.exp(2j * np.pi * kx[:, None] * (s0[0] + d)[None, :] / N)   # [kx][a]
    Ey = np.exp(2j * np.pi * k[:, None] * (s0[1] + d)[None, :] / N)                  # [ky][b]
    Ez = np.exp(2j * np.pi * k[:, None] * (s0[2] + d)[None, :] / N)                  # [kz][c]
    vals = np.real(np.einsum("zyx,xa,yb,zc->cba", X, Ex, Ey, Ez)) / N ** 3           # [c][b][a]
    flatv = vals.ravel()
    i = int(np.flatnonzero(flatv == flatv.max())[0])
    jc, jb, ja = i // (m * m), (i // m) % m, i % m
    return s0 + np.array([d[ja], d[jb], d[jc]]), float(flatv[i])


def shift_volume(f: np.ndarray, s) -> np.ndarray:
    """f(x + s) by the phase ramp, Nyquist planes zeroed."""
    N = f.shape[0]
    F = np.fft.rfftn(f)
    kx = np.arange(N // 2 + 1)
    k = _signed(np.arange(N), N)
    ph = (np.exp(2j * np.pi * k * s[2] / N)[:, None, None] * np.exp(2j * np.pi * k * s[1] / N)[None, :, None] *
          np.exp(2j * np.pi * kx * s[0] / N)[None, None, :])
    F = F * ph
    F[N // 2, :, :] = 0
    F[:, N // 2, :] = 0
    F[:, :, N // 2] = 0
    return np.fft.irfftn(F, s=f.shape, axes=(0, 1, 2))
