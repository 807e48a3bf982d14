"""Ball-harmonic front end (matcha_ball_transform, App. A.1) against the FP64 oracle (oracle/ball.py).

Tolerance.  The kernels form each coefficient as an FP32 sum over the octant voxels of products of
an FP32 table entry and a sign-symmetrised volume value (a sum of 8 FP32 samples); with
S = (2/N)^3 sum_v |u psi| the absolute sum of the full-grid terms, the error stays below about
(4 + sqrt(V)) * 4 u32 * S (a few roundings per product, the sum's rounding a random walk over the
terms), u32 = 2^-24, V the voxel count.  A wrong sign, index or
normalisation moves an entry by its own size, about S / sqrt(V) for a random volume, far above.
Structural zeros (k >= |K_l|) must be exactly zero.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ball as B  # noqa: E402
from paper_2603_15285_amd import synth as S  # noqa: E402

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_15285_amd import matcha
    matcha.lib()
    return matcha


@pytest.fixture(scope="module")
def ctx(M):
    c = M.Context(0)
    yield c
    c.close()


def abs_scale(u, lam):
    """S_klm = (2/N)^3 sum_v |u(x_v) psi_klm(x_v)| in the output layout (the oracle's basis)."""
    N = u.shape[0]
    L, zeros = B.ball_index(lam)
    pts, inside = B.voxel_centres(N)
    au = np.abs(u[inside].astype(np.float64))
    out = np.zeros((zeros[0].size, (L + 1) ** 2))
    for l in range(L + 1):
        for k, lk in enumerate(zeros[l]):
            for m in range(-l, l + 1):
                out[k, l * l + l + m] = (2.0 / N) ** 3 * np.sum(au * np.abs(B.psi(l, m, lk, pts[inside])))
    return out


def structural_zero_mask(lam):
    L, zeros = B.ball_index(lam)
    z = np.ones((zeros[0].size, (L + 1) ** 2), dtype=bool)
    for l in range(L + 1):
        z[: zeros[l].size, l * l: (l + 1) ** 2] = False
    return z


def grid_rotation(u, g):
    """u(g^-1 x) on the voxel grid for a cube rotation g (a permutation of the voxels); u [..., N, N, N]."""
    N = u.shape[-1]
    pts, _ = B.voxel_centres(N)
    idx = np.rint((pts @ g + 1.0) * N / 2.0 - 0.5).astype(int)
    return u[..., idx[..., 2], idx[..., 1], idx[..., 0]]


def check_against_oracle(got, u, lam):
    N = u.shape[0]
    V = int(B.voxel_centres(N)[1].sum())
    ref = B.ball_transform(u.astype(np.float64), lam)
    sc = abs_scale(u, lam)
    zero = structural_zero_mask(lam)
    assert got.shape == ref.shape
    assert np.all(got[zero] == 0)
    err = np.abs(got.astype(np.complex128) - ref)
    tol = (4 + math.sqrt(V)) * 4 * U32 * sc
    bad = err > tol
    assert not bad.any(), (err[bad].max(), tol[bad].min(), np.argwhere(bad)[:5])
    return err, ref


# ---------------------------------------------------------------- element by element
@pytest.mark.parametrize("N,lam,P", [
    (12, 9.0, 3),     # even grid, two radial indices at l = 0
    (13, 14.0, 37),   # odd grid: voxels on the mirror planes and one at r = 0
    (20, 14.0, 130),  # three 64-volume row tiles, the last ragged; ragged column tiles in every class
    (31, 20.0, 2),    # odd, several K splits over the octant voxels, partial last chunk
    (12, 9.0, 300),   # 128-volume row tiles (from 256 volumes on), the last one ragged
    (14, 9.0, 600),   # from 512 volumes on the partial sums are reduced per volume through LDS
])
def test_ball_transform_matches_oracle(M, ctx, N, lam, P):
    rng = np.random.default_rng(1000 + N)
    u = rng.standard_normal((P, N, N, N)).astype(np.float32)
    print(f"ball N={N} lam={lam} P={P}", flush=True)
    got = M.ball_transform(ctx, torch.from_numpy(u).cuda(), lam).cpu().numpy()
    # every volume of small batches; the first, last and tile-edge volumes of the large one
    sample = range(P) if P <= 40 else sorted({0, 1, 63, 64, 127, 128, 255, 256, 511, 512, P - 2, P - 1} & set(range(P)))
    for p in sample:
        check_against_oracle(got[p], u[p], lam)


def test_ball_transform_widest_degree(M, ctx):
    """Lambda = 70.5: L = 62, 603 radial indices, 23517 columns (about 3000 per sign class, many
    128-column tiles), on a small grid."""
    N, lam = 8, 70.5
    u = np.random.default_rng(7).standard_normal((N, N, N)).astype(np.float32)
    L, zeros = M.ball_index(lam)
    assert L == 62
    got = M.ball_transform(ctx, torch.from_numpy(u).cuda(), lam).cpu().numpy()
    check_against_oracle(got, u, lam)


def test_single_volume_and_out_buffer(M, ctx):
    N, lam = 12, 9.0
    u = np.random.default_rng(5).standard_normal((N, N, N)).astype(np.float32)
    ut = torch.from_numpy(u).cuda()
    a = M.ball_transform(ctx, ut, lam)
    out = torch.full((1,) + tuple(a.shape), float("nan"), dtype=torch.complex64, device="cuda")
    b = M.ball_transform(ctx, ut.unsqueeze(0), lam, out=out)
    assert torch.equal(a, b[0])  # every entry written, structural zeros included


# ---------------------------------------------------------------- full size
def test_full_size_covariance_and_samples(M, ctx):
    """N = 64, Lambda = 38 (L = 31, 170 radial indices), eight volumes in one launch.  Rotations of
    the cube group permute the voxels inside the ball, so T(u o g^-1)_l = D^l(g) T(u)_l holds for
    the voxel sum at any size; and sampled entries are recomputed one by one by the oracle."""
    N, lam, P = 64, 38.0, 8
    rng = np.random.default_rng(64)
    u = rng.standard_normal((P, N, N, N)).astype(np.float32)
    ut = torch.from_numpy(u).cuda()
    got = M.ball_transform(ctx, ut, lam).cpu().numpy().astype(np.complex128)
    L, zeros = M.ball_index(lam)
    assert L == 31 and sum(z.size for z in zeros) == 170
    assert np.all(got[:, structural_zero_mask(lam)] == 0)
    # cube rotations about z and about y: D^l diagonal, and D^l mixing every m
    V = int(B.voxel_centres(N)[1].sum())
    for euler in ((np.pi / 2, 0.0, 0.0), (0.0, np.pi / 2, 0.0)):
        ur = np.ascontiguousarray(grid_rotation(u, S.euler_zyz_to_matrix(*euler)))
        got_r = M.ball_transform(ctx, torch.from_numpy(ur).cuda(), lam).cpu().numpy()
        for p in range(P):
            rot = S.rotate_coeffs(got[p], L, np.array([euler]))[0]
            # |entry error| <= (4 + sqrt V) 4 u32 S on each side, and S <= sqrt((2/N)^3 sum u^2) by
            # Cauchy-Schwarz (the voxel-sum norm of psi is 1 to within 1e-2 at this size)
            s_max = 1.01 * math.sqrt((2.0 / N) ** 3 * np.sum(u[p].astype(np.float64)[B.voxel_centres(N)[1]] ** 2))
            assert np.abs(rot - got_r[p]).max() <= 2 * (4 + math.sqrt(V)) * 4 * U32 * s_max, euler
    # sampled entries of volume 3 against the oracle, one at a time
    samples = [(0, 0, 0), (11, 0, 0), (0, 31, 31), (0, 31, -31), (5, 7, -3), (zeros[20].size - 1, 20, 19), (zeros[25].size - 1, 25, 2)]
    pts, inside = B.voxel_centres(N)
    pts_in = pts[inside]
    for k, l, m in samples:
        ref = B.ball_coefficient(u[3], lam, k, l, m)
        sc = (2.0 / N) ** 3 * np.sum(np.abs(u[3][inside].astype(np.float64)) *
                                      np.abs(B.psi(l, m, zeros[l][k], pts_in)))
        err = abs(got[3, k, l * l + l + m] - ref)
        assert err <= (4 + math.sqrt(V)) * 4 * U32 * sc, (k, l, m, err, sc)


# ---------------------------------------------------------------- into the path
def test_volumes_to_rotation(M, ctx):
    """Front end and path together: two band-limited volumes, the second the first rotated, both
    synthesised by the oracle at the voxel centres; their transforms, aligned with unit shell
    weights, give back the rotation (the voxel sum is close to the exact coefficients here)."""
    N, lam = 32, 16.0
    L, zeros = B.ball_index(lam)
    K = zeros[0].size
    rng = np.random.default_rng(21)
    c = np.zeros((K, (L + 1) ** 2), dtype=np.complex128)
    for l in range(L + 1):
        g = S.hermitian_gaussian(rng, zeros[l].size, l, np.full(l + 1, 1.0 / (1 + l)))
        c[: zeros[l].size, l * l:(l + 1) ** 2] = g[:, l * l:(l + 1) ** 2]
    euler = np.array([[1.1, 0.7, -2.0]])
    cf = S.rotate_coeffs(c, L, euler, hermitian=True)[0]
    pts, inside = B.voxel_centres(N)
    vols = np.zeros((2, N, N, N))
    vols[0][inside] = B.ball_synthesize(cf, lam, pts[inside])
    vols[1][inside] = B.ball_synthesize(c, lam, pts[inside])
    coef = M.ball_transform(ctx, torch.from_numpy(vols.astype(np.float32)).cuda(), lam)
    f = coef[0].contiguous().view(torch.float32).reshape(-1)
    h = coef[1].contiguous().view(torch.float32).reshape(-1)
    w = torch.ones(K, dtype=torch.float32, device="cuda")
    batch = M.Batch.make([L], [K], L, K)
    Bs = 6
    best, _, _ = M.align(ctx, batch, f, h, w, Bs, 4 * Bs, 8, (8, L), 4)
    best = best.cpu().numpy().astype(np.float64)
    err = S.geodesic_deg(S.euler_zyz_to_matrix(*best[0, :3]), S.euler_zyz_to_matrix(*euler[0]))
    assert err < 0.01, err


# ---------------------------------------------------------------- edges
def test_ball_edges(M, ctx):
    lib = M.lib()
    import ctypes as ct
    u = torch.zeros((1, 6, 6, 6), dtype=torch.float32, device="cuda")
    out = torch.zeros((1, 1, 4), dtype=torch.complex64, device="cuda")
    ws = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    s = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    U, O, W = (ct.c_void_p(t.data_ptr()) for t in (u, out, ws))
    # not prepared for N = 6
    assert lib.matcha_ball_workspace_size(ctx.handle, 6, 5.0, 1) == 0
    assert lib.matcha_ball_transform(ctx.handle, 6, 5.0, 1, U, O, W, ws.numel(), s) == M.ERR_NOT_PREPARED
    assert lib.matcha_ball_prepare(ctx.handle, 1, 5.0) == M.ERR_INVALID_ARG
    assert lib.matcha_ball_prepare(ctx.handle, 6, 0.0) == M.ERR_INVALID_ARG
    assert lib.matcha_ball_prepare(ctx.handle, 6, 80.0) == M.ERR_INVALID_ARG
    assert lib.matcha_ball_prepare(ctx.handle, 6, 5.0) == M.OK
    assert lib.matcha_ball_prepare(ctx.handle, 6, 5.0) == M.OK  # idempotent
    need = lib.matcha_ball_workspace_size(ctx.handle, 6, 5.0, 1)
    assert 0 < need <= ws.numel()
    # zero volumes: nothing written, null pointers allowed
    out.fill_(7.0)
    assert lib.matcha_ball_transform(ctx.handle, 6, 5.0, 0, None, None, None, 0, s) == M.OK
    assert lib.matcha_ball_transform(ctx.handle, 6, 5.0, -1, None, None, None, 0, s) == M.ERR_INVALID_ARG
    assert lib.matcha_ball_transform(ctx.handle, 6, 5.0, 1, None, O, W, need, s) == M.ERR_INVALID_ARG
    assert lib.matcha_ball_transform(ctx.handle, 6, 5.0, 1, U, O, W, need - 1, s) == M.ERR_WORKSPACE
    assert lib.matcha_ball_transform(ctx.handle, 6, 5.0, 1, U, O, None, need, s) == M.ERR_WORKSPACE
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    # a zero volume has zero coefficients; a constant one has the symmetry of the cube, which leaves
    # no invariant at degrees 1, 2 and 3
    got = M.ball_transform(ctx, u, 5.0)
    assert torch.all(got == 0)
    got = M.ball_transform(ctx, torch.ones((6, 6, 6), dtype=torch.float32, device="cuda"), 9.0).cpu().numpy()
    assert np.abs(got[:, 1:16]).max() <= 1e-5 * np.abs(got[:, 0]).max()


def test_repeat_calls_are_bitwise_reproducible(M, ctx):
    """The split count depends on the volume count and the device only: the same call twice gives
    the same bits, and a volume's coefficients do not depend on the batch it is in beyond rounding."""
    N, lam = 20, 14.0
    u = torch.from_numpy(np.random.default_rng(9).standard_normal((70, N, N, N)).astype(np.float32)).cuda()
    a = M.ball_transform(ctx, u, lam)
    b = M.ball_transform(ctx, u, lam)
    assert torch.equal(a, b)
    c = M.ball_transform(ctx, u[3:4].contiguous(), lam)
    assert torch.allclose(a[3], c[0], rtol=0, atol=1e-5 * float(a[3].abs().max()))
