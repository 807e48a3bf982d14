"""Singular values and effective ranks of the correlation blocks (matcha_lowrank_spectrum,
App. A.6 and B.1) against the FP64 oracle (oracle/lowrank.py: numpy's SVD of the assembled blocks).

Tolerance.  Both sides start from the same FP32 inputs and compute in FP64.  The kernel passes
through Gram matrices (squared values) and stops each pivoted Cholesky at 1e-13 of the largest
diagonal, so singular values below sqrt(1e-13) s_1 = 3.2e-7 s_1 come out as 0 and larger ones carry
an absolute error of about 1e-16 s_1^2 / s_j: |ds| <= 4e-7 s_1 for every value.  Effective ranks are
compared where the oracle's cut falls at a value >= 1e-4 s_1 and no ratio between values >= 1e-4 s_1
lies within 1e-3 of rho (where the two may legitimately differ)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import ball as OB  # noqa: E402
from oracle import lowrank as LR  # noqa: E402
from paper_2603_15285_amd import synth as S  # noqa: E402


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


def upload(M, b, f_parts):
    flat = np.concatenate([x.reshape(-1) for x in f_parts]).astype(np.complex64)
    batch = M.Batch.make(b["L"], b["R"], b["Lh"], b["Rh"])
    f = torch.from_numpy(flat.view(np.float32).copy()).cuda()
    h = torch.from_numpy(b["h"].astype(np.complex64).view(np.float32).reshape(-1).copy()).cuda()
    w = torch.from_numpy(b["w"].astype(np.float32)).cuda()
    return batch, f, h, w


def check(sv, reff, f_parts, b, rho=0.2):
    h32 = b["h"].astype(np.complex64).astype(np.complex128)
    w32 = b["w"].astype(np.float32).astype(np.float64)
    for p, fp in enumerate(f_parts):
        Lp, Rp = int(b["L"][p]), int(b["R"][p])
        ref = LR.block_singular_values(Lp, Rp, fp.astype(np.complex64).astype(np.complex128), Lp, h32, b["Lh"], w32)
        s1 = max(float(r[0]) for r in ref if r.size)
        for l in range(Lp + 1):
            k = ref[l].size
            assert np.all(np.abs(sv[p, l, :k] - ref[l]) <= 4e-7 * s1), (p, l, sv[p, l, :k], ref[l])
            assert np.all(sv[p, l, k:] == 0)
            r = ref[l]
            cut = LR.effective_rank(r, rho)
            big = r >= 1e-4 * r[0] if r.size and r[0] > 0 else np.zeros(r.size, bool)
            ratios = r[1:] / np.where(r[:-1] > 0, r[:-1], 1.0)
            near = np.any(np.abs(ratios[big[1:]] - rho) < 1e-3 * rho)
            if cut == 0 or (r[cut - 1] >= 1e-4 * r[0] and not near):
                assert reff[p, l] == cut, (p, l, reff[p, l], r)
        assert np.all(sv[p, Lp + 1:] == 0) and np.all(reff[p, Lp + 1:] == 0)


def test_ragged_batch_matches_oracle(M, ctx):
    rng = np.random.default_rng(5)
    Lh, Rh = 24, 16
    L = np.array([8, 16, 24, 24, 12, 20, 1, 0])
    R = np.array([4, 16, 16, 8, 12, 16, 3, 2])
    var = 1.0 / (1.0 + np.arange(Lh + 1)) ** 2
    h = S.hermitian_gaussian(rng, Rh, Lh, var)
    w = (1.0 + np.arange(Rh)) ** 2
    f_parts = [S.hermitian_gaussian(rng, int(r), int(l), var[: l + 1]) for l, r in zip(L, R)]
    # a particle whose f repeats one shell: rank 1 in every degree
    f_parts[3][:] = f_parts[3][0][None, :] * (1.0 + np.arange(8))[:, None]
    b = dict(L=L, R=R, Lh=Lh, Rh=Rh, h=h, w=w)
    batch, f, hh, ww = upload(M, b, f_parts)
    sv, reff = M.lowrank_spectrum(ctx, batch, f, hh, ww, rho=0.2, n_sv=16)
    sv, reff = sv.cpu().numpy(), reff.cpu().numpy()
    check(sv, reff, f_parts, b)
    assert np.all(reff[3, :25] == 1)


def test_ball_coefficients_rank_at_most_K_l(M, ctx):
    """Volumes through the front end: shells k >= |K_l| are zero, so every block's rank is at most
    |K_l| (eq. rank_bound), and the GPU values match the oracle's."""
    N, lam = 16, 14.0
    Lb, zeros = OB.ball_index(lam)
    Kl = np.array([z.size for z in zeros])
    rng = np.random.default_rng(8)
    vols = torch.from_numpy(rng.standard_normal((3, N, N, N)).astype(np.float32)).cuda()
    coef = M.ball_transform(ctx, vols, lam).cpu().numpy()  # [3, K, (L+1)^2]
    K = coef.shape[1]
    b = dict(L=np.array([Lb, Lb]), R=np.array([K, K]), Lh=Lb, Rh=K, h=coef[2].astype(np.complex128), w=np.ones(K))
    f_parts = [coef[0].astype(np.complex128), coef[1].astype(np.complex128)]
    batch, f, hh, ww = upload(M, b, f_parts)
    sv, reff = M.lowrank_spectrum(ctx, batch, f, hh, ww, rho=0.2, n_sv=K)
    sv, reff = sv.cpu().numpy(), reff.cpu().numpy()
    check(sv, reff, f_parts, b)
    for l in range(Lb + 1):
        assert np.all(sv[:, l, Kl[l]:] <= 1e-9 * sv[:, l, :1]), l
        assert np.all(reff[:, l] <= Kl[l])


def test_bench_workload_sampled(M, ctx):
    """The L = 32, 32-shell workload (1024 particles) in one launch; sampled particles against the
    oracle, and rotation invariance: the noiseless particle f = D(g) h has the spectrum of h with
    itself."""
    b0 = S.make_workload("L32_R32_B12_K16", n_particles=1024)
    parts = [b0.f(p) for p in range(b0.n_particles)]
    b = dict(L=b0.L, R=b0.R, Lh=b0.L_h, Rh=b0.R_h, h=b0.h, w=b0.w)
    batch, f, hh, ww = upload(M, b, parts)
    sv, reff = M.lowrank_spectrum(ctx, batch, f, hh, ww, rho=0.2)
    torch.cuda.synchronize()
    sv, reff = sv.cpu().numpy(), reff.cpu().numpy()
    sample = [0, 511, 1023]
    check(sv[sample], reff[sample], [parts[p] for p in sample],
          dict(L=b0.L[sample], R=b0.R[sample], Lh=b0.L_h, Rh=b0.R_h, h=b0.h, w=b0.w))
    nb = S.make_batch(32, 32, 1, seed=12, noiseless=True)
    b1 = dict(L=nb.L, R=nb.R, Lh=nb.L_h, Rh=nb.R_h, h=nb.h, w=nb.w)
    batch1, f1, h1, w1 = upload(M, b1, [nb.f(0)])
    s_rot, _ = M.lowrank_spectrum(ctx, batch1, f1, h1, w1)
    b2 = dict(L=nb.L, R=nb.R, Lh=nb.L_h, Rh=nb.R_h, h=nb.h, w=nb.w)
    batch2, f2, h2, w2 = upload(M, b2, [nb.h[:, : 33 * 33]])
    s_id, _ = M.lowrank_spectrum(ctx, batch2, f2, h2, w2)
    s_rot, s_id = s_rot.cpu().numpy(), s_id.cpu().numpy()
    assert np.abs(s_rot - s_id).max() <= 1e-5 * s_id.max()  # FP32 rounding of the rotated input


def test_lowrank_edges(M, ctx):
    import ctypes as ct
    lib = M.lib()
    rng = np.random.default_rng(2)
    h = S.hermitian_gaussian(rng, 50, 4, np.ones(5))
    b = dict(L=np.array([4]), R=np.array([50]), Lh=4, Rh=50, h=h, w=np.ones(50))
    batch, f, hh, ww = upload(M, b, [h])
    with pytest.raises(M.MatchaError, match="unsupported"):
        M.lowrank_spectrum(ctx, batch, f, hh, ww)
    b = dict(L=np.array([4]), R=np.array([8]), Lh=4, Rh=8, h=h[:8], w=np.ones(8))
    batch, f, hh, ww = upload(M, b, [h[:8]])
    for rho in (0.0, 1.0, -0.5):
        with pytest.raises(M.MatchaError, match="invalid"):
            M.lowrank_spectrum(ctx, batch, f, hh, ww, rho=rho)
    with pytest.raises(M.MatchaError, match="invalid"):
        M.lowrank_spectrum(ctx, batch, f, hh, ww, n_sv=65)
    empty = M.Batch.make([], [], 4, 8)
    bs = empty.c_struct()
    assert lib.matcha_lowrank_spectrum(ctx.handle, ct.byref(bs), None, None, None, 0.2, 4, None, None, None) == M.OK
    # a zero block: all singular values 0, r_eff 0
    batch, f, hh, ww = upload(M, dict(L=np.array([4]), R=np.array([8]), Lh=4, Rh=8, h=h[:8], w=np.ones(8)),
                              [np.zeros_like(h[:8])])
    sv, reff = M.lowrank_spectrum(ctx, batch, f, hh, ww)
    assert torch.all(sv == 0) and torch.all(reff == 0)


def test_maximum_shell_count_matches_oracle(M, ctx):
    """MATCHA_LOWRANK_MAX_SHELLS = 48 shells (the kernel's LDS then holds three 48 x 48 complex
    FP64 matrices, 110.6 KB) at degrees up to 30, where 2l + 1 crosses the shell count: ranks are
    min(2l + 1, 48) for generic inputs."""
    rng = np.random.default_rng(48)
    Lh, Rh = 30, 48
    var = 1.0 / (1.0 + np.arange(Lh + 1))
    h = S.hermitian_gaussian(rng, Rh, Lh, var)
    w = 1.0 + rng.uniform(0.0, 1.0, Rh)
    L = np.array([30, 12])
    R = np.array([48, 48])
    f_parts = [S.hermitian_gaussian(rng, int(r), int(l), var[: l + 1]) for l, r in zip(L, R)]
    b = dict(L=L, R=R, Lh=Lh, Rh=Rh, h=h, w=w)
    batch, f, hh, ww = upload(M, b, f_parts)
    sv, reff = M.lowrank_spectrum(ctx, batch, f, hh, ww, rho=0.2, n_sv=64)
    sv, reff = sv.cpu().numpy(), reff.cpu().numpy()
    check(sv, reff, f_parts, b)
