"""Adjoint (matcha_grad_template) on the GPU against the FP64 oracle and finite differences.

At fixed rotations F = sum_p g_p C_{L_p}(R_p*) is bilinear in (f, h), so central differences are
exact up to rounding for any step: the oracle check uses the 1e-3 step in FP64; the check on
the GPU's own FP32 objective uses a larger step so that FP32 rounding of F stays below the
tolerance.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
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


def upload(M, b):
    batch = M.Batch.make(b.L, b.R, b.L_h, b.R_h, f_offset=b.f_offset)
    f = torch.from_numpy(b.f_flat.astype(np.complex64).view(np.float32).copy()).cuda()
    h = torch.from_numpy(b.h.astype(np.complex64).view(np.float32).reshape(-1).copy()).cuda()
    w = torch.from_numpy(b.w.astype(np.float32)).cuda()
    return batch, f, h, w


def test_adjoint_matches_oracle_gradient(M, ctx):
    """The full 1024-particle launch; the upstream weights are non-zero on 16 sampled particles,
    so the oracle gradient of those 16 is the exact reference for the template gradient."""
    b = S.make_workload("adjoint_L32")
    P = b.n_particles
    rng = np.random.default_rng(4)
    eul = S.haar_euler(rng, P)
    sample = np.sort(rng.choice(P, 16, replace=False))
    g = np.zeros(P, dtype=np.float32)
    g[sample] = rng.standard_normal(16).astype(np.float32)
    batch, f, h, w = upload(M, b)
    best = torch.from_numpy(np.c_[eul, np.zeros(P)].astype(np.float32)).cuda()
    gh, gf = M.grad_template(ctx, batch, f, h, w, best, torch.from_numpy(g).cuda())
    gh = gh.cpu().numpy().view(np.complex64).reshape(b.R_h, -1)
    gf = gf.cpu().numpy().view(np.complex64)
    e32 = best.cpu().numpy().astype(np.float64)
    ref_h = np.zeros_like(b.h)
    for p in sample.tolist():
        ref_h, ref_f = O.grad_one(32, 32, b.f(p), b.h, 32, b.w, e32[p, :3], float(g[p]), grad_h=ref_h)
        o = b.f_offset[p]
        got = gf[o: o + ref_f.size].reshape(ref_f.shape)
        assert np.abs(got - ref_f).max() <= 2e-5 * np.abs(ref_f).max(), p
    assert np.abs(gh - ref_h).max() <= 2e-5 * np.abs(ref_h).max()


def test_adjoint_uneven_and_deterministic(M, ctx):
    b = S.make_batch(24, 20, 5, seed=8, snr=0.2, L_per=[24, 10, 17, 3, 24], R_per=[20, 7, 12, 2, 5])
    rng = np.random.default_rng(5)
    eul = S.haar_euler(rng, 5)
    g = rng.standard_normal(5).astype(np.float32)
    batch, f, h, w = upload(M, b)
    best = torch.from_numpy(np.c_[eul, np.zeros(5)].astype(np.float32)).cuda()
    gt = torch.from_numpy(g).cuda()
    gh1, gf1 = M.grad_template(ctx, batch, f, h, w, best, gt)
    gh2, gf2 = M.grad_template(ctx, batch, f, h, w, best, gt)
    assert torch.equal(gh1, gh2) and torch.equal(gf1, gf2)  # fixed-order reduction
    gh = gh1.cpu().numpy().view(np.complex64).reshape(b.R_h, -1)
    gfa = gf1.cpu().numpy().view(np.complex64)
    e32 = best.cpu().numpy().astype(np.float64)
    ref_h = np.zeros_like(b.h)
    for p in range(5):
        Lp, Rp = int(b.L[p]), int(b.R[p])
        ref_h, ref_f = O.grad_one(Lp, Rp, b.f(p), b.h, 24, b.w, e32[p, :3], float(g[p]), grad_h=ref_h)
        o = b.f_offset[p]
        got = gfa[o: o + ref_f.size].reshape(ref_f.shape)
        assert np.abs(got - ref_f).max() <= 2e-5 * np.abs(ref_f).max()
    assert np.abs(gh - ref_h).max() <= 2e-5 * np.abs(ref_h).max()


def test_adjoint_padded_and_permuted_f_offsets(M, ctx):
    """f_offset need not be packed: particles stored out of order with gaps between them (the
    library packs its own workspace).  grad_f lands at each particle's own offset, nothing is
    written into the gaps, and grad_h matches the oracle."""
    b = S.make_batch(16, 12, 4, seed=12, snr=0.2, L_per=[16, 9, 16, 5], R_per=[12, 6, 3, 12])
    rng = np.random.default_rng(13)
    eul = S.haar_euler(rng, 4)
    g = rng.standard_normal(4).astype(np.float32)
    sizes = [b.f(p).size for p in range(4)]
    order = [2, 0, 3, 1]  # storage order in f
    gap = 1000
    offs = np.zeros(4, dtype=np.int64)
    o = gap
    for p in order:
        offs[p] = o
        o += sizes[p] + gap
    flat = np.zeros(o, dtype=np.complex64)
    for p in range(4):
        flat[offs[p]: offs[p] + sizes[p]] = b.f(p).reshape(-1)
    batch = M.Batch.make(b.L, b.R, b.L_h, b.R_h, f_offset=offs)
    f = torch.from_numpy(flat.view(np.float32).copy()).cuda()
    h = torch.from_numpy(b.h.astype(np.complex64).view(np.float32).reshape(-1).copy()).cuda()
    w = torch.from_numpy(b.w.astype(np.float32)).cuda()
    best = torch.from_numpy(np.c_[eul, np.zeros(4)].astype(np.float32)).cuda()
    gh, gf = M.grad_template(ctx, batch, f, h, w, best, torch.from_numpy(g).cuda())
    packed = M.Batch.make(b.L, b.R, b.L_h, b.R_h)
    assert M.grad_workspace_bytes(batch) == M.grad_workspace_bytes(packed)  # not sized by the padded f
    gh = gh.cpu().numpy().view(np.complex64).reshape(b.R_h, -1)
    gfa = gf.cpu().numpy().view(np.complex64)
    e32 = best.cpu().numpy().astype(np.float64)
    ref_h = np.zeros_like(b.h)
    used = np.zeros(o, dtype=bool)
    for p in range(4):
        Lp, Rp = int(b.L[p]), int(b.R[p])
        ref_h, ref_f = O.grad_one(Lp, Rp, b.f(p), b.h, 16, b.w, e32[p, :3], float(g[p]), grad_h=ref_h)
        got = gfa[offs[p]: offs[p] + sizes[p]].reshape(ref_f.shape)
        assert np.abs(got - ref_f).max() <= 2e-5 * np.abs(ref_f).max(), p
        used[offs[p]: offs[p] + sizes[p]] = True
    assert np.abs(gh - ref_h).max() <= 2e-5 * np.abs(ref_h).max()
    # grad_f only, through the C ABI into a pre-filled buffer: the gaps keep their contents
    gf2 = torch.full_like(f, 3.0)
    bs = batch.c_struct()
    nb = M.grad_workspace_bytes(batch)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    rc = M.lib().matcha_grad_template(ctx.handle, M.ct.byref(bs), M._ptr(f), M._ptr(h), M._ptr(w), M._ptr(best),
                                      M._ptr(torch.from_numpy(g).cuda()), None, M._ptr(gf2), M.FP32, M._ptr(ws), nb,
                                      M.ct.c_void_p(M._stream()))
    assert rc == M.OK
    gf2 = gf2.cpu().numpy().view(np.complex64)
    assert np.all(gf2[~used] == 3.0 + 3.0j)  # the gaps are untouched
    assert np.array_equal(gf2[used], gfa[used])


def test_adjoint_central_differences(M, ctx):
    b = S.make_workload("adjoint_L32", n_particles=4)
    rng = np.random.default_rng(6)
    eul = S.haar_euler(rng, 4)
    g = rng.standard_normal(4)
    batch, f, h, w = upload(M, b)
    best = torch.from_numpy(np.c_[eul, np.zeros(4)].astype(np.float32)).cuda()
    gh, gf = M.grad_template(ctx, batch, f, h, w, best, torch.from_numpy(g.astype(np.float32)).cuda())
    gh = gh.cpu().numpy()
    gf = gf.cpu().numpy()
    e32 = best.cpu().numpy().astype(np.float64)

    def oracle_loss(hc, fs):
        return sum(g[p] * O.evaluate_F(32, O.coeff_assemble(32, 32, fs[p], 32, hc, 32, b.w), e32[p, :3]) for p in range(4))

    def gpu_loss(hv, fv):
        C = M.coeff_assemble(ctx, batch, fv, hv, w)
        F = M.evaluate(ctx, batch, C, 0, best)[:, 0].double().cpu().numpy()
        return float(np.dot(g, F))

    fs = [b.f(p).copy() for p in range(4)]
    Sc = [np.sqrt(np.sum(b.w[:, None] * np.abs(fs[p]) ** 2) * np.sum(b.w[:, None] * np.abs(b.h) ** 2)) for p in range(4)]
    S_tot = float(np.dot(np.abs(g), Sc))
    for _ in range(6):
        # template entry: oracle FD at step 1e-3 (FP64) and GPU FD at a larger step (FP32)
        r, j = rng.integers(32), rng.integers(33 * 33)
        for part, unit in ((0, 1.0), (1, 1j)):
            hp, hm = b.h.copy(), b.h.copy()
            hp[r, j] += 1e-3 * unit
            hm[r, j] -= 1e-3 * unit
            fd = (oracle_loss(hp, fs) - oracle_loss(hm, fs)) / 2e-3
            an = gh[2 * (r * 33 * 33 + j) + part]
            assert abs(fd - an) <= 1e-4 * max(1.0, abs(an)), (r, j, part, fd, an)
            # The GPU assembly forms the half plane m >= 0 and completes C by the symmetry of
            # real-space functions, so its finite difference moves h along a direction that keeps
            # c_{l,-n} = (-1)^n conj(c_ln): the entry and its mirror together.  The analytic
            # directional derivative is then the sum of both entries' partials.
            l = int(np.sqrt(j))
            n = j - l * l - l
            jm = l * l + l - n
            sgn = -1.0 if (n & 1) else 1.0
            if n == 0 and part == 1:
                continue  # c_l0 is real: no symmetric imaginary direction
            ia, ib = 2 * (r * 33 * 33 + j) + part, 2 * (r * 33 * 33 + jm) + part
            # mirror moves by (-1)^n conj(unit): +(-1)^n on the real part, -(-1)^n on the imaginary
            mir = sgn if part == 0 else -sgn
            an_dir = an if jm == j else an + mir * gh[ib]
            step = 0.5
            hv = h.clone()
            hv[ia] += step
            if jm != j:
                hv[ib] += mir * step
            lp = gpu_loss(hv, f)
            hv[ia] -= 2 * step
            if jm != j:
                hv[ib] -= 2 * mir * step
            lm = gpu_loss(hv, f)
            # FP32 objective: each F carries ~1e-6 S of rounding, divided by the 2 * step of the difference
            assert abs((lp - lm) / (2 * step) - an_dir) <= 2e-6 * S_tot / step + 1e-3 * abs(an_dir), (lp, lm, an_dir)
        # particle entry
        p, r, j = rng.integers(4), rng.integers(32), rng.integers(33 * 33)
        o = int(b.f_offset[p]) + r * 33 * 33 + j
        for part, unit in ((0, 1.0), (1, 1j)):
            fp_, fm_ = [x.copy() for x in fs], [x.copy() for x in fs]
            fp_[p][r, j] += 1e-3 * unit
            fm_[p][r, j] -= 1e-3 * unit
            fd = (oracle_loss(b.h, fp_) - oracle_loss(b.h, fm_)) / 2e-3
            an = gf[2 * o + part]
            assert abs(fd - an) <= 1e-4 * max(1.0, abs(an)), (p, r, j, part, fd, an)


def test_objective_autograd(M, ctx):
    b = S.make_workload("adjoint_L32", n_particles=3)
    rng = np.random.default_rng(7)
    eul = S.haar_euler(rng, 3)
    batch, f, h, w = upload(M, b)
    best = torch.from_numpy(np.c_[eul, np.zeros(3)].astype(np.float32)).cuda()
    fr = f.clone().requires_grad_(True)
    hr = h.clone().requires_grad_(True)
    F = M.Objective.apply(ctx, batch, fr, hr, w, best)
    g = torch.tensor([0.5, -1.0, 2.0], device="cuda")
    (F * g).sum().backward()
    gh, gf = M.grad_template(ctx, batch, f, h, w, best, g)
    assert torch.allclose(hr.grad, gh) and torch.allclose(fr.grad, gf)
    e32 = best.cpu().numpy().astype(np.float64)
    for p in range(3):
        ref = O.evaluate_F(32, O.coeff_assemble(32, 32, b.f(p), 32, b.h, 32, b.w), e32[p, :3])
        Sc = np.sqrt(np.sum(b.w[:, None] * np.abs(b.f(p)) ** 2) * np.sum(b.w[:, None] * np.abs(b.h) ** 2))
        assert abs(F[p].item() - ref) <= 1e-5 * Sc
