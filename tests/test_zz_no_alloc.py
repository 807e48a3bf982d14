"""matcha_soft_search_noalloc (the search on the library's static device scratch) against
matcha_soft_search (the search on a caller-owned workspace): the same candidates and status bits,
bit for bit, on two calls in a row -- a batch larger than one scratch chunk, then a smaller batch on
a smaller grid -- called through the C ABI."""
import ctypes as ct

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2603_15285_amd import synth as S  # noqa: E402


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_15285_amd import matcha
    matcha.lib()
    return matcha


def upload(M, b):
    batch = M.Batch.make(b.L, b.R, b.L_h, b.R_h, f_offset=b.f_offset)
    f = torch.from_numpy(b.f_flat.astype(np.complex64).view(np.float32).copy()).cuda()
    h = torch.from_numpy(b.h.astype(np.complex64).view(np.float32).reshape(-1).copy()).cuda()
    w = torch.from_numpy(b.w.astype(np.float32)).cuda()
    return batch, f, h, w


def search_both(M, ctx, batch, C, B, n, Kc):
    ctx.prepare(B, n)
    bs = batch.c_struct()
    cfg = M._SoftCfg(B, n, Kc)
    stream = ct.c_void_p(M._stream())
    cand_ws = torch.full((batch.n, Kc, 4), -1.0, dtype=torch.float32, device="cuda")
    st_ws = torch.full((batch.n,), -1, dtype=torch.int32, device="cuda")
    nb = M.workspace_bytes(batch, B, n)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    rc = M.lib().matcha_soft_search(ctx.handle, ct.byref(bs), M._ptr(C), ct.byref(cfg), M._ptr(cand_ws),
                                    M._ptr(st_ws), M._ptr(ws), nb, stream)
    assert rc == M.OK
    cand_na = torch.full((batch.n, Kc, 4), -2.0, dtype=torch.float32, device="cuda")
    st_na = torch.full((batch.n,), -2, dtype=torch.int32, device="cuda")
    rc = M.lib().matcha_soft_search_noalloc(ctx.handle, ct.byref(bs), M._ptr(C), ct.byref(cfg), M._ptr(cand_na),
                                            M._ptr(st_na), stream)
    assert rc == M.OK
    torch.cuda.synchronize()
    return (cand_ws, st_ws), (cand_na, st_na)


def test_noalloc_search_matches_workspace_search(M):
    ctx = M.Context(0)
    # first call: 300 particles at B = 12 on a 48^3 grid, more than one chunk of the 128 MiB scratch
    # (575 KB per particle: 227 particles per chunk)
    wl = S.WORKLOADS["L32_R32_B12_K16"]
    b1 = S.make_workload("L32_R32_B12_K16", n_particles=300)
    batch1, f1, h1, w1 = upload(M, b1)
    C1 = M.coeff_assemble(ctx, batch1, f1, h1, w1)
    ref, got = search_both(M, ctx, batch1, C1, wl.B, wl.n_grid, wl.Kc)
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
    assert torch.all(got[0][:, :, 1] > 0)  # every candidate written (b lies in (0, pi))
    # second call, smaller: 5 particles at B = 8 on a 32^3 grid, on the scratch the first call left
    b2 = S.make_batch(16, 8, 5, seed=17, snr=0.1)
    batch2, f2, h2, w2 = upload(M, b2)
    C2 = M.coeff_assemble(ctx, batch2, f2, h2, w2)
    ref, got = search_both(M, ctx, batch2, C2, 8, 32, 8)
    assert torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])
    # an unprepared shape is refused before anything runs
    bs = batch2.c_struct()
    cfg = M._SoftCfg(7, 28, 8)
    cand = torch.zeros((5, 8, 4), dtype=torch.float32, device="cuda")
    st = torch.zeros(5, dtype=torch.int32, device="cuda")
    rc = M.lib().matcha_soft_search_noalloc(ctx.handle, ct.byref(bs), M._ptr(C2), ct.byref(cfg), M._ptr(cand),
                                            M._ptr(st), ct.c_void_p(M._stream()))
    assert rc == M.ERR_NOT_PREPARED
    ctx.close()
