"""Batched execution: HIP-graph replay, launch-shape tuning and longest-first ordering must not
change any result (every kernel is deterministic, so results are compared bit for bit)."""
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


def eager(M, ctx, batch, f, h, w, wl):
    best, bi, st = M.align(ctx, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps)
    torch.cuda.synchronize()
    return best.clone(), bi.clone(), st.clone()


def test_graph_replays_match_eager(M, ctx):
    wl = S.WORKLOADS["L32_R32_B12_K16"]
    b1 = S.make_workload("L32_R32_B12_K16", n_particles=64)
    b2 = S.make_workload("L32_R32_B12_K16", n_particles=64, seed_offset=1)
    batch, f, h, w = upload(M, b1)
    _, f2, _, _ = upload(M, b2)
    ref1 = eager(M, ctx, batch, f, h, w, wl)
    ref2 = eager(M, ctx, batch, f2, h, w, wl)
    g = M.AlignGraph(ctx, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps)
    f_orig = f.clone()
    for rep in range(3):
        if rep == 1:
            f.copy_(f2)  # the graph reads its buffers at replay time
        else:
            f.copy_(f_orig)
        eager(M, ctx, batch, f2, h, w, wl)  # unrelated eager work between replays
        best, bi, st = g.launch()
        torch.cuda.synchronize()
        ref = ref2 if rep == 1 else ref1
        assert torch.equal(best, ref[0]) and torch.equal(bi, ref[1]) and torch.equal(st, ref[2]), rep
    g.close()


def test_autotune_keeps_results(M):
    """The tuner's choice and every other launch or tile shape (assembly row tiles per wave, grid
    nodes per wave, ranking workgroup, march candidates per wave, persistent march) give the same
    C, candidates and selections, bit for bit."""
    c = M.Context(0)
    wl = S.WORKLOADS["L32_R32_B12_K16"]
    b = S.make_workload("L32_R32_B12_K16", n_particles=128)
    batch, f, h, w = upload(M, b)
    ref = eager(M, c, batch, f, h, w, wl)
    refC = M.coeff_assemble(c, batch, f, h, w).clone()
    t = M.autotune(c, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, reps=1)
    assert t["march_nc"] in (2, 4, 8) and t["soft_threads"] in (256, 512) and t["asm_tiles"] in (1, 2, 4, 8)
    assert t["grid_nodes"] in (8, 16, 32, 48, 64) and t["march_persistent"] in (0, 1)
    assert c.get_tuning() == t
    got = eager(M, c, batch, f, h, w, wl)
    for x, y in zip(got, ref):
        assert torch.equal(x, y)
    for shape in [(2, 256, 1, 8, 1), (8, 512, 8, 32, 0), (4, 256, 2, 16, 1), (4, 256, 4, 48, 1), (2, 512, 2, 64, 0),
                  (1, 0, 0, 0, 1)]:
        c.set_tuning(*shape)
        assert torch.equal(M.coeff_assemble(c, batch, f, h, w), refC), shape
        got = eager(M, c, batch, f, h, w, wl)
        for x, y in zip(got, ref):
            assert torch.equal(x, y), shape
    with pytest.raises(M.MatchaError):
        c.set_tuning(0, 0, 3, 0, 0)  # not a supported tile count
    with pytest.raises(M.MatchaError):
        c.set_tuning(0, 0, 0, 12, 0)
    c.close()


def test_persistent_march_uneven_longest_first(M):
    """The persistent march (workgroups taking particles from a counter) on the uneven workload in
    longest-first order, with more particles than resident workgroups: the same results, bit for
    bit, as one workgroup per particle."""
    c = M.Context(0)
    wl = S.WORKLOADS["uneven_L24to48"]
    b = S.make_workload("uneven_L24to48", n_particles=600)
    batch, f, h, w = upload(M, b)
    batch.set_lpt_order(wl.levels, wl.steps)
    C = M.coeff_assemble(c, batch, f, h, w)
    cand0, st0 = M.soft_search(c, batch, C, wl.B, wl.n_grid, wl.Kc)
    out = {}
    for pers in (0, 1):
        c.set_tuning(4, 0, 0, 0, pers)
        cand, st = cand0.clone(), st0.clone()
        best, bi, st = M.march_newton(c, batch, C, wl.levels, wl.steps, cand, st, fp64_above=40)
        torch.cuda.synchronize()
        out[pers] = (cand, best, bi, st)
    for x, y in zip(out[0], out[1]):
        assert torch.equal(x, y)
    c.close()


def test_longest_first_order_keeps_results(M, ctx):
    wl = S.WORKLOADS["uneven_L24to48"]
    b = S.make_workload("uneven_L24to48", n_particles=48)
    batch, f, h, w = upload(M, b)
    ref = eager(M, ctx, batch, f, h, w, wl)
    order = batch.set_lpt_order(wl.levels, wl.steps)
    assert sorted(order.tolist()) == list(range(48))
    Ls = b.L[order]
    assert np.all(np.diff(Ls) <= 0)  # longer bands (more work) first
    got = eager(M, ctx, batch, f, h, w, wl)
    for x, y in zip(got, ref):
        assert torch.equal(x, y)


def test_march_near_pole_candidates_independent_of_grouping(M):
    """Candidates at and next to the poles beside ordinary ones: every candidate's result must be the
    same however the candidates are grouped into waves (march_nc)."""
    c = M.Context(0)
    wl = S.WORKLOADS["L32_R32_B12_K16"]
    b = S.make_workload("L32_R32_B12_K16", n_particles=6)
    batch, f, h, w = upload(M, b)
    C = M.coeff_assemble(c, batch, f, h, w)
    cand0, st0 = M.soft_search(c, batch, C, wl.B, wl.n_grid, wl.Kc)
    cand0[:, 1, 1] = 5e-5
    cand0[:, 6, 1] = float(np.pi - 3e-5)
    cand0[::2, 9, 1] = 2e-4
    cand0[1::2, 13, 1] = 0.0
    out = {}
    for nc in (1, 2, 4, 8):
        c.set_tuning(nc, 0, 0, 0, nc % 2 == 0)
        cand, st = cand0.clone(), st0.clone()
        best, bi, st = M.march_newton(c, batch, C, wl.levels, wl.steps, cand, st)
        torch.cuda.synchronize()
        out[nc] = (cand, best, bi, st)
    for nc in (2, 4, 8):
        for x, y in zip(out[nc], out[1]):
            assert torch.equal(x, y), nc
    assert torch.isfinite(out[1][0]).all()
    c.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_uneven_graph_and_assembly_order(M, ctx, prec):
    """Mixed band limits: the assembly covers each degree's rows only for particles with L_p >= l,
    in an order it computes on the device.  The graph (its own order buffer) must replay the
    eager results, and the assembled C must not depend on the particles' order in the batch."""
    wl = S.WORKLOADS["uneven_L24to48"]
    b = S.make_workload("uneven_L24to48", n_particles=40)
    batch, f, h, w = upload(M, b)
    p = M.BF16_FP32ACC if prec == "bf16" else M.FP32
    if prec == "bf16":
        f, h = f.to(torch.bfloat16), h.to(torch.bfloat16)
    C0 = M.coeff_assemble(ctx, batch, f, h, w, prec=p)
    cand, st = M.soft_search(ctx, batch, C0, wl.B, wl.n_grid, wl.Kc)
    best, bi, st = M.march_newton(ctx, batch, C0, wl.levels, wl.steps, cand, st, fp64_above=40)
    torch.cuda.synchronize()
    ref = (best.clone(), bi.clone(), st.clone())
    g = M.AlignGraph(ctx, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, prec=p, fp64_above=40)
    for rep in range(2):
        M.coeff_assemble(ctx, batch, f, h, w, prec=p)  # eager work on the context's own order buffer
        got = g.launch()
        torch.cuda.synchronize()
        for x, y in zip(got, ref):
            assert torch.equal(x, y), rep
    g.close()
    # the same particles in reverse order: each particle's C is unchanged bit for bit
    C = M.coeff_assemble(ctx, batch, f, h, w, prec=p).cpu().numpy()
    rev = np.arange(b.n_particles)[::-1].copy()
    sizes = [b.f(q).size for q in rev]
    br = S.Batch(L_h=b.L_h, R_h=b.R_h, h=b.h, w=b.w, L=b.L[rev].copy(), R=b.R[rev].copy(),
                 f_offset=np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64),
                 f_flat=np.concatenate([b.f(q).reshape(-1) for q in rev]), euler_true=b.euler_true[rev],
                 snr=np.asarray(b.snr)[rev])
    batch_r, fr, _, _ = upload(M, br)
    if prec == "bf16":
        fr = fr.to(torch.bfloat16)
    Cr = M.coeff_assemble(ctx, batch_r, fr, h, w, prec=p).cpu().numpy()
    for i, q in enumerate(rev):
        n = 2 * M.c_elems(int(b.L[q]))
        o, orv = 2 * int(batch.C_offset[q]), 2 * int(batch_r.C_offset[i])
        assert np.array_equal(C[o: o + n], Cr[orv: orv + n]), q


def test_bf16_graph_with_fp32_final_level_matches_eager(M, ctx):
    """The BF16 path whose final level marches on FP32-assembled coefficients, as one graph (two
    assemblies, search, march) against the same calls made eagerly: bit for bit."""
    wl = S.WORKLOADS["L32_R32_B12_K16"]
    b = S.make_workload("L32_R32_B12_K16", n_particles=32)
    batch, f, h, w = upload(M, b)
    f16, h16 = f.to(torch.bfloat16), h.to(torch.bfloat16)
    best, bi, st = M.align(ctx, batch, f16, h16, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps,
                           prec=M.BF16_FP32ACC, f32=f, h32=h)
    torch.cuda.synchronize()
    ref = (best.clone(), bi.clone(), st.clone())
    g = M.AlignGraph(ctx, batch, f16, h16, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, prec=M.BF16_FP32ACC,
                     f32=f, h32=h)
    for rep in range(3):
        eager(M, ctx, batch, f, h, w, wl)  # unrelated eager work between replays
        got = g.launch()
        torch.cuda.synchronize()
        for x, y in zip(got, ref):
            assert torch.equal(x, y), rep
    g.close()


def test_caller_captures_the_path_with_its_own_workspace(M):
    """Every enqueue call allocates nothing and never synchronises, so a caller can capture the whole
    path (assembly of mixed band limits, search, march) into a graph of its own with a workspace it
    owns (torch.cuda.CUDAGraph here).  Each replay, with eager work and synchronisations between
    replays, matches the eager result bit for bit."""
    c = M.Context(0)
    wl = S.WORKLOADS["uneven_L24to48"]
    b = S.make_workload("uneven_L24to48", n_particles=24)
    batch, f, h, w = upload(M, b)
    c.prepare(wl.B, wl.n_grid)
    nb = M.workspace_bytes(batch, wl.B, wl.n_grid)
    ws = c.workspace(nb)
    bufs = dict(C=torch.empty(2 * batch.c_total, dtype=torch.float32, device="cuda"),
                cand=torch.empty((batch.n, wl.Kc, 4), dtype=torch.float32, device="cuda"),
                status=torch.empty(batch.n, dtype=torch.int32, device="cuda"),
                best=torch.empty((batch.n, 4), dtype=torch.float32, device="cuda"),
                best_idx=torch.empty(batch.n, dtype=torch.int32, device="cuda"))

    def run():
        return M.align(c, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, fp64_above=40, bufs=bufs)

    run()
    torch.cuda.synchronize()
    ref = tuple(x.clone() for x in (bufs["best"], bufs["best_idx"], bufs["status"]))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run()
    assert c.workspace(nb) is ws  # no workspace was allocated during capture
    for rep in range(3):
        for t in bufs.values():
            t.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (bufs["best"], bufs["best_idx"], bufs["status"])
        for x, y in zip(got, ref):
            assert torch.equal(x, y), rep
        M.soft_search(c, batch, bufs["C"], 8, 24, 8)  # eager work between replays
        torch.cuda.synchronize()
    del graph
    c.close()


def test_tune_cache_persists_results(M, tmp_path):
    """matcha_create(tune_cache): autotune stores its choice in the file; a new context on the same
    file applies the stored choice for the same batch and configuration without timing again (no
    new line), and a different configuration is timed and added."""
    path = str(tmp_path / "tune.txt")
    wl = S.WORKLOADS["L32_R32_B12_K16"]
    b = S.make_workload("L32_R32_B12_K16", n_particles=64)
    batch, f, h, w = upload(M, b)
    c1 = M.Context(0, tune_cache=path)
    t1 = M.autotune(c1, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, reps=1)
    c1.close()
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:] == [str(t1[k]) for k in M.TUNING_FIELDS]
    c2 = M.Context(0, tune_cache=path)
    assert c2.get_tuning() == {k: 0 for k in M.TUNING_FIELDS}
    t2 = M.autotune(c2, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, reps=1)
    assert t2 == t1 and c2.get_tuning() == t1
    assert len(open(path).read().splitlines()) == 1
    M.autotune(c2, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, 2, reps=1)  # another schedule
    assert len(open(path).read().splitlines()) == 2
    c2.close()


def test_graph_survives_other_shapes_on_its_context(M):
    """A graph keeps pointing at the context's tables: searches at another (B, n) and evaluations at
    a larger band on the same context between replays must not disturb it (tables are freed only
    with the context)."""
    c = M.Context(0)
    wl = S.WORKLOADS["L32_R32_B12_K16"]
    b = S.make_workload("L32_R32_B12_K16", n_particles=16)
    batch, f, h, w = upload(M, b)
    ref = eager(M, c, batch, f, h, w, wl)
    g = M.AlignGraph(c, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps)
    bb = S.make_batch(48, 8, 2, seed=5, snr=0.1)
    batch2, f2, h2, w2 = upload(M, bb)
    for rep in range(2):
        C = M.coeff_assemble(c, batch, f, h, w)
        M.soft_search(c, batch, C, 8, 24, 8)
        C2 = M.coeff_assemble(c, batch2, f2, h2, w2)
        M.evaluate(c, batch2, C2, 48, torch.zeros((2, 4), dtype=torch.float32, device="cuda"), fp64_above=40)
        M.soft_search(c, batch2, C2, 16, 40, 8)
        got = g.launch()
        torch.cuda.synchronize()
        for x, y in zip(got, ref):
            assert torch.equal(x, y), rep
    g.close()
    c.close()
