"""Host-side logic that needs no GPU: longest-first ordering, workspace sizing, the ball-harmonic
index set and the bench's use of the recorded march traffic."""
import ctypes as ct

import numpy as np

from paper_2603_15285_amd import matcha as M


def host_batch(L, R, L_h, R_h):
    L = np.ascontiguousarray(L, dtype=np.int32)
    R = np.ascontiguousarray(R, dtype=np.int32)
    b = M._Batch()
    b.n_particles = L.size
    b.L_max = int(L.max()) if L.size else 0
    b.L_host = L.ctypes.data_as(ct.POINTER(ct.c_int32))
    b.R_host = R.ctypes.data_as(ct.POINTER(ct.c_int32))
    # device arrays are only checked for presence on the host; never dereferenced here
    dummy = ct.c_void_p(16)
    b.L_dev = b.R_dev = b.f_offset = b.C_offset = dummy
    b.L_h, b.R_h = L_h, R_h
    b.order = None
    return b, (L, R)


def lpt(L, levels, steps=3):
    b, keep = host_batch(L, [1] * len(L), 64, 1)
    cfg = M._march_cfg(levels, steps)
    out = np.zeros(len(L), dtype=np.int32)
    rc = M.lib().matcha_lpt_order(ct.byref(b), ct.byref(cfg), out.ctypes.data_as(ct.POINTER(ct.c_int32)))
    return rc, out


def test_lpt_order_longest_first_and_stable():
    L = [24, 48, 31, 48, 24, 40]
    rc, out = lpt(L, [12, 16, 24, 32, 40, 48])
    assert rc == M.OK
    assert out.tolist() == [1, 3, 5, 2, 0, 4]  # by decreasing cost, ties by index


def test_lpt_order_cost_model():
    """cost = sum over the schedule (levels below L_p, then L_p) of the wedge terms (L+1)(L+2)(2L+3)/6."""
    def cost(Lp, levels):
        sched = [x for x in levels if x < Lp] + [Lp]
        return sum((x + 1) * (x + 2) * (2 * x + 3) // 6 for x in sched)
    rng = np.random.default_rng(0)
    L = rng.integers(1, 65, size=50).tolist()
    levels = [8, 16, 32, 48]
    rc, out = lpt(L, levels)
    c = [cost(L[i], levels) for i in out]
    assert rc == M.OK and all(c[i] >= c[i + 1] for i in range(len(c) - 1))


def test_lpt_order_rejects_bad_arguments():
    rc, _ = lpt([70], [8])  # L above the build limit
    assert rc == M.ERR_INVALID_ARG


def align256(x):
    return (x + 255) // 256 * 256


def soft_particle(n, B):
    """Per particle: n^3 floats of grid, 1024 maxima keys, a count, n (B+1)(2B+1) complex node transforms."""
    return n ** 3 * 4, 1024 * 8, 4, n * (B + 1) * (2 * B + 1) * 8


def soft_chunk(pc, n, B):
    g, l, c, s = soft_particle(n, B)
    return align256(pc * g) + align256(pc * l) + align256(pc * c) + align256(pc * s)


def test_workspace_size_is_the_largest_call_need():
    """matcha_workspace_size = max(assembly order buffer, SOFFT chunk of the whole batch, the
    persistent march's 256-byte counter);
    matcha_grad_workspace_size = the adjoint's offsets and per-particle template terms."""
    L, R = [32, 10, 3], [32, 5, 2]
    b, keep = host_batch(L, R, 32, 32)
    E = 32 * 33 * 33  # template entries
    seg = min(64, 3, -(-2048 // -(-E // 256)))
    grad = align256(8 * 3) + align256(seg * E * 8) + 8 * sum(r * (l + 1) ** 2 for l, r in zip(L, R))
    assert M.lib().matcha_grad_workspace_size(ct.byref(b)) == grad
    assert M.lib().matcha_workspace_size(None, ct.byref(b), None, None) == 256  # the march's work counter
    soft = M._SoftCfg(3, 12, 4)
    want = max(soft_chunk(3, 12, 3), 4 * 3, 256)
    assert M.lib().matcha_workspace_size(None, ct.byref(b), ct.byref(soft), None) == want
    soft = M._SoftCfg(12, 48, 16)
    assert M.lib().matcha_workspace_size(None, ct.byref(b), ct.byref(soft), None) == soft_chunk(3, 48, 12)
    # empty or invalid batches need nothing
    e, keep2 = host_batch([], [], 32, 32)
    e.n_particles = 0
    assert M.lib().matcha_workspace_size(None, ct.byref(e), ct.byref(soft), None) == 0
    bad, keep3 = host_batch([40], [4], 32, 32)  # L_p above the template's band
    assert M.lib().matcha_workspace_size(None, ct.byref(bad), None, None) == 0
    assert M.lib().matcha_grad_workspace_size(ct.byref(bad)) == 0
    assert M.lib().matcha_grad_workspace_size(ct.byref(e)) == 0


def test_workspace_too_small_is_reported_before_the_context():
    """Every enqueue call checks its workspace on the host, before it needs a context or a device: a
    short workspace gives MATCHA_ERR_WORKSPACE, an adequate one then fails only on the NULL context."""
    lib = M.lib()
    dev = ct.c_void_p(1 << 20)  # aligned stand-in for device buffers: never dereferenced by these checks
    L, R = [8, 6, 8], [4, 4, 3]
    b, keep = host_batch(L, R, 8, 4)
    b.f_offset = dev
    # assembly of mixed band limits needs P int32
    rc = lib.matcha_coeff_assemble(None, ct.byref(b), dev, dev, dev, dev, M.FP32, dev, 11, None)
    assert rc == M.ERR_WORKSPACE
    rc = lib.matcha_coeff_assemble(None, ct.byref(b), dev, dev, dev, dev, M.FP32, None, 0, None)
    assert rc == M.ERR_WORKSPACE
    rc = lib.matcha_coeff_assemble(None, ct.byref(b), dev, dev, dev, dev, M.FP32, dev, 12, None)
    assert rc == M.ERR_INVALID_ARG
    # equal band limits need no workspace
    bu, keepu = host_batch([8, 8], [4, 4], 8, 4)
    bu.f_offset = dev
    assert lib.matcha_coeff_assemble(None, ct.byref(bu), dev, dev, dev, dev, M.FP32, None, 0, None) == M.ERR_INVALID_ARG
    # search: one particle's share at least
    soft = M._SoftCfg(4, 16, 8)
    one = soft_chunk(1, 16, 4)
    rc = lib.matcha_soft_search(None, ct.byref(b), dev, ct.byref(soft), dev, dev, dev, one - 1, None)
    assert rc == M.ERR_WORKSPACE
    rc = lib.matcha_soft_search(None, ct.byref(b), dev, ct.byref(soft), dev, dev, dev, one, None)
    assert rc == M.ERR_INVALID_ARG
    rc = lib.matcha_soft_search(None, ct.byref(b), dev, ct.byref(soft), dev, dev, ct.c_void_p((1 << 20) + 8), one,
                                None)
    assert rc == M.ERR_WORKSPACE  # misaligned
    # adjoint with grad_h: offsets and terms
    E = 4 * 9 * 9
    seg = min(64, 3, -(-2048 // -(-E // 256)))
    need = align256(8 * 3) + align256(seg * E * 8) + 8 * sum(r * (l + 1) ** 2 for l, r in zip(L, R))
    args = (None, ct.byref(b), dev, dev, dev, dev, dev, dev, None, M.FP32)
    assert lib.matcha_grad_template(*args, dev, need - 1, None) == M.ERR_WORKSPACE
    assert lib.matcha_grad_template(*args, dev, need, None) == M.ERR_INVALID_ARG
    # grad_f only: no workspace
    args_f = (None, ct.byref(b), dev, dev, dev, dev, dev, None, dev, M.FP32)
    assert lib.matcha_grad_template(*args_f, None, 0, None) == M.ERR_INVALID_ARG
    # only FP32 is offered
    args_b = (None, ct.byref(b), dev, dev, dev, dev, dev, dev, None, M.BF16_FP32ACC)
    assert lib.matcha_grad_template(*args_b, dev, need, None) == M.ERR_UNSUPPORTED


def test_march_traffic_reported_only_for_its_workload_and_sources(tmp_path, monkeypatch):
    """The bench's HBM-traffic figure comes from a counter summary; it is used only while the
    summary names the timed workload and the march sources still hash to the recorded digest."""
    import bench

    def summary(workload, digest, nbytes):
        p = tmp_path / f"traffic_{workload}_{digest[:8]}.txt"
        p.write_text(f"workload: {workload}\nkernel_source_sha256: {digest}\nhbm_bytes_per_launch: {nbytes}\n")
        return str(p)

    digest = bench.march_source_digest()
    monkeypatch.setattr(bench, "TRAFFIC_FILE", summary("L32_R32_B12_K16", digest, 123456))
    assert bench.measured_march_traffic("L32_R32_B12_K16") == 123456.0
    assert bench.measured_march_traffic("uneven_L24to48") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", summary("L32_R32_B12_K16", "0" * 64, 123456))
    assert bench.measured_march_traffic("L32_R32_B12_K16") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.txt"))
    assert bench.measured_march_traffic("L32_R32_B12_K16") is None


def test_ball_index_matches_the_oracle_and_rejects_bad_cutoffs():
    """matcha_ball_index (host FP64 zeros) against the oracle's scipy-based zeros (App. A.1)."""
    from oracle import ball as OB
    for lam in (3.2, 9.0, 14.0, 38.0, 71.0):
        L, zeros = M.ball_index(lam)
        Lo, zo = OB.ball_index(lam)
        assert L == Lo and [z.size for z in zeros] == [z.size for z in zo]
        for a, b in zip(zeros, zo):
            assert np.abs(a - b).max() <= 4e-15 * lam
    L, K = ct.c_int32(), ct.c_int32()
    for lam in (0.0, -1.0, 3.0, 71.5, float("nan")):
        assert M.lib().matcha_ball_index(lam, ct.byref(L), ct.byref(K), None, None) == M.ERR_INVALID_ARG
    assert M.lib().matcha_ball_index(9.0, None, ct.byref(K), None, None) == M.ERR_INVALID_ARG


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and says why, before any GPU work."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
