"""Host-side logic that needs no GPU: longest-first ordering, workspace sizing and the bench's
use of the recorded march traffic."""
import ctypes as ct

import numpy as np

from paper_2603_15285_amd import matcha as M


def host_batch(L, R, L_h, R_h):
    L = np.ascontiguousarray(L, dtype=np.int32)
    R = np.ascontiguousarray(R, dtype=np.int32)
    b = M._Batch()
    b.n_particles = L.size
    b.L_max = int(L.max())
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


def test_workspace_is_one_template_term_per_particle():
    L, R = [32, 10, 3], [32, 5, 2]
    b, keep = host_batch(L, R, 32, 32)
    n = M.lib().matcha_workspace_size(ct.byref(b), 16)
    assert n == 8 * sum(r * (l + 1) ** 2 for l, r in zip(L, R))


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
