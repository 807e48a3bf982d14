"""Throughput of the rotational-alignment path on one GPU.

A step is one pass of the whole path -- coefficient assembly, SOFFT search, frequency
march and selection -- over one batch of synthetic particles already resident in HBM.
Prints one JSON line (see the fields below).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particles/sec rotationally refined at L=32, batched vs plain; % of roofline"
# MI355X's published FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2 (packed FP32)
# x 2.4 GHz.  This build issues no packed FP32 instructions, so its own ceiling is half of that.
VALU_FP32_PEAK_TFLOPS = 157.3
VALU_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def wedge_terms(L):
    """(l, wedge pair) recurrence steps of one evaluation at band L: sum_{l<=L} (l+1)^2."""
    return (L + 1) * (L + 2) * (2 * L + 3) // 6


def march_flops_per_particle(levels, L, steps, Kc):
    """Algorithmic FP32 flops of the march for one particle (FMA = 2 flops).

    Per wedge term and candidate: value + 2 derivative recurrences (16 flops) and 12
    complex-by-real accumulations (24) for a derivative evaluation; 12 flops for the
    value-only evaluation at the final point.  Per pair and candidate: the two phase
    products, the real / imaginary parts and the 10 weighted sums (~100 flops; 40 for the
    value only)."""
    sched = [x for x in levels if x < L] + [L]
    f = 0
    for Lj in sched:
        f += steps * (40 * wedge_terms(Lj) + 100 * (Lj + 1) ** 2)
    f += 12 * wedge_terms(L) + 40 * (L + 1) ** 2
    return Kc * f


# HBM traffic of k_march, from two rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE) over
# `bench.py --pmc-probe`, scaled by the same counters on a copy of known size.  Only used while
# the kernel's sources are the ones the counters were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_march_L32_R32_B12_K16_hbm_traffic.txt")
MARCH_SOURCES = ["paper_2603_15285_amd/csrc/k_march.hip", "paper_2603_15285_amd/csrc/matcha_dev.hpp"]
LAUNCH_HEADER = "paper_2603_15285_amd/csrc/matcha_launch.hpp"


def march_source_digest():
    """SHA-256 over the march kernel's source, the device header and the MarchArgs block of the
    launch header (the other kernels' argument blocks do not reach the march)."""
    h = hashlib.sha256()
    for rel in MARCH_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, LAUNCH_HEADER)) as fh:
        text = fh.read()
    i = text.index("struct MarchArgs {")
    h.update(text[i:text.index("};", i) + 2].encode())
    return h.hexdigest()


def measured_march_traffic(workload):
    """Bytes per k_march launch, or None when no summary matches this workload and source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("workload") != workload or fields.get("kernel_source_sha256") != march_source_digest():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pmc_probe(args):
    """One device copy of known size (the counters' scale reference), then one pass of the batched
    path on the bench workload with the default launch shapes; prints no JSON line."""
    import torch

    from paper_2603_15285_amd import matcha as M
    from paper_2603_15285_amd import synth as S

    torch.cuda.set_device(0)
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    src.fill_(1.0)  # writes nbytes
    dst = torch.empty_like(src)
    dst.copy_(src)  # reads nbytes, writes nbytes
    torch.cuda.synchronize()
    del src, dst
    print(f"reference: fill then copy of {nbytes} bytes", flush=True)
    wl = S.WORKLOADS[args.workload]
    b = S.make_workload(args.workload, n_particles=args.particles)
    ctx = M.Context(0)
    ctx.prepare(wl.B, wl.n_grid)
    batch = M.Batch.make(b.L, b.R, b.L_h, b.R_h, f_offset=b.f_offset)
    f = torch.from_numpy(b.f_flat.astype(np.complex64).view(np.float32)).cuda()
    h = torch.from_numpy(b.h.astype(np.complex64).view(np.float32).reshape(-1)).cuda()
    w = torch.from_numpy(b.w.astype(np.float32)).cuda()
    if int(b.L.max()) != int(b.L.min()):
        batch.set_lpt_order(wl.levels, wl.steps)
    fp64_above = 40 if int(b.L.max()) > 40 else 0
    best, _, _ = M.align(ctx, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, fp64_above=fp64_above)
    torch.cuda.synchronize()
    print(f"probe pass done: {b.n_particles} particles, march source {march_source_digest()}", flush=True)
    ctx.close()


HBM_PEAK_GBPS = 8000.0
MFMA_FP32_PEAK_TFLOPS = 157.3


def wedge_rows(L):
    """float4 entries of one particle's wedge-layout C up to band L: sum_{l<=L} (l+1)^2."""
    return (L + 1) * (L + 2) * (2 * L + 3) // 6


def assemble_work(L, R):
    """(HBM bytes, useful MFMA flops) of the assembly for one particle: f read (R (L+1)^2 complex64),
    C written (16 bytes per wedge entry); 8 real flops per complex multiply-add over the half plane
    sum_l (l+1)(2l+1) R."""
    byts = R * (L + 1) ** 2 * 8 + wedge_rows(L) * 16
    flops = 8 * R * sum((l + 1) * (2 * l + 1) for l in range(L + 1))
    return byts, flops


def soft_work(B, n):
    """(HBM bytes, useful DFT flops) of the SOFFT search for one particle: the n^3 grid written
    and read back (4 bytes each way), C read up to band B; the two real DFT products per polar node,
    8 (B+1)(2B+1) n for the first stage and 4 (B+1) n^2 for the second."""
    byts = 2 * 4 * n ** 3 + wedge_rows(B) * 16
    flops = n * (8 * (B + 1) * (2 * B + 1) * n + 4 * (B + 1) * n * n)
    return byts, flops


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(b, wl, budget_s=15.0):
    """The FP64 oracle's whole path (built -O3 -march=native on this host) on an evenly spread
    sample of the batch: OpenMP over particles on every available core, and one core on a few
    particles.  Returns (report, sample, oracle best, oracle candidates)."""
    import oracle as O
    O.use_native()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    O.set_num_threads(1)
    n1 = 2
    t0 = time.time()
    O.align_batch(b, wl.B, wl.n_grid, wl.Kc, list(wl.levels), wl.steps, particles=[0, b.n_particles - 1][:n1])
    t1 = (time.time() - t0) / n1
    O.set_num_threads(threads)
    n = int(max(threads, min(b.n_particles, round(budget_s / max(t1, 1e-3) * threads))))
    sample = np.linspace(0, b.n_particles - 1, n).astype(int)
    t0 = time.time()
    ob, obi, ost, ocand = O.align_batch(b, wl.B, wl.n_grid, wl.Kc, list(wl.levels), wl.steps, particles=sample)
    dt = time.time() - t0
    rep = {"value": n / dt, "unit": "particles/s", "cores": threads, "kind": "oracle",
           "single_core": {"value": 1.0 / t1, "unit": "particles/s", "particles": n1},
           "cpu": cpu_model(),
           "sample": f"{n} particles of the same workload spread over the batch, whole path "
                     f"(assembly, SOFFT, march, selection) in FP64, OpenMP over particles, {dt:.1f} s"}
    return rep, sample, ob, ocand


def norm_bound(b, p):
    """S = |f_p|_w |h|_w over the particle's shells and degrees: the Cauchy-Schwarz bound on |C_L|."""
    Lp, Rp = int(b.L[p]), int(b.R[p])
    f = b.f(p)
    hh = b.h[:Rp, : (Lp + 1) ** 2]
    w = b.w[:Rp, None]
    return math.sqrt(float(np.sum(w * np.abs(f) ** 2))) * math.sqrt(float(np.sum(w * np.abs(hh) ** 2)))


def errors_vs_oracle(S_mod, b, sample, ob, ocand, best):
    """Rotation (degrees, geodesic) and objective (|dF| / S) errors of GPU results against the FP64
    oracle on the sampled particles.  Particles whose two best oracle candidates lie within 1e-5 S of
    each other are skipped: either basin is a correct selection."""
    rot, obj = [], []
    skipped = 0
    for t, p in enumerate(sample):
        Sb = norm_bound(b, p)
        top = np.sort(ocand[t, :, 3])[::-1]
        if top.size > 1 and top[0] - top[1] <= 1e-5 * Sb:
            skipped += 1
            continue
        g = best[p].astype(np.float64)
        rot.append(float(S_mod.geodesic_deg(S_mod.euler_zyz_to_matrix(g[0], g[1], g[2]),
                                            S_mod.euler_zyz_to_matrix(ob[t, 0], ob[t, 1], ob[t, 2]))))
        obj.append(abs(g[3] - ob[t, 3]) / Sb)
    rot, obj = np.asarray(rot), np.asarray(obj)
    return {"rot_err_vs_oracle_deg": {"max": float(rot.max()), "p90": float(np.percentile(rot, 90)),
                                      "median": float(np.median(rot))},
            "obj_err_vs_oracle_rel_S": {"max": float(obj.max()), "p90": float(np.percentile(obj, 90))},
            "compared": int(rot.size), "near_ties_skipped": skipped}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="L32_R32_B12_K16")
    ap.add_argument("--particles", type=int, default=None)
    ap.add_argument("--plain", type=int, default=32, help="particles timed on the one-particle path")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run the counter probe (reference copy + one pass) instead of the benchmark")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); particles shard across GPUs "
              "with no exchange in the forward path, so run one process per GPU.", file=sys.stderr)
        sys.exit(2)
    if args.pmc_probe:
        pmc_probe(args)
        return

    import torch

    from paper_2603_15285_amd import matcha as M
    from paper_2603_15285_amd import synth as S

    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    wl = S.WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    t0 = time.time()
    b = S.make_workload(args.workload, n_particles=args.particles)
    log(f"generated {b.n_particles} particles in {time.time() - t0:.1f} s")
    P = b.n_particles
    ctx = M.Context(0)
    ctx.prepare(wl.B, wl.n_grid)
    batch = M.Batch.make(b.L, b.R, b.L_h, b.R_h, f_offset=b.f_offset)
    f = torch.from_numpy(b.f_flat.astype(np.complex64).view(np.float32)).cuda()
    h = torch.from_numpy(b.h.astype(np.complex64).view(np.float32).reshape(-1)).cuda()
    w = torch.from_numpy(b.w.astype(np.float32)).cuda()
    stream = torch.cuda.current_stream()
    if int(b.L.max()) != int(b.L.min()):
        batch.set_lpt_order(wl.levels, wl.steps)
    fp64_above = 40 if int(b.L.max()) > 40 else 0

    # tune the launch shapes on this batch, then capture the whole path in a HIP graph
    C0 = M.coeff_assemble(ctx, batch, f, h, w)
    tuning = M.autotune(ctx, batch, C0, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, reps=1, fp64_above=fp64_above)
    del C0
    log(f"tuning: {tuning}")
    graph = M.AlignGraph(ctx, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, fp64_above=fp64_above)
    bufs = graph.bufs

    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()
    log("warmup done")
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for k in range(args.steps):
        graph.launch()
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    value = P / (ms_step / 1e3)

    # each stage alone, timed with events on the stream its kernels run on
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for k in range(args.steps):
        ev[k][0].record(stream)
        M.coeff_assemble(ctx, batch, f, h, w, C=bufs["C"])
        ev[k][1].record(stream)
        M.soft_search(ctx, batch, bufs["C"], wl.B, wl.n_grid, wl.Kc, cand=bufs["cand"], status=bufs["status"])
        ev[k][2].record(stream)
        M.march_newton(ctx, batch, bufs["C"], wl.levels, wl.steps, bufs["cand"], bufs["status"], best=bufs["best"],
                       best_idx=bufs["best_idx"], fp64_above=fp64_above)
        ev[k][3].record(stream)
    torch.cuda.synchronize()
    ms_asm = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    ms_soft = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    ms_march = float(np.mean([e[2].elapsed_time(e[3]) for e in ev]))
    log(f"batched: {ms_step:.3f} ms/step (assembly {ms_asm:.3f}, search {ms_soft:.3f}, march {ms_march:.3f} ms), "
        f"{value:.0f} particles/s")

    best = bufs["best"].cpu().numpy().astype(np.float64)
    err = S.geodesic_deg(b.R_true(), S.euler_zyz_to_matrix(best[:, 0], best[:, 1], best[:, 2]))

    # plain path: one particle per call sequence, same kernels, no graph
    n_plain = min(args.plain, P)
    singles = []
    for p in range(n_plain):
        sb = M.Batch.make(b.L[p:p + 1], b.R[p:p + 1], b.L_h, b.R_h, f_offset=[0])
        o, sz = int(b.f_offset[p]), int(b.R[p]) * (int(b.L[p]) + 1) ** 2
        singles.append((sb, f[2 * o: 2 * (o + sz)], {}))
    plain_tuning = ctx.get_tuning()
    ctx.set_tuning(0, 0)  # the one-particle path runs the library's default launch shapes

    def plain_one(sb, fp, bb):
        M.align(ctx, sb, fp, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, fp64_above=fp64_above, bufs=bb)

    for sb, fp, bb in singles[:2]:
        plain_one(sb, fp, bb)
    torch.cuda.synchronize()
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    for sb, fp, bb in singles:
        plain_one(sb, fp, bb)
    p1.record(stream)
    torch.cuda.synchronize()
    plain_value = n_plain / (p0.elapsed_time(p1) / 1e3)
    log(f"plain: {plain_value:.0f} particles/s over {n_plain} particles")
    ctx.set_tuning(plain_tuning["march_nc"], plain_tuning["soft_threads"])

    # batched with BF16 coefficients on the matrix cores (FP32 accumulation) for the search and the
    # lower levels, and each particle's final level on FP32-assembled coefficients (FP32 march)
    f16 = f.to(torch.bfloat16)
    h16 = h.to(torch.bfloat16)

    def time_graph(g):
        g.launch()
        torch.cuda.synchronize()
        q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        q0.record(stream)
        for k in range(args.steps):
            g.launch()
        q1.record(stream)
        torch.cuda.synchronize()
        return P / (q0.elapsed_time(q1) / args.steps / 1e3), g.bufs["best"].cpu().numpy().astype(np.float64)

    g16 = M.AlignGraph(ctx, batch, f16, h16, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, prec=M.BF16_FP32ACC,
                       fp64_above=fp64_above, f32=f, h32=h)
    bf16_value, b16 = time_graph(g16)
    g16.close()
    del g16
    g16o = M.AlignGraph(ctx, batch, f16, h16, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, prec=M.BF16_FP32ACC,
                        fp64_above=fp64_above)
    bf16o_value, b16o = time_graph(g16o)
    g16o.close()
    del g16o
    err16 = S.geodesic_deg(b.R_true(), S.euler_zyz_to_matrix(b16[:, 0], b16[:, 1], b16[:, 2]))
    d16 = S.geodesic_deg(S.euler_zyz_to_matrix(best[:, 0], best[:, 1], best[:, 2]),
                         S.euler_zyz_to_matrix(b16[:, 0], b16[:, 1], b16[:, 2]))
    log(f"batched bf16 (FP32 final level): {bf16_value:.0f} particles/s; BF16 throughout: {bf16o_value:.0f}")

    flops = sum(march_flops_per_particle(wl.levels, int(Lp), wl.steps, wl.Kc) for Lp in b.L)
    traffic = measured_march_traffic(wl.name) if args.particles is None else None
    a_b, a_f = np.sum([assemble_work(int(Lp), int(Rp)) for Lp, Rp in zip(b.L, b.R)], axis=0)
    s_b, s_f = soft_work(wl.B, wl.n_grid)
    s_b, s_f = s_b * P, s_f * P
    stages = {
        "assemble": {"kernel": "k_assemble_f32", "ms": ms_asm,
                     "hbm_GBps": a_b / (ms_asm / 1e3) / 1e9, "hbm_frac": a_b / (ms_asm / 1e3) / 1e9 / HBM_PEAK_GBPS,
                     "mfma_TFLOPs": a_f / (ms_asm / 1e3) / 1e12,
                     "mfma_frac": a_f / (ms_asm / 1e3) / 1e12 / MFMA_FP32_PEAK_TFLOPS},
        "soft_search": {"kernels": ("k_soft_wigner + k_soft_grid_reg (or k_soft_grid) + k_soft_maxima_q "
                                    "(or k_soft_maxima) + k_soft_rank"), "ms": ms_soft,
                        "hbm_GBps": s_b / (ms_soft / 1e3) / 1e9,
                        "hbm_frac": s_b / (ms_soft / 1e3) / 1e9 / HBM_PEAK_GBPS,
                        "mfma_TFLOPs": s_f / (ms_soft / 1e3) / 1e12,
                        "mfma_frac": s_f / (ms_soft / 1e3) / 1e12 / MFMA_FP32_PEAK_TFLOPS},
        "march": {"kernel": "k_march", "ms": ms_march, "valu_TFLOPs": flops / (ms_march / 1e3) / 1e12,
                  "valu_frac": flops / (ms_march / 1e3) / 1e12 / VALU_FP32_PEAK_TFLOPS},
    }
    achieved = flops / (ms_march / 1e3) / 1e12
    out = {
        "metric": METRIC, "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "particles": P, "L": int(b.L.max()), "shells": int(b.R.max()),
                   "B": wl.B, "n_grid": wl.n_grid, "Kc": wl.Kc, "levels": list(wl.levels),
                   "newton_steps_per_level": wl.steps, "snr": list(wl.snr) if isinstance(wl.snr, tuple) else wl.snr},
        "roofline": {"kernel": "k_march (frequency march: value, gradient, Hessian, Newton, selection)",
                     "bound": "alu", "achieved": achieved, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / VALU_FP32_PEAK_TFLOPS, "traffic": traffic, "traffic_unit": "bytes/launch",
                     "ms_per_launch": ms_march,
                     "peak_without_packed_fp32": VALU_FP32_NONPACKED_TFLOPS,
                     "frac_without_packed_fp32": achieved / VALU_FP32_NONPACKED_TFLOPS},
        "plain": {"value": plain_value, "unit": "particles/s", "particles": n_plain},
        "batched_over_plain": value / plain_value,
        "batched_bf16": {"value": bf16_value, "unit": "particles/s", "over_plain": bf16_value / plain_value,
                         "scheme": ("BF16 f, h on the matrix cores (FP32 accumulation) for the search and the lower "
                                    "levels; FP32 assembly for each particle's final level; FP32 march"),
                         "rot_diff_vs_fp32_deg": {"median": float(np.median(d16)), "p99": float(np.percentile(d16, 99)),
                                                  "n_over_0.05": int(np.sum(d16 > 0.05))},
                         "rot_err_vs_truth_deg": {"median": float(np.median(err16)), "p90": float(np.percentile(err16, 90))}},
        "stages": stages,
        "tuning": tuning,
        "rot_err_vs_truth_deg": {"median": float(np.median(err)), "p90": float(np.percentile(err, 90)),
                                 "max": float(err.max())},
    }
    out["batched_bf16"]["without_fp32_final_level"] = {"value": bf16o_value, "unit": "particles/s"}
    if not args.no_cpu:
        log("cpu baseline ...")
        rep, sample, ob, ocand = cpu_baseline(b, wl)
        out["cpu_baseline"] = rep
        # the GPU's selected rotations against the FP64 oracle on the particles the oracle ran
        out["vs_oracle"] = {"fp32": errors_vs_oracle(S, b, sample, ob, ocand, best),
                            "bf16": errors_vs_oracle(S, b, sample, ob, ocand, b16),
                            "bf16_without_fp32_final_level": errors_vs_oracle(S, b, sample, ob, ocand, b16o)}
        out["rot_err_vs_oracle_deg"] = {k: v["rot_err_vs_oracle_deg"] for k, v in out["vs_oracle"].items()}
        log(f"vs oracle: {json.dumps(out['rot_err_vs_oracle_deg'])}")
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
