"""Accuracy report: the batched path (FP32; BF16 assembly with the final level on FP32 coefficients;
BF16 throughout) against the FP64 oracle on evenly spaced sampled particles of three workloads,
and the adjoint's time and error.  Needs a GPU:

    python tests/accuracy_report.py

Particles whose two best oracle candidates lie within 1e-5 S of each other are skipped (either
basin is a correct selection); S = |f|_w |h|_w bounds |C_L|.  Not collected by pytest."""
import sys, os, time, math, numpy as np, torch
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))  # the repository
sys.path.insert(0, ROOT)
from paper_2603_15285_amd import matcha as M, synth as S
import oracle as O

def upload(b):
    batch = M.Batch.make(b.L, b.R, b.L_h, b.R_h, f_offset=b.f_offset)
    f = torch.from_numpy(b.f_flat.astype(np.complex64).view(np.float32).copy()).cuda()
    h = torch.from_numpy(b.h.astype(np.complex64).view(np.float32).reshape(-1).copy()).cuda()
    w = torch.from_numpy(b.w.astype(np.float32)).cuda()
    return batch, f, h, w

def scale(b, p, L):
    f = b.f(p)[:, : (L + 1) ** 2]
    R = f.shape[0]
    w = b.w[:R, None]
    return math.sqrt(np.sum(w * np.abs(f) ** 2)) * math.sqrt(np.sum(w * np.abs(b.h[:R, : (L + 1) ** 2]) ** 2))

def rot(e):
    return S.euler_zyz_to_matrix(e[..., 0], e[..., 1], e[..., 2])

ctx = M.Context(0)
for name, npart, nsamp in [("L32_R32_B12_K16", 4096, 64), ("uneven_L24to48", 1024, 48), ("L64_R64_B16_K32", 128, 16)]:
    wl = S.WORKLOADS[name]
    t0 = time.time()
    b = S.make_workload(name, n_particles=npart)
    batch, f, h, w = upload(b)
    fp64 = 40 if int(b.L.max()) > 40 else 0
    res = {}
    f16, h16 = f.to(torch.bfloat16), h.to(torch.bfloat16)
    for tag, ff, hh, prec, fin in [("fp32", f, h, M.FP32, False), ("bf16", f16, h16, M.BF16_FP32ACC, True),
                                   ("bf16 throughout", f16, h16, M.BF16_FP32ACC, False)]:
        kw = dict(f32=f, h32=h) if fin else {}
        best, bi, st = M.align(ctx, batch, ff, hh, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps, prec=prec,
                               fp64_above=fp64, **kw)
        res[tag] = best.cpu().numpy().astype(np.float64)
    sample = np.linspace(0, npart - 1, nsamp).astype(int)
    ob, obi, ost, ocand = O.align_batch(b, wl.B, wl.n_grid, wl.Kc, list(wl.levels), wl.steps, particles=sample)
    for tag in res:
        e_rot, e_obj, ties = [], [], 0
        for t, p in enumerate(sample):
            Sc = scale(b, p, int(b.L[p]))
            top = np.sort(ocand[t, :, 3])[::-1]
            if top[0] - top[1] <= 1e-5 * Sc:
                ties += 1
                continue
            e_rot.append(float(S.geodesic_deg(rot(res[tag][p, :3]), rot(ob[t, :3]))))
            e_obj.append(abs(res[tag][p, 3] - ob[t, 3]) / Sc)
        e_rot, e_obj = np.array(e_rot), np.array(e_obj)
        print(f"{name} {tag}: {len(e_rot)} of {nsamp} sampled particles (skipped {ties} near-ties): rotation error vs FP64 oracle "
              f"max {e_rot.max():.2e} deg, p90 {np.percentile(e_rot, 90):.2e} deg; objective |dF|/S max {e_obj.max():.2e}, "
              f"p90 {np.percentile(e_obj, 90):.2e}  ({time.time()-t0:.0f} s)", flush=True)
    del f, h, batch, b
    torch.cuda.empty_cache()

# adjoint (c4): gradient of sum_p g_p C_L(R_p*) at the aligned rotations, 1024 particles at L = R = 32
wl = S.WORKLOADS["adjoint_L32"]
b = S.make_workload("adjoint_L32", n_particles=1024)
batch, f, h, w = upload(b)
best, _, _ = M.align(ctx, batch, f, h, w, wl.B, wl.n_grid, wl.Kc, wl.levels, wl.steps)
g = torch.ones(1024, dtype=torch.float32, device="cuda")
gh, gf = M.grad_template(ctx, batch, f, h, w, best, g)
torch.cuda.synchronize()
e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
e0.record()
for _ in range(5):
    M.grad_template(ctx, batch, f, h, w, best, g)
e1.record(); torch.cuda.synchronize()
ms = e0.elapsed_time(e1) / 5
bn = best.cpu().numpy().astype(np.float64)
gfn = gf.cpu().numpy().view(np.complex64)
rel = []
for p in (0, 511, 1023):
    _, gfo = O.grad_one(int(b.L[p]), int(b.R[p]), b.f(p), b.h, b.L_h, b.w, bn[p, :3], 1.0)
    o = int(b.f_offset[p])
    x = gfn[o: o + gfo.size].reshape(gfo.shape)
    rel.append(np.abs(x - gfo).max() / np.abs(gfo).max())
gm = torch.zeros(1024, dtype=torch.float32, device="cuda")
gm[:64] = 1.0  # template gradient over the first 64 particles, against the oracle
gh64, _ = M.grad_template(ctx, batch, f, h, w, best, gm, want_f=False)
ghn = gh64.cpu().numpy().view(np.complex64).reshape(b.h.shape)
gho = np.zeros_like(b.h, dtype=np.complex128)
for p in range(64):
    O.grad_one(int(b.L[p]), int(b.R[p]), b.f(p), b.h, b.L_h, b.w, bn[p, :3], 1.0, grad_h=gho, want_f=False)
relh = np.abs(ghn - gho).max() / np.abs(gho).max()
print(f"adjoint_L32: grad_template {ms:.3f} ms for 1024 particles ({1024/ms*1e3:.0f} particles/s); grad_f rel err vs FP64 oracle "
      f"max {max(rel):.2e} (3 particles), grad_h rel err {relh:.2e} (sum over 64 particles)", flush=True)
