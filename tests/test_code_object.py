"""Properties of the gfx950 code in the built libmatcha.so, read from its own disassembly (CPU only).

* Every kernel addresses LDS scratch with LDS instructions: no flat loads / stores / atomics, whose
  generic addresses are checked against the apertures (a base formed as pointer - offset can
  leave the shared aperture).
* No kernel calls a function (every device function is inlined).
* No kernel writes through the scalar data cache: scalar stores, scalar atomics and the scalar
  cache write-back / discard never appear.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_15285_amd", "libmatcha.so")
LLVM = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
KERNELS = {"k_assemble_f32", "k_assemble_bf16", "k_soft_grid", "k_soft_maxima", "k_soft_rank", "k_march",
           "k_evaluate", "k_grad_particle", "k_grad_reduce", "k_ball_sym", "k_ball_gemm", "k_ball_scatter", "k_ball_scatter_vol", "k_lowrank_sv",
           "k_rotate_volume", "k_phase_shift", "k_cross_spectrum", "k_corr_peak", "k_upsample_tables", "k_upsample_xy", "k_upsample_z"}


def _disassembly(tmp_path):
    for tool in ("clang-offload-bundler", "llvm-objdump"):
        if not os.path.exists(os.path.join(LLVM, tool)):
            pytest.skip(f"{tool} not available")
    if shutil.which("objcopy") is None:
        pytest.skip("objcopy not available")
    if not os.path.exists(LIB):
        pytest.skip("libmatcha.so not built")
    fat = tmp_path / "fatbin.bin"
    subprocess.run(["objcopy", "--dump-section", f".hip_fatbin={fat}", LIB, str(tmp_path / "lib.copy")], check=True,
                   capture_output=True)
    data = fat.read_bytes()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)] + [len(data)]
    text = []
    for k in range(len(starts) - 1):
        part = tmp_path / f"bundle{k}.bin"
        part.write_bytes(data[starts[k]:starts[k + 1]])
        co = tmp_path / f"code{k}.o"
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o", f"--input={part}",
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"], check=True, capture_output=True)
        text.append(subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", str(co)], check=True,
                                   capture_output=True, text=True).stdout)
    return "\n".join(text)


def _functions(dis):
    """{mangled kernel name: [instruction mnemonics]}"""
    out, cur = {}, None
    for line in dis.split("\n"):
        m = re.match(r"^[0-9a-f]+ <(\S+)>:", line)
        if m:
            cur = m.group(1)
            out[cur] = []
            continue
        if cur is not None:
            m = re.match(r"^\s+([a-z][a-z0-9_]+)\b", line)
            if m:
                out[cur].append(m.group(1))
    return out


def test_code_object_rules(tmp_path):
    fns = _functions(_disassembly(tmp_path))
    names = {re.sub(r"^_ZN6matcha\d+", "", k) for k in fns}
    for kname in KERNELS:
        assert any(n.startswith(kname) for n in names), (kname, sorted(names))
    for fn, ops in fns.items():
        assert ops, fn
        flat = [o for o in ops if o.startswith(("flat_load", "flat_store", "flat_atomic"))]
        assert not flat, (fn, flat[:4])
        calls = [o for o in ops if o in ("s_swappc_b64", "s_call_b64")]
        assert not calls, fn
        scalar_writes = [o for o in ops if o.startswith(("s_store", "s_buffer_store", "s_atomic", "s_buffer_atomic",
                                                         "s_scratch_store", "s_dcache_wb", "s_dcache_discard"))]
        assert not scalar_writes, (fn, scalar_writes[:4])
