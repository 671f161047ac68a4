"""Properties of the compiled kernels that the tests on the GPU cannot see (CPU, no GPU).

The FP32 Poisson passes run their sine transforms on the matrix cores and are compiled for
high occupancy: the listing must hold the FP16 matrix instructions and no scratch spills for
the boxes up to 64^3, forward and reverse, at every finite-difference order.  The particle step stages windows into LDS with direct-to-LDS loads: a
wave must wait for them before the barrier after which other waves read the staged words.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2003_04925_amd", "csrc")


def _compile(tmp_path, source):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path / (source + ".s")
    cmd = [hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only", "-S",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(CSRC, source),
           "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


def kernel_bodies(asm_text, pattern):
    """{mangled name: body text} of the kernels whose names match `pattern`."""
    out = {}
    for m in re.finditer(r"^(_Z\w+):[^\n]*\n(.*?)^\.Lfunc_end", asm_text, re.M | re.S):
        if re.search(pattern, m.group(1)):
            out[m.group(1)] = m.group(2)
    return out


def kernel_meta(asm_text, name):
    """The code-object metadata entry (.name, .private_segment_fixed_size, .vgpr_count, ...)
    of one kernel: the kernel list's entries start at two spaces of indentation."""
    pos = asm_text.index(".name:           " + name + "\n")
    start = asm_text.rfind("\n  - ", 0, pos)
    end = asm_text.find("\n  - ", pos)
    return asm_text[start:end if end > 0 else len(asm_text)]


def test_fp32_poisson_passes_use_the_matrix_cores_without_spills(tmp_path):
    asm = _compile(tmp_path, "kernels_poisson.hip")
    # FP32 passes of boxes of 16, 32, 48 and 64 nodes (R = 1..4): P1 and P3 of the forward
    # solve at orders 2, 4, 6 and of the reverse solve (order 2), and P2
    bodies = kernel_bodies(asm, r"k_poisson_p([13]IfLi[1-4]ELb[01]ELi[123]E|2IfLi[1-4]E)")
    names = sorted(bodies)
    assert len(names) == 2 * 4 * 4 + 4, names
    for n in names:
        assert "v_mfma_f32_16x16x32_f16" in bodies[n], n
        meta = kernel_meta(asm, n)
        spill = re.search(r"\.private_segment_fixed_size:\s+(\d+)", meta)
        assert spill and int(spill.group(1)) == 0, (n, spill.group(0) if spill else None)
    # the FP64 passes keep the FFT (no matrix instructions)
    for n, body in kernel_bodies(asm, r"k_poisson_p[123]IdLi4E").items():
        assert "v_mfma" not in body, n


def is_lds_dma(t):
    """A load that writes LDS directly: global_load_lds_* or a buffer load with the lds bit."""
    return t.startswith("global_load_lds") or (t.startswith("buffer_load") and
                                               re.search(r"\blds\b", t) is not None)


def lds_dma_waits(asm_text):
    """(number of direct-to-LDS loads, list of problems): after each direct-to-LDS load, the
    next s_barrier must be preceded by an s_waitcnt that waits for every vector memory
    operation (vmcnt(0)), so that other waves read the staged words only once they landed."""
    lines = [l.strip() for l in asm_text.split("\n")]
    loads, problems = 0, []
    for i, t in enumerate(lines):
        if not is_lds_dma(t):
            continue
        loads += 1
        waited = False
        for u in lines[i + 1:]:
            if u.startswith("s_waitcnt") and re.search(r"vmcnt\(0\)", u):
                waited = True
            if is_lds_dma(u):
                waited = False
            if u.startswith("s_barrier"):
                if not waited:
                    problems.append((i, t))
                break
            if u.startswith("s_endpgm"):
                break
    return loads, problems


def test_lds_dma_scan_flags_a_missing_wait():
    bad = "\tglobal_load_lds_dword v1, s[0:1]\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier"
    assert lds_dma_waits(bad)[1]
    ok = "\tglobal_load_lds_dword v1, s[0:1]\n\ts_waitcnt vmcnt(0)\n\ts_barrier"
    assert lds_dma_waits(ok) == (1, [])
    bad = "\tbuffer_load_dword v0, s[0:3], s4 offen lds\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier"
    assert lds_dma_waits(bad)[1]
    ok = "\tbuffer_load_dword v0, s[0:3], s4 offen lds\n\ts_waitcnt vmcnt(0)\n\ts_barrier"
    assert lds_dma_waits(ok) == (1, [])
    assert lds_dma_waits("\tbuffer_load_dword v0, s[0:3], s4 offen\n\ts_barrier") == (0, [])


def test_particle_direct_lds_staging_waits_before_barrier(tmp_path):
    loads, problems = lds_dma_waits(_compile(tmp_path, "kernels_particles.hip"))
    assert loads > 0
    assert not problems, problems[:5]
