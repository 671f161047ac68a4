"""Wait states around the hand-placed DPP multiply-adds of the FFT stages (CPU, no GPU).

The Poisson passes fold each radix-2 stage's cross-lane move into the multiply-add with
inline assembly that begins with two wait states, which covers a DPP read of a VGPR written
by the previous VALU instruction.  The other DPP hazard, a VALU write of EXEC, needs five;
the compiler's hazard recognizer does not look inside inline assembly, so this test compiles
the Poisson kernels for gfx950 and requires that no EXEC-writing VALU instruction and no
branch target lies among the four instructions before any of those blocks.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2003_04925_amd", "csrc")


def _is_instruction(line):
    t = line.strip()
    return bool(t) and not t.startswith((";", ".")) and not t.endswith(":")


def dpp_hazards(asm_text, mnemonic="v_fmac_f32_dpp", window=4):
    """(number of inline DPP multiply-adds, list of problems) for an assembly listing."""
    lines = asm_text.split("\n")
    problems, count = [], 0
    for i, line in enumerate(lines):
        if mnemonic not in line:
            continue
        count += 1
        before, j = [], i - 1
        while j >= 0 and len(before) < window + 1:
            t = lines[j].strip()
            if re.match(r"^[\w.$]+:", t):
                before.append("label " + t)
                break
            if _is_instruction(lines[j]):
                before.append(t)
            j -= 1
        # before[0] is the block's own s_nop; the next `window` entries precede the block
        assert before and before[0].startswith("s_nop"), before[:2]
        for t in before[1:window + 1]:
            if t.startswith("label") or t.startswith("v_cmpx") or re.search(r"\bexec\b", t):
                problems.append((i, t))
    return count, problems


def test_scan_flags_an_exec_write_and_a_label():
    bad = "\n".join(["\tv_cmpx_eq_u32_e32 0, v1", "\ts_nop 1",
                     "\tv_fmac_f32_dpp v4, v4, v3 row_mirror row_mask:0xf bank_mask:0xf"])
    assert dpp_hazards(bad)[1]
    lab = "\n".join([".LBB0_3:", "\tv_add_f32_e32 v1, v2, v3", "\ts_nop 1",
                     "\tv_fmac_f32_dpp v4, v4, v3 row_mirror row_mask:0xf bank_mask:0xf"])
    assert dpp_hazards(lab)[1]
    ok = "\n".join(["\tv_add_f32_e32 v1, v2, v3", "\tv_mul_f32_e32 v5, v2, v3",
                    "\tv_mul_f32_e32 v6, v2, v3", "\tv_mul_f32_e32 v7, v2, v3",
                    "\tv_mul_f32_e32 v8, v2, v3", "\ts_nop 1",
                    "\tv_fmac_f32_dpp v4, v4, v3 row_mirror row_mask:0xf bank_mask:0xf"])
    assert dpp_hazards(ok) == (1, [])


def test_poisson_dpp_blocks_have_no_exec_hazard(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path / "poisson.s"
    cmd = [hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only", "-S",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "kernels_poisson.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    count, problems = dpp_hazards(out.read_text())
    assert count > 0
    assert not problems, problems[:5]


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
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path / "particles.s"
    cmd = [hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only", "-S",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "kernels_particles.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    loads, problems = lds_dma_waits(out.read_text())
    assert loads > 0
    assert not problems, problems[:5]
