"""Build-level checks that need no GPU: every HIP kernel the host side
registers exists under the same (mangled) name in the gfx950 code object.
A mismatch (for example a parameter type that differs between the host and
device compilation passes) leaves a kernel the runtime cannot launch."""
import glob
import os
import re
import subprocess
import tempfile

import pytest

from paper_1308_0653_amd import build as B


@pytest.mark.parametrize("src", sorted(glob.glob(os.path.join(B.CSRC, "*.hip"))))
def test_host_and_device_kernel_names_match(src):
    with tempfile.TemporaryDirectory() as tmp:
        cmd = [B.HIPCC, *[f for f in B.FLAGS if f != "-shared"], f"-I{B.INCLUDE}", f"-I{B.CSRC}", "-c", src,
               "-o", os.path.join(tmp, "k.o"), "--save-temps"]
        subprocess.run(cmd, cwd=tmp, check=True, capture_output=True)
        host = glob.glob(os.path.join(tmp, "*host-x86_64*.s"))
        dev = glob.glob(os.path.join(tmp, "*amdgcn-amd-amdhsa-gfx950.s"))
        assert host and dev
        pat = re.compile(r"_ZN4pdbm[A-Za-z0-9_]*\bk_[A-Za-z0-9_]*|_ZN4pdbm12_GLOBAL__N_1[0-9]+k_[A-Za-z0-9_]+")
        htxt = open(host[0]).read()
        dtxt = open(dev[0]).read()
        dev_names = set(re.findall(r"^(_ZN4pdbm[A-Za-z0-9_]+):", dtxt, flags=re.M))
        dev_kernels = {n for n in dev_names if re.search(r"k_[a-z]", n)}
        host_kernels = {n for n in pat.findall(htxt) if n.startswith("_ZN4pdbm")}
        if not dev_kernels:
            pytest.skip("no kernels in this source")
        assert host_kernels == dev_kernels, (host_kernels ^ dev_kernels)


STEP_SOURCES = ("pdbm_step.hip", "pdbm_step2.hip")  # k_step and k_step2


def _step_kernels_asm() -> str:
    """gfx950 assembly of the sources holding the step kernels."""
    out = []
    with tempfile.TemporaryDirectory() as tmp:
        for name in STEP_SOURCES:
            dst = os.path.join(tmp, name + ".s")
            cmd = [B.HIPCC, *[f for f in B.FLAGS if f not in ("-shared", "-fPIC")], f"-I{B.INCLUDE}", f"-I{B.CSRC}",
                   "--cuda-device-only", "-S", os.path.join(B.CSRC, name), "-o", dst]
            subprocess.run(cmd, cwd=tmp, check=True, capture_output=True)
            out.append(open(dst).read())
    return "\n".join(out)


def _kernel_bodies(asm: str, key: str):
    for name in re.findall(r"^(_Z\S*" + key + r"\S*):", asm, flags=re.M):
        i = asm.index(name + ":")
        yield name, asm[i:asm.index(".Lfunc_end", i)].split("\n")


SREG = r"s\[\d+:\d+\]"


def _narrowing(t, regions):
    """Applies one instruction to the open exec-narrowing regions (a tuple
    of frozensets, each the registers holding one region's saved mask).  A
    region opens with s_and_saveexec_b64 sX and closes with s_or_b64 exec,
    exec, sY where sY holds the saved mask; the mask may move on the way
    (s_xor_b64 sA, exec, sX before an else-arm, s_or_saveexec_b64 /
    s_andn2_saveexec_b64 sA, sX, s_mov_b64)."""
    m = re.match(r"s_and_saveexec_b64\s+(" + SREG + ")", t)
    if m:
        return regions + (frozenset({m.group(1)}),)
    m = re.match(r"s_(?:xor_b64|mov_b64|or_saveexec_b64|andn2_saveexec_b64)\s+(" + SREG + r"),\s*(?:exec,\s*)?("
                 + SREG + ")", t)
    if m:
        return tuple(r | {m.group(1)} if m.group(2) in r else r for r in regions)
    m = re.match(r"s_or_b64\s+exec,\s*exec,\s*(" + SREG + ")", t)
    if m:
        return tuple(r for r in regions if m.group(1) not in r)
    return regions


def _dpp_under_narrowed_exec(lines):
    """Counts the DPP instructions that some path reaches with an exec-
    narrowing region open: the regions are followed along the control flow
    graph of the kernel's basic blocks (labels, branches, fall-through), not
    the text order, since the compiler lays blocks out out of order."""
    blocks, cur = [], []
    label_of = {}
    for line in lines:
        t = line.split(";")[0].strip()
        if not t or t.startswith("."):
            m = re.match(r"^(\.LBB\S+):", t)
            if m:
                if cur:
                    blocks.append(cur)
                cur = []
                label_of[m.group(1)] = len(blocks)
            continue
        if t.endswith(":"):
            continue
        cur.append(t)
        if re.match(r"s_(cbranch_\w+|branch|endpgm|setpc_b64)\b", t):
            blocks.append(cur)
            cur = []
    if cur:
        blocks.append(cur)
    # label_of maps a label to the index of the block that starts at it
    succ = []
    for i, blk in enumerate(blocks):
        last = blk[-1] if blk else ""
        m = re.match(r"s_(cbranch_\w+|branch)\s+(\.LBB\S+)", last)
        out = []
        if m:
            out.append(label_of[m.group(2)])
            if m.group(1) != "branch" and i + 1 < len(blocks):
                out.append(i + 1)
        elif not re.match(r"s_(endpgm|setpc_b64)\b", last) and i + 1 < len(blocks):
            out.append(i + 1)
        succ.append(out)
    entry = [set() for _ in blocks]
    entry[0].add(())
    work = [0]
    while work:
        i = work.pop()
        for state in list(entry[i]):
            for t in blocks[i]:
                state = _narrowing(t, state)
            for j in succ[i]:
                if state not in entry[j]:
                    entry[j].add(state)
                    work.append(j)
    flagged = 0
    for i, blk in enumerate(blocks):
        for state in entry[i]:
            for t in blk:
                state = _narrowing(t, state)
                if re.search(r"\b(wave_sh[lr]|row_|quad_perm)", t) and state:
                    flagged += 1
    return flagged


def test_step_kernel_takes_lane_shifts_with_every_lane_active():
    """The step kernel's azimuthal neighbours come from DPP whole-wave lane
    shifts.  A shift executed while some lanes are switched off (inside a
    divergent branch) reads 0 from those lanes, silently corrupting their
    neighbours' update; the source takes every shift unconditionally and
    selects afterwards.  The same holds for the other cross-lane DPP moves
    (the lane permutations of the two-step kernel's edge cells, the
    wavefront sums of the drift records).  Checked on the gfx950 assembly:
    no path through k_step or k_step2 reaches a DPP instruction between an
    exec-narrowing instruction and the matching restore."""
    asm = _step_kernels_asm()
    bodies = list(_kernel_bodies(asm, "k_step"))
    # k_step and k_step2: 2 precisions x (full annulus, rotated sector) x (tau of the solve, per-cell tau)
    assert len(bodies) == 16
    for name, lines in bodies:
        shifts = sum(("wave_shr:1" in t or "wave_shl:1" in t) for t in lines)
        dpp = sum(bool(re.search(r"\b(wave_sh[lr]|row_|quad_perm)", t)) for t in lines)
        assert shifts >= 66, (name, shifts)
        assert dpp >= shifts, (name, dpp)
        assert _dpp_under_narrowed_exec(lines) == 0, name
    # the multi-step single-column kernel: 2 precisions x the two kinds of tau
    columns = list(_kernel_bodies(asm, "k_column"))
    assert len(columns) == 4
    for name, lines in columns:
        assert sum(("wave_shr:1" in t or "wave_shl:1" in t) for t in lines) >= 66, name
        assert _dpp_under_narrowed_exec(lines) == 0, name


def test_narrowed_exec_check_finds_a_dpp_inside_a_branch():
    """The checker itself: a DPP move inside an s_and_saveexec region is
    flagged, on the path that enters the region; one reached only around the
    region (a uniform branch over it, a block laid out after it) is not."""
    inside = ["s_and_saveexec_b64 s[2:3], vcc", "s_cbranch_execz .LBB0_2", ".LBB0_1:",
              "v_mov_b32_dpp v1, v2 wave_shr:1 row_mask:0xf bank_mask:0xf", ".LBB0_2:",
              "s_or_b64 exec, exec, s[2:3]", "s_endpgm"]
    assert _dpp_under_narrowed_exec(inside) == 1
    around = ["s_cbranch_vccz .LBB0_3", "s_and_saveexec_b64 s[2:3], vcc", "s_cbranch_execnz .LBB0_1",
              "s_branch .LBB0_2", ".LBB0_3:", "v_mov_b32_dpp v1, v2 row_bcast:15 row_mask:0xa bank_mask:0xf",
              "s_endpgm", ".LBB0_1:", "v_add_f32_e32 v1, v1, v1", ".LBB0_2:", "s_or_b64 exec, exec, s[2:3]",
              "s_endpgm"]
    assert _dpp_under_narrowed_exec(around) == 0


def test_step_kernel_uses_no_scratch_memory():
    """Register spills of the step kernels must stay in registers (AGPRs): a
    spill to scratch memory inside the row loop adds memory round trips to
    every row.  Checked on the code-object metadata of every variant of the
    one-step, the two-step and the single-column kernel."""
    asm = _step_kernels_asm()
    seen = 0
    for block in asm.split("- .agpr_count:")[1:]:
        name = re.search(r"\.name:\s+(\S+)", block).group(1)
        if "k_step" not in name and "k_column" not in name:
            continue
        seen += 1
        assert int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", block).group(1)) == 0, name
    assert seen == 20
