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


def test_step_kernel_takes_lane_shifts_with_every_lane_active():
    """The step kernel's azimuthal neighbours come from DPP whole-wave lane
    shifts.  A shift executed while some lanes are switched off (inside a
    divergent branch) reads 0 from those lanes, silently corrupting their
    neighbours' update; the source takes every shift unconditionally and
    selects afterwards.  The same holds for the other cross-lane DPP moves
    (the lane-pair swap of the two-step kernel's edge cells).  Checked on the
    gfx950 assembly: no
    DPP instruction of k_step or k_step2 sits between an exec-narrowing
    instruction and the matching restore."""
    asm = _step_kernels_asm()
    bodies = list(_kernel_bodies(asm, "k_step"))
    # k_step: 2 precisions x (full annulus, rotated sector) x (tau of the solve, per-cell tau); k_step2: 2
    # precisions x the two kinds of tau
    assert len(bodies) == 12
    sreg = r"s\[\d+:\d+\]"
    for name, lines in bodies:
        # An exec-narrowing region opens with s_and_saveexec_b64 sX (on every
        # path that enters it, so possibly more than once in the text) and
        # closes with s_or_b64 exec, exec, sY where sY holds the saved mask.
        # The mask may move on the way (s_xor_b64 sA, exec, sX before an
        # else-arm, s_or_saveexec_b64 / s_andn2_saveexec_b64 sA, sX, s_mov):
        # each region is the set of registers its mask has been copied to.
        regions, shifts, dpp, narrowed = [], 0, 0, 0
        for line in lines:
            t = line.strip()
            m = re.match(r"s_and_saveexec_b64\s+(" + sreg + ")", t)
            if m:
                regions.append({m.group(1)})
                continue
            m = re.match(r"s_(?:xor_b64|mov_b64|or_saveexec_b64|andn2_saveexec_b64)\s+(" + sreg + r"),\s*(?:exec,\s*)?("
                         + sreg + ")", t)
            if m:
                for reg in regions:
                    if m.group(2) in reg:
                        reg.add(m.group(1))
                continue
            m = re.match(r"s_or_b64\s+exec,\s*exec,\s*(" + sreg + ")", t)
            if m:
                regions = [reg for reg in regions if m.group(1) not in reg]
            if "wave_shr:1" in t or "wave_shl:1" in t:
                shifts += 1
            if re.search(r"\b(wave_sh[lr]|row_|quad_perm)", t):
                dpp += 1
                narrowed += bool(regions)
        assert shifts >= 66, (name, shifts)
        assert dpp >= shifts, (name, dpp)
        assert narrowed == 0, (name, narrowed)


def test_step_kernel_uses_no_scratch_memory():
    """Register spills of the step kernels must stay in registers (AGPRs): a
    spill to scratch memory inside the row loop adds memory round trips to
    every row.  Checked on the code-object metadata of every variant of the
    one-step and the two-step kernel."""
    asm = _step_kernels_asm()
    seen = 0
    for block in asm.split("- .agpr_count:")[1:]:
        name = re.search(r"\.name:\s+(\S+)", block).group(1)
        if "k_step" not in name:
            continue
        seen += 1
        assert int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", block).group(1)) == 0, name
    assert seen == 12
