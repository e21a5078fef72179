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
