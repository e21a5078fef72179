"""Host-side checks of the library's own code, with no GPU.

- Bounds of the step kernels' buffer accesses: tests/host/offsets_check.cpp
  evaluates the kernels' offset functions (pdbm_offsets.h) for every strip,
  lane and row of the largest grids of each kind, the strip-edge test grids
  and the benchmark workloads, and checks every access against its buffer
  and every 32-bit offset against wrapping.  It must also flag the grids one
  row larger than the largest accepted ones, whose offsets wrap.
- AddressSanitizer on host code: the library built with the sanitizer on its
  host part only, driven by the plain C client's host entry points
  (validation, sizes, the moment-inversion matrix, a create that must fail
  cleanly without a GPU), with leak detection.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1308_0653_amd", "csrc")
INC = os.path.join(ROOT, "include")


def _build_offsets_check(out, extra=()):
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{INC}",
                    f"-I{CSRC}", *extra, os.path.join(ROOT, "tests", "host", "offsets_check.cpp"), "-o", out],
                   check=True, capture_output=True, text=True)


def test_kernel_buffer_offsets_in_bounds(tmp_path):
    exe = str(tmp_path / "offsets_check")
    _build_offsets_check(exe)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0 and "0 out of bounds" in r.stdout, r.stderr[-3000:]
    # one row more than the largest accepted grids: the check sees the wrap
    for grid in (["4035", "4000", "8", "8"], ["8134408", "1", "8", "8"]):
        r = subprocess.run([exe, *grid], capture_output=True, text=True, timeout=300)
        assert r.returncode == 1 and "OUT OF BOUNDS" in r.stderr, grid


def test_offsets_check_is_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "offsets_check_san")
    _build_offsets_check(exe, ("-fsanitize=address,undefined", "-fno-sanitize-recover=all"))
    r = subprocess.run([exe, "986", "462", "8", "4"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]


@pytest.mark.slow
def test_library_host_code_under_address_sanitizer(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    clang = "/opt/rocm/llvm/bin/clang"
    if not (shutil.which(hipcc) or os.path.exists(hipcc)) or not os.path.exists(clang):
        pytest.skip("no ROCm toolchain")
    lib = str(tmp_path / "libpdbm.so")
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    host_asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-Xclang",
                    "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
                    *host_asan, f"-I{INC}", f"-I{CSRC}", *srcs, "-o", lib, "-lpthread"],
                   check=True, capture_output=True, text=True)
    rtdir = os.path.dirname(subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                           capture_output=True, text=True, check=True).stdout.strip())
    exe = str(tmp_path / "client")
    subprocess.run([clang, "-std=c11", "-O1", "-g", "-fsanitize=address", "-shared-libsan", f"-I{INC}",
                    os.path.join(ROOT, "tests", "c_abi", "pdbm_c_client.c"), "-o", exe, f"-L{tmp_path}", "-lpdbm",
                    f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath,/opt/rocm/lib", f"-Wl,-rpath,{rtdir}", "-lm"],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe, "cpu"], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "cpu ok" in r.stdout, (r.stdout + r.stderr)[-3000:]
    assert "AddressSanitizer" not in r.stderr
