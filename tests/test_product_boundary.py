"""Rules of the product path, checked without a GPU (and one with it):

- the product package never imports the CPU oracle (only tests, the smoke
  check and the benchmark's CPU-baseline leg may);
- a missing library that cannot be built fails loudly, with no fallback;
- bench.py measures one GPU and refuses other counts;
- the bench line carries the fields its consumers read."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1308_0653_amd")


def _run(code, env=None, timeout=300):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=timeout,
                          env=e)


def test_product_package_never_imports_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, flags=re.M), f
                assert "liboracle" not in src and "pdbm_oracle" not in src, f
    r = _run("import sys; import paper_1308_0653_amd.pdbm, paper_1308_0653_amd.workloads, paper_1308_0653_amd.build; "
             "bad = [m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]; "
             "assert not bad, bad; print('clean')")
    assert r.returncode == 0 and "clean" in r.stdout, r.stderr


def test_missing_library_fails_loudly():
    code = ("from paper_1308_0653_amd import pdbm as P\n"
            "P.LIB_PATH = '/nonexistent/libpdbm.so'\n"
            "try:\n"
            "    P.lib()\n"
            "except Exception as e:\n"
            "    print('raised', type(e).__name__)\n"
            "else:\n"
            "    print('loaded')\n")
    r = _run(code, env={"HIPCC": "/bin/false"})
    assert "raised" in r.stdout, r.stdout + r.stderr


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.gpu
def test_bench_line_contract():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "5", "--warmup", "1",
                        "--no-serving", "--no-fp32", "--cpu-steps", "1"], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 1 and d["value"] > 0
    assert d["config"]["workload"] == "outward1024_fp64"
    rl = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in rl, key
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and 0 < rl["frac"] < 1
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0
    assert cb["single_core"]["cores"] == 1 and cb["single_core"]["value"] > 0
    side = d["side_kernels"]
    assert side["noneq"]["avg_us"] > 0 and 0 < side["noneq"]["frac_of_peak"] < 1
    assert side["tau_field"]["avg_launch_us"] > 0 and side["tau_field"]["plain_avg_launch_us"] > 0
    assert side["sector"]["avg_launch_us"] > 0 and 0 < side["sector"]["effective_frac_of_peak"] < 1
