"""The buffer-parity rules of packed chunks (pdbm_schedule.h) on the CPU,
under AddressSanitizer and UndefinedBehaviorSanitizer, against a
step-by-step model of the launches a chunk enqueues: two-step launches (an
odd chunk ending with single steps) and single-column launches of up to k
steps, for members that finish before, inside or after the chunk."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pack_schedule(tmp_path):
    exe = str(tmp_path / "schedule_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", f"-I{ROOT}/paper_1308_0653_amd/csrc",
                    os.path.join(ROOT, "tests", "host", "schedule_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "schedule ok" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
