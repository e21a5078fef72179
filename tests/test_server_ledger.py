"""The request server's admission accounting (pdbm_ledger.h) on the CPU,
under AddressSanitizer and UndefinedBehaviorSanitizer: memory in use and
request counts stay balanced, and a request reached twice (a failed set-up,
then a scheduler error) is retired once."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_server_ledger(tmp_path):
    exe = str(tmp_path / "ledger_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", f"-I{ROOT}/include",
                    f"-I{ROOT}/paper_1308_0653_amd/csrc", os.path.join(ROOT, "tests", "host", "ledger_check.cpp"),
                    "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and "ledger ok" in r.stdout, r.stderr
