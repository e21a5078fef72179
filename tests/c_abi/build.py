"""Builds the plain C client of the ABI against include/pdbm.h and the
in-tree libpdbm.so (gcc; the library is found through the binary's run
path)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "pdbm_c_client.c")
BIN = os.path.join(HERE, "pdbm_c_client")


def build() -> str:
    pkg = os.path.join(ROOT, "paper_1308_0653_amd")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", f"-I{os.path.join(ROOT, 'include')}", SRC, "-o", BIN + ".tmp",
           f"-L{pkg}", "-lpdbm", "-Wl,-rpath,$ORIGIN/../../paper_1308_0653_amd", "-Wl,-rpath,/opt/rocm/lib", "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build())
