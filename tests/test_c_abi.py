"""The ABI from a plain C program (tests/c_abi/pdbm_c_client.c): no Python
and no torch in the calling process.  Built by __graft_entry__.build()."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_0653_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
CLIENT = os.path.join(HERE, "c_abi", "pdbm_c_client")


def _client():
    if not os.path.exists(CLIENT):
        import importlib.util
        spec = importlib.util.spec_from_file_location("cb", os.path.join(HERE, "c_abi", "build.py"))
        cb = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(cb)
        cb.build()
    return CLIENT


def test_c_client_host_entry_points():
    """Validation, error strings, the F_k matrix and state sizing from C;
    without a usable GPU creating a solve fails with PDBM_ENOSYS or
    PDBM_EHIP (with a GPU present the client skips nothing: it runs the same
    checks and a solve may be created, so this test only runs without one)."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = subprocess.run([_client(), "cpu"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert "cpu ok" in r.stdout


@pytest.mark.gpu
def test_c_client_solves_match_oracle():
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "fields.bin")
        r = subprocess.run([_client(), "gpu", out], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "gpu ok" in r.stdout
        F = np.fromfile(out, dtype=np.float64).reshape(6, 64, 64)
    w = W.small_fp64()
    o = O.Solver(O.make_params(**w.params_kw()))
    o.init_ic(**w.ic_kw())
    o.step(50)
    R = o.fields()
    for k in (0, 3, 5):
        assert np.abs(F[k] - R[k]).max() <= 1e-10 * np.abs(R[k]).max(), k
