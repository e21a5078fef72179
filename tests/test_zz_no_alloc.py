"""pdbm_create_noalloc through the C ABI against pdbm_create: the same
solve, with its auxiliary device memory in the library's static scratch and
its state in a caller-owned buffer, gives the same fields, drift report and
drift history bit for bit.  Two solves in a row, the second smaller and in
the other precision, so the second runs over what the first left in the
scratch."""
from dataclasses import replace

import numpy as np
import pytest

from paper_1308_0653_amd import pdbm as P
from paper_1308_0653_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [
    # a ragged grid (strips and row blocks with tails), float64, odd steps
    (replace(W.small_fp64(), nr=200, ntheta=300, r_min=0.2, dt=4e-6, tau=1e-5, r_split=0.35, w1=3.0, w2=7.0,
             m=1, n=3), P.PDBM_FP64, 31),
    # smaller, float32, even steps
    (replace(W.small_fp64(), nr=70, ntheta=90, r_min=0.2, dt=1e-5, tau=2e-5, r_split=0.35), P.PDBM_FP32, 24),
]


def _run(s, n):
    s.step(n)
    F, d = s.moments(check=False)
    return F, d, s.diag_history()


def test_noalloc_matches_create_two_calls_in_a_row():
    torch = pytest.importorskip("torch")
    stream = torch.cuda.current_stream()
    for w, prec, n in CASES:
        print(f"noalloc case {w.nr}x{w.ntheta} precision {prec} steps {n}", flush=True)
        p = P.make_params(**w.params_kw(), precision=prec, diag_every=1)
        ic = P.make_ic(**w.ic_kw())
        nbytes = P.pdbm_noalloc_state_bytes(p)
        state = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        s = P.pdbm_create_noalloc(p, ic, state, stream=stream)
        # the device's static slot is taken while s lives
        with pytest.raises(P.PdbmError) as e:
            P.pdbm_create_noalloc(p, ic, torch.empty(nbytes, dtype=torch.uint8, device="cuda"), stream=stream)
        assert e.value.code == P.PDBM_EAGAIN
        got = _run(s, n)
        ref_s = P.Solver(p, ic, stream=stream)
        ref = _run(ref_s, n)
        ref_s.close()
        s.close()
        assert np.array_equal(got[0], ref[0])
        assert got[1] == ref[1]
        assert len(got[2]) == n and got[2] == ref[2]
        assert got[1]["n_nonfinite"] == 0 and got[1]["n_nonphys"] == 0
