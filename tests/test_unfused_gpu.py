"""PDBM_FUSE=0: every launch takes a single step (the one-step kernel, also
for single theta columns, whose lanes then run along r one step at a time),
for single solves and packs alike.  The switch is read once per process, so
a child process runs the cases with it set; its results must equal those of
the multi-step launches (two steps per launch, up to 8 for a single column)
to rounding, drift records included, and the oracle."""
import os
import subprocess
import sys
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_0653_amd import pdbm as P
from paper_1308_0653_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def cases():
    """(workload, steps, flags): a single column, a disc of the 1/8 sector
    as a single column, and a full annulus of three strips."""
    col = replace(W.small_fp64(), name="column", nr=97, ntheta=1, r_min=0.3, r_max=1.0, dt=2e-5 * 64 / 97,
                  tau=5e-5, r_split=0.5513, p_noise=1e-3, seed=41, nsteps=0)
    disc = W.Workload("col_disc", 96, 1, 0.0, 1.0, dt=1e-4, tau=2e-4, w1=1.0, w2=50.0, m=1, n=1, Q=1.0, T_th=1.1,
                      r_split=0.3, inner=(1.5, 1.55556, 0.666667, 0.0, 1.0), outer=(1.0, 1.0, 0.0, 0.0, 0.0),
                      p_noise=1e-3, seed=42, nsteps=0, sector=1)
    wide = replace(W.small_fp64(), name="wide", nr=40, ntheta=150, r_min=0.3, dt=1e-5, r_split=0.5, p_noise=1e-3,
                   seed=43, nsteps=0)
    return [(col, 29, 0), (disc, 20, P.PDBM_ALLOW_CFL), (wide, 15, 0)]


def run_all():
    """Each case alone, then all of them in one pack (chunks of 7 steps):
    fields and drift totals."""
    out = {}
    for w, n, flags in cases():
        s = P.Solver(P.make_params(**w.params_kw(), diag_every=3, flags=flags), P.make_ic(**w.ic_kw()))
        s.step(n)
        F, d = s.moments(check=False)
        out[f"solo_{w.name}"] = F
        out[f"solo_{w.name}_drift"] = np.array([d["mass"], d["energy"], d["chem"]])
        s.close()
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=4, chunk_steps=7)
    ids = [(w, srv.submit(P.make_params(**w.params_kw(), diag_every=3, flags=flags), P.make_ic(**w.ic_kw()), n,
                          keep_fields=True)) for w, n, flags in cases()]
    assert srv.wait(60.0)
    for w, rid in ids:
        state, F, d = srv.poll(rid, fields=True)
        assert state == P.PDBM_DONE
        out[f"pack_{w.name}"] = F
        out[f"pack_{w.name}_drift"] = np.array([d["mass"], d["energy"], d["chem"]])
    srv.close()
    return out


CHILD = """
import sys
import numpy as np
sys.path.insert(0, {root!r})
from tests.test_unfused_gpu import run_all
np.savez({out!r}, **run_all())
print("child done", flush=True)
"""


def _errs(F, R):
    us = max(np.abs(R[1]).max(), np.abs(R[2]).max(), np.sqrt(np.abs(R[3]).max()))
    return np.array([np.abs(F[k] - R[k]).max() / (us if k in (1, 2) else max(np.abs(R[k]).max(), 1e-300))
                     for k in range(6)])


def test_single_steps_per_launch_equal_multi_step_launches(tmp_path):
    out = str(tmp_path / "unfused.npz")
    env = dict(os.environ, PDBM_FUSE="0")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, out=out)], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    one = dict(np.load(out))
    multi = run_all()
    for w, n, _ in cases():
        o = O.Solver(O.make_params(**w.params_kw()))
        o.init_ic(**w.ic_kw())
        o.step(n)
        R = o.fields()
        for how in ("solo", "pack"):
            key = f"{how}_{w.name}"
            err = _errs(one[key], multi[key])
            drift = np.abs(one[key + "_drift"] - multi[key + "_drift"]) / np.abs(multi[key + "_drift"])
            print(f"{key} n={n}: single vs multi-step {err.max():.1e}, drift {drift.max():.1e}", flush=True)
            assert err.max() < 1e-12, (key, err)
            assert drift.max() < 1e-12, (key, drift)
            err = _errs(one[key], R)
            assert max(err[k] for k in (0, 3, 5)) < 1e-10, (key, err)
