"""Per-cell relaxation time (Sec. IV, point (ii)) on the GPU, through the C
ABI, against the oracle given the same tau field.

The paper notes that tau should depend on the local state and so vary in
space and time, and gives no form; the library takes the field from the
caller (pdbm_set_tau, pdbm_set_tau_async on a solve created with
PDBM_TAU_FIELD).  The fields here are seeded, smooth in r and theta with a
random factor per cell, and include cells of tau = +inf (no relaxation).
The float64 bar is the parity bar of every other float64 path (normwise
relative L_inf 1e-10); float32 is held to its stated 1e-4.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_0653_amd import pdbm as P
from paper_1308_0653_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-10, 1e-4


def _field(w, seed, inf_cells=3):
    """tau(r, theta) = tau0 (1 + 0.5 sin(2 theta + 3 r)) U[0.7, 1.3]; a few
    cells get tau = +inf."""
    rng = np.random.default_rng(seed)
    dr = (w.r_max - w.r_min) / w.nr
    r = w.r_min + (np.arange(w.nr) + 0.5) * dr
    th = (np.arange(w.ntheta) + 0.5) * w.sector * np.pi / 4 / w.ntheta
    R, TH = np.meshgrid(r, th, indexing="ij")
    tau = w.tau * (1 + 0.5 * np.sin(2 * TH + 3 * R)) * rng.uniform(0.7, 1.3, R.shape)
    for _ in range(inf_cells):
        tau[rng.integers(w.nr), rng.integers(w.ntheta)] = np.inf
    return tau


def _gpu(w, precision=P.PDBM_FP64, flags=P.PDBM_TAU_FIELD):
    return P.Solver(P.make_params(**w.params_kw(), precision=precision, flags=flags), P.make_ic(**w.ic_kw()))


def _oracle(w):
    o = O.Solver(O.make_params(**w.params_kw()))
    o.init_ic(**w.ic_kw())
    return o


def _errors(got, ref):
    sc = [np.abs(ref[k]).max() for k in range(6)]
    us = max(sc[1], sc[2], np.sqrt(np.abs(ref[3]).max()))
    sc[1] = sc[2] = us
    return [np.abs(got[k] - ref[k]).max() / (sc[k] if sc[k] > 0 else 1.0) for k in range(6)]


CASES = {
    # one strip (the edge cells of the two-step kernel are the strip's own periodic images)
    "annulus64": replace(W.small_fp64(), nsteps=121),
    # three strips, ragged last strip, a != b
    "wide": replace(W.small_fp64(), nr=20, ntheta=150, r_min=0.3, dt=1e-5, w1=3.0, w2=7.0, m=1, n=3, r_split=0.5,
                    p_noise=1e-3, nsteps=41),
    # rotated sector, two steps per launch
    "sector3": replace(W.small_fp64(), nr=24, ntheta=24, sector=3, r_min=0.5, dt=1e-4, tau=4e-4, r_split=0.7,
                       nsteps=60),
    # one theta column: lanes along r
    "ntheta1": W.Workload("vv1d", 300, 1, 1000.0, 1000.1, dt=2.5e-6, tau=2e-4, w1=10.0, w2=1000.0, m=1, n=1, Q=1.0,
                          T_th=1.1, r_split=1000.01, inner=(1.35826, 2.59709, 0.81650, 0.0, 1.0),
                          outer=(1.0, 1.0, 0.0, 0.0, 0.0), p_noise=0.0, seed=0, nsteps=150),
    # the paper's 1/8-sector disc
    "disc_s1": W.Workload("disc_s1", 40, 2, 0.0, 1.0, dt=2e-4, tau=2e-4, w1=1.0, w2=50.0, m=1, n=1, Q=1.0, T_th=1.1,
                          r_split=0.3, inner=(1.5, 1.55556, 0.666667, 0.0, 1.0), outer=(1.0, 1.0, 0.0, 0.0, 0.0),
                          p_noise=1e-6, seed=4, nsteps=80, sector=1),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_tau_field_parity_with_oracle(case):
    """The field is set, stepped over (an odd count: pairs and a single
    step), replaced by another, stepped over again."""
    w = CASES[case]
    s, o = _gpu(w), _oracle(w)
    n1 = w.nsteps // 2 + 1
    for seed, n in ((1, n1), (2, w.nsteps - n1)):
        tau = _field(w, seed)
        s.set_tau(tau)
        o.set_tau(tau)
        s.step(n)
        o.step(n)
    F, _ = s.moments(check=False)
    err = _errors(F, o.fields())
    print(case, [f"{e:.1e}" for e in err], flush=True)
    assert max(err) <= TOL64, (case, err)


def test_tau_field_fp32_within_its_bound():
    w = CASES["annulus64"]
    s, o = _gpu(w, P.PDBM_FP32), _oracle(w)
    tau = _field(w, 5)
    s.set_tau(tau)
    o.set_tau(tau)
    s.step(w.nsteps)
    o.step(w.nsteps)
    F, _ = s.moments(check=False)
    err = _errors(F, o.fields())
    print("fp32", [f"{e:.1e}" for e in err], flush=True)
    for k in (0, 3, 5):
        assert err[k] <= TOL32, err


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_uniform_field_equals_the_solves_own_tau(precision):
    """A solve with PDBM_TAU_FIELD starts with the parameters' tau in every
    cell; set back with NULL it returns to it.  Either way it steps as the
    same solve without the flag."""
    w = replace(CASES["wide"], nsteps=21)
    a, b = _gpu(w, precision), _gpu(w, precision, flags=0)
    a.step(11)
    b.step(11)
    a.set_tau(_field(w, 3))
    a.set_tau(None)
    a.step(10)
    b.step(10)
    fa, la = a.read_f()
    fb, lb = b.read_f()
    df = np.abs(fa - fb).max() / np.abs(fb).max()
    print("uniform field vs none", precision, df, np.abs(la - lb).max(), flush=True)
    assert df <= (1e-14 if precision == P.PDBM_FP64 else 1e-6)
    assert np.abs(la - lb).max() <= 1e-13


def test_set_tau_async_equals_the_host_call():
    torch = pytest.importorskip("torch")
    w = replace(CASES["wide"], nsteps=15)
    tau = _field(w, 7)
    stream = torch.cuda.current_stream()
    a = P.Solver(P.make_params(**w.params_kw(), flags=P.PDBM_TAU_FIELD), P.make_ic(**w.ic_kw()), stream=stream)
    b = P.Solver(P.make_params(**w.params_kw(), flags=P.PDBM_TAU_FIELD), P.make_ic(**w.ic_kw()), stream=stream)
    a.set_tau(tau)
    t = torch.from_numpy(tau).to("cuda")
    b.set_tau_async(t)
    a.step(w.nsteps)
    b.step(w.nsteps)
    fa, la = a.read_f()
    fb, lb = b.read_f()
    assert np.array_equal(fa, fb) and np.array_equal(la, lb)


def test_tau_field_refusals():
    w = replace(CASES["wide"], nsteps=1)
    plain = _gpu(w, flags=0)
    with pytest.raises(P.PdbmError) as e:
        plain.set_tau(_field(w, 1))
    assert e.value.code == P.PDBM_EINVAL
    s = _gpu(w)
    for bad in (0.0, -1e-5, np.nan):
        tau = _field(w, 1)
        tau[3, 4] = bad
        with pytest.raises(P.PdbmError) as e:
            s.set_tau(tau)
        assert e.value.code == P.PDBM_EINVAL
