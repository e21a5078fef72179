"""Two steps per launch against one step per launch.

Solver.step(n) advances a full-annulus solve with ntheta > 1 in pairs of
steps, each pair in one pass over f (k_step2: one wavefront per SIMD in
float64, two in float32, whose drift sums are added across the wavefront row
by row); step(1) always takes the one-step kernel.  Both do the same
arithmetic per cell in the same order, so their states agree to rounding.  The cases cover strip and row-block edges
(blocks of one row up to the 16-row limit, marched both ways), rings close
to the axis, both precisions, odd step counts (pairs and one single step), the
drift records of both steps of a pair, and checkpoints taken after an odd
number of pairs, when the state sits in the buffer of the other parity.
Parity of the paired path with the oracle is covered by the parity and
strip-edge tests, which step in pairs.
"""
from dataclasses import replace

import numpy as np
import pytest

from paper_1308_0653_amd import pdbm as P
from paper_1308_0653_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(nr, nt, r_min=0.3, seed=0):
    # a reacting, moving, noisy state: ignition inside r < 0.55; dt keeps
    # the radial Courant number of the fastest speed (12.5) at about 0.35
    dt = min(2e-5, 0.35 * (1.0 - r_min) / nr / 12.5)
    return replace(W.small_fp64(), nr=nr, ntheta=nt, r_min=r_min, r_max=1.0, dt=dt, tau=2.5 * dt, r_split=0.55,
                   p_noise=1e-3, seed=seed)


def _solver(w, precision, diag_every=0):
    return P.Solver(P.make_params(**w.params_kw(), precision=precision, diag_every=diag_every),
                    P.make_ic(**w.ic_kw()))


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# The two paths round differently (the compiler contracts multiply-adds per
# inlined context, and the float32 form converts to and from float64 in
# places): after 7 steps float64 differs by up to about 15 units of its
# rounding (1.7e-15) and float32 by up to about 30 of its own (1.9e-6),
# relative to the largest f.  The bounds allow about 100 and 160.
TOL = {P.PDBM_FP64: 1e-13, P.PDBM_FP32: 1e-5}


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
@pytest.mark.parametrize("nr,nt,r_min", [(1, 64, 0.3), (1, 64, 0.05), (2, 65, 0.3), (2, 130, 0.05), (5, 2, 0.3),
                                         (33, 65, 0.3), (17, 200, 0.05), (40, 130, 0.05), (64, 64, 0.3),
                                         (8192, 130, 0.3)])
def test_pairs_match_single_steps(precision, nr, nt, r_min):
    w = _case(nr, nt, r_min)
    n = 7  # three pairs and one single step
    a = _solver(w, precision)
    a.step(n)
    b = _solver(w, precision)
    for _ in range(n):
        b.step(1)
    assert a.step_count == b.step_count == n
    fa, la = a.read_f()
    fb, lb = b.read_f()
    ef, el = _rel(fa, fb), _rel(la, lb)
    print(f"nr={nr} nt={nt} r_min={r_min} prec={precision}: f {ef:.2e} lambda {el:.2e}", flush=True)
    assert ef <= TOL[precision] and el <= TOL[precision]
    Fa, _ = a.moments()
    Fb, _ = b.moments()
    assert np.abs(Fa - Fb).max() <= TOL[precision] * max(np.abs(Fb).max(), 1.0)


# drift sums of states equal to rounding: float32 states differ in the last
# bits of f between the two paths
DTOL = {P.PDBM_FP64: 1e-13, P.PDBM_FP32: 1e-6}


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_pair_drift_records_match_single_steps(precision):
    w = _case(33, 130)
    a = _solver(w, precision, diag_every=1)
    a.step(130)  # more records than the partial-sum ring holds
    b = _solver(w, precision, diag_every=1)
    for _ in range(130):
        b.step(1)
    ha, hb = a.diag_history(), b.diag_history()
    assert len(ha) == len(hb) == 130
    for ra, rb in zip(ha, hb):
        assert ra["step"] == rb["step"]
        assert ra["n_nonfinite"] == rb["n_nonfinite"] == 0 and ra["n_nonphys"] == rb["n_nonphys"] == 0
        for k in ("mass", "energy", "chem"):
            assert abs(ra[k] - rb[k]) <= DTOL[precision] * abs(rb[k]), (ra, rb)


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_checkpoint_after_odd_number_of_pairs(precision):
    w = _case(20, 70, r_min=0.05)
    ref = _solver(w, precision)
    ref.step(10)
    a = _solver(w, precision)
    a.step(6)  # three pairs: the state sits in the buffer of the other parity
    blob = a.get_state()
    b = _solver(w, precision)
    b.set_state(blob)
    assert b.step_count == 6
    for s in (a, b):
        s.step(4)
    fr, lr = ref.read_f()
    for s in (a, b):
        f, lam = s.read_f()
        assert np.array_equal(f, fr) and np.array_equal(lam, lr)
    # the non-equilibrium measures read the current buffer too
    assert np.array_equal(a.noneq(), ref.noneq())


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_pair_drift_records_every_third_step(precision):
    """Records every third step: a pair holds one record step or none, and
    the records of both kinds of pair match single steps."""
    w = _case(20, 70)
    a = _solver(w, precision, diag_every=3)
    a.step(61)
    b = _solver(w, precision, diag_every=3)
    for _ in range(61):
        b.step(1)
    ha, hb = a.diag_history(), b.diag_history()
    assert [r["step"] for r in ha] == [r["step"] for r in hb] == list(range(0, 61, 3))
    for ra, rb in zip(ha, hb):
        for k in ("mass", "energy", "chem"):
            assert abs(ra[k] - rb[k]) <= DTOL[precision] * abs(rb[k]), (ra, rb)


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_pairs_from_an_odd_step_after_restore(precision):
    """A state restored at an odd step count: the pairs then start at odd
    steps (the other buffer parity and record slots) and agree with single
    steps; the records made after the restore match too."""
    w = _case(24, 130, r_min=0.05)
    src = _solver(w, precision)
    for _ in range(7):
        src.step(1)
    blob = src.get_state()
    a = P.Solver(P.make_params(**w.params_kw(), precision=precision, diag_every=1), P.make_ic(**w.ic_kw()))
    b = P.Solver(P.make_params(**w.params_kw(), precision=precision, diag_every=1), P.make_ic(**w.ic_kw()))
    a.set_state(blob)
    b.set_state(blob)
    a.step(9)
    for _ in range(9):
        b.step(1)
    assert a.step_count == b.step_count == 16
    fa, la = a.read_f()
    fb, lb = b.read_f()
    assert _rel(fa, fb) <= TOL[precision] and _rel(la, lb) <= TOL[precision]
    ha, hb = a.diag_history(), b.diag_history()
    assert [r["step"] for r in ha] == [r["step"] for r in hb] == list(range(7, 16))
    for ra, rb in zip(ha, hb):
        assert abs(ra["mass"] - rb["mass"]) <= max(DTOL[precision], 1e-12) * abs(rb["mass"])


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_pair_drift_counts_match_single_steps(precision):
    """Non-finite and non-physical cells in the drift records: one cell of
    NaN f (whose NaN reaches its four neighbours in each step) and one cell
    with every f negated (rho < 0, T unchanged), both inside strips and
    rows, far apart.  The counts of pairs equal those of single steps, and
    the sums, which leave non-finite cells out, agree."""
    w = _case(40, 130)
    a = _solver(w, precision, diag_every=1)
    f, lam = a.read_f()
    f[:, 10, 30] = np.nan
    f[:, 30, 100] *= -1.0
    a.write_f(f, lam)
    b = _solver(w, precision, diag_every=1)
    b.write_f(f, lam)
    a.step(2)
    b.step(1)
    b.step(1)
    ha, hb = a.diag_history(), b.diag_history()
    assert [r["step"] for r in ha] == [r["step"] for r in hb] == [0, 1]
    assert ha[0]["n_nonfinite"] == hb[0]["n_nonfinite"] == 1
    assert ha[1]["n_nonfinite"] == hb[1]["n_nonfinite"] == 5
    assert ha[0]["n_nonphys"] == hb[0]["n_nonphys"] == 1
    for ra, rb in zip(ha, hb):
        for k in ("mass", "energy", "chem"):
            assert np.isfinite(ra[k]) and abs(ra[k] - rb[k]) <= DTOL[precision] * abs(rb[k]), (ra, rb)
