"""Single-column solves (ntheta = 1, the quasi-one-dimensional runs of
Sec. III) advance up to 8 steps per launch: each wavefront holds 64 rows and
owns the 48 in the middle, the 8 on either side going wrong one lane per
step.  These cases check the state against the oracle after step counts
that split into launches of every length, row counts around the 48-row
blocks, the radial ghosts (zero-gradient ends, the disc centre on the
paper's 1/8 sector), drift records of every step (several rings of records
added up on the way), checkpoints taken between launches of odd length,
and single columns stepped in packed launches (also up to 8 steps each,
alone or beside grids of more than one column)."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_0653_amd import pdbm as P
from paper_1308_0653_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _case(nr, sector=8, disc=False, seed=0):
    # a reacting, outward-moving, noisy state
    if disc:
        return W.Workload("col_disc", nr, 1, 0.0, 1.0, dt=2e-4 * 48 / max(nr, 48), tau=2e-4, w1=1.0, w2=50.0,
                          m=1, n=1, Q=1.0, T_th=1.1, r_split=0.3, inner=(1.5, 1.55556, 0.666667, 0.0, 1.0),
                          outer=(1.0, 1.0, 0.0, 0.0, 0.0), p_noise=1e-3, seed=seed, nsteps=0, sector=sector)
    # (r_split falls on no cell centre of these grids: a centre exactly at
    # r_split would be inner or outer by the rounding of r_i)
    return replace(W.small_fp64(), nr=nr, ntheta=1, r_min=0.3, r_max=1.0, dt=2e-5 * 64 / max(nr, 64), tau=5e-5,
                   r_split=0.5513, sector=sector, p_noise=1e-3, seed=seed, nsteps=0)


def _params(w, precision=P.PDBM_FP64, diag_every=0):
    flags = P.PDBM_ALLOW_CFL if w.r_min == 0.0 else 0
    return P.make_params(**w.params_kw(), precision=precision, diag_every=diag_every, flags=flags)


def _oracle(w, nsteps):
    o = O.Solver(O.make_params(**w.params_kw()))
    o.init_ic(**w.ic_kw())
    o.step(nsteps)
    return o


def _errs(F, R):
    us = max(np.abs(R[1]).max(), np.abs(R[2]).max(), np.sqrt(np.abs(R[3]).max()))
    out = []
    for k in range(6):
        sc = us if k in (1, 2) else np.abs(R[k]).max()
        out.append(np.abs(F[k] - R[k]).max() / (sc if sc > 0 else 1.0))
    return np.array(out)


CHUNKS = {"ones": [1] * 11, "mixed": [3, 8, 13, 2, 9, 1], "long": [37]}


@pytest.mark.parametrize("nr", [1, 2, 7, 47, 48, 49, 96, 97, 300])
@pytest.mark.parametrize("chunks", sorted(CHUNKS))
def test_single_column_against_oracle(nr, chunks):
    w = _case(nr, seed=nr)
    s = P.Solver(_params(w), P.make_ic(**w.ic_kw()))
    for n in CHUNKS[chunks]:
        s.step(n)
    total = sum(CHUNKS[chunks])
    assert s.step_count == total
    F, _ = s.moments(check=False)
    err = _errs(F, _oracle(w, total).fields())
    assert np.isfinite(err).all() and err.max() < TOL64, (nr, chunks, err)


@pytest.mark.parametrize("sector", [1, 2, 4])
def test_single_column_disc_centre(sector):
    """The disc centre (r_min = 0): below row 0 its ghost, row 0 with the
    directions turned by 4, set again before every step of a launch."""
    w = _case(60, sector=sector, disc=True, seed=sector)
    s = P.Solver(_params(w), P.make_ic(**w.ic_kw()))
    for n in (5, 8, 8, 3, 16):
        s.step(n)
    F, _ = s.moments(check=False)
    err = _errs(F, _oracle(w, 40).fields())
    print("disc sector", sector, [f"{e:.1e}" for e in err], flush=True)
    assert np.isfinite(err).all() and err.max() < TOL64, err


def test_single_column_records_every_step():
    """Drift records of every step, taken inside launches of several steps,
    over more steps than the ring of partial sums holds, against the oracle's
    drift report of the same steps."""
    w = _case(130, seed=5)
    s = P.Solver(_params(w, diag_every=1), P.make_ic(**w.ic_kw()))
    for n in (5, 64, 7, 80, 3):
        s.step(n)
    hist = s.diag_history()
    assert [h["step"] for h in hist] == list(range(159))
    o = O.Solver(O.make_params(**w.params_kw()))
    o.init_ic(**w.ic_kw())
    for h in hist[::9]:
        o.step(h["step"] - o.step_count)
        ref = o.diag()
        for k in ("mass", "energy", "chem"):
            assert abs(h[k] - ref[k]) <= 1e-12 * abs(ref[k]), (h["step"], k)
        assert h["n_nonfinite"] == 0 and h["n_nonphys"] == 0


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_single_column_checkpoint_between_odd_launches(precision):
    """The state's buffer parity after launches of odd and even lengths:
    a checkpoint taken after 13 steps and resumed gives the same state,
    bitwise, as the run that went on."""
    w = _case(100, seed=9)
    a = P.Solver(_params(w, precision), P.make_ic(**w.ic_kw()))
    a.step(5)
    a.step(8)
    blob = a.get_state()
    a.step(11)
    b = P.Solver(_params(w, precision), P.make_ic(**w.ic_kw()))
    b.set_state(blob)
    b.step(11)
    fa, la = a.read_f()
    fb, lb = b.read_f()
    assert np.array_equal(fa, fb) and np.array_equal(la, lb)


def test_single_column_float32_bound():
    w = _case(300, seed=11)
    s = P.Solver(_params(w, P.PDBM_FP32), P.make_ic(**w.ic_kw()))
    s.step(60)
    F, _ = s.moments(check=False)
    err = _errs(F, _oracle(w, 60).fields())
    print("float32 single column", [f"{e:.1e}" for e in err], flush=True)
    for k in (0, 3, 5):
        assert err[k] < 1e-4, (k, err)


def test_single_column_solver_equals_packed_steps():
    """The same solve alone and in a pack, both up to 8 steps per launch but
    cut at other steps (launches of 8 alone, chunks of 7 in the pack): equal
    to rounding, drift records included."""
    w = _case(200, seed=13)
    s = P.Solver(_params(w, diag_every=4), P.make_ic(**w.ic_kw()))
    s.step(40)
    Fs, ds = s.moments(check=False)
    b = P.Batch([_params(w, diag_every=4)], [P.make_ic(**w.ic_kw())], chunk_steps=7)
    b.step(40)
    Fb, db = b.moments(0, check=False)
    err = _errs(Fs, Fb)
    assert err.max() < 1e-13, err
    for k in ("mass", "energy", "chem"):
        assert abs(ds[k] - db[k]) <= 1e-13 * abs(db[k]), k


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_packed_single_columns_several_steps_per_launch(precision):
    """A pack of single columns only (row counts around the 48-row blocks,
    a disc of the 1/8 sector, a 3/8 sector) takes up to 8 steps per launch:
    members with odd counts finish inside a launch and leave the pack,
    chunks of 7 steps cut launches at other steps than the solo runs, and
    each member's buffer parity follows the launch lengths it took.  Every
    result equals its solo run to rounding, drift records included, and the
    oracle."""
    ws = [_case(47, seed=21), _case(97, seed=22), _case(150, sector=3, seed=23), _case(96, sector=1, disc=True, seed=24)]
    counts = [29, 40, 17, 33]
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=4, chunk_steps=7)
    ids = [srv.submit(_params(w, precision, diag_every=3), P.make_ic(**w.ic_kw()), n, keep_fields=True)
           for w, n in zip(ws, counts)]
    assert srv.wait(60.0)
    tol = 1e-13 if precision == P.PDBM_FP64 else 1e-5
    otol = TOL64 if precision == P.PDBM_FP64 else 1e-4
    for rid, w, n in zip(ids, ws, counts):
        state, F, d = srv.poll(rid, fields=True)
        assert state == P.PDBM_DONE
        solo = P.Solver(_params(w, precision, diag_every=3), P.make_ic(**w.ic_kw()))
        solo.step(n)
        Fs, ds = solo.moments(check=False)
        err = _errs(F, Fs)
        print(f"nr={w.nr} sector={w.sector} n={n} precision={precision}: vs solo {err.max():.1e}", flush=True)
        assert err.max() < tol, (w.nr, err)
        for k in ("mass", "energy", "chem"):
            assert abs(d[k] - ds[k]) <= tol * abs(ds[k]), (w.nr, k)
        err = _errs(F, _oracle(w, n).fields())
        assert max(err[k] for k in (0, 3, 5)) < otol, (w.nr, err)
    srv.close()


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_packs_mixing_columns_and_wider_grids(precision):
    """A pack holding single columns (one of them a disc of the 1/8 sector)
    beside grids of more than one column (a full annulus of three strips and
    a 3/8 sector): the wider grids step in pairs and the columns up to 8
    steps per launch of their own kernel, in the same chunks of 7 steps,
    each member's buffer parity following the launches it took.  Members
    with odd counts leave mid-chunk.  Every result equals its solo run to
    rounding, drift records included, and the oracle."""
    ws = [_case(97, seed=31), _case(96, sector=1, disc=True, seed=32),
          replace(W.small_fp64(), name="wide", nr=40, ntheta=150, r_min=0.3, dt=1e-5, r_split=0.5, p_noise=1e-3,
                  seed=33, nsteps=0),
          replace(W.small_fp64(), name="sector3", nr=24, ntheta=24, sector=3, r_min=0.5, dt=1e-4, tau=4e-4,
                  r_split=0.7, p_noise=1e-3, seed=34, nsteps=0)]
    counts = [29, 40, 33, 26]
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=4, chunk_steps=7)
    ids = [srv.submit(_params(w, precision, diag_every=3), P.make_ic(**w.ic_kw()), n, keep_fields=True)
           for w, n in zip(ws, counts)]
    assert srv.wait(60.0)
    tol = 1e-12 if precision == P.PDBM_FP64 else 1e-5
    otol = TOL64 if precision == P.PDBM_FP64 else 1e-4
    for rid, w, n in zip(ids, ws, counts):
        state, F, d = srv.poll(rid, fields=True)
        assert state == P.PDBM_DONE
        solo = P.Solver(_params(w, precision, diag_every=3), P.make_ic(**w.ic_kw()))
        solo.step(n)
        Fs, ds = solo.moments(check=False)
        err = _errs(F, Fs)
        print(f"{w.name} {w.nr}x{w.ntheta} sector={w.sector} n={n} precision={precision}: vs solo {err.max():.1e}",
              flush=True)
        assert err.max() < tol, (w.name, err)
        for k in ("mass", "energy", "chem"):
            assert abs(d[k] - ds[k]) <= tol * abs(ds[k]), (w.name, k)
        err = _errs(F, _oracle(w, n).fields())
        assert max(err[k] for k in (0, 3, 5)) < otol, (w.name, err)
    srv.close()
