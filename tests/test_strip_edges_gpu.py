"""Strip and row-block edges of the step kernel against the oracle (FP64).

A wavefront owns 64 theta columns and a block of rows; columns past the last
one hold periodic images, the two halo columns come from gathers, rows are
padded to a multiple of 64.  These cases put the last column of the grid at
every position relative to the strip (widths around 1, 16, 64 and 128), use
row counts that leave blocks of one or two rows, march blocks in both
directions, and rotate the halo for a sector."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_0653_amd import pdbm as P
from paper_1308_0653_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
WIDTHS = [1, 2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 200]


def _case(nr, nt, sector=8, seed=0, r_min=0.3):
    # a reacting, moving, noisy state: ignition inside r < 0.55
    return replace(W.small_fp64(), nr=nr, ntheta=nt, r_min=r_min, r_max=1.0, dt=2e-5, tau=5e-5, r_split=0.55,
                   sector=sector, p_noise=1e-3, seed=seed, nsteps=12)


def _scales(R):
    sc = [np.abs(R[k]).max() for k in range(6)]
    us = max(sc[1], sc[2], np.sqrt(np.abs(R[3]).max()))
    sc[1] = sc[2] = us
    return [v if v > 0 else 1.0 for v in sc]  # a field that is zero everywhere (lambda) is compared absolutely


def _check(F, w):
    o = O.Solver(O.make_params(**w.params_kw()))
    o.init_ic(**w.ic_kw())
    o.step(w.nsteps)
    R = o.fields()
    sc = _scales(R)
    err = np.array([np.abs(F[k] - R[k]).max() / sc[k] for k in range(6)])
    assert np.isfinite(err).all() and err.max() < TOL64, (w.nr, w.ntheta, w.sector, err)


@pytest.mark.parametrize("nt", WIDTHS)
def test_strip_widths_single_solve(nt):
    for nr in (1, 2, 5, 33):
        w = _case(nr, nt)
        s = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP64), P.make_ic(**w.ic_kw()))
        s.step(w.nsteps)
        F, _ = s.moments(check=False)
        _check(F, w)


def test_strip_widths_packed_short_blocks():
    """Packed launches use 4-row blocks: every nr below gives a last block
    of 1, 2 or 3 rows, marched outward or inward by block parity."""
    ws = [_case(nr, nt, seed=i) for i, (nr, nt) in enumerate([(5, 65), (6, 63), (7, 129), (9, 17), (10, 128),
                                                              (13, 1), (3, 200)])]
    b = P.Batch([P.make_params(**w.params_kw(), precision=P.PDBM_FP64) for w in ws],
                [P.make_ic(**w.ic_kw()) for w in ws], chunk_steps=4)
    b.step(ws[0].nsteps)
    for i, w in enumerate(ws):
        F, _ = b.moments(i, check=False)
        _check(F, w)


@pytest.mark.parametrize("nt,sector", [(65, 1), (130, 3), (17, 5), (64, 2)])
def test_rotated_sector_halos(nt, sector):
    w = _case(6, nt, sector=sector)
    s = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP64), P.make_ic(**w.ic_kw()))
    s.step(w.nsteps)
    F, _ = s.moments(check=False)
    _check(F, w)


@pytest.mark.parametrize("nt", [256, 512, 768])
@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_strip_groups_of_whole_workgroups(nt, precision):
    """Widths of whole workgroups of strips (multiples of 256: 4, 8 and 12
    strips, so that the four wavefronts of a workgroup hold adjacent strips
    of one row block, the last one's right neighbour being the first
    strip).  Row counts leave blocks of one or a few rows; odd step counts
    end with a one-step launch.  Float64 against the oracle at the parity
    bound, float32 at its own."""
    tol = TOL64 if precision == P.PDBM_FP64 else 1e-4
    for nr, nsteps in ((1, 12), (5, 13), (33, 12), (70, 9)):
        w = replace(_case(nr, nt), nsteps=nsteps)
        s = P.Solver(P.make_params(**w.params_kw(), precision=precision), P.make_ic(**w.ic_kw()))
        s.step(w.nsteps)
        F, _ = s.moments(check=False)
        o = O.Solver(O.make_params(**w.params_kw()))
        o.init_ic(**w.ic_kw())
        o.step(w.nsteps)
        R = o.fields()
        sc = _scales(R)
        err = np.array([np.abs(F[k] - R[k]).max() / sc[k] for k in range(6)])
        print(f"nt={nt} nr={nr} steps={nsteps} precision={precision}: max err {err.max():.2e}", flush=True)
        assert np.isfinite(err).all() and err.max() < tol, (nr, nt, err)


@pytest.mark.parametrize("sector", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_rotated_sectors_in_pairs(sector, precision):
    """Annular sectors step two steps per launch: the periodic images past
    the last column, and the edge cells at the sector's ends, carry the
    directions and the angles turned by the sector.  Widths leave none, one
    or most lanes of the last strip to images (of several turns where the
    sector is narrow), row counts give blocks of one or two rows, and odd
    step counts end with a one-step launch.  Against the oracle: float64 at
    the parity bound, float32 at its own."""
    tol = TOL64 if precision == P.PDBM_FP64 else 1e-4
    for nr, nt, nsteps in ((1, 17, 12), (5, 63, 13), (33, 65, 12), (12, 130, 9)):
        w = replace(_case(nr, nt, sector=sector), nsteps=nsteps)
        s = P.Solver(P.make_params(**w.params_kw(), precision=precision), P.make_ic(**w.ic_kw()))
        s.step(w.nsteps)
        F, _ = s.moments(check=False)
        o = O.Solver(O.make_params(**w.params_kw()))
        o.init_ic(**w.ic_kw())
        o.step(w.nsteps)
        R = o.fields()
        sc = _scales(R)
        err = np.array([np.abs(F[k] - R[k]).max() / sc[k] for k in range(6)])
        print(f"sector={sector} nr={nr} nt={nt} steps={nsteps} precision={precision}: max err {err.max():.2e}",
              flush=True)
        assert np.isfinite(err).all() and err.max() < tol, (sector, nr, nt, err)


@pytest.mark.parametrize("sector", [1, 2, 4])
@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_rotated_discs_in_pairs(sector, precision):
    """Discs of the sectors with the disc-centre rule (Sec. II.D) step two
    steps per launch too: below row 0 the ghost is row 0 with every
    direction turned by 4, for stage A's rows, for stage B's row behind the
    first block and for the edge cells' radial neighbours.  Against the
    oracle, as above."""
    tol = TOL64 if precision == P.PDBM_FP64 else 1e-4
    for nr, nt, nsteps in ((1, 17, 12), (5, 65, 13), (33, 17, 12), (12, 130, 9)):
        w = replace(_case(nr, nt, sector=sector, r_min=0.0), nsteps=nsteps)
        s = P.Solver(P.make_params(**w.params_kw(), precision=precision), P.make_ic(**w.ic_kw()))
        s.step(w.nsteps)
        F, _ = s.moments(check=False)
        o = O.Solver(O.make_params(**w.params_kw()))
        o.init_ic(**w.ic_kw())
        o.step(w.nsteps)
        R = o.fields()
        sc = _scales(R)
        err = np.array([np.abs(F[k] - R[k]).max() / sc[k] for k in range(6)])
        print(f"disc sector={sector} nr={nr} nt={nt} steps={nsteps} precision={precision}: max err {err.max():.2e}",
              flush=True)
        assert np.isfinite(err).all() and err.max() < tol, (sector, nr, nt, err)


@pytest.mark.parametrize("sector", [1, 3, 4])
def test_rotated_sector_pairs_equal_single_steps(sector):
    """A rotated sector (the half one as a disc) stepped two steps per launch
    equals the same steps taken one launch at a time (step(1) calls take the
    one-step kernel), to rounding."""
    w = _case(33, 65, sector=sector, r_min=0.0 if sector == 4 else 0.3)  # the half disc with its centre rule
    a = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP64), P.make_ic(**w.ic_kw()))
    b = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP64), P.make_ic(**w.ic_kw()))
    for _ in range(10):
        a.step(1)
    b.step(10)
    Fa, _ = a.moments(check=False)
    Fb, _ = b.moments(check=False)
    sc = _scales(Fa)
    err = np.array([np.abs(Fa[k] - Fb[k]).max() / sc[k] for k in range(6)])
    assert err.max() < 1e-13, (sector, err)
