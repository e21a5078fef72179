"""The packed sweep and the serving stream at their full sizes.

- The 256-solve float32 sweep (seed 1; grids up to 1021 x 512, 4.3e7 cells)
  packed into one set of launches, as the benchmark runs it (two steps per
  launch, graph chunks of 50): four members, among them the one of most
  cells (986 x 462) and the one of fewest (141 x 84), are bitwise equal to
  the same solve packed alone, and within the float32 bound of the oracle.
- The Poisson serving stream (seed 2): its request of most cells, 2015 x
  1935 for 4542 steps, served while other requests of the stream come and
  go, is bitwise equal to the same request run alone.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_0653_amd import pdbm as P
from paper_1308_0653_amd import workloads as W

pytestmark = pytest.mark.gpu


def _params(w, precision=P.PDBM_FP32):
    return P.make_params(**w.params_kw(), precision=precision)


def _errs(F, R):
    us = max(np.abs(R[1]).max(), np.abs(R[2]).max(), np.sqrt(np.abs(R[3]).max()))
    return [np.abs(F[k] - R[k]).max() / (us if k in (1, 2) else max(np.abs(R[k]).max(), 1e-300)) for k in range(6)]


def test_full_sweep_pack_members_equal_solo_and_oracle():
    ws = W.batch_sweep(count=256, nsteps=500)
    cells = np.array([w.cells for w in ws])
    picks = [int(np.argmax(cells)), int(np.argmin(cells)), 0, 255]
    assert (ws[picks[0]].nr, ws[picks[0]].ntheta) == (986, 462) and cells.sum() == 43412078
    params = [_params(w) for w in ws]
    ics = [P.make_ic(**w.ic_kw()) for w in ws]
    nsteps = 100  # two graph chunks
    pack = P.Batch(params, ics, chunk_steps=50)
    pack.step(nsteps)
    print("pack of", len(ws), "stepped", nsteps, flush=True)
    for i in picks:
        Fp, dp = pack.moments(i)
        alone = P.Batch([params[i]], [ics[i]], chunk_steps=50)
        alone.step(nsteps)
        Fa, da = alone.moments(0)
        alone.close()
        assert np.array_equal(Fp, Fa), i
        assert dp == da, i
        w = ws[i]
        o = O.Solver(O.make_params(**w.params_kw()))
        o.init_ic(**w.ic_kw())
        o.step(nsteps)
        err = _errs(Fp, o.fields())
        print(f"member {i} {w.nr}x{w.ntheta}: vs oracle", [f"{e:.1e}" for e in err], flush=True)
        for k in (0, 3, 5):
            assert err[k] <= 1e-4, (i, k, err)
    pack.close()


def test_largest_served_request_equals_its_solo_run():
    stream = W.serving_stream(count=1000, rate=30.0)
    k_big = int(np.argmax([w.cells for _, w in stream]))
    big = stream[k_big][1]
    assert big.cells >= 1024 * 1024 and (big.nr, big.ntheta, big.nsteps) == (2015, 1935, 4542)
    others = [w for _, w in stream[:12] if w.cells <= 600_000]
    srv = P.Server(hbm_cap_bytes=200 * 10**9, max_slots=16, chunk_steps=24)
    ids = [srv.submit(_params(w), P.make_ic(**w.ic_kw()), min(w.nsteps, 600)) for w in others[:4]]
    bid = srv.submit(_params(big), P.make_ic(**big.ic_kw()), big.nsteps, keep_fields=True)
    ids += [srv.submit(_params(w), P.make_ic(**w.ic_kw()), min(w.nsteps, 600)) for w in others[4:]]
    assert srv.wait(300.0), srv.stats()
    state, F, d = srv.poll(bid, fields=True)
    assert state == P.PDBM_DONE
    assert all(srv.poll(i)[0] == P.PDBM_DONE for i in ids)
    t_big = srv.times(bid)
    # it shared the GPU: some other request was running while it ran
    assert any(srv.times(i)[1] < t_big[2] and srv.times(i)[2] > t_big[1] for i in ids)
    srv.close()
    alone = P.Batch([_params(big)], [P.make_ic(**big.ic_kw())], chunk_steps=24)
    alone.step(big.nsteps)
    Fa, da = alone.moments(0)
    assert np.array_equal(F, Fa)
    for key in ("mass", "energy", "chem", "n_nonfinite", "n_nonphys"):
        assert d[key] == da[key], key
