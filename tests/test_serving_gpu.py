"""Packed batches and the continuous-batching server on the GPU.

A solve's fields must be bitwise the same alone and in any mix (members
never read each other's data), its drift report equal to rounding, and each
result must match the CPU oracle."""
import time
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_1308_0653_amd import pdbm as P
from paper_1308_0653_amd import workloads as W

pytestmark = pytest.mark.gpu


def _params(w, precision, diag_every=0):
    return P.make_params(**w.params_kw(), precision=precision, diag_every=diag_every)


def _small_sweep(n, seed=0, nsteps=60):
    """A few solves with the sweep's parameter ranges on small grids."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nr, nt = int(rng.integers(24, 90)), int(rng.integers(20, 140))
        w = replace(W.batch_sweep(count=i + 1, nsteps=nsteps)[i], nr=nr, ntheta=nt)
        out.append(w)
    return out


def _oracle_fields(w, nsteps):
    o = O.Solver(O.make_params(**w.params_kw()))
    o.init_ic(**w.ic_kw())
    o.step(nsteps)
    return o.fields()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _field_errs(F, R):
    """Normwise error of each of the six fields; the velocity components share
    the scale max(|u_r|, |u_theta|, sqrt(T)), as u_theta can be near zero."""
    us = max(np.abs(R[1]).max(), np.abs(R[2]).max(), np.sqrt(np.abs(R[3]).max()))
    return [np.abs(F[k] - R[k]).max() / (us if k in (1, 2) else max(np.abs(R[k]).max(), 1e-300)) for k in range(6)]


@pytest.mark.parametrize("chunk", [0, 7])
def test_batch_members_match_single_solves_and_oracle(chunk):
    ws = _small_sweep(4, seed=1)
    params = [_params(w, P.PDBM_FP64, diag_every=5) for w in ws]
    ics = [P.make_ic(**w.ic_kw()) for w in ws]
    b = P.Batch(params, ics, chunk_steps=chunk)
    b.step(30)
    for i, w in enumerate(ws):
        assert b.step_count(i) == 30
        F, d = b.moments(i)
        # packed members and the solo solve both step in pairs, but with
        # chunks of 7 the pack's pairs and single steps fall elsewhere, and
        # the row blocks differ: equal to rounding
        solo = P.Solver(params[i], ics[i])
        solo.step(30)
        Fs, ds = solo.moments()
        errs = _field_errs(F, Fs)
        assert max(errs) <= 1e-12, (i, errs)
        for k in ("mass", "energy", "chem"):
            assert abs(d[k] - ds[k]) <= 1e-13 * abs(ds[k])
        R = _oracle_fields(w, 30)
        for k in (0, 3, 5):
            assert _rel(F[k], R[k]) < 1e-10, (i, k)


@pytest.mark.parametrize("precision", [P.PDBM_FP32, P.PDBM_FP64])
def test_batch_graph_replay_equals_plain_launches(precision):
    """Chunks replayed from the captured graph against plain launches, after
    every call: whole chunks, remainders run as plain launches in between,
    and the synchronising moments reads between the replays."""
    ws = _small_sweep(3, seed=2)
    params = [_params(w, precision, diag_every=4) for w in ws]
    ics = [P.make_ic(**w.ic_kw()) for w in ws]
    a = P.Batch(params, ics, chunk_steps=6)
    b = P.Batch(params, ics, chunk_steps=0)
    for n in (13, 6, 1, 12, 6, 18):  # whole chunks and remainders
        a.step(n)
        b.step(n)
        for i in range(len(ws)):
            Fa, da = a.moments(i)
            Fb, db = b.moments(i)
            assert np.array_equal(Fa, Fb), (n, i)
            assert da == db, (n, i)


def test_batch_member_alone_equals_in_mix_fp32():
    ws = _small_sweep(5, seed=3)
    params = [_params(w, P.PDBM_FP32) for w in ws]
    ics = [P.make_ic(**w.ic_kw()) for w in ws]
    mix = P.Batch(params, ics, chunk_steps=10)
    mix.step(40)
    for i in (0, 3):
        alone = P.Batch([params[i]], [ics[i]], chunk_steps=10)
        alone.step(40)
        Fm, dm = mix.moments(i)
        Fa, da = alone.moments(0)
        assert np.array_equal(Fm, Fa)
        assert dm == da


def _wait_all(srv, ids, timeout=60.0):
    assert srv.wait(timeout), srv.stats()
    return {rid: srv.poll(rid, fields=True) for rid in ids}


def test_server_results_equal_solo_runs():
    ws = _small_sweep(6, seed=4, nsteps=40)
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=3, chunk_steps=8)
    ids = []
    for k, w in enumerate(ws):
        prec = P.PDBM_FP64 if k % 2 else P.PDBM_FP32
        ids.append((srv.submit(_params(w, prec), P.make_ic(**w.ic_kw()), nsteps=w.nsteps + 7 * k,
                               keep_fields=True), w, prec, w.nsteps + 7 * k))
    res = _wait_all(srv, [i for i, *_ in ids])
    for rid, w, prec, n in ids:
        state, F, d = res[rid]
        assert state == P.PDBM_DONE
        solo = P.Batch([_params(w, prec)], [P.make_ic(**w.ic_kw())], chunk_steps=0)
        solo.step(n)
        Fs, ds = solo.moments(0)
        assert np.array_equal(F, Fs), rid
        t = srv.times(rid)
        assert 0 <= t[0] <= t[1] <= t[2]
    st = srv.stats()
    assert st["done"] == len(ws) and st["failed"] == 0 and st["queued"] == 0 and st["running"] == 0
    srv.close()


def test_server_admission_by_slots_and_memory():
    w0 = _small_sweep(1, seed=5, nsteps=30)[0]
    ws = [replace(w0, seed=k) for k in range(5)]  # same size, different noise
    p0 = _params(ws[0], P.PDBM_FP32)
    need = P.pdbm_state_bytes(p0)
    # memory for only one running solve at a time
    srv = P.Server(hbm_cap_bytes=need + need // 2, max_slots=8, chunk_steps=5)
    ids = [srv.submit(_params(w, P.PDBM_FP32), P.make_ic(**w.ic_kw()), nsteps=30) for w in ws]
    assert srv.wait(60.0)
    spans = sorted(tuple(srv.times(i)[1:]) for i in ids)
    for (a1, d1), (a2, d2) in zip(spans, spans[1:]):
        assert a2 >= d1 - 1e-9  # admitted only after the previous one left
    assert srv.stats()["done"] == len(ws)
    # and by slots: two at a time
    srv2 = P.Server(hbm_cap_bytes=8 << 30, max_slots=2, chunk_steps=5)
    ids = [srv2.submit(_params(w, P.PDBM_FP32), P.make_ic(**w.ic_kw()), nsteps=30) for w in ws]
    assert srv2.wait(60.0)
    spans = [tuple(srv2.times(i)[1:]) for i in ids]
    for t in np.linspace(0, max(d for _, d in spans), 200):
        assert sum(a <= t < d for a, d in spans) <= 2
    srv2.close()
    # a solve that can never fit is refused at submission
    small = P.Server(hbm_cap_bytes=1 << 20, max_slots=2, chunk_steps=5)
    with pytest.raises(P.PdbmError) as e:
        small.submit(p0, P.make_ic(**ws[0].ic_kw()), 10)
    assert e.value.code == P.PDBM_ENOMEM
    with pytest.raises(P.PdbmError) as e:
        small.poll(12345)
    assert e.value.code == P.PDBM_ENOENT
    small.close()
    srv.close()


def test_server_failure_is_isolated():
    """A solve whose state blows up (burnt gas at T = 20 is outside the
    model's stable range) fails alone; the others are bitwise unaffected."""
    good = _small_sweep(3, seed=6, nsteps=60)
    bad = W.Workload("unstable", 48, 1024, 0.05, 0.2, dt=1e-5, tau=2e-5, w1=2.0, w2=2.0, m=2, n=2, Q=1.0,
                     T_th=1.1, r_split=0.1, inner=(1.5, 20.0, 0.0, 0.0, 1.0), outer=(1.0, 1.0, 0.0, 0.0, 0.0),
                     p_noise=1e-6, seed=0, nsteps=100)
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=8, chunk_steps=10)
    gid = [srv.submit(_params(w, P.PDBM_FP32), P.make_ic(**w.ic_kw()), w.nsteps, keep_fields=True) for w in good]
    bid = srv.submit(_params(bad, P.PDBM_FP32), P.make_ic(**bad.ic_kw()), bad.nsteps)
    assert srv.wait(60.0)
    state, _, d = srv.poll(bid)
    assert state == P.PDBM_FAILED and (d["n_nonfinite"] > 0 or d["n_nonphys"] > 0)
    for rid, w in zip(gid, good):
        state, F, _ = srv.poll(rid, fields=True)
        assert state == P.PDBM_DONE
        solo = P.Batch([_params(w, P.PDBM_FP32)], [P.make_ic(**w.ic_kw())])
        solo.step(w.nsteps)
        assert np.array_equal(F, solo.moments(0)[0])
    assert srv.stats()["failed"] == 1
    srv.close()


def test_stream_request_that_turns_nonphysical_is_reported_failed():
    """Request 138 of the 1000-request serving stream (430 x 1952, m = 2,
    n = 3) is one the model cannot carry: the oracle's own run has no bad
    cell at step 350 and non-finite and non-physical cells at step 400
    (tests/golden/unstable_request.json, written from the oracle alone).
    The float64 path reaches the same verdict at both steps, and the server,
    serving it in float32 beside a stable request of the stream, reports it
    failed and the other done."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "unstable_request.json")))
    stream = W.serving_stream(count=1000, rate=30.0)
    w = stream[g["index"]][1]
    assert (w.nr, w.ntheta, w.nsteps, w.m, w.n) == (g["nr"], g["ntheta"], g["nsteps"], g["m"], g["n"])
    s = P.Solver(P.make_params(**w.params_kw(), precision=P.PDBM_FP64, diag_every=50), P.make_ic(**w.ic_kw()))
    s.step(401)  # the record of step s holds the state the step starts from
    hist = {r["step"]: r for r in s.diag_history()}
    s.close()
    for step in (350, 400):
        oracle_bad = sum(g["oracle_bad_cells"][str(step)].values()) > 0
        gpu_bad = hist[step]["n_nonfinite"] + hist[step]["n_nonphys"] > 0
        print("step", step, "oracle bad", oracle_bad, "float64 path", hist[step], flush=True)
        assert gpu_bad == oracle_bad, step
    ok = stream[1][1]
    srv = P.Server(hbm_cap_bytes=50 * 10**9, max_slots=8, chunk_steps=24)
    bid = srv.submit(_params(w, P.PDBM_FP32), P.make_ic(**w.ic_kw()), w.nsteps)
    oid = srv.submit(_params(ok, P.PDBM_FP32), P.make_ic(**ok.ic_kw()), ok.nsteps)
    assert srv.wait(120.0)
    state, _, d = srv.poll(bid)
    assert state == P.PDBM_FAILED and d["n_nonfinite"] + d["n_nonphys"] > 0
    assert srv.poll(oid)[0] == P.PDBM_DONE
    srv.close()


def test_server_shutdown_with_pending_work():
    w = _small_sweep(1, seed=7)[0]
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=1, chunk_steps=5)
    ids = [srv.submit(_params(w, P.PDBM_FP32), P.make_ic(**w.ic_kw()), 100000) for _ in range(3)]
    time.sleep(0.2)
    t0 = time.perf_counter()
    srv.close()  # must not wait for the 100000-step solves
    assert time.perf_counter() - t0 < 10.0
    assert ids


def test_server_admits_arrivals_while_others_run():
    """Continuous batching, not a queue: a short request that arrives while
    two long ones are on the GPU is admitted at the next chunk boundary and
    finishes first, while they keep running."""
    w = _small_sweep(1, seed=8)[0]
    p = _params(w, P.PDBM_FP32)
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=4, chunk_steps=10)
    long_ids = [srv.submit(p, P.make_ic(**replace(w, seed=k).ic_kw()), 20000) for k in range(2)]
    t0 = time.perf_counter()
    while srv.stats()["running"] < 2:
        assert time.perf_counter() - t0 < 30.0
        time.sleep(0.005)
    short = srv.submit(p, P.make_ic(**w.ic_kw()), 50, keep_fields=True)
    assert srv.wait(120.0)
    ts, tl = srv.times(short), [srv.times(i) for i in long_ids]
    for t in tl:
        assert ts[1] > t[1]  # admitted after the long ones started ...
        assert ts[2] < t[2]  # ... and done before they were
    state, F, _ = srv.poll(short, fields=True)
    assert state == P.PDBM_DONE
    solo = P.Batch([p], [P.make_ic(**w.ic_kw())])
    solo.step(50)
    assert np.array_equal(F, solo.moments(0)[0])
    srv.close()


def test_server_submit_from_many_threads():
    import threading
    ws = _small_sweep(4, seed=9, nsteps=30)
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=3, chunk_steps=5)
    ids, errors = [], []
    lock = threading.Lock()

    def client(k):
        try:
            for j in range(4):
                w = ws[(k + j) % len(ws)]
                rid = srv.submit(_params(w, P.PDBM_FP32), P.make_ic(**w.ic_kw()), w.nsteps + j)
                with lock:
                    ids.append(rid)
        except Exception as e:  # pragma: no cover - reported below
            errors.append(e)

    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors
    assert srv.wait(60.0)
    assert len(set(ids)) == 16
    for rid in ids:
        assert srv.poll(rid)[0] == P.PDBM_DONE
    st = srv.stats()
    assert st["submitted"] == 16 and st["done"] == 16
    srv.close()


def test_zero_steps_change_nothing():
    """Zero steps are a no-op for a solve and a pack, and a request for zero
    steps comes back DONE with the initial fields; waiting on a server with
    no requests returns at once."""
    w = _small_sweep(1, seed=10)[0]
    for prec in (P.PDBM_FP64, P.PDBM_FP32):
        s = P.Solver(_params(w, prec), P.make_ic(**w.ic_kw()))
        F0, _ = s.moments()
        f0, l0 = s.read_f()
        s.step(0)
        assert s.step_count == 0
        f1, l1 = s.read_f()
        assert np.array_equal(f0, f1) and np.array_equal(l0, l1)
        b = P.Batch([_params(w, prec)], [P.make_ic(**w.ic_kw())], chunk_steps=5)
        b.step(0)
        assert b.step_count(0) == 0
        assert np.array_equal(b.moments(0)[0], F0)
        srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=2, chunk_steps=5)
        t0 = time.perf_counter()
        assert srv.wait(10.0)
        assert time.perf_counter() - t0 < 1.0
        rid = srv.submit(_params(w, prec), P.make_ic(**w.ic_kw()), 0, keep_fields=True)
        assert srv.wait(60.0)
        state, F, _ = srv.poll(rid, fields=True)
        assert state == P.PDBM_DONE
        assert np.array_equal(F, F0)
        assert srv.stats()["done"] == 1
        srv.close()


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_packed_pairs_with_odd_counts(precision):
    """Packs step in pairs (two steps per launch), with a launch of single
    steps closing a chunk of odd length and a single step for a member with
    one step left.  Requests of 31, 24, 17 and 30 steps in chunks of 7 finish
    inside chunks, and the pack is rebuilt as they leave, so each member's
    buffer parity is carried across rebuilds.  The results agree with solo
    solves (pairs from step 0) to rounding and with the oracle."""
    ws = _small_sweep(4, seed=11)
    counts = [31, 24, 17, 30]
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=4, chunk_steps=7)
    ids = [srv.submit(_params(w, precision, diag_every=5), P.make_ic(**w.ic_kw()), n, keep_fields=True)
           for w, n in zip(ws, counts)]
    assert srv.wait(60.0)
    tol = 1e-12 if precision == P.PDBM_FP64 else 1e-5
    for rid, w, n in zip(ids, ws, counts):
        state, F, d = srv.poll(rid, fields=True)
        assert state == P.PDBM_DONE
        solo = P.Solver(_params(w, precision, diag_every=5), P.make_ic(**w.ic_kw()))
        solo.step(n)
        Fs, ds = solo.moments()
        errs = _field_errs(F, Fs)
        print(f"n={n} prec={precision}: max rel {max(errs):.2e}", flush=True)
        assert max(errs) <= tol, (n, errs)
        R = _oracle_fields(w, n)
        for k in (0, 3, 5):
            assert _rel(F[k], R[k]) < (1e-10 if precision == P.PDBM_FP64 else 1e-4), (n, k)
    srv.close()


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_single_columns_join_a_pack_stepping_in_pairs(precision):
    """Single-column solves join a pack whose members have been stepping in
    pairs (chunks of 6 steps are 3 pairs, so that parity changes with every
    chunk): the wider grids keep stepping in pairs, the columns take
    launches of up to 8 steps of their own kernel in the same chunks, and
    the pack goes on with pairs alone when they leave.  Every result agrees
    with its solo solve to rounding and with the oracle."""
    ws = _small_sweep(2, seed=12)
    sec = replace(W.small_fp64(), name="column", nr=40, ntheta=1, r_min=0.5, dt=1e-4, tau=4e-4, r_split=0.7)
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=4, chunk_steps=6)
    n_long, n_sec = 601, 31
    long_ids = [srv.submit(_params(w, precision), P.make_ic(**w.ic_kw()), n_long, keep_fields=True) for w in ws]
    sec_ids = []
    t0 = time.perf_counter()
    for launched in (6, 18):
        while srv.stats()["steps_launched"] < launched:
            assert time.perf_counter() - t0 < 30.0
            time.sleep(0.0005)
        sec_ids.append(srv.submit(_params(sec, precision), P.make_ic(**sec.ic_kw()), n_sec, keep_fields=True))
    assert srv.wait(120.0)
    for sid in sec_ids:  # the single-column solves ran while the long ones did
        assert max(srv.times(i)[1] for i in long_ids) < srv.times(sid)[1] < min(srv.times(i)[2] for i in long_ids)
    tol = 1e-12 if precision == P.PDBM_FP64 else 1e-4
    otol = 1e-10 if precision == P.PDBM_FP64 else 1e-4
    for rid, w, n in [(i, w, n_long) for i, w in zip(long_ids, ws)] + [(i, sec, n_sec) for i in sec_ids]:
        state, F, _ = srv.poll(rid, fields=True)
        assert state == P.PDBM_DONE
        solo = P.Solver(_params(w, precision), P.make_ic(**w.ic_kw()))
        solo.step(n)
        errs = _field_errs(F, solo.moments()[0])
        print(f"{w.name} n={n} prec={precision}: max rel {max(errs):.2e}", flush=True)
        assert max(errs) <= tol, (w.name, errs)
        errs = _field_errs(F, _oracle_fields(w, n))
        assert max(errs[k] for k in (0, 3, 5)) <= otol, (w.name, errs)
    srv.close()


@pytest.mark.parametrize("precision", [P.PDBM_FP64, P.PDBM_FP32])
def test_packs_with_rotated_sectors_step_in_pairs(precision):
    """A pack holding rotated sectors, an annular one and a half disc with
    its centre rule, beside full annuli, still steps in pairs (the rotated
    variant of the two-step kernel takes every member).  Odd counts in
    chunks of 7; every result agrees with its solo solve to rounding and
    with the oracle."""
    ws = _small_sweep(2, seed=13)
    ws.append(replace(W.small_fp64(), name="sector3", nr=24, ntheta=24, sector=3, r_min=0.5, dt=1e-4, tau=4e-4,
                      r_split=0.7))
    ws.append(W.Workload("halfdisc", 40, 8, 0.0, 1.0, dt=2e-4, tau=2e-4, w1=1.0, w2=50.0, m=1, n=1, Q=1.0,
                         T_th=1.1, r_split=0.3, inner=(1.5, 1.55556, 0.666667, 0.0, 1.0),
                         outer=(1.0, 1.0, 0.0, 0.0, 0.0), p_noise=1e-6, seed=3, nsteps=40, sector=4))
    counts = [33, 26, 29, 40]
    srv = P.Server(hbm_cap_bytes=8 << 30, max_slots=4, chunk_steps=7)
    ids = [srv.submit(_params(w, precision, diag_every=5), P.make_ic(**w.ic_kw()), n, keep_fields=True)
           for w, n in zip(ws, counts)]
    assert srv.wait(60.0)
    tol = 1e-12 if precision == P.PDBM_FP64 else 1e-5
    otol = 1e-10 if precision == P.PDBM_FP64 else 1e-4
    for rid, w, n in zip(ids, ws, counts):
        state, F, _ = srv.poll(rid, fields=True)
        assert state == P.PDBM_DONE
        solo = P.Solver(_params(w, precision, diag_every=5), P.make_ic(**w.ic_kw()))
        solo.step(n)
        errs = _field_errs(F, solo.moments()[0])
        print(f"{w.name} n={n} prec={precision}: max rel {max(errs):.2e}", flush=True)
        assert max(errs) <= tol, (w.name, errs)
        errs = _field_errs(F, _oracle_fields(w, n))
        assert max(errs[k] for k in (0, 3, 5)) <= otol, (w.name, errs)
    srv.close()
