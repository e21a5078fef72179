"""Seeded synthetic workloads: problem statements and initial states only.

This module holds no arithmetic of the method.  It describes each workload
as plain numbers (grid, domain, gas, reaction, initial two-region state,
noise seed, step count) that the GPU path and the CPU oracle both take as
input.  The initial states follow the two-region form of the paper's
experiments (Sec. III.B-D of arXiv:1308.0653): burnt, compressed gas inside
a radius, unburnt gas at rest outside, with a tiny uniform pressure noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    nr: int
    ntheta: int
    r_min: float
    r_max: float
    dt: float
    tau: float
    w1: float
    w2: float
    m: int
    n: int
    Q: float
    T_th: float
    r_split: float
    inner: tuple  # (rho, T, u_r, u_theta, lambda)
    outer: tuple
    p_noise: float
    seed: int
    nsteps: int
    sector: int = 8
    fp32: bool = False
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.nr * self.ntheta

    def params_kw(self) -> dict:
        return dict(nr=self.nr, ntheta=self.ntheta, r_min=self.r_min, r_max=self.r_max, dt=self.dt,
                    tau=self.tau, w1=self.w1, w2=self.w2, m=self.m, n=self.n, Q=self.Q, T_th=self.T_th,
                    sector=self.sector)

    def ic_kw(self) -> dict:
        return dict(r_split=self.r_split, inner=self.inner, outer=self.outer, p_noise=self.p_noise,
                    seed=self.seed)


def _state(rho, p, ur=0.0, ut=0.0, lam=0.0):
    """(rho, T, u_r, u_theta, lambda) from a (rho, p) specification, T = p/rho."""
    return (float(rho), float(p) / float(rho), float(ur), float(ut), float(lam))


# Temperature of burnt ignition gas where only its pressure is specified.  The
# D2V33 equilibrium turns strongly non-positive above T ~ 8 (the moment-matched
# weights F_k swing in sign) and the scheme then amplifies perturbations, so
# ignition regions given by pressure alone are put at T = 5 with rho = p / 5.
T_IGNITION = 5.0


def _ignition(p):
    return _state(float(p) / T_IGNITION, p, lam=1.0)


UNBURNT = _state(1.0, 1.0)

# Gas, reaction and relaxation shared by the single-solve workloads.
_GAS = dict(dt=1e-5, tau=2e-5, w1=2.0, w2=2.0, m=2, n=2, Q=1.0, T_th=1.1)


def small_fp64() -> Workload:
    """64 x 64 annulus r in [0.1, 1.0], 200 steps; ignition disc r < 0.2 of
    rho = 1.5, p = 20, burnt; unburnt gas rho = p = 1 at rest outside."""
    return Workload("annulus64_fp64", 64, 64, 0.1, 1.0, r_split=0.2, inner=_state(1.5, 20.0, lam=1.0),
                    outer=UNBURNT, p_noise=1e-6, seed=0, nsteps=200, **_GAS)


def outward_fp64() -> Workload:
    """Outward detonation, 1024 x 1024 on r in [0.05, 2.0], 2000 steps;
    ignition ring r < 0.1 of burnt gas at p = 30 (T = 5, rho = 6)."""
    return Workload("outward1024_fp64", 1024, 1024, 0.05, 2.0, r_split=0.1, inner=_ignition(30.0),
                    outer=UNBURNT, p_noise=1e-6, seed=0, nsteps=2000, **_GAS)


def outward_fp32() -> Workload:
    """The outward detonation with f stored and updated in float32."""
    return replace(outward_fp64(), name="outward1024_fp32", fp32=True)


def batch_sweep(count: int = 256, nsteps: int = 500) -> list[Workload]:
    """Independent solves of a parameter sweep (seed 1), float32.  Per solve,
    in this order: Nr ~ U{128..1024}, Ntheta ~ U{64..512}, w1, w2 ~
    U[0.5, 5], m, n ~ U{1, 2, 3}, ignition p ~ U[5, 50], tau ~ U[1e-5,
    1e-4].  Domain, ignition radius, ignition temperature and dt as the
    outward detonation; noise seed = solve index."""
    rng = np.random.default_rng(1)
    out = []
    for i in range(count):
        nr = int(rng.integers(128, 1025))
        nt = int(rng.integers(64, 513))
        w1, w2 = (float(x) for x in rng.uniform(0.5, 5.0, 2))
        m, n = (int(x) for x in rng.integers(1, 4, 2))
        p_ign = float(rng.uniform(5.0, 50.0))
        tau = float(rng.uniform(1e-5, 1e-4))
        out.append(Workload(f"sweep{i}", nr, nt, 0.05, 2.0, dt=1e-5, tau=tau, w1=w1, w2=w2, m=m, n=n, Q=1.0,
                            T_th=1.1, r_split=0.1, inner=_ignition(p_ign), outer=UNBURNT,
                            p_noise=1e-6, seed=i, nsteps=nsteps, fp32=True))
    return out


def _log_uniform(rng, lo, hi):
    return math.exp(rng.uniform(math.log(lo), math.log(hi)))


def serving_stream(count: int = 1000, rate: float = 1.0, seed: int = 2,
                   max_cells: int | None = None, max_steps: int | None = None):
    """Poisson arrivals (exponential gaps of mean 1/rate seconds) of solves
    with Nr ~ round(logU[128, 2048]), Ntheta ~ round(logU[64, 2048]), steps ~
    round(logU[200, 5000]) and the sweep's reaction parameters, float32.
    Returns a list of (arrival_time_s, Workload).  `max_cells` and
    `max_steps` cap the draws for short runs."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        nr = int(round(_log_uniform(rng, 128, 2048)))
        nt = int(round(_log_uniform(rng, 64, 2048)))
        steps = int(round(_log_uniform(rng, 200, 5000)))
        w1, w2 = (float(x) for x in rng.uniform(0.5, 5.0, 2))
        m, n = (int(x) for x in rng.integers(1, 4, 2))
        p_ign = float(rng.uniform(5.0, 50.0))
        tau = float(rng.uniform(1e-5, 1e-4))
        if max_cells is not None:
            while nr * nt > max_cells:
                nr, nt = max(2, nr // 2), max(1, nt // 2)
        if max_steps is not None:
            steps = min(steps, max_steps)
        out.append((t, Workload(f"req{i}", nr, nt, 0.05, 2.0, dt=1e-5, tau=tau, w1=w1, w2=w2, m=m, n=n, Q=1.0,
                                T_th=1.1, r_split=0.1, inner=_ignition(p_ign), outer=UNBURNT,
                                p_noise=1e-6, seed=1000 + i, nsteps=steps, fp32=True)))
    return out


def mean_work_serving(samples: int = 20000, seed: int = 12345) -> float:
    """Expected cell-updates per request of the serving stream (Monte Carlo
    over the same distributions)."""
    rng = np.random.default_rng(seed)
    nr = np.round(np.exp(rng.uniform(math.log(128), math.log(2048), samples)))
    nt = np.round(np.exp(rng.uniform(math.log(64), math.log(2048), samples)))
    st = np.round(np.exp(rng.uniform(math.log(200), math.log(5000), samples)))
    return float((nr * nt * st).mean())
