"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than the oracle itself:
an exact rational solution, a moment identity, a closed form, a numerical
ODE solution, the exact transport solution, a symmetry of the scheme, values
printed in the paper, or an extended-precision build.  Every plausible slip
(a dropped term, a wrong sign or index, a transposed operand) breaks at least
one of them.  Citations refer to Lin, Xu, Zhang, Li, arXiv:1308.0653.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
SPEEDS = GOLD["speeds"]["value"]


def _k_of(q):
    return 0 if q == 0 else 1 + (q - 1) // 8


def _i_of(q):
    return 0 if q == 0 else (q - 1) % 8


def _q_of(k, i):
    return 0 if k == 0 else 1 + 8 * (k - 1) + i


# ---------------------------------------------------------------- P1 ------
def _exact_weights(T: Fraction):
    """Solve sum_k 8 F_k v_k^(2n) = 2^n n! T^n (n = 1..4) exactly with
    rationals: the isotropic Gaussian moments that the weights of Sec. II.B
    are built to reproduce.  F_0 = 1 - 8 sum F_k."""
    x = [Fraction(v) ** 2 for v in SPEEDS[1:]]
    A = [[8 * xk ** n for xk in x] for n in range(1, 5)]
    b = [2 ** n * math.factorial(n) * T ** n for n in range(1, 5)]
    n = 4
    for c in range(n):  # Gauss-Jordan, exact
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        b[c], b[piv] = b[piv], b[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                fac = A[r][c] / A[c][c]
                A[r] = [A[r][j] - fac * A[c][j] for j in range(n)]
                b[r] -= fac * b[c]
    F = [b[i] / A[i][i] for i in range(n)]
    return [1 - 8 * sum(F)] + F


@pytest.mark.parametrize("T", [Fraction(3, 10), Fraction(1), Fraction(12, 5), Fraction(133, 10), Fraction(50)])
def test_P1_weights_match_exact_moment_inversion(T):
    exact = [float(v) for v in _exact_weights(T)]
    got = O.weights(float(T))
    scale = max(abs(v) for v in exact)
    for k in range(5):
        assert abs(got[k] - exact[k]) <= 1e-13 * scale + 1e-13 * abs(exact[k]), (k, got[k], exact[k])


def test_P1_weights_moment_constraints():
    for T in np.linspace(0.3, 50, 37):
        F = O.weights(T)
        for n in range(1, 5):
            lhs = sum(8 * F[k] * SPEEDS[k] ** (2 * n) for k in range(1, 5))
            rhs = 2 ** n * math.factorial(n) * T ** n
            assert abs(lhs - rhs) <= 1e-12 * rhs
        assert abs(F[0] + 8 * F[1:].sum() - 1) < 1e-15


# ---------------------------------------------------------------- P2 ------
def _central(feq, theta, ur, ut):
    vr, vt = O.velocities(theta)
    c = np.stack([vr - ur, vt - ut])
    return vr, vt, c


@pytest.mark.parametrize("seed", range(6))
def test_P2_equilibrium_moments(seed):
    """Sec. II.B defines rho, u, T as moments of f; f^eq must return them and
    match a 2-D Maxwellian's central moments up to 4th order (the ones the
    non-equilibrium measures of Sec. II.E rely on: M3*(f^eq) = 0,
    M31*(f^eq) = 0)."""
    rng = np.random.default_rng(seed)
    rho, T = rng.uniform(0.5, 3.0), rng.uniform(0.5, 30.0)
    ur, ut = rng.uniform(-1.4, 1.4, 2)
    theta = rng.uniform(0, 2 * np.pi)
    feq = O.equilibrium(rho, ur, ut, T, theta)
    vr, vt, c = _central(feq, theta, ur, ut)
    s = T + ur * ur + ut * ut  # velocity scale squared
    tol = 1e-12
    assert abs(feq.sum() - rho) <= tol * rho
    assert abs((feq * vr).sum() - rho * ur) <= tol * rho * math.sqrt(s)
    assert abs((feq * vt).sum() - rho * ut) <= tol * rho * math.sqrt(s)
    assert abs(0.5 * (feq * (c * c).sum(0)).sum() - rho * T) <= tol * rho * s
    M2 = np.einsum("q,aq,bq->ab", feq, c, c)
    assert np.abs(M2 - rho * T * np.eye(2)).max() <= tol * rho * s
    M3 = np.einsum("q,aq,bq,cq->abc", feq, c, c, c)
    assert np.abs(M3).max() <= tol * rho * s ** 1.5
    c2 = (c * c).sum(0)
    M31 = 0.5 * np.einsum("q,q,aq->a", feq, c2, c)
    assert np.abs(M31).max() <= tol * rho * s ** 1.5
    M42 = 0.5 * np.einsum("q,q,aq,bq->ab", feq, c2, c, c)
    assert np.abs(M42 - 2 * rho * T * T * np.eye(2)).max() <= 1e-11 * rho * s * s
    # energy identity of the model (gamma = 2): sum 1/2 f v^2 = rho T + rho u^2/2
    e = 0.5 * (feq * (vr * vr + vt * vt)).sum()
    assert abs(e - (rho * T + 0.5 * rho * (ur * ur + ut * ut))) <= tol * rho * s


def test_P2_moments_roundtrip_and_frame():
    """The oracle's moments of f^eq give back (rho, u_r, u_theta, T), and the
    velocity components are the polar components of the fixed Cartesian
    directions i pi/4 (Sec. II.B)."""
    theta = 0.7
    vr, vt = O.velocities(theta)
    for q in range(1, 33):
        k, i = _k_of(q), _i_of(q)
        vx, vy = SPEEDS[k] * math.cos(i * math.pi / 4), SPEEDS[k] * math.sin(i * math.pi / 4)
        # e_r = (cos th, sin th), e_th = (-sin th, cos th)
        assert abs(vr[q] - (vx * math.cos(theta) + vy * math.sin(theta))) < 1e-13
        assert abs(vt[q] - (-vx * math.sin(theta) + vy * math.cos(theta))) < 1e-13
    m = O.moments(O.equilibrium(1.3, 0.4, -0.25, 2.2, theta), theta)
    np.testing.assert_allclose(m, [1.3, 0.4, -0.25, 2.2], rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------- P3 ------
def _noneq_f(rng, theta):
    rho, T = rng.uniform(0.8, 2.0), rng.uniform(1.5, 8.0)
    ur, ut = rng.uniform(-0.8, 0.8, 2)
    feq = O.equilibrium(rho, ur, ut, T, theta)
    return feq * (1 + 0.05 * rng.uniform(-1, 1, 33))


@pytest.mark.parametrize("seed", range(5))
def test_P3_collision_conserves_and_heats_by_QR(seed):
    """Sec. II.A: the chemical term changes neither mass nor momentum and adds
    rho Q R(lambda) to the energy; BGK relaxation conserves all three.  Over
    one step the collision must therefore give d(rho)=0, d(rho u)=0,
    d(E_total) = rho Q R dt exactly (up to rounding)."""
    rng = np.random.default_rng(100 + seed)
    theta = rng.uniform(0, 2 * np.pi)
    f = _noneq_f(rng, theta)
    p = O.make_params(4, 4, 0.1, 1.0, dt=1e-4, tau=2e-4, w1=rng.uniform(0.5, 5), w2=rng.uniform(0.5, 5),
                      m=int(rng.integers(1, 4)), n=int(rng.integers(1, 4)), Q=rng.uniform(0.5, 2.0), T_th=1.1)
    lam = rng.uniform(0.05, 0.95)
    out, info = O.collide(p, f, lam, theta)
    vr, vt = O.velocities(theta)
    rho, T = info[0], info[3]
    assert info[6] == 1.0  # T > T_th: reacting
    P = rho * T
    R = p.w1 * P ** p.m * (1 - lam) + p.w2 * P ** p.n * lam * (1 - lam)
    assert abs(out.sum() - f.sum()) <= 1e-13 * rho
    assert abs((out * vr).sum() - (f * vr).sum()) <= 1e-12 * rho
    assert abs((out * vt).sum() - (f * vt).sum()) <= 1e-12 * rho
    e0 = 0.5 * (f * (vr * vr + vt * vt)).sum()
    e1 = 0.5 * (out * (vr * vr + vt * vt)).sum()
    dE = rho * p.Q * R * p.dt
    assert abs((e1 - e0) - dE) <= 1e-12 * e0 + 1e-10 * abs(dE)
    # the rate the oracle used is Cochran's
    np.testing.assert_allclose(info[4], p.w1 * P ** p.m, rtol=1e-14)
    np.testing.assert_allclose(info[5], p.w2 * P ** p.n, rtol=1e-14)


def test_P3_no_reaction_at_or_below_threshold():
    """Sec. III.A: T > T_th is necessary for the reaction."""
    theta = 0.3
    p = O.make_params(4, 4, 0.1, 1.0, dt=1e-4, tau=2e-4, w1=3, w2=3, m=1, n=1, Q=1.0, T_th=1.1)
    f = O.equilibrium(1.0, 0.0, 0.0, 1.0, theta)
    out, info = O.collide(p, f, 0.3, theta)
    assert info[6] == 0.0
    np.testing.assert_allclose(out, f, rtol=1e-14, atol=1e-18)


# ---------------------------------------------------------------- P4 ------
@pytest.mark.parametrize("ux,uy,T", [(0.0, 0.0, 1.0), (0.35, -0.2, 1.0), (0.6, 0.45, 1.05)])
def test_P4_uniform_state_stays_uniform(ux, uy, T):
    """A state uniform in the Cartesian sense (same rho, T, u_x, u_y in every
    cell; unreactive since T <= T_th) has f_ki equal in every cell, so every
    upwind difference vanishes and the state is steady, including at the
    zero-gradient radial boundaries."""
    nr, nt = 6, 16
    p = O.make_params(nr, nt, 0.2, 1.0, dt=2e-4, tau=1e-3, w1=2, w2=2, m=2, n=2, Q=1.0, T_th=1.1)
    s = O.Solver(p)
    dr, dth = 0.8 / nr, 2 * np.pi / nt
    th = (np.arange(nt) + 0.5) * dth
    fields = np.zeros((5, nr, nt))
    fields[0] = 1.2
    fields[1] = T
    fields[2] = ux * np.cos(th) + uy * np.sin(th)
    fields[3] = -ux * np.sin(th) + uy * np.cos(th)
    fields[4] = 0.25
    s.init_fields(fields)
    f0, l0 = s.get_state()
    s.step(20)
    f1, l1 = s.get_state()
    np.testing.assert_allclose(f1, f0, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(l1, l0, rtol=0, atol=1e-13)
    # and f_ki is indeed the same in every cell (Cartesian-uniform)
    np.testing.assert_allclose(f0, np.broadcast_to(f0[0, 0], f0.shape), rtol=1e-12, atol=1e-16)


# ---------------------------------------------------------------- P5 ------
def test_P5_pure_relaxation_is_exponential():
    """With no reaction and no gradients the LB evolution equation of
    Sec. II.C reduces to f(n dt) = f^eq + (f0 - f^eq) exp(-n dt / tau), with
    f^eq fixed because collisions conserve rho, u, T."""
    rng = np.random.default_rng(7)
    nr, nt = 4, 8
    p = O.make_params(nr, nt, 0.5, 1.0, dt=1e-5, tau=3e-5, w1=0, w2=0, m=1, n=1, Q=0.0, T_th=1.1)
    # A uniform non-equilibrium f at rest: only f_{k,i} symmetric under the
    # direction set keeps cells equal; use the same f in every cell with u=0
    # directions chosen so that the state is Cartesian-uniform.
    feq = O.equilibrium(1.1, 0.0, 0.0, 1.7, 0.0)
    pert = 0.03 * rng.uniform(-1, 1, 33)
    f0 = feq * (1 + pert)
    # make the perturbation carry no mass, momentum or energy so f^eq is that of feq
    vr, vt = O.velocities(0.0)
    Bm = np.stack([np.ones(33), vr, vt, 0.5 * (vr * vr + vt * vt)])
    d = f0 - feq
    d -= Bm.T @ np.linalg.lstsq(Bm.T, d, rcond=None)[0]
    f0 = feq + d
    s = O.Solver(p)
    s.set_state(np.broadcast_to(f0, (nr, nt, 33)).copy(), np.zeros((nr, nt)))
    n = 25
    s.step(n)
    f, _ = s.get_state()
    expect = feq + (f0 - feq) * math.exp(-n * p.dt / p.tau)
    np.testing.assert_allclose(f[2, 3], expect, rtol=1e-11, atol=1e-16)


# ---------------------------------------------------------------- P6 ------
def _ode_lambda(lam0, a, b, t):
    sol = solve_ivp(lambda _t, y: [(1 - y[0]) * (a + b * y[0])], (0, t), [lam0],
                    method="DOP853", rtol=1e-13, atol=1e-16)
    return sol.y[0, -1]


@pytest.mark.parametrize("lam0,a,b,dt", [(0.5, 1.0, 3.0, 0.3), (0.0, 40.0, 7.0, 1e-3), (0.2, 0.3, 900.0, 2e-3),
                                         (0.97, 5.0, 5.0, 1e-2), (0.1, 0.0, 4.0, 0.5)])
def test_P6_cochran_closed_form_solves_the_rate_equation(lam0, a, b, dt):
    """Sec. III.A: the lambda update integrates d lambda/dt = a(1-lambda) +
    b lambda(1-lambda) exactly over dt at frozen a, b.  Checked against an
    independent high-order ODE solution, and the semigroup property (two
    half steps = one step) that any exact flow has."""
    got = O.cochran(lam0, a, b, dt)
    assert abs(got - _ode_lambda(lam0, a, b, dt)) < 1e-11
    half = O.cochran(O.cochran(lam0, a, b, dt / 2), a, b, dt / 2)
    assert abs(half - got) < 1e-14
    assert abs(O.cochran(lam0, a, b, 0.0) - lam0) < 1e-15


def test_P6_fixed_pressure_cell_follows_logistic():
    """Reaction-only uniform cell at rest with Q = 0: P stays fixed, and
    lambda after n steps is the exact solution of Cochran's law at t = n dt."""
    nr, nt = 3, 8
    w1, w2, m, n = 2.0, 3.0, 2, 1
    p = O.make_params(nr, nt, 0.5, 1.0, dt=1e-3, tau=2e-3, w1=w1, w2=w2, m=m, n=n, Q=0.0, T_th=1.1)
    s = O.Solver(p)
    rho, T, lam0 = 1.2, 1.5, 0.05
    s.init_ic(0.0, [rho, T, 0, 0, lam0], [rho, T, 0, 0, lam0])
    P = rho * T
    nsteps = 60
    s.step(nsteps)
    F = s.fields()
    expect = _ode_lambda(lam0, w1 * P ** m, w2 * P ** n, nsteps * p.dt)
    assert np.abs(F[5] - expect).max() < 1e-11
    assert np.abs(F[4] - P).max() < 1e-12


def test_P6_heat_release_recurrence():
    """With Q != 0 a uniform cell at rest heats by exactly Q R dt per step
    (energy gain rho Q R dt at fixed rho, u), while lambda advances by the
    exact solution over dt at the current a, b."""
    nr, nt = 3, 8
    w1, w2, m, n, Q, dt = 1.5, 2.5, 1, 2, 0.8, 2e-3
    p = O.make_params(nr, nt, 0.5, 1.0, dt=dt, tau=3e-3, w1=w1, w2=w2, m=m, n=n, Q=Q, T_th=1.1)
    s = O.Solver(p)
    rho, T, lam = 1.1, 1.3, 0.1
    s.init_ic(0.0, [rho, T, 0, 0, lam], [rho, T, 0, 0, lam])
    for _ in range(15):
        P = rho * T
        a, b = w1 * P ** m, w2 * P ** n
        R = a * (1 - lam) + b * lam * (1 - lam)
        T = T + Q * R * dt
        lam = _ode_lambda(lam, a, b, dt)
    s.step(15)
    F = s.fields()
    assert np.abs(F[3] - T).max() < 1e-11 * T
    assert np.abs(F[5] - lam).max() < 1e-10


# ---------------------------------------------------------------- P7 ------
def _advect_params(nr, nt, r0, r1, dt):
    # tau = inf: exp(-dt/tau) = 1, pure free streaming; Q = 0, no reaction
    return O.make_params(nr, nt, r0, r1, dt=dt, tau=float("inf"), w1=0, w2=0, m=1, n=1, Q=0.0, T_th=1e9)


def test_P7_donor_cell_is_monotone():
    """First-order upwind (donor cell) with |C_r| + |C_theta| <= 1 writes each
    new value as a convex combination of the cell and its upwind neighbours:
    it never leaves the range of the stencil.  Taking the downwind side, or
    adding the flux instead of subtracting it, breaks this."""
    rng = np.random.default_rng(3)
    nr, nt = 10, 24
    p = _advect_params(nr, nt, 0.5, 1.0, dt=2.5e-3)  # max |C_r|+|C_theta| = 0.86
    s = O.Solver(p)
    # random positive f around an equilibrium (so rounding in f^eq + (f - f^eq)
    # stays at the size of f itself)
    base = O.equilibrium(1.0, 0.0, 0.0, 2.0, 0.0)
    f0 = base * rng.uniform(0.5, 1.5, (nr, nt, 33))
    s.set_state(f0, np.zeros((nr, nt)))
    s.step(1)
    f1, _ = s.get_state()
    tol = 1e-13 * np.abs(base)
    pad = np.pad(f0, ((1, 1), (0, 0), (0, 0)), mode="edge")
    pad = np.concatenate([pad[:, -1:], pad, pad[:, :1]], axis=1)  # periodic theta, sector 8
    lo = np.minimum.reduce([pad[1:-1, 1:-1], pad[:-2, 1:-1], pad[2:, 1:-1], pad[1:-1, :-2], pad[1:-1, 2:]])
    hi = np.maximum.reduce([pad[1:-1, 1:-1], pad[:-2, 1:-1], pad[2:, 1:-1], pad[1:-1, :-2], pad[1:-1, 2:]])
    assert (f1 >= lo - tol).all() and (f1 <= hi + tol).all()
    # and the flux did something for every moving q
    assert (np.abs(f1 - f0)[:, :, 1:] > 1e-3 * np.abs(base[1:])).mean() > 0.5


def _transport_error(h):
    """One free-streaming step of a smooth field, against the exact solution
    f(x - v dt) of df/dt + v.grad f = 0 written in Cartesian coordinates."""
    r0, r1 = 0.6, 1.0
    nr = int(round(0.4 / h))
    nt = int(round(2 * np.pi * 0.8 / h / 8)) * 8
    dt = 0.4 * h / 12.5
    p = _advect_params(nr, nt, r0, r1, dt)
    s = O.Solver(p)
    dr, dth = (r1 - r0) / nr, 2 * np.pi / nt
    r = r0 + (np.arange(nr) + 0.5) * dr
    th = (np.arange(nt) + 0.5) * dth
    R, TH = np.meshgrid(r, th, indexing="ij")
    X, Y = R * np.cos(TH), R * np.sin(TH)

    def g(x, y):
        return 1.0 + 0.2 * np.sin(3.0 * x + 1.0) * np.cos(2.0 * y - 0.5)

    f0 = np.repeat(g(X, Y)[:, :, None], 33, axis=2)
    s.set_state(f0, np.zeros((nr, nt)))
    s.step(1)
    f1, _ = s.get_state()
    err = 0.0
    inner = slice(2, nr - 2)
    for q in range(1, 33):
        k, i = _k_of(q), _i_of(q)
        vx, vy = SPEEDS[k] * math.cos(i * math.pi / 4), SPEEDS[k] * math.sin(i * math.pi / 4)
        exact = g(X - vx * dt, Y - vy * dt)
        err = max(err, np.abs(f1[inner, :, q] - exact[inner]).max())
    return err


def test_P7_free_streaming_matches_exact_transport():
    """The per-step error of a consistent first-order scheme against the exact
    transport is O(h^2) (C h^2 f''); a missing 1/r, a wrong Courant number
    or swapped components leave an O(h) error.  Halving h must cut the error
    about four-fold."""
    e1, e2 = _transport_error(0.02), _transport_error(0.01)
    assert e2 < e1 / 3.2, (e1, e2)
    assert e1 < 2e-3


def _lambda_transport_error(h):
    """One step of a smooth lambda field carried by a uniform, unreactive flow
    (T = 1 < T_th, Cartesian-uniform f so f itself stays put), against the
    exact solution lambda(x - u dt) of d lambda/dt + u.grad lambda = 0."""
    r0, r1 = 0.6, 1.0
    nr = int(round(0.4 / h))
    nt = int(round(2 * np.pi * 0.8 / h / 8)) * 8
    dt = 0.4 * h / 12.5
    p = O.make_params(nr, nt, r0, r1, dt=dt, tau=1e-3, w1=2, w2=2, m=1, n=1, Q=1.0, T_th=1.1)
    s = O.Solver(p)
    dr, dth = (r1 - r0) / nr, 2 * np.pi / nt
    r = r0 + (np.arange(nr) + 0.5) * dr
    th = (np.arange(nt) + 0.5) * dth
    R, TH = np.meshgrid(r, th, indexing="ij")
    X, Y = R * np.cos(TH), R * np.sin(TH)
    ux, uy = 0.7, -0.45

    def g(x, y):
        return 0.5 + 0.3 * np.sin(3.0 * x + 1.0) * np.cos(2.0 * y - 0.5)

    fields = np.stack([np.ones_like(R), np.ones_like(R), ux * np.cos(TH) + uy * np.sin(TH),
                       -ux * np.sin(TH) + uy * np.cos(TH), g(X, Y)])
    s.init_fields(fields)
    s.step(1)
    lam = s.fields()[5]
    exact = g(X - ux * dt, Y - uy * dt)
    return np.abs(lam - exact)[2:-2].max()


def test_P7_lambda_is_carried_by_the_flow():
    """Sec. III.A: lambda is advected upwind by the cell's own u (radial and
    azimuthal parts, the latter with 1/r).  Consistency shows as an O(h^2)
    per-step error against exact transport; a wrong sign or side of either
    flux leaves O(h)."""
    e1, e2 = _lambda_transport_error(0.02), _lambda_transport_error(0.01)
    assert e2 < e1 / 3.2, (e1, e2)
    assert e1 < 1e-4


def test_P7_lambda_advection_is_monotone():
    """The lambda fluxes are donor-cell in the direction of the own-cell u:
    each new lambda is a convex combination of the cell and its upwind
    neighbours (a downwind pick is not)."""
    rng = np.random.default_rng(11)
    nr, nt = 12, 32
    r0, r1 = 0.5, 1.0
    p = O.make_params(nr, nt, r0, r1, dt=2e-3, tau=1e-3, w1=2, w2=2, m=1, n=1, Q=1.0, T_th=1.1)
    s = O.Solver(p)
    th = (np.arange(nt) + 0.5) * 2 * np.pi / nt
    TH = np.broadcast_to(th, (nr, nt))
    ux, uy = 0.8, 0.5
    lam0 = rng.uniform(0, 1, (nr, nt))
    fields = np.stack([np.ones((nr, nt)), np.ones((nr, nt)), ux * np.cos(TH) + uy * np.sin(TH),
                       -ux * np.sin(TH) + uy * np.cos(TH), lam0])
    s.init_fields(fields)
    s.step(1)
    lam1 = s.fields()[5]
    pad = np.pad(lam0, ((1, 1), (0, 0)), mode="edge")
    pad = np.concatenate([pad[:, -1:], pad, pad[:, :1]], axis=1)
    nb = [pad[1:-1, 1:-1], pad[:-2, 1:-1], pad[2:, 1:-1], pad[1:-1, :-2], pad[1:-1, 2:]]
    lo, hi = np.minimum.reduce(nb), np.maximum.reduce(nb)
    assert (lam1 >= lo - 1e-14).all() and (lam1 <= hi + 1e-14).all()
    assert np.abs(lam1 - lam0).max() > 1e-2


# ---------------------------------------------------------------- P8 ------
def test_P8_rotation_and_mirror_symmetry():
    """With an axisymmetric initial state, the full annulus and N_theta a
    multiple of 8, the scheme commutes with rotation by pi/4 (cells shift by
    N_theta/8, direction index i -> i+1) and with the mirror theta -> -theta
    (j -> N_theta-1-j, i -> -i mod 8)."""
    nr, nt = 12, 24
    p = O.make_params(nr, nt, 0.1, 1.0, dt=1e-4, tau=2e-4, w1=2, w2=2, m=2, n=2, Q=1.0, T_th=1.1)
    s = O.Solver(p)
    s.init_ic(0.35, [1.5, 20 / 1.5, 0, 0, 1], [1, 1, 0, 0, 0])
    s.step(40)
    f, lam = s.get_state()
    rot = np.empty_like(f)
    mir = np.empty_like(f)
    for q in range(33):
        k, i = _k_of(q), _i_of(q)
        rot[:, :, _q_of(k, (i + 1) % 8) if k else 0] = np.roll(f[:, :, q], nt // 8, axis=1)
        mir[:, :, _q_of(k, (-i) % 8) if k else 0] = f[:, ::-1, q]
    scale = np.abs(f).max()
    assert np.abs(rot - f).max() < 1e-12 * scale
    assert np.abs(mir - f).max() < 1e-12 * scale
    # lambda is a scalar: it only moves with the cells
    assert np.abs(np.roll(lam, nt // 8, axis=1) - lam).max() < 1e-12
    assert np.abs(lam[:, ::-1] - lam).max() < 1e-12
    # the run did react and move
    F = s.fields()
    assert F[5].min() < 0.99 and F[5].max() > 0.99 and np.abs(F[1]).max() > 0.1


# ---------------------------------------------------------------- P10 -----
def test_P10_gamma_two_reproduces_printed_states():
    """The model's equation of state (p = rho T, internal energy rho T for
    D = 2, i.e. gamma = 2) reproduces the paper's printed shocked state and
    CJ detonation state and speed (Sec. III.B-D initial states)."""
    gam, rho0, p0, Q = 2.0, 1.0, 1.0, 1.0
    rho1 = GOLD["shocked_state"]["value"]["rho"]
    # Rankine-Hugoniot for a shock into (rho0, p0, 0)
    p1 = p0 * ((gam + 1) * rho1 - (gam - 1) * rho0) / ((gam + 1) * rho0 - (gam - 1) * rho1)
    u1 = math.sqrt((p1 - p0) * (1 / rho0 - 1 / rho1))
    assert abs(p1 / rho1 - GOLD["shocked_state"]["value"]["T"]) < 1e-5
    assert abs(u1 - GOLD["shocked_state"]["value"]["u_r_abs"]) < 1e-6
    # CJ state with heat release Q
    c0sq = gam * p0 / rho0
    D = math.sqrt((gam * gam - 1) * Q / 2 + c0sq) + math.sqrt((gam * gam - 1) * Q / 2)
    rho_cj = rho0 * (gam + 1) * D * D / (gam * D * D + c0sq)
    u_cj = D * (1 - rho0 / rho_cj)
    p_cj = p0 + rho0 * D * u_cj
    cj = GOLD["cj_state"]["value"]
    assert abs(D - GOLD["cj_speed"]["value"]) < 1e-5
    assert abs(rho_cj - cj["rho"]) < 1e-5
    assert abs(p_cj / rho_cj - cj["T"]) < 1e-5
    assert abs(u_cj - cj["u_r"]) < 1e-5
    # and the oracle's f^eq carries exactly that equation of state
    theta = 0.4
    feq = O.equilibrium(cj["rho"], cj["u_r"], 0.0, cj["T"], theta)
    vr, vt = O.velocities(theta)
    E = 0.5 * (feq * (vr * vr + vt * vt)).sum()
    assert abs(E - (cj["rho"] * cj["T"] + 0.5 * cj["rho"] * cj["u_r"] ** 2)) < 1e-13


# ---------------------------------------------------------------- P12 -----
def test_P12_rounding_drift_is_far_below_parity_tolerance():
    """The same 200 steps in long double arithmetic: the double oracle's own
    rounding drift must sit orders of magnitude below the 1e-10 parity bar."""
    p = O.make_params(8, 8, 0.1, 1.0, dt=1e-5, tau=2e-5, w1=2, w2=2, m=2, n=2, Q=1.0, T_th=1.1)
    outs = []
    for real in ("double", "long double"):
        s = O.Solver(p, real=real)
        s.init_ic(0.35, [1.5, 20 / 1.5, 0, 0, 1], [1, 1, 0, 0, 0], 1e-6, 0)
        s.step(200)
        outs.append(s.fields())
    assert O.lib("long double").ora_real_bytes() > 8
    for fld in (0, 3, 5):
        a, b = outs[0][fld], outs[1][fld]
        assert np.abs(a - b).max() / np.abs(b).max() < 1e-13


# ------------------------------------------------------------ drift report
# The drift report sums cell values times the cell area r_i dr dtheta over the
# grid (reading R20).  The midpoint rule is exact for the weight r, so for a
# uniform state each sum is the state's density times the exact area of the
# annular sector, s pi (r_max^2 - r_min^2) / 8.
def _sector_area(r_min, r_max, sector):
    return sector * math.pi / 8.0 * (r_max * r_max - r_min * r_min)


@pytest.mark.parametrize("nr,nt,r_min,r_max,sector", [(7, 16, 0.3, 1.0, 8), (5, 9, 0.5, 2.0, 3),
                                                      (6, 4, 0.0, 0.8, 1)])
def test_drift_report_of_uniform_states(nr, nt, r_min, r_max, sector):
    """Uniform states on an annulus, a 3/8 sector and a 1/8 disc: mass
    rho A, total energy (rho T + rho |u|^2 / 2) A (gamma = 2: internal energy
    rho T, Sec. II.A), unreleased chemical energy rho Q (1 - lambda) A, and no
    cell counted as bad."""
    rho, T, ur, ut, lam, Q = 1.3, 2.1, 0.4, -0.25, 0.35, 0.7
    s = O.Solver(O.make_params(nr, nt, r_min, r_max, dt=1e-4, tau=2e-4, Q=Q, sector=sector))
    s.init_ic(0.0, [rho, T, ur, ut, lam], [rho, T, ur, ut, lam])
    d = s.diag()
    A = _sector_area(r_min, r_max, sector)
    for key, want in (("mass", rho * A), ("energy", (rho * T + 0.5 * rho * (ur * ur + ut * ut)) * A),
                      ("chem", rho * Q * (1.0 - lam) * A)):
        assert abs(d[key] - want) <= 1e-13 * want, (key, d[key], want)
    assert d["n_nonfinite"] == 0 and d["n_nonphys"] == 0


def test_drift_report_counts_each_bad_cell_once():
    """Cells made bad through the raw state: a non-finite f, a non-finite
    lambda, and a non-finite f in a cell of negative density are each one
    non-finite cell and leave the sums; a cell of negative density (f turned
    over: rho and the energy change sign, u and T do not) and a cell of zero
    temperature (all mass at rest) are each one non-physical cell and stay in
    the sums with their own values."""
    nr, nt, r_min, r_max, Q = 6, 8, 0.2, 1.0, 0.9
    rho, T, lam = 1.2, 1.5, 0.25
    s = O.Solver(O.make_params(nr, nt, r_min, r_max, dt=1e-4, tau=2e-4, Q=Q))
    s.init_ic(0.0, [rho, T, 0, 0, lam], [rho, T, 0, 0, lam])
    f, la = s.get_state()
    dr, dth = (r_max - r_min) / nr, 2 * math.pi / nt
    w = [(r_min + (i + 0.5) * dr) * dr * dth for i in range(nr)]
    f[1, 2, :] = np.nan                    # non-finite
    la[3, 1] = np.nan                      # non-finite
    f[5, 3, :] *= -1.0
    f[5, 3, 7] = np.inf                    # non-finite (not also non-physical)
    f[2, 5, :] *= -1.0                     # rho < 0
    f[4, 6, :] = 0.0
    f[4, 6, 0] = rho                       # T = 0
    s.set_state(f, la)
    d = s.diag()
    assert d["n_nonfinite"] == 3 and d["n_nonphys"] == 2, d
    A = _sector_area(r_min, r_max, 8)
    gone = w[1] + w[3] + w[5]
    e, c = rho * T, rho * Q * (1.0 - lam)
    np.testing.assert_allclose(d["mass"], rho * (A - gone - 2 * w[2]), rtol=1e-13)
    np.testing.assert_allclose(d["energy"], e * (A - gone - 2 * w[2] - w[4]), rtol=1e-13)
    np.testing.assert_allclose(d["chem"], c * (A - gone - 2 * w[2]), rtol=1e-13)


# ------------------------------------------------------------ initial state
def test_initial_state_noise_and_regions():
    """Reading of the two-region initial state with +-p_noise uniform noise on
    p: the splitmix64 generator matches its published test vector, the inner
    region is chosen by cell-centre radius, and T = p / rho."""
    assert O.splitmix64(0) == 0xE220A8397B1DCDAF
    assert O.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4
    nr, nt = 16, 16
    p = O.make_params(nr, nt, 0.1, 1.0, dt=1e-5, tau=2e-5, w1=2, w2=2, m=2, n=2, Q=1.0, T_th=1.1)
    s = O.Solver(p)
    amp, seed = 1e-6, 5
    s.init_ic(0.2, [1.5, 20 / 1.5, 0, 0, 1], [1, 1, 0, 0, 0], amp, seed)
    F = s.fields()
    r = 0.1 + (np.arange(nr) + 0.5) * 0.9 / nr
    inner = r < 0.2
    assert inner.sum() == 2
    assert np.abs(F[0][inner] - 1.5).max() < 1e-13 and np.abs(F[0][~inner] - 1).max() < 1e-13
    assert np.abs(F[5][inner] - 1).max() == 0 and np.abs(F[5][~inner]).max() == 0
    for ir in range(nr):
        for jt in range(nt):
            h = O.splitmix64(seed ^ (((ir * nt + jt) * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF))
            U = (h >> 11) * 2.0 ** -53
            p_exp = (1.5 * (20 / 1.5) if inner[ir] else 1.0) + amp * (2 * U - 1)
            assert abs(F[4][ir, jt] - p_exp) < 1e-13 * p_exp


# ---------------------------------------------------------------- P9 ------
@pytest.mark.slow
def test_P9_steady_detonation_runs_at_cj_speed():
    """The paper's validation run (Sec. III.B.1): an annulus at r = 1000 (flat
    to within 1e-4), CJ state behind r = 1000.01, unburnt gas ahead, tau =
    2e-4, omega1 = 10, omega2 = 1000, m = n = 1, to t = 0.025.  Run here on a
    4x coarser grid with dt scaled alike (same Courant number).  The wave
    must run at the Chapman-Jouguet speed the paper prints (D = 3.09557,
    within 3 %; the paper's own run is 1.8 % off) and leave the post-wave
    state the paper prints for its run (within 1 %)."""
    g = GOLD["vv_setup"]["value"]
    nr = g["nr"] // 8
    dt = g["dt"] * 8
    p = O.make_params(nr, 1, g["r_min"], g["r_max"], dt=dt, tau=g["tau"], w1=g["w1"], w2=g["w2"], m=1, n=1,
                      Q=1.0, T_th=GOLD["ignition_temperature"]["value"])
    s = O.Solver(p)
    cj, un = GOLD["cj_state"]["value"], GOLD["unburnt_state"]["value"]
    s.init_ic(g["r_split"], [cj["rho"], cj["T"], cj["u_r"], 0, 1], [un["rho"], un["T"], 0, 0, 0])
    dr = (g["r_max"] - g["r_min"]) / nr
    r = g["r_min"] + (np.arange(nr) + 0.5) * dr
    chunk = int(round(5e-4 / dt))
    ts, xs = [], []
    for k in range(int(round(g["t_end"] / dt)) // chunk):
        s.step(chunk)
        lam = s.fields()[5][:, 0]
        i = np.where(lam >= 0.5)[0].max()
        xs.append(r[i] + (lam[i] - 0.5) / (lam[i] - lam[i + 1]) * dr)
        ts.append((k + 1) * chunk * dt)
    h = 3 * len(ts) // 4
    D = np.polyfit(ts[h:], xs[h:], 1)[0]
    assert abs(D - GOLD["cj_speed"]["value"]) / GOLD["cj_speed"]["value"] < 0.03, D
    F = s.fields()
    post = i - int(round(0.01 / dr))
    lb = GOLD["lb_post_state"]["value"]
    assert abs(F[0][post, 0] - lb["rho"]) / lb["rho"] < 0.01
    assert abs(F[3][post, 0] - lb["T"]) / lb["T"] < 0.01
    assert abs(F[1][post, 0] - lb["u_r"]) / lb["u_r"] < 0.01
    assert abs(F[5][post, 0] - 1.0) < 1e-3


# -------------------------------------- per-cell relaxation time (Sec. IV) --
# The paper (Sec. IV, point (ii)) says tau should depend on the local state
# but gives no form; the oracle takes a field tau[ir][jt] as input.
def _tau_case(seed=11):
    rng = np.random.default_rng(seed)
    nr, nt = 6, 8
    p = O.make_params(nr, nt, 0.3, 1.0, dt=2e-5, tau=5e-5, w1=2.0, w2=3.0, m=1, n=2, Q=1.0, T_th=1.1)
    s = O.Solver(p)
    s.init_ic(0.55, [1.5, 20 / 1.5, 0.2, -0.1, 1], [1, 1, 0, 0, 0], 1e-3, 3)
    f, lam = s.get_state()
    f = f * (1 + 0.05 * rng.uniform(-1, 1, f.shape))  # off equilibrium everywhere
    lam = np.clip(lam + 0.1 * rng.uniform(0, 1, lam.shape), 0, 1)
    tau = rng.uniform(1e-5, 2e-4, (nr, nt))
    return p, f, lam, tau


def test_tau_field_step_is_each_cells_own_uniform_step():
    """In the unsplit update (reading R8) the fluxes use time-t f, so one
    step of cell c with a tau field is the step with a uniform tau equal to
    tau[c]: checked cell by cell, bitwise, on a reacting, moving, off-
    equilibrium state with a tau field of distinct values (a transposed or
    shifted index would take another cell's value)."""
    p, f, lam, tau = _tau_case()
    nr, nt = p.nr, p.ntheta
    s = O.Solver(p)
    s.set_state(f, lam)
    s.set_tau(tau)
    s.step(1)
    gf, gl = s.get_state()
    for ir in range(nr):
        for jt in range(nt):
            q = O.make_params(nr, nt, 0.3, 1.0, dt=p.dt, tau=tau[ir, jt], w1=p.w1, w2=p.w2, m=p.m, n=p.n, Q=p.Q,
                              T_th=p.T_th)
            u = O.Solver(q)
            u.set_state(f, lam)
            u.step(1)
            uf, ul = u.get_state()
            assert np.array_equal(gf[ir, jt], uf[ir, jt]) and gl[ir, jt] == ul[ir, jt], (ir, jt)


def test_tau_field_collision_conserves_every_cell():
    """Whatever tau a cell relaxes with, the collision conserves its mass,
    momentum and energy (Sec. II.A): one step with the tau field and one with
    no relaxation at all (tau = inf) differ in every cell by
    (e^(-dt/tau) - 1)(f - f^eq), whose mass, momentum and energy are zero."""
    p, f, lam, tau = _tau_case(12)
    s = O.Solver(p)
    s.set_state(f, lam)
    s.set_tau(tau)
    s.step(1)
    a, _ = s.get_state()
    s.set_state(f, lam)
    s.set_tau(np.full_like(tau, np.inf))
    s.step(1)
    b, _ = s.get_state()
    d = a - b
    assert np.abs(d).max() > 1e-3 * np.abs(f).max()  # the relaxation did act
    dth = 2 * np.pi / p.ntheta
    for jt in range(p.ntheta):
        vr, vt = O.velocities((jt + 0.5) * dth)
        for ir in range(p.nr):
            scale = np.abs(f[ir, jt]).sum()
            w = np.abs(d[ir, jt]).sum()
            for mom in (np.ones(33), vr, vt, 0.5 * (vr * vr + vt * vt)):
                assert abs((d[ir, jt] * mom).sum()) <= 1e-13 * scale * max(1.0, np.abs(mom).max()), (ir, jt)
            assert w > 0


def test_tau_field_pure_relaxation_decays_with_the_cells_own_tau():
    """A single cell (its radial ghosts and its periodic azimuthal neighbours
    are itself, so nothing streams) off equilibrium with no reaction: f(n dt)
    = f^eq + (f0 - f^eq) exp(-n dt / tau_cell) with tau_cell from the field,
    not the parameters; tau = inf in the field freezes it."""
    rng = np.random.default_rng(9)
    p = O.make_params(1, 1, 0.5, 1.0, dt=1e-5, tau=3e-5, w1=0, w2=0, m=1, n=1, Q=0.0, T_th=1.1)
    feq = O.equilibrium(1.1, 0.0, 0.0, 1.7, np.pi / 4)
    vr, vt = O.velocities(np.pi / 4)
    Bm = np.stack([np.ones(33), vr, vt, 0.5 * (vr * vr + vt * vt)])
    d = feq * 0.03 * rng.uniform(-1, 1, 33)
    d -= Bm.T @ np.linalg.lstsq(Bm.T, d, rcond=None)[0]
    f0 = feq + d
    for tau_cell in (1.2e-5, 8e-5, np.inf):
        s = O.Solver(p)
        s.set_state(f0.reshape(1, 1, 33), np.zeros((1, 1)))
        s.set_tau(np.full((1, 1), tau_cell))
        s.step(40)
        f, _ = s.get_state()
        np.testing.assert_allclose(f[0, 0], feq + d * math.exp(-40 * p.dt / tau_cell), rtol=1e-11, atol=1e-16)


def test_tau_field_of_the_uniform_value_changes_nothing():
    p, f, lam, _ = _tau_case(13)
    a, b = O.Solver(p), O.Solver(p)
    for s in (a, b):
        s.set_state(f, lam)
    a.set_tau(np.full((p.nr, p.ntheta), p.tau))
    a.step(5)
    b.step(5)
    assert all(np.array_equal(x, y) for x, y in zip(a.get_state(), b.get_state()))
    a.set_tau(None)  # back to the parameters' tau
    a.step(3)
    b.step(3)
    assert all(np.array_equal(x, y) for x, y in zip(a.get_state(), b.get_state()))


# ------------------------------------------------ sector and disc centre --
def test_sector_halo_equals_full_annulus():
    """Reading of the periodic azimuthal boundary on a sector (Sec. II.D):
    the halo rotates the direction index by the sector angle.  For an
    axisymmetric state, a 1/8 sector (s = 1, N cells) must evolve exactly as
    the first N columns of the full annulus (s = 8, 8N cells); a 3/8 sector
    likewise as the first 3N."""
    nr, n = 10, 6
    common = dict(r_min=0.3, r_max=1.0, dt=1e-4, tau=2e-4, w1=2, w2=3, m=1, n=2, Q=1.0, T_th=1.1)
    full = O.Solver(O.make_params(nr, 8 * n, sector=8, **common))
    full.init_ic(0.55, [1.5, 20 / 1.5, 0.1, 0.05, 1], [1, 1, 0, 0, 0])
    full.step(30)
    Ff = full.fields()
    for s in (1, 3):
        part = O.Solver(O.make_params(nr, s * n, sector=s, **common))
        part.init_ic(0.55, [1.5, 20 / 1.5, 0.1, 0.05, 1], [1, 1, 0, 0, 0])
        part.step(30)
        Fp = part.fields()
        scale = np.abs(Ff).max(axis=(1, 2))[:, None, None]
        assert (np.abs(Fp - Ff[:, :, : s * n]) / scale).max() < 1e-12, s


def test_disc_centre_rule_keeps_rest_and_symmetry():
    """Disc-centre ghost rule f(-1, j, k, i) = f(0, j, k, (i+4)%8) (Sec.
    II.D): a gas at rest is mirror-symmetric in velocity, so the rule keeps
    it at rest and uniform; and an axisymmetric explosion on the full disc
    keeps the pi/4 rotation symmetry through the centre."""
    nr, nt = 12, 16
    p = O.make_params(nr, nt, 0.0, 1.0, dt=2e-4, tau=2e-4, w1=1, w2=50, m=1, n=1, Q=1.0, T_th=1.1)
    s = O.Solver(p)
    s.init_ic(0.0, [1.3, 1.05, 0, 0, 0], [1.3, 1.05, 0, 0, 0])
    f0, _ = s.get_state()
    s.step(25)
    f1, _ = s.get_state()
    np.testing.assert_allclose(f1, f0, rtol=1e-12, atol=1e-15)
    s = O.Solver(p)
    s.init_ic(0.3, list(GOLD["shocked_state"]["value"].values())[:2] + [0.666667, 0, 1], [1, 1, 0, 0, 0])
    s.step(60)
    f, lam = s.get_state()
    rot = np.empty_like(f)
    for q in range(33):
        k, i = _k_of(q), _i_of(q)
        rot[:, :, _q_of(k, (i + 1) % 8) if k else 0] = np.roll(f[:, :, q], nt // 8, axis=1)
    assert np.abs(rot - f).max() < 1e-12 * np.abs(f).max()
    F = s.fields()
    assert np.abs(F[1]).max() > 0.05  # the explosion did move


def _disc_ring_errors(nr, nt=16):
    """One free-streaming step on a disc of radius 0.5 with a smooth field
    f_q(x) = g(x . v_q, |x|) (unchanged when position and velocity are
    rotated together), against the exact transport f_q(x - v_q dt): the
    largest error on each ring."""
    h = 0.5 / nr
    dt = 0.08 * h / 12.5
    p = O.make_params(nr, nt, 0.0, 0.5, dt=dt, tau=float("inf"), w1=0, w2=0, m=1, n=1, Q=0.0, T_th=1e9)
    s = O.Solver(p)
    r = (np.arange(nr) + 0.5) * h
    th = (np.arange(nt) + 0.5) * 2 * np.pi / nt
    R, TH = np.meshgrid(r, th, indexing="ij")
    X, Y = R * np.cos(TH), R * np.sin(TH)
    vx = np.zeros(33)
    vy = np.zeros(33)
    for q in range(1, 33):
        k, i = _k_of(q), _i_of(q)
        vx[q], vy[q] = SPEEDS[k] * math.cos(i * math.pi / 4), SPEEDS[k] * math.sin(i * math.pi / 4)

    def g(x, y, q):
        return 1.0 + 0.3 * np.sin(0.8 * (x * vx[q] + y * vy[q]) + 5.0 * (x * x + y * y))

    f0 = np.stack([g(X, Y, q) for q in range(33)], axis=-1)
    s.set_state(f0, np.zeros((nr, nt)))
    s.step(1)
    f1, _ = s.get_state()
    err = np.zeros(nr)
    for q in range(1, 33):
        exact = g(X - vx[q] * dt, Y - vy[q] * dt, q)
        err = np.maximum(err, np.abs(f1[:, :, q] - exact).max(axis=1))
    return err


def test_disc_centre_rule_is_consistent_transport():
    """For such a field the paper's rule gives the ghost the exact value of
    the field at the mirrored point, so the innermost ring, whose upwind
    stencil crosses the centre, is no less accurate than the next ring; a
    ghost rotated by anything but pi adds an error there."""
    for nr in (20, 40):
        e = _disc_ring_errors(nr)
        assert e[0] <= 1.2 * e[1], (nr, e[:3])


# ------------------------------------------------- non-equilibrium (II.E) --
# component order of the Delta*_m output: M*_2 rr, rt, tt; M*_3 rrr, rrt,
# rtt, ttt; M*_{3,1} r, t; M*_{4,2} rr, rt, tt
_THETA_PARITY = np.array([1, -1, 1, 1, -1, 1, -1, 1, -1, 1, -1, 1])


def _two_beam_expected(rho, T, dr, dt_):
    """Delta*_m of f = (f^eq(rho, u + d, T) + f^eq(rho, u - d, T)) / 2, a
    mixture of two equilibria drifting at +-d relative to the mean u.  From
    the Maxwellian moments (which f^eq reproduces up to M*_{4,2}, Sec. II.B):
    central M*_2 = rho T I + rho d d and the mixture temperature is
    T + |d|^2/2, so Delta*_2 = rho (d d - |d|^2/2 I); odd moments cancel
    between the beams; and
    Delta*_{4,2} = rho (3T d d - 3/2 T |d|^2 I + 1/2 |d|^2 d d - 1/2 |d|^4 I)."""
    d = np.array([dr, dt_])
    d2 = d @ d
    I = np.eye(2)
    D2 = rho * (np.outer(d, d) - 0.5 * d2 * I)
    D42 = rho * (3 * T * np.outer(d, d) - 1.5 * T * d2 * I + 0.5 * d2 * np.outer(d, d) - 0.5 * d2 * d2 * I)
    return np.array([D2[0, 0], D2[0, 1], D2[1, 1], 0, 0, 0, 0, 0, 0, D42[0, 0], D42[0, 1], D42[1, 1]])


@pytest.mark.parametrize("rho,T,ur,ut,dr,dt_", [(1.3, 2.0, 0.2, -0.1, 0.3, 0.15), (0.7, 5.0, -0.5, 0.4, -0.2, 0.6),
                                                 (2.0, 1.2, 0.0, 0.0, 0.05, -0.02)])
def test_noneq_two_beam_mixture_closed_form(rho, T, ur, ut, dr, dt_):
    """Sec. II.E on a state whose non-equilibrium is known in closed form:
    two interpenetrating equilibria (a mixture of beams at u +- d)."""
    p = O.make_params(1, 1, 0.5, 1.0, dt=1e-5, tau=2e-5)
    theta = math.pi  # the single cell of a full annulus with N_theta = 1
    f = 0.5 * (O.equilibrium(rho, ur + dr, ut + dt_, T, theta) + O.equilibrium(rho, ur - dr, ut - dt_, T, theta))
    s = O.Solver(p)
    s.set_state(f.reshape(1, 1, 33), np.zeros((1, 1)))
    got = s.noneq()[:, 0, 0]
    ref = _two_beam_expected(rho, T, dr, dt_)
    scale = rho * (T + dr * dr + dt_ * dt_) ** 2
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * scale)
    # the mixture does depart from equilibrium
    assert np.abs(got).max() > 0.1 * rho * (dr * dr + dt_ * dt_)


def test_noneq_relations_of_the_paper():
    """Sec. II.E: Delta*_{3,1,r} = (Delta*_{3,rrr} + Delta*_{3,r theta theta})/2,
    Delta*_{3,1,theta} = (Delta*_{3,rr theta} + Delta*_{3,theta theta theta})/2,
    and Delta*_{2,rr} = -Delta*_{2,theta theta} (f^eq carries the cell's own
    energy), for an arbitrary non-equilibrium state."""
    rng = np.random.default_rng(11)
    nr, nt = 6, 16
    p = O.make_params(nr, nt, 0.2, 1.0, dt=1e-5, tau=2e-5)
    f = np.empty((nr, nt, 33))
    for ir in range(nr):
        for jt in range(nt):
            th = (jt + 0.5) * 2 * math.pi / nt
            feq = O.equilibrium(rng.uniform(0.5, 2), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5),
                                rng.uniform(0.8, 6), th)
            f[ir, jt] = feq * (1 + 0.05 * rng.uniform(-1, 1, 33))
    s = O.Solver(p)
    s.set_state(f, np.zeros((nr, nt)))
    D = s.noneq()
    F = s.fields()
    s3 = (F[0] * F[3] ** 1.5).max()
    assert np.abs(D[7] - 0.5 * (D[3] + D[5])).max() < 1e-12 * s3
    assert np.abs(D[8] - 0.5 * (D[4] + D[6])).max() < 1e-12 * s3
    assert np.abs(D[0] + D[2]).max() < 1e-12 * (F[0] * F[3]).max()
    assert np.abs(D[0]).max() > 1e-4 * (F[0] * F[3]).max()


def test_noneq_central_moments_match_cartesian_tensors():
    """The polar central moments equal the Cartesian tensors of the same
    distribution, built here from the speeds and the directions i pi/4 alone,
    rotated into the frame (e_r, e_theta) at theta."""
    rng = np.random.default_rng(12)
    g = rng.uniform(-1, 1, 33)
    theta, ux, uy = 0.7, 0.3, -0.2
    vx, vy = np.zeros(33), np.zeros(33)
    for q in range(1, 33):
        v, a = SPEEDS[_k_of(q)], _i_of(q) * math.pi / 4
        vx[q], vy[q] = v * math.cos(a), v * math.sin(a)
    cx, cy = vx - ux, vy - uy
    c = np.stack([cx, cy])
    h = 0.5 * (cx * cx + cy * cy)
    M2 = np.einsum("q,aq,bq->ab", g, c, c)
    M3 = np.einsum("q,aq,bq,cq->abc", g, c, c, c)
    M31 = np.einsum("q,q,aq->a", g, h, c)
    M42 = np.einsum("q,q,aq,bq->ab", g, h, c, c)
    R = np.array([[math.cos(theta), math.sin(theta)], [-math.sin(theta), math.cos(theta)]])  # rows e_r, e_theta
    M2p = R @ M2 @ R.T
    M3p = np.einsum("ia,jb,kc,abc->ijk", R, R, R, M3)
    M31p = R @ M31
    M42p = R @ M42 @ R.T
    ref = np.array([M2p[0, 0], M2p[0, 1], M2p[1, 1], M3p[0, 0, 0], M3p[0, 0, 1], M3p[0, 1, 1], M3p[1, 1, 1],
                    M31p[0], M31p[1], M42p[0, 0], M42p[0, 1], M42p[1, 1]])
    ur, ut = R @ np.array([ux, uy])
    got = O.central_moments(g, theta, ur, ut)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_noneq_rotation_and_mirror_symmetry():
    """An axisymmetric run is invariant under rotation by pi/4 and under the
    mirror theta -> -theta (P8).  Polar components are frame-relative: they
    repeat under the rotation, and those with an odd number of theta indices
    change sign under the mirror."""
    nr, nt = 12, 24
    p = O.make_params(nr, nt, 0.1, 1.0, dt=1e-4, tau=2e-4, w1=2, w2=2, m=2, n=2, Q=1.0, T_th=1.1)
    s = O.Solver(p)
    s.init_ic(0.35, [1.5, 20 / 1.5, 0, 0, 1], [1, 1, 0, 0, 0])
    s.step(40)
    D = s.noneq()
    scale = np.abs(D).max()
    assert np.abs(np.roll(D, nt // 8, axis=2) - D).max() < 1e-11 * scale
    assert np.abs(_THETA_PARITY[:, None, None] * D[:, :, ::-1] - D).max() < 1e-11 * scale
    assert np.abs(D[0]).max() > 1e-3 * scale  # the detonation front is out of equilibrium


def test_noneq_decays_with_pure_relaxation():
    """With no reaction and no gradients (P5), f - f^eq decays as
    exp(-t/tau) at fixed moments, so every Delta*_m does too."""
    rng = np.random.default_rng(13)
    nr, nt = 4, 8
    p = O.make_params(nr, nt, 0.5, 1.0, dt=1e-5, tau=3e-5, w1=0, w2=0, m=1, n=1, Q=0.0, T_th=1.1)
    feq = O.equilibrium(1.1, 0.0, 0.0, 1.7, 0.0)
    vr, vt = O.velocities(0.0)
    Bm = np.stack([np.ones(33), vr, vt, 0.5 * (vr * vr + vt * vt)])
    d = 0.03 * feq * rng.uniform(-1, 1, 33)
    d -= Bm.T @ np.linalg.lstsq(Bm.T, d, rcond=None)[0]
    s = O.Solver(p)
    s.set_state(np.broadcast_to(feq + d, (nr, nt, 33)).copy(), np.zeros((nr, nt)))
    D0 = s.noneq()
    n = 20
    s.step(n)
    D1 = s.noneq()
    np.testing.assert_allclose(D1, D0 * math.exp(-n * p.dt / p.tau), rtol=0, atol=1e-11 * np.abs(D0).max())
