"""Pins of the oracle's pseudo-transient relaxation (Section 2.2)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import apt, assembly, design

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def _closed_form_heavy_ball(kappa, F, dt, theta, n):
    """e_n = u_n - F/kappa for the 1-unknown damped wave, from the roots of
    z^2 - (1 + a - b) z + a = 0 with a = theta/(theta+dt), b = dt^2 kappa/(theta+dt)."""
    a = theta / (theta + dt)
    b = dt * dt * kappa / (theta + dt)
    e0 = -F / kappa
    e1 = (1.0 - b) * e0
    z = np.roots([1.0, -(1.0 + a - b), a]).astype(complex)
    if abs(z[0] - z[1]) < 1e-12:
        zz = z[0]
        c1 = e0
        c2 = (e1 - c1 * zz) / zz
        return (c1 + c2 * n) * zz ** n
    c2 = (e1 - e0 * z[0]) / (z[1] - z[0])
    c1 = e0 - c2
    return (c1 * z[0] ** n + c2 * z[1] ** n).real


@pytest.mark.parametrize("theta,dt", [(1.0, 0.3), (1.0, 0.9), (0.0, 0.15), (4.0, 0.5)])
def test_single_unknown_recurrence(theta, dt):
    kappa, F = 2.5, 0.7
    for n in (1, 2, 7, 40):
        res = apt.apt_solve(lambda u: F - kappa * u, np.zeros(1), dt=dt, theta=theta, hd=1.0,
                            fnorm=F, ncell=1, n_iter=n, check_every=10**9)
        assert res.u[0] - F / kappa == pytest.approx(_closed_form_heavy_ball(kappa, F, dt, theta, n),
                                                     rel=1e-9, abs=1e-14)


def test_pt_is_theta_zero():
    kappa, F, dt = 3.0, 1.0, 0.2
    res = apt.apt_solve(lambda u: F - kappa * u, np.zeros(1), dt=dt, theta=0.0, hd=1.0, fnorm=1.0,
                        ncell=1, n_iter=5, check_every=10**9)
    u = 0.0
    for _ in range(5):
        u = u + dt * (F - kappa * u)
    assert res.u[0] == pytest.approx(u, rel=1e-14)


def test_step_above_stability_bound_diverges():
    """Stable iff dt^2 kappa < 2 (2 theta + dt)."""
    kappa, theta = 4.0, 1.0
    # boundary kappa dt^2 = 4 theta + 2 dt  ->  dt = (2 + sqrt(4 + 16 kappa theta)) / (2 kappa)
    dt_bound = (2 + math.sqrt(4 + 16 * kappa * theta)) / (2 * kappa)
    good = apt.apt_solve(lambda u: 1.0 - kappa * u, np.zeros(1), dt=0.95 * dt_bound, theta=theta,
                         hd=1.0, fnorm=1.0, ncell=1, tol=1e-10, check_every=10)
    bad = apt.apt_solve(lambda u: 1.0 - kappa * u, np.zeros(1), dt=1.05 * dt_bound, theta=theta,
                        hd=1.0, fnorm=1.0, ncell=1, tol=1e-10, check_every=10, max_iter=10**5)
    assert good.converged and not good.diverged
    assert bad.diverged


def test_default_steps_match_printed_values():
    """The damped-wave step h sqrt(theta/(2 d M)) is the printed dx/2 for 2D
    unit-conductivity heat with theta = 1; the PT step h^2/(2 d M) is the printed
    dx^2/4 (2D) and dx^2/6 (3D)."""
    h = GOLD["heat2d"]["dx"]
    assert apt.default_dt(h, 2, 1.0, GOLD["mbb2d"]["theta"]) == pytest.approx(GOLD["heat2d"]["dt_apt_over_dx"] * h)
    assert apt.default_dt(h, 2, 1.0, 0.0) == pytest.approx(GOLD["heat2d"]["dt_pt_over_dx2"] * h * h)
    assert apt.default_dt(h, 3, 1.0, 0.0) == pytest.approx(GOLD["cantilever3d"]["dt_pt_over_dx2"] * h * h)


@pytest.mark.parametrize("which", ["cant2d", "cant3d", "heat"])
def test_fixed_point_equals_direct_solve(which):
    if which == "cant2d":
        prob = W.cantilever2d(12, 6)
        phi = W.random_phi(prob, 2, 0.3, 1.0)
    elif which == "cant3d":
        prob = W.cantilever3d(6, 4, 4)
        phi = W.random_phi(prob, 3, 0.3, 1.0)
    else:
        probs, phis, _ = W.heat_batch(1, 10, 14, seed=5)
        prob, phi = probs[0], np.clip(phis[0], 0.3, 1.0)
    res, _ = design.solve(phi, prob, params=design.AptParams(theta=4.0, tol=1e-11, check_every=20))
    assert res.converged
    E = design.material(phi, prob)
    ud = assembly.direct_solve(design.stiffness(E, prob), design.load_vector(prob), prob)
    assert np.linalg.norm(res.u - ud) / np.linalg.norm(ud) < 1e-9


def test_stop_rule_reports_checked_residual():
    prob = W.cantilever2d(8, 4)
    phi = W.initial_phi(prob)
    res, _ = design.solve(phi, prob, params=design.AptParams(tol=1e-3, check_every=10))
    assert res.converged and res.iters % 10 == 0 and res.rho <= 1e-3
    # replaying the same count reproduces the same state
    res2, _ = design.solve(phi, prob, params=design.AptParams(tol=1e-3, check_every=10), n_iter=res.iters)
    np.testing.assert_array_equal(res.u, res2.u)


def test_adapted_theta_single_unknown():
    """For one unknown K = kappa the Rayleigh quotient is kappa exactly, so the
    critically damping choice is theta = 1 / (4 kappa) (floored)."""
    kappa, F = 0.02, 1.0
    u = np.array([3.0])
    r = F - kappa * u
    assert apt.adapted_theta(u, r, np.array([F]), 1.0, 1.0) == pytest.approx(1.0 / (4 * kappa))
    assert apt.adapted_theta(u, r, np.array([F]), 1.0, 100.0) == pytest.approx(100.0)
    assert apt.adapted_theta(np.zeros(1), r, np.array([F]), 1.0, 1.0) is None


def _scalar_sweeps(u, v, theta, dt, kappa, F, n):
    for _ in range(n):
        v = (theta * v + dt * (F - kappa * u)) / (theta + dt)
        u = u + dt * v
    return u, v


@pytest.mark.parametrize("u0", [3.0, 0.0])
def test_adaptive_damping_starts_from_the_state_it_is_given(u0):
    """One unknown K = kappa, h^d = 1: a warm start (u0 != 0) runs its first
    sweeps at the critical damping 1 / (4 kappa) of its own state; a start from
    zero has no quotient and runs them at the floor.  Checked against the
    damped-wave recurrence written out for the first block."""
    kappa, F, floor = 0.02, 1.0, 1.0
    dt_of = lambda th: 0.05 * np.sqrt(th)
    res = apt.apt_solve(lambda u: F - kappa * u, np.array([u0]), dt=dt_of(floor), theta=floor, hd=1.0,
                        fnorm=F, ncell=1, check_every=10, n_iter=10, adapt=(np.array([F]), dt_of))
    th = 1.0 / (4 * kappa) if u0 != 0.0 else floor
    u_want, v_want = _scalar_sweeps(u0, 0.0, th, dt_of(th), kappa, F, 10)
    assert res.u[0] == pytest.approx(u_want, rel=1e-14)
    assert res.v[0] == pytest.approx(v_want, rel=1e-14)


def test_adaptive_damping_reaches_direct_solution_faster():
    prob = W.cantilever2d(16, 8)
    phi = W.initial_phi(prob)
    plain, _ = design.solve(phi, prob, params=design.AptParams(theta=1.0, tol=1e-9, check_every=20))
    fast, _ = design.solve(phi, prob, params=design.AptParams(theta=1.0, tol=1e-9, check_every=20, adapt=True))
    assert plain.converged and fast.converged
    assert fast.iters < plain.iters / 2
    assert fast.theta > 1.0
    E = design.material(phi, prob)
    ud = assembly.direct_solve(design.stiffness(E, prob), design.load_vector(prob), prob)
    assert np.linalg.norm(fast.u - ud) / np.linalg.norm(ud) < 1e-7
