"""Pseudo-transient relaxation (oracle; test infrastructure only).

Section 2.2: the stationary problem R(u) = 0 is relaxed in pseudo-time.

* Plain PT (Eq. (2.4), elastic Eq. (3.11)):  u^{n+1} = u^n + dt R(u^n).
* Accelerated PT (damped wave, Eqs. (2.5)-(2.6), elastic Eq. (3.12)):
      theta (u^{n+1} - 2u^n + u^{n-1})/dt^2 + (u^{n+1} - u^n)/dt = R(u^n).
  With the pseudo-velocity v^{n+1} = (u^{n+1} - u^n)/dt this is
      v^{n+1} = (theta v^n + dt R(u^n)) / (theta + dt),   u^{n+1} = u^n + dt v^{n+1},
  and theta = 0 gives back plain PT.

R is the residual density: the force residual r = F - K u divided by the cell
volume h^d.  The stop rule checks rho = ||r||_2 / ||F||_2 on every
``check_every``-th sweep (computed from the state the sweep starts from) and
returns the state that sweep produces.  ``r_pde`` is the residual norm of
Eq. (3.5): sqrt(sum R^2) / (number of cells).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class SolveResult:
    u: np.ndarray
    v: np.ndarray
    iters: int
    rho: float
    r_pde: float
    converged: bool
    diverged: bool
    theta: float = 0.0
    dt: float = 0.0


def default_dt(h, ndim, m_max, theta):
    """Pseudo-time step: h * sqrt(theta / (2 d M_max)) for the damped wave (the
    paper's dx/2 for unit-conductivity 2D heat), h^2 / (2 d M_max) for plain PT."""
    if theta > 0:
        return h * math.sqrt(theta / (2.0 * ndim * m_max))
    return h * h / (2.0 * ndim * m_max)


def adapted_theta(u, r, F, hd, theta_min, theta_max=1e6):
    """Damping that critically damps the mode of the current state: with the
    Rayleigh quotient lam = u.Ku / (h^d u.u) (u.Ku = u.F - u.r) of the pseudo-time
    operator, the damped wave theta u'' + u' + lam u = 0 is critically damped at
    theta = 1 / (4 lam); never below theta_min.  Returns None when u is zero."""
    uu = float(np.sum(u * u))
    if uu <= 0.0:
        return None
    uKu = float(np.sum(u * F)) - float(np.sum(u * r))
    if not uKu > 0.0:
        return None
    lam = uKu / (hd * uu)
    return min(max(theta_min, 0.25 / lam), theta_max)


def apt_solve(residual_fn, u0, *, dt, theta, hd, fnorm, ncell, tol=1e-6, check_every=100,
              max_iter=10**7, n_iter=None, v0=None, div_factor=1e4, adapt=None):
    """Run sweeps from (u0, v0=0).  With n_iter given, run exactly that many sweeps
    (the stop rule is still evaluated for reporting).  adapt = (F, dt_of_theta):
    theta is chosen with `adapted_theta` (floor: the given theta) from the
    starting state before the first sweep (a state of zeros has no quotient and
    keeps the floor) and again after every checking sweep that does not stop the
    iteration, from the state that sweep produced, with the step
    dt_of_theta(theta); the new values apply from the next sweep."""
    theta_min = theta
    u = np.array(u0, dtype=np.float64)
    v = np.zeros_like(u) if v0 is None else np.array(v0, dtype=np.float64)
    it = 0
    rho = math.inf
    r_pde = math.inf
    first = None
    limit = n_iter if n_iter is not None else max_iter
    converged = diverged = False
    if adapt is not None:
        th = adapted_theta(u, residual_fn(u), adapt[0], hd, theta_min)
        if th is not None:
            theta, dt = th, adapt[1](th)
    while it < limit:
        r = residual_fn(u)
        it += 1
        check = (it % check_every == 0) or (n_iter is not None and it == n_iter)
        if check:
            ss = float(np.sum(r * r))
            rho = math.sqrt(ss) / fnorm
            r_pde = math.sqrt(ss) / hd / ncell
            if first is None:
                first = rho
        v = (theta * v + dt * (r / hd)) / (theta + dt)
        u = u + dt * v
        if check:
            if not math.isfinite(rho) or rho > div_factor * max(first, tol):
                diverged = True
                break
            if n_iter is None and rho <= tol:
                converged = True
                break
            if adapt is not None and it < limit:
                th = adapted_theta(u, residual_fn(u), adapt[0], hd, theta_min)
                if th is not None:
                    theta, dt = th, adapt[1](th)
    if n_iter is not None:
        converged = rho <= tol
    return SolveResult(u, v, it, rho, r_pde, converged, diverged, theta, dt)
