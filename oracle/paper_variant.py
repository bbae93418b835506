"""The paper's own update schedule (oracle; test infrastructure only).

Besides the solve-to-tolerance / Allen-Cahn / exact-projection loop of
`oracle.design`, the paper runs (Sections 2.4-2.5 and the examples of Section 3):

* a hybrid relaxation with fixed counts: n_APT damped-wave sweeps (Eqs. (2.5)-(2.6),
  elastic Eq. (3.12)) followed by n_PT plain pseudo-transient sweeps (Eq. (2.4),
  elastic Eq. (3.11)), with no stop rule;
* the penalty update of Eq. (2.13) in its normalised form of Section 3.1,
      phi_i <- phi_i - (alpha_h g_i / max|g_i| + alpha_v dJ_v/dphi_i + alpha_1 dJ_1/dphi_i),
  with the volume penalty J_v = sum_i (int phi_i dOmega - V_i)^2 (Eq. (2.10)) and the
  partition-of-unity penalty J_1 = int (sum_i phi_i - 1)^2 dOmega (Eq. (2.11));
* one explicit Cahn-Hilliard step (Eq. (2.14), forward Euler in time, finite
  differences in space, Section 2.4): mu = w'(phi) - gamma Lap(phi),
  phi <- phi + dt3 D Lap(mu), no-flux (mirror) boundaries for both fields;
* the void-region penalty of the drone example (Section 3.4):
  alpha_b dJ_b/dphi with J_b = (int_{Omega_b} phi dOmega - V^b)^2, V^b = 0 for a
  solid phase (the void phase, V^b = 1, is implicit here); passive-solid cells are
  reset to phase 0 after the step.

Readings (the paper leaves them open): the integral is the cell sum times h^d; the
target V_i of J_v is the volume V_f,i |Omega| (the printed form compares an
integral with a fraction, which agrees when |Omega| = 1); the gradient of every
penalty is taken at the design before the step (one Jacobi step for all phases).
The CH step uses the same mirror Laplacian as the Allen-Cahn step, so Lap(Lap) is
the 13-point (2D) / 25-point (3D) biharmonic stencil.  Default dt3 = 500 h^4
capped at 0.9 of the step's stability limit (binding in 3D), D = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import design


@dataclass
class PenaltyParams:
    alpha_h: float = 0.1          # normalised-sensitivity weight (Section 3.1)
    alpha_v: float = 1e5          # volume-penalty weight
    alpha_1: float = 0.0          # partition-of-unity weight (1e4 in the paper, whose
                                  # void phase is a stored field)
    alpha_b: float = 0.0          # void-region weight (the drone example, Section 3.4;
                                  # the region is the problem's REGION_VOID cells)
    gamma: float = 3e-5           # interface parameter of Eq. (2.14)
    mobility: float = 1.0         # D of Eq. (2.14)
    dt_ch: float | None = None    # None: 500 h^4
    vol_frac: tuple = ()          # default: the problem's


def default_dt_ch(h, ndim=2, gamma=3e-5, mobility=1.0):
    """The printed 500 h^4, capped at 0.9 of the explicit stability limit of the
    step on the mirror Laplacian: a mode with Lap = -lam grows by
    1 - dt D lam (w'' + gamma lam), so dt < 2 / (D lam (pi^2/32 + gamma lam)) for
    the largest lam = 4 d / h^2.  (The printed step was set for the paper's wider
    jnp.gradient stencil; with the compact stencil it exceeds the limit in 3D.)"""
    lam = 4.0 * ndim / (h * h)
    limit = 2.0 / (mobility * lam * (math.pi ** 2 / 32.0 + gamma * lam))
    return min(500.0 * h ** 4, 0.9 * limit)


def volume_penalty_gradient(phi_m, vf, h, ndim):
    """dJ_v/dphi_c of one phase: 2 (h^d sum(phi) - V_f N h^d) h^d, the same for
    every cell."""
    hd = h ** ndim
    n = phi_m.size
    return 2.0 * (hd * float(np.sum(phi_m)) - vf * n * hd) * hd


def partition_penalty_gradient(phi, h, ndim):
    """dJ_1/dphi_{i,c} = 2 (sum_i phi_{i,c} - 1) h^d (the same for every phase i)."""
    return 2.0 * (np.sum(phi, axis=0) - 1.0) * h ** ndim


def void_region_gradient(phi_m, region, h, ndim):
    """dJ_b/dphi_c of one solid phase, J_b = (int_{Omega_b} phi dOmega - 0)^2:
    2 (h^d sum_{Omega_b} phi) h^d on the region's cells, 0 elsewhere."""
    hd = h ** ndim
    inb = region == 1
    return np.where(inb, 2.0 * (hd * float(np.sum(phi_m[inb]))) * hd, 0.0)


def cahn_hilliard_step(p, h, gamma, mobility, dt):
    """phi + dt D Lap(w'(phi) - gamma Lap(phi)), mirror boundaries."""
    mu = design.double_well_derivative(p) - gamma * design.laplacian_mirror(p, h)
    return p + dt * mobility * design.laplacian_mirror(mu, h)


def penalty_update(phi, g, prob, params=PenaltyParams()):
    """The sensitivity / penalty step and one Cahn-Hilliard step, every phase
    from the same old design.  Returns (phi_new, info) with info.shift the uniform
    volume-penalty term -alpha_v dJ_v/dphi of each phase."""
    h, nd = prob.h, prob.ndim
    dt = params.dt_ch if params.dt_ch else default_dt_ch(h, nd, params.gamma, params.mobility)
    vf = params.vol_frac if params.vol_frac else prob.vol_frac
    pgrad = partition_penalty_gradient(phi, h, nd) if params.alpha_1 != 0.0 else 0.0
    out = np.empty_like(phi)
    info = design.PhaseInfo()
    for m in range(phi.shape[0]):
        gmax = float(np.max(np.abs(g[m])))
        ghat = g[m] / gmax if gmax > 0 else np.zeros_like(g[m])
        vpen = params.alpha_v * volume_penalty_gradient(phi[m], vf[m], h, nd)
        p1 = phi[m] - params.alpha_h * ghat - vpen - params.alpha_1 * pgrad
        if params.alpha_b != 0.0 and prob.region is not None:
            p1 = p1 - params.alpha_b * void_region_gradient(phi[m], prob.region, h, nd)
        out[m] = cahn_hilliard_step(p1, h, params.gamma, params.mobility, dt)
        if prob.region is not None:
            # passive-solid cells: phase 0 held at 1, the others at 0
            out[m] = np.where(prob.region == 2, 1.0 if m == 0 else 0.0, out[m])
        info.shift.append(-vpen)
        info.volume.append(float(np.mean(out[m])))
        info.gmax.append(gmax)
    return out, info


def hybrid_solve(phi, prob, u0, n_apt, n_pt, theta=1.0, dt=None, dt_pt=None, check_every=None):
    """n_apt damped-wave sweeps, then n_pt plain PT sweeps (theta = 0; the
    velocity plays no part), from u0 and zero velocity.  Returns (u, iters, rho)
    with rho the stop-rule ratio of the last sweep."""
    ce = check_every if check_every else max(n_apt, 2)
    res1, _ = design.solve(phi, prob, u0, design.AptParams(theta=theta, dt=dt, check_every=ce), n_iter=n_apt)
    u, rho, iters = res1.u, res1.rho, res1.iters
    if n_pt > 0:
        res2, _ = design.solve(phi, prob, u, design.AptParams(theta=0.0, dt=dt_pt, check_every=max(n_pt, 2)),
                               n_iter=n_pt)
        u, rho, iters = res2.u, res2.rho, iters + res2.iters
    return u, iters, rho


def paper_step(phi, u, prob, n_apt, n_pt, params=PenaltyParams(), theta=1.0):
    """One loop of Fig. 4 in the paper's schedule: hybrid relaxation from the
    previous state, sensitivity, penalty update, Cahn-Hilliard step."""
    u, iters, rho = hybrid_solve(phi, prob, u, n_apt, n_pt, theta=theta)
    g = design.sensitivity(u, phi, prob)
    C = design.compliance(u, prob)
    phi_new, info = penalty_update(phi, g, prob, params)
    return phi_new, u, g, C, info
