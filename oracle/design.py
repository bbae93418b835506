"""Compliance, sensitivity, phase-field update and the design step (oracle; test
infrastructure only).

* Compliance: C = F . u, the discrete form of the thermal compliance of Eq. (2.7)
  and of the mechanical compliance of Eq. (3.7); at equilibrium it equals
  u^T K u = 2 Pi(u).
* Sensitivity (Section 2.3): the total derivative of the solved compliance,
  dC/dphi_c = -u^T (dK/dphi_c) u = -E'(phi_c) * 2 W_c(u) / E_c, because K is linear
  in the cell moduli and compliance is self-adjoint.  (The code of Fig. 2
  differentiates at fixed state, which is the same magnitude with the opposite
  sign; the total derivative is what a finite difference of the solved compliance
  measures.)  For a general adjoint state w the bilinear form replaces 2 W_c.
* Phase update: the normalised sensitivity step of Eqs. (3.2)-(3.3) without the
  penalty terms, one explicit Allen-Cahn step with the double-well of Eq. (2.15)
  (forward Euler in time and finite differences in space as in Section 2.4, with
  no-flux mirror boundaries), then the volume constraint enforced exactly by a
  uniform shift s found by bisection in FP64 (the role of the penalty J_v of
  Eq. (2.10)).  Several solid phases are projected one after another, each bounded
  above by what the earlier phases leave; cells of a void region are held at 0 and
  passive-solid cells at 1 (phase 0) by the same bounds.
* Design step (Fig. 4): relax the state, evaluate compliance and sensitivity,
  update the design.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from workloads import ELASTIC, HEAT
from . import apt, assembly, elastic, heat


# ------------------------------------------------------------------------------ physics dispatch

def material(phi, prob):
    return elastic.modulus(phi, prob) if prob.physics == ELASTIC else heat.conductivity(phi, prob)


def material_derivative(phi, prob):
    if prob.physics == ELASTIC:
        return elastic.modulus_derivative(phi, prob)
    return heat.conductivity_derivative(phi, prob)


def residual(u, E, prob, F=None):
    if prob.physics == ELASTIC:
        return elastic.residual(u, E, prob, F)
    return heat.residual(u, E, prob, F)


def cell_energy(u, E, prob):
    if prob.physics == ELASTIC:
        return elastic.cell_energy(u, E, prob)
    return heat.cell_energy(u, E, prob)


def load_vector(prob):
    if prob.physics == ELASTIC:
        F = np.array(prob.load, dtype=np.float64)
        F[prob.fixed.astype(bool)] = 0.0
        return F
    return heat.source(prob)


def wave_modulus_max(E, prob):
    return elastic.p_wave_max(E, prob) if prob.physics == ELASTIC else float(np.max(E))


# ------------------------------------------------------------------------------ solve

@dataclass
class AptParams:
    theta: float = 1.0
    dt: float | None = None       # None: h sqrt(theta / (2 d M_max))
    tol: float = 1e-6
    check_every: int = 100
    max_iter: int = 10**7
    adapt: bool = False           # re-choose theta at every check (critical damping of the state's mode)


def stiffness(E, prob):
    if prob.physics == ELASTIC:
        return assembly.elastic_stiffness(E, prob)
    return assembly.heat_stiffness(E, prob)


def assembled_residual(K, F, prob):
    """r(u) = F - K u with the element-assembled stiffness (equal to the matrix-free
    gradient of the energy; the tests pin the two against each other), zero on
    Dirichlet and padding slots."""
    free = assembly.free_mask(prob).reshape(F.shape)

    def fn(u):
        r = F - (K @ u.ravel()).reshape(F.shape)
        r[~free] = 0.0
        return r
    return fn


def solve(phi, prob, u0=None, params=AptParams(), n_iter=None):
    E = material(phi, prob)
    F = load_vector(prob)
    u0 = np.zeros_like(F) if u0 is None else u0
    dt = params.dt if params.dt else apt.default_dt(prob.h, prob.ndim, wave_modulus_max(E, prob),
                                                    params.theta)
    fnorm = float(np.sqrt(np.sum(F * F)))
    rfn = assembled_residual(stiffness(E, prob), F, prob)
    mmax = wave_modulus_max(E, prob)
    adapt = (F, lambda th: apt.default_dt(prob.h, prob.ndim, mmax, th)) if params.adapt else None
    res = apt.apt_solve(rfn, u0, dt=dt, theta=params.theta,
                        hd=prob.h ** prob.ndim, fnorm=fnorm, ncell=prob.ncell, tol=params.tol,
                        check_every=params.check_every, max_iter=params.max_iter, n_iter=n_iter,
                        adapt=adapt)
    return res, dt


# ------------------------------------------------------------------------------ compliance / sensitivity

def compliance(u, prob):
    return float(np.sum(load_vector(prob) * u))


def strain_energy_total(u, phi, prob):
    return float(np.sum(cell_energy(u, material(phi, prob), prob)))


def sensitivity(u, phi, prob, w=None):
    """g_m = dC/dphi_m (shape of phi): -E'_m(phi_c) B_c(w, u) / E_c with the cell
    bilinear form B_c(w, u) = (W_c(w + u) - W_c(w - u)) / 2, so that
    B_c(u, u) = 2 W_c(u) (w defaults to u, the self-adjoint compliance case)."""
    E = material(phi, prob)
    if w is None:
        B = 2.0 * cell_energy(u, E, prob)
    else:
        B = 0.5 * (cell_energy(w + u, E, prob) - cell_energy(w - u, E, prob))
    dE = material_derivative(phi, prob)
    return -dE * (B / E)[None]


# ------------------------------------------------------------------------------ phase update

@dataclass
class PhaseParams:
    alpha_h: float = 0.1          # Eq. (3.2) weight
    gamma: float = 3e-5           # interface parameter of Eq. (2.14)
    dt_ac: float | None = None    # None: 0.9 min(h^2 / (4 d gamma), 32 / pi^2)
    bisect_iters: int = 64
    vol_frac: tuple = ()          # default: the problem's


def default_dt_ac(h, ndim, gamma):
    return 0.9 * min(h * h / (4.0 * ndim * gamma), 32.0 / math.pi ** 2)


def double_well_derivative(phi):
    """w'(phi) for w = sin^2(pi phi)/64 (Eq. (2.15))."""
    return (math.pi / 64.0) * np.sin(2.0 * math.pi * phi)


def laplacian_mirror(phi, h):
    """Five/seven-point Laplacian with mirror (no-flux) boundaries."""
    p = np.pad(phi, 1, mode="edge")
    out = np.zeros_like(phi)
    nd = phi.ndim
    for A in range(nd):
        lo = [slice(1, -1)] * nd
        hi = [slice(1, -1)] * nd
        lo[A] = slice(0, -2)
        hi[A] = slice(2, None)
        out += p[tuple(lo)] + p[tuple(hi)] - 2.0 * phi
    return out / (h * h)


def volume(phi_shifted_clamped):
    return float(np.sum(phi_shifted_clamped))


def bisect_shift(x, ub, target, iters=64, lb=0.0):
    """s with sum(clip(x + s, lb, ub)) = target, by bisection on [-max x, max(ub) - min x]."""
    lo = -float(np.max(x))
    hi = float(np.max(ub)) - float(np.min(x))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if float(np.sum(np.clip(x + mid, lb, ub))) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def region_bounds(prob, m, used):
    """Per-cell bounds of phase m: void-region cells held at 0, passive-solid cells
    hold phase 0 at 1 (later phases then have no room), design cells in
    [0, 1 - used] (Section 3.4's void region as a hard constraint)."""
    ub = 1.0 - used
    lb = np.zeros_like(ub)
    reg = prob.region
    if reg is not None:
        ub = np.where(reg == 1, 0.0, ub)
        if m == 0:
            lb = np.where(reg == 2, 1.0, lb)
            ub = np.where(reg == 2, 1.0, ub)
    return lb, ub


@dataclass
class PhaseInfo:
    shift: list = field(default_factory=list)
    volume: list = field(default_factory=list)
    gmax: list = field(default_factory=list)


def sensitivity_step(phi_m, g_m, alpha_h):
    """Eqs. (3.2)-(3.3) without the penalty terms: the sensitivity is divided by its
    largest magnitude over the cells of the phase, and the design moves against it
    by alpha_h (downhill for the compliance, whose sensitivity g = dC/dphi this is).
    Returns (phi', max|g|); a zero sensitivity leaves the phase unchanged."""
    gmax = float(np.max(np.abs(g_m)))
    ghat = g_m / gmax if gmax > 0 else np.zeros_like(g_m)
    return phi_m - alpha_h * ghat, gmax


def allen_cahn_step(p, h, gamma, dt_ac):
    """One forward-Euler step of the Allen-Cahn gradient flow of the interface
    energy of Section 2.4 (double well of Eq. (2.15) plus gamma/2 |grad phi|^2,
    mobility 1): phi <- phi - dt_ac (w'(phi) - gamma Lap_h phi), with the mirror
    (no-flux) Laplacian."""
    return p - dt_ac * (double_well_derivative(p) - gamma * laplacian_mirror(p, h))


def phase_update(phi, g, prob, params=PhaseParams()):
    """Normalised sensitivity step, Allen-Cahn step, exact volume projection.
    ``params.dt_ac`` None selects the default step; 0 skips the Allen-Cahn step."""
    h, nd = prob.h, prob.ndim
    dt_ac = params.dt_ac if params.dt_ac is not None else default_dt_ac(h, nd, params.gamma)
    vf = params.vol_frac if params.vol_frac else prob.vol_frac
    out = np.empty_like(phi)
    info = PhaseInfo()
    used = np.zeros(phi.shape[1:])
    N = phi[0].size
    for m in range(phi.shape[0]):
        p1, gmax = sensitivity_step(phi[m], g[m], params.alpha_h)
        p2 = allen_cahn_step(p1, h, params.gamma, dt_ac) if dt_ac != 0.0 else p1
        lb, ub = region_bounds(prob, m, used)
        s = bisect_shift(p2, ub, vf[m] * N, params.bisect_iters, lb)
        out[m] = np.clip(p2 + s, lb, ub)
        used = used + out[m]
        info.shift.append(s)
        info.volume.append(float(np.mean(out[m])))
        info.gmax.append(gmax)
    return out, info


# ------------------------------------------------------------------------------ design loop

@dataclass
class StepRecord:
    iters: int
    rho: float
    r_pde: float
    compliance: float
    energy2: float
    shift: list
    volume: list
    gmax: list
    dt: float


def design_step(phi, u, prob, apt_params=AptParams(), phase_params=PhaseParams(), n_iter=None):
    """One loop of Fig. 4: state relaxation (warm-started u, zero velocity),
    compliance and sensitivity at the relaxed state, design update."""
    res, dt = solve(phi, prob, u, apt_params, n_iter)
    u = res.u
    C = compliance(u, prob)
    e2 = 2.0 * strain_energy_total(u, phi, prob)
    g = sensitivity(u, phi, prob)
    phi_new, info = phase_update(phi, g, prob, phase_params)
    rec = StepRecord(res.iters, res.rho, res.r_pde, C, e2, info.shift, info.volume, info.gmax, dt)
    return phi_new, u, g, rec


def optimize(prob, phi0, steps, apt_params=AptParams(), phase_params=PhaseParams(),
             replay_iters=None, u0=None):
    phi = np.array(phi0, dtype=np.float64)
    u = np.zeros(prob.u_shape() if prob.physics == ELASTIC else prob.cell_shape()) if u0 is None else u0
    hist = []
    for s in range(steps):
        n_iter = None if replay_iters is None else int(replay_iters[s])
        phi, u, g, rec = design_step(phi, u, prob, apt_params, phase_params, n_iter)
        hist.append(rec)
    return phi, u, hist
