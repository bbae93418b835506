"""Staggered-grid linear elasticity (oracle; test infrastructure only).

The paper discretises the momentum balance of Eq. (3.6) with the stresses of
Eq. (3.9) and the Lame parameters of Eq. (3.10) by finite differences.  The
oracle writes that discretisation as an energy on a staggered (MAC) grid and
takes its exact gradient:

* normal strains eps_aa live at cell centres, from the two face displacements of
  component a bounding the cell;
* engineering shear strains gamma_ab live on cell edges (vertices in 2D), from
  the differences of u_a across b and u_b across a;
* the cell energy is h^d [ lam/2 (sum_a eps_aa)^2 + mu sum_a eps_aa^2 ]
  plus, for each active edge of the cell, h^d (mu_c/4) gamma^2 / 2, so an edge
  carries the arithmetic mean of the (in-domain) cells around it;
* an edge is active only if every boundary side it lies on is clamped; on a
  clamped side the tangential displacement is reflected (ghost = -interior), the
  normal displacement is a Dirichlet unknown held at zero.

In 2D the Lame parameters are used as printed (plane strain).  The residual is
r = F - dPi/du in force units, zero on Dirichlet unknowns.
"""
from __future__ import annotations

import numpy as np

from workloads import CLAMPED


def lame(E, nu):
    """Lame parameters of Eq. (3.10) (the paper writes Poisson's ratio as gamma)."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def ax(ndim, a):
    """Array axis of spatial axis a (arrays are stored z, y, x)."""
    return ndim - 1 - a


def split(u, ndim, n):
    """Canonical padded array -> list of natural component arrays."""
    comps = []
    for a in range(ndim):
        sl = []
        for r in range(ndim):
            sa = ndim - 1 - r
            sl.append(slice(0, n[sa] + 1) if sa == a else slice(0, n[sa]))
        comps.append(np.array(u[a][tuple(sl)], dtype=np.float64))
    return comps


def join(comps, ndim, n):
    """Natural component arrays -> canonical padded array (padding zero)."""
    out = np.zeros((ndim,) + tuple(int(x) + 1 for x in reversed(n)))
    for a in range(ndim):
        sl = []
        for r in range(ndim):
            sa = ndim - 1 - r
            sl.append(slice(0, n[sa] + 1) if sa == a else slice(0, n[sa]))
        out[a][tuple(sl)] = comps[a]
    return out


def _extend_tangential(ua, ndim, b, side):
    """Append ghost layers to u_a along axis b (b != a): index -1 and n_b.
    Ghost = -interior on a clamped side, 0 otherwise (edges there are inactive)."""
    axb = ax(ndim, b)
    first = np.take(ua, [0], axis=axb)
    last = np.take(ua, [ua.shape[axb] - 1], axis=axb)
    lo = -first if side[2 * b] == CLAMPED else np.zeros_like(first)
    hi = -last if side[2 * b + 1] == CLAMPED else np.zeros_like(last)
    return np.concatenate([lo, ua, hi], axis=axb)


def _fold_tangential(g_ext, ndim, b, side):
    """Transpose of _extend_tangential: fold ghost gradients back onto the interior."""
    axb = ax(ndim, b)
    m = g_ext.shape[axb]
    g = np.array(np.take(g_ext, np.arange(1, m - 1), axis=axb))
    if side[2 * b] == CLAMPED:
        sl = [slice(None)] * ndim
        sl[axb] = slice(0, 1)
        g[tuple(sl)] -= np.take(g_ext, [0], axis=axb)
    if side[2 * b + 1] == CLAMPED:
        sl = [slice(None)] * ndim
        sl[axb] = slice(m - 3, m - 2)
        g[tuple(sl)] -= np.take(g_ext, [m - 1], axis=axb)
    return g


def _diff(x, axis):
    return np.diff(x, axis=axis)


def _diff_T(g, axis):
    """Adjoint of np.diff along axis: maps shape m-1 -> m."""
    pad_lo = [(0, 0)] * g.ndim
    pad_hi = [(0, 0)] * g.ndim
    pad_lo[axis] = (1, 0)
    pad_hi[axis] = (0, 1)
    return np.pad(g, pad_lo) - np.pad(g, pad_hi)


def shear_pairs(ndim):
    return [(0, 1)] if ndim == 2 else [(0, 1), (0, 2), (1, 2)]


def edge_active(ndim, n, a, b, side):
    """Activity mask of the (a, b) shear edges: shape has n_a+1 along a,
    n_b+1 along b, n_c along the remaining axis."""
    shape = [0] * ndim
    for s in range(ndim):
        shape[ax(ndim, s)] = n[s] + 1 if s in (a, b) else n[s]
    act = np.ones(shape, dtype=bool)
    for s in (a, b):
        for hi in (0, 1):
            if side[2 * s + hi] != CLAMPED:
                sl = [slice(None)] * ndim
                sl[ax(ndim, s)] = n[s] if hi else 0
                act[tuple(sl)] = False
    return act


def edge_mean(mu, ndim, a, b):
    """Arithmetic-mean weight at (a, b) edges: (1/4) * sum of the in-domain cells
    around the edge (cells outside the domain are absent)."""
    pad = [(0, 0)] * ndim
    pad[ax(ndim, a)] = (1, 1)
    pad[ax(ndim, b)] = (1, 1)
    m = np.pad(mu, pad)
    A, B = ax(ndim, a), ax(ndim, b)
    s = 0.0
    for da in (0, 1):
        for db in (0, 1):
            sl = [slice(None)] * ndim
            sl[A] = slice(da, da + m.shape[A] - 1)
            sl[B] = slice(db, db + m.shape[B] - 1)
            s = s + m[tuple(sl)]
    return 0.25 * s


def strains(u, prob):
    """Normal strains at cells and engineering shear strains on edges.
    Returns (eps[a] arrays of cell shape, gam dict {(a,b): edge array})."""
    ndim, n, h, side = prob.ndim, prob.n, prob.h, prob.side
    comps = split(u, ndim, n)
    eps = [_diff(comps[a], ax(ndim, a)) / h for a in range(ndim)]
    gam = {}
    for (a, b) in shear_pairs(ndim):
        ua_ext = _extend_tangential(comps[a], ndim, b, side)
        ub_ext = _extend_tangential(comps[b], ndim, a, side)
        gam[(a, b)] = _diff(ua_ext, ax(ndim, b)) / h + _diff(ub_ext, ax(ndim, a)) / h
    return eps, gam


def cell_energy(u, E, prob):
    """Per-cell strain energy W_c (cell shape); sum equals the total energy Pi."""
    ndim, n, h = prob.ndim, prob.n, prob.h
    lam, mu = lame(E, prob.nu)
    eps, gam = strains(u, prob)
    tr = sum(eps)
    W = h ** ndim * (0.5 * lam * tr * tr + mu * sum(e * e for e in eps))
    for (a, b), g in gam.items():
        act = edge_active(ndim, n, a, b, prob.side)
        e2 = np.where(act, 0.5 * g * g, 0.0)
        # every cell gets (mu_c/4) * gamma^2/2 from each of its 4 edges of this family
        A, B = ax(ndim, a), ax(ndim, b)
        acc = np.zeros_like(E)
        for da in (0, 1):
            for db in (0, 1):
                sl = [slice(None)] * ndim
                sl[A] = slice(da, da + n[a])
                sl[B] = slice(db, db + n[b])
                acc = acc + e2[tuple(sl)]
        W = W + h ** ndim * 0.25 * mu * acc
    return W


def energy(u, E, prob):
    return float(np.sum(cell_energy(u, E, prob)))


def internal_force(u, E, prob):
    """Gradient dPi/du of the elastic energy, in the canonical padded layout."""
    ndim, n, h, side = prob.ndim, prob.n, prob.h, prob.side
    lam, mu = lame(E, prob.nu)
    eps, gam = strains(u, prob)
    tr = sum(eps)
    grads = [None] * ndim
    for a in range(ndim):
        sig = lam * tr + 2.0 * mu * eps[a]                      # sigma_aa at cells
        grads[a] = _diff_T(h ** ndim * sig / h, ax(ndim, a))
    for (a, b), g in gam.items():
        act = edge_active(ndim, n, a, b, side)
        tau = np.where(act, edge_mean(mu, ndim, a, b) * g, 0.0)   # shear stress on edges
        coef = h ** ndim * tau / h
        ga_ext = _diff_T(coef, ax(ndim, b))
        gb_ext = _diff_T(coef, ax(ndim, a))
        grads[a] = grads[a] + _fold_tangential(ga_ext, ndim, b, side)
        grads[b] = grads[b] + _fold_tangential(gb_ext, ndim, a, side)
    return join(grads, ndim, n)


def residual(u, E, prob, F=None):
    """r = F - dPi/du (force units), zero on Dirichlet and padding slots."""
    F = prob.load if F is None else F
    r = F - internal_force(u, E, prob)
    r[prob.fixed.astype(bool)] = 0.0
    r = join(split(r, prob.ndim, prob.n), prob.ndim, prob.n)
    return r


def modulus(phi, prob):
    """Young's modulus per cell.  Single phase: the modified SIMP law
    E = Emin + phi^p (E0 - Emin).  Several solid phases plus void: the sum of
    E_m phi_m^p over the solid phases and the void phase 1 - sum(phi) (Eq. (3.8)).
    The laws take every phase fraction clamped to [0, 1] (a reading: fractions can
    leave the range under the penalty update of Eq. (2.13))."""
    q = np.clip(phi, 0.0, 1.0)
    if prob.nphase > 1:
        void = np.clip(1.0 - q.sum(axis=0), 0.0, 1.0)
        E = prob.e_phase[-1] * void ** prob.p
        for m in range(prob.nphase):
            E = E + prob.e_phase[m] * q[m] ** prob.p
        return E
    return prob.emin + q[0] ** prob.p * (prob.e0 - prob.emin)


def _inside(x):
    return ((x >= 0.0) & (x <= 1.0)).astype(np.float64)


def modulus_derivative(phi, prob):
    """dE/dphi_m per stored phase (shape of phi); zero where a clamped fraction
    is outside [0, 1]."""
    p = prob.p
    q = np.clip(phi, 0.0, 1.0)
    if prob.nphase > 1:
        vraw = 1.0 - q.sum(axis=0)
        void = np.clip(vraw, 0.0, 1.0)
        out = np.empty_like(phi)
        for m in range(prob.nphase):
            out[m] = p * (prob.e_phase[m] * q[m] ** (p - 1) * _inside(phi[m])
                          - prob.e_phase[-1] * void ** (p - 1) * _inside(vraw))
        return out
    return (p * q[0] ** (p - 1) * (prob.e0 - prob.emin) * _inside(phi[0]))[None]


def p_wave_max(E, prob):
    """Largest P-wave modulus lam + 2 mu over the cells (sets the explicit step)."""
    lam, mu = lame(np.max(E), prob.nu)
    return lam + 2.0 * mu
