"""Cell-centred steady heat conduction (oracle; test infrastructure only).

Eq. (2.2): -div(kappa grad T) = f, with Neumann (no-flux) sides except the
Dirichlet T=0 faces listed per cell.  Discretised as the energy

  Pi = sum over interior faces (a,b) of  (1/2) k_ab (T_b - T_a)^2 h^(d-2)
     + sum over Dirichlet faces of cell c of  k_c T_c^2 h^(d-2),

with k_ab the arithmetic mean of the two cells and the Dirichlet face realised by
the reflected ghost T = -T_c (face value zero).  The residual is r = F - dPi/dT
with F_c = f_c h^d; per cell, W_c takes k_c/4 (dT)^2 h^(d-2) from each interior
face and its Dirichlet-face terms, so sum_c W_c = Pi.
"""
from __future__ import annotations

import numpy as np


def conductivity(phi, prob):
    """k = kmin + phi^p (k0 - kmin): the modified SIMP form of Eq. (3.1), on phi
    clamped to [0, 1] (as the elastic laws)."""
    q = np.clip(phi[0], 0.0, 1.0)
    return prob.emin + q ** prob.p * (prob.e0 - prob.emin)


def conductivity_derivative(phi, prob):
    """dk/dphi; zero where phi is outside [0, 1]."""
    q = np.clip(phi[0], 0.0, 1.0)
    inside = ((phi[0] >= 0.0) & (phi[0] <= 1.0)).astype(np.float64)
    return (prob.p * q ** (prob.p - 1) * (prob.e0 - prob.emin) * inside)[None]


def _ax(ndim, a):
    return ndim - 1 - a


def dirichlet_counts(prob):
    """Number of Dirichlet faces of every cell."""
    f = prob.fixed.astype(np.int64)
    cnt = np.zeros(prob.cell_shape(), dtype=np.int64)
    for bit in range(2 * prob.ndim):
        cnt += (f >> bit) & 1
    return cnt


def source(prob):
    if prob.load is not None:
        return np.array(prob.load, dtype=np.float64)
    return np.full(prob.cell_shape(), prob.q * prob.h ** prob.ndim)


def cell_energy(T, k, prob):
    ndim, h = prob.ndim, prob.h
    s = h ** (ndim - 2)
    W = dirichlet_counts(prob) * k * T * T * s
    for a in range(ndim):
        A = _ax(ndim, a)
        dT = np.diff(T, axis=A)
        e = dT * dT
        lo = [(0, 0)] * ndim
        hi = [(0, 0)] * ndim
        lo[A] = (1, 0)
        hi[A] = (0, 1)
        # each cell gets k_c/4 * dT^2 from each interior face it touches
        W = W + 0.25 * k * (np.pad(e, lo) + np.pad(e, hi)) * s
    return W


def energy(T, k, prob):
    return float(np.sum(cell_energy(T, k, prob)))


def internal_flux(T, k, prob):
    """dPi/dT per cell."""
    ndim, h = prob.ndim, prob.h
    s = h ** (ndim - 2)
    g = 2.0 * dirichlet_counts(prob) * k * T * s
    for a in range(ndim):
        A = _ax(ndim, a)
        kf = 0.5 * (np.take(k, range(0, k.shape[A] - 1), axis=A) +
                    np.take(k, range(1, k.shape[A]), axis=A))
        flux = kf * np.diff(T, axis=A) * s            # k_f (T_b - T_a) h^(d-2)
        lo = [(0, 0)] * ndim
        hi = [(0, 0)] * ndim
        lo[A] = (1, 0)
        hi[A] = (0, 1)
        # d/dT_a of 1/2 k_f (T_b-T_a)^2 = -flux, d/dT_b = +flux
        g = g + np.pad(flux, lo) - np.pad(flux, hi)
    return g


def residual(T, k, prob, F=None):
    F = source(prob) if F is None else F
    return F - internal_flux(T, k, prob)


def kmax(k):
    return float(np.max(k))
