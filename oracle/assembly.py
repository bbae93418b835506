"""Element-by-element sparse assembly and direct solves (oracle; test infrastructure only).

An independent construction of the stiffness that ``elastic.internal_force`` and
``heat.internal_flux`` apply matrix-free: here every strain is written as an
explicit row of (unknown index, coefficient) pairs from the grid indices, and
K = sum over strains of B^T C B is summed entry by entry with scipy.sparse.
Unknowns are numbered by their flat index in the canonical padded layout;
padding and Dirichlet slots are removed before a solve.  Used for the direct
solves that pin the pseudo-transient fixed point on small grids.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import CLAMPED, ELASTIC, dof_valid_mask
from .elastic import lame


def _flat(shape, comp, idx3):
    """Flat canonical index of component comp at spatial index tuple (i, j[, k])."""
    ndim = len(idx3)
    # canonical array axes: comp, (z,) y, x
    sub = (comp,) + tuple(idx3[ndim - 1 - r] for r in range(ndim))
    return np.ravel_multi_index(sub, shape)


def _grid(ranges):
    mesh = np.meshgrid(*[np.arange(r) for r in ranges], indexing="ij")
    return [m.ravel() for m in mesh]


def elastic_stiffness(E, prob):
    """Assemble K (size = canonical padded array length) for cell moduli E."""
    ndim, n, h, side = prob.ndim, prob.n, prob.h, prob.side
    shape = prob.u_shape()
    N = int(np.prod(shape))
    lam, mu = lame(E, prob.nu)
    hd = h ** ndim
    rows, cols, vals = [], [], []

    # --- normal strains at cells: eps_aa = (u_a(c + e_a) - u_a(c)) / h
    cell_idx = _grid(n)                      # i, j[, k] arrays over all cells
    ncell = cell_idx[0].size
    cell_flat_E = np.ravel_multi_index(tuple(cell_idx[ndim - 1 - r] for r in range(ndim)),
                                       prob.cell_shape())
    lam_c = lam.ravel()[cell_flat_E]
    mu_c = mu.ravel()[cell_flat_E]
    D = []
    for a in range(ndim):
        hi = list(cell_idx)
        hi[a] = cell_idx[a] + 1
        r = np.arange(ncell)
        D.append(sp.csr_matrix((np.concatenate([np.full(ncell, 1.0 / h), np.full(ncell, -1.0 / h)]),
                                (np.concatenate([r, r]),
                                 np.concatenate([_flat(shape, a, hi), _flat(shape, a, cell_idx)]))),
                               shape=(ncell, N)))
    K = sp.csr_matrix((N, N))
    for a in range(ndim):
        for b in range(ndim):
            c = hd * (lam_c + (2.0 * mu_c if a == b else 0.0))
            K = K + D[a].T @ sp.diags(c) @ D[b]

    # --- shear strains on edges
    pairs = [(0, 1)] if ndim == 2 else [(0, 1), (0, 2), (1, 2)]
    mu_grid = mu
    for (a, b) in pairs:
        ranges = [n[s] + 1 if s in (a, b) else n[s] for s in range(ndim)]
        eidx = _grid(ranges)
        ne = eidx[0].size
        active = np.ones(ne, dtype=bool)
        for s in (a, b):
            if side[2 * s] != CLAMPED:
                active &= eidx[s] != 0
            if side[2 * s + 1] != CLAMPED:
                active &= eidx[s] != n[s]
        eidx = [x[active] for x in eidx]
        ne = eidx[0].size
        # edge modulus: mean over the 4 surrounding cells, absent cells contribute 0
        mu_e = np.zeros(ne)
        for da in (-1, 0):
            for db in (-1, 0):
                ci = list(eidx)
                ci[a] = eidx[a] + da
                ci[b] = eidx[b] + db
                ok = (ci[a] >= 0) & (ci[a] < n[a]) & (ci[b] >= 0) & (ci[b] < n[b])
                sub = tuple(np.where(ok, ci[ndim - 1 - r], 0) for r in range(ndim))
                mu_e += np.where(ok, mu_grid[sub], 0.0) * 0.25
        er, ec, ev = [], [], []
        rowid = np.arange(ne)
        # gamma = (u_a(.., j) - u_a(.., j-1))/h along b  +  (u_b(i) - u_b(i-1))/h along a
        for (comp, along) in ((a, b), (b, a)):
            for (off, sgn) in ((0, 1.0), (-1, -1.0)):
                pos = list(eidx)
                pos[along] = eidx[along] + off
                coef = np.full(ne, sgn / h)
                # ghost reflection on clamped sides: index -1 -> -(index 0), index n -> -(index n-1)
                lo_ghost = pos[along] < 0
                hi_ghost = pos[along] >= n[along]
                p2 = list(pos)
                p2[along] = np.where(lo_ghost, 0, np.where(hi_ghost, n[along] - 1, pos[along]))
                coef = np.where(lo_ghost | hi_ghost, -coef, coef)
                er.append(rowid)
                ec.append(_flat(shape, comp, p2))
                ev.append(coef)
        G = sp.csr_matrix((np.concatenate(ev), (np.concatenate(er), np.concatenate(ec))),
                          shape=(ne, N))
        K = K + G.T @ sp.diags(hd * mu_e) @ G
    return K.tocsr()


def heat_stiffness(k, prob):
    """Assemble the heat conduction matrix (cells in the canonical [nz][ny][nx] order)."""
    ndim, n, h = prob.ndim, prob.n, prob.h
    shape = prob.cell_shape()
    N = int(np.prod(shape))
    s = h ** (ndim - 2)
    kf = k.ravel()
    rows, cols, vals = [], [], []
    cells = _grid(n)
    flat = np.ravel_multi_index(tuple(cells[ndim - 1 - r] for r in range(ndim)), shape)
    for a in range(ndim):
        ok = cells[a] < n[a] - 1
        nb = list(cells)
        nb[a] = cells[a] + 1
        fa = flat[ok]
        fb = np.ravel_multi_index(tuple(nb[ndim - 1 - r][ok] for r in range(ndim)), shape)
        w = 0.5 * (kf[fa] + kf[fb]) * s
        rows += [fa, fb, fa, fb]
        cols += [fa, fb, fb, fa]
        vals += [w, w, -w, -w]
    fixed = prob.fixed.ravel().astype(np.int64)
    nd = np.zeros(N)
    for bit in range(2 * ndim):
        nd += (fixed >> bit) & 1
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(2.0 * nd * kf * s)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def free_mask(prob):
    if prob.physics == ELASTIC:
        m = dof_valid_mask(prob.ndim, prob.n) & ~prob.fixed.astype(bool)
        return m.ravel()
    return np.ones(prob.ncell, dtype=bool)


def direct_solve(K, F, prob):
    """Solve K u = F on the free unknowns; returns u in the canonical layout."""
    free = free_mask(prob)
    Kf = K[free][:, free].tocsc()
    u = np.zeros(F.size)
    u[free] = spla.spsolve(Kf, F.ravel()[free])
    return u.reshape(F.shape)
