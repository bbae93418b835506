"""Seeded synthetic problem generators shared by the oracle, the tests and the bench.

This module only builds inputs: grid sizes, boundary-side types, Dirichlet masks,
load vectors and initial designs.  It holds none of the method's arithmetic (no
stiffness, residual, sensitivity or phase-field update) and imports neither the
oracle nor the GPU package.

Canonical layouts (shared interface of the C library, the oracle and the tests):

* Elastic displacement-like arrays (u, v, F, Dirichlet mask) are component-major
  and padded: ``[d][nz+1][ny+1][nx+1]`` (2D: ``[d][ny+1][nx+1]``), x fastest.
  Component ``a`` lives on the faces normal to axis ``a``: its index along axis
  ``a`` runs over ``0..n_a`` and along every other axis ``b`` over ``0..n_b-1``;
  the slot with index ``n_b`` on a foreign axis is padding and stays zero.
* Cell arrays (design phi, sensitivity g, temperature T) are ``[nz][ny][nx]``;
  several phases stack as ``[nphase][...]``.
* Heat Dirichlet faces are given per cell as a bit set: bit ``2a`` marks the face
  on the low side of axis ``a``, bit ``2a+1`` the face on the high side.

Boundary-side codes follow the order -x, +x, -y, +y, -z, +z.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FREE, CLAMPED, ROLLER = 0, 1, 2
ELASTIC, HEAT = 0, 1
REGION_DESIGN, REGION_VOID, REGION_SOLID = 0, 1, 2   # cell roles (passive regions)


@dataclass
class Problem:
    """One design problem on a regular grid (the PDE-constrained statement, Eq. 2.1)."""
    physics: int
    ndim: int
    n: tuple                      # cells per axis (nx, ny[, nz])
    h: float
    e0: float = 1.0
    emin: float = 1e-9
    nu: float = 0.3
    p: float = 3.0
    side: tuple = (FREE,) * 6
    fixed: np.ndarray | None = None   # uint8, canonical layout (see module doc)
    load: np.ndarray | None = None    # float64, canonical layout (force units)
    q: float = 0.0                    # heat: uniform source density used when load is None
    nphase: int = 1                   # >1: solid phases + implicit void
    e_phase: tuple = ()               # moduli of the solid phases, then the void
    vol_frac: tuple = (0.5,)
    name: str = ""
    region: np.ndarray | None = None  # uint8 per cell: 0 design, REGION_VOID, REGION_SOLID

    @property
    def ncell(self) -> int:
        return int(np.prod(self.n))

    def u_shape(self):
        """Canonical padded shape of a displacement-like array."""
        nn = tuple(int(x) + 1 for x in reversed(self.n))
        return (self.ndim,) + nn

    def cell_shape(self):
        return tuple(int(x) for x in reversed(self.n))

    def phi_shape(self):
        nst = self.nphase if self.nphase > 1 else 1
        return (nst,) + self.cell_shape()


def dof_valid_mask(ndim, n):
    """Boolean canonical-layout mask of the slots that hold a real face unknown."""
    shape = (ndim,) + tuple(int(x) + 1 for x in reversed(n))
    m = np.zeros(shape, dtype=bool)
    for a in range(ndim):
        sl = [a]
        for ax_rev in range(ndim):            # array axis order is z, y, x
            ax = ndim - 1 - ax_rev
            sl.append(slice(0, n[ax] + 1) if ax == a else slice(0, n[ax]))
        m[tuple(sl)] = True
    return m


def _side_normal_fixed(ndim, n, side):
    """Dirichlet mask implied by the sides: the normal component on every
    clamped or roller side."""
    fixed = np.zeros((ndim,) + tuple(int(x) + 1 for x in reversed(n)), dtype=np.uint8)
    for a in range(ndim):
        for hi in (0, 1):
            if side[2 * a + hi] in (CLAMPED, ROLLER):
                idx = [a]
                for ax_rev in range(ndim):
                    ax = ndim - 1 - ax_rev
                    if ax == a:
                        idx.append(n[a] if hi else 0)
                    else:
                        idx.append(slice(0, n[ax]))
                fixed[tuple(idx)] = 1
    return fixed


def _idx(ndim, comp, i, j, k=0):
    """Canonical index tuple of component ``comp`` at face position (i, j, k)."""
    return (comp, k, j, i) if ndim == 3 else (comp, j, i)


# --------------------------------------------------------------------------------------
# Elastic configurations (2D / 3D cantilevers, multi-material block)
# --------------------------------------------------------------------------------------

def cantilever2d(nx=64, ny=32, e0=1.0, emin=1e-9, nu=0.3, p=3.0, vol_frac=0.5):
    """2D cantilever: left side clamped, unit point load -y on the y-face nearest
    the middle of the right side (u_y at cell column nx-1, face row ny/2)."""
    side = (CLAMPED, FREE, FREE, FREE, FREE, FREE)
    n = (nx, ny)
    fixed = _side_normal_fixed(2, n, side)
    load = np.zeros((2, ny + 1, nx + 1))
    load[_idx(2, 1, nx - 1, ny // 2)] = -1.0
    return Problem(ELASTIC, 2, n, 1.0 / ny, e0, emin, nu, p, side, fixed, load,
                   vol_frac=(vol_frac,), name=f"cantilever2d_{nx}x{ny}")


def cantilever3d(nx=128, ny=64, nz=64, e0=1.0, emin=1e-9, nu=0.3, p=3.0, vol_frac=0.3):
    """3D cantilever: x=0 face clamped, line load -z of total 1 spread over the
    bottom z-faces of the last cell column along the bottom edge of the x=end face."""
    side = (CLAMPED, FREE, FREE, FREE, FREE, FREE)
    n = (nx, ny, nz)
    fixed = _side_normal_fixed(3, n, side)
    load = np.zeros((3, nz + 1, ny + 1, nx + 1))
    for j in range(ny):
        load[_idx(3, 2, nx - 1, j, 0)] = -1.0 / ny
    return Problem(ELASTIC, 3, n, 1.0 / ny, e0, emin, nu, p, side, fixed, load,
                   vol_frac=(vol_frac,), name=f"cantilever3d_{nx}x{ny}x{nz}")


def multimaterial3d(nx=256, ny=128, nz=128, e_phase=(1.0, 0.5, 1e-9), nu=0.3, p=3.0,
                    vol_frac=(0.2, 0.1)):
    """3D block with two solid phases plus void: distributed -z load of total 1 on
    the top face, the four bottom corner cells pinned on their outer faces."""
    side = (FREE,) * 6
    n = (nx, ny, nz)
    fixed = np.zeros((3, nz + 1, ny + 1, nx + 1), dtype=np.uint8)
    for (ci, cj) in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)):
        fx = 0 if ci == 0 else nx
        fy = 0 if cj == 0 else ny
        fixed[_idx(3, 0, fx, cj, 0)] = 1
        fixed[_idx(3, 1, ci, fy, 0)] = 1
        fixed[_idx(3, 2, ci, cj, 0)] = 1
    load = np.zeros((3, nz + 1, ny + 1, nx + 1))
    load[2, nz, :ny, :nx] = -1.0 / (nx * ny)
    return Problem(ELASTIC, 3, n, 1.0 / ny, 1.0, 0.0, nu, p, side, fixed, load,
                   nphase=len(e_phase) - 1, e_phase=tuple(e_phase), vol_frac=tuple(vol_frac),
                   name=f"multimaterial3d_{nx}x{ny}x{nz}")


def mbb2d(nx=512, ny=128, e_phase=(1.0, 0.775, 0.55, 0.325, 0.1, 1e-6), nu=0.3, p=3.0,
          vol_frac=(0.08,) * 5):
    """The paper's 2D multi-material MBB beam (Section 3.2): a 4 x 1 domain, five
    solid phases plus void (moduli and fractions as printed), a downward unit force
    at the middle of the top side (split over the two top y-faces next to it),
    rollers under both bottom corners (u_y of their bottom faces held).  Reading:
    u_x of the bottom-left corner face is held too, removing the rigid x
    translation the rollers leave free (its reaction is zero by symmetry)."""
    side = (FREE,) * 6
    n = (nx, ny)
    fixed = np.zeros((2, ny + 1, nx + 1), dtype=np.uint8)
    fixed[_idx(2, 1, 0, 0)] = 1
    fixed[_idx(2, 1, nx - 1, 0)] = 1
    fixed[_idx(2, 0, 0, 0)] = 1
    load = np.zeros((2, ny + 1, nx + 1))
    if nx % 2 == 0:
        load[_idx(2, 1, nx // 2 - 1, ny)] = -0.5
        load[_idx(2, 1, nx // 2, ny)] = -0.5
    else:
        load[_idx(2, 1, nx // 2, ny)] = -1.0
    return Problem(ELASTIC, 2, n, 1.0 / ny, 1.0, 0.0, nu, p, side, fixed, load,
                   nphase=len(e_phase) - 1, e_phase=tuple(e_phase), vol_frac=tuple(vol_frac),
                   name=f"mbb2d_{nx}x{ny}")


def drone3d(nx=128, ny=64, nz=128, vol_frac=0.15, void_box=((0.25, 0.75), (0.2, 1.0), (0.25, 0.75)),
            nu=0.3, p=3.0):
    """A synthetic stand-in for the paper's drone skeleton (Section 3.4; the
    geometry of the cited source is not given): a 1 x 0.5 x 1 block (y up), u_y of
    the top faces of the four top corner cells held (the printed rollers), a unit
    downward load on the bottom face of the middle cell, and a void region Omega_b
    (the battery bay) given as a box in units of the sides (default: 20 % of the
    volume).  Reading: u_x and u_z of one top corner face and u_z of a second one
    are held too, removing the rigid motions the rollers leave free."""
    side = (FREE,) * 6
    n = (nx, ny, nz)
    fixed = np.zeros((3, nz + 1, ny + 1, nx + 1), dtype=np.uint8)
    corners = ((0, 0), (nx - 1, 0), (0, nz - 1), (nx - 1, nz - 1))
    for (ci, ck) in corners:
        fixed[_idx(3, 1, ci, ny, ck)] = 1
    fixed[_idx(3, 0, 0, ny - 1, 0)] = 1
    fixed[_idx(3, 2, 0, ny - 1, 0)] = 1
    fixed[_idx(3, 2, nx - 1, ny - 1, 0)] = 1
    load = np.zeros((3, nz + 1, ny + 1, nx + 1))
    load[_idx(3, 1, nx // 2, 0, nz // 2)] = -1.0
    region = np.zeros((nz, ny, nx), dtype=np.uint8)
    (x0, x1), (y0, y1), (z0, z1) = void_box
    xs = slice(int(round(x0 * nx)), int(round(x1 * nx)))
    ys = slice(int(round(y0 * ny)), int(round(y1 * ny)))
    zs = slice(int(round(z0 * nz)), int(round(z1 * nz)))
    region[zs, ys, xs] = REGION_VOID
    return Problem(ELASTIC, 3, n, 1.0 / nx, 1.0, 1e-6, nu, p, side, fixed, load,
                   vol_frac=(vol_frac,), name=f"drone3d_{nx}x{ny}x{nz}", region=region)


def uniform_bar(ndim, n, t=1.0, E=1.0, nu=0.3):
    """Bar under uniform axial traction: roller on x=0, symmetry-plane pins on the
    mid y-face row (and mid z-face layer in 3D), traction t on the x=end faces.
    Returns (problem, phi) with phi chosen so that the SIMP modulus is E exactly
    (e0=E, emin=0, phi=1)."""
    side = (ROLLER,) + (FREE,) * 5
    fixed = _side_normal_fixed(ndim, n, side)
    load = np.zeros((ndim,) + tuple(int(x) + 1 for x in reversed(n)))
    h = 1.0 / n[1]
    if ndim == 2:
        nx, ny = n
        assert ny % 2 == 0
        fixed[1, ny // 2, :nx] = 1
        load[0, :ny, nx] = t * h
    else:
        nx, ny, nz = n
        assert ny % 2 == 0 and nz % 2 == 0
        fixed[1, :nz, ny // 2, :nx] = 1
        fixed[2, nz // 2, :ny, :nx] = 1
        load[0, :nz, :ny, nx] = t * h * h
    prob = Problem(ELASTIC, ndim, tuple(n), h, E, 0.0, nu, 3.0, side, fixed, load,
                   vol_frac=(0.5,), name=f"bar{ndim}d")
    phi = np.ones((1,) + tuple(int(x) for x in reversed(n)))
    return prob, phi


def manufactured_elastic(ndim, n, E=1.0, nu=0.3, amp=(1.0, -0.7, 0.4)):
    """All sides clamped, body force of the smooth field u_a = amp_a * prod sin(pi x_b / L_b),
    sampled at the face centres and scaled by the cell volume (force units).
    Returns (problem, phi, exact_u_canonical).  The body force is the negative
    divergence of the constant-coefficient stress of that field (Navier form)."""
    h = 1.0 / n[1]
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    Ls = [n[a] * h for a in range(ndim)]
    w = [math.pi / L for L in Ls]
    side = (CLAMPED,) * (2 * ndim) + (FREE,) * (6 - 2 * ndim)
    fixed = _side_normal_fixed(ndim, n, side)
    shape = (ndim,) + tuple(int(x) + 1 for x in reversed(n))
    load = np.zeros(shape)
    exact = np.zeros(shape)
    valid = dof_valid_mask(ndim, n)
    for b in range(ndim):
        # face-centre coordinates of component b
        grids = []
        for ax_rev in range(ndim):
            ax = ndim - 1 - ax_rev
            m = n[ax] + 1
            idx = np.arange(m, dtype=float)
            pos = idx * h if ax == b else (idx + 0.5) * h
            grids.append(pos)
        mesh = np.meshgrid(*grids, indexing="ij")       # z, y, x order (or y, x)
        X = list(reversed(mesh))                          # X[ax] is coordinate along axis ax
        s = [np.sin(w[a] * X[a]) for a in range(ndim)]
        c = [np.cos(w[a] * X[a]) for a in range(ndim)]
        prod_s = np.ones_like(X[0])
        for a in range(ndim):
            prod_s = prod_s * s[a]
        lap_sum = sum(wa * wa for wa in w)
        # d/dx_b (div u)
        grad_div = -amp[b] * w[b] ** 2 * prod_s
        for a in range(ndim):
            if a == b:
                continue
            term = amp[a] * w[a] * w[b] * c[a] * c[b]
            for e in range(ndim):
                if e not in (a, b):
                    term = term * s[e]
            grad_div = grad_div + term
        lap_ub = -amp[b] * lap_sum * prod_s
        f_b = -((lam + mu) * grad_div + mu * lap_ub)
        load[b] = f_b * h ** ndim
        exact[b] = amp[b] * prod_s
    load[~valid] = 0.0
    exact[~valid] = 0.0
    load[fixed.astype(bool)] = 0.0
    prob = Problem(ELASTIC, ndim, tuple(n), h, E, 0.0, nu, 3.0, side, fixed, load,
                   vol_frac=(0.5,), name=f"manufactured{ndim}d")
    phi = np.ones((1,) + tuple(int(x) for x in reversed(n)))
    return prob, phi, exact


# --------------------------------------------------------------------------------------
# Heat configurations
# --------------------------------------------------------------------------------------

def heat_slab(n, k=1.0, q=1.0):
    """Dirichlet T=0 on the whole x=0 and x=L sides, Neumann elsewhere, uniform k, q."""
    ndim = len(n)
    fixed = np.zeros(tuple(int(x) for x in reversed(n)), dtype=np.uint8)
    idx_lo = [slice(None)] * ndim
    idx_hi = [slice(None)] * ndim
    idx_lo[ndim - 1] = 0
    idx_hi[ndim - 1] = n[0] - 1
    fixed[tuple(idx_lo)] |= 1
    fixed[tuple(idx_hi)] |= 2
    prob = Problem(HEAT, ndim, tuple(n), 1.0 / n[1], k, 0.0, 0.0, 3.0, (FREE,) * 6, fixed, None,
                   q=q, vol_frac=(0.3,), name="heat_slab")
    phi = np.ones((1,) + tuple(int(x) for x in reversed(n)))
    return prob, phi


def manufactured_heat(n, k=1.0):
    """All sides Dirichlet, source -div(k grad T*) for T* = prod sin(pi x_a / L_a),
    sampled at cell centres and scaled by the cell volume.  Returns (problem, phi, T*)."""
    ndim = len(n)
    h = 1.0 / n[1]
    shape = tuple(int(x) for x in reversed(n))
    fixed = np.zeros(shape, dtype=np.uint8)
    for a in range(ndim):
        ax = ndim - 1 - a
        lo = [slice(None)] * ndim
        hi = [slice(None)] * ndim
        lo[ax] = 0
        hi[ax] = n[a] - 1
        fixed[tuple(lo)] |= np.uint8(1 << (2 * a))
        fixed[tuple(hi)] |= np.uint8(1 << (2 * a + 1))
    grids = [(np.arange(n[ndim - 1 - r]) + 0.5) * h for r in range(ndim)]
    mesh = list(reversed(np.meshgrid(*grids, indexing="ij")))
    Tex = np.ones(shape)
    wsum = 0.0
    for a in range(ndim):
        L = n[a] * h
        Tex = Tex * np.sin(math.pi * mesh[a] / L)
        wsum += (math.pi / L) ** 2
    f = k * wsum * Tex
    prob = Problem(HEAT, ndim, tuple(n), h, k, 0.0, 0.0, 3.0, (FREE,) * 6, fixed, f * h ** ndim,
                   vol_frac=(0.3,), name="manufactured_heat")
    phi = np.ones((1,) + shape)
    return prob, phi, Tex


def paper_heat2d(n=512, kmin=1e-6, q=0.01):
    """The paper's 2D single-material heat set-up (Section 3.1): an n x n grid,
    T = 0 on the top and left sides, no flux on the right and bottom, a uniform
    source f = 0.01, void conductivity 1e-6, target solid fraction 0.3; h = 1/n
    (the printed grid size)."""
    fixed = np.zeros((n, n), dtype=np.uint8)
    fixed[:, 0] |= 1          # left side (x = 0)
    fixed[n - 1, :] |= 8      # top side (y = L)
    prob = Problem(HEAT, 2, (n, n), 1.0 / n, 1.0, kmin, 0.0, 3.0, (FREE,) * 6, fixed, None, q=q,
                   vol_frac=(0.3,), name=f"paper_heat2d_{n}")
    return prob


def heat_batch(ndesign=64, lo=128, hi=1024, seed=0, kmin=1e-3, q=1.0):
    """Batch of independent 2D heat designs of uneven size.

    Draw order from ``numpy.random.default_rng(seed)``: all nx, then all ny
    (uniform integers in [lo, hi]); then per design the patch count U{1..4} and per
    patch its side U{0..3}, length U{ceil(L/16)..ceil(L/4)} and start offset; finally
    per design a U(0,1) design field.  Each patch marks a run of boundary faces as
    Dirichlet T=0 sinks.  Conductivity k = kmin + phi^3 (1 - kmin), source density q."""
    rng = np.random.default_rng(seed)
    nxs = rng.integers(lo, hi + 1, ndesign)
    nys = rng.integers(lo, hi + 1, ndesign)
    probs, phis, patches = [], [], []
    for d in range(ndesign):
        nx, ny = int(nxs[d]), int(nys[d])
        fixed = np.zeros((ny, nx), dtype=np.uint8)
        plist = []
        for _ in range(int(rng.integers(1, 5))):
            s = int(rng.integers(0, 4))
            L = ny if s in (0, 1) else nx
            ln = int(rng.integers(math.ceil(L / 16), math.ceil(L / 4) + 1))
            st = int(rng.integers(0, L - ln + 1))
            plist.append((s, st, ln))
            if s == 0:
                fixed[st:st + ln, 0] |= 1
            elif s == 1:
                fixed[st:st + ln, nx - 1] |= 2
            elif s == 2:
                fixed[0, st:st + ln] |= 4
            else:
                fixed[ny - 1, st:st + ln] |= 8
        probs.append(Problem(HEAT, 2, (nx, ny), 1.0 / ny, 1.0, kmin, 0.0, 3.0, (FREE,) * 6, fixed,
                             None, q=q, vol_frac=(0.3,), name=f"heat{d}_{nx}x{ny}"))
        patches.append(plist)
    for d in range(ndesign):
        nx, ny = probs[d].n
        phis.append(rng.random((1, ny, nx)))
    return probs, phis, patches


def heat_batch_small(ndesign=6, lo=24, hi=80, seed=3, kmin=1e-3, q=1.0):
    """A small uneven heat batch for parity tests (same recipe, smaller sides)."""
    return heat_batch(ndesign, lo, hi, seed, kmin, q)


# --------------------------------------------------------------------------------------
# Seeded fields
# --------------------------------------------------------------------------------------

def random_u(prob, seed=0, scale=1.0):
    """Random displacement-like canonical array: U(-1,1)*scale on real, non-fixed
    slots, zero on padding and Dirichlet slots."""
    rng = np.random.default_rng(seed)
    if prob.physics == HEAT:
        return rng.uniform(-1, 1, prob.cell_shape()) * scale
    u = rng.uniform(-1, 1, prob.u_shape()) * scale
    u[~dof_valid_mask(prob.ndim, prob.n)] = 0.0
    u[prob.fixed.astype(bool)] = 0.0
    return u


def random_phi(prob, seed=0, lo=0.0, hi=1.0):
    rng = np.random.default_rng(seed)
    phi = rng.uniform(lo, hi, prob.phi_shape())
    if prob.nphase > 1:
        # keep the solid phases inside the simplex: phi_1 + phi_2 <= 1
        s = phi.sum(axis=0)
        over = s > 1.0
        phi[:, over] /= s[over]
    return phi


def initial_phi(prob):
    """Uniform initial design at the target volume fractions."""
    phi = np.empty(prob.phi_shape())
    for m in range(phi.shape[0]):
        phi[m] = prob.vol_frac[m]
    return phi


# --------------------------------------------------------------------------------------
# Named configurations
# --------------------------------------------------------------------------------------

@dataclass
class Config:
    name: str
    make: object
    steps: int
    precision: str
    tol: float = 1e-6
    kwargs: dict = field(default_factory=dict)

    def problem(self):
        return self.make(**self.kwargs)


CONFIGS = {
    "cantilever2d_64x32": Config("cantilever2d_64x32", cantilever2d, 20, "fp64",
                                 kwargs=dict(nx=64, ny=32)),
    "cantilever2d_1024x512": Config("cantilever2d_1024x512", cantilever2d, 100, "fp32",
                                    kwargs=dict(nx=1024, ny=512)),
    "cantilever3d_128x64x64": Config("cantilever3d_128x64x64", cantilever3d, 50, "fp32",
                                     kwargs=dict(nx=128, ny=64, nz=64)),
    "multimaterial3d_256x128x128": Config("multimaterial3d_256x128x128", multimaterial3d, 30,
                                          "fp32", kwargs=dict(nx=256, ny=128, nz=128)),
}
