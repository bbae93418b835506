"""Pins of the oracle's design update that fix the sign of each of its terms:
the Allen-Cahn step (Section 2.4, Eqs. (2.14)-(2.15)) on Neumann eigenmodes,
the normalised sensitivity step (Eqs. (3.2)-(3.3)) in closed form, the descent
of the directly solved compliance along a small step, and the material laws at
interior points with a nonzero minimum stiffness."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import assembly, design, elastic, heat

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "material_laws.json")))


def _neumann_mode(shape, modes):
    """Product of cos(pi m (i + 1/2) / n) over the axes: an eigenvector of the
    cell-centred Laplacian with no-flux (mirror) sides."""
    v = np.ones(shape)
    for ax, (n, m) in enumerate(zip(shape, modes)):
        c = np.cos(math.pi * m * (np.arange(n) + 0.5) / n)
        sh = [1] * len(shape)
        sh[ax] = n
        v = v * c.reshape(sh)
    return v


def _neumann_eig(shape, modes, h):
    """lam with Lap v = -lam v for the mode above (h the grid spacing)."""
    return sum((2.0 - 2.0 * math.cos(math.pi * m / n)) / h ** 2 for n, m in zip(shape, modes))


def _w2(base):
    """w''(phi) for w = sin^2(pi phi)/64: (pi^2/32) cos(2 pi phi)."""
    return (math.pi ** 2 / 32.0) * math.cos(2.0 * math.pi * base)


# a low mode (interface term small next to the well) and a mode near the grid
# scale (interface term as large as the well's curvature)
_MODES = [((32, 16), (1, 0)), ((32, 16), (29, 14)), ((8, 6, 10), (1, 2, 3)), ((8, 6, 10), (7, 5, 8))]


@pytest.mark.parametrize("shape,modes", _MODES)
@pytest.mark.parametrize("base", [0.0, 0.5])
def test_allen_cahn_step_on_a_neumann_mode(shape, modes, base):
    """Around a stationary point of the double well (phi = 0: w'' = pi^2/32;
    phi = 1/2: w'' = -pi^2/32), a small Neumann eigenmode eps v (Lap v = -lam v)
    is scaled by 1 - dt (w'' + gamma lam) to first order in eps.  Flipping the
    sign of the well term, of the interface term or of the whole step changes
    that factor by more than the tolerance on every case here."""
    h = 1.0 / shape[1]
    gamma = 3e-5
    dt = design.default_dt_ac(h, len(shape), gamma)
    v = _neumann_mode(shape, modes)
    lam = _neumann_eig(shape, modes, h)
    eps = 1e-7
    out = design.allen_cahn_step(base + eps * v, h, gamma, dt)
    amp = 1.0 - dt * (_w2(base) + gamma * lam)
    # the remainder is O(eps^2) (w''' vanishes at both points)
    tol = 1e-6
    np.testing.assert_allclose((out - base) / eps, amp * v, rtol=0, atol=tol)
    # a flipped sign of either term would move the factor by far more than tol
    assert abs(2 * dt * gamma * lam) > 100 * tol
    assert abs(2 * dt * _w2(base)) > 100 * tol


@pytest.mark.parametrize("grid,modes", [((32, 16), (3, 2)), ((32, 16), (14, 29))])
def test_phase_update_applies_the_allen_cahn_step(grid, modes):
    """phase_update with zero sensitivity and default parameters on phi = 1/2 + eps v
    (mean 1/2 = the volume target, no clamping): the projection shift is of second
    order, so the result is the Allen-Cahn factor of the default step and gamma.
    ``grid`` is (nx, ny); ``modes`` follow the array axes (y, x)."""
    prob = W.cantilever2d(grid[0], grid[1], vol_frac=0.5)
    v = _neumann_mode(prob.cell_shape(), modes)
    eps = 1e-7
    phi = (0.5 + eps * v)[None]
    out, info = design.phase_update(phi, np.zeros_like(phi), prob)
    dt = design.default_dt_ac(prob.h, 2, 3e-5)
    amp = 1.0 - dt * (_w2(0.5) + 3e-5 * _neumann_eig(prob.cell_shape(), modes, prob.h))
    np.testing.assert_allclose((out[0] - 0.5) / eps, amp * v, rtol=0, atol=1e-6)
    assert abs(info.shift[0]) < 1e-12


def test_sensitivity_step_closed_form():
    """Eq. (3.3) without penalties: with the Allen-Cahn step off (dt_ac = 0), a
    zero-mean sensitivity and a design at the target volume whose step stays in
    [0, 1], the update is exactly phi - alpha_h g / max|g| (shift 0).  With a
    nonzero-mean g, the shift returns the mean: phi - alpha_h g/max|g| + mean."""
    prob = W.cantilever2d(16, 8, vol_frac=0.5)
    rng = np.random.default_rng(7)
    g = rng.normal(size=prob.phi_shape())
    g -= g.mean()
    phi = np.full(prob.phi_shape(), 0.5)
    pp = design.PhaseParams(dt_ac=0.0)
    out, info = design.phase_update(phi, g, prob, pp)
    gmax = np.abs(g).max()
    np.testing.assert_allclose(out, phi - 0.1 * g / gmax, rtol=0, atol=2e-15)
    assert info.gmax[0] == gmax
    # nonzero mean: the exact shift is alpha_h mean(g)/max|g|
    g2 = g + 0.3 * gmax
    out2, info2 = design.phase_update(phi, g2, prob, pp)
    gm2 = np.abs(g2).max()
    expect = phi - 0.1 * g2 / gm2 + 0.1 * g2.mean() / gm2
    np.testing.assert_allclose(out2, expect, rtol=0, atol=2e-15)
    assert info2.shift[0] == pytest.approx(0.1 * g2.mean() / gm2, abs=1e-15)
    # scaling g by a positive factor changes nothing (normalisation, Eq. (3.2))
    out3, _ = design.phase_update(phi, 37.0 * g, prob, pp)
    np.testing.assert_allclose(out3, out, rtol=0, atol=2e-15)


def _direct_compliance(phi, prob):
    E = design.material(phi, prob)
    u = assembly.direct_solve(design.stiffness(E, prob), design.load_vector(prob), prob)
    return design.compliance(u, prob), u


@pytest.mark.parametrize("ac", [False, True])
def test_small_design_step_lowers_the_compliance(ac):
    """One design update with a small alpha_h on a 12x6 cantilever: the directly
    solved compliance drops, and by g . dphi to first order (dphi the actual
    change).  Without the Allen-Cahn step the start is a non-uniform design; with
    it the start is the uniform phi = 1/2, where the step only scales the small
    sensitivity move (by 1 - dt(w''(1/2) + gamma lam) > 0 on every mode) instead of
    reshaping the design.  A step taken with the wrong sign raises the compliance."""
    prob = W.cantilever2d(12, 6, vol_frac=0.5)
    rng = np.random.default_rng(3)
    if ac:
        phi = np.full(prob.phi_shape(), 0.5)
    else:
        phi = 0.5 + 0.1 * rng.uniform(-1, 1, prob.phi_shape())
        phi += 0.5 - phi.mean()
    C0, u = _direct_compliance(phi, prob)
    g = design.sensitivity(u, phi, prob)
    pp = design.PhaseParams(alpha_h=1e-4, dt_ac=None if ac else 0.0)
    out, _ = design.phase_update(phi, g, prob, pp)
    dphi = out - phi
    C1, _ = _direct_compliance(out, prob)
    pred = float(np.sum(g * dphi))
    assert C1 < C0
    assert (C1 - C0) == pytest.approx(pred, rel=2e-2)
    if not ac:
        # the pure sensitivity step: first-order change -alpha_h sum(g ghat - mean) < 0
        gh = g / np.abs(g).max()
        assert pred == pytest.approx(-1e-4 * float(np.sum(g * (gh - gh.mean()))), rel=1e-9)


def test_simp_law_interior_point():
    d = GOLD["simp_single"]
    prob = W.cantilever2d(4, 2, e0=d["e0"], emin=d["emin"], p=d["p"])
    phi = np.full(prob.phi_shape(), d["phi"])
    np.testing.assert_array_equal(elastic.modulus(phi, prob), d["E"])
    np.testing.assert_array_equal(elastic.modulus_derivative(phi, prob), d["dE"])


def test_heat_law_interior_point():
    d = GOLD["heat_single"]
    prob = W.Problem(W.HEAT, 2, (4, 2), 0.5, e0=d["k0"], emin=d["kmin"], p=d["p"])
    phi = np.full(prob.phi_shape(), d["phi"])
    np.testing.assert_allclose(heat.conductivity(phi, prob), d["k"], rtol=2e-16)
    np.testing.assert_allclose(heat.conductivity_derivative(phi, prob), d["dk"], rtol=2e-16)


def test_mixture_law_interior_point():
    d = GOLD["mixture_two_phase"]
    prob = W.Problem(W.ELASTIC, 3, (2, 2, 2), 0.5, p=d["p"], nphase=2,
                     e_phase=tuple(d["e_phase"]), vol_frac=(0.2, 0.1))
    phi = np.stack([np.full(prob.cell_shape(), x) for x in d["phi"]])
    np.testing.assert_allclose(elastic.modulus(phi, prob), d["E"], rtol=2e-16)
    dE = elastic.modulus_derivative(phi, prob)
    np.testing.assert_allclose(dE[0], d["dE"][0], rtol=2e-16)
    np.testing.assert_allclose(dE[1], d["dE"][1], rtol=2e-16)
