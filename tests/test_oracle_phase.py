"""Pins of the oracle's phase-field design update."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import design

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def _exact_shift(x, ub, target):
    """Root of the piecewise-linear V(s) = sum clip(x + s, 0, ub) by sorting its breakpoints."""
    x = x.ravel(); ub = np.broadcast_to(ub, x.shape).ravel()
    bps = np.unique(np.concatenate([-x, ub - x]))
    V = np.array([np.sum(np.clip(x + s, 0, ub)) for s in bps])
    k = np.searchsorted(V, target)
    if k == 0:
        return bps[0]
    s0, s1, v0, v1 = bps[k - 1], bps[k], V[k - 1], V[k]
    return s0 + (target - v0) * (s1 - s0) / (v1 - v0)


def test_double_well_printed_form():
    w = lambda p: np.sin(np.pi * p) ** 2 / 64.0
    assert w(0.5) == pytest.approx(GOLD["double_well"]["w_at_half"])
    for m in GOLD["double_well"]["minima"]:
        assert abs(design.double_well_derivative(np.array(m))) < 1e-15
        assert w(m + 1e-3) > w(m) and w(m - 1e-3) > w(m)
    p = np.linspace(0, 1, 11)
    fd = (w(p + 1e-6) - w(p - 1e-6)) / 2e-6
    np.testing.assert_allclose(design.double_well_derivative(p), fd, atol=1e-9)


def test_bisection_matches_sorted_root():
    rng = np.random.default_rng(0)
    for trial in range(5):
        x = rng.normal(0.4, 0.5, 300)
        ub = 1.0 if trial % 2 == 0 else rng.uniform(0.3, 1.0, 300)
        target = 0.35 * 300 * (1.0 if np.isscalar(ub) else np.mean(ub))
        s = design.bisect_shift(x, ub, target)
        assert s == pytest.approx(_exact_shift(x, ub, target), abs=1e-12)
        assert np.sum(np.clip(x + s, 0, ub)) == pytest.approx(target, abs=1e-10)


def test_mirror_laplacian_sums_to_zero():
    rng = np.random.default_rng(1)
    for shape in ((7, 9), (4, 5, 6)):
        phi = rng.random(shape)
        assert abs(np.sum(design.laplacian_mirror(phi, 0.1))) < 1e-9
        # uniform fields are harmonic, a linear ramp has zero interior Laplacian
        assert np.abs(design.laplacian_mirror(np.full(shape, 0.3), 0.1)).max() == 0.0


@pytest.mark.parametrize("value", [0.0, 0.5, 1.0])
def test_fixed_points(value):
    """With zero sensitivity a uniform design at a double-well extremum stays put."""
    prob = W.cantilever2d(8, 4, vol_frac=0.5)
    phi = np.full(prob.phi_shape(), value)
    out, info = design.phase_update(phi, np.zeros_like(phi), prob,
                                    design.PhaseParams(vol_frac=(value,)))
    np.testing.assert_allclose(out, phi, atol=1e-15)


def test_volume_and_bounds_single_phase():
    prob = W.cantilever2d(16, 8, vol_frac=0.4)
    rng = np.random.default_rng(2)
    phi = rng.random(prob.phi_shape())
    g = -rng.random(prob.phi_shape())
    out, info = design.phase_update(phi, g, prob)
    assert np.mean(out) == pytest.approx(0.4, abs=1e-12)
    assert out.min() >= 0.0 and out.max() <= 1.0
    assert info.gmax[0] == pytest.approx(np.abs(g).max())


def test_volume_and_simplex_two_phases():
    prob = W.multimaterial3d(6, 4, 4)
    rng = np.random.default_rng(3)
    phi = W.random_phi(prob, 4)
    g = -rng.random(phi.shape)
    out, info = design.phase_update(phi, g, prob)
    assert np.mean(out[0]) == pytest.approx(0.2, abs=1e-12)
    assert np.mean(out[1]) == pytest.approx(0.1, abs=1e-12)
    assert out.min() >= 0.0 and (out[0] + out[1]).max() <= 1.0 + 1e-15


def test_volume_and_simplex_five_phases():
    """Five solid phases, each bounded by what the earlier ones leave: every
    volume exact, fractions in [0, 1], their sum at most 1."""
    prob = W.mbb2d(16, 8)
    rng = np.random.default_rng(5)
    phi = W.random_phi(prob, 6, 0.0, 0.4)
    g = -rng.random(phi.shape)
    out, info = design.phase_update(phi, g, prob)
    for m in range(5):
        assert np.mean(out[m]) == pytest.approx(0.08, abs=1e-12)
    assert out.min() >= 0.0 and out.sum(axis=0).max() <= 1.0 + 1e-12


def test_default_allen_cahn_step_is_stable():
    """dt (4 d gamma / h^2 + max w'') stays below 2 for the default step."""
    for h, nd in ((1 / 32, 2), (1 / 512, 2), (1 / 64, 3), (1 / 128, 3)):
        dt = design.default_dt_ac(h, nd, 3e-5)
        assert dt * (4 * nd * 3e-5 / h ** 2 + math.pi ** 2 / 32) < 2.0
