"""Pins of the oracle's compliance sensitivity (Section 2.3) against exact
identities and finite differences of direct solves."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly, design


def _direct(phi, prob):
    E = design.material(phi, prob)
    u = assembly.direct_solve(design.stiffness(E, prob), design.load_vector(prob), prob)
    return u, design.compliance(u, prob)


def _problems():
    p2 = W.cantilever2d(10, 6)
    p3 = W.cantilever3d(5, 4, 4)
    pm = W.multimaterial3d(6, 4, 4)
    probs, phis, _ = W.heat_batch(1, 9, 13, seed=11)
    p5 = W.mbb2d(12, 4)
    return [(p2, W.random_phi(p2, 1, 0.05, 1.0)), (p3, W.random_phi(p3, 2, 0.05, 1.0)),
            (pm, W.random_phi(pm, 3, 0.05, 0.5)), (probs[0], phis[0]), (p5, W.random_phi(p5, 4, 0.02, 0.3))]


@pytest.mark.parametrize("case", range(5))
def test_euler_homogeneity(case):
    """C is homogeneous of degree -1 in the moduli, so sum_c E_c dC/dE_c = -C."""
    prob, phi = _problems()[case]
    u, C = _direct(phi, prob)
    g = design.sensitivity(u, phi, prob)
    E = design.material(phi, prob)
    dE = design.material_derivative(phi, prob)
    # chain rule: dC/dE_c = g_m,c / dE_m,c for any stored phase m
    s = np.sum(E * g[0] / dE[0])
    assert s == pytest.approx(-C, rel=1e-10)
    assert C > 0
    assert C == pytest.approx(design.strain_energy_total(u, phi, prob) * 2.0, rel=1e-10)


def test_uniform_bar_sensitivity():
    """Uniform strain: every cell holds C/(2N) energy, so g_c = -(E'/E) C / N."""
    prob, phi = W.uniform_bar(2, (8, 4), t=1.0, E=1.5)
    u, C = _direct(phi, prob)
    g = design.sensitivity(u, phi, prob)
    np.testing.assert_allclose(g[0], -prob.p * C / prob.ncell, rtol=1e-12)


@pytest.mark.parametrize("case", range(5))
def test_finite_differences(case):
    prob, phi = _problems()[case]
    u, C = _direct(phi, prob)
    g = design.sensitivity(u, phi, prob)
    gmax = np.abs(g).max()
    rng = np.random.default_rng(case)
    d = 1e-5
    for _ in range(4):
        idx = tuple(int(rng.integers(0, s)) for s in phi.shape)
        pp = phi.copy(); pp[idx] += d
        pm = phi.copy(); pm[idx] -= d
        fd = (_direct(pp, prob)[1] - _direct(pm, prob)[1]) / (2 * d)
        assert abs(fd - g[idx]) <= 1e-7 * gmax + 1e-6 * abs(g[idx])


def test_general_adjoint_bilinear_form():
    """For L = a . u(phi) the adjoint state w solves K w = a and
    dL/dphi_c = -E'_c B_c(w, u) / E_c; checked by finite differences."""
    prob = W.cantilever2d(8, 4)
    phi = W.random_phi(prob, 5, 0.2, 1.0)
    a = W.random_u(prob, 9)
    free = assembly.free_mask(prob).reshape(a.shape)
    a[~free] = 0.0

    def L(ph):
        E = design.material(ph, prob)
        return float(np.sum(a * assembly.direct_solve(design.stiffness(E, prob), design.load_vector(prob), prob)))

    E = design.material(phi, prob)
    K = design.stiffness(E, prob)
    u = assembly.direct_solve(K, design.load_vector(prob), prob)
    w = assembly.direct_solve(K, a, prob)
    g = design.sensitivity(u, phi, prob, w=w)
    # w = u reproduces the compliance form
    np.testing.assert_allclose(design.sensitivity(u, phi, prob, w=u), design.sensitivity(u, phi, prob), rtol=1e-12)
    d = 1e-5
    for idx in [(0, 1, 2), (0, 3, 7), (0, 0, 0)]:
        pp = phi.copy(); pp[idx] += d
        pm = phi.copy(); pm[idx] -= d
        fd = (L(pp) - L(pm)) / (2 * d)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-8 * np.abs(g).max())
