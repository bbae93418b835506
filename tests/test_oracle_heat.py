"""Pins of the oracle's cell-centred heat conduction."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly, heat


@pytest.mark.parametrize("n", [(12, 5), (6, 4, 3)])
def test_slab_closed_form(n):
    """Dirichlet x-sides, uniform k and q: T_c = q/(2k) x_c (L - x_c) + q h^2/(8k) exactly."""
    k, q = 2.0, 1.5
    prob, phi = W.heat_slab(n, k=k, q=q)
    K = assembly.heat_stiffness(heat.conductivity(phi, prob), prob)
    T = assembly.direct_solve(K, heat.source(prob), prob)
    h = prob.h
    L = n[0] * h
    xc = (np.arange(n[0]) + 0.5) * h
    Tex = q / (2 * k) * xc * (L - xc) + q * h * h / (8 * k)
    np.testing.assert_allclose(T, np.broadcast_to(Tex, T.shape), atol=1e-13)
    r = heat.residual(T, heat.conductivity(phi, prob), prob)
    assert np.abs(r).max() < 1e-13


def test_manufactured_second_order():
    errs = []
    for n in ((16, 8), (32, 16), (64, 32)):
        prob, phi, Tex = W.manufactured_heat(n)
        K = assembly.heat_stiffness(heat.conductivity(phi, prob), prob)
        T = assembly.direct_solve(K, heat.source(prob), prob)
        errs.append(np.abs(T - Tex).max())
    assert errs[0] / errs[1] > 3.8 and errs[1] / errs[2] > 3.9


@pytest.mark.parametrize("ndim", [2, 3])
def test_matrix_free_equals_assembled_and_energy(ndim):
    probs, phis, _ = W.heat_batch(2, 6, 11, seed=7)
    if ndim == 2:
        prob, phi = probs[0], phis[0]
    else:
        prob, phi = W.heat_slab((5, 4, 3))
        prob.fixed[0, 0, :] |= 4
        prob.fixed[:, -1, 2] |= 8
        prob.fixed[-1, :, :] |= 32
        phi = np.random.default_rng(2).random(phi.shape)
    prob.emin = 1e-3
    k = heat.conductivity(phi, prob)
    K = assembly.heat_stiffness(k, prob)
    rng = np.random.default_rng(1)
    T = rng.uniform(-1, 1, prob.cell_shape())
    S = rng.uniform(-1, 1, prob.cell_shape())
    g = heat.internal_flux(T, k, prob)
    np.testing.assert_allclose(g, (K @ T.ravel()).reshape(T.shape), atol=1e-13)
    assert np.sum(T * g) == pytest.approx(2.0 * heat.energy(T, k, prob), rel=1e-12)
    assert np.sum(S * g) == pytest.approx(np.sum(T * heat.internal_flux(S, k, prob)), rel=1e-12)
