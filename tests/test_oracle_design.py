"""Whole design steps of the oracle: invariants along a trajectory.  The paper
prints no trajectory values, so the trajectory itself is parity unpinned; these
tests pin its symmetry and constraints."""
import numpy as np

import workloads as W
from oracle import design


def test_cantilever_mirror_symmetry_and_volume():
    """Clamped left side, load on the mid-height face: the design stays mirror
    symmetric about y = H/2 and keeps its volume."""
    prob = W.cantilever2d(16, 8)
    phi = W.initial_phi(prob)
    u = None
    for step in range(3):
        phi, u, g, rec = design.design_step(phi, np.zeros(prob.u_shape()) if u is None else u, prob,
                                            design.AptParams(theta=16.0, tol=1e-8, check_every=50))
        np.testing.assert_allclose(phi[0], phi[0][::-1, :], atol=1e-10)
        np.testing.assert_allclose(g[0], g[0][::-1, :], rtol=1e-7, atol=1e-12 * np.abs(g).max())
        assert abs(np.mean(phi) - 0.5) < 1e-12
        assert rec.rho <= 1e-8
        assert rec.compliance > 0
        assert abs(rec.compliance - rec.energy2) < 1e-5 * rec.compliance
