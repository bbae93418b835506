"""Pins of the oracle's staggered-grid elasticity against closed forms, a
manufactured solution, an independent assembly and operator invariants."""
import numpy as np
import pytest

import workloads as W
from oracle import assembly, elastic


@pytest.mark.parametrize("ndim,n", [(2, (10, 6)), (3, (6, 4, 4))])
def test_uniform_bar_closed_form(ndim, n):
    """A bar under uniform traction has the exact linear solution
    u_x = eps_xx x, u_y = eps_yy (y - H/2) (plane strain in 2D, uniaxial stress in 3D)."""
    t, E, nu = 1.3, 2.0, 0.3
    prob, phi = W.uniform_bar(ndim, n, t=t, E=E, nu=nu)
    Ec = elastic.modulus(phi, prob)
    K = assembly.elastic_stiffness(Ec, prob)
    u = assembly.direct_solve(K, prob.load, prob)
    comps = elastic.split(u, ndim, n)
    h = prob.h
    if ndim == 2:
        exx, eyy = t * (1 - nu ** 2) / E, -t * nu * (1 + nu) / E
    else:
        exx, eyy = t / E, -nu * t / E
    x = np.arange(n[0] + 1) * h
    y = np.arange(n[1] + 1) * h - n[1] * h / 2
    if ndim == 2:
        np.testing.assert_allclose(comps[0], np.broadcast_to(exx * x, comps[0].shape), atol=1e-13)
        np.testing.assert_allclose(comps[1], np.broadcast_to(eyy * y[:, None], comps[1].shape), atol=1e-13)
        L, H = n[0] * h, n[1] * h
        C_exact = t * t * L * H * (1 - nu ** 2) / E
    else:
        z = np.arange(n[2] + 1) * h - n[2] * h / 2
        np.testing.assert_allclose(comps[0], np.broadcast_to(exx * x, comps[0].shape), atol=1e-13)
        np.testing.assert_allclose(comps[1], np.broadcast_to(eyy * y[None, :, None], comps[1].shape), atol=1e-13)
        np.testing.assert_allclose(comps[2], np.broadcast_to(eyy * z[:, None, None], comps[2].shape), atol=1e-13)
        L, H, D = n[0] * h, n[1] * h, n[2] * h
        C_exact = t * t * L * H * D / E
    C = float(np.sum(prob.load * u))
    assert C == pytest.approx(C_exact, rel=1e-12)
    # the residual of the exact field vanishes on the matrix-free operator too
    r = elastic.residual(u, Ec, prob)
    assert np.abs(r).max() < 1e-12


@pytest.mark.parametrize("ndim,grids,min_ratio", [(2, [(16, 8), (32, 16), (64, 32)], 3.9),
                                                  (3, [(8, 4, 4), (16, 8, 8)], 3.4)])
def test_manufactured_second_order(ndim, grids, min_ratio):
    """Clamped box with the body force of a smooth field: the discrete solution
    converges to it at second order (catches wrong Lame factors, signs, transposes)."""
    errs = []
    for n in grids:
        prob, phi, ex = W.manufactured_elastic(ndim, n)
        K = assembly.elastic_stiffness(elastic.modulus(phi, prob), prob)
        u = assembly.direct_solve(K, prob.load, prob)
        errs.append(np.abs(u - ex).max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert min(ratios) > min_ratio, ratios
    assert errs[-1] < 0.04


def _mixed_problem(ndim):
    if ndim == 2:
        n = (9, 6)
        side = (W.CLAMPED, W.FREE, W.CLAMPED, W.ROLLER, 0, 0)
    else:
        n = (5, 4, 3)
        side = (W.CLAMPED, W.FREE, W.ROLLER, W.CLAMPED, W.CLAMPED, W.FREE)
    fixed = W._side_normal_fixed(ndim, n, side)
    prob = W.Problem(W.ELASTIC, ndim, n, 1.0 / n[1], 1.0, 1e-3, 0.3, 3.0, side, fixed,
                     np.zeros((ndim,) + tuple(x + 1 for x in reversed(n))))
    return prob


@pytest.mark.parametrize("ndim", [2, 3])
def test_matrix_free_equals_assembled(ndim):
    prob = _mixed_problem(ndim)
    rng = np.random.default_rng(4)
    E = rng.uniform(0.01, 2.0, prob.cell_shape())
    K = assembly.elastic_stiffness(E, prob)
    valid = W.dof_valid_mask(ndim, prob.n)
    for seed in range(3):
        u = W.random_u(prob, seed)
        f1 = elastic.internal_force(u, E, prob)
        f2 = (K @ u.ravel()).reshape(u.shape)
        np.testing.assert_allclose(f1[valid], f2[valid], atol=1e-11 * np.abs(f2).max())


@pytest.mark.parametrize("ndim", [2, 3])
def test_symmetry_and_energy_identity(ndim):
    prob = _mixed_problem(ndim)
    rng = np.random.default_rng(5)
    E = rng.uniform(0.01, 2.0, prob.cell_shape())
    u = W.random_u(prob, 1)
    w = W.random_u(prob, 2)
    Ku = elastic.internal_force(u, E, prob)
    Kw = elastic.internal_force(w, E, prob)
    assert np.sum(w * Ku) == pytest.approx(np.sum(u * Kw), rel=1e-12)
    assert np.sum(u * Ku) == pytest.approx(2.0 * elastic.energy(u, E, prob), rel=1e-12)
    # the per-cell split is nonnegative and sums to the energy
    Wc = elastic.cell_energy(u, E, prob)
    assert Wc.min() >= 0.0


@pytest.mark.parametrize("ndim,n,nzero", [(2, (6, 4), 3), (3, (4, 4, 2), 6)])
def test_rigid_modes_free_body(ndim, n, nzero):
    """All sides free: exactly the rigid-body modes are in the null space."""
    prob, phi = W.uniform_bar(ndim, n)
    prob.side = (W.FREE,) * 6
    prob.fixed[:] = 0
    K = assembly.elastic_stiffness(elastic.modulus(phi, prob), prob).toarray()
    free = assembly.free_mask(prob)
    ev = np.linalg.eigvalsh(K[np.ix_(free, free)])
    assert int(np.sum(np.abs(ev) < 1e-10 * ev.max())) == nzero
    assert ev.min() > -1e-10 * ev.max()


def test_cantilever_is_positive_definite():
    prob = W.cantilever2d(8, 4)
    E = elastic.modulus(W.random_phi(prob, 3, 0.1, 1.0), prob)
    K = assembly.elastic_stiffness(E, prob).toarray()
    free = assembly.free_mask(prob)
    assert np.linalg.eigvalsh(K[np.ix_(free, free)]).min() > 0


def test_clamped_wall_tangential_factor():
    """Closed form of one diagonal entry next to a clamped wall.  A unit u_y on the
    first cell column (face row j) strains the two cells it bounds (eps_yy = +-1/h,
    energy lam/2 + mu each), the interior vertex to its right (gamma = -1/h, full
    edge modulus mu) and the wall vertex (reflected ghost: gamma = 2/h, half the
    cells so modulus mu/2).  Pi = lam + 2 mu + mu/2 + mu, and K_jj = 2 Pi."""
    prob = W.cantilever2d(4, 4)
    E = np.ones(prob.cell_shape())
    lam, mu = elastic.lame(1.0, prob.nu)
    u = np.zeros(prob.u_shape())
    u[1, 2, 0] = 1.0
    f = elastic.internal_force(u, E, prob)
    assert f[1, 2, 0] == pytest.approx(2.0 * (lam + 3.5 * mu), rel=1e-13)
    assert elastic.energy(u, E, prob) == pytest.approx(lam + 3.5 * mu, rel=1e-13)


def test_multiphase_modulus():
    prob = W.multimaterial3d(4, 2, 2)
    phi = W.random_phi(prob, 1)
    E = elastic.modulus(phi, prob)
    void = 1 - phi[0] - phi[1]
    np.testing.assert_allclose(E, 1.0 * phi[0] ** 3 + 0.5 * phi[1] ** 3 + 1e-9 * void ** 3, rtol=1e-14)
    d = elastic.modulus_derivative(phi, prob)
    eps = 1e-6
    for m in range(2):
        pp = phi.copy(); pp[m] += eps
        pm = phi.copy(); pm[m] -= eps
        fd = (elastic.modulus(pp, prob) - elastic.modulus(pm, prob)) / (2 * eps)
        np.testing.assert_allclose(d[m], fd, rtol=1e-7, atol=1e-12)
