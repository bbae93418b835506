"""Pins of the oracle's paper-schedule variant: hybrid APT + PT relaxation, the
penalty update and the explicit Cahn-Hilliard step."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import assembly, design, elastic, heat
from oracle import paper_variant as pv

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def _neumann_mode(shape, modes):
    """Product of cos(pi m (i + 1/2) / n): an eigenvector of the mirror Laplacian
    (cell-centred grid, no-flux sides) with eigenvalue -sum (2 - 2 cos(pi m / n)) / h^2."""
    v = np.ones(shape)
    for ax, (n, m) in enumerate(zip(shape, modes)):
        c = np.cos(math.pi * m * (np.arange(n) + 0.5) / n)
        sh = [1] * len(shape)
        sh[ax] = n
        v = v * c.reshape(sh)
    return v


def _eig(shape, modes, h):
    return sum((2.0 - 2.0 * math.cos(math.pi * m / n)) / h ** 2 for n, m in zip(shape, modes))


def test_default_ch_step_is_the_printed_value():
    h = GOLD["heat2d"]["dx"]
    assert pv.default_dt_ch(h) == pytest.approx(GOLD["heat2d"]["dt_ch_over_dx4"] * h ** 4)
    # 3D on a coarser grid: the printed step is above the stability limit and is capped
    assert pv.default_dt_ch(1 / 128, 3) < 500 * (1 / 128) ** 4


@pytest.mark.parametrize("ndim,h", [(2, 1 / 512), (3, 1 / 128), (3, 1 / 64)])
def test_default_ch_step_is_stable(ndim, h):
    """The highest mirror-Laplacian mode (checkerboard, lam = 4 d / h^2) neither
    grows nor flips sign unboundedly under the default step around a well."""
    dt = pv.default_dt_ch(h, ndim)
    lam = 4 * ndim / h ** 2
    amp = 1 - dt * lam * (math.pi ** 2 / 32 + 3e-5 * lam)
    assert abs(amp) < 1.0
    assert pv.PenaltyParams().alpha_v == GOLD["penalty"]["alpha_v"]
    assert pv.PenaltyParams().alpha_h == GOLD["penalty"]["alpha_h"]


@pytest.mark.parametrize("shape,modes", [((16, 24), (3, 2)), ((6, 8, 10), (1, 2, 3))])
@pytest.mark.parametrize("base", [0.0, 0.5])
def test_ch_step_on_a_neumann_mode(shape, modes, base):
    """Around phi = 0 (w'' = pi^2/32) and phi = 1/2 (w'' = -pi^2/32), a small
    Neumann eigenmode eps v (Lap v = -lam v) moves by
    -dt D lam (w'' + gamma lam) eps v to first order in eps: this fixes the mirror
    stencil, the composition Lap(w' - gamma Lap), every sign and the scalings."""
    h, gamma, D, dt = 0.05, 3e-5, 0.7, 1e-3
    v = _neumann_mode(shape, modes)
    lam = _eig(shape, modes, h)
    eps = 1e-7
    w2 = (math.pi ** 2 / 32.0) * (1.0 if base == 0.0 else -1.0)
    got = pv.cahn_hilliard_step(base + eps * v, h, gamma, D, dt) - base
    want = eps * v * (1.0 - dt * D * lam * (w2 + gamma * lam))
    assert abs(dt * D * lam * (w2 + gamma * lam)) > 0.01        # the step is visible
    # first order in eps; the rest is the rounding of base + eps v
    assert np.max(np.abs(got - want)) < 1e-8 * eps


@pytest.mark.parametrize("shape", [(13, 9), (5, 7, 6)])
def test_ch_step_conserves_mass(shape):
    rng = np.random.default_rng(1)
    p = rng.uniform(0, 1, shape)
    out = pv.cahn_hilliard_step(p, 0.1, 3e-5, 1.0, 500 * 0.1 ** 4)
    assert abs(out.sum() - p.sum()) < 1e-12 * p.size
    assert np.max(np.abs(out - p)) > 1e-6    # it did move


def test_ch_step_keeps_the_wells():
    for c in (0.0, 1.0):
        p = np.full((7, 5), c)
        np.testing.assert_array_equal(pv.cahn_hilliard_step(p, 0.1, 3e-5, 1.0, 1e-3), p)


def _jv(phi_m, vf, h, nd):
    hd = h ** nd
    return (hd * np.sum(phi_m) - vf * phi_m.size * hd) ** 2


def _j1(phi, h, nd):
    return h ** nd * np.sum((np.sum(phi, axis=0) - 1.0) ** 2)


def test_penalty_gradients_against_finite_differences():
    rng = np.random.default_rng(2)
    h, nd = 0.125, 2
    phi = rng.uniform(0, 1, (2, 6, 5))
    vf = 0.3
    d = 1e-3
    gv = pv.volume_penalty_gradient(phi[0], vf, h, nd)
    g1 = pv.partition_penalty_gradient(phi, h, nd)
    for c in [(0, 0), (3, 2), (5, 4)]:
        pp, pm = phi.copy(), phi.copy()
        pp[0][c] += d
        pm[0][c] -= d
        fd_v = (_jv(pp[0], vf, h, nd) - _jv(pm[0], vf, h, nd)) / (2 * d)
        fd_1 = (_j1(pp, h, nd) - _j1(pm, h, nd)) / (2 * d)
        assert gv == pytest.approx(fd_v, rel=1e-9)
        assert g1[c] == pytest.approx(fd_1, rel=1e-9)
    # uniform design: 2 (a - V_f) N h^(2d)
    a = np.full((6, 5), 0.7)
    assert pv.volume_penalty_gradient(a, vf, h, nd) == pytest.approx(2 * (0.7 - vf) * 30 * h ** 4)


def test_penalty_update_fixed_point():
    """No sensitivity, the design uniform at its target volume where w' = 0:
    unchanged."""
    prob = W.cantilever2d(8, 4)
    phi = np.full((1, 4, 8), 0.5)             # mean 0.5 = V_f, w'(1/2) = 0
    g = np.zeros_like(phi)
    out, info = pv.penalty_update(phi, g, prob, pv.PenaltyParams())
    np.testing.assert_array_equal(out, phi)
    assert info.shift == [0.0]


def test_penalty_update_moves_volume_toward_target():
    prob = W.cantilever2d(16, 8)
    phi = np.full((1, 8, 16), 0.8)            # above V_f = 0.5
    g = np.zeros_like(phi)
    out, info = pv.penalty_update(phi, g, prob, pv.PenaltyParams())
    assert info.shift[0] < 0 and np.mean(out) < 0.8


def test_hybrid_relaxation_fixed_point_and_pt_progress():
    """The APT stage reaches the direct solve, and PT sweeps at theta = 0 with the
    PT step keep it (the step is stable); from a partly relaxed state the PT stage
    lowers the error."""
    prob = W.cantilever2d(8, 4)
    phi = np.ones((1, 4, 8))
    E = design.material(phi, prob)
    ud = assembly.direct_solve(design.stiffness(E, prob), design.load_vector(prob), prob)
    err = lambda u: np.linalg.norm(u - ud) / np.linalg.norm(ud)
    u, iters, rho = pv.hybrid_solve(phi, prob, None, n_apt=20000, n_pt=2000)
    assert iters == 22000 and err(u) < 1e-12
    u1, _, _ = pv.hybrid_solve(phi, prob, None, n_apt=600, n_pt=0)
    u2, _, _ = pv.hybrid_solve(phi, prob, None, n_apt=600, n_pt=4000)
    assert err(u2) < 0.5 * err(u1)


def test_material_laws_clamp_the_fractions():
    prob = W.cantilever2d(4, 2)
    phi = np.array([[[-0.2, 0.3, 1.4, 1.0], [0.0, 0.5, 0.9, -1e-3]]])
    np.testing.assert_array_equal(elastic.modulus(phi, prob), elastic.modulus(np.clip(phi, 0, 1), prob))
    d = elastic.modulus_derivative(phi, prob)
    assert d[0, 0, 0] == 0.0 and d[0, 0, 2] == 0.0 and d[0, 1, 3] == 0.0 and d[0, 0, 1] > 0.0
    probs, phis, _ = W.heat_batch(1, 6, 6, seed=1)
    assert heat.conductivity(phi, probs[0]).min() >= probs[0].emin


def _region_problem():
    prob = W.cantilever2d(16, 8)
    reg = np.zeros((8, 16), dtype=np.uint8)
    reg[2:6, 6:10] = W.REGION_VOID
    reg[:, 0] = W.REGION_SOLID
    prob.region = reg
    return prob


def test_void_region_gradient_against_finite_differences():
    prob = _region_problem()
    rng = np.random.default_rng(3)
    phi = rng.uniform(0, 1, (8, 16))
    h, nd = prob.h, 2
    jb = lambda p: (h ** nd * np.sum(p[prob.region == 1])) ** 2
    gb = pv.void_region_gradient(phi, prob.region, h, nd)
    d = 1e-4
    for c in [(3, 7), (0, 3), (5, 9)]:
        pp, pm = phi.copy(), phi.copy()
        pp[c] += d
        pm[c] -= d
        assert gb[c] == pytest.approx((jb(pp) - jb(pm)) / (2 * d), rel=1e-8, abs=1e-20)


def test_regions_in_the_allen_cahn_update():
    """Void-region cells end at 0, passive-solid cells at 1, the volume is exact."""
    prob = _region_problem()
    rng = np.random.default_rng(4)
    phi = rng.uniform(0, 1, (1, 8, 16))
    g = -rng.random(phi.shape)
    out, info = design.phase_update(phi, g, prob)
    assert np.all(out[0][prob.region == 1] == 0.0)
    assert np.all(out[0][prob.region == 2] == 1.0)
    assert np.mean(out[0]) == pytest.approx(prob.vol_frac[0], abs=1e-12)
    assert out.min() >= 0.0 and out.max() <= 1.0


def test_regions_in_the_penalty_update():
    """The void-region term lowers the region's material; passive-solid cells are
    reset to 1."""
    prob = _region_problem()
    phi = np.full((1, 8, 16), 0.5)
    g = np.zeros_like(phi)
    a, _ = pv.penalty_update(phi, g, prob, pv.PenaltyParams(alpha_b=0.0))
    b, _ = pv.penalty_update(phi, g, prob, pv.PenaltyParams(alpha_b=1e5))
    assert np.all(b[0][prob.region == 2] == 1.0)
    inb = prob.region == 1
    assert np.sum(b[0][inb]) < np.sum(a[0][inb])
