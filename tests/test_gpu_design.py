"""Sensitivity, phase update and whole design trajectories (GPU against oracle)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import assembly, design
from _gpu import announce, context, dev, host, rel_l2, require_gpu
from paper_2509_06971_amd import _lib as L

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,make", [("mixed2d", None), ("cant3d", lambda: W.cantilever3d(20, 8, 6)),
                                       ("multi3d", lambda: W.multimaterial3d(24, 10, 8))])
@pytest.mark.parametrize("with_w", [False, True])
def test_adjoint_parity(name, make, with_w):
    require_gpu()
    from _gpu import mixed_elastic
    prob = mixed_elastic(2) if make is None else make()
    announce(f"adjoint {name} w={with_w}")
    phi = W.random_phi(prob, 4, 0.05, 1.0)
    u = W.random_u(prob, 5)
    w = W.random_u(prob, 6) if with_w else None
    ctx = context(prob, "fp64")
    g = ctx.new_cells()
    comp = ctx.adjoint(dev(phi, torch.float64), dev(u, torch.float64), g,
                       w=dev(w, torch.float64) if with_w else None)
    torch.cuda.synchronize()
    want = design.sensitivity(u, phi, prob, w=w)
    got = host(g, phi.shape)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    c = comp.cpu().numpy()
    assert c[0] == pytest.approx(float(np.sum(design.load_vector(prob) * u)), rel=1e-12)
    assert c[1] == pytest.approx(2.0 * design.strain_energy_total(u, phi, prob), rel=1e-12)
    ctx.close()


@pytest.mark.parametrize("name,make,prec", [("cant3d_128x64x64", lambda: W.cantilever3d(128, 64, 64), "fp64"),
                                            ("multi3d_256x128x18", lambda: W.multimaterial3d(256, 128, 18), "fp32")])
def test_adjoint_parity_large_3d(name, make, prec):
    """3D grids on which the sensitivity launch has several times the workgroups
    of any sweep tiling, so every one of its partial-sum slots must fit the
    context's buffers: gradient and both compliance sums against the oracle."""
    require_gpu()
    prob = make()
    announce(f"adjoint large {name} {prec}")
    phi = W.random_phi(prob, 4, 0.05, 1.0)
    u = W.random_u(prob, 5)
    ctx = context(prob, prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
    g = ctx.new_cells()
    comp = ctx.adjoint(dev(phi, dt), dev(u, torch.float64), g, state_fp64=True)
    torch.cuda.synchronize()
    want = design.sensitivity(u, phi, prob)
    got = host(g, phi.shape)
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert np.abs(got - want).max() <= tol * np.abs(want).max()
    c = comp.cpu().numpy()
    assert c[0] == pytest.approx(float(np.sum(design.load_vector(prob) * u)), rel=1e-12)
    assert c[1] == pytest.approx(2.0 * design.strain_energy_total(u, phi, prob), rel=1e-12)
    ctx.close()


def test_heat_adjoint_parity():
    require_gpu()
    probs, phis, _ = W.heat_batch_small()
    announce("heat adjoint")
    ctx = context(probs, "fp64")
    rng = np.random.default_rng(3)
    us = [rng.uniform(-1, 1, p.cell_shape()) for p in probs]
    g = ctx.new_cells()
    comp = ctx.adjoint(dev(np.concatenate([x.ravel() for x in phis]), torch.float64),
                       dev(np.concatenate([x.ravel() for x in us]), torch.float64), g)
    torch.cuda.synchronize()
    got = host(g)
    c = comp.cpu().numpy()
    for d, p in enumerate(probs):
        o0, o1 = ctx.offset(d, 1), ctx.offset(d + 1, 1)
        want = design.sensitivity(us[d], phis[d], p)[0]
        assert np.abs(got[o0:o1].reshape(want.shape) - want).max() <= 1e-12 * np.abs(want).max()
        assert c[2 * d] == pytest.approx(design.compliance(us[d], p), rel=1e-12)
        assert c[2 * d + 1] == pytest.approx(2.0 * design.strain_energy_total(us[d], phis[d], p), rel=1e-12)
    ctx.close()


def test_adjoint_against_finite_differences_on_gpu_solves():
    """dC/dphi from the adjoint kernel against central differences of GPU FP64
    solves (warm-started, relaxed to the FP64 floor), on seeded cells with
    non-negligible sensitivity."""
    require_gpu()
    prob = W.cantilever2d(48, 24)
    announce("adjoint vs finite differences")
    phi = W.random_phi(prob, 9, 0.3, 1.0)
    ctx = context(prob, "fp64")
    u = ctx.new_state()
    v = ctx.new_state()
    kw = dict(theta=16.0, tol=1e-11, check_every=50, max_iter=2000000)
    ctx.solve(dev(phi, torch.float64), u, v, **kw)
    g = ctx.new_cells()
    comp = ctx.adjoint(dev(phi, torch.float64), u, g)
    gh = host(g, phi.shape)
    u0 = u.clone()
    rng = np.random.default_rng(0)
    cand = np.argwhere(np.abs(gh) >= 0.1 * np.abs(gh).max())
    def central(idx, d):
        vals = []
        for sgn in (1, -1):
            pp = phi.copy()
            pp[idx] += sgn * d
            uu = u0.clone()
            ctx.solve(dev(pp, torch.float64), uu, v, **kw)
            c = ctx.adjoint(dev(pp, torch.float64), uu, ctx.new_cells())
            # variational estimate 2 F.u - u.K.u: its error is quadratic in the solve error
            vals.append(2.0 * c[0].item() - c[1].item())
        return (vals[0] - vals[1]) / (2 * d)

    d = 1e-3
    for idx in cand[rng.choice(len(cand), 4, replace=False)]:
        idx = tuple(idx)
        # Richardson: the O(d^2) truncation term of the two central differences cancels
        fd = (4.0 * central(idx, d / 2) - central(idx, d)) / 3.0
        assert fd == pytest.approx(gh[idx], rel=1e-5), idx
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make", [("cant2d", lambda: W.cantilever2d(150, 37)),
                                       ("multi3d", lambda: W.multimaterial3d(24, 10, 8))])
def test_phase_update_parity(name, make, prec):
    require_gpu()
    prob = make()
    announce(f"phase update {name} {prec}")
    rng = np.random.default_rng(1)
    phi = W.random_phi(prob, 2, 0.0, 0.6)
    g = -rng.random(phi.shape)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    ctx = context(prob, prec)
    phi_t = dev(phi, dtype)
    info = ctx.phase_update(phi_t, dev(g, dtype), vol_frac=prob.vol_frac)
    want, winfo = design.phase_update(phi, g, prob, design.PhaseParams(vol_frac=prob.vol_frac))
    got = host(phi_t, phi.shape)
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert np.abs(got - want).max() < tol
    for m in range(phi.shape[0]):
        assert info[0]["shift"][m] == pytest.approx(winfo.shift[m], abs=1e-12 if prec == "fp64" else 1e-6)
        assert info[0]["volume"][m] == pytest.approx(prob.vol_frac[m], abs=1e-12 if prec == "fp64" else 1e-7)
        assert info[0]["gmax"][m] == pytest.approx(winfo.gmax[m], rel=1e-12 if prec == "fp64" else 1e-6)
    assert got.min() >= 0.0 and got.sum(axis=0).max() <= 1.0 + 1e-6
    ctx.close()


@pytest.mark.timeout(900)
def test_cantilever_64x32_design_trajectory_fp64():
    """The small configuration: 20 design steps, FP64, tolerance 1e-6.  The oracle
    replays the GPU's sweep count of every solve; designs, states and compliance
    agree to 1e-10 relative at every step, and the design stays mirror symmetric."""
    require_gpu()
    prob = W.cantilever2d(64, 32)
    announce("trajectory cantilever 64x32 fp64, 20 steps")
    ctx = context(prob, "fp64")
    phi0 = W.initial_phi(prob)
    phi = dev(phi0, torch.float64)
    u = ctx.new_state()
    v = ctx.new_state()
    g = ctx.new_cells()
    hist = []
    for s in range(20):
        st, si, pi, comp = ctx.step(phi, u, v, g, vol_frac=prob.vol_frac,
                                    apt=dict(theta=1.0, tol=1e-6, check_every=100))
        assert st == L.OK
        hist.append((si[0]["iters"], host(phi, phi0.shape), host(u, prob.u_shape()), comp.cpu().numpy().copy()))
    ph, uo, ohist = phi0, None, []
    for s in range(20):
        ph, uo, go, rec = design.design_step(ph, np.zeros(prob.u_shape()) if uo is None else uo, prob,
                                             design.AptParams(theta=1.0, tol=1e-6, check_every=100),
                                             n_iter=hist[s][0])
        # the oracle's own stop rule agrees with the GPU's on this step
        assert rec.rho <= 1e-6
        assert rel_l2(hist[s][1], ph) < 1e-10, s
        assert rel_l2(hist[s][2], uo) < 1e-10, s
        assert hist[s][3][0] == pytest.approx(rec.compliance, rel=1e-10)
        assert np.abs(hist[s][1][0] - hist[s][1][0][::-1, :]).max() < 1e-9
        assert abs(hist[s][1].mean() - 0.5) < 1e-12
    ctx.close()


def test_compliance_autograd_function():
    require_gpu()
    from paper_2509_06971_amd.api import ComplianceFn
    prob = W.cantilever2d(32, 16)
    announce("ComplianceFn")
    phi0 = W.random_phi(prob, 3, 0.3, 1.0)
    ctx = context(prob, "fp64")
    phi = dev(phi0, torch.float64).requires_grad_(True)
    u = ctx.new_state()
    v = ctx.new_state()
    C = ComplianceFn.apply(phi, ctx, u, v, dict(theta=8.0, tol=1e-11, check_every=50))
    (2.0 * C.sum()).backward()
    E = design.material(phi0, prob)
    ud = assembly.direct_solve(design.stiffness(E, prob), design.load_vector(prob), prob)
    assert C.item() == pytest.approx(design.compliance(ud, prob), rel=1e-8)
    want = 2.0 * design.sensitivity(ud, phi0, prob)
    got = host(phi.grad, phi0.shape)
    assert np.abs(got - want).max() < 1e-7 * np.abs(want).max()
    ctx.close()
