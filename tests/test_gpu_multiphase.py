"""Several solid phases (the paper's five-material MBB beam) on the GPU against the
oracle: modulus and residual, sensitivity, both design updates, a short trajectory."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import design, elastic
from oracle import paper_variant as pv
from _gpu import announce, context, dev, host, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


def _mbb():
    return W.mbb2d(40, 12)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_five_phase_residual_parity(prec):
    require_gpu()
    prob = _mbb()
    announce(f"five-phase residual {prec}")
    phi = W.random_phi(prob, 3, -0.02, 0.35)       # some fractions outside [0, 1]
    u = W.random_u(prob, 4)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        u = u.astype(np.float32).astype(np.float64)
    ctx = context(prob, prec)
    r = ctx.new_state()
    ctx.residual(dev(phi, dtype), dev(u, dtype), r)
    torch.cuda.synchronize()
    got = host(r, prob.u_shape())
    E = elastic.modulus(phi, prob)
    want = elastic.residual(u, E, prob, design.load_vector(prob))
    scale = np.abs(elastic.internal_force(np.abs(u), E, prob)).max() + np.abs(want).max()
    assert np.abs(got - want).max() / scale < (1e-13 if prec == "fp64" else 2e-6)
    ctx.close()


def test_five_phase_adjoint_parity():
    require_gpu()
    prob = _mbb()
    announce("five-phase adjoint")
    phi = W.random_phi(prob, 5, 0.02, 0.35)
    u = W.random_u(prob, 6)
    ctx = context(prob, "fp64")
    g = ctx.new_cells()
    comp = ctx.adjoint(dev(phi, torch.float64), dev(u, torch.float64), g)
    torch.cuda.synchronize()
    want = design.sensitivity(u, phi, prob)
    got = host(g, phi.shape)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    assert comp.cpu().numpy()[0] == pytest.approx(design.compliance(u, prob), rel=1e-12)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_five_phase_allen_cahn_update_parity(prec):
    """Each phase bounded by what the already updated phases leave."""
    require_gpu()
    prob = _mbb()
    announce(f"five-phase Allen-Cahn update {prec}")
    rng = np.random.default_rng(7)
    phi = W.random_phi(prob, 8, 0.0, 0.4)
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
    assert np.abs(got - want).max() < (1e-12 if prec == "fp64" else 2e-6)
    for m in range(5):
        assert info[0]["volume"][m] == pytest.approx(0.08, abs=1e-12 if prec == "fp64" else 1e-7)
        assert info[0]["shift"][m] == pytest.approx(winfo.shift[m], abs=1e-12 if prec == "fp64" else 1e-6)
    assert got.min() >= 0.0 and got.sum(axis=0).max() <= 1.0 + 1e-6
    ctx.close()


def test_five_phase_penalty_update_parity():
    """The penalty update with the partition-of-unity term over five stored phases."""
    require_gpu()
    prob = _mbb()
    announce("five-phase penalty update")
    rng = np.random.default_rng(9)
    phi = W.random_phi(prob, 10, -0.02, 0.4)
    g = -rng.random(phi.shape)
    params = pv.PenaltyParams(alpha_1=1e4)
    ctx = context(prob, "fp64")
    phi_t = dev(phi, torch.float64)
    ctx.phase_update(phi_t, dev(g, torch.float64), vol_frac=prob.vol_frac, model="penalty",
                     alpha_h=params.alpha_h, alpha_v=params.alpha_v, alpha_1=params.alpha_1, gamma=params.gamma)
    want, _ = pv.penalty_update(phi, g, prob, params)
    got = host(phi_t, phi.shape)
    assert np.abs(got - want).max() < 1e-12 * max(1.0, np.abs(want).max())
    ctx.close()


@pytest.mark.timeout(600)
def test_mbb_trajectory_fp64():
    """Six design steps of the five-material MBB beam (300 sweeps per solve, the
    Allen-Cahn update), FP64: designs and compliance equal the oracle's to 1e-10."""
    require_gpu()
    prob = W.mbb2d(64, 16)
    announce("mbb five-phase trajectory fp64")
    ctx = context(prob, "fp64")
    phi_np = W.initial_phi(prob)
    phi = dev(phi_np, torch.float64)
    u = ctx.new_state()
    v = ctx.new_state()
    g = ctx.new_cells()
    comp = torch.zeros(2, dtype=torch.float64, device="cuda")
    u_np = None
    params = design.AptParams(theta=1.0, check_every=100)
    for step in range(6):
        st, si, pi, _ = ctx.step(phi, u, v, g, vol_frac=prob.vol_frac, compliance=comp,
                                 apt=dict(theta=1.0, replay_iters=300, check_every=100))
        phi_np, u_np, g_np, rec = design.design_step(phi_np, u_np if u_np is not None else np.zeros(prob.u_shape()),
                                                     prob, params, design.PhaseParams(vol_frac=prob.vol_frac),
                                                     n_iter=300)
        assert si[0]["iters"] == 300
        assert rel_l2(host(phi, phi_np.shape), phi_np) < 1e-10, step
        assert comp[0].item() == pytest.approx(rec.compliance, rel=1e-10), step
    ctx.close()
