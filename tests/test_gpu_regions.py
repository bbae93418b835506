"""Void and passive-solid regions (the drone example's battery bay) on the GPU against
the oracle: both design updates and short trajectories through petto_step."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import design
from oracle import paper_variant as pv
from _gpu import announce, context, dev, host, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


def _cantilever_with_regions():
    prob = W.cantilever2d(96, 40)
    reg = np.zeros((40, 96), dtype=np.uint8)
    reg[10:30, 40:60] = W.REGION_VOID
    reg[:, :3] = W.REGION_SOLID
    prob.region = reg
    return prob


def _block3d_with_regions():
    prob = W.multimaterial3d(24, 10, 12)
    reg = np.zeros((12, 10, 24), dtype=np.uint8)
    reg[4:8, 3:7, 8:16] = W.REGION_VOID
    reg[:2, :, :] = W.REGION_SOLID
    prob.region = reg
    return prob


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make", [("cant2d", _cantilever_with_regions), ("block3d", _block3d_with_regions)])
def test_allen_cahn_update_with_regions(name, make, prec):
    require_gpu()
    prob = make()
    announce(f"Allen-Cahn update with regions {name} {prec}")
    rng = np.random.default_rng(3)
    phi = W.random_phi(prob, 4, 0.0, 0.5)
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
    assert np.all(got[:, prob.region == W.REGION_VOID] == 0.0)
    assert np.all(got[0][prob.region == W.REGION_SOLID] == 1.0)
    for m in range(phi.shape[0]):
        assert info[0]["volume"][m] == pytest.approx(prob.vol_frac[m], abs=1e-12 if prec == "fp64" else 1e-7)
    ctx.close()


def test_penalty_update_with_void_region():
    require_gpu()
    prob = _cantilever_with_regions()
    announce("penalty update with void region")
    rng = np.random.default_rng(5)
    phi = W.random_phi(prob, 6, 0.0, 0.8)
    g = -rng.random(phi.shape)
    params = pv.PenaltyParams(alpha_b=3e4)
    ctx = context(prob, "fp64")
    phi_t = dev(phi, torch.float64)
    ctx.phase_update(phi_t, dev(g, torch.float64), vol_frac=prob.vol_frac, model="penalty",
                     alpha_h=params.alpha_h, alpha_v=params.alpha_v, alpha_b=params.alpha_b, gamma=params.gamma)
    want, _ = pv.penalty_update(phi, g, prob, params)
    got = host(phi_t, phi.shape)
    assert np.abs(got - want).max() < 1e-12 * max(1.0, np.abs(want).max())
    assert np.all(got[0][prob.region == W.REGION_SOLID] == 1.0)
    ctx.close()


@pytest.mark.timeout(600)
def test_drone_standin_paper_schedule_trajectory_fp64():
    """Four loops of the paper's schedule on a small drone stand-in (void region,
    rollers at the top corners), FP64, through petto_step."""
    require_gpu()
    prob = W.drone3d(24, 12, 24)
    announce("drone stand-in paper schedule fp64")
    hd = prob.h ** 3
    nb = int(np.sum(prob.region == W.REGION_VOID))
    params = pv.PenaltyParams(alpha_v=0.25 / (prob.ncell * hd * hd), alpha_b=0.25 / (nb * hd * hd))
    ctx = context(prob, "fp64")
    phi_np = W.initial_phi(prob)
    phi = dev(phi_np, torch.float64)
    u = ctx.new_state()
    v = ctx.new_state()
    g = ctx.new_cells()
    comp = torch.zeros(2, dtype=torch.float64, device="cuda")
    u_np = np.zeros(prob.u_shape())
    for step in range(4):
        ctx.step(phi, u, v, g, vol_frac=prob.vol_frac, compliance=comp,
                 apt=dict(theta=1.0, replay_iters=50, check_every=50, n_pt=50),
                 phase=dict(model="penalty", alpha_h=params.alpha_h, alpha_v=params.alpha_v,
                            alpha_b=params.alpha_b, gamma=params.gamma))
        phi_np, u_np, g_np, C, info = pv.paper_step(phi_np, u_np, prob, 50, 50, params)
        assert rel_l2(host(phi, phi_np.shape), phi_np) < 1e-10, step
        assert comp[0].item() == pytest.approx(C, rel=1e-10), step
    inb = prob.region == W.REGION_VOID
    assert np.mean(phi_np[0][inb]) < np.mean(phi_np[0][~inb])   # the bay empties
    ctx.close()
