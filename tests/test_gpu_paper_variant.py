"""The paper's schedule on the GPU against the oracle: hybrid APT + PT relaxation,
the penalty update with one Cahn-Hilliard step, and a short design trajectory."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import design
from oracle import paper_variant as pv
from _gpu import announce, context, dev, host, mixed_elastic, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


def _penalty_kw(p):
    return dict(model="penalty", alpha_h=p.alpha_h, alpha_v=p.alpha_v, alpha_1=p.alpha_1, gamma=p.gamma,
                dt_ch=p.dt_ch or 0.0, mobility=p.mobility)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make,alpha_1", [
    ("cant2d", lambda: W.cantilever2d(150, 37), 0.0),
    ("cant3d", lambda: W.cantilever3d(20, 9, 7), 0.0),
    ("multi3d", lambda: W.multimaterial3d(24, 10, 8), 1e4),
])
def test_penalty_update_parity(name, make, alpha_1, prec):
    """Fractions partly outside [0, 1], a design off its target volume, random
    sensitivities: the GPU update equals the oracle's element by element."""
    require_gpu()
    prob = make()
    announce(f"penalty update {name} {prec}")
    rng = np.random.default_rng(7)
    phi = W.random_phi(prob, 8, -0.05, 0.9)
    g = -rng.random(phi.shape)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    params = pv.PenaltyParams(alpha_1=alpha_1, dt_ch=2e3 * prob.h ** 4, mobility=0.8)
    ctx = context(prob, prec)
    phi_t = dev(phi, dtype)
    info = ctx.phase_update(phi_t, dev(g, dtype), vol_frac=prob.vol_frac, **_penalty_kw(params))
    want, winfo = pv.penalty_update(phi, g, prob, params)
    got = host(phi_t, phi.shape)
    tol = 1e-12 if prec == "fp64" else 3e-7
    assert np.abs(got - want).max() < tol * max(1.0, np.abs(want).max())
    assert np.abs(got - phi).max() > 1e-4          # the update did move the design
    for m in range(phi.shape[0]):
        assert info[0]["shift"][m] == pytest.approx(winfo.shift[m], rel=1e-12 if prec == "fp64" else 1e-6)
        assert info[0]["volume"][m] == pytest.approx(winfo.volume[m], abs=1e-12 if prec == "fp64" else 1e-7)
        assert info[0]["gmax"][m] == pytest.approx(winfo.gmax[m], rel=1e-12 if prec == "fp64" else 1e-6)
    ctx.close()


def test_penalty_update_heat_batch():
    require_gpu()
    probs, phis, _ = W.heat_batch_small()
    announce("penalty update heat batch")
    rng = np.random.default_rng(9)
    gs = [-rng.random(x.shape) for x in phis]
    params = pv.PenaltyParams()
    ctx = context(probs, "fp64")
    phi_t = dev(np.concatenate([x.ravel() for x in phis]), torch.float64)
    g_t = dev(np.concatenate([x.ravel() for x in gs]), torch.float64)
    ctx.phase_update(phi_t, g_t, vol_frac=(0.3,), **_penalty_kw(params))
    got = host(phi_t)
    for d, p in enumerate(probs):
        o0, o1 = ctx.offset(d, 1), ctx.offset(d + 1, 1)
        want, _ = pv.penalty_update(phis[d], gs[d], p, pv.PenaltyParams(vol_frac=(0.3,)))
        assert np.abs(got[o0:o1].reshape(want.shape) - want).max() < 1e-12 * max(1.0, np.abs(want).max()), d
    ctx.close()


@pytest.mark.parametrize("name,make", [("mixed2d", lambda: mixed_elastic(2)),
                                       ("cant3d", lambda: W.cantilever3d(20, 9, 7))])
def test_hybrid_schedule_parity(name, make):
    """n_APT damped-wave sweeps then n_PT plain PT sweeps, FP64, against the oracle."""
    require_gpu()
    prob = make()
    announce(f"hybrid schedule {name}")
    phi = W.random_phi(prob, 6, 0.2, 1.0)
    u0 = W.random_u(prob, 7, scale=1e-2)
    ctx = context(prob, "fp64")
    u = dev(u0, torch.float64)
    v = ctx.new_state()
    st, info = ctx.solve(dev(phi, torch.float64), u, v, theta=1.0, replay_iters=120, check_every=40, n_pt=60)
    assert info[0]["iters"] == 180
    want, iters, rho = pv.hybrid_solve(phi, prob, u0, n_apt=120, n_pt=60, theta=1.0, check_every=40)
    assert iters == 180
    assert rel_l2(host(u, prob.u_shape()), want) < 1e-12
    assert info[0]["rel_res"] == pytest.approx(rho, rel=1e-9)
    ctx.close()


def test_hybrid_schedule_refined_fp32():
    """The FP32 refined mode: damped-wave sweeps to a tolerance, then a fixed PT
    stage; the oracle replays the damped-wave count."""
    require_gpu()
    prob = W.cantilever2d(64, 32)
    announce("hybrid schedule refined fp32")
    phi = W.random_phi(prob, 3, 0.3, 1.0).astype(np.float32).astype(np.float64)
    ctx = context(prob, "fp32")
    u = ctx.new_state(torch.float64)
    v = ctx.new_state()
    st, info = ctx.solve(dev(phi, torch.float32), u, v, theta=4.0, tol=1e-7, refine=True, check_every=100,
                         n_pt=200)
    n_apt = info[0]["iters"] - 200
    assert n_apt > 0 and n_apt % 100 == 0
    want, _, _ = pv.hybrid_solve(phi, prob, None, n_apt=n_apt, n_pt=200, theta=4.0, check_every=100)
    assert rel_l2(host(u, prob.u_shape()), want) < 1e-5
    ctx.close()


@pytest.mark.timeout(600)
def test_paper_schedule_trajectory_fp64():
    """Eight design steps of the paper's loop (20 APT + 20 PT sweeps, penalty update,
    one Cahn-Hilliard step) on the 64 x 32 cantilever, FP64, through petto_step:
    designs and compliance agree with the oracle to 1e-10 at every step."""
    require_gpu()
    prob = W.cantilever2d(64, 32)
    announce("paper schedule trajectory 64x32 fp64")
    ctx = context(prob, "fp64")
    phi_np = W.initial_phi(prob)
    phi = dev(phi_np, torch.float64)
    u = ctx.new_state()
    v = ctx.new_state()
    g = ctx.new_cells()
    comp = torch.zeros(2, dtype=torch.float64, device="cuda")
    params = pv.PenaltyParams()
    u_np = np.zeros(prob.u_shape())
    for step in range(8):
        st, si, pi, _ = ctx.step(phi, u, v, g, vol_frac=prob.vol_frac, compliance=comp,
                                 apt=dict(theta=1.0, replay_iters=20, check_every=20, n_pt=20),
                                 phase=_penalty_kw(params))
        phi_np, u_np, g_np, C, info = pv.paper_step(phi_np, u_np, prob, 20, 20, params)
        assert si[0]["iters"] == 40
        assert rel_l2(host(phi, phi_np.shape), phi_np) < 1e-10, step
        assert comp[0].item() == pytest.approx(C, rel=1e-10), step
    ctx.close()


def test_hybrid_schedule_heat_parity():
    """The paper's 2D heat set-up (small grid): 60 damped-wave + 40 PT sweeps, FP64."""
    require_gpu()
    prob = W.paper_heat2d(40)
    announce("hybrid schedule paper heat 40x40")
    phi = W.random_phi(prob, 2, 0.1, 1.0)
    ctx = context(prob, "fp64")
    u = ctx.new_state()
    v = ctx.new_state()
    st, info = ctx.solve(dev(phi, torch.float64), u, v, theta=1.0, replay_iters=60, check_every=20, n_pt=40)
    want, iters, rho = pv.hybrid_solve(phi, prob, None, n_apt=60, n_pt=40, theta=1.0, check_every=20)
    assert info[0]["iters"] == iters == 100
    assert rel_l2(host(u, prob.cell_shape()), want) < 1e-12
    ctx.close()


@pytest.mark.parametrize("name,make", [("cant2d", lambda: W.cantilever2d(64, 32)),
                                       ("mbb2d", lambda: W.mbb2d(48, 16))])
def test_detached_steps_match_reported_steps(name, make):
    """Fixed-count loops called without records are only enqueued; five loops with
    records, and five with records only on some of them (detached loops before and
    after reported ones), give bit-identical designs, states and compliance."""
    require_gpu()
    prob = make()
    announce(f"detached paper-schedule steps {name}")
    ctx = context(prob, "fp32")
    params = pv.PenaltyParams()
    hd = prob.h ** prob.ndim
    if prob.nphase > 1:
        params = pv.PenaltyParams(alpha_v=0.25 / (prob.ncell * hd * hd))
    out = []
    for pattern in ((True,) * 5, (False, False, True, False, True)):
        phi = dev(W.initial_phi(prob), torch.float32)
        u = ctx.new_state()
        v = ctx.new_state()
        g = ctx.new_cells()
        comp = torch.zeros(2, dtype=torch.float64, device="cuda")
        for info in pattern:
            st, si, pi, _ = ctx.step(phi, u, v, g, vol_frac=prob.vol_frac, compliance=comp,
                                     apt=dict(theta=1.0, replay_iters=20, check_every=20, n_pt=20),
                                     phase=_penalty_kw(params), info=info)
            assert (si is None) == (not info)
            if info:
                assert si[0]["iters"] == 40
        torch.cuda.synchronize()
        out.append((phi.clone(), u.clone(), comp.clone()))
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][2], out[1][2])
    assert torch.isfinite(out[1][0]).all()
    ctx.close()
