"""Relaxation to tolerance, FP32 refinement, failure statuses (GPU against oracle)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import assembly, design
from _gpu import announce, context, dev, host, rel_l2, require_gpu
from paper_2509_06971_amd import _lib as L

pytestmark = pytest.mark.gpu


def test_fp64_solve_matches_oracle_stop_and_state():
    """Cantilever 64x32 (the small configuration) from rest to rho <= 1e-6: the
    GPU stops on the same check as the oracle and the states agree to 1e-10."""
    require_gpu()
    prob = W.cantilever2d(64, 32)
    announce("fp64 solve cantilever 64x32")
    phi = W.random_phi(prob, 1, 0.3, 1.0)
    ctx = context(prob, "fp64")
    u = ctx.new_state()
    v = ctx.new_state()
    st, info = ctx.solve(dev(phi, torch.float64), u, v, theta=1.0, tol=1e-6, check_every=100)
    assert st == L.OK and info[0]["status"] == L.OK
    res, _ = design.solve(phi, prob, params=design.AptParams(theta=1.0, tol=1e-6, check_every=100))
    assert res.converged
    assert info[0]["iters"] == res.iters
    assert rel_l2(host(u, prob.u_shape()), res.u) < 1e-10
    assert info[0]["rel_res"] <= 1e-6
    ctx.close()


@pytest.mark.parametrize("name,make,theta", [("cant2d", lambda: W.cantilever2d(64, 32), 1.0),
                                             ("cant3d", lambda: W.cantilever3d(16, 8, 8), 8.0),
                                             ("multi3d", lambda: W.multimaterial3d(16, 8, 8), 8.0)])
def test_fp32_refined_solve_matches_direct(name, make, theta):
    """FP32 sweeps on corrections of a double state reach rho <= 1e-6; the state
    and the compliance agree with the exact (direct) solution to 1e-4."""
    require_gpu()
    prob = make()
    announce(f"fp32 refine {name}")
    phi = W.random_phi(prob, 2, 0.3, 1.0).astype(np.float32).astype(np.float64)
    ctx = context(prob, "fp32")
    u = ctx.new_state(torch.float64)
    v = ctx.new_state()
    st, info = ctx.solve(dev(phi, torch.float32), u, v, theta=theta, tol=1e-6, refine=True, check_every=100)
    assert st == L.OK, info
    assert info[0]["rel_res"] <= 1e-6 and info[0]["outer"] >= 1
    E = design.material(phi, prob)
    ud = assembly.direct_solve(design.stiffness(E, prob), design.load_vector(prob), prob)
    got = host(u, prob.u_shape())
    assert rel_l2(got, ud) < 1e-4
    C_gpu = float(np.sum(design.load_vector(prob) * got))
    assert abs(C_gpu - design.compliance(ud, prob)) / design.compliance(ud, prob) < 1e-4
    ctx.close()


def test_heat_batch_solve_matches_direct():
    require_gpu()
    probs, phis, _ = W.heat_batch_small()
    announce("heat batch fp64 solve")
    ctx = context(probs, "fp64")
    phi_t = dev(np.concatenate([x.ravel() for x in phis]), torch.float64)
    u = ctx.new_state()
    v = ctx.new_state()
    st, info = ctx.solve(phi_t, u, v, theta=1.0, tol=1e-8, check_every=50)
    assert st == L.OK
    got = host(u)
    for d, p in enumerate(probs):
        o0, o1 = ctx.offset(d, 1), ctx.offset(d + 1, 1)
        k = design.material(phis[d], p)
        Td = assembly.direct_solve(design.stiffness(k, p), design.load_vector(p), p)
        assert rel_l2(got[o0:o1].reshape(p.cell_shape()), Td) < 1e-5, d
        # every design stops on its own check, like a solve of that design alone
        res, _ = design.solve(phis[d], p, params=design.AptParams(theta=1.0, tol=1e-8, check_every=50))
        assert info[d]["iters"] == res.iters, d
        assert rel_l2(got[o0:o1].reshape(p.cell_shape()), res.u) < 1e-10, d
    ctx.close()


def test_heat_batch_adaptive_damping_matches_oracle():
    """Adaptive damping on a batch of heat designs: each design takes its own
    damping from its own state (before its first sweep, then at every check).
    From rest and warm-started on new designs, the FP64 batch solve stops every
    design on the oracle's sweep, with the oracle's damping and state."""
    require_gpu()
    probs, phis, _ = W.heat_batch_small()
    announce("heat batch adaptive damping fp64")
    phis2 = [W.random_phi(p, 100 + d, 0.0, 1.0) for d, p in enumerate(probs)]
    ctx = context(probs, "fp64")
    u = ctx.new_state()
    v = ctx.new_state()
    uo = [np.zeros(p.cell_shape()) for p in probs]
    for batch in (phis, phis2):
        phi_t = dev(np.concatenate([x.ravel() for x in batch]), torch.float64)
        st, info = ctx.solve(phi_t, u, v, theta=0.1, tol=1e-8, check_every=50, adapt=True)
        assert st == L.OK
        got = host(u)
        for d, p in enumerate(probs):
            res, _ = design.solve(batch[d], p, u0=uo[d],
                                  params=design.AptParams(theta=0.1, tol=1e-8, check_every=50, adapt=True))
            assert res.converged
            assert info[d]["iters"] == res.iters, d
            assert info[d]["theta"] == pytest.approx(res.theta, rel=1e-9), d
            o0, o1 = ctx.offset(d, 1), ctx.offset(d + 1, 1)
            assert rel_l2(got[o0:o1].reshape(p.cell_shape()), res.u) < 1e-10, d
            uo[d] = res.u
    ctx.close()


def test_heat_batch_fp32_refined():
    require_gpu()
    probs, phis, _ = W.heat_batch_small()
    announce("heat batch fp32 refine")
    phis = [x.astype(np.float32).astype(np.float64) for x in phis]
    ctx = context(probs, "fp32")
    phi_t = dev(np.concatenate([x.ravel() for x in phis]), torch.float32)
    u = ctx.new_state(torch.float64)
    v = ctx.new_state()
    st, info = ctx.solve(phi_t, u, v, theta=1.0, tol=1e-7, refine=True, check_every=50)
    assert st == L.OK
    got = host(u)
    for d, p in enumerate(probs):
        o0, o1 = ctx.offset(d, 1), ctx.offset(d + 1, 1)
        k = design.material(phis[d], p)
        Td = assembly.direct_solve(design.stiffness(k, p), design.load_vector(p), p)
        assert rel_l2(got[o0:o1].reshape(p.cell_shape()), Td) < 1e-4, d
    ctx.close()


def test_step_above_bound_diverges():
    require_gpu()
    prob = W.cantilever2d(32, 16)
    announce("divergence status")
    ctx = context(prob, "fp64")
    phi = dev(W.initial_phi(prob), torch.float64)
    u = ctx.new_state()
    v = ctx.new_state()
    res_dt = design.solve(W.initial_phi(prob), prob, n_iter=2)[1]
    with pytest.raises(L.PettoError) as e:
        ctx.solve(phi, u, v, theta=1.0, dt=10 * res_dt, tol=1e-6, max_iter=200000, check_every=20)
    assert e.value.status == L.ERR_DIVERGED
    # the oracle diverges on the same step
    res, _ = design.solve(W.initial_phi(prob), prob, params=design.AptParams(dt=10 * res_dt, check_every=20))
    assert res.diverged
    ctx.close()


def test_not_converged_status_and_invalid_params():
    require_gpu()
    prob = W.cantilever2d(32, 16)
    announce("status codes")
    ctx = context(prob, "fp64")
    phi = dev(W.initial_phi(prob), torch.float64)
    u = ctx.new_state()
    v = ctx.new_state()
    st, info = ctx.solve(phi, u, v, tol=1e-12, max_iter=400, check_every=100)
    assert st == L.NOT_CONVERGED and info[0]["iters"] == 400
    for kw in (dict(check_every=3), dict(theta=-1.0), dict(tol=0.0), dict(replay_iters=150),
               dict(refine=True)):
        with pytest.raises(L.PettoError) as e:
            ctx.solve(phi, u, v, **kw)
        assert e.value.status == L.ERR_INVALID, kw
    with pytest.raises(TypeError):
        ctx.solve(phi.float(), u, v)
    ctx.close()


def test_two_runs_bit_identical():
    require_gpu()
    prob = W.cantilever2d(100, 40)
    announce("determinism")
    ctx = context(prob, "fp32")
    phi = dev(W.random_phi(prob, 3, 0.2, 1.0), torch.float32)
    outs = []
    for use_graph in (True, True, False):
        u = ctx.new_state(torch.float64)
        v = ctx.new_state()
        ctx.solve(phi, u, v, tol=1e-6, refine=True, theta=4.0, use_graph=use_graph)
        outs.append(u.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    ctx.close()


@pytest.mark.parametrize("name,make", [("cant2d", lambda: W.cantilever2d(64, 32)),
                                       ("multi3d", lambda: W.multimaterial3d(24, 10, 8))])
def test_adaptive_damping_matches_oracle(name, make):
    """Damping chosen from the starting state and re-chosen at every check from
    the Rayleigh quotient of the state: the FP64 GPU solve stops on the oracle's
    sweep with the oracle's state, from rest and warm-started after a design
    change."""
    require_gpu()
    prob = make()
    announce(f"adaptive damping fp64 {name}")
    ctx = context(prob, "fp64")
    phi0 = W.initial_phi(prob)
    phi1 = W.random_phi(prob, 4, 0.3, 1.0)
    u = ctx.new_state()
    v = ctx.new_state()
    uo = np.zeros(prob.u_shape())
    for phi in (phi0, phi1):
        st, info = ctx.solve(dev(phi, torch.float64), u, v, theta=1.0, tol=1e-6, check_every=100, adapt=True)
        res, _ = design.solve(phi, prob, u0=uo, params=design.AptParams(theta=1.0, tol=1e-6, check_every=100,
                                                                       adapt=True))
        assert res.converged and st == L.OK
        assert info[0]["iters"] == res.iters
        assert info[0]["theta"] == pytest.approx(res.theta, rel=1e-9)
        assert rel_l2(host(u, prob.u_shape()), res.u) < 1e-10
        uo = res.u
    ctx.close()


def test_adaptive_damping_refined_fp32():
    require_gpu()
    prob = W.cantilever2d(128, 64)
    announce("adaptive damping fp32 refined")
    phi = W.random_phi(prob, 5, 0.3, 1.0).astype(np.float32).astype(np.float64)
    ctx = context(prob, "fp32")
    u = ctx.new_state(torch.float64)
    v = ctx.new_state()
    st, info = ctx.solve(dev(phi, torch.float32), u, v, theta=1.0, tol=1e-7, refine=True, adapt=True)
    st1, info1 = ctx.solve(dev(phi, torch.float32), ctx.new_state(torch.float64), v, theta=1.0, tol=1e-7,
                           refine=True)
    assert st == L.OK and info[0]["iters"] < info1[0]["iters"]
    E = design.material(phi, prob)
    ud = assembly.direct_solve(design.stiffness(E, prob), design.load_vector(prob), prob)
    assert rel_l2(host(u, prob.u_shape()), ud) < 1e-4
    ctx.close()


def test_warm_started_adaptive_fp64_3d_design_steps():
    """Two design steps of the multi-material 3D cantilever at 128x64x64 with
    adaptive damping, FP64 plain against the FP32 refined mode: the warm-started
    second solve of either converges, with sweep counts within 20 % of each
    other (the damping of a warm start comes from its own state from the first
    sweep on, in both modes)."""
    require_gpu()
    prob = W.multimaterial3d(128, 64, 64)
    announce("adaptive warm start multimaterial3d_128x64x64")
    counts = {}
    for prec in ("fp32", "fp64"):
        ctx = context(prob, prec)
        phi = dev(W.initial_phi(prob), torch.float32 if prec == "fp32" else torch.float64)
        u = ctx.new_state(torch.float64)
        v = ctx.new_state()
        g = ctx.new_cells()
        apt = dict(theta=1.0, tol=1e-6, adapt=True, refine=prec == "fp32", max_iter=200000)
        counts[prec] = []
        for _ in range(2):
            st, si, _, _ = ctx.step(phi, u, v, g, vol_frac=prob.vol_frac, apt=apt)
            assert st == L.OK and si[0]["status"] == L.OK, (prec, si)
            counts[prec].append(si[0]["iters"])
        ctx.close()
    for a, b in zip(counts["fp32"], counts["fp64"]):
        assert abs(a - b) <= 0.2 * a, counts
