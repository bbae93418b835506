"""Multi-sweep launches are bit-identical to one sweep per launch, and agree with
the oracle; the autotuner's choice is one of the supported values."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import design
from _gpu import announce, context, dev, host, mixed_elastic, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,ks", [("fp32", (1, 2, 4, 5, 8, 10)), ("fp64", (1, 2, 4, 5))])
@pytest.mark.parametrize("name", ["mixed2d", "cant2d_ragged", "cant2d_wide"])
def test_blocking_bit_identical(name, prec, ks):
    """Windows on the boundary and (ragged, wide) windows strictly inside the grid,
    which take the kernel's ghost-free path."""
    require_gpu()
    prob = {"mixed2d": lambda: mixed_elastic(2), "cant2d_ragged": lambda: W.cantilever2d(203, 61),
            "cant2d_wide": lambda: W.cantilever2d(300, 150)}[name]()
    announce(f"blocking {name} {prec} ks={ks}")
    phi = W.random_phi(prob, 6, 0.2, 1.0)
    u0 = W.random_u(prob, 7, scale=1e-2)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        u0 = u0.astype(np.float32).astype(np.float64)
    ctx = context(prob, prec)
    outs = {}
    for k in ks:
        ctx.set_blocking(k)
        u = dev(u0, dtype)
        v = ctx.new_state()
        st, info = ctx.solve(dev(phi, dtype), u, v, theta=1.0, replay_iters=400, check_every=80)
        assert info[0]["iters"] == 400
        outs[k] = (u.cpu().numpy().copy(), v.cpu().numpy().copy(), info[0]["rel_res"])
    ref = outs[ks[0]]
    for k in ks[1:]:
        assert np.array_equal(outs[k][0], ref[0]), k
        assert np.array_equal(outs[k][1], ref[1]), k
        # the norm is summed per tile, and the tiling differs: equal up to summation order
        assert outs[k][2] == pytest.approx(ref[2], rel=1e-12), k
    res, _ = design.solve(phi, prob, u0=u0, params=design.AptParams(theta=1.0, check_every=80), n_iter=400)
    assert rel_l2(ref[0].reshape(prob.u_shape()), res.u) < (1e-12 if prec == "fp64" else 2e-5)
    ctx.close()


def test_refined_solve_same_for_every_blocking_and_autotune():
    require_gpu()
    prob = W.cantilever2d(128, 64)
    announce("refined solve, blocking and autotune")
    phi = dev(W.random_phi(prob, 3, 0.3, 1.0), torch.float32)
    ctx = context(prob, "fp32")
    outs = []
    for k in (1, 5, 0):
        ctx.set_blocking(k)
        u = ctx.new_state(torch.float64)
        v = ctx.new_state()
        st, info = ctx.solve(phi, u, v, theta=4.0, tol=1e-7, refine=True, check_every=100)
        outs.append((u.cpu().numpy(), info[0]["iters"]))
    assert ctx.blocking() in (1, 2, 5, 10)
    for u, it in outs[1:]:
        assert it == outs[0][1]
        assert np.array_equal(u, outs[0][0])
    ctx.close()


@pytest.mark.parametrize("prec,ks", [("fp32", (1, 2, 4, 5, 8, 10)), ("fp64", (1, 2, 5))])
def test_heat_batch_blocking_bit_identical(prec, ks):
    require_gpu()
    probs, phis, _ = W.heat_batch_small()
    announce(f"heat blocking {prec} ks={ks}")
    dtype = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(2)
    u0 = [rng.uniform(-1, 1, p.cell_shape()) * 1e-3 for p in probs]
    if prec == "fp32":
        u0 = [x.astype(np.float32).astype(np.float64) for x in u0]
        phis = [x.astype(np.float32).astype(np.float64) for x in phis]
    ctx = context(probs, prec)
    phi_t = dev(np.concatenate([x.ravel() for x in phis]), dtype)
    outs = {}
    for k in ks:
        ctx.set_blocking(k)
        u = dev(np.concatenate([x.ravel() for x in u0]), dtype)
        v = ctx.new_state()
        st, info = ctx.solve(phi_t, u, v, theta=1.0, replay_iters=400, check_every=80)
        outs[k] = (u.cpu().numpy().copy(), v.cpu().numpy().copy(), [x["rel_res"] for x in info])
    ref = outs[ks[0]]
    for k in ks[1:]:
        assert np.array_equal(outs[k][0], ref[0]), k
        assert np.array_equal(outs[k][1], ref[1]), k
        assert outs[k][2] == pytest.approx(ref[2], rel=1e-12), k
    got = ref[0]
    for d, p in enumerate(probs):
        o0, o1 = ctx.offset(d, 1), ctx.offset(d + 1, 1)
        res, _ = design.solve(phis[d], p, u0=u0[d], params=design.AptParams(theta=1.0, check_every=80), n_iter=400)
        assert rel_l2(got[o0:o1].reshape(p.cell_shape()), res.u) < (1e-12 if prec == "fp64" else 2e-5), d
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("name", ["cant3d", "multi3d", "duty3d", "thin3d"])
def test_3d_tilings_bit_identical(name, prec):
    """Every candidate tiling of the 3D sweep gives the same state and velocity,
    bit for bit (the norm only up to its summation order)."""
    require_gpu()
    prob = {"cant3d": lambda: W.cantilever3d(70, 40, 24), "multi3d": lambda: W.multimaterial3d(64, 20, 18),
            "duty3d": lambda: mixed_elastic(3, 3), "thin3d": lambda: mixed_elastic(3, 2)}[name]()
    announce(f"3D tilings {name} {prec}")
    phi = W.random_phi(prob, 6, 0.2, 1.0)
    u0 = W.random_u(prob, 7, scale=1e-2)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        u0 = u0.astype(np.float32).astype(np.float64)
    ctx = context(prob, prec)
    outs = {}
    for t in (1, 2, 3):
        ctx.set_tile3d(t)
        u = dev(u0, dtype)
        v = ctx.new_state()
        st, info = ctx.solve(dev(phi, dtype), u, v, theta=1.0, replay_iters=200, check_every=100)
        assert ctx.tile3d() == t
        outs[t] = (u.cpu().numpy().copy(), v.cpu().numpy().copy(), info[0]["rel_res"])
    for t in (2, 3):
        assert np.array_equal(outs[t][0], outs[1][0]), t
        assert np.array_equal(outs[t][1], outs[1][1]), t
        assert outs[t][2] == pytest.approx(outs[1][2], rel=1e-12), t
    ctx.close()


@pytest.mark.parametrize("name,prec", [("cant2d", "fp64"), ("cant2d", "fp32"), ("heat", "fp64"), ("cant3d", "fp32"),
                                       ("cant3d", "fp64")])
def test_autotuned_choice_reported_and_cached(name, prec):
    """The first solve times the launch choices (2D sweeps per launch, 3D tiling)
    and reports the one kept; a second context of the same shape gets the same
    choice from the process cache; the state equals that of an explicit choice."""
    require_gpu()
    if name == "heat":
        probs = W.heat_batch_small()[0]
        prob = probs
        phi = np.concatenate([x.ravel() for x in W.heat_batch_small()[1]])
    else:
        prob = W.cantilever2d(300, 150) if name == "cant2d" else W.cantilever3d(70, 40, 24)
        phi = W.random_phi(prob, 3, 0.2, 1.0).ravel()
    announce(f"autotune {name} {prec}")
    dtype = torch.float64 if prec == "fp64" else torch.float32
    three = name == "cant3d"
    choices, states = [], []
    for rep in range(2):
        ctx = context(prob, prec)
        if not three:
            assert ctx.blocking() == 0          # open until the first solve
        u, v = ctx.new_state(), ctx.new_state()
        ctx.solve(dev(phi, dtype), u, v, theta=1.0, replay_iters=200, check_every=100)
        c = ctx.tile3d() if three else ctx.blocking()
        allowed = (1, 2, 3) if three else ((1, 2, 4, 5) if prec == "fp64" else (1, 2, 4, 5, 10))
        assert c in allowed, c
        choices.append(c)
        states.append(u.cpu().numpy().copy())
        ctx.close()
    assert choices[0] == choices[1]
    assert np.array_equal(states[0], states[1])
    # the same solve with one sweep per launch (2D) or the large tiling (3D)
    ctx = context(prob, prec)
    if three:
        ctx.set_tile3d(1)
    else:
        ctx.set_blocking(1)
    u, v = ctx.new_state(), ctx.new_state()
    ctx.solve(dev(phi, dtype), u, v, theta=1.0, replay_iters=200, check_every=100)
    assert np.array_equal(u.cpu().numpy(), states[0])
    ctx.close()
