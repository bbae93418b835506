"""Parity of the GPU residual and sweep kernels with the oracle, element by element."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import apt, design, elastic, heat
from _gpu import announce, context, dev, host, mixed_elastic, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-13
TOL_FP32 = 2e-6


def _elastic_cases():
    return [("mixed2d", lambda: mixed_elastic(2)), ("mixed3d", lambda: mixed_elastic(3)),
            ("mixed3d64", lambda: mixed_elastic(3, 1)), ("thin3d", lambda: mixed_elastic(3, 2)),
            ("cant2d", lambda: W.cantilever2d(64, 32)), ("cant3d", lambda: W.cantilever3d(20, 8, 6)),
            ("multi3d", lambda: W.multimaterial3d(24, 10, 8)), ("duty3d", lambda: mixed_elastic(3, 3))]


def _tilings(prob):
    """3D contexts: every sweep tiling; 2D: the default."""
    return [1, 2, 3] if prob.ndim == 3 else [None]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make", _elastic_cases())
def test_elastic_residual_parity(name, make, prec):
    require_gpu()
    prob = make()
    announce(f"elastic residual {name} {prec} n={prob.n}")
    phi = W.random_phi(prob, 3, 0.05, 1.0)
    u = W.random_u(prob, 4)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        u = u.astype(np.float32).astype(np.float64)
    ctx = context(prob, prec)
    E = elastic.modulus(phi, prob)
    want = elastic.residual(u, E, prob, design.load_vector(prob))
    scale = np.abs(elastic.internal_force(np.abs(u), E, prob)).max() + np.abs(want).max()
    for t in _tilings(prob):
        if t is not None:
            ctx.set_tile3d(t)
        r = ctx.new_state()
        r.fill_(7.0)    # padding slots must come back as zero
        ctx.residual(dev(phi, dtype), dev(u, dtype), r)
        torch.cuda.synchronize()
        got = host(r, prob.u_shape())
        err = np.abs(got - want).max() / scale
        assert err < (TOL_FP64 if prec == "fp64" else TOL_FP32), (t, err)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_heat_batch_residual_parity(prec):
    require_gpu()
    probs, phis, _ = W.heat_batch_small()
    announce(f"heat batch residual {prec} sizes={[p.n for p in probs]}")
    dtype = torch.float64 if prec == "fp64" else torch.float32
    ctx = context(probs, prec)
    rng = np.random.default_rng(5)
    us = [rng.uniform(-1, 1, p.cell_shape()) for p in probs]
    if prec == "fp32":
        us = [x.astype(np.float32).astype(np.float64) for x in us]
        phis = [x.astype(np.float32).astype(np.float64) for x in phis]
    phi_t = dev(np.concatenate([x.ravel() for x in phis]), dtype)
    u_t = dev(np.concatenate([x.ravel() for x in us]), dtype)
    r = ctx.new_state()
    ctx.residual(phi_t, u_t, r)
    torch.cuda.synchronize()
    got = host(r)
    for d, p in enumerate(probs):
        o0, o1 = ctx.offset(d, 1), ctx.offset(d + 1, 1)
        k = heat.conductivity(phis[d], p)
        want = heat.residual(us[d], k, p)
        scale = np.abs(heat.internal_flux(np.abs(us[d]), k, p)).max() + np.abs(want).max()
        err = np.abs(got[o0:o1].reshape(p.cell_shape()) - want).max() / scale
        assert err < (TOL_FP64 if prec == "fp64" else TOL_FP32), (d, err)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,make", _elastic_cases()[:4] + _elastic_cases()[4:6] + _elastic_cases()[7:])
def test_sweeps_parity(name, make, prec):
    """200 damped-wave sweeps from a random state equal the oracle's sweeps (3D:
    with every sweep tiling)."""
    require_gpu()
    prob = make()
    for t in _tilings(prob):
        _sweeps_case(name, prob, prec, t)


def _sweeps_case(name, prob, prec, tiling):
    announce(f"sweeps {name} {prec} tiling={tiling}")
    phi = W.random_phi(prob, 6, 0.2, 1.0)
    u0 = W.random_u(prob, 7, scale=1e-2)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        u0 = u0.astype(np.float32).astype(np.float64)
    ctx = context(prob, prec)
    if tiling is not None:
        ctx.set_tile3d(tiling)
        assert ctx.tile3d() == tiling
    u = dev(u0, dtype)
    v = ctx.new_state()
    for use_graph in (True, False):
        u.copy_(dev(u0, dtype))
        st, info = ctx.solve(dev(phi, dtype), u, v, theta=1.0, replay_iters=200, check_every=100,
                             use_graph=use_graph)
        assert info[0]["iters"] == 200
        got = host(u, prob.u_shape())
        res, dt = design.solve(phi, prob, u0=u0, params=design.AptParams(theta=1.0, check_every=100), n_iter=200)
        assert info[0]["dt"] == pytest.approx(dt, rel=1e-12 if prec == "fp64" else 1e-6)
        err = rel_l2(got, res.u)
        assert err < (1e-12 if prec == "fp64" else 2e-5), (use_graph, err)
        assert info[0]["rel_res"] == pytest.approx(res.rho, rel=1e-9 if prec == "fp64" else 1e-3)
    ctx.close()


@pytest.mark.parametrize("name,make,sample", [
    ("cantilever2d_1024x512", lambda: W.cantilever2d(1024, 512), None),
    ("cantilever3d_128x64x64", lambda: W.cantilever3d(128, 64, 64), None),
    ("multimaterial3d_256x128x128", lambda: W.multimaterial3d(256, 128, 128), 200000),
])
def test_full_size_residual_parity(name, make, sample):
    """At the configurations' full sizes (the launch shapes the bench times): the
    FP32 residual of a random state against the oracle's FP64 residual of the same
    (FP32-rounded) inputs, on every unknown or a seeded sample of them."""
    require_gpu()
    prob = make()
    announce(f"full-size residual {name}")
    phi = W.random_phi(prob, 8, 0.05, 1.0).astype(np.float32).astype(np.float64)
    u = W.random_u(prob, 9, scale=1e-3).astype(np.float32).astype(np.float64)
    ctx = context(prob, "fp32")
    r = ctx.new_state()
    ctx.residual(dev(phi, torch.float32), dev(u, torch.float32), r)
    torch.cuda.synchronize()
    got = host(r, prob.u_shape())
    ctx.close()
    E = elastic.modulus(phi, prob)
    want = elastic.residual(u, E, prob, design.load_vector(prob))
    scale = np.abs(elastic.internal_force(np.abs(u), E, prob)).max() + np.abs(want).max()
    if sample:
        rng = np.random.default_rng(0)
        flat = rng.choice(got.size, sample, replace=False)
        got, want = got.ravel()[flat], want.ravel()[flat]
    err = np.abs(got - want).max() / scale
    assert err < 2e-6, err


def _fp32(a):
    return np.asarray(a).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("name,make", [
    ("cantilever2d_1024x512", lambda: W.cantilever2d(1024, 512)),
    ("cantilever3d_128x64x64", lambda: W.cantilever3d(128, 64, 64)),
])
def test_full_size_sweeps_parity(name, make):
    """At full size and in the launch configuration the bench times (FP32 graphs,
    autotuned sweeps per launch in 2D, the automatic 3D tiling): 20 sweeps from a
    random state against the oracle's 20 FP64 sweeps, every unknown."""
    require_gpu()
    prob = make()
    announce(f"full-size sweeps {name}")
    phi = _fp32(W.random_phi(prob, 12, 0.05, 1.0))
    u0 = _fp32(W.random_u(prob, 13, scale=1e-3))
    ctx = context(prob, "fp32")
    phi_t = dev(phi, torch.float32)
    u = dev(u0, torch.float32)
    v = ctx.new_state()
    # a first solve runs the autotuner (2D), as in the bench
    ctx.solve(phi_t, ctx.new_state(), ctx.new_state(), theta=1.0, replay_iters=20, check_every=20)
    st, info = ctx.solve(phi_t, u, v, theta=1.0, replay_iters=20, check_every=20)
    assert info[0]["iters"] == 20
    got = host(u, prob.u_shape())
    blocking, tiling = ctx.blocking(), (ctx.tile3d() if prob.ndim == 3 else None)
    ctx.close()
    res, _ = design.solve(phi, prob, u0=u0, params=design.AptParams(theta=1.0, check_every=20), n_iter=20)
    err = rel_l2(got, res.u)
    assert err < 2e-5, (blocking, tiling, err)
    assert info[0]["rel_res"] == pytest.approx(res.rho, rel=1e-3)


def test_full_size_multimaterial3d_sweeps_parity():
    """The multi-material 3D configuration at full size (256x128x128, 12.8 M
    unknowns) in the launch configuration the bench times (FP32, the tiling the
    first solve times and keeps): 4 sweeps from a random state against 4 FP64
    sweeps on the oracle's matrix-free residual, every unknown."""
    require_gpu()
    prob = W.multimaterial3d(256, 128, 128)
    announce("full-size sweeps multimaterial3d_256x128x128")
    phi = _fp32(W.random_phi(prob, 12, 0.05, 1.0))
    u0 = _fp32(W.random_u(prob, 13, scale=1e-3))
    ctx = context(prob, "fp32")
    u = dev(u0, torch.float32)
    v = ctx.new_state()
    st, info = ctx.solve(dev(phi, torch.float32), u, v, theta=1.0, replay_iters=4, check_every=4)
    assert info[0]["iters"] == 4
    got = host(u, prob.u_shape())
    tiling = ctx.tile3d()
    ctx.close()
    E = elastic.modulus(phi, prob)
    F = design.load_vector(prob)
    dt = apt.default_dt(prob.h, prob.ndim, design.wave_modulus_max(E, prob), 1.0)
    assert info[0]["dt"] == pytest.approx(dt, rel=1e-6)
    res = apt.apt_solve(lambda x: elastic.residual(x, E, prob, F), u0, dt=dt, theta=1.0, hd=prob.h ** 3,
                        fnorm=float(np.sqrt(np.sum(F * F))), ncell=prob.ncell, check_every=4, n_iter=4)
    err = rel_l2(got, res.u)
    assert err < 2e-5, (tiling, err)
    assert info[0]["rel_res"] == pytest.approx(res.rho, rel=1e-3)


@pytest.mark.timeout(900)
@pytest.mark.oracle_job("heat_batch64_20")
def test_full_size_heat_batch_sweeps_parity(oracle_jobs):
    """The 64-design heat batch at full size (22.0 M cells), 20 FP32 sweeps in the
    bench's launch configuration, every design compared with the oracle on every
    cell (the oracle's sweeps run in a child process started at session start)."""
    require_gpu()
    from oracle_jobs import heat_batch_start
    probs, phis, u0 = heat_batch_start()
    announce("full-size heat batch sweeps")
    ctx = context(probs, "fp32")
    phi_t = dev(np.concatenate([x.ravel() for x in phis]), torch.float32)
    ctx.solve(phi_t, ctx.new_state(), ctx.new_state(), theta=1.0, replay_iters=20, check_every=20)
    u = dev(np.concatenate([x.ravel() for x in u0]), torch.float32)
    v = ctx.new_state()
    st, info = ctx.solve(phi_t, u, v, theta=1.0, replay_iters=20, check_every=20)
    got = host(u)
    offs = [(ctx.offset(d, 1), ctx.offset(d + 1, 1)) for d in range(len(probs))]
    ctx.close()
    want = oracle_jobs.result("heat_batch64_20")["u"]
    assert got.shape == want.shape
    for d, p in enumerate(probs):
        o0, o1 = offs[d]
        assert rel_l2(got[o0:o1], want[o0:o1]) < 2e-5, d
