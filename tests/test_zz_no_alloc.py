"""The allocation-free sensitivity entry point (petto_adjoint_noalloc) against
petto_adjoint, through the C ABI (GPU).

Calls run back to back on decreasing problem sizes, so every call after the
first finds the fixed scratch array holding a larger launch's partial sums: the
outputs must still equal petto_adjoint's bit for bit, and the oracle's to the
FP64 / FP32 parity bars.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import design
from _gpu import announce, context, dev, host, mixed_elastic, require_gpu

pytestmark = pytest.mark.gpu


def _elastic_case(prob, prec, state_fp64, seed):
    ctx = context(prob, prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    phi = W.random_phi(prob, seed, 0.05, 1.0)
    u = W.random_u(prob, seed + 1)
    if prec == "fp32":
        phi = phi.astype(np.float32).astype(np.float64)
        if not state_fp64:
            u = u.astype(np.float32).astype(np.float64)
    udt = torch.float64 if (prec == "fp64" or state_fp64) else torch.float32
    phi_t, u_t = dev(phi, dt), dev(u, udt)
    g_ref, g_na = ctx.new_cells(), ctx.new_cells()
    c_ref = ctx.adjoint(phi_t, u_t, g_ref, state_fp64=state_fp64)
    c_na = ctx.adjoint(phi_t, u_t, g_na, state_fp64=state_fp64, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(g_ref, g_na)
    assert torch.equal(c_ref, c_na)
    want = design.sensitivity(u, phi, prob)
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert np.abs(host(g_na, phi.shape) - want).max() <= tol * np.abs(want).max()
    c = c_na.cpu().numpy()
    assert c[0] == pytest.approx(float(np.sum(design.load_vector(prob) * u)), rel=1e-12 if udt == torch.float64
                                 else 2e-6)
    assert c[1] == pytest.approx(2.0 * design.strain_energy_total(u, phi, prob), rel=1e-12 if udt == torch.float64
                                 else 2e-6)
    ctx.close()


def test_adjoint_noalloc_matches_adjoint_on_shrinking_calls():
    require_gpu()
    announce("adjoint_noalloc: 3D cantilever 96x48x32 fp64")
    _elastic_case(W.cantilever3d(96, 48, 32), "fp64", False, 21)
    announce("adjoint_noalloc: 2D cantilever 256x128 fp32 (fp64 state)")
    _elastic_case(W.cantilever2d(256, 128), "fp32", True, 23)
    announce("adjoint_noalloc: 2D mixed sides 150x37 fp32")
    _elastic_case(mixed_elastic(2), "fp32", False, 25)


def test_adjoint_noalloc_heat_batch():
    require_gpu()
    probs, phis, _ = W.heat_batch_small()
    announce("adjoint_noalloc: heat batch")
    ctx = context(probs, "fp64")
    rng = np.random.default_rng(7)
    us = [rng.uniform(-1, 1, p.cell_shape()) for p in probs]
    phi_t = dev(np.concatenate([x.ravel() for x in phis]), torch.float64)
    u_t = dev(np.concatenate([x.ravel() for x in us]), torch.float64)
    g_ref, g_na = ctx.new_cells(), ctx.new_cells()
    c_ref = ctx.adjoint(phi_t, u_t, g_ref)
    c_na = ctx.adjoint(phi_t, u_t, g_na, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(g_ref, g_na) and torch.equal(c_ref, c_na)
    got = host(g_na)
    c = c_na.cpu().numpy()
    for d, p in enumerate(probs):
        o0, o1 = ctx.offset(d, 1), ctx.offset(d + 1, 1)
        want = design.sensitivity(us[d], phis[d], p)[0]
        assert np.abs(got[o0:o1].reshape(want.shape) - want).max() <= 1e-12 * np.abs(want).max()
        assert c[2 * d] == pytest.approx(design.compliance(us[d], p), rel=1e-12)
    ctx.close()
