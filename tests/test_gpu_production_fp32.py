"""The FP32 production design loop against the oracle (GPU).

The production mode relaxes the state with FP32 sweeps on corrections of an FP64
state (refine), replays captured graphs of check blocks and runs the autotuned
number of sweeps per launch; the sensitivity then reads the FP64 state.  The
tolerance on designs, states and compliance is 1e-4 relative (the FP32 target of
the configurations); the observed agreement is printed.

A batch of heat designs runs the same production loop (one context, every
design stopping on its own check).

Also here: direct parity of the 2D sensitivity kernel when its state or its
arithmetic is FP32, and the finite-difference check of the sensitivity on 8
seeded cells of the 1024 x 512 cantilever, at the initial design and after 20
production design steps (Section 2.3, Eq. 2.7 and Fig. 2's gradient).
"""
import time

import numpy as np
import pytest
import torch

import workloads as W
from oracle import design
from _gpu import announce, context, dev, host, rel_l2, require_gpu
from paper_2509_06971_amd import _lib as L

pytestmark = pytest.mark.gpu

TOL32 = 1e-4


def _say(capsys, msg):
    """A progress line that reaches the terminal while the test runs."""
    with capsys.disabled():
        print(f"\n[fp32-production] {msg}", flush=True)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


# ------------------------------------------------------------------ sensitivity kernel in FP32 contexts

@pytest.mark.parametrize("state_fp64", [True, False])
@pytest.mark.parametrize("name", ["mixed2d", "cant2d_256x128"])
def test_adjoint_parity_2d_fp32_context(name, state_fp64):
    """The 2D sensitivity kernel of an FP32 context, reading an FP64 state (the
    refined production loop) or an FP32 state: gradient and both compliance sums
    against the oracle evaluated on the same (rounded) inputs."""
    require_gpu()
    from _gpu import mixed_elastic
    prob = mixed_elastic(2) if name == "mixed2d" else W.cantilever2d(256, 128)
    announce(f"adjoint fp32 context {name} state_fp64={state_fp64}")
    phi = _f32(W.random_phi(prob, 4, 0.05, 1.0))
    u = W.random_u(prob, 5)
    if not state_fp64:
        u = _f32(u)
    ctx = context(prob, "fp32")
    g = ctx.new_cells()
    comp = ctx.adjoint(dev(phi, torch.float32), dev(u, torch.float64 if state_fp64 else torch.float32), g,
                       state_fp64=state_fp64)
    torch.cuda.synchronize()
    want = design.sensitivity(u, phi, prob)
    got = host(g, phi.shape)
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 2e-6, err
    c = comp.cpu().numpy()
    # the compliance sums accumulate in FP64 on both sides; with an FP32 state the
    # per-cell energies are FP32 products
    rel = 1e-12 if state_fp64 else 2e-6
    assert c[0] == pytest.approx(float(np.sum(design.load_vector(prob) * u)), rel=rel)
    assert c[1] == pytest.approx(2.0 * design.strain_energy_total(u, phi, prob), rel=rel)
    ctx.close()


# ------------------------------------------------------------------ FP32 design trajectories

def _gpu_trajectory(prob, steps, apt, capsys, label):
    """`steps` production design steps (FP32 refined, graphs, autotuned sweeps per
    launch) from the uniform initial design; records after every step."""
    ctx = context(prob, "fp32")
    phi0 = W.initial_phi(prob)
    phi = dev(phi0, torch.float32)
    u = ctx.new_state(torch.float64)
    v = ctx.new_state()
    g = ctx.new_cells()
    comp = torch.zeros(2, dtype=torch.float64, device="cuda")
    hist = []
    t0 = time.time()
    for s in range(steps):
        st, si, pi, _ = ctx.step(phi, u, v, g, vol_frac=prob.vol_frac, compliance=comp,
                                 apt=dict(apt, refine=True, use_graph=True))
        assert st == L.OK, (s, si)
        hist.append(dict(iters=si[0]["iters"], rho=si[0]["rel_res"], phi=host(phi, phi0.shape),
                         u=host(u, prob.u_shape()), C=comp[0].item(), E2=comp[1].item(),
                         volume=pi[0]["volume"][:phi0.shape[0]]))
    blocking = ctx.blocking()
    ctx.close()
    _say(capsys, f"{label}: GPU {steps} steps in {time.time() - t0:.1f} s, sweeps per launch {blocking}, "
                 f"sweeps {[h['iters'] for h in hist]}")
    return hist, blocking


def _compare(hist, ref, prob, label, capsys):
    """Designs, states and compliance of every step within TOL32 (relative)."""
    worst = dict(phi=0.0, dphi=0.0, u=0.0, C=0.0)
    for s, (h, r) in enumerate(zip(hist, ref)):
        e_phi = rel_l2(h["phi"], r["phi"])
        d_phi = float(np.abs(h["phi"] - r["phi"]).max())
        e_u = rel_l2(h["u"], r["u"])
        e_c = abs(h["C"] - r["C"]) / abs(r["C"])
        for k, x in (("phi", e_phi), ("dphi", d_phi), ("u", e_u), ("C", e_c)):
            worst[k] = max(worst[k], x)
        assert e_phi < TOL32 and e_u < TOL32 and e_c < TOL32, (s, e_phi, e_u, e_c)
        # the volume constraints hold exactly in the stored FP32 design
        for m, vol in enumerate(h["volume"]):
            assert abs(vol - prob.vol_frac[m]) < 1e-6
    _say(capsys, f"{label}: worst over steps rel-L2(phi) {worst['phi']:.2e}, max|dphi| {worst['dphi']:.2e}, "
                 f"rel-L2(u) {worst['u']:.2e}, |dC|/C {worst['C']:.2e}")


@pytest.mark.timeout(600)
def test_cantilever_64x32_trajectory_fp32_production(capsys):
    """The small configuration's 20 design steps in the production FP32 mode; the
    oracle replays the GPU's sweep count of every solve from the same start."""
    require_gpu()
    prob = W.cantilever2d(64, 32)
    announce("trajectory cantilever 64x32 fp32 refined, 20 steps")
    apt = dict(theta=1.0, tol=1e-6, check_every=100)
    hist, _ = _gpu_trajectory(prob, 20, apt, capsys, "64x32")
    ph, uo, ref = W.initial_phi(prob), np.zeros(prob.u_shape()), []
    for h in hist:
        ph, uo, go, rec = design.design_step(ph, uo, prob, design.AptParams(theta=1.0, tol=1e-6, check_every=100),
                                             n_iter=h["iters"])
        # the oracle's own stop rule agrees that the replayed count converged
        assert rec.rho <= 1e-6
        ref.append(dict(phi=ph, u=uo, C=rec.compliance))
    _compare(hist, ref, prob, "64x32", capsys)


@pytest.mark.timeout(600)
def test_heat_batch_trajectory_fp32_production(capsys):
    """Six heat designs of uneven size in one context (their own Dirichlet patches,
    24-80 cells a side): 8 production design steps (FP32 refined sweeps, graphs,
    autotuned sweeps per launch, every design stopping on its own check) against
    the oracle run design by design, replaying each design's sweep counts."""
    require_gpu()
    probs, _, _ = W.heat_batch_small()
    steps = 8
    announce(f"trajectory heat batch ({len(probs)} designs) fp32 refined, {steps} steps")
    ctx = context(probs, "fp32")
    phi0 = [W.initial_phi(p) for p in probs]
    phi = dev(np.concatenate([x.ravel() for x in phi0]), torch.float32)
    u = ctx.new_state(torch.float64)
    v = ctx.new_state()
    g = ctx.new_cells()
    comp = torch.zeros(2 * len(probs), dtype=torch.float64, device="cuda")
    apt = dict(theta=1.0, tol=1e-6, check_every=100, refine=True, use_graph=True)
    hist = []
    t0 = time.time()
    for s in range(steps):
        st, si, pi, _ = ctx.step(phi, u, v, g, vol_frac=probs[0].vol_frac, compliance=comp, apt=apt)
        assert st == L.OK, (s, si)
        ph, uh, c = host(phi), host(u), comp.cpu().numpy()
        rec = []
        for d, p in enumerate(probs):
            c0, c1 = ctx.offset(d, L.FIELD_CELL), ctx.offset(d + 1, L.FIELD_CELL)
            s0, s1 = ctx.offset(d, L.FIELD_STATE), ctx.offset(d + 1, L.FIELD_STATE)
            rec.append(dict(iters=si[d]["iters"], rho=si[d]["rel_res"], phi=ph[c0:c1].reshape(p.phi_shape()),
                            u=uh[s0:s1].reshape(p.cell_shape()), C=float(c[2 * d]), volume=pi[d]["volume"][0]))
        hist.append(rec)
    ctx.close()
    _say(capsys, f"heat batch: GPU {steps} steps in {time.time() - t0:.1f} s, sweeps per design and step "
                 f"{[[h[d]['iters'] for h in hist] for d in range(len(probs))]}")
    worst = dict(phi=0.0, u=0.0, C=0.0)
    for d, p in enumerate(probs):
        ph, uo = phi0[d], np.zeros(p.cell_shape())
        for s in range(steps):
            h = hist[s][d]
            ph, uo, _, r = design.design_step(ph, uo, p, design.AptParams(theta=1.0, tol=1e-6, check_every=100),
                                              n_iter=h["iters"])
            # the GPU's FP64 check of its refined state met the tolerance, and the
            # FP64 oracle after the same sweep count sits at it too: the FP32 sweeps
            # reach a state 1e-4 close to the FP64 iteration's, whose residual at the
            # stop can lie a little either side (one design ends 0.5 % above)
            assert h["rho"] <= 1e-6, (d, s, h["rho"])
            assert r.rho <= 1.02e-6, (d, s, r.rho)
            e_phi, e_u = rel_l2(h["phi"], ph), rel_l2(h["u"], uo)
            e_c = abs(h["C"] - r.compliance) / abs(r.compliance)
            assert e_phi < TOL32 and e_u < TOL32 and e_c < TOL32, (d, s, e_phi, e_u, e_c)
            assert abs(h["volume"] - p.vol_frac[0]) < 1e-6, (d, s, h["volume"])
            worst = dict(phi=max(worst["phi"], e_phi), u=max(worst["u"], e_u), C=max(worst["C"], e_c))
    _say(capsys, f"heat batch: worst over designs and steps rel-L2(phi) {worst['phi']:.2e}, "
                 f"rel-L2(T) {worst['u']:.2e}, |dC|/C {worst['C']:.2e}")


@pytest.mark.timeout(1500)
@pytest.mark.oracle_job("cantilever2d_256x128_adapt_10")
def test_cantilever_256x128_trajectory_fp32_production(capsys, oracle_jobs):
    """Ten production design steps with adaptive damping on a 256 x 128 grid (some
    64 x 32 sweep windows lie strictly inside it and take the kernel's fast path),
    against the oracle's own trajectory: the oracle runs its own stop rule in a
    child process started at session start, with nothing from the GPU path."""
    require_gpu()
    prob = W.cantilever2d(256, 128)
    announce("trajectory cantilever 256x128 fp32 refined adaptive, 10 steps")
    apt = dict(theta=1.0, tol=1e-6, check_every=100, adapt=True)
    hist, blocking = _gpu_trajectory(prob, 10, apt, capsys, "256x128")
    assert blocking > 1
    ref = oracle_jobs.result("cantilever2d_256x128_adapt_10", progress=lambda m: _say(capsys, m))
    refs = [dict(phi=ref["phi"][s], u=ref["u"][s], C=float(ref["compliance"][s])) for s in range(10)]
    _say(capsys, f"256x128: oracle sweeps {ref['iters'].tolist()}")
    for h, n in zip(hist, ref["iters"]):
        # the two stop rules see residuals that differ by rounding (and the adaptive
        # damping follows each side's own state), so the stops may fall a few
        # checks apart; the sweep counts stay within a few percent
        assert abs(h["iters"] - int(n)) <= 0.03 * int(n), (h["iters"], int(n))
    _compare(hist, refs, prob, "256x128", capsys)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("job,make,steps", [
    pytest.param("cantilever3d_32x16x16_adapt_6", lambda: W.cantilever3d(32, 16, 16), 6,
                 marks=pytest.mark.oracle_job("cantilever3d_32x16x16_adapt_6")),
    pytest.param("multimaterial3d_32x16x16_adapt_4", lambda: W.multimaterial3d(32, 16, 16), 4,
                 marks=pytest.mark.oracle_job("multimaterial3d_32x16x16_adapt_4"))])
def test_3d_trajectory_fp32_production(job, make, steps, capsys, oracle_jobs):
    """The 3D production loop (FP32 refined 3D sweeps with graphs and the timed
    tiling, FP64 state, the 3D sensitivity and, for two phases, the bounded
    second projection) against the oracle's own trajectory with its own stop
    rule, computed in a child process."""
    require_gpu()
    prob = make()
    announce(f"trajectory {job} fp32 refined adaptive")
    oracle_jobs.start(job)
    apt = dict(theta=1.0, tol=1e-6, check_every=100, adapt=True)
    hist, _ = _gpu_trajectory(prob, steps, apt, capsys, job)
    ref = oracle_jobs.result(job, progress=lambda m: _say(capsys, m))
    refs = [dict(phi=ref["phi"][s], u=ref["u"][s], C=float(ref["compliance"][s])) for s in range(steps)]
    _say(capsys, f"{job}: oracle sweeps {ref['iters'].tolist()}")
    for h, n in zip(hist, ref["iters"]):
        assert abs(h["iters"] - int(n)) <= 0.05 * int(n) + 200, (h["iters"], int(n))
    _compare(hist, refs, prob, job, capsys)


# ------------------------------------------------------------------ finite differences at 1024 x 512

def _solve64(ctx, phi_t, u, v, tol, cap):
    st, info = ctx.solve(phi_t, u, v, tol=tol, max_iter=cap, check_every=100, adapt=True)
    assert st in (L.OK, L.NOT_CONVERGED)
    return info[0]


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("steps", [0, 20])
def test_cantilever_1024x512_sensitivity_finite_differences(steps, capsys):
    """dC/dphi of the hand-written adjoint against central differences of the
    solved compliance on 8 seeded cells with |g| >= 0.1 max|g| (and fractions at
    least 2 delta inside [0, 1]), at the initial
    design and after 20 production (FP32 refined) design steps.  Every solve is
    FP64, warm-started from the converged state, and runs until rho <= 1e-13 or
    until it stalls at the FP64 floor; the compliance is taken in its variational
    form 2 F.u - u.K.u (error quadratic in the solve error); delta = 1e-3 and
    delta/2 are Richardson-combined; tolerance 1e-5 relative."""
    require_gpu()
    prob = W.cantilever2d(1024, 512)
    announce(f"finite differences cantilever 1024x512 after {steps} steps")
    phi0 = W.initial_phi(prob)
    if steps:
        ctx32 = context(prob, "fp32")
        p32 = dev(phi0, torch.float32)
        u32 = ctx32.new_state(torch.float64)
        v32 = ctx32.new_state()
        g32 = ctx32.new_cells()
        t0 = time.time()
        for s in range(steps):
            st, si, _, _ = ctx32.step(p32, u32, v32, g32, vol_frac=prob.vol_frac,
                                      apt=dict(theta=1.0, tol=1e-6, check_every=100, refine=True, adapt=True))
            assert st == L.OK
        phi = host(p32, phi0.shape)
        ctx32.close()
        _say(capsys, f"1024x512: {steps} FP32 design steps in {time.time() - t0:.1f} s")
    else:
        phi = phi0
    ctx = context(prob, "fp64")
    ctx.set_blocking(5)
    phi_t = dev(phi, torch.float64)
    u = ctx.new_state()
    v = ctx.new_state()
    t0 = time.time()
    # base state: to 1e-13 or the FP64 floor (the cap is far beyond the sweeps
    # this grid needs to reach the floor from rest)
    info = _solve64(ctx, phi_t, u, v, 1e-13, 800_000)
    rho_floor = info["rel_res"]
    g = ctx.new_cells()
    ctx.adjoint(phi_t, u, g)
    gh = host(g, phi.shape)
    _say(capsys, f"1024x512 base solve: {info['iters']} sweeps, rho {rho_floor:.3e}, {time.time() - t0:.1f} s")
    assert rho_floor < 1e-9
    # perturbed solves stop once they reach the base solve's level (1e-13 if it got there)
    tol = max(1e-13, 1.5 * rho_floor)
    u0 = u.clone()
    rng = np.random.default_rng(8 + steps)
    d = 1e-3
    # cells whose perturbed fractions stay inside [0, 1]: the material law takes
    # fractions clamped to [0, 1], so at a bound the central difference would see
    # a one-sided change (half the derivative)
    inside = (phi >= 2 * d) & (phi <= 1.0 - 2 * d)
    cand = np.argwhere((np.abs(gh) >= 0.1 * np.abs(gh).max()) & inside)
    assert len(cand) >= 8
    cells = [tuple(c) for c in cand[rng.choice(len(cand), 8, replace=False)]]

    def cvar(pp):
        uu = u0.clone()
        pt = dev(pp, torch.float64)
        inf = _solve64(ctx, pt, uu, v, tol, 400_000)
        c = ctx.adjoint(pt, uu, ctx.new_cells()).cpu().numpy()
        return 2.0 * c[0] - c[1], inf

    def central(idx, d):
        vals = []
        for sgn in (1.0, -1.0):
            pp = phi.copy()
            pp[idx] += sgn * d
            cv, inf = cvar(pp)
            vals.append(cv)
        return (vals[0] - vals[1]) / (2.0 * d), inf

    worst = 0.0
    for n, idx in enumerate(cells):
        f1, i1 = central(idx, d)
        f2, i2 = central(idx, d / 2)
        fd = (4.0 * f2 - f1) / 3.0
        err = abs(fd - gh[idx]) / abs(gh[idx])
        worst = max(worst, err)
        _say(capsys, f"cell {idx}: g {gh[idx]:.9e} fd {fd:.9e} rel {err:.2e} "
                     f"(last solve {i2['iters']} sweeps, rho {i2['rel_res']:.2e}), {time.time() - t0:.0f} s")
        assert err < 1e-5, (idx, gh[idx], fd)
    _say(capsys, f"1024x512 after {steps} steps: worst relative FD difference {worst:.2e}")
    ctx.close()
