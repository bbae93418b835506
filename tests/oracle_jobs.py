"""Long oracle computations run in a child process beside the GPU tests (test
infrastructure only; imports the oracle and the input generators, nothing of the
GPU package).

    python tests/oracle_jobs.py <job> <out.npz>

Each job is a pure function of its name: the oracle's own design trajectory from
the seeded initial design, with its own stop rule (no count or state from the
GPU path), written to <out.npz>.  The GPU tests start the jobs at session start
(tests/conftest.py) so the single-threaded oracle runs while other GPU tests use
the device, and read the file when they need it.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import design  # noqa: E402


def trajectory(prob, steps, adapt):
    """`steps` design steps (Fig. 4 loop: relax to rho <= 1e-6, sensitivity, phase
    update) from the problem's uniform initial design, recording the design,
    state and compliance after every step."""
    phi = W.initial_phi(prob)
    u = np.zeros(prob.u_shape())
    ap = design.AptParams(theta=1.0, tol=1e-6, check_every=100, adapt=adapt)
    out = {"phi": [], "u": [], "compliance": [], "energy2": [], "iters": [], "rho": []}
    t0 = time.time()
    for s in range(steps):
        phi, u, g, rec = design.design_step(phi, u, prob, ap)
        out["phi"].append(phi.copy())
        out["u"].append(u.copy())
        out["compliance"].append(rec.compliance)
        out["energy2"].append(rec.energy2)
        out["iters"].append(rec.iters)
        out["rho"].append(rec.rho)
        print(f"[oracle-job] {prob.name} step {s + 1}/{steps}: {rec.iters} sweeps, rho {rec.rho:.3e}, "
              f"{time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    return {k: np.asarray(v) for k, v in out.items()}


def heat_batch_start():
    """The 64-design heat batch at full size with a seeded starting temperature:
    designs, starting states (both rounded to FP32, the precision the GPU reads)."""
    probs, phis, _ = W.heat_batch()
    rng = np.random.default_rng(14)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    u0 = [f32(rng.uniform(0.0, 1e-2, p.cell_shape())) for p in probs]
    return probs, [f32(x) for x in phis], u0


def heat_batch_sweeps(n):
    """n damped-wave sweeps (theta = 1, default step) of every design of the batch
    from heat_batch_start(), concatenated in batch order."""
    probs, phis, u0 = heat_batch_start()
    out = []
    t0 = time.time()
    for d, p in enumerate(probs):
        res, _ = design.solve(phis[d], p, u0=u0[d], params=design.AptParams(theta=1.0, check_every=n), n_iter=n)
        out.append(res.u.ravel())
        if d % 8 == 7:
            print(f"[oracle-job] heat batch: {d + 1}/64 designs, {time.time() - t0:.1f} s", file=sys.stderr,
                  flush=True)
    return {"u": np.concatenate(out)}


JOBS = {
    # 20 sweeps of all 64 heat designs at full size (22.0 M cells)
    "heat_batch64_20": lambda: heat_batch_sweeps(20),
    # ten adaptive-damping design steps on a grid whose 64 x 32 sweep windows
    # include some strictly inside the grid (the multi-sweep kernel's fast path)
    "cantilever2d_256x128_adapt_10": lambda: trajectory(W.cantilever2d(256, 128), 10, True),
    # the 3D cantilever and the two-phase 3D cantilever at 32 x 16 x 16
    "cantilever3d_32x16x16_adapt_6": lambda: trajectory(W.cantilever3d(32, 16, 16), 6, True),
    "multimaterial3d_32x16x16_adapt_4": lambda: trajectory(W.multimaterial3d(32, 16, 16), 4, True),
}


def main(argv):
    if len(argv) != 3 or argv[1] not in JOBS:
        print(f"usage: {argv[0]} <{'|'.join(JOBS)}> <out.npz>", file=sys.stderr)
        return 2
    res = JOBS[argv[1]]()
    tmp = argv[2] + ".part.npz"
    np.savez(tmp, **res)
    os.replace(tmp, argv[2])
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
