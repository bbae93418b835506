"""Fixed-length runs of the relaxation kernels for profiling (rocprofv3).

    python -m paper_2509_06971_amd.profile_run --workload cantilever2d_1024x512 --sweeps 2000

runs exactly `sweeps` FP32 sweeps of the named workload (random design, state
from rest, refinement off so only the sweep kernel runs), then a device copy of
a known size (256 MiB read + 256 MiB written) that calibrates HBM byte counters.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def make(name):
    import workloads as W
    if name.startswith("cantilever2d_"):
        nx, ny = (int(x) for x in name.split("_")[1].split("x"))
        return [W.cantilever2d(nx, ny)]
    if name.startswith("cantilever3d_"):
        nx, ny, nz = (int(x) for x in name.split("_")[1].split("x"))
        return [W.cantilever3d(nx, ny, nz)]
    if name.startswith("multimaterial3d_"):
        nx, ny, nz = (int(x) for x in name.split("_")[1].split("x"))
        return [W.multimaterial3d(nx, ny, nz)]
    if name == "heat_batch64":
        return W.heat_batch()[0]
    raise ValueError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cantilever2d_1024x512")
    ap.add_argument("--sweeps", type=int, default=2000)
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--blocking", type=int, default=0, help="sweeps per launch (0: autotune)")
    ap.add_argument("--tile3d", type=int, default=0, help="3D sweep tiling (0: autotune)")
    ap.add_argument("--copy-mib", type=int, default=256)
    a = ap.parse_args()
    import numpy as np
    import torch

    import workloads as W
    from paper_2509_06971_amd.api import Context

    probs = make(a.workload)
    ctx = Context(probs, "fp32")
    ctx.set_blocking(a.blocking)
    if probs[0].ndim == 3 and probs[0].physics == W.ELASTIC:
        ctx.set_tile3d(a.tile3d)
    if len(probs) == 1:
        phi = W.random_phi(probs[0], 1, 0.05, 1.0).ravel()
    else:
        phi = np.concatenate([W.random_phi(p, d, 0.0, 1.0).ravel() for d, p in enumerate(probs)])
    phi_t = torch.tensor(phi, dtype=torch.float32, device="cuda")
    u = ctx.new_state()
    v = ctx.new_state()
    st, info = ctx.solve(phi_t, u, v, theta=1.0, replay_iters=a.sweeps, check_every=a.check_every)
    torch.cuda.synchronize()
    n = a.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"workload={a.workload} sweeps={info[0]['iters']} blocking={ctx.blocking()} "
          f"copy_bytes_each_way={n * 4}", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
