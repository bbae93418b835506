"""Shared helpers of the GPU parity tests (test code only)."""
import sys

import numpy as np
import pytest
import torch

import workloads as W

HAS_GPU = torch.cuda.is_available()


def require_gpu():
    if not HAS_GPU:
        pytest.skip("no GPU")


def announce(msg):
    """Name the case before a GPU step (flushed, so it survives a lost box)."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a).ravel(), dtype=dtype, device="cuda")


def host(t, shape=None):
    a = t.detach().cpu().numpy().astype(np.float64)
    return a.reshape(shape) if shape is not None else a


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def context(prob, prec):
    from paper_2509_06971_amd.api import Context
    return Context([prob] if not isinstance(prob, list) else prob, prec)


def mixed_elastic(ndim, variant=0):
    """Ragged grid with clamped, roller and free sides and a few extra pins.
    3D variant 1 has n_x a multiple of 64 and a clamped x = n_x side (the face
    column that the 3D tiling hands to the last x-tile); variant 2 is thinner than
    one tile in y and z and barely over one tile in x, clamped on every side;
    variant 3 has n_x a multiple of 64 and n_y of 8, and several z-tiles."""
    if ndim == 2:
        n = (150, 37)
        side = (W.CLAMPED, W.ROLLER, W.FREE, W.CLAMPED, 0, 0)
    elif variant == 0:
        n = (70, 9, 19)
        side = (W.CLAMPED, W.FREE, W.ROLLER, W.CLAMPED, W.CLAMPED, W.FREE)
    elif variant == 1:
        n = (64, 7, 11)
        side = (W.FREE, W.CLAMPED, W.CLAMPED, W.ROLLER, W.FREE, W.CLAMPED)
    elif variant == 2:
        n = (66, 3, 2)
        side = (W.CLAMPED,) * 6
    else:
        # n_x a multiple of 64 and n_y of 8: the face column and the face row are
        # the extra duties of the last x- and y-tiles (with the corner); several
        # z-tiles with a short top tile, clamped z sides (ghost layers)
        n = (128, 16, 35)
        side = (W.CLAMPED, W.CLAMPED, W.ROLLER, W.CLAMPED, W.CLAMPED, W.CLAMPED)
    fixed = W._side_normal_fixed(ndim, n, side)
    valid = W.dof_valid_mask(ndim, n)
    rng = np.random.default_rng(11)
    idx = np.argwhere(valid & (fixed == 0))
    for q in idx[rng.choice(len(idx), 5, replace=False)]:
        fixed[tuple(q)] = 1
    load = rng.uniform(-1, 1, fixed.shape)
    load[~valid] = 0
    load[fixed.astype(bool)] = 0
    prob = W.Problem(W.ELASTIC, ndim, n, 1.0 / n[1], 1.0, 1e-3, 0.3, 3.0, side, fixed, load)
    return prob
