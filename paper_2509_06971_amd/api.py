"""Torch-facing wrapper of the C ABI.  PyTorch supplies device memory and the
stream; every step of the computation runs in the HIP library."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _problem_struct(p, keep):
    s = L.Problem()
    s.physics = int(p.physics)
    s.ndim = int(p.ndim)
    n = list(p.n) + [1] * (3 - len(p.n))
    for a in range(3):
        s.n[a] = int(n[a])
    s.h = float(p.h)
    s.e0, s.emin, s.nu, s.p = float(p.e0), float(p.emin), float(p.nu), float(p.p)
    s.nphase = int(getattr(p, "nphase", 1))
    ep = list(getattr(p, "e_phase", ())) + [0.0] * (L.MAX_PHASES + 1)
    for m in range(L.MAX_PHASES + 1):
        s.e_phase[m] = float(ep[m])
    side = list(getattr(p, "side", (0,) * 6)) + [0] * 6
    for k in range(6):
        s.side[k] = int(side[k])
    if getattr(p, "fixed", None) is not None:
        f = np.ascontiguousarray(p.fixed, dtype=np.uint8)
        keep.append(f)
        s.fixed = f.ctypes.data_as(C.POINTER(C.c_uint8))
    if getattr(p, "load", None) is not None:
        ld = np.ascontiguousarray(p.load, dtype=np.float64)
        keep.append(ld)
        s.load = ld.ctypes.data_as(C.POINTER(C.c_double))
    s.q = float(getattr(p, "q", 0.0))
    if getattr(p, "region", None) is not None:
        rg = np.ascontiguousarray(p.region, dtype=np.uint8)
        keep.append(rg)
        s.region = rg.ctypes.data_as(C.POINTER(C.c_uint8))
    return s


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class Context:
    """A set of design problems resident on the GPU (see petto_create)."""

    def __init__(self, problems, precision: str = "fp64"):
        self.lib = L.load()
        probs = list(problems) if isinstance(problems, (list, tuple)) else [problems]
        self.problems = probs
        self.prec = L.FP64 if precision == "fp64" else L.FP32
        self.dtype = torch.float64 if self.prec == L.FP64 else torch.float32
        arr = (L.Problem * len(probs))()
        keep = []
        for i, p in enumerate(probs):
            arr[i] = _problem_struct(p, keep)
        h = C.c_void_p()
        L.check(self.lib.petto_create(arr, len(probs), self.prec, C.byref(h)))
        self.h = h
        self.nprob = len(probs)
        self.nstate = self.lib.petto_field_offset(h, self.nprob, L.FIELD_STATE)
        self.ncell = self.lib.petto_field_offset(h, self.nprob, L.FIELD_CELL)
        self.nphase = int(getattr(probs[0], "nphase", 1))

    # ------------------------------------------------------------------ helpers
    def offset(self, i, field):
        return self.lib.petto_field_offset(self.h, i, field)

    def _ptr(self, t, dtype, numel, name):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a GPU tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
        return C.c_void_p(t.data_ptr())

    def new_state(self, dtype=None):
        return torch.zeros(self.nstate, dtype=dtype or self.dtype, device="cuda")

    def new_cells(self, dtype=None):
        return torch.zeros(self.nphase * self.ncell, dtype=dtype or self.dtype, device="cuda")

    @staticmethod
    def apt_params(theta=1.0, dt=0.0, tol=1e-6, max_iter=10**8, check_every=100, refine=False,
                   use_graph=True, replay_iters=0, adapt=False, n_pt=0, dt_pt=0.0):
        p = L.AptParams()
        p.theta, p.dt, p.tol = float(theta), float(dt), float(tol)
        p.max_iter, p.check_every = int(max_iter), int(check_every)
        p.refine, p.use_graph = int(bool(refine)), int(bool(use_graph))
        p.replay_iters = int(replay_iters)
        p.adapt = int(bool(adapt))
        p.n_pt, p.dt_pt = int(n_pt), float(dt_pt)
        return p

    @staticmethod
    def phase_params(vol_frac, alpha_h=0.1, gamma=3e-5, dt_ac=0.0, bisect_passes=0, model="allen_cahn",
                     alpha_v=1e5, alpha_1=0.0, dt_ch=0.0, mobility=1.0, alpha_b=0.0):
        """model: "allen_cahn" (Allen-Cahn step + exact volume projection) or
        "penalty" (the paper's penalty update + one Cahn-Hilliard step)."""
        p = L.PhaseParams()
        p.alpha_h, p.gamma, p.dt_ac = float(alpha_h), float(gamma), float(dt_ac)
        vf = list(vol_frac) + [0.0] * L.MAX_PHASES
        for m in range(L.MAX_PHASES):
            p.vol_frac[m] = float(vf[m])
        p.bisect_passes = int(bisect_passes)
        p.model = {"allen_cahn": 0, "penalty": 1}[model]
        p.alpha_v, p.alpha_1, p.dt_ch, p.mobility = float(alpha_v), float(alpha_1), float(dt_ch), float(mobility)
        p.alpha_b = float(alpha_b)
        return p

    # ------------------------------------------------------------------ entry points
    def solve(self, phi, u, v, stream=None, **kw):
        """Relax the state in place (petto_apt_solve).  Returns (status, infos)."""
        p = self.apt_params(**kw)
        udt = torch.float64 if p.refine else self.dtype
        infos = (L.SolveInfo * self.nprob)()
        st = self.lib.petto_apt_solve(self.h, self._ptr(phi, self.dtype, self.nphase * self.ncell, "phi"),
                                      self._ptr(u, udt, self.nstate, "u"),
                                      self._ptr(v, self.dtype, self.nstate, "v"), C.byref(p), _stream(stream),
                                      infos)
        L.check(st)
        return st, [infos[i].as_dict() for i in range(self.nprob)]

    def residual(self, phi, u, r, stream=None):
        L.check(self.lib.petto_residual(self.h, self._ptr(phi, self.dtype, self.nphase * self.ncell, "phi"),
                                        self._ptr(u, self.dtype, self.nstate, "u"),
                                        self._ptr(r, self.dtype, self.nstate, "r"), _stream(stream)))

    def adjoint(self, phi, u, grad, w=None, compliance=None, state_fp64=False, stream=None, noalloc=False):
        """Compliance and sensitivity (petto_adjoint; noalloc: petto_adjoint_noalloc,
        whose partial sums live in the library's fixed device array)."""
        sdt = torch.float64 if (state_fp64 or self.prec == L.FP64) else self.dtype
        comp = compliance if compliance is not None else torch.empty(2 * self.nprob, dtype=torch.float64,
                                                                     device="cuda")
        fn = self.lib.petto_adjoint_noalloc if noalloc else self.lib.petto_adjoint
        L.check(fn(self.h, self._ptr(phi, self.dtype, self.nphase * self.ncell, "phi"),
                                       self._ptr(u, sdt, self.nstate, "u"),
                                       self._ptr(w, sdt, self.nstate, "w") if w is not None else None,
                                       int(bool(state_fp64)),
                                       self._ptr(grad, self.dtype, self.nphase * self.ncell, "grad"),
                                       self._ptr(comp, torch.float64, 2 * self.nprob, "compliance"),
                                       _stream(stream)))
        return comp

    def phase_update(self, phi, grad, vol_frac, stream=None, info=True, **kw):
        p = self.phase_params(vol_frac, **kw)
        infos = (L.PhaseInfo * self.nprob)() if info else None
        L.check(self.lib.petto_phase_update(self.h, self._ptr(phi, self.dtype, self.nphase * self.ncell, "phi"),
                                            self._ptr(grad, self.dtype, self.nphase * self.ncell, "grad"),
                                            C.byref(p), _stream(stream), infos))
        return [infos[i].as_dict() for i in range(self.nprob)] if info else None

    def step(self, phi, u, v, grad, vol_frac, compliance=None, stream=None, apt=None, phase=None, info=True):
        """One design loop.  info=False asks for no solve / update records: with a
        fixed sweep count the loop is then only enqueued (no host wait) and the two
        record lists come back as None."""
        ap = self.apt_params(**(apt or {}))
        pp = self.phase_params(vol_frac, **(phase or {}))
        udt = torch.float64 if ap.refine else self.dtype
        comp = compliance if compliance is not None else torch.empty(2 * self.nprob, dtype=torch.float64,
                                                                     device="cuda")
        si = (L.SolveInfo * self.nprob)() if info else None
        pi = (L.PhaseInfo * self.nprob)() if info else None
        st = self.lib.petto_step(self.h, self._ptr(phi, self.dtype, self.nphase * self.ncell, "phi"),
                                 self._ptr(u, udt, self.nstate, "u"), self._ptr(v, self.dtype, self.nstate, "v"),
                                 self._ptr(grad, self.dtype, self.nphase * self.ncell, "grad"),
                                 self._ptr(comp, torch.float64, 2 * self.nprob, "compliance"),
                                 C.byref(ap), C.byref(pp), _stream(stream), si, pi)
        L.check(st)
        if not info:
            return st, None, None, comp
        return st, [si[i].as_dict() for i in range(self.nprob)], [pi[i].as_dict() for i in range(self.nprob)], comp

    def set_blocking(self, k):
        """Sweeps per launch of the 2D elastic relaxation (0: autotune)."""
        L.check(self.lib.petto_set_blocking(self.h, int(k)))

    def blocking(self):
        return int(self.lib.petto_blocking(self.h))

    def set_tile3d(self, t):
        """Tiling of the 3D elastic sweeps: 1 large columns, 2 small, 3 short, 0 automatic."""
        L.check(self.lib.petto_set_tile3d(self.h, int(t)))

    def tile3d(self):
        return int(self.lib.petto_tile3d(self.h))

    def time_sweeps(self, launches=200, stream=None):
        """Mean milliseconds per launch of the dominant sweep kernel and the sweeps
        per launch, from HIP events around back-to-back launches on `stream`."""
        ms = C.c_double()
        k = C.c_int32()
        L.check(self.lib.petto_time_sweeps(self.h, int(launches), _stream(stream), C.byref(ms), C.byref(k)))
        return ms.value, k.value

    def set_timing(self, on=True):
        L.check(self.lib.petto_set_timing(self.h, int(bool(on))))

    def last_sweep_ms(self):
        n = C.c_int64()
        ms = self.lib.petto_last_sweep_ms(self.h, C.byref(n))
        return ms, n.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.petto_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ComplianceFn(torch.autograd.Function):
    """C(phi) = F . u(phi) with u the relaxed state; the backward pass applies the
    hand-written adjoint sensitivity (compliance is self-adjoint, so no second
    solve).  Returns one compliance per design (float64)."""

    @staticmethod
    def forward(fctx, phi, context, u, v, solve_kw):
        solve_kw = dict(solve_kw or {})
        context.solve(phi, u, v, **solve_kw)
        g = torch.empty_like(phi)
        comp = context.adjoint(phi, u, g, state_fp64=bool(solve_kw.get("refine", False)))
        fctx.save_for_backward(g)
        fctx.context = context
        return comp[0::2].clone()

    @staticmethod
    def backward(fctx, grad_out):
        (g,) = fctx.saved_tensors
        context = fctx.context
        grad = torch.empty_like(g)
        for d in range(context.nprob):
            o0 = context.offset(d, L.FIELD_CELL)
            o1 = context.offset(d + 1, L.FIELD_CELL)
            for m in range(context.nphase):
                sl = slice(m * context.ncell + o0, m * context.ncell + o1)
                grad[sl] = g[sl] * grad_out[d].to(g.dtype)
        return grad, None, None, None, None
