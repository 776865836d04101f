"""Python binding of the gfx950 RBF-FD library (argument marshalling only).

Every function takes/returns torch tensors on a ROCm device and forwards
device pointers and the current HIP stream to the C ABI; all arithmetic
runs in the HIP kernels of librbffd.so.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import OP_ID, OP_DX, OP_DY, OP_LAP, check, lib

__all__ = ["build_nodes", "knn", "assemble_weights", "ell_apply", "ell_autotune", "ELL_SHAPES", "cast_f32", "Solver", "LidRollout",
           "OP_ID", "OP_DX", "OP_DY", "OP_LAP"]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a ROCm device")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def build_nodes(kind, K, jitter=0.3, seed=0):
    """Host node sets from rbf_build_nodes: dict of numpy arrays."""
    nv = ctypes.c_int64()
    npn = ctypes.c_int64()
    check(lib.rbf_build_nodes(kind, K, jitter, seed, ctypes.byref(nv), None, None,
                              ctypes.byref(npn), None, None, None))
    N, M = nv.value, npn.value
    xv = np.empty((2, N), np.float64)
    vt = np.empty(N, np.int8)
    xp = np.empty((2, M), np.float64)
    pt = np.empty(M, np.int8)
    pn = np.empty((2, M), np.float64)
    c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    check(lib.rbf_build_nodes(kind, K, jitter, seed, ctypes.byref(nv), c(xv), c(vt),
                              ctypes.byref(npn), c(xp), c(pt), c(pn)))
    return {"xv": xv, "v_tag": vt, "xp": xp, "p_tag": pt, "p_normal": pn}


def knn(xq, xs, k):
    """int32 [k, nq] stencil indices (slot-major) of the k nearest xs-nodes."""
    _dev(xq, torch.float64, name="xq")
    _dev(xs, torch.float64, name="xs")
    if xq.dim() != 2 or xq.shape[0] != 2 or xs.dim() != 2 or xs.shape[0] != 2:
        raise ValueError("coordinates must have shape [2, n]")
    nq, ns = xq.shape[1], xs.shape[1]
    idx = torch.empty((k, nq), dtype=torch.int32, device=xq.device)
    check(lib.rbf_knn(_ptr(xq), nq, _ptr(xs), ns, k, _ptr(idx), _stream()))
    return idx


def assemble_weights(xq, xs, idx, m=7, q=3, op_mask=OP_DX | OP_DY | OP_LAP, force=False,
                     cond=False):
    """FP64 weights [nops, k, nq] for the operators in op_mask (bit order);
    with cond=True also the FP64 [nq] 1-norm condition estimates of the local
    systems, returned as (w, cond_est)."""
    _dev(xq, torch.float64, name="xq")
    _dev(xs, torch.float64, name="xs")
    _dev(idx, torch.int32, name="idx")
    k, nq = idx.shape
    if xq.shape != (2, nq) or xs.dim() != 2 or xs.shape[0] != 2:
        raise ValueError("shape mismatch between xq, xs and idx")
    nops = bin(op_mask & 15).count("1")
    w = torch.empty((max(nops, 1), k, nq), dtype=torch.float64, device=xq.device)
    bad = ctypes.c_int64(-1)
    mask = op_mask | (_lib.FORCE_SMALL_STENCIL if force else 0)
    c = torch.empty(nq, dtype=torch.float64, device=xq.device) if cond else None
    check(lib.rbf_assemble_weights(_ptr(xq), nq, _ptr(xs), xs.shape[1], _ptr(idx), k, m, q,
                                   ctypes.c_uint32(mask), _ptr(w), _ptr(c) if cond else None,
                                   ctypes.byref(bad), _stream()))
    return (w, c) if cond else w


ELL_SHAPES = [(b, xcd, nt) for nt in (True, False) for xcd in (True, False)
              for b in (256, 64, 128, 512)]  # (block, XCD remap, non-temporal), shape order


def ell_autotune(idx, w, x, reps=20):
    """Time the launch shapes of ell_apply for this operator size and record
    the fastest for later ell_apply calls (rbf_ell_autotune); returns
    (shape, [ms per application of each shape])."""
    _dev(idx, torch.int32, name="idx")
    k, rows = idx.shape
    if w.dtype not in (torch.float64, torch.float32):
        raise ValueError("w must be float64 or float32")
    _dev(w, w.dtype, (k, rows), name="w")
    _dev(x, w.dtype, name="x")
    y = torch.empty(rows, dtype=w.dtype, device=w.device)
    shape = ctypes.c_int32(-1)
    ms = (ctypes.c_float * 16)()
    check(lib.rbf_ell_autotune(rows, k, _ptr(idx), _ptr(w), _ptr(x), _ptr(y),
                               0 if w.dtype == torch.float64 else 1, int(reps),
                               ctypes.byref(shape), ms, _stream()))
    return shape.value, list(ms)


def ell_apply(idx, w, x, out=None):
    """y = D x for ELL (idx [k, rows], w [k, rows]); FP64 or FP32 (w, x, y alike)."""
    _dev(idx, torch.int32, name="idx")
    k, rows = idx.shape
    if w.dtype not in (torch.float64, torch.float32):
        raise ValueError("w must be float64 or float32")
    _dev(w, w.dtype, (k, rows), name="w")
    _dev(x, w.dtype, name="x")
    if out is None:
        out = torch.empty(rows, dtype=w.dtype, device=w.device)
    _dev(out, w.dtype, (rows,), name="out")
    dtype = 0 if w.dtype == torch.float64 else 1
    check(lib.rbf_ell_apply(rows, k, _ptr(idx), _ptr(w), _ptr(x), _ptr(out), dtype, _stream()))
    return out


class Transpose:
    """Column structure of D^T for one ELL index array (rbf_ell_transpose):
    colptr int64 [ncols + 1], src and slot int32 [k * rows]."""

    def __init__(self, idx, ncols):
        _dev(idx, torch.int32, name="idx")
        self.k, self.rows = idx.shape
        self.ncols = int(ncols)
        dev = idx.device
        self.colptr = torch.empty(self.ncols + 1, dtype=torch.int64, device=dev)
        nnz = max(1, self.k * self.rows)
        self.src = torch.empty(nnz, dtype=torch.int32, device=dev)
        self.slot = torch.empty(nnz, dtype=torch.int32, device=dev)
        bad = ctypes.c_int64(-1)
        rc = lib.rbf_ell_transpose(self.rows, self.k, _ptr(idx), self.ncols, _ptr(self.colptr),
                                   _ptr(self.src), _ptr(self.slot), ctypes.byref(bad), _stream())
        self.bad_entry = bad.value
        check(rc)

    def weights(self, w):
        """w [k, rows] (FP64 or FP32) permuted into column order: wt [k * rows]."""
        if w.dtype not in (torch.float64, torch.float32):
            raise ValueError("w must be float64 or float32")
        _dev(w, w.dtype, (self.k, self.rows), name="w")
        wt = torch.empty(max(1, self.k * self.rows), dtype=w.dtype, device=w.device)
        dtype = 0 if w.dtype == torch.float64 else 1
        check(lib.rbf_ell_transpose_weights(self.rows, self.k, _ptr(self.src), _ptr(self.slot),
                                            _ptr(w), _ptr(wt), dtype, _stream()))
        return wt

    def apply(self, wt, y, out=None):
        """z = D^T y with column-ordered weights wt (from weights())."""
        if wt.dtype not in (torch.float64, torch.float32):
            raise ValueError("wt must be float64 or float32")
        _dev(wt, wt.dtype, (max(1, self.k * self.rows),), name="wt")
        _dev(y, wt.dtype, (self.rows,), name="y")
        if out is None:
            out = torch.empty(self.ncols, dtype=wt.dtype, device=wt.device)
        _dev(out, wt.dtype, (self.ncols,), name="out")
        dtype = 0 if wt.dtype == torch.float64 else 1
        check(lib.rbf_ell_apply_transpose(self.ncols, _ptr(self.colptr), _ptr(self.src), _ptr(wt),
                                          _ptr(y), _ptr(out), dtype, _stream()))
        return out


def ell_transpose(idx, ncols):
    """Transposed-product structure of the ELL index array idx [k, rows]."""
    return Transpose(idx, ncols)


def cast_f32(a):
    """FP32 copy of an FP64 device tensor (round to nearest), on the GPU."""
    _dev(a, torch.float64, name="a")
    out = torch.empty(a.shape, dtype=torch.float32, device=a.device)
    check(lib.rbf_cast_f32(_ptr(a), _ptr(out), a.numel(), _stream()))
    return out


class Solver:
    """Fractional-step solver handle (rbf_solver_create / rbf_step / ...).

    grid: dict with device tensors xv [2,N], xp [2,M], v_tag int8 [N],
    p_tag int8 [M], p_normal [2,M].  ops: dict with k and the ELL arrays
    idx_vv, vv_dx, vv_dy, vv_lap, idx_pv, pv_dx, pv_dy, idx_pp, pp_dx, pp_dy,
    pp_lap, idx_vp, vp_dx, vp_dy (device, [k, rows]).
    """

    PRECOND = {"auto": 0, "none": 1, "lattice": 2, "aux": 3}
    PRECISION = {"fp64": 0, "mixed": 1}

    def __init__(self, grid, ops, u_bc, v_bc, re, dt, rtol_h=1e-13, rtol_p=1e-12,
                 maxit_h=2000, maxit_p=20000, precond="auto", precision="fp64", u_conv=1.0):
        N = grid["xv"].shape[1]
        M = grid["xp"].shape[1]
        self.N, self.M = N, M
        self.device = grid["xv"].device
        _dev(grid["xv"], torch.float64, (2, N), "xv")
        _dev(grid["xp"], torch.float64, (2, M), "xp")
        _dev(grid["v_tag"], torch.int8, (N,), "v_tag")
        _dev(grid["p_tag"], torch.int8, (M,), "p_tag")
        _dev(grid["p_normal"], torch.float64, (2, M), "p_normal")
        k = int(ops["k"])
        for name, rows in (("vv", N), ("pv", M), ("pp", M), ("vp", N)):
            _dev(ops["idx_" + name], torch.int32, (k, rows), "idx_" + name)
        for name, rows in (("vv_dx", N), ("vv_dy", N), ("vv_lap", N), ("pv_dx", M), ("pv_dy", M),
                           ("pp_dx", M), ("pp_dy", M), ("pp_lap", M), ("vp_dx", N), ("vp_dy", N)):
            _dev(ops[name], torch.float64, (k, rows), name)
        _dev(u_bc, torch.float64, (N,), "u_bc")
        _dev(v_bc, torch.float64, (N,), "v_bc")
        g = _lib.Grid(N, M, grid["xv"].data_ptr(), grid["xp"].data_ptr(), grid["v_tag"].data_ptr(),
                      grid["p_tag"].data_ptr(), grid["p_normal"].data_ptr())
        o = _lib.Ops(k, *[ops[n].data_ptr() for n in (
            "idx_vv", "vv_dx", "vv_dy", "vv_lap", "idx_pv", "pv_dx", "pv_dy",
            "idx_pp", "pp_dx", "pp_dy", "pp_lap", "idx_vp", "vp_dx", "vp_dy")])
        prm = _lib.Params(float(re), float(dt), float(rtol_h), float(rtol_p), int(maxit_h),
                          int(maxit_p), self.PRECISION[precision], self.PRECOND[precond],
                          float(u_conv))
        h = ctypes.c_void_p()
        check(lib.rbf_solver_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(o),
                                    _ptr(u_bc), _ptr(v_bc), ctypes.byref(prm), _stream()))
        self._h = h

    def new_state(self, u, v):
        """Caller-owned state tensors with u, v given and p~ = p = C = 0."""
        z = lambda n: torch.zeros(n, dtype=torch.float64, device=self.device)  # noqa: E731
        return {"u": u.clone(), "v": v.clone(), "p_tilde": z(self.M), "p": z(self.M),
                "cu_prev": z(self.N), "cv_prev": z(self.N), "step": 0}

    def step(self, state, nsteps=1):
        """Advance the state dict in place; returns the step statistics."""
        st = self._state_struct(state)
        stats = _lib.StepStats()
        rc = lib.rbf_step(self._h, int(nsteps), ctypes.byref(st), ctypes.byref(stats))
        state["step"] = st.step
        check(rc)
        return stats

    def _state_struct(self, state):
        for key, n in (("u", self.N), ("v", self.N), ("cu_prev", self.N), ("cv_prev", self.N),
                       ("p_tilde", self.M), ("p", self.M)):
            _dev(state[key], torch.float64, (n,), key)
        return _lib.State(*[state[k].data_ptr() for k in ("u", "v", "p_tilde", "p", "cu_prev",
                                                            "cv_prev")], int(state["step"]))

    def solve_pressure(self, rhs, p_tilde):
        _dev(rhs, torch.float64, (self.M,), "rhs")
        _dev(p_tilde, torch.float64, (self.M,), "p_tilde")
        stats = _lib.SolveStats()
        check(lib.rbf_solve_pressure(self._h, _ptr(rhs), _ptr(p_tilde), ctypes.byref(stats)))
        return stats

    def apply_precond(self, y):
        """z = P^-1 y, one application of the pressure preconditioner (lattice
        or auxiliary-lattice)."""
        _dev(y, torch.float64, (self.M,), "y")
        z = torch.empty_like(y)
        check(lib.rbf_solver_apply_precond(self._h, _ptr(y), _ptr(z)))
        return z

    def profile(self, sample_every=-1):
        """Sampled kernel durations so far: {"gemm", "spmv", "smooth", "gs"}, each
        (avg_ms, count) (slots RBF_PROF_*); with sample_every >= 0, reset and
        sample every sample_every-th pressure iteration from now on."""
        avg = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int64 * 4)()
        check(lib.rbf_solver_profile(self._h, int(sample_every), avg, cnt))
        return {name: (avg[q], cnt[q]) for q, name in enumerate(("gemm", "spmv", "smooth", "gs"))}

    def forces(self, grid, state, tag=1, center=(0.0, 0.0), radius=0.5):
        """(F_x, F_y) on the circular body whose nodes carry `tag`
        (rbf_solver_forces); C_D, C_L = 2 F / (rho U^2 D)."""
        g = _lib.Grid(self.N, self.M, grid["xv"].data_ptr(), grid["xp"].data_ptr(),
                      grid["v_tag"].data_ptr(), grid["p_tag"].data_ptr(),
                      grid["p_normal"].data_ptr())
        st = self._state_struct(state)
        f = (ctypes.c_double * 2)()
        check(lib.rbf_solver_forces(self._h, ctypes.byref(g), ctypes.byref(st), int(tag),
                                    float(center[0]), float(center[1]), float(radius), f))
        return f[0], f[1]

    def info(self):
        """How the solves run: {"viscous_jacobi", "lattice_precond", "jacobi_bound",
        "aux_precond", "aux_cells", "viscous_mixed", "aux_smooth_weight"}."""
        inf = _lib.SolverInfo()
        check(lib.rbf_solver_query(self._h, ctypes.byref(inf)))
        return {"viscous_jacobi": bool(inf.viscous_jacobi),
                "lattice_precond": bool(inf.lattice_precond), "jacobi_bound": inf.jacobi_bound,
                "aux_precond": bool(inf.aux_precond), "aux_cells": int(inf.aux_cells),
                "viscous_mixed": bool(inf.viscous_mixed),
                "aux_smooth_weight": float(inf.aux_smooth_weight)}

    def run(self, state, nsteps, every=10, log=None):
        """Advance `state` by `nsteps` in rbf_step calls of `every` steps and,
        after each call, append one JSON line to the open file `log` (if given)
        with the step, the Krylov iterations per step and the last solves'
        relative residuals (rbf_step_stats) and the state's diagnostics
        (rbf_solver_diagnostics).  Each call starts its initial-guess history
        afresh, so the chunk size changes the iterates within the solver
        tolerance.  Returns the list of records."""
        import json
        every = max(1, int(every))
        records = []
        done = 0
        while done < nsteps:
            k = min(every, nsteps - done)
            s = self.step(state, k)
            done += k
            rec = {"step": int(state["step"]),
                   "poisson_iters_per_step": s.poisson_iters / k,
                   "helmholtz_iters_per_step": s.helmholtz_iters / k,
                   "poisson_rel_residual": s.last_poisson.rel_residual,
                   "helmholtz_rel_residual": max(s.last_helmholtz_u.rel_residual,
                                                 s.last_helmholtz_v.rel_residual),
                   **self.diagnostics(state)}
            records.append(rec)
            if log is not None:
                log.write(json.dumps(rec) + "\n")
                log.flush()
        return records

    def adjoint_step(self, fwd, adj, grad_bc):
        """rbf_adjoint_step: `adj` (dict of device tensors u, v, p_tilde,
        cu_prev, cv_prev) holds the adjoints of the state one step after
        `fwd` on entry and of `fwd` on return; grad_bc (device [2, N])
        accumulates the boundary-value adjoints.  Returns dJ/dnu of the step."""
        f = self._state_struct(fwd)
        for key, n in (("u", self.N), ("v", self.N), ("cu_prev", self.N), ("cv_prev", self.N),
                       ("p_tilde", self.M)):
            _dev(adj[key], torch.float64, (n,), "adj " + key)
        _dev(grad_bc, torch.float64, (2, self.N), "grad_bc")
        a = _lib.State(adj["u"].data_ptr(), adj["v"].data_ptr(), adj["p_tilde"].data_ptr(),
                       adj["p_tilde"].data_ptr(), adj["cu_prev"].data_ptr(),
                       adj["cv_prev"].data_ptr(), 0)
        dnu = ctypes.c_double(0.0)
        check(lib.rbf_adjoint_step(self._h, ctypes.byref(f), ctypes.byref(a), _ptr(grad_bc),
                                   ctypes.byref(dnu)))
        return dnu.value

    def diagnostics(self, state):
        """Health figures of a state: {"div_max", "div_rms", "kinetic_energy",
        "speed_max", "cfl"} (rbf_solver_diagnostics)."""
        st = self._state_struct(state)
        d = _lib.Diagnostics()
        check(lib.rbf_solver_diagnostics(self._h, ctypes.byref(st), ctypes.byref(d)))
        return {f: getattr(d, f) for f, _ in d._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.rbf_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(solvers, states, nsteps=1, nthreads=0):
    """Advance independent instances concurrently (rbf_step_batch): solvers[b]
    with the state dict states[b], nsteps steps each, on nthreads host threads
    (0: the library's default).  Give each solver its own stream (create it
    under ``torch.cuda.stream(s)``) for their work to overlap.  Returns the
    per-instance step statistics and statuses; raises RbfError for the
    lowest-numbered failed instance after all were attempted (its
    ``statuses`` and ``stats`` attributes hold every instance's)."""
    n = len(solvers)
    if len(states) != n:
        raise ValueError("step_batch: one state per solver")
    hs = (ctypes.c_void_p * n)(*[s._h for s in solvers])
    sts = (_lib.State * n)(*[s._state_struct(st) for s, st in zip(solvers, states)])
    stats = (_lib.StepStats * n)()
    codes = (ctypes.c_int32 * n)()
    rc = lib.rbf_step_batch(hs, n, int(nsteps), sts, stats, codes, int(nthreads))
    for st, c in zip(states, sts):
        st["step"] = c.step
    try:
        check(rc)
    except _lib.RbfError as e:
        e.statuses, e.stats = list(codes), list(stats)
        raise
    return list(stats), list(codes)


class LidRollout:
    """Differentiable lid-driven cavity rollout: J(nu, coef) = kinetic energy
    (rbf_solver_diagnostics: 1/2 mean over V-nodes of u^2 + v^2) after
    `nsteps` steps from rest, with nu = 1/Re and the lid velocity
    u_lid = sum_k coef[k] modes[k] on the lid V-nodes (modes: device
    [nmodes, N], zero off the lid).  Calling it returns a torch scalar whose
    backward runs rbf_adjoint_step backwards through the rollout from
    checkpoints taken every `every` steps (the states inside a segment are
    recomputed, one rbf_step each, as the forward pass takes them).
    grid, ops: as for Solver; solver_kw: further Solver arguments."""

    def __init__(self, grid, ops, modes, dt, nsteps, every=10, **solver_kw):
        self.grid, self.ops, self.modes = grid, ops, modes
        self.dt, self.nsteps, self.every = float(dt), int(nsteps), max(1, int(every))
        self.solver_kw = solver_kw
        self.N = grid["xv"].shape[1]
        self.wall = grid["v_tag"] != 0

    def _solver(self, nu, coef):
        u_bc = (coef.to(self.modes) @ self.modes).contiguous()
        v_bc = torch.zeros_like(u_bc)
        S = Solver(self.grid, self.ops, u_bc, v_bc, 1.0 / float(nu), self.dt, **self.solver_kw)
        st = S.new_state(torch.where(self.wall, u_bc, torch.zeros_like(u_bc)), v_bc)
        return S, st

    @staticmethod
    def _clone(st):
        return {k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in st.items()}

    def __call__(self, nu, coef):
        return _LidRolloutFn.apply(nu, coef, self)


class _LidRolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, nu, coef, R):
        S, st = R._solver(nu, coef)
        checkpoints = []
        for j in range(R.nsteps):
            if j % R.every == 0:
                checkpoints.append(R._clone(st))
            S.step(st, 1)
        J = S.diagnostics(st)["kinetic_energy"]
        ctx.R, ctx.S, ctx.checkpoints, ctx.final = R, S, checkpoints, st
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        R, S, final = ctx.R, ctx.S, ctx.final
        N, M = S.N, S.M
        z = lambda n: torch.zeros(n, dtype=torch.float64, device=S.device)  # noqa: E731
        adj = {"u": final["u"] / N, "v": final["v"] / N, "p_tilde": z(M), "cu_prev": z(N),
               "cv_prev": z(N)}
        grad_bc = torch.zeros((2, N), dtype=torch.float64, device=S.device)
        dnu = 0.0
        for c in range(len(ctx.checkpoints) - 1, -1, -1):
            st = R._clone(ctx.checkpoints[c])
            seg = [R._clone(st)]
            stop = min(R.nsteps, (c + 1) * R.every)
            for _ in range(c * R.every, stop - 1):
                S.step(st, 1)
                seg.append(R._clone(st))
            for fwd in reversed(seg):
                dnu += S.adjoint_step(fwd, adj, grad_bc)
        # The initial state's wall values are the boundary data as well.
        gu = grad_bc[0] + torch.where(R.wall, adj["u"], torch.zeros_like(adj["u"]))
        S.close()
        g = float(gJ)
        d_coef = (R.modes @ gu) * g
        return torch.tensor(dnu * g, dtype=torch.float64), d_coef.to(torch.float64).cpu(), None
