"""Semi-implicit fractional-step solver on staggered nodes (oracle).

Sec. 3 advances (u, v, p) from step j to j+1 in three stages:
  1. AB2 advection (eqs. (14)-(15)):
       C_j(q) = -[u_j o (D_x^VV q) + v_j o (D_y^VV q)],
       u* = u_j + dt (3/2 C_j(u_j) - 1/2 C_{j-1}(u_{j-1})), same for v.
  2. Crank-Nicolson viscous step (eq. (16)), a = dt / (2 Re):
       (I - a D_Lap^VV) u** = (I + a D_Lap^VV) u*, same for v,
     with the Kim-Moin intermediate boundary values (eq. (21)) on wall rows:
       u** = u_{j+1} + dt D_x^VP p~_j,  v** = v_{j+1} + dt D_y^VP p~_j.
  3. Projection (eqs. (17)-(20)):
       F = D_x^PV u** + D_y^PV v**,  D_Lap^PP p~_{j+1} = F / dt,
       p_{j+1} = p~_{j+1} - a D_Lap^PP p~_{j+1},
       u_{j+1} = u** - dt D_x^VP p~_{j+1},  v_{j+1} = v** - dt D_y^VP p~_{j+1}.
The implicit matrices are factored once by LU and reused every step, as the
paper does at the end of Sec. 3 (dense LU for small grids, SuperLU above).

Readings where the paper is silent or ambiguous:
  * AB2 start: C_{-1} := C_0.
  * The CN right-hand side acts on u* (eq. (16) as printed).
  * Pressure boundary rows: homogeneous Neumann, with the Neumann system
    bordered by a uniform source and a zero-mean condition on p~ (see
    ``operators.poisson_matrix``); the right-hand side is F/dt on interior
    P-rows and 0 on wall rows.
  * Eq. (20) is applied on every V row, wall rows included, and the Kim-Moin
    values enter u** (and hence the divergence F) on wall rows: the scheme as
    printed.  Wall velocities then equal the boundary values to O(dt^2) and are
    re-imposed through eq. (21) on the next step.
  * Initial state: fluid at rest, walls at their boundary values, p~ = p = 0.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .operators import CavityOperators, helmholtz_matrix, poisson_matrix


class _Factored:
    def __init__(self, A, dense):
        self.dense = dense
        if dense:
            self.lu = sla.lu_factor(A.toarray())
        else:
            self.lu = spla.splu(A.tocsc())

    def solve(self, b):
        if self.dense:
            return sla.lu_solve(self.lu, b)
        return self.lu.solve(b)


class CavityState:
    def __init__(self, u, v, pt, p, cu_prev, cv_prev, step=0):
        self.u, self.v, self.pt, self.p = u, v, pt, p
        self.cu_prev, self.cv_prev = cu_prev, cv_prev
        self.step = step

    def copy(self):
        return CavityState(self.u.copy(), self.v.copy(), self.pt.copy(), self.p.copy(),
                           self.cu_prev.copy(), self.cv_prev.copy(), self.step)


class CavityOracle:
    def __init__(self, nodes, u_bc, v_bc, re, dt, n=28, m=7, q=3, dense=None,
                 ops=None):
        self.nodes = nodes
        self.ops = ops if ops is not None else CavityOperators(nodes, n, m, q)
        self.re = float(re)
        self.dt = float(dt)
        self.a = self.dt / (2.0 * self.re)
        self.u_bc = np.asarray(u_bc, np.float64)
        self.v_bc = np.asarray(v_bc, np.float64)
        self.vwall = nodes.v_tag != 0
        self.pint = nodes.p_tag == 0
        if dense is None:
            dense = max(nodes.n_v, nodes.n_p) <= 6000
        self.H = helmholtz_matrix(self.ops, self.a)
        self.A0, self.chi, self.Lp = poisson_matrix(self.ops)
        self.H_lu = _Factored(self.H, dense)
        self.Lp_lu = _Factored(self.Lp, dense)

    def initial_state(self):
        N, M = self.nodes.n_v, self.nodes.n_p
        u = np.where(self.vwall, self.u_bc, 0.0)
        v = np.where(self.vwall, self.v_bc, 0.0)
        return CavityState(u, v, np.zeros(M), np.zeros(M), np.zeros(N), np.zeros(N), 0)

    def advection(self, u, v):
        """C_j(u_j), C_j(v_j) of eq. (15)."""
        o = self.ops
        cu = -(u * (o.Dx_vv @ u) + v * (o.Dy_vv @ u))
        cv = -(u * (o.Dx_vv @ v) + v * (o.Dy_vv @ v))
        return cu, cv

    def pressure_rhs(self, F):
        return np.where(self.pint, F / self.dt, 0.0)

    def solve_pressure(self, rhs):
        """p~ (zero mean) and the uniform source lam of the bordered system."""
        sol = self.Lp_lu.solve(np.concatenate([rhs, [0.0]]))
        return sol[:-1], sol[-1]

    def predictor(self, q, c, c_prev):
        """Eq. (14): second-order Adams-Bashforth, q + dt (3/2 c - 1/2 c_prev)."""
        return q + self.dt * (1.5 * c - 0.5 * c_prev)

    def viscous(self, us, vs, pt_j):
        """Eq. (16) with the Kim-Moin wall values of eq. (21): (I - a D_Lap)
        u** = (I + a D_Lap) u* on interior rows, u** = u_bc + dt D_x^VP p~_j
        (v: D_y^VP) on wall rows.  Returns (u**, v**, ru, rv)."""
        o, dt, a = self.ops, self.dt, self.a
        ru = us + a * (o.L_vv @ us)
        rv = vs + a * (o.L_vv @ vs)
        ru = np.where(self.vwall, self.u_bc + dt * (o.Dx_vp @ pt_j), ru)
        rv = np.where(self.vwall, self.v_bc + dt * (o.Dy_vp @ pt_j), rv)
        return self.H_lu.solve(ru), self.H_lu.solve(rv), ru, rv

    def pressure_update(self, pt):
        """Eq. (19): p = p~ - a D_Lap^PP p~."""
        return pt - self.a * (self.ops.L_pp @ pt)

    def projection(self, uss, vss):
        """Eqs. (17), (18), (20): F = D^PV [u**, v**], the bordered Poisson
        solve for p~, and u = u** - dt D^VP p~.  Returns (u, v, p~, F, rhs, lam)."""
        o, dt = self.ops, self.dt
        F = o.Dx_pv @ uss + o.Dy_pv @ vss
        prhs = self.pressure_rhs(F)
        pt, lam = self.solve_pressure(prhs)
        return uss - dt * (o.Dx_vp @ pt), vss - dt * (o.Dy_vp @ pt), pt, F, prhs, lam

    def step(self, s, stages=None):
        """Advance one step; returns the new state.  ``stages`` (a dict), if
        given, receives the intermediate vectors for stage-level checks."""
        # Stage 1: AB2 advection.
        cu, cv = self.advection(s.u, s.v)
        cu_prev, cv_prev = (cu, cv) if s.step == 0 else (s.cu_prev, s.cv_prev)
        us = self.predictor(s.u, cu, cu_prev)
        vs = self.predictor(s.v, cv, cv_prev)
        # Stage 2: Crank-Nicolson with Kim-Moin wall values.
        uss, vss, ru, rv = self.viscous(us, vs, s.pt)
        # Stage 3: divergence, pressure Poisson, pressure and correction.
        un, vn, pt, F, prhs, lam = self.projection(uss, vss)
        p = self.pressure_update(pt)
        if stages is not None:
            stages.update(cu=cu, cv=cv, us=us, vs=vs, ru=ru, rv=rv, uss=uss, vss=vss,
                          F=F, prhs=prhs, lam=lam)
        return CavityState(un, vn, pt, p, cu, cv, s.step + 1)

    def run(self, nsteps, state=None, every=None, callback=None):
        s = state if state is not None else self.initial_state()
        for _ in range(nsteps):
            s = self.step(s)
            if callback is not None and every and s.step % every == 0:
                callback(s)
        return s

    def divergence(self, u, v):
        """D_x^PV u + D_y^PV v on the P-grid (eq. (17))."""
        return self.ops.Dx_pv @ u + self.ops.Dy_pv @ v
