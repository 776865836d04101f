"""Discrete adjoint of the fractional-step scheme (oracle; test
infrastructure).

The forward map is ``CavityOracle.step`` (Sec. 3, eqs. (14)-(21)); its
exact transpose, stage by stage in reverse order, gives the gradient of a
scalar objective of the final state with respect to the viscosity
nu = 1/Re and to the boundary velocities (here a lid profile).  The paper
has no adjoint; this is the reverse-mode derivative of the scheme as the
oracle reads it, written out with the transposed sparse matrices.

Forward step j -> j+1 (state u, v, p~, C_{j-1}; a = dt nu / 2):
  C(u) = -(u o Dx u + v o Dy u), C(v) likewise           (eq. (15))
  u* = u + dt (3/2 C_j - 1/2 C_{j-1})  (C_{-1} = C_0)       (eq. (14))
  r_u = (I + a L) u* on interior rows, u_bc + dt Gx p~_j on walls
  u** = H^-1 r_u, H = I - a chi L                          (eqs. (16), (21))
  F = Dx^PV u** + Dy^PV v**,  rhs = chi_P F / dt            (eq. (17))
  p~ = zero-mean solution of the bordered Poisson system   (eq. (18))
  u_{j+1} = u** - dt Gx p~, v_{j+1} likewise                (eq. (20))
Reverse step: the adjoint (u_bar, v_bar, pt_bar, cu_bar, cv_bar) of the
state at j+1 (cu_bar: adjoint of C_j as the next step's C_{j-1}) gives the
adjoint of the state at j and adds to nu_bar and to the boundary-value
adjoints ubc_bar, vbc_bar.

Objective used by the tests: J = 1/2 mean over V-nodes of u^2 + v^2 of the
final state (the unweighted kinetic energy of rbf_solver_diagnostics).
"""
import numpy as np
import scipy.linalg as sla

from .cavity import CavityOracle, CavityState


class AdjointCavity:
    """Forward steps that keep their intermediates, and their transposes."""

    def __init__(self, orc: CavityOracle):
        self.o = orc
        ops = orc.ops
        nd = orc.nodes
        self.wall = nd.v_tag != 0
        self.chi_p = (nd.p_tag == 0).astype(np.float64)
        self.chi_v = (~self.wall).astype(np.float64)
        self.DxT, self.DyT = ops.Dx_vv.T.tocsr(), ops.Dy_vv.T.tocsr()
        self.LT = ops.L_vv.T.tocsr()
        self.GxT, self.GyT = ops.Dx_vp.T.tocsr(), ops.Dy_vp.T.tocsr()
        self.DpxT, self.DpyT = ops.Dx_pv.T.tocsr(), ops.Dy_pv.T.tocsr()
        M = nd.n_p
        # Transposes of the factored systems (dense LU: solve with trans=1).
        self.Hd = sla.lu_factor(orc.H.toarray())
        self.Bd = sla.lu_factor(orc.Lp.toarray())
        self.M = M

    def step(self, s):
        """Forward step with the intermediates the reverse step needs."""
        o = self.o
        cu, cv = o.advection(s.u, s.v)
        cu_prev, cv_prev = (cu, cv) if s.step == 0 else (s.cu_prev, s.cv_prev)
        us = o.predictor(s.u, cu, cu_prev)
        vs = o.predictor(s.v, cv, cv_prev)
        uss, vss, ru, rv = o.viscous(us, vs, s.pt)
        un, vn, pt, F, prhs, lam = o.projection(uss, vss)
        p = o.pressure_update(pt)
        tape = dict(u=s.u, v=s.v, us=us, vs=vs, uss=uss, vss=vss, first=(s.step == 0))
        return CavityState(un, vn, pt, p, cu, cv, s.step + 1), tape

    def reverse(self, tape, ub, vb, ptb, cub, cvb):
        """Adjoint of one step.  Inputs: adjoints of u_{j+1}, v_{j+1},
        p~_{j+1} and of C_j (as the next step's C_{j-1}).  Returns the
        adjoints of (u_j, v_j, p~_j, C_{j-1}) and the contributions
        (nu_bar, ubc_bar, vbc_bar)."""
        o, ops = self.o, self.o.ops
        dt, a = o.dt, o.a
        M = self.M
        # eq. (20): u_{j+1} = u** - dt Gx p~, v likewise
        ussb = ub.copy()
        vssb = vb.copy()
        ptb = ptb - dt * (self.GxT @ ub) - dt * (self.GyT @ vb)
        # eq. (18): p~ = P0 (A0 + border)^-1 [rhs; 0] with the zero-mean
        # border; the bordered LU carries the mean condition, so the
        # transposed solve takes [pt_bar; 0].
        sol = sla.lu_solve(self.Bd, np.concatenate([ptb, [0.0]]), trans=1)
        rhsb = sol[:M]
        # eq. (17): rhs = chi_P F / dt
        Fb = self.chi_p * rhsb / dt
        ussb = ussb + self.DpxT @ Fb
        vssb = vssb + self.DpyT @ Fb
        # eq. (16): u** = H^-1 r_u
        rub = sla.lu_solve(self.Hd, ussb, trans=1)
        rvb = sla.lu_solve(self.Hd, vssb, trans=1)
        # d/d nu: H = I - a chi L and r = (I + a L) u* (interior), a = dt nu / 2
        half = dt / 2.0
        nub = half * (np.dot(rub, self.chi_v * (ops.L_vv @ (tape["us"] + tape["uss"])))
                      + np.dot(rvb, self.chi_v * (ops.L_vv @ (tape["vs"] + tape["vss"]))))
        # r_u: interior (I + a L) u*, wall u_bc + dt Gx p~_j (eq. (21))
        ri, rw = self.chi_v * rub, (1.0 - self.chi_v) * rub
        si, sw = self.chi_v * rvb, (1.0 - self.chi_v) * rvb
        usb = ri + a * (self.LT @ ri)
        vsb = si + a * (self.LT @ si)
        ubcb, vbcb = rw, sw
        ptb_prev = dt * (self.GxT @ rw) + dt * (self.GyT @ sw)
        # eq. (14): u* = u + dt (3/2 C_j - 1/2 C_{j-1})
        uj_b = usb.copy()
        vj_b = vsb.copy()
        cu_b = 1.5 * dt * usb + cub
        cv_b = 1.5 * dt * vsb + cvb
        cprev_u = -0.5 * dt * usb
        cprev_v = -0.5 * dt * vsb
        if tape["first"]:  # C_{-1} = C_0
            cu_b = cu_b + cprev_u
            cv_b = cv_b + cprev_v
            cprev_u = np.zeros_like(cprev_u)
            cprev_v = np.zeros_like(cprev_v)
        # eq. (15): C(u) = -(u o Dx u + v o Dy u), C(v) = -(u o Dx v + v o Dy v)
        u, v = tape["u"], tape["v"]
        Dxu, Dyu = ops.Dx_vv @ u, ops.Dy_vv @ u
        Dxv, Dyv = ops.Dx_vv @ v, ops.Dy_vv @ v
        uj_b = uj_b - Dxu * cu_b - self.DxT @ (u * cu_b) - self.DyT @ (v * cu_b) - Dxv * cv_b
        vj_b = vj_b - Dyu * cu_b - Dyv * cv_b - self.DxT @ (u * cv_b) - self.DyT @ (v * cv_b)
        return uj_b, vj_b, ptb_prev, cprev_u, cprev_v, nub, ubcb, vbcb


def kinetic_energy(u, v):
    return 0.5 * np.mean(u * u + v * v)


def rollout_gradient(orc, s0, nsteps, init_from_bc=True):
    """J = kinetic_energy of the state after nsteps from s0, and dJ/dnu and
    dJ/du_bc, dJ/dv_bc (the boundary-value adjoints, per V-node; with
    init_from_bc the wall values of s0 count as boundary data too, as in
    CavityOracle.initial_state)."""
    adj = AdjointCavity(orc)
    s = s0
    tapes = []
    for _ in range(nsteps):
        s, tape = adj.step(s)
        tapes.append(tape)
    N = orc.nodes.n_v
    J = kinetic_energy(s.u, s.v)
    ub, vb = s.u / N, s.v / N
    ptb = np.zeros(orc.nodes.n_p)
    cub = np.zeros(N)
    cvb = np.zeros(N)
    nub = 0.0
    ubc_b = np.zeros(N)
    vbc_b = np.zeros(N)
    for tape in reversed(tapes):
        ub, vb, ptb, cub, cvb, dn, du, dv = adj.reverse(tape, ub, vb, ptb, cub, cvb)
        nub += dn
        ubc_b += du
        vbc_b += dv
    if init_from_bc:  # the initial state takes its wall values from u_bc, v_bc
        ubc_b = ubc_b + np.where(adj.wall, ub, 0.0)
        vbc_b = vbc_b + np.where(adj.wall, vb, 0.0)
    return J, nub, ubc_b, vbc_b, (ub, vb, ptb)
