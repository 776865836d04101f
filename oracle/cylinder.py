"""Flow past a cylinder (Sec. 5.2), oracle; test infrastructure only.

The step is the cavity's (``CavityOracle``: Sec. 3, eqs. (14)-(21), factor
once, SuperLU or dense LU) on the channel node set of
``rbf_inputs.cylinder_nodes``, with the channel's boundary rows.  Every
boundary V row carries a value through the Kim-Moin form of eq. (21),
u** = u_bc^{j+1} + dt D_x^VP p~_j (v: D_y^VP), where u_bc^{j+1} is

  inflow  (tag 3): U_inf, 0                    (uniform inflow)
  cylinder (tag 1): 0, 0                       (no slip)
  sides   (tag 5): u: the D_y^VV row of the node solved for the node's own
                   value with its neighbours at step j (du/dy = 0), v: 0
                   (symmetry: v = du/dy = 0)
  outflow (tag 4): q_i^j - dt U_c (D_x^VV q^j)_i for q = u, v (convective
                   outflow dq/dt + U_c dq/dx = 0, explicit Euler, U_c = U_inf)

Readings (the paper is silent on the discrete form of its open boundaries;
the workload asks for a convective outflow where the paper has a
stress-free one): the open rows are updated explicitly from step j; the
pressure keeps the homogeneous Neumann rows and the zero-mean border of the
cavity on every boundary (the forces only see pressure differences).

Initial state (Sec. 5.2): U_0 = (U_inf, 0) everywhere off the cylinder,
(0, 0) on it; p~ = p = 0.

Forces (Sec. 5.2): F = the closed integral over the cylinder of
(-p I + (1/Re)(grad U + grad U^T)) n ds, n the unit normal pointing out of
the body, with p (eq. (19)) at the cylinder's P-nodes and the velocity
gradients (D^VV rows) at its V-nodes, each set integrated over its own
equally spaced angles by the periodic composite Simpson's rule
(weights 4/3 and 2/3 of the angle step alternating, times the radius);
C_D = F_x / (rho U_inf^2 D / 2), C_L = F_y / (rho U_inf^2 D / 2), rho = 1.
"""
import numpy as np
import scipy.sparse as sp

from .cavity import CavityOracle, CavityState

TAG_CYLINDER, TAG_INFLOW, TAG_OUTFLOW, TAG_SIDE = 1, 3, 4, 5


class ChannelOracle(CavityOracle):
    def __init__(self, nodes, re, dt, u_inf=1.0, **kw):
        vt = nodes.v_tag
        u_bc = np.where(vt == TAG_INFLOW, u_inf, 0.0)
        v_bc = np.zeros(nodes.n_v)
        super().__init__(nodes, u_bc, v_bc, re, dt, **kw)
        self.u_inf = float(u_inf)
        self.side = vt == TAG_SIDE
        self.outflow = vt == TAG_OUTFLOW
        Dy = self.ops.Dy_vv.tocsr()
        self.dy_diag = Dy.diagonal()
        self.Dy_off = (Dy - sp.diags(self.dy_diag)).tocsr()
        self.u_bc0, self.v_bc0 = self.u_bc.copy(), self.v_bc.copy()

    def initial_state(self):
        N, M = self.nodes.n_v, self.nodes.n_p
        cyl = self.nodes.v_tag == TAG_CYLINDER
        u = np.where(cyl, 0.0, self.u_inf)
        return CavityState(u, np.zeros(N), np.zeros(M), np.zeros(M), np.zeros(N), np.zeros(N), 0)

    def open_values(self, u, v):
        """Boundary values u_bc^{j+1}, v_bc^{j+1} of every V row from the
        state at step j (fixed rows keep their values)."""
        ub, vb = self.u_bc0.copy(), self.v_bc0.copy()
        with np.errstate(divide="ignore", invalid="ignore"):
            us = -(self.Dy_off @ u) / self.dy_diag
        ub = np.where(self.side, us, ub)
        vb = np.where(self.side, 0.0, vb)
        cx = self.dt * self.u_inf
        ub = np.where(self.outflow, u - cx * (self.ops.Dx_vv @ u), ub)
        vb = np.where(self.outflow, v - cx * (self.ops.Dx_vv @ v), vb)
        return ub, vb

    def step(self, s, stages=None):
        self.u_bc, self.v_bc = self.open_values(s.u, s.v)
        return super().step(s, stages)


def simpson_periodic_weights(n):
    """Composite Simpson weights over one period of n equally spaced angles
    (n even): (4/3, 2/3, ...) times the angle step, starting with 2/3 at
    index 0 (the closing endpoint folded onto it)."""
    if n % 2:
        raise ValueError("Simpson's rule needs an even number of intervals")
    d = 2.0 * np.pi / n
    return np.where(np.arange(n) % 2 == 1, 4.0 * d / 3.0, 2.0 * d / 3.0)


def _ring(xy, rows, center):
    """rows ordered by their angle about center, in [0, 2 pi)."""
    ang = np.arctan2(xy[1, rows] - center[1], xy[0, rows] - center[0])
    ang = np.where(ang < 0.0, ang + 2.0 * np.pi, ang)
    order = np.argsort(ang, kind="stable")
    return rows[order], ang[order]


def cylinder_forces(nodes, ops, u, v, p, re, center=(0.0, 0.0), radius=0.5):
    """(F_x, F_y) on the cylinder as the module docstring states; C_D and
    C_L are 2 F_x and 2 F_y for U_inf = D = rho = 1."""
    prow, pang = _ring(nodes.xp, np.flatnonzero(nodes.p_tag == TAG_CYLINDER), center)
    vrow, vang = _ring(nodes.xv, np.flatnonzero(nodes.v_tag == TAG_CYLINDER), center)
    wp = simpson_periodic_weights(prow.size) * radius
    wv = simpson_periodic_weights(vrow.size) * radius
    nxp, nyp = np.cos(pang), np.sin(pang)
    fx = -np.sum(wp * p[prow] * nxp)
    fy = -np.sum(wp * p[prow] * nyp)
    ux, uy = (ops.Dx_vv @ u)[vrow], (ops.Dy_vv @ u)[vrow]
    vx, vy = (ops.Dx_vv @ v)[vrow], (ops.Dy_vv @ v)[vrow]
    nxv, nyv = np.cos(vang), np.sin(vang)
    sxy = uy + vx
    fx += np.sum(wv * (2.0 * ux * nxv + sxy * nyv)) / re
    fy += np.sum(wv * (sxy * nxv + 2.0 * vy * nyv)) / re
    return fx, fy
