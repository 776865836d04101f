"""Truncation-error metrics of Sec. 4 (oracle).

* Test-function error, eqs. (23)-(24): for each alpha-node j,
  g_j(x) = cos(x / dr_j) cos(y / dr_j) (so that k~ dr_j = sqrt(2)), and
      E = (1/R) sum_j |delta_j g_j - L g_j(x_j)| / max|L g_j|.
  Readings: dr_j ("locally averaged distance between adjacent nodes",
  Sec. 3) is the mean, over the stencil nodes of row j, of each stencil
  node's mean distance to its 6 nearest other beta-nodes (6 being the
  typical number of edge neighbours of a vertex in a 2-D triangulation, the
  paper's mesh type); the denominator is
  the analytic amplitude of L g_j (1 for the identity, 1/dr_j for D_x and
  D_y, 2/dr_j^2 for the Laplacian); the 1/N prefactor is 1/(number of rows).
* Modified wavenumber, eq. (22): k* = -i delta_r{e^{i k~ r~}} e^{-i k~ r~} with
  delta_r = cos(theta) D_x + sin(theta) D_y; for the second derivative the
  Laplacian is used, k*^2 = -D_Lap{e^{i k.x}} e^{-i k.x}.
"""
import numpy as np
from scipy.spatial import cKDTree

from .weights import OP_ID, OP_DX, OP_DY, OP_LAP


N_ADJACENT = 6


def adjacent_distance(xs, n_adj=N_ADJACENT):
    """Mean distance from every node to its n_adj nearest other nodes."""
    d, _ = cKDTree(xs.T).query(xs.T, k=n_adj + 1)
    return d[:, 1:].mean(axis=1)


def local_spacing(idx, xs):
    """dr_j: the adjacent-node distance averaged over the stencil of row j."""
    return adjacent_distance(xs)[idx].mean(axis=0)


def relative_error_E(xq, xs, idx, w, op):
    """E^(alpha,beta) of eq. (24) for one operator (weights w[s, r])."""
    dr = local_spacing(idx, xs)
    sx = xs[0][idx] / dr[None, :]
    sy = xs[1][idx] / dr[None, :]
    approx = np.sum(w * (np.cos(sx) * np.cos(sy)), axis=0)
    qx = xq[0] / dr
    qy = xq[1] / dr
    if op == OP_ID:
        exact, amp = np.cos(qx) * np.cos(qy), np.ones_like(dr)
    elif op == OP_DX:
        exact, amp = -np.sin(qx) * np.cos(qy) / dr, 1.0 / dr
    elif op == OP_DY:
        exact, amp = -np.cos(qx) * np.sin(qy) / dr, 1.0 / dr
    elif op == OP_LAP:
        exact, amp = -2.0 * np.cos(qx) * np.cos(qy) / dr ** 2, 2.0 / dr ** 2
    else:
        raise ValueError(op)
    return float(np.mean(np.abs(approx - exact) / amp))


def modified_wavenumber(xq, xs, idx, wx, wy, wlap, kdr=np.sqrt(2.0), thetas=None):
    """Mean normalised modified wavenumbers k*/k~ (first derivative) and
    (k*/k~)^2 (Laplacian) over the rows, for each wave angle theta."""
    if thetas is None:
        thetas = np.linspace(0.0, np.pi, 37)
    dr = local_spacing(idx, xs)
    kt = kdr / dr
    first, second = [], []
    for th in thetas:
        kx = kt * np.cos(th)
        ky = kt * np.sin(th)
        ph = np.exp(1j * (kx[None, :] * (xs[0][idx] - xq[0][None, :])
                          + ky[None, :] * (xs[1][idx] - xq[1][None, :])))
        d1 = np.sum((np.cos(th) * wx + np.sin(th) * wy) * ph, axis=0)
        first.append(np.mean((-1j * d1).real / kt))
        d2 = np.sum(wlap * ph, axis=0)
        second.append(np.mean((-d2).real / kt ** 2))
    return np.asarray(thetas), np.asarray(first), np.asarray(second)
