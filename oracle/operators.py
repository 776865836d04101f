"""Global sparse differentiation matrices and the implicit system matrices.

Sec. 2.2 (eq. (10)): D_L^(alpha,beta) has, in row j, the n weights of the
alpha-node x_j at the columns of its stencil and zeros elsewhere (M x n
nonzeros).  Sec. 4 lists the eight matrices the fractional-step scheme needs:
D_x, D_y, D_Lap on (V,V); D_x, D_y on (P,V); D_Lap on (P,P); D_x, D_y on (V,P).
The pressure boundary rows use D_x, D_y on (P,P) as well (see ``poisson``).

Storage: slot-major ELL ``idx[s, r]``, ``w[s, r]``; the oracle converts to
SciPy CSR for application and factorisation.
"""
import numpy as np
import scipy.sparse as sp

from . import knn as _knn
from . import weights as _w


def ell_to_csr(idx, w, ncols):
    n, R = idx.shape
    rows = np.repeat(np.arange(R), n)
    return sp.csr_matrix((np.asarray(w).T.ravel(), (rows, np.asarray(idx).T.ravel())),
                         shape=(R, ncols))


def ell_apply(idx, w, x):
    """y_r = sum_s w[s, r] x[idx[s, r]] (eq. (10) applied to a vector)."""
    return np.einsum("sr,sr->r", w, x[idx])


def ell_apply_transpose(idx, w, y, ncols):
    """z = D^T y for the matrix of eq. (10) held as ELL: z_c is the sum of
    w[s, r] y[r] over the entries with idx[s, r] = c (the transposed product
    an adjoint of the scheme applies)."""
    idx = np.asarray(idx)
    z = np.zeros(ncols)
    np.add.at(z, idx.ravel(), (np.asarray(w) * np.asarray(y)[None, :]).ravel())
    return z


class StencilSet:
    """Stencils and weights of one (alpha, beta) pair."""

    def __init__(self, xq, xs, n, m, q, ops, knn_fn=None, force=False):
        knn_fn = knn_fn or _knn.knn
        self.idx = knn_fn(xq, xs, n)
        self.ops = list(ops)
        self.w = _w.stencil_weights(xq, xs, self.idx, m, q, self.ops, force=force)
        self.nrows = xq.shape[1]
        self.ncols = xs.shape[1]

    def weights(self, op):
        return self.w[self.ops.index(op)]

    def csr(self, op):
        return ell_to_csr(self.idx, self.weights(op), self.ncols)


class CavityOperators:
    """The four stencil sets of the staggered scheme (Sec. 4, items 1-4).

    VV: D_x, D_y, D_Lap      (N x N)
    PV: D_x, D_y             (M x N), velocity divergence on the P-grid
    PP: D_x, D_y, D_Lap      (M x M), Laplacian + Neumann boundary rows
    VP: D_x, D_y             (N x M), pressure gradient on the V-grid
    """

    def __init__(self, nodes, n=28, m=7, q=3, knn_fn=None):
        X, Y, L = _w.OP_DX, _w.OP_DY, _w.OP_LAP
        self.nodes = nodes
        self.vv = StencilSet(nodes.xv, nodes.xv, n, m, q, (X, Y, L), knn_fn)
        self.pv = StencilSet(nodes.xp, nodes.xv, n, m, q, (X, Y), knn_fn)
        self.pp = StencilSet(nodes.xp, nodes.xp, n, m, q, (X, Y, L), knn_fn)
        self.vp = StencilSet(nodes.xv, nodes.xp, n, m, q, (X, Y), knn_fn)
        self.Dx_vv = self.vv.csr(X)
        self.Dy_vv = self.vv.csr(Y)
        self.L_vv = self.vv.csr(L)
        self.Dx_pv = self.pv.csr(X)
        self.Dy_pv = self.pv.csr(Y)
        self.Dx_pp = self.pp.csr(X)
        self.Dy_pp = self.pp.csr(Y)
        self.L_pp = self.pp.csr(L)
        self.Dx_vp = self.vp.csr(X)
        self.Dy_vp = self.vp.csr(Y)


def helmholtz_matrix(ops, a):
    """Crank-Nicolson matrix of eq. (16): I - a D_Lap^(V,V) on interior V rows,
    identity on wall rows (which carry the Dirichlet/Kim-Moin values)."""
    N = ops.nodes.n_v
    interior = (ops.nodes.v_tag == 0).astype(np.float64)
    Dint = sp.diags(interior) @ ops.L_vv
    return (sp.identity(N, format="csr") - a * Dint).tocsr()


def poisson_matrix(ops):
    """Pressure-Poisson operator of eq. (18) with boundary rows, bordered.

    The paper states no pressure boundary condition.  Reading: the pressure
    correction of the Kim-Moin scheme satisfies a homogeneous Neumann
    condition, so wall P-rows are n_x D_x^(P,P) + n_y D_y^(P,P); interior rows
    are D_Lap^(P,P).  With Neumann rows the constants span the null space and
    the right-hand side F/dt is in general not compatible with the discrete
    operator, so the system is bordered: one Lagrange multiplier lam enters
    every interior row as a uniform source and one row fixes mean(p~) = 0,

        [ A0   chi ] [p~ ]   [ F/dt on interior rows, 0 on wall rows ]
        [ 1/M  0   ] [lam] = [ 0                                     ]

    (chi = indicator of interior rows).  Returns (A0, chi) in CSR/ndarray
    form and the bordered (M+1) x (M+1) matrix.
    """
    nd = ops.nodes
    M = nd.n_p
    interior = (nd.p_tag == 0).astype(np.float64)
    wall = 1.0 - interior
    A0 = (sp.diags(interior) @ ops.L_pp + sp.diags(wall * nd.p_normal[0]) @ ops.Dx_pp
          + sp.diags(wall * nd.p_normal[1]) @ ops.Dy_pp).tocsr()
    border_col = sp.csr_matrix(interior[:, None])
    border_row = sp.csr_matrix(np.full((1, M), 1.0 / M))
    B = sp.bmat([[A0, border_col], [border_row, None]], format="csr")
    return A0, interior, B
