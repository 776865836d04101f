"""Local PHS+poly RBF-FD weights (oracle).

Sec. 2.1: the weights w of L f(x_0) ~ sum_j w_j f(x_j) (eq. (4)) are the first
n unknowns of the augmented saddle-point system (eq. (9))

    [ A   P ] [w]   [ L phi ]
    [ P^T 0 ] [c] = [ L P   ]

with A_ij = phi(||x_i - x_j||), phi(r) = r^m for odd m (eq. (3)), P_jk the
monomials of total degree <= q at the stencil nodes (eqs. (6)-(8)), and the
right-hand side L applied to phi(||x - x_j||) and to the monomials, evaluated
at x = x_0.  The vector c is discarded (eq. (4) is what is applied).

Readings where the paper is silent (it defers to Flyer et al. 2016):
  * Local coordinates.  Nodes are shifted to x_0 and divided by s = 2^e, the
    power of two with 1/4 <= max_j |x_j - x_0|^2 / s^2 < 1, i.e.
    e = ceil(E/2) where max d^2 = f 2^E, 1/2 <= f < 1.  In exact arithmetic
    PHS+poly weights are invariant under translation and scale as s^-k for a
    k-th derivative, so this only affects rounding; a power of two makes the
    scaling itself exact.  Weights in physical units are the local ones times
    s^-k.
  * Monomial order: graded, x^a y^b for degree d = 0..q, b = 0..d with a = d-b
    (1; x, y; x^2, xy, y^2; x^3, x^2 y, x y^2, y^3 for q = 3).
  * Arithmetic: squared distances as dx*dx + dy*dy without fused multiply-add,
    r = sqrt(d^2), r^m = (d^2)^((m-1)/2) * r by left-to-right products, so the
    FP64 system is a fixed function of the coordinates.
  * Solve: LAPACK LU with partial pivoting (numpy.linalg.solve), then
    iterative refinement with the residual accumulated in extended precision,
    so the returned weights are the solution of the FP64 system to within a
    few ulps rather than to within cond(A_aug) * eps.

Operators (bit codes): ID = 1 (interpolation, L = identity), DX = 2, DY = 4,
LAP = 8 (Laplacian); ``ops`` lists codes in increasing bit order.
"""
import numpy as np

OP_ID, OP_DX, OP_DY, OP_LAP = 1, 2, 4, 8
_DERIV_ORDER = {OP_ID: 0, OP_DX: 1, OP_DY: 1, OP_LAP: 2}


def n_monomials(q):
    """K_p = (q+1)(q+2)/2 monomials of degree <= q in 2-D (0 for q < 0)."""
    return 0 if q < 0 else (q + 1) * (q + 2) // 2


def monomial_exponents(q):
    """Graded list of (a, b) with x^a y^b, degree 0..q."""
    return [(d - b, b) for d in range(q + 1) for b in range(d + 1)]


def ops_from_mask(mask):
    return [c for c in (OP_ID, OP_DX, OP_DY, OP_LAP) if mask & c]


def _ipow(b, n):
    """b**n as a left-to-right product chain (1 for n = 0)."""
    if n == 0:
        return np.ones_like(b)
    t = b
    for _ in range(n - 1):
        t = t * b
    return t


def _powers(t, n):
    """[t^0, t^1, ..., t^n] with t^a = t^(a-1) * t."""
    out = [np.ones_like(t)]
    for _ in range(n):
        out.append(out[-1] * t)
    return out


def scale_exponent(d2max):
    """e with s = 2^e: e = ceil(E/2) where d2max = f 2^E, 1/2 <= f < 1."""
    _, E = np.frexp(d2max)
    return -((-E) // 2)


def local_coordinates(xq, xs, idx):
    """Shifted, scaled stencil coordinates xt, yt [R, n] and exponents e [R]."""
    qx = xq[0][:, None]
    qy = xq[1][:, None]
    dx = xs[0][idx.T] - qx
    dy = xs[1][idx.T] - qy
    d2 = dx * dx + dy * dy
    e = scale_exponent(d2.max(axis=1))
    xt = np.ldexp(dx, -e[:, None])
    yt = np.ldexp(dy, -e[:, None])
    return xt, yt, e


def monomials(xt, yt, q):
    """P[..., t] = x^a y^b for the graded exponents (a, b)."""
    px = _powers(xt, q)
    py = _powers(yt, q)
    return np.stack([px[a] * py[b] for a, b in monomial_exponents(q)], axis=-1)


def phs_matrix(xt, yt, m):
    """A[r, i, j] = ||x_i - x_j||^m over each stencil (eq. (2))."""
    ddx = xt[:, :, None] - xt[:, None, :]
    ddy = yt[:, :, None] - yt[:, None, :]
    d2 = ddx * ddx + ddy * ddy
    return _ipow(d2, (m - 1) // 2) * np.sqrt(d2)


def rhs_phs(xt, yt, m, op):
    """L phi(||x - x_j||) at x = x_0 = 0 (right-hand side of eq. (5))."""
    d2 = xt * xt + yt * yt
    r = np.sqrt(d2)
    if op == OP_ID:
        return _ipow(d2, (m - 1) // 2) * r
    # d/dx r^m = m r^(m-2) (x - x_j); at x_0 = 0 this is -m r^(m-2) xt_j.
    rm2 = _ipow(d2, (m - 3) // 2) * r
    if op == OP_DX:
        return -float(m) * rm2 * xt
    if op == OP_DY:
        return -float(m) * rm2 * yt
    if op == OP_LAP:
        # In 2-D, Laplacian of r^m = m^2 r^(m-2).
        return float(m * m) * rm2
    raise ValueError(f"unknown operator code {op}")


def rhs_poly(q, op):
    """L applied to each monomial, evaluated at x_0 = 0 (eq. (7))."""
    out = np.zeros(n_monomials(q))
    for t, (a, b) in enumerate(monomial_exponents(q)):
        if op == OP_ID and (a, b) == (0, 0):
            out[t] = 1.0
        elif op == OP_DX and (a, b) == (1, 0):
            out[t] = 1.0
        elif op == OP_DY and (a, b) == (0, 1):
            out[t] = 1.0
        elif op == OP_LAP and (a, b) in ((2, 0), (0, 2)):
            out[t] = 2.0
    return out


def augmented_system(xt, yt, m, q, ops):
    """A_aug [R, s, s] and right-hand sides [R, s, nops] of eq. (9)."""
    R, n = xt.shape
    kp = n_monomials(q)
    s = n + kp
    A = np.zeros((R, s, s))
    A[:, :n, :n] = phs_matrix(xt, yt, m)
    if kp:
        P = monomials(xt, yt, q)
        A[:, :n, n:] = P
        A[:, n:, :n] = np.transpose(P, (0, 2, 1))
    B = np.zeros((R, s, len(ops)))
    for o, op in enumerate(ops):
        B[:, :n, o] = rhs_phs(xt, yt, m, op)
        if kp:
            B[:, n:, o] = rhs_poly(q, op)[None, :]
    return A, B


def solve_refined(A, B, refinements=2):
    """Solve A X = B (batched), refining with an extended-precision residual."""
    X = np.linalg.solve(A, B)
    Al = A.astype(np.longdouble)
    Bl = B.astype(np.longdouble)
    for _ in range(refinements):
        res = Bl - np.einsum("rij,rjo->rio", Al, X.astype(np.longdouble))
        X = X + np.linalg.solve(A, res.astype(np.float64))
    return X


def check_args(n, m, q, ops, ns, force=False):
    if n < 1 or n > ns:
        raise ValueError("stencil size must be in [1, number of source nodes]")
    if m < 1 or m % 2 == 0:
        raise ValueError("PHS exponent m must be an odd positive integer")
    if any(op != OP_ID for op in ops) and m < 3:
        raise ValueError("derivative operators need m >= 3 (L phi continuous)")
    if n_monomials(q) >= n:
        raise ValueError("stencil must have more nodes than monomials")
    if not force and q >= 0 and n < (q + 1) * (q + 2):
        raise ValueError("stencil smaller than (q+1)(q+2) (stability rule, Sec. 4)")


def stencil_weights(xq, xs, idx, m=7, q=3, ops=(OP_DX, OP_DY, OP_LAP),
                    chunk=4096, force=False):
    """Weights ``w[o, s, r]`` (slot-major ELL values) for each operator.

    xq: [2, R] evaluation nodes (alpha grid); xs: [2, ns] stencil nodes (beta
    grid); idx: [n, R] stencil indices (int32).
    """
    xq = np.asarray(xq, np.float64)
    xs = np.asarray(xs, np.float64)
    idx = np.asarray(idx)
    n, R = idx.shape
    ops = list(ops)
    check_args(n, m, q, ops, xs.shape[1], force)
    W = np.empty((len(ops), n, R))
    for a in range(0, R, chunk):
        b = min(R, a + chunk)
        xt, yt, e = local_coordinates(xq[:, a:b], xs, idx[:, a:b])
        A, B = augmented_system(xt, yt, m, q, ops)
        X = solve_refined(A, B)
        for o, op in enumerate(ops):
            W[o, :, a:b] = np.ldexp(X[:, :n, o], -_DERIV_ORDER[op] * e[:, None]).T
    return W
