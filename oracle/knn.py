"""n-nearest-neighbour stencils (oracle).

Sec. 2.2: row j of D^(alpha,beta) uses the n nearest beta-nodes of the
alpha-node x_j; Sec. 4 fixes n = 28.  The paper is silent on ties, which are
common on lattices, so the stencil is defined as the first n beta-nodes in
the order of the key (d^2, beta index), with d^2 = dx*dx + dy*dy evaluated in
FP64 as two rounded products and one rounded sum (no fused multiply-add).
When alpha = beta and nodes are distinct, the node itself is slot 0.

Output layout is slot-major: ``idx[s, r]`` is slot s of row r (int32).
"""
import numpy as np


def _d2(qx, qy, sx, sy):
    dx = sx - qx
    dy = sy - qy
    return dx * dx + dy * dy


def knn_bruteforce(xq, xs, k, chunk=256):
    """Exact stencils by comparing every query with every source node."""
    xq = np.asarray(xq, np.float64)
    xs = np.asarray(xs, np.float64)
    nq = xq.shape[1]
    ns = xs.shape[1]
    if k > ns:
        raise ValueError("k exceeds the number of source nodes")
    out = np.empty((k, nq), np.int32)
    for a in range(0, nq, chunk):
        b = min(nq, a + chunk)
        d2 = _d2(xq[0, a:b, None], xq[1, a:b, None], xs[0][None, :], xs[1][None, :])
        # Every node whose d2 is at most the k-th smallest d2 of its row is a
        # candidate (ties at the k-th distance included); the candidates are
        # ordered by (d2, index) and the first k kept.
        kth = np.partition(d2, k - 1, axis=1)[:, k - 1]
        for r in range(b - a):
            cand = np.nonzero(d2[r] <= kth[r])[0]
            order = np.lexsort((cand, d2[r, cand]))
            out[:, a + r] = cand[order[:k]]
    return out


def knn(xq, xs, k, extra=12):
    """Exact stencils for large node sets.

    A k-d tree proposes k+extra candidates per query; the candidates are
    re-ranked with the exact key (d^2, index).  Rows where the proposal might
    have cut a tie at the k-th distance are recomputed by brute force.
    """
    from scipy.spatial import cKDTree

    xq = np.asarray(xq, np.float64)
    xs = np.asarray(xs, np.float64)
    nq = xq.shape[1]
    ns = xs.shape[1]
    if k > ns:
        raise ValueError("k exceeds the number of source nodes")
    kc = min(ns, k + extra)
    if kc == ns:
        return knn_bruteforce(xq, xs, k)
    tree = cKDTree(xs.T)
    _, cand = tree.query(xq.T, k=kc)
    cand = cand.astype(np.int64)
    d2 = _d2(xq[0][:, None], xq[1][:, None], xs[0][cand], xs[1][cand])
    # Sort candidates by (d2, index): lexsort uses the last key as primary.
    order = np.lexsort((cand, d2), axis=1)
    cand = np.take_along_axis(cand, order, axis=1)
    d2 = np.take_along_axis(d2, order, axis=1)
    # Every node with d2 <= d2_k must be among the candidates: require the
    # farthest candidate to be strictly (with margin) beyond the k-th.
    bad = np.nonzero(d2[:, -1] <= d2[:, k - 1] * (1.0 + 1e-9))[0]
    out = cand[:, :k].T.astype(np.int32).copy()
    if bad.size:
        out[:, bad] = knn_bruteforce(xq[:, bad], xs, k)
    return out
