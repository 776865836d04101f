"""GPU (HIP, through the C ABI) against the CPU oracle on identical seeded
inputs.  Bars: stencil indices bit-exact; weights within 1e-12 relative per
row; FP64 fields within 1e-10 relative; ELL products within the rounding
bound of their summation."""
import numpy as np
import pytest

import rbf_inputs as ri
from oracle import knn as oknn, weights as ow, operators as oops, cavity as ocav
from tests.helpers import (OP_ID, OP_DX, OP_DY, OP_LAP, rel_err, row_rel_err, to_dev,
                           gpu_cavity_ops)

pytestmark = pytest.mark.gpu

OPS_ALL = [OP_ID, OP_DX, OP_DY, OP_LAP]


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P(gpu):
    import paper_2206_06495_amd as P
    return P


def _pairs(nd):
    return {"vv": (nd.xv, nd.xv), "pv": (nd.xp, nd.xv), "pp": (nd.xp, nd.xp), "vp": (nd.xv, nd.xp)}


@pytest.mark.parametrize("K,jit,seed", [(40, 0.3, 0), (13, 0.0, 1), (7, 0.25, 2)])
def test_knn_cavity_bit_exact(P, gpu, K, jit, seed):
    _say("knn cavity", K, jit, seed)
    nd = ri.cavity_nodes(K, jit, seed)
    for name, (xq, xs) in _pairs(nd).items():
        idx = P.knn(to_dev(xq, gpu), to_dev(xs, gpu), 28).cpu().numpy()
        ref = oknn.knn_bruteforce(xq, xs, 28)
        assert np.array_equal(idx, ref), name
        if name in ("vv", "pp"):
            assert np.array_equal(idx[0], np.arange(xq.shape[1]))


@pytest.mark.parametrize("jit", [0.0, 0.3])
@pytest.mark.parametrize("k", [1, 5, 28, 33, 64])
def test_knn_square_ties_and_widths(P, gpu, jit, k):
    _say("knn square", jit, k)
    nd = ri.square_nodes(23, jit, 3)
    for xq, xs in ((nd.xv, nd.xv), (nd.xp, nd.xv)):
        idx = P.knn(to_dev(xq, gpu), to_dev(xs, gpu), k).cpu().numpy()
        assert np.array_equal(idx, oknn.knn_bruteforce(xq, xs, k))


def test_knn_degenerate_inputs(P, gpu):
    import torch
    _say("knn degenerate")
    xs = np.array([[0.0, 1.0, 2.0], [0.0, 0.0, 0.0]])  # collinear sources
    xq = np.array([[0.4, 5.0, -3.0], [0.0, 7.0, 0.0]])  # queries outside the box too
    idx = P.knn(to_dev(xq, gpu), to_dev(xs, gpu), 3).cpu().numpy()
    assert np.array_equal(idx, oknn.knn_bruteforce(xq, xs, 3))
    empty = P.knn(torch.zeros((2, 0), dtype=torch.float64, device=gpu), to_dev(xs, gpu), 2)
    assert empty.shape == (2, 0)
    with pytest.raises(P.RbfError):
        P.knn(to_dev(xq, gpu), to_dev(xs, gpu), 4)  # k > ns


def test_knn_rejects_non_finite_coordinates(P, gpu):
    """A NaN or infinite coordinate in the queries or the sources is refused
    with RBF_E_ARG by the host-side check, before any search runs, and the
    output stencils are left untouched."""
    import ctypes
    import torch
    from paper_2206_06495_amd import _lib
    _say("knn non-finite")
    nd = ri.cavity_nodes(6, 0.3, 0)
    for which, bad in (("query", np.nan), ("query", np.inf), ("source", np.nan),
                       ("source", -np.inf)):
        xq, xs = nd.xp.copy(), nd.xv.copy()
        (xq if which == "query" else xs)[1, 3] = bad
        dq, ds = to_dev(xq, gpu), to_dev(xs, gpu)
        idx = torch.full((28, xq.shape[1]), -5, dtype=torch.int32, device=gpu)
        rc = _lib.lib.rbf_knn(ctypes.c_void_p(dq.data_ptr()), xq.shape[1],
                              ctypes.c_void_p(ds.data_ptr()), xs.shape[1], 28,
                              ctypes.c_void_p(idx.data_ptr()), None)
        torch.cuda.synchronize()
        assert rc == _lib.RBF_E_ARG, (which, bad, rc)
        assert "non-finite " + which in _lib.lib.rbf_last_error().decode()
        assert bool((idx == -5).all())


def test_weights_out_of_range_index_reported(P, gpu):
    """A stencil index outside [0, ns) marks its row bad (RBF_E_SINGULAR,
    lowest such row in bad_row, NaN weights) without a load through it;
    other rows keep their weights."""
    import ctypes
    import torch
    from paper_2206_06495_amd import _lib
    _say("weights index range")
    nd = ri.cavity_nodes(6, 0.3, 0)
    d = to_dev(nd.xv, gpu)
    n = nd.n_v
    idx = P.knn(d, d, 28)
    good = P.assemble_weights(d, d, idx, 7, 3, 2).cpu().numpy()
    idx[7, 11] = n            # one past the end
    idx[2, 40] = -1           # negative
    idx[0, 90] = 2 ** 31 - 1  # far out
    w = torch.empty((1, 28, n), dtype=torch.float64, device=gpu)
    c = torch.empty(n, dtype=torch.float64, device=gpu)
    bad = ctypes.c_int64(-7)
    rc = _lib.lib.rbf_assemble_weights(ctypes.c_void_p(d.data_ptr()), n,
                                       ctypes.c_void_p(d.data_ptr()), n,
                                       ctypes.c_void_p(idx.data_ptr()), 28, 7, 3, 2,
                                       ctypes.c_void_p(w.data_ptr()),
                                       ctypes.c_void_p(c.data_ptr()), ctypes.byref(bad), None)
    torch.cuda.synchronize()
    assert rc == _lib.RBF_E_SINGULAR
    assert bad.value == 11
    wh = w.cpu().numpy()[0]
    ch = c.cpu().numpy()
    for r in (11, 40, 90):
        assert np.isnan(wh[:, r]).all() and np.isnan(ch[r])
    keep = np.setdiff1d(np.arange(n), [11, 40, 90])
    assert np.array_equal(wh[:, keep], good[0][:, keep])


@pytest.mark.parametrize("K,seed", [(40, 0), (9, 1)])
def test_weights_cavity_parity(P, gpu, K, seed):
    _say("weights cavity", K, seed)
    nd = ri.cavity_nodes(K, 0.3, seed)
    worst = 0.0
    for name, (xq, xs) in _pairs(nd).items():
        dq, ds = to_dev(xq, gpu), to_dev(xs, gpu)
        idx = P.knn(dq, ds, 28)
        w = P.assemble_weights(dq, ds, idx, 7, 3, 15).cpu().numpy()
        ref = ow.stencil_weights(xq, xs, idx.cpu().numpy(), 7, 3, OPS_ALL)
        for o in range(4):
            e = row_rel_err(w[o], ref[o])
            worst = max(worst, e)
            assert e <= 1e-12, (name, o, e)
    _say("worst weight error", worst)


@pytest.mark.parametrize("kind,K", [("cavity", 12), ("hex", 10), ("square", 16)])
def test_weights_unjittered_sets(P, gpu, kind, K):
    """Node sets without jitter: a local system then holds many equal
    entries, so the elimination meets exactly tied pivot candidates (taken
    by the lowest lane); the weights stay within 1e-12 of the oracle."""
    _say("weights unjittered", kind, K)
    nd = {"cavity": lambda: ri.cavity_nodes(K, 0.0, 0), "hex": lambda: ri.hex_cavity_nodes(K, 0.0, 0),
          "square": lambda: ri.square_nodes(K, 0.0, 0)}[kind]()
    worst = 0.0
    for name, (xq, xs) in _pairs(nd).items():
        dq, ds = to_dev(xq, gpu), to_dev(xs, gpu)
        idx = P.knn(dq, ds, 28)
        w = P.assemble_weights(dq, ds, idx, 7, 3, 15).cpu().numpy()
        ref = ow.stencil_weights(xq, xs, idx.cpu().numpy(), 7, 3, OPS_ALL)
        for o in range(4):
            e = row_rel_err(w[o], ref[o])
            worst = max(worst, e)
            assert e <= 1e-12, (name, o, e)
    _say("worst weight error", worst)


def test_weights_pairing_independent(P, gpu):
    """The paper's stencil is solved two systems per wavefront: a system's
    weights must not depend on which system shares its wavefront, nor on an
    empty second half (odd counts).  Subsets of 1, 2, 3 and 5 queries taken
    at odd offsets reproduce the full assembly's rows bit for bit."""
    nd = ri.hex_cavity_nodes(12, 0.3, 5)
    dq, ds = to_dev(nd.xv, gpu), to_dev(nd.xp, gpu)
    idx = P.knn(dq, ds, 28)
    full = P.assemble_weights(dq, ds, idx, 7, 3, 6).cpu().numpy()
    ref = ow.stencil_weights(nd.xv, nd.xp, idx.cpu().numpy(), 7, 3, [OP_DX, OP_DY])
    for o in range(2):
        assert row_rel_err(full[o], ref[o]) <= 1e-12
    for start, cnt in ((0, 1), (7, 1), (3, 2), (11, 3), (101, 5)):
        sub = P.assemble_weights(dq[:, start:start + cnt].contiguous(), ds,
                                 idx[:, start:start + cnt].contiguous(), 7, 3, 6).cpu().numpy()
        assert np.array_equal(sub, full[:, :, start:start + cnt]), (start, cnt)


@pytest.mark.parametrize("n,m,q,mask", [(28, 7, -1, 15), (12, 3, 1, 15), (20, 5, 2, 7),
                                        (36, 9, 4, 15), (45, 7, 3, 8), (28, 1, 2, 1),
                                        (40, 9, 3, 6), (43, 7, 5, 15)])
def test_weights_parameter_variants(P, gpu, n, m, q, mask):
    _say("weights variant", n, m, q, mask)
    nd = ri.cavity_nodes(11, 0.3, 4)
    xq, xs = nd.xv, nd.xp
    dq, ds = to_dev(xq, gpu), to_dev(xs, gpu)
    idx = P.knn(dq, ds, n)
    force = q >= 0 and n < (q + 1) * (q + 2)
    w = P.assemble_weights(dq, ds, idx, m, q, mask, force=force).cpu().numpy()
    ops = [c for c in OPS_ALL if mask & c]
    ref = ow.stencil_weights(xq, xs, idx.cpu().numpy(), m, q, ops, force=True)
    for o in range(len(ops)):
        assert row_rel_err(w[o], ref[o]) <= 1e-12, (ops[o], row_rel_err(w[o], ref[o]))


@pytest.mark.parametrize("n,m,q", [(28, 7, 3), (12, 3, 1), (40, 7, 4), (28, 7, -1)])
def test_weights_condition_estimate(P, gpu, n, m, q):
    """cond_est (Sec. 4's conditioning of the local systems) against the
    1-norm condition number of the oracle's augmented matrix in the same
    local coordinates, numpy.linalg.cond(A_aug, 1): Hager's estimate is a
    lower bound of ||A^-1||_1, usually exact; the weights do not change when
    the estimate is asked for."""
    _say("weights condition estimate", n, m, q)
    nd = ri.cavity_nodes(12, 0.3, 2)
    xq, xs = nd.xv, nd.xp
    dq, ds = to_dev(xq, gpu), to_dev(xs, gpu)
    idx = P.knn(dq, ds, n)
    force = q >= 0 and n < (q + 1) * (q + 2)
    w0 = P.assemble_weights(dq, ds, idx, m, q, 6, force=force)
    w1, c = P.assemble_weights(dq, ds, idx, m, q, 6, force=force, cond=True)
    assert bool((w0 == w1).all())
    est = c.cpu().numpy()
    xt, yt, _ = ow.local_coordinates(xq, xs, idx.cpu().numpy())
    A, _ = ow.augmented_system(xt, yt, m, q, [ow.OP_DX, ow.OP_DY])
    true = np.linalg.cond(A, 1)
    ratio = est / true
    _say("cond range", true.min(), true.max(), "ratio min/median", ratio.min(), np.median(ratio))
    assert np.all(np.isfinite(est))
    assert ratio.max() <= 1.0 + 1e-3
    assert ratio.min() >= 0.1
    assert np.mean(ratio >= 0.5) >= 0.9


def test_weights_argument_checks(P, gpu):
    nd = ri.cavity_nodes(6, 0.3, 0)
    dq = to_dev(nd.xv, gpu)
    idx = P.knn(dq, dq, 28)
    for m, q, mask in ((6, 3, 15), (7, 6, 15), (1, 3, 2), (7, 3, 0), (7, 4, 15)):
        with pytest.raises(P.RbfError) as ei:
            P.assemble_weights(dq, dq, idx, m, q, mask)
        assert ei.value.status == -1


def test_weights_singular_row_reported(P, gpu):
    import torch
    _say("weights singular")
    nd = ri.cavity_nodes(8, 0.3, 0)
    xs = nd.xv.copy()
    xs[:, 5] = xs[:, 4]  # duplicated node -> singular local systems
    d = to_dev(xs, gpu)
    idx = P.knn(d, d, 28)
    import ctypes
    from paper_2206_06495_amd import _lib
    w = torch.empty((1, 28, xs.shape[1]), dtype=torch.float64, device=gpu)
    bad = ctypes.c_int64(-7)
    rc = _lib.lib.rbf_assemble_weights(ctypes.c_void_p(d.data_ptr()), xs.shape[1],
                                       ctypes.c_void_p(d.data_ptr()), xs.shape[1],
                                       ctypes.c_void_p(idx.data_ptr()), 28, 7, 3, 2,
                                       ctypes.c_void_p(w.data_ptr()), None, ctypes.byref(bad),
                                       None)
    torch.cuda.synchronize()
    assert rc == _lib.RBF_E_SINGULAR
    idxh = idx.cpu().numpy()
    rows_with_both = np.nonzero(np.isin(idxh, [4]).any(0) & np.isin(idxh, [5]).any(0))[0]
    assert bad.value == rows_with_both.min()
    assert np.isnan(w.cpu().numpy()[0][:, bad.value]).all()


def test_weights_bench_square_sampled(P, gpu):
    """Operator-bench size (10^6 + 10^6 nodes): full GPU assembly, oracle on
    sampled rows."""
    _say("weights bench square 1000")
    nd = ri.square_nodes(1000, 0.3, 0)
    rng = np.random.default_rng(5)
    for xq, xs, mask in ((nd.xv, nd.xv, OP_DX | OP_DY | OP_LAP), (nd.xp, nd.xv, OP_ID)):
        dq, ds = to_dev(xq, gpu), to_dev(xs, gpu)
        idx = P.knn(dq, ds, 28)
        w = P.assemble_weights(dq, ds, idx, 7, 3, mask)
        rows = np.sort(np.concatenate([rng.choice(xq.shape[1], 1500, replace=False),
                                       [0, xq.shape[1] - 1]]))
        idx_h = idx.cpu().numpy()
        ref_idx = oknn.knn_bruteforce(xq[:, rows], xs, 28)
        assert np.array_equal(idx_h[:, rows], ref_idx)
        ops = [c for c in OPS_ALL if mask & c]
        ref = ow.stencil_weights(xq[:, rows], xs, ref_idx, 7, 3, ops)
        wh = w.cpu().numpy()
        for o in range(len(ops)):
            assert row_rel_err(wh[o][:, rows], ref[o]) <= 1e-12
        assert np.isfinite(wh).all()


def test_stencils_and_weights_graded_cylinder_nodes(P, gpu):
    """The graded cylinder-in-channel node set of the paper's second workload
    (spacing 0.02 on the cylinder growing to 0.25 at the channel ends;
    132,692 P + 397,066 V nodes): kNN and weights for all four pairs on the
    GPU, checked on 400 sampled rows per pair (the 100 nearest the cylinder,
    the channel edges and random rows) against the oracle: stencils bit for
    bit, weights within 1e-12 per row."""
    _say("graded cylinder nodes: kNN + weights")
    nd = ri.cylinder_nodes()
    rng = np.random.default_rng(11)
    pairs = (("vv", nd.xv, nd.xv, nd.v_tag, OP_DX | OP_DY | OP_LAP),
             ("pv", nd.xp, nd.xv, nd.p_tag, OP_DX | OP_DY),
             ("pp", nd.xp, nd.xp, nd.p_tag, OP_DX | OP_DY | OP_LAP),
             ("vp", nd.xv, nd.xp, nd.v_tag, OP_DX | OP_DY))
    for name, xq, xs, tag, mask in pairs:
        dq, ds = to_dev(xq, gpu), to_dev(xs, gpu)
        idx = P.knn(dq, ds, 28)
        w = P.assemble_weights(dq, ds, idx, 7, 3, mask)
        near = np.argsort(np.hypot(xq[0], xq[1]))[:100]
        edge = np.flatnonzero(tag > 1)
        rows = np.unique(np.concatenate([near, rng.choice(edge, min(100, edge.size), replace=False),
                                         rng.choice(xq.shape[1], 200, replace=False)]))
        ref_idx = oknn.knn_bruteforce(xq[:, rows], xs, 28)
        assert np.array_equal(idx.cpu().numpy()[:, rows], ref_idx), name
        ops = [c for c in OPS_ALL if mask & c]
        ref = ow.stencil_weights(xq[:, rows], xs, ref_idx, 7, 3, ops)
        wh = w.cpu().numpy()
        for o in range(len(ops)):
            assert row_rel_err(wh[o][:, rows], ref[o]) <= 1e-12, (name, o)
        assert np.isfinite(wh).all(), name


def _sum_bound(idx, w, x, u):
    return 2.0 * idx.shape[0] * u * np.sum(np.abs(w * x[idx]), axis=0) + 1e-300


def test_ell_apply_parity(P, gpu):
    import torch
    _say("ell apply")
    nd = ri.cavity_nodes(40, 0.3, 0)
    for n in (28, 17):
        dv = to_dev(nd.xv, gpu)
        idx = P.knn(dv, dv, n)
        w = P.assemble_weights(dv, dv, idx, 7, 3, OP_DX | OP_LAP, force=True)
        x = ri.random_vector(nd.n_v, 11)
        idx_h, w_h = idx.cpu().numpy(), w.cpu().numpy()
        for o in range(2):
            y = P.ell_apply(idx, w[o].contiguous(), to_dev(x, gpu)).cpu().numpy()
            ref = oops.ell_apply(idx_h, w_h[o], x)
            assert np.all(np.abs(y - ref) <= _sum_bound(idx_h, w_h[o], x, 2.0 ** -53))
            # FP32-stored: inputs rounded to FP32 on the GPU, FP32 accumulation.
            w32 = P.cast_f32(w[o].contiguous())
            x32 = P.cast_f32(to_dev(x, gpu))
            y32 = P.ell_apply(idx, w32, x32).cpu().numpy().astype(np.float64)
            w32h = w32.cpu().numpy().astype(np.float64)
            x32h = x32.cpu().numpy().astype(np.float64)
            assert np.array_equal(w32h, w_h[o].astype(np.float32).astype(np.float64))
            ref32 = oops.ell_apply(idx_h, w32h, x32h)
            assert np.all(np.abs(y32 - ref32) <= _sum_bound(idx_h, w32h, x32h, 2.0 ** -24))
    # Ragged tail and one-row operators.
    idx = torch.zeros((28, 1), dtype=torch.int32, device=gpu)
    w = torch.ones((28, 1), dtype=torch.float64, device=gpu)
    y = P.ell_apply(idx, w, torch.full((1,), 0.5, dtype=torch.float64, device=gpu))
    assert float(y.cpu()[0]) == 14.0


def _transpose_ref(idx, ncols):
    """Column structure of D^T by definition: entries (s, r) grouped by
    column idx[s, r], ordered by (r, s) inside a column."""
    k, rows = idx.shape
    s_, r_ = np.meshgrid(np.arange(k), np.arange(rows), indexing="ij")
    c, r, s = idx.ravel(), r_.ravel(), s_.ravel()
    order = np.lexsort((s, r, c))
    colptr = np.concatenate([[0], np.cumsum(np.bincount(c, minlength=ncols))])
    return colptr, r[order], s[order]


def _t_bound(idx, w, y, ncols, u):
    lens = np.bincount(idx.ravel(), minlength=ncols)
    mag = np.zeros(ncols)
    np.add.at(mag, idx.ravel(), np.abs(w * y[None, :]).ravel())
    return 2.0 * np.maximum(lens, 1) * u * mag + 1e-300


def test_ell_autotune(P, gpu):
    """rbf_ell_autotune times the 16 launch shapes of the 28-wide product,
    records the fastest, and ell_apply then uses it: results bit-identical
    to the default shape (same per-row summation order) in FP64 and FP32;
    other widths keep the default shape."""
    import torch
    _say("ell autotune")
    nd = ri.square_nodes(200, 0.3, 1)
    xv = to_dev(nd.xv, gpu)
    idx = P.knn(xv, xv, 28)
    w = P.assemble_weights(xv, xv, idx, 7, 3, 2)[0].contiguous()
    x = to_dev(ri.random_vector(nd.xv.shape[1], 3), gpu)
    for ww, xx in ((w, x), (P.cast_f32(w), P.cast_f32(x))):
        y0 = P.ell_apply(idx, ww, xx)
        shape, ms = P.ell_autotune(idx, ww, xx, reps=5)
        assert len(ms) == 16 and all(t > 0.0 for t in ms), ms
        assert shape == int(np.argmin(ms)), (shape, ms)
        y1 = P.ell_apply(idx, ww, xx)
        torch.cuda.synchronize()
        assert bool((y0 == y1).all())
        _say("dtype", ww.dtype, "shape", shape, P.ELL_SHAPES[shape], "ms", min(ms), "default", ms[0])
    i17 = idx[:17].contiguous()
    shape, ms = P.ell_autotune(i17, w[:17].contiguous(), x, reps=2)
    assert shape == 0 and ms[0] == 0.0 and all(t == -1.0 for t in ms[1:])


def test_ell_transpose_parity(P, gpu):
    """z = D^T y (the transposed product of the adjoint): the column
    structure and the column-ordered weights equal their definitions
    exactly; FP64 and FP32 products agree
    with the oracle within the rounding bound of each column's sum and are
    bit-identical on repetition; rectangular PV (M x N) and square VV
    operators, k = 28 and 17, with columns no row references."""
    import torch
    _say("ell transpose")
    nd = ri.cavity_nodes(40, 0.3, 0)
    xv, xp = to_dev(nd.xv, gpu), to_dev(nd.xp, gpu)
    for xq, xs, k in ((xp, xv, 28), (xv, xv, 17)):
        idx = P.knn(xq, xs, k)
        w = P.assemble_weights(xq, xs, idx, 7, 3, OP_DX | OP_DY, force=True)
        rows, ncols = xq.shape[1], xs.shape[1] + 3
        T = P.ell_transpose(idx, ncols)
        idx_h, w_h = idx.cpu().numpy(), w.cpu().numpy()
        colptr, src, slot = _transpose_ref(idx_h, ncols)
        assert np.array_equal(T.colptr.cpu().numpy(), colptr)
        assert np.array_equal(T.src.cpu().numpy(), src)
        assert np.array_equal(T.slot.cpu().numpy(), slot)
        y = ri.random_vector(rows, 21)
        for o in range(2):
            wt = T.weights(w[o].contiguous())
            perm = np.asarray(T.src.cpu().numpy(), np.int64) + rows * T.slot.cpu().numpy()
            assert np.array_equal(wt.cpu().numpy(), w_h[o].ravel()[perm])
            z = T.apply(wt, to_dev(y, gpu))
            ref = oops.ell_apply_transpose(idx_h, w_h[o], y, ncols)
            zh = z.cpu().numpy()
            assert np.all(np.abs(zh - ref) <= _t_bound(idx_h, w_h[o], y, ncols, 2.0 ** -53))
            assert np.all(zh[ncols - 3:] == 0.0)
            assert torch.equal(z, T.apply(wt, to_dev(y, gpu)))
            w32 = P.cast_f32(w[o].contiguous())
            y32 = P.cast_f32(to_dev(y, gpu))
            z32 = T.apply(T.weights(w32), y32).cpu().numpy().astype(np.float64)
            w32h = w32.cpu().numpy().astype(np.float64)
            y32h = y32.cpu().numpy().astype(np.float64)
            ref32 = oops.ell_apply_transpose(idx_h, w32h, y32h, ncols)
            assert np.all(np.abs(z32 - ref32) <= _t_bound(idx_h, w32h, y32h, ncols, 2.0 ** -24))


def test_ell_transpose_edge_cases(P, gpu):
    """No rows: every column empty and z = 0.  An index outside
    [0, ncols) is reported with the lowest offending ELL position; a column
    with more than 4096 entries is rejected before any entry is placed."""
    import torch
    _say("ell transpose edge cases")
    T = P.ell_transpose(torch.zeros((28, 0), dtype=torch.int32, device=gpu), 4)
    assert T.colptr.cpu().tolist() == [0] * 5
    z = T.apply(T.weights(torch.zeros((28, 0), dtype=torch.float64, device=gpu)),
                torch.zeros(0, dtype=torch.float64, device=gpu))
    assert z.cpu().tolist() == [0.0] * 4
    idx = torch.zeros((28, 10), dtype=torch.int32)
    idx[3, 7] = 6
    idx[5, 2] = -1
    with pytest.raises(P.RbfError) as ei:
        P.ell_transpose(idx.to(gpu), 6)
    assert ei.value.status == -1 and "entry 37" in str(ei.value)
    with pytest.raises(P.RbfError) as ei:
        P.ell_transpose(torch.zeros((28, 200), dtype=torch.int32, device=gpu), 3)
    assert ei.value.status == -1 and "5600 entries" in str(ei.value)


def _gpu_solver(P, nd, gpu, re, dt, **kw):
    grid, ops = gpu_cavity_ops(nd, gpu)
    u_bc, v_bc = ri.cavity_bc(nd.v_tag)
    S = P.Solver(grid, ops, to_dev(u_bc, gpu), to_dev(v_bc, gpu), re, dt, **kw)
    return S, ops, u_bc, v_bc


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cavity_parity_small_workload(P, gpu, precision):
    """K=40 cavity (N=4880, M=1681), Re=100, dt=2e-3, 200 steps: GPU BiCGSTAB
    against the oracle's LU, u, v, p within 1e-10 every 20 steps (mixed: FP32
    preconditioner transforms, FP64 residuals, same bar)."""
    _say("cavity parity K=40", precision)
    nd = ri.cavity_nodes(40, 0.3, 0)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 100.0, 2e-3, precision=precision)
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 100.0, 2e-3)
    s0 = orc.initial_state()
    st = S.new_state(to_dev(s0.u, gpu), to_dev(s0.v, gpu))
    so = s0
    worst = 0.0
    for chunk in range(10):
        stats = S.step(st, 20)
        so = orc.run(20, so)
        for key, ref in (("u", so.u), ("v", so.v), ("p", so.p), ("p_tilde", so.pt)):
            e = rel_err(st[key].cpu().numpy(), ref)
            worst = max(worst, e)
            assert e <= 1e-10, (chunk, key, e)
        assert stats.steps_done == 20
        assert stats.last_poisson.converged and stats.last_poisson.rel_residual < 1e-11
    assert st["step"] == 200
    _say("cavity worst rel err", worst, "poisson iters/step", stats.poisson_iters / 20)
    S.close()


def test_cavity_parity_jacobi_viscous_solve(P, gpu):
    """K=40 cavity at the bench's Re=1e4 and dt=2e-4 (a = 1e-8): the Jacobi
    iteration matrix of H has a small infinity norm, so the viscous solve
    runs Jacobi sweeps; 40 steps against the oracle's LU within 1e-10.  At
    Re=100, dt=2e-3 (a = 1e-5) the same grid keeps BiCGSTAB."""
    _say("cavity parity K=40 Jacobi viscous solve")
    nd = ri.cavity_nodes(40, 0.3, 0)
    # Viscous tolerance 1e-13 (the binding's default): at dt = 2e-4 an error
    # in u** reaches p~ multiplied by 1/dt through F/dt.
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 1e4, 2e-4)
    info = S.info()
    _say("solver info", info)
    assert info["viscous_jacobi"] and info["jacobi_bound"] <= 0.25 and info["lattice_precond"]
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 1e4, 2e-4)
    s0 = orc.initial_state()
    st = S.new_state(to_dev(s0.u, gpu), to_dev(s0.v, gpu))
    so = s0
    for chunk in range(2):
        stats = S.step(st, 20)
        so = orc.run(20, so)
        assert stats.last_helmholtz_u.converged and stats.last_helmholtz_u.rel_residual <= 1e-12
        for key, ref in (("u", so.u), ("v", so.v), ("p", so.p), ("p_tilde", so.pt)):
            assert rel_err(st[key].cpu().numpy(), ref) <= 1e-10, (chunk, key)
    S.close()
    S2, _, _, _ = _gpu_solver(P, nd, gpu, 100.0, 2e-3)
    info2 = S2.info()
    _say("solver info at Re=100, dt=2e-3", info2)
    assert not info2["viscous_jacobi"] and info2["jacobi_bound"] > 0.25
    S2.close()
    # One sweep allowed: the sweeps stop with RBF_E_NOCONV and the failed
    # step is not committed.
    S3, _, _, _ = _gpu_solver(P, nd, gpu, 1e4, 2e-4, maxit_h=1)
    st3 = S3.new_state(to_dev(s0.u, gpu), to_dev(s0.v, gpu))
    with pytest.raises(P.RbfError) as ei:
        S3.step(st3, 3)
    assert ei.value.status == -3 and "Jacobi" in str(ei.value)
    assert st3["step"] < 3
    S3.close()


@pytest.mark.parametrize("precond", ["none", "lattice"])
def test_solve_pressure_parity(P, gpu, precond):
    _say("solve_pressure", precond)
    nd = ri.cavity_nodes(24, 0.3, 1)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 100.0, 1e-3, precond=precond)
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 100.0, 1e-3)
    rhs = ri.random_vector(nd.n_p, 3)
    rhs[nd.p_tag != 0] = 0.0
    x = to_dev(np.zeros(nd.n_p), gpu)
    stats = S.solve_pressure(to_dev(rhs, gpu), x)
    ref, _ = orc.solve_pressure(rhs)
    assert stats.converged and stats.rel_residual <= 1e-10
    assert rel_err(x.cpu().numpy(), ref) <= 1e-10
    S.close()


def test_lattice_preconditioner_cuts_iterations(P, gpu):
    """K=64 cavity pressure solve from a zero guess: both variants reach the
    oracle's bordered solution; the lattice preconditioner needs at most a
    fifth of the unpreconditioned iterations."""
    _say("lattice preconditioner K=64")
    nd = ri.cavity_nodes(64, 0.3, 2)
    grid, ops = gpu_cavity_ops(nd, gpu)
    u_bc, v_bc = ri.cavity_bc(nd.v_tag)
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 100.0, 1e-3)
    rhs = ri.random_vector(nd.n_p, 5)
    rhs[nd.p_tag != 0] = 0.0
    ref, _ = orc.solve_pressure(rhs)
    its = {}
    for precond in ("none", "lattice"):
        S = P.Solver(grid, ops, to_dev(u_bc, gpu), to_dev(v_bc, gpu), 100.0, 1e-3,
                     rtol_p=1e-12, precond=precond)
        x = to_dev(np.zeros(nd.n_p), gpu)
        stats = S.solve_pressure(to_dev(rhs, gpu), x)
        assert stats.converged and stats.rel_residual <= 1e-11, precond
        assert rel_err(x.cpu().numpy(), ref) <= 1e-9, precond
        its[precond] = stats.iterations
        S.close()
    _say("iterations", its)
    assert its["lattice"] * 5 <= its["none"], its


def _lattice_precond_reference(nd, ops, y):
    """Plain numpy statement of the lattice preconditioner (header of
    rbf_params.precond): z = J (L5 + chi c 1^T)^-1 D^-1 y, with L5 solved by
    sparse LU on the full lattice, bordered (no transforms, no wall
    elimination)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    K = nd.K
    n1 = K + 1
    M = n1 * n1
    h = 1.0 / K
    # D: signed inverse row norms of the stored Poisson rows.
    wall = nd.p_tag != 0
    lap = ops["pp_lap"].cpu().numpy()
    dx = ops["pp_dx"].cpu().numpy()
    dy = ops["pp_dy"].cpu().numpy()
    rows = np.where(wall[None, :], nd.p_normal[0][None, :] * dx + nd.p_normal[1][None, :] * dy, lap)
    rs = np.where(wall, 1.0, -1.0) / np.sqrt((rows * rows).sum(axis=0))
    u1 = np.where(wall, 0.0, rs)
    c = ((~wall).sum() / np.abs(u1).sum()) / M
    # L5 with one-sided Neumann rows, bordered by chi c 1^T.
    r_, c_, v_ = [], [], []
    for j in range(n1):
        for i in range(n1):
            r = j * n1 + i
            if 0 < i < K and 0 < j < K:
                r_ += [r] * 5
                c_ += [r, r - 1, r + 1, r - n1, r + n1]
                v_ += [-4 / h**2] + [1 / h**2] * 4
            else:
                di = 1 if i == 0 else (-1 if i == K else 0)
                dj = 1 if j == 0 else (-1 if j == K else 0)
                d = h * np.hypot(di, dj)
                r_ += [r, r]
                c_ += [r, (j + dj) * n1 + i + di]
                v_ += [1 / d, -1 / d]
    # (L5 + c chi 1^T) zl = y / rs as the sparse bordered system
    # [L5 chi; c 1^T -1] [zl; mu] = [y / rs; 0].
    L5 = sp.csr_matrix((v_, (r_, c_)), shape=(M, M))
    Bd = sp.bmat([[L5, sp.csr_matrix((~wall).astype(float)[:, None])],
                  [sp.csr_matrix(np.full((1, M), c)), sp.csr_matrix([[-1.0]])]], format="csc")
    zl = spla.spsolve(Bd, np.concatenate([y / rs, [0.0]]))[:M]
    # J: bilinear interpolation from the lattice points to the nodes.
    sx, sy = nd.xp[0] * K, nd.xp[1] * K
    i0 = np.clip(np.floor(sx).astype(int), 0, K - 1)
    j0 = np.clip(np.floor(sy).astype(int), 0, K - 1)
    fx, fy = sx - i0, sy - j0
    z = lambda i, j: zl[j * n1 + i]  # noqa: E731
    return ((1 - fy) * ((1 - fx) * z(i0, j0) + fx * z(i0 + 1, j0))
            + fy * ((1 - fx) * z(i0, j0 + 1) + fx * z(i0 + 1, j0 + 1)))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-5)])
@pytest.mark.parametrize("K", [12, 23, 40, 150, 300])
def test_lattice_preconditioner_matches_its_definition(P, gpu, K, precision, tol):
    """One application of P^-1 through the C ABI against its plain statement
    (K=23: interior size 22, a ragged 16x16 tiling; K=150 and K=300: 64
    chunks of 2-3 and of 4-5 rows per lane in the tridiagonal stage).  Mixed
    precision runs the transforms in FP32: the bound is a few hundred FP32
    roundings.  Both bars grow with the condition number of the lattice
    Poisson solve, about 0.4 K^2: 4e-16 K^2 (FP64) and 2e-5 (K/40)^2 (FP32)
    beyond K = 50 and K = 40."""
    _say("apply_precond K=", K, precision)
    nd = ri.cavity_nodes(K, 0.3, 4)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 100.0, 1e-3, precond="lattice",
                                     precision=precision)
    y = ri.random_vector(nd.n_p, 11)
    z = S.apply_precond(to_dev(y, gpu)).cpu().numpy()
    ref = _lattice_precond_reference(nd, ops, y)
    tol = max(tol, 4e-16 * K * K) if precision == "fp64" else tol * max(1.0, (K / 40) ** 2)
    assert rel_err(z, ref) <= tol
    S.close()


def test_lattice_preconditioner_needs_a_lattice(P, gpu):
    """A P-node moved out of its lattice cell: 'lattice' is refused with
    RBF_E_ARG, 'auto' falls back to the auxiliary-lattice preconditioner
    (the nodes still fill a square)."""
    _say("lattice detection")
    nd = ri.cavity_nodes(12, 0.3, 0)
    v = 5 * 13 + 6
    assert nd.p_tag[v] == 0
    nd.xp[0, v] = (6 + 0.7) * nd.h  # vertex (6, 5), now outside its lattice cell
    grid, ops = gpu_cavity_ops(nd, gpu)
    u_bc, v_bc = ri.cavity_bc(nd.v_tag)
    with pytest.raises(P.RbfError) as ei:
        P.Solver(grid, ops, to_dev(u_bc, gpu), to_dev(v_bc, gpu), 100.0, 1e-3, precond="lattice")
    assert ei.value.status == -1
    S = P.Solver(grid, ops, to_dev(u_bc, gpu), to_dev(v_bc, gpu), 100.0, 1e-3, precond="auto")
    assert not S.info()["lattice_precond"] and S.info()["aux_precond"]
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 100.0, 1e-3)
    rhs = ri.random_vector(nd.n_p, 7)
    rhs[nd.p_tag != 0] = 0.0
    x = to_dev(np.zeros(nd.n_p), gpu)
    stats = S.solve_pressure(to_dev(rhs, gpu), x)
    ref, _ = orc.solve_pressure(rhs)
    assert stats.converged and rel_err(x.cpu().numpy(), ref) <= 1e-10
    S.close()


@pytest.mark.parametrize("n", [24, 32])
def test_cavity_parity_other_stencil_sizes(P, gpu, n):
    """Stencils of n = 24 and 32 nodes (the generic-width kernels of every
    stage and of both pressure variants): K=16 cavity, 20 steps at Re=100,
    u, v, p, p~ within 1e-10 of the oracle built with the same n."""
    _say("cavity parity K=16, n =", n)
    nd = ri.cavity_nodes(16, 0.3, 3)
    grid, ops = gpu_cavity_ops(nd, gpu, n=n)
    u_bc, v_bc = ri.cavity_bc(nd.v_tag)
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 100.0, 2e-3, n=n)
    so = orc.run(20, orc.initial_state())
    for precond in ("lattice", "none"):
        S = P.Solver(grid, ops, to_dev(u_bc, gpu), to_dev(v_bc, gpu), 100.0, 2e-3, precond=precond)
        st = S.new_state(to_dev(np.where(nd.v_tag != 0, u_bc, 0.0), gpu), to_dev(v_bc, gpu))
        S.step(st, 20)
        for key, ref in (("u", so.u), ("v", so.v), ("p", so.p), ("p_tilde", so.pt)):
            assert rel_err(st[key].cpu().numpy(), ref) <= 1e-10, (precond, key)
        S.close()


def test_cavity_parity_unpreconditioned(P, gpu):
    """The unpreconditioned pressure iteration on the K=24 cavity, 40 steps."""
    _say("cavity parity K=24, precond none")
    nd = ri.cavity_nodes(24, 0.3, 1)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 100.0, 2e-3, precond="none")
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 100.0, 2e-3)
    s0 = orc.initial_state()
    st = S.new_state(to_dev(s0.u, gpu), to_dev(s0.v, gpu))
    S.step(st, 40)
    so = orc.run(40, s0)
    for key, ref in (("u", so.u), ("v", so.v), ("p", so.p), ("p_tilde", so.pt)):
        assert rel_err(st[key].cpu().numpy(), ref) <= 1e-10, key
    S.close()


def test_cavity_parity_near_equilateral_nodes(P, gpu):
    """A cavity on the jittered near-equilateral triangulation (node kind 2;
    not a lattice, so the pressure iteration runs FGMRES with the
    auxiliary-lattice preconditioner): 60 steps at Re = 1e3, dt = 1e-3, u, v,
    p, p~ within 1e-10 of the oracle."""
    _say("cavity parity, near-equilateral nodes K=20")
    nd = ri.hex_cavity_nodes(20, 0.3, 0)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 1000.0, 1e-3)
    assert not S.info()["lattice_precond"] and S.info()["aux_precond"]
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 1000.0, 1e-3)
    s0 = orc.initial_state()
    st = S.new_state(to_dev(s0.u, gpu), to_dev(s0.v, gpu))
    for _ in range(3):
        S.step(st, 20)
        s0 = orc.run(20, s0)
        for key, ref in (("u", s0.u), ("v", s0.v), ("p", s0.p), ("p_tilde", s0.pt)):
            assert rel_err(st[key].cpu().numpy(), ref) <= 1e-10, (st["step"], key)
    S.close()


def test_long_run_on_near_equilateral_nodes(P, gpu):
    """400 steps at the bench's Re = 1e4 and dt = 2e-4 on the jittered
    near-equilateral K = 60 triangulation (stable there, unlike the
    right-triangle lattice):
    the fields follow the oracle every 100 steps and the run stays bounded
    (maximum speed, CFL and interior divergence from rbf_solver_diagnostics).
    With the default pressure tolerance 1e-12 p drifts to 1.03e-10 by step
    200; at 1e-13 the fields stay well inside the bar."""
    _say("long run, near-equilateral nodes K=60")
    nd = ri.hex_cavity_nodes(60, 0.3, 0)
    # At dt = 2e-4 an error in u** reaches p~ multiplied by 1/dt: the
    # pressure tolerance is one decade below the binding's default.
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 1e4, 2e-4, rtol_p=1e-13)
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 1e4, 2e-4)
    s0 = orc.initial_state()
    st = S.new_state(to_dev(s0.u, gpu), to_dev(s0.v, gpu))
    for _ in range(4):
        S.step(st, 100)
        s0 = orc.run(100, s0)
        errs = {key: rel_err(st[key].cpu().numpy(), ref)
                for key, ref in (("u", s0.u), ("v", s0.v), ("p", s0.p), ("p_tilde", s0.pt))}
        d = S.diagnostics(st)
        _say(st["step"], errs, d)
        assert all(e <= 1e-10 for e in errs.values()), (st["step"], errs)
        assert d["speed_max"] < 1.05 and d["cfl"] < 0.1 and d["div_max"] < 0.01, d
    S.close()


def test_step_error_paths_are_transactional(P, gpu):
    import torch
    _say("error paths")
    nd = ri.cavity_nodes(12, 0.3, 0)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 100.0, 2e-3, maxit_p=1)
    st = S.new_state(to_dev(np.where(nd.v_tag != 0, u_bc, 0.0), gpu), to_dev(v_bc, gpu))
    before = {k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in st.items()}
    with pytest.raises(P.RbfError) as ei:
        S.step(st, 3)
    assert ei.value.status == -3  # RBF_E_NOCONV
    for k, v in before.items():
        if isinstance(v, torch.Tensor):
            assert torch.equal(v, st[k]), k
    assert st["step"] == 0
    S.close()
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 100.0, 2e-3)
    u0 = np.where(nd.v_tag != 0, u_bc, 0.0)
    u0[np.nonzero(nd.v_tag == 0)[0][3]] = np.nan
    st = S.new_state(to_dev(u0, gpu), to_dev(v_bc, gpu))
    with pytest.raises(P.RbfError) as ei:
        S.step(st, 1)
    assert ei.value.status == -6  # RBF_E_NAN
    assert st["step"] == 0
    S.close()


def test_solver_create_rejects_out_of_range_stencils(P, gpu):
    """A stencil index outside its source node range (one too large in VP,
    negative in PV) is refused by rbf_solver_create with RBF_E_ARG naming the
    array, slot and row, before any kernel gathers through it."""
    _say("stencil range check")
    nd = ri.cavity_nodes(8, 0.3, 0)
    grid, ops = gpu_cavity_ops(nd, gpu)
    u_bc, v_bc = ri.cavity_bc(nd.v_tag)
    for name, slot, row, val in (("idx_vp", 5, 7, nd.n_p), ("idx_pv", 27, 0, -1)):
        bad = dict(ops)
        bad[name] = ops[name].clone()
        bad[name][slot, row] = val
        with pytest.raises(P.RbfError) as ei:
            P.Solver(grid, bad, to_dev(u_bc, gpu), to_dev(v_bc, gpu), 100.0, 2e-3)
        assert ei.value.status == -1
        assert f"{name}[{slot}][{row}] = {val}" in str(ei.value), str(ei.value)
    S = P.Solver(grid, ops, to_dev(u_bc, gpu), to_dev(v_bc, gpu), 100.0, 2e-3)
    S.close()


def test_solver_diagnostics(P, gpu):
    """rbf_solver_diagnostics after 10 steps of the K=24 cavity against
    their definitions evaluated on the downloaded fields: divergence of
    eq. (17) on interior P rows (within its summation bound), kinetic
    energy, maximum speed and CFL number (nearest stencil neighbour
    distance) to rounding; repeatable bit for bit; a NaN shows as NaN."""
    import torch
    _say("diagnostics K=24")
    nd = ri.cavity_nodes(24, 0.3, 1)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 100.0, 2e-3)
    st = S.new_state(to_dev(np.where(nd.v_tag != 0, u_bc, 0.0), gpu), to_dev(v_bc, gpu))
    S.step(st, 10)
    d = S.diagnostics(st)
    assert d == S.diagnostics(st)
    u, v = st["u"].cpu().numpy(), st["v"].cpu().numpy()
    idx = ops["idx_pv"].cpu().numpy()
    wx, wy = ops["pv_dx"].cpu().numpy(), ops["pv_dy"].cpu().numpy()
    F = oops.ell_apply(idx, wx, u) + oops.ell_apply(idx, wy, v)
    bound = 4.0 * 28 * 2.0 ** -53 * (np.abs(wx * u[idx]) + np.abs(wy * v[idx])).sum(axis=0)
    inner = nd.p_tag == 0
    assert abs(d["div_max"] - np.max(np.abs(F[inner]))) <= np.max(bound[inner])
    assert abs(d["div_rms"] - np.sqrt(np.mean(F[inner] ** 2))) <= np.max(bound[inner])
    sp = np.sqrt(u * u + v * v)
    assert abs(d["kinetic_energy"] - 0.5 * np.mean(u * u + v * v)) <= 1e-14 * d["kinetic_energy"]
    assert abs(d["speed_max"] - np.max(sp)) <= 4e-16 * np.max(sp)
    iv = ops["idx_vv"].cpu().numpy()
    dx = nd.xv[0][iv] - nd.xv[0][None, :]
    dy = nd.xv[1][iv] - nd.xv[1][None, :]
    d2 = np.where(iv == np.arange(nd.n_v)[None, :], np.inf, dx * dx + dy * dy)
    cfl = 2e-3 * np.max(sp / np.sqrt(d2.min(axis=0)))
    assert abs(d["cfl"] - cfl) <= 1e-14 * cfl
    bad = dict(st)
    bad["u"] = st["u"].clone()
    bad["u"][5] = float("nan")
    dn = S.diagnostics(bad)
    assert np.isnan(dn["speed_max"]) and np.isnan(dn["cfl"]) and np.isnan(dn["kinetic_energy"])
    S.close()


def test_run_writes_jsonl_records(P, gpu):
    """Solver.run: one JSON line per rbf_step call with the step, Krylov
    statistics and diagnostics; the state equals the one from plain calls of
    the same chunk size (bit for bit)."""
    import io
    import json
    import torch
    _say("run / JSONL log")
    nd = ri.cavity_nodes(12, 0.3, 0)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 100.0, 2e-3)
    u0 = to_dev(np.where(nd.v_tag != 0, u_bc, 0.0), gpu)
    st = S.new_state(u0, to_dev(v_bc, gpu))
    ref = S.new_state(u0, to_dev(v_bc, gpu))
    buf = io.StringIO()
    recs = S.run(st, 25, every=10, log=buf)
    lines = [json.loads(x) for x in buf.getvalue().splitlines()]
    assert lines == recs and [r["step"] for r in recs] == [10, 20, 25]
    for r in recs:
        assert r["poisson_rel_residual"] <= 1e-12 and r["cfl"] > 0 and r["speed_max"] >= 1.0
        assert set(r) >= {"div_max", "div_rms", "kinetic_energy", "poisson_iters_per_step"}
    for k in (10, 10, 5):
        S.step(ref, k)
    for key in ("u", "v", "p", "p_tilde", "cu_prev", "cv_prev"):
        assert torch.equal(st[key], ref[key]), key
    S.close()


def test_checkpoint_resume_is_bitwise(P, gpu):
    """(u, v, p~, p, C_{j-1}(u), C_{j-1}(v), j) is the whole carried state of
    the scheme (AB2, eq. (14), needs the previous advection terms): saved
    with torch.save after 6 steps and loaded (weights_only) for a new solver
    built from the same operators, 6 more steps give fields bit-identical to
    6 + 6 steps on the first solver.  The Krylov initial guesses are rebuilt
    within each rbf_step call, the launch plan only decides how many
    iterations are queued, and every reduction runs in a fixed order."""
    import io
    import torch
    _say("checkpoint / resume K=24")
    nd = ri.cavity_nodes(24, 0.3, 2)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, 400.0, 2e-3)
    st = S.new_state(to_dev(np.where(nd.v_tag != 0, u_bc, 0.0), gpu), to_dev(v_bc, gpu))
    S.step(st, 6)
    buf = io.BytesIO()
    torch.save(st, buf)
    S.step(st, 6)
    grid2, ops2 = gpu_cavity_ops(nd, gpu)
    S2 = P.Solver(grid2, ops2, to_dev(u_bc, gpu), to_dev(v_bc, gpu), 400.0, 2e-3)
    buf.seek(0)
    st2 = torch.load(buf, weights_only=True, map_location=gpu)
    assert st2["step"] == 6
    S2.step(st2, 6)
    assert st2["step"] == st["step"] == 12
    for key in ("u", "v", "p", "p_tilde", "cu_prev", "cv_prev"):
        assert torch.equal(st[key], st2[key]), key
    S.close()
    S2.close()


def _sampled_stencils(xq, xs, rows, ops):
    """Oracle kNN + weights for the listed evaluation rows only."""
    idx = oknn.knn_bruteforce(xq[:, rows], xs, 28)
    return idx, ow.stencil_weights(xq[:, rows], xs, idx, 7, 3, ops)


def test_cavity_full_size_sampled(P, gpu):
    """The bench workload (K=400: N=480,800, M=160,801; Re=1e4, dt=2e-4,
    tolerances 1e-12), three GPU steps, the third checked on sampled rows
    with oracle stencils and weights computed for those rows only:
    advection C_j(u_j) (eq. (15)) and the pressure update (eq. (19)) to
    1e-10; the viscous solve (eq. (16)) through its residual at sampled rows,
    u** rebuilt from u_{j+1} and p~_{j+1} (eq. (20)); the bordered Poisson
    solve (eq. (18)) through its residual, which on interior rows must be the
    one constant -lam and on wall rows the Neumann value 0."""
    import torch
    _say("cavity full size sampled K=400")
    K, re, dt = 400, 1e4, 2e-4
    a = dt / (2.0 * re)
    nd = ri.cavity_nodes(K, 0.3, 0)
    S, ops, u_bc, v_bc = _gpu_solver(P, nd, gpu, re, dt, rtol_h=1e-12, rtol_p=1e-12)
    del ops
    st = S.new_state(to_dev(np.where(nd.v_tag != 0, u_bc, 0.0), gpu),
                     to_dev(np.where(nd.v_tag != 0, v_bc, 0.0), gpu))
    S.step(st, 2)
    before = {k: st[k].cpu().numpy().copy() for k in ("u", "v", "p_tilde", "cu_prev", "cv_prev")}
    stats = S.step(st, 1)
    after = {k: st[k].cpu().numpy() for k in ("u", "v", "p_tilde", "p", "cu_prev", "cv_prev")}
    S.close()
    torch.cuda.empty_cache()
    assert stats.last_poisson.converged and stats.last_helmholtz_u.converged
    xv, xp = nd.xv, nd.xp
    vwall, pwall = nd.v_tag != 0, nd.p_tag != 0
    rng = np.random.default_rng(7)
    rv = np.unique(np.concatenate([rng.choice(np.nonzero(~vwall)[0], 24, replace=False),
                                   rng.choice(np.nonzero(vwall)[0], 8, replace=False)]))
    rp = np.unique(np.concatenate([rng.choice(np.nonzero(~pwall)[0], 24, replace=False),
                                   rng.choice(np.nonzero(pwall)[0], 8, replace=False)]))
    uj, vj, ptj = before["u"], before["v"], before["p_tilde"]
    un, vn, ptn = after["u"], after["v"], after["p_tilde"]

    def advect(rows):
        idx, (wx, wy) = _sampled_stencils(xv, xv, rows, (OP_DX, OP_DY))
        dxu, dyu = (wx * uj[idx]).sum(0), (wy * uj[idx]).sum(0)
        dxv, dyv = (wx * vj[idx]).sum(0), (wy * vj[idx]).sum(0)
        return -(uj[rows] * dxu + vj[rows] * dyu), -(uj[rows] * dxv + vj[rows] * dyv)

    # Stage 1 at the sampled rows: C_j(u_j), C_j(v_j) are the new cu_prev, cv_prev.
    cu_r, cv_r = advect(rv)
    for got, ref in ((after["cu_prev"][rv], cu_r), (after["cv_prev"][rv], cv_r)):
        assert np.max(np.abs(got - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))

    # u** = u_{j+1} + dt D_x^VP p~_{j+1} at the given V rows.
    def ustar2(rows):
        idx, (wx, wy) = _sampled_stencils(xv, xp, rows, (OP_DX, OP_DY))
        return un[rows] + dt * (wx * ptn[idx]).sum(0), vn[rows] + dt * (wy * ptn[idx]).sum(0)

    # Stage 2: H u** = ru on the sampled V rows.
    idx_l, (wl,) = _sampled_stencils(xv, xv, rv, (OP_LAP,))
    nb = np.unique(idx_l)
    pos = {r: i for i, r in enumerate(nb)}
    cu_n, cv_n = advect(nb)
    us_n = uj[nb] + dt * (1.5 * cu_n - 0.5 * before["cu_prev"][nb])
    vs_n = vj[nb] + dt * (1.5 * cv_n - 0.5 * before["cv_prev"][nb])
    uss_n, vss_n = ustar2(nb)
    loc = np.vectorize(pos.get)(idx_l)
    self_ = np.array([pos[r] for r in rv])
    idx_w, (wxw, wyw) = _sampled_stencils(xv, xp, rv, (OP_DX, OP_DY))
    for comp, (s_n, x_n, bc, ww) in enumerate(((us_n, uss_n, u_bc, wxw), (vs_n, vss_n, v_bc, wyw))):
        rhs = np.where(vwall[rv], bc[rv] + dt * (ww * ptj[idx_w]).sum(0),
                       s_n[self_] + a * (wl * s_n[loc]).sum(0))
        hx = np.where(vwall[rv], x_n[self_], x_n[self_] - a * (wl * x_n[loc]).sum(0))
        assert np.max(np.abs(hx - rhs)) <= 1e-9 * max(1.0, np.max(np.abs(rhs))), comp

    # Stage 3: F = D_x^PV u** + D_y^PV v**, D_Lap^PP p~ + lam = F / dt inside,
    # n . grad p~ = 0 on the walls; p = p~ - a D_Lap^PP p~.
    idx_pv, (wpx, wpy) = _sampled_stencils(xp, xv, rp, (OP_DX, OP_DY))
    nbv = np.unique(idx_pv)
    posv = {r: i for i, r in enumerate(nbv)}
    uss_v, vss_v = ustar2(nbv)
    locv = np.vectorize(posv.get)(idx_pv)
    F = (wpx * uss_v[locv]).sum(0) + (wpy * vss_v[locv]).sum(0)
    idx_pp, (plap, pdx, pdy) = _sampled_stencils(xp, xp, rp, (OP_LAP, OP_DX, OP_DY))
    lap = (plap * ptn[idx_pp]).sum(0)
    scale = np.abs(plap * ptn[idx_pp]).sum(0) + np.abs(F / dt)
    inner = ~pwall[rp]
    d = lap[inner] - F[inner] / dt
    assert np.ptp(d) <= 1e-9 * np.max(scale[inner]), (np.ptp(d), np.max(scale[inner]))
    nx, ny = nd.p_normal[0][rp], nd.p_normal[1][rp]
    dn = nx * (pdx * ptn[idx_pp]).sum(0) + ny * (pdy * ptn[idx_pp]).sum(0)
    dscale = np.abs(pdx * ptn[idx_pp]).sum(0) + np.abs(pdy * ptn[idx_pp]).sum(0)
    assert np.max(np.abs(dn[~inner])) <= 1e-9 * np.max(dscale[~inner])
    p_ref = ptn[rp] - a * lap
    assert np.max(np.abs(after["p"][rp] - p_ref)) <= 1e-10 * max(1e-30, np.max(np.abs(p_ref)))
