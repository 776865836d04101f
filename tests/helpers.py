"""Shared test helpers: build the four stencil sets on the GPU (through the C
ABI) and on the CPU oracle from the same seeded node sets."""
import numpy as np

import rbf_inputs as ri

OP_ID, OP_DX, OP_DY, OP_LAP = 1, 2, 4, 8


def rel_err(a, b):
    """||a - b||_inf / ||b||_inf."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.max(np.abs(a - b)) if a.size else 0.0
    s = np.max(np.abs(b)) if b.size else 0.0
    return d / s if s > 0 else d


def row_rel_err(w_gpu, w_ora):
    """max over rows of max_s |dw| / max_s |w_ora| (weights metric)."""
    num = np.max(np.abs(w_gpu - w_ora), axis=-2)
    den = np.max(np.abs(w_ora), axis=-2)
    return float(np.max(num / den))


def to_dev(a, dev, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def gpu_cavity_ops(nd, dev, n=28, m=7, q=3):
    """kNN + weights for VV, PV, PP, VP on the GPU; returns (grid, ops) dicts."""
    import torch
    import paper_2206_06495_amd as P
    xv = to_dev(nd.xv, dev)
    xp = to_dev(nd.xp, dev)
    grid = {"xv": xv, "xp": xp, "v_tag": to_dev(nd.v_tag, dev), "p_tag": to_dev(nd.p_tag, dev),
            "p_normal": to_dev(nd.p_normal, dev)}
    ops = {"k": n}
    for name, xq, xs, mask in (("vv", xv, xv, OP_DX | OP_DY | OP_LAP), ("pv", xp, xv, OP_DX | OP_DY),
                               ("pp", xp, xp, OP_DX | OP_DY | OP_LAP), ("vp", xv, xp, OP_DX | OP_DY)):
        idx = P.knn(xq, xs, n)
        w = P.assemble_weights(xq, xs, idx, m, q, mask)
        ops["idx_" + name] = idx
        ops[name + "_dx"] = w[0].contiguous()
        ops[name + "_dy"] = w[1].contiguous()
        if mask & OP_LAP:
            ops[name + "_lap"] = w[2].contiguous()
    torch.cuda.synchronize()
    return grid, ops


def cavity_nodes(K, jitter=0.3, seed=0):
    return ri.cavity_nodes(K, jitter, seed)
