"""Concurrent stepping of independent instances (rbf_step_batch) against
stepping each instance alone, and one instance against the oracle."""
import numpy as np
import pytest

import rbf_inputs as ri
from oracle import cavity as ocav
from tests.helpers import rel_err, to_dev, gpu_cavity_ops

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "p", "p_tilde", "cu_prev", "cv_prev")


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P(gpu):
    import paper_2206_06495_amd as P
    return P


def _instances(P, gpu, cases, **kw):
    """One solver per (K, Re, seed), each created on its own stream."""
    import torch
    out = []
    for K, re, seed in cases:
        nd = ri.cavity_nodes(K, 0.3, seed)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            grid, ops = gpu_cavity_ops(nd, gpu)
            u_bc, v_bc = ri.cavity_bc(nd.v_tag)
            S = P.Solver(grid, ops, to_dev(u_bc, gpu), to_dev(v_bc, gpu), re, DT, **kw)
            st = S.new_state(to_dev(np.where(nd.v_tag != 0, u_bc, 0.0), gpu),
                             to_dev(np.where(nd.v_tag != 0, v_bc, 0.0), gpu))
        out.append({"S": S, "st": st, "stream": s, "nd": nd, "bc": (u_bc, v_bc),
                    "keep": (grid, ops), "re": re, "dt": DT})
    torch.cuda.synchronize()
    return out


DT = 2e-3
CASES = [(10, 100.0, 0), (14, 400.0, 1), (17, 1000.0, 2), (21, 250.0, 5), (12, 3000.0, 4)]


def test_step_batch_matches_single_instances(P, gpu):
    """Five cavities of different sizes and Reynolds numbers, each on its own
    stream, 12 steps on 3 host threads: every field bit-identical to 12
    rbf_step calls on a second copy of each instance alone (all reductions
    run in a fixed order); the smallest instance also matches the oracle."""
    import torch
    _say("step_batch vs single instances")
    A = _instances(P, gpu, CASES)
    B = _instances(P, gpu, CASES)
    stats, codes = P.step_batch([a["S"] for a in A], [a["st"] for a in A], 12, nthreads=3)
    assert codes == [0] * len(CASES)
    assert all(s.steps_done == 12 for s in stats)
    for b in B:
        with torch.cuda.stream(b["stream"]):
            b["S"].step(b["st"], 12)
    torch.cuda.synchronize()
    for a, b, case in zip(A, B, CASES):
        assert a["st"]["step"] == b["st"]["step"] == 12, case
        for key in FIELDS:
            assert torch.equal(a["st"][key], b["st"][key]), (case, key)
    a = A[0]
    orc = ocav.CavityOracle(a["nd"], a["bc"][0], a["bc"][1], a["re"], a["dt"])
    so = orc.run(12, orc.initial_state())
    for key, ref in (("u", so.u), ("v", so.v), ("p", so.p), ("p_tilde", so.pt)):
        assert rel_err(a["st"][key].cpu().numpy(), ref) <= 1e-10, key
    for x in A + B:
        x["S"].close()


def test_step_batch_failure_is_per_instance(P, gpu):
    """An instance that cannot converge (pressure cap of one iteration) fails
    alone: its status is RBF_E_NOCONV and its state keeps step 0, while the
    other instances of the call complete their steps; the call raises for
    it after all were attempted."""
    import torch
    _say("step_batch failure")
    cases = CASES[:3]
    A = _instances(P, gpu, cases)
    bad = _instances(P, gpu, [cases[1]], maxit_p=1)[0]
    A[1] = bad
    before = {k: bad["st"][k].clone() for k in FIELDS}
    with pytest.raises(P.RbfError) as ei:
        P.step_batch([a["S"] for a in A], [a["st"] for a in A], 4, nthreads=2)
    assert ei.value.status == -3
    assert ei.value.statuses == [0, -3, 0]
    assert "instance 1" in str(ei.value)
    torch.cuda.synchronize()
    assert A[0]["st"]["step"] == 4 and A[2]["st"]["step"] == 4
    assert bad["st"]["step"] == 0
    for k in FIELDS:
        assert torch.equal(bad["st"][k], before[k]), k
    twin = {k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in A[0]["st"].items()}
    with pytest.raises(P.RbfError) as ei:  # the same solver twice would race with itself
        P.step_batch([A[0]["S"], A[0]["S"]], [A[0]["st"], twin], 1)
    assert ei.value.status == -1 and A[0]["st"]["step"] == 4
    for x in A:
        x["S"].close()
