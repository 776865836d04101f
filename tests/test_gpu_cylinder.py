"""Flow past a cylinder (Sec. 5.2) through the C ABI, against the oracle.

Coarse graded cylinder-in-channel nodes (diameter 1 at the origin, channel
[-4, 8] x [-4, 4], spacing 0.1 on the cylinder growing by 0.1 per unit of
radius: N = 3,218 V + M = 1,111 P), uniform inflow, symmetry sides,
convective outflow (rbf_grid tags RBF_VTAG_SYMMETRY and RBF_VTAG_OUTFLOW),
no slip on the cylinder, impulsive start from U_0 = (1, 0).  u, v, p, p~
and the drag and lift of rbf_solver_forces against oracle.cylinder within
1e-10 every 2 steps over an 8-step window (Re = 1000, dt = 5e-3, pressure
tolerance 1e-13).  The window is short because on these ring-and-Delaunay
node sets the scheme has growing modes near the curved wall (the lift
coefficient, 0.015 after 4 steps, reaches 0.36 after 10), which amplify the
solver-tolerance differences between the two sides (forces 1.2e-10 after
10 steps, fields 3e-10 after 15).
"""
import numpy as np
import pytest

import rbf_inputs as ri
from oracle import cylinder as oc
from tests.helpers import rel_err, to_dev, gpu_cavity_ops

pytestmark = pytest.mark.gpu

BOX = (-4.0, 8.0, -4.0, 4.0)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P(gpu):
    import paper_2206_06495_amd as P
    return P


def test_cylinder_flow_against_oracle(P, gpu):
    _say("cylinder flow, coarse channel")
    nd = ri.cylinder_nodes(h_wall=0.1, grading=0.1, box=BOX)
    re, dt = 1000.0, 5e-3
    grid, ops = gpu_cavity_ops(nd, gpu)
    orc = oc.ChannelOracle(nd, re, dt)
    S = P.Solver(grid, ops, to_dev(orc.u_bc, gpu), to_dev(orc.v_bc, gpu), re, dt, u_conv=1.0,
                 rtol_p=1e-13)
    assert S.info()["aux_precond"]
    so = orc.initial_state()
    st = S.new_state(to_dev(so.u, gpu), to_dev(so.v, gpu))
    worst = worst_f = 0.0
    for _ in range(4):
        stats = S.step(st, 2)
        so = orc.run(2, so)
        for key, ref in (("u", so.u), ("v", so.v), ("p", so.p), ("p_tilde", so.pt)):
            e = rel_err(st[key].cpu().numpy(), ref)
            worst = max(worst, e)
            assert e <= 1e-10, (st["step"], key, e)
        fg = np.array(S.forces(grid, st))
        fo = np.array(oc.cylinder_forces(nd, orc.ops, so.u, so.v, so.p, re))
        ef = np.max(np.abs(fg - fo)) / np.max(np.abs(fo))
        worst_f = max(worst_f, ef)
        assert ef <= 1e-10, (st["step"], fg, fo)
        _say("step", st["step"], "C_D, C_L", 2 * fg, "pressure steps per time step",
             stats.poisson_iters / 2)
    _say("worst field error", worst, "worst force error", worst_f)
    S.close()


def test_forces_argument_checks(P, gpu):
    nd = ri.cylinder_nodes(h_wall=0.1, grading=0.1, box=BOX)
    grid, ops = gpu_cavity_ops(nd, gpu)
    orc = oc.ChannelOracle(nd, 100.0, 1e-2)
    S = P.Solver(grid, ops, to_dev(orc.u_bc, gpu), to_dev(orc.v_bc, gpu), 100.0, 1e-2)
    so = orc.initial_state()
    st = S.new_state(to_dev(so.u, gpu), to_dev(so.v, gpu))
    with pytest.raises(P.RbfError) as ei:
        S.forces(grid, st, tag=0)
    assert ei.value.status == -1
    with pytest.raises(P.RbfError) as ei:
        S.forces(grid, st, tag=7)  # no node carries it
    assert ei.value.status == -1 and "even counts" in str(ei.value)
    S.close()
