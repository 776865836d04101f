"""Flow past a cylinder (Sec. 5.2) through the C ABI, against the oracle.

Graded cylinder-in-channel nodes (diameter 1 at the origin, channel
[-2.5, 5] x [-2.5, 2.5], spacing 0.03 on the cylinder -- the paper's --
growing by 0.05 per unit of radius: N = 13,961 V + M = 4,736 P), uniform
inflow, symmetry sides, convective outflow (rbf_grid tags RBF_VTAG_SYMMETRY
and RBF_VTAG_OUTFLOW), no slip on the cylinder, impulsive start from
U_0 = (1, 0), Re = 100, dt = 5e-3, solver tolerances 1e-13 (pressure) and
1e-14 (viscous).  u, v, p, p~ and the drag and lift of rbf_solver_forces
against oracle.cylinder every 20 steps: within 1e-10 after 20 and 40 steps,
within 3e-10 after 60 steps (t = 0.3).  The bound widens because the
wake's asymmetric mode grows from the start and amplifies the
rounding-level differences between the two sides (an iterative solve to
rtol 1e-13 against LU, and summation orders): the pressure differs by
0.9-1.0e-10 of its largest value after 60 steps, 1.9e-10 after 80 (and
1.3e-10 after 40 steps at dt = 2e-3, where differences in u** reach p~
times 1/dt).  Coarser cylinders, 0.05 or 0.1 on the wall, carry growing
modes at the wall within tens of steps.
"""
import numpy as np
import pytest

import rbf_inputs as ri
from oracle import cylinder as oc
from tests.helpers import rel_err, to_dev, gpu_cavity_ops

pytestmark = pytest.mark.gpu

BOX = (-2.5, 5.0, -2.5, 2.5)
H_WALL, GRADING = 0.03, 0.05


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P(gpu):
    import paper_2206_06495_amd as P
    return P


def test_cylinder_flow_against_oracle(P, gpu):
    _say("cylinder flow, coarse channel")
    nd = ri.cylinder_nodes(h_wall=H_WALL, grading=GRADING, box=BOX)
    re, dt = 100.0, 5e-3
    grid, ops = gpu_cavity_ops(nd, gpu)
    orc = oc.ChannelOracle(nd, re, dt)
    S = P.Solver(grid, ops, to_dev(orc.u_bc, gpu), to_dev(orc.v_bc, gpu), re, dt, u_conv=1.0,
                 rtol_p=1e-13, rtol_h=1e-14)
    assert S.info()["aux_precond"]
    so = orc.initial_state()
    st = S.new_state(to_dev(so.u, gpu), to_dev(so.v, gpu))
    worst = worst_f = 0.0
    for tol in (1e-10, 1e-10, 3e-10):
        stats = S.step(st, 20)
        so = orc.run(20, so)
        for key, ref in (("u", so.u), ("v", so.v), ("p", so.p), ("p_tilde", so.pt)):
            e = rel_err(st[key].cpu().numpy(), ref)
            worst = max(worst, e)
            _say("step", st["step"], key, "rel err", e)
            assert e <= tol, (st["step"], key, e)
        fg = np.array(S.forces(grid, st))
        fo = np.array(oc.cylinder_forces(nd, orc.ops, so.u, so.v, so.p, re))
        ef = np.max(np.abs(fg - fo)) / np.max(np.abs(fo))
        worst_f = max(worst_f, ef)
        assert ef <= tol, (st["step"], fg, fo)
        _say("step", st["step"], "C_D, C_L", 2 * fg, "pressure steps per time step",
             stats.poisson_iters / 20)
    _say("worst field error", worst, "worst force error", worst_f)
    S.close()


def test_forces_argument_checks(P, gpu):
    nd = ri.cylinder_nodes(h_wall=H_WALL, grading=GRADING, box=BOX)
    grid, ops = gpu_cavity_ops(nd, gpu)
    orc = oc.ChannelOracle(nd, 100.0, 2e-3)
    S = P.Solver(grid, ops, to_dev(orc.u_bc, gpu), to_dev(orc.v_bc, gpu), 100.0, 2e-3)
    so = orc.initial_state()
    st = S.new_state(to_dev(so.u, gpu), to_dev(so.v, gpu))
    with pytest.raises(P.RbfError) as ei:
        S.forces(grid, st, tag=0)
    assert ei.value.status == -1
    with pytest.raises(P.RbfError) as ei:
        S.forces(grid, st, tag=7)  # no node carries it
    assert ei.value.status == -1 and "even counts" in str(ei.value)
    S.close()
