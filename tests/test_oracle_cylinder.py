"""Pins of the cylinder-flow oracle (Sec. 5.2) against closed forms (CPU).

* Simpson's periodic rule integrates trigonometric polynomials of degree
  below the node count exactly, and its weights sum to the period.
* Forces: for a linear pressure field p = x the pressure force is
  -(pi r^2, 0); for u = y^2, v = 0 the viscous force is (1/Re) times the
  closed integral of 2y n_y ds = (2 pi r r_v / Re, 0), r_v the radius of the
  V-nodes (chord midpoints) -- exact because the RBF-FD rows reproduce
  polynomials of degree <= 3 and the rule is exact for sin^2.  A dropped
  term, a wrong sign or a transposed stress component fails one of them.
* Open boundary rows: for fields the stencils reproduce exactly, the
  symmetry row returns the node's own value when du/dy = 0 and the
  convective row moves a linear profile by -dt U_c du/dx.
"""
import numpy as np
import pytest

import rbf_inputs as ri
from oracle import cylinder as oc, operators as oops

BOX = (-4.0, 8.0, -4.0, 4.0)


@pytest.fixture(scope="module")
def coarse():
    nd = ri.cylinder_nodes(h_wall=0.1, grading=0.1, box=BOX)
    return nd, oops.CavityOperators(nd)


@pytest.mark.parametrize("n", [8, 32, 158])
def test_simpson_periodic_weights(n):
    w = oc.simpson_periodic_weights(n)
    th = 2 * np.pi * np.arange(n) / n
    assert abs(w.sum() - 2 * np.pi) < 1e-13
    for f, exact in ((np.cos(th) ** 2, np.pi), (np.sin(th) * np.cos(th), 0.0),
                     (np.sin(3 * th) ** 2, np.pi if n > 6 else None)):
        if exact is not None:
            assert abs(np.sum(w * f) - exact) < 1e-12
    with pytest.raises(ValueError):
        oc.simpson_periodic_weights(n + 1)


def test_pressure_force_of_linear_field(coarse):
    nd, ops = coarse
    z = np.zeros(nd.n_v)
    fx, fy = oc.cylinder_forces(nd, ops, z, z, nd.xp[0].copy(), 100.0)
    assert abs(fx + np.pi * 0.25) < 1e-12 and abs(fy) < 1e-12
    fx, fy = oc.cylinder_forces(nd, ops, z, z, 2.0 * nd.xp[1], 100.0)
    assert abs(fx) < 1e-12 and abs(fy + 2.0 * np.pi * 0.25) < 1e-12


def test_viscous_force_of_polynomial_field(coarse):
    nd, ops = coarse
    re = 50.0
    ncyl = int((nd.v_tag == oc.TAG_CYLINDER).sum())
    r_v = 0.5 * np.cos(np.pi / ncyl)
    assert np.allclose(np.hypot(*nd.xv[:, nd.v_tag == oc.TAG_CYLINDER]), r_v, atol=1e-14)
    u = nd.xv[1] ** 2
    zp = np.zeros(nd.n_p)
    fx, fy = oc.cylinder_forces(nd, ops, u, np.zeros(nd.n_v), zp, re)
    assert abs(fx - 2 * np.pi * 0.5 * r_v / re) < 1e-9 and abs(fy) < 1e-9
    # v = x^2: (u_y + v_x) n_x = 2x n_x gives the lift
    fx, fy = oc.cylinder_forces(nd, ops, np.zeros(nd.n_v), nd.xv[0] ** 2, zp, re)
    assert abs(fy - 2 * np.pi * 0.5 * r_v / re) < 1e-9 and abs(fx) < 1e-9


def test_open_boundary_rows(coarse):
    nd, ops = coarse
    dt = 0.01
    orc = oc.ChannelOracle(nd, 100.0, dt, ops=ops)
    x, y = nd.xv
    side = nd.v_tag == oc.TAG_SIDE
    out = nd.v_tag == oc.TAG_OUTFLOW
    inflow = nd.v_tag == oc.TAG_INFLOW
    cyl = nd.v_tag == oc.TAG_CYLINDER
    u = 1.0 + 0.3 * x - 0.02 * x ** 2  # du/dy = 0, du/dx = 0.3 - 0.04 x
    v = 0.5 * x + 0.1                  # dv/dx = 0.5
    ub, vb = orc.open_values(u, v)
    assert np.max(np.abs(ub[side] - u[side])) < 1e-9 and np.all(vb[side] == 0.0)
    assert np.max(np.abs(ub[out] - (u[out] - dt * (0.3 - 0.04 * x[out])))) < 1e-9
    assert np.max(np.abs(vb[out] - (v[out] - dt * 0.5))) < 1e-9
    assert np.all(ub[inflow] == 1.0) and np.all(vb[inflow] == 0.0)
    assert np.all(ub[cyl] == 0.0) and np.all(vb[cyl] == 0.0)
