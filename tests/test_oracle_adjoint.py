"""The oracle's discrete adjoint against central finite differences of the
oracle itself (CPU only): gradients of the final kinetic energy with respect
to the viscosity and to a 16-mode Fourier lid profile.  A pin of
oracle/adjoint.py that does not use it: the finite differences only run the
forward scheme."""
import numpy as np
import pytest

import rbf_inputs as ri
from oracle import adjoint as oadj, cavity as ocav, operators as oops

NMODES = 16


def lid_profile(nd, coef):
    """u on the lid V-nodes: sum_k coef[k] sin((k+1) pi x) (zero at the
    corners); no slip elsewhere."""
    x = nd.xv[0]
    lid = nd.v_tag == ri.TAG_LID
    modes = np.sin(np.pi * np.outer(np.arange(1, NMODES + 1), x))  # [16, N]
    u = np.where(lid, coef @ modes, 0.0)
    return u, modes * lid


def _objective(nd, ops, nu, coef, nsteps, dt):
    u_bc, _ = lid_profile(nd, coef)
    v_bc = np.zeros(nd.n_v)
    orc = ocav.CavityOracle(nd, u_bc, v_bc, 1.0 / nu, dt, ops=ops, dense=True)
    s = orc.run(nsteps)
    return oadj.kinetic_energy(s.u, s.v)


@pytest.mark.parametrize("kind", [0, 2])
def test_oracle_adjoint_matches_central_differences(kind):
    K, nsteps, dt, nu = (8, 12, 2e-3, 1e-2)
    nd = ri.cavity_nodes(K, 0.3, 0) if kind == 0 else ri.hex_cavity_nodes(K, 0.3, 0)
    ops = oops.CavityOperators(nd)
    coef = np.zeros(NMODES)
    coef[0] = 1.0
    coef[2] = -0.3
    u_bc, modes = lid_profile(nd, coef)
    orc = ocav.CavityOracle(nd, u_bc, np.zeros(nd.n_v), 1.0 / nu, dt, ops=ops, dense=True)
    J, nub, ubc_b, vbc_b, _ = oadj.rollout_gradient(orc, orc.initial_state(), nsteps)
    g_coef = modes @ ubc_b
    assert abs(J - _objective(nd, ops, nu, coef, nsteps, dt)) <= 1e-15 * J
    eps = 1e-6
    fd_nu = (_objective(nd, ops, nu * (1 + eps), coef, nsteps, dt)
             - _objective(nd, ops, nu * (1 - eps), coef, nsteps, dt)) / (2 * eps * nu)
    assert abs(fd_nu - nub) <= 1e-6 * max(abs(fd_nu), 1e-12 * J / nu), (fd_nu, nub)
    scale = np.max(np.abs(g_coef))
    for k in (0, 1, 2, 7, 15):
        e = np.zeros(NMODES)
        e[k] = eps
        fd = (_objective(nd, ops, nu, coef + e, nsteps, dt)
              - _objective(nd, ops, nu, coef - e, nsteps, dt)) / (2 * eps)
        assert abs(fd - g_coef[k]) <= 1e-6 * scale, (k, fd, g_coef[k])
