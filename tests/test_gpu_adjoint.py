"""The adjoint step (rbf_adjoint_step) and the differentiable rollout
(LidRollout, checkpoints every 10 steps) against the oracle's discrete
adjoint and against central differences of the GPU forward scheme:
gradients of the final kinetic energy with respect to nu = 1/Re and a
16-mode Fourier lid profile."""
import numpy as np
import pytest

import rbf_inputs as ri
from oracle import adjoint as oadj, cavity as ocav, operators as oops
from tests.helpers import to_dev, gpu_cavity_ops

pytestmark = pytest.mark.gpu
NMODES = 16


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def P(gpu):
    import paper_2206_06495_amd as P
    return P


def _modes(nd):
    lid = nd.v_tag == ri.TAG_LID
    return np.sin(np.pi * np.outer(np.arange(1, NMODES + 1), nd.xv[0])) * lid


def _case(kind, K):
    nd = ri.cavity_nodes(K, 0.3, 0) if kind == 0 else ri.hex_cavity_nodes(K, 0.3, 0)
    coef = np.zeros(NMODES)
    coef[0], coef[2] = 1.0, -0.3
    return nd, coef


@pytest.mark.parametrize("kind,K,nsteps", [(0, 8, 12), (2, 10, 25)])
def test_rollout_gradient_matches_oracle_adjoint(P, gpu, kind, K, nsteps):
    """d(final KE)/d nu and d/d coef through LidRollout (GPU adjoint steps,
    checkpoints every 10 steps) against oracle.adjoint.rollout_gradient on
    the same nodes: within 1e-8 relative to the largest component."""
    import torch
    _say("adjoint vs oracle", kind, K, nsteps)
    nd, coef = _case(kind, K)
    dt, nu = 2e-3, 1e-2
    grid, ops = gpu_cavity_ops(nd, gpu)
    modes = _modes(nd)
    R = P.LidRollout(grid, ops, to_dev(modes, gpu), dt, nsteps, every=10, rtol_p=1e-13)
    nu_t = torch.tensor(nu, dtype=torch.float64, requires_grad=True)
    c_t = torch.tensor(coef, dtype=torch.float64, requires_grad=True)
    J = R(nu_t, c_t)
    J.backward()
    u_bc = coef @ modes
    orc = ocav.CavityOracle(nd, u_bc, np.zeros(nd.n_v), 1.0 / nu, dt, dense=True)
    Jo, nub, ubc_b, _, _ = oadj.rollout_gradient(orc, orc.initial_state(), nsteps)
    go = modes @ ubc_b
    _say("J", float(J), Jo, "dnu", float(nu_t.grad), nub)
    assert abs(float(J) - Jo) <= 1e-10 * Jo
    assert abs(float(nu_t.grad) - nub) <= 1e-8 * abs(nub)
    gc = c_t.grad.numpy()
    assert np.max(np.abs(gc - go)) <= 1e-8 * np.max(np.abs(go)), (gc, go)


def test_rollout_gradient_matches_central_differences(P, gpu):
    """GPU adjoint gradient against central differences of the GPU forward
    rollout with eps = 1e-6 (relative for nu): within 1e-6 relative to the
    largest gradient component."""
    import torch
    _say("adjoint vs central differences")
    nd, coef = _case(2, 10)
    dt, nu, nsteps = 2e-3, 1e-2, 25
    grid, ops = gpu_cavity_ops(nd, gpu)
    modes = to_dev(_modes(nd), gpu)
    R = P.LidRollout(grid, ops, modes, dt, nsteps, every=10, rtol_p=1e-13)
    nu_t = torch.tensor(nu, dtype=torch.float64, requires_grad=True)
    c_t = torch.tensor(coef, dtype=torch.float64, requires_grad=True)
    R(nu_t, c_t).backward()
    g_nu, g_c = float(nu_t.grad), c_t.grad.numpy()
    eps = 1e-6
    J = lambda n, c: float(R(torch.tensor(n, dtype=torch.float64),  # noqa: E731
                              torch.tensor(c, dtype=torch.float64)))
    fd_nu = (J(nu * (1 + eps), coef) - J(nu * (1 - eps), coef)) / (2 * eps * nu)
    _say("dnu", g_nu, fd_nu)
    assert abs(fd_nu - g_nu) <= 1e-6 * abs(g_nu)
    scale = np.max(np.abs(g_c))
    for k in (0, 2, 5, 15):
        e = np.zeros(NMODES)
        e[k] = eps
        fd = (J(nu, coef + e) - J(nu, coef - e)) / (2 * eps)
        _say("coef", k, g_c[k], fd)
        assert abs(fd - g_c[k]) <= 1e-6 * scale, (k, fd, g_c[k])
