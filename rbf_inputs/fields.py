"""Seeded input fields and boundary values (no RBF-FD arithmetic here)."""
import numpy as np

from .nodes import TAG_LID


def wave_field(x, k):
    """f = sin(k x) cos(k y) on nodes ``x[2, n]`` (operator-bench input)."""
    return np.sin(k * x[0]) * np.cos(k * x[1])


def random_vector(n, seed, dtype=np.float64):
    """Standard-normal vector of length n from a seeded PCG64 stream."""
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)


def cavity_bc(v_tag, lid_u=1.0):
    """Dirichlet velocity on the V-grid walls of the lid-driven cavity
    (Sec. 5.1): u = lid_u on the lid, no slip elsewhere.  Interior entries are
    zero and unused."""
    u_bc = np.where(v_tag == TAG_LID, lid_u, 0.0).astype(np.float64)
    v_bc = np.zeros(v_tag.shape[0], np.float64)
    return u_bc, v_bc
