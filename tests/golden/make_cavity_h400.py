"""Writes cavity_h400_100steps.json: the oracle's state after 100 steps of the
lid-driven cavity at h = 1/400 (jittered near-equilateral nodes, K = 400,
jitter 0.3 h, seed 0; Re = 1e4, dt = 2e-4), on sampled rows, plus whole-field
sums.  Calls only the oracle and the seeded input generators.

Run from the repository root:  python tests/golden/make_cavity_h400.py
(about 11 minutes of operator assembly and LU factorisation, then about 3 s
per step, single-threaded).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import rbf_inputs as ri  # noqa: E402
from oracle import cavity as ocav  # noqa: E402
from oracle import operators as oops  # noqa: E402

K, JITTER, SEED = 400, 0.3, 0
RE, DT, STEPS = 1e4, 2e-4, 100
N_SAMPLE_V, N_SAMPLE_P = 600, 300


def sample_rows(n, k, rng):
    """k distinct rows drawn uniformly (wall rows included in proportion)."""
    return np.sort(rng.choice(n, size=k, replace=False))


def field_sums(x):
    return {"sum": float(np.sum(x)), "sum_sq": float(np.sum(x * x)),
            "max_abs": float(np.max(np.abs(x)))}


def main():
    t0 = time.perf_counter()
    nd = ri.hex_cavity_nodes(K, JITTER, SEED)
    u_bc, v_bc = ri.cavity_bc(nd.v_tag)
    ops = oops.CavityOperators(nd)
    orc = ocav.CavityOracle(nd, u_bc, v_bc, RE, DT, ops=ops)
    print(f"set-up {time.perf_counter() - t0:.0f} s  N={nd.n_v} M={nd.n_p}", flush=True)
    s = orc.initial_state()
    for j in range(STEPS):
        s = orc.step(s)
        if (j + 1) % 10 == 0:
            print(f"step {j + 1}  {time.perf_counter() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(20240601)
    iv = sample_rows(nd.n_v, N_SAMPLE_V, rng)
    ip = sample_rows(nd.n_p, N_SAMPLE_P, rng)
    out = {
        "workload": {"kind": "near-equilateral cavity", "K": K, "jitter": JITTER, "seed": SEED,
                     "re": RE, "dt": DT, "steps": STEPS, "n_v": int(nd.n_v), "n_p": int(nd.n_p),
                     "n": 28, "m": 7, "q": 3},
        "written_by": "tests/golden/make_cavity_h400.py (oracle: scipy SuperLU solves)",
        "v_rows": iv.tolist(),
        "p_rows": ip.tolist(),
        "u": s.u[iv].tolist(),
        "v": s.v[iv].tolist(),
        "p": s.p[ip].tolist(),
        "pt": s.pt[ip].tolist(),
        "sums": {"u": field_sums(s.u), "v": field_sums(s.v), "p": field_sums(s.p),
                 "pt": field_sums(s.pt)},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cavity_h400_100steps.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
