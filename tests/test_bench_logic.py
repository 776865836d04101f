"""Host logic of bench.py (CPU only): step statistics summed over rbf_step
calls, the algorithmic bytes of the roofline kernels, and the refusal of
more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
torch = pytest.importorskip("torch")
import bench  # noqa: E402


class _FakeSolver:
    def __init__(self):
        self.calls = []

    def step(self, st, k):
        self.calls.append(k)
        st["step"] += k

        class _S:
            poisson_iters, helmholtz_iters, last_poisson = 3 * k, k, None
        return _S()


def test_run_sums_statistics():
    S = _FakeSolver()
    st = {"step": 0}
    r = bench.Run(S, st)
    r.advance(7)
    r.advance(0)
    r.advance(5)
    assert S.calls == [7, 5] and st["step"] == 12
    assert r.poisson_iters == 36 and r.helmholtz_iters == 12
    r.clear()
    assert r.poisson_iters == 0 and r.last is None


def test_kernel_bytes():
    M = 1000
    b = bench.kernel_bytes(M, {}, 21.0)  # mean Arnoldi index 10: 11 basis vectors
    assert b["k_aux_post2"] == M * 368
    assert b["k_fg_av2"] == M * (352 + 8 * 11)
    assert b["k_fg_gs<2>"] == M * (32 + 8 * 11)


def test_shedding_statistics():
    """Strouhal number from the upward zero crossings of C_L over the second
    half of the series, and the force amplitudes, for a synthetic limit
    cycle; None before three periods."""
    import numpy as np
    t = np.arange(0.0, 100.0, 0.02)
    cl = 0.3 * np.sin(2 * np.pi * 0.17 * t + 0.4)
    cd = 1.35 + 0.01 * np.sin(4 * np.pi * 0.17 * t)
    ser = [{"t": a, "C_D": b, "C_L": c} for a, b, c in zip(t, cd, cl)]
    r = bench.shedding_stats(ser, 0.02)
    assert abs(r["St"] - 0.17) < 1e-6 and abs(r["C_D_mean"] - 1.35) < 1e-3
    assert abs(r["C_L_amp"] - 0.3) < 1e-3 and abs(r["C_D_amp"] - 0.01) < 1e-4
    assert bench.shedding_stats(ser[:700], 0.02) is None


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode == 2 and "one GPU" in res.stderr
