"""Host C++ under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The node builder (csrc/nodes.cpp) and the error state (csrc/common.cpp) are
compiled for the host alone with clang (HIP language, no device code),
instrumented with ASan and UBSan (every report fatal), linked with a small
driver (tests/host/nodes_driver.cpp) and run on cavity and square node sets
through the two-call pattern and the argument checks; the coordinates must
match the NumPy generator bit for bit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import rbf_inputs as ri

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2206_06495_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ of the ROCm toolchain not found")
    out = tmp_path_factory.mktemp("san")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    common = [CLANG, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
              "-I" + os.path.join(ROOT, "include")] + san
    objs = []
    for src, lang in (("nodes.cpp", ["-x", "hip", "--offload-host-only", "-ffp-contract=off"]),
                      ("common.cpp", ["-x", "hip", "--offload-host-only"]),
                      (os.path.join(HERE, "host", "nodes_driver.cpp"), [])):
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = str(out / (os.path.basename(src) + ".o"))
        subprocess.run(common + lang + ["-c", path, "-o", obj], check=True)
        objs.append(obj)
    exe = str(out / "nodes_driver")
    subprocess.run([CLANG] + san + objs + ["-o", exe], check=True)
    return exe, out


def _read(path, nv, npn):
    raw = open(path, "rb").read()
    off = 16
    def take(n, dt):
        nonlocal off
        a = np.frombuffer(raw, dtype=dt, count=n, offset=off)
        off += a.nbytes
        return a
    xv = take(2 * nv, np.float64).reshape(2, nv)
    xp = take(2 * npn, np.float64).reshape(2, npn)
    pn = take(2 * npn, np.float64).reshape(2, npn)
    vt = take(nv, np.int8)
    pt = take(npn, np.int8)
    assert off == len(raw)
    return xv, xp, pn, vt, pt


@pytest.mark.parametrize("kind,K,jit,seed", [(0, 2, 0.3, 0), (0, 13, 0.3, 3), (0, 40, 0.0, 1),
                                             (1, 1, 0.3, 0), (1, 25, 0.45, 7), (2, 2, 0.3, 0),
                                             (2, 17, 0.4, 5), (2, 60, 0.0, 1)])
def test_node_builder_clean_under_sanitizers(driver, kind, K, jit, seed):
    exe, out = driver
    path = str(out / f"nodes_{kind}_{K}_{seed}.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe, str(kind), str(K), repr(jit), str(seed), path], env=env,
                         capture_output=True, text=True)
    assert res.returncode == 0, (res.returncode, res.stderr[-2000:])
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
    nv, npn = np.frombuffer(open(path, "rb").read(16), dtype=np.int64)
    xv, xp, pn, vt, pt = _read(path, int(nv), int(npn))
    nd = ri.build_nodes(kind, K, jit, seed)
    assert np.array_equal(xv, nd.xv) and np.array_equal(xp, nd.xp)
    if kind != 1:
        assert np.array_equal(vt, nd.v_tag) and np.array_equal(pt, nd.p_tag)
        assert np.array_equal(pn, nd.p_normal)
    else:
        assert not vt.any() and not pt.any() and not pn.any()
