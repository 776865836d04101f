"""Benchmark of the staggered-node RBF-FD Navier-Stokes hot path on one MI355X.

Workload (one JSON line on stdout):
  * step throughput: lid-driven cavity, Re = 1e4, dt = 2e-4, h = 1/400 on the
    paper's staggered layout over a seed-jittered near-equilateral
    triangulation (node kind 2: P on the vertices, V on the edge midpoints,
    N = 555,955, M = 185,894), 28-point PHS r^7 + cubic stencils, FP64,
    pressure by flexible GMRES with the two-level auxiliary-lattice
    preconditioner.  Setup (stencils, weights, system matrices) is timed
    separately; `warmup` steps run untimed, then `steps` steps are timed from
    the state the warm-up left.  value = (N + M) * steps / seconds
    (node-steps/s).
  * roofline of the dominant kernel of the step (the longest of the sampled
    pressure-solve kernels: the FGMRES product k_fg_av2, the smoothing product
    k_aux_post2, the Gram-Schmidt update k_fg_gs<2>, the auxiliary
    lattice transform k_pc_gemm<0>), its average duration sampled with the
    launch's own start/end stamps on the solver's stream during the timed
    steps, against its algorithmic bytes per launch.
  * mixed: the same steps with FP32 restart cycles inside FP64 iterative
    refinement, and the relative difference of the fields from the FP64 run.
  * lattice: the right-triangle lattice cavity (node kind 0) of the same size
    with the lattice fast-Poisson preconditioner and BiCGSTAB, 100 steps
    (context: that layout diverges after about 490 steps from rest).
  * batch: `batch` independent near-equilateral cavities, N uniform in
    [5000, 60000] V-nodes and Re log-uniform in [100, 5000] (dt = 0.08 h),
    each solver on its own stream, advanced `batch_steps` steps by
    rbf_step_batch on one host thread and on `batch_threads` threads, from
    the same states; aggregate node-steps/s and bit-identity of the two.
  * operator bench: 10^6 V + 10^6 P jittered square nodes, weights for VV
    {D_x, D_y, Lap} and PV {I}, the launch shape of each operator size and
    precision chosen by the library's autotuner, then `spmv_reps`
    applications of each operator in FP64 and FP32-stored ELL, timed with
    HIP events; achieved GB/s from the algorithmic bytes; truncation error against closed-form derivatives of
    sin(kx)cos(ky), k = 2 pi {4, 16, 64}, over interior rows and over all
    rows; the distribution of the 1-norm condition estimates of the VV
    systems.
  * cylinder: flow past a cylinder (Sec. 5.2) on the graded channel set
    (N = 396,685 V + M = 132,565 P), Re = 100, dt = 2e-3, uniform inflow,
    symmetry sides, convective outflow; `cyl_steps` steps from an impulsive
    start (with a small transverse disturbance), node-steps/s, the drag and
    lift coefficients every 10 steps and, for runs long enough to shed, the
    mean drag, the force amplitudes and the Strouhal number.
  * cpu_baseline: the CPU oracle (SciPy sparse LU solves, as the paper's
    factor-once scheme) on a bounded sample of the headline workload: the
    same node kind, Re, dt, jitter and stencils at h = 1/100 (`--cpu-K`;
    at h = 1/400 its set-up alone takes about 11 minutes), a few steps after
    an untimed set-up.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TFLOPS = 78.6

# Traffic beyond L2 per launch of the roofline kernels at the headline
# workload, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE scaled by the same
# counters on a plain 256 MiB copy (2.0 and 1.0), mean over the working
# launches of 3 steps from rest (mean Arnoldi index 11.9 for k_fg_av2 and
# k_fg_gs<2>); None for a kernel changed since it was measured.
TRAFFIC_BYTES = {"k_fg_av2": 87.05e6, "k_aux_post2": 68.84e6, "k_fg_gs<2>": 26.30e6,
                 "k_pc_gemm<0>": 22.76e6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--K", type=int, default=400, help="cavity cells per side (h = 1/K)")
    ap.add_argument("--re", type=float, default=1e4)
    ap.add_argument("--dt", type=float, default=2e-4)
    ap.add_argument("--jitter", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--spmv-K", type=int, default=1000)
    ap.add_argument("--spmv-reps", type=int, default=1000)
    ap.add_argument("--no-spmv", action="store_true")
    ap.add_argument("--no-lattice", action="store_true",
                    help="skip the right-triangle lattice cavity leg")
    ap.add_argument("--lattice-steps", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run (FP32 cycles in FP64 refinement)")
    ap.add_argument("--cpu-K", type=int, default=100,
                    help="cells per side of the oracle's sample (same node kind, Re, dt); "
                         "h = 1/400 needs about 11 minutes of oracle set-up")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--prof-every", type=int, default=25)
    ap.add_argument("--rtol-p", type=float, default=1e-12)
    ap.add_argument("--rtol-h", type=float, default=1e-13)
    ap.add_argument("--batch", type=int, default=64,
                    help="independent cavities of the concurrent-instance run (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-threads", type=int, default=8)
    ap.add_argument("--no-cylinder", action="store_true",
                    help="skip the cylinder-flow leg")
    ap.add_argument("--cyl-steps", type=int, default=50)
    ap.add_argument("--cyl-re", type=float, default=100.0)
    ap.add_argument("--cyl-dt", type=float, default=2e-3)
    ap.add_argument("--cyl-perturb", type=float, default=0.1)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 256 MiB device copy first (HBM counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dev_tensor(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def build_ops(P, xv, xp):
    """28-point stencils and PHS r^7 + cubic weights of the four stencil
    sets (VV: D_x, D_y, Lap; PV: D_x, D_y; PP: D_x, D_y, Lap; VP: D_x, D_y)."""
    ops = {"k": 28}
    for name, xq, xs, mask in (("vv", xv, xv, 14), ("pv", xp, xv, 6),
                               ("pp", xp, xp, 14), ("vp", xv, xp, 6)):
        idx = P.knn(xq, xs, 28)
        w = P.assemble_weights(xq, xs, idx, 7, 3, mask)
        ops["idx_" + name] = idx
        ops[name + "_dx"] = w[0].contiguous()
        ops[name + "_dy"] = w[1].contiguous()
        if mask & 8:
            ops[name + "_lap"] = w[2].contiguous()
        del w
    return ops


def cavity_setup(P, args, dev, precision="fp64", kind=2, precond="auto"):
    """Nodes (rbf_build_nodes `kind`), stencils, weights and the solver, on
    the device; returns the solver, a rest state, the nodes and the set-up
    time."""
    import torch
    nodes = P.build_nodes(kind, args.K, args.jitter, args.seed)
    t0 = time.perf_counter()
    g = {k: dev_tensor(v, dev) for k, v in nodes.items()}
    ops = build_ops(P, g["xv"], g["xp"])
    vt = nodes["v_tag"]
    u_bc = np.where(vt == 2, 1.0, 0.0)
    S = P.Solver(g, ops, dev_tensor(u_bc, dev), dev_tensor(np.zeros_like(u_bc), dev),
                 args.re, args.dt, rtol_h=args.rtol_h, rtol_p=args.rtol_p, maxit_h=2000,
                 maxit_p=200000, precision=precision, precond=precond)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    del ops
    st = S.new_state(dev_tensor(u_bc, dev), dev_tensor(np.zeros_like(u_bc), dev))
    return S, st, nodes, setup_s


class Run:
    """Steps of one solver; sums the statistics of its rbf_step calls."""

    def __init__(self, S, st):
        self.S, self.st = S, st
        self.clear()

    def clear(self):
        self.poisson_iters = self.helmholtz_iters = 0
        self.last = None

    def advance(self, n):
        if n > 0:
            s = self.S.step(self.st, n)
            self.poisson_iters += s.poisson_iters
            self.helmholtz_iters += s.helmholtz_iters
            self.last = s
        return self


def spmv_bench(P, args, dev):
    import torch
    import rbf_inputs as ri
    nd = ri.square_nodes(args.spmv_K, 0.3, 0)
    xv, xp = dev_tensor(nd.xv, dev), dev_tensor(nd.xp, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx_vv = P.knn(xv, xv, 28)
    w_vv = P.assemble_weights(xv, xv, idx_vv, 7, 3, 14)
    idx_pv = P.knn(xp, xv, 28)
    w_pv = P.assemble_weights(xp, xv, idx_pv, 7, 3, 1)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    nsys = xv.shape[1] + xp.shape[1]
    # Weight kernel alone (FP64 throughput): one more VV assembly, timed by events.
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    P.assemble_weights(xv, xv, idx_vv, 7, 3, 14)
    e1.record()
    torch.cuda.synchronize()
    wt_ms = e0.elapsed_time(e1)
    s_sz = 38
    flops_per_sys = (2.0 / 3.0) * s_sz ** 3 + 2 * s_sz ** 2 * 3 + 5.0e3
    ops = {"dx_vv": (idx_vv, w_vv[0].contiguous(), xv.shape[1]),
           "dy_vv": (idx_vv, w_vv[1].contiguous(), xv.shape[1]),
           "lap_vv": (idx_vv, w_vv[2].contiguous(), xv.shape[1]),
           "id_pv": (idx_pv, w_pv[0].contiguous(), xv.shape[1])}
    out = {"setup_s": setup_s, "systems": nsys,
           "weights_vv_ms": wt_ms,
           "weights_vv_tflops": xv.shape[1] * flops_per_sys / (wt_ms * 1e-3) / 1e12}
    out["weights_vv_frac_fp64_peak"] = out["weights_vv_tflops"] / FP64_VALU_PEAK_TFLOPS
    # 1-norm condition estimates of the VV systems (local scaled coordinates).
    e0.record()
    _, cond = P.assemble_weights(xv, xv, idx_vv, 7, 3, 14, cond=True)
    e1.record()
    torch.cuda.synchronize()
    c = cond.cpu().numpy()
    q = np.percentile(c, [0, 1, 50, 99, 100])
    out["weights_vv_cond_est"] = {"ms_with_estimate": e0.elapsed_time(e1),
                                  "min": q[0], "p1": q[1], "median": q[2], "p99": q[3],
                                  "max": q[4], "log10_mean": float(np.mean(np.log10(c)))}
    del cond
    res = {}
    for k_wave in (4, 16, 64):
        kk = 2 * math.pi * k_wave
        fv = dev_tensor(ri.wave_field(nd.xv, kk), dev)
        errs = {}
        xh, yh = nd.xv
        inner = (np.minimum.reduce([xh, yh, 1 - xh, 1 - yh]) > 4.0 / args.spmv_K)
        exact = {"dx_vv": kk * np.cos(kk * xh) * np.cos(kk * yh),
                 "dy_vv": -kk * np.sin(kk * xh) * np.sin(kk * yh),
                 "lap_vv": -2 * kk * kk * np.sin(kk * xh) * np.cos(kk * yh)}
        xpp, ypp = nd.xp
        inner_p = (np.minimum.reduce([xpp, ypp, 1 - xpp, 1 - ypp]) > 4.0 / args.spmv_K)
        exact["id_pv"] = np.sin(kk * xpp) * np.cos(kk * ypp)
        for name, (idx, w, _) in ops.items():
            y = P.ell_apply(idx, w, fv).cpu().numpy()
            amp = {"dx_vv": kk, "dy_vv": kk, "lap_vv": 2 * kk * kk, "id_pv": 1.0}[name]
            msk = inner_p if name == "id_pv" else inner
            d = np.abs(y - exact[name]) / amp
            errs[name] = {"interior": float(np.max(d[msk])), "all_rows": float(np.max(d))}
        res[f"k=2pi*{k_wave}"] = errs
    out["trunc_err_rel_amp"] = res
    gbs = {}
    x64 = dev_tensor(ri.random_vector(xv.shape[1], 1), dev)
    x32 = P.cast_f32(x64)
    # Launch shape of each operator size and precision chosen by the
    # library's autotuner (rbf_ell_autotune); the timings below use it.
    tune = {}
    for prec in ("fp64", "fp32"):
        for name in ("dx_vv", "id_pv"):
            idx, w, _ = ops[name]
            w = P.cast_f32(w) if prec == "fp32" else w
            shape, ms = P.ell_autotune(idx, w, x32 if prec == "fp32" else x64, reps=20)
            tune[f"{name}_{prec}"] = {"shape": P.ELL_SHAPES[shape], "us": ms[shape] * 1e3,
                                      "default_us": ms[0] * 1e3}
    out["ell_autotune"] = tune
    for prec in ("fp64", "fp32"):
        for name, (idx, w, ncols) in ops.items():
            rows = idx.shape[1]
            if prec == "fp32":
                w = P.cast_f32(w)
                x = x32
                bytes_row = 28 * (4 + 4) + 4 + 4  # idx + w + x (once) + y
            else:
                x = x64
                bytes_row = 28 * (4 + 8) + 8 + 8
            y = torch.empty(rows, dtype=w.dtype, device=dev)
            for _ in range(10):
                P.ell_apply(idx, w, x, y)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.spmv_reps):
                P.ell_apply(idx, w, x, y)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / args.spmv_reps
            gbs[f"{name}_{prec}"] = {"us": ms * 1e3, "GB/s": bytes_row * rows / (ms * 1e-3) / 1e9}
    out["ell_apply"] = gbs
    # Transposed product z = D_x^VV^T y: structure built once (timed as
    # set-up), weights permuted into column order once per precision, then
    # applications timed like the forward products.
    idx, w, ncols = ops["dx_vv"]
    rows = idx.shape[1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = P.ell_transpose(idx, ncols)
    torch.cuda.synchronize()
    tr = {"build_ms": (time.perf_counter() - t0) * 1e3}
    for prec in ("fp64", "fp32"):
        ww = T.weights(w if prec == "fp64" else P.cast_f32(w))
        y = x64 if prec == "fp64" else x32
        vb = 8 if prec == "fp64" else 4
        z = torch.empty(ncols, dtype=ww.dtype, device=dev)
        for _ in range(10):
            T.apply(ww, y, z)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.spmv_reps):
            T.apply(ww, y, z)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.spmv_reps
        # src + wt per entry, y once per row, colptr + z per column.
        nbytes = 28 * rows * (4 + vb) + rows * vb + ncols * (8 + vb)
        tr[prec] = {"us": ms * 1e3, "GB/s": nbytes / (ms * 1e-3) / 1e9}
    out["ell_apply_transpose_dx_vv"] = tr
    return out


def cpu_baseline(args):
    """The oracle on a bounded sample of the headline workload (same node
    kind, Re, dt, jitter, stencils; h = 1/cpu_K): set-up (kNN, weights,
    SuperLU factorisations of both implicit matrices, as the paper factors
    them once) untimed, then `cpu_steps` timed steps (triangular solves and
    CSR products)."""
    import rbf_inputs as ri
    from oracle import cavity as ocav
    nd = ri.hex_cavity_nodes(args.cpu_K, args.jitter, args.seed)
    u_bc, v_bc = ri.cavity_bc(nd.v_tag)
    t0 = time.perf_counter()
    orc = ocav.CavityOracle(nd, u_bc, v_bc, args.re, args.dt)
    setup = time.perf_counter() - t0
    s = orc.initial_state()
    t0 = time.perf_counter()
    s = orc.run(args.cpu_steps, s)
    el = time.perf_counter() - t0
    return {"value": (nd.n_v + nd.n_p) * args.cpu_steps / el, "unit": "node-steps/s",
            "cores": 1, "kind": "oracle", "host_cpu_count": os.cpu_count(),
            "sample": f"the headline cavity kind at h=1/{args.cpu_K} (N={nd.n_v}, M={nd.n_p}, "
                      f"Re={args.re:g}, dt={args.dt:g}, jitter {args.jitter}h), "
                      f"{args.cpu_steps} steps from rest ({el:.1f} s) after an untimed set-up "
                      f"of {setup:.1f} s (stencils, weights, SuperLU factorisations).  The "
                      "timed steps are SuperLU triangular solves and SciPy CSR products, both "
                      "single-threaded, so one core does the work whatever the host has.  The "
                      "oracle's cost per node-step grows with the grid (fill of the LU "
                      f"factors), so this overstates its rate at h=1/{args.K}",
            "setup_s": setup, "u_abs_max": float(np.abs(s.u).max())}


def mixed_run(P, args, dev, st64, value64):
    """The same steps with RBF_PRECISION_MIXED; fields compared with the FP64
    run after the same number of steps."""
    import torch
    S, st, _, setup_s = cavity_setup(P, args, dev, precision="mixed")
    run = Run(S, st)
    run.advance(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.clear()
    stats = run.advance(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S.close()
    value = (S.N + S.M) * args.steps / el
    err = {}
    for key in ("u", "v", "p", "p_tilde"):
        a, b = st[key], st64[key]
        err[key] = float((a - b).abs().max() / b.abs().max())
    log(f"mixed: {value:.3e} node-steps/s, rel err vs FP64 {err}")
    return {"value": value, "unit": "node-steps/s", "ms_per_step": el / args.steps * 1e3,
            "speedup_vs_fp64": value / value64,
            "poisson_steps_per_step": stats.poisson_iters / max(1, args.steps),
            "rel_err_vs_fp64": err, "setup_s": setup_s,
            "what": "pressure: each FGMRES restart cycle is one iterative-refinement step "
                    "(FP64 residual from FP64 weights; FP32 weights, vectors, smoother and "
                    "lattice transforms inside, FP64 dots); weights, viscous solve, "
                    "projection and tolerance FP64"}


def batch_run(P, args, dev):
    """Concurrent stepping of many small independent cavities."""
    import torch
    rng = np.random.default_rng(args.seed + 2206)
    inst = []
    t0 = time.perf_counter()
    for b in range(args.batch):
        n_target = rng.uniform(5000.0, 60000.0)
        K = max(8, int(round(math.sqrt(n_target / 3.47))))  # kind 2: N ~ 3.47 K^2
        re = math.exp(rng.uniform(math.log(100.0), math.log(5000.0)))
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            sub = argparse.Namespace(**vars(args))
            sub.K, sub.re, sub.dt, sub.seed = K, re, 0.08 / K, args.seed + 1 + b
            S, st, _, _ = cavity_setup(P, sub, dev)
        inst.append({"S": S, "st0": st, "K": K, "re": re, "stream": s})
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    nodes = sum(x["S"].N + x["S"].M for x in inst)
    log(f"batch: {len(inst)} cavities, {nodes} nodes, setup {setup_s:.1f}s")
    solvers = [x["S"] for x in inst]

    def fresh():
        out = []
        for x in inst:
            with torch.cuda.stream(x["stream"]):
                out.append({k: (v.clone() if isinstance(v, torch.Tensor) else v)
                            for k, v in x["st0"].items()})
        torch.cuda.synchronize()
        return out

    P.step_batch(solvers, fresh(), 2, nthreads=args.batch_threads)  # warm-up
    res = {}
    for label, nt in (("sequential", 1), ("concurrent", args.batch_threads)):
        states = fresh()
        t0 = time.perf_counter()
        try:
            stats, codes = P.step_batch(solvers, states, args.batch_steps, nthreads=nt)
        except P.RbfError as e:  # an instance that failed keeps its last committed step
            stats, codes = e.stats, e.statuses
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        done = sum((x["S"].N + x["S"].M) * s.steps_done for x, s in zip(inst, stats))
        res[label] = (el, states, stats, codes, done)
        log(f"batch {label} ({nt} threads): {el:.3f}s, {done / el:.3e} node-steps/s")
    same = all(torch.equal(a[k], b[k]) for a, b in zip(res["sequential"][1], res["concurrent"][1])
               for k in ("u", "v", "p", "p_tilde", "cu_prev", "cv_prev"))
    el_s, el_c = res["sequential"][0], res["concurrent"][0]
    codes = res["concurrent"][3]
    failed = [{"instance": b, "K": inst[b]["K"], "re": inst[b]["re"], "status": codes[b],
               "steps_done": res["concurrent"][2][b].steps_done}
              for b in range(len(inst)) if codes[b] != 0]
    its = [s.poisson_iters / max(1, s.steps_done) for s in res["concurrent"][2]]
    for x in inst:
        x["S"].close()
    return {"instances": len(inst), "nodes_total": nodes,
            "K_range": [min(x["K"] for x in inst), max(x["K"] for x in inst)],
            "re_range": [min(x["re"] for x in inst), max(x["re"] for x in inst)],
            "steps": args.batch_steps, "threads": args.batch_threads, "setup_s": setup_s,
            "sequential_node_steps_per_s": res["sequential"][4] / el_s,
            "concurrent_node_steps_per_s": res["concurrent"][4] / el_c,
            "speedup": el_s / el_c, "bit_identical": bool(same),
            "failed": failed,
            "poisson_iters_per_step_mean": float(np.mean(its)),
            "what": "independent near-equilateral cavities (node kind 2), one stream each, "
                    "rbf_step_batch"}


def shedding_stats(series, dt):
    """Mean and amplitude of C_D, amplitude of C_L and the Strouhal number
    St = f D / U (D = U = 1) from the second half of a force series, f from
    the upward zero crossings of C_L - mean (linear interpolation); None
    when fewer than three crossings."""
    if len(series) < 8:
        return None
    half = series[len(series) // 2:]
    t = np.array([r["t"] for r in half])
    cd = np.array([r["C_D"] for r in half])
    cl = np.array([r["C_L"] for r in half])
    c = cl - cl.mean()
    up = [t[i] - c[i] * (t[i + 1] - t[i]) / (c[i + 1] - c[i])
          for i in range(len(c) - 1) if c[i] < 0.0 <= c[i + 1]]
    if len(up) < 3:
        return None
    period = (up[-1] - up[0]) / (len(up) - 1)
    return {"St": float(1.0 / period), "C_D_mean": float(cd.mean()),
            "C_D_amp": float(0.5 * (cd.max() - cd.min())),
            "C_L_amp": float(0.5 * (cl.max() - cl.min())), "periods": len(up) - 1,
            "window_t": [float(t[0]), float(t[-1])]}


def cylinder_run(P, args, dev):
    """Flow past a cylinder (Sec. 5.2) on the graded channel nodes of
    rbf_inputs.cylinder_nodes (channel [-10, 30] x [-10, 10], spacing 0.02
    on the cylinder): uniform inflow, symmetry sides, convective outflow,
    start from U_0 = (1, 0) plus `cyl_perturb` times a smooth transverse
    blob behind the cylinder (v = eps exp(-((x - 1.5)^2 + y^2)), which seeds
    the shedding that the paper's asymmetric grids seed by themselves);
    `cyl_steps` timed steps after 5, drag and lift (rbf_solver_forces,
    Simpson's rule) every 10 steps, and the shedding statistics of the
    second half of the run when it holds three or more periods."""
    import torch
    import rbf_inputs as ri
    nd = ri.cylinder_nodes()
    xv, xp = dev_tensor(nd.xv, dev), dev_tensor(nd.xp, dev)
    grid = {"xv": xv, "xp": xp, "v_tag": torch.from_numpy(nd.v_tag).to(dev),
            "p_tag": torch.from_numpy(nd.p_tag).to(dev), "p_normal": dev_tensor(nd.p_normal, dev)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ops = build_ops(P, xv, xp)
    u_bc = np.where(nd.v_tag == 3, 1.0, 0.0)
    S = P.Solver(grid, ops, dev_tensor(u_bc, dev), dev_tensor(np.zeros(nd.n_v), dev),
                 args.cyl_re, args.cyl_dt, u_conv=1.0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    x, y = nd.xv
    u0 = np.where(nd.v_tag == 1, 0.0, 1.0)
    v0 = np.where(nd.v_tag == 0, args.cyl_perturb * np.exp(-((x - 1.5) ** 2 + y ** 2)), 0.0)
    st = S.new_state(dev_tensor(u0, dev), dev_tensor(v0, dev))
    out = {"workload": f"cylinder D=1 in [-10,30]x[-10,10], N={S.N} V + M={S.M} P graded from "
                       f"0.02 on the cylinder, Re={args.cyl_re:g}, dt={args.cyl_dt:g}, uniform "
                       "inflow, symmetry sides, convective outflow, start from U_0 = (1, 0) + "
                       f"{args.cyl_perturb:g} transverse blob",
           "setup_s": setup_s, "aux_lattice_cells": S.info()["aux_cells"],
           "aux_smooth_weight": S.info()["aux_smooth_weight"]}
    series = []
    try:
        S.step(st, 5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = 0
        for c in range(0, args.cyl_steps, 10):
            n = min(10, args.cyl_steps - c)
            s = S.step(st, n)
            iters += s.poisson_iters
            fx, fy = S.forces(grid, st)
            series.append({"step": int(st["step"]), "t": st["step"] * args.cyl_dt,
                           "C_D": 2.0 * fx, "C_L": 2.0 * fy})
            if len(series) % 500 == 0:
                log(f"cylinder step {st['step']}: C_D {2 * fx:.4f} C_L {2 * fy:.4f}")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out.update({"value": (S.N + S.M) * args.cyl_steps / el, "unit": "node-steps/s",
                    "ms_per_step": el / args.cyl_steps * 1e3, "steps": args.cyl_steps,
                    "poisson_fgmres_steps_per_step": iters / args.cyl_steps,
                    "final_state": S.diagnostics(st)})
    except P.RbfError as e:
        out["error"] = f"step {st['step']}: {e}"
    keep = max(1, len(series) // 50)
    out["forces"] = series[::keep] + (series[-1:] if series and (len(series) - 1) % keep else [])
    out["shedding"] = shedding_stats(series, args.cyl_dt)
    S.close()
    log(f"cylinder: {out.get('value', float('nan')):.3e} node-steps/s, last "
        f"{series[-1] if series else None}, shedding {out['shedding']}")
    return out


def lattice_run(P, args, dev):
    """The right-triangle lattice cavity (node kind 0) of the same h with the
    lattice fast-Poisson preconditioner and BiCGSTAB (context only: the
    scheme is unstable on that layout beyond about 490 steps from rest)."""
    import torch
    S, st, _, setup_s = cavity_setup(P, args, dev, kind=0, precond="lattice")
    S.step(st, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = S.step(st, args.lattice_steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"value": (S.N + S.M) * args.lattice_steps / el, "unit": "node-steps/s",
           "ms_per_step": el / args.lattice_steps * 1e3, "steps": args.lattice_steps,
           "poisson_iters_per_step": s.poisson_iters / args.lattice_steps,
           "final_state": S.diagnostics(st),
           "workload": f"right-triangle lattice cavity h=1/{args.K} (N={S.N} V + M={S.M} P), "
                       f"Re={args.re:g}, dt={args.dt:g}, steps 10-{10 + args.lattice_steps} "
                       "from rest, BiCGSTAB with the lattice preconditioner"}
    S.close()
    log(f"lattice: {out['value']:.3e} node-steps/s")
    return out


def kernel_bytes(M, prof, steps_per_cycle):
    """Algorithmic bytes per launch of the sampled pressure-solve kernels
    (28-point rows: int32 index + FP64 weight per entry)."""
    jbar = max(0.0, (steps_per_cycle - 1.0) / 2.0)  # mean Arnoldi index in a cycle
    return {
        # product (idx + w, z gathered once, w written) + dots with jbar + 1
        # basis vectors
        "k_fg_av2": M * (28 * 12 + 8 + 8 + 8 * (jbar + 1)),
        # idx + w, t1 gathered once, y, dinv, z written
        "k_aux_post2": M * (28 * 12 + 8 + 8 + 8 + 8),
        # w read and written, jbar + 1 basis vectors, dinv read, W w written
        "k_fg_gs<2>": M * (8 + 8 + 8 + 8 + 8 * (jbar + 1)),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding "
              "is designed but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2206_06495_amd as P
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        a = torch.empty(32 * 2 ** 20, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)  # 256 MiB read + 256 MiB write per copy
        torch.cuda.synchronize()
        del a, b
    log("cavity setup K =", args.K)
    S, st, nodes, setup_s = cavity_setup(P, args, dev)
    N, M = S.N, S.M
    info = S.info()
    log(f"N={N} M={M} setup {setup_s:.2f}s (aux lattice {info['aux_cells']} cells); "
        f"warmup {args.warmup} steps")
    run = Run(S, st)
    run.advance(args.warmup)
    torch.cuda.synchronize()
    S.profile(args.prof_every)
    log("timed steps", args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.clear()
    stats = run.advance(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = S.profile(0)
    value = (N + M) * args.steps / el
    umax = float(st["u"].abs().max())
    diag = S.diagnostics(st)
    steps_per_ts = stats.poisson_iters / max(1, args.steps)
    cycles = stats.last.last_poisson.restarts + 1 if stats.last else 1
    log(f"{el:.3f}s  {value:.3e} node-steps/s  pressure FGMRES steps per time step "
        f"{steps_per_ts:.1f}  |u|max {umax:.3f}")
    # Dominant kernel among the sampled ones (each runs once per FGMRES step).
    names = {"spmv": "k_fg_av2", "smooth": "k_aux_post2", "gs": "k_fg_gs<2>",
             "gemm": "k_pc_gemm<0>"}
    nbytes = kernel_bytes(M, prof, steps_per_ts / max(1, cycles))
    kern = {}
    for slot, name in names.items():
        ms, cnt = prof[slot]
        if cnt:
            kern[name] = {"avg_us": ms * 1e3, "samples": cnt}
            if name in nbytes:
                kern[name]["bytes_per_launch"] = nbytes[name]
                kern[name]["GB/s"] = nbytes[name] / (ms * 1e-3) / 1e9
    dom = max(kern, key=lambda k: kern[k]["avg_us"]) if kern else None
    if dom == "k_pc_gemm<0>":
        n = info["aux_cells"] - 1
        flops = 2.0 * n ** 3
        ach = flops / (kern[dom]["avg_us"] * 1e-6) / 1e12
        roof = {"kernel": f"{dom} (auxiliary-lattice transform, {n}^3 FP64 product)",
                "bound": "mfma", "achieved": ach, "peak": FP64_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_MFMA_PEAK_TFLOPS, "traffic": None}
    elif dom:
        ach = kern[dom]["GB/s"]
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": TRAFFIC_BYTES.get(dom),
                "avg_us": kern[dom]["avg_us"], "samples": kern[dom]["samples"],
                "bytes_per_launch": kern[dom]["bytes_per_launch"]}
    else:
        roof = None
    out = {
        "metric": "node-steps/s + ELL SpMV HBM GB/s, mixed/batched vs FP64 at rel err 1e-8",
        "value": value, "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"lid-driven cavity Re={args.re:g} dt={args.dt:g} h=1/{args.K} on "
                               f"the seed-jittered near-equilateral triangulation (node kind 2, "
                               f"N={N} V + M={M} P nodes, jitter {args.jitter}h, seed "
                               f"{args.seed}), 28-point PHS r^7 + cubic, FP64, pressure by "
                               "FGMRES with the two-level auxiliary-lattice preconditioner",
                   "poisson_rtol": args.rtol_p, "helmholtz_rtol": args.rtol_h,
                   "setup_s": setup_s, "aux_lattice_cells": info["aux_cells"],
                   "aux_smooth_weight": info["aux_smooth_weight"],
                   "poisson_fgmres_steps_per_step": steps_per_ts,
                   "helmholtz_iters_per_step": stats.helmholtz_iters / max(1, args.steps),
                   "last_poisson_rel_residual": stats.last.last_poisson.rel_residual
                   if stats.last else None,
                   "final_state": diag, "u_abs_max": umax,
                   "pressure_kernels": kern},
        "roofline": roof,
    }
    S.close()
    if not args.no_mixed:
        log("mixed precision: same workload, FP32 cycles inside FP64 refinement")
        out["mixed"] = mixed_run(P, args, dev, st, value)
    del st
    torch.cuda.empty_cache()
    if not args.no_lattice:
        log("right-triangle lattice cavity K =", args.K)
        out["lattice"] = lattice_run(P, args, dev)
        torch.cuda.empty_cache()
    if not args.no_cylinder:
        log("cylinder flow")
        out["cylinder"] = cylinder_run(P, args, dev)
        torch.cuda.empty_cache()
    if args.batch > 0:
        log("concurrent instances:", args.batch)
        out["batch"] = batch_run(P, args, dev)
        torch.cuda.empty_cache()
    if not args.no_spmv:
        log("operator bench K =", args.spmv_K)
        out["spmv"] = spmv_bench(P, args, dev)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
