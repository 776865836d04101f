"""Benchmark of the staggered-node RBF-FD Navier-Stokes hot path on one MI355X.

Workload (one JSON line on stdout):
  * step throughput: lid-driven cavity, Re = 1e4, dt = 2e-4, h = 1/400 on the
    paper's staggered layout (P on triangulation vertices, V on edge
    midpoints: N = 480,800, M = 160,801), 28-point PHS r^7 + cubic stencils,
    FP64.  Setup (stencils, weights, system matrices) is timed separately;
    `warmup` steps run untimed, then `steps` steps are timed.  value =
    (N + M) * steps / seconds (node-steps/s).  The run restarts from the
    rest state every `segment` steps (the restore is a device copy inside the
    timed region): on this jittered node set the scheme diverges after about
    490 steps from rest (near-wall modes of the approximate projection), so
    longer runs are made of segments of the same flow.
  * operator bench: 10^6 V + 10^6 P jittered square nodes, weights for VV
    {D_x, D_y, Lap} and PV {I}, then `spmv_reps` applications of each operator
    in FP64 and FP32-stored ELL, timed with HIP events; achieved GB/s from the
    algorithmic bytes; truncation error against closed-form derivatives of
    sin(kx)cos(ky), k = 2 pi {4, 16, 64}.
  * roofline of the dominant kernel of the step: the FP64 MFMA transform
    k_pc_gemm<0> of the lattice preconditioner (2 n^3 flops per launch,
    n = K - 1), its average duration sampled with the launch's own start/end
    stamps on the solver's stream during the timed steps; the pressure SpMV
    k_pc_av (HBM bytes per launch) is reported beside it.
  * mixed: the same steps with FP32 preconditioner arrays, and the relative
    difference of the fields from the FP64 run.
  * batch: `batch` independent cavities, N uniform in [5000, 60000] V-nodes
    and Re log-uniform in [100, 5000] (dt = 0.08 h), each solver on its own
    stream, advanced `batch_steps` steps by rbf_step_batch on one host thread
    (one instance after another) and on `batch_threads` threads (concurrent),
    from the same states; aggregate node-steps/s of both and whether the
    fields agree bit for bit.
  * hex: the same Re and dt on a near-equilateral triangulation at
    h = 1/100 (no lattice, so no lattice preconditioner): the cost of the
    general path.
  * cpu_baseline: the CPU oracle (SciPy sparse LU solves) on a bounded
    sample: the same cavity at h = 1/200.
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

# Traffic beyond L2 per launch at K=400 from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE, scaled by the same counters on a plain 256 MiB copy
# (profiles/k_pc_gemm_cavity_K400_pmc.md): k_pc_gemm<0> and the pressure
# SpMV k_pc_av<28,0>.  Set to None when the kernel changes until it is
# measured again.
GEMM_TRAFFIC_BYTES = 21.96e6
SPMV_TRAFFIC_BYTES = 59.95e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--segment", type=int, default=400,
                    help="steps from rest after which the state is restored to rest")
    ap.add_argument("--K", type=int, default=400, help="cavity cells per side (h = 1/K)")
    ap.add_argument("--re", type=float, default=1e4)
    ap.add_argument("--dt", type=float, default=2e-4)
    ap.add_argument("--jitter", type=float, default=0.3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--spmv-K", type=int, default=1000)
    ap.add_argument("--spmv-reps", type=int, default=1000)
    ap.add_argument("--no-spmv", action="store_true")
    ap.add_argument("--no-hex", action="store_true",
                    help="skip the near-equilateral (non-lattice) cavity leg")
    ap.add_argument("--hex-K", type=int, default=100)
    ap.add_argument("--hex-steps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run (FP32 preconditioner transforms)")
    ap.add_argument("--cpu-K", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--prof-every", type=int, default=25)
    ap.add_argument("--rtol-p", type=float, default=1e-12)
    ap.add_argument("--rtol-h", type=float, default=1e-13)
    ap.add_argument("--batch", type=int, default=64,
                    help="independent cavities of the concurrent-instance run (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-threads", type=int, default=8)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 256 MiB device copy first (HBM counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dev_tensor(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def cavity_setup(P, args, dev, precision="fp64"):
    import torch
    nodes = P.build_nodes(0, args.K, args.jitter, args.seed)
    t0 = time.perf_counter()
    g = {k: dev_tensor(v, dev) for k, v in nodes.items()}
    ops = {"k": 28}
    for name, xq, xs, mask in (("vv", g["xv"], g["xv"], 14), ("pv", g["xp"], g["xv"], 6),
                               ("pp", g["xp"], g["xp"], 14), ("vp", g["xv"], g["xp"], 6)):
        idx = P.knn(xq, xs, 28)
        w = P.assemble_weights(xq, xs, idx, 7, 3, mask)
        ops["idx_" + name] = idx
        ops[name + "_dx"] = w[0].contiguous()
        ops[name + "_dy"] = w[1].contiguous()
        if mask & 8:
            ops[name + "_lap"] = w[2].contiguous()
        del w
    vt = nodes["v_tag"]
    u_bc = np.where(vt == 2, 1.0, 0.0)
    S = P.Solver(g, ops, dev_tensor(u_bc, dev), dev_tensor(np.zeros_like(u_bc), dev),
                 args.re, args.dt, rtol_h=args.rtol_h, rtol_p=args.rtol_p, maxit_h=2000,
                 maxit_p=200000, precision=precision)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    del ops
    st = S.new_state(dev_tensor(u_bc, dev), dev_tensor(np.zeros_like(u_bc), dev))
    return S, st, nodes, setup_s


class Run:
    """Steps of one solver in segments of `segment` steps from the rest
    state; sums the statistics of its rbf_step calls."""

    def __init__(self, S, st, segment):
        self.S, self.st, self.segment = S, st, segment
        self.rest = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in st.items()}
        self.clear()

    def clear(self):
        self.poisson_iters = self.helmholtz_iters = 0
        self.last = None
        self.restarts = 0

    def advance(self, n):
        st = self.st
        while n > 0:
            if st["step"] >= self.segment:
                for k, v in self.rest.items():
                    if hasattr(v, "copy_"):
                        st[k].copy_(v)
                    else:
                        st[k] = v
                self.restarts += 1
            k = min(n, self.segment - st["step"])
            s = self.S.step(st, k)
            self.poisson_iters += s.poisson_iters
            self.helmholtz_iters += s.helmholtz_iters
            self.last = s
            n -= k
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
            errs[name] = float(np.max(np.abs(y - exact[name])[msk]) / amp)
        res[f"k=2pi*{k_wave}"] = errs
    out["trunc_err_interior_rel_amp"] = res
    gbs = {}
    x64 = dev_tensor(ri.random_vector(xv.shape[1], 1), dev)
    x32 = P.cast_f32(x64)
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
    import rbf_inputs as ri
    from oracle import cavity as ocav
    nd = ri.cavity_nodes(args.cpu_K, args.jitter, args.seed)
    u_bc, v_bc = ri.cavity_bc(nd.v_tag)
    t0 = time.perf_counter()
    orc = ocav.CavityOracle(nd, u_bc, v_bc, args.re, args.dt)
    setup = time.perf_counter() - t0
    s = orc.initial_state()
    t0 = time.perf_counter()
    s = orc.run(args.cpu_steps, s)
    el = time.perf_counter() - t0
    return {"value": (nd.n_v + nd.n_p) * args.cpu_steps / el, "unit": "node-steps/s",
            "cores": 1, "kind": "oracle",
            "sample": f"cavity h=1/{args.cpu_K} (N={nd.n_v}, M={nd.n_p}), {args.cpu_steps} steps "
                      f"({el:.1f} s) after an untimed setup with SuperLU factorisations "
                      f"({setup:.1f} s); same Re, dt and stencils as the GPU run. The timed "
                      f"steps are SuperLU triangular solves and CSR products, single-threaded. "
                      f"The oracle's cost per node grows with K, so this overstates its rate "
                      f"at h=1/{args.K}",
            "u_abs_max": float(np.abs(s.u).max())}


def mixed_run(P, args, dev, st64, value64):
    """The same steps with RBF_PRECISION_MIXED; fields compared with the FP64
    run after the same number of steps."""
    import torch
    S, st, _, setup_s = cavity_setup(P, args, dev, precision="mixed")
    run = Run(S, st, args.segment)
    run.advance(args.warmup)
    S.profile(args.prof_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run.clear()
    stats = run.advance(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = S.profile(0)
    S.close()
    value = (S.N + S.M) * args.steps / el
    err = {}
    for key in ("u", "v", "p", "p_tilde"):
        a, b = st[key], st64[key]
        err[key] = float((a - b).abs().max() / b.abs().max())
    log(f"mixed: {value:.3e} node-steps/s, rel err vs FP64 {err}")
    n = args.K - 1
    gemm_ms = prof["gemm"][0]
    return {"value": value, "unit": "node-steps/s", "ms_per_step": el / args.steps * 1e3,
            "speedup_vs_fp64": value / value64,
            "poisson_iters_per_step": stats.poisson_iters / max(1, args.steps),
            "rel_err_vs_fp64": err, "setup_s": setup_s,
            "gemm_fp32_avg_us": gemm_ms * 1e3,
            "gemm_fp32_tflops": (2.0 * n ** 3 / (gemm_ms * 1e-3) / 1e12) if gemm_ms > 0 else None,
            "what": "FP32 lattice-preconditioner transforms (FP32 matrix cores); operators, "
                    "residuals, Krylov iteration, weights and projection FP64"}


def batch_run(P, args, dev):
    """Concurrent stepping of many small independent cavities."""
    import torch
    rng = np.random.default_rng(args.seed + 2206)
    inst = []
    t0 = time.perf_counter()
    for b in range(args.batch):
        n_target = rng.uniform(5000.0, 60000.0)
        K = max(8, int(round((-2.0 + math.sqrt(4.0 + 12.0 * n_target)) / 6.0)))  # N = 3K^2 + 2K
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
            "what": "independent lattice cavities, one stream each, rbf_step_batch"}


def hex_run(P, args, dev):
    """The general-triangulation path: the cavity on a near-equilateral
    triangulation (hexagonal rows, Delaunay edges; stable where the lattice
    is not) at the same Re and dt, which has no lattice preconditioner."""
    import torch
    import rbf_inputs as ri
    nd = ri.hex_cavity_nodes(args.hex_K)
    g = {"xv": dev_tensor(nd.xv, dev), "xp": dev_tensor(nd.xp, dev),
         "v_tag": dev_tensor(nd.v_tag, dev), "p_tag": dev_tensor(nd.p_tag, dev),
         "p_normal": dev_tensor(nd.p_normal, dev)}
    ops = {"k": 28}
    for name, xq, xs, mask in (("vv", g["xv"], g["xv"], 14), ("pv", g["xp"], g["xv"], 6),
                               ("pp", g["xp"], g["xp"], 14), ("vp", g["xv"], g["xp"], 6)):
        idx = P.knn(xq, xs, 28)
        w = P.assemble_weights(xq, xs, idx, 7, 3, mask)
        ops["idx_" + name] = idx
        ops[name + "_dx"] = w[0].contiguous()
        ops[name + "_dy"] = w[1].contiguous()
        if mask & 8:
            ops[name + "_lap"] = w[2].contiguous()
    u_bc = np.where(nd.v_tag == 2, 1.0, 0.0)
    S = P.Solver(g, ops, dev_tensor(u_bc, dev), dev_tensor(np.zeros_like(u_bc), dev), args.re,
                 args.dt, rtol_h=args.rtol_h, rtol_p=args.rtol_p, maxit_h=2000, maxit_p=200000)
    st = S.new_state(dev_tensor(u_bc, dev), dev_tensor(np.zeros_like(u_bc), dev))
    S.step(st, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = S.step(st, args.hex_steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"value": (S.N + S.M) * args.hex_steps / el, "unit": "node-steps/s",
           "ms_per_step": el / args.hex_steps * 1e3, "steps": args.hex_steps,
           "poisson_iters_per_step": s.poisson_iters / args.hex_steps,
           "lattice_precond": S.info()["lattice_precond"], "final_state": S.diagnostics(st),
           "workload": f"cavity on a near-equilateral triangulation, h = 1/{args.hex_K} "
                       f"(N={S.N} V + M={S.M} P), Re={args.re:g}, dt={args.dt:g}, "
                       "unpreconditioned pressure iteration"}
    S.close()
    log(f"hex: {out['value']:.3e} node-steps/s, {out['poisson_iters_per_step']:.0f} pressure "
        "iterations per step")
    return out


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
    log(f"N={N} M={M} setup {setup_s:.2f}s; warmup {args.warmup} steps")
    run = Run(S, st, args.segment)
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
    log(f"{el:.3f}s  {value:.3e} node-steps/s  poisson iters/step "
        f"{stats.poisson_iters / max(1, args.steps):.1f}  |u|max {umax:.3f}")
    # Dominant kernel: k_pc_gemm, the n x n x n FP64 products of the
    # preconditioner (n = K - 1); the first of the two per application is
    # sampled with its own start/end stamps.
    n = args.K - 1
    gemm_ms, gemm_cnt = prof["gemm"]
    gemm_flops = 2.0 * n ** 3
    gemm_tf = gemm_flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else None
    # Pressure SpMV k_pc_av<28, 0>: idx + w (28 each), p^ gathered (once),
    # rh read, v written.
    spmv_ms, spmv_cnt = prof["spmv"]
    spmv_bytes = M * (28 * (4 + 8) + 8 + 8 + 8)
    spmv_gbs = spmv_bytes / (spmv_ms * 1e-3) / 1e9 if spmv_ms > 0 else None
    out = {
        "metric": "node-steps/s + ELL SpMV HBM GB/s, mixed/batched vs FP64 at rel err 1e-8",
        "value": value, "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"lid-driven cavity Re={args.re:g} dt={args.dt:g} h=1/{args.K} "
                               f"(N={N} V + M={M} P nodes, jitter {args.jitter}h), "
                               "28-point PHS r^7 + cubic, FP64 BiCGSTAB with the lattice "
                               "fast-Poisson preconditioner",
                   "poisson_rtol": args.rtol_p, "helmholtz_rtol": args.rtol_h,
                   "setup_s": setup_s,
                   "poisson_iters_per_step": stats.poisson_iters / max(1, args.steps),
                   "helmholtz_iters_per_step": stats.helmholtz_iters / max(1, args.steps),
                   "last_poisson_rel_residual": stats.last.last_poisson.rel_residual
                   if stats.last else None,
                   "segment": args.segment, "restores_in_timed_steps": stats.restarts,
                   "final_state": diag,
                   "u_abs_max": umax},
        "roofline": {"kernel": f"k_pc_gemm<0> (preconditioner transform, FP64 MFMA, "
                               f"{n}x{n}x{n})",
                     "bound": "mfma", "achieved": gemm_tf, "peak": FP64_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s",
                     "frac": (gemm_tf / FP64_MFMA_PEAK_TFLOPS) if gemm_tf else None,
                     "traffic": GEMM_TRAFFIC_BYTES, "avg_us": gemm_ms * 1e3,
                     "samples": gemm_cnt, "flops_per_launch": gemm_flops},
        "spmv_roofline": {"kernel": "k_pc_av<28,0> (pressure SpMV v = A p^)", "bound": "hbm",
                          "achieved": spmv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": (spmv_gbs / HBM_PEAK_GBS) if spmv_gbs else None,
                          "traffic": SPMV_TRAFFIC_BYTES, "avg_us": spmv_ms * 1e3,
                          "samples": spmv_cnt,
                          "bytes_per_launch": spmv_bytes},
    }
    S.close()
    if not args.no_mixed:
        log("mixed precision: same workload, FP32 preconditioner transforms")
        out["mixed"] = mixed_run(P, args, dev, st, value)
    del st
    torch.cuda.empty_cache()
    if args.batch > 0:
        log("concurrent instances:", args.batch)
        out["batch"] = batch_run(P, args, dev)
        torch.cuda.empty_cache()
    if not args.no_hex:
        log("near-equilateral cavity K =", args.hex_K)
        out["hex"] = hex_run(P, args, dev)
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
