#!/usr/bin/env python
"""Throughput of the LABFM hot path on one MI355X.

One benchmark step is the whole periodic Taylor-Green job of the workload:
stencil search, weight construction (six operators, filter coefficients),
time step, then the RK steps of the run (four fused RK stages and one filter
pass each). All inputs (node positions, spacings, orders, initial state) are
resident in device memory before the timed region starts.

value  = node-updates per second per RK stage for the whole job
         (nodes x 4 stages x RK steps / job time), float64 path;
roofline: the fused RK stage kernel, algorithmic bytes per launch
         (44 K + 104 bytes per node, K = mean neighbours) over its mean
         duration from HIP events recorded on its stream during the timed
         region; traffic: HBM bytes per launch from the committed rocprofv3
         FETCH_SIZE / WRITE_SIZE summary of the same kernel, if it was taken
         on the current source;
graph_replayed_steps: the same RK steps replayed from a HIP graph;
build: stencil search and weight build of the workload (HIP events) and
         the build's algorithmic FP64 FLOP/s against the FP64 peak and the
         FP64 MFMA rate measured on the device (labfm_mfma_f64_rate);
stream_copy: measured bandwidth of plain streaming kernels on 1 GiB (a
         device copy, read + write, and a read-only sum; best of 5 each), the
         measured ceiling the stage kernel's bandwidth is also compared with;
f32w, f32_comp: the same job with float32 weights (float64 sums, or
         float32 compensated Dot2 sums), speedup and per-field error against
         the float64 run;
mixed_precision_4m: the 4,194,304-node workload (m = 8): float64 build,
         then its 500 graph-replayed RK steps in float64 and in compensated
         float32, run rates, stage-kernel fractions, per-field and
         per-operator errors of the float32 run against the float64 run;
cpu_baseline: the FP64 CPU oracle on a bounded sample of the same workload.

Launch shapes of the gather kernels are autotuned on the workload before the
timed region. --profile-run runs a 1 GiB calibration copy, the tuner and one
job per precision, for rocprofv3 counter passes.

Other lines (each one JSON line of its own, same conventions):
--poiseuille  the channel between no-slip walls (boundary strips, wall
              equation) at 1.05M nodes, with the start-up's convergence;
--lagrangian  the Lagrangian mode on the workload's nodes (stencils and
              weights rebuilt at every RK stage);
--adjoint     the adjoint of the filtered RK loop (65,536 nodes, 200 steps);
--stencil-opt the stencil optimisation on the workload and 1.0M graded nodes;
--batched-build the weight build of the 1.0M graded nodes (orders 10 / 6 / 4,
              uneven stencils) in each distribution and the autotuner's.

Prints one JSON line.
"""
import os

# the oracle's BLAS runs single-threaded so the core count is known
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("OMP_NUM_THREADS", "1")

import argparse  # noqa: E402
import json  # noqa: E402
import math  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-updates/s per RK stage + HBM roofline frac, FP32-comp vs FP64 at stated err"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# the solver jobs time one RK step in this many with HIP events around each
# launch (the kernel means of the roofline); the others run without events
TIMING_EVERY = 10


def log(msg: str) -> None:
    """A progress line on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed benchmark steps (whole jobs)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tg512_m8")
    ap.add_argument("--rk-steps", type=int, default=None,
                    help="RK steps per job (default: the workload's run length)")
    ap.add_argument("--no-f32", action="store_true", help="skip the float32 compensated job")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-4m", action="store_true",
                    help="skip the 4,194,304-node mixed-precision leg (tg2048_m8)")
    ap.add_argument("--launch-shapes", default=None,
                    help="pin the gather kernels' launch shapes instead of tuning: JSON "
                         "{prec: {kernel: [lanes_per_node, flags]}} inline, or the path of a "
                         "JSON file holding it under 'launch_shapes' (a bench output line)")
    ap.add_argument("--poiseuille", action="store_true",
                    help="print the channel (no-slip walls) line instead: Poiseuille start-up\n"
                         "throughput at 1.05M nodes, convergence at t* = 1, oracle baseline")
    ap.add_argument("--adjoint", action="store_true",
                    help="print the adjoint line instead: the gradient of a loss of the state\n"
                         "after 200 steps (tg256_m6) with respect to the initial state")
    ap.add_argument("--lagrangian", action="store_true",
                    help="print the Lagrangian-mode line instead: nodes advected, stencils and\n"
                         "weights rebuilt at every RK stage, on the workload's node set")
    ap.add_argument("--stencil-opt", action="store_true",
                    help="instead of the solver job: time the stencil optimisation on the "
                         "workload and on the 1.0M-node graded set (one JSON line)")
    ap.add_argument("--batched-build", action="store_true",
                    help="instead of the solver job: the weight build of the 1.0M-node graded "
                         "set (orders 10 / 6 / 4) in each distribution (one JSON line)")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for rocprofv3: a 1 GiB copy, then warmup jobs only")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is designed, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2102_02019_amd import inputs, labfm, profiling

    dev = torch.device("cuda:0")
    if args.stencil_opt:
        print(json.dumps(stencil_opt_bench(args, inputs, labfm, torch, np, dev)))
        return
    if args.batched_build:
        print(json.dumps(batched_build_bench(args, inputs, labfm, torch, np, dev)))
        return
    if args.poiseuille:
        print(json.dumps(poiseuille_bench(args, inputs, labfm, torch, np, dev)))
        return
    if args.lagrangian:
        print(json.dumps(lagrangian_bench(args, inputs, labfm, torch, np, dev)))
        return
    if args.adjoint:
        print(json.dumps(adjoint_bench(args, inputs, labfm, torch, np, dev)))
        return
    wl = inputs.WORKLOADS[args.workload]
    rk_steps = wl.steps if args.rk_steps is None else args.rk_steps
    nodes = wl.nodes()
    N = nodes.n
    prm = inputs.taylor_green_params(L=wl.L)
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y, L=wl.L)
    q0_h = np.concatenate([np.log(rho), u, v])

    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    x, y, h, s, m = T(nodes.x), T(nodes.y), T(nodes.h), T(nodes.s), T(nodes.m)
    q0 = T(q0_h)
    q = torch.empty_like(q0)
    ws = labfm.rk_workspace(N, dev)
    torch.cuda.synchronize()

    if args.profile_run:
        # a plain copy of known size calibrates the HBM byte counters
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()

    def tune(prec):
        """Autotune the gather kernels' launch shapes on this workload (outside
        the timed region); the timed jobs then use the installed shapes."""
        rp, col = labfm.build_neighbours(x, y, h, nodes.box)
        ops = labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=True)
        return labfm.tune(ops, q0, prec, reps=10, workspace=ws)

    setup_ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def job(prec):
        setup_ev[0].record()
        rp, col = labfm.build_neighbours(x, y, h, nodes.box)
        ops = labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=(prec != labfm.F64))
        q.copy_(q0)
        dt = labfm.time_step(q, s, prm.c2, prm.mu, visc=wl.visc_coef)
        setup_ev[1].record()
        tm = labfm.rk_step(q, ops, prm, dt, rk_steps, prec=prec, workspace=ws, timing=True,
                           timing_every=TIMING_EVERY)
        # the stencil search, build, tiles and dt of this job (the RK call
        # synchronises, so both events have completed)
        tm["setup_ms"] = setup_ev[0].elapsed_time(setup_ev[1])
        return ops, tm

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            job(prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tms = []
        ops = None
        for _ in range(steps):
            ops, tm = job(prec)
            tms.append(tm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return ops, tms, (t1 - t0) / max(1, steps)

    precs = {"f64": labfm.F64, "f32w": labfm.F32W, "f32_comp": labfm.F32_COMP}
    if args.no_f32:
        precs = {"f64": labfm.F64}
    log(f"workload {wl.name}: {N} nodes, m = {wl.m}, {rk_steps} RK steps per job")
    if args.launch_shapes:
        tuned = pinned_shapes(args.launch_shapes, precs, labfm)
    else:
        tuned = {key: tune(p) for key, p in precs.items()}
    # the stage kernels the jobs launch (names as a profiler shows them)
    use_tiles = True
    rp0, _ = labfm.build_neighbours(x, y, h, nodes.box)
    nnz0 = int(rp0[-1].item())
    names = {k: stage_kernel_name(v["stage"], use_tiles, PREC_TAG[k], nnz0)
             for k, v in tuned.items()}

    if args.profile_run:
        # the tuned shapes stay installed; the counters of the last dispatches
        # of each stage kernel belong to these jobs
        job(labfm.F64)
        if not args.no_f32:
            job(labfm.F32W)
            job(labfm.F32_COMP)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": "done", "workload": wl.name, "nodes": N,
                          "rk_steps": rk_steps, "stage_kernels": names, "launch_shapes": tuned}))
        return

    log(f"launch shapes {json.dumps(tuned)}; timing {args.steps} float64 jobs")
    ops, tms, sec = timed(labfm.F64, args.steps, args.warmup)
    q64 = q.clone()
    nnz = ops.nnz
    kbar = nnz / N
    launches = sum(t["stage_launches"] for t in tms)
    stage_ms = sum(t["stage_ms"] for t in tms) / launches
    filter_ms = sum(t["filter_ms"] for t in tms) / max(1, sum(t["filter_launches"] for t in tms))
    value = N * 4 * rk_steps / sec
    bytes_stage = (44.0 * kbar + 104.0) * N
    bytes_filter = (12.0 * kbar + 56.0) * N
    achieved = bytes_stage / (stage_ms * 1e-3) / 1e9
    traffic = profiling.load_traffic("rk_stage_f64", wl.name, names["f64"])
    status_hist = np.bincount(ops.status.cpu().numpy().astype(np.int64), minlength=5).tolist()
    finite = bool(torch.isfinite(q64).all().item())

    # full RK steps replayed from a HIP graph (4 stages + filter), per stage
    q.copy_(q0)
    dt = labfm.time_step(q, s, prm.c2, prm.mu, visc=wl.visc_coef)
    labfm.rk_step(q, ops, prm, dt, 10, workspace=ws, use_graph=True)
    torch.cuda.synchronize()
    q.copy_(q0)
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    labfm.rk_step(q, ops, prm, dt, rk_steps, workspace=ws, use_graph=True)
    torch.cuda.synchronize()
    graph_s = time.perf_counter() - tg0
    graph_equal = bool(torch.equal(q, q64))

    log("graph replay done; build and copy rates")
    build = build_rate(labfm, torch, np, nodes, x, y, h, s, m)
    stream = stream_copy_rate(torch, dev)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "nodes": N, "order_m": wl.m,
                   "mean_neighbours": round(kbar, 2), "rk_steps_per_job": rk_steps,
                   "filter": "every step", "domain": "[0,2pi)^2 periodic, +/-0.3s jitter",
                   "flow": "Taylor-Green, Re=100, Ma=0.1"},
        "roofline": {"bound": "hbm", "kernel": names["f64"], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "bytes_per_node_stage": 44.0 * kbar + 104.0,
                     "algorithmic_bytes_per_launch": bytes_stage,
                     "mean_launch_ms": stage_ms, "launches": launches,
                     "frac_of_stream_copy": achieved / stream["GBs"]},
        "stream_copy": stream,
        "stage_kernel_node_updates_per_s": N / (stage_ms * 1e-3),
        "graph_replayed_steps": {"node_updates_per_s": N * 4 * rk_steps / graph_s,
                                 "ms_per_rk_step": graph_s * 1e3 / rk_steps,
                                 "bitwise_equal_to_eager": graph_equal},
        "filter_kernel": {"mean_launch_ms": filter_ms,
                          "achieved_GBs": bytes_filter / (filter_ms * 1e-3) / 1e9,
                          "frac": bytes_filter / (filter_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "bytes_per_node": 12.0 * kbar + 56.0},
        "build": build,
        "setup_ms_per_job": sum(t["setup_ms"] for t in tms) / len(tms),
        "timed_launches": f"one RK step in {TIMING_EVERY} of every job carries HIP events",
        "final_state_finite": finite,
        "node_status_histogram": status_hist,
        "launch_shapes": tuned,
    }

    for prec, key in ((labfm.F32W, "f32w"), (labfm.F32_COMP, "f32_comp")):
        if args.no_f32:
            break
        log(f"timing {args.steps} {key} jobs")
        ops32, tms32, sec32 = timed(prec, args.steps, args.warmup)
        q32 = q.clone()
        st32 = sum(t["stage_ms"] for t in tms32) / sum(t["stage_launches"] for t in tms32)
        a64 = q64.cpu().numpy().reshape(3, -1)
        a32 = q32.cpu().numpy().reshape(3, -1)
        err = {
            "rho": float(np.linalg.norm(np.exp(a32[0]) - np.exp(a64[0])) / np.linalg.norm(np.exp(a64[0]))),
            "u": float(np.linalg.norm(a32[1] - a64[1]) / np.linalg.norm(a64[1])),
            "v": float(np.linalg.norm(a32[2] - a64[2]) / np.linalg.norm(a64[2])),
        }
        # per-operator error of one application on the initial velocity
        uu = q0[N:2 * N].contiguous()
        d64 = labfm.apply_operators(ops32, uu, 0x1F, labfm.F64).cpu().numpy()
        d32 = labfm.apply_operators(ops32, uu, 0x1F, prec).cpu().numpy()
        op_err = {labfm.OPS[d]: float(np.linalg.norm(d32[d] - d64[d]) / np.linalg.norm(d64[d]))
                  for d in range(5)}
        b32 = (24.0 * kbar + 104.0) * N
        out[key] = {
            "value": N * 4 * rk_steps / sec32,
            "ms_per_step": sec32 * 1e3,
            "speedup_job": sec / sec32,
            "speedup_stage_kernel": stage_ms / st32,
            "stage_mean_launch_ms": st32,
            "stage_achieved_GBs": b32 / (st32 * 1e-3) / 1e9,
            "stage_frac": b32 / (st32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "stage_kernel": names[key],
            "bytes_per_node_stage": 24.0 * kbar + 104.0,
            "final_state_rel_err_vs_f64": err,
            "operator_rel_err_vs_f64": op_err,
        }

    if not args.no_f32 and not args.no_4m:
        log("mixed-precision leg on 4,194,304 nodes")
        out["mixed_precision_4m"] = mixed_precision_bench(inputs, labfm, torch, np, dev)

    if not args.no_cpu_baseline:
        log("oracle baseline on the host cores")
        out["cpu_baseline"] = cpu_baseline(wl, rk_steps, N)
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(wl, rk_steps, N)

    print(json.dumps(out))


PREC_TAG = {"f64": "F64", "f32w": "F32W", "f32_comp": "F32Comp"}


def stencil_opt_bench(args, inputs, labfm, torch, np, dev):
    """The stencil optimisation (h_i from 2.8 s_i shrunk by 0.99 while the
    node passes the residual and amplitude tests) on the workload's nodes and
    on the 1.0M-node graded set: time (HIP events around the call, which
    includes its h0 stencil search), tests per node, the FP64 FLOP/s of the
    node systems it builds, neighbours before and after; and the oracle's
    per-node loop timed on a sample of the workload."""
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    res = {"metric": "stencil optimisation: nodes/s and FP64 FLOP/s of the per-node systems",
           "runs": []}
    sets = [(args.workload, inputs.WORKLOADS[args.workload].nodes()),
            ("holes1m", inputs.graded_holes(1_000_000, seed=3))]
    for name, nodes in sets:
        x, y, s, m = T(nodes.x), T(nodes.y), T(nodes.s), T(nodes.m)
        h0 = (inputs.STENCIL_H0_OVER_S * s).contiguous()
        labfm.optimise_stencils(x, y, s, m, nodes.box, h0=h0)  # warm-up
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        h, k = labfm.optimise_stencils(x, y, s, m, nodes.box, h0=h0)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        rp0, _ = labfm.build_neighbours(x, y, h0, nodes.box)
        rp1, _ = labfm.build_neighbours(x, y, h, nodes.box)
        rpu, _ = labfm.build_neighbours(x, y, T(nodes.h), nodes.box)
        K0 = np.diff(rp0.cpu().numpy()).astype(np.float64)
        kk = k.cpu().numpy().astype(np.float64)
        tests = kk + 2.0  # the accepted scales and the one that failed
        fl = float(np.sum(tests * build_flops(nodes.m.astype(np.float64), K0)))
        res["runs"].append({
            "nodes": nodes.n, "set": name, "orders": sorted(set(int(v) for v in nodes.m)),
            "ms": ms, "nodes_per_s": nodes.n / (ms * 1e-3),
            "tests_per_node": float(tests.mean()),
            "gflop": fl / 1e9, "achieved_TFLOPs": fl / (ms * 1e-3) / 1e12,
            "frac_fp64_peak": fl / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "h_over_s_mean": float((h / s).mean().item()),
            "neighbours_mean": {"h0": float(K0.mean()),
                                "uniform_h_over_s": float(rpu[-1].item() / nodes.n),
                                "optimised": float(rp1[-1].item() / nodes.n)}})
    # the oracle's loop on a sample of the workload (one core)
    from oracle import labfm_oracle as O

    nodes = sets[0][1]
    sample = list(range(0, nodes.n, nodes.n // 24))
    t0 = time.perf_counter()
    O.optimise_stencils(nodes.x, nodes.y, nodes.s, nodes.m, nodes.box,
                        h0=O.STENCIL_H0_OVER_S * nodes.s, nodes=sample)
    t1 = time.perf_counter()
    res["cpu_baseline"] = {"value": len(sample) / (t1 - t0), "unit": "nodes/s", "cores": 1,
                           "kind": "oracle", "sample": f"{len(sample)} nodes of {sets[0][0]}"}
    return res


def batched_build_bench(args, inputs, labfm, torch, np, dev):
    """The weight build of the 1.0M-node graded set (24 holes, orders 10 / 6
    / 4 by wall distance, uneven stencils; node arrays and stencils resident
    on the device): each distribution timed with HIP events (best of 3), its
    FP64 FLOP/s against the spec peak and the measured MFMA rate, the
    autotuner's choice; and the oracle's build timed on a sample of nodes of
    every order."""
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    nodes = inputs.graded_holes(1_000_000, seed=3)
    log(f"graded set: {nodes.n} nodes")
    x, y, h, s, m = T(nodes.x), T(nodes.y), T(nodes.h), T(nodes.s), T(nodes.m)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    rp, col = labfm.build_neighbours(x, y, h, nodes.box)
    ev[1].record()
    torch.cuda.synchronize()
    nb_ms = ev[0].elapsed_time(ev[1])
    K = np.diff(rp.cpu().numpy()).astype(np.float64)
    fl = float(np.sum(build_flops(nodes.m.astype(np.float64), K)))
    measured = labfm.mfma_f64_rate()
    modes = {"rows-in-registers": labfm.BUILD_ROWS, "workgroup-per-node": labfm.BUILD_BLOCK,
             "persistent": labfm.BUILD_PERSISTENT, "per-order-class": labfm.BUILD_BUCKETED}
    runs = {}
    status = None
    try:
        for name, mode in modes.items():
            labfm.set_build_config(mode)
            labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=True, tiles=False)
            best = None
            for _ in range(3):
                ev[0].record()
                ops = labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=True,
                                          tiles=False)
                ev[1].record()
                torch.cuda.synchronize()
                t = ev[0].elapsed_time(ev[1])
                best = t if best is None else min(best, t)
            tf = fl / (best * 1e-3) / 1e12
            runs[name] = {"ms": best, "achieved_TFLOPs": tf, "frac": tf / FP64_PEAK_TFLOPS,
                          "frac_of_measured_mfma": tf / measured}
            log(f"{name}: {best:.2f} ms")
            if mode == labfm.BUILD_ROWS:
                status = np.bincount(ops.status.cpu().numpy().astype(np.int64), minlength=5)
        labfm.set_build_config(0)
        labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=True, tiles=False, tune=True)
        tuned = labfm.build_weights.last_tuned
    finally:
        labfm.set_build_config(0)
    names = {v: k for k, v in modes.items()}
    names[labfm.BUILD_WAVE] = "wavefront-per-node"
    dominant = runs["rows-in-registers"]
    res = {"metric": "batched weight build: FP64 FLOP/s, orders 10 / 6 / 4 in one call",
           "value": dominant["achieved_TFLOPs"], "unit": "TFLOP/s", "dtype": "f64",
           "config": {"workload": "holes1m", "nodes": nodes.n,
                      "orders": {int(o): int(np.sum(nodes.m == o)) for o in np.unique(nodes.m)},
                      "mean_neighbours": float(K.mean())},
           "gflop": fl / 1e9, "neighbours_ms": nb_ms,
           "roofline": {"bound": "mfma", "kernel": "build_rows_kernel<10>",
                        "achieved": dominant["achieved_TFLOPs"], "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": dominant["frac"], "traffic": None},
           "measured_mfma_f64_TFLOPs": measured, "distributions": runs,
           "autotuner": {"choice": names.get(tuned[0], str(tuned[0])),
                         "workgroups_per_cu": tuned[1], "ms": tuned[2]},
           "node_status_histogram": [int(v) for v in status]}
    # the oracle's build on a sample of every order (one core)
    from oracle import labfm_oracle as O

    sample = []
    for o in np.unique(nodes.m):
        idx = np.nonzero(nodes.m == o)[0]
        sample += [int(i) for i in idx[:: max(1, idx.size // 8)][:8]]
    t0 = time.perf_counter()
    srp, scol = O.neighbours_rows(nodes.x, nodes.y, nodes.h, nodes.box, sample)
    O.weights(nodes.x, nodes.y, nodes.h, nodes.s, nodes.m, srp, scol, nodes.box, nodes=sample)
    t1 = time.perf_counter()
    res["cpu_baseline"] = {"value": len(sample) / (t1 - t0), "unit": "nodes/s", "cores": 1,
                           "kind": "oracle",
                           "sample": f"{len(sample)} nodes, 8 of each order: stencils + weights"}
    return res


def poiseuille_bench(args, inputs, labfm, torch, np, dev, n_x=1024, rk_steps=400):
    """Channel between no-slip walls (5-node strips, 1D LABFM rows, wall
    equation) driven from rest by a body force at Re = 10, Ma = 0.05: the
    whole job (stencils, weights, boundary weights, dt, RK steps with the
    filter; node arrays resident on the device beforehand) at n_x = 1024
    (1.05M nodes, m = 6 in the bulk), the stage kernel against the HBM
    roofline (44 K + 120 bytes per node: the periodic stage's 44 K + 104 plus
    the wall normal), the velocity error against the analytic start-up at the
    final time, the convergence at t* = 1 for s = H/20, H/40, H/80, and the
    oracle's steps timed on the 20 x 21 channel.

    At n_x = 1024 the viscous term sets dt; the paper's coefficient 0.4 puts
    the stiffest viscous mode outside the RK stability interval there (as for
    the 2048^2 periodic case), so this job uses 0.25. The convergence runs are
    convective-limited and use the paper's 0.4."""
    from paper_2102_02019_amd import profiling

    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    P = inputs.POISEUILLE
    flow = P.flow()

    def resident(nodes, strips):
        return tuple(T(a) for a in (nodes.x, nodes.y, nodes.h, nodes.s, nodes.m,
                                    strips.column, strips.normal))

    def setup(box, dev_arrays):
        x, y, h, s, m, column, normal = dev_arrays
        rp, col = labfm.build_neighbours(x, y, h, box)
        ops = labfm.build_weights(x, y, h, s, m, box, rp, col)
        labfm.boundary_weights(x, y, h, s, box, ops, column, normal)
        return ops

    def dt_for(q, s_dev, t_end, visc):
        """dt = t_end / ceil(t_end / dt_max), dt_max from eq. dt on q."""
        dt_max = labfm.time_step(q, s_dev, flow.c2, flow.mu, conv=1.0, visc=visc)
        n = max(1, int(math.ceil(t_end / dt_max - 1e-9)))
        return t_end / n, n

    def vel_err(g, y, t):
        ua = inputs.poiseuille_startup(y, t, P.H, P.mu / P.rho0, P.gx)
        return float(math.sqrt(np.sum((g[1] - ua) ** 2 + g[2] ** 2) / np.sum(ua * ua)))

    def run(nx, t_star):
        nodes, st = inputs.channel(nx)
        arr = resident(nodes, st)
        ops = setup(nodes.box, arr)
        q = torch.zeros(3 * nodes.n, dtype=torch.float64, device=dev)
        dt, n = dt_for(q, arr[3], P.time(t_star), 0.4)
        labfm.rk_step(q, ops, flow, dt, n, use_graph=True, check_finite=True)
        return nodes, vel_err(q.cpu().numpy().reshape(3, -1), nodes.y, dt * n), dt * n

    big, strips = inputs.channel(n_x)
    N = big.n
    arrays = resident(big, strips)
    if args.profile_run:
        # a plain copy of known size calibrates the HBM byte counters
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
    # launch shapes tuned on this node set, outside the timed region
    ops = setup(big.box, arrays)
    q = torch.zeros(3 * N, dtype=torch.float64, device=dev)
    labfm.tune(ops, q, labfm.F64, reps=10)
    torch.cuda.synchronize()
    if args.profile_run:
        # one short job with the tuned shape: its stage launches are the last
        # dispatches of the stage kernel in this process
        qq = torch.zeros(3 * N, dtype=torch.float64, device=dev)
        dt = labfm.time_step(qq, arrays[3], flow.c2, flow.mu, conv=1.0, visc=0.25)
        labfm.rk_step(qq, ops, flow, dt, args.rk_steps or 10)
        torch.cuda.synchronize()
        return {"profile_run": "done", "workload": "channel1024_m6", "nodes": N,
                "rk_steps": args.rk_steps or 10,
                "stage_kernel": stage_kernel_name(labfm.get_launch_config(
                    labfm.KERNEL_STAGE, labfm.F64, N, ops.nnz), True, "F64", ops.nnz)}

    def job():
        o = setup(big.box, arrays)
        qq = torch.zeros(3 * N, dtype=torch.float64, device=dev)
        dt = labfm.time_step(qq, arrays[3], flow.c2, flow.mu, conv=1.0, visc=0.25)
        tm = labfm.rk_step(qq, o, flow, dt, rk_steps, timing=True, timing_every=TIMING_EVERY)
        return o, qq, dt, tm

    job()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tms = []
    for _ in range(args.steps):
        o, qq, dt, tm = job()
        tms.append(tm)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / max(1, args.steps)
    launches = sum(t["stage_launches"] for t in tms)
    stage_ms = sum(t["stage_ms"] for t in tms) / launches
    kbar = o.nnz / N
    bytes_stage = (44.0 * kbar + 120.0) * N
    achieved = bytes_stage / (stage_ms * 1e-3) / 1e9
    g = qq.cpu().numpy().reshape(3, -1)
    err_big = vel_err(g, big.y, dt * rk_steps)
    conv = []
    for nx in (20, 40, 80):
        nn, err, t_end = run(nx, 1.0)
        conv.append({"n_x": nx, "nodes": nn.n, "t_star": t_end * P.U0 / P.H, "vel_rel_err": err})
    rates = [math.log(conv[k]["vel_rel_err"] / conv[k + 1]["vel_rel_err"]) / math.log(2.0)
             for k in range(2)]
    stage_name = stage_kernel_name(labfm.get_launch_config(labfm.KERNEL_STAGE, labfm.F64, N,
                                                           o.nnz), True, "F64", o.nnz)
    out = {
        "metric": "Poiseuille channel: node-updates/s per RK stage + stage-kernel HBM roofline",
        "value": N * 4 * rk_steps / sec, "unit": "node-updates/s", "dtype": "f64",
        "config": {"workload": "channel1024_m6", "nodes": N, "order_bulk": 6, "order_walls": 4,
                   "mean_neighbours": round(kbar, 2), "rk_steps_per_job": rk_steps,
                   "dt_coefficients": {"conv": 1.0, "visc": 0.25},
                   "flow": "Poiseuille start-up, Re=10, Ma=0.05, from rest",
                   "domain": "[0,1) periodic x [0,1] walls, 5-node strips, +/-0.3s bulk jitter"},
        "ms_per_job": sec * 1e3,
        "roofline": {"bound": "hbm", "kernel": stage_name, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiling.load_traffic("rk_stage_walls_f64", "channel1024_m6",
                                                       stage_name),
                     "bytes_per_node_stage": 44.0 * kbar + 120.0,
                     "algorithmic_bytes_per_launch": bytes_stage, "mean_launch_ms": stage_ms,
                     "launches": launches},
        "final_time": dt * rk_steps, "vel_rel_err_at_final_time": err_big,
        "final_state_finite": bool(np.all(np.isfinite(g))),
        "convergence_t1": conv, "rates_t1": rates,
    }
    out["cpu_baseline"] = poiseuille_cpu_baseline(inputs, np)
    return out


def poiseuille_cpu_baseline(inputs, np, n_x=20, n_steps=60):
    """The oracle's filtered RK steps of the 20 x 21 channel on one core."""
    from oracle import boundaries_oracle as B

    P = inputs.POISEUILLE
    flow = P.flow()
    small, strips = inputs.channel(n_x)
    W = B.channel_weights(small, strips)
    dt, _ = B.poiseuille_steps(small, P, flow, 1.0)
    z = np.zeros(small.n)
    c0 = time.perf_counter()
    B.channel_run(z, z, z, W, flow, dt, n_steps)
    c1 = time.perf_counter()
    return {"value": small.n * 4 * n_steps / (c1 - c0), "unit": "node-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_steps} filtered RK steps of the {n_x} x {n_x + 1} channel "
                      f"({small.n} nodes)"}


def lagrangian_bench(args, inputs, labfm, torch, np, dev, rk_steps=10):
    """Lagrangian mode on the workload's nodes (Taylor-Green): each job
    advances positions and fields by rk_steps RK steps with stencils and
    weights rebuilt at every stage's positions (4 builds per step plus one),
    inputs resident on the device. Reports node-updates/s per RK stage, the
    share of the job in the builds, the weight build kernel against the FP64
    peak (the dominant kernel: its algorithmic flops over the mean of HIP
    events around labfm_build_weights on the moved nodes), the Eulerian job's
    rate on the same nodes for comparison, and the oracle's Lagrangian step on
    a 32 x 32 sample."""
    wl = inputs.WORKLOADS[args.workload]
    nodes = wl.nodes()
    N = nodes.n
    prm = inputs.taylor_green_params(L=wl.L)
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y, L=wl.L)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    x0, y0, h, s, m = T(nodes.x), T(nodes.y), T(nodes.h), T(nodes.s), T(nodes.m)
    q0 = T(np.concatenate([np.log(rho), u, v]))
    x, y, q = torch.empty_like(x0), torch.empty_like(y0), torch.empty_like(q0)
    dt = labfm.time_step(q0, s, prm.c2, prm.mu, visc=wl.visc_coef)
    rp, _ = labfm.build_neighbours(x0, y0, h, nodes.box)
    cap = int(1.5 * rp[-1].item()) + 1024
    ws = torch.empty(labfm.lib().labfm_lagrangian_workspace_bytes(N, cap), dtype=torch.uint8,
                     device=dev)

    def job():
        x.copy_(x0)
        y.copy_(y0)
        q.copy_(q0)
        return labfm.lagrangian_step(x, y, q, h, s, m, nodes.box, prm, dt, rk_steps,
                                     nnz_capacity=cap, workspace=ws)

    job()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        stats.append(job())
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / max(1, args.steps)
    build_ms = sum(st["build_ms"] for st in stats) / len(stats)
    stage_ms = sum(st["stage_ms"] for st in stats) / len(stats)
    finite = bool(torch.isfinite(q).all().item())
    # the build kernel on the moved nodes (final positions of the last job)
    br = build_rate(labfm, torch, np, nodes_at(inputs, nodes, x, y), x, y, h, s, m)
    # the Eulerian job on the same nodes (stencils and weights once)
    x.copy_(x0)
    y.copy_(y0)
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for _ in range(args.steps):
        rp, col = labfm.build_neighbours(x0, y0, h, nodes.box)
        ops = labfm.build_weights(x0, y0, h, s, m, nodes.box, rp, col)
        q.copy_(q0)
        labfm.rk_step(q, ops, prm, dt, rk_steps)
    torch.cuda.synchronize()
    e_sec = (time.perf_counter() - e0) / max(1, args.steps)
    out = {
        "metric": "Lagrangian LABFM: node-updates/s per RK stage with a stencil and weight "
                  "rebuild at every stage",
        "value": N * 4 * rk_steps / sec, "unit": "node-updates/s", "dtype": "f64",
        "config": {"workload": wl.name + "_lagrangian", "nodes": N, "order_m": wl.m,
                   "rk_steps_per_job": rk_steps, "builds_per_job": stats[-1]["builds"],
                   "flow": "Taylor-Green, Re=100, Ma=0.1, nodes advected"},
        "ms_per_job": sec * 1e3,
        "build_share": build_ms / (sec * 1e3),
        "build_ms_per_build": build_ms / stats[-1]["builds"],
        "stage_and_filter_ms_per_job": stage_ms,
        "max_nnz": stats[-1]["max_nnz"], "nnz_capacity": cap,
        "final_state_finite": finite,
        "roofline": {"bound": "mfma", "kernel": build_kernel_name(labfm, wl.m),
                     "achieved": br["achieved_TFLOPs"], "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": br["frac"], "traffic": None,
                     "gflop_per_build": br["gflop"], "mean_build_ms": br["weights_ms"]},
        "eulerian_same_nodes": {"value": N * 4 * rk_steps / e_sec, "ms_per_job": e_sec * 1e3,
                                "lagrangian_slowdown": sec / e_sec},
    }
    out["cpu_baseline"] = lagrangian_cpu_baseline(inputs, np, wl)
    return out


def adjoint_bench(args, inputs, labfm, torch, np, dev, ckpt_every=20):
    """The adjoint of the filtered RK loop on tg256_m6 (65,536 nodes, m = 6,
    200 steps, a checkpoint every 20 steps): forward run, then the gradient
    of a scalar loss of the final state with respect to the initial state
    (labfm_rk_adjoint: each checkpoint segment recomputed once, then per step
    the filter adjoint and four stage adjoints, each a forward gather and a
    transposed gather). Inputs resident on the device. Reports the adjoint's
    node-updates/s (N x 4 stages x steps / its time), its cost relative to the
    forward run, and the pass's algorithmic bytes per second. At this size a
    stage's data (~180 MB) stays in the 256 MB last-level cache, so the rate is
    a cache-resident one, not an HBM roofline (per-kernel times:
    profiles/adjoint_tg256_m6_kernel_trace.md)."""
    wl = inputs.TG256_M6
    nodes = wl.nodes()
    N = nodes.n
    steps = wl.steps
    prm = inputs.taylor_green_params(L=wl.L)
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y, L=wl.L)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    x, y, h, s, m = T(nodes.x), T(nodes.y), T(nodes.h), T(nodes.s), T(nodes.m)
    q0 = T(np.concatenate([np.log(rho), u, v]))
    rp, col = labfm.build_neighbours(x, y, h, nodes.box)
    ops = labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, rowsum=True)
    labfm.build_transpose(ops)
    dt = labfm.time_step(q0, s, prm.c2, prm.mu, visc=wl.visc_coef)
    qbar = T(np.random.default_rng(5).standard_normal(3 * N))
    q = torch.empty_like(q0)
    ws = labfm.rk_workspace(N, dev)

    def forward():
        q.copy_(q0)
        labfm.rk_step(q, ops, prm, dt, steps, workspace=ws)

    def adjoint():
        return labfm.rk_adjoint(q0, qbar, ops, prm, dt, steps, ckpt_every)

    forward()
    g = adjoint()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd_ms, adj_ms = [], []
    for _ in range(max(1, args.steps)):
        ev[0].record()
        forward()
        ev[1].record()
        g = adjoint()
        ev[2].record()
        torch.cuda.synchronize()
        fwd_ms.append(ev[0].elapsed_time(ev[1]))
        adj_ms.append(ev[1].elapsed_time(ev[2]))
    fwd, adj = sum(fwd_ms) / len(fwd_ms), sum(adj_ms) / len(adj_ms)
    kbar = ops.nnz / N
    # algorithmic bytes per node and step: the recomputed forward step
    # (4 stages of 44K + 104 and a filter of 12K + 56), four forward gathers
    # (44K + 216) and four transposed gathers (44K + 240), and the filter
    # adjoint (12K + 80)
    per_node_step = (4 * (44 * kbar + 104) + 12 * kbar + 56 + 4 * (44 * kbar + 216)
                     + 4 * (44 * kbar + 240) + 12 * kbar + 80)
    achieved = per_node_step * N * steps / (adj * 1e-3) / 1e9
    return {
        "metric": "adjoint of the filtered RK loop: node-updates/s (N x 4 stages x steps / time)",
        "value": N * 4 * steps / (adj * 1e-3), "unit": "node-updates/s", "dtype": "f64",
        "config": {"workload": wl.name + "_adjoint", "nodes": N, "order_m": wl.m,
                   "mean_neighbours": round(kbar, 2), "rk_steps": steps,
                   "checkpoint_every": ckpt_every, "filter": "every step"},
        "forward_ms": fwd, "adjoint_ms": adj, "adjoint_over_forward": adj / fwd,
        "gradient_finite": bool(torch.isfinite(g).all().item()),
        "pass_bytes": {"bound": "cache-resident gathers", "achieved_GBs": achieved,
                       "bytes_per_node_step": per_node_step,
                       "note": "about 180 MB per stage at this size: last-level cache"},
        "cpu_baseline": adjoint_cpu_baseline(inputs, np, wl),
    }


def adjoint_cpu_baseline(inputs, np, wl, n_side=32, n_steps=10):
    """The oracle's adjoint (explicit sparse operator matrices, every forward
    state stored) on a 32 x 32 sample with the workload's order and h/s, one
    core, scaled per node-update."""
    from oracle import labfm_oracle as O

    nodes = inputs.jittered_lattice(n_side, L=wl.L, seed=wl.seed, m=wl.m)
    prm = inputs.taylor_green_params(L=wl.L)
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y, L=wl.L)
    rp, col = O.neighbours(nodes.x, nodes.y, nodes.h, nodes.box)
    W = O.weights_batched(nodes.x, nodes.y, nodes.h, nodes.s, wl.m, rp, col, nodes.box)
    W.update(row_ptr=rp, col=col)
    dt = O.time_step(nodes.s, np.log(rho), u, v, prm, visc_coef=wl.visc_coef)
    qbar = tuple(np.random.default_rng(5).standard_normal((3, nodes.n)))
    c0 = time.perf_counter()
    O.rk_adjoint(np.log(rho), u, v, W, prm, dt, n_steps, qbar)
    c1 = time.perf_counter()
    return {"value": nodes.n * 4 * n_steps / (c1 - c0), "unit": "node-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"adjoint of {n_steps} filtered steps on a {n_side}x{n_side} lattice "
                      f"(m={wl.m})"}


def nodes_at(inputs, nodes, x, y):
    """The node set with positions taken from device tensors x, y."""
    return inputs.NodeSet(x.cpu().numpy(), y.cpu().numpy(), nodes.s, nodes.h, nodes.m, nodes.box,
                          nodes.meta)


def lagrangian_cpu_baseline(inputs, np, wl, n_side=32, n_steps=1):
    """The oracle's Lagrangian step (5 stencil and weight builds, 4 stages, the
    filter) on a 32 x 32 sample with the workload's order and h/s, one core."""
    from oracle import labfm_oracle as O
    from oracle import lagrangian_oracle as G

    nodes = inputs.jittered_lattice(n_side, L=wl.L, seed=wl.seed, m=wl.m)
    prm = inputs.taylor_green_params(L=wl.L)
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y, L=wl.L)
    dt = O.time_step(nodes.s, np.log(rho), u, v, prm, visc_coef=wl.visc_coef)
    c0 = time.perf_counter()
    G.lagrangian_run(nodes.x, nodes.y, np.log(rho), u, v, nodes.h, nodes.s, nodes.m, nodes.box,
                     prm, dt, n_steps)
    c1 = time.perf_counter()
    return {"value": nodes.n * 4 * n_steps / (c1 - c0), "unit": "node-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_steps} Lagrangian step of a {n_side}x{n_side} lattice (m={wl.m}): "
                      f"5 builds, 4 stages, filter"}


def mixed_precision_bench(inputs, labfm, torch, np, dev, eager_steps=10):
    """The mixed-precision workload: 2048^2 = 4,194,304 jittered nodes, m = 8,
    weights built in float64 and stored in float32 as well, then the
    workload's 500 filtered RK steps replayed from a HIP graph in float64 and
    in the compensated float32 precision (Dot2 sums), each timed once around
    the replay (after a short captured warm-up). The per-field relative
    errors of the float32 run are taken against the float64 run of the same
    weights, and the per-operator errors of one application on the initial
    velocity. Stage-kernel durations come from a short eager run with HIP
    events. The launch shapes are the ones installed for the main job."""
    wl = inputs.TG2048_M8
    nodes = wl.nodes()
    N = nodes.n
    prm = inputs.taylor_green_params(L=wl.L)
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y, L=wl.L)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    x, y, h, s, m = T(nodes.x), T(nodes.y), T(nodes.h), T(nodes.s), T(nodes.m)
    q0 = T(np.concatenate([np.log(rho), u, v]))
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    rp, col = labfm.build_neighbours(x, y, h, nodes.box)
    ev[1].record()
    ops = labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=True)
    ev[2].record()
    torch.cuda.synchronize()
    nnz = ops.nnz
    kbar = nnz / N
    K = np.diff(rp.cpu().numpy()).astype(np.float64)
    gflop = float(np.sum(build_flops(float(wl.m), K))) / 1e9
    build_ms = ev[1].elapsed_time(ev[2])
    statuses = np.bincount(ops.status.cpu().numpy().astype(np.int64), minlength=5).tolist()
    ws = labfm.rk_workspace(N, dev)
    q = torch.empty_like(q0)
    dt = labfm.time_step(q0, s, prm.c2, prm.mu, visc=wl.visc_coef)
    res, state = {}, {}
    for key, prec, bpn in (("f64", labfm.F64, 44.0 * kbar + 104.0),
                           ("f32_comp", labfm.F32_COMP, 24.0 * kbar + 104.0)):
        log(f"{wl.name} {key}: {eager_steps} eager steps, then {wl.steps} graph-replayed steps")
        q.copy_(q0)
        tm = labfm.rk_step(q, ops, prm, dt, eager_steps, prec=prec, workspace=ws, timing=True)
        st = tm["stage_ms"] / tm["stage_launches"]
        fl = tm["filter_ms"] / max(1, tm["filter_launches"])
        q.copy_(q0)
        labfm.rk_step(q, ops, prm, dt, 5, prec=prec, workspace=ws, use_graph=True)
        q.copy_(q0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        labfm.rk_step(q, ops, prm, dt, wl.steps, prec=prec, workspace=ws, use_graph=True)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        state[key] = q.view(3, -1).cpu().numpy()
        gbs = bpn * N / (st * 1e-3) / 1e9
        res[key] = {"node_updates_per_s": N * 4 * wl.steps / sec,
                    "ms_per_rk_step": sec * 1e3 / wl.steps,
                    "run_s": sec,
                    "stage_mean_launch_ms": st, "filter_mean_launch_ms": fl,
                    "bytes_per_node_stage": bpn,
                    "stage_achieved_GBs": gbs, "stage_frac": gbs / HBM_PEAK_GBS}
    a64, a32 = state["f64"], state["f32_comp"]

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    res["f32_comp"]["final_state_rel_err_vs_f64"] = {
        "rho": rel(np.exp(a32[0]), np.exp(a64[0])), "u": rel(a32[1], a64[1]),
        "v": rel(a32[2], a64[2])}
    uu = q0[N:2 * N].contiguous()
    d64 = labfm.apply_operators(ops, uu, 0x1F, labfm.F64).cpu().numpy()
    d32 = labfm.apply_operators(ops, uu, 0x1F, labfm.F32_COMP).cpu().numpy()
    res["f32_comp"]["operator_rel_err_vs_f64"] = {
        labfm.OPS[d]: rel(d32[d], d64[d]) for d in range(5)}
    res["f32_comp"]["speedup_run"] = res["f64"]["run_s"] / res["f32_comp"]["run_s"]
    res["f32_comp"]["speedup_stage_kernel"] = (res["f64"]["stage_mean_launch_ms"]
                                               / res["f32_comp"]["stage_mean_launch_ms"])
    decay = math.exp(-2.0 * prm.mu * dt * wl.steps)
    return {"workload": wl.name, "nodes": N, "order_m": wl.m, "mean_neighbours": round(kbar, 2),
            "rk_steps": wl.steps, "dt": dt, "graph_replayed": True,
            "neighbours_ms": ev[0].elapsed_time(ev[1]), "build_ms": build_ms,
            "build_TFLOPs": gflop / build_ms, "node_status_histogram": statuses,
            "f64_u_decay_vs_exact": float(np.abs(a64[1]).max() / (np.abs(u).max() * decay)),
            **res}


def pinned_shapes(spec, precs, labfm):
    """Install the launch shapes given on the command line (see --launch-shapes)."""
    text = spec if spec.lstrip().startswith("{") else open(spec).read().strip().splitlines()[-1]
    d = json.loads(text)
    d = d.get("launch_shapes", d)
    kernels = {"stage": labfm.KERNEL_STAGE, "filter": labfm.KERNEL_FILTER,
               "apply": labfm.KERNEL_APPLY}
    out = {}
    for key, p in precs.items():
        out[key] = {}
        for kname, kid in kernels.items():
            lpn, flags = d[key][kname][0], d[key][kname][1]
            labfm.set_launch_config(kid, p, lpn, flags)
            out[key][kname] = [lpn, flags, None]
    return out


def stage_kernel_name(shape, tiled, prec_tag, nnz=None):
    """Name pattern of the fused RK stage kernel for a tuned launch shape
    (lanes per node, flags); '*' joins the parts of a profiler's name. With
    tiles the library launches the quad-loading variant for the float32
    weights (four edges per lane load, rows at the padded stride) and the
    pair-loading variant for float64 (its last template argument tells an odd
    stencil count)."""
    lpn, flags = shape[0], shape[1]
    kern = "rk_stage_kernel"
    tail = ""
    if tiled:
        if prec_tag in ("F32W", "F32Comp"):
            kern = "rk_stage_tiled_quad_kernel"
        else:
            kern = "rk_stage_tiled_packed_kernel"
            if nnz is not None:
                tail = ", " + ("true" if nnz % 2 else "false")
    return f"{kern}<{lpn}, {flags}, *{prec_tag}{tail}>"


def stream_copy_rate(torch, dev, reps=5):
    """Measured bandwidth ceilings of plain streaming kernels on 1 GiB of
    float64 (torch's own): a device copy (read + write, 2 GiB moved) and a
    sum (read only, 1 GiB), each the best of reps, timed with events on
    torch's stream (the one both run on). GBs is the larger of the two."""
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    r = a.sum()

    def best_ms(fn):
        best = float("inf")
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    nb = float(a.numel() * a.element_size())
    t_copy = best_ms(lambda: b.copy_(a))
    t_sum = best_ms(lambda: torch.sum(a, 0, out=r))
    del a, b, r
    copy_gbs = 2.0 * nb / (t_copy * 1e-3) / 1e9
    read_gbs = nb / (t_sum * 1e-3) / 1e9
    best = max(copy_gbs, read_gbs)
    return {"GBs": best, "copy_GBs": copy_gbs, "copy_ms": t_copy, "read_GBs": read_gbs,
            "read_ms": t_sum, "bytes": nb, "frac_of_hbm_peak": best / HBM_PEAK_GBS}


def build_kernel_name(labfm, m):
    """The weight-build kernel the library launches for order m under the
    installed distribution: one wavefront per node with the rows in
    registers for orders up to 10 (the default), else the workgroup-per-node
    kernel."""
    mode = labfm.get_build_config()[0]
    if mode == labfm.BUILD_ROWS and m <= 10:
        return "build_rows_kernel<%d>" % m
    return "build_block_kernel<%d>" % m


def build_flops(m, K):
    """Algorithmic FP64 flops of one node's weight build: assembly 2Kn^2,
    LU (2/3)n^3, six solves 12n^2, weights 12Kn, basis K(3n + 4m + 20)."""
    n = (m * m + 3 * m) // 2
    return 2 * K * n * n + (2.0 / 3.0) * n ** 3 + 12 * n * n + 12 * K * n + K * (3 * n + 4 * m + 20)


def build_rate(labfm, torch, np, nodes, x, y, h, s, m):
    """Stencil search and weight build of the workload, timed with HIP events
    on the current stream (best of 3), and the weight build's FP64 FLOP/s."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    best = None
    for _ in range(3):
        ev[0].record()
        rp, col = labfm.build_neighbours(x, y, h, nodes.box)
        ev[1].record()
        labfm.build_weights(x, y, h, s, m, nodes.box, rp, col, f32=True, tiles=False)
        ev[2].record()
        torch.cuda.synchronize()
        t = (ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]))
        best = t if best is None or t[1] < best[1] else best
    K = np.diff(rp.cpu().numpy()).astype(np.float64)
    fl = float(np.sum(build_flops(nodes.m.astype(np.float64), K)))
    mode = labfm.get_build_config()
    measured = labfm.mfma_f64_rate()
    return {"neighbours_ms": best[0], "weights_ms": best[1], "gflop": fl / 1e9,
            "achieved_TFLOPs": fl / (best[1] * 1e-3) / 1e12,
            "peak_TFLOPs": FP64_PEAK_TFLOPS,
            "frac": fl / (best[1] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "measured_mfma_f64_TFLOPs": measured,
            "frac_of_measured_mfma": fl / (best[1] * 1e-3) / 1e12 / measured,
            "distribution": {1: "wavefront-per-node", 2: "workgroup-per-node",
                             3: "persistent", 4: "per-order-class",
                             5: "rows-in-registers"}.get(mode[0], str(mode[0])),
            "kernel": build_kernel_name(labfm, int(np.max(nodes.m)))}


def _oracle_sample(args):
    """One oracle sample run (in a worker process): the same steps as
    cpu_baseline on a 64 x 64 lattice of its own seed; returns the nodes,
    the stencil + weight time and the RK time."""
    wl_name, seed, k = args
    import numpy as np

    from oracle import labfm_oracle as O
    from paper_2102_02019_amd import inputs

    wl = inputs.WORKLOADS[wl_name]
    nodes = inputs.jittered_lattice(64, L=wl.L, seed=seed, m=wl.m)
    prm = inputs.taylor_green_params(L=wl.L)
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y, L=wl.L)
    t0 = time.perf_counter()
    rp, col = O.neighbours(nodes.x, nodes.y, nodes.h, nodes.box)
    W = O.weights_batched(nodes.x, nodes.y, nodes.h, nodes.s, wl.m, rp, col, nodes.box)
    W.update(row_ptr=rp, col=col)
    dt = O.time_step(nodes.s, np.log(rho), u, v, prm, visc_coef=wl.visc_coef)
    t1 = time.perf_counter()
    O.rk_run(np.log(rho), u, v, W, prm, dt, k)
    t2 = time.perf_counter()
    return nodes.n, t1 - t0, t2 - t1


def cpu_baseline_all_cores(wl, rk_steps, N_full):
    """The oracle on every host core: one single-threaded oracle process per
    core, each on its own 64 x 64 sample (the node set splits into
    independent pieces the way the GPU job would shard), aggregate
    throughput over the wall time of the slowest, scaled per node to the
    full job like cpu_baseline."""
    import multiprocessing as mp

    cores = min(len(os.sched_getaffinity(0)), 16)
    k = 20
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_sample, [(wl.name, 100 + c, k) for c in range(cores)])
    wall = time.perf_counter() - t0
    n_tot = sum(r[0] for r in res)
    setup = max(r[1] for r in res)
    step = max(r[2] for r in res)
    setup_per_node = setup / (n_tot / cores)
    step_per_node = step / (n_tot / cores * k)
    job_s = N_full * (setup_per_node + rk_steps * step_per_node) / cores
    return {
        "value": N_full * 4 * rk_steps / job_s,
        "unit": "node-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{cores} processes x {n_tot // cores} nodes (64x64, m={wl.m}), stencils + "
                   f"weights and {k} RK steps each, {wall:.1f} s wall; scaled per node to "
                   f"{N_full} nodes and {rk_steps} steps"),
        "cpu_model": cpu_model(),
    }


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), for the CPU baselines."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, rk_steps, N_full):
    """The oracle on a 64 x 64 node sample of the workload (same order m,
    h/s and so the same stencils per node): stencil search, weight build and
    40 RK steps, timed, then scaled per node to the full job."""
    import numpy as np

    from oracle import labfm_oracle as O
    from paper_2102_02019_amd import inputs

    nodes = inputs.jittered_lattice(64, L=wl.L, seed=wl.seed, m=wl.m)
    n = nodes.n
    prm = inputs.taylor_green_params(L=wl.L)
    rho, u, v = inputs.taylor_green_state(nodes.x, nodes.y, L=wl.L)
    t0 = time.perf_counter()
    rp, col = O.neighbours(nodes.x, nodes.y, nodes.h, nodes.box)
    W = O.weights_batched(nodes.x, nodes.y, nodes.h, nodes.s, wl.m, rp, col, nodes.box)
    W.update(row_ptr=rp, col=col)
    dt = O.time_step(nodes.s, np.log(rho), u, v, prm, visc_coef=wl.visc_coef)
    t1 = time.perf_counter()
    k = 40
    O.rk_run(np.log(rho), u, v, W, prm, dt, k)
    t2 = time.perf_counter()
    setup_per_node = (t1 - t0) / n
    step_per_node = (t2 - t1) / (n * k)
    job_s = N_full * (setup_per_node + rk_steps * step_per_node)
    return {
        "value": N_full * 4 * rk_steps / job_s,
        "unit": "node-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{n} nodes (64x64, m={wl.m}): stencils + weights {t1 - t0:.1f} s, "
                   f"{k} RK steps {t2 - t1:.1f} s; scaled per node to {N_full} nodes "
                   f"and {rk_steps} steps"),
        "rk_stage_only_node_updates_per_s": 4 * n * k / (t2 - t1),
        "cpu_model": cpu_model(),
    }


if __name__ == "__main__":
    main()
