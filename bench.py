#!/usr/bin/env python3
"""Throughput of the amplitude path on one MI355X.

A "step" is one qgm_amplitudes call over the whole batch, with bitstrings,
workspace and output already resident in HBM, launched on one stream; the same
call captured in a HIP graph (qgm_graph_create) and replayed is reported beside
it.  Default workload: the 5x5 depth-25 random grid circuit (seed 201) with
1024 uniform bitstrings, planned with ordering 1 (bucket elimination along a
greedy treewidth order), which runs as one LDS-resident launch (one work-group
per bitstring, every result of the elimination tree in LDS; the factor tables
and the composed leaf tables, subtrees over few output bits for every value of
those bits, are built once per plan by its first call, whose time is reported
as plan_setup_ms).  --tree-exec 1 times the same plan with one launch per
elimination-tree level instead (results in HBM); --ordering 0 the
vertical-order path (worldline steps, autotuned kernels).

Prints one JSON line.  The roofline object is for the dominant kernel: for the
LDS-resident launch, the plan's algorithmic LDS bytes over its launch time
against the LDS rate of the chip (its HBM traffic is a few megabytes; its
flops against the FP32 vector peak are given beside); for the level launches
and the worldline steps, algorithmic bytes per launch (every input result read
once, every result written once, from the plan) against HBM; launch times from
HIP events on the stream the kernels run on.  The cpu_baseline leg times the FP64 state-vector
oracle on the host cores over the same circuit and bitstrings, and its
amplitudes give the max error of the GPU result.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
LDS_PEAK_TBS = 157.3        # 256 B/clk per CU (LDS reads and writes), 256 CUs, 2.4 GHz
LDS_HEADER = 4 * 256 + 16   # LDS bytes before the data of the LDS-resident launch (table output bits, phase)
# HBM bytes per dominant-kernel launch on the default workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000, the factors a
# plain 1 GiB copy gives), valid for the kernel source with this hash and the
# plan with these figures; for the LDS launch also its SQ_INSTS_VALU per wave.
MEASURED_TRAFFIC = {
    ("c2_5x5_d25", 0): {"bytes_per_launch": 226794653.4, "source": "kernels.hip", "sha256_16": "a72736aaae65f038"},
    ("c2_5x5_d25", 1): {"bytes_per_launch": 12430049.3, "source": "tree.hip", "sha256_16": "50fd2ea026f0b985",
                        "plan": {"bytes_per_amp": 41096, "level_launches": 5}},
    ("c2_5x5_d25", "lds"): {"bytes_per_launch": 6717849.6, "source": "tree_lds.hip", "sha256_16": "371a4a84ae1b6d6a",
                            "plan": {"lds_entries": 3540, "lds_jobs": 16, "lds_threads": 256},
                            "valu_per_wave": 694},
}
METRIC = "amplitudes/sec at max err vs FP64 oracle; % FP32-MFMA/HBM roofline; grad/sec"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2_5x5_d25")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-single-core", action="store_true", help="skip the one-core oracle timing")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary workloads (C4 gradients, C3 sliced, C5 four-circuit graph)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for the HBM byte counters)")
    ap.add_argument("--ordering", type=int, default=1,
                    help="1 bucket elimination along a greedy treewidth order (default), 0 vertical order")
    ap.add_argument("--no-autotune", action="store_true", help="ordering 0: keep the policy's kernels")
    ap.add_argument("--kernel-policy", type=int, default=0,
                    help="ordering 0: 0 auto, 1 vector ALU one row per thread, 2 FP32 matrix cores where supported")
    ap.add_argument("--section", default=None, choices=None,
                    help="run only this secondary workload (launch_forms, batch_scaling, sets, c4_grad, "
                         "per_bitstring, c3, c3_mfma, c5_graph, xeb, paper_circuits) and print its JSON, for profiling it "
                         "alone")
    ap.add_argument("--tree-exec", type=int, default=0,
                    help="ordering 1: 0 auto (LDS-resident launch when the plan fits), 1 one launch per level, "
                         "3 LDS-resident")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(bitstrings and slices would shard across GPUs with no exchange but a final sum)"}))
        return 2

    import numpy as np
    import torch
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8, "copies": 3}))
        return 0
    import paper_1712_05384_amd as Q
    from paper_1712_05384_amd import circuits as C

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.section is not None:
        if args.section not in SECTIONS:
            print(json.dumps({"error": f"unknown section {args.section}; one of {sorted(SECTIONS)}"}))
            return 2
        print(json.dumps(extras(Q, C, torch, np, torch.cuda.current_stream(dev), args, args.section)), flush=True)
        return 0
    c, bits = C.workload(args.workload)
    B = len(bits)
    t0 = time.perf_counter()
    p = Q.plan(c, kernel_policy=args.kernel_policy, ordering=args.ordering,
               **({"tree_exec": args.tree_exec} if args.ordering == 1 else {}))
    plan_s = time.perf_counter() - t0
    info = p.info(0)
    print(f"# plan: n={c.n} ordering={args.ordering} max_rank={info['max_rank']} "
          f"bytes/amp={info['bytes_per_amp']:.3g} flops/amp={info['flops_per_amp']:.3g} plan_s={plan_s:.3f}",
          file=sys.stderr, flush=True)
    gv = None if c.gate_vals is None else torch.tensor(c.gate_vals.astype(np.complex64), device=dev)
    bits_d = torch.from_numpy(bits.view(np.int64)).to(dev)
    out = torch.empty((B, 1), dtype=torch.complex64, device=dev)
    ws = torch.empty(p.workspace_bytes(B), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    kernels = None
    if args.ordering == 0 and not args.no_autotune:
        kernels = p.autotune(bits_d, gv, stream=stream)   # per-step kernel by measurement (complex64 kernels only)
        info = p.info(0)

    for _ in range(args.warmup):
        p.amplitudes(bits_d, gv, out=out, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        p.amplitudes(bits_d, gv, out=out, workspace=ws, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    # phase split from separate calls with the plan's own HIP events between
    # the phases (each event adds a few microseconds, so not in the timed loop)
    p.set_timing(True)
    for _ in range(args.steps):
        p.amplitudes(bits_d, gv, out=out, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    phases, ncalls = p.timings()
    p.set_timing(False)
    eager_ms = total_ms / args.steps
    ms_per_step = eager_ms
    value = B / (ms_per_step / 1e3)
    print(f"# timed {args.steps} calls: {eager_ms:.4f} ms/call, {value:.4g} amplitudes/s", file=sys.stderr, flush=True)

    # The one-time cost of a plan on the device: the first call of a second plan of the same circuit uploads
    # its constant tables and, for a circuit without gate values, builds its factor and composed leaf tables
    # (wall clock around that call; the kernels are already loaded)
    # (ordering 0 with autotuning: a second plan would have to be tuned again, so none; setup_ms is then a call)
    p2 = p if kernels is not None else Q.plan(c, kernel_policy=args.kernel_policy, ordering=args.ordering,
                                              **({"tree_exec": args.tree_exec} if args.ordering == 1 else {}))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p2.amplitudes(bits_d, gv, out=out, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    del p2

    # Beside it: the same call captured once in a HIP graph (qgm_graph_create) and replayed K times.
    g = Q.Graph([p], [bits_d], [gv])
    for _ in range(args.warmup):
        g.launch(stream)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        g.launch(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    graph_ms = ev0.elapsed_time(ev1) / args.steps
    assert torch.equal(g.outs[0], out), "graph replay differs from the eager call"
    del g
    print(f"# {args.steps} graph replays: {graph_ms:.4f} ms/step, {B / (graph_ms / 1e3):.4g} amplitudes/s",
          file=sys.stderr, flush=True)

    # a call that is exactly one k_tree_lds launch (no gate values: the tables are the plan's): the timed
    # region's time per call is that kernel's average launch duration on the launch stream; otherwise the
    # elimination phase's own events
    one_launch = (info["ordering"] == 1 and info.get("lds_ok") and args.tree_exec in (0, 3)
                  and not info.get("n_open") and gv is None)
    elim_ms = eager_ms if one_launch else phases[2] / max(ncalls, 1)
    roofline, cfg = dominant_kernel(args, p, info, B, elim_ms, kernels, args.tree_exec)
    roofline["launch_ms_from"] = ("the timed region (one launch per call)" if one_launch
                                  else "HIP events around the elimination phase")
    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "amplitudes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": dict({"workload": f"{c.name}: {c.rows}x{c.cols} grid, depth {c.depth()}, {B} uniform bitstrings, "
                                    f"complex64, one plan for the batch", "global_batch": B,
                        "qubits": c.n, "ordering": args.ordering, "max_rank": info["max_rank"],
                        "execution": "qgm_amplitudes launched on one stream, K calls back to back"}, **cfg),
        "graph_ms_per_call": round(graph_ms, 5),
        "graph_amplitudes_per_sec": round(B / (graph_ms / 1e3), 1),
        "phases_ms_per_call_with_events": {k: round(v / max(ncalls, 1), 5) for k, v in
                                           zip(("boundary", "tables", "elimination", "output"), phases)},
        "plan_seconds": round(plan_s, 4),
        "plan_setup_ms": round(setup_ms, 4),
        "amplitudes_per_sec_incl_plan_setup": round(B * args.steps / ((total_ms + setup_ms) / 1e3), 1),
        "roofline": roofline,
    }

    if not args.no_extras:
        result["extras"] = extras(Q, C, torch, np, stream, args)

    if not args.no_cpu_baseline and c.n <= 30:
        import oracle
        got = out.cpu().numpy()[:, 0]
        cores = len(os.sched_getaffinity(0))
        omp = os.environ.get("OMP_NUM_THREADS")
        if omp and omp.isdigit():
            cores = min(cores, int(omp))
        times = []
        ref = None
        for _ in range(args.cpu_reps):
            t = time.perf_counter()
            ref = oracle.sv_amplitudes(c.n, c.gates, c.gate_vals, bits)
            times.append(time.perf_counter() - t)
        tmed = sorted(times)[len(times) // 2]
        err = float(np.abs(got - ref).max())
        result["cpu_baseline"] = {"value": round(B / tmed, 2), "unit": "amplitudes/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": f"FP64 state vector of the same circuit (2^{c.n} entries), "
                                            f"{args.cpu_reps} full sweeps, median; each sweep yields the {B} "
                                            f"amplitudes; {tmed:.2f} s per sweep"}
        if not args.no_single_core:
            # the same oracle on one host core (OpenMP limited to one thread in a child process): the 5x5 depth-25
            # batch (one sweep) and the 4x4 depth-16 batch (64 bitstrings, five sweeps)
            import subprocess
            code = ("import json, time, oracle\n"
                    "from paper_1712_05384_amd import circuits as C\n"
                    "r = {}\n"
                    "for name, reps in (('c2_5x5_d25', 1), ('c1_4x4_d16', 5)):\n"
                    "    c, b = C.workload(name)\n"
                    "    t = time.perf_counter()\n"
                    "    for _ in range(reps):\n"
                    "        oracle.sv_amplitudes(c.n, c.gates, c.gate_vals, b)\n"
                    "    dt = (time.perf_counter() - t) / reps\n"
                    "    r[name] = {'amplitudes_per_sec': round(len(b) / dt, 2), 'seconds_per_sweep': round(dt, 4),\n"
                    "               'bitstrings': len(b)}\n"
                    "print(json.dumps(r))\n")
            env = dict(os.environ, OMP_NUM_THREADS="1")
            r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                               timeout=600)
            if r.returncode == 0:
                result["cpu_baseline"]["single_core"] = dict(json.loads(r.stdout.strip().splitlines()[-1]),
                                                             note="FP64 state-vector oracle, one thread")
        result["max_abs_err"] = err
        result["max_abs_err_x_2^(n/2)"] = err * 2 ** (c.n / 2)
        result["tolerance_x_2^(n/2)"] = 1e-5
    print(json.dumps(result), flush=True)
    return 0


def dominant_kernel(args, p, info, B, elim_ms, kernels, tree_exec=0):
    """Roofline object of the dominant kernel and its config keys.  elim_ms is
    the per-call time of all its launches (HIP events around them)."""
    B_eff = ((B + 63) // 64 * 64) << info["n_sliced"]
    if info["ordering"] == 1 and info.get("lds_ok") and tree_exec in (0, 3) and not info.get("n_open"):
        # one launch, every result in LDS: its HBM traffic is the bitstrings, the table entries at their
        # output bits (served by L2) and the amplitudes, so its roofs are on chip.  The plan's LDS bytes
        # (per result row kept: 2^k input and table reads plus one write; plus the copied table entries)
        # against the LDS read/write rate, and its flops against the vector ALU; the LDS roof is the
        # higher time floor of the two, so it is the one reported.
        lds_bytes = info["lds_bytes_per_amp"] * B
        flops = info["flops_per_amp"] * B
        t = elim_ms / 1e3
        achieved = lds_bytes / t / 1e12
        cfg = {"buckets": info["n_buckets"], "tree_levels": info["n_levels"], "launches": 1,
               "execution_form": "LDS-resident: one work-group of %d threads per bitstring" % info["lds_threads"],
               "lds_bytes_per_workgroup": 8 * info["lds_entries"] + LDS_HEADER, "lds_jobs": info["lds_jobs"],
               "flops_per_amp": info["flops_per_amp"], "lds_bytes_per_amp": info["lds_bytes_per_amp"],
               "bytes_per_amp_of_the_level_launches": info["bytes_per_amp"]}
        roofline = {"bound": "lds", "achieved": round(achieved, 3), "peak": LDS_PEAK_TBS, "unit": "TB/s",
                    "frac": round(achieved / LDS_PEAK_TBS, 4), "traffic": None,
                    "kernel": "k_tree_lds (bucket elimination with every result in LDS, one launch per call)",
                    "lds_bytes_per_launch": lds_bytes, "launch_ms": elim_ms, "launches_per_step": 1,
                    "peak_note": "LDS peak from unit counts: 256 B/clk per CU x 256 CUs x 2.4 GHz",
                    "alu": {"flops_per_launch": flops, "achieved_TFLOPs": round(flops / t / 1e12, 3),
                            "peak_TFLOPs": FP32_VECTOR_PEAK_TFLOPS,
                            "frac": round(flops / t / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4)}}
        rec = MEASURED_TRAFFIC.get((args.workload, "lds"))
        if rec:
            import hashlib
            path = os.path.join(ROOT, "paper_1712_05384_amd", "csrc", rec["source"])
            same_plan = all(info.get(k) == v for k, v in rec.get("plan", {}).items())
            if same_plan and hashlib.sha256(open(path, "rb").read()).hexdigest()[:16] == rec["sha256_16"]:
                roofline["traffic"] = round(rec["bytes_per_launch"] / t / 1e9, 2)
                roofline["traffic_bytes_per_launch"] = rec["bytes_per_launch"]
                roofline["traffic_unit"] = "GB/s of HBM"
                vi = rec.get("valu_per_wave")
                if vi:   # the vector-ALU issue floor from the same record's SQ_INSTS_VALU count
                    waves_per_simd = B * (info["lds_threads"] // 64) / (4 * 256)
                    floor_s = vi * 4 * waves_per_simd / 2.4e9
                    roofline["valu_issue"] = {"instructions_per_wave": vi, "floor_ms": round(floor_s * 1e3, 5),
                                              "frac": round(floor_s / t, 3),
                                              "note": "4 cycles per wave64 instruction on a SIMD, 1024 SIMDs "
                                                      "at 2.4 GHz, every wave of the launch"}
        return roofline, cfg
    if info["ordering"] == 1:
        kernel = ("k_tree_level + k_tree_tail (bucket elimination: one launch per elimination-tree level, "
                  "the last small levels and the FP64 output in one launch)")
        n_launch = info["level_launches"]
        alg_bytes = B_eff * sum(s["bytes_per_b"] for s in info["buckets"])
        # row loads and stores the kernel issues (cache-served re-reads of broadcast inputs, constant-1
        # padding, factor-table entries), from the plan's per-bucket count
        issued = sum(s["issued_bytes_per_b"] for s in info["buckets"]) * B_eff
        cfg = {"buckets": info["n_buckets"], "tree_levels": info["n_levels"], "launches": n_launch,
               "bytes_per_amp": info["bytes_per_amp"]}
        extra = {"issued_load_store_bytes_per_launch": issued / n_launch}
        src = "tree.hip"
    else:
        kernel = "k_step (worldline elimination step)"
        n_launch = info["n_steps"]
        alg_bytes = B_eff * sum(s["bytes_per_b"] for s in info["steps"])
        cfg = {"sliced_vars": info["n_sliced"], "kernel_policy": args.kernel_policy,
               "autotuned": not args.no_autotune,
               "step_kernels": {k: (kernels or [st["kernel"] for st in info["steps"]]).count(k)
                                for k in ("valu", "valu_pair", "mfma_f32", "mfma_bf16x3")}}
        extra = {}
        src = "kernels.hip"
    achieved = alg_bytes / (elim_ms / 1e3) / 1e9
    traffic, tb = None, None
    rec = MEASURED_TRAFFIC.get((args.workload, info["ordering"]))
    if rec and args.kernel_policy == 0 and (info["ordering"] == 1 or args.no_autotune):
        import hashlib
        path = os.path.join(ROOT, "paper_1712_05384_amd", "csrc", rec["source"])
        same_plan = all(info.get(k) == v for k, v in rec.get("plan", {}).items())
        if rec["source"] == src and same_plan and \
                hashlib.sha256(open(path, "rb").read()).hexdigest()[:16] == rec["sha256_16"]:
            tb = rec["bytes_per_launch"]
            traffic = round(tb / (elim_ms / n_launch / 1e3) / 1e9, 1)   # GB/s of HBM traffic
    roofline = dict({"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_bytes_per_launch": tb, "kernel": kernel, "bytes_per_launch": alg_bytes / n_launch,
                     "launch_ms": elim_ms / n_launch, "launches_per_step": n_launch}, **extra)
    return roofline, cfg


def _time(fn, reps, stream, torch):
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _amps_per_sec(Q, C, torch, np, stream, name, reps=5, autotune=True, **plan_kw):
    """Eager amplitudes/s of one workload with inputs resident; returns (value, plan, ms, out)."""
    dev = torch.device("cuda", 0)
    c, bits = C.workload(name)
    p = Q.plan(c, **plan_kw)
    gv = None if c.gate_vals is None else torch.tensor(c.gate_vals.astype(np.complex64), device=dev)
    bd = torch.from_numpy(bits.view(np.int64)).to(dev)
    o = torch.empty((len(bits), 1), dtype=torch.complex128 if plan_kw.get("out_c128") else torch.complex64,
                    device=dev)
    w = torch.empty(max(p.workspace_bytes(len(bits)), 256), dtype=torch.uint8, device=dev)
    if plan_kw.get("ordering", 0) == 0 and autotune:
        p.autotune(bd, gv, stream=stream)
    ms = _time(lambda: p.amplitudes(bd, gv, out=o, workspace=w, stream=stream), reps, stream, torch)
    return len(bits) / (ms / 1e3), p, ms, o


def _kernel_ms(p, bd, out, ws, stream, torch, reps=5):
    """Per-call time of the elimination phase (HIP events the plan records around its launches)."""
    p.set_timing(True)
    for _ in range(reps):
        p.amplitudes(bd, None, out=out, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    ph, nc = p.timings()
    p.set_timing(False)
    return ph[2] / max(nc, 1)


def _sec_launch_forms(Q, C, torch, np, stream, args, out):
    """The default plan with one launch per elimination-tree level (results in HBM), and the vertical order."""
    dev = torch.device("cuda", 0)
    c, bits = C.workload(args.workload)
    bd = torch.from_numpy(bits.view(np.int64)).to(dev)
    for key, kw in (("ordering_1_level_launches", {"ordering": 1, "tree_exec": 1}),
                    ("ordering_0", {"ordering": 0})):
        v, p, ms, o = _amps_per_sec(Q, C, torch, np, stream, args.workload, 10, **kw)
        info = p.info(0)
        w = torch.empty(max(p.workspace_bytes(len(bits)), 256), dtype=torch.uint8, device=dev)
        kms = _kernel_ms(p, bd, o, w, stream, torch)
        rf, _ = dominant_kernel(argparse.Namespace(workload=args.workload, kernel_policy=0, no_autotune=False),
                                p, info, len(bits), kms, None, kw.get("tree_exec", 0))
        out[key] = {"workload": args.workload, "amplitudes_per_sec": round(v, 1), "ms_per_call": round(ms, 4),
                    "bytes_per_amp": info["bytes_per_amp"], "max_rank": info["max_rank"], "roofline": rf}
        print(f"# {key}: {ms:.4f} ms per call, roofline frac {rf['frac']}", file=sys.stderr, flush=True)


def _sec_batch_scaling(Q, C, torch, np, stream, args, out):
    """Batch scaling on the default circuit, both launch forms of the bucket plan (graph replay)."""
    dev = torch.device("cuda", 0)
    c, _ = C.workload(args.workload)
    scale = {}
    for mode in (0, 1):
        p = Q.plan(c, ordering=1, tree_exec=mode)
        info = p.info(0)
        form = "lds" if mode == 0 and info["lds_ok"] else "level_launches"
        for Bs in (4096, 16384, 65536):
            bs = C.random_bitstrings(c.n, Bs, 77)
            bdx = torch.from_numpy(bs.view(np.int64)).to(dev)
            o = torch.empty((Bs, 1), dtype=torch.complex64, device=dev)
            w = torch.empty(max(p.workspace_bytes(Bs), 256), dtype=torch.uint8, device=dev)
            g = Q.Graph([p], [bdx])
            ms = _time(lambda: g.launch(stream), 10, stream, torch)
            kms = _kernel_ms(p, bdx, o, w, stream, torch)
            rf, _ = dominant_kernel(argparse.Namespace(workload="", kernel_policy=0, no_autotune=True), p, info, Bs,
                                    kms, None, mode)
            scale.setdefault(form, {})[str(Bs)] = {"amplitudes_per_sec": round(Bs / (ms / 1e3), 1),
                                                   "ms_per_call": round(ms, 4), "roofline_bound": rf["bound"],
                                                   "roofline_frac": rf["frac"], "achieved": rf["achieved"],
                                                   "achieved_unit": rf["unit"]}
            print(f"# {form} B={Bs}: {ms:.4f} ms, roofline frac {rf['frac']} ({rf['bound']})", file=sys.stderr,
                  flush=True)
            del g, w, o
    out["batch_scaling"] = {"workload": f"{args.workload} with B uniform bitstrings (seed 77), graph replay",
                            **scale}


def _sec_sets(Q, C, torch, np, stream, args, out):
    """Sets of amplitudes (Sec. III.A): 2^k amplitudes per bitstring with k open qubits, counted as amplitudes."""
    dev = torch.device("cuda", 0)
    c, bits = C.workload(args.workload)
    bd = torch.from_numpy(bits.view(np.int64)).to(dev)
    sets = {}
    for oq in ((0, 6, 12, 18), (0, 3, 6, 9, 12, 15, 18, 21)):
        p = Q.plan(c, oq, ordering=1)
        o = torch.empty((len(bits), 1 << len(oq)), dtype=torch.complex64, device=dev)
        w = torch.empty(max(p.workspace_bytes(len(bits)), 256), dtype=torch.uint8, device=dev)
        ms = _time(lambda: p.amplitudes(bd, None, out=o, workspace=w, stream=stream), 10, stream, torch)
        n_amp = len(bits) << len(oq)
        sets[f"open_{len(oq)}"] = {"open_qubits": list(oq), "amplitudes_per_call": n_amp,
                                   "amplitudes_per_sec": round(n_amp / (ms / 1e3), 1), "ms_per_call": round(ms, 4),
                                   "max_rank": p.info(0)["max_rank"]}
        print(f"# sets of {1 << len(oq)} amplitudes: {ms:.4f} ms per call ({n_amp} amplitudes)", file=sys.stderr,
              flush=True)
        del w, o
    out["sets_of_amplitudes"] = {"workload": f"{args.workload}, {len(bits)} bitstrings, k open qubits "
                                             "(one level-launch plan per set; every completion of the open bits)",
                                 **sets}


def _sec_c4_grad(Q, C, torch, np, stream, args, out):
    """Gradients: 5x5 depth 20 with parameterised gates, 256 bitstrings, L = sum log |A|^2."""
    dev = torch.device("cuda", 0)
    c, bits = C.workload("c4_5x5_d20_U")
    gv = torch.tensor(c.gate_vals.astype(np.complex64), device=dev)
    bd = torch.from_numpy(bits.view(np.int64)).to(dev)
    out["c4_grad"] = {"workload": "5x5 depth 20, every 1q gate U(theta, n), 256 bitstrings, d(sum log p)/dU for "
                                  f"{c.n_slots} gate tensors (one backward call: forward, seed, adjoint)"}
    for ordering in (1, 0):
        p = Q.plan(c, ordering=ordering)
        amps = p.amplitudes(bd, gv)
        gamps = (2.0 / torch.conj(amps)).contiguous()
        ws = torch.empty(p.backward_workspace_bytes(len(bits)), dtype=torch.uint8, device=dev)
        gg = torch.empty((c.n_slots, 2, 2), dtype=torch.complex64, device=dev)
        ao = torch.empty_like(amps)
        ms = _time(lambda: p.backward(bd, gamps, gv, workspace=ws, stream=stream, gate_grads=gg, amps_out=ao),
                   10, stream, torch)
        wf = torch.empty(max(p.workspace_bytes(len(bits)), 256), dtype=torch.uint8, device=dev)
        msf = _time(lambda: p.amplitudes(bd, gv, out=ao, workspace=wf, stream=stream), 10, stream, torch)
        out["c4_grad"]["ordering_%d" % ordering] = {"grad_evals_per_sec": round(1e3 / ms, 2),
                                                    "ms_per_grad_eval": round(ms, 4),
                                                    "ms_forward_only": round(msf, 4)}
        print(f"# c4 gradient ordering {ordering}: {ms:.3f} ms per evaluation (forward alone {msf:.3f} ms)",
              file=sys.stderr, flush=True)
        del ws


def _sec_per_bitstring(Q, C, torch, np, stream, args, out):
    """Plain per-bitstring baseline: the default workload's plan called with B = 1 in a host loop (no graph)."""
    dev = torch.device("cuda", 0)
    c, bits = C.workload(args.workload)
    p = Q.plan(c, ordering=args.ordering)
    one = [torch.from_numpy(bits[i:i + 1].view(np.int64)).to(dev) for i in range(64)]
    o1 = torch.empty((1, 1), dtype=torch.complex64, device=dev)
    w1 = torch.empty(max(p.workspace_bytes(1), 256), dtype=torch.uint8, device=dev)
    ms = _time(lambda: [p.amplitudes(b1, None, out=o1, workspace=w1, stream=stream) for b1 in one], 3, stream, torch)
    out["per_bitstring_baseline"] = {"workload": f"{c.name}, same plan, B = 1 per call, 64 calls",
                                     "amplitudes_per_sec": round(64 / (ms / 1e3), 1),
                                     "ms_per_amplitude": round(ms / 64, 4)}
    print(f"# per-bitstring baseline: {ms / 64:.3f} ms per amplitude", file=sys.stderr, flush=True)


def _sec_c3(Q, C, torch, np, stream, args, out, mfma_only=False):
    """5x6 depth 30: bucket path (no slicing needed) and vertical path with 2 sliced variables (FP64 slice sum)
    in three precisions of its steps: autotuned vector ALU, FP32 matrix cores, BF16x3 matrix cores; each against
    the stored FP64 state-vector amplitudes (tests/golden, written by the oracle)."""
    golden = np.load(os.path.join(ROOT, "tests", "golden", "c3_5x6_d30_amps.npy"), allow_pickle=False)
    n3 = C.workload("c3_5x6_d30")[0].n

    def c3_row(**kw):
        v, p, ms, o = _amps_per_sec(Q, C, torch, np, stream, "c3_5x6_d30", 3, out_c128=True, **kw)
        err = np.abs(o.cpu().numpy()[:, 0] - golden) * 2 ** (n3 / 2)
        info = p.info(0)
        row = {"amplitudes_per_sec": round(v, 1), "ms_per_call": round(ms, 4), "bytes_per_amp": info["bytes_per_amp"],
               "max_err_x_2^(n/2)": float(err.max()), "median_err_x_2^(n/2)": float(np.median(err))}
        if kw.get("ordering") == 0:
            kinds = [st["kernel"] for st in info["steps"]]
            row["step_kernels"] = {k: kinds.count(k) for k in sorted(set(kinds))}
        return row, ms
    out["c3"] = {"workload": "5x6 depth 30, 1024 bitstrings, complex128 output"}
    if not mfma_only:
        out["c3"]["ordering_1"], ms1 = c3_row(ordering=1)
        print(f"# c3: bucket {ms1:.3f} ms per 1024 amplitudes", file=sys.stderr, flush=True)
    rows = (("ordering_0_sliced_2_valu", 0, True), ("ordering_0_sliced_2_fp32_mfma", 2, False),
            ("ordering_0_sliced_2_bf16x3", 4, False))
    for key, pol, tune in rows[1:] if mfma_only else rows:
        out["c3"][key], ms0 = c3_row(ordering=0, min_sliced_vars=2, kernel_policy=pol, autotune=tune)
        print(f"# c3 {key}: {ms0:.3f} ms per 1024 amplitudes, max err x 2^(n/2) "
              f"{out['c3'][key]['max_err_x_2^(n/2)']:.3g}", file=sys.stderr, flush=True)


def _sec_c5_graph(Q, C, torch, np, stream, args, out):
    """Uneven batch: 4x5 d20, 5x5 d24, 6x6 d24, 6x7 d27, 1024 bitstrings each, one graph."""
    names = ("c5_4x5_d20", "c5_5x5_d24", "c5_6x6_d24", "c5_6x7_d27")
    cs, bs = zip(*[C.workload(nm) for nm in names])
    total = sum(len(b) for b in bs)
    out["c5_graph"] = {"workload": "4x5 d20 + 5x5 d24 + 6x6 d24 + 6x7 d27, 1024 bitstrings each, one HIP graph "
                                   "with one branch per circuit"}
    for ordering in (1, 0):
        plans = [Q.plan(ci, ordering=ordering) for ci in cs]
        g = Q.Graph(plans, list(bs))
        ms = _time(lambda: g.launch(stream), 3, stream, torch)
        out["c5_graph"]["ordering_%d" % ordering] = {"amplitudes_per_sec": round(total / (ms / 1e3), 1),
                                                     "ms_per_launch": round(ms, 4)}
        print(f"# c5 graph ordering {ordering}: {ms:.3f} ms per launch ({total} amplitudes)", file=sys.stderr,
              flush=True)
        del g


def _sec_xeb(Q, C, torch, np, stream, args, out):
    """Cross-entropy statistics and sampling from a set (App. B, App. C) over 2^22 complex64 amplitudes."""
    dev = torch.device("cuda", 0)
    nx = 1 << 22
    ax = torch.from_numpy(C.random_amplitudes(30, nx, 1).astype(np.complex64)).to(dev)
    ux = torch.from_numpy(C.random_uniforms(1 << 20, 1)).to(dev)
    wsx = Q.api.xeb_workspace(nx)
    ox = torch.empty(8, dtype=torch.float64, device=dev)
    ix = torch.empty(1 << 20, dtype=torch.int64, device=dev)
    ms_x = _time(lambda: Q.xeb(ax, 30, stream=stream, workspace=wsx, out=ox), 10, stream, torch)
    ms_s = _time(lambda: Q.sample_from_set(ax, ux, stream=stream, workspace=wsx, out=ix), 10, stream, torch)
    out["xeb"] = {"workload": "2^22 complex64 amplitudes (Porter-Thomas statistics); 2^20 draws from the set",
                  "xeb_ms": round(ms_x, 4), "xeb_read_GBps": round(8 * nx / (ms_x / 1e3) / 1e9, 1),
                  "xeb_frac_of_hbm": round(8 * nx / (ms_x / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                  "sample_set_ms": round(ms_s, 4),
                  "note": "workspace and outputs allocated once, outside the timing; each call is timed from Python "
                          "(its launches and the binding included); the XEB partial kernel is bound by its FP64 logarithm "
                          "chains (one round of 4 waves per SIMD), not by its reads"}
    print(f"# xeb: {ms_x:.3f} ms, sample_set: {ms_s:.3f} ms", file=sys.stderr, flush=True)


def _sec_c3_mfma(Q, C, torch, np, stream, args, out):
    """The two matrix-core rows of the 5x6 depth-30 workload alone (no autotuning), for counter runs."""
    _sec_c3(Q, C, torch, np, stream, args, out, mfma_only=True)


def _sec_paper_circuits(Q, C, torch, np, stream, args, out):
    """The 5x9 depth-40 and 7x8 depth-30 circuits of the Abstract (seed 1), 64 uniform bitstrings per call,
    bucket plans sliced until every result fits the kernels; for context, the paper's workstation aims at
    about 100 s per amplitude (Sec. II)."""
    dev = torch.device("cuda", 0)
    out["paper_circuits"] = {"workload": "random grid circuits of the Abstract, 64 bitstrings per call, ordering 1"}
    for r, cc, d in ((5, 9, 40), (7, 8, 30)):
        c = C.random_grid_circuit(r, cc, d, 1)
        bits = C.random_bitstrings(c.n, 64, 1)
        t0 = time.perf_counter()
        p = Q.plan(c, ordering=1)
        plan_s = time.perf_counter() - t0
        info = p.info(0)
        bd = torch.from_numpy(bits.view(np.int64)).to(dev)
        o = torch.empty((64, 1), dtype=torch.complex64, device=dev)
        w = torch.empty(max(p.workspace_bytes(64), 256), dtype=torch.uint8, device=dev)
        ms = _time(lambda: p.amplitudes(bd, None, out=o, workspace=w, stream=stream), 3, stream, torch)
        kms = _kernel_ms(p, bd, o, w, stream, torch, reps=3)
        rf, _ = dominant_kernel(argparse.Namespace(workload="", kernel_policy=0, no_autotune=True), p, info, 64, kms,
                                None, 0)
        out["paper_circuits"][f"{r}x{cc}_d{d}"] = {
            "qubits": c.n, "sliced_vars": info["n_sliced"], "max_rank": info["max_rank"],
            "workspace_GB": round(p.workspace_bytes(64) / 1e9, 3), "plan_seconds": round(plan_s, 3),
            "bytes_per_amp": info["bytes_per_amp"], "ms_per_call": round(ms, 3),
            "amplitudes_per_sec": round(64 / (ms / 1e3), 1), "roofline_frac": rf["frac"], "roofline_bound": rf["bound"]}
        print(f"# {r}x{cc} d{d}: {ms:.3f} ms per 64 amplitudes ({info['n_sliced']} sliced), roofline frac {rf['frac']}",
              file=sys.stderr, flush=True)
        del w, o


SECTIONS = {"launch_forms": _sec_launch_forms, "batch_scaling": _sec_batch_scaling, "sets": _sec_sets,
            "c4_grad": _sec_c4_grad, "per_bitstring": _sec_per_bitstring, "c3": _sec_c3, "c5_graph": _sec_c5_graph,
            "xeb": _sec_xeb, "paper_circuits": _sec_paper_circuits, "c3_mfma": _sec_c3_mfma}


def extras(Q, C, torch, np, stream, args, only=None):
    """Secondary workloads, timed the same way (inputs resident, HIP events)."""
    out = {}
    for name, fn in SECTIONS.items():
        if (only is None and name != "c3_mfma") or name == only:
            fn(Q, C, torch, np, stream, args, out)
    return out


if __name__ == "__main__":
    sys.exit(main())
