#!/usr/bin/env python3
"""Throughput of the amplitude path on one MI355X.

A "step" is one qgm_amplitudes call over the whole batch: boundary kernel,
G build, every elimination step and the FP64 output stage, with bitstrings,
workspace and output already resident in HBM.  Default workload: the 5x5
depth-25 random grid circuit (seed 201) with 1024 uniform bitstrings.

Prints one JSON line.  The roofline object is for the dominant kernel (the
elimination-step kernel): algorithmic bytes per launch (read F + write F' +
variant ids, from the plan) over its average launch duration, timed with HIP
events on the stream the kernels run on.  The cpu_baseline leg times the FP64
state-vector oracle on the host cores over the same circuit and bitstrings,
and its amplitudes give the max error of the GPU result.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per elimination-step launch on the default workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000, the factors a
# plain 1 GiB copy gives), valid for the step-kernel source with this hash.
MEASURED_TRAFFIC = {"c2_5x5_d25": {"bytes_per_launch": 226794653.4, "kernels_sha256_16": "a72736aaae65f038"}}
METRIC = "amplitudes/sec at max err vs FP64 oracle; % FP32-MFMA/HBM roofline; grad/sec"


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2_5x5_d25")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary workloads (C4 gradients, C3 sliced, C5 four-circuit graph)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for the HBM byte counters)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the policy's kernels instead of timing them")
    ap.add_argument("--kernel-policy", type=int, default=0,
                    help="0 auto, 1 vector ALU one row per thread, 2 FP32 matrix cores where supported")
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
    c, bits = C.workload(args.workload)
    B = len(bits)
    t0 = time.perf_counter()
    p = Q.plan(c, kernel_policy=args.kernel_policy)
    plan_s = time.perf_counter() - t0
    info = p.info(0)
    print(f"# plan: n={c.n} steps={info['n_steps']} max_rank={info['max_rank']} "
          f"bytes/amp={info['bytes_per_amp']:.3g} flops/amp={info['flops_per_amp']:.3g} plan_s={plan_s:.3f}",
          file=sys.stderr, flush=True)
    gv = None if c.gate_vals is None else torch.tensor(c.gate_vals.astype(np.complex64), device=dev)
    bits_d = torch.from_numpy(bits.view(np.int64)).to(dev)
    out = torch.empty((B, 1), dtype=torch.complex64, device=dev)
    ws = torch.empty(p.workspace_bytes(B), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    kernels = None
    if not args.no_autotune:
        kernels = p.autotune(bits_d, gv, stream=stream)   # per-step kernel by measurement (complex64 kernels only)
        info = p.info(0)

    for _ in range(args.warmup):
        p.amplitudes(bits_d, gv, out=out, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    p.set_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        p.amplitudes(bits_d, gv, out=out, workspace=ws, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    phases, ncalls = p.timings()
    p.set_timing(False)
    ms_per_step = total_ms / args.steps
    value = B / (ms_per_step / 1e3)
    print(f"# timed {args.steps} steps: {ms_per_step:.4f} ms/step, {value:.4g} amplitudes/s", file=sys.stderr,
          flush=True)

    # dominant kernel: the elimination steps
    B_eff = ((B + 63) // 64 * 64) << info["n_sliced"]
    step_bytes = B_eff * sum(s["bytes_per_b"] for s in info["steps"])
    n_launch = info["n_steps"]
    step_ms = phases[2] / max(ncalls, 1)
    achieved = step_bytes / (step_ms / 1e3) / 1e9
    traffic = None
    rec = MEASURED_TRAFFIC.get(args.workload)
    if rec and args.kernel_policy == 0 and args.no_autotune:
        import hashlib
        src = os.path.join(ROOT, "paper_1712_05384_amd", "csrc", "kernels.hip")
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] == rec["kernels_sha256_16"]:
            traffic = round(rec["bytes_per_launch"] / (step_ms / n_launch / 1e3) / 1e9, 1)   # GB/s of HBM traffic
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_bytes_per_launch": rec["bytes_per_launch"] if traffic is not None else None,
                "kernel": "k_step (elimination step)", "bytes_per_launch": step_bytes / n_launch,
                "launch_ms": step_ms / n_launch, "launches_per_step": n_launch}

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "amplitudes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{c.name}: {c.rows}x{c.cols} grid, depth {c.depth()}, {B} uniform bitstrings, "
                               f"complex64, one plan for the batch", "global_batch": B,
                   "qubits": c.n, "max_rank": info["max_rank"], "sliced_vars": info["n_sliced"],
                   "kernel_policy": args.kernel_policy, "autotuned": not args.no_autotune,
                   "step_kernels": {k: (kernels or [st["kernel"] for st in info["steps"]]).count(k)
                                    for k in ("valu", "valu_pair", "mfma_f32", "mfma_bf16x3")}},
        "phases_ms_per_step": {k: round(v / max(ncalls, 1), 5) for k, v in
                               zip(("boundary", "g_build", "elimination", "output"), phases)},
        "plan_seconds": round(plan_s, 4),
        "roofline": roofline,
    }

    # the same call replayed from a HIP graph (no per-launch host work)
    g = Q.Graph([p], [bits_d], [gv])
    for _ in range(args.warmup):
        g.launch(stream)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        g.launch(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    result["graph_ms_per_step"] = round(ev0.elapsed_time(ev1) / args.steps, 5)
    result["graph_amplitudes_per_sec"] = round(B / (result["graph_ms_per_step"] / 1e3), 1)
    assert torch.equal(g.outs[0], out), "graph replay differs from the eager call"
    del g

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
        result["max_abs_err"] = err
        result["max_abs_err_x_2^(n/2)"] = err * 2 ** (c.n / 2)
        result["tolerance_x_2^(n/2)"] = 1e-5
    print(json.dumps(result), flush=True)
    return 0


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


def extras(Q, C, torch, np, stream, args):
    """Secondary workloads, timed the same way (inputs resident, HIP events)."""
    out = {}
    dev = torch.device("cuda", 0)
    # gradients: 5x5 depth 20 with parameterised gates, 256 bitstrings, L = sum log |A|^2
    c, bits = C.workload("c4_5x5_d20_U")
    p = Q.plan(c)
    gv = torch.tensor(c.gate_vals.astype(np.complex64), device=dev)
    bd = torch.from_numpy(bits.view(np.int64)).to(dev)
    amps = p.amplitudes(bd, gv)
    gamps = (2.0 / torch.conj(amps)).contiguous()
    ws = torch.empty(p.backward_workspace_bytes(len(bits)), dtype=torch.uint8, device=dev)
    ms = _time(lambda: p.backward(bd, gamps, gv, workspace=ws, stream=stream), 10, stream, torch)
    msf = _time(lambda: p.amplitudes(bd, gv, stream=stream), 10, stream, torch)
    out["c4_grad"] = {"workload": "5x5 depth 20, every 1q gate U(theta, n), 256 bitstrings, d(sum log p)/dU for "
                                  f"{c.n_slots} gate tensors, checkpointed", "grad_evals_per_sec": round(1e3 / ms, 2),
                      "ms_per_grad_eval": round(ms, 4), "ms_forward_only": round(msf, 4)}
    print(f"# c4 gradient: {ms:.3f} ms per evaluation (forward alone {msf:.3f} ms)", file=sys.stderr, flush=True)
    del ws
    # plain per-bitstring baseline: the default workload's plan called with B = 1
    # in a host loop (no graph, no autotuning; B is padded to one 64-wide wave)
    c, bits = C.workload(args.workload)
    p = Q.plan(c)
    one = [torch.from_numpy(bits[i:i + 1].view(np.int64)).to(dev) for i in range(64)]
    o1 = torch.empty((1, 1), dtype=torch.complex64, device=dev)
    w1 = torch.empty(p.workspace_bytes(1), dtype=torch.uint8, device=dev)
    ms = _time(lambda: [p.amplitudes(b1, None, out=o1, workspace=w1, stream=stream) for b1 in one], 3, stream, torch)
    out["per_bitstring_baseline"] = {"workload": f"{c.name}, same plan, B = 1 per call, 64 calls",
                                     "amplitudes_per_sec": round(64 / (ms / 1e3), 1), "ms_per_amplitude": round(ms / 64, 4)}
    print(f"# per-bitstring baseline: {ms / 64:.3f} ms per amplitude", file=sys.stderr, flush=True)
    # 5x6 depth 30, 2 sliced variables, FP64 slice sum
    c, bits = C.workload("c3_5x6_d30")
    p = Q.plan(c, min_sliced_vars=2, out_c128=True)
    bd = torch.from_numpy(bits.view(np.int64)).to(dev)
    g = Q.Graph([p], [bd])
    ms = _time(lambda: g.launch(stream), 5, stream, torch)
    out["c3_sliced"] = {"workload": "5x6 depth 30, 1024 bitstrings, 2 sliced variables, FP64 slice sum",
                        "amplitudes_per_sec": round(len(bits) / (ms / 1e3), 1), "ms_per_call": round(ms, 4),
                        "bytes_per_amp": p.info(0)["bytes_per_amp"]}
    print(f"# c3 sliced: {ms:.3f} ms per 1024 amplitudes", file=sys.stderr, flush=True)
    del g
    # uneven batch: 4x5 d20, 5x5 d24, 6x6 d24, 6x7 d27, 1024 bitstrings each, one graph
    names = ("c5_4x5_d20", "c5_5x5_d24", "c5_6x6_d24", "c5_6x7_d27")
    cs, bs = zip(*[C.workload(nm) for nm in names])
    plans = [Q.plan(ci) for ci in cs]
    g = Q.Graph(plans, list(bs))
    ms = _time(lambda: g.launch(stream), 3, stream, torch)
    total = sum(len(b) for b in bs)
    out["c5_graph"] = {"workload": "4x5 d20 + 5x5 d24 + 6x6 d24 + 6x7 d27, 1024 bitstrings each, one HIP graph "
                                   "with one branch per circuit", "amplitudes_per_sec": round(total / (ms / 1e3), 1),
                       "ms_per_launch": round(ms, 4)}
    print(f"# c5 graph: {ms:.3f} ms per launch ({total} amplitudes)", file=sys.stderr, flush=True)
    del g
    return out


if __name__ == "__main__":
    sys.exit(main())
