"""Throughput benchmark of the CoNet-Rx forward pass on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload bf16_b64_f3276] [--dtype bf16]
                    [--no-cpu] [--json-out PATH]

A step is one forward pass of the whole network (input layer, L residual blocks per
branch with product fusion + LayerNorm, LLR head) over one batch of synthetic slots
that is already resident in HBM. Default workload: 64 slots of 3276 subcarriers x 14
OFDM symbols, 4 rx (16 input channels), 16-QAM, K=3 branches x L=4 blocks x C=64
channels, BF16 operands with FP32 accumulation.

Prints one JSON line. `value` is LLR REs per second. `roofline` covers the dominant
kernel (per-launch algorithmic MFMA FLOPs / its mean HIP-event duration over the
timed steps). `cpu_baseline` times the FP64 oracle on a bounded sample of slots on the
host cores and also reports the LLR error of the GPU result on those slots.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LLR REs/sec (BF16/FP8 vs FP32) at stated LLR err; p99 slot latency"
PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0, "f32": 157.3}
HBM_PEAK_GBS = 8000.0
LLR_TOL = {"bf16": "rel-L2 <= 3e-2 vs FP64, sign agreement >= 0.99",
           "fp8": "rel-L2 <= 0.25 vs FP64, sign agreement >= 0.93",
           "f32": "rel-L2 <= 1e-5 vs FP64"}


def kernel_source_hash() -> str:
    """Hash of the HIP sources; a stored HBM-traffic measurement is valid only for it."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2510_12739_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def flops_per_re(K, L, C, C_in, m):
    return 2 * 9 * C_in * K * C + K * L * 2 * (2 * 9 * C * C) + 2 * C * m


def cpu_baseline(workload, blob, X_sample, llr_gpu_sample, budget_s=15.0, max_slots=8):
    """Time the FP64 oracle on whole slots until the budget is spent (at least one slot)."""
    from oracle import conet64 as o
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    mc = workload.model
    p = o.unpack(blob, mc.K, mc.L, mc.C, mc.C_in, mc.m)
    t0 = time.perf_counter()
    n, res, outs = 0, 0, []
    while n < min(max_slots, X_sample.shape[0]):
        outs.append(o.forward(p, X_sample[n:n + 1].astype(np.float64)))
        res += X_sample.shape[1] * X_sample.shape[2]
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    ref = np.concatenate(outs)
    got = llr_gpu_sample[:n].astype(np.float64)
    err = {"rel_l2_vs_fp64": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
           "sign_agreement": float(np.mean((got > 0) == (ref > 0))),
           "slots": n}
    return {"value": res / dt, "unit": "REs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} whole slot(s) of {X_sample.shape[1]}x{X_sample.shape[2]} REs, FP64 NumPy "
                      f"(im2col + BLAS), {dt:.1f} s"}, err


def load_traffic(kernel: str, workload: str, dtype: str):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{workload}/{dtype}/{kernel}")
    except Exception:
        return None
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def kernel_kind(name: str):
    """Roofline kind of a kernel dispatch, from the demangled name rocprofv3 reports."""
    if "block_pair_kernel<" in name or "block32_pair_kernel<" in name:
        return "block_fused_pair"
    if "block_kernel<" in name:  # <Arith, C, TWO, MAIN, HEAD, NSUP>
        args = name.split("block_kernel<", 1)[1].split(">", 1)[0].split(",")
        return "block_fused_main" if args[3].strip() == "true" else "block_fused_supports"
    if "block32_kernel<" in name:  # FP8, 96 channels: <TWO, MAIN, HEAD, NSUP>
        args = name.split("block32_kernel<", 1)[1].split(">", 1)[0].split(",")
        return "block_fused_main" if args[1].strip() == "true" else "block_fused_supports"
    if "conv3x3_kernel<" in name:
        mode = name.split("conv3x3_kernel<", 1)[1].split(",")[1].strip()
        return {"0": "input_layer", "1": "block_conv1", "2": "block_conv2_supports",
                "4": "block_conv2_main_fused"}.get(mode)
    return None


def pmc_summary(dirs, copy_bytes, workload_name, dtype, out_md=None):
    """HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this bench
    and of --copy-probe (calibration), written to profiles/traffic.json for the current
    kernel sources. dirs: (bench FETCH, bench WRITE, copy FETCH, copy WRITE) output dirs."""
    import csv
    import glob

    def rows(d):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise SystemExit(f"no counter_collection.csv under {d}")
        return list(csv.DictReader(open(f[0])))

    def per_kind(rs, counter):
        acc = {}
        for r in rs:
            if r["Counter_Name"] != counter:
                continue
            k = kernel_kind(r["Kernel_Name"])
            if k:
                acc.setdefault(k, []).append(float(r["Counter_Value"]) * 1024.0)
        return {k: (float(np.mean(v)), len(v)) for k, v in acc.items()}

    def copy_bytes_read(rs, counter):
        v = [float(r["Counter_Value"]) * 1024.0 for r in rs if r["Counter_Name"] == counter and "opy" in r["Kernel_Name"]]
        if not v:
            raise SystemExit("no copy kernel in the calibration run")
        return float(np.median(v))

    fetch, write = per_kind(rows(dirs[0]), "FETCH_SIZE"), per_kind(rows(dirs[1]), "WRITE_SIZE")
    fscale = copy_bytes / copy_bytes_read(rows(dirs[2]), "FETCH_SIZE")
    wscale = copy_bytes / copy_bytes_read(rows(dirs[3]), "WRITE_SIZE")
    h = kernel_source_hash()
    path = os.path.join(ROOT, "profiles", "traffic.json")
    db = json.load(open(path)) if os.path.exists(path) else {}
    db = {k: v for k, v in db.items() if v.get("source_hash") == h}
    lines = ["| Kernel | Dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | Scaled read GB | Scaled write GB | Total GB/launch |",
             "|---|---|---|---|---|---|---|"]
    for k in sorted(set(fetch) & set(write)):
        rd, wr = fetch[k][0] * fscale, write[k][0] * wscale
        db[f"{workload_name}/{dtype}/{k}"] = {"bytes_per_launch": int(rd + wr), "read_bytes": int(rd), "write_bytes": int(wr),
                                             "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4),
                                             "source_hash": h}
        lines.append(f"| {k} | {fetch[k][1]} | {fetch[k][0] / 1024:.0f} | {write[k][0] / 1024:.0f} | {rd / 1e9:.3f} | "
                     f"{wr / 1e9:.3f} | {(rd + wr) / 1e9:.3f} |")
    json.dump(db, open(path, "w"), indent=1)
    table = "\n".join(lines)
    print(f"FETCH_SIZE scale {fscale:.4f}, WRITE_SIZE scale {wscale:.4f}, source hash {h}")
    print(table)
    if out_md:
        with open(out_md, "w") as f:
            f.write(table + "\n")


def serve_measure(loads=(0.5,), duration_s=1.5, n_streams=3, seed=13, grid=False, pinned=False):
    """Serving on the continuous-batching server: first a saturating burst gives the
    capacity (requests/s); then, for each load fraction, Poisson arrivals at that
    fraction of capacity for duration_s. Latency = submit -> LLRs in host memory.
    grid: the requests carry the received grid (featurised on the GPU) instead of features.
    pinned: the callers' input and LLR buffers are page-locked (the server copies them by DMA)."""
    import collections
    import threading
    from paper_2510_12739_amd import Conet, Server, pinned_array
    from synth import make_blob, workload
    from synth.requests import make_requests, poisson_arrivals

    w = workload("serve_bf16")
    mc = w.model
    model = Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, make_blob(mc, seed=w.weight_seed), dtype="bf16",
                  max_res=14 * 3276)
    pool = make_requests(32, seed=seed)
    mean_res = float(np.mean([14 * 12 * r.n_prb for r in pool]))
    srv = Server(model, mem_budget=16 << 30, n_streams=n_streams, max_batch_res=600_000, max_queue=1 << 16)
    inputs = [r.y if grid else r.x for r in pool]
    free_out = None
    if pinned:   # page-locked copies of the inputs; per request shape, a stock of LLR buffers
        inputs = [pinned_array(a.shape) for a in inputs]
        for a, r in zip(inputs, pool):
            a[...] = r.y if grid else r.x
        free_out = [collections.deque(pinned_array((14, 12 * r.n_prb, r.m)) for _ in range(24)) for r in pool]

    def run(arrivals):
        pending, lock, done = [], threading.Lock(), threading.Event()

        def collect():
            i = 0
            while True:
                with lock:
                    t = pending[i] if i < len(pending) else None
                if t is None:
                    if done.is_set() and i >= len(pending):
                        return
                    time.sleep(50e-6)
                    continue
                srv.wait(t[0])
                if t[1] is not None:
                    free_out[t[1]].append(t[2])
                i += 1
        th = threading.Thread(target=collect)
        th.start()
        srv.reset_stats()
        t0 = time.perf_counter()
        for i, ta in enumerate(arrivals):
            while time.perf_counter() - t0 < ta:
                pass
            q = i % len(pool)
            r = pool[q]
            out = None
            if pinned:
                with lock:
                    out = free_out[q].popleft() if free_out[q] else None
                if out is None:
                    out = pinned_array((14, 12 * r.n_prb, r.m))
            t, _ = srv.submit(inputs[q], r.n_prb, r.n_rx, r.m, out=out, grid=grid)
            with lock:
                pending.append((t, q if pinned else None, out))
        done.set()
        th.join()
        return srv.stats()

    burst = run(np.zeros(600))
    cap = burst["res_per_s"] / mean_res
    out = {"workload": "serve_bf16", "requests": "n_PRB U{4..273} x 12 subcarriers x 14 symbols, n_rx {2,4}, "
           "QPSK/16/64-QAM; K=3 L=4 C=64 BF16, inputs zero-padded to 16 channels, head width 6",
           "input": "received grid, featurised on the GPU" if grid else "features",
           "caller_buffers": "page-locked (DMA to and from them)" if pinned else "pageable (host copies via pinned staging)",
           "lanes": n_streams, "capacity_req_s": round(cap, 1), "capacity_res_s": round(burst["res_per_s"], 1),
           "points": []}
    for f in loads:
        rate = f * cap
        n = max(200, int(rate * duration_s))
        st = run(poisson_arrivals(rate, n, seed=int(f * 1000)))
        out["points"].append({"load": f, "offered_req_s": round(rate, 1), "p50_us": round(st["p50_us"], 1),
                              "p99_us": round(st["p99_us"], 1), "max_us": round(st["max_us"], 1),
                              "res_per_s": round(st["res_per_s"], 1), "requests": int(st["completed"]),
                              "mean_batch_requests": round(st["mean_batch_requests"], 2),
                              "mean_us": round(st["mean_us"], 1),
                              "mean_phase_us": {k: round(st["mean_" + k + "_us"], 1)
                                                for k in ("queue", "prep", "device", "scatter", "h2d", "forward", "d2h")},
                              "slowest_phase_us": {k: round(st["slowest_" + k + "_us"], 1)
                                                   for k in ("queue", "prep", "device", "scatter")}})
        print(f"[bench] serving ({'grid' if grid else 'features'}{', pinned' if pinned else ''}) load {f:.2f}: {rate:.0f} req/s, "
              f"p50 {st['p50_us']:.0f} us, p99 {st['p99_us']:.0f} us, "
              f"phases {out['points'][-1]['mean_phase_us']}, slowest {round(st['max_us'])} us: "
              f"{out['points'][-1]['slowest_phase_us']}", file=sys.stderr, flush=True)
    srv.close()
    model.close()
    return out


def depth_latency(args):
    """Depth vs latency on this GPU (the paper's claim that inference time follows the number
    of sequentially dependent layers): CoNet with K = 2 branches of L = 6 blocks (2L + 2 = 14
    sequential conv layers) against a single pre-activation ResNet of L = 11 blocks (24
    layers), both fed the same synthetic slots with random He-normal weights and near-equal
    parameter counts. Reports the latency of one slot (median of `--steps` forwards, each
    timed by HIP events with the GPU otherwise idle) and the throughput at a 32-slot batch."""
    import torch
    from paper_2510_12739_amd import Conet
    from synth import features_fast, make_blob, workload
    from synth.weights import ModelConfig

    w = workload("bf16_b64_f3276")
    F, T, Ci, m = w.sim.F, w.sim.T, w.model.C_in, w.model.m
    X = torch.from_numpy(features_fast(w.sim, 32, n_distinct=8)).cuda()
    stream = torch.cuda.current_stream()
    out_rows = []
    for C in (64, 96):
        for name, K, L, mask in (("conet_K2_L6", 2, 6, -1), ("resnet_K1_L11", 1, 11, 0)):
            mc = ModelConfig(K, L, C, Ci, m, mask)
            model = Conet(K, L, C, Ci, m, make_blob(mc, seed=11), dtype="bf16", fuse_mask=mc.mask, max_res=32 * T * F)
            block_params = K * L * 2 * 9 * C * C
            seq_layers = 2 * L + 2
            x1 = X[:1].contiguous()
            o1 = torch.empty((1, T, F, m), dtype=torch.float32, device="cuda")
            for _ in range(5):
                model.forward(x1, out=o1)
            torch.cuda.synchronize()
            lat = []
            for _ in range(args.steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                model.forward(x1, out=o1)
                e1.record(stream)
                torch.cuda.synchronize()
                lat.append(e0.elapsed_time(e1) * 1e3)
            ob = torch.empty((32, T, F, m), dtype=torch.float32, device="cuda")
            for _ in range(2):
                model.forward(X, out=ob)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(5):
                model.forward(X, out=ob)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 5
            row = {"model": name, "C": C, "K": K, "L": L, "sequential_conv_layers": seq_layers,
                   "block_params": block_params, "fused_block_tile_width": model.block_tile_width,
                   "latency_1slot_us": {"p50": round(float(np.median(lat)), 1),
                                        "p10": round(float(np.percentile(lat, 10)), 1),
                                        "p90": round(float(np.percentile(lat, 90)), 1)},
                   "batch32_ms": round(ms, 3), "batch32_res_per_s": round(32 * T * F / (ms * 1e-3), 1)}
            out_rows.append(row)
            print(f"[depth] {name} C={C}: 1-slot p50 {row['latency_1slot_us']['p50']} us, "
                  f"32 slots {ms:.3f} ms", file=sys.stderr, flush=True)
            model.close()
    res = {"experiment": "depth_vs_latency", "slot": f"{T}x{F} REs, C_in={Ci}, m={m}, BF16", "rows": out_rows}
    for C in (64, 96):
        a = [r for r in out_rows if r["C"] == C]
        res[f"C{C}_latency_ratio_conet_over_resnet"] = round(a[0]["latency_1slot_us"]["p50"] / a[1]["latency_1slot_us"]["p50"], 3)
        res[f"C{C}_throughput_ratio_conet_over_resnet"] = round(a[0]["batch32_res_per_s"] / a[1]["batch32_res_per_s"], 3)
    print(json.dumps(res), flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(json.dumps(res) + "\n")


def train_bench(args):
    """One training step = forward with saved activations + bitwise BCE + backward + Adam,
    on a batch resident in HBM (the simulator's slots tiled to the batch size)."""
    import torch
    from paper_2510_12739_amd import Conet
    from synth import make_blob, simulate_slot, workload
    from synth.ofdm import data_mask

    w = workload(args.workload)
    mc = w.model
    dtype = args.dtype or w.dtype
    B, T, F = w.batch, w.sim.T, w.sim.F
    res = B * T * F
    nd = min(8, B)
    slots = [simulate_slot(w.sim, s) for s in range(nd)]
    reps = -(-B // nd)
    X = np.concatenate([np.stack([s.features for s in slots])] * reps)[:B]
    bits = np.concatenate([np.stack([s.bits for s in slots])] * reps)[:B]
    dm = data_mask(T, F)
    model = Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, make_blob(mc, seed=w.weight_seed), dtype=dtype, max_res=res,
                  train=True)
    x = torch.from_numpy(X).cuda()
    bt = torch.from_numpy(bits).cuda()
    dmt = torch.from_numpy(dm.astype(np.uint8)).cuda()
    n_data = int(dm.sum())
    llr = torch.empty((B, T, F, mc.m), dtype=torch.float32, device="cuda")

    def step():
        model.forward(x, out=llr, save=True)
        loss, dllr = model.bce(llr, bt, dmt, n_data)
        model.backward(dllr)
        model.adam_step(lr=1e-3)
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    losses = []
    ev0.record()
    for _ in range(args.steps):
        losses.append(step())
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    fl_fwd = flops_per_re(mc.K, mc.L, mc.C, mc.C_in, mc.m)
    fl_bwd = 2 * mc.K * mc.L * 2 * (2 * 9 * mc.C * mc.C) + 2 * 9 * mc.C_in * mc.K * mc.C + 4 * mc.C * mc.m
    tf = (fl_fwd + fl_bwd) * res / (ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[dtype]
    result = {"metric": "training REs/sec (forward + BCE + backward + Adam)", "value": round(res / (ms * 1e-3), 1),
              "unit": "REs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
              "data": "synthetic (seeded OFDM simulator; He-normal weights; FP32 master + Adam)",
              "config": {"workload": w.name, "slots": B, "T": T, "F": F, "K": mc.K, "L": mc.L, "C": mc.C,
                         "C_in": mc.C_in, "m": mc.m, "res_per_step": res, "parallelism": "single-gpu"},
              "loss_first_last": [round(float(losses[0].cpu()), 5), round(float(losses[-1].cpu()), 5)],
              "roofline": {"bound": "mfma", "kernel": "whole training step", "achieved": round(tf, 2), "peak": peak,
                           "unit": "TFLOP/s", "frac": round(tf / peak, 4), "traffic": None,
                           "flops_per_step": (fl_fwd + fl_bwd) * res}}
    line = json.dumps(result)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="bf16_b64_f3276")
    ap.add_argument("--dtype", default=None, help="override the workload's dtype (f32, bf16, fp8)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--serve", action="store_true", help="only the serving load sweep (10 %% .. 120 %% of capacity)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving point of the default run")
    ap.add_argument("--depth-latency", action="store_true",
                    help="only the depth-vs-latency experiment (CoNet K=2 L=6 vs ResNet K=1 L=11)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device 3 times (HBM counter calibration)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="no GPU work: turn rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this bench and of "
                         "--copy-probe into profiles/traffic.json (needs --copy-bytes)")
    ap.add_argument("--copy-bytes", type=int, default=268435456)
    ap.add_argument("--pmc-md", default=None, help="with --pmc-summary: also write the table here")
    args = ap.parse_args()

    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.copy_bytes, args.workload, args.dtype or "bf16", args.pmc_md)
        return

    if args.copy_probe:
        import torch
        src = torch.empty(args.copy_probe, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 3}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (slots shard across GPUs "
              "with no exchange; see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.depth_latency:
        depth_latency(args)
        return

    if args.serve:
        for grid, pinned in ((False, False), (True, False), (False, True), (True, True)):
            out = serve_measure(loads=(0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2), duration_s=2.0, grid=grid, pinned=pinned)
            ok = [p["offered_req_s"] for p in out["points"] if p["p99_us"] < 500.0]
            out["max_load_req_s_p99_under_500us"] = max(ok) if ok else None
            print(json.dumps(out), flush=True)
        return

    if args.workload.startswith("train"):
        train_bench(args)
        return

    import torch
    from paper_2510_12739_amd import Conet
    from synth import features_fast, make_blob, workload

    w = workload(args.workload)
    dtype = args.dtype or w.dtype
    mc = w.model
    B, T, F = w.batch, w.sim.T, w.sim.F
    res = B * T * F
    print(f"[bench] workload {w.name} dtype {dtype}: B={B} T={T} F={F} K={mc.K} L={mc.L} C={mc.C} "
          f"C_in={mc.C_in} m={mc.m}", file=sys.stderr, flush=True)
    blob = make_blob(mc, seed=w.weight_seed)
    X = features_fast(w.sim, B, n_distinct=min(8, B))
    x = torch.from_numpy(X).cuda()
    model = Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, dtype=dtype, max_res=res)
    if dtype == "fp8":
        model.calibrate(x[:min(4, B)])
    out = torch.empty((B, T, F, mc.m), dtype=torch.float32, device="cuda")

    # attainable dense-MFMA peak and shader clock on this device (context for `frac`)
    from paper_2510_12739_amd import mfma_peak
    peak_meas, clock_ghz = mfma_peak(dtype)
    print(f"[bench] measured MFMA peak {peak_meas:.1f} TFLOP/s at {clock_ghz:.3f} GHz", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        model.forward(x, out=out)
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # ---- timed region: K steps; each records a HIP event before every kernel launch
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stage_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    stage_units = None
    for _ in range(args.steps):
        _, ms, stage_units = model.forward_profiled(x, out=out, units=True)
        stage_ms.append(ms)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    stage_ms = np.array(stage_ms)                          # [steps, 1 + 2L]
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall {wall:.2f} s)", file=sys.stderr, flush=True)

    # ---- roofline of the dominant kernel. Stages: input layer, then per block (a) conv 1 of
    # all branches / a fused block without fusion after it, (b) support branches (their conv 2,
    # or with fused residual blocks both convs, paired with the previous block's main branch
    # when it was deferred to this launch), (c) a main branch launched alone. The library
    # reports each stage's conv-branch units (one conv of one branch over the batch), so the
    # FLOPs are algorithmic: units x REs x 2*9*C*C (the fused kernel's halo recompute of conv 1
    # and padded M-tiles are not counted).
    blk_fl = res * 2 * 9 * mc.C * mc.C                   # MFMA FLOPs of one block conv over one branch
    fused_tw = model.block_tile_width
    names = (("block_fused_all", "block_fused_supports", "block_fused_main") if fused_tw else
             ("block_conv1", "block_conv2_supports", "block_conv2_main_fused"))
    kinds = {}
    for i in range(1, stage_ms.shape[1]):
        u = int(stage_units[i])
        if u == 0:
            continue
        name = names[(i - 1) % 3]
        if fused_tw and (i - 1) % 3 == 1 and u == 2 * mc.K:
            name = "block_fused_pair"
        kinds.setdefault(name, []).append((stage_ms[:, i], u * blk_fl))
    tot = {k: sum(float(ms.sum()) for ms, _ in v) for k, v in kinds.items() if v}
    dom = max(tot, key=tot.get)
    launches = kinds[dom]
    fl_launch = float(np.mean([fl for _, fl in launches]))
    dom_ms = float(np.mean([ms.mean() for ms, _ in launches]))
    achieved = float(np.mean([fl / (ms.mean() * 1e-3) for ms, fl in launches])) / 1e12
    peak = PEAK_TFLOPS[dtype]
    traffic = load_traffic(dom, w.name, dtype)
    roofline = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "flops_per_launch": fl_launch, "mean_launch_ms": round(dom_ms, 4),
                "fused_block_tile_width": fused_tw,
                "measured_peak": round(peak_meas, 1), "measured_clock_ghz": round(clock_ghz, 3),
                "frac_of_measured_peak": round(achieved / peak_meas, 4) if peak_meas > 0 else None,
                "stage_mean_ms": [round(float(v), 4) for v in stage_ms.mean(axis=0)],
                "stage_conv_units": [int(u) for u in stage_units],
                "whole_step_tflops": round(flops_per_re(mc.K, mc.L, mc.C, mc.C_in, mc.m) * res / (ms_per_step * 1e-3) / 1e12, 2)}

    result = {"metric": METRIC, "value": round(res / (ms_per_step * 1e-3), 1), "unit": "REs/s",
              "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
              "data": "synthetic (seeded OFDM simulator: Rayleigh + Jakes channel, AWGN, LS features; He-normal weights)",
              "config": {"workload": w.name, "slots": B, "T": T, "F": F, "n_rx": w.sim.n_rx, "K": mc.K, "L": mc.L,
                         "C": mc.C, "C_in": mc.C_in, "m": mc.m, "res_per_step": res, "parallelism": "single-gpu"},
              "llr_tolerance": LLR_TOL[dtype],
              "roofline": roofline}

    # input featuriser (LS + interpolation, conet_featurise) on the same grid: reported beside
    # the forward, not part of `value` (the forward's boundary takes features)
    from paper_2510_12739_amd import featurise
    from synth import simulate_slot
    ys = np.stack([simulate_slot(w.sim, s).y for s in range(min(8, B))])
    ys = np.concatenate([ys] * (-(-B // ys.shape[0])), axis=0)[:B]
    y_dev = torch.from_numpy(np.ascontiguousarray(np.stack([ys.real, ys.imag], axis=-1).astype(np.float32))).cuda()
    del ys
    xf = torch.empty_like(x)
    for _ in range(3):
        featurise(y_dev, mc.C_in, out=xf)
    fe0, fe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fe0.record(stream)
    for _ in range(10):
        featurise(y_dev, mc.C_in, out=xf)
    fe1.record(stream)
    torch.cuda.synchronize()
    f_ms = fe0.elapsed_time(fe1) / 10
    f_bytes = y_dev.numel() * 4 + xf.numel() * 4
    result["featuriser"] = {"ms": round(f_ms, 4), "bytes": f_bytes, "GB_per_s": round(f_bytes / (f_ms * 1e-3) / 1e9, 1),
                            "frac_of_hbm_peak": round(f_bytes / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del y_dev, xf

    if not args.no_cpu:
        n_s = min(8, B)
        llr_s = out[:n_s].cpu().numpy()
        cb, err = cpu_baseline(w, blob, X[:n_s], llr_s, budget_s=args.cpu_budget)
        result["cpu_baseline"] = cb
        result["llr_err"] = err
    else:
        result["cpu_baseline"] = None

    if not args.no_serve and args.workload == "bf16_b64_f3276" and dtype == "bf16":
        del model, x, out
        torch.cuda.empty_cache()
        # received grids in page-locked buffers (the server's fastest input path); --serve sweeps all four
        result["serving"] = serve_measure(loads=(0.1, 0.5), duration_s=1.5, grid=True, pinned=True)

    line = json.dumps(result)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
