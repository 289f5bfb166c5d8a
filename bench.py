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


# Sources that define the forward kernels and the layouts they read (a stored HBM-traffic
# measurement is valid only for these exact sources).
FORWARD_KERNEL_SOURCES = ("conet_common.h", "conet_kernels.h", "conet_model.h", "conet_conv_impl.h",
                          "conet_block_impl.h", "conet_block32_impl.h", "conet_conv.hip", "conet_conv_f32.hip",
                          "conet_conv_bf16.hip", "conet_conv_fp8.hip", "conet_forward.hip", "conet_api.hip")


def kernel_source_hash() -> str:
    """Hash of the forward-kernel sources; a stored HBM-traffic measurement is valid only for it."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2510_12739_amd", "csrc")
    for f in FORWARD_KERNEL_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def flops_per_re(K, L, C, C_in, m):
    return 2 * 9 * C_in * K * C + K * L * 2 * (2 * 9 * C * C) + 2 * C * m


def cpu_baseline(workload, blob, X_sample, budget_s=15.0, max_slots=8, extra=None):
    """The FP64 oracle timed on the host cores: whole slots of the headline workload until the
    budget is spent (at least one slot). `extra`: (name, workload, blob, [(X_window, keep_slice)])
    samples of other workloads (sampled subcarrier windows, each with the margin its outputs
    depend on), timed the same way. Returns the baseline record and the FP64 LLRs of every
    sample, which the GPU legs' LLR errors are measured against."""
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
    rec = {"value": res / dt, "unit": "REs/s", "cores": int(threads), "kind": "oracle",
           "cpu_model": cpu_model_name(), "host_cpus": os.cpu_count(),
           "sample": f"{n} whole slot(s) of {X_sample.shape[1]}x{X_sample.shape[2]} REs of {workload.name}, "
                     f"FP64 NumPy (im2col + BLAS), {dt:.1f} s"}
    refs = {workload.name: np.concatenate(outs)}
    for name, w2, blob2, wins in (extra or []):
        m2 = w2.model
        p2 = o.unpack(blob2, m2.K, m2.L, m2.C, m2.C_in, m2.m)
        t1 = time.perf_counter()
        r2, got = 0, []
        for Xw, keep in wins:
            got.append(o.forward(p2, Xw.astype(np.float64))[:, :, keep])
            r2 += Xw.shape[1] * Xw.shape[2]
        d2 = time.perf_counter() - t1
        rec.setdefault("other_workloads", {})[name] = {
            "value": r2 / d2, "unit": "REs/s",
            "sample": f"{len(wins)} subcarrier windows ({r2} REs incl. margins) of {w2.name}, {d2:.1f} s"}
        refs[name] = got
    return rec, refs


def cpu_model_name() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def llr_error(got, ref) -> dict:
    """rel-L2, max |d| / RMS(ref) with the worst element's index, and sign agreement."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.abs(got - ref)
    i = np.unravel_index(int(np.argmax(d)), d.shape)
    rms = float(np.sqrt(np.mean(ref ** 2)))
    return {"rel_l2_vs_fp64": float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)),
            "max_abs_over_rms": float(d.max() / max(rms, 1e-300)), "worst_index": [int(v) for v in i],
            "sign_agreement": float(np.mean((got > 0) == (ref > 0))), "n": int(ref.size)}


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


def depth_latency_measure(calls=100):
    """Depth vs latency on this GPU (the paper's claim that inference time follows the number of
    sequentially dependent layers, Sec. IV): CoNet with K = 2 branches of L = 6 blocks (2L + 2 =
    14 sequential conv layers) against single pre-activation ResNets of L = 11 blocks (24 layers,
    the depth the paper compares with; 8 % fewer block parameters at equal width) and L = 12
    blocks (26 layers, exactly CoNet's 24 block convolutions of C x C, so equal parameters), at
    C = 64 and C = 96, all fed the same synthetic slots with random He-normal weights. Reports
    the latency of one slot (`calls` forwards, each timed alone by HIP events) and the
    throughput at a 32-slot batch."""
    import torch
    from paper_2510_12739_amd import Conet
    from synth import features_fast, make_blob, workload
    from synth.weights import ModelConfig, blob_size

    w = workload("bf16_b64_f3276")
    F, T, Ci, m = w.sim.F, w.sim.T, w.model.C_in, w.model.m
    X = torch.from_numpy(features_fast(w.sim, 32, n_distinct=8)).cuda()
    stream = torch.cuda.current_stream()
    out_rows = []
    for C in (64, 96):
        for name, K, L, mask in (("conet_K2_L6", 2, 6, -1), ("resnet_K1_L11", 1, 11, 0), ("resnet_K1_L12", 1, 12, 0)):
            mc = ModelConfig(K, L, C, Ci, m, mask)
            model = Conet(K, L, C, Ci, m, make_blob(mc, seed=11), dtype="bf16", fuse_mask=mc.mask, max_res=32 * T * F)
            params = blob_size(mc)
            x1 = X[:1].contiguous()
            o1 = torch.empty((1, T, F, m), dtype=torch.float32, device="cuda")
            for _ in range(5):
                model.forward(x1, out=o1)
            torch.cuda.synchronize()
            lat = []
            for _ in range(calls):
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
            row = {"model": name, "C": C, "K": K, "L": L, "sequential_conv_layers": 2 * L + 2,
                   "params": params, "block_params": K * L * 2 * 9 * C * C,
                   "fused_block_tile_width": model.block_tile_width,
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
        a = {r["model"]: r for r in out_rows if r["C"] == C}
        for rn in ("resnet_K1_L11", "resnet_K1_L12"):
            res[f"C{C}_latency_ratio_conet_over_{rn}"] = round(
                a["conet_K2_L6"]["latency_1slot_us"]["p50"] / a[rn]["latency_1slot_us"]["p50"], 3)
            res[f"C{C}_throughput_ratio_conet_over_{rn}"] = round(
                a["conet_K2_L6"]["batch32_res_per_s"] / a[rn]["batch32_res_per_s"], 3)
    return res


def variants_measure(steps=10):
    """The block and fusion variants on the BF16 headline batch (64 slots of 3276 x 14, K=3, L=4,
    C=64, random He-normal weights): depthwise-separable blocks with product fusion, fusion by
    concatenation after standard blocks, and support nets of 2 blocks. Per variant: time per
    forward and REs/s; for the separable network also the roofline of its block kernel (HBM-
    bound: algorithmic bytes = block inputs read + outputs written, per launch) and of the
    fusion epilogue pass, from the per-stage HIP events of conet_forward_profiled."""
    import torch
    from paper_2510_12739_amd import Conet
    from synth import ModelConfig, features_fast, make_blob, workload

    w = workload("bf16_b64_f3276")
    X = torch.from_numpy(features_fast(w.sim, w.batch, n_distinct=8)).cuda()
    B, T, F = X.shape[:3]
    res = B * T * F
    K, L, C, Ci, m = 3, 4, 64, w.model.C_in, w.model.m
    out = torch.empty((B, T, F, m), dtype=torch.float32, device="cuda")
    rows = {}
    for name, kw in (("separable_product", dict(block="ds")), ("standard_concat", dict(fusion="concat")),
                     ("standard_product_support2", dict(support_blocks=2))):
        mc = ModelConfig(K, L, C, Ci, m, -1, kw.get("support_blocks", 0), kw.get("fusion", "product"),
                         kw.get("block", "standard"))
        print(f"[bench] variant {name}", file=sys.stderr, flush=True)
        model = Conet(K, L, C, Ci, m, make_blob(mc, seed=21), dtype="bf16", max_res=res, **kw)
        for _ in range(2):
            model.forward(X, out=out)
        torch.cuda.synchronize()
        stage = []
        for _ in range(steps):
            _, ms, units = model.forward_profiled(X, out=out, units=True)
            stage.append(ms)
        stage = np.array(stage, dtype=np.float64)
        call = stage.sum(axis=1)
        row = {"call_ms_p50": round(float(np.median(call)), 4), "res_per_s": round(res / (np.median(call) * 1e-3), 1)}
        if name == "separable_product":
            # stage 1 + 3l: the block launch over the branches; 2 + 3l: the fusion epilogue pass
            blk = [(stage[:, 1 + 3 * l].mean(), (K if l < L - 1 else 1)) for l in range(L)]
            fused = [blk[l] for l in range(L - 1)]
            main_extra = 2 * C  # the main branch's FP32 output (4 C bytes instead of 2 C)
            by = [res * (n * 4 * C + main_extra) for _, n in fused]
            gbs = [b / (ms * 1e-3) / 1e9 for (ms, _), b in zip(fused, by)]
            row["block_kernel"] = {"mean_launch_ms": round(float(np.mean([ms for ms, _ in fused])), 4),
                                   "bytes_per_launch": int(np.mean(by)), "achieved_GB_per_s": round(float(np.mean(gbs)), 1),
                                   "frac_of_hbm_peak": round(float(np.mean(gbs)) / HBM_PEAK_GBS, 4),
                                   "per_re_branch_bytes": 4 * C, "flops_per_re_branch": 2 * (18 * C + 2 * C * C)}
            epi = [stage[:, 2 + 3 * l].mean() for l in range(L - 1)]
            eb = res * (4 * C + (K - 1) * 2 * C + 2 * C)  # FP32 main + BF16 supports read, A written
            row["fusion_epilogue"] = {"mean_ms": round(float(np.mean(epi)), 4), "bytes": eb,
                                      "achieved_GB_per_s": round(eb / (float(np.mean(epi)) * 1e-3) / 1e9, 1)}
        if name == "standard_concat":
            epi = [stage[:, 3 + 3 * l].mean() for l in range(L)]
            row["concat_stage_ms"] = [round(float(v), 4) for v in epi]
        rows[name] = row
        model.close()
    return {"workload": f"{B} slots x {T} x {F}, K={K} L={L} C={C} BF16, random weights", "variants": rows}


def depth_latency(args):
    res = depth_latency_measure(calls=args.steps)
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

    sim_bufs = None
    counter = [0]

    def step():
        nonlocal sim_bufs
        if args.device_data:  # a fresh batch every step, generated and featurised on the GPU
            from paper_2510_12739_amd import featurise, simulate
            sim_bufs = simulate(F, w.sim.n_rx, mc.m, counter[0] * B, B, n_taps=w.sim.n_taps,
                                max_doppler_hz=w.sim.max_doppler_hz, seed=w.sim.seed + 7000, out=sim_bufs)
            counter[0] += 1
            featurise(sim_bufs[0], mc.C_in, out=x)
        model.forward(x, out=llr, save=True)
        loss, dllr = model.bce(llr, sim_bufs[1] if args.device_data else bt, dmt, n_data)
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
              "data": ("synthetic, a fresh batch per step generated and featurised on the GPU (conet_simulate + "
                       "conet_featurise, inside the timed step)" if args.device_data else
                       "synthetic (seeded OFDM simulator, batch resident in HBM)") + "; He-normal weights; FP32 master + Adam",
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


# ----------------------------------------------------------------------------- forward legs

def trained_blob(name: str):
    """Weights trained on simulator data by tests/golden/train_weights.py (CPU), if present."""
    path = os.path.join(ROOT, "tests", "golden", f"trained_{name}.npy")
    return np.load(path).astype(np.float32) if os.path.exists(path) else None


def leg_inputs(w):
    """Blob (trained if available, else He-normal) and features of a workload's batch (8 distinct
    simulated slots tiled to the batch; the cost does not depend on the values)."""
    from synth import features_fast, make_blob
    blob = trained_blob(w.name)
    kind = "trained on simulator data (CPU trainer)" if blob is not None else "He-normal random"
    if blob is None:
        blob = make_blob(w.model, seed=w.weight_seed)
    return blob, kind, features_fast(w.sim, w.batch, n_distinct=min(8, w.batch))


def dominant_roofline(stage_ms, stage_units, mc, res, dtype, fused_tw, wl_name):
    """Roofline of the kernel kind that takes most of the step. Stages: input layer, then per
    block (a) a block without fusion after it (fused) or conv 1 of all branches, (b) support
    branches (paired with the previous block's main branch when deferred to this launch),
    (c) a main branch launched alone. Units are conv-branch executions (one conv of one branch
    over the batch), so FLOPs are algorithmic: units x REs x 2*9*C*C."""
    blk_fl = res * 2 * 9 * mc.C * mc.C
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
    return {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": load_traffic(dom, wl_name, dtype),
            "flops_per_launch": fl_launch, "launches_per_step": len(launches), "mean_launch_ms": round(dom_ms, 4),
            "fused_block_tile_width": fused_tw,
            "stage_mean_ms": [round(float(v), 4) for v in stage_ms.mean(axis=0)],
            "stage_conv_units": [int(u) for u in stage_units]}


def forward_leg(w, dtype, blob, X, steps, warmup, label):
    """W untimed forwards, then exactly `steps` timed ones (a HIP event before every launch, on
    the stream the kernels run on). Returns the leg's record and the LLRs of the last step."""
    import torch
    from paper_2510_12739_amd import Conet
    mc = w.model
    B, T, F = X.shape[0], X.shape[1], X.shape[2]
    res = B * T * F
    print(f"[bench] {label}: {w.name} {dtype} B={B} T={T} F={F} K={mc.K} L={mc.L} C={mc.C}", file=sys.stderr, flush=True)
    x = torch.from_numpy(X).cuda()
    model = Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, dtype=dtype, max_res=res)
    if dtype == "fp8":
        model.calibrate(x[:min(4, B)])
    out = torch.empty((B, T, F, mc.m), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        model.forward(x, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stage_ms, units = [], None
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        _, ms, units = model.forward_profiled(x, out=out, units=True)
        stage_ms.append(ms)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / steps
    stage_ms = np.array(stage_ms, dtype=np.float64)
    per_call = stage_ms.sum(axis=1)                    # first to last event of each forward
    rec = {"workload": w.name, "dtype": dtype, "value": round(res / (ms_per_step * 1e-3), 1), "unit": "REs/s",
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms_per_step, 4),
           "call_ms": {"p10": round(float(np.percentile(per_call, 10)), 4), "p50": round(float(np.median(per_call)), 4),
                       "p90": round(float(np.percentile(per_call, 90)), 4)},
           "res_per_step": res, "K": mc.K, "L": mc.L, "C": mc.C, "C_in": mc.C_in, "m": mc.m,
           "whole_step_tflops": round(flops_per_re(mc.K, mc.L, mc.C, mc.C_in, mc.m) * res / (ms_per_step * 1e-3) / 1e12, 2),
           "roofline": dominant_roofline(stage_ms, units, mc, res, dtype, model.block_tile_width, w.name)}
    print(f"[bench] {label}: {ms_per_step:.3f} ms/step, median call {rec['call_ms']['p50']:.3f} ms, "
          f"{rec['roofline']['kernel']} at {rec['roofline']['frac']:.3f} of peak", file=sys.stderr, flush=True)
    model.close()
    return rec, out


def c1_latency(calls=100, warmup=10):
    """The single-slot FP32 workload (72 x 14 grid, K=2 L=2 C=32): latency of one forward, each
    call timed alone by HIP events on its stream with the GPU otherwise idle."""
    import torch
    from paper_2510_12739_amd import Conet
    from synth import make_blob, simulate_slot, workload
    w = workload("fp32_b1_f72")
    mc = w.model
    X = np.stack([simulate_slot(w.sim, s).features for s in range(w.batch)])
    x = torch.from_numpy(X).cuda()
    model = Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, make_blob(mc, seed=w.weight_seed), dtype="f32",
                  max_res=X.shape[0] * 14 * 72)
    out = torch.empty((w.batch, 14, 72, mc.m), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        model.forward(x, out=out)
    torch.cuda.synchronize()
    lat = []
    for _ in range(calls):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        model.forward(x, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        lat.append(e0.elapsed_time(e1) * 1e3)
    # the same forward recorded once as a HIP graph and replayed with one launch
    g = model.record(x, out)
    for _ in range(warmup):
        g.launch()
    torch.cuda.synchronize()
    lat_g = []
    for _ in range(calls):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.launch()
        e1.record(stream)
        torch.cuda.synchronize()
        lat_g.append(e0.elapsed_time(e1) * 1e3)
    g.close()
    model.close()
    q = lambda v: {"p10": round(float(np.percentile(v, 10)), 1), "p50": round(float(np.median(v)), 1),
                   "p90": round(float(np.percentile(v, 90)), 1)}
    return {"workload": w.name, "dtype": "f32", "calls": calls, "latency_us": q(lat),
            "latency_us_recorded_graph": q(lat_g)}


def snr_at(snr, ber, target):
    """SNR where a BER curve crosses `target` (log-linear interpolation), or None."""
    lt = np.log10(target)
    lb = np.log10(np.maximum(np.asarray(ber, float), 1e-12))
    for i in range(len(snr) - 1):
        if (lb[i] - lt) * (lb[i + 1] - lt) <= 0 and lb[i] != lb[i + 1]:
            return float(snr[i] + (lt - lb[i]) * (snr[i + 1] - snr[i]) / (lb[i + 1] - lb[i]))
    return None


def ber_leg(wl, dtypes):
    """BER against SNR of the trained network at each GPU precision on the slots whose FP64 BER
    tests/golden/ber_<wl>.json holds (common random numbers), and the horizontal gap to the FP64
    curve at BER 1e-3 (else the lowest of 1e-2, 1e-1 that the FP64 curve reaches)."""
    import torch
    from paper_2510_12739_amd import Conet
    from synth import SimConfig, simulate_slot, workload
    from synth.ofdm import data_mask
    path = os.path.join(ROOT, "tests", "golden", f"ber_{wl}.json")
    blob = trained_blob(wl)
    if blob is None or not os.path.exists(path):
        return None
    g = json.load(open(path))
    w = workload(wl)
    mc, s0 = w.model, w.sim
    snr = [r["snr_db"] for r in g["points"]]
    F, n_sl, T = g["F"], g["slots_per_point"], g["T"]
    X, bits = [], []
    for i, v in enumerate(snr):
        sim = SimConfig(**{**s0.__dict__, "F": F, "snr_db": float(v), "seed": g["sim_seed"]})
        for s in range(n_sl):
            sl = simulate_slot(sim, i * 1000 + s)
            X.append(sl.features)
            bits.append(sl.bits)
    X = np.stack(X)
    bits = np.stack(bits).reshape(len(snr), n_sl, T, F, mc.m)
    mask = np.broadcast_to(data_mask(T, F)[None, None, :, :, None], bits.shape)
    ber64 = np.array([r["errors_fp64"] / r["bits"] for r in g["points"]])
    target = next(v for v in (1e-3, 1e-2, 1e-1, 2e-1) if ber64.min() <= v)  # the lowest the FP64 curve reaches
    s64 = snr_at(snr, ber64, target)
    out = {"workload": wl, "weights": g["weights"], "slots": f"{len(snr)} SNR points x {n_sl} slots of {T}x{F} REs",
           "target_ber": target, "snr_db_at_target": {"fp64": s64}, "delta_db": {}, "ber": {"snr_db": snr,
           "fp64": [float(v) for v in ber64]}}
    if "errors_fp8_contract" in g["points"][0]:  # the FP8 contract alone (oracle emulation)
        ber8 = np.array([r["errors_fp8_contract"] / r["bits"] for r in g["points"]])
        s8 = snr_at(snr, ber8, target)
        out["ber"]["fp8_contract_oracle"] = [float(v) for v in ber8]
        out["delta_db"]["fp8_contract_oracle"] = None if (s8 is None or s64 is None) else round(s8 - s64, 4)
    x = torch.from_numpy(X).cuda()
    for dt in dtypes:
        model = Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, dtype=dt, max_res=X.shape[0] * T * F)
        if dt == "fp8":
            from synth import features_fast
            model.calibrate(torch.from_numpy(features_fast(s0.__class__(**{**s0.__dict__, "F": F}), 8)).cuda())
        llr = model(x)
        torch.cuda.synchronize()
        err = ((llr.cpu().numpy() > 0).reshape(bits.shape) != bits) & mask
        b = err.reshape(len(snr), -1).sum(axis=1) / mask.reshape(len(snr), -1).sum(axis=1)
        sx = snr_at(snr, b, target)
        out["ber"][dt] = [float(v) for v in b]
        out["snr_db_at_target"][dt] = sx
        out["delta_db"][dt] = None if (sx is None or s64 is None) else round(sx - s64, 4)
        model.close()
        print(f"[bench] BER {wl} {dt}: delta {out['delta_db'][dt]} dB at {target:g}", file=sys.stderr, flush=True)
    return out


def window_samples(X, windows, R):
    """(X window with its R-subcarrier margin, slice of its own outputs) per (slot, f0, f1)."""
    outs = []
    for s, f0, f1 in windows:
        a, b = max(f0 - R, 0), min(f1 + R, X.shape[2])
        outs.append((X[s:s + 1, :, a:b], slice(f0 - a, f0 - a + (f1 - f0))))
    return outs


def headline(args):
    """The default run: the BF16 batched-inference workload (the metric's configuration) with its
    roofline and the FP64 oracle beside it, plus the comparison legs the metric names."""
    import torch
    from synth import workload

    dtype = args.dtype or workload(args.workload).dtype
    w = workload(args.workload)
    blob, wkind, X = leg_inputs(w)
    from paper_2510_12739_amd import mfma_peak
    peak_meas, clock_ghz = mfma_peak(dtype)
    print(f"[bench] measured MFMA peak {peak_meas:.1f} TFLOP/s at {clock_ghz:.3f} GHz", file=sys.stderr, flush=True)
    rec, out = forward_leg(w, dtype, blob, X, args.steps, args.warmup, "headline")
    n_s = min(8, w.batch)
    llr_head = out[:n_s].cpu().numpy()
    del out
    rl = dict(rec["roofline"])
    rl.update({"measured_peak": round(peak_meas, 1), "measured_clock_ghz": round(clock_ghz, 3),
               "frac_of_measured_peak": round(rl["achieved"] / peak_meas, 4) if peak_meas > 0 else None,
               "whole_step_tflops": rec["whole_step_tflops"]})
    mc = w.model
    B, T, F = X.shape[:3]
    result = {"metric": METRIC, "value": rec["value"], "unit": "REs/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": rec["ms_per_step"], "call_ms": rec["call_ms"],
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
              "data": f"synthetic (seeded OFDM simulator: Rayleigh + Jakes channel, AWGN, LS features; {wkind} weights)",
              "config": {"workload": w.name, "slots": B, "T": T, "F": F, "n_rx": w.sim.n_rx, "K": mc.K, "L": mc.L,
                         "C": mc.C, "C_in": mc.C_in, "m": mc.m, "res_per_step": B * T * F, "parallelism": "single-gpu"},
              "llr_tolerance": LLR_TOL[dtype], "roofline": rl}
    legs = {}
    full = not args.quick and args.workload == "bf16_b64_f3276" and dtype == "bf16"
    llr_legs = {}
    if full:
        # FP32 on the same shape (the metric's comparison point)
        r32, o32 = forward_leg(w, "f32", blob, X, max(3, args.steps // 10), 1, "fp32 on the BF16 shape")
        llr_legs[("bf16_b64_f3276", "f32")] = o32[:n_s].cpu().numpy()
        del o32
        r32["speedup_of_bf16"] = round(rec["value"] / r32["value"], 3)
        legs["f32_" + w.name] = r32
        # the FP8 workload, and BF16 / FP32 on its shape
        w3 = workload("fp8_b128_f3276")
        blob3, wkind3, X3 = leg_inputs(w3)
        R = 2 * w3.model.L + 1
        wins = [(0, 0, 128), (3, 1600, 1728), (7, 3148, 3276)]
        for dt3, st in (("fp8", max(5, args.steps // 5)), ("bf16", max(3, args.steps // 10)), ("f32", 2)):
            r3, o3 = forward_leg(w3, dt3, blob3, X3, st, 1, f"{dt3} on the FP8 shape")
            llr_legs[("fp8_b128_f3276", dt3)] = [o3[s:s + 1, :, f0:f1].cpu().numpy() for s, f0, f1 in wins]
            del o3
            r3["weights"] = wkind3
            legs[f"{dt3}_{w3.name}"] = r3
            torch.cuda.empty_cache()
        v8 = legs["fp8_fp8_b128_f3276"]["value"]
        legs["fp8_fp8_b128_f3276"]["speedup_over_bf16"] = round(v8 / legs["bf16_fp8_b128_f3276"]["value"], 3)
        legs["fp8_fp8_b128_f3276"]["speedup_over_f32"] = round(v8 / legs["f32_fp8_b128_f3276"]["value"], 3)
        legs["c1_latency"] = c1_latency()
    if not args.no_cpu:
        extra = []
        if full:
            extra = [("fp8_b128_f3276", w3, blob3, window_samples(X3, wins, R))]
        cb, refs = cpu_baseline(w, blob, X[:n_s], budget_s=args.cpu_budget, extra=extra)
        result["cpu_baseline"] = cb
        ref = refs[w.name]
        result["llr_err"] = llr_error(llr_head[:ref.shape[0]], ref)
        for (wl, dt), got in llr_legs.items():
            if wl == w.name:
                legs[f"{dt}_{wl}"]["llr_err"] = llr_error(got[:ref.shape[0]], ref)
            else:
                legs[f"{dt}_{wl}"]["llr_err"] = llr_error(np.concatenate([g.ravel() for g in got]),
                                                          np.concatenate([r.ravel() for r in refs[wl]]))
                legs[f"{dt}_{wl}"]["llr_err"]["sample"] = f"{len(wins)} windows of 128 subcarriers"
    else:
        result["cpu_baseline"] = None
    if full:
        ber = {}
        for wl, dts in (("bf16_b64_f3276", ("f32", "bf16")), ("fp8_b128_f3276", ("f32", "bf16", "fp8")),
                        ("interf_bf16_b64_f3276", ("f32", "bf16"))):
            b = ber_leg(wl, dts)
            if b is not None:
                ber[wl] = b
        result["ber_delta"] = ber or None
    result["legs"] = legs or None

    # input featuriser (LS + interpolation, conet_featurise) on the headline grid: reported
    # beside the forward, not part of `value` (the forward's boundary takes features)
    if not args.quick:
        from paper_2510_12739_amd import featurise
        from synth import simulate_slot
        stream = torch.cuda.current_stream()
        ys = np.stack([simulate_slot(w.sim, s).y for s in range(min(8, B))])
        ys = np.concatenate([ys] * (-(-B // ys.shape[0])), axis=0)[:B]
        y_dev = torch.from_numpy(np.ascontiguousarray(np.stack([ys.real, ys.imag], axis=-1).astype(np.float32))).cuda()
        del ys
        xf = torch.empty((B, T, F, mc.C_in), dtype=torch.float32, device="cuda")
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
        result["featuriser"] = {"ms": round(f_ms, 4), "bytes": f_bytes,
                                "GB_per_s": round(f_bytes / (f_ms * 1e-3) / 1e9, 1),
                                "frac_of_hbm_peak": round(f_bytes / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        # the forward straight from the received grid (features formed in the input layer's
        # staging) against the featuriser pass followed by the forward on features
        from paper_2510_12739_amd import Conet
        model = Conet(mc.K, mc.L, mc.C, mc.C_in, mc.m, blob, dtype=dtype, max_res=B * T * F)
        if dtype == "fp8":
            model.calibrate(xf[:min(4, B)])
        yo = torch.empty((B, T, F, mc.m), dtype=torch.float32, device="cuda")
        timings = {}
        for name, fn in (("featurise_then_forward", lambda: (featurise(y_dev, mc.C_in, out=xf), model.forward(xf, out=yo))),
                         ("forward_from_grid", lambda: model.forward_grid(y_dev, out=yo))):
            for _ in range(2):
                fn()
            fe0.record(stream)
            for _ in range(5):
                fn()
            fe1.record(stream)
            torch.cuda.synchronize()
            timings[name] = round(fe0.elapsed_time(fe1) / 5, 4)
        model.close()
        result["featuriser"]["ms_per_batch"] = timings
        result["featuriser"]["grid_to_llr_res_per_s"] = round(B * T * F / (timings["forward_from_grid"] * 1e-3), 1)
        del y_dev, xf, yo
        torch.cuda.empty_cache()

    if full:
        result["depth_vs_latency"] = depth_latency_measure(calls=50)
        result["variants"] = variants_measure()

    if full and not args.no_serve:
        result["serving"] = serve_measure(loads=args.serve_loads, duration_s=args.serve_seconds, grid=True, pinned=True)
        ok = [p["offered_req_s"] for p in result["serving"]["points"] if p["p99_us"] < 500.0]
        result["serving"]["max_load_req_s_p99_under_500us"] = max(ok) if ok else None

    line = json.dumps(result)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="bf16_b64_f3276")
    ap.add_argument("--dtype", default=None, help="override the workload's dtype (f32, bf16, fp8)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--serve", action="store_true", help="only the serving load sweep (10 %% .. 120 %% of capacity)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sweep of the default run")
    ap.add_argument("--quick", action="store_true", help="only the headline workload (no comparison legs, BER, "
                    "featuriser or serving)")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.1, 0.25, 0.5, 0.75, 1.0])
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--device-data", action="store_true",
                    help="with --train: generate every step's batch on the GPU (conet_simulate), inside the timed step")
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

    headline(args)


if __name__ == "__main__":
    main()
