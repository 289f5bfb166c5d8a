"""FP64 BER-vs-SNR curves of a trained CoNet, written by the oracle (no GPU library involved).

    python tests/golden/ber_curves.py bf16_b64_f3276 [--slots 16] [--F 288]

The paper compares receivers by their uncoded BER against SNR (Sec. IV, Figs. 6-8). The
precision bar here is the horizontal gap, in dB at a target BER, between the curve of an
arithmetic precision (FP32, BF16, FP8 on the GPU) and the FP64 curve of the same network
on the same slots (common random numbers). This script evaluates the FP64 side once:

  * weights: tests/golden/trained_<workload>.npy (trained by train_weights.py on the CPU);
  * slots: the workload's simulator settings at a fixed SNR per point, on narrower grids
    (F subcarriers; the network's receptive field is 2L + 2 REs each way, so the width
    only sets how many REs sit near a slot edge) and many slots per point, so that each
    point averages many channel realisations; slot s of point i is slot i * 1000 + s of
    the evaluation seed 2000 + the workload's simulator seed (training used 1000 + it);
  * per point: data bits, bit errors of the FP64 network, and for context the errors of
    the classical receiver (MRC + max-log) with the LS-interpolated and the true channel;
    with --fp8-contract also those of the oracle's FP8 emulation (the FP8 precision
    contract with static activation scales), which separates what the number format
    costs from what the GPU kernels add.

Writes tests/golden/ber_<workload>.json.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import classical as cl  # noqa: E402
from oracle import conet64 as o  # noqa: E402
from synth import SimConfig, simulate_slot, workload  # noqa: E402
from synth.ofdm import data_mask  # noqa: E402

SNR_GRID = {"bf16_b64_f3276": list(range(-5, 26)), "fp8_b128_f3276": list(range(-5, 26)),
            "interf_bf16_b64_f3276": list(range(-5, 26))}


def eval_sim(wl: str, F: int, snr_db: float) -> SimConfig:
    """The workload's simulator (interferer and variance channels included) at one SNR."""
    s = workload(wl).sim
    return SimConfig(**{**s.__dict__, "F": F, "snr_db": float(snr_db), "seed": 2000 + s.seed})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--F", type=int, default=288)
    ap.add_argument("--fp8-contract", action="store_true",
                    help="also count the errors of the oracle's FP8 emulation (the precision contract alone), "
                         "with static scales calibrated on the slots the GPU test calibrates on")
    args = ap.parse_args()
    wl = args.workload
    w = workload(wl)
    mc = w.model
    blob = np.load(os.path.join(HERE, f"trained_{wl}.npy"))
    p = o.unpack(blob.astype(np.float32), mc.K, mc.L, mc.C, mc.C_in, mc.m)
    dm = data_mask(w.sim.T, args.F)
    q8 = None
    if args.fp8_contract:
        from synth import features_fast
        cal = features_fast(SimConfig(**{**w.sim.__dict__, "F": args.F}), 8).astype(np.float64)
        q8 = o.Quant("fp8", o.calibrate(p, cal))
    rows = []
    t0 = time.time()
    for i, snr in enumerate(SNR_GRID[wl]):
        sim = eval_sim(wl, args.F, snr)
        slots = [simulate_slot(sim, i * 1000 + s) for s in range(args.slots)]
        X = np.stack([s.features for s in slots]).astype(np.float64)
        bits = np.stack([s.bits for s in slots])
        llr = o.forward(p, X)
        mask = np.broadcast_to(dm[None, :, :, None], bits.shape)
        n_bits = int(mask.sum())
        err = int(((cl.hard_bits(llr) != bits) & mask).sum())
        e_ls = e_pc = 0
        for s, sl in zip(range(args.slots), slots):
            for H, acc in ((sl.H_ls, "ls"), (sl.H, "pc")):
                l_c = cl.classical_rx(sl.y, H, sl.noise_var, mc.m)
                e = int(((cl.hard_bits(l_c) != sl.bits) & mask[s]).sum())
                if acc == "ls":
                    e_ls += e
                else:
                    e_pc += e
        row = {"snr_db": snr, "bits": n_bits, "errors_fp64": err, "errors_mrc_ls": e_ls, "errors_mrc_true_h": e_pc}
        if q8 is not None:
            row["errors_fp8_contract"] = int(((cl.hard_bits(o.forward(p, X, quant=q8)) != bits) & mask).sum())
        rows.append(row)
        print(f"{wl} SNR {snr:+d} dB: BER fp64 {err / n_bits:.3e}, MRC-LS {e_ls / n_bits:.3e}, "
              f"MRC-true {e_pc / n_bits:.3e} ({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": wl, "weights": f"trained_{wl}.npy", "F": args.F, "slots_per_point": args.slots,
           "slot_index": "i * 1000 + s for point i, slot s",
           "sim_seed": 2000 + w.sim.seed, "T": w.sim.T, "points": rows}
    with open(os.path.join(HERE, f"ber_{wl}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", os.path.join(HERE, f"ber_{wl}.json"))


if __name__ == "__main__":
    main()
