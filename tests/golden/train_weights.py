"""Train the CoNet weights that the BER experiments use, with the CPU trainer of oracle/.

    python tests/golden/train_weights.py bf16_b64_f3276 --minutes 60

Starts from the workload's He-normal blob and trains on simulator batches of the
workload's channel, antennas and modulation (training slots come from their own seed,
1000 + the workload's simulator seed, so they never coincide with evaluation slots) on
narrower grids (the receptive field of the network is 2L + 2 REs each way, so the grid
width only sets how often slot edges are seen). Writes tests/golden/trained_<workload>.npy
(FP32 blob) and its training log (.json). Nothing here touches the GPU library.
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import conet64 as o  # noqa: E402
from oracle import trainer  # noqa: E402
from synth import make_blob, workload  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--minutes", type=float, default=60.0)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--F", type=int, default=144)
    ap.add_argument("--threads", type=int, default=6)
    ap.add_argument("--workers", type=int, default=2)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--resume", action="store_true",
                    help="start from the blob already written (fresh Adam state, training slots after those used)")
    ap.add_argument("--fake-quant", default=None, choices=["fp8"],
                    help="fine-tune with the FP8 contract's roundings in the forward (straight-through)")
    args = ap.parse_args()
    w = workload(args.workload)
    mc = w.model
    p0 = o.unpack(make_blob(mc, seed=w.weight_seed), mc.K, mc.L, mc.C, mc.C_in, mc.m)
    sim = dict(w.sim.__dict__)
    sim.update(F=args.F, seed=1000 + w.sim.seed)
    out = os.path.join(HERE, f"trained_{args.workload}.npy")
    first = 0
    if args.resume:
        import json
        import numpy as np
        p0 = o.unpack(np.load(out), mc.K, mc.L, mc.C, mc.C_in, mc.m)
        prev = json.load(open(os.path.splitext(out)[0] + ".json"))
        first = prev.get("first_slot", 0) + prev["steps_done"] * prev["batch"]
    trainer.train(p0, sim, steps=args.steps, batch=args.batch, out_path=out, lr=args.lr,
                  threads=args.threads, workers=args.workers, max_seconds=args.minutes * 60.0, first_slot=first,
                  fake_quant=args.fake_quant)
    print("wrote", out)


if __name__ == "__main__":
    main()
