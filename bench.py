"""Throughput of the qNEP force evaluation on one MI355X.

One step = one full evaluation (neighbour lists, descriptors, network, charge
correction, real-space and PPPM electrostatics, forces, virial, Born charges,
polarization) of the 975,560-atom perovskite-like box with a 256^3 PPPM mesh.
Inputs are resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 3] [--precision fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--variant", default="full")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build evaluates one structure on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2601_19034_amd import inputs
    from paper_2601_19034_amd.api import QNEP, to_device_inputs

    w = inputs.workload(args.workload, args.variant)
    n = w.system.n
    print(f"# workload {w.name}: N={n}, mesh={w.es.mesh}, precision={args.precision}", file=sys.stderr, flush=True)
    model = QNEP(w.hp, args.precision)
    pos, types, th = to_device_inputs(w.system, w.theta, "cuda:0")
    stream = torch.cuda.current_stream()
    out = model.compute(pos, types, w.system.cell, th, w.es)
    flags = model.check_status()
    if flags:
        raise SystemExit(f"device status flags {flags}")
    for _ in range(args.warmup):
        model.compute(pos, types, w.system.cell, th, w.es, out=out)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(args.steps):
        model.compute(pos, types, w.system.cell, th, w.es, out=out)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1) / args.steps
    value = n / (ms * 1e-3)
    print(f"# {ms:.3f} ms/step ({wall / args.steps * 1e3:.3f} ms wall), E={float(out['energy'][0]):.6f}",
          file=sys.stderr, flush=True)
    rec = {
        "metric": "atom-steps/s (E+F+virial+Z*) at 1M atoms PPPM",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_atoms": n, "method": "PPPM", "mesh": list(w.es.mesh),
                   "mlp": args.precision},
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
