"""Throughput of the qNEP force evaluation on one MI355X.

One step = one full evaluation (neighbour lists, descriptors, network, charge
correction, real-space and PPPM electrostatics, forces, virial, Born charges,
polarization) of the 975,560-atom perovskite-like box (58^3 ABO3 cells) with a
256^3 PPPM mesh.  Inputs are resident in HBM before the timed region.  Prints one
JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP32_VALU_PEAK_TF = 157.3  # MI355X FP32 vector


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pair_counts(system, radii):
    """Ordered neighbour-pair counts within each radius (host bookkeeping for the
    algorithmic work of a launch; periodic KD-tree, cubic or orthorhombic boxes)."""
    import numpy as np
    from scipy.spatial import cKDTree

    box = np.diag(system.cell)
    x = np.mod(system.pos, box)
    tree = cKDTree(x, boxsize=box)
    return {r: int(tree.query_ball_point(x, r, return_length=True, workers=-1).sum()) - system.n for r in radii}


# FP32 operations of one ordered pair inside the real-space cutoff (FMA = 2): image
# displacement 6, r^2 5, rsqrt and r 2, corrected charge 1, alpha r 1, exp(-a^2 r^2) 2,
# erfc from that exponential by the Abramowitz-Stegun 7.1.26 form 12, potential 3,
# force factor 5, force 6, virial (six products and sums) 18.
REAL_SPACE_FLOPS_PER_PAIR = 61


KERNEL_HEADERS = ("common.h", "plan.h", "nep_math.h")

# Algorithmic budget of one atom-step of the perovskite workload (design notes, the
# measurement section): FP32 operations (descriptors, network, electrostatics,
# FFTs and forces) and HBM bytes (per-atom inputs and outputs plus each mesh field
# written and read once, 17.2 mesh points per atom).
STEP_FLOPS_PER_ATOM = 1.3e5
STEP_BYTES_PER_ATOM = 940.0


def traffic_from_profile(kernel, workload, source):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary,
    or None when there is none or the kernel's source changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in (source,) + KERNEL_HEADERS:  # the kernel's source and the headers it includes
        h.update(open(os.path.join(ROOT, "paper_2601_19034_amd", "csrc", f), "rb").read())
    sha = h.hexdigest()
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            fields = dict(kv.split("=") for kv in line.split(":", 1)[1].split())
            if fields.get("source_sha256") == sha:
                return float(fields["bytes"])
    return None


def angular_flops_per_pair(hp):
    """Algorithmic FP32 operations of one (atom, angular neighbour) pair in the angular
    partial-force kernel, which serves the energy and the charge gradient at once
    (FMA = 2): radial basis and derivative, g_n and g_n' (4 NA NB) and the harmonics
    once; per gradient the P_n and Q_lm contractions (4 NA LM), the harmonic gradient,
    projection and accumulation."""
    NA, NB, LM = hp.n_max_A + 1, hp.basis_A + 1, 24
    basis = 13 * (NB - 2) + 16 + 12
    shared = 4 * NA * NB + basis + 80
    per_gradient = 4 * NA * LM + 2 * NA + 130 + 50
    return shared + 2 * per_gradient


def timed_run(model, pos, types, th, w, steps, warmup, torch):
    out = model.compute(pos, types, w.system.cell, th, w.es)
    flags = model.check_status()
    if flags:
        raise SystemExit(f"device status flags {flags}")
    for _ in range(warmup):
        model.compute(pos, types, w.system.cell, th, w.es, out=out)
    torch.cuda.synchronize()
    model.enable_timing(True)
    model.read_timing()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(steps):
        model.compute(pos, types, w.system.cell, th, w.es, out=out)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_stage, launches, calls = model.read_timing()
    model.enable_timing(False)
    ms = t0.elapsed_time(t1) / steps
    return ms, wall / steps * 1e3, ms_stage, launches, calls, float(out["energy"][0])


def crop_errors(torch, forms):
    """|dE|/N, max |dF|, max |dW|/N and max |dZ*| of every network form against the stored
    FP64 oracle values of the 5,000-atom perovskite crop (PPPM 45^3), written by
    tests/golden/make_fixtures.py from the oracle alone."""
    import numpy as np

    from paper_2601_19034_amd import inputs
    from paper_2601_19034_amd.api import QNEP, to_device_inputs

    ref = np.load(os.path.join(ROOT, "tests", "golden", "perovskite5000_oracle.npz"))
    w = inputs.workload(3, "crop")
    pos, types, th = to_device_inputs(w.system, w.theta, "cuda:0")
    n = w.system.n
    res = {}
    for form in forms:
        model = QNEP(w.hp, form)
        out = model.compute(pos, types, w.system.cell, th, w.es)
        if model.check_status():
            raise SystemExit("crop evaluation: device status flags set")
        g = {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
        res[form] = {
            "dE_per_atom": abs(g["energy"][0] - float(ref["energy"])) / n,
            "max_dF": float(np.abs(g["forces"].T - ref["forces"]).max()),
            "max_dW_per_atom": float(np.abs(g["virial"].reshape(3, 3) - ref["virial"]).max() / n),
            "max_dZ": float(np.abs(g["bec"].T.reshape(-1, 3, 3) - ref["bec"]).max()),
        }
        log(f"# crop errors {form}: " + ", ".join(f"{k}={v:.2e}" for k, v in res[form].items()))
        del model
    return {"workload": f"{w.name} (PPPM {'x'.join(map(str, w.es.mesh))}) vs FP64 oracle", "forms": res}


def workload_bench(torch, steps, warmup):
    """The other workloads of the method on one GPU: water-24,000 with PPPM 64^3 and with
    direct Ewald (27,200 wave vectors); garnet-153,600 with PPPM 128^3, forward and the
    adjoint (qnep_backward: forward recomputed plus the reverse pass); and NVE molecular
    dynamics of the water box (velocity Verlet, one full evaluation per step)."""
    import numpy as np

    from paper_2601_19034_amd import inputs
    from paper_2601_19034_amd.api import QNEP, to_device_inputs

    lines = []

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for wid, method in ((1, 1), (1, 0), (2, 1)):
        w = inputs.workload(wid, "full")
        w.es.method = method
        model = QNEP(w.hp, "fp32")
        pos, types, th = to_device_inputs(w.system, w.theta, "cuda:0")
        out = model.compute(pos, types, w.system.cell, th, w.es)
        if model.check_status():
            raise SystemExit(f"{w.name}: device status flags set")
        ms = timed(lambda: model.compute(pos, types, w.system.cell, th, w.es, out=out), steps)
        rec = {"workload": w.name, "n_atoms": w.system.n, "method": "PPPM" if method == 1 else "Ewald",
               "ms_per_step": ms, "atom_steps_per_s": w.system.n / (ms * 1e-3), "mlp": "fp32"}
        if method == 1:
            rec["mesh"] = list(w.es.mesh)
        else:
            rec["k_vectors"] = int(out["energy_terms"][7].item())
        if wid == 2:
            ms_b = timed(lambda: model.backward(pos, types, w.system.cell, th, w.es, 1.0, None,
                                                want=("pos", "cell", "theta")), max(steps // 2, 3))
            rec["adjoint_ms"] = ms_b
            rec["adjoint_atom_steps_per_s"] = w.system.n / (ms_b * 1e-3)
        log(f"# {w.name} {rec['method']}: {ms:.3f} ms/step ({rec['atom_steps_per_s']:.3e} atom-steps/s)"
            + (f", adjoint {rec['adjoint_ms']:.3f} ms" if "adjoint_ms" in rec else ""))
        lines.append(rec)
        del model, out
        torch.cuda.empty_cache()
    # NVE MD of the water box with PPPM: the paper's speed figures are MD rates
    w = inputs.workload(1, "full")
    model = QNEP(w.hp, "fp32")
    pos, types, th = to_device_inputs(w.system, w.theta, "cuda:0")
    masses = [15.999, 1.008]
    rng = np.random.default_rng(5)
    mt = np.array([masses[t] for t in w.system.types])
    v = rng.normal(size=(3, w.system.n)) * np.sqrt(0.025 / (mt * 103.6427))[None, :]
    vel = torch.from_numpy(v.astype(np.float32)).cuda()
    # the random-weight model has no physical repulsion, so the run is kept short (the
    # rate does not depend on the trajectory as long as no list overflows)
    md_steps, dt = 5 * steps, 0.25
    model.md_nve(pos, vel, types, w.system.cell, th, w.es, masses, dt, warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    model.md_nve(pos, vel, types, w.system.cell, th, w.es, masses, dt, md_steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / md_steps
    rec = {"workload": f"{w.name} NVE MD", "n_atoms": w.system.n, "method": "PPPM", "mesh": list(w.es.mesh),
           "dt_fs": dt, "steps": md_steps, "ms_per_step": ms, "atom_steps_per_s": w.system.n / (ms * 1e-3),
           "status_flags": model.check_status()}
    log(f"# {rec['workload']}: {ms:.3f} ms/step ({rec['atom_steps_per_s']:.3e} atom-steps/s), "
        f"{md_steps} steps of {dt} fs, status flags {rec['status_flags']}")
    lines.append(rec)
    return lines


def batch_bench(torch, reps=3):
    """The batched training evaluation: 512 uneven structures x 64 candidate parameter
    vectors, Ewald, in one persistent launch (plus the loss reduction); then the
    loss gradient (forward + adjoint launches).  Targets are seeded synthetic values;
    the work does not depend on them."""
    import numpy as np

    from paper_2601_19034_amd import inputs
    from paper_2601_19034_amd.api import QNEP, QNEPBatch

    wl = inputs.batch_workload()
    res = {}
    for form in ("fp32", "bf16"):
        model = QNEP(wl.hp, form)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        batch = QNEPBatch(model, wl.systems, wl.es, max_candidates=64, gradient=(form == "fp32"))
        e1.record()
        torch.cuda.synchronize()
        prep = e0.elapsed_time(e1)
        th = torch.from_numpy(wl.thetas.astype(np.float32)).cuda()
        rng = np.random.default_rng(7)
        E_ref = torch.from_numpy(rng.normal(-5.0, 1.0, batch.S) * batch.sizes).cuda()
        F_ref = torch.from_numpy(rng.normal(0, 1.0, (3, batch.n_total)).astype(np.float32)).cuda()
        choice = batch.tune(th, E_ref, F_ref)
        batch.compute(th, E_ref, F_ref)
        torch.cuda.synchronize()
        if batch.check_status():
            raise SystemExit("batched evaluation: device status flags set")
        e0.record()
        for _ in range(reps):
            batch.compute(th, E_ref, F_ref)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        evals = batch.n_total * th.shape[0]
        rec = {"ms_per_launch": ms, "atom_evaluations_per_s": evals / (ms * 1e-3), "prepare_ms": prep,
               "tuned": {"lanes_per_class": choice[:4], "workgroups_per_cu": choice[4]}}
        if form == "fp32":
            batch.gradient(th, E_ref, F_ref)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                batch.gradient(th, E_ref, F_ref)
            e1.record()
            torch.cuda.synchronize()
            rec["gradient_ms"] = e0.elapsed_time(e1) / reps
        res[form] = rec
        log(f"# batch {form}: {ms:.2f} ms per 512 x 64 launch ({evals / (ms * 1e-3):.3e} atom-evaluations/s), "
            f"prepare {prep:.1f} ms" + (f", gradient {rec['gradient_ms']:.2f} ms" if "gradient_ms" in rec else ""))
        del batch, model
        torch.cuda.empty_cache()
    return {"workload": f"{len(wl.systems)} structures ({int(sum(len(s.types) for s in wl.systems))} atoms) x "
                        f"{wl.thetas.shape[0]} candidates, Ewald", "forms": res}


def cpu_baseline(budget_s=12.0):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    a 20^3-cell (40,000-atom) perovskite box of the same generator, PPPM with a
    90^3 mesh (0.89 A spacing), full evaluation repeated until the budget is used."""
    import oracle
    from paper_2601_19034_amd import inputs

    oracle.build(force=False)
    sysm = inputs.perovskite_box(20, seed=inputs.SEED_BASE + 3, name="perovskite-40000")
    hp = inputs.PEROV_HP
    es = inputs.ESParams(mode=1, method=1, alpha=0.3, rc_coul=9.0, mesh=(90, 90, 90), order=5)
    th = inputs.theta0(hp, inputs.SEED_BASE + 3)
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.compute(hp, es, sysm.pos, sysm.types, sysm.cell, th, cells=True)
        reps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": sysm.n * reps / dt, "unit": "atom-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"perovskite 20^3 cells ({sysm.n} atoms), PPPM 90^3, FP64 oracle, {reps} evaluation(s) "
                      f"in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--variant", default="full")
    ap.add_argument("--method", choices=("pppm", "ewald"), default=None,
                    help="reciprocal-space method of the timed workload (default: the workload's own)")
    ap.add_argument("--forms", default="fp32,bf16x3,bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched (structures x candidates) line")
    ap.add_argument("--batch-only", action="store_true", help="only the batched line")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the water, garnet and MD lines and the per-form crop errors")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run three 1 GiB device copies first (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library evaluates one structure on one GPU; run with --gpus 1"}))
        sys.exit(2)

    import torch

    from paper_2601_19034_amd import inputs
    from paper_2601_19034_amd.api import QNEP, to_device_inputs

    if args.batch_only:  # the batched line alone (for profiling its kernels)
        print(json.dumps({"batch": batch_bench(torch)}), flush=True)
        return
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("# copy calibration: 3 x 1 GiB device-to-device copies")
        del a, b
    w = inputs.workload(args.workload, args.variant)
    if args.method is not None:
        w.es.method = 1 if args.method == "pppm" else 0
    n = w.system.n
    log(f"# workload {w.name}: N={n}, " + (f"mesh={w.es.mesh}" if w.es.method == 1 else f"Ewald kmax={w.es.kmax:.4f}"))
    pos, types, th = to_device_inputs(w.system, w.theta, "cuda:0")
    forms = {}
    stages = {}
    for form in args.forms.split(","):
        model = QNEP(w.hp, form)
        ms, wall_ms, ms_stage, launches, calls, energy = timed_run(model, pos, types, th, w, args.steps,
                                                                    args.warmup, torch)
        forms[form] = {"ms_per_step": ms, "atom_steps_per_s": n / (ms * 1e-3), "energy": energy}
        stages[form] = ({k: v / calls for k, v in ms_stage.items() if v > 0},
                        {k: v / calls for k, v in launches.items() if v > 0})
        log(f"# {form}: {ms:.3f} ms/step ({wall_ms:.3f} ms wall), E={energy:.6f}")
        log("#   " + ", ".join(f"{k}={v:.3f}" for k, v in sorted(stages[form][0].items(), key=lambda x: -x[1])))
        del model
        torch.cuda.empty_cache()

    head = "fp32" if "fp32" in forms else list(forms)[0]
    if "bf16x3" in forms and forms["bf16x3"]["ms_per_step"] < forms[head]["ms_per_step"]:
        head = "bf16x3"
    ms = forms[head]["ms_per_step"]
    # roofline of the dominant kernel (largest stage time of the headline form)
    st_ms, st_launch = stages[head]
    dom = max(st_ms, key=st_ms.get)
    roof = None
    t_launch = st_ms[dom] / st_launch[dom] * 1e-3
    if dom.startswith("angular_forces"):
        pairs = pair_counts(w.system, [w.hp.rc_A])[w.hp.rc_A]
        per_launch_flops = pairs * angular_flops_per_pair(w.hp)
        ach = per_launch_flops / t_launch / 1e12
        roof = {"bound": "alu", "kernel": "k_angular_forces", "achieved": ach,
                "peak": FP32_VALU_PEAK_TF, "unit": "TFLOP/s", "frac": ach / FP32_VALU_PEAK_TF,
                "traffic": traffic_from_profile("k_angular_forces", w.name, "nep.hip"),
                "units_per_launch": pairs, "flops_per_unit": angular_flops_per_pair(w.hp),
                "launch_ms": t_launch * 1e3}
    elif dom == "real_space":
        pairs = pair_counts(w.system, [w.es.rc_coul])[w.es.rc_coul]
        ach = pairs * REAL_SPACE_FLOPS_PER_PAIR / t_launch / 1e12
        roof = {"bound": "alu", "kernel": "k_real_space", "achieved": ach, "peak": FP32_VALU_PEAK_TF,
                "unit": "TFLOP/s", "frac": ach / FP32_VALU_PEAK_TF,
                "traffic": traffic_from_profile("k_real_space", w.name, "coul.hip"),
                "units_per_launch": pairs, "flops_per_unit": REAL_SPACE_FLOPS_PER_PAIR,
                "launch_ms": t_launch * 1e3}
    if roof is None:
        log(f"# no roofline model for the dominant stage {dom}")
    rec = {
        "metric": "atom-steps/s (E+F+virial+Z*) at 1M atoms PPPM",
        "value": n / (ms * 1e-3),
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else "bf16+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_atoms": n, "method": "PPPM" if w.es.method == 1 else "Ewald",
                   "mesh": list(w.es.mesh), "mlp": head},
        "forms": {k: {"atom_steps_per_s": v["atom_steps_per_s"], "ms_per_step": v["ms_per_step"]}
                  for k, v in forms.items()},
        "stage_ms": {k: round(v, 4) for k, v in stages[head][0].items()},
        "roofline": roof,
    }
    # the whole step against the per-atom-step budgets of the path (algorithmic FP32
    # operations and HBM bytes per atom-step for this workload, derived in the design notes)
    rec["step_roofline"] = {
        "flops_per_atom_step": STEP_FLOPS_PER_ATOM, "hbm_bytes_per_atom_step": STEP_BYTES_PER_ATOM,
        "valu_tflops": rec["value"] * STEP_FLOPS_PER_ATOM / 1e12,
        "valu_frac": rec["value"] * STEP_FLOPS_PER_ATOM / 1e12 / FP32_VALU_PEAK_TF,
        "hbm_gbs": rec["value"] * STEP_BYTES_PER_ATOM / 1e9,
        "hbm_frac": rec["value"] * STEP_BYTES_PER_ATOM / 1e9 / HBM_PEAK_GBS}
    if not args.no_workloads and args.workload == 3:
        rec["accuracy"] = crop_errors(torch, list(forms))
        rec["workloads"] = workload_bench(torch, args.steps, args.warmup)
    if not args.no_batch:
        rec["batch"] = batch_bench(torch)
    if not args.no_cpu_baseline:
        log("# cpu baseline (FP64 oracle)")
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
