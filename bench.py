#!/usr/bin/env python3
"""Benchmark: NNP energy + force throughput (atom-steps/s) on one MI355X.

One step is one full energy + force evaluation through the C ABI
(``nnp_compute``): cell list, neighbour lists, descriptors, per-species
networks (forward + backward), FP64 energy sum, descriptor adjoint and FP64
force gather.  The neighbour search reruns every step; inputs stay resident
in device memory.  The timed steps use the library's production path (one
HIP-graph replay per step); a second pass of the same length with per-stage
HIP events gives the kernel durations used for the roofline entry.

Default workload: periodic water box, 4,096 molecules (12,288 atoms,
L = 49.7 A), the FP32 form; the BF16 form is timed on the same input and both
are checked against the FP64 oracle (force relative RMSE, energy error per
atom).  ``--workload`` also accepts the 98,304- and 261,000-atom boxes and
the batch of 256 open H/C/N/O molecules.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NNP energy+force atom-steps/s (BF16 vs FP32 form) at stated force RMSE"

WORKLOADS = {
    "c1": dict(kind="water", n_mol=64, L=12.42, desc="periodic water box, 64 molecules (192 atoms), L=12.42 A"),
    "c2": dict(kind="water", n_mol=4096, L=49.7, desc="periodic water box, 4,096 molecules (12,288 atoms), L=49.7 A"),
    "c3": dict(kind="water", n_mol=32768, L=99.4, desc="periodic water box, 32,768 molecules (98,304 atoms), L=99.4 A"),
    "c5a": dict(kind="water", n_mol=87000, L=137.7,
                desc="periodic water box, 87,000 molecules (261,000 atoms), L=137.7 A"),
    "c4": dict(kind="batch", n_sys=256, desc="256 open H/C/N/O walk molecules of 24-300 atoms, one batched call"),
}

# Peaks (MI355X, published): HBM 8 TB/s; dense MFMA FP32 157.3 TFLOP/s, BF16 2.5 PFLOP/s.
# VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 lane-operations/s (unpacked FP32
# and FP64 issue at that rate; transcendentals at a quarter of it, counted as 4 operations).
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic VALU lane-operations per unit of work (transcendental = 4), derived in the design doc.
OPS_FWD_RAD_PAIR = 155
OPS_FWD_TRIPLET = 150
OPS_BWD_RAD_PAIR = 200
OPS_BWD_TRIPLET = 300


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def network_flops_per_atom(widths):
    """2 x multiply-adds of the forward chain plus the three backward products."""
    K0, N1, N2, N3 = widths[0], widths[1], widths[2], widths[3]
    fwd = K0 * N1 + N1 * N2 + N2 * N3 + N3
    bwd = N3 * N2 + N2 * N1 + N1 * K0
    return 2 * (fwd + bwd)


def build_inputs(name):
    import numpy as np
    import synthetic as sy
    w = WORKLOADS[name]
    if w["kind"] == "water":
        cfg = sy.model_config("water")
        pos, Z, box = sy.water_box(w["n_mol"], w["L"], seed=0)
        return cfg, dict(pos=pos, Z=Z, box=box, offsets=None)
    cfg = sy.model_config("hcno")
    pos, Z, off = sy.walk_batch(w["n_sys"], seed=0)
    return cfg, dict(pos=pos, Z=Z, box=None, offsets=np.asarray(off, np.int32))


def run_form(P, cfg, flat, inp, prec, steps, warmup, autotune=True):
    """Time `steps` production calls (HIP-graph replay, preallocated outputs, topology
    reused), then the same number of calls with per-stage HIP-event timing."""
    import numpy as np
    import torch
    m = P.NNPModel(cfg, weights=flat, precision=prec)
    d = torch.from_numpy(inp["pos"]).cuda()
    n = d.shape[0]
    batched = inp["offsets"] is not None
    if batched:
        n_sys = len(inp["offsets"]) - 1
        m.reserve(n, n_sys)
        E = torch.empty(n_sys, dtype=torch.float64, device="cuda")
        F = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        first = lambda: m.compute_batch(d, inp["Z"], inp["offsets"], out=(E, F))
        call = lambda: m.compute_batch(d, None, inp["offsets"], out=(E, F))
    else:
        m.reserve(n)
        E = torch.empty(1, dtype=torch.float64, device="cuda")
        F = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        first = lambda: m.compute(d, inp["Z"], inp["box"], out=(E, F, None))
        call = lambda: m.compute(d, None, inp["box"], out=(E, F, None))
    first()
    torch.cuda.synchronize()
    st = m.status()
    if st != 0:
        raise RuntimeError(f"device status {st} after the first call")
    E_first = E.detach().cpu().numpy().astype(float)
    F_first = F.detach().cpu().numpy()
    tuned = m.autotune(5) if autotune else None
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if m.status() != 0:
        raise RuntimeError("device status flagged an error during the timed steps")
    # per-stage event timing (stage launches issued directly; same kernels)
    P.nnp_profile_enable(m.h, steps)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    stage_ms, calls = P.nnp_profile_read(m.h)
    P.nnp_profile_enable(m.h, 0)
    cnt = m.read(P._lib.NNP_BUF_NBR_COUNT)
    out = {
        "ms_per_step": (t1 - t0) * 1e3 / steps,
        "profiled_ms_per_step": (tp1 - tp0) * 1e3 / steps,
        "stage_ms": {k: v / max(calls, 1) for k, v in stage_ms.items()},
        "E": E_first,
        "F": F_first,
        "rad_pairs": int(cnt[:, 0].sum()),
        "triplets": int((cnt[:, 1].astype(np.int64) * (cnt[:, 1] - 1) // 2).sum()),
        "n": n,
        "tuned": tuned,
    }
    m.close()
    return out


def oracle_reference(cfg, w, inp, sample_centres):
    """FP64 oracle energy/forces.  Full evaluation, or exact forces on sampled atoms."""
    import numpy as np
    import oracle as orc
    if inp["offsets"] is not None:
        E, F = orc.evaluate_batch(inp["pos"], inp["Z"], inp["offsets"], cfg, w)
        return {"E": E, "F": F, "atoms": np.arange(len(inp["Z"]))}
    if sample_centres is None:
        r = orc.evaluate(inp["pos"], inp["Z"], cfg, w, box=inp["box"])
        return {"E": np.array([r["E"]]), "F": r["F"], "atoms": np.arange(len(inp["Z"]))}
    I, J = orc.neighbour_pairs(inp["pos"], float(cfg["rc_rad"]), inp["box"], centres=sample_centres)
    cs = np.unique(np.concatenate([sample_centres, J]))
    r = orc.evaluate(inp["pos"], inp["Z"], cfg, w, box=inp["box"], centres=cs)
    return {"E": None, "F": r["F"], "atoms": sample_centres}


def cpu_baseline(cfg, w, inp, reps):
    """The oracle as it stands, timed on the host cores on a bounded sample of the workload."""
    import numpy as np
    import torch
    import oracle as orc
    n = len(inp["Z"])
    if inp["offsets"] is not None:
        off = inp["offsets"]
        k = min(16, len(off) - 1)
        sub = slice(0, int(off[k]))
        sample = f"first {k} molecules ({int(off[k])} atoms) of the batch, E+F, median of {reps}"
        atoms = int(off[k])
        fn = lambda: orc.evaluate_batch(inp["pos"][sub], inp["Z"][sub], off[:k + 1], cfg, w)
    elif n <= 20000:
        sample = f"full {n}-atom system, E+F, median of {reps}"
        atoms = n
        fn = lambda: orc.evaluate(inp["pos"], inp["Z"], cfg, w, box=inp["box"])
    else:
        rng = np.random.default_rng(0)
        cs = np.sort(rng.choice(n, 8192, replace=False))
        sample = f"atomic energies of 8,192 random atoms of the {n}-atom box and their gradients, median of {reps}"
        atoms = cs.size
        fn = lambda: orc.evaluate(inp["pos"], inp["Z"], cfg, w, box=inp["box"], centres=cs)
    # about 10 s of CPU work: at least `reps` evaluations, more when one is short
    t = time.perf_counter()
    fn()
    times = [time.perf_counter() - t]
    total = max(reps, min(30, math.ceil(10.0 / max(times[0], 1e-3))))
    for _ in range(total - 1):
        t = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t)
    sample = sample.replace(f"median of {reps}", f"median of {len(times)}")
    t = statistics.median(times)
    return {"value": atoms / t, "unit": "atom-steps/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": sample, "seconds_per_eval": t}


def roofline(res, widths, prec, stage):
    """Roofline entry for one stage from its live event time and its algorithmic work."""
    n = res["n"]
    t = res["stage_ms"][stage] * 1e-3
    D = widths[0]
    if stage == "network":
        flops = network_flops_per_atom(widths) * n
        ach = flops / t / 1e12
        return {"kernel": "k_mlp", "bound": "mfma", "achieved": ach, "peak": PEAK_MFMA_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": ach / PEAK_MFMA_TFLOPS[prec], "traffic": None,
                "algorithmic_per_launch": flops}
    if stage in ("adjoint", "descriptor"):
        if stage == "adjoint":
            ops = OPS_BWD_RAD_PAIR * res["rad_pairs"] + OPS_BWD_TRIPLET * res["triplets"]
            byts = n * (4 * D + 16) + 16 * res["rad_pairs"] + 24 * n
        else:
            ops = OPS_FWD_RAD_PAIR * res["rad_pairs"] + OPS_FWD_TRIPLET * res["triplets"]
            byts = n * (16 + 4 * D)
        ach = ops / t / 1e12
        return {"kernel": "k_desc_bwd" if stage == "adjoint" else "k_desc_fwd", "bound": "alu",
                "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TOP/s", "frac": ach / PEAK_VALU_TOPS,
                "traffic": None, "algorithmic_per_launch": ops, "hbm_GBs": byts / t / 1e9}
    # memory-bound stages
    byts = {"neighbours": n * 16 + 4 * res["rad_pairs"] + 8 * res["rad_pairs"],
            "gather": 16 * res["rad_pairs"] + 24 * n + 48 * n,
            "cells": 16 * n + 16 * n,
            "energy": 8 * (n // 16)}.get(stage, 16 * n)
    ach = byts / t / 1e9
    return {"kernel": stage, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": None, "algorithmic_per_launch": byts}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--form", default="fp32", choices=["fp32", "bf16"], help="form reported as `value`")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (no RMSE, no cpu_baseline)")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-autotune", action="store_true", help="use the built-in kernel variant choices")
    ap.add_argument("--nve", type=int, default=0,
                    help="also run this many velocity-Verlet NVE steps (dt 0.5 fs, 300 K) and report drift")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path.", file=sys.stderr)
        return 2
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: launched with WORLD_SIZE > 1; this build runs on one GPU only.", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import synthetic as sy
    import paper_2604_21441_amd as P

    if args.calib_copy:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": nbytes, "launches": 5}))
        return 0

    torch.set_num_threads(len(os.sched_getaffinity(0)))
    cfg, inp = build_inputs(args.workload)
    w = sy.model_weights(cfg, seed=1)
    flat = sy.flat_weights(w)
    widths = list(cfg["widths"])
    n = len(inp["Z"])
    log(f"[bench] workload {args.workload}: {WORKLOADS[args.workload]['desc']} ({n} atoms)")

    forms = {}
    for prec in ("fp32", "bf16"):
        log(f"[bench] timing {prec}: {args.warmup} warmup + {args.steps} steps")
        forms[prec] = run_form(P, cfg, flat, inp, prec, args.steps, args.warmup, not args.no_autotune)
        log(f"[bench] {prec}: {forms[prec]['ms_per_step']:.4f} ms/step, "
            f"{n / forms[prec]['ms_per_step'] * 1e3:.4e} atom-steps/s")

    report_forms = {}
    ref = None
    if not args.no_cpu:
        log("[bench] oracle reference")
        sample = None
        if args.workload in ("c3", "c5a"):
            sample = np.sort(np.random.default_rng(1).choice(n, 64, replace=False))
        ref = oracle_reference(cfg, w, inp, sample)
    for prec, r in forms.items():
        entry = {"atom_steps_per_s": n / r["ms_per_step"] * 1e3, "ms_per_step": r["ms_per_step"],
                 "profiled_ms_per_step": r["profiled_ms_per_step"], "stage_ms": r["stage_ms"],
                 "tuned_variants": r["tuned"]}
        if ref is not None:
            a = ref["atoms"]
            dF = r["F"][a] - ref["F"][a]
            entry["force_rel_rmse"] = float(np.linalg.norm(dF) / np.linalg.norm(ref["F"][a]))
            entry["force_rmse_eV_per_A"] = float(np.sqrt(np.mean(dF ** 2)))
            if ref["E"] is not None:
                sizes = np.diff(inp["offsets"]) if inp["offsets"] is not None else np.array([n])
                entry["energy_err_per_atom_eV"] = float(np.max(np.abs(r["E"] - ref["E"]) / sizes))
            entry["rmse_over"] = "all atoms" if a.size == n else f"{a.size} sampled atoms"
        report_forms[prec] = entry
    r32, r16 = forms["fp32"], forms["bf16"]
    report_forms["bf16"]["force_rel_rmse_vs_fp32"] = float(np.linalg.norm(r16["F"] - r32["F"]) /
                                                           np.linalg.norm(r32["F"]))
    report_forms["bf16"]["speedup_vs_fp32"] = r32["ms_per_step"] / r16["ms_per_step"]

    main_form = forms[args.form]
    dom = max(main_form["stage_ms"], key=lambda k: main_form["stage_ms"][k])
    roof = roofline(main_form, widths, args.form, dom)
    stage_roofs = {s: roofline(main_form, widths, args.form, s) for s in ("descriptor", "network", "adjoint")}

    cpu = None
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle on host cores)")
        cpu = cpu_baseline(cfg, w, inp, args.cpu_reps)
        log(f"[bench] cpu: {cpu['value']:.4e} atom-steps/s on {cpu['cores']} threads")

    nve = None
    if args.nve > 0 and inp["offsets"] is None:
        from paper_2604_21441_amd.md import run_nve
        log(f"[bench] NVE: {args.nve} steps, dt 0.5 fs, {args.form}")
        masses = np.array([sy.WATER_MASS[int(z)] for z in inp["Z"]])
        v0 = sy.maxwell_boltzmann(inp["Z"], 300.0, seed=2)
        mdl = P.NNPModel(cfg, weights=flat, precision=args.form)
        r = run_nve(mdl, inp["pos"], inp["Z"], inp["box"], masses, v0, dt=0.5, steps=args.nve)
        mdl.close()
        nve = {"steps": args.nve, "dt_fs": 0.5, "drift_eV_per_atom_per_ps": r["drift_eV_per_atom_per_ps"],
               "max_abs_dev_eV_per_atom": r["max_abs_dev_eV_per_atom"], "ms_per_step": r["ms_per_step"],
               "T_start_K": 300.0}
        log(f"[bench] NVE drift {r['drift_eV_per_atom_per_ps']:.3e} eV/atom/ps, {r['ms_per_step']:.3f} ms/step")

    value = n / main_form["ms_per_step"] * 1e3
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.form,
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload]["desc"] + f", {args.form.upper()} form",
                   "atoms": n, "form": args.form, "seeds": {"geometry": 0, "weights": 1}},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": report_forms,
        "stage_roofline": stage_roofs,
        "nve": nve,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
