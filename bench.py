#!/usr/bin/env python3
"""Throughput of the per-electron PIC step with MC photon emission on one
MI355X, in electron-steps/s.

Default workload: the 2D3V gold-slab configuration (2048x1024 cells at
lambda/64, Au q=69 slab 2 um thick at n_e = 200 n_c, 16 electrons/cell =
2,097,152 electrons, a0 = 270 Gaussian w0 = 3 um, 2000 steps), FP32 bulk with
FP64 optical depth, weights and energy sums; the same run in FP64 is timed
beside it.  A "step" is one full step of every electron (gather, push, eta,
NCS, bremsstrahlung, recoil, append, move + deposit) plus the field solve.

    python bench.py [--gpus 1] [--steps 2000] [--warmup 20]

Prints one JSON line.  The timed region starts from a freshly created
context (all state already resident in HBM) and covers exactly --steps
steps, bracketed by torch.cuda.synchronize().
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Non-packed FP32 (and FP64) VALU issue of MI355X: 256 CU x 4 SIMD x 16 lanes
# x 2.4 GHz, one lane operation per lane and cycle (packed FP32 is disabled).
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic lane operations per electron-step that every live electron
# executes (gather, Boris, eta, NCS decrement, move, deposit, stats), quarter-
# rate operations counted 4; the conditional brem test and event sampling are
# not included
ALU_OPS = {1: 292, 2: 548, 3: 1366}
KERNEL_SOURCES = ["step.hip", "pic_internal.hpp", "philox.hpp"]
# algorithmic bytes per electron-step of the step kernel: the electron state
# read once (positions, momenta, tau, weight, id) and written once (positions,
# momenta, tau); fields and tables are amortised over the electrons of a cell
STATE_BYTES = {("fp32", 1): 60, ("fp32", 2): 68, ("fp32", 3): 76,
               ("fp64", 1): 92, ("fp64", 2): 108, ("fp64", 3): 124}


def _workload(name, precision, steps):
    from paper_1612_07592_amd import workloads as W
    if name == "c2":
        w = W.c2(steps=steps, precision=precision)
    elif name == "c1":
        w = W.c1(steps)
        w["precision"] = precision
    elif name == "c5":
        w = W.c5(steps)
        w["precision"] = precision
    elif name == "thick":
        w = W.thick_target(steps, precision)
    else:
        raise SystemExit(f"unknown workload {name}")
    return w


def _kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1612_07592_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _measured_traffic(workload, precision):
    """Calibrated HBM-counter bytes per launch of the step kernel, from the
    committed rocprofv3 summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    for e in d.get("entries", []):
        if (e["kernel_sha"] == _kernel_hash() and e["workload"] == workload
                and e["precision"] == precision):
            return e["bytes_per_launch"]
    return None


def _num_electrons(w):
    from paper_1612_07592_amd import workloads as W
    return W.num_electrons(w)


def _pencil_beam(w):
    """Electrons of a thick-target recipe as a pencil beam along +x at the
    front face, kinetic energy w["beam_energy_mev"] (set before timing)."""
    import numpy as np

    def f(s):
        e = s.electrons()
        x = np.zeros_like(e["x"])
        x[:, 0] = (np.arange(s.N) % 1024 + 0.5) / 1024 * 2 * np.pi * w["dx_lambda"][0]
        T = w["beam_energy_mev"] / 0.51099895
        p = np.zeros_like(e["p"])
        p[:, 0] = (T * (T + 2.0)) ** 0.5
        s.set_electrons(x, p, e["tau"])
    return f if "beam_energy_mev" in w else None


def run_gpu(w, tables, steps, warmup, torch, photons=False, kernel_times=True):
    """Time `steps` steps from a fresh context.  The wall-clock run records no
    events; a second identical run, with HIP events on the context's stream
    around every launch group, gives the per-kernel times."""
    from paper_1612_07592_amd import binding
    beam = _pencil_beam(w)
    if warmup > 0:
        s = binding.Sim(w, tables)
        if beam:
            beam(s)
        s.pic_step(warmup)
        s.pic_emission_stats()
        s.pic_destroy()
    s = binding.Sim(w, tables)
    if beam:
        beam(s)
    s.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.pic_step(steps)
    s.synchronize()          # libpic's own HIP runtime (torch's does not see its queues)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = s.pic_emission_stats()
    ph = s.photons() if photons else None
    s.pic_destroy()
    out = dict(wall_s=t1 - t0, stats=st, photons=ph, step_kernel_ms=None, field_ms=None,
               sort_ms=None, step_launches=0)
    if kernel_times:
        s = binding.Sim(w, tables)
        if beam:
            beam(s)
        s.profile(True)
        s.pic_step(steps)
        ms, n = s.profile_read()
        s.pic_destroy()
        out.update(step_kernel_ms=float(ms[0]), field_ms=float(ms[1]), sort_ms=float(ms[2]),
                   step_launches=int(n[0]), profiled_wall_ms=float(ms.sum()))
    return out


def thick_target_line(args, tables, torch):
    """Bremsstrahlung-dominated workload: 100 MeV pencil beam of 2.1M
    electrons into 5 mm of solid gold, particle-only, FP32, 2000 steps; the
    per-step Eq. (4) trial against the free-path form."""
    from paper_1612_07592_amd import workloads as W
    res = {"workload": "thick-au-5mm", "electrons": None, "steps": 2000}
    for form, fp in (("per_step_trial", False), ("free_path", True)):
        w = W.thick_target(2000, "fp32")
        w["brem_freepath"] = fp
        r = run_gpu(w, tables, 2000, 0, torch, kernel_times=True)
        st = r["stats"]
        res["electrons"] = _num_electrons(w)
        res[form] = {"value": st["electron_steps"] / r["wall_s"],
                     "kernel_avg_us": r["step_kernel_ms"] * 1e3 / max(1, r["step_launches"]),
                     "brem_events": st["events"][1], "e_rad_brem": st["e_rad_kept"][1]}
    res["free_path_speedup"] = res["free_path"]["value"] / res["per_step_trial"]["value"]
    print(f"[bench] thick target: per-step {res['per_step_trial']['value']:.3e}, free path "
          f"{res['free_path']['value']:.3e} e-steps/s ({res['free_path_speedup']:.2f}x)",
          file=sys.stderr, flush=True)
    return res


def precision_check(r32, r64):
    """FP32-mixed against FP64 on the same workload and Philox streams:
    kept-photon count within 3 sigma (Poisson), photon-energy spectrum
    two-sample KS p > 0.01, total radiated energy within 1%."""
    from scipy import stats as sst
    s32, s64 = r32["stats"], r64["stats"]
    n32, n64 = sum(s32["kept"]), sum(s64["kept"])
    sigma = max(n64, 1) ** 0.5
    e32 = s32["e_rad_kept"][0] + s32["e_rad_kept"][1] + s32["e_rad_dropped"]
    e64 = s64["e_rad_kept"][0] + s64["e_rad_kept"][1] + s64["e_rad_dropped"]
    out = {"photon_count": {"fp32": n32, "fp64": n64, "z": (n32 - n64) / sigma,
                            "pass": abs(n32 - n64) <= 3 * sigma},
           "radiated_energy": {"fp32": e32, "fp64": e64, "rel": (e32 - e64) / e64 if e64 else None,
                               "pass": bool(e64) and abs(e32 - e64) <= 0.01 * abs(e64)}}
    p32, p64 = r32["photons"], r64["photons"]
    if p32 is not None and p64 is not None and len(p32["energy"]) and len(p64["energy"]):
        ks = sst.ks_2samp(p32["energy"], p64["energy"])
        out["spectrum_ks"] = {"statistic": float(ks.statistic), "p": float(ks.pvalue),
                              "n": [len(p32["energy"]), len(p64["energy"])],
                              "pass": float(ks.pvalue) > 0.01}
    else:
        out["spectrum_ks"] = {"p": None, "pass": None, "n": [0, 0]}
    return out


def serving(args, torch):
    """Scan jobs through the continuous-batching server: the 8-job
    intensity x target batch (FP32, FP64, and FP32 one job after another),
    then the first --c4-jobs jobs of the Poisson stream."""
    from paper_1612_07592_amd import binding, serving as SV
    from paper_1612_07592_amd import workloads as W
    tb = {13: binding.pic_build_tables(13, 1.0, 16), 79: binding.pic_build_tables(79, 1.0, 16)}
    log = lambda m: print(f"[serve] {m}", file=sys.stderr, flush=True)
    out = {}
    jobs = W.c3_jobs(args.c3_steps)
    _, out["c3_fp32"] = SV.run_batch(jobs, tb)
    log(f"c3 fp32 {out['c3_fp32']['electron_steps_per_s']:.3e} e-steps/s")
    _, out["c3_fp64"] = SV.run_batch([dict(w, precision="fp64") for w in jobs], tb)
    log(f"c3 fp64 {out['c3_fp64']['electron_steps_per_s']:.3e} e-steps/s")
    out["c3_fp32_sequential"] = SV.run_sequential(jobs, tb)
    log(f"c3 fp32 one at a time {out['c3_fp32_sequential']['electron_steps_per_s']:.3e} e-steps/s")
    if args.c4_jobs > 0:
        arr = W.c4_stream()[:args.c4_jobs]
        _, c4 = SV.run_stream(arr, tb, log=log)
        offered = sum(W.num_electrons(w) * w["steps"] for _, w in arr) / max(arr[-1][0], 1e-9)
        c4["offered_electron_steps_per_s"] = offered
        c4["arrival_rate_per_s"] = 4.0
        out["c4_stream"] = c4
        log(f"c4 {c4['jobs']} jobs: p50 {c4['latency_p50_s']:.2f} s p99 {c4['latency_p99_s']:.2f} s "
            f"{c4['electron_steps_per_s']:.3e} e-steps/s")
    out["scan_fp32_over_fp64"] = out["c3_fp32"]["electron_steps_per_s"] / out["c3_fp64"]["electron_steps_per_s"]
    return out


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle, as is, on the host cores: a bounded number of steps of
    the same workload from t = 0."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import conftest
    import oracle
    oracle.build(force=False)
    tables = conftest.oracle_tables(int(w["Z"]))
    ww = dict(w)
    ww["precision"] = "fp64"
    ww["photon_capacity"] = 1 << 22
    nt = min(16, os.cpu_count() or 1)
    o = oracle.OracleSim(ww, tables, nthreads=nt)
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    k = max(1, min(200, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t0
    live = o.stats()["live"]
    o.close()
    return dict(value=live * k / dt, unit="electron-steps/s", cores=nt, kind="oracle",
                sample=f"FP64 oracle, steps 1..{k + 1} of the same workload from t=0 "
                       f"({live} electrons, {dt:.1f} s on {nt} threads)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sort-every", type=int, default=0,
                    help="tile-sort interval in steps (0 = library default, -1 = never)")
    ap.add_argument("--no-serving", action="store_true", help="skip the scan-job server runs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--c3-steps", type=int, default=1000)
    ap.add_argument("--brem-freepath", action="store_true",
                    help="time the free-path form of the bremsstrahlung test instead of the per-step trial")
    ap.add_argument("--no-freepath-line", action="store_true",
                    help="skip the free-path bremsstrahlung run reported beside the main one")
    ap.add_argument("--c4-jobs", type=int, default=24,
                    help="jobs of the Poisson stream served (0 = none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is a "
                                   "design note, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1612_07592_amd import binding
    binding.load()
    if args.copy_calibration > 0:
        n = args.copy_calibration << 18
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)  # an elementwise kernel: reads and writes n floats
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {n * 4} bytes read, {n * 4} written", file=sys.stderr, flush=True)
        del a, b
    w = _workload(args.workload, args.precision, args.steps)
    if args.sort_every or "sort_every" not in w:
        w["sort_every"] = args.sort_every
    w["brem_freepath"] = args.brem_freepath
    t0 = time.perf_counter()
    tables = binding.pic_build_tables(int(w["Z"]), 1.0, 16)
    t_tables = time.perf_counter() - t0
    print(f"[bench] tables built in {t_tables:.1f} s; {args.workload} {args.precision} "
          f"{args.steps} steps", file=sys.stderr, flush=True)
    r = run_gpu(w, tables, args.steps, args.warmup, torch, photons=not args.no_fp64)
    st = r["stats"]
    esteps = int(st["electron_steps"])
    value = esteps / r["wall_s"]
    dims = int(w["dims"])
    bpe = STATE_BYTES[(args.precision, dims)]
    achieved = bpe * esteps / (r["step_kernel_ms"] * 1e-3) / 1e9
    ops = ALU_OPS[dims]
    alu = ops * esteps / (r["step_kernel_ms"] * 1e-3) / 1e12
    launches = max(1, r["step_launches"])
    out = {
        "metric": "electron-steps/s",
        "value": value,
        "unit": "electron-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "dims": dims, "cells": list(w["n"]),
                   "electrons": _num_electrons(w),
                   "precision": args.precision, "a0": w["a0"], "Z": w["Z"],
                   "brem": "free-path" if args.brem_freepath else "per-step trial"},
        "roofline": {"bound": "alu", "achieved": alu, "peak": ALU_PEAK_TOPS, "unit": "TFLOP/s",
                     "frac": alu / ALU_PEAK_TOPS,
                     "traffic": _measured_traffic(w["name"], args.precision),
                     "kernel": f"k_electron_step<{'float' if args.precision == 'fp32' else 'double'},{dims}>",
                     "ops_per_electron_step": ops,
                     "electron_steps_per_launch": esteps / launches,
                     "kernel_avg_us": r["step_kernel_ms"] * 1e3 / launches,
                     "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved / HBM_PEAK_GBS, "bytes_per_electron_step": bpe}},
        "time_share": {"electron_step": r["step_kernel_ms"] / (r["wall_s"] * 1e3),
                       "field_solve": r["field_ms"] / (r["wall_s"] * 1e3),
                       "sort": r["sort_ms"] / (r["wall_s"] * 1e3)},
        "kernel_ms": {"electron_step": r["step_kernel_ms"], "field_solve": r["field_ms"],
                      "sort": r["sort_ms"]},
        "untiled_fraction": st["untiled_steps"] / max(1, esteps),
        "emission": {"events": st["events"], "kept": st["kept"], "dropped_ncs": st["dropped_ncs"],
                     "overflow": st["overflow"], "e_rad_kept": st["e_rad_kept"]},
    }
    print(f"[bench] {args.precision}: {value:.3e} e-steps/s, step kernel "
          f"{out['roofline']['kernel_avg_us']:.1f} us, {alu:.2f} Tops/s, {achieved:.0f} GB/s",
          file=sys.stderr, flush=True)
    if not args.no_freepath_line and not args.brem_freepath:
        # the same workload with the free-path form of the collision test
        rf = run_gpu(dict(w, brem_freepath=True), tables, args.steps, 0, torch, kernel_times=True)
        vf = rf["stats"]["electron_steps"] / rf["wall_s"]
        out["brem_free_path"] = {
            "value": vf, "over_per_step_trial": vf / value,
            "kernel_avg_us": rf["step_kernel_ms"] * 1e3 / max(1, rf["step_launches"]),
            "events": rf["stats"]["events"], "kept": rf["stats"]["kept"]}
        print(f"[bench] free-path brem: {vf:.3e} e-steps/s ({vf / value:.3f}x)", file=sys.stderr, flush=True)
    if not args.no_freepath_line and args.workload == "c2":
        out["thick_target"] = thick_target_line(args, tables, torch)
    if not args.no_fp64 and args.precision == "fp32":
        w64 = _workload(args.workload, "fp64", args.steps)
        w64["sort_every"] = w["sort_every"]
        w64["brem_freepath"] = args.brem_freepath
        r64 = run_gpu(w64, tables, args.steps, 0, torch, photons=True, kernel_times=True)
        v64 = r64["stats"]["electron_steps"] / r64["wall_s"]
        out["fp64"] = {"value": v64, "ms_per_step": r64["wall_s"] * 1e3 / args.steps,
                       "kernel_avg_us": r64["step_kernel_ms"] * 1e3 / max(1, r64["step_launches"]),
                       "events": r64["stats"]["events"], "kept": r64["stats"]["kept"]}
        out["fp32_over_fp64"] = value / v64
        out["fp32_vs_fp64"] = precision_check(r, r64)
        # run-to-run spread of the full PIC run: FP64 with the next two seeds
        refs = []
        for k in (1, 2):
            rref = run_gpu(dict(w64, seed=int(w64["seed"]) + k), tables, args.steps, 0, torch,
                           photons=True, kernel_times=False)
            refs.append(precision_check(rref, r64))
        pc = out["fp32_vs_fp64"]
        pc["reference_fp64_other_seeds"] = refs
        dn = max(abs(q["photon_count"]["fp32"] - q["photon_count"]["fp64"]) for q in refs)
        de = max(abs(q["radiated_energy"]["rel"]) for q in refs)
        dk = max(q["spectrum_ks"]["statistic"] or 0.0 for q in refs)
        n64 = pc["photon_count"]["fp64"]
        pc["within_seed_spread"] = {
            "photon_count": abs(pc["photon_count"]["fp32"] - n64) <= 2.0 * max(dn, 3.0 * n64 ** 0.5),
            "radiated_energy": abs(pc["radiated_energy"]["rel"]) <= max(0.01, 2.0 * de),
            "spectrum_ks": (pc["spectrum_ks"]["statistic"] or 0.0) <= 2.0 * dk}
        print(f"[bench] fp64: {v64:.3e} e-steps/s; {out['fp32_vs_fp64']}", file=sys.stderr, flush=True)
    if not args.no_serving and args.workload == "c2":
        out["serving"] = serving(args, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(_workload(args.workload, "fp64", args.steps))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
