#!/usr/bin/env python3
"""Throughput of the per-electron PIC step with MC photon emission on one
MI355X, in electron-steps/s.

Headline workload: the 2D3V gold-slab configuration (2048x1024 cells at
lambda/64, Au q=69 slab 2 um thick at n_e = 200 n_c, 16 electrons/cell =
2,097,152 electrons, a0 = 270 Gaussian w0 = 3 um, 2000 steps), FP32 bulk with
FP64 optical depth, weights and energy sums, with the same run in FP64 beside
it.  A "step" is one full step of every electron (gather, push, eta, NCS,
bremsstrahlung, recoil, append, move + deposit) plus the field solve and the
periodic tile sort.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

The K timed steps are a window of the workload's own run, placed so that it is
centred on the step at which the peak of the laser envelope reaches the slab
front (the laser-plasma interaction, where emission happens); the steps
before the window are an untimed lead-in on the same context ("lead_in_steps"
in the output).  K >= the workload's length times the whole run.  W warm-up
steps run first on a separate context.  The timed region starts with all state
resident in HBM and is bracketed by a synchronisation of libpic's stream and
torch.cuda.synchronize().

Beside the headline, the JSON line carries (each leg's failure is recorded in
"errors" and never suppresses the line):
  fp64 / fp32_over_fp64  the same window in FP64;
  full_run               the whole 2000-step run in both precisions, with the
                         FP32-vs-FP64 criteria (photon count within 3 sigma,
                         spectrum KS p > 0.01, radiated energy within 1%) and
                         two more FP64 seeds as the run-to-run spread;
  roofline               the electron-step kernel on the 3D gold slab (134M
                         electrons, whose 10 GB of state no cache holds), HBM
                         bound: algorithmic bytes per launch / average launch
                         time from HIP events on the kernel's stream;
  cpu_baseline           the FP64 oracle on the host over the same window of a
                         transverse slice of the headline workload;
  serving, thick_target  scan-job server runs and the bremsstrahlung benchmark;
  solid                  (--only solid) the laser-solid study of Sec. III at
                         its own size, with mobile ions: throughput and energy
                         partition of every run;
  pairs                  (--only pairs) the gold run at 10^24 W/cm^2 with
                         photons in flight and pair production.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time
import traceback

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Non-packed FP32 (and FP64) VALU issue of MI355X: 256 CU x 4 SIMD x 16 lanes
# x 2.4 GHz, one lane operation per lane and cycle (packed FP32 is disabled).
ALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# wave64 VALU instructions per second: 256 CUs x 4 SIMDs, one instruction per SIMD every 4 cycles
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
# algorithmic lane operations per electron-step that every live electron
# executes (gather, Boris, eta, NCS decrement, move, deposit, stats), quarter-
# rate operations counted 4; the conditional brem test and event sampling are
# not included.  An estimate from the method, not a counter.
ALU_OPS = {1: 292, 2: 548, 3: 1366}
KERNEL_SOURCES = ["step.hip", "particle.hpp", "pic_internal.hpp", "philox.hpp", "fpmath.hpp"]
# algorithmic bytes per electron-step of the step kernel: the electron state
# read once (positions, momenta, tau, weight, id) and written once (positions,
# momenta, tau); fields and tables are amortised over the electrons of a cell
STATE_BYTES = {("fp32", 1): 60, ("fp32", 2): 68, ("fp32", 3): 76,
               ("fp64", 1): 92, ("fp64", 2): 108, ("fp64", 3): 124}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _workload(name, precision, steps=None):
    from paper_1612_07592_amd import workloads as W
    if name == "c2":
        w = W.c2(precision=precision)
    elif name == "c1":
        w = W.c1()
    elif name == "c5":
        w = W.c5()
    elif name == "thick":
        w = W.thick_target(precision=precision)
    else:
        raise SystemExit(f"unknown workload {name}")
    w["precision"] = precision
    if steps is not None:
        w["steps"] = steps
    return w


def step_dt(w):
    """Time step in 1/omega0 (cell sizes in c/omega0 = lambda / (2 pi))."""
    dx = [d * 2.0 * math.pi for d in w["dx_lambda"][:w["dims"]]]
    return w.get("cfl", 0.95) / math.sqrt(sum(1.0 / (d * d) for d in dx))


def peak_step(w):
    """Step at which the peak of the sin^2 envelope (emitted at the left
    boundary at half the pulse length) reaches the slab front."""
    t = math.pi * w.get("duration_cycles", 10.0) + 2.0 * math.pi * w["x0_lambda"]
    return int(round(t / step_dt(w)))


def window(w, k):
    """(lead_in, k) of a k-step window centred on peak_step, inside the run."""
    total = int(w["steps"])
    if k >= total:
        return 0, k
    lead = peak_step(w) - k // 2
    return max(0, min(lead, total - k)), k


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
                and e["precision"] == precision and e.get("bytes_per_launch")):
            return e
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


def _esteps(s):
    return int(s.pic_emission_stats()["electron_steps"])


def run_window(w, tables, lead, k, torch, warmup=0, photons=False, events=True, wall=True):
    """Lead-in of `lead` untimed steps, then k steps timed on the wall clock
    (no events recorded), on a fresh context; optionally a second identical
    context whose k window steps carry HIP events for per-kernel times (the
    events are recorded on libpic's stream, around every launch group)."""
    from paper_1612_07592_amd import binding
    beam = _pencil_beam(w)
    out = dict(lead_in=lead, steps=k)
    if warmup > 0:
        s = binding.Sim(w, tables)
        if beam:
            beam(s)
        s.pic_step(warmup)
        s.synchronize()
        s.pic_destroy()
    if wall:
        s = binding.Sim(w, tables)
        if beam:
            beam(s)
        if lead:
            s.pic_step(lead)
        s.synchronize()
        e0 = _esteps(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.pic_step(k)
        s.synchronize()          # libpic's own HIP runtime (torch's does not see its queues)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = s.pic_emission_stats()
        out.update(wall_s=t1 - t0, window_esteps=int(st["electron_steps"]) - e0, stats=st,
                   photons=s.photons() if photons else None)
        s.pic_destroy()
    if events:
        s = binding.Sim(w, tables)
        if beam:
            beam(s)
        if lead:
            s.pic_step(lead)
        s.synchronize()
        e0 = _esteps(s)
        s.profile(True)
        s.pic_step(k)
        ms, n = s.profile_read()
        st = s.pic_emission_stats()
        if not wall:
            out.update(stats=st, photons=s.photons() if photons else None)
        s.pic_destroy()
        out.update(window_esteps=int(st["electron_steps"]) - e0,
                   step_kernel_ms=float(ms[0]), field_ms=float(ms[1]), sort_ms=float(ms[2]),
                   ion_ms=float(ms[3]), photon_ms=float(ms[4]), step_launches=int(n[0]),
                   profiled_ms=float(ms.sum()))
    return out


def precision_check(s32, s64, p32=None, p64=None):
    """FP32-mixed against FP64 on the same workload and Philox streams, each
    criterion stated per result: kept-photon count within 3 sigma (Poisson),
    photon-energy spectrum two-sample KS p > 0.01, total radiated energy
    within 1%.  Missing data (no photons yet) gives None, never an error."""
    n32, n64 = sum(s32["kept"]), sum(s64["kept"])
    sigma = max(n64, 1) ** 0.5
    e32 = s32["e_rad_kept"][0] + s32["e_rad_kept"][1] + s32["e_rad_dropped"]
    e64 = s64["e_rad_kept"][0] + s64["e_rad_kept"][1] + s64["e_rad_dropped"]
    out = {"photon_count": {"fp32": n32, "fp64": n64, "z": (n32 - n64) / sigma,
                            "pass": abs(n32 - n64) <= 3 * sigma},
           "radiated_energy": {"fp32": e32, "fp64": e64,
                               "rel": (e32 - e64) / e64 if e64 else None,
                               "pass": (abs(e32 - e64) <= 0.01 * abs(e64)) if e64 else None}}
    ks = {"statistic": None, "p": None, "pass": None, "n": [0, 0]}
    if p32 is not None and p64 is not None and len(p32["energy"]) and len(p64["energy"]):
        from scipy import stats as sst
        r = sst.ks_2samp(p32["energy"], p64["energy"])
        ks = {"statistic": float(r.statistic), "p": float(r.pvalue),
              "n": [len(p32["energy"]), len(p64["energy"])], "pass": float(r.pvalue) > 0.01}
    out["spectrum_ks"] = ks
    out["spectrum_all_kept"] = binned_spectra(s32, s64)
    if n64 == 0 and n32 == 0:
        out["note"] = "no photons kept in this window"
    return out


def binned_spectra(s32, s64):
    """The kept-photon spectra of the statistics (every kept photon, stored
    in the buffer or not, in quarter-octave bins; NCS and bremsstrahlung
    pooled): the largest difference of the two binned distribution
    functions and the chi-square homogeneity p-value of the 2 x bins table."""
    import numpy as np
    a = np.asarray(s32.get("spectrum", np.zeros((2, 64))), dtype=np.float64).sum(axis=0)
    b = np.asarray(s64.get("spectrum", np.zeros((2, 64))), dtype=np.float64).sum(axis=0)
    res = {"n": [int(a.sum()), int(b.sum())], "D": None, "chi2_p": None, "pass": None}
    if a.sum() == 0 or b.sum() == 0:
        return res
    D = float(np.abs(np.cumsum(a) / a.sum() - np.cumsum(b) / b.sum()).max())
    keep = (a + b) > 0
    from scipy import stats as sst
    chi2, p, _, _ = sst.chi2_contingency(np.vstack([a[keep], b[keep]]))
    res.update(D=D, chi2_p=float(p), pass_=None)
    res.pop("pass_")
    res["pass"] = float(p) > 0.01
    return res


def _max_or_none(vals):
    vals = [v for v in vals if v is not None]
    return max(vals) if vals else None


def seed_spread(pc, refs):
    """Each FP32 difference against twice the largest difference between the
    FP64 run and FP64 runs with other seeds (None where a figure is absent)."""
    n64 = pc["photon_count"]["fp64"]
    dn = _max_or_none([abs(q["photon_count"]["fp32"] - q["photon_count"]["fp64"]) for q in refs])
    de = _max_or_none([abs(q["radiated_energy"]["rel"]) if q["radiated_energy"]["rel"] is not None
                       else None for q in refs])
    dk = _max_or_none([q["spectrum_ks"]["statistic"] for q in refs])
    rel = pc["radiated_energy"]["rel"]
    ks = pc["spectrum_ks"]["statistic"]
    db = _max_or_none([q.get("spectrum_all_kept", {}).get("D") for q in refs])
    bd = pc.get("spectrum_all_kept", {}).get("D")
    return {
        "spectrum_all_kept": (bd <= 2.0 * db) if (bd is not None and db) else None,
        "photon_count": abs(pc["photon_count"]["fp32"] - n64) <= 2.0 * max(dn or 0, 3.0 * n64 ** 0.5),
        "radiated_energy": (abs(rel) <= max(0.01, 2.0 * (de or 0.0))) if rel is not None else None,
        "spectrum_ks": (ks <= 2.0 * dk) if (ks is not None and dk) else None}


def full_run_leg(w32, tables, torch):
    """The whole run in FP32 and FP64 (wall clock), the FP32-vs-FP64 criteria
    on it, and FP64 with the next two seeds as the run-to-run spread."""
    total = int(w32["steps"])
    r32 = run_window(w32, tables, 0, total, torch, photons=True, events=False)
    w64 = dict(w32, precision="fp64")
    r64 = run_window(w64, tables, 0, total, torch, photons=True, events=False)
    v32 = r32["window_esteps"] / r32["wall_s"]
    v64 = r64["window_esteps"] / r64["wall_s"]
    pc = precision_check(r32["stats"], r64["stats"], r32["photons"], r64["photons"])
    refs = []
    for k in (1, 2):
        rr = run_window(dict(w64, seed=int(w64["seed"]) + k), tables, 0, total, torch,
                        photons=True, events=False)
        refs.append(precision_check(rr["stats"], r64["stats"], rr["photons"], r64["photons"]))
    pc["reference_fp64_other_seeds"] = refs
    pc["within_seed_spread"] = seed_spread(pc, refs)
    st = r32["stats"]
    out = {"steps": total, "fp32": {"value": v32, "ms_per_step": r32["wall_s"] * 1e3 / total,
                                    "events": st["events"], "kept": st["kept"],
                                    "overflow": st["overflow"]},
           "fp64": {"value": v64, "ms_per_step": r64["wall_s"] * 1e3 / total,
                    "events": r64["stats"]["events"], "kept": r64["stats"]["kept"]},
           "fp32_over_fp64": v32 / v64, "fp32_vs_fp64": pc}
    log(f"full run {total} steps: fp32 {v32:.3e}, fp64 {v64:.3e} e-steps/s; count z "
        f"{pc['photon_count']['z']:+.2f}, energy rel {pc['radiated_energy']['rel']}, "
        f"KS p {pc['spectrum_ks']['p']}")
    return out


def roofline_leg(name, k, tables, torch, with_fp64=True):
    """HBM roofline of the electron-step kernel on the 3D gold slab: the
    window of k steps centred on the interaction, HIP events around every
    launch from step 0 (so that the average covers the same launches as a
    kernel trace of this process)."""
    from paper_1612_07592_amd import binding
    w = _workload(name, "fp32")
    lead, k = window(w, k)
    s = binding.Sim(w, tables)
    s.synchronize()
    s.profile(True)
    if lead:
        s.pic_step(lead)
    ms_a, n_a = s.profile_read()
    e_a = _esteps(s)
    s.profile(True)
    s.pic_step(k)
    ms_b, n_b = s.profile_read()
    st = s.pic_emission_stats()
    s.pic_destroy()
    e_b = int(st["electron_steps"]) - e_a
    dims = int(w["dims"])
    bpe = STATE_BYTES[("fp32", dims)]
    launches = int(n_a[0] + n_b[0])
    kern_ms = float(ms_a[0] + ms_b[0])
    esteps = e_a + e_b
    avg_us = kern_ms * 1e3 / max(1, launches)
    achieved = bpe * esteps / (kern_ms * 1e-3) / 1e9
    lane_ops = ALU_OPS[dims] * esteps / (kern_ms * 1e-3)
    tr = _measured_traffic(w["name"], "fp32")
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (tr["bytes_per_launch"] / 1e9 * launches / (kern_ms * 1e-3)) if tr else None,
            "traffic_bytes_per_launch": tr["bytes_per_launch"] if tr else None,
            "traffic_over_algorithmic": (tr["bytes_per_launch"] / (bpe * esteps / launches)) if tr else None,
            "kernel": f"k_electron_step<float, {dims}>", "workload": w["name"],
            "electrons": _num_electrons(w), "bytes_per_electron_step": bpe,
            "electron_steps_per_launch": esteps / max(1, launches),
            "launches": launches, "kernel_avg_us": avg_us,
            "steps": f"0..{lead + k} (lead-in {lead} + window {k}, all launches of the context)",
            "window_kernel_avg_us": float(ms_b[0]) * 1e3 / max(1, int(n_b[0])),
            "window_frac": bpe * e_b / (float(ms_b[0]) * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "window_electron_steps_per_s": e_b / (float(ms_b.sum()) * 1e-3),
            "untiled_fraction": st["untiled_steps"] / max(1, int(st["electron_steps"])),
            "alu_lane_ops": {"estimate_per_electron_step": ALU_OPS[dims],
                             "achieved_per_s": lane_ops, "peak_per_s": ALU_PEAK_LANE_OPS,
                             "frac": lane_ops / ALU_PEAK_LANE_OPS,
                             "note": "lane operations counted from the method with the general "
                                     "(cell-crossing) deposit for every electron-step: an upper "
                                     "bound; valu_issue holds the counter figure"},
            "valu_issue": ({"valu_instructions_per_launch": tr["valu_instructions_per_launch"],
                            "achieved_per_s": tr["valu_instructions_per_launch"] / (avg_us * 1e-6),
                            "peak_per_s": VALU_PEAK_WAVE_INSTS,
                            "frac": tr["valu_instructions_per_launch"] / (avg_us * 1e-6) / VALU_PEAK_WAVE_INSTS,
                            "source": "SQ_INSTS_VALU averaged over the launches, profiles/traffic.json"}
                           if tr and tr.get("valu_instructions_per_launch") else None)}
    log(f"roofline {w['name']}: {avg_us:.1f} us per launch, {achieved:.0f} GB/s "
        f"(frac {roof['frac']:.3f}); window {roof['window_kernel_avg_us']:.1f} us")
    out = {"roofline": roof}
    if with_fp64:
        w64 = dict(w, precision="fp64")
        r64 = run_window(w64, tables, lead, k, torch, events=False)
        r32 = run_window(w, tables, lead, k, torch, events=False)
        v64 = r64["window_esteps"] / r64["wall_s"]
        v32 = r32["window_esteps"] / r32["wall_s"]
        out["fp32_vs_fp64_3d"] = {"workload": w["name"], "lead_in_steps": lead, "steps": k,
                                  "fp32": v32, "fp64": v64, "fp32_over_fp64": v32 / v64,
                                  "precision": precision_check(r32["stats"], r64["stats"])}
        log(f"3D window: fp32 {v32:.3e}, fp64 {v64:.3e} e-steps/s")
    return out


def thick_target_line(tables, torch):
    """Bremsstrahlung-dominated workload: 100 MeV pencil beam of 2.1M
    electrons into 5 mm of solid gold, particle-only, FP32, 2000 steps; the
    per-step Eq. (4) trial against the free-path form."""
    from paper_1612_07592_amd import workloads as W
    res = {"workload": "thick-au-5mm", "electrons": None, "steps": 2000}
    for form, fp in (("per_step_trial", False), ("free_path", True)):
        w = W.thick_target(2000, "fp32")
        w["brem_freepath"] = fp
        r = run_window(w, tables, 0, 2000, torch)
        st = r["stats"]
        res["electrons"] = _num_electrons(w)
        res[form] = {"value": r["window_esteps"] / r["wall_s"],
                     "kernel_avg_us": r["step_kernel_ms"] * 1e3 / max(1, r["step_launches"]),
                     "brem_events": st["events"][1], "e_rad_brem": st["e_rad_kept"][1]}
    res["free_path_speedup"] = res["free_path"]["value"] / res["per_step_trial"]["value"]
    log(f"thick target: per-step {res['per_step_trial']['value']:.3e}, free path "
        f"{res['free_path']['value']:.3e} e-steps/s ({res['free_path_speedup']:.2f}x)")
    return res


def laser_energy(w):
    """Energy the laser source injects over the pulse, in the statistics'
    units (n_c m c^2 (c/omega0)^dims): a flat envelope of length T carries a
    time-averaged flux a0^2 / 2 through a 2D Gaussian profile of integral
    w0 sqrt(pi / 2) over y (per unit length in z)."""
    T = w["duration_cycles"] * 2.0 * math.pi
    w0 = w["w0_lambda"] * 2.0 * math.pi
    assert w["dims"] == 2 and w.get("envelope") == "flat" and w0 > 0
    return 0.5 * w["a0"] ** 2 * w0 * math.sqrt(math.pi / 2.0) * T


def solid_leg(torch, targets=("al", "au"), intensities=None, processes=("ncs", "brem"),
              precision="fp32"):
    """The laser-solid study of Sec. III at its own size: Al (1000^2 cells,
    13.4M electrons, 3.3M mobile ions) and Au (2000^2 cells, 53.3M electrons,
    13.3M ions), 80 electrons and 20 ions per cell, flat 30 fs pulse, one
    NCS-only and one brem-only run per intensity, each run to its end.  Per
    run: throughput, kernel time shares, and the energy partition as fractions
    of the injected laser energy (radiated by the run's process, electrons,
    ions, field left in the box)."""
    from paper_1612_07592_amd import binding
    from paper_1612_07592_amd import workloads as W
    intensities = intensities or W.SOLID_INTENSITIES
    tb = {}
    runs = []
    for tgt in targets:
        for I in intensities:
            for proc in processes:
                w = W.solid(tgt, I, proc, precision=precision)
                Z = int(w["Z"])
                if Z not in tb:
                    tb[Z] = binding.pic_build_tables(Z, 1.0, 16)
                r = run_window(w, tb[Z], 0, int(w["steps"]), torch, events=True, wall=True)
                st = r["stats"]
                EL = laser_energy(w)
                pr = 0 if proc == "ncs" else 1
                rec = {"run": w["name"], "steps": int(w["steps"]), "electrons": _num_electrons(w),
                       "ions": _num_electrons(w) // w["ppc"] * w["ion_ppc"],
                       "value": r["window_esteps"] / r["wall_s"], "wall_s": r["wall_s"],
                       "kernel_ms": {"electron_step": r["step_kernel_ms"], "field_solve": r["field_ms"],
                                     "sort": r["sort_ms"], "ions": r["ion_ms"]},
                       "events": st["events"][pr], "photons_kept": st["kept"][pr],
                       "overflow": st["overflow"],
                       "fraction_of_laser_energy": {
                           "photons": (st["e_rad_kept"][pr] + (st["e_rad_dropped"] if pr == 0 else 0.0)) / EL,
                           "photons_kept": st["e_rad_kept"][pr] / EL,
                           "electrons": st["e_kin_e"] / EL, "ions": st["e_kin_i"] / EL,
                           "field_in_box": st["e_field"] / EL},
                       "ions_live": st["ions_live"], "electrons_live": st["live"]}
                f = rec["fraction_of_laser_energy"]
                log(f"solid {w['name']}: {rec['value']:.3e} e-steps/s over {w['steps']} steps "
                    f"({r['wall_s']:.1f} s); photons {f['photons']:.2e}, e {f['electrons']:.3f}, "
                    f"i {f['ions']:.3f} of the laser energy")
                runs.append(rec)
    return {"runs": runs, "laser_energy_note": "a0^2/2 * w0 sqrt(pi/2) * T (flat pulse, 2D)",
            "precision": precision}


def pairs_leg(torch, precision="fp32"):
    """Pair production on the Sec. III gold run at 10^24 W/cm^2 (NCS and
    bremsstrahlung on, photons from 1 mc^2 kept and followed, Breit-Wheeler
    and Bethe-Heitler on): the cost of photons in flight beside the rest of
    the step, the pairs made, and the same run without them."""
    from paper_1612_07592_amd import binding
    from paper_1612_07592_amd import workloads as W
    w = W.solid("au", 1e24, "both", precision=precision)
    w.update(bw=True, bh=True, pair_capacity=50_000_000)
    Z = int(w["Z"])
    tb = dict(binding.pic_build_tables(Z, 1.0, 16))
    tb.update(binding.pic_build_pair_tables(Z, 16))
    out = {"run": w["name"] + "-pairs", "steps": int(w["steps"]), "electrons": _num_electrons(w)}
    r = run_window(w, tb, 0, int(w["steps"]), torch, events=True, wall=True)
    st = r["stats"]
    EL = laser_energy(w)
    out.update(value=r["window_esteps"] / r["wall_s"], wall_s=r["wall_s"],
               kernel_ms={"electron_step": r["step_kernel_ms"], "field_solve": r["field_ms"],
                          "sort": r["sort_ms"], "ions": r["ion_ms"], "photons": r["photon_ms"]},
               photons_stored=st["photons_stored"], overflow=st["overflow"],
               pairs=st["pairs"], pairs_stored=st["pairs_stored"],
               fraction_of_laser_energy={"into_pairs_bw": st["e_pair"][0] / EL,
                                         "into_pairs_bh": st["e_pair"][1] / EL,
                                         "photons_kept": [v / EL for v in st["e_rad_kept"]]})
    w0 = dict(w, bw=False, bh=False)
    r0 = run_window(w0, tb, 0, int(w["steps"]), torch, events=False, wall=True)
    out["without_pairs"] = {"value": r0["window_esteps"] / r0["wall_s"], "wall_s": r0["wall_s"]}
    log(f"pairs {out['run']}: {out['value']:.3e} e-steps/s ({r['wall_s']:.1f} s; without pair "
        f"production {r0['wall_s']:.1f} s); pairs BW {st['pairs'][0]}, BH {st['pairs'][1]}; photons "
        f"in flight {r['photon_ms'] / int(w['steps']) * 1e3:.0f} us per step")
    return out


def serving(args):
    """Scan jobs through the continuous-batching server: the 8-job
    intensity x target batch (FP32, FP64, and FP32 one job after another),
    then the first --c4-jobs jobs of the Poisson stream."""
    from paper_1612_07592_amd import binding, serving as SV
    from paper_1612_07592_amd import workloads as W
    tb = {13: binding.pic_build_tables(13, 1.0, 16), 79: binding.pic_build_tables(79, 1.0, 16)}
    slog = lambda m: print(f"[serve] {m}", file=sys.stderr, flush=True)
    out = {}
    jobs = W.c3_jobs(args.c3_steps)
    _, out["c3_fp32"] = SV.run_batch(jobs, tb)
    slog(f"c3 fp32 {out['c3_fp32']['electron_steps_per_s']:.3e} e-steps/s")
    _, out["c3_fp64"] = SV.run_batch([dict(w, precision="fp64") for w in jobs], tb)
    slog(f"c3 fp64 {out['c3_fp64']['electron_steps_per_s']:.3e} e-steps/s")
    out["c3_fp32_sequential"] = SV.run_sequential(jobs, tb)
    slog(f"c3 fp32 one at a time {out['c3_fp32_sequential']['electron_steps_per_s']:.3e} e-steps/s")
    out["scan_fp32_over_fp64"] = (out["c3_fp32"]["electron_steps_per_s"]
                                  / out["c3_fp64"]["electron_steps_per_s"])
    out["batched_over_sequential"] = (out["c3_fp32"]["electron_steps_per_s"]
                                      / out["c3_fp32_sequential"]["electron_steps_per_s"])
    if args.c4_jobs > 0:
        arr = W.c4_stream()[:args.c4_jobs]
        _, c4 = SV.run_stream(arr, tb, log=slog)
        offered = sum(W.num_electrons(w) * w["steps"] for _, w in arr) / max(arr[-1][0], 1e-9)
        c4["offered_electron_steps_per_s"] = offered
        c4["arrival_rate_per_s"] = 4.0
        c4["jobs_of_stream"] = f"first {len(arr)} of 500"
        out["c4_stream"] = c4
        slog(f"c4 {c4['jobs']} jobs: p50 {c4['latency_p50_s']:.2f} s p99 "
             f"{c4['latency_p99_s']:.2f} s {c4['electron_steps_per_s']:.3e} e-steps/s")
    return out


def host_cpu():
    """Host processor of the machine the benchmark runs on, as the OS reports it."""
    info = {"nproc": None, "affinity": None, "model": None, "lscpu_cpus": None}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except Exception:
        pass
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() == "Model name":
                info["model"] = v.strip()
            elif k.strip() == "CPU(s)":
                info["lscpu_cpus"] = v.strip()
    except Exception:
        pass
    return info


def cpu_baseline(w_full, lead, k, ny=64, budget_s=12.0):
    """The FP64 oracle, as it stands, on the host cores, over the same window
    of a transverse slice of the workload (all of its x extent, ny of its
    cells across the laser axis, so the slice holds the most intense part of
    the interaction).  The lead-in is untimed; the window is extended past k
    steps, if needed, to about budget_s seconds of CPU work."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import conftest
    import oracle
    oracle.build(force=False)
    tables = conftest.oracle_tables(int(w_full["Z"]))
    w = dict(w_full, precision="fp64", photon_capacity=1 << 22)
    if w["dims"] >= 2:
        w["n"] = [w["n"][0], min(ny, w["n"][1])] + list(w["n"][2:])
    cpu = host_cpu()
    nt = max(1, min(16, cpu["affinity"] or os.cpu_count() or 1))
    o = oracle.OracleSim(w, tables, nthreads=nt)
    t0 = time.perf_counter()
    if lead:
        o.step(lead)
    t_lead = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    kk = max(k - 1, int(budget_s / max(one, 1e-6)))
    kk = min(kk, max(1, int(w_full["steps"]) - lead - 1))
    t0 = time.perf_counter()
    o.step(kk)
    dt = time.perf_counter() - t0
    live = o.stats()["live"]
    o.close()
    return dict(value=live * kk / dt, unit="electron-steps/s", cores=nt, kind="oracle",
                sample=f"FP64 oracle on {nt} threads, {w['name']} sliced to {w['n'][:w['dims']]} "
                       f"cells ({o.N} electrons), steps {lead + 1}..{lead + 1 + kk} after an "
                       f"untimed lead-in of {lead + 1} steps ({t_lead:.1f} s); {live} live, "
                       f"{dt:.1f} s timed",
                host=cpu)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed steps: a window of the workload's run centred on the interaction")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--roofline-workload", default="c5")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison runs")
    ap.add_argument("--no-full-run", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the scan-job server runs")
    ap.add_argument("--no-thick", action="store_true", help="skip the thick-target runs")
    ap.add_argument("--only", default=None,
                    help="run only the headline and this leg (roofline, full, cpu, serving, thick, "
                         "solid, pairs)")
    ap.add_argument("--solid-targets", default="al,au")
    ap.add_argument("--solid-intensities", default="1e21,1e22,1e23,1e24")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--c3-steps", type=int, default=1000)
    ap.add_argument("--brem-freepath", action="store_true",
                    help="time the free-path form of the bremsstrahlung test instead of the per-step trial")
    ap.add_argument("--c4-jobs", type=int, default=24,
                    help="jobs of the Poisson stream served (0 = none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; splitting the run over "
                                   "several GPUs is described, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    legs = {"roofline": not args.no_roofline, "full": not args.no_full_run and not args.no_fp64,
            "cpu": not args.no_cpu_baseline, "serving": not args.no_serving,
            "thick": not args.no_thick, "fp64": not args.no_fp64, "solid": False, "pairs": False}
    if args.only:
        legs = {k: (k == args.only) for k in legs}
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
        log(f"copy calibration: {n * 4} bytes read, {n * 4} written")
        del a, b
    w = _workload(args.workload, args.precision)
    w["brem_freepath"] = args.brem_freepath
    lead, k = window(w, args.steps)
    t0 = time.perf_counter()
    tables = binding.pic_build_tables(int(w["Z"]), 1.0, 16)
    log(f"tables built in {time.perf_counter() - t0:.1f} s; {w['name']} {args.precision}: "
        f"{k} timed steps after a lead-in of {lead} (run of {w['steps']}, envelope peak at the "
        f"slab front at step {peak_step(w)})")
    dims = int(w["dims"])
    out = {
        "metric": "electron-steps/s", "value": None, "unit": "electron-steps/s", "n_gpus": 1,
        "steps": k, "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": w["name"], "dims": dims, "cells": list(w["n"]),
                   "electrons": _num_electrons(w), "precision": args.precision,
                   "a0": w["a0"], "Z": w["Z"], "run_steps": int(w["steps"]),
                   "lead_in_steps": lead, "window": [lead, lead + k],
                   "brem": "free-path" if args.brem_freepath else "per-step trial"},
        "roofline": None, "cpu_baseline": None, "errors": {},
    }

    def leg(name, fn):
        try:
            return fn()
        except Exception as e:  # record the failure in the line and go on
            out["errors"][name] = f"{type(e).__name__}: {e}"
            traceback.print_exc()
            return None

    try:
        r = run_window(w, tables, lead, k, torch, warmup=args.warmup)
        st = r["stats"]
        value = r["window_esteps"] / r["wall_s"]
        out.update(value=value, ms_per_step=r["wall_s"] * 1e3 / k)
        out["kernel_ms"] = {"electron_step": r["step_kernel_ms"], "field_solve": r["field_ms"],
                            "sort": r["sort_ms"], "launches": r["step_launches"]}
        out["time_share"] = {kk: v / r["profiled_ms"] for kk, v in
                             (("electron_step", r["step_kernel_ms"]), ("field_solve", r["field_ms"]),
                              ("sort", r["sort_ms"]), ("ions", r["ion_ms"]))}
        avg = r["step_kernel_ms"] * 1e3 / max(1, r["step_launches"])
        bpe = STATE_BYTES[(args.precision, dims)]
        out["headline_kernel"] = {
            "kernel": f"k_electron_step<{'float' if args.precision == 'fp32' else 'double'}, {dims}>",
            "kernel_avg_us": avg,
            "hbm_GBs": bpe * r["window_esteps"] / (r["step_kernel_ms"] * 1e-3) / 1e9,
            "note": "this state fits the 256 MB Infinity Cache: not an HBM figure"}
        out["emission"] = {"events": st["events"], "kept": st["kept"],
                           "dropped_ncs": st["dropped_ncs"], "overflow": st["overflow"],
                           "e_rad_kept": st["e_rad_kept"],
                           "untiled_fraction": st["untiled_steps"] / max(1, st["electron_steps"])}
        log(f"{args.precision}: {value:.3e} e-steps/s over steps {lead}..{lead + k}, step kernel "
            f"{avg:.1f} us")
        if legs["fp64"] and args.precision == "fp32":
            def fp64_window():
                r64 = run_window(dict(w, precision="fp64"), tables, lead, k, torch)
                v64 = r64["window_esteps"] / r64["wall_s"]
                out["fp64"] = {"value": v64, "ms_per_step": r64["wall_s"] * 1e3 / k,
                               "kernel_avg_us": r64["step_kernel_ms"] * 1e3 / max(1, r64["step_launches"])}
                out["fp32_over_fp64"] = value / v64
                out["fp32_vs_fp64_window"] = precision_check(r["stats"], r64["stats"])
                log(f"fp64 window: {v64:.3e} e-steps/s (fp32 {value / v64:.2f}x)")
            leg("fp64", fp64_window)
        if legs["full"] and args.precision == "fp32":
            out["full_run"] = leg("full_run", lambda: full_run_leg(w, tables, torch))
        if legs["roofline"]:
            def roof():
                tb = tables if args.roofline_workload in ("c2", "c5") else \
                    binding.pic_build_tables(int(_workload(args.roofline_workload, "fp32")["Z"]), 1.0, 16)
                res = roofline_leg(args.roofline_workload, k, tb, torch, with_fp64=legs["fp64"])
                out["roofline"] = res["roofline"]
                if "fp32_vs_fp64_3d" in res:
                    out["fp32_vs_fp64_3d"] = res["fp32_vs_fp64_3d"]
            leg("roofline", roof)
        if legs["thick"] and args.workload == "c2":
            out["thick_target"] = leg("thick_target", lambda: thick_target_line(tables, torch))
        if legs["serving"] and args.workload == "c2":
            out["serving"] = leg("serving", lambda: serving(args))
        if legs["solid"]:
            out["solid"] = leg("solid", lambda: solid_leg(
                torch, tuple(args.solid_targets.split(",")),
                tuple(float(v) for v in args.solid_intensities.split(","))))
        if legs["pairs"]:
            out["pairs"] = leg("pairs", lambda: pairs_leg(torch))
        if legs["cpu"]:
            out["cpu_baseline"] = leg("cpu_baseline", lambda: cpu_baseline(
                _workload(args.workload, "fp64"), lead, k))
    except Exception as e:
        out["errors"]["headline"] = f"{type(e).__name__}: {e}"
        traceback.print_exc()
    finally:
        print(json.dumps(out), flush=True)
    if "headline" in out["errors"]:
        sys.exit(1)


if __name__ == "__main__":
    main()
