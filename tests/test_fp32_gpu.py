"""The FP32-mixed path against the FP64 path on the GPU, on the same workload
and the same Philox streams.  Criteria, each stated per result:
  photon count   |N32 - N64| <= 3 sqrt(N64)        (kept photons)
  spectrum       two-sample KS p > 0.01            (kept photon energies)
  radiated energy |E32 - E64| <= 1% E64            (kept + dropped, both processes)

Particle-only runs (prescribed fields) have no collective dynamics, so the
two precisions see the same fields and the criteria apply as stated.  In the
full 2D PIC run the laser-plasma interaction is chaotic: two FP64 runs that
differ only in the seed already fail the Poisson count and KS criteria, so
there the KS distance is judged against that seed-to-seed distance."""
from __future__ import annotations

import numpy as np
import pytest
from scipy import stats as sst

import scenarios as S
from paper_1612_07592_amd import workloads as W

pytestmark = pytest.mark.gpu


def _run(gpu_lib, w, tables, steps, beam=None):
    s = gpu_lib.Sim(w, tables)
    if beam is not None:
        e = s.electrons()
        s.set_electrons(e["x"], beam(s.N), e["tau"])
    s.pic_step(steps)
    st = s.stats()
    ph = s.photons()
    s.close()
    erad = st["e_rad_kept"][0] + st["e_rad_kept"][1] + st["e_rad_dropped"]
    return dict(n=sum(st["kept"]), erad=erad, eps=ph["energy"], events=st["events"])


def _criteria(r32, r64, label):
    z = (r32["n"] - r64["n"]) / max(r64["n"], 1) ** 0.5
    rel = (r32["erad"] - r64["erad"]) / r64["erad"]
    ks = sst.ks_2samp(r32["eps"], r64["eps"]) if len(r32["eps"]) and len(r64["eps"]) else None
    print(f"\n[fp32-vs-fp64] {label}: kept {r32['n']} vs {r64['n']} (z = {z:+.2f}); "
          f"radiated energy rel {rel:+.3e}; KS D = {ks.statistic if ks else float('nan'):.5f} "
          f"p = {ks.pvalue if ks else float('nan'):.3g}", flush=True)
    return z, rel, ks


def test_fp32_particle_only_uniform_B(gpu_lib, tables_al):
    w = S.frozen_B_beam(B=3000.0, seed=5)
    beam = lambda n: S.beam_momenta(n, 50.0, 3000.0, 9)
    r64 = _run(gpu_lib, dict(w, precision="fp64"), tables_al, 200, beam)
    r32 = _run(gpu_lib, dict(w, precision="fp32"), tables_al, 200, beam)
    z, rel, ks = _criteria(r32, r64, "uniform B = 3000, beam 50..3000 mc, 200 steps")
    assert r64["n"] > 10000
    assert abs(z) <= 3.0
    assert abs(rel) <= 0.01
    assert ks.pvalue > 0.01


def test_fp32_particle_only_plane_wave(gpu_lib, tables_al):
    w = S.frozen_plane_wave(a=270.0, seed=6)
    r64 = _run(gpu_lib, dict(w, precision="fp64"), tables_al, 600)
    r32 = _run(gpu_lib, dict(w, precision="fp32"), tables_al, 600)
    z, rel, ks = _criteria(r32, r64, "plane wave a = 270, cold slab, 600 steps")
    assert r64["n"] > 100
    assert abs(z) <= 3.0
    assert abs(rel) <= 0.01
    assert ks.pvalue > 0.01


def test_fp32_full_pic_2d_gold_a270(gpu_lib, tables_au):
    """2048x1024 cells, Au q = 69 slab at 200 n_c, a0 = 270, 2000 steps.

    The strict criteria are printed per result; the assertions hold each
    FP32 difference to twice the largest difference between the FP64 run and
    FP64 runs with the next two seeds (floored at the strict bounds)."""
    w = W.c2(steps=2000)
    r64 = _run(gpu_lib, dict(w, precision="fp64"), tables_au, 2000)
    r32 = _run(gpu_lib, dict(w, precision="fp32"), tables_au, 2000)
    z, rel, ks = _criteria(r32, r64, "2D Au a0=270 full PIC")
    print(f"[fp32-vs-fp64] strict: count {'pass' if abs(z) <= 3 else 'FAIL'}, energy "
          f"{'pass' if abs(rel) <= 0.01 else 'FAIL'}, KS {'pass' if ks.pvalue > 0.01 else 'FAIL'}")
    dn, de, dk = [], [], []
    for k in (1, 2):
        ref = _run(gpu_lib, dict(w, precision="fp64", seed=w["seed"] + k), tables_au, 2000)
        zr, relr, ksr = _criteria(ref, r64, f"2D Au a0=270 full PIC, FP64 seed +{k} (reference)")
        dn.append(abs(ref["n"] - r64["n"]))
        de.append(abs(relr))
        dk.append(ksr.statistic)
    assert r64["n"] > 100000
    assert abs(r32["n"] - r64["n"]) <= 2.0 * max(max(dn), 3.0 * r64["n"] ** 0.5)
    assert abs(rel) <= max(0.01, 2.0 * max(de))
    assert ks.statistic <= 2.0 * max(dk)
