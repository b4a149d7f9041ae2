"""Free-path bremsstrahlung (PIC_BREM_FREEPATH) on the GPU.

FP64 parity with the oracle's free-path form: identical events, collision
optical depths within 1e-12 relative (absolute below 1), the usual state and
photon bars.  Against the per-step Eq. (4) trial the free-path form draws
different random numbers, so the two agree in distribution: event counts
within 3 sigma, photon spectra by two-sample KS (p > 0.01), radiated energy
within 3 sigma of the compound-Poisson spread.  FP32 against FP64, both
free-path: the FP32 criteria (count 3 sigma, KS p > 0.01, energy 1%)."""
from __future__ import annotations

import math

import numpy as np
import pytest
from scipy import stats as sst

import scenarios as S
from parity import compare

pytestmark = pytest.mark.gpu


def _announce(name):
    print(f"\n[gpu-case] {name}", flush=True)


def _beam(seed, pmin=5.0, pmax=2000.0):
    def f(sim):
        e = sim.electrons()
        return e["x"], S.beam_momenta(sim.N, pmin, pmax, seed), e["tau"]
    return f


def _dense(**kw):
    w = S.frozen_B_beam(B=50.0, ne=5e7, Z=79, charge_state=79, **kw)
    w["brem_freepath"] = True
    return w


def _compare_depth(o, g, label):
    to, tg = o.tau_brem(), g.brem_depth()
    d = np.abs(tg - to) / np.maximum(np.abs(to), 1.0)
    assert float(d.max()) <= 1e-12, f"{label}: collision depth mismatch {d.max():.3e}"
    return float(d.max())


def test_freepath_parity_dense_target(oracle_lib, gpu_lib, tables_au):
    """Particle-only mode, dense gold target, NCS and recoil on."""
    _announce("free-path brem, frozen uniform B, dense target")
    w = _dense()
    o = oracle_lib.OracleSim(w, tables_au)
    g = gpu_lib.Sim(w, tables_au)
    x, p, tau = _beam(22)(o)
    o.set_electrons(x, p, tau)
    g.set_electrons(x, p, tau)
    _compare_depth(o, g, "initial")
    o.step(150)
    g.step(150)
    # momenta relative to the beam's |p|: see compare()
    rep = compare(o, g, label="freepath-dense", p_scale=np.linalg.norm(p, axis=1))
    rep["max_dtaub"] = _compare_depth(o, g, "freepath-dense")
    print(rep, flush=True)
    assert rep["events"][1] > 100


def test_freepath_parity_16_electrons(oracle_lib, gpu_lib, tables_au):
    """The 16-electron free-path case the oracle is pinned on by replay."""
    _announce("free-path brem, 16 electrons at a table node")
    Tk = math.exp(tables_au["ln_T0"] + 100 * tables_au["dln_T"])
    pm = math.sqrt(Tk * (Tk + 2))
    w = S.base(name="brem-16-fp", dims=1, n=[64], dx_lambda=[1.0], ppc=1, x0_lambda=0.0,
               thickness_lambda=16.0, frozen=True, frozen_kind=0, Z=79, charge_state=79,
               ne_over_nc=1.4e5, ncs=False, brem=True, no_recoil=True, seed=13,
               brem_freepath=True)
    o = oracle_lib.OracleSim(w, tables_au)
    g = gpu_lib.Sim(w, tables_au)
    e = o.electrons()
    p = np.zeros((o.N, 3))
    p[:, 1] = pm
    o.set_electrons(e["x"], p, e["tau"])
    g.set_electrons(e["x"], p, e["tau"])
    o.step(300)
    g.step(300)
    rep = compare(o, g, label="16-freepath")
    rep["max_dtaub"] = _compare_depth(o, g, "16-freepath")
    print(rep, flush=True)
    assert rep["events"][1] > 10


def test_freepath_parity_small_2d_full_pic(oracle_lib, gpu_lib, tables_au):
    """Full 2D PIC (fields, deposit, sort) with the free-path form."""
    _announce("free-path brem, 2D small full PIC")
    w = S.small_2d()
    w.update(brem_freepath=True, ne_over_nc=400.0)
    o = oracle_lib.OracleSim(w, tables_au)
    g = gpu_lib.Sim(w, tables_au)
    o.step(w["steps"])
    g.step(w["steps"])
    rep = compare(o, g, label="2D-freepath")
    rep["max_dtaub"] = _compare_depth(o, g, "2D-freepath")
    fo, fg = o.fields(), g.fields()
    rep["max_dfield"] = float(np.abs(fo - fg).max())
    print(rep, flush=True)
    assert rep["max_dfield"] <= 1e-12 * max(1.0, np.abs(fo).max())


def _run(gpu_lib, w, tables, steps, beam):
    s = gpu_lib.Sim(w, tables)
    x, p, tau = beam(s)
    s.set_electrons(x, p, tau)
    s.pic_step(steps)
    st = s.stats()
    ph = s.photons()
    s.close()
    br = ph["proc"] == 1
    return dict(n=st["events"][1], eps=ph["energy"][br], wgt=ph["w"][br],
                erad=st["e_rad_kept"][1])


def test_freepath_same_law_as_per_step_trial(gpu_lib, tables_au):
    """Per-step Eq. (4) trial and free path on the same beam: same event law."""
    _announce("free path vs per-step trial, dense target, 400 steps")
    w = _dense()
    w["ncs"] = False
    a = _run(gpu_lib, dict(w, brem_freepath=False), tables_au, 400, _beam(31))
    b = _run(gpu_lib, w, tables_au, 400, _beam(31))
    z = (b["n"] - a["n"]) / math.sqrt(a["n"] + b["n"])
    ks = sst.ks_2samp(a["eps"], b["eps"])
    de = b["erad"] - a["erad"]
    sd = math.sqrt(float(np.sum((a["wgt"] * a["eps"]) ** 2) + np.sum((b["wgt"] * b["eps"]) ** 2)))
    print(f"[freepath-vs-trial] events {b['n']} vs {a['n']} (z = {z:+.2f}); KS p = {ks.pvalue:.3g}; "
          f"radiated energy {b['erad']:.6e} vs {a['erad']:.6e} ({de / sd:+.2f} sigma)", flush=True)
    assert a["n"] > 5000
    assert abs(z) <= 3.0
    assert ks.pvalue > 0.01
    assert abs(de) <= 3.0 * sd


def test_freepath_fp32_against_fp64(gpu_lib, tables_au):
    _announce("free path: FP32 vs FP64, dense target, 400 steps")
    w = _dense()
    r64 = _run(gpu_lib, dict(w, precision="fp64"), tables_au, 400, _beam(32))
    r32 = _run(gpu_lib, dict(w, precision="fp32"), tables_au, 400, _beam(32))
    z = (r32["n"] - r64["n"]) / math.sqrt(max(r64["n"], 1))
    rel = (r32["erad"] - r64["erad"]) / r64["erad"]
    ks = sst.ks_2samp(r32["eps"], r64["eps"])
    print(f"[fp32-vs-fp64 free path] brem events {r32['n']} vs {r64['n']} (z = {z:+.2f}); "
          f"radiated energy rel {rel:+.3e}; KS p = {ks.pvalue:.3g}", flush=True)
    assert r64["n"] > 5000
    assert abs(z) <= 3.0
    assert abs(rel) <= 0.01
    assert ks.pvalue > 0.01


def test_freepath_runs_same_alone_and_batched(gpu_lib, tables_au):
    """Free-path runs (2D full PIC, FP32 and FP64) advanced with pic_step_many
    beside a per-step-trial run end bit-identical to the same runs alone,
    collision depths included (the sort carries them in both)."""
    _announce("free path: pic_step_many against pic_step")
    from test_serving_gpu import assert_same_run
    mix = []
    for prec, n in (("fp32", 60), ("fp64", 45)):
        w = S.small_2d(precision=prec)
        w.update(brem_freepath=True, ne_over_nc=400.0, seed=41 if prec == "fp32" else 42)
        mix.append((w, n))
    mix.append((S.small_2d(precision="fp32"), 50))
    alone = []
    for w, n in mix:
        s = gpu_lib.Sim(w, tables_au)
        s.pic_step(n)
        alone.append(s)
    sims = [gpu_lib.Sim(w, tables_au) for w, _ in mix]
    b = gpu_lib.Batch()
    b.step_many(sims, [min(n, 17) for _, n in mix])
    b.step_many(sims, [n - min(n, 17) for _, n in mix])
    for (w, n), a, g in zip(mix, alone, sims):
        st = assert_same_run(a, g, f"{w['name']}/{w['precision']}/freepath={w.get('brem_freepath', False)}")
        assert st["steps"] == n
        if w.get("brem_freepath"):
            assert np.array_equal(a.brem_depth(), g.brem_depth())
    b.close()
