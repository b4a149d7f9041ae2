"""GPU parity of photons in flight and pair production (Breit-Wheeler,
Bethe-Heitler) against the FP64 oracle, through the C-ABI.

FP64 bar: the same photons convert, by the same process, at the same step,
into pairs of identical energies at identical positions (records compared
as sets keyed by the photon's parent, emission step and process, since the
device's append order is not deterministic); the state in flight of every
photon (position, pair optical depth, state) identical; pair counts exact,
radiated-into-pairs energy within 1e-11 relative."""
from __future__ import annotations

import math

import numpy as np
import pytest

import scenarios as S
import test_oracle_pins_pairs as PP
from parity import SUM_TOL, compare

pytestmark = pytest.mark.gpu


def _announce(name):
    print(f"\n[gpu-case] {name}", flush=True)


def _key(d):
    return np.lexsort((d["proc"], d["pstep"], d["parent"]))


def compare_pairs(o, g, label=""):
    po, pg = o.pairs(), g.pairs()
    assert len(po["e_minus"]) == len(pg["e_minus"]), (label, len(po["e_minus"]), len(pg["e_minus"]))
    io, ig = _key(po), _key(pg)
    for k in ("parent", "pstep", "proc", "step"):
        assert np.array_equal(po[k][io], pg[k][ig]), (label, k)
    for k in ("e_minus", "e_plus", "w"):
        assert np.array_equal(po[k][io], pg[k][ig]), (label, k)
    assert np.array_equal(po["x"][io], pg["x"][ig]), label
    assert np.array_equal(po["k"][io], pg["k"][ig]), label
    so, sg = o.stats(), g.stats()
    assert list(so["pairs"]) == list(sg["pairs"]), (label, so["pairs"], sg["pairs"])
    assert so["pairs_overflow"] == sg["pairs_overflow"], label
    for i in range(2):
        assert abs(sg["e_pair"][i] - so["e_pair"][i]) <= SUM_TOL * max(abs(so["e_pair"][i]), 1e-300), label
    return dict(pairs=list(sg["pairs"]))


def compare_flight(o, g, label=""):
    """In-flight state of every stored photon, joined on (parent, step, proc)."""
    fo, fg = o.flight(), g.flight()
    ph_o, ph_g = o.photons(), g.photons()
    ko = np.lexsort((ph_o["proc"], ph_o["step"], ph_o["parent"]))
    kg = np.lexsort((ph_g["proc"], ph_g["step"], ph_g["parent"]))
    for k in ("parent", "step", "proc"):
        assert np.array_equal(ph_o[k][ko], ph_g[k][kg]), (label, k)
    assert np.array_equal(fo["state"][ko], fg["state"][kg]), label
    assert np.array_equal(fo["x"][ko], fg["x"][kg]), label
    assert np.array_equal(fo["tau"][ko], fg["tau"][kg]), label
    return dict(travelling=int((fg["state"] == 1).sum()), converted=int((fg["state"] == 2).sum()),
                absorbed=int((fg["state"] == 3).sum()))


def _pair(oracle_lib, gpu_lib, w, tables):
    o = oracle_lib.OracleSim(w, tables)
    g = gpu_lib.Sim(w, tables)
    assert g.N == o.N
    return o, g


def test_breit_wheeler_in_prescribed_fields(oracle_lib, gpu_lib, tables_al):
    """Photons injected along +x, -x and +z in crossed E and B (three chi,
    one of them between the others and zero along none): conversions,
    shares, positions and depths bit for bit."""
    _announce("pairs: Breit-Wheeler, injected photons")
    w = PP._bw_w()
    o, g = _pair(oracle_lib, gpu_lib, w, tables_al)
    x0 = 0.5 * 1024 * o.derived()["dx"][0]
    ph = PP._field_photons(1500, 2400.0, x0)
    o.add_photons(*ph)
    g.add_photons(*ph)
    o.step(90)
    g.step(90)
    rep = compare_pairs(o, g, "bw")
    rep.update(compare_flight(o, g, "bw"))
    print(rep, flush=True)
    assert rep["pairs"][0] > 1000
    # injected photons are stored records, not photons lost to a full buffer
    assert g.stats()["overflow"] == 0 == o.stats()["overflow"]


def test_bethe_heitler_on_a_dense_target(oracle_lib, gpu_lib, tables_au):
    _announce("pairs: Bethe-Heitler, injected photons in a dense target")
    w = S.frozen_B_beam(B=0.0, ne=4e7, Z=79, charge_state=79, ppc=1)
    w.update(ncs=False, brem=False, bw=False, bh=True, photon_capacity=1 << 16, pair_capacity=1 << 16)
    o, g = _pair(oracle_lib, gpu_lib, w, tables_au)
    dx = o.derived()["dx"][0]
    n = 6000
    rng = np.random.default_rng(3)
    k = np.zeros((n, 3))
    k[:, 0] = rng.choice([-1.0, 1.0], n)        # crossing the slab (cells 480..543) and out
    x = np.zeros((n, 3)); x[:, 0] = (rng.uniform(470, 554, n)) * dx
    x[:600, 0] = rng.uniform(2, 40, 600) * dx   # near the left wall, leaving through it
    k[:600, 0] = -1.0
    eps = np.exp(rng.uniform(math.log(3.0), math.log(5000.0), n))
    par = 0x40000000 + np.arange(n, dtype=np.uint32)
    o.add_photons(x, k, eps, np.full(n, 0.7), par)
    g.add_photons(x, k, eps, np.full(n, 0.7), par)
    o.step(120)
    g.step(120)
    rep = compare_pairs(o, g, "bh")
    rep.update(compare_flight(o, g, "bh"))
    print(rep, flush=True)
    assert rep["pairs"][1] > 500 and rep["absorbed"] > 0


def test_pairs_from_emitted_photons_full_pic(oracle_lib, gpu_lib, tables_au):
    """1D laser slab at a0 = 855: NCS photons of the interaction turn into
    Breit-Wheeler pairs in the laser field; everything bit for bit."""
    _announce("pairs: 1D full PIC at a0 = 855")
    w = S.ions_1d(steps=500)
    w.update(ion_ppc=0, a0=855.0, ne_over_nc=100.0, bw=True, bh=True, pair_capacity=1 << 18,
             photon_cut_mc2=1.0, photon_capacity=1 << 22)
    o, g = _pair(oracle_lib, gpu_lib, w, tables_au)
    o.step(500)
    g.step(500)
    rep = compare(o, g, label="pairs-1d")
    rep.update(compare_pairs(o, g, "pairs-1d"))
    rep.update(compare_flight(o, g, "pairs-1d"))
    fo, fg = o.fields(), g.fields()
    rep["max_dfield"] = float(np.abs(fo - fg).max())
    print(rep, flush=True)
    assert rep["max_dfield"] <= 1e-12 * max(1.0, np.abs(fo).max())
    assert rep["pairs"][0] > 1000


def test_pairs_fp32_against_fp64(gpu_lib, tables_al):
    """FP32 photons in flight against FP64 on the same random streams: the
    pair optical depth is FP64 in both, the rate FP32 in one, so the same
    photons convert up to the few whose depth ends within the rate's
    rounding of zero; the shares agree in distribution."""
    _announce("pairs: FP32 against FP64")
    res = []
    for prec in ("fp64", "fp32"):
        w = PP._bw_w(precision=prec)
        g = gpu_lib.Sim(w, tables_al)
        x0 = 0.5 * 1024 * g.derived()["dx"][0]
        g.add_photons(*PP._field_photons(3000, 2400.0, x0))
        g.step(90)
        res.append((g.stats(), g.pairs()))
    (s64, p64), (s32, p32) = res
    n64, n32 = s64["pairs"][0], s32["pairs"][0]
    assert abs(n32 - n64) <= max(3, 0.002 * n64), (n32, n64)
    from scipy import stats
    xi64 = p64["e_minus"] / (p64["e_minus"] + p64["e_plus"])
    xi32 = p32["e_minus"] / (p32["e_minus"] + p32["e_plus"])
    assert stats.ks_2samp(xi64, xi32).pvalue > 0.01
    assert abs(s32["e_pair"][0] / s64["e_pair"][0] - 1) < 0.01


def test_step_many_with_pairs_matches_step(gpu_lib, tables_au):
    _announce("pairs: pic_step_many vs pic_step")
    w = S.ions_1d(steps=300)
    w.update(ion_ppc=0, a0=855.0, ne_over_nc=100.0, bw=True, bh=True, pair_capacity=1 << 18,
             photon_cut_mc2=1.0, photon_capacity=1 << 22)
    ws = [w, dict(w, precision="fp32", seed=77), S.small_2d(steps=60)]
    solo = []
    for x in ws:
        s = gpu_lib.Sim(x, tables_au)
        s.step(300 if x is not ws[2] else 60)
        solo.append(s)
    batch = gpu_lib.Batch()
    many = [gpu_lib.Sim(x, tables_au) for x in ws]
    for _ in range(5):
        batch.step_many(many, [60, 60, 12])
    for a, b in zip(solo, many):
        ea, eb = a.electrons(), b.electrons()
        for k in ("x", "p", "tau", "alive"):
            assert np.array_equal(ea[k], eb[k]), k
        assert np.array_equal(a.fields(), b.fields())
        if a.workload.get("bw"):
            pa, pb = a.pairs(), b.pairs()
            ia, ib = _key(pa), _key(pb)
            for k in ("e_minus", "e_plus", "parent", "pstep", "step"):
                assert np.array_equal(pa[k][ia], pb[k][ib]), k
            assert a.stats()["pairs"] == b.stats()["pairs"]
    batch.close()


def test_pair_buffer_overflow(oracle_lib, gpu_lib, tables_al):
    """A pair buffer of 100 records: every pair is still counted (and its
    energy summed), 100 are stored, none is written beyond; the stored ones
    are pairs the oracle made (its buffer large enough for all)."""
    _announce("pairs: pair buffer overflow")
    w = PP._bw_w()
    o = oracle_lib.OracleSim(w, tables_al)
    g = gpu_lib.Sim(dict(w, pair_capacity=100), tables_al)
    x0 = 0.5 * 1024 * o.derived()["dx"][0]
    ph = PP._field_photons(1500, 2400.0, x0)
    o.add_photons(*ph)
    g.add_photons(*ph)
    o.step(60)
    g.step(60)
    so, sg = o.stats(), g.stats()
    assert sg["pairs"] == so["pairs"] and sg["pairs"][0] > 100
    assert sg["pairs_stored"] == 100 and sg["pairs_overflow"] == sg["pairs"][0] - 100
    assert abs(sg["e_pair"][0] - so["e_pair"][0]) <= SUM_TOL * so["e_pair"][0]
    po, pg = o.pairs(), g.pairs()
    assert len(pg["e_minus"]) == 100
    ko = {(int(a), int(b), int(c)): (em, ep) for a, b, c, em, ep in
          zip(po["parent"], po["pstep"], po["proc"], po["e_minus"], po["e_plus"])}
    for a, b, c, em, ep in zip(pg["parent"], pg["pstep"], pg["proc"], pg["e_minus"], pg["e_plus"]):
        assert ko[(int(a), int(b), int(c))] == (em, ep)


def test_pair_call_errors(gpu_lib, tables_au):
    _announce("pairs: call errors")
    from paper_1612_07592_amd.binding import PicError
    g = gpu_lib.Sim(S.small_2d())               # no pair production
    with pytest.raises(PicError) as e:
        g.pic_load_pair_tables(tables_au)
    assert e.value.code == 4
    w = PP._bw_w()
    g = gpu_lib.Sim(w)                          # pair tables not loaded
    with pytest.raises(PicError) as e:
        g.pic_step(1)
    assert e.value.code == 4
    bad = dict(tables_au)
    bad["bw_cdf"] = np.array(tables_au["bw_cdf"])
    bad["bw_cdf"][5, 3] = 2.0                   # not monotone
    g2 = gpu_lib.Sim(dict(w, Z=79, charge_state=79))
    with pytest.raises(PicError) as e:
        g2.pic_load_pair_tables(bad)
    assert e.value.code == 6
    g2.pic_load_pair_tables(tables_au)          # the context survives a rejection
