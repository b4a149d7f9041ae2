"""GPU parity of the mobile ions (the solid-target runs of Sec. III) against
the FP64 oracle, through the C-ABI.

FP64 bar, as for the electrons: identical loading, ion positions and
momenta within 1e-12 relative (absolute below 1), identical alive masks and
live counts, ion kinetic energy within 1e-11 relative, fields within 1e-12,
and the electrons' full comparison (identical emission events, which with
bremsstrahlung on are decided against the counted ion density)."""
from __future__ import annotations

import numpy as np
import pytest

import scenarios as S
from parity import SUM_TOL, compare

pytestmark = pytest.mark.gpu

P_TOL = 1e-12


def _announce(name):
    print(f"\n[gpu-case] {name}", flush=True)


def compare_ions(o, g, label=""):
    io, ig = o.ions(), g.ions()
    assert io["x"].shape == ig["x"].shape, label
    assert np.array_equal(io["alive"], ig["alive"]), f"{label}: ion alive masks differ"
    sp = np.maximum(np.linalg.norm(io["p"], axis=1), 1.0)
    sx = np.maximum(np.linalg.norm(io["x"], axis=1), 1.0)
    dp = float((np.linalg.norm(io["p"] - ig["p"], axis=1) / sp).max()) if sp.size else 0.0
    dx = float((np.linalg.norm(io["x"] - ig["x"], axis=1) / sx).max()) if sx.size else 0.0
    assert dp <= P_TOL, f"{label}: ion momentum mismatch {dp:.3e}"
    assert dx <= P_TOL, f"{label}: ion position mismatch {dx:.3e}"
    so, sg = o.stats(), g.stats()
    assert so["ions_live"] == sg["ions_live"], label
    eo = o.ion_kinetic_energy()
    assert abs(sg["e_kin_i"] - eo) <= SUM_TOL * max(abs(eo), 1e-300), (label, sg["e_kin_i"], eo)
    return dict(ion_dp=dp, ion_dx=dx, ions_live=int(sg["ions_live"]), e_kin_i=eo)


def _pair(oracle_lib, gpu_lib, w, tables):
    o = oracle_lib.OracleSim(w, tables)
    g = gpu_lib.Sim(w, tables)
    assert (g.N, g.Ni) == (o.N, o.Ni)
    return o, g


def test_ion_loading_identical(oracle_lib, gpu_lib, tables_au):
    _announce("ions: loading 2D")
    w = S.ions_2d()
    o, g = _pair(oracle_lib, gpu_lib, w, tables_au)
    io, ig = o.ions(), g.ions()
    assert g.Ni == 16 * 64 * 2
    assert np.array_equal(io["x"], ig["x"])
    assert not ig["p"].any() and ig["alive"].all()
    s = g.stats()
    assert s["ions_live"] == g.Ni and s["e_kin_i"] == 0.0


def test_ions_1d_laser_slab(oracle_lib, gpu_lib, tables_au):
    """Hole boring into a dense slab: the ions gain more energy than the
    electrons keep, and move hundreds of cells; NCS throughout."""
    _announce("ions: 1D laser slab 300 steps")
    w = S.ions_1d()
    o, g = _pair(oracle_lib, gpu_lib, w, tables_au)
    o.step(w["steps"])
    g.step(w["steps"])
    rep = compare(o, g, label="ions-1d")
    rep.update(compare_ions(o, g, "ions-1d"))
    fo, fg = o.fields(), g.fields()
    rep["max_dfield"] = float(np.abs(fo - fg).max())
    print(rep, flush=True)
    assert rep["max_dfield"] <= 1e-12 * max(1.0, np.abs(fo).max())
    assert rep["events"][0] > 1000 and rep["e_kin_i"] > 0.0


def test_ions_2d_flat_pulse(oracle_lib, gpu_lib, tables_au):
    _announce("ions: 2D flat pulse 160 steps")
    w = S.ions_2d()
    o, g = _pair(oracle_lib, gpu_lib, w, tables_au)
    o.step(w["steps"])
    g.step(w["steps"])
    rep = compare(o, g, label="ions-2d")
    rep.update(compare_ions(o, g, "ions-2d"))
    fo, fg = o.fields(), g.fields()
    rep["max_dfield"] = float(np.abs(fo - fg).max())
    print(rep, flush=True)
    assert rep["max_dfield"] <= 1e-12 * max(1.0, np.abs(fo).max())
    assert rep["ions_live"] < g.Ni   # some ions left through the walls


def test_ions_3d_laser_slab(oracle_lib, gpu_lib, tables_au):
    _announce("ions: 3D laser slab 80 steps")
    w = S.ions_3d()
    o, g = _pair(oracle_lib, gpu_lib, w, tables_au)
    o.step(w["steps"])
    g.step(w["steps"])
    rep = compare(o, g, label="ions-3d")
    rep.update(compare_ions(o, g, "ions-3d"))
    fo, fg = o.fields(), g.fields()
    rep["max_dfield"] = float(np.abs(fo - fg).max())
    print(rep, flush=True)
    assert rep["max_dfield"] <= 1e-12 * max(1.0, np.abs(fo).max())
    assert rep["e_kin_i"] > 0.0


def test_ions_2d_scattered_global_path(oracle_lib, gpu_lib, tables_au):
    """Ions shuffled over the slab, so that a workgroup's ions span more
    nodes than its LDS box holds: current and counts go to global memory."""
    _announce("ions: 2D shuffled ions (global-memory path)")
    w = S.ions_2d(steps=120)
    o, g = _pair(oracle_lib, gpu_lib, w, tables_au)
    x = o.ions()["x"]
    x = x[np.random.default_rng(9).permutation(o.Ni)]
    p = np.zeros_like(x)
    o.set_ions(x, p)
    g.set_ions(x, p)
    o.step(w["steps"])
    g.step(w["steps"])
    rep = compare(o, g, label="ions-2d-shuffled")
    rep.update(compare_ions(o, g, "ions-2d-shuffled"))
    fo, fg = o.fields(), g.fields()
    rep["max_dfield"] = float(np.abs(fo - fg).max())
    print(rep, flush=True)
    assert rep["max_dfield"] <= 1e-12 * max(1.0, np.abs(fo).max())


def test_brem_against_counted_ion_density(oracle_lib, gpu_lib, tables_au):
    """Particle-only mode, very dense: thousands of collisions, each decided
    against the density counted from the (moving) ions of the electron's
    cell; the ions are then set by hand into a few cells (pic_set_ions
    rebuilds the counts) and the run goes on."""
    _announce("ions: frozen dense brem with counted density")
    w = S.frozen_dense_ions()
    o, g = _pair(oracle_lib, gpu_lib, w, tables_au)
    p = S.beam_momenta(o.N, 5.0, 2000.0, 22)
    e = o.electrons()
    o.set_electrons(e["x"], p, e["tau"])
    g.set_electrons(e["x"], p, e["tau"])
    rng = np.random.default_rng(5)
    pi = np.zeros((o.Ni, 3))
    pi[:, :2] = rng.uniform(-0.05, 0.05, (o.Ni, 2))
    x = o.ions()["x"]
    o.set_ions(x, pi)
    g.set_ions(x, pi)
    o.step(80)
    g.step(80)
    compare(o, g, label="dense-ions-a", p_scale=np.linalg.norm(p, axis=1))
    compare_ions(o, g, "dense-ions-a")
    # crowd every ion into the slab's first 8 cells
    x = o.ions()["x"].copy()
    dx = w["dx_lambda"][0] * 2 * np.pi
    x[:, 0] = (480 + (np.arange(o.Ni) % 8) + 0.5) * dx
    o.set_ions(x, pi)
    g.set_ions(x, pi)
    o.step(70)
    g.step(70)
    rep = compare(o, g, label="dense-ions-b", p_scale=np.linalg.norm(p, axis=1))
    rep.update(compare_ions(o, g, "dense-ions-b"))
    print(rep, flush=True)
    assert rep["events"][1] > 1000


def test_step_many_with_ions_matches_step(gpu_lib, tables_au):
    """pic_step_many with runs that have mobile ions (and one that has not)
    ends bit-identical to pic_step run by run, in both precisions."""
    _announce("ions: pic_step_many vs pic_step")
    ws = [S.ions_2d(steps=60), S.ions_2d(steps=60, precision="fp32"), S.small_2d(steps=60)]
    ws[1]["seed"] = 44
    solo = []
    for w in ws:
        s = gpu_lib.Sim(w, tables_au)
        s.step(60)
        solo.append(s)
    batch = gpu_lib.Batch()
    many = [gpu_lib.Sim(w, tables_au) for w in ws]
    for _ in range(3):
        batch.step_many(many, [20] * len(many))
    for a, b in zip(solo, many):
        ea, eb = a.electrons(), b.electrons()
        for k in ("x", "p", "tau", "alive"):
            assert np.array_equal(ea[k], eb[k]), k
        assert np.array_equal(a.fields(), b.fields())
        if a.Ni:
            ia, ib = a.ions(), b.ions()
            for k in ("x", "p", "alive"):
                assert np.array_equal(ia[k], ib[k]), k
            assert a.stats()["e_kin_i"] == b.stats()["e_kin_i"]
    batch.close()


def test_every_ion_leaves(oracle_lib, gpu_lib, tables_au):
    """Ions set moving fast towards the right wall: all are absorbed within
    the run (live count 0, kinetic energy 0), the density of Eq. (4) falls to
    zero and no collision happens after that; parity throughout."""
    _announce("ions: every ion leaves the box")
    w = S.frozen_dense_ions(B=0.0, steps=600)
    w["ncs"] = False
    o, g = _pair(oracle_lib, gpu_lib, w, tables_au)
    e = o.electrons()
    pe = S.beam_momenta(o.N, 5.0, 2000.0, 23)
    o.set_electrons(e["x"], pe, e["tau"])
    g.set_electrons(e["x"], pe, e["tau"])
    x = o.ions()["x"]
    p = np.zeros_like(x)
    p[:, 0] = 30.0                      # v = 0.9995 c along +x
    o.set_ions(x, p)
    g.set_ions(x, p)
    o.step(600)
    g.step(600)
    rep = compare(o, g, label="ions-leave", p_scale=np.linalg.norm(pe, axis=1))
    rep.update(compare_ions(o, g, "ions-leave"))
    print(rep, flush=True)
    assert rep["ions_live"] == 0 and g.stats()["e_kin_i"] == 0.0


def test_ion_config_errors(gpu_lib):
    _announce("ions: config and call errors")
    from paper_1612_07592_amd.binding import PicError
    w = S.ions_2d()
    w["ion_mass_me"] = 0.5
    with pytest.raises(PicError):
        gpu_lib.Sim(w)
    g = gpu_lib.Sim(S.small_2d())
    assert g.Ni == 0
    with pytest.raises(PicError):
        g.ions()
    g2 = gpu_lib.Sim(S.ions_2d())
    x = g2.ions()["x"]
    x[0, 0] = -1.0       # a live ion outside the box is refused
    with pytest.raises(PicError):
        g2.set_ions(x, np.zeros_like(x))
