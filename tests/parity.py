"""Element-by-element comparison of a HIP run with the oracle on the same
seeded inputs.  Bar for FP64: identical emission events (parent, step,
process), momenta and positions within 1e-12 relative (absolute below 1 mc /
1 c/w0), photon energies within 1e-12 relative, exact counts, energy sums
within 1e-11 relative."""
from __future__ import annotations

import numpy as np

P_TOL = 1e-12
SUM_TOL = 1e-11


def _rel(a, b, floor=1.0):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def photon_table(ph):
    """Photons sorted by (parent id, step, process) for set comparison."""
    order = np.lexsort((ph["proc"], ph["step"], ph["parent"]))
    return {k: np.asarray(v)[order] for k, v in ph.items()}


def compare(o, g, p_tol=P_TOL, label="", check_tau=True, p_scale=None):
    """p_scale: optional per-electron momentum scale (e.g. the |p| a beam
    started with).  Recoil computes the new momentum from gamma - eps, a
    difference of two numbers of the size of the old energy, so after an
    emission that takes most of the energy the remaining momentum carries the
    absolute rounding of the old one; momenta are then compared relative to
    the larger of the two scales."""
    eo, eg = o.electrons(), g.electrons()
    rep = {}
    assert eo["x"].shape == eg["x"].shape, label
    assert np.array_equal(eo["alive"], eg["alive"]), f"{label}: alive masks differ at " \
        f"{np.nonzero(eo['alive'] != eg['alive'])[0][:10]}"
    scale = np.maximum(np.linalg.norm(eo["p"], axis=1), 1.0)
    if p_scale is not None:
        scale = np.maximum(scale, np.asarray(p_scale))
    dpn = np.linalg.norm(eo["p"] - eg["p"], axis=1) / scale
    dxn = np.linalg.norm(eo["x"] - eg["x"], axis=1) / np.maximum(np.linalg.norm(eo["x"], axis=1), 1.0)
    rep["max_dp"] = float(dpn.max()) if dpn.size else 0.0
    rep["max_dx"] = float(dxn.max()) if dxn.size else 0.0
    assert rep["max_dp"] <= p_tol, f"{label}: momentum mismatch {rep['max_dp']:.3e} at id {int(np.argmax(dpn))}"
    assert rep["max_dx"] <= p_tol, f"{label}: position mismatch {rep['max_dx']:.3e} at id {int(np.argmax(dxn))}"
    assert np.array_equal(eo["w"], eg["w"]), label
    if check_tau:
        dt = _rel(eg["tau"], eo["tau"])
        rep["max_dtau"] = float(dt.max()) if dt.size else 0.0
        assert rep["max_dtau"] <= p_tol, f"{label}: optical depth mismatch {rep['max_dtau']:.3e}"
    so, sg = o.stats(), g.stats()
    for k in ("events", "kept"):
        assert list(so[k]) == list(sg[k]), f"{label}: {k} oracle {so[k]} gpu {sg[k]}"
    assert so["dropped_ncs"] == sg["dropped_ncs"], label
    assert so["overflow"] == sg["overflow"], label
    assert so["live"] == sg["live"], label
    assert np.array_equal(so["spectrum"], sg["spectrum"]), f"{label}: kept-photon spectra differ"
    for i in range(2):
        assert abs(sg["e_rad_kept"][i] - so["e_rad_kept"][i]) <= SUM_TOL * max(abs(so["e_rad_kept"][i]), 1e-300), label
    assert abs(sg["e_rad_dropped"] - so["e_rad_dropped"]) <= SUM_TOL * max(abs(so["e_rad_dropped"]), 1e-300), label
    po, pg = photon_table(o.photons()), photon_table(g.photons())
    assert len(po["energy"]) == len(pg["energy"]), f"{label}: photon count {len(po['energy'])} vs {len(pg['energy'])}"
    for k in ("parent", "step", "proc"):
        assert np.array_equal(po[k], pg[k]), f"{label}: photon {k} lists differ"
    if len(po["energy"]):
        rep["max_deps"] = float(_rel(pg["energy"], po["energy"], 1e-300).max())
        assert rep["max_deps"] <= p_tol, f"{label}: photon energy mismatch {rep['max_deps']:.3e}"
        assert np.abs(pg["k"] - po["k"]).max() <= p_tol, label
        assert np.abs(pg["x"] - po["x"]).max() <= p_tol * max(1.0, np.abs(po["x"]).max()), label
        assert np.array_equal(pg["w"], po["w"]), label
    rep["events"] = list(so["events"])
    rep["photons"] = int(len(po["energy"]))
    return rep
