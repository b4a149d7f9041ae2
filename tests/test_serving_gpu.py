"""Batched stepping and the scan-job server on the GPU: every run advanced in
a batch, or served in a mix of other jobs, ends in the same state as the same
run stepped alone with pic_step.

Bar: electron positions, momenta, optical depths, alive masks, fields and the
fixed-point current identical; photon records identical as sets (append order
is not deterministic); event counts identical; FP64 energy sums within 1e-12
relative (their order inside a wave slot follows the in-tile order of the
sort, which is not deterministic)."""
from __future__ import annotations

import numpy as np
import pytest

import scenarios as S
from parity import photon_table

pytestmark = pytest.mark.gpu
SUM_REL = 1e-12


def _mix(tables_al, tables_au):
    """Uneven runs: 1D/2D/3D, FP64 and FP32, different step counts."""
    c1 = S.c1_parity(64)
    c1f = dict(S.c1_parity(64), precision="fp32", seed=21, job_id=5)
    out = [
        (S.small_2d(precision="fp32"), tables_au, 70),
        (S.small_2d(precision="fp64"), tables_au, 45),
        (c1, tables_al, 64),
        (c1f, tables_al, 50),
        (S.small_3d(precision="fp32"), tables_au, 30),
        (S.ions_2d(steps=40), tables_au, 40),            # a run with mobile ions
    ]
    return out


def assert_same_run(a, b, label):
    ea, eb = a.electrons(), b.electrons()
    assert np.array_equal(ea["alive"], eb["alive"]), label
    for k in ("x", "p", "tau", "w"):
        assert np.array_equal(ea[k], eb[k]), f"{label}: electron {k} differs " \
            f"(max {np.max(np.abs(ea[k] - eb[k])):.3e})"
    assert np.array_equal(a.fields(), b.fields()), f"{label}: fields differ"
    assert np.array_equal(a.current(), b.current()), f"{label}: current differs"
    sa, sb = a.stats(), b.stats()
    for k in ("steps", "live", "electron_steps", "events", "kept", "dropped_ncs", "overflow",
              "brem_clamped", "photons_stored"):
        assert sa[k] == sb[k], f"{label}: {k} {sa[k]} vs {sb[k]}"
    for k in ("e_rad_dropped", "e_kin_e", "e_field"):
        assert abs(sa[k] - sb[k]) <= SUM_REL * max(abs(sa[k]), 1e-300), f"{label}: {k}"
    for i in range(2):
        assert abs(sa["e_rad_kept"][i] - sb["e_rad_kept"][i]) <= SUM_REL * max(abs(sa["e_rad_kept"][i]), 1e-300), label
    pa, pb = photon_table(a.photons()), photon_table(b.photons())
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), f"{label}: photon {k} differs"
    return sa


def _alone(gpu_lib, w, t, n):
    s = gpu_lib.Sim(w, t)
    s.pic_step(n)
    return s


def test_step_many_equals_step(gpu_lib, tables_al, tables_au):
    mix = _mix(tables_al, tables_au)
    # particle-only run with a beam in the mix too
    fz = S.frozen_B_beam(B=2000.0, seed=31)
    mix.append((fz, tables_al, 40))
    alone = []
    for w, t, n in mix:
        print(f"alone {w['name']} {w['precision']} steps={n}", flush=True)
        s = gpu_lib.Sim(w, t)
        if w.get("frozen"):
            e = s.electrons()
            s.set_electrons(e["x"], S.beam_momenta(s.N, 5.0, 2e3, 31), e["tau"])
        s.pic_step(n)
        alone.append(s)
    sims = []
    for w, t, n in mix:
        s = gpu_lib.Sim(w, t)
        if w.get("frozen"):
            e = s.electrons()
            s.set_electrons(e["x"], S.beam_momenta(s.N, 5.0, 2e3, 31), e["tau"])
        sims.append(s)
    b = gpu_lib.Batch()
    first = [min(n, 24) for _, _, n in mix]
    print("step_many", first, flush=True)
    b.step_many(sims, first)
    rest = [n - f for (_, _, n), f in zip(mix, first)]
    print("step_many", rest, flush=True)
    b.step_many(sims, rest)
    for (w, _, n), a, g in zip(mix, alone, sims):
        st = assert_same_run(a, g, f"{w['name']}/{w['precision']}")
        assert st["steps"] == n
    b.close()


def test_step_many_rejects_bad_lists(gpu_lib, tables_al):
    s = gpu_lib.Sim(S.c1_parity(8), tables_al)
    b = gpu_lib.Batch()
    with pytest.raises(gpu_lib.PicError):
        b.step_many([s, s], [1, 1])            # the same run twice
    with pytest.raises(gpu_lib.PicError):
        b.step_many([s], [-1])
    t = gpu_lib.Sim(S.c1_parity(8))           # no tables, emission on
    with pytest.raises(gpu_lib.PicError):
        b.step_many([s, t], [1, 1])
    assert s.stats()["steps"] == 0             # nothing moved
    b.step_many([s], [0])
    b.close()


def test_server_results_same_alone_and_in_mix(gpu_lib, tables_al, tables_au):
    mix = _mix(tables_al, tables_au)
    srv = gpu_lib.Server(max_jobs=3, quantum_steps=8, keep_finished=True, hbm_reserve_bytes=0)
    jobs = {}
    results = {}
    pending = list(enumerate(mix))
    rounds = 0
    # two arrivals per round: later jobs join while earlier ones are resident
    while pending or len(results) < len(mix):
        for _ in range(2):
            if pending:
                k, (w, t, n) = pending.pop(0)
                jobs[srv.submit(w, t, n)] = k
        print(f"round {rounds}", flush=True)
        srv.run()
        for r in srv.poll():
            results[r["job"]] = r
        rounds += 1
        assert rounds < 200
    resident_max = 0
    spans = [(r["t_admit"], r["t_finish"]) for r in results.values()]
    for t0, _ in spans:
        resident_max = max(resident_max, sum(1 for a, f in spans if a <= t0 < f))
    assert resident_max <= 3
    for job, r in results.items():
        w, t, n = mix[jobs[job]]
        assert r["status"] == "PIC_OK", r
        assert r["steps"] == n and r["stats"]["steps"] == n
        assert r["t_submit"] <= r["t_admit"] <= r["t_finish"]
        mixed = srv.job_sim(job, w)
        a = _alone(gpu_lib, w, t, n)
        assert_same_run(a, mixed, f"served {w['name']}/{w['precision']}")
        a.close()
        srv.release(job)
    srv.close()


def test_server_refuses_pair_production(gpu_lib, tables_au):
    from paper_1612_07592_amd.binding import PicError
    srv = gpu_lib.Server(max_jobs=2, quantum_steps=8, hbm_reserve_bytes=0)
    w = dict(S.small_2d(), bw=True, bh=True)
    with pytest.raises(PicError) as e:
        srv.submit(w, tables_au, 10)
    assert e.value.code == 1
    srv.close()


def test_server_admits_by_free_memory(gpu_lib, tables_au):
    import gc
    gc.collect()  # contexts of earlier tests
    # a photon buffer large enough that allocation rounding is small beside it
    w = dict(S.small_2d(precision="fp32"), photon_capacity=1 << 24)
    need = gpu_lib.pic_memory_required(w)
    free, _ = gpu_lib.pic_device_memory()
    # leave room for two such runs at most
    reserve = max(0, int(free - 2.5 * need))
    srv = gpu_lib.Server(max_jobs=16, quantum_steps=10, hbm_reserve_bytes=reserve)
    for k in range(5):
        srv.submit(dict(w, seed=100 + k, job_id=k), tables_au, 30)
    huge = dict(w, photon_capacity=1 << 40)
    big = srv.submit(huge, tables_au, 10)
    res = []
    for _ in range(100):
        r, q = srv.run()
        res += srv.poll()
        if r == 0 and q == 0:
            break
    assert len(res) == 6
    by = {r["job"]: r for r in res}
    assert by[big]["status"] == "PIC_ERR_NOMEM"
    ok = [r for r in res if r["job"] != big]
    assert all(r["status"] == "PIC_OK" for r in ok)
    spans = [(r["t_admit"], r["t_finish"]) for r in ok]
    most = max(sum(1 for a, f in spans if a <= t0 < f) for t0, _ in spans)
    assert most == 2, spans
    srv.close()
