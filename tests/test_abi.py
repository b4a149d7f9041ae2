"""The C-ABI library on the host: it loads, exports every entry point the
header declares, validates configs and builds tables (no GPU calls)."""
from __future__ import annotations

import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1612_07592_amd import binding as B
from paper_1612_07592_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = declared_symbols()
    for n in ("pic_create", "pic_load_tables", "pic_step", "pic_emission_stats", "pic_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = B.load()
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pic_\w+)", out))
    missing = [n for n in declared_symbols() if n not in exported]
    assert not missing, missing
    for n in declared_symbols():
        assert getattr(L, n) is not None
    assert set(B.EXPORTS) == set(declared_symbols())


def test_binding_struct_layouts_match_header():
    """The ctypes mirrors have the sizes a C compiler gives the header structs."""
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "pic.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(pic_config), sizeof(pic_tables),
         sizeof(pic_stats), offsetof(pic_config, stream), offsetof(pic_tables, br_cdf),
         sizeof(pic_server_config), offsetof(pic_server_config, stream), sizeof(pic_job_result),
         offsetof(pic_job_result, stats), sizeof(pic_buffers), offsetof(pic_buffers, photon_proc));
  return 0;
}'''
    d = os.path.join(ROOT, "_build")
    os.makedirs(d, exist_ok=True)
    c = os.path.join(d, "layout.c")
    exe = os.path.join(d, "layout")
    open(c, "w").write(src)
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
    got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(B.pic_config), C.sizeof(B.pic_tables), C.sizeof(B.pic_stats),
            B.pic_config.stream.offset, B.pic_tables.br_cdf.offset,
            C.sizeof(B.pic_server_config), B.pic_server_config.stream.offset,
            C.sizeof(B.pic_job_result), B.pic_job_result.stats.offset,
            C.sizeof(B.pic_buffers), B.pic_buffers.photon_proc.offset]
    assert got == want


def _mem(w):
    L = B.load()
    c = B.config_from(w)
    n = C.c_uint64()
    return L.pic_memory_required(C.byref(c), C.byref(n)), n.value


def test_memory_required_counts_buffers():
    code, n1 = _mem(W.c1())
    assert code == 0 and n1 > 0
    code, n2 = _mem(W.c2())
    assert code == 0
    # C2 holds 2M electrons, a 2048x1024 grid and a 4e8-photon buffer
    assert n2 > 400_000_000 * 40


@pytest.mark.parametrize("field,value", [
    ("dims", 4), ("ppc", 0), ("cfl", 1.2), ("cfl", 0.0), ("Z", 0), ("charge_state", 100),
    ("lambda_m", -1.0), ("ne_over_nc", float("nan")), ("a0", float("inf")),
    ("photon_cut_mc2", -1.0), ("thickness_lambda", -0.5)])
def test_invalid_configs_rejected(field, value):
    w = W.c1()
    w[field] = value
    code, _ = _mem(w)
    assert code == 1  # PIC_ERR_INVALID
    msg = B.load().pic_last_error(None)
    assert msg and len(msg) > 3


def test_mobile_ion_configs():
    """The Sec. III solid runs fit one GPU; mobile ions add their arrays and
    per-cell counts; bad ion parameters are refused."""
    code, n_au = _mem(W.solid("au"))
    assert code == 0 and n_au < 64 * 2**30, n_au
    w = W.solid("al", cells=200)
    code, with_ions = _mem(w)
    assert code == 0
    w0 = dict(w, ion_ppc=0)
    code, without = _mem(w0)
    ni = W.num_electrons(w) // w["ppc"] * w["ion_ppc"]
    assert with_ions - without >= ni * (2 * 8 + 3 * 8 + 1)
    for k, v in (("ion_ppc", -1), ("ion_ppc", 5000), ("ion_mass_me", 0.5),
                 ("ion_mass_me", float("nan"))):
        assert _mem(dict(w, **{k: v}))[0] == 1, (k, v)
    c = B.config_from(w)
    c.envelope = 2
    n = C.c_uint64()
    assert B.load().pic_memory_required(C.byref(c), C.byref(n)) == 1
    c = B.config_from(w)
    c.reserved0 = 1
    assert B.load().pic_memory_required(C.byref(c), C.byref(n)) == 1


def test_invalid_grid_rejected():
    w = W.c1()
    w["n"] = [4]
    assert _mem(w)[0] == 1
    w = W.c1()
    w["dx_lambda"] = [0.0]
    assert _mem(w)[0] == 1


def test_abi_version_checked():
    L = B.load()
    c = B.config_from(W.c1())
    c.abi_version = 99
    n = C.c_uint64()
    assert L.pic_memory_required(C.byref(c), C.byref(n)) == 1


def test_batch_and_server_argument_checks():
    """Argument checks that fail before any device call."""
    L = B.load()
    h = C.c_void_p()
    assert L.pic_batch_create(None, None) == 1
    assert L.pic_step_many(None, None, None, 0) == 1
    sc = B.pic_server_config()
    sc.abi_version = B.PIC_ABI_VERSION
    sc.max_jobs = 0
    sc.quantum_steps = 8
    assert L.pic_server_create(C.byref(sc), C.byref(h)) == 1
    sc.max_jobs = 4
    sc.quantum_steps = 0
    assert L.pic_server_create(C.byref(sc), C.byref(h)) == 1
    sc.quantum_steps = 8
    sc.abi_version = 7
    assert L.pic_server_create(C.byref(sc), C.byref(h)) == 1
    job = C.c_uint64()
    cfg = B.config_from(W.c1())
    assert L.pic_server_submit(None, C.byref(cfg), None, 1, -1.0, C.byref(job)) == 1
    n = C.c_int32()
    assert L.pic_server_poll(None, None, 0, C.byref(n)) == 1
    assert L.pic_server_run(None, None, None) == 1
    L.pic_server_destroy(None)
    L.pic_batch_destroy(None)
    assert L.pic_server_clock(None) == 0.0


def test_null_arguments():
    L = B.load()
    h = C.c_void_p()
    assert L.pic_create(None, C.byref(h)) == 1
    assert L.pic_step(None, 1) == 1
    L.pic_destroy(None)  # NULL is a no-op


@pytest.mark.slow
def test_library_tables_match_oracle_tables(tables_au):
    """Two independent quadratures of the same formulas agree (library:
    trapezoid Bessel sums + adaptive Simpson; oracle: scipy K, adaptive GL)."""
    t = B.pic_build_tables(79, 1.0, 0)
    assert abs(t["ln_eta0"] - tables_au["ln_eta0"]) < 1e-15
    assert np.allclose(t["ln_xi"], tables_au["ln_xi"], rtol=0, atol=1e-13)
    assert np.max(np.abs(t["h"] / tables_au["h"] - 1)) < 1e-9
    assert np.max(np.abs(t["ncs_cdf"] - tables_au["ncs_cdf"])) < 1e-9
    pos = tables_au["sigma"] > 0
    assert np.array_equal(t["sigma"] > 0, pos)
    assert np.max(np.abs(t["sigma"][pos] / tables_au["sigma"][pos] - 1)) < 1e-9
    assert np.max(np.abs(t["br_cdf"] - tables_au["br_cdf"])) < 1e-9


def test_library_pair_tables_match_oracle_tables(tables_au):
    """Two independent quadratures of the pair spectra and cross-sections
    (library: trapezoid Bessel sums + adaptive Simpson; oracle: scipy K and
    adaptive Gauss-Legendre) agree."""
    t = B.pic_build_pair_tables(79, 8)
    assert t["pair_checksum"] != 0
    assert abs(t["ln_chi0"] - tables_au["ln_chi0"]) < 1e-15 and abs(t["ln_k0"] - tables_au["ln_k0"]) < 1e-15
    assert np.abs(t["bw_lnT"] - tables_au["bw_lnT"]).max() < 1e-9
    assert np.abs(t["bw_cdf"] - tables_au["bw_cdf"]).max() < 1e-9
    pos = tables_au["bh_sigma"] > 0
    assert np.array_equal(t["bh_sigma"] > 0, pos)
    assert np.max(np.abs(t["bh_sigma"][pos] / tables_au["bh_sigma"][pos] - 1)) < 1e-8
    assert np.abs(t["bh_cdf"] - tables_au["bh_cdf"]).max() < 1e-8


def test_build_tables_rejects_bad_args():
    L = B.load()
    out = B.pic_tables()
    z = np.zeros(256 * 256)
    assert L.pic_build_tables(0, 1.0, 1, z.ctypes.data, z.ctypes.data, z.ctypes.data,
                              z.ctypes.data, z.ctypes.data, C.byref(out)) == 1
    assert L.pic_build_tables(13, 0.0, 1, z.ctypes.data, z.ctypes.data, z.ctypes.data,
                              z.ctypes.data, z.ctypes.data, C.byref(out)) == 1


def test_free_path_flag_checked_and_counted():
    """PIC_BREM_FREEPATH needs PIC_BREM, and its collision depths (one
    double per electron in each of the two electron buffers) are counted by
    pic_memory_required."""
    w = W.c2()
    code, n0 = _mem(w)
    assert code == 0
    code, n1 = _mem(dict(w, brem_freepath=True))
    assert code == 0
    assert n1 - n0 >= 2 * 8 * W.num_electrons(w)
    assert _mem(dict(w, brem_freepath=True, brem=False))[0] == 1


def test_workload_sizes():
    """Electron counts of the recipes as the configurations state them."""
    assert W.num_electrons(W.c1()) == 8192
    assert W.num_electrons(W.c2()) == 2_097_152
    assert W.num_electrons(W.c5()) == 134_217_728
    assert W.num_electrons(W.thick_target()) == 5000 * 420
    assert sum(W.num_electrons(j) for j in W.c3_jobs()) == 5_898_240  # 5.9e9 e-steps over 1000 steps


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N > 1 exits with a message (one GPU only), before it
    touches torch or the GPU."""
    r = subprocess.run(["python3", os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _zero_stats():
    return dict(kept=[0, 0], e_rad_kept=[0.0, 0.0], e_rad_dropped=0.0, events=[0, 0])


def test_bench_precision_check_without_photons():
    """A window that ends before anything radiates (no photons, zero
    radiated energy) yields None figures, not an exception, all the way
    through the seed-spread summary."""
    import numpy as np
    b = _bench()
    empty = dict(energy=np.zeros(0))
    pc = b.precision_check(_zero_stats(), _zero_stats(), empty, empty)
    assert pc["radiated_energy"]["rel"] is None and pc["radiated_energy"]["pass"] is None
    assert pc["spectrum_ks"]["statistic"] is None and pc["spectrum_ks"]["p"] is None
    assert pc["photon_count"]["z"] == 0.0
    refs = [b.precision_check(_zero_stats(), _zero_stats()) for _ in range(2)]
    s = b.seed_spread(pc, refs)
    assert s["radiated_energy"] is None and s["spectrum_ks"] is None
    assert s["photon_count"] is True
    # one side radiated, the other not
    one = dict(_zero_stats(), kept=[3, 0], e_rad_kept=[5.0, 0.0])
    pc = b.precision_check(one, _zero_stats())
    assert pc["radiated_energy"]["rel"] is None and pc["photon_count"]["fp32"] == 3


def test_bench_window_is_centred_on_the_interaction():
    """The timed window of the 2D gold slab sits around the step at which
    the envelope peak reaches the slab front, inside the run; a window as
    long as the run starts at step 0."""
    b = _bench()
    from paper_1612_07592_amd import workloads as W
    w = W.c2()
    pk = b.peak_step(w)
    # the peak leaves the source at 5 periods and crosses 2 um: 7 periods
    assert abs(pk * b.step_dt(w) - 14 * math.pi) < b.step_dt(w)
    lead, k = b.window(w, 20)
    assert lead <= pk <= lead + k and lead + k <= w["steps"]
    assert b.window(w, w["steps"]) == (0, w["steps"])
    lead, k = b.window(w, 1990)
    assert lead + k <= w["steps"]
    w5 = W.c5()
    lead, k = b.window(w5, 20)
    assert lead <= b.peak_step(w5) <= lead + k


def test_hot_path_declarations_cite_the_paper():
    """Each of the calls of the hot path says which passage defines what it
    computes (a section or an equation of the paper)."""
    text = open(HEADER).read()
    for name in ("pic_create", "pic_load_tables", "pic_step", "pic_emission_stats"):
        m = re.search(r"/\*((?:(?!\*/).)*)\*/\s*pic_status\s+" + name + r"\(", text, flags=re.S)
        assert m, name
        assert re.search(r"Sec\. I|Eq\. \(", m.group(1)), name
    m = re.search(r"/\*((?:(?!\*/).)*)\*/\s*void\s+pic_destroy\(", text, flags=re.S)
    assert m and "no passage" in m.group(1)


def test_device_pointer_convention_names_get_buffers():
    text = open(HEADER).read()
    head = text[:text.index("#ifndef LIBPIC_PIC_H")]
    assert "never exposed." not in head
    assert "pic_get_buffers" in head


def test_bench_laser_energy_is_what_the_source_injects():
    """The laser energy the Sec. III energy fractions are taken of: a flat
    pulse of 30 fs through a 1 um Gaussian waist, a0^2/2 w0 sqrt(pi/2) T,
    equals the field energy of an oracle vacuum run at the moment the last of
    the pulse has left the source (box wide enough to hold the beam)."""
    import oracle
    import conftest
    import scenarios as S
    b = _bench()
    w = S.base(name="vacuum", dims=2, n=[512, 384], dx_lambda=[1 / 32, 1 / 32], ppc=1,
               x0_lambda=0.0, thickness_lambda=0.0, a0=10.0, w0_lambda=1.0,
               focus_x_lambda=2.0, duration_cycles=30e-15 * 299792458.0 / 1e-6,
               envelope="flat", ncs=False, brem=False, ne_over_nc=0.0)
    o = oracle.OracleSim(w, conftest.oracle_tables(13))
    assert o.N == 0
    T = w["duration_cycles"] * 2 * math.pi
    o.step(int(T / o.derived()["dt"]))
    assert abs(o.field_energy() / b.laser_energy(w) - 1.0) < 0.01
