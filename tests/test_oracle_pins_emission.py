"""Pins of the oracle's emission side against closed forms, independent
numbers and direct quadrature of the paper's formulas:

  eta          closed forms in pure E (p parallel / normal to E), in crossed
               E = B fields, in pure B, and invariance under Lorentz boosts;
  NCS          the per-step optical depth at eta between table points against
               K_N (eta/gamma) h(eta) dt with h by direct quadrature of F/chi;
               sampled photon fractions at eta = 0.3, 1, 3 (between rows)
               against the cumulative F(eta, chi)/chi spectrum by quadrature;
  brem         sigma(T) between table points against the Tsai bracket of
               Eq. (1) integrated directly; sampled photon energies between
               rows against the cumulative Tsai spectrum;
  constants    E_S, K_N, K_BR and n_c against independently computed values.

Each check takes the oracle library to run (None = the oracle itself), so that
tests/test_oracle_mutants.py can show it fails on a planted mistake.  CPU only.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

import oracle
import scenarios as S
from oracle import tables as T


def _probe(Z, lib=None):
    import conftest
    w = S.frozen_B_beam(n_cells=8, ppc=1, slab=(3, 4), B=0.0, Z=Z, charge_state=Z)
    return oracle.OracleSim(w, conftest.oracle_tables(Z), nthreads=1, lib=lib), conftest.oracle_tables(Z)


# ------------------------------------------------------------------- eta
def _boost(E, B, p, beta):
    """Fields and momentum seen from a frame moving with velocity beta."""
    b2 = beta @ beta
    g = 1.0 / math.sqrt(1.0 - b2)
    n = beta / math.sqrt(b2)
    Ep = (E @ n) * n
    Bp = (B @ n) * n
    E2 = Ep + g * (E - Ep + np.cross(beta, B))
    B2 = Bp + g * (B - Bp - np.cross(beta, E))
    ge = math.sqrt(1.0 + p @ p)
    pp = (p @ n) * n
    p2 = p - pp + g * (pp - ge * beta)
    return E2, B2, p2


def check_eta_closed_forms(lib=None):
    o, _ = _probe(13, lib)
    ES = 1e-6 / (2.0 * math.pi * 3.8615926796e-13)   # lambda / (2 pi reduced Compton)
    rel = lambda a, b: abs(a - b) / max(abs(b), 1e-300)
    zero = np.zeros(3)
    worst = 0.0
    for g0 in (1.5, 40.0, 3000.0):
        pm = math.sqrt(g0 * g0 - 1.0)
        for Em in (0.7, 300.0):
            # pure E, p parallel to E: eta = |E| / E_S whatever gamma
            worst = max(worst, rel(o.probe_eta([Em, 0, 0], zero, [pm, 0, 0]), Em / ES))
            worst = max(worst, rel(o.probe_eta([0, -Em, 0], zero, [0, 2 * pm / 2, 0]), Em / ES))
            # pure E, p normal to E: eta = gamma |E| / E_S
            worst = max(worst, rel(o.probe_eta([0, Em, 0], zero, [pm, 0, 0]), g0 * Em / ES))
            worst = max(worst, rel(o.probe_eta([0, 0, Em], zero, [0, pm, 0]), g0 * Em / ES))
            # pure B, p normal to B: eta = |p| |B| / E_S
            worst = max(worst, rel(o.probe_eta(zero, [0, 0, Em], [pm, 0, 0]), pm * Em / ES))
    # crossed fields of a plane wave along x, E_y = B_z: eta = |gamma - p_x| E / E_S
    rng = np.random.default_rng(3)
    for _ in range(50):
        Em = rng.uniform(1, 500)
        p = rng.normal(size=3) * rng.uniform(1, 2000)
        ge = math.sqrt(1.0 + p @ p)
        worst = max(worst, rel(o.probe_eta([0, Em, 0], [0, 0, Em], p), abs(ge - p[0]) * Em / ES))
        worst = max(worst, rel(o.probe_eta([0, 0, Em], [0, -Em, 0], p), abs(ge - p[0]) * Em / ES))
    # invariance under boosts
    for _ in range(50):
        E = rng.normal(size=3) * 50
        B = rng.normal(size=3) * 50
        p = rng.normal(size=3) * 30
        beta = rng.normal(size=3)
        beta *= rng.uniform(0.1, 0.9) / np.linalg.norm(beta)
        E2, B2, p2 = _boost(E, B, p, beta)
        eta = o.probe_eta(E, B, p)
        assert eta > 0.0, (E, B, p)
        worst = max(worst, rel(o.probe_eta(E2, B2, p2), eta))
    o.close()
    assert worst < 1e-9, worst
    return worst


def test_eta_closed_forms_and_invariance(oracle_lib):
    print(check_eta_closed_forms())


# -------------------------------------------------------------- NCS rate
def _off_node(ln0, dln, x, frac):
    """A point between table nodes: the node at or below x, plus frac of the
    spacing (in the log coordinate)."""
    i = math.floor((math.log(x) - ln0) / dln)
    return math.exp(ln0 + (i + frac) * dln), i


def check_ncs_rate_off_node(lib=None):
    """Optical depth per step between eta nodes: K_N (eta/gamma) h(eta) dt,
    h(eta) = int_0^1 F(eta, xi)/xi dxi by direct quadrature, within the
    error of linear interpolation in ln eta (h'' from the table's second
    differences) and the quadrature's own accuracy."""
    o, tb = _probe(13, lib)
    d = o.derived()
    worst = 0.0
    for eta_t, frac in ((1e-3, 0.12), (0.05, 0.83), (0.3, 0.1), (1.0, 0.9), (3.0, 0.15), (20.0, 0.8)):
        eta, i = _off_node(tb["ln_eta0"], tb["dln_eta"], eta_t, frac)
        h = T.ncs_h_g(eta)[0]
        gamma = 1234.5
        want = d["K_N"] * eta / gamma * h * d["dt"]
        got = o.probe_ncs_dtau(eta, gamma)
        h2 = abs(tb["h"][i + 1] - 2 * tb["h"][i] + tb["h"][i - 1]) + abs(tb["h"][i + 2] - 2 * tb["h"][i + 1] + tb["h"][i])
        tol = (frac * (1 - frac) * 0.5 * h2 + 1e-9 * h) / h
        err = abs(got / want - 1)
        worst = max(worst, err / tol)
        assert err <= tol, (eta, got, want, err, tol)
    o.close()
    return worst


def test_ncs_rate_between_table_points(oracle_lib):
    print(check_ncs_rate_off_node())


# ---------------------------------------------------------- NCS sampling
def _ncs_cdf_direct(eta, n=3000):
    """The cumulative photon-fraction spectrum at eta, int_0^xi F/x dx / h,
    on a fine ln(xi) grid (direct quadrature of every interval)."""
    lx = np.linspace(math.log(T.XI_MIN), 0.0, n)
    f = lambda u: T.ncs_F(eta, np.exp(u))
    scale = float(np.sum(T._gl_panel(f, lx[:-1], lx[1:])))
    per = T.adaptive_integrals(f, lx[:-1], lx[1:], atol=1e-15 * scale)
    # mass below the grid: F/xi ~ xi^(-2/3) there, int = 3 xi0 F(xi0)/xi0 ... use the same panels below
    below_e = np.linspace(lx[0] - 60.0, lx[0], 31)
    below = float(np.sum(T.adaptive_integrals(f, below_e[:-1], below_e[1:], atol=1e-16 * scale)))
    cum = np.concatenate([[below], below + np.cumsum(per)])
    return lx, cum / cum[-1]


def check_ncs_sampling_quantum(lib=None):
    """Photon fractions drawn at eta = 0.3, 1 and 3 (between table rows) by
    the inverse-CDF step: at stratified uniforms u_k = (k + 1/2)/N the drawn
    xi_k are the quantiles of the sampled law, so max_k |C(xi_k) - u_k| with
    C the directly integrated spectrum is its Kolmogorov distance."""
    o, tb = _probe(13, lib)
    N = 4000
    u = (np.arange(N) + 0.5) / N
    out = []
    for eta_t, frac in ((0.3, 0.1), (1.0, 0.9), (3.0, 0.15)):
        eta, _ = _off_node(tb["ln_eta0"], tb["dln_eta"], eta_t, frac)
        xi = o.probe_ncs_xi(eta, u)
        lx, C = _ncs_cdf_direct(eta)
        Ck = np.interp(np.log(xi), lx, C)
        D = float(np.abs(Ck - u).max())
        out.append((eta, D))
        assert D < 2e-3, (eta, D)
    o.close()
    return out


def test_ncs_sampling_quantum_regime(oracle_lib):
    print(check_ncs_sampling_quantum())


# ------------------------------------------------------------ brem sigma
def _sigma_direct(T_mc2, Z, k_cut=1.0):
    E = T_mc2 + 1.0
    f = lambda lk: float(T.tsai_bracket(np.exp(lk) / E, E, Z))
    v, _ = integrate.quad(f, math.log(k_cut), math.log(T_mc2), epsabs=0, epsrel=1e-12, limit=200)
    return v


def check_brem_sigma_off_node(lib=None):
    """sigma(T) between table points against int_{k_cut}^{T} B(k/E) dk/k by
    direct quadrature (scipy), within the error of linear interpolation in
    ln T (sigma'' from the table's second differences)."""
    o, tb = _probe(79, lib)
    worst = 0.0
    for Tmev, frac in ((0.8, 0.2), (2.0, 0.85), (7.0, 0.1), (30.0, 0.9), (150.0, 0.3), (800.0, 0.75)):
        Tk, i = _off_node(tb["ln_T0"], tb["dln_T"], Tmev / T.MC2_MEV, frac)
        want = _sigma_direct(Tk, 79)
        got = o.probe_brem_sigma(Tk)
        s = tb["sigma"]
        s2 = abs(s[i + 1] - 2 * s[i] + s[i - 1]) + abs(s[i + 2] - 2 * s[i + 1] + s[i])
        tol = frac * (1 - frac) * 0.5 * s2 + 1e-8 * want
        worst = max(worst, abs(got - want) / tol)
        assert abs(got - want) <= tol, (Tmev, got, want, tol)
    o.close()
    return worst


def test_brem_sigma_between_table_points(oracle_lib):
    print(check_brem_sigma_off_node())


def check_brem_sampling_off_node(lib=None):
    """Photon energies drawn at electron energies between table rows: at
    stratified uniforms the drawn k are the quantiles of the sampled law;
    compared with the directly integrated Tsai spectrum
    S(k) = int_{k_cut}^{k} B dk'/k' / sigma(T) (Kolmogorov distance)."""
    o, tb = _probe(79, lib)
    N = 3000
    u = (np.arange(N) + 0.5) / N
    out = []
    for Tmev, frac in ((3.0, 0.1), (40.0, 0.85), (400.0, 0.2)):
        Tk, _ = _off_node(tb["ln_T0"], tb["dln_T"], Tmev / T.MC2_MEV, frac)
        E = Tk + 1.0
        eps = o.probe_brem_eps(Tk, u)
        lk = np.linspace(0.0, math.log(Tk), 2001)
        f = lambda x: T.tsai_bracket(np.exp(x) / E, E, 79)
        per = T.adaptive_integrals(f, lk[:-1], lk[1:], atol=1e-14)
        cum = np.concatenate([[0.0], np.cumsum(per)])
        Sk = np.interp(np.log(eps), lk, cum / cum[-1])
        D = float(np.abs(Sk - u).max())
        out.append((Tmev, D))
        assert D < 2e-3, (Tmev, D)
    o.close()
    return out


def test_brem_sampling_between_table_rows(oracle_lib):
    print(check_brem_sampling_off_node())


# -------------------------------------------------------------- constants
def check_constants(lib=None):
    """Derived constants of a lambda = 1 um run against values computed
    independently of the oracle's formulas (survey of the method):
    E_S = m c^2 / (hbar w0) = 4.12148e5, K_N = 829.09 per 1/w0,
    K_BR = n_c (c/w0) alpha r_e^2 = 1.02817e-11, n_c = 1.11485e27 m^-3."""
    o, _ = _probe(13, lib)
    d = o.derived()
    o.close()
    for key, want, tol in (("E_S", 4.12148e5, 2e-6), ("K_N", 829.09, 2e-5),
                           ("K_BR", 1.02817e-11, 2e-5), ("n_c", 1.11485e27, 2e-5)):
        assert abs(d[key] / want - 1) < tol, (key, d[key], want)
    return d


def test_constants_against_independent_values(oracle_lib):
    print(check_constants())


# ------------------------------------------------------- exp, log, expm1
def check_math_against_libm(lib=None):
    """The oracle's own exp, log and expm1 against the platform libm over
    wide random arguments: within 1, 3 and 4 ulp, exact at the special
    points."""
    rng = np.random.default_rng(1)
    ulps = lambda a, b: np.abs(a - b) / np.spacing(np.abs(b))
    x = np.concatenate([rng.uniform(-30, 30, 20000), rng.uniform(-1, 1, 10000),
                        rng.uniform(-700, 700, 5000)])
    y = np.concatenate([np.exp(rng.uniform(-740, 709, 20000)), rng.uniform(0.5, 2, 10000),
                        1 + rng.normal(scale=1e-6, size=5000)])
    z = np.concatenate([rng.uniform(-0.35, 0.35, 10000), -np.exp(rng.uniform(-40, 0, 10000)),
                        rng.uniform(-30, 5, 10000)])
    e1 = ulps(oracle.math("exp", x, lib), np.exp(x)).max()
    e2 = ulps(oracle.math("log", y, lib), np.log(y)).max()
    e3 = ulps(oracle.math("expm1", z, lib), np.expm1(z)).max()
    assert e1 <= 1.0 and e2 <= 3.0 and e3 <= 4.0, (e1, e2, e3)
    assert oracle.math("exp", [0.0], lib)[0] == 1.0 and oracle.math("log", [1.0], lib)[0] == 0.0
    assert oracle.math("expm1", [0.0], lib)[0] == 0.0
    assert oracle.math("log", [0.5], lib)[0] == -math.log(2.0)
    return e1, e2, e3


def test_oracle_math_against_libm(oracle_lib):
    print(check_math_against_libm())


def check_spectrum_bins(lib=None):
    """The kept-photon spectrum of the statistics counts every kept photon in
    its quarter octave: against floor(4 log2(eps)) + 8 of the stored records
    (a run with every photon stored), per process."""
    import conftest
    w = S.frozen_B_beam(B=50.0, ne=5e7, Z=79, charge_state=79, photon_cut_mc2=0.0,
                        photon_capacity=1 << 20)
    o = oracle.OracleSim(w, conftest.oracle_tables(79), nthreads=1, lib=lib)
    e = o.electrons()
    o.set_electrons(e["x"], S.beam_momenta(o.N, 5.0, 2000.0, 22), e["tau"])
    o.step(60)
    st = o.stats()
    ph = o.photons()
    assert st["overflow"] == 0 and len(ph["energy"]) == sum(st["kept"])
    ref = np.zeros((2, 64), dtype=np.uint64)
    b = np.clip(np.floor(4.0 * np.log2(ph["energy"])).astype(np.int64) + 8, 0, 63)
    np.add.at(ref, (ph["proc"].astype(np.int64), b), 1)
    assert np.array_equal(st["spectrum"], ref), np.nonzero(st["spectrum"] != ref)
    assert ref[0].sum() > 1000 and ref[1].sum() > 1000
    return ref.sum(axis=1)


def test_kept_photon_spectrum_bins(oracle_lib):
    print(check_spectrum_bins())
