"""Pins of the oracle's pair production (Breit-Wheeler in the fields,
Bethe-Heitler on the nuclei; photons in flight):

  tables      T(chi) of the Breit-Wheeler spectrum against its two published
              limits, (3/16) sqrt(3/2) exp(-8/(3 chi)) for chi << 1 and
              0.3796 chi^(-1/3) for chi >> 1 (the latter from Beta functions
              of the large-chi form); the Bethe-Heitler cross-section against
              the complete-screening limit (A / (X0 N_A)) (1 - 4/3 x (1 - x))
              and (7/9) A / (X0 N_A) at high energy, with the radiation
              lengths of the Particle Data Group (independent numbers);
  flight      photons injected in prescribed E and B: the number converting
              in m steps follows 1 - exp(-m dtau) with dtau = alpha (m c^2 /
              hbar w0) (chi / eps) T(chi) dt, chi = eps |E_perp + k x B| / E_S,
              and T by direct quadrature at off-node chi (three directions,
              three chi, one of them zero); Bethe-Heitler conversions on a
              dense target follow 1 - exp(-n sigma c dt) per step with sigma
              by direct quadrature at an off-node k;
  shares      the pair energy shares against the quadrature spectra (KS);
  kinematics  pair records at the emission point + k c dt per step travelled,
              e- + e+ = eps, both at least m c^2.

Each check takes the oracle library (None = the oracle itself).  CPU only."""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special, stats

import oracle
import scenarios as S
from oracle import tables as TB

ALPHA = 7.2973525693e-3
NA = 6.02214076e23
RE_CM = 2.8179403262e-13


def _tables(Z):
    import conftest
    return conftest.oracle_tables(Z)


# ---------------------------------------------------------------- tables ----
def check_bw_table_asymptotes(t=None):
    t = t or _tables(13)
    chi = np.exp(t["ln_chi0"] + np.arange(int(t["n_chi"])) * t["dln_chi"])
    T = np.exp(t["bw_lnT"])
    small = 3.0 / 16.0 * math.sqrt(1.5) * np.exp(-8.0 / (3.0 * chi))
    # Gamma(2/3)/2 3^(2/3) 2 B(8/3, 2/3) / (sqrt(3) pi)
    big = special.gamma(2 / 3) / 2 * 3 ** (2 / 3) * 2 * special.beta(8 / 3, 2 / 3) / (math.sqrt(3) * math.pi)
    assert abs(big - 0.3796) < 1e-3
    r_small = T[chi < 0.03] / small[chi < 0.03]
    assert np.all(np.abs(r_small - 1) < 0.01), r_small
    r_big = T[chi > 500] * chi[chi > 500] ** (1 / 3) / big
    assert np.all(np.abs(r_big - 1) < 0.03), r_big
    # the approach to both limits is monotone
    assert np.all(np.diff(r_small) < 0) and np.all(np.diff(r_big) > 0)
    # rows: symmetric in xi <-> 1 - xi, from 0 to 1
    C = t["bw_cdf"]
    assert np.all(C[:, 0] == 0.0) and np.all(C[:, -1] == 1.0)
    assert np.abs(C + C[:, ::-1] - 1.0).max() < 1e-9
    return float(np.abs(r_small - 1).max()), float(np.abs(r_big - 1).max())


def check_bh_table_limits(t=None, Z=79, A=196.966569, X0=6.46):
    t = t or _tables(Z)
    unit = ALPHA * RE_CM ** 2
    axn = A / (X0 * NA)                     # cm^2
    k = np.exp(t["ln_k0"] + np.arange(int(t["n_k"])) * t["dln_k"])
    sig = t["bh_sigma"] * unit
    hi = k > 1e4
    r = sig[hi] / (7.0 / 9.0 * axn)
    assert np.all(np.abs(r - 1) < 0.03), r
    assert np.all(np.diff(t["bh_sigma"][k > 20]) > 0)           # rises to the plateau
    # complete screening at very high energy: the shape 1 - 4/3 x (1 - x)
    x = np.linspace(0.05, 0.95, 19)
    d = TB.bh_dcs(x, 1e8, Z) * unit
    ref = axn * (1 - 4.0 / 3.0 * x * (1 - x))
    assert np.all(np.abs(d / ref - 1) < 0.03), d / ref
    assert np.allclose(TB.bh_dcs(x, 300.0, Z), TB.bh_dcs(1 - x, 300.0, Z), rtol=1e-12)
    C = t["bh_cdf"]
    assert np.all(C[:, -1] == 1.0)
    return float(np.abs(r - 1).max())


# ---------------------------------------------------------------- flight ----
E0, B0 = 300.0, 700.0


def _flight_sim(lib, w, photons):
    o = oracle.OracleSim(w, _tables(int(w["Z"])), nthreads=1, lib=lib)
    x, k, eps, wt, par = photons
    o.add_photons(x, k, eps, wt, par)
    return o


def _field_photons(n_per, eps, x0):
    """Three groups of n_per photons: along +x, -x and +z."""
    dirs = [(1.0, 0.0, 0.0), (-1.0, 0.0, 0.0), (0.0, 0.0, 1.0)]
    k = np.repeat(np.array(dirs), n_per, axis=0)
    n = k.shape[0]
    x = np.zeros((n, 3)); x[:, 0] = x0
    return x, k, np.full(n, eps), np.full(n, 0.5), 0x40000000 + np.arange(n, dtype=np.uint32)


def _bw_w(**kw):
    w = S.frozen_B_beam(B=B0, ne=1.0, ppc=1, slab=(0, 8))
    w.update(frozen_E=[0.0, E0, 0.0], ncs=False, brem=False, bw=True, bh=False,
             photon_capacity=1 << 16, pair_capacity=1 << 16)
    w.update(kw)
    return w


def check_bw_conversion_law(lib=None, n_per=4000, m=60):
    w = _bw_w()
    o0 = oracle.OracleSim(w, _tables(13), nthreads=1, lib=lib)
    d = o0.derived()
    ES, dt, x0 = d["E_S"], d["dt"], 0.5 * 1024 * d["dx"][0]
    o0.close()
    eps = 2400.0
    o = _flight_sim(lib, w, _field_photons(n_per, eps, x0))
    o.step(m + 1)                              # the first step only starts them
    f = o.flight()
    conv = (f["state"] == 2).reshape(3, n_per).sum(axis=1)
    chis = [eps * abs(E0 - B0) / ES, eps * (E0 + B0) / ES, eps * E0 / ES]
    zs = []
    for g, chi in enumerate(chis):
        T = TB.bw_T(chi)
        dtau = ALPHA * ES * chi / eps * T * dt
        p = 1.0 - math.exp(-m * dtau)
        sd = math.sqrt(n_per * p * (1 - p))
        zs.append((conv[g] - n_per * p) / sd)
        assert 0.05 < p < 0.95, (chi, p)
    assert max(abs(z) for z in zs) < 4.0, (chis, conv, zs)
    st = o.stats()
    assert st["pairs"] == [int(conv.sum()), 0]
    return zs


def check_bh_conversion_law(lib=None, n=20000, m=40, Z=79, ne=4e7):
    w = S.frozen_B_beam(B=0.0, ne=ne, Z=Z, charge_state=Z, ppc=1)
    w.update(ncs=False, brem=False, bw=False, bh=True, photon_capacity=1 << 16,
             pair_capacity=1 << 16)
    o = oracle.OracleSim(w, _tables(Z), nthreads=1, lib=lib)
    d = o.derived()
    dt = d["dt"]
    xc = 500.5 * d["dx"][0]                 # inside the slab (cells 480..543)
    eps = 37.0
    k = np.zeros((n, 3)); k[:, 2] = 1.0     # along z: never leaves its cell in 1D
    x = np.zeros((n, 3)); x[:, 0] = xc
    o.add_photons(x, k, np.full(n, eps), np.full(n, 1.0), 0x40000000 + np.arange(n, dtype=np.uint32))
    o.step(m + 1)
    conv = int((o.flight()["state"] == 2).sum())
    sig = integrate.quad(lambda u: TB.bh_dcs(u, eps, Z), 1 / eps, 1 - 1 / eps, epsabs=0,
                         epsrel=1e-11, limit=200)[0]
    nion = ne / Z
    X = d["K_BR"] * nion * sig * dt
    p = 1.0 - math.exp(-m * X)
    z = (conv - n * p) / math.sqrt(n * p * (1 - p))
    assert 0.05 < p < 0.95, p
    assert abs(z) < 4.0, (conv, n * p, z)
    return z


def _ks_against(samples, cdf_fn):
    return stats.kstest(samples, cdf_fn).statistic


def check_pair_shares(lib=None):
    """Breit-Wheeler electron shares at off-node chi, Bethe-Heitler positron
    shares at an off-node k, against the quadrature spectra."""
    w = _bw_w()
    o0 = oracle.OracleSim(w, _tables(13), nthreads=1, lib=lib)
    d = o0.derived()
    ES, x0 = d["E_S"], 0.5 * 1024 * d["dx"][0]
    o0.close()
    eps = 2400.0
    n_per = 6000
    o = _flight_sim(lib, w, _field_photons(n_per, eps, x0))
    o.step(400)
    pr = o.pairs()
    xi = pr["e_minus"] / (pr["e_minus"] + pr["e_plus"])
    grp = ((pr["parent"] - 0x40000000) // n_per).astype(int)
    chis = [eps * abs(E0 - B0) / ES, eps * (E0 + B0) / ES]
    ds = []
    for g, chi in enumerate(chis):
        s = np.sort(xi[grp == g])
        assert s.size > 2000, s.size
        grid = np.linspace(1e-6, 1 - 1e-6, 2001)
        f = TB.bw_bracket(chi, grid)
        cum = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(grid))])
        cum /= cum[-1]
        D = _ks_against(s, lambda v: np.interp(v, grid, cum))
        ds.append(D)
        assert D < 1.63 / math.sqrt(s.size) + 0.01, (chi, D)
    # Bethe-Heitler
    Z, k = 79, 37.0
    w = S.frozen_B_beam(B=0.0, ne=4e8, Z=Z, charge_state=Z, ppc=1)
    w.update(ncs=False, brem=False, bw=False, bh=True, photon_capacity=1 << 16, pair_capacity=1 << 16)
    o = oracle.OracleSim(w, _tables(Z), nthreads=1, lib=lib)
    dd = o.derived()
    n = 8000
    kk = np.zeros((n, 3)); kk[:, 2] = 1.0
    x = np.zeros((n, 3)); x[:, 0] = 500.5 * dd["dx"][0]
    o.add_photons(x, kk, np.full(n, k), np.full(n, 1.0), 0x40000000 + np.arange(n, dtype=np.uint32))
    o.step(200)
    pr = o.pairs()
    xp = np.sort(pr["e_plus"] / k)
    assert xp.size > 3000, xp.size
    grid = np.linspace(1 / k, 1 - 1 / k, 4001)
    f = TB.bh_dcs(grid, k, Z)
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(grid))])
    cum /= cum[-1]
    D = _ks_against(xp, lambda v: np.interp(v, grid, cum))
    ds.append(D)
    assert D < 1.63 / math.sqrt(xp.size) + 0.01, D
    return ds


def check_pair_kinematics(lib=None):
    w = _bw_w()
    o0 = oracle.OracleSim(w, _tables(13), nthreads=1, lib=lib)
    d = o0.derived()
    x0, dt = 0.5 * 1024 * d["dx"][0], d["dt"]
    o0.close()
    eps = np.array([2400.0, 900.0, 30.0, 1.5])
    n = 2000
    ph = _field_photons(n // 3 + 1, 1.0, x0)
    e = np.resize(eps, ph[0].shape[0])
    o = _flight_sim(lib, w, (ph[0], ph[1], e, ph[3], ph[4]))
    o.step(150)
    pr = o.pairs()
    assert pr["e_minus"].size > 100
    j = (pr["parent"] - 0x40000000).astype(int)
    eps_j = e[j]
    assert np.allclose(pr["e_minus"] + pr["e_plus"], eps_j, rtol=1e-14, atol=0)
    assert np.all(pr["e_minus"] >= 1.0) and np.all(pr["e_plus"] >= 1.0)
    travelled = (pr["step"].astype(np.int64) - pr["pstep"].astype(np.int64) - 1)
    want = x0 + ph[1][j, 0] * dt * travelled
    assert np.allclose(pr["x"][:, 0], want, rtol=0, atol=1e-9)
    assert np.array_equal(pr["k"], ph[1][j])
    # below 2 mc^2 nothing travels or converts
    f = o.flight()
    assert np.all(f["state"][e < 2.0] == 4)
    return int(pr["e_minus"].size)


def test_bw_table_asymptotes():
    print(check_bw_table_asymptotes())


def test_bh_table_limits():
    print(check_bh_table_limits())
    print(check_bh_table_limits(_tables(13), Z=13, A=26.9815385, X0=24.01))


def test_bw_conversion_follows_the_rate(oracle_lib):
    print(check_bw_conversion_law())


def test_bh_conversion_follows_eq4_with_the_pair_cross_section(oracle_lib):
    print(check_bh_conversion_law())


def test_pair_shares_follow_the_spectra(oracle_lib):
    print(check_pair_shares())


def test_pair_kinematics(oracle_lib):
    print(check_pair_kinematics())
