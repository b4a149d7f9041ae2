"""Pins of the oracle's mobile ions (the solid-target runs of Sec. III):

  push      ions at q/M in a uniform B turn by exactly 2 atan(q B dt / (2 gamma M))
            per step (the Boris rotation), at constant |p|;
  coupling  a cold two-species slab oscillates at the leapfrog form of
            w^2 = n_e + n_i q^2 / M (electron and ion plasma frequencies);
  deposit   charge continuity with both species moving;
  density   the n of Eq. (4) is the count of ions in the electron's cell times
            the ion weight over the cell volume: a 16-electron replay of the
            collision test against densities counted from the ion positions.

Each check takes the oracle library to run (None = the oracle itself).  CPU only."""
from __future__ import annotations

import math

import numpy as np

import oracle
import scenarios as S
import test_oracle_pins as P0
import test_oracle_pins_fields as PF


def _tables(Z):
    import conftest
    return conftest.oracle_tables(Z)


def check_ion_gyration(lib=None):
    q, M, B = 3.0, 40.0, 7.0
    w = S.base(name="ion-gyro", dims=1, n=[64], dx_lambda=[1 / 16], ppc=1, x0_lambda=1.0,
               thickness_lambda=1.0, frozen=True, frozen_kind=0, frozen_B=[0.0, 0.0, B],
               ncs=False, brem=False, charge_state=int(q), ion_ppc=2, ion_mass_me=M)
    o = oracle.OracleSim(w, _tables(13), nthreads=1, lib=lib)
    dt = o.derived()["dt"]
    x = o.ions()["x"]
    rng = np.random.default_rng(4)
    u = rng.uniform(0.01, 1.0, o.Ni)            # |p| / (M c): gyroradius < 2 c/w0, inside the box
    th0 = rng.uniform(0, 2 * math.pi, o.Ni)
    p = np.stack([u * np.cos(th0), u * np.sin(th0), np.zeros(o.Ni)], axis=1)
    o.set_ions(x, p)
    steps = 50
    o.step(steps)
    io = o.ions()
    assert io["alive"].all()
    pn = io["p"]
    g = np.sqrt(1 + u * u)
    turn = steps * 2 * np.arctan(q * B * dt / (2 * g * M))
    # positive charge in B along +z turns clockwise (dp/dt = q v x B)
    th = np.arctan2(pn[:, 1], pn[:, 0])
    err = np.abs(np.angle(np.exp(1j * (th - (th0 - turn)))))
    o.close()
    assert np.abs(np.linalg.norm(pn, axis=1) / u - 1).max() < 1e-13
    assert err.max() < 1e-11, err.max()
    return float(err.max())


def test_ion_gyration_is_the_boris_rotation(oracle_lib):
    print(check_ion_gyration())


def check_two_fluid_plasma_frequency(lib=None):
    """Electrons given a small drift in a cold slab with light mobile ions
    (q = 1, M = 25) oscillate at 2/dt asin(w dt/2), w^2 = n_e (1 + 1/M);
    with static ions at n_e alone (the 2% difference is 50 times the
    tolerance)."""
    out = []
    for M in (25.0, 0.0):
        w = S.base(name="plasma2", dims=1, n=[512], dx_lambda=[1 / 128], ppc=16, x0_lambda=1.0,
                   thickness_lambda=2.0, a0=0.0, ne_over_nc=4.0, ncs=False, brem=False,
                   charge_state=1, ion_ppc=16 if M else 0, ion_mass_me=M)
        o = oracle.OracleSim(w, _tables(13), nthreads=4, lib=lib)
        dt = o.derived()["dt"]
        e = o.electrons()
        p = np.zeros((o.N, 3))
        p[:, 0] = 1e-4
        o.set_electrons(e["x"], p, e["tau"])
        xs = e["x"][:, 0]
        mid = (xs > 1.6 * 2 * math.pi) & (xs < 2.4 * 2 * math.pi)
        ser = []
        for _ in range(300):
            o.step(1)
            ser.append(o.electrons()["p"][mid, 0].mean())
        o.close()
        s = np.array(ser)
        zc = np.nonzero(np.diff(np.sign(s)) != 0)[0]
        tz = [(k + s[k] / (s[k] - s[k + 1])) for k in zc]
        wm = 2 * math.pi / (2 * np.mean(np.diff(tz)) * dt)
        w2 = 4.0 * (1 + (1.0 / M if M else 0.0))
        want = 2 / dt * math.asin(math.sqrt(w2) * dt / 2)
        out.append((M, wm, want))
        assert abs(wm / want - 1) < 4e-4, (M, wm, want)
    return out


def test_two_fluid_plasma_frequency(oracle_lib):
    print(check_two_fluid_plasma_frequency())


def check_continuity_with_ions(lib=None):
    """2D, both species thermal (ions q = 2, M = 50, hotter per unit mass so
    that they move): div E - (rho - rho_0) with rho = rho_e + rho_i stays
    within the stated current-rounding bound."""
    w = S.base(name="thermal2", dims=2, n=[40, 32], dx_lambda=[1 / 32, 1 / 24], ppc=4,
               x0_lambda=0.3, thickness_lambda=0.6, a0=0.0, ncs=False, brem=False,
               ne_over_nc=20.0, seed=31, charge_state=2, ion_ppc=3, ion_mass_me=50.0)
    o = oracle.OracleSim(w, _tables(13), nthreads=8, lib=lib)
    L = PF.Layout(o, 2)
    rng = np.random.default_rng(5)
    e = o.electrons()
    o.set_electrons(e["x"], rng.normal(scale=0.08, size=(o.N, 3)), e["tau"])
    io = o.ions()
    o.set_ions(io["x"], rng.normal(scale=0.05, size=(o.Ni, 3)))
    wi = 20.0 / 2 * float(np.prod(L.dx[:2])) / 3       # n_i V / ion_ppc
    e0, i0 = o.electrons(), o.ions()
    o.step(30)
    e1, i1 = o.electrons(), o.ions()
    rho = lambda ee, ii: (PF._rho_nodes(L, ee["x"], ee["w"], ee["alive"])
                          - 2.0 * PF._rho_nodes(L, ii["x"], np.full(o.Ni, wi), ii["alive"]))
    res = np.abs(PF._div_E(L, o.fields()) - (rho(e1, i1) - rho(e0, i0)))
    sel = L.interior(4)
    bound = PF.current_rounding_bound(L, 30, 4 * (4 + 3))
    o.close()
    assert res[sel].max() <= bound, (res[sel].max(), bound)
    # the ions moved enough to matter: their charge density changed
    assert np.abs(rho(e0, i1) - rho(e0, i0))[sel].max() > 1e3 * bound
    return float(res[sel].max()), bound


def test_continuity_with_mobile_ions(oracle_lib):
    print(check_continuity_with_ions())


def check_brem_with_counted_ion_density(lib=None):
    """16 electrons at fixed energy in a dense target of mobile ions at rest
    (zero fields): each step's collision probability uses the ions counted
    in the electron's cell (3 per cell on average, Poisson-scattered)."""
    tab = _tables(79)
    i = 100
    Tk = math.exp(tab["ln_T0"] + i * tab["dln_T"])
    pm = math.sqrt(Tk * (Tk + 2))
    gam = math.sqrt(1 + pm * pm)
    q = 79
    ni = 0.03 / (P0._K_BR() * tab["sigma"][i] * (pm / gam) * 0.95 * 2 * math.pi)
    w = S.base(name="brem-16-ions", dims=1, n=[64], dx_lambda=[1.0], ppc=1, x0_lambda=0.0,
               thickness_lambda=16.0, frozen=True, frozen_kind=0, Z=79, charge_state=q,
               ne_over_nc=ni * q, ncs=False, brem=True, no_recoil=True, seed=17,
               ion_ppc=3, ion_mass_me=196.97 * 1822.888)
    o = oracle.OracleSim(w, tab, nthreads=1, lib=lib)
    assert o.N == 16 and o.Ni == 48
    d = o.derived()
    e = o.electrons()
    p = np.zeros((16, 3))
    p[:, 1] = pm
    o.set_electrons(e["x"], p, e["tau"])
    # ion positions -> counts per cell (the ions stay at rest in zero fields)
    dx = d["dx"][0]
    cnt = np.bincount(np.floor(o.ions()["x"][:, 0] / dx).astype(int), minlength=64)
    assert cnt.sum() == 48 and cnt.std() > 0
    M = 300
    o.step(M)
    wiv = ni / 3                                        # ion weight / cell volume
    key = (17, 0)
    want = []
    cell = np.floor(e["x"][:, 0] / dx).astype(int)
    for idv in range(16):
        X = d["K_BR"] * (cnt[cell[idv]] * wiv) * tab["sigma"][i] * (pm / gam) * d["dt"]
        P = -math.expm1(-X)
        for n in range(M):
            r = P0._philox_py((idv, n, 0, 0), key)
            k = r[0] * 2 ** 20 + (r[1] >> 12)
            if (k + 0.5) * 2.0 ** -52 < P:
                want.append((idv, n))
    ph = o.photons()
    got = sorted(zip(ph["parent"].tolist(), ph["step"].tolist()))
    o.close()
    assert len(want) > 50
    assert got == sorted(want)
    return len(want)


def test_brem_uses_the_counted_ion_density(oracle_lib):
    print(check_brem_with_counted_ion_density())
