"""Pins of the FP64 oracle to values fixed outside it: published known answers,
closed forms, textbook limits, exact distributions of the Monte-Carlo steps
and conservation laws.  CPU only."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
from scipy import stats
from scipy.integrate import quad
from scipy.special import gamma as Gamma
from scipy.special import kv

import oracle
import scenarios as S
from oracle import tables as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALPHA = 7.2973525693e-3
N_A = 6.02214076e23
RE_CM = 2.8179403262e-13


# --------------------------------------------------------------------- Philox
def test_philox_known_answers(oracle_lib):
    """Philox4x32-10 (Salmon et al., SC'11) on the published known-answer set."""
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        assert list(oracle.philox(v[0:4], v[4:6])) == v[6:10]


def test_philox_counter_sensitivity(oracle_lib):
    """Each counter or key bit changes about half of the 128 output bits."""
    base = oracle.philox([1, 2, 3, 4], [5, 6])
    flips = []
    for word in range(6):
        for bit in (0, 13, 31):
            ctr, key = [1, 2, 3, 4], [5, 6]
            if word < 4:
                ctr[word] ^= 1 << bit
            else:
                key[word - 4] ^= 1 << bit
            out = oracle.philox(ctr, key)
            flips.append(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, out)))
    assert 50 < np.mean(flips) < 78


# ----------------------------------------------------------------- NCS tables
def test_ncs_classical_limit_rate_and_power():
    """eta -> 0: h -> Gamma(1/6) Gamma(11/6) = 5 pi / 3 (classical photon number)
    and g -> 1 (Larmor power)."""
    h, g = T.ncs_h_g(1e-8)
    assert abs(h / (Gamma(1 / 6) * Gamma(11 / 6)) - 1) < 1e-6
    assert abs(g - 1) < 1e-6


def test_ncs_quantum_power_fit():
    """g(eta) against the published fit [1 + 4.8(1+eta) ln(1+1.7 eta) + 2.44 eta^2]^(-2/3)."""
    for eta in (0.01, 0.1, 1.0, 10.0):
        _, g = T.ncs_h_g(eta)
        fit = (1 + 4.8 * (1 + eta) * math.log(1 + 1.7 * eta) + 2.44 * eta ** 2) ** (-2 / 3)
        assert abs(g / fit - 1) < 0.03, (eta, g, fit)


def test_ncs_h_decreases_and_g_below_one(tables_al):
    h = tables_al["h"]
    assert np.all(np.diff(h) < 0)
    assert h[0] < 5 * math.pi / 3 and h[0] > 5 * math.pi / 3 * (1 - 3e-4)


def test_int_k53_against_library():
    """int_y^inf K_{5/3} from the cosh representation vs quadrature of scipy's K."""
    for y in (1e-3, 0.1, 1.0, 5.0, 30.0):
        # K decays like exp(-t): a finite range of 80 is exact in double
        ref = quad(lambda t: kv(5 / 3, t), y, y + 80.0, epsrel=1e-14, limit=400)[0]
        assert abs(T.int_k53(np.array([y]))[0] / ref - 1) < 1e-10


def test_ncs_spectrum_classical_shape(tables_al):
    """The first CDF row (eta = 1e-4) is the classical synchrotron number
    spectrum in x = xi/(1.5 eta): CDF(x) = (3/(5 pi)) int_0^x int_t^inf K_{5/3}."""
    eta = math.exp(tables_al["ln_eta0"])
    lnxi = tables_al["ln_xi"]
    row = tables_al["ncs_cdf"][0]
    norm = 5 * math.pi / 3
    for j in range(0, 256, 1):
        xi = math.exp(lnxi[j])
        x = xi / (1.5 * eta)
        if not (0.01 < x < 5.0):
            continue
        ref = quad(lambda t: T.int_k53(np.array([t]))[0], 0, x, limit=200)[0] / norm
        # quantum corrections are O(eta) = 1e-4
        assert abs(row[j] - ref) < 5e-4, (x, row[j], ref)


def test_ncs_mean_fraction_classical():
    """<xi> = (4/(5 sqrt 3)) eta in the classical limit (mean synchrotron photon
    energy (8/(15 sqrt 3)) eps_c with eps_c = 1.5 eta gamma)."""
    eta = 1e-6
    h, g = T.ncs_h_g(eta)
    mean = 4 * math.pi * eta * g / (3 * math.sqrt(3) * h)
    assert abs(mean / (4 * eta / (5 * math.sqrt(3))) - 1) < 1e-5


# ----------------------------------------------------------------- Brem (Tsai)
def test_tsai_complete_screening_reproduces_pdg_x0():
    """Eq. (1) at complete screening (E -> infinity): int_0^1 y dsigma/dy dy
    without the (Z^2+Z)/9 (1-y) term is 4 alpha r_e^2 [Z^2(L_rad - f) + Z L'_rad],
    the radiation length tabulated by the PDG."""
    for line in open(os.path.join(GOLDEN, "radiation_length_pdg.txt")):
        if line.startswith("#") or not line.strip():
            continue
        Z, A, X0, tol = line.split()
        Z, A, X0, tol = int(Z), float(A), float(X0), float(tol)
        E = 1e9  # mc^2: screening parameters -> 0
        val = quad(lambda y: T.tsai_bracket(np.array([y]), E, Z)[0], 0.0, 1.0 - 1e-9,
                   limit=400, epsrel=1e-12)[0]
        val -= (2.0 / 9.0) * (Z * Z + Z)  # int_0^1 (2/3)(1-y)(2/3)(Z^2+Z) dy
        x0 = A / (N_A * ALPHA * RE_CM ** 2 * val)
        assert abs(x0 / X0 - 1) < tol, (Z, x0, X0)


def test_tsai_unscreened_bethe_heitler_limit():
    """Without screening (gamma, eps large) phi1 - 4/3 ln Z and psi1 - 8/3 ln Z
    both tend to the unscreened Bethe-Heitler value 4 ln(2 E E'/(m k)) - 2,
    where gamma = 100 m k/(E E' Z^(1/3)) and eps = 100 m k/(E E' Z^(2/3))."""
    for Z in (13, 79):
        for E, k in ((3.0, 1.5), (40.0, 39.0)):
            Ep = E - k
            # scale the ratio k/(E E') by 1e3 so that screening is negligible
            s_ = 1e3
            gs = 100 * k * s_ / (E * Ep * Z ** (1 / 3))
            es = 100 * k * s_ / (E * Ep * Z ** (2 / 3))
            phi1, _, psi1, _ = T.screening(np.array([gs]), np.array([es]))
            rhs = 4 * math.log(2 * E * Ep / (k * s_)) - 2
            assert abs(phi1[0] - 4 / 3 * math.log(Z) - rhs) < 2e-3, (Z, E, phi1[0], rhs)
            assert abs(psi1[0] - 8 / 3 * math.log(Z) - rhs) < 2e-3, (Z, E, psi1[0], rhs)


def test_tsai_complete_screening_constants():
    """gamma = eps = 0: phi1 = 20.863, phi1 - phi2 = 2/3, psi1 = 28.340, psi1 - psi2 = 2/3;
    4 L_rad = 4 ln 184.15 and 4 L'_rad = 4 ln 1194 to the printed digits."""
    phi1, phi2, psi1, psi2 = T.screening(np.array([0.0]), np.array([0.0]))
    assert abs(phi1[0] - 4 * math.log(184.15)) < 2e-3
    assert abs(psi1[0] - 4 * math.log(1194.0)) < 2e-3
    assert abs(phi1[0] - phi2[0] - 2 / 3) < 1e-12
    assert abs(psi1[0] - psi2[0] - 2 / 3) < 1e-12


def test_brem_sigma_scales_as_z2(tables_al, tables_au):
    """sigma ~ alpha r_e^2 Z^2 (Sec. II.A): at high energy the Au/Al ratio is
    Z^2 times the ratio of the screened logarithms, between (79/13)^2 / 2 and
    (79/13)^2 * 1.1."""
    r = tables_au["sigma"][-1] / tables_al["sigma"][-1]
    assert 0.5 * (79 / 13) ** 2 < r < 1.1 * (79 / 13) ** 2


def test_brem_tables_monotone(tables_al, tables_au):
    for t in (tables_al, tables_au):
        assert np.all(np.diff(t["br_cdf"], axis=1) >= 0)
        assert np.all(t["br_cdf"][:, 0] == 0) and np.all(t["br_cdf"][:, -1] == 1)
        assert np.all(np.diff(t["ncs_cdf"], axis=1) >= 0)
        pos = t["sigma"] > 0
        assert np.all(np.diff(t["sigma"][pos]) > 0)


# ------------------------------------------------------------- step: pusher
def _frozen(**kw):
    w = S.frozen_B_beam(**kw)
    w["ncs"] = False
    w["brem"] = False
    return w


def test_boris_pure_B_rotation(oracle_lib, tables_al):
    """Uniform B only: |p| is conserved and the momentum turns by exactly
    2 atan(B dt / (2 gamma)) per step (Boris rotation)."""
    w = _frozen(n_cells=4096, ppc=1, slab=(2016, 2080), B=3.0)
    o = oracle.OracleSim(w, tables_al)
    e = o.electrons()
    p = np.zeros((o.N, 3))
    p[:, 0] = np.linspace(0.1, 50.0, o.N)
    x = e["x"].copy()
    x[:, 0] = 2048 * o.derived()["dx"][0]   # gyro-radius p/B <= 17 << half box
    o.set_electrons(x, p, e["tau"])
    n = 500
    dt = o.derived()["dt"]
    o.step(n)
    q = o.electrons()["p"]
    assert np.allclose(np.linalg.norm(q, axis=1), p[:, 0], rtol=1e-13, atol=0)
    gam = np.sqrt(1 + p[:, 0] ** 2)
    theta = n * 2 * np.arctan(3.0 * dt / (2 * gam))
    # the rotation angle (its sense is set by the charge) from the x component
    assert np.allclose(q[:, 0] / p[:, 0], np.cos(theta), atol=1e-9)


def test_boris_pure_E_exact(oracle_lib, tables_al):
    """Uniform E only: p(t) = p0 - E t exactly (q = -1)."""
    w = _frozen(n_cells=64, ppc=1, slab=(0, 64), B=0.0)
    w["frozen_E"] = [0.5, -0.25, 0.125]
    o = oracle.OracleSim(w, tables_al)
    dt = o.derived()["dt"]
    o.step(7)
    q = o.electrons()["p"]
    assert np.allclose(q, -7 * dt * np.array([0.5, -0.25, 0.125]), rtol=1e-14, atol=1e-15)


def _plane_wave_error(dx_lambda, a=5.0, steps_per_unit=None):
    w = S.frozen_plane_wave(a=a)
    w["ncs"] = False
    w["brem"] = False
    w["dx_lambda"] = [dx_lambda]
    w["n"] = [int(round(40 / dx_lambda))]
    w["ppc"] = 1
    w["x0_lambda"] = 1.0
    w["thickness_lambda"] = dx_lambda * 8
    o = oracle.OracleSim(w, oracle_tables_al())
    dt = o.derived()["dt"]
    nsteps = int(round(6 * 2 * math.pi / dt))  # six laser periods
    o.step(nsteps)
    e = o.electrons()
    p, x = e["p"], e["x"][:, 0]
    gam = np.sqrt(1 + (p ** 2).sum(axis=1))
    # invariant of the exact orbit: gamma - p_x = 1
    return np.abs(gam - p[:, 0] - 1).max(), np.abs(p[:, 0] - 0.5 * (p[:, 1] ** 2 + p[:, 2] ** 2) * 1.0
                                                    + 0.0 * gam).max()


def oracle_tables_al():
    import conftest
    return conftest.oracle_tables(13)


def test_plane_wave_orbit_invariants_second_order(oracle_lib):
    """Plane wave E_y = B_z = a sin(t - x): the exact orbit keeps gamma - p_x = 1
    and p_x = p_perp^2 / 2; the Boris error in these falls like dt^2."""
    e1, _ = _plane_wave_error(1 / 32)
    e2, _ = _plane_wave_error(1 / 64)
    e3, _ = _plane_wave_error(1 / 128)
    assert e1 < 0.05
    r12, r23 = e1 / e2, e2 / e3
    assert 3.0 < r12 < 5.0 and 3.0 < r23 < 5.0, (e1, e2, e3)


def test_plane_wave_transverse_momentum(oracle_lib):
    """p_y = a (cos phi - 1) with phi = t - x along the orbit (electron at rest
    before the wave front)."""
    w = S.frozen_plane_wave(a=2.0)
    w["ncs"] = False
    w["brem"] = False
    w["ppc"] = 2
    o = oracle.OracleSim(w, oracle_tables_al())
    dt = o.derived()["dt"]
    n = 400
    o.step(n)
    e = o.electrons()
    x, p = e["x"][:, 0], e["p"]
    # p^{n-1/2} belongs to t_{n-1/2}; position at t_{n-1/2} ~ x^n - v dt/2
    gam = np.sqrt(1 + (p ** 2).sum(axis=1))
    xh = x - 0.5 * dt * p[:, 0] / gam
    phi = (n - 0.5) * dt - xh
    ref = np.where(phi > 0, 2.0 * (np.cos(phi) - 1), 0.0)
    assert np.abs(p[:, 1] - ref).max() < 2e-3


# ---------------------------------------------------------- step: emission MC
def _ncs_rate_case(eta_target, B=100.0, gamma_target=1000.0):
    """Electrons perpendicular to a uniform B: eta = |p| B / E_S, constant."""
    w = S.frozen_B_beam(n_cells=256, ppc=16, slab=(112, 144), B=B)
    w["brem"] = False
    w["no_recoil"] = True
    return w


def test_ncs_event_counts_are_binomial(oracle_lib, tables_al):
    """Optical-depth emission with a fresh tau after each event and a constant
    rate R: each step emits with probability 1 - exp(-R dt), independently, so
    the per-electron count over M steps is Binomial(M, 1 - exp(-R dt)), with
    R = (sqrt 3/(2 pi)) alpha (m c^2/hbar w0) (eta/gamma) h(eta)."""
    B = 200.0
    w = _ncs_rate_case(0.0, B=B)
    o = oracle.OracleSim(w, tables_al)
    d = o.derived()
    pmag = 600.0
    e = o.electrons()
    p = np.zeros((o.N, 3))
    p[:, 0] = pmag
    o.set_electrons(e["x"], p, e["tau"])
    M = 400
    o.step(M)
    st = o.stats()
    eta = pmag * B / d["E_S"]
    gam = math.sqrt(1 + pmag ** 2)
    h, _ = T.ncs_h_g(eta)
    lam = 7.2973525693e-3
    E_S = 1e-6 / (2 * math.pi * 3.8615926796e-13)
    R = math.sqrt(3) / (2 * math.pi) * lam * E_S * eta / gam * h
    pe = 1 - math.exp(-R * d["dt"])
    n = o.N * M
    mean, sd = n * pe, math.sqrt(n * pe * (1 - pe))
    assert abs(st["events"][0] - mean) < 4 * sd + 2e-3 * mean, (st["events"][0], mean, sd)
    # per-electron counts: dispersion of a binomial
    ph = o.photons()
    counts = np.bincount(ph["parent"], minlength=o.N)
    assert abs(counts.var() / (M * pe * (1 - pe)) - 1) < 0.25


def test_ncs_photon_spectrum_classical(oracle_lib, tables_al):
    """At small eta the drawn photon fraction follows the classical
    synchrotron number spectrum: <xi> = (4/(5 sqrt 3)) eta (1 + O(eta)) and the
    distribution of x = xi/(1.5 eta) is (3/(5 pi)) int_x^inf K_{5/3}."""
    pmag, eta_target = 20.0, 2e-3
    w = _ncs_rate_case(0.0, B=1.0)
    o0 = oracle.OracleSim(w, tables_al)
    B = eta_target * o0.derived()["E_S"] / pmag     # gyro-radius p/B ~ 0.5 c/w0
    o0.close()
    w = _ncs_rate_case(0.0, B=B)
    w["photon_cut_mc2"] = 0.0
    o = oracle.OracleSim(w, tables_al)
    d = o.derived()
    e = o.electrons()
    p = np.zeros((o.N, 3))
    p[:, 0] = pmag
    o.set_electrons(e["x"], p, e["tau"])
    o.step(3000)
    assert o.stats()["live"] == o.N
    ph = o.photons()
    gam = math.sqrt(1 + pmag ** 2)
    eta = pmag * B / d["E_S"]
    xi = ph["energy"] / gam
    assert len(xi) > 10000
    m = xi.mean() / (4 * eta / (5 * math.sqrt(3)))
    assert abs(m - 1) < 4 * xi.std() / xi.mean() / math.sqrt(len(xi)) + 2 * eta, m
    x = xi / (1.5 * eta)
    xs = np.sort(x)
    grid = np.geomspace(0.003, 8, 60)
    cdf = np.array([quad(lambda t: T.int_k53(np.array([t]))[0], 0, g, limit=200)[0] for g in grid])
    cdf /= 5 * math.pi / 3
    emp = np.searchsorted(xs, grid) / len(xs)
    assert np.abs(emp - cdf).max() < 1.8 / math.sqrt(len(xs)) + 2 * eta


def _brem_case(Z, q, ne, T_kin, nT_cells=4096):
    """Zero fields, electrons along +x through a uniform slab filling the box."""
    w = S.base(name="brem-thick", dims=1, n=[nT_cells], dx_lambda=[1.0], ppc=1,
               x0_lambda=0.0, thickness_lambda=float(nT_cells), frozen=True, frozen_kind=0,
               Z=Z, charge_state=q, ne_over_nc=ne, ncs=False, brem=True)
    return w


def test_brem_event_counts_binomial(oracle_lib, tables_au):
    """Eq. (4): with the energy fixed (no recoil) each step is an independent
    trial with P = 1 - exp(-n sigma(E) v dt); the total count over M steps of N
    electrons is Binomial(N M, P).  sigma at a table node is the tabulated
    integral of Eq. (1)."""
    i = 110
    Tk = math.exp(tables_au["ln_T0"] + i * tables_au["dln_T"])
    w = _brem_case(79, 79, 7900.0, Tk)
    w["no_recoil"] = True
    o = oracle.OracleSim(w, tables_au)
    d = o.derived()
    e = o.electrons()
    p = np.zeros((o.N, 3))
    pm = math.sqrt(Tk * (Tk + 2))
    p[:, 0] = pm
    x = e["x"].copy()
    x[:, 0] = 0.5 * d["dx"][0] * (np.arange(o.N) % 64 + 0.5)
    o.set_electrons(x, p, e["tau"])
    M = 2000
    o.step(M)
    st = o.stats()
    gam = math.sqrt(1 + pm * pm)
    v = pm / gam
    ni = 7900.0 / 79
    X = d["K_BR"] * ni * tables_au["sigma"][i] * v * d["dt"]
    P = -math.expm1(-X)
    n = o.N * M
    mean, sd = n * P, math.sqrt(n * P * (1 - P))
    assert abs(st["events"][1] - mean) < 4 * sd + 1e-4 * mean, (st["events"][1], mean, sd)


def test_brem_photon_energies_follow_tsai(oracle_lib, tables_au):
    """Photon energies drawn at a table node follow sigma(k, E)/sigma(E) of
    Eq. (1) (KS test against the direct integral of the Tsai bracket)."""
    i = 100
    Tk = math.exp(tables_au["ln_T0"] + i * tables_au["dln_T"])
    w = _brem_case(79, 79, 7900.0, Tk)
    w["no_recoil"] = True
    o = oracle.OracleSim(w, tables_au)
    e = o.electrons()
    p = np.zeros((o.N, 3))
    p[:, 0] = math.sqrt(Tk * (Tk + 2))
    x = e["x"].copy()
    x[:, 0] = 0.5 * o.derived()["dx"][0] * (np.arange(o.N) % 64 + 0.5)
    o.set_electrons(x, p, e["tau"])
    o.step(1500)
    k = o.photons()["energy"]
    assert len(k) > 3000
    E = Tk + 1.0
    kc = tables_au["k_cut"]
    tot = quad(lambda lk: T.tsai_bracket(np.array([math.exp(lk) / E]), E, 79)[0],
               math.log(kc), math.log(Tk), limit=400, epsrel=1e-11)[0]

    def cdf(kk):
        kk = np.atleast_1d(kk)
        return np.array([quad(lambda lk: T.tsai_bracket(np.array([math.exp(lk) / E]), E, 79)[0],
                              math.log(kc), math.log(v), limit=200, epsrel=1e-10)[0] / tot
                         for v in kk])
    ks = stats.kstest(k, lambda v: cdf(np.clip(v, kc, Tk)))
    assert ks.pvalue > 1e-3, ks
    assert k.min() >= kc and k.max() <= Tk


def test_recoil_conserves_energy(oracle_lib, tables_au):
    """Zero fields: the electrons' kinetic-energy loss equals the radiated
    energy (kept + dropped) to rounding (energy-conserving recoil)."""
    i = 100
    Tk = math.exp(tables_au["ln_T0"] + i * tables_au["dln_T"])
    w = _brem_case(79, 79, 7900.0, Tk)
    o = oracle.OracleSim(w, tables_au)
    e = o.electrons()
    p = np.zeros((o.N, 3))
    p[:, 0] = math.sqrt(Tk * (Tk + 2))
    x = e["x"].copy()
    x[:, 0] = 0.5 * o.derived()["dx"][0] * (np.arange(o.N) % 64 + 0.5)
    o.set_electrons(x, p, e["tau"])
    ke0 = o.kinetic_energy()
    o.step(1000)
    st = o.stats()
    rad = st["e_rad_kept"][0] + st["e_rad_kept"][1] + st["e_rad_dropped"]
    assert st["events"][1] > 100
    assert abs((ke0 - o.kinetic_energy()) - rad) <= 1e-10 * ke0


# ------------------------------------------------------------ full PIC pins
def test_vacuum_wave_amplitude_and_speed(oracle_lib, tables_al):
    """No plasma: the current-sheet source launches E_y = a0 env sin(t - (x - x_s))
    to the right at the Yee phase speed (within 1% of a0 at lambda/128)."""
    w = S.c1_parity(0)
    w["ne_over_nc"] = 0.0
    w["thickness_lambda"] = 0.0
    w["a0"] = 1.0
    o = oracle.OracleSim(w, tables_al)
    d = o.derived()
    dx, dt = d["dx"][0], d["dt"]
    n = 800
    o.step(n)
    F = o.fields()
    Ey = F[1]
    i = np.arange(len(Ey)) - 2
    x = i * dx
    xs = 4 * dx
    t = n * dt - 0.5 * dt   # source phase of the last half step
    tl = 10 * 2 * math.pi
    tau = (n * dt) - (x - xs)
    env = np.where((tau > 0) & (tau < tl), np.sin(math.pi * tau / tl) ** 2, 0.0)
    ref = env * np.sin(tau)
    sel = (i > 10) & (i < 1000)
    assert np.abs(Ey[sel] - ref[sel]).max() < 0.01
    assert t > 0


def test_charge_conservation_gauss_law(oracle_lib, tables_al):
    """With the charge-conserving deposit, d(div E)/dt = -div J = d rho_e/dt:
    div E(t) - rho_e(t) stays at its initial value (0) on every node."""
    w = S.c1_parity(0)
    o = oracle.OracleSim(w, tables_al)
    d = o.derived()
    dx = d["dx"][0]
    e0 = o.electrons()
    o.step(300)
    e1 = o.electrons()
    F = o.fields()
    Ex = F[0]
    nn = len(Ex)

    def rho(x, wt, alive):
        r = np.zeros(nn)
        g = x[alive, 0] / dx
        i = np.floor(g).astype(int)
        f = g - i
        np.add.at(r, i + 2, -(1 - f) * wt[alive] / dx)
        np.add.at(r, i + 3, -f * wt[alive] / dx)
        return r
    r0 = rho(e0["x"], e0["w"], e0["alive"])
    r1 = rho(e1["x"], e1["w"], e1["alive"])
    div = np.zeros(nn)
    div[1:] = (Ex[1:] - Ex[:-1]) / dx   # node i sits between faces i-1/2 and i+1/2
    sel = slice(40, 900)
    assert e1["alive"].all()
    assert np.abs(div[sel] - (r1[sel] - r0[sel])).max() < 1e-9 * np.abs(r0).max()


def test_cold_plasma_oscillation_frequency(oracle_lib, tables_al):
    """A thick slab given a uniform velocity oscillates at the plasma
    frequency; for the leapfrog scheme sin(w dt/2) = w_p dt/2, w_p^2 = n_e."""
    w = S.base(name="plasma", dims=1, n=[512], dx_lambda=[1 / 128], ppc=16, x0_lambda=1.0,
               thickness_lambda=2.0, a0=0.0, ne_over_nc=4.0, ncs=False, brem=False)
    o = oracle.OracleSim(w, tables_al)
    d = o.derived()
    dt = d["dt"]
    e = o.electrons()
    p = np.zeros((o.N, 3))
    p[:, 0] = 1e-4
    o.set_electrons(e["x"], p, e["tau"])
    xs = e["x"][:, 0]
    mid = (xs > 1.6 * 2 * math.pi) & (xs < 2.4 * 2 * math.pi)
    series = []
    for _ in range(200):
        o.step(1)
        series.append(o.electrons()["p"][mid, 0].mean())
    s = np.array(series)
    zc = np.nonzero(np.diff(np.sign(s)) != 0)[0]
    # linear interpolation of zero crossings
    tz = [(k + s[k] / (s[k] - s[k + 1])) for k in zc]
    period_steps = 2 * np.mean(np.diff(tz))
    w_meas = 2 * math.pi / (period_steps * dt)
    wp = math.sqrt(4.0)
    w_leap = 2 / dt * math.asin(wp * dt / 2)
    assert abs(w_meas / w_leap - 1) < 5e-3, (w_meas, w_leap)


# ----------------------------------------------- 16-particle brute force (MC)
# An independent Philox4x32-10 (Salmon et al., SC'11) in plain Python, checked
# against the published known answers, drives a step-by-step replay of the
# emission decisions of 16 electrons; the oracle's event lists must equal the
# replay exactly.
_PH_M = (0xD2511F53, 0xCD9E8D57)
_PH_W = (0x9E3779B9, 0xBB67AE85)


def _philox_py(ctr, key):
    c = [int(v) & 0xFFFFFFFF for v in ctr]
    k = [int(v) & 0xFFFFFFFF for v in key]
    for _ in range(10):
        p0 = _PH_M[0] * c[0]
        p1 = _PH_M[1] * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k[0]) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k[1]) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
        k = [(k[0] + _PH_W[0]) & 0xFFFFFFFF, (k[1] + _PH_W[1]) & 0xFFFFFFFF]
    return c


def _u32(r):
    return (r + 0.5) * 2.0 ** -32


def test_python_philox_matches_known_answers():
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        assert _philox_py(v[0:4], v[4:6]) == v[6:10]


def _E_S():
    return 1e-6 / (2 * math.pi * 3.8615926796e-13)


def _K_BR():
    eps0, me, e, c = 8.8541878128e-12, 9.1093837015e-31, 1.602176634e-19, 299792458.0
    lam = 1e-6
    n_c = eps0 * me * (2 * math.pi * c / lam) ** 2 / e ** 2
    return n_c * (lam / (2 * math.pi)) * ALPHA * (RE_CM * 1e-2) ** 2


def test_ncs_events_16_electrons_brute_force(oracle_lib, tables_al):
    """16 electrons gyrating in a uniform B (no recoil, no brem): eta and gamma
    are constant, so each step lowers tau by K_N (eta/gamma) h(eta) dt; an
    event when tau <= 0, then tau = -ln u(r3 of the step's counter).  Replayed
    independently with eta at a table node."""
    i_eta = 170
    eta = math.exp(tables_al["ln_eta0"] + i_eta * tables_al["dln_eta"])
    pm = 600.0
    B = eta * _E_S() / pm
    w = S.frozen_B_beam(n_cells=256, ppc=16, slab=(128, 129), B=B, seed=11)
    w.update(brem=False, no_recoil=True, photon_cut_mc2=0.0)
    o = oracle.OracleSim(w, tables_al)
    assert o.N == 16
    d = o.derived()
    assert abs(d["E_S"] / _E_S() - 1) < 1e-14
    e = o.electrons()
    p = np.zeros((16, 3))
    p[:, 0] = pm
    o.set_electrons(e["x"], p, e["tau"])
    M = 300
    o.step(M)
    gam = math.sqrt(1 + pm * pm)
    K_N = math.sqrt(3) / (2 * math.pi) * ALPHA * _E_S()
    dtau = K_N * eta / gam * tables_al["h"][i_eta] * d["dt"]
    key = (11, 0)
    want = []
    for idv in range(16):
        tau = -math.log(_u32(_philox_py((idv, 0xFFFFFFFF, 0, 0), key)[3]))
        assert abs(tau - e["tau"][idv]) <= 1e-15 * tau
        for n in range(M):
            tau -= dtau
            if tau <= 0.0:
                want.append((idv, n))
                tau = -math.log(_u32(_philox_py((idv, n, 0, 0), key)[3]))
    ph = o.photons()
    got = sorted(zip(ph["parent"].tolist(), ph["step"].tolist()))
    assert len(want) > 100
    assert got == sorted(want)


def test_brem_events_16_electrons_brute_force(oracle_lib, tables_au):
    """16 electrons at fixed energy (no recoil, zero fields, NCS off) in a
    dense static target: Eq. (4) per step with P = -expm1(-K_BR n_i sigma v dt)
    and the 52-bit uniform of (r0, r1).  Replayed independently at a table
    node of sigma."""
    i = 100
    Tk = math.exp(tables_au["ln_T0"] + i * tables_au["dln_T"])
    pm = math.sqrt(Tk * (Tk + 2))
    q = 79
    gam = math.sqrt(1 + pm * pm)
    # ion density for X = 0.05 per step (dt = 0.95 dx, dx = 2 pi c/w0)
    ni = 0.05 / (_K_BR() * tables_au["sigma"][i] * (pm / gam) * 0.95 * 2 * math.pi)
    w = S.base(name="brem-16", dims=1, n=[64], dx_lambda=[1.0], ppc=1, x0_lambda=0.0,
               thickness_lambda=16.0, frozen=True, frozen_kind=0, Z=79, charge_state=q,
               ne_over_nc=ni * q, ncs=False, brem=True, no_recoil=True, seed=13)
    o = oracle.OracleSim(w, tables_au)
    assert o.N == 16
    d = o.derived()
    assert abs(d["K_BR"] / _K_BR() - 1) < 1e-9
    e = o.electrons()
    p = np.zeros((16, 3))
    p[:, 1] = pm                     # along y: the 1D cell does not change
    o.set_electrons(e["x"], p, e["tau"])
    M = 300
    o.step(M)
    X = d["K_BR"] * ni * tables_au["sigma"][i] * (pm / gam) * d["dt"]
    P = -math.expm1(-X)
    assert 0.01 < P < 0.2
    key = (13, 0)
    want = []
    for idv in range(16):
        for n in range(M):
            r = _philox_py((idv, n, 0, 0), key)
            k = r[0] * 2 ** 20 + (r[1] >> 12)
            if (k + 0.5) * 2.0 ** -52 < P:
                want.append((idv, n))
    ph = o.photons()
    got = sorted(zip(ph["parent"].tolist(), ph["step"].tolist()))
    assert len(want) > 100
    assert got == sorted(want)


# ------------------------------------------------ free-path bremsstrahlung
def test_brem_freepath_16_electrons_brute_force(oracle_lib, tables_au):
    """Free-path form of Eq. (4): each electron carries the number of mean free
    paths to its next collision, tau_b = -ln u (word 0 of counter
    (id, 0xFFFFFFFF, 1, 0) at load); every step uses up X = K_BR n_i sigma v dt
    of it; a collision when tau_b <= 0, then tau_b = -ln u (word 1 of the
    event's energy-draw counter (id, n, 1, 0)).  Replayed independently at a
    table node of sigma with the pinned Python Philox."""
    i = 100
    Tk = math.exp(tables_au["ln_T0"] + i * tables_au["dln_T"])
    pm = math.sqrt(Tk * (Tk + 2))
    q = 79
    gam = math.sqrt(1 + pm * pm)
    ni = 0.05 / (_K_BR() * tables_au["sigma"][i] * (pm / gam) * 0.95 * 2 * math.pi)
    w = S.base(name="brem-16-fp", dims=1, n=[64], dx_lambda=[1.0], ppc=1, x0_lambda=0.0,
               thickness_lambda=16.0, frozen=True, frozen_kind=0, Z=79, charge_state=q,
               ne_over_nc=ni * q, ncs=False, brem=True, no_recoil=True, seed=13,
               brem_freepath=True)
    o = oracle.OracleSim(w, tables_au)
    assert o.N == 16
    d = o.derived()
    e = o.electrons()
    key = (13, 0)
    tb0 = o.tau_brem()
    for idv in range(16):
        want0 = -math.log(_u32(_philox_py((idv, 0xFFFFFFFF, 1, 0), key)[0]))
        # the oracle's own log series is within 3 ulp of the platform log
        assert abs(tb0[idv] - want0) <= 4 * np.spacing(want0)
    p = np.zeros((16, 3))
    p[:, 1] = pm
    o.set_electrons(e["x"], p, e["tau"])
    M = 300
    o.step(M)
    X = d["K_BR"] * ni * tables_au["sigma"][i] * (pm / gam) * d["dt"]
    assert 0.01 < X < 0.2
    want, tb_end = [], []
    for idv in range(16):
        tb = float(tb0[idv])
        for n in range(M):
            tb -= X
            if tb <= 0.0:
                want.append((idv, n))
                tb = -math.log(_u32(_philox_py((idv, n, 1, 0), key)[1]))
        tb_end.append(tb)
    ph = o.photons()
    got = sorted(zip(ph["parent"].tolist(), ph["step"].tolist()))
    assert len(want) > 100
    assert got == sorted(want)
    np.testing.assert_allclose(o.tau_brem(), tb_end, rtol=0, atol=1e-9)
    # mean number of steps between collisions: 1 / P with P = 1 - exp(-X)
    P = -math.expm1(-X)
    assert abs(len(want) / (16 * M) - P) < 4 * math.sqrt(P * (1 - P) / (16 * M))


def test_brem_freepath_event_counts_binomial(oracle_lib, tables_au):
    """With the energy fixed, the steps between collisions of the free-path
    form are geometric with P = 1 - exp(-X) (the exponential free path cut into
    steps), so the count over M steps of N electrons is Binomial(N M, P): the
    same law as the per-step trial of Eq. (4)."""
    i = 110
    Tk = math.exp(tables_au["ln_T0"] + i * tables_au["dln_T"])
    w = _brem_case(79, 79, 7900.0, Tk)
    w.update(no_recoil=True, brem_freepath=True)
    o = oracle.OracleSim(w, tables_au)
    d = o.derived()
    e = o.electrons()
    p = np.zeros((o.N, 3))
    pm = math.sqrt(Tk * (Tk + 2))
    p[:, 0] = pm
    x = e["x"].copy()
    x[:, 0] = 0.5 * d["dx"][0] * (np.arange(o.N) % 64 + 0.5)
    o.set_electrons(x, p, e["tau"])
    M = 2000
    o.step(M)
    st = o.stats()
    gam = math.sqrt(1 + pm * pm)
    X = d["K_BR"] * (7900.0 / 79) * tables_au["sigma"][i] * (pm / gam) * d["dt"]
    P = -math.expm1(-X)
    n = o.N * M
    mean, sd = n * P, math.sqrt(n * P * (1 - P))
    assert abs(st["events"][1] - mean) < 4 * sd + 1e-4 * mean, (st["events"][1], mean, sd)
    # and the first-collision step k (1-based) is geometric, truncated at M:
    # randomised probability-integral transform of k against
    # F(k) = (1 - (1 - P)^k) / (1 - (1 - P)^M), then KS against uniform
    ph = o.photons()
    first = {}
    for par, stp in zip(ph["parent"].tolist(), ph["step"].tolist()):
        first[par] = min(stp, first.get(par, stp))
    k = np.array(sorted(first.values()), dtype=np.float64) + 1.0
    assert len(k) > 0.99 * o.N
    F = lambda t: -np.expm1(t * math.log1p(-P)) / -math.expm1(M * math.log1p(-P))
    u = F(k - 1) + (F(k) - F(k - 1)) * np.random.default_rng(5).random(len(k))
    ks = stats.kstest(u, "uniform")
    assert ks.pvalue > 1e-3, ks
