"""Oracle table builder: NCS and bremsstrahlung tables by direct quadrature.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Shares no code with the
HIP library's own table builder; the two are compared in the tests.

NCS (Sec. II.A; the paper takes its emission module from EPOCH, i.e. the
quantum-synchrotron rates of the works it cites there).  With xi = 2 chi/eta
the photon energy is xi*gamma*mc^2 and

    F(eta, xi) = xi^2 y K_{2/3}(y) + (1 - xi) y int_y^inf K_{5/3}(t) dt,
    y = 2 xi / (3 eta (1 - xi)),
    h(eta) = int_0^1 F/xi dxi,            dN/dt = K_N (eta/gamma) h(eta),
    g(eta) = 3 sqrt(3)/(4 pi eta) * int_0^1 F dxi  (radiated power / Larmor).

Bremsstrahlung (Sec. II.B, Eq. (1)): Tsai's bracket B(y; E, Z) with the
screening functions and the Coulomb correction named there, dsigma/dy =
alpha r_e^2 B / y, sigma(E) = int_{y_cut}^{y_max} dsigma (Eq. (4) text).

Quadrature here: adaptive Gauss-Legendre (16 points, bisection error
estimate) on every table interval in ln(xi) / ln(k);
K_{2/3} from scipy.special.kv; int_y^inf K_{5/3} from its representation
int_0^inf exp(-y cosh s) cosh(5s/3)/cosh(s) ds on Gauss-Legendre panels.
"""
from __future__ import annotations

import math
import numpy as np
from scipy.special import kv

MC2_MEV = 0.51099895000
ALPHA = 7.2973525693e-3

# --- table geometry (the layout the C-ABI consumes) -------------------------
N_ETA, ETA_MIN, ETA_MAX = 256, 1e-4, 1e2
N_XI, XI_MIN = 256, 1e-12
N_T, T_MIN_MEV, T_MAX_MEV = 128, 1e-3, 1e3
N_Y = 64

_GL16 = np.polynomial.legendre.leggauss(16)
_GL8 = np.polynomial.legendre.leggauss(8)


def _gl_nodes(a, b, gl):
    """Nodes and weights of one Gauss-Legendre panel on [a, b] (broadcasts)."""
    x, w = gl
    a = np.asarray(a, dtype=np.float64)[..., None]
    b = np.asarray(b, dtype=np.float64)[..., None]
    half = 0.5 * (b - a)
    return a + half * (x + 1.0), half * w


def int_k53(y):
    """int_y^inf K_{5/3}(t) dt for an array of y > 0 (0 where it underflows)."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(y)
    ok = y < 700.0
    yy = y[ok]
    if yy.size == 0:
        return out
    # integrand exp(-y cosh s) cosh(5s/3)/cosh s is negligible once y cosh s > 60
    smax = np.arccosh(np.maximum(60.0 / yy, 1.0)) + 2.0
    npan = 24
    edges = smax[:, None] * np.linspace(0.0, 1.0, npan + 1)[None, :]
    s, w = _gl_nodes(edges[:, :-1], edges[:, 1:], _GL8)          # (n, npan, 8)
    ch = np.cosh(s)
    f = np.exp(-yy[:, None, None] * ch) * np.cosh(s * (5.0 / 3.0)) / ch
    out[ok] = np.sum(f * w, axis=(1, 2))
    return out


def ncs_F(eta, xi):
    """Quantum-synchrotron emissivity F(eta, xi); xi in (0, 1)."""
    eta = np.asarray(eta, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    y = 2.0 * xi / (3.0 * eta * (1.0 - xi))
    big = y > 700.0
    ys = np.where(big, 1.0, y)
    k23 = kv(2.0 / 3.0, ys)
    F = xi * xi * ys * k23 + (1.0 - xi) * ys * int_k53(ys)
    return np.where(big, 0.0, F)


def _gl_panel(f, a, b):
    """16-point Gauss-Legendre integral of vectorised f on each [a_i, b_i]."""
    t, w = _gl_nodes(a, b, _GL16)
    return np.sum(f(t.ravel()).reshape(t.shape) * w, axis=-1)


def adaptive_integrals(f, a, b, atol, rtol=1e-13, max_levels=48):
    """Integral of f over each interval [a_i, b_i]: Gauss-Legendre 16 on the
    panel and on its two halves; panels whose two estimates differ by more
    than max(atol, rtol*|I|) are bisected (vectorised over all panels)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    res = np.zeros(a.size)
    pa, pb, po = a.copy(), b.copy(), np.arange(a.size)
    whole = _gl_panel(f, pa, pb)
    for _ in range(max_levels):
        m = 0.5 * (pa + pb)
        left = _gl_panel(f, pa, m)
        right = _gl_panel(f, m, pb)
        two = left + right
        ok = np.abs(two - whole) <= np.maximum(atol, rtol * np.abs(two))
        np.add.at(res, po[ok], two[ok])
        if ok.all():
            return res
        nk = ~ok
        pa = np.concatenate([pa[nk], m[nk]])
        pb = np.concatenate([m[nk], pb[nk]])
        po = np.concatenate([po[nk], po[nk]])
        whole = np.concatenate([left[nk], right[nk]])
    np.add.at(res, po, whole)
    return res


def _ncs_row(eta, lnxi_grid, with_first=True):
    """Cumulative integral of F d(ln xi) on the grid (index 0 holds the mass
    below the first grid point); also returns int F dxi for g(eta)."""
    lo = lnxi_grid[0]
    fa = lambda u: ncs_F(eta, np.exp(u))
    fb = lambda u: ncs_F(eta, np.exp(u)) * np.exp(u)
    # edges: 60 units of ln(xi) below the grid (integrand ~ xi^(1/3)), then the grid
    below_e = np.linspace(lo - 60.0, lo, 31)
    edges_a = np.concatenate([below_e[:-1], lnxi_grid[:-1]])
    edges_b = np.concatenate([below_e[1:], lnxi_grid[1:]])
    scale = np.sum(_gl_panel(fa, edges_a, edges_b))
    I = adaptive_integrals(fa, edges_a, edges_b, atol=1e-16 * scale)
    below = np.sum(I[:30])
    cum = np.concatenate([[below], below + np.cumsum(I[30:])])
    if not with_first:
        return cum, None
    scale1 = np.sum(_gl_panel(fb, edges_a, edges_b))
    first = np.sum(adaptive_integrals(fb, edges_a, edges_b, atol=1e-16 * scale1))
    return cum, first


def ncs_h_g(eta):
    """h(eta) and g(eta) for a scalar eta, on the table's xi grid."""
    lnxi = np.linspace(math.log(XI_MIN), 0.0, N_XI)
    cum, first = _ncs_row(float(eta), lnxi)
    h = cum[-1]
    g = 3.0 * math.sqrt(3.0) / (4.0 * math.pi) * first / eta
    return h, g


def _ncs_table_row(i):
    ln_eta0 = math.log(ETA_MIN)
    dln_eta = math.log(ETA_MAX / ETA_MIN) / (N_ETA - 1)
    lnxi = np.linspace(math.log(XI_MIN), 0.0, N_XI)
    eta = math.exp(ln_eta0 + i * dln_eta)
    cum, _ = _ncs_row(eta, lnxi, with_first=False)
    return i, cum


def build_ncs(workers=None):
    """NCS tables: h on the eta grid, shared ln(xi) grid, CDF rows (rows are
    independent and are computed in a process pool)."""
    import concurrent.futures as cf
    import os
    ln_eta0 = math.log(ETA_MIN)
    dln_eta = math.log(ETA_MAX / ETA_MIN) / (N_ETA - 1)
    lnxi = np.linspace(math.log(XI_MIN), 0.0, N_XI)
    lnxi[-1] = 0.0
    h = np.empty(N_ETA)
    cdf = np.empty((N_ETA, N_XI))
    nw = workers or min(16, os.cpu_count() or 1)
    if nw > 1:
        with cf.ProcessPoolExecutor(max_workers=nw) as ex:
            rows = list(ex.map(_ncs_table_row, range(N_ETA), chunksize=4))
    else:
        rows = [_ncs_table_row(i) for i in range(N_ETA)]
    for i, cum in rows:
        h[i] = cum[-1]
        c = cum / cum[-1]
        c[-1] = 1.0
        cdf[i] = c
    return dict(n_eta=N_ETA, ln_eta0=ln_eta0, dln_eta=dln_eta, h=h,
                n_xi=N_XI, ln_xi=lnxi, ncs_cdf=cdf)


# --- Tsai bremsstrahlung, Eq. (1) -------------------------------------------
def coulomb_f(Z):
    """Coulomb correction f(Z) (Davies-Bethe-Maximon form used by Tsai)."""
    a2 = (ALPHA * Z) ** 2
    return a2 * (1.0 / (1.0 + a2) + 0.20206 - 0.0369 * a2 + 0.0083 * a2 ** 2 - 0.002 * a2 ** 3)


def screening(gs, es):
    """Tsai's screening functions phi1, phi2 (of gamma) and psi1, psi2 (of eps)."""
    phi1 = 20.863 - 2.0 * np.log(1.0 + (0.55846 * gs) ** 2) \
        - 4.0 * (1.0 - 0.6 * np.exp(-0.9 * gs) - 0.4 * np.exp(-1.5 * gs))
    phi2 = phi1 - (2.0 / 3.0) / (1.0 + 6.5 * gs + 6.0 * gs * gs)
    psi1 = 28.340 - 2.0 * np.log(1.0 + (3.621 * es) ** 2) \
        - 4.0 * (1.0 - 0.7 * np.exp(-8.0 * es) - 0.3 * np.exp(-29.2 * es))
    psi2 = psi1 - (2.0 / 3.0) / (1.0 + 40.0 * es + 400.0 * es * es)
    return phi1, phi2, psi1, psi2


def tsai_bracket(y, E, Z, clamp=True):
    """Curly bracket of Eq. (1): dsigma/dy = alpha r_e^2 * B / y.
    E is the total electron energy in mc^2, y = k/E."""
    y = np.asarray(y, dtype=np.float64)
    k = y * E
    Ep = E - k
    gs = 100.0 * k / (E * Ep * Z ** (1.0 / 3.0))
    es = 100.0 * k / (E * Ep * Z ** (2.0 / 3.0))
    phi1, phi2, psi1, psi2 = screening(gs, es)
    lnZ = math.log(Z)
    fz = coulomb_f(Z)
    B = (4.0 / 3.0 - 4.0 / 3.0 * y + y * y) * (Z * Z * (phi1 - 4.0 / 3.0 * lnZ - 4.0 * fz)
                                               + Z * (psi1 - 8.0 / 3.0 * lnZ)) \
        + 2.0 / 3.0 * (1.0 - y) * (Z * Z * (phi1 - phi2) + Z * (psi1 - psi2))
    return np.maximum(B, 0.0) if clamp else B


def build_brem(Z, k_cut_mc2=1.0):
    """sigma(T) in units of alpha r_e^2 and cumulative rows on the scaled
    coordinate s = (ln k - ln k_cut)/(ln T - ln k_cut), 64 points."""
    T0 = T_MIN_MEV / MC2_MEV
    ln_T0 = math.log(T0)
    dln_T = math.log(T_MAX_MEV / T_MIN_MEV) / (N_T - 1)
    sig = np.zeros(N_T)
    cdf = np.empty((N_T, N_Y))
    sgrid = np.arange(N_Y) / (N_Y - 1.0)
    for i in range(N_T):
        T = math.exp(ln_T0 + i * dln_T)
        E = T + 1.0
        if not (T > k_cut_mc2):
            cdf[i] = sgrid
            continue
        lk = np.log(k_cut_mc2) + sgrid * (math.log(T) - math.log(k_cut_mc2))
        # B d(ln y) = B d(ln k) on each interval, adaptive Gauss-Legendre
        fB = lambda u, E=E: tsai_bracket(np.exp(u) / E, E, Z)
        scale = np.sum(_gl_panel(fB, lk[:-1], lk[1:]))
        per = adaptive_integrals(fB, lk[:-1], lk[1:], atol=1e-16 * scale)
        cum = np.concatenate([[0.0], np.cumsum(per)])
        sig[i] = cum[-1]
        c = cum / cum[-1]
        c[-1] = 1.0
        cdf[i] = c
    return dict(n_T=N_T, ln_T0=ln_T0, dln_T=dln_T, sigma=sig, n_y=N_Y, br_cdf=cdf,
                k_cut=float(k_cut_mc2), Z=int(Z))


# --- pair production (the channels the paper names beside its two) ---------
# Breit-Wheeler, a photon of energy eps (mc^2) with quantum parameter chi
# turning into a pair in the laser field (named in Sec. I and II.A as the
# companion of NCS in the QED-PIC codes it builds on): with xi the electron's
# share of eps and y = 2 / (3 chi xi (1 - xi)),
#
#     d2N/(dt dxi) = alpha m c^2 / (sqrt(3) pi hbar eps)
#                    * [ int_y^inf K_{1/3}(t) dt + (xi/(1-xi) + (1-xi)/xi) K_{2/3}(y) ],
#
# so dN/dt = alpha (m c^2/hbar) (chi/eps) T(chi) with
# T(chi) = 1/(sqrt(3) pi chi) int_0^1 [..] dxi.
N_CHI, CHI_MIN, CHI_MAX = 128, 1e-2, 1e3
N_XP = 128
# Bethe-Heitler, a photon of energy k pair-converting on a nucleus ("similar
# to the bremsstrahlung", Sec. II.B): Tsai's cross-section, the crossing of
# Eq. (1), with x the positron's share of k and the screening variables at
# E+ E- = x (1 - x) k^2:
#
#     dsigma/dx = alpha r_e^2 { [x^2 + (1-x)^2 + 2/3 x (1-x)] [Z^2 (phi1 - 4/3 ln Z - 4 f)
#                               + Z (psi1 - 8/3 ln Z)]
#                               - 2/3 x (1-x) [Z^2 (phi1 - phi2) + Z (psi1 - psi2)] },
#
# both pair members above rest (1/k < x < 1 - 1/k).
N_K, K_MIN, K_MAX = 128, 2.0, 2.0e4
N_S = 64


def int_k13(y):
    """int_y^inf K_{1/3}(t) dt for an array of y > 0 (0 where it underflows)."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(y)
    ok = y < 700.0
    yy = y[ok]
    if yy.size == 0:
        return out
    smax = np.arccosh(np.maximum(60.0 / yy, 1.0)) + 2.0
    npan = 24
    edges = smax[:, None] * np.linspace(0.0, 1.0, npan + 1)[None, :]
    s, w = _gl_nodes(edges[:, :-1], edges[:, 1:], _GL8)
    ch = np.cosh(s)
    f = np.exp(-yy[:, None, None] * ch) * np.cosh(s * (1.0 / 3.0)) / ch
    out[ok] = np.sum(f * w, axis=(1, 2))
    return out


def bw_bracket(chi, xi):
    """The square bracket of the Breit-Wheeler spectrum; xi in (0, 1)."""
    xi = np.asarray(xi, dtype=np.float64)
    y = 2.0 / (3.0 * chi * xi * (1.0 - xi))
    big = y > 700.0
    ys = np.where(big, 1.0, y)
    val = int_k13(ys) + (xi / (1.0 - xi) + (1.0 - xi) / xi) * kv(2.0 / 3.0, ys)
    return np.where(big, 0.0, val)


def _bw_row(chi):
    """Cumulative integral of the bracket over the xi grid, and T(chi)."""
    xg = np.linspace(0.0, 1.0, N_XP)
    f = lambda u: bw_bracket(chi, u)
    # the bracket diverges like xi^(-1/3) at both ends: panels on a graded mesh
    scale = np.sum(_gl_panel(f, xg[:-1], xg[1:]))
    per = adaptive_integrals(f, xg[:-1], xg[1:], atol=1e-16 * max(scale, 1e-300))
    cum = np.concatenate([[0.0], np.cumsum(per)])
    T = cum[-1] / (math.sqrt(3.0) * math.pi * chi)
    return cum, T


def bw_T(chi):
    return _bw_row(float(chi))[1]


def build_bw():
    """ln T on the chi grid and CDF rows of the electron share xi (uniform
    grid on [0, 1], symmetric about 1/2)."""
    ln_chi0 = math.log(CHI_MIN)
    dln_chi = math.log(CHI_MAX / CHI_MIN) / (N_CHI - 1)
    lnT = np.empty(N_CHI)
    cdf = np.empty((N_CHI, N_XP))
    for i in range(N_CHI):
        chi = math.exp(ln_chi0 + i * dln_chi)
        cum, T = _bw_row(chi)
        lnT[i] = math.log(T)
        c = cum / cum[-1]
        c[-1] = 1.0
        cdf[i] = c
    return dict(n_chi=N_CHI, ln_chi0=ln_chi0, dln_chi=dln_chi, bw_lnT=lnT, n_xp=N_XP,
                bw_cdf=cdf)


def bh_dcs(x, k, Z, clamp=True):
    """Curly bracket of the pair cross-section: dsigma/dx = alpha r_e^2 * B."""
    x = np.asarray(x, dtype=np.float64)
    q = x * (1.0 - x)
    gs = 100.0 / (k * q * Z ** (1.0 / 3.0))
    es = 100.0 / (k * q * Z ** (2.0 / 3.0))
    phi1, phi2, psi1, psi2 = screening(gs, es)
    lnZ = math.log(Z)
    fz = coulomb_f(Z)
    B = (x * x + (1.0 - x) ** 2 + 2.0 / 3.0 * q) * (Z * Z * (phi1 - 4.0 / 3.0 * lnZ - 4.0 * fz)
                                                    + Z * (psi1 - 8.0 / 3.0 * lnZ)) \
        - 2.0 / 3.0 * q * (Z * Z * (phi1 - phi2) + Z * (psi1 - psi2))
    return np.maximum(B, 0.0) if clamp else B


def build_bh(Z):
    """sigma(k) in alpha r_e^2 on a ln k grid from 2 mc^2, and CDF rows of
    the positron share on s = (x - 1/k) / (1 - 2/k), 64 points."""
    ln_k0 = math.log(K_MIN)
    dln_k = math.log(K_MAX / K_MIN) / (N_K - 1)
    sig = np.zeros(N_K)
    cdf = np.empty((N_K, N_S))
    sgrid = np.arange(N_S) / (N_S - 1.0)
    for i in range(N_K):
        k = math.exp(ln_k0 + i * dln_k)
        lo, hi = 1.0 / k, 1.0 - 1.0 / k
        if not (hi > lo):
            cdf[i] = sgrid
            continue
        xg = lo + sgrid * (hi - lo)
        f = lambda u, k=k: bh_dcs(u, k, Z)
        scale = np.sum(_gl_panel(f, xg[:-1], xg[1:]))
        if not (scale > 0.0):
            cdf[i] = sgrid
            continue
        per = adaptive_integrals(f, xg[:-1], xg[1:], atol=1e-16 * scale)
        cum = np.concatenate([[0.0], np.cumsum(per)])
        sig[i] = cum[-1]
        c = cum / cum[-1]
        c[-1] = 1.0
        cdf[i] = c
    return dict(n_k=N_K, ln_k0=ln_k0, dln_k=dln_k, bh_sigma=sig, n_s=N_S, bh_cdf=cdf)


def build_tables(Z, k_cut_mc2=1.0):
    t = build_ncs()
    t.update(build_brem(Z, k_cut_mc2))
    t.update(build_bw())
    t.update(build_bh(Z))
    return t
