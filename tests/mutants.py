"""Planted errors in the oracle, for checking that its pins bite.

A mutant is a copy of oracle/oracle.c with one plausible mistake written into
it (a dropped term, a wrong sign, index or weight), compiled with the
oracle's own flags into a separate shared object under _build/.  A pin is
shown to pin its function when it passes on the oracle and fails on the
mutant.  Nothing here runs on a GPU.
"""
from __future__ import annotations

import hashlib
import os
import shutil

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MUT_DIR = os.path.join(ROOT, "_build", "mutants")

# name -> list of (text in oracle.c, replacement); each text must occur once
MUTANTS = {
    # charge-conserving deposit
    "deposit2d_jx_weight": [("double W = 0.5 * (S1[0][i] - S0[0][i]) * (S0[1][j] + S1[1][j]);",
                             "double W = 0.5 * (S1[0][i] - S0[0][i]) * (S0[1][j] + S0[1][j]);")],
    "deposit2d_jz_weights": [("(S0[0][i] * S0[1][j] + S1[0][i] * S1[1][j]) * (1.0 / 3.0) +\n"
                              "                   (S0[0][i] * S1[1][j] + S1[0][i] * S0[1][j]) * (1.0 / 6.0);",
                              "(S0[0][i] * S0[1][j] + S1[0][i] * S1[1][j]) * (1.0 / 2.0) +\n"
                              "                   (S0[0][i] * S1[1][j] + S1[0][i] * S0[1][j]) * (0.0 / 6.0);")],
    "deposit3d_T_weight": [("double T = (S0[1][j] * S0[2][k] + S1[1][j] * S1[2][k]) * (1.0 / 3.0) +",
                            "double T = (S0[1][j] * S0[2][k] + S1[1][j] * S1[2][k]) * (1.0 / 2.0) +")],
    "current_quantum_2e-30": [("int64_t q = (int64_t)llrint(v * 0x1p40);", "int64_t q = (int64_t)llrint(v * 0x1p30) << 10;")],
    # gather
    "gather_stagger_sign": [("double ga = g[a] - 0.5 * (double)st[a];", "double ga = g[a] + 0.5 * (double)st[a];")],
    "gather3d_z_fraction": [("return (1.0 - f[2]) * a2 + f[2] * b2;", "return (1.0 - f[1]) * a2 + f[1] * b2;")],
    # Yee field solve
    "bhalf_curl_sign": [("if (s->act[1]) b = b - s->hd[1] * (Ez[fidx(s, i, j + 1, k)] - Ez[m]);",
                         "if (s->act[1]) b = b + s->hd[1] * (Ez[fidx(s, i, j + 1, k)] - Ez[m]);")],
    "efull_curl_index": [("if (s->act[1]) e = e + s->cd[1] * (Bz[m] - Bz[fidx(s, i, j - 1, k)]);",
                          "if (s->act[1]) e = e + s->cd[1] * (Bz[fidx(s, i, j + 1, k)] - Bz[m]);")],
    "mur_coefficient_sign": [("s->cm[a] = (s->dt - s->dx[a]) / (s->dt + s->dx[a]);",
                              "s->cm[a] = (s->dx[a] - s->dt) / (s->dt + s->dx[a]);")],
    # Gaussian source
    "source3d_amplitude": [("A = (w0n / wz) * exp(-r2 / (wz * wz));", "A = sqrt(w0n / wz) * exp(-r2 / (wz * wz));")],
    "source2d_gouy": [("ph = 0.5 * r2 * Rinv - 0.5 * psi;", "ph = 0.5 * r2 * Rinv - psi;")],
    "source_curvature_sign": [("double Rinv = zz / (zz * zz + zR * zR);", "double Rinv = -zz / (zz * zz + zR * zR);")],
    # quantum parameter
    "eta_pxB_sign": [("double cx = gamma * E[0] + (py * B[2] - pz * B[1]);\n"
                      "  double cy = gamma * E[1] + (pz * B[0] - px * B[2]);\n"
                      "  double cz = gamma * E[2] + (px * B[1] - py * B[0]);",
                      "double cx = gamma * E[0] - (py * B[2] - pz * B[1]);\n"
                      "  double cy = gamma * E[1] - (pz * B[0] - px * B[2]);\n"
                      "  double cz = gamma * E[2] - (px * B[1] - py * B[0]);")],
    "eta_pE_sign": [("double q2 = (cx * cx + cy * cy + cz * cz) - pe * pe;",
                     "double q2 = (cx * cx + cy * cy + cz * cz) + pe * pe;")],
    "eta_gamma_dropped": [("double cy = gamma * E[1] + (pz * B[0] - px * B[2]);",
                           "double cy = E[1] + (pz * B[0] - px * B[2]);")],
    # table interpolation and sampling
    "ncs_rate_blend": [("double h = s->h[i] + f * (s->h[i + 1] - s->h[i]);",
                        "double h = s->h[i] + (1.0 - f) * (s->h[i + 1] - s->h[i]);")],
    "ncs_row_blend": [("double lx = la + f * (lb - la);", "double lx = la + (1.0 - f) * (lb - la);")],
    "ncs_row_search": [("int lo = 0, hi = s->n_xi - 1;\n  while (hi - lo > 1) {\n    int mid = (lo + hi) / 2;\n"
                        "    if (C[mid] <= u) lo = mid; else hi = mid;",
                        "int lo = 0, hi = s->n_xi - 1;\n  while (hi - lo > 1) {\n    int mid = (lo + hi) / 2;\n"
                        "    if (C[mid] < u) hi = mid; else lo = mid;")],
    "brem_sigma_blend": [("return s->sigma[i] + f * (s->sigma[i + 1] - s->sigma[i]);",
                          "return s->sigma[i + 1] + f * (s->sigma[i + 1] - s->sigma[i]);")],
    "brem_row_blend": [("double sv = sa + f * (sb - sa);", "double sv = sa + (1.0 - f) * (sb - sa);")],
    "brem_energy_map": [("double eps = or_exp(lk + sv * (lt - lk));",
                         "double eps = or_exp(lk + sv * (or_log(T + 1.0) - lk));")],
    # the oracle's own exp / log series
    "exp_series_short": [("  for (int n = 13; n >= 0; --n) p = p * r + INV_FACT[n];",
                          "  for (int n = 7; n >= 0; --n) p = p * r + INV_FACT[n];")],
    "log_split_dropped": [("  return de * L_HI + (de * L_LO + lm);", "  return de * L_HI + lm;")],
    # mobile ions
    "ion_push_charge_sign": [("const double hq = 0.5 * s->dt * (s->iq / s->imass);",
                              "const double hq = -0.5 * s->dt * (s->iq / s->imass);")],
    "ion_mass_dropped": [("const double hq = 0.5 * s->dt * (s->iq / s->imass);",
                          "const double hq = 0.5 * s->dt * s->iq;")],
    "ion_deposit_charge": [("deposit(s, s->ix + 3 * e, x1 + 3 * e, vv + 3 * e, s->iq * s->iw);",
                            "deposit(s, s->ix + 3 * e, x1 + 3 * e, vv + 3 * e, s->iw);")],
    "ion_density_volume": [("for (int64_t m = 0; m < s->ncell_tot; ++m) s->ni[m] = (double)s->icount[m] * s->iwv;",
                            "for (int64_t m = 0; m < s->ncell_tot; ++m) s->ni[m] = (double)s->icount[m] * s->iw;")],
    # pair production
    "chi_cross_sign": [("  double cy = E[1] + (k[2] * B[0] - k[0] * B[2]);",
                        "  double cy = E[1] - (k[2] * B[0] - k[0] * B[2]);")],
    "bw_rate_alpha": [("const double K_P = 7.2973525693e-3 * s->E_S;", "const double K_P = s->E_S;")],
    "bh_density_dropped": [("double X = s->K_BR * ni * sig * s->dt;\n          double P = -or_expm1(-X);\n          or_philox(par",
                            "double X = s->K_BR * sig * s->dt;\n          double P = -or_expm1(-X);\n          or_philox(par")],
    "bw_share_row_length": [("double xa = share_inv_row(s->bw_cdf + (int64_t)bi * s->n_xp, s->n_xp, u32(r[2]));",
                             "double xa = share_inv_row(s->bw_cdf + (int64_t)bi * s->n_xp, s->n_s, u32(r[2]));"),
                            ("double xb = share_inv_row(s->bw_cdf + (int64_t)(bi + 1) * s->n_xp, s->n_xp, u32(r[2]));",
                             "double xb = share_inv_row(s->bw_cdf + (int64_t)(bi + 1) * s->n_xp, s->n_s, u32(r[2]));")],
    "photon_move_sign": [("      x[a] = x[a] + k[a] * s->dt;", "      x[a] = x[a] - k[a] * s->dt;")],
    "spectrum_bin_offset": [("  int b = 4 * (e + 2);\n  if (m >= 0x1.306fe0a31b715p+0) b++;",
                             "  int b = 4 * (e + 1);\n  if (m >= 0x1.306fe0a31b715p+0) b++;")],
    # constants
    "K_BR_factor": [("s->K_BR = s->n_c * (lam / twopi) * alpha * re * re;",
                     "s->K_BR = s->n_c * lam * alpha * re * re;")],
    "E_S_factor": [("s->E_S = lam / (twopi * lC);", "s->E_S = lam / lC;")],
}


def build(name: str) -> str:
    """Shared object of mutant `name` (cached by the text of the mutated source)."""
    src = open(os.path.join(oracle.HERE, "oracle.c")).read()
    for old, new in MUTANTS[name]:
        n = src.count(old)
        if n != 1:
            # not an AssertionError: a mutant that cannot be built must not
            # count as a pin that failed on it
            raise RuntimeError(f"mutant {name}: pattern found {n} times: {old!r}")
        src = src.replace(old, new)
    key = hashlib.sha256(src.encode()).hexdigest()[:12]
    d = os.path.join(MUT_DIR, f"{name}-{key}")
    so = os.path.join(d, "liboracle_mutant.so")
    if not os.path.exists(so):
        os.makedirs(d, exist_ok=True)
        shutil.copy(os.path.join(oracle.HERE, "oracle.h"), d)
        c = os.path.join(d, "oracle.c")
        open(c, "w").write(src)
        oracle.compile_source(c, so + ".tmp")
        os.replace(so + ".tmp", so)
    return so
