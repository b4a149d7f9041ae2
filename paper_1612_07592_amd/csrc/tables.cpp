// Emission-table builder of libpic (host, FP64), exported as pic_build_tables.
//
// NCS (the paper's Sec. II.A defers to the quantum-synchrotron emission of
// the works it cites; EPOCH's module): with xi = hbar w/(gamma m c^2) and
// y = 2 xi / (3 eta (1 - xi)),
//   F(eta, xi) = xi^2 y K_{2/3}(y) + (1 - xi) y Int_y^inf K_{5/3},
//   h(eta) = Int_0^1 F / xi dxi,  CDF(xi) = Int_0^xi F/xi' dxi' / h.
// Both Bessel quantities come from one trapezoid sum over t of
// exp(-y cosh t) [cosh(2t/3), cosh(5t/3)/cosh t] (exponentially convergent),
// and the xi integrals from adaptive Simpson panels in ln(xi).
//
// Bremsstrahlung (Sec. II.B, Eq. (1)): Tsai's bracket with his screening
// functions and the Coulomb correction; sigma(T) = Int_{k_cut}^{T} B d ln k in
// alpha r_e^2; cumulative rows on s = ln(k/k_cut)/ln(T/k_cut).
//
// Pairs: the Breit-Wheeler spectrum bracket Int_y^inf K_{1/3} + (xi/(1-xi) +
// (1-xi)/xi) K_{2/3}(y), y = 2/(3 chi xi (1-xi)), integrated over the
// electron share xi on a uniform grid (T(chi) = Int / (sqrt(3) pi chi)); the
// Bethe-Heitler cross-section in Tsai's form for pair production (the same
// screening functions and Coulomb correction, arguments at E+ E- =
// x (1-x) k^2), integrated over the positron share x between 1/k and 1 - 1/k.
#include <cmath>
#include <thread>
#include <vector>
#include "../../include/pic.h"
#include "pic_internal.hpp"

namespace {

constexpr int kNeta = 256, kNxi = 256, kNT = 128, kNy = 64;
constexpr double kEtaMin = 1e-4, kEtaMax = 1e2, kXiMin = 1e-12;
constexpr double kMc2MeV = 0.51099895000;
constexpr double kTMinMeV = 1e-3, kTMaxMeV = 1e3;
constexpr double kAlpha = 7.2973525693e-3;
constexpr int kNchi = 128, kNxp = 128, kNk = 128, kNs = 64;
constexpr double kChiMin = 1e-2, kChiMax = 1e3, kKMin = 2.0, kKMax = 2.0e4;

// K_{2/3}(y) and Int_y^inf K_{5/3}(t) dt by the trapezoid rule in t.
void bessel_pair(double y, double* k23, double* i53) {
  if (y > 700.0) { *k23 = 0.0; *i53 = 0.0; return; }
  const double h = 1.0 / 32.0;
  double a = 0.5 * std::exp(-y);  // t = 0 term, weight 1/2; cosh(0) = 1
  double b = a;
  for (int k = 1;; ++k) {
    const double t = k * h;
    const double ch = std::cosh(t);
    const double ex = std::exp(-y * ch);
    const double ta = ex * std::cosh(t * (2.0 / 3.0));
    const double tb = ex * std::cosh(t * (5.0 / 3.0)) / ch;
    a += ta;
    b += tb;
    if (y * ch > 40.0 && tb < 1e-18 * b) break;
    if (k > 200000) break;
  }
  *k23 = a * h;
  *i53 = b * h;
}

double ncs_F(double eta, double xi) {
  if (!(xi < 1.0)) return 0.0;
  const double y = 2.0 * xi / (3.0 * eta * (1.0 - xi));
  if (y > 700.0) return 0.0;
  double k23, i53;
  bessel_pair(y, &k23, &i53);
  return xi * xi * y * k23 + (1.0 - xi) * y * i53;
}

// Adaptive Simpson (Lyness): refine [a, b] until the Richardson difference
// of the two half-panel estimates is below 15 * dens * (b - a).
template <class Fn>
double asimpson(const Fn& f, double a, double b, double fa, double fm, double fb, double whole,
                double dens, int depth) {
  const double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
  const double flm = f(lm), frm = f(rm);
  const double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
  const double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
  const double delta = left + right - whole;
  if (depth <= 0 || std::fabs(delta) <= 15.0 * dens * (b - a) ||
      std::fabs(delta) <= 1e-14 * std::fabs(left + right))
    return left + right + delta / 15.0;
  return asimpson(f, a, m, fa, flm, fm, left, dens, depth - 1) +
         asimpson(f, m, b, fm, frm, fb, right, dens, depth - 1);
}

// Integral over [a, b] as 4 adaptive Simpson panels.
template <class Fn>
double integrate(const Fn& f, double a, double b, double dens) {
  double sum = 0.0;
  const int np = 4;
  for (int q = 0; q < np; ++q) {
    const double pa = a + (b - a) * q / np, pb = a + (b - a) * (q + 1) / np;
    const double fa = f(pa), fb = f(pb), fm = f(0.5 * (pa + pb));
    const double whole = (pb - pa) / 6.0 * (fa + 4.0 * fm + fb);
    sum += asimpson(f, pa, pb, fa, fm, fb, whole, dens, 24);
  }
  return sum;
}

void ncs_row(double eta, const double* lnxi, double* h_out, double* cdf) {
  auto f = [eta](double u) { return ncs_F(eta, std::exp(u)); };
  // coarse total for the error density (integrand ~ xi^(1/3) below the grid)
  const double lo = lnxi[0] - 50.0;
  double coarse = 0.0;
  for (int q = 0; q < 400; ++q) {
    const double a = lo + (0.0 - lo) * q / 400, b = lo + (0.0 - lo) * (q + 1) / 400;
    coarse += (b - a) / 6.0 * (f(a) + 4.0 * f(0.5 * (a + b)) + f(b));
  }
  const double dens = 1e-15 * coarse / (0.0 - lo);
  double cum = integrate(f, lo, lnxi[0], dens);
  cdf[0] = cum;
  for (int j = 0; j + 1 < kNxi; ++j) {
    cum += integrate(f, lnxi[j], lnxi[j + 1], dens);
    cdf[j + 1] = cum;
  }
  *h_out = cum;
  for (int j = 0; j < kNxi; ++j) cdf[j] /= cum;
  cdf[kNxi - 1] = 1.0;
}

// Tsai's screening terms at the screening variables gs (gamma) and es
// (epsilon): the unscreened-charge bracket A = Z^2 (phi1 - 4/3 ln Z - 4 f) +
// Z (psi1 - 8/3 ln Z) and the difference D = Z^2 (phi1 - phi2) + Z (psi1 - psi2).
void tsai_terms(double gs, double es, double Z, double* A, double* D) {
  const double phi1 = 20.863 - 2.0 * std::log(1.0 + (0.55846 * gs) * (0.55846 * gs)) -
                      4.0 * (1.0 - 0.6 * std::exp(-0.9 * gs) - 0.4 * std::exp(-1.5 * gs));
  const double phi2 = phi1 - (2.0 / 3.0) / (1.0 + 6.5 * gs + 6.0 * gs * gs);
  const double psi1 = 28.340 - 2.0 * std::log(1.0 + (3.621 * es) * (3.621 * es)) -
                      4.0 * (1.0 - 0.7 * std::exp(-8.0 * es) - 0.3 * std::exp(-29.2 * es));
  const double psi2 = psi1 - (2.0 / 3.0) / (1.0 + 40.0 * es + 400.0 * es * es);
  const double a2 = (kAlpha * Z) * (kAlpha * Z);
  const double fz = a2 * (1.0 / (1.0 + a2) + 0.20206 - 0.0369 * a2 + 0.0083 * a2 * a2 - 0.002 * a2 * a2 * a2);
  const double lnZ = std::log(Z);
  *A = Z * Z * (phi1 - (4.0 / 3.0) * lnZ - 4.0 * fz) + Z * (psi1 - (8.0 / 3.0) * lnZ);
  *D = Z * Z * (phi1 - phi2) + Z * (psi1 - psi2);
}

// Bremsstrahlung bracket of Eq. (1) at y = k/E.
double tsai_B(double y, double E, double Z) {
  const double k = y * E, Ep = E - k;
  double A, D;
  tsai_terms(100.0 * k / (E * Ep * std::cbrt(Z)), 100.0 * k / (E * Ep * std::cbrt(Z * Z)), Z, &A, &D);
  const double B = (4.0 / 3.0 - (4.0 / 3.0) * y + y * y) * A + (2.0 / 3.0) * (1.0 - y) * D;
  return B > 0.0 ? B : 0.0;
}

// Pair-production bracket at positron share x of a photon k (mc^2).
double tsai_pair(double x, double k, double Z) {
  const double q = x * (1.0 - x);
  double A, D;
  tsai_terms(100.0 / (k * q * std::cbrt(Z)), 100.0 / (k * q * std::cbrt(Z * Z)), Z, &A, &D);
  const double B = (1.0 - (4.0 / 3.0) * q) * A - (2.0 / 3.0) * q * D;
  return B > 0.0 ? B : 0.0;
}

// K_{2/3}(y) and Int_y^inf K_{1/3}(t) dt by the trapezoid rule in t.
void bessel_bw(double y, double* k23, double* i13) {
  if (y > 700.0) { *k23 = 0.0; *i13 = 0.0; return; }
  const double h = 1.0 / 32.0;
  double a = 0.5 * std::exp(-y), b = a;
  for (int k = 1;; ++k) {
    const double t = k * h;
    const double ch = std::cosh(t);
    const double ex = std::exp(-y * ch);
    const double ta = ex * std::cosh(t * (2.0 / 3.0));
    const double tb = ex * std::cosh(t * (1.0 / 3.0)) / ch;
    a += ta;
    b += tb;
    if (y * ch > 40.0 && ta < 1e-18 * a) break;
    if (k > 200000) break;
  }
  *k23 = a * h;
  *i13 = b * h;
}

double bw_bracket(double chi, double xi) {
  if (!(xi > 0.0 && xi < 1.0)) return 0.0;
  const double y = 2.0 / (3.0 * chi * xi * (1.0 - xi));
  if (y > 700.0) return 0.0;
  double k23, i13;
  bessel_bw(y, &k23, &i13);
  return i13 + (xi / (1.0 - xi) + (1.0 - xi) / xi) * k23;
}

void bw_row(double chi, double* lnT, double* cdf) {
  auto f = [chi](double xi) { return bw_bracket(chi, xi); };
  double coarse = 0.0;
  for (int q = 0; q < 512; ++q) {
    const double a = (double)q / 512, b = (double)(q + 1) / 512;
    coarse += (b - a) / 6.0 * (f(a) + 4.0 * f(0.5 * (a + b)) + f(b));
  }
  const double dens = 1e-15 * coarse;
  double cum = 0.0;
  cdf[0] = 0.0;
  for (int j = 0; j + 1 < kNxp; ++j) {
    cum += integrate(f, (double)j / (kNxp - 1), (double)(j + 1) / (kNxp - 1), dens);
    cdf[j + 1] = cum;
  }
  *lnT = std::log(cum / (std::sqrt(3.0) * M_PI * chi));
  for (int j = 0; j < kNxp; ++j) cdf[j] /= cum;
  cdf[kNxp - 1] = 1.0;
}

void bh_row(double k, double Z, double* sigma, double* cdf) {
  const double lo = 1.0 / k, hi = 1.0 - 1.0 / k;
  auto f = [k, Z](double x) { return tsai_pair(x, k, Z); };
  double coarse = 0.0;
  if (hi > lo)
    for (int q = 0; q < 256; ++q) {
      const double a = lo + (hi - lo) * q / 256, b = lo + (hi - lo) * (q + 1) / 256;
      coarse += (b - a) / 6.0 * (f(a) + 4.0 * f(0.5 * (a + b)) + f(b));
    }
  if (!(coarse > 0.0)) {
    *sigma = 0.0;
    for (int j = 0; j < kNs; ++j) cdf[j] = (double)j / (kNs - 1);
    return;
  }
  const double dens = 1e-15 * coarse / (hi - lo);
  double cum = 0.0;
  cdf[0] = 0.0;
  for (int j = 0; j + 1 < kNs; ++j) {
    cum += integrate(f, lo + (hi - lo) * j / (kNs - 1), lo + (hi - lo) * (j + 1) / (kNs - 1), dens);
    cdf[j + 1] = cum;
  }
  *sigma = cum;
  for (int j = 0; j < kNs; ++j) cdf[j] /= cum;
  cdf[kNs - 1] = 1.0;
}

void brem_row(int i, double Z, double kcut, double ln_T0, double dln_T, double* sigma, double* cdf) {
  const double T = std::exp(ln_T0 + i * dln_T);
  const double E = T + 1.0;
  if (!(T > kcut)) {
    *sigma = 0.0;
    for (int j = 0; j < kNy; ++j) cdf[j] = (double)j / (kNy - 1);
    return;
  }
  const double lk0 = std::log(kcut), lk1 = std::log(T);
  const double ds = (lk1 - lk0) / (kNy - 1);
  auto f = [E, Z](double u) { return tsai_B(std::exp(u) / E, E, Z); };
  double coarse = 0.0;
  for (int q = 0; q < 256; ++q) {
    const double a = lk0 + (lk1 - lk0) * q / 256, b = lk0 + (lk1 - lk0) * (q + 1) / 256;
    coarse += (b - a) / 6.0 * (f(a) + 4.0 * f(0.5 * (a + b)) + f(b));
  }
  const double dens = 1e-15 * coarse / (lk1 - lk0);
  double cum = 0.0;
  cdf[0] = 0.0;
  for (int j = 0; j + 1 < kNy; ++j) {
    cum += integrate(f, lk0 + j * ds, lk0 + (j + 1) * ds, dens);
    cdf[j + 1] = cum;
  }
  *sigma = cum;
  for (int j = 0; j < kNy; ++j) cdf[j] /= cum;
  cdf[kNy - 1] = 1.0;
}

}  // namespace

extern "C" pic_status pic_build_tables(uint32_t Z, double k_cut_mc2, int32_t nthreads, double* h,
                                       double* ln_xi, double* ncs_cdf, double* sigma,
                                       double* br_cdf, pic_tables* out) {
  if (!h || !ln_xi || !ncs_cdf || !sigma || !br_cdf || !out) return PIC_ERR_INVALID;
  if (Z < 1 || Z > 120 || !(k_cut_mc2 > 0.0) || !std::isfinite(k_cut_mc2)) return PIC_ERR_INVALID;
  const double ln_eta0 = std::log(kEtaMin);
  const double dln_eta = std::log(kEtaMax / kEtaMin) / (kNeta - 1);
  const double l0 = std::log(kXiMin);
  for (int j = 0; j < kNxi; ++j) ln_xi[j] = l0 + (0.0 - l0) * j / (kNxi - 1);
  ln_xi[kNxi - 1] = 0.0;
  const double ln_T0 = std::log(kTMinMeV / kMc2MeV);
  const double dln_T = std::log(kTMaxMeV / kTMinMeV) / (kNT - 1);
  int nt = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
  if (nt < 1) nt = 1;
  if (nt > 64) nt = 64;
  std::vector<std::thread> pool;
  for (int w = 0; w < nt; ++w)
    pool.emplace_back([=]() {
      for (int i = w; i < kNeta; i += nt)
        ncs_row(std::exp(ln_eta0 + i * dln_eta), ln_xi, &h[i], ncs_cdf + (size_t)i * kNxi);
      for (int i = w; i < kNT; i += nt)
        brem_row(i, (double)Z, k_cut_mc2, ln_T0, dln_T, &sigma[i], br_cdf + (size_t)i * kNy);
    });
  for (auto& t : pool) t.join();
  out->version = PIC_TABLES_VERSION;
  out->Z = Z;
  out->k_cut_mc2 = k_cut_mc2;
  out->n_eta = kNeta;
  out->n_xi = kNxi;
  out->ln_eta0 = ln_eta0;
  out->dln_eta = dln_eta;
  out->h = h;
  out->ln_xi = ln_xi;
  out->ncs_cdf = ncs_cdf;
  out->n_T = kNT;
  out->n_y = kNy;
  out->ln_T0 = ln_T0;
  out->dln_T = dln_T;
  out->sigma = sigma;
  out->br_cdf = br_cdf;
  out->checksum = pic::tables_checksum(*out);
  return PIC_OK;
}

extern "C" pic_status pic_build_pair_tables(uint32_t Z, int32_t nthreads, double* bw_lnT,
                                            double* bw_cdf, double* bh_sigma, double* bh_cdf,
                                            pic_pair_tables* out) {
  if (!bw_lnT || !bw_cdf || !bh_sigma || !bh_cdf || !out) return PIC_ERR_INVALID;
  if (Z < 1 || Z > 120) return PIC_ERR_INVALID;
  const double ln_chi0 = std::log(kChiMin), dln_chi = std::log(kChiMax / kChiMin) / (kNchi - 1);
  const double ln_k0 = std::log(kKMin), dln_k = std::log(kKMax / kKMin) / (kNk - 1);
  int nt = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
  if (nt < 1) nt = 1;
  if (nt > 64) nt = 64;
  std::vector<std::thread> pool;
  for (int w = 0; w < nt; ++w)
    pool.emplace_back([=]() {
      for (int i = w; i < kNchi; i += nt)
        bw_row(std::exp(ln_chi0 + i * dln_chi), &bw_lnT[i], bw_cdf + (size_t)i * kNxp);
      for (int i = w; i < kNk; i += nt)
        bh_row(std::exp(ln_k0 + i * dln_k), (double)Z, &bh_sigma[i], bh_cdf + (size_t)i * kNs);
    });
  for (auto& t : pool) t.join();
  out->version = PIC_PAIR_TABLES_VERSION;
  out->Z = Z;
  out->n_chi = kNchi;
  out->n_xp = kNxp;
  out->ln_chi0 = ln_chi0;
  out->dln_chi = dln_chi;
  out->bw_lnT = bw_lnT;
  out->bw_cdf = bw_cdf;
  out->n_k = kNk;
  out->n_s = kNs;
  out->ln_k0 = ln_k0;
  out->dln_k = dln_k;
  out->bh_sigma = bh_sigma;
  out->bh_cdf = bh_cdf;
  out->checksum = pic::pair_tables_checksum(*out);
  return PIC_OK;
}
