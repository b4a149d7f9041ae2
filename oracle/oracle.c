/*
 * FP64 CPU oracle: the per-electron step of a PIC code with Monte-Carlo
 * nonlinear Compton scattering (NCS) and bremsstrahlung, written step by step
 * from Wan et al. (arXiv:1612.07592).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; the product path never calls it.  It
 * shares no code with the HIP library.
 *
 * Paper references used below:
 *   Sec. II.A  - the quantum parameter eta and the NCS process (photon
 *                emission handled "the same as EPOCH": optical depth plus
 *                sampling from the quantum-synchrotron spectrum).
 *   Sec. II.B  - Tsai cross-section, Eq. (1); collision probability Eq. (4);
 *                the R1 < P_br test, the R2 energy draw, photon energy E*y and
 *                photon direction v/|v|; dropping low-energy photons.
 *   Sec. II.B (benchmark paragraph) - particle-only mode: field updater and
 *                weighting switched off.
 *   Sec. III   - laser and target set-up, absorbing boundaries, the
 *                m_e c^2 photon cut.
 * Where the paper is silent (pusher, shapes, recoil, RNG, interpolation) the
 * readings are the ones listed in the design notes; each is marked READING.
 *
 * Every floating-point expression is written in a fixed left-to-right order
 * and the file is compiled without FP contraction, so that an independent
 * implementation of the same readings can reproduce it bit for bit (apart from
 * libm rounding of log/exp/expm1/sin).
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------- Philox4x32-10 (Salmon et al., SC'11) ------------------ */
/* Counter-based generator: 10 rounds of the Philox S-box on a 4x32-bit
 * counter, with a 2x32-bit key bumped by the Weyl constants between rounds. */
void or_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
               uint32_t k0, uint32_t k1, uint32_t out[4]) {
  const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  for (int r = 0; r < 10; ++r) {
    uint64_t a = M0 * (uint64_t)c0;   /* multiplies the first counter word  */
    uint64_t b = M1 * (uint64_t)c2;   /* multiplies the third counter word  */
    uint32_t hi0 = (uint32_t)(a >> 32), lo0 = (uint32_t)a;
    uint32_t hi1 = (uint32_t)(b >> 32), lo1 = (uint32_t)b;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u in (0,1) from one 32-bit word, exact in double. */
static double u32(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }
/* 52-bit uniform in (0,1) from two words, exact in double: needed because the
 * per-step bremsstrahlung probability is far below 2^-32. */
static double u52(uint32_t r0, uint32_t r1) {
  uint64_t k = ((uint64_t)r0 << 20) | (uint64_t)(r1 >> 12);
  return ((double)k + 0.5) * 0x1p-52;
}

/* ------------------- exp, log and expm1 in FP64 -------------------------- */
/* The method only needs these functions to double precision; their last bit
 * differs between math libraries, and in a chaotic run one differing bit
 * (say, in the photon energy of an emission) grows until runs part.  The
 * oracle therefore evaluates them by the series below, whose every operation
 * is an IEEE-rounded add, multiply or divide in a fixed order (accurate to
 * about one ulp; pinned against the platform libm in the tests).
 *   exp(x):   x = k ln2 + r, k the nearest integer to x/ln2, r formed in two
 *             parts with ln2 = L_HI + L_LO (L_HI has 42 significant bits, so
 *             k L_HI is exact); exp(r) = sum_{n<=14} r^n/n!, |r| <= ln2/2
 *             (the first omitted term is below 2^-60); times 2^k.
 *   log(x):   x = m 2^e with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh s,
 *             s = (m-1)/(m+1), |s| <= 0.1716, = 2 s sum_{j<=11} s^(2j)/(2j+1);
 *             plus e L_HI + e L_LO.
 *   expm1(x): x sum_{n<=13} x^n/(n+1)! for |x| < ln2/2, else exp(x) - 1. */
static const double L_HI = 0x1.62e42fefa38p-1;
static const double L_LO = 0x1.ef35793c7673p-45;
static const double INV_LN2 = 0x1.71547652b82fep+0;
/* 1/n!, n = 0..14 (each an exactly representable n! divided once) */
static const double INV_FACT[15] = {
    1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0,
    1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0,
    1.0 / 6227020800.0, 1.0 / 87178291200.0};

static double or_exp(double x) {
  if (x != x) return x;
  if (x > 709.8) return INFINITY;
  if (x < -745.2) return 0.0;
  double k = rint(x * INV_LN2);
  double r = (x - k * L_HI) - k * L_LO;
  double p = INV_FACT[14];
  for (int n = 13; n >= 0; --n) p = p * r + INV_FACT[n];
  return ldexp(p, (int)k);
}

static double or_log(double x) {
  if (x != x) return x;
  if (!(x > 0.0)) return x == 0.0 ? -INFINITY : NAN;
  if (isinf(x)) return x;
  int e;
  double m = frexp(x, &e);                          /* x = m 2^e, m in [1/2, 1) */
  if (m < 0x1.6a09e667f3bcdp-1) { m = m * 2.0; e = e - 1; }
  double s = (m - 1.0) / (m + 1.0);
  double z = s * s;
  double p = 1.0 / 23.0;
  for (int j = 10; j >= 0; --j) p = p * z + 1.0 / (double)(2 * j + 1);
  double lm = (2.0 * s) * p;
  double de = (double)e;
  return de * L_HI + (de * L_LO + lm);
}

static double or_expm1(double x) {
  if (fabs(x) < 0x1.62e42fefa39efp-2) {             /* |x| < ln2/2 */
    double p = INV_FACT[14];
    for (int n = 12; n >= 0; --n) p = p * x + INV_FACT[n + 1];
    return x * p;
  }
  return or_exp(x) - 1.0;
}

double or_math(int which, double x) {
  return which == 0 ? or_exp(x) : (which == 1 ? or_log(x) : or_expm1(x));
}

/* ---------------------------- state --------------------------------------- */
#define G 2 /* guard cells per side on active axes */

struct or_sim {
  or_config c;
  /* tables (owned copies) */
  int n_eta, n_xi, n_T, n_y;
  double ln_eta0, dln_eta, idln_eta, ln_T0, dln_T, idln_T, k_cut, iny1;
  double *h, *ln_xi, *ncs_cdf, *sigma, *br_cdf;
  int n_chi, n_xp, n_k, n_s;
  double ln_chi0, idln_chi, ln_k0, idln_k;
  double *bw_lnT, *bw_cdf, *bh_sigma, *bh_cdf;
  /* derived */
  int dims, n[3], act[3], gg[3], sz[3];
  double dx[3], idx[3], L[3], dt, invV, E_S, iES, K_N, K_BR, n_c;
  double cm[3];      /* Mur coefficients */
  double hd[3], cd[3];
  int i_src;
  int64_t ncell_tot, nfield;
  uint32_t key0, key1;
  /* fields: E (current), En (next), B; J in 2^-40 fixed point */
  double *E[3], *En[3], *B[3];
  int64_t* J[3];
  double *ni;        /* ion density per cell */
  double *srcA, *srcC, *srcS; /* transverse source profile (ny_s*nz_s) */
  int nsrc_y, nsrc_z;
  /* electrons (id order, never reordered) */
  int64_t N;
  double *x, *p, *tau, *w;
  double* taub;      /* collision optical depth (free-path bremsstrahlung only) */
  uint32_t* id;
  uint8_t* alive;
  /* mobile ions (id order): positions, momenta per unit mass, weight,
   * charge, mass; the ion density of every cell, recomputed each step from
   * the ions (count times iw / V) */
  int64_t Ni;
  double *ix, *ip;
  uint8_t* ialive;
  double iw, iwv, iq, imass;
  uint32_t* icount;
  /* photons */
  int64_t pcap, pcount;
  double *ph_x, *ph_k, *ph_e, *ph_w;
  uint32_t *ph_step, *ph_parent, *ph_proc;
  /* photons in flight (OR_BW / OR_BH): position, pair optical depth, state
   * (0 not yet started, 1 travelling, 2 converted, 3 left the box, 4 below
   * the pair threshold) */
  double *gx, *gtau;
  uint8_t* gst;
  /* pairs */
  int64_t rcap, rcount;
  double *pr_x, *pr_k, *pr_em, *pr_ep, *pr_w;
  uint32_t *pr_step, *pr_parent, *pr_pstep, *pr_proc;
  or_stats st;
  uint64_t step;
  int nthreads;
};

static int64_t fidx(const or_sim* s, int i, int j, int k) {
  return (int64_t)(i + s->gg[0]) +
         (int64_t)s->sz[0] * ((int64_t)(j + s->gg[1]) + (int64_t)s->sz[1] * (int64_t)(k + s->gg[2]));
}

/* ------------------------ table interpolation ----------------------------- */
/* Inverse of one NCS cumulative row at uniform u; returns ln(xi).  Below the
 * first grid point F/xi ~ xi^(-2/3), so the CDF ~ xi^(1/3) (READING). */
static double ncs_inv_row(const or_sim* s, int row, double u) {
  const double* C = s->ncs_cdf + (int64_t)row * s->n_xi;
  if (u < C[0]) return s->ln_xi[0] + 3.0 * or_log(u / C[0]);
  int lo = 0, hi = s->n_xi - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (C[mid] <= u) lo = mid; else hi = mid;
  }
  double t = (u - C[lo]) / (C[lo + 1] - C[lo]);
  return s->ln_xi[lo] + t * (s->ln_xi[lo + 1] - s->ln_xi[lo]);
}

/* Inverse of one bremsstrahlung cumulative row; returns the scaled coordinate
 * in [0,1] between ln k_cut and ln T (READING of the R2 draw, Sec. II.B). */
static double br_inv_row(const or_sim* s, int row, double u) {
  const double* S = s->br_cdf + (int64_t)row * s->n_y;
  int lo = 0, hi = s->n_y - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (S[mid] <= u) lo = mid; else hi = mid;
  }
  double t = (u - S[lo]) / (S[lo + 1] - S[lo]);
  return ((double)lo + t) * s->iny1;
}

/* ----------------------------- set-up ------------------------------------- */
static double* dalloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

or_sim* or_create(const or_config* c, const or_tables* t, int nthreads) {
  or_sim* s = (or_sim*)calloc(1, sizeof(or_sim));
  s->c = *c;
  s->nthreads = nthreads > 0 ? nthreads : 1;
  s->dims = c->dims;
  const double twopi = 2.0 * M_PI;
  for (int a = 0; a < 3; ++a) {
    s->act[a] = a < c->dims;
    s->n[a] = s->act[a] ? c->n[a] : 1;
    s->gg[a] = s->act[a] ? G : 0;
    s->sz[a] = s->act[a] ? s->n[a] + 1 + 2 * G : 1;
    s->dx[a] = s->act[a] ? c->dx_lambda[a] * twopi : 1.0;
    s->idx[a] = 1.0 / s->dx[a];
    s->L[a] = (double)s->n[a] * s->dx[a];
  }
  double q = 0.0;
  for (int a = 0; a < c->dims; ++a) q = q + 1.0 / (s->dx[a] * s->dx[a]);
  s->dt = c->cfl / sqrt(q);
  double V = 1.0;
  for (int a = 0; a < c->dims; ++a) V = V * s->dx[a];
  s->invV = 1.0 / V;
  for (int a = 0; a < 3; ++a) {
    s->hd[a] = (0.5 * s->dt) / s->dx[a];
    s->cd[a] = s->dt / s->dx[a];
    s->cm[a] = (s->dt - s->dx[a]) / (s->dt + s->dx[a]);
  }
  /* physical constants (CODATA 2018) */
  const double alpha = 7.2973525693e-3, re = 2.8179403262e-15, lC = 3.8615926796e-13;
  const double eps0 = 8.8541878128e-12, me = 9.1093837015e-31, qe = 1.602176634e-19, cl = 299792458.0;
  double lam = c->lambda_m;
  double w0 = twopi * cl / lam;
  s->n_c = eps0 * me * w0 * w0 / (qe * qe);
  s->E_S = lam / (twopi * lC);                    /* m c^2 / (hbar w0) */
  s->iES = 1.0 / s->E_S;
  s->K_N = sqrt(3.0) / twopi * alpha * s->E_S;    /* NCS rate prefactor, per 1/w0 */
  s->K_BR = s->n_c * (lam / twopi) * alpha * re * re; /* n[n_c] sigma[alpha re^2] v dt[1/w0] */
  s->key0 = (uint32_t)c->seed;
  s->key1 = (uint32_t)(c->seed >> 32) ^ (uint32_t)c->job_id;

  /* tables */
  s->n_eta = t->n_eta; s->n_xi = t->n_xi; s->n_T = t->n_T; s->n_y = t->n_y;
  s->ln_eta0 = t->ln_eta0; s->dln_eta = t->dln_eta; s->idln_eta = 1.0 / t->dln_eta;
  s->ln_T0 = t->ln_T0; s->dln_T = t->dln_T; s->idln_T = 1.0 / t->dln_T;
  s->k_cut = t->k_cut; s->iny1 = 1.0 / (double)(t->n_y - 1);
  s->h = dalloc(s->n_eta); memcpy(s->h, t->h, sizeof(double) * s->n_eta);
  s->ln_xi = dalloc(s->n_xi); memcpy(s->ln_xi, t->ln_xi, sizeof(double) * s->n_xi);
  s->ncs_cdf = dalloc((int64_t)s->n_eta * s->n_xi);
  memcpy(s->ncs_cdf, t->ncs_cdf, sizeof(double) * (size_t)s->n_eta * s->n_xi);
  s->sigma = dalloc(s->n_T); memcpy(s->sigma, t->sigma, sizeof(double) * s->n_T);
  s->br_cdf = dalloc((int64_t)s->n_T * s->n_y);
  memcpy(s->br_cdf, t->br_cdf, sizeof(double) * (size_t)s->n_T * s->n_y);
  if (c->flags & OR_BW) {
    s->n_chi = t->n_chi; s->n_xp = t->n_xp;
    s->ln_chi0 = t->ln_chi0; s->idln_chi = 1.0 / t->dln_chi;
    s->bw_lnT = dalloc(s->n_chi); memcpy(s->bw_lnT, t->bw_lnT, sizeof(double) * s->n_chi);
    s->bw_cdf = dalloc((int64_t)s->n_chi * s->n_xp);
    memcpy(s->bw_cdf, t->bw_cdf, sizeof(double) * (size_t)s->n_chi * s->n_xp);
  }
  if (c->flags & OR_BH) {
    s->n_k = t->n_k; s->n_s = t->n_s;
    s->ln_k0 = t->ln_k0; s->idln_k = 1.0 / t->dln_k;
    s->bh_sigma = dalloc(s->n_k); memcpy(s->bh_sigma, t->bh_sigma, sizeof(double) * s->n_k);
    s->bh_cdf = dalloc((int64_t)s->n_k * s->n_s);
    memcpy(s->bh_cdf, t->bh_cdf, sizeof(double) * (size_t)s->n_k * s->n_s);
  }

  /* fields */
  s->nfield = (int64_t)s->sz[0] * s->sz[1] * s->sz[2];
  for (int a = 0; a < 3; ++a) {
    s->E[a] = dalloc(s->nfield); s->En[a] = dalloc(s->nfield);
    s->B[a] = dalloc(s->nfield);
    s->J[a] = (int64_t*)calloc((size_t)s->nfield, sizeof(int64_t));
  }
  /* ions: static, n_i = n_e / q in the slab cells (Sec. III, fully or
   * partially ionised target; READING: charge enters only through n_i) */
  s->ncell_tot = (int64_t)s->n[0] * s->n[1] * s->n[2];
  s->ni = dalloc(s->ncell_tot);
  int i0 = (int)llround(c->x0_lambda / c->dx_lambda[0]);
  int i1 = i0 + (int)llround(c->thickness_lambda / c->dx_lambda[0]);
  if (i0 < 0) i0 = 0;
  if (i1 > s->n[0]) i1 = s->n[0];
  if (i1 < i0) i1 = i0;
  double nion = c->ne_over_nc / (double)c->charge_state;
  for (int k = 0; k < s->n[2]; ++k)
    for (int j = 0; j < s->n[1]; ++j)
      for (int i = i0; i < i1; ++i)
        s->ni[i + (int64_t)s->n[0] * (j + (int64_t)s->n[1] * k)] = nion;

  /* laser source plane: a current sheet at x = i_src*dx radiating a0 (READING) */
  s->i_src = 4;
  s->nsrc_y = s->act[1] ? s->n[1] : 1;
  s->nsrc_z = s->act[2] ? s->n[2] + 1 : 1;
  int64_t ns = (int64_t)s->nsrc_y * s->nsrc_z;
  s->srcA = dalloc(ns); s->srcC = dalloc(ns); s->srcS = dalloc(ns);
  {
    double w0n = c->w0_lambda * twopi;
    double xs = (double)s->i_src * s->dx[0];
    double xf = c->focus_x_lambda * twopi;
    double zz = xs - xf;
    double zR = 0.5 * w0n * w0n;
    double wz = w0n * sqrt(1.0 + (zz / zR) * (zz / zR));
    double Rinv = zz / (zz * zz + zR * zR);
    double psi = atan(zz / zR);
    for (int k = 0; k < s->nsrc_z; ++k)
      for (int j = 0; j < s->nsrc_y; ++j) {
        int64_t m = j + (int64_t)s->nsrc_y * k;
        if (c->dims == 1 || !(c->w0_lambda > 0.0)) {
          s->srcA[m] = 1.0; s->srcC[m] = 1.0; s->srcS[m] = 0.0;
          continue;
        }
        double yr = ((double)j + 0.5) * s->dx[1] - 0.5 * s->L[1];
        double r2 = yr * yr;
        double A, ph;
        if (c->dims == 3) {
          double zr = (double)k * s->dx[2] - 0.5 * s->L[2];
          r2 = r2 + zr * zr;
          A = (w0n / wz) * exp(-r2 / (wz * wz));
          ph = 0.5 * r2 * Rinv - psi;
        } else {
          A = sqrt(w0n / wz) * exp(-r2 / (wz * wz));
          ph = 0.5 * r2 * Rinv - 0.5 * psi;
        }
        s->srcA[m] = A; s->srcC[m] = cos(ph); s->srcS[m] = -sin(ph);
      }
  }

  /* electrons: ppc per slab cell, uniform-random in-cell, cold, tau0 = -ln u */
  int nslab = i1 - i0;
  s->N = (int64_t)nslab * s->n[1] * s->n[2] * c->ppc;
  s->x = dalloc(3 * s->N); s->p = dalloc(3 * s->N);
  s->tau = dalloc(s->N); s->w = dalloc(s->N);
  s->taub = (c->flags & OR_BREM_FREEPATH) ? dalloc(s->N) : NULL;
  s->id = (uint32_t*)calloc((size_t)(s->N > 0 ? s->N : 1), 4);
  s->alive = (uint8_t*)calloc((size_t)(s->N > 0 ? s->N : 1), 1);
  double wgt = c->ne_over_nc * V / (double)c->ppc;
  for (int k = 0; k < s->n[2]; ++k)
    for (int j = 0; j < s->n[1]; ++j)
      for (int i = i0; i < i1; ++i) {
        int64_t rank = ((int64_t)k * s->n[1] + j) * nslab + (i - i0);
        for (int m = 0; m < c->ppc; ++m) {
          int64_t e = rank * c->ppc + m;
          uint32_t r[4];
          or_philox((uint32_t)e, 0xFFFFFFFFu, 0u, 0u, s->key0, s->key1, r);
          s->x[3 * e + 0] = ((double)i + u32(r[0])) * s->dx[0];
          s->x[3 * e + 1] = s->act[1] ? ((double)j + u32(r[1])) * s->dx[1] : 0.0;
          s->x[3 * e + 2] = s->act[2] ? ((double)k + u32(r[2])) * s->dx[2] : 0.0;
          s->tau[e] = -or_log(u32(r[3]));
          if (s->taub) {  /* first free path, in mean free paths: -ln u */
            uint32_t rb[4];
            or_philox((uint32_t)e, 0xFFFFFFFFu, 1u, 0u, s->key0, s->key1, rb);
            s->taub[e] = -or_log(u32(rb[0]));
          }
          s->w[e] = wgt;
          s->id[e] = (uint32_t)e;
          s->alive[e] = 1;
        }
      }
  s->st.live = (uint64_t)s->N;

  /* mobile ions: ion_ppc per slab cell at uniform-random in-cell positions
   * (Philox counter (j, 0xFFFFFFFE, 0, 0)), at rest, weight n_i V / ion_ppc */
  if (c->ion_ppc > 0) {
    s->Ni = (int64_t)nslab * s->n[1] * s->n[2] * c->ion_ppc;
    s->ix = dalloc(3 * s->Ni); s->ip = dalloc(3 * s->Ni);
    s->ialive = (uint8_t*)calloc((size_t)(s->Ni > 0 ? s->Ni : 1), 1);
    s->icount = (uint32_t*)calloc((size_t)s->ncell_tot, 4);
    s->iq = (double)c->charge_state;
    s->imass = c->ion_mass;
    s->iw = nion * V / (double)c->ion_ppc;
    s->iwv = s->iw * s->invV;
    for (int k = 0; k < s->n[2]; ++k)
      for (int j = 0; j < s->n[1]; ++j)
        for (int i = i0; i < i1; ++i) {
          int64_t rank = ((int64_t)k * s->n[1] + j) * nslab + (i - i0);
          for (int m = 0; m < c->ion_ppc; ++m) {
            int64_t e = rank * c->ion_ppc + m;
            uint32_t r[4];
            or_philox((uint32_t)e, 0xFFFFFFFEu, 0u, 0u, s->key0, s->key1, r);
            s->ix[3 * e + 0] = ((double)i + u32(r[0])) * s->dx[0];
            s->ix[3 * e + 1] = s->act[1] ? ((double)j + u32(r[1])) * s->dx[1] : 0.0;
            s->ix[3 * e + 2] = s->act[2] ? ((double)k + u32(r[2])) * s->dx[2] : 0.0;
            s->ialive[e] = 1;
          }
        }
    s->st.ions_live = (uint64_t)s->Ni;
  }

  s->pcap = (int64_t)c->photon_capacity;
  s->ph_x = dalloc(3 * s->pcap); s->ph_k = dalloc(3 * s->pcap);
  s->ph_e = dalloc(s->pcap); s->ph_w = dalloc(s->pcap);
  s->ph_step = (uint32_t*)calloc((size_t)(s->pcap > 0 ? s->pcap : 1), 4);
  s->ph_parent = (uint32_t*)calloc((size_t)(s->pcap > 0 ? s->pcap : 1), 4);
  s->ph_proc = (uint32_t*)calloc((size_t)(s->pcap > 0 ? s->pcap : 1), 4);
  if (c->flags & (OR_BW | OR_BH)) {
    s->gx = dalloc(3 * s->pcap); s->gtau = dalloc(s->pcap);
    s->gst = (uint8_t*)calloc((size_t)(s->pcap > 0 ? s->pcap : 1), 1);
    s->rcap = (int64_t)c->pair_capacity;
    s->pr_x = dalloc(3 * s->rcap); s->pr_k = dalloc(3 * s->rcap);
    s->pr_em = dalloc(s->rcap); s->pr_ep = dalloc(s->rcap); s->pr_w = dalloc(s->rcap);
    s->pr_step = (uint32_t*)calloc((size_t)(s->rcap > 0 ? s->rcap : 1), 4);
    s->pr_parent = (uint32_t*)calloc((size_t)(s->rcap > 0 ? s->rcap : 1), 4);
    s->pr_pstep = (uint32_t*)calloc((size_t)(s->rcap > 0 ? s->rcap : 1), 4);
    s->pr_proc = (uint32_t*)calloc((size_t)(s->rcap > 0 ? s->rcap : 1), 4);
  }
  return s;
}

void or_destroy(or_sim* s) {
  if (!s) return;
  for (int a = 0; a < 3; ++a) { free(s->E[a]); free(s->En[a]); free(s->B[a]); free(s->J[a]); }
  free(s->ni); free(s->srcA); free(s->srcC); free(s->srcS);
  free(s->h); free(s->ln_xi); free(s->ncs_cdf); free(s->sigma); free(s->br_cdf);
  free(s->x); free(s->p); free(s->tau); free(s->taub); free(s->w); free(s->id); free(s->alive);
  free(s->ph_x); free(s->ph_k); free(s->ph_e); free(s->ph_w);
  free(s->ph_step); free(s->ph_parent); free(s->ph_proc);
  free(s->bw_lnT); free(s->bw_cdf); free(s->bh_sigma); free(s->bh_cdf);
  free(s->gx); free(s->gtau); free(s->gst);
  free(s->pr_x); free(s->pr_k); free(s->pr_em); free(s->pr_ep); free(s->pr_w);
  free(s->pr_step); free(s->pr_parent); free(s->pr_pstep); free(s->pr_proc);
  free(s->ix); free(s->ip); free(s->ialive); free(s->icount);
  free(s);
}

/* ----------------------------- fields ------------------------------------- */
/* Yee staggering: E_a is half-integer along a; B_a is half-integer along the
 * two other axes.  stag[c][a] = 1 when component c is half-integer along a. */
static const int ESTAG[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
static const int BSTAG[3][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

/* B <- B - (dt/2) curl E  (half step, on every valid B node) */
static void b_half(or_sim* s) {
  double* Ex = s->E[0]; double* Ey = s->E[1]; double* Ez = s->E[2];
  for (int c = 0; c < 3; ++c) {
    int lim[3];
    for (int a = 0; a < 3; ++a) lim[a] = s->act[a] ? (BSTAG[c][a] ? s->n[a] : s->n[a] + 1) : 1;
    double* Bc = s->B[c];
#ifdef _OPENMP
#pragma omp parallel for collapse(2) schedule(static) num_threads(s->nthreads)
#endif
    for (int k = 0; k < lim[2]; ++k)
      for (int j = 0; j < lim[1]; ++j)
        for (int i = 0; i < lim[0]; ++i) {
          int64_t m = fidx(s, i, j, k);
          double b = Bc[m];
          if (c == 0) {        /* dBx/dt = -dEz/dy + dEy/dz */
            if (s->act[1]) b = b - s->hd[1] * (Ez[fidx(s, i, j + 1, k)] - Ez[m]);
            if (s->act[2]) b = b + s->hd[2] * (Ey[fidx(s, i, j, k + 1)] - Ey[m]);
          } else if (c == 1) { /* dBy/dt = -dEx/dz + dEz/dx */
            if (s->act[2]) b = b - s->hd[2] * (Ex[fidx(s, i, j, k + 1)] - Ex[m]);
            b = b + s->hd[0] * (Ez[fidx(s, i + 1, j, k)] - Ez[m]);
          } else {             /* dBz/dt = -dEy/dx + dEx/dy */
            b = b - s->hd[0] * (Ey[fidx(s, i + 1, j, k)] - Ey[m]);
            if (s->act[1]) b = b + s->hd[1] * (Ex[fidx(s, i, j + 1, k)] - Ex[m]);
          }
          Bc[m] = b;
        }
  }
}

/* Laser source current added to J_y on the source plane: a sheet current
 * -2a/dx radiates E_y = a on both sides. */
static double src_val(const or_sim* s, int j, int k, double lsin, double lcos) {
  int64_t m = j + (int64_t)s->nsrc_y * k;
  double v = lsin * s->srcC[m] + lcos * s->srcS[m];
  return (-2.0 / s->dx[0]) * (s->srcA[m] * v);
}

/* interior Ampere update of E_c at node (i,j,k) from E (old), B, J */
static double e_interior(const or_sim* s, int c, int i, int j, int k, double lsin, double lcos) {
  int64_t m = fidx(s, i, j, k);
  const double* Bx = s->B[0]; const double* By = s->B[1]; const double* Bz = s->B[2];
  double e = s->E[c][m];
  double jj = (double)s->J[c][m] * 0x1p-40;
  if (c == 0) {        /* dEx/dt = dBz/dy - dBy/dz - Jx */
    if (s->act[1]) e = e + s->cd[1] * (Bz[m] - Bz[fidx(s, i, j - 1, k)]);
    if (s->act[2]) e = e - s->cd[2] * (By[m] - By[fidx(s, i, j, k - 1)]);
  } else if (c == 1) { /* dEy/dt = dBx/dz - dBz/dx - Jy */
    if (s->act[2]) e = e + s->cd[2] * (Bx[m] - Bx[fidx(s, i, j, k - 1)]);
    e = e - s->cd[0] * (Bz[m] - Bz[fidx(s, i - 1, j, k)]);
    if (i == s->i_src) jj = jj + src_val(s, j, k, lsin, lcos);
  } else {             /* dEz/dt = dBy/dx - dBx/dy - Jz */
    e = e + s->cd[0] * (By[m] - By[fidx(s, i - 1, j, k)]);
    if (s->act[1]) e = e - s->cd[1] * (Bx[m] - Bx[fidx(s, i, j - 1, k)]);
  }
  return e - s->dt * jj;
}

/* E^{n+1} into En: interior Yee update; first-order Mur on the faces for the
 * tangential components; nodes on two boundary faces are held at zero
 * (READING: the paper states absorbing boundaries, Sec. III). */
static void e_full(or_sim* s, double lsin, double lcos) {
  for (int c = 0; c < 3; ++c) {
    double* Fn = s->En[c];
    memset(Fn, 0, sizeof(double) * (size_t)s->nfield);
    int lim[3];
    for (int a = 0; a < 3; ++a) lim[a] = s->act[a] ? (ESTAG[c][a] ? s->n[a] : s->n[a] + 1) : 1;
    /* interior */
#ifdef _OPENMP
#pragma omp parallel for collapse(2) schedule(static) num_threads(s->nthreads)
#endif
    for (int k = 0; k < lim[2]; ++k)
      for (int j = 0; j < lim[1]; ++j)
        for (int i = 0; i < lim[0]; ++i) {
          int ijk[3] = {i, j, k}, nb = 0;
          for (int a = 0; a < 3; ++a)
            if (s->act[a] && !ESTAG[c][a] && (ijk[a] == 0 || ijk[a] == s->n[a])) ++nb;
          if (nb == 0) Fn[fidx(s, i, j, k)] = e_interior(s, c, i, j, k, lsin, lcos);
        }
    /* faces (Mur), using the already computed interior neighbour */
#ifdef _OPENMP
#pragma omp parallel for collapse(2) schedule(static) num_threads(s->nthreads)
#endif
    for (int k = 0; k < lim[2]; ++k)
      for (int j = 0; j < lim[1]; ++j)
        for (int i = 0; i < lim[0]; ++i) {
          int ijk[3] = {i, j, k}, nb = 0, ax = -1;
          for (int a = 0; a < 3; ++a)
            if (s->act[a] && !ESTAG[c][a] && (ijk[a] == 0 || ijk[a] == s->n[a])) { ++nb; ax = a; }
          if (nb != 1) continue;
          int in[3] = {i, j, k};
          in[ax] += (ijk[ax] == 0) ? 1 : -1;
          int64_t mb = fidx(s, i, j, k), mi = fidx(s, in[0], in[1], in[2]);
          Fn[mb] = s->E[c][mi] + s->cm[ax] * (Fn[mi] - s->E[c][mb]);
        }
  }
  for (int c = 0; c < 3; ++c) { double* t = s->E[c]; s->E[c] = s->En[c]; s->En[c] = t; }
}

/* linear (CIC) interpolation of one staggered component at grid coords g */
static double gather1(const or_sim* s, const double* F, const int* st, const double* g) {
  int i[3] = {0, 0, 0};
  double f[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < s->dims; ++a) {
    double ga = g[a] - 0.5 * (double)st[a];
    double fl = floor(ga);
    i[a] = (int)fl;
    f[a] = ga - fl;
  }
  if (s->dims == 1)
    return (1.0 - f[0]) * F[fidx(s, i[0], 0, 0)] + f[0] * F[fidx(s, i[0] + 1, 0, 0)];
  double v0 = (1.0 - f[0]) * F[fidx(s, i[0], i[1], i[2])] + f[0] * F[fidx(s, i[0] + 1, i[1], i[2])];
  double v1 = (1.0 - f[0]) * F[fidx(s, i[0], i[1] + 1, i[2])] + f[0] * F[fidx(s, i[0] + 1, i[1] + 1, i[2])];
  double a2 = (1.0 - f[1]) * v0 + f[1] * v1;
  if (s->dims == 2) return a2;
  double w0 = (1.0 - f[0]) * F[fidx(s, i[0], i[1], i[2] + 1)] + f[0] * F[fidx(s, i[0] + 1, i[1], i[2] + 1)];
  double w1 = (1.0 - f[0]) * F[fidx(s, i[0], i[1] + 1, i[2] + 1)] + f[0] * F[fidx(s, i[0] + 1, i[1] + 1, i[2] + 1)];
  double b2 = (1.0 - f[1]) * w0 + f[1] * w1;
  return (1.0 - f[2]) * a2 + f[2] * b2;
}

/* ------------------------ per-electron step ------------------------------- */
typedef struct {
  double x1[3], v[3];
  int nph;
  double px[2][3], pk[2][3], pe[2];
  int pproc[2], pkeep[2];
  int clamped;
} eres;

/* E and B at x (grid coordinates g = x/dx per axis) from the Yee arrays:
 * component c of E (c < 3) or of B (c >= 3). */
static double field_at(const or_sim* s, int c, const double* g) {
  return c < 3 ? gather1(s, s->E[c], ESTAG[c], g) : gather1(s, s->B[c - 3], BSTAG[c - 3], g);
}

/* Relativistic Boris push of p (q = -1, m = 1) through E, B over dt. */
static void boris(double hq, const double E[3], const double B[3], double* px, double* py, double* pz) {
  double umx = *px + hq * E[0], umy = *py + hq * E[1], umz = *pz + hq * E[2];
  double gm = sqrt(1.0 + (umx * umx + umy * umy + umz * umz));
  double fq = hq / gm;
  double tx = fq * B[0], ty = fq * B[1], tz = fq * B[2];
  double sf = 2.0 / (1.0 + (tx * tx + ty * ty + tz * tz));
  double sx = sf * tx, sy = sf * ty, sz = sf * tz;
  double upx = umx + (umy * tz - umz * ty);
  double upy = umy + (umz * tx - umx * tz);
  double upz = umz + (umx * ty - umy * tx);
  double uqx = umx + (upy * sz - upz * sy);
  double uqy = umy + (upz * sx - upx * sz);
  double uqz = umz + (upx * sy - upy * sx);
  *px = uqx + hq * E[0]; *py = uqy + hq * E[1]; *pz = uqz + hq * E[2];
}

/* Quantum parameter eta of an electron of momentum p and energy gamma in E, B:
 * the Lorentz invariant |gamma E + p x B|^2 - (p.E)^2, square-rooted and in
 * units of the Schwinger field (Sec. II.A; READING of the printed form). */
static double eta_of(const double E[3], const double B[3], double px, double py, double pz,
                     double gamma, double iES) {
  double cx = gamma * E[0] + (py * B[2] - pz * B[1]);
  double cy = gamma * E[1] + (pz * B[0] - px * B[2]);
  double cz = gamma * E[2] + (px * B[1] - py * B[0]);
  double pe = px * E[0] + py * E[1] + pz * E[2];
  double q2 = (cx * cx + cy * cy + cz * cz) - pe * pe;
  if (q2 < 0.0) q2 = 0.0;
  return sqrt(q2) * iES;
}

/* Position of eta on the NCS table: row i and fraction f in ln eta (clamped
 * to the last interval above the grid).  Returns 0 below the first point:
 * no emission there (READING). */
static int ncs_row(const or_sim* s, double eta, int* i, double* f) {
  double le = or_log(eta);
  double sl = (le - s->ln_eta0) * s->idln_eta;
  if (!(sl >= 0.0)) return 0;
  if (sl >= (double)(s->n_eta - 1)) { *i = s->n_eta - 2; *f = 1.0; }
  else { *i = (int)sl; *f = sl - (double)*i; }
  return 1;
}

/* Optical depth used up in one step: dN/dt = K_N (eta/gamma) h(eta) with h
 * linear in ln eta between table points (Sec. II.A, NCS "the same as EPOCH"). */
static double ncs_dtau(const or_sim* s, int i, double f, double eta, double gamma) {
  double h = s->h[i] + f * (s->h[i + 1] - s->h[i]);
  return s->K_N * eta / gamma * h * s->dt;
}

/* Photon fraction xi = hbar w / (gamma m c^2) at uniform u: each of the two
 * rows around eta inverted, blended in ln eta (READING). */
static double ncs_xi(const or_sim* s, int i, double f, double u) {
  double la = ncs_inv_row(s, i, u);
  double lb = ncs_inv_row(s, i + 1, u);
  double lx = la + f * (lb - la);
  return or_exp(lx);
}

/* Position of the kinetic energy T on the bremsstrahlung table: row i,
 * fraction f in ln T, ln T itself; clamps (and flags) above the last point.
 * Returns 0 below the first point. */
static int brem_row(const or_sim* s, double T, int* i, double* f, double* lt, int* clamped) {
  *lt = or_log(T);
  double sl = (*lt - s->ln_T0) * s->idln_T;
  if (!(sl >= 0.0)) return 0;
  if (sl >= (double)(s->n_T - 1)) { *i = s->n_T - 2; *f = 1.0; *clamped = 1; }
  else { *i = (int)sl; *f = sl - (double)*i; }
  return 1;
}

/* sigma(E) of Eq. (4): the Tsai cross-section of Eq. (1) integrated from the
 * photon cut to T, in alpha r_e^2, linear in ln T between table points. */
static double brem_sigma(const or_sim* s, int i, double f) {
  return s->sigma[i] + f * (s->sigma[i + 1] - s->sigma[i]);
}

/* Photon energy of a bremsstrahlung event: sigma(y, E) = R2 sigma(E) solved
 * on the two rows around T, blended in ln T, mapped from the scaled
 * coordinate between ln k_cut and ln T, capped at T (Sec. II.B; READING). */
static double brem_eps(const or_sim* s, int i, double f, double lt, double T, double u) {
  double sa = br_inv_row(s, i, u);
  double sb = br_inv_row(s, i + 1, u);
  double sv = sa + f * (sb - sa);
  double lk = or_log(s->k_cut);
  double eps = or_exp(lk + sv * (lt - lk));
  if (eps > T) eps = T;
  return eps;
}

/* Recoil of an emission of energy eps: the electron keeps its direction and
 * loses eps of its energy (READING: energy-conserving along p). */
static void recoil(double eps, double pm, double* px, double* py, double* pz, double* gamma) {
  double gn = *gamma - eps;
  double pn = sqrt((gn - 1.0) * (gn + 1.0));
  double sc = pn / pm;
  *px = *px * sc; *py = *py * sc; *pz = *pz * sc; *gamma = gn;
}

static void add_photon(eres* out, const double* x, double px, double py, double pz, double pm,
                       double eps, int proc, int keep) {
  int k = out->nph++;
  out->px[k][0] = x[0]; out->px[k][1] = x[1]; out->px[k][2] = x[2];
  out->pk[k][0] = px / pm; out->pk[k][1] = py / pm; out->pk[k][2] = pz / pm;
  out->pe[k] = eps; out->pproc[k] = proc; out->pkeep[k] = keep;
}

/* Steps in the order of the method: RNG, gather, Boris push, eta, NCS
 * (optical depth + inverse-CDF draw), bremsstrahlung (Eq. (4) test + R2 draw),
 * recoil, move.  Deposit, append and sums happen afterwards in id order. */
static void electron_one(or_sim* s, int64_t e, double tn, eres* out) {
  const or_config* c = &s->c;
  const uint32_t n = (uint32_t)s->step;
  double* x = s->x + 3 * e;
  double* p = s->p + 3 * e;
  out->nph = 0; out->clamped = 0;
  uint32_t r[4];
  or_philox(s->id[e], n, 0u, 0u, s->key0, s->key1, r);

  /* gather E^n, B^n at x^n (or prescribed fields in particle-only mode) */
  double E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
  if (c->flags & OR_FROZEN) {
    if (c->frozen_kind == OR_FROZEN_UNIFORM) {
      for (int a = 0; a < 3; ++a) { E[a] = c->frozen_E[a]; B[a] = c->frozen_B[a]; }
    } else {
      double phi = tn - x[0];
      if (phi > 0.0) { double v = c->frozen_a * sin(phi); E[1] = v; B[2] = v; }
    }
  } else {
    double g[3];
    for (int a = 0; a < 3; ++a) g[a] = x[a] * s->idx[a];
    for (int a = 0; a < 3; ++a) {
      E[a] = field_at(s, a, g);
      B[a] = field_at(s, 3 + a, g);
    }
  }

  double px = p[0], py = p[1], pz = p[2];
  boris(-0.5 * s->dt, E, B, &px, &py, &pz);
  double gamma = sqrt(1.0 + (px * px + py * py + pz * pz));
  double eta = eta_of(E, B, px, py, pz, gamma, s->iES);

  /* nonlinear Compton scattering: optical-depth decrement, one emission at
   * most per step, photon fraction from the inverse cumulative spectrum */
  int i; double f;
  if ((c->flags & OR_NCS) && ncs_row(s, eta, &i, &f)) {
    s->tau[e] = s->tau[e] - ncs_dtau(s, i, f, eta, gamma);
    if (s->tau[e] <= 0.0) {
      double eps = ncs_xi(s, i, f, u32(r[2])) * gamma;
      if (eps > gamma - 1.0) eps = gamma - 1.0;
      double pm = sqrt(px * px + py * py + pz * pz);
      add_photon(out, x, px, py, pz, pm, eps, 0, eps >= c->photon_cut_mc2);
      if (!(c->flags & OR_NO_RECOIL)) recoil(eps, pm, &px, &py, &pz, &gamma);
      s->tau[e] = -or_log(u32(r[3]));
    }
  }

  /* bremsstrahlung: Eq. (4) with n the ion density of the electron's cell,
   * sigma(E) integrated from the cut, event iff R1 < P_br (Sec. II.B).
   * Free-path form (OR_BREM_FREEPATH): the exponent X = n sigma v dt of Eq. (4)
   * is the path of the step in mean free paths, Delta s / lambda; the electron
   * carries the number of mean free paths left to its next collision,
   * exponentially distributed, and collides in the step in which that number
   * is used up.  Given no collision so far, the chance of one within a step is
   * 1 - exp(-X): the per-step law of Eq. (4), with no draw until the collision
   * (the random free path of Sec. II.B, the cheaper sampling suggested in
   * Sec. IV). */
  if (c->flags & OR_BREM) {
    double T = gamma - 1.0;
    if (T >= s->k_cut) {
      int ci[3] = {0, 0, 0};
      for (int a = 0; a < s->dims; ++a) {
        int q = (int)floor(x[a] * s->idx[a]);
        if (q < 0) q = 0;
        if (q > s->n[a] - 1) q = s->n[a] - 1;
        ci[a] = q;
      }
      double ni = s->ni[ci[0] + (int64_t)s->n[0] * (ci[1] + (int64_t)s->n[1] * ci[2])];
      double lt;
      if (ni > 0.0 && brem_row(s, T, &i, &f, &lt, &out->clamped)) {
        double sig = brem_sigma(s, i, f);
        if (sig > 0.0) {
          double pm = sqrt(px * px + py * py + pz * pz);
          double v = pm / gamma;
          double X = s->K_BR * ni * sig * v * s->dt;
          int hit;
          if (c->flags & OR_BREM_FREEPATH) {
            s->taub[e] = s->taub[e] - X;
            hit = s->taub[e] <= 0.0;
          } else {
            double P = -or_expm1(-X);
            hit = u52(r[0], r[1]) < P;
          }
          if (hit) {
            uint32_t r2[4];
            or_philox(s->id[e], n, 1u, 0u, s->key0, s->key1, r2);
            /* the next free path: word 1 of the event's second draw */
            if (c->flags & OR_BREM_FREEPATH) s->taub[e] = -or_log(u32(r2[1]));
            double eps = brem_eps(s, i, f, lt, T, u32(r2[0]));
            add_photon(out, x, px, py, pz, pm, eps, 1, 1);
            if (!(c->flags & OR_NO_RECOIL)) recoil(eps, pm, &px, &py, &pz, &gamma);
          }
        }
      }
    }
  }

  p[0] = px; p[1] = py; p[2] = pz;
  double ig = 1.0 / gamma;
  out->v[0] = px * ig; out->v[1] = py * ig; out->v[2] = pz * ig;
  for (int a = 0; a < 3; ++a)
    out->x1[a] = s->act[a] ? x[a] + out->v[a] * s->dt : x[a];
}

/* node-based linear weights of a point on a 4-node window starting at base */
static void shape4(double g, int base, double S[4]) {
  double fl = floor(g);
  int i = (int)fl;
  double f = g - fl;
  S[0] = S[1] = S[2] = S[3] = 0.0;
  S[i - base] = 1.0 - f;
  S[i - base + 1] = f;
}

/* Current accumulation in 2^-40 fixed point: every contribution is rounded to
 * the nearest multiple of 2^-40 and summed as an integer, so the total does
 * not depend on the order in which electrons are visited (READING: the paper
 * leaves the weighting procedure unspecified). */
static void jadd(int64_t* J, int64_t m, double v) {
  int64_t q = (int64_t)llrint(v * 0x1p40);
#ifdef _OPENMP
#pragma omp atomic
#endif
  J[m] += q;
}

/* charge-conserving current of one particle of charge times weight qw (-w
 * for an electron) moving x0 -> x1 (Esirkepov form; in 1D the exact 1D
 * continuity solution) */
static void deposit(or_sim* s, const double* x0, const double* x1, const double* v, double qw) {
  double c0 = qw * s->invV;
  double S0[3][4], S1[3][4];
  int b[3] = {0, 0, 0};
  for (int a = 0; a < s->dims; ++a) {
    double g0 = x0[a] * s->idx[a], g1 = x1[a] * s->idx[a];
    b[a] = (int)floor(g0) - 1;
    shape4(g0, b[a], S0[a]);
    shape4(g1, b[a], S1[a]);
  }
  int64_t* Jx = s->J[0]; int64_t* Jy = s->J[1]; int64_t* Jz = s->J[2];
  if (s->dims == 1) {
    double qx = c0 * (s->dx[0] / s->dt);
    double acc = 0.0;
    for (int i = 0; i < 3; ++i) {
      acc = acc - qx * (S1[0][i] - S0[0][i]);
      jadd(Jx, fidx(s, b[0] + i, 0, 0), acc);
    }
    double cy = c0 * v[1], cz = c0 * v[2];
    for (int i = 0; i < 4; ++i) {
      double sa = 0.5 * (S0[0][i] + S1[0][i]);
      jadd(Jy, fidx(s, b[0] + i, 0, 0), cy * sa);
      jadd(Jz, fidx(s, b[0] + i, 0, 0), cz * sa);
    }
    return;
  }
  if (s->dims == 2) {
    double qx = c0 * (s->dx[0] / s->dt), qy = c0 * (s->dx[1] / s->dt), cz = c0 * v[2];
    for (int j = 0; j < 4; ++j) {
      double acc = 0.0;
      for (int i = 0; i < 3; ++i) {
        double W = 0.5 * (S1[0][i] - S0[0][i]) * (S0[1][j] + S1[1][j]);
        acc = acc - qx * W;
        jadd(Jx, fidx(s, b[0] + i, b[1] + j, 0), acc);
      }
    }
    for (int i = 0; i < 4; ++i) {
      double acc = 0.0;
      for (int j = 0; j < 3; ++j) {
        double W = 0.5 * (S0[0][i] + S1[0][i]) * (S1[1][j] - S0[1][j]);
        acc = acc - qy * W;
        jadd(Jy, fidx(s, b[0] + i, b[1] + j, 0), acc);
      }
    }
    for (int j = 0; j < 4; ++j)
      for (int i = 0; i < 4; ++i) {
        double W = (S0[0][i] * S0[1][j] + S1[0][i] * S1[1][j]) * (1.0 / 3.0) +
                   (S0[0][i] * S1[1][j] + S1[0][i] * S0[1][j]) * (1.0 / 6.0);
        jadd(Jz, fidx(s, b[0] + i, b[1] + j, 0), cz * W);
      }
    return;
  }
  /* 3D */
  double qx = c0 * (s->dx[0] / s->dt), qy = c0 * (s->dx[1] / s->dt), qz = c0 * (s->dx[2] / s->dt);
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 4; ++j) {
      double acc = 0.0;
      for (int i = 0; i < 3; ++i) {
        double T = (S0[1][j] * S0[2][k] + S1[1][j] * S1[2][k]) * (1.0 / 3.0) +
                   (S1[1][j] * S0[2][k] + S0[1][j] * S1[2][k]) * (1.0 / 6.0);
        acc = acc - qx * ((S1[0][i] - S0[0][i]) * T);
        jadd(Jx, fidx(s, b[0] + i, b[1] + j, b[2] + k), acc);
      }
    }
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 4; ++i) {
      double acc = 0.0;
      for (int j = 0; j < 3; ++j) {
        double T = (S0[0][i] * S0[2][k] + S1[0][i] * S1[2][k]) * (1.0 / 3.0) +
                   (S1[0][i] * S0[2][k] + S0[0][i] * S1[2][k]) * (1.0 / 6.0);
        acc = acc - qy * ((S1[1][j] - S0[1][j]) * T);
        jadd(Jy, fidx(s, b[0] + i, b[1] + j, b[2] + k), acc);
      }
    }
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) {
        double T = (S0[0][i] * S0[1][j] + S1[0][i] * S1[1][j]) * (1.0 / 3.0) +
                   (S1[0][i] * S0[1][j] + S0[0][i] * S1[1][j]) * (1.0 / 6.0);
        acc = acc - qz * ((S1[2][k] - S0[2][k]) * T);
        jadd(Jz, fidx(s, b[0] + i, b[1] + j, b[2] + k), acc);
      }
    }
}

/* Ion density of every cell for the collision test of Eq. (4): the number
 * of live ions whose position lies in the cell (nearest grid cell), times
 * the ion weight over the cell volume. */
static void ion_density(or_sim* s) {
  memset(s->icount, 0, sizeof(uint32_t) * (size_t)s->ncell_tot);
  for (int64_t e = 0; e < s->Ni; ++e) {
    if (!s->ialive[e]) continue;
    int ci[3] = {0, 0, 0};
    for (int a = 0; a < s->dims; ++a) {
      int q = (int)floor(s->ix[3 * e + a] * s->idx[a]);
      if (q < 0) q = 0;
      if (q > s->n[a] - 1) q = s->n[a] - 1;
      ci[a] = q;
    }
    s->icount[ci[0] + (int64_t)s->n[0] * (ci[1] + (int64_t)s->n[1] * ci[2])]++;
  }
  for (int64_t m = 0; m < s->ncell_tot; ++m) s->ni[m] = (double)s->icount[m] * s->iwv;
}

/* Mobile ions (Sec. III): gather, Boris push with charge q and mass M (the
 * momentum is per unit mass, p/(M c)), move, charge-conserving deposit of
 * charge +q w, absorbing walls.  No photon emission. */
static void ion_step(or_sim* s, double tn, int frozen) {
  const or_config* c = &s->c;
  const double hq = 0.5 * s->dt * (s->iq / s->imass);
  double* x1 = dalloc(3 * s->Ni);
  double* vv = dalloc(3 * s->Ni);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
#endif
  for (int64_t e = 0; e < s->Ni; ++e) {
    if (!s->ialive[e]) continue;
    double* x = s->ix + 3 * e;
    double* p = s->ip + 3 * e;
    double E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
    if (frozen) {
      if (c->frozen_kind == OR_FROZEN_UNIFORM) {
        for (int a = 0; a < 3; ++a) { E[a] = c->frozen_E[a]; B[a] = c->frozen_B[a]; }
      } else {
        double phi = tn - x[0];
        if (phi > 0.0) { double v = c->frozen_a * sin(phi); E[1] = v; B[2] = v; }
      }
    } else {
      double g[3];
      for (int a = 0; a < 3; ++a) g[a] = x[a] * s->idx[a];
      for (int a = 0; a < 3; ++a) {
        E[a] = field_at(s, a, g);
        B[a] = field_at(s, 3 + a, g);
      }
    }
    double px = p[0], py = p[1], pz = p[2];
    boris(hq, E, B, &px, &py, &pz);
    double gamma = sqrt(1.0 + (px * px + py * py + pz * pz));
    p[0] = px; p[1] = py; p[2] = pz;
    double ig = 1.0 / gamma;
    double* v = vv + 3 * e;
    v[0] = px * ig; v[1] = py * ig; v[2] = pz * ig;
    for (int a = 0; a < 3; ++a)
      x1[3 * e + a] = s->act[a] ? x[a] + v[a] * s->dt : x[a];
  }
  if (!frozen) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
#endif
    for (int64_t e = 0; e < s->Ni; ++e)
      if (s->ialive[e]) deposit(s, s->ix + 3 * e, x1 + 3 * e, vv + 3 * e, s->iq * s->iw);
  }
  uint64_t live = 0;
  for (int64_t e = 0; e < s->Ni; ++e) {
    if (!s->ialive[e]) continue;
    int out = 0;
    for (int a = 0; a < s->dims; ++a) {
      s->ix[3 * e + a] = x1[3 * e + a];
      if (x1[3 * e + a] < 0.0 || x1[3 * e + a] >= s->L[a]) out = 1;
    }
    if (out) s->ialive[e] = 0; else ++live;
  }
  s->st.ions_live = live;
  free(x1);
  free(vv);
}

/* ------------------------ pair production --------------------------------- */
/* Quantum parameter of a photon of energy eps (mc^2) travelling along the
 * unit vector k in E, B: eps |E_perp + k x B| / E_S, i.e. the electron's
 * invariant with p = eps k and gamma = eps. */
static double chi_of(const double E[3], const double B[3], const double* k, double eps, double iES) {
  double cx = E[0] + (k[1] * B[2] - k[2] * B[1]);
  double cy = E[1] + (k[2] * B[0] - k[0] * B[2]);
  double cz = E[2] + (k[0] * B[1] - k[1] * B[0]);
  double ke = k[0] * E[0] + k[1] * E[1] + k[2] * E[2];
  double q2 = (cx * cx + cy * cy + cz * cz) - ke * ke;
  if (q2 < 0.0) q2 = 0.0;
  return eps * sqrt(q2) * iES;
}

/* Share of a uniform-grid CDF row on [0, 1] at u (linear between points). */
static double share_inv_row(const double* C, int n, double u) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (C[mid] <= u) lo = mid; else hi = mid;
  }
  double t = (u - C[lo]) / (C[lo + 1] - C[lo]);
  return ((double)lo + t) / (double)(n - 1);
}

/* Photons in flight.  Every recorded photon of at least 2 mc^2 travels on
 * along its direction at c from the step after its emission (Breit-Wheeler
 * and Bethe-Heitler, the pair channels the paper names beside its two; the
 * latter "similar to the bremsstrahlung", Sec. II.B):
 *   Breit-Wheeler: a pair optical depth, -ln u at the start, used up at
 *     dN/dt = alpha (m c^2 / hbar) (chi / eps) T(chi) with ln T linear in
 *     ln chi between table points (none below the first point); the photon
 *     converts when it runs out;
 *   Bethe-Heitler: the Eq. (4) trial with the pair cross-section,
 *     P = 1 - exp(-n sigma_BH(k) c dt), n the ion density of the photon's
 *     cell, against the 52-bit uniform of the step's draw;
 *   the pair energies from the inverse CDF rows (electron share for
 *   Breit-Wheeler, positron share for Bethe-Heitler), the two rows around
 *   chi or k blended in its logarithm; both members keep at least mc^2;
 *   the pair record at the photon's position, along its direction;
 *   a photon that converts stops; the others move x += k dt, and are
 *   absorbed at the walls (READINGS).
 * Random numbers: Philox counter (parent, emission step, 2 + process, n)
 * per step, (.., 0xFFFFFFFF) for the initial depth. */
static void photon_step(or_sim* s, double tn, int frozen) {
  const or_config* c = &s->c;
  const uint32_t n = (uint32_t)s->step;
  const int64_t nst = s->pcount < s->pcap ? s->pcount : s->pcap;
  const double K_P = 7.2973525693e-3 * s->E_S;   /* alpha m c^2 / (hbar w0) */
  for (int64_t q = 0; q < nst; ++q) {
    uint8_t st = s->gst[q];
    const uint32_t par = s->ph_parent[q], pst = s->ph_step[q], pr = s->ph_proc[q];
    if (st == 0) {
      if (pst == n) continue;                      /* emitted in this step */
      for (int a = 0; a < 3; ++a) s->gx[3 * q + a] = s->ph_x[3 * q + a];
      if (s->ph_e[q] >= 2.0) {
        uint32_t r0[4];
        or_philox(par, pst, 2u + pr, 0xFFFFFFFFu, s->key0, s->key1, r0);
        s->gtau[q] = -or_log(u32(r0[0]));
        st = 1;
      } else {
        st = 4;
      }
      s->gst[q] = st;
    }
    if (st != 1) continue;
    double* x = s->gx + 3 * q;
    const double* k = s->ph_k + 3 * q;
    const double eps = s->ph_e[q];
    int conv = -1, bi = 0;
    double bf = 0.0;
    uint32_t r[4];
    int have_r = 0;
    if (c->flags & OR_BW) {
      double E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
      if (frozen) {
        if (c->frozen_kind == OR_FROZEN_UNIFORM) {
          for (int a = 0; a < 3; ++a) { E[a] = c->frozen_E[a]; B[a] = c->frozen_B[a]; }
        } else {
          double phi = tn - x[0];
          if (phi > 0.0) { double v = c->frozen_a * sin(phi); E[1] = v; B[2] = v; }
        }
      } else {
        double g[3];
        for (int a = 0; a < 3; ++a) g[a] = x[a] * s->idx[a];
        for (int a = 0; a < 3; ++a) { E[a] = field_at(s, a, g); B[a] = field_at(s, 3 + a, g); }
      }
      double chi = chi_of(E, B, k, eps, s->iES);
      if (chi > 0.0) {
        double sl = (or_log(chi) - s->ln_chi0) * s->idln_chi;
        if (sl >= 0.0) {
          if (sl >= (double)(s->n_chi - 1)) { bi = s->n_chi - 2; bf = 1.0; }
          else { bi = (int)sl; bf = sl - (double)bi; }
          double lT = s->bw_lnT[bi] + bf * (s->bw_lnT[bi + 1] - s->bw_lnT[bi]);
          double dtau = K_P * chi / eps * or_exp(lT) * s->dt;
          s->gtau[q] = s->gtau[q] - dtau;
          if (s->gtau[q] <= 0.0) conv = 0;
        }
      }
    }
    int ki = 0;
    double kf = 0.0;
    if (conv < 0 && (c->flags & OR_BH)) {
      int ci[3] = {0, 0, 0};
      for (int a = 0; a < s->dims; ++a) {
        int qq = (int)floor(x[a] * s->idx[a]);
        if (qq < 0) qq = 0;
        if (qq > s->n[a] - 1) qq = s->n[a] - 1;
        ci[a] = qq;
      }
      double ni = s->ni[ci[0] + (int64_t)s->n[0] * (ci[1] + (int64_t)s->n[1] * ci[2])];
      double sl = (or_log(eps) - s->ln_k0) * s->idln_k;
      if (ni > 0.0 && sl >= 0.0) {
        if (sl >= (double)(s->n_k - 1)) { ki = s->n_k - 2; kf = 1.0; }
        else { ki = (int)sl; kf = sl - (double)ki; }
        double sig = s->bh_sigma[ki] + kf * (s->bh_sigma[ki + 1] - s->bh_sigma[ki]);
        if (sig > 0.0) {
          double X = s->K_BR * ni * sig * s->dt;
          double P = -or_expm1(-X);
          or_philox(par, pst, 2u + pr, n, s->key0, s->key1, r);
          have_r = 1;
          if (u52(r[0], r[1]) < P) conv = 1;
        }
      }
    }
    if (conv >= 0) {
      if (!have_r) or_philox(par, pst, 2u + pr, n, s->key0, s->key1, r);
      double em, ep;
      if (conv == 0) {   /* electron share xi */
        double xa = share_inv_row(s->bw_cdf + (int64_t)bi * s->n_xp, s->n_xp, u32(r[2]));
        double xb = share_inv_row(s->bw_cdf + (int64_t)(bi + 1) * s->n_xp, s->n_xp, u32(r[2]));
        double xi = xa + bf * (xb - xa);
        double lo = 1.0 / eps, hi = 1.0 - lo;
        if (xi < lo) xi = lo;
        if (xi > hi) xi = hi;
        em = xi * eps;
        ep = eps - em;
      } else {           /* positron share x on s = (x - 1/k) / (1 - 2/k) */
        double sa = share_inv_row(s->bh_cdf + (int64_t)ki * s->n_s, s->n_s, u32(r[3]));
        double sb = share_inv_row(s->bh_cdf + (int64_t)(ki + 1) * s->n_s, s->n_s, u32(r[3]));
        double sv = sa + kf * (sb - sa);
        double lo = 1.0 / eps;
        double xp = lo + sv * (1.0 - 2.0 * lo);
        ep = xp * eps;
        em = eps - ep;
      }
      s->st.pairs[conv]++;
      s->st.e_pair[conv] += s->ph_w[q] * eps;
      if (s->rcount < s->rcap) {
        int64_t m = s->rcount;
        for (int a = 0; a < 3; ++a) { s->pr_x[3 * m + a] = x[a]; s->pr_k[3 * m + a] = k[a]; }
        s->pr_em[m] = em; s->pr_ep[m] = ep; s->pr_w[m] = s->ph_w[q];
        s->pr_step[m] = n; s->pr_parent[m] = par; s->pr_pstep[m] = pst;
        s->pr_proc[m] = pr | ((uint32_t)conv << 1);
      } else {
        s->st.pairs_overflow++;
      }
      s->rcount++;
      s->gst[q] = 2;
      continue;
    }
    int out = 0;
    for (int a = 0; a < s->dims; ++a) {
      x[a] = x[a] + k[a] * s->dt;
      if (x[a] < 0.0 || x[a] >= s->L[a]) out = 1;
    }
    if (out) s->gst[q] = 3;
  }
}

/* Quarter-octave bin of a photon energy: eps = m 2^e with 1 <= m < 2 gives
 * 4 (e + 2) plus the number of the thresholds 2^(1/4), 2^(1/2), 2^(3/4)
 * (rounded to double) that m reaches; clamped to [0, 64). */
static int spectrum_bin(double eps) {
  int e;
  double m = 2.0 * frexp(eps, &e);
  e = e - 1;
  int b = 4 * (e + 2);
  if (m >= 0x1.306fe0a31b715p+0) b++;
  if (m >= 0x1.6a09e667f3bcdp+0) b++;
  if (m >= 0x1.ae89f995ad3adp+0) b++;
  if (b < 0) b = 0;
  if (b > 63) b = 63;
  return b;
}

static void laser_scalars(const or_sim* s, uint64_t step, double* lsin, double* lcos) {
  double t = ((double)step + 0.5) * s->dt;
  double TL = s->c.duration_cycles * (2.0 * M_PI);
  double env = 0.0;
  if (t >= 0.0 && t <= TL) {
    if (s->c.envelope == OR_ENV_FLAT) env = 1.0;   /* constant over the pulse (Sec. III) */
    else { env = sin(M_PI * t / TL); env = env * env; }
  }
  *lsin = s->c.a0 * env * sin(t);
  *lcos = s->c.a0 * env * cos(t);
}

void or_step(or_sim* s, int nsteps) {
  eres* res = (eres*)malloc(sizeof(eres) * (size_t)(s->N > 0 ? s->N : 1));
  const int frozen = (s->c.flags & OR_FROZEN) != 0;
  for (int it = 0; it < nsteps; ++it) {
    double tn = (double)s->step * s->dt;
    if (!frozen) {
      for (int a = 0; a < 3; ++a) memset(s->J[a], 0, sizeof(int64_t) * (size_t)s->nfield);
      b_half(s);                                  /* B^{n-1/2} -> B^n */
    }
    if (s->Ni > 0) ion_density(s);               /* n of Eq. (4) from the ions at x^n */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
#endif
    for (int64_t e = 0; e < s->N; ++e)
      if (s->alive[e]) electron_one(s, e, tn, &res[e]);
    if (s->Ni > 0) ion_step(s, tn, frozen);
    /* charge-conserving deposit of every move (integer sums: the order in
     * which electrons add to a node does not change the result) */
    if (!frozen) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
#endif
      for (int64_t e = 0; e < s->N; ++e)
        if (s->alive[e]) deposit(s, s->x + 3 * e, res[e].x1, res[e].v, -s->w[e]);
    }
    /* id-ordered pass: photon append, sums, absorbing walls */
    uint64_t live = 0;
    for (int64_t e = 0; e < s->N; ++e) {
      if (!s->alive[e]) continue;
      eres* r = &res[e];
      for (int k = 0; k < r->nph; ++k) {
        int pr = r->pproc[k];
        double we = s->w[e] * r->pe[k];
        s->st.events[pr]++;
        if (!r->pkeep[k]) { s->st.dropped_ncs++; s->st.e_rad_dropped += we; continue; }
        s->st.kept[pr]++;
        s->st.e_rad_kept[pr] += we;
        s->st.spectrum[pr][spectrum_bin(r->pe[k])]++;
        if (s->pcount < s->pcap) {
          int64_t q = s->pcount;
          for (int a = 0; a < 3; ++a) { s->ph_x[3 * q + a] = r->px[k][a]; s->ph_k[3 * q + a] = r->pk[k][a]; }
          s->ph_e[q] = r->pe[k]; s->ph_w[q] = s->w[e];
          s->ph_step[q] = (uint32_t)s->step; s->ph_parent[q] = s->id[e]; s->ph_proc[q] = (uint32_t)pr;
        } else {
          s->st.overflow++;
        }
        s->pcount++;
      }
      s->st.brem_clamped += (uint64_t)r->clamped;
      int out = 0;
      for (int a = 0; a < s->dims; ++a) {
        s->x[3 * e + a] = r->x1[a];
        if (r->x1[a] < 0.0 || r->x1[a] >= s->L[a]) out = 1;
      }
      if (out) s->alive[e] = 0; else ++live;
    }
    s->st.live = live;
    if (s->c.flags & (OR_BW | OR_BH)) photon_step(s, tn, frozen);  /* E^n, B^n, n at x^n */
    if (!frozen) {
      double ls, lc;
      laser_scalars(s, s->step, &ls, &lc);
      b_half(s);                                  /* B^n -> B^{n+1/2} */
      e_full(s, ls, lc);                          /* E^n -> E^{n+1}   */
    }
    s->step++;
    s->st.steps = s->step;
  }
  free(res);
}

/* ----------------------------- accessors ---------------------------------- */
int64_t or_num_electrons(const or_sim* s) { return s->N; }
int64_t or_num_photons(const or_sim* s) { return s->pcount; }

void or_get_electrons(const or_sim* s, double* x, double* p, double* tau,
                      double* w, uint32_t* id, uint8_t* alive) {
  memcpy(x, s->x, sizeof(double) * 3 * (size_t)s->N);
  memcpy(p, s->p, sizeof(double) * 3 * (size_t)s->N);
  memcpy(tau, s->tau, sizeof(double) * (size_t)s->N);
  memcpy(w, s->w, sizeof(double) * (size_t)s->N);
  memcpy(id, s->id, sizeof(uint32_t) * (size_t)s->N);
  memcpy(alive, s->alive, (size_t)s->N);
}

void or_get_tau_brem(const or_sim* s, double* out) {
  if (s->taub) memcpy(out, s->taub, sizeof(double) * (size_t)s->N);
}

void or_set_tau_brem(or_sim* s, const double* in) {
  if (s->taub) memcpy(s->taub, in, sizeof(double) * (size_t)s->N);
}

void or_set_electrons(or_sim* s, const double* x, const double* p, const double* tau) {
  memcpy(s->x, x, sizeof(double) * 3 * (size_t)s->N);
  memcpy(s->p, p, sizeof(double) * 3 * (size_t)s->N);
  memcpy(s->tau, tau, sizeof(double) * (size_t)s->N);
}

void or_get_photons(const or_sim* s, double* x, double* k, double* eps, double* w,
                    uint32_t* step, uint32_t* parent, uint32_t* proc) {
  int64_t n = s->pcount < s->pcap ? s->pcount : s->pcap;
  memcpy(x, s->ph_x, sizeof(double) * 3 * (size_t)n);
  memcpy(k, s->ph_k, sizeof(double) * 3 * (size_t)n);
  memcpy(eps, s->ph_e, sizeof(double) * (size_t)n);
  memcpy(w, s->ph_w, sizeof(double) * (size_t)n);
  memcpy(step, s->ph_step, 4 * (size_t)n);
  memcpy(parent, s->ph_parent, 4 * (size_t)n);
  memcpy(proc, s->ph_proc, 4 * (size_t)n);
}

void or_get_stats(const or_sim* s, or_stats* out) { *out = s->st; }

/* Test hook: n photons appended as NCS records of the coming step (they
 * start travelling one step later), with the caller's parent ids. */
void or_add_photons(or_sim* s, int64_t n, const double* x, const double* k, const double* eps,
                    const double* w, const uint32_t* parent) {
  for (int64_t j = 0; j < n; ++j) {
    if (s->pcount < s->pcap) {
      int64_t q = s->pcount;
      for (int a = 0; a < 3; ++a) { s->ph_x[3 * q + a] = x[3 * j + a]; s->ph_k[3 * q + a] = k[3 * j + a]; }
      s->ph_e[q] = eps[j]; s->ph_w[q] = w[j];
      s->ph_step[q] = (uint32_t)s->step; s->ph_parent[q] = parent[j]; s->ph_proc[q] = 0u;
    }
    s->pcount++;
  }
}

/* Test hook: the photons' state in flight (positions, pair optical depths,
 * states; min(count, capacity) of each). */
void or_get_flight(const or_sim* s, double* x, double* tau, uint8_t* st) {
  int64_t n = s->pcount < s->pcap ? s->pcount : s->pcap;
  if (!s->gx || n <= 0) return;
  memcpy(x, s->gx, sizeof(double) * 3 * (size_t)n);
  memcpy(tau, s->gtau, sizeof(double) * (size_t)n);
  memcpy(st, s->gst, (size_t)n);
}

int64_t or_num_pairs(const or_sim* s) { return s->rcount; }

void or_get_pairs(const or_sim* s, double* x, double* k, double* e_minus, double* e_plus,
                  double* w, uint32_t* step, uint32_t* parent, uint32_t* pstep, uint32_t* proc) {
  int64_t n = s->rcount < s->rcap ? s->rcount : s->rcap;
  if (n <= 0) return;
  memcpy(x, s->pr_x, sizeof(double) * 3 * (size_t)n);
  memcpy(k, s->pr_k, sizeof(double) * 3 * (size_t)n);
  memcpy(e_minus, s->pr_em, sizeof(double) * (size_t)n);
  memcpy(e_plus, s->pr_ep, sizeof(double) * (size_t)n);
  memcpy(w, s->pr_w, sizeof(double) * (size_t)n);
  memcpy(step, s->pr_step, 4 * (size_t)n);
  memcpy(parent, s->pr_parent, 4 * (size_t)n);
  memcpy(pstep, s->pr_pstep, 4 * (size_t)n);
  memcpy(proc, s->pr_proc, 4 * (size_t)n);
}

int64_t or_num_ions(const or_sim* s) { return s->Ni; }

void or_get_ions(const or_sim* s, double* x, double* p, uint8_t* alive) {
  if (s->Ni == 0) return;
  memcpy(x, s->ix, sizeof(double) * 3 * (size_t)s->Ni);
  memcpy(p, s->ip, sizeof(double) * 3 * (size_t)s->Ni);
  memcpy(alive, s->ialive, (size_t)s->Ni);
}

void or_set_ions(or_sim* s, const double* x, const double* p) {
  if (s->Ni == 0) return;
  memcpy(s->ix, x, sizeof(double) * 3 * (size_t)s->Ni);
  memcpy(s->ip, p, sizeof(double) * 3 * (size_t)s->Ni);
}

double or_ion_kinetic_energy(const or_sim* s) {
  double sum = 0.0;
  for (int64_t e = 0; e < s->Ni; ++e) {
    if (!s->ialive[e]) continue;
    const double* p = s->ip + 3 * e;
    double g = sqrt(1.0 + (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));
    sum += s->iw * s->imass * (g - 1.0);
  }
  return sum;
}

double or_kinetic_energy(const or_sim* s) {
  double sum = 0.0;
  for (int64_t e = 0; e < s->N; ++e) {
    if (!s->alive[e]) continue;
    const double* p = s->p + 3 * e;
    double g = sqrt(1.0 + (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));
    sum += s->w[e] * (g - 1.0);
  }
  return sum;
}

double or_field_energy(const or_sim* s) {
  double sum = 0.0;
  for (int c = 0; c < 3; ++c)
    for (int64_t m = 0; m < s->nfield; ++m)
      sum += s->E[c][m] * s->E[c][m] + s->B[c][m] * s->B[c][m];
  double V = 1.0 / s->invV;
  return 0.5 * sum * V;
}

int64_t or_field_size(const or_sim* s) { return s->nfield; }

void or_get_fields(const or_sim* s, double* out) {
  for (int c = 0; c < 3; ++c) memcpy(out + (int64_t)c * s->nfield, s->E[c], sizeof(double) * (size_t)s->nfield);
  for (int c = 0; c < 3; ++c) memcpy(out + (int64_t)(3 + c) * s->nfield, s->B[c], sizeof(double) * (size_t)s->nfield);
}

void or_get_current(const or_sim* s, int64_t* out) {
  for (int c = 0; c < 3; ++c) memcpy(out + (int64_t)c * s->nfield, s->J[c], sizeof(int64_t) * (size_t)s->nfield);
}

void or_get_derived(const or_sim* s, double* o) {
  o[0] = s->dx[0]; o[1] = s->dx[1]; o[2] = s->dx[2]; o[3] = s->dt;
  o[4] = s->E_S; o[5] = s->K_N; o[6] = s->K_BR; o[7] = s->n_c;
}

/* ---------------- probes of single steps (for the pins) ------------------ */
void or_set_fields(or_sim* s, const double* in) {
  for (int c = 0; c < 3; ++c) memcpy(s->E[c], in + (int64_t)c * s->nfield, sizeof(double) * (size_t)s->nfield);
  for (int c = 0; c < 3; ++c) memcpy(s->B[c], in + (int64_t)(3 + c) * s->nfield, sizeof(double) * (size_t)s->nfield);
}

double or_probe_field(const or_sim* s, int comp, const double x[3]) {
  double g[3];
  for (int a = 0; a < 3; ++a) g[a] = x[a] * s->idx[a];
  return field_at(s, comp, g);
}

void or_probe_boris(const or_sim* s, const double E[3], const double B[3], double p[3]) {
  boris(-0.5 * s->dt, E, B, &p[0], &p[1], &p[2]);
}

double or_probe_eta(const or_sim* s, const double E[3], const double B[3], const double p[3]) {
  double gamma = sqrt(1.0 + (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));
  return eta_of(E, B, p[0], p[1], p[2], gamma, s->iES);
}

double or_probe_ncs_dtau(const or_sim* s, double eta, double gamma) {
  int i; double f;
  if (!ncs_row(s, eta, &i, &f)) return 0.0;
  return ncs_dtau(s, i, f, eta, gamma);
}

double or_probe_ncs_xi(const or_sim* s, double eta, double u) {
  int i; double f;
  if (!ncs_row(s, eta, &i, &f)) return 0.0;
  return ncs_xi(s, i, f, u);
}

double or_probe_brem_sigma(const or_sim* s, double T) {
  int i, cl = 0; double f, lt;
  if (!(T >= s->k_cut) || !brem_row(s, T, &i, &f, &lt, &cl)) return 0.0;
  return brem_sigma(s, i, f);
}

double or_probe_brem_eps(const or_sim* s, double T, double u) {
  int i, cl = 0; double f, lt;
  if (!(T >= s->k_cut) || !brem_row(s, T, &i, &f, &lt, &cl)) return 0.0;
  return brem_eps(s, i, f, lt, T, u);
}
