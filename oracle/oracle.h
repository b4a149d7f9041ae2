/*
 * FP64 CPU oracle for the per-electron PIC step with Monte-Carlo photon
 * emission (Wan et al., "Photon emission by bremsstrahlung and nonlinear
 * Compton scattering in the interaction of ultraintense laser and plasmas").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may build, load or call this code.
 * It shares no code, header or helper with the HIP library; the two agree only
 * through the written method (the paper's equations plus the readings listed
 * in the design notes) and through the caller-supplied tables and configs.
 *
 * Units are normalised to the laser: length c/w0, time 1/w0, momentum mc,
 * energy mc^2, field m c w0 / e, density n_c.  Charge of the electron is -1.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

/* OR_BREM_FREEPATH: bremsstrahlung by a per-electron free path (collision
 * optical depth) instead of a fresh Eq. (4) trial every step; the same
 * per-step event law, see electron_one. */
/* OR_BW / OR_BH: recorded photons of at least 2 mc^2 travel on at c and may
 * turn into an electron-positron pair, in the fields (Breit-Wheeler) or on a
 * nucleus (Bethe-Heitler); see photon_step. */
enum { OR_NCS = 1, OR_BREM = 2, OR_FROZEN = 4, OR_NO_RECOIL = 16, OR_BREM_FREEPATH = 32,
       OR_BW = 64, OR_BH = 128 };
enum { OR_FROZEN_UNIFORM = 0, OR_FROZEN_PLANE_WAVE = 1 };

typedef struct {
  int32_t dims, flags, frozen_kind, ppc;
  int32_t n[3];
  int32_t Z, charge_state;
  double dx_lambda[3];
  double cfl, lambda_m;
  double a0, w0_lambda, duration_cycles, focus_x_lambda;
  double ne_over_nc, x0_lambda, thickness_lambda;
  double photon_cut_mc2;
  double frozen_E[3], frozen_B[3], frozen_a;
  uint64_t seed, job_id, photon_capacity;
  /* mobile ions (paper Sec. III): ion_ppc per slab cell (0 = static ions),
   * charge charge_state, mass ion_mass in electron masses */
  int32_t ion_ppc, envelope;          /* envelope: OR_ENV_SIN2 or OR_ENV_FLAT */
  double ion_mass;
  uint64_t pair_capacity;             /* pair records held (OR_BW / OR_BH) */
} or_config;
enum { OR_ENV_SIN2 = 0, OR_ENV_FLAT = 1 };

typedef struct {
  int32_t n_eta, n_xi;
  double ln_eta0, dln_eta;
  const double *h, *ln_xi, *ncs_cdf;   /* n_eta, n_xi, n_eta*n_xi */
  int32_t n_T, n_y;
  double ln_T0, dln_T, k_cut;
  const double *sigma, *br_cdf;        /* n_T, n_T*n_y */
  /* pair production (read only with OR_BW / OR_BH):
   * Breit-Wheeler ln T(chi) on chi_i = exp(ln_chi0 + i dln_chi) and CDF rows
   * of the electron share xi on the uniform grid j/(n_xp-1) of [0, 1];
   * Bethe-Heitler sigma(k) in alpha r_e^2 on k_i = exp(ln_k0 + i dln_k) and
   * CDF rows of the positron share on s = (x - 1/k)/(1 - 2/k), uniform grid */
  int32_t n_chi, n_xp;
  double ln_chi0, dln_chi;
  const double *bw_lnT, *bw_cdf;       /* n_chi, n_chi*n_xp */
  int32_t n_k, n_s;
  double ln_k0, dln_k;
  const double *bh_sigma, *bh_cdf;     /* n_k, n_k*n_s */
} or_tables;

typedef struct {
  uint64_t steps, live, events[2], kept[2], dropped_ncs, overflow, brem_clamped;
  double e_rad_kept[2], e_rad_dropped;
  uint64_t ions_live;
  uint64_t pairs[2];                   /* [0] Breit-Wheeler, [1] Bethe-Heitler */
  uint64_t pairs_overflow;             /* pairs not stored (buffer full) */
  double e_pair[2];                    /* sum w eps of the converted photons */
  /* kept photons per process by energy: bin b holds 2^((b-8)/4) <= eps <
   * 2^((b-7)/4) (mc^2), the first and last bins open */
  uint64_t spectrum[2][64];
} or_stats;

typedef struct or_sim or_sim;

or_sim*  or_create(const or_config* c, const or_tables* t, int nthreads);
void     or_destroy(or_sim* s);
void     or_step(or_sim* s, int nsteps);
int64_t  or_num_electrons(const or_sim* s);
int64_t  or_num_photons(const or_sim* s);          /* may exceed capacity */
void     or_get_electrons(const or_sim* s, double* x, double* p, double* tau,
                          double* w, uint32_t* id, uint8_t* alive);
void     or_set_electrons(or_sim* s, const double* x, const double* p,
                          const double* tau);
/* collision optical depths of the free-path form (id order); no-ops without
 * OR_BREM_FREEPATH */
void     or_get_tau_brem(const or_sim* s, double* out);
void     or_set_tau_brem(or_sim* s, const double* in);
void     or_get_photons(const or_sim* s, double* x, double* k, double* eps,
                        double* w, uint32_t* step, uint32_t* parent,
                        uint32_t* proc);
void     or_get_stats(const or_sim* s, or_stats* out);
/* pair records (min(count, capacity) of them): position, photon direction,
 * electron and positron total energies (mc^2), weight, step, the photon's
 * parent electron and emission step, and proc = photon process | 2 * pair
 * process (0 Breit-Wheeler, 1 Bethe-Heitler) */
int64_t  or_num_pairs(const or_sim* s);          /* may exceed capacity */
/* test hooks: append photons as NCS records of the coming step (they start
 * travelling a step later); read the state in flight (0 not started,
 * 1 travelling, 2 converted, 3 left the box, 4 below 2 mc^2) */
void     or_add_photons(or_sim* s, int64_t n, const double* x, const double* k,
                        const double* eps, const double* w, const uint32_t* parent);
void     or_get_flight(const or_sim* s, double* x, double* tau, uint8_t* st);
void     or_get_pairs(const or_sim* s, double* x, double* k, double* e_minus,
                      double* e_plus, double* w, uint32_t* step, uint32_t* parent,
                      uint32_t* pstep, uint32_t* proc);
double   or_kinetic_energy(const or_sim* s);
double   or_field_energy(const or_sim* s);
/* full field arrays incl. guard cells, component order Ex,Ey,Ez,Bx,By,Bz */
int64_t  or_field_size(const or_sim* s);
void     or_get_fields(const or_sim* s, double* out);
/* J^{n+1/2} of the last step in 2^-40 fixed point, 3*size values */
void     or_get_current(const or_sim* s, int64_t* out);
void     or_get_derived(const or_sim* s, double* out8);  /* dx[3], dt, E_S, K_N, K_BR, n_c */
void     or_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                   uint32_t k0, uint32_t k1, uint32_t out[4]);

/* Probes of single steps of the method, on a run's tables and fields (test
 * pins only).  field: component comp (0..2 E, 3..5 B) at position x by the
 * gather of the step; boris: one push of p over the run's dt; eta: the quantum
 * parameter of momentum p in E, B; ncs_dtau: the optical depth one step uses
 * up (0 below the table); ncs_xi: the photon fraction at uniform u;
 * brem_sigma: sigma(T) in alpha r_e^2 (0 below the cut or the table);
 * brem_eps: the photon energy at uniform u. */
void     or_set_fields(or_sim* s, const double* in);   /* 6*size: Ex,Ey,Ez,Bx,By,Bz */
double   or_math(int which, double x);                 /* 0 exp, 1 log, 2 expm1 of the oracle */
/* mobile ions: count, state in id order (x, p per unit mass, alive),
 * sum w M (gamma - 1) over live ions */
int64_t  or_num_ions(const or_sim* s);
void     or_get_ions(const or_sim* s, double* x, double* p, uint8_t* alive);
void     or_set_ions(or_sim* s, const double* x, const double* p);
double   or_ion_kinetic_energy(const or_sim* s);
double   or_probe_field(const or_sim* s, int comp, const double x[3]);
void     or_probe_boris(const or_sim* s, const double E[3], const double B[3], double p[3]);
double   or_probe_eta(const or_sim* s, const double E[3], const double B[3], const double p[3]);
double   or_probe_ncs_dtau(const or_sim* s, double eta, double gamma);
double   or_probe_ncs_xi(const or_sim* s, double eta, double u);
double   or_probe_brem_sigma(const or_sim* s, double T);
double   or_probe_brem_eps(const or_sim* s, double T, double u);

#endif
