/*
 * libpic - C ABI of the MI355X (gfx950) per-electron PIC step with Monte-Carlo
 * photon emission by nonlinear Compton scattering (NCS) and bremsstrahlung,
 * after Wan et al., arXiv:1612.07592.
 *
 * Method (one step of every live electron, in this order):
 *   field gather at x^n (Yee-staggered, linear weights)
 *   relativistic Boris push p^{n-1/2} -> p^{n+1/2}            (Sec. II.B: "particle pusher")
 *   quantum parameter eta (Lorentz invariant of Sec. II.A)
 *   NCS: optical depth tau -= dt * K_N (eta/gamma) h(eta); an emission when
 *        tau <= 0, photon fraction drawn from the tabulated inverse CDF
 *        (Sec. II.A/II.B: NCS module "the same with EPOCH")
 *   bremsstrahlung: P = 1 - exp(-n sigma(E) v dt) with n the ion density of
 *        the electron's cell; an event when R1 < P; photon energy from
 *        sigma(y,E) = R2 sigma(E)                              (Sec. II.B, Eqs. (1), (4))
 *   electron recoil along p (energy conserving), photon direction v/|v|
 *   photon-macroparticle append (NCS photons below the record cut are
 *        counted, not stored: Sec. III keeps photons >= m_e c^2)
 *   move x^{n+1} = x^n + dt p/gamma and charge-conserving current deposit
 * plus the supporting Yee field solve (B half steps around the push, E full
 * step, first-order Mur absorbing faces) and a current-sheet laser source.
 *
 * Units: lengths c/w0, time 1/w0, momentum mc, energy mc^2, field m c w0/e,
 * density n_c, with w0 = 2 pi c / lambda.  Electron charge -1.
 *
 * Conventions for every entry point:
 *   - Every call returns pic_status (PIC_OK = 0).  No C++ exception crosses
 *     the ABI.  A failed call leaves its outputs untouched.
 *   - Host pointers are read during the call only; configs and tables are
 *     copied, so the caller may free them on return.
 *   - The context owns all device memory it allocates (hipMalloc at
 *     pic_create); pic_destroy frees it.  Device pointers are exposed only by
 *     pic_get_buffers, borrowed and valid until the next step or destroy.
 *   - A context is not thread-safe; distinct contexts are independent and may
 *     be driven from different threads.
 *   - Work is enqueued on cfg->stream (a hipStream_t, NULL = the default
 *     stream).  Errors raised asynchronously by a kernel surface at the next
 *     call that synchronises (pic_emission_stats, pic_copy_*).  After a device
 *     error the context is "broken": every call except pic_destroy and
 *     pic_last_error returns PIC_ERR_DEVICE.
 */
#ifndef LIBPIC_PIC_H
#define LIBPIC_PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 2u
#define PIC_TABLES_VERSION 2u
#define PIC_SPECTRUM_BINS 64

typedef struct pic_ctx pic_ctx; /* opaque; owned by the library */

typedef enum {
  PIC_OK = 0,
  PIC_ERR_INVALID = 1,  /* bad argument or config (message in pic_last_error) */
  PIC_ERR_NOMEM = 2,    /* device allocation failed */
  PIC_ERR_DEVICE = 3,   /* HIP runtime / kernel error; context is broken */
  PIC_ERR_STATE = 4,    /* call out of order (e.g. step before tables) */
  PIC_ERR_OVERFLOW = 5, /* photon buffer full: stats valid, excess photons counted not stored */
  PIC_ERR_TABLES = 6    /* tables rejected (version, sizes, non-finite, non-monotone CDF) */
} pic_status;

enum { PIC_FP64 = 0, PIC_FP32_MIXED = 1 };

/* flags */
enum {
  PIC_NCS = 1u << 0,           /* nonlinear Compton emission on */
  PIC_BREM = 1u << 1,          /* bremsstrahlung on */
  PIC_FIELDS_FROZEN = 1u << 2, /* particle-only mode: prescribed fields, no field
                                  solve, no deposit (the benchmark mode of Sec. II.B) */
  PIC_NO_RECOIL = 1u << 4,     /* emit without changing the electron (tests only) */
  PIC_BREM_FREEPATH = 1u << 5, /* with PIC_BREM: collision by free path.  Each electron
                                  carries its collision optical depth (the mean free
                                  paths left to its next collision, -ln u at load and
                                  after each collision); a step uses up the exponent
                                  n sigma v dt of Eq. (4) and collides when it runs
                                  out.  Same per-step law as the Eq. (4) trial (Sec.
                                  II.B, random free path), no draw between collisions
                                  (Sec. IV); different random streams, so runs agree
                                  with the per-step form in distribution, not event
                                  by event.  8 more bytes per electron (16 when
                                  the electrons are re-sorted: two buffers). */
  PIC_BW = 1u << 6,            /* photons in flight: Breit-Wheeler pairs in the fields */
  PIC_BH = 1u << 7             /* photons in flight: Bethe-Heitler pairs on the nuclei */
};
/* Pair production (PIC_BW, PIC_BH; the channels the paper names beside NCS
 * and bremsstrahlung, Sec. I, II.A and II.B, where Bethe-Heitler is "similar
 * to the bremsstrahlung").  Every stored photon record of at least 2 mc^2
 * travels on along its direction at c from the step after its emission:
 *   Breit-Wheeler: a pair optical depth (-ln u at the start) used up at
 *     dN/dt = alpha (m c^2/hbar) (chi/eps) T(chi), chi = eps |E_perp + k x B|
 *     / E_S, ln T linear in ln chi between table points; converts when it
 *     runs out;
 *   Bethe-Heitler: the per-step trial of Eq. (4) with the pair
 *     cross-section, P = 1 - exp(-n sigma_BH(eps) c dt), n as for the
 *     bremsstrahlung;
 *   the pair's energies from the inverse-CDF rows of the pair tables; the
 *   pair is recorded (position, direction, electron and positron energies,
 *   weight, step, the photon's parent and emission step, process), not
 *   pushed; a photon that converts stops, the others are absorbed at the
 *   walls.  Photons beyond the photon buffer's capacity are not followed. */
enum { PIC_FROZEN_UNIFORM = 0, PIC_FROZEN_PLANE_WAVE = 1 };
/* laser temporal envelope over [0, duration]: sin^2, or constant (the flat
   30 fs pulse of Sec. III) */
enum { PIC_ENV_SIN2 = 0, PIC_ENV_FLAT = 1 };

/* Run configuration.  Lengths in laser wavelengths unless stated.
 * Electrons are loaded cold (p = 0), ppc per cell at uniform-random in-cell
 * positions from the run's Philox stream, in the slab cells
 * [round(x0/dx), round(x0/dx) + round(thickness/dx)) x all transverse cells;
 * ions fill the same cells at n_i = ne_over_nc / charge_state: static (a
 * fixed background density), or, with ion_ppc > 0, mobile macro-ions of
 * Sec. III (ion_ppc per slab cell at uniform-random in-cell positions, at
 * rest, charge charge_state, mass ion_mass_me electron masses, weight
 * n_i V / ion_ppc; Boris push, charge-conserving deposit, absorbing walls;
 * always FP64).  With mobile ions, n of Eq. (4) in a cell is the count of
 * live ions in it (nearest cell) times their weight over the cell volume,
 * taken before each step's push. */
typedef struct {
  uint32_t abi_version;     /* must be PIC_ABI_VERSION */
  uint32_t dims;            /* 1, 2 or 3 (x, then y, then z) */
  uint32_t precision;       /* PIC_FP64 or PIC_FP32_MIXED (FP32 push/gather/tables,
                               FP64 optical depth, weights and energy sums) */
  uint32_t flags;           /* PIC_* flags */
  int32_t n[3];             /* cells per axis; unused axes ignored */
  int32_t ppc;              /* electrons per slab cell, >= 1 */
  uint32_t Z;               /* nuclear charge (bremsstrahlung screening) */
  uint32_t charge_state;    /* ion charge q: n_i = n_e / q */
  uint32_t frozen_kind;     /* PIC_FROZEN_* when PIC_FIELDS_FROZEN */
  double dx_lambda[3];      /* cell size per axis */
  double cfl;               /* dt = cfl / sqrt(sum 1/dx^2), in (0, 1) */
  double lambda_m;          /* laser wavelength in metres (sets n_c, E_S, K_BR) */
  double a0;                /* peak normalised laser amplitude, linear pol. along y */
  double w0_lambda;         /* Gaussian waist (2D/3D); <= 0 means plane wave */
  double duration_cycles;   /* full length of the envelope in laser periods */
  double focus_x_lambda;    /* focal plane */
  double ne_over_nc;        /* electron density in the slab */
  double x0_lambda;         /* slab front */
  double thickness_lambda;  /* slab thickness */
  double photon_cut_mc2;    /* NCS photons below this energy are counted, not stored */
  double frozen_E[3];       /* PIC_FROZEN_UNIFORM fields */
  double frozen_B[3];
  double frozen_a;          /* PIC_FROZEN_PLANE_WAVE: E_y = B_z = a sin(t - x) for t > x */
  uint64_t photon_capacity; /* photon records the buffer holds */
  uint64_t seed;            /* Philox key = (seed_lo, seed_hi ^ job_id_lo) */
  uint64_t job_id;
  int32_t sort_every;       /* re-sort electrons by cell tile every this many steps;
                               0 = default for dims, < 0 = never (results do not
                               depend on it) */
  int32_t ion_ppc;          /* mobile macro-ions per slab cell; 0 = static ions */
  double ion_mass_me;       /* ion mass in electron masses (>= 1; mobile ions only) */
  uint64_t pair_capacity;   /* pair records the pair buffer holds (PIC_BW / PIC_BH) */
  uint32_t envelope;        /* PIC_ENV_SIN2 or PIC_ENV_FLAT */
  uint32_t reserved0;       /* must be 0 */
  void* stream;             /* hipStream_t of the HIP runtime libpic links
                               (/opt/rocm), or NULL for its default stream */
} pic_config;

/* Emission tables (host arrays, copied by pic_load_tables).
 * NCS: eta_i = exp(ln_eta0 + i dln_eta), i < n_eta; h(eta_i) is the
 *   dimensionless total rate, dN/dt = K_N (eta/gamma) h(eta) with
 *   K_N = sqrt(3)/(2 pi) alpha m c^2/(hbar w0); ncs_cdf[i*n_xi + j] is the
 *   probability that the photon fraction xi = hbar w/(gamma m c^2) is below
 *   exp(ln_xi[j]); ln_xi ascending, last value 0; rows non-decreasing,
 *   first entry > 0 (mass below the grid), last entry 1.
 * Bremsstrahlung: T_i = exp(ln_T0 + i dln_T) kinetic energy in mc^2;
 *   sigma[i] = integral of Tsai's Eq. (1) from k_cut to T_i in alpha r_e^2;
 *   br_cdf[i*n_y + j] = fraction of sigma[i] below photon energy
 *   k_cut (T_i/k_cut)^(j/(n_y-1)); rows start at 0, end at 1, non-decreasing.
 */
typedef struct {
  uint32_t version;   /* PIC_TABLES_VERSION */
  uint32_t Z;         /* must equal the config's Z */
  double k_cut_mc2;   /* bremsstrahlung photon cut (> 0) */
  int32_t n_eta, n_xi;
  double ln_eta0, dln_eta;
  const double* h;       /* n_eta */
  const double* ln_xi;   /* n_xi */
  const double* ncs_cdf; /* n_eta * n_xi */
  int32_t n_T, n_y;
  double ln_T0, dln_T;
  const double* sigma;   /* n_T */
  const double* br_cdf;  /* n_T * n_y */
  uint64_t checksum;     /* 64-bit FNV-1a of the bytes of h, ln_xi, ncs_cdf, sigma
                            and br_cdf, in that order (pic_build_tables fills it);
                            0 = not checked.  A mismatch is PIC_ERR_TABLES. */
} pic_tables;

/* Pair-production tables (host arrays, copied by pic_load_pair_tables;
 * required before pic_step when PIC_BW or PIC_BH is set).
 * Breit-Wheeler: chi_i = exp(ln_chi0 + i dln_chi), i < n_chi; bw_lnT[i] =
 *   ln T(chi_i) with T(chi) = (sqrt(3) pi chi)^-1 Int_0^1 [Int_y^inf K_{1/3}
 *   + (xi/(1-xi) + (1-xi)/xi) K_{2/3}(y)] dxi, y = 2/(3 chi xi (1-xi));
 *   bw_cdf[i*n_xp + j] = fraction of that integral below xi = j/(n_xp-1)
 *   (the electron's share of the photon energy); rows 0 .. 1.
 * Bethe-Heitler: k_i = exp(ln_k0 + i dln_k) photon energy in mc^2;
 *   bh_sigma[i] = Int dsigma/dx over 1/k < x < 1 - 1/k in alpha r_e^2 (Tsai's
 *   pair cross-section, the crossing of Eq. (1)); bh_cdf[i*n_s + j] =
 *   fraction below the positron share x = 1/k + s (1 - 2/k), s = j/(n_s-1). */
#define PIC_PAIR_TABLES_VERSION 1u
typedef struct {
  uint32_t version;          /* PIC_PAIR_TABLES_VERSION */
  uint32_t Z;                /* must equal the config's Z */
  int32_t n_chi, n_xp;       /* 128, 128 */
  double ln_chi0, dln_chi;
  const double* bw_lnT;      /* n_chi */
  const double* bw_cdf;      /* n_chi * n_xp */
  int32_t n_k, n_s;          /* 128, 64 */
  double ln_k0, dln_k;
  const double* bh_sigma;    /* n_k */
  const double* bh_cdf;      /* n_k * n_s */
  uint64_t checksum;         /* 64-bit FNV-1a of the bytes of bw_lnT, bw_cdf,
                                bh_sigma and bh_cdf, in that order; 0 = not checked */
} pic_pair_tables;

/* Emission statistics.  Energies in mc^2 times the macro-particle weight
 * unit (n_c (c/w0)^dims).  Counts are exact; sums are FP64 with Neumaier
 * compensation per wave slot, reduced in a fixed order. */
typedef struct {
  uint64_t steps;            /* steps taken so far */
  uint64_t electrons_live;   /* electrons inside the box */
  uint64_t electron_steps;   /* sum over steps of live electrons pushed */
  uint64_t events[2];        /* [0] NCS, [1] bremsstrahlung emissions */
  uint64_t kept[2];          /* photons recorded (or counted as overflow) */
  uint64_t dropped_ncs;      /* NCS photons below the record cut */
  uint64_t overflow;         /* kept photons that did not fit the buffer */
  uint64_t brem_clamped;     /* sigma evaluated above the table's last energy */
  uint64_t photons_stored;   /* records in the photon buffer */
  uint64_t untiled_steps;    /* electron-steps whose workgroup box did not fit LDS
                                (deposit and gather went to global memory) */
  double e_rad_kept[2];      /* sum w*eps of kept photons per process */
  double e_rad_dropped;      /* sum w*eps of dropped NCS photons */
  double e_kin_e;            /* sum w*(gamma-1) over live electrons (snapshot) */
  double e_field;            /* (1/2) sum (E^2 + B^2) dV (snapshot) */
  uint64_t ions_live;        /* mobile ions inside the box (0 with static ions) */
  double e_kin_i;            /* sum w M (gamma - 1) over live mobile ions (snapshot) */
  uint64_t pairs[2];         /* pairs created: [0] Breit-Wheeler, [1] Bethe-Heitler */
  uint64_t pairs_stored;     /* pair records in the pair buffer */
  uint64_t pairs_overflow;   /* pairs that did not fit the buffer */
  double e_pair[2];          /* sum w eps of the photons that converted, per process */
  uint64_t spectrum[2][PIC_SPECTRUM_BINS]; /* kept photons per process by energy, stored
                                or not: bin b holds 2^((b-8)/4) <= eps/mc^2 < 2^((b-7)/4)
                                (quarter octaves from 0.25 mc^2; the first and last
                                bins take everything below and above) */
} pic_stats;

/* ---- the five calls of the hot path ------------------------------------- */

/* Validate cfg, allocate the context's device memory and load the electrons
 * and ions on the device: the laser-target set-up of Sec. III (a slab target
 * of fully or partly ionised Al or Au at a given electron density, ppc
 * macro-electrons per cell, the laser entering from the left boundary,
 * absorbing boundaries).  On success *out owns everything.
 * Errors: PIC_ERR_INVALID (bad cfg), PIC_ERR_NOMEM, PIC_ERR_DEVICE. */
pic_status pic_create(const pic_config* cfg, pic_ctx** out);

/* Copy and check the emission tables: NCS tables of the quantum-synchrotron
 * spectrum (Sec. II.A, the emission module "the same with EPOCH"), and
 * bremsstrahlung tables of Tsai's cross-section, Eq. (1), integrated from the
 * photon cut to give sigma(E) of Eq. (4) and its cumulative rows for the R2
 * energy draw (Sec. II.B).  Required before pic_step when PIC_NCS or PIC_BREM
 * is set.  Errors: PIC_ERR_TABLES (version, Z, sizes, a non-finite value, a
 * CDF row not rising from its first entry to exactly 1, a checksum that does
 * not match the arrays), PIC_ERR_INVALID,
 * PIC_ERR_DEVICE. */
pic_status pic_load_tables(pic_ctx* ctx, const pic_tables* t);

/* Enqueue nsteps >= 0 full steps on the context's stream; returns without
 * waiting for the device.  One step of every live electron, in order:
 * gather, Boris push, eta (Sec. II.A), NCS optical depth and photon draw
 * (Sec. II.A-B), the bremsstrahlung collision test P = 1 - exp(-n sigma v dt)
 * of Eq. (4) with the photon energy from sigma(y, E) = R2 sigma(E) and the
 * cross-section of Eq. (1) (Sec. II.B), recoil, photon append (records of
 * photons >= the cut, Sec. III), move and current deposit; then the field
 * solve.  Errors: PIC_ERR_STATE (no tables while emission is on),
 * PIC_ERR_INVALID, PIC_ERR_DEVICE. */
pic_status pic_step(pic_ctx* ctx, int32_t nsteps);

/* Wait for the context's stream and return the statistics: event and photon
 * counts per process and the energy partition of Sec. III (energy radiated
 * into kept and dropped photons per process, electron kinetic energy, field
 * energy).  Returns PIC_ERR_OVERFLOW (with *out filled) when photons did not
 * fit the buffer. */
pic_status pic_emission_stats(pic_ctx* ctx, pic_stats* out);

/* Release everything the context owns (no passage of the paper: resource
 * management).  NULL is a no-op. */
void pic_destroy(pic_ctx* ctx);

/* ---- helpers (tests, tools, serving) ------------------------------------ */

/* Last error message of ctx (or, when ctx is NULL, of the last failed
 * pic_create or pic_philox_noalloc of the calling thread).  Never NULL. */
const char* pic_last_error(const pic_ctx* ctx);

/* Device bytes pic_create would allocate for cfg (tables included). */
pic_status pic_memory_required(const pic_config* cfg, uint64_t* bytes);

/* Wait until the context's stream has drained (the work of every pic_step
 * so far); surfaces asynchronous kernel errors.  libpic links the system
 * HIP runtime, which is a separate instance from the one bundled with
 * PyTorch: a torch synchronisation does not wait for libpic's work, this
 * call does. */
pic_status pic_synchronize(pic_ctx* ctx);

/* Number of macro-electrons loaded (live or not) and photon records the
 * buffer holds / photons kept so far (may exceed the capacity). */
pic_status pic_counts(pic_ctx* ctx, uint64_t* electrons, uint64_t* photons_stored,
                      uint64_t* photons_kept);

/* Copy all electrons to host arrays of pic_counts' electron count, ordered by
 * id and widened to double: x[3n] (unused axes 0), p[3n], tau[n], w[n],
 * id[n], alive[n] (0/1).  Any pointer may be NULL.  Synchronises. */
pic_status pic_copy_electrons(pic_ctx* ctx, double* x, double* p, double* tau,
                              double* w, uint32_t* id, uint8_t* alive);

/* Overwrite positions, momenta and optical depths (host arrays ordered by
 * id, layout as pic_copy_electrons).  For tests that set up beams. */
pic_status pic_set_electrons(pic_ctx* ctx, const double* x, const double* p,
                             const double* tau);

/* Mobile ions (ion_ppc > 0): their number (live or not; 0 with static
 * ions), a copy of all of them ordered by id (x[3n] with unused axes 0,
 * p[3n] the momentum per unit mass p/(M c), alive[n] 0/1; any pointer may
 * be NULL; synchronises), and an overwrite of positions and momenta (same
 * layout; the cell counts behind n of Eq. (4) are rebuilt).  Errors:
 * PIC_ERR_INVALID (no mobile ions for copy/set, null arrays for set). */
pic_status pic_ion_count(pic_ctx* ctx, uint64_t* ions);
pic_status pic_copy_ions(pic_ctx* ctx, double* x, double* p, uint8_t* alive);
pic_status pic_set_ions(pic_ctx* ctx, const double* x, const double* p);

/* Borrowed device pointers to the context's live buffers, for callers that
 * read them in place (on libpic's HIP runtime).  Valid until the next
 * pic_step, pic_step_many or pic_destroy: a step swaps the E buffers and a
 * tile sort swaps the electron buffers.  Electrons are in the library's
 * sorted order (id[] gives each one's id, with bit 31 set once absorbed);
 * in PIC_FP32_MIXED runs x[] holds int32 fixed point in cells with fb[]
 * fraction bits and p[], fields and photon x/k/eps are float, else double.
 * The field arrays use the pic_copy_fields layout; J is int64 in units of
 * 2^-40.  Unused axes and absent buffers (taub without PIC_BREM_FREEPATH)
 * are NULL.  Synchronises (the photon count is read from the device). */
typedef struct {
  uint32_t precision, dims;
  int32_t fb[3];
  uint64_t electrons, photons_stored, field_size;
  void* x[3];
  void* p[3];
  double* tau;
  double* taub;
  double* w;
  uint32_t* id;
  void* E[3];
  void* B[3];
  int64_t* J[3];
  void* photon_x[3];
  void* photon_k[3];
  void* photon_eps;
  double* photon_w;
  uint32_t* photon_step;
  uint32_t* photon_parent;
  uint32_t* photon_proc;
} pic_buffers;
pic_status pic_get_buffers(pic_ctx* ctx, pic_buffers* out);

/* Collision optical depths of PIC_BREM_FREEPATH runs, n = pic_counts'
 * electron count doubles ordered by id (copy: synchronises; set: for tests
 * that set up beams, finite values only).  PIC_ERR_STATE without the flag. */
pic_status pic_copy_brem_depth(pic_ctx* ctx, double* out);
pic_status pic_set_brem_depth(pic_ctx* ctx, const double* in);

/* Copy photon records [off, off+n) of the buffer (n <= stored - off):
 * x[3n] emission point, k[3n] unit direction, eps[n] energy (mc^2), w[n]
 * weight, step[n], parent[n] electron id, proc[n] (0 NCS, 1 brem).
 * Record order is the device append order (not deterministic). */
pic_status pic_copy_photons(pic_ctx* ctx, uint64_t off, uint64_t n, double* x,
                            double* k, double* eps, double* w, uint32_t* step,
                            uint32_t* parent, uint32_t* proc);

/* Pair production (PIC_BW / PIC_BH; PIC_ERR_STATE without them).
 * pic_load_pair_tables: copy and check the pair tables (PIC_ERR_TABLES on a
 *   wrong version, Z or size, a non-finite value, a row not rising from 0 to
 *   exactly 1, or a checksum that does not match).
 * pic_pair_counts: records in the pair buffer and pairs created so far.
 * pic_copy_pairs: pair records [off, off+n): x[3n] position, k[3n] photon
 *   direction, e_minus[n], e_plus[n] total energies (mc^2), w[n], step[n]
 *   of the conversion, parent[n] and pstep[n] the photon's parent electron
 *   and emission step, proc[n] = photon process | 2 * pair process
 *   (0 Breit-Wheeler, 1 Bethe-Heitler); device append order.
 * pic_copy_flight: the state in flight of photon records [off, off+n), in
 *   record order: position x[3n], pair optical depth tau[n], state[n]
 *   (0 not started, 1 travelling, 2 converted, 3 absorbed, 4 below 2 mc^2).
 * pic_add_photons: for tests, append n photon records (NCS, emitted in the
 *   coming step, so they start travelling one step later) with the
 *   caller's positions, unit directions, energies, weights and parent ids
 *   ((parent, step) must not repeat); PIC_ERR_OVERFLOW when the photon
 *   buffer cannot take them all (nothing is added). */
pic_status pic_load_pair_tables(pic_ctx* ctx, const pic_pair_tables* t);
pic_status pic_pair_counts(pic_ctx* ctx, uint64_t* stored, uint64_t* created);
pic_status pic_copy_pairs(pic_ctx* ctx, uint64_t off, uint64_t n, double* x, double* k,
                          double* e_minus, double* e_plus, double* w, uint32_t* step,
                          uint32_t* parent, uint32_t* pstep, uint32_t* proc);
pic_status pic_copy_flight(pic_ctx* ctx, uint64_t off, uint64_t n, double* x, double* tau,
                           uint8_t* state);
pic_status pic_add_photons(pic_ctx* ctx, uint64_t n, const double* x, const double* k,
                           const double* eps, const double* w, const uint32_t* parent);

/* Size (elements per component, guard cells included) of the field arrays
 * and a copy of Ex,Ey,Ez,Bx,By,Bz (6*size doubles) in the library layout:
 * index (i+g) + sx*((j+g) + sy*(k+g)), g = 2 on active axes.  After n steps
 * E is E^n and B is B^{n-1/2} (the leapfrog state the next step starts from). */
pic_status pic_field_size(pic_ctx* ctx, uint64_t* size);
pic_status pic_copy_fields(pic_ctx* ctx, double* out);

/* Copy the current density of the last step, J^{n+1/2}, as the library keeps
 * it: 3*size int64 values (Jx, Jy, Jz) in units of 2^-40 (n_c e c), same
 * layout as pic_copy_fields.  Zero before the first step. */
pic_status pic_copy_current(pic_ctx* ctx, int64_t* out);

/* Build the emission tables with the library's own quadrature (host, FP64).
 * Caller provides arrays of the standard sizes: h[256], ln_xi[256],
 * ncs_cdf[256*256], sigma[128], br_cdf[128*64]; *out is filled to point at
 * them.  nthreads <= 0 uses all host cores. */
pic_status pic_build_tables(uint32_t Z, double k_cut_mc2, int32_t nthreads,
                            double* h, double* ln_xi, double* ncs_cdf,
                            double* sigma, double* br_cdf, pic_tables* out);

/* Build the pair-production tables the same way: caller arrays bw_lnT[128],
 * bw_cdf[128*128], bh_sigma[128], bh_cdf[128*64]. */
pic_status pic_build_pair_tables(uint32_t Z, int32_t nthreads, double* bw_lnT, double* bw_cdf,
                                 double* bh_sigma, double* bh_cdf, pic_pair_tables* out);

/* Device Philox4x32-10 of n counters (ctr[4n]) under one key (key[2]) into
 * out[4n]; host buffers.  Exposes the generator the step kernels use. */
pic_status pic_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n);

/* pic_philox for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same generator and the same host-buffer arguments and results, staged
 * through a fixed device array the library holds (2 MiB per GPU it runs on,
 * for the life of the process) instead of per-call allocations.  Calls no
 * hipMalloc or hipFree.  n <= 65536 counters; larger n returns
 * PIC_ERR_INVALID (message in pic_last_error(NULL)).  Every call on a GPU
 * uses that GPU's one array: calls that overlap on one GPU (from several
 * threads) race and must be serialised by the caller.  Synchronous, on the
 * current device's default stream.  Errors: PIC_ERR_INVALID, PIC_ERR_DEVICE. */
pic_status pic_philox_noalloc(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n);

/* Kernel timing with HIP events recorded on the context's stream around
 * every electron-step launch, every field-solve group and every tile sort
 * (enable != 0 starts a fresh accumulation).  pic_profile_read synchronises
 * and returns the summed milliseconds and launch counts in ms5/launches5:
 * [0] electron step, [1] field solve, [2] sort, [3] mobile ions (density
 * pass and push), [4] photons in flight. */
pic_status pic_profile(pic_ctx* ctx, int32_t enable);
pic_status pic_profile_read(pic_ctx* ctx, double* ms5, uint64_t* launches5);

/* Derived constants of ctx: dx[3], dt, E_S, K_N, K_BR, n_c (8 doubles). */
pic_status pic_derived(pic_ctx* ctx, double* out8);

/* ---- batched stepping (several runs, one launch per kernel and step) ---- */

typedef struct pic_batch pic_batch; /* opaque staging for pic_step_many */

/* Staging buffers (pinned host + device) for pic_step_many on `stream`
 * (hipStream_t or NULL).  Every context passed to pic_step_many with this
 * batch must have been created on the same stream.
 * Errors: PIC_ERR_INVALID (out NULL), PIC_ERR_NOMEM, PIC_ERR_DEVICE. */
pic_status pic_batch_create(void* stream, pic_batch** out);
void pic_batch_destroy(pic_batch* b); /* NULL is a no-op; waits for its last upload */
const char* pic_batch_last_error(const pic_batch* b);

/* Advance run j of ctxs[0..njobs) by nsteps[j] >= 0 steps, all on the batch's
 * stream, returning without waiting for the device.  Step s of the call
 * issues, for the runs with nsteps[j] > s: their due tile sorts, then one
 * batched launch per kernel of the step (B half step, electron step per
 * dims and precision, B half step, E step) whose workgroups walk a table of
 * the runs' parameters (runs with mobile ions add their ion density pass
 * before, and their ion push after, the electron step, one launch each).
 * Each run's electrons, ions, fields, photons and
 * statistics end bit-identical to pic_step(ctxs[j], nsteps[j]) (up to the
 * order of photon records and of FP64 sums inside a wave slot, which no
 * result depends on beyond rounding).  The runs must be distinct.  Nothing
 * moves unless every run passes validation.
 * Errors: PIC_ERR_INVALID (bad list, duplicate run, stream mismatch),
 * PIC_ERR_STATE (a run without tables), PIC_ERR_DEVICE (every run of the
 * call is then broken). */
pic_status pic_step_many(pic_batch* b, pic_ctx* const* ctxs, const int32_t* nsteps,
                         int32_t njobs);

/* ---- serving: continuous batching of scan jobs on one device ------------ */

typedef struct pic_server pic_server; /* opaque */

typedef struct {
  uint32_t abi_version;       /* PIC_ABI_VERSION */
  int32_t max_jobs;           /* runs resident on the device at once, >= 1 */
  int32_t quantum_steps;      /* steps each resident run advances per round, >= 1 */
  uint32_t keep_finished;     /* 1: a finished run keeps its context (for read-back)
                                 until pic_server_release; 0: freed at completion */
  uint64_t hbm_reserve_bytes; /* device memory admission leaves free */
  void* stream;               /* hipStream_t every run is created on, or NULL */
} pic_server_config;

typedef struct {
  uint64_t job;          /* handle from pic_server_submit */
  int32_t status;        /* PIC_OK, PIC_ERR_OVERFLOW (stats valid) or the error
                            that ended the run (PIC_ERR_NOMEM: larger than the device) */
  int32_t steps;         /* steps requested */
  double t_submit;       /* arrival time, seconds on the server clock */
  double t_admit;        /* admission (context creation) */
  double t_finish;       /* completion observed (statistics read) */
  uint64_t device_bytes; /* pic_memory_required of the run */
  pic_stats stats;       /* statistics at completion */
} pic_job_result;

/* Free and total memory of the current device as the HIP runtime reports
 * them (hipMemGetInfo): the figure admission compares against.
 * Errors: PIC_ERR_INVALID (NULL), PIC_ERR_DEVICE. */
pic_status pic_device_memory(uint64_t* free_bytes, uint64_t* total_bytes);

/* Create a server (one pic_batch on sc->stream).  Errors: PIC_ERR_INVALID. */
pic_status pic_server_create(const pic_server_config* sc, pic_server** out);
/* Destroy the server and every context it still holds.  NULL is a no-op. */
void pic_server_destroy(pic_server* s);
/* Seconds since pic_server_create (monotonic). */
double pic_server_clock(const pic_server* s);
const char* pic_server_last_error(const pic_server* s);

/* Queue a job: a run of cfg (cfg->stream is replaced by the server's) for
 * nsteps steps, with tables t (deep-copied; NULL if no emission is on).
 * t_arrival < 0 stamps the current server time, otherwise it is taken as the
 * arrival time for latency.  Thread-safe with respect to pic_server_run.
 * Jobs may have mobile ions; pair production (PIC_BW / PIC_BH) is refused,
 * since a job carries no pair tables.
 * Errors: PIC_ERR_INVALID (bad cfg: nothing queued), PIC_ERR_TABLES. */
pic_status pic_server_submit(pic_server* s, const pic_config* cfg, const pic_tables* t,
                             int32_t nsteps, double t_arrival, uint64_t* job);

/* One scheduling round: admit waiting jobs in arrival order while a slot is
 * free and hipMemGetInfo's free memory covers the job's
 * pic_memory_required plus the reserve; advance every resident run by up to
 * quantum_steps steps with one pic_step_many call; wait for the device and
 * retire the runs that are done.  Returns the resident and waiting counts
 * after the round.  A device error ends every resident run with that
 * status.  Call from one thread. */
pic_status pic_server_run(pic_server* s, int32_t* resident, int32_t* queued);

/* Move up to max finished jobs into out (completion order); *n = count. */
pic_status pic_server_poll(pic_server* s, pic_job_result* out, int32_t max, int32_t* n);

/* Borrow the context of a finished job (keep_finished = 1) for pic_copy_*;
 * valid until pic_server_release or pic_server_destroy.
 * Errors: PIC_ERR_STATE (unknown, unfinished or released job). */
pic_status pic_server_job_ctx(pic_server* s, uint64_t job, pic_ctx** ctx);
pic_status pic_server_release(pic_server* s, uint64_t job);

#ifdef __cplusplus
}
#endif
#endif /* LIBPIC_PIC_H */
