// Internal declarations of libpic: context layout, kernel parameter blocks,
// launcher prototypes.  gfx950 (CDNA4) only: wave64, 160 KB LDS per CU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>
#include "../../include/pic.h"

namespace pic {

constexpr uint32_t kDead = 0x80000000u;   // id bit marking an absorbed electron
constexpr int kGuard = 2;                 // guard cells per side on active axes
constexpr int kBlock = 256;               // threads per block (4 waves)
constexpr int kSlotCnt = 8;               // u64 counters per wave slot
// Step-kernel workgroups go to the 8 XCDs round robin; chunks are dealt to
// them in groups of kXcdGroup consecutive chunks, and grids are padded to a
// multiple of kGridQuantum so that the deal is a bijection.
constexpr uint32_t kXcdGroup = 16;
constexpr int64_t kGridQuantum = 8 * kXcdGroup;
constexpr int kSlotSum = 6;               // doubles per wave slot (3 Neumaier pairs)
constexpr int kSpecCopies = 2048;         // copies of the kept-photon spectrum (by chunk)
constexpr double kJScale = 0x1p40;        // current fixed point: units of 2^-40
constexpr double kJInv = 0x1p-40;

// counter slots
enum { SC_ESTEPS = 0, SC_EV_NCS, SC_EV_BR, SC_KEPT_NCS, SC_KEPT_BR, SC_DROPPED, SC_CLAMPED, SC_UNTILED };

// Geometry shared by the field kernels (grid layout identical in every mode).
struct Grid {
  int dims;
  int n[3], act[3], gg[3], sz[3];
  double dx[3], idx[3], L[3];
  double dt, invV;
  double hd[3], cd[3], cm[3];   // (dt/2)/dx, dt/dx, Mur coefficients
  int i_src, nsrc_y, nsrc_z;
  int64_t nfield;               // elements per component
  int fb[3];                    // FP32 path: fraction bits of the fixed-point positions
};

// Parameter block of the field kernels (one run).
struct FieldArgs {
  int n[3], act[3], gg[3], sz[3];
  double hd[3], cd[3], cm[3], dt, srcfac;
  int i_src, nsrc_y;
  int64_t nfield;
  // node index -> (i, j, k) by multiply-shift division (nfield < 2^31):
  // q = (n * mg) >> sh equals n / d for every n < 2^31, d = sz[0] (mg0, sh0)
  // and d = sz[1] (mg1, sh1)
  uint32_t mg0, mg1;
  int sh0, sh1;
};

struct EPtrs {
  const void* E[3];
  void* En[3];
  const void* B[3];
  const unsigned long long* J[3];
  const double *srcA, *srcC, *srcS;
};

// One run's entry in a batched field launch.
struct FieldJob {
  FieldArgs A;
  EPtrs P;
  void* Bw[3];
  unsigned long long* Jw[3];
  double lsin, lcos;
};

// 64-bit FNV-1a of the bytes of the five table arrays, in declaration order
// (the pic_tables checksum).
inline uint64_t tables_checksum(const pic_tables& t) {
  uint64_t h = 0xcbf29ce484222325ull;
  auto feed = [&](const double* a, size_t n) {
    const unsigned char* b = reinterpret_cast<const unsigned char*>(a);
    for (size_t i = 0; i < n * sizeof(double); ++i) {
      h ^= b[i];
      h *= 0x100000001b3ull;
    }
  };
  feed(t.h, (size_t)t.n_eta);
  feed(t.ln_xi, (size_t)t.n_xi);
  feed(t.ncs_cdf, (size_t)t.n_eta * t.n_xi);
  feed(t.sigma, (size_t)t.n_T);
  feed(t.br_cdf, (size_t)t.n_T * t.n_y);
  return h;
}

// 64-bit FNV-1a of the bytes of the four pair-table arrays, in declaration
// order (the pic_pair_tables checksum).
inline uint64_t pair_tables_checksum(const pic_pair_tables& t) {
  uint64_t h = 0xcbf29ce484222325ull;
  auto feed = [&](const double* a, size_t n) {
    const unsigned char* b = reinterpret_cast<const unsigned char*>(a);
    for (size_t i = 0; i < n * sizeof(double); ++i) {
      h ^= b[i];
      h *= 0x100000001b3ull;
    }
  };
  feed(t.bw_lnT, (size_t)t.n_chi);
  feed(t.bw_cdf, (size_t)t.n_chi * t.n_xp);
  feed(t.bh_sigma, (size_t)t.n_k);
  feed(t.bh_cdf, (size_t)t.n_k * t.n_s);
  return h;
}

// Emission tables resident on the device (FP64 copy, FP32 copy).
// Guide of an inverse-CDF row: kGuide + 1 entries, entry b is the largest
// index j <= n - 2 with C[j] <= b / kGuide (0 if none).  A uniform u then has
// its bracket (the largest j <= n - 2 with C[j] <= u) between entries
// floor(u kGuide) and that + 1, plus one, so the search covers a few points
// instead of the whole row and returns the same bracket.  With as many
// guide entries as row points (256) the search takes at most a step or two,
// which keeps the chain of dependent table loads of an emission short.
constexpr int kGuide = 256;

struct DevTables {
  int n_eta = 0, n_xi = 0, n_T = 0, n_y = 0;
  double ln_eta0 = 0, idln_eta = 0, ln_T0 = 0, idln_T = 0, k_cut = 0, lnk = 0, iny1 = 0;
  double *h = nullptr, *lnxi = nullptr, *ncs = nullptr, *sig = nullptr, *br = nullptr;
  float *hf = nullptr, *lnxif = nullptr, *ncsf = nullptr, *sigf = nullptr, *brf = nullptr;
  // guides of the CDF rows as compared in each precision (row-major, kGuide + 1 per row)
  uint8_t *gncs = nullptr, *gncsf = nullptr, *gbr = nullptr, *gbrf = nullptr;
  // pair production (FP64 and FP32 copies)
  int n_chi = 0, n_xp = 0, n_k = 0, n_s = 0;
  double ln_chi0 = 0, idln_chi = 0, ln_k0 = 0, idln_k = 0;
  double *bwT = nullptr, *bwC = nullptr, *bhS = nullptr, *bhC = nullptr;
  float *bwTf = nullptr, *bwCf = nullptr, *bhSf = nullptr, *bhCf = nullptr;
};

// Parameters the electron-step kernel needs only on rare paths (prescribed
// fields, event sampling, photon append, statistics).  They live in device
// memory and are read with scalar loads where used, which keeps the kernel's
// argument block, and so its scalar-register pressure, small.
template <class R>
struct StepCold {
  uint32_t frozen_kind;
  double fE[3], fB[3], fa;
  double photon_cut;
  int n_xi, n_y;
  double iny1, lnk;
  const R* ncs;
  const R* lnxi;
  const R* br;
  const uint8_t* gncs;  // guides of the rows of ncs and br
  const uint8_t* gbr;
  uint64_t pcap;
  R* px[3];
  R* pk[3];
  R* pe;
  double* pw;
  uint32_t* pstep;
  uint32_t* ppar;
  uint32_t* pproc;
  unsigned long long* pcount;
  uint32_t* pfull;            // set once a reservation reached the capacity
  unsigned long long* spec;   // kept-photon spectrum, kSpecCopies x [2][PIC_SPECTRUM_BINS]
  unsigned long long* slot_cnt;
  double* slot_sum;
};

// Parameter block of the electron-step kernel (passed by value).
template <class R>
struct StepParams {
  int64_t N;
  uint32_t step, key0, key1;
  uint32_t flags;
  const StepCold<R>* cold;
  // constants in the working precision (a float holds half the scalar
  // registers of a double in the kernel's argument block)
  R dt, tn;
  // electrons
  R* x[3];
  R* p[3];
  double* tau;
  double* taub;  // collision optical depth (free-path bremsstrahlung), else null
  const double* w;
  uint32_t* id;
  // fields: Ex, Ey, Ez, Bx, By, Bz
  const R* F[6];
  unsigned long long* J[3];
  int n[3], gg[3], sz[3];
  R idx[3], L[3], dxdt[3], invV;
  const double* ni;
  // physics constants
  R iES, K_N, K_BR;
  // tables (decrement and collision test; the sampling rows are cold)
  int n_eta, n_T;
  R ln_eta0, idln_eta, ln_T0, idln_T, k_cut;
  R eta_skip;  // slightly below the first eta of the table
  const R* h;
  const R* sig;
  // cell-sorted layout: live electrons are [0, *n_active); LDS tile capacity
  const uint32_t* n_active;
  int lds_nodes;
  // FP32 path: current contributions rounded to 2^-jbits (int32 in LDS), widened
  // to the 2^-40 grid when flushed; jbits is chosen so a chunk sum fits int32
  int jbits;
  // FP32 path: positions are int32 fixed point in cell units with fb fraction
  // bits (uniform resolution 2^-fb cell over the whole box)
  int fb[3];
  float iqs[3];   // 2^-fb
  float iqd[3];   // dx 2^-fb: fixed point -> absolute position
  float mvq[3];   // dt/dx 2^fb: velocity -> fixed-point displacement per step
};

// Arguments of the tile sort (sort.hip).
struct SortArgs {
  int64_t N;
  int dims;
  int n[3], tile[3];
  double idx[3];
  int fb[3];                // FP32 fixed-point positions: cell = q >> fb
  uint32_t nkeys;           // keys of the tiles + 1 bucket for absorbed electrons
  // tile key: the low mbits bits of every axis interleaved (Morton order),
  // the remaining hb[a] high bits of each axis above them
  int mbits;
  int hb[3];
  const void* x[3];
  const void* p[3];
  const double* tau;
  const double* taub;       // null unless free-path bremsstrahlung
  const double* w;
  const uint32_t* id;
  void* x2[3];
  void* p2[3];
  double* tau2;
  double* taub2;
  double* w2;
  uint32_t* id2;
  uint32_t* key;
  uint32_t* count;
  uint32_t* offset;
  uint32_t* cursor;
  uint32_t* n_active;
};
void launch_sort(const SortArgs& A, bool fp32, hipStream_t s);

// Mobile ions (always FP64): one thread per ion, id order (never sorted).
struct IonArgs {
  int64_t Ni;
  int dims, ion_ppc, nslab, i0, ny;
  int n[3], gg[3], sz[3];
  uint32_t flags, frozen_kind, key0, key1;
  int fp32;                 // field arrays are float
  double dx[3], idx[3], L[3], dxdt[3], invV, dt;
  double hq;                // (dt / 2) (q / M)
  double qw;                // -(q w): the deposit's weight argument (charge density +q w / V)
  double iwv;               // w / V: density of one ion in its cell
  double tn;                // t^n (prescribed plane wave)
  double fE[3], fB[3], fa;
  const void* F[6];         // E^n, B^n
  unsigned long long* J[3];
  double* x[3];
  double* p[3];
  uint8_t* alive;
  uint32_t* count;          // live ions per cell (for the next step's density)
  double* ni;
  int64_t ncell;
};
void fill_ion_args(const struct Ctx& c, IonArgs& A);
void launch_ion_init(const IonArgs& A, hipStream_t s);     // load, then count
void launch_ion_recount(const IonArgs& A, hipStream_t s);  // clear and count again
void launch_ion_density(const IonArgs& A, hipStream_t s);  // ni <- count w / V, count <- 0
void launch_ion_step(const IonArgs& A, hipStream_t s);     // push, deposit, walls, count

// Photons in flight and pair production (PIC_BW / PIC_BH), precision of the
// run; one grid-stride pass over the stored photon records per step.
struct PhotonArgs {
  int dims;
  uint32_t flags, frozen_kind, step, key0, key1;
  int n[3], gg[3], sz[3];
  double idx[3], L[3], dt, tn, iES, K_P, K_BR;
  double fE[3], fB[3], fa;
  const void* F[6];           // E^n, B^n
  const double* ni;
  // photon records and their state in flight
  const unsigned long long* pcount;
  uint64_t pcap;
  const void* px[3];
  const void* pk[3];
  const void* pe;
  const double* pw;
  const uint32_t* pstep;
  const uint32_t* ppar;
  const uint32_t* pproc;
  void* gx[3];
  double* gtau;
  uint8_t* gst;
  // tables (precision of the run)
  int n_chi, n_xp, n_k, n_s;
  double ln_chi0, idln_chi, ln_k0, idln_k;
  const void* bwT;
  const void* bwC;
  const void* bhS;
  const void* bhC;
  // pair records
  uint64_t rcap;
  unsigned long long* rcount;
  uint32_t* rfull;
  void* rx[3];
  void* rk[3];
  void* rem;
  void* rep;
  double* rw;
  uint32_t* rstep;
  uint32_t* rpar;
  uint32_t* rpst;
  uint32_t* rproc;
  unsigned long long* ev;    // [2] pairs created per process
  double* esum;              // [2] sum w eps per process
};
void fill_photon_args(const struct Ctx& c, PhotonArgs& A);
void launch_photon_step(const PhotonArgs& A, bool fp32, hipStream_t s);

void launch_step(int dims, bool fp32, const void* params, hipStream_t s);
int chunk_electrons(bool fp32, int dims);   // electrons per step-kernel workgroup
// batched forms (device-resident tables of per-run entries; first[] is the
// exclusive prefix of chunks / workgroups per run, with first[njobs] = total)
void launch_step_batch(int dims, bool fp32, const void* tab, const uint32_t* first, int njobs,
                       uint32_t total, int lds_nodes, hipStream_t s);
void launch_b_both_batch(bool fp32, const FieldJob* tab, const uint32_t* first, int njobs,
                         uint32_t total, hipStream_t s);
void launch_e_full_batch(bool fp32, const FieldJob* tab, const uint32_t* first, int njobs,
                         uint32_t total, hipStream_t s);
uint32_t field_blocks(const struct Ctx& c);
void fill_field_job(const struct Ctx& c, double lsin, double lcos, FieldJob& F);
void launch_init_electrons(const struct Ctx& c, hipStream_t s);
void launch_b_both(const struct Ctx& c, hipStream_t s);
void launch_e_full(struct Ctx& c, double lsin, double lcos, hipStream_t s);
// Statistics reduction: cnt_out[kRedCnt] = the kSlotCnt slot counters, live
// electrons, live mobile ions; sum_out[kRedSum] = kept NCS, kept brem,
// dropped NCS, electron kinetic, sum (E^2 + B^2), ion kinetic energy.
constexpr int kRedCnt = kSlotCnt + 2;
constexpr int kRedSum = 6;
void launch_stats_reduce(const struct Ctx& c, unsigned long long* cnt_out, double* sum_out,
                         hipStream_t s);
void launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, uint64_t n,
                   hipStream_t s);

// Context: everything one run owns.
struct Ctx {
  pic_config cfg{};
  std::string err;
  bool broken = false;
  bool fp32 = false;
  hipStream_t stream = nullptr;
  Grid g{};
  double E_S = 0, iES = 0, K_N = 0, K_BR = 0, n_c = 0;
  uint32_t key0 = 0, key1 = 0;
  uint64_t step = 0;
  int64_t N = 0;            // electrons loaded
  int64_t Ni = 0;           // mobile ions loaded (0: static ions)
  double iw = 0, iq = 0, imass = 0;
  int i0 = 0, i1 = 0;       // slab cells [i0, i1)
  double wgt = 0;           // electron weight
  // device memory (one arena of allocations, freed in ~Ctx)
  void* E[3] = {};
  void* En[3] = {};
  void* B[3] = {};
  unsigned long long* J[3] = {};
  double* ni = nullptr;
  double* srcA = nullptr;
  double* srcC = nullptr;
  double* srcS = nullptr;
  void* x[3] = {};
  void* p[3] = {};
  double* tau = nullptr;
  double* taub = nullptr;     // free-path bremsstrahlung only
  double* w = nullptr;
  uint32_t* id = nullptr;
  double* ix[3] = {};         // mobile ions: positions (active axes), momenta per unit mass
  double* ip[3] = {};
  uint8_t* ialive = nullptr;
  uint32_t* icount = nullptr; // live ions per cell
  uint64_t pcap = 0;
  void* px[3] = {};
  void* pk[3] = {};
  void* pe = nullptr;
  double* pw = nullptr;
  uint32_t* pstep = nullptr;
  uint32_t* ppar = nullptr;
  uint32_t* pproc = nullptr;
  unsigned long long* pcount = nullptr;
  uint32_t* pfull = nullptr;  // photon buffer full (set by the step kernel)
  unsigned long long* spec = nullptr;  // kept-photon spectrum [2][PIC_SPECTRUM_BINS]
  // photons in flight and pair records (PIC_BW / PIC_BH)
  void* gx[3] = {};
  double* gtau = nullptr;
  uint8_t* gst = nullptr;
  uint64_t rcap = 0;
  void* rx[3] = {};
  void* rk[3] = {};
  void* rem = nullptr;
  void* rep = nullptr;
  double* rw = nullptr;
  uint32_t* rstep = nullptr;
  uint32_t* rpar = nullptr;
  uint32_t* rpst = nullptr;
  uint32_t* rproc = nullptr;
  unsigned long long* rcount = nullptr;   // [0] count; then rfull, ev[2], esum[2] in one block
  uint32_t* rfull = nullptr;
  unsigned long long* rev = nullptr;
  double* resum = nullptr;
  bool pair_tables_loaded = false;
  int64_t nslots = 0;
  int64_t nblocks_step = 0;   // step-kernel grid (a multiple of kGridQuantum)
  // cell-tile sort
  int sort_every = 0;
  int tile[3] = {1, 1, 1};
  uint32_t nkeys = 0;
  int key_mbits = 0;
  int key_hb[3] = {0, 0, 0};
  void* x2[3] = {};
  void* p2[3] = {};
  double* tau2 = nullptr;
  double* taub2 = nullptr;
  double* w2 = nullptr;
  uint32_t* id2 = nullptr;
  uint32_t* skey = nullptr;
  uint32_t* scount = nullptr;
  uint32_t* soffset = nullptr;
  uint32_t* scursor = nullptr;
  uint32_t* n_active = nullptr;
  int lds_nodes = 0;
  int jbits = 40;
  unsigned long long* slot_cnt = nullptr;
  double* slot_sum = nullptr;
  // reduction scratch
  unsigned long long* red_cnt = nullptr;
  double* red_sum = nullptr;
  void* cold = nullptr;       // device copy of StepCold<R>
  bool tables_loaded = false;
  // optional kernel timing (pairs of events per launch group)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;   // 0 electron step, 1 field solve, 2 sort, 3 ions, 4 photons
  size_t ev_used = 0;
  DevTables t{};
  std::vector<void*> allocs;
  ~Ctx();
  hipEvent_t prof_event();
};

}  // namespace pic
