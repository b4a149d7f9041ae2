// libpic host runtime: the C ABI of include/pic.h.
// Validation, device allocation, per-step kernel sequencing on the context's
// stream, statistics read-back and the test/tool helpers.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <new>
#include <mutex>
#include <string>
#include <utility>
#include <vector>
#include "pic_internal.hpp"
#include "philox.hpp"
#include "fpmath.hpp"

namespace pic {
int sort_scratch_words(uint32_t nkeys);
int reduce_scratch_cnt();
int reduce_scratch_sum();

Ctx::~Ctx() {
  for (void* p : allocs) { hipError_t e = hipFree(p); (void)e; }
  for (hipEvent_t ev : ev_pool) { hipError_t e = hipEventDestroy(ev); (void)e; }
}

// Timing events skip the system-scope fence on record: that fence writes back
// and invalidates the caches between launches, which both adds to the measured
// interval and slows the launch after it.  pic_profile_read synchronises the
// stream before it reads the events.
hipEvent_t Ctx::prof_event() {
  if (ev_used == ev_pool.size()) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    ev_pool.push_back(ev);
  }
  return ev_pool[ev_used++];
}
}  // namespace pic

using namespace pic;

struct pic_ctx {
  Ctx c;
  uint64_t injected = 0;  // photon records added by pic_add_photons (not kept by the method)
};

static thread_local std::string g_create_err;

#define FAIL(ctx, code, ...)                                   \
  do {                                                         \
    char _b[512];                                              \
    snprintf(_b, sizeof(_b), __VA_ARGS__);                     \
    (ctx).err = _b;                                            \
    return code;                                               \
  } while (0)

#define HIPCHK(ctx, expr)                                                          \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      (ctx).err = std::string(#expr) + ": " + hipGetErrorString(_e);               \
      (ctx).broken = true;                                                         \
      return PIC_ERR_DEVICE;                                                       \
    }                                                                              \
  } while (0)

namespace {

size_t real_size(const pic_config& c) { return c.precision == PIC_FP32_MIXED ? 4 : 8; }

bool is_fin(double v) { return std::isfinite(v); }

// Fills grid geometry and derived constants; returns an error message or "".
std::string derive(const pic_config& cfg, Ctx& c) {
  if (cfg.abi_version != PIC_ABI_VERSION) return "abi_version mismatch";
  if (cfg.dims < 1 || cfg.dims > 3) return "dims must be 1, 2 or 3";
  if (cfg.precision != PIC_FP64 && cfg.precision != PIC_FP32_MIXED) return "unknown precision";
  if (cfg.flags & ~(uint32_t)(PIC_NCS | PIC_BREM | PIC_FIELDS_FROZEN | PIC_NO_RECOIL | PIC_BREM_FREEPATH |
                              PIC_BW | PIC_BH))
    return "unknown flag bits";
  if ((cfg.flags & PIC_BREM_FREEPATH) && !(cfg.flags & PIC_BREM)) return "PIC_BREM_FREEPATH needs PIC_BREM";
  if (cfg.ppc < 1) return "ppc must be >= 1";
  if (cfg.Z < 1 || cfg.Z > 120) return "Z out of range";
  if (cfg.charge_state < 1 || cfg.charge_state > cfg.Z) return "charge_state must be in [1, Z]";
  if (!(cfg.cfl > 0.0 && cfg.cfl < 1.0)) return "cfl must be in (0, 1)";
  if (!(cfg.lambda_m > 0.0) || !is_fin(cfg.lambda_m)) return "lambda_m must be > 0";
  if (!is_fin(cfg.a0) || !is_fin(cfg.w0_lambda) || !is_fin(cfg.duration_cycles) ||
      !is_fin(cfg.focus_x_lambda) || !is_fin(cfg.frozen_a))
    return "non-finite laser parameter";
  if (!(cfg.ne_over_nc >= 0.0) || !is_fin(cfg.ne_over_nc)) return "ne_over_nc must be finite and >= 0";
  if (!is_fin(cfg.x0_lambda) || !(cfg.thickness_lambda >= 0.0) || !is_fin(cfg.thickness_lambda))
    return "bad slab geometry";
  if (!(cfg.photon_cut_mc2 >= 0.0) || !is_fin(cfg.photon_cut_mc2)) return "photon_cut_mc2 must be >= 0";
  for (int a = 0; a < 3; ++a)
    if (!is_fin(cfg.frozen_E[a]) || !is_fin(cfg.frozen_B[a])) return "non-finite frozen field";
  if (cfg.frozen_kind > PIC_FROZEN_PLANE_WAVE) return "unknown frozen_kind";
  if (cfg.photon_capacity > (1ull << 40)) return "photon_capacity too large";
  if (cfg.pair_capacity > (1ull << 36)) return "pair_capacity too large";
  if (cfg.envelope > PIC_ENV_FLAT) return "unknown envelope";
  if (cfg.ion_ppc < 0 || cfg.ion_ppc > 4096) return "ion_ppc must be in [0, 4096]";
  if (cfg.ion_ppc > 0 && !(cfg.ion_mass_me >= 1.0 && is_fin(cfg.ion_mass_me)))
    return "ion_mass_me must be finite and >= 1 with mobile ions";
  Grid& g = c.g;
  g.dims = (int)cfg.dims;
  const double twopi = 2.0 * M_PI;
  for (int a = 0; a < 3; ++a) {
    g.act[a] = a < g.dims;
    if (g.act[a]) {
      if (cfg.n[a] < 8 || cfg.n[a] > (1 << 24)) return "cells per axis must be in [8, 2^24]";
      if (!(cfg.dx_lambda[a] > 0.0) || !is_fin(cfg.dx_lambda[a])) return "dx must be > 0";
    }
    g.n[a] = g.act[a] ? cfg.n[a] : 1;
    g.gg[a] = g.act[a] ? kGuard : 0;
    g.sz[a] = g.act[a] ? g.n[a] + 1 + 2 * kGuard : 1;
    g.dx[a] = g.act[a] ? cfg.dx_lambda[a] * twopi : 1.0;
    g.idx[a] = 1.0 / g.dx[a];
    g.L[a] = (double)g.n[a] * g.dx[a];
  }
  double q = 0.0;
  for (int a = 0; a < g.dims; ++a) q = q + 1.0 / (g.dx[a] * g.dx[a]);
  g.dt = cfg.cfl / sqrt(q);
  double V = 1.0;
  for (int a = 0; a < g.dims; ++a) V = V * g.dx[a];
  g.invV = 1.0 / V;
  for (int a = 0; a < 3; ++a) {
    g.hd[a] = (0.5 * g.dt) / g.dx[a];
    g.cd[a] = g.dt / g.dx[a];
    g.cm[a] = (g.dt - g.dx[a]) / (g.dt + g.dx[a]);
  }
  g.i_src = 4;
  g.nsrc_y = g.act[1] ? g.n[1] : 1;
  g.nsrc_z = g.act[2] ? g.n[2] + 1 : 1;
  g.nfield = (int64_t)g.sz[0] * g.sz[1] * g.sz[2];
  if (g.nfield >= (int64_t)1 << 31) return "grid too large (nodes per field component must stay below 2^31)";
  // CODATA 2018
  const double alpha = 7.2973525693e-3, re = 2.8179403262e-15, lC = 3.8615926796e-13;
  const double eps0 = 8.8541878128e-12, me = 9.1093837015e-31, qe = 1.602176634e-19, cl = 299792458.0;
  const double lam = cfg.lambda_m;
  const double w0 = twopi * cl / lam;
  c.n_c = eps0 * me * w0 * w0 / (qe * qe);
  c.E_S = lam / (twopi * lC);
  c.iES = 1.0 / c.E_S;
  c.K_N = sqrt(3.0) / twopi * alpha * c.E_S;
  c.K_BR = c.n_c * (lam / twopi) * alpha * re * re;
  c.key0 = (uint32_t)cfg.seed;
  c.key1 = (uint32_t)(cfg.seed >> 32) ^ (uint32_t)cfg.job_id;
  int i0 = (int)llround(cfg.x0_lambda / cfg.dx_lambda[0]);
  int i1 = i0 + (int)llround(cfg.thickness_lambda / cfg.dx_lambda[0]);
  if (i0 < 0) i0 = 0;
  if (i1 > g.n[0]) i1 = g.n[0];
  if (i1 < i0) i1 = i0;
  c.i0 = i0;
  c.i1 = i1;
  const int64_t N = (int64_t)(i1 - i0) * g.n[1] * g.n[2] * cfg.ppc;
  if (N >= (int64_t)kDead) return "too many electrons (ids are 31-bit)";
  if (g.i_src + 2 >= g.n[0]) return "grid too short for the laser source plane";
  c.N = N;
  c.wgt = cfg.ne_over_nc * V / (double)cfg.ppc;
  // mobile ions: ion_ppc per slab cell, weight n_i V / ion_ppc
  const int64_t Ni = (int64_t)(i1 - i0) * g.n[1] * g.n[2] * cfg.ion_ppc;
  if (Ni >= ((int64_t)1 << 31)) return "too many ions (more than 2^31 - 1)";
  c.Ni = Ni;
  c.iq = (double)cfg.charge_state;
  c.imass = cfg.ion_mass_me;
  c.iw = cfg.ion_ppc > 0 ? (cfg.ne_over_nc / (double)cfg.charge_state) * V / (double)cfg.ion_ppc : 0.0;
  c.fp32 = cfg.precision == PIC_FP32_MIXED;
  c.pcap = cfg.photon_capacity;
  c.rcap = (cfg.flags & (PIC_BW | PIC_BH)) ? cfg.pair_capacity : 0;
  const int64_t per_chunk = chunk_electrons(c.fp32, g.dims);
  c.nblocks_step = ((N + per_chunk - 1) / per_chunk + kGridQuantum - 1) / kGridQuantum * kGridQuantum;
  c.nslots = c.nblocks_step * (kBlock / 64);
  // FP32 positions: int32 fixed point in cells; n << fb stays below 2^30 so a
  // move of less than a cell past either wall cannot overflow, and fb <= 24
  // keeps the in-cell fraction exact in a float
  for (int a = 0; a < 3; ++a) {
    int bits = 0;
    while ((1 << bits) < g.n[a]) ++bits;
    g.fb[a] = g.act[a] ? std::min(24, 30 - bits) : 0;
  }
  // cell tiles for the sort and the LDS box of the step kernel
  if (cfg.reserved0 != 0) return "reserved0 must be 0";
  const int dflt_every[4] = {0, 16, 8, 4};
  const int tiles[4] = {0, 16, 4, 2};
  // LDS box capacity in nodes (2D: fields + current, 36 B/node in FP32;
  // 3D: current only, 12 B/node); chosen by measurement on the 2D and 3D
  // gold-slab workloads
  const int ldsn[4] = {0, 64, 576, 2048};
  c.sort_every = cfg.sort_every == 0 ? dflt_every[g.dims] : (cfg.sort_every < 0 ? 0 : cfg.sort_every);
  c.lds_nodes = ldsn[g.dims];
  // FP32 current quantum: the largest 2^-jbits (jbits <= 40) with which the
  // sum of one chunk's contributions to a node stays below 2^30 in int32
  {
    double vmax = cfg.ne_over_nc / (double)cfg.ppc;   // |c0| = w / V
    double dxdt = 1.0;
    for (int a = 0; a < g.dims; ++a) dxdt = std::max(dxdt, g.dx[a] / g.dt);
    vmax = vmax * dxdt * 1.5 + 1e-30;                 // |W| <= 1, |acc| <= 1.5, |v| < 1
    c.jbits = 40;
    while (c.jbits > 0 && (double)kBlock * vmax * ldexp(1.0, c.jbits) >= ldexp(1.0, 30)) --c.jbits;
    // (particle-only runs deposit nothing)
    if (c.fp32 && c.jbits < 8 && !(cfg.flags & PIC_FIELDS_FROZEN))
      return "electron weight too large for the FP32 current quantum";
  }
  // tuning overrides (layout only; results do not depend on them)
  if (const char* v = getenv("PIC_TUNE_LDS_NODES")) c.lds_nodes = atoi(v) & ~1;
  int tile_edge = tiles[g.dims];
  if (const char* v = getenv("PIC_TUNE_TILE")) tile_edge = atoi(v) > 0 ? atoi(v) : tile_edge;
  // tile keys: Morton order over the bits all axes share, the extra high
  // bits of the longer axes on top, so a 2:1 grid of tiles needs 2^(bx+by)
  // keys rather than the 2^(2 bx) of a square Morton range
  int ntl[3] = {1, 1, 1}, bits[3] = {0, 0, 0}, bmin = 31, btot = 0;
  for (int a = 0; a < g.dims; ++a) {
    c.tile[a] = tile_edge;
    ntl[a] = (g.n[a] + c.tile[a] - 1) / c.tile[a];
    while ((1 << bits[a]) < ntl[a]) ++bits[a];
    bmin = std::min(bmin, bits[a]);
    btot += bits[a];
  }
  c.key_mbits = g.dims == 1 ? 0 : bmin;
  for (int a = 0; a < 3; ++a) c.key_hb[a] = a < g.dims ? bits[a] - c.key_mbits : 0;
  if (g.dims == 1) c.nkeys = (uint32_t)ntl[0] + 1;
  else if (btot > 30 || bmin > (g.dims == 2 ? 15 : 10)) return "grid too large for the tile sort";
  else c.nkeys = (1u << btot) + 1;
  return "";
}

// Every device buffer of a context, in allocation order.
struct Plan {
  struct Item { void** dst; size_t bytes; };
  std::vector<Item> items;
  uint64_t total = 0;
  void add(void** dst, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    items.push_back({dst, bytes});
    total += bytes;
  }
};

Plan make_plan(Ctx& c) {
  Plan P;
  const size_t rs = c.fp32 ? 4 : 8;
  const Grid& g = c.g;
  const size_t nf = (size_t)g.nfield;
  for (int a = 0; a < 3; ++a) {
    P.add(&c.E[a], nf * rs);
    P.add(&c.En[a], nf * rs);
    P.add(&c.B[a], nf * rs);
    P.add((void**)&c.J[a], nf * 8);
  }
  const size_t ncell = (size_t)g.n[0] * g.n[1] * g.n[2];
  P.add((void**)&c.ni, ncell * 8);
  const size_t ns = (size_t)g.nsrc_y * g.nsrc_z;
  P.add((void**)&c.srcA, ns * 8);
  P.add((void**)&c.srcC, ns * 8);
  P.add((void**)&c.srcS, ns * 8);
  const size_t N = (size_t)(c.N > 0 ? c.N : 1);
  for (int a = 0; a < 3; ++a) {
    if (a < g.dims) P.add(&c.x[a], N * rs);
    P.add(&c.p[a], N * rs);
  }
  P.add((void**)&c.tau, N * 8);
  const bool fp = (c.cfg.flags & PIC_BREM_FREEPATH) != 0;
  if (fp) P.add((void**)&c.taub, N * 8);
  P.add((void**)&c.w, N * 8);
  P.add((void**)&c.id, N * 4);
  if (c.Ni > 0) {
    const size_t Ni = (size_t)c.Ni;
    for (int a = 0; a < 3; ++a) {
      if (a < g.dims) P.add((void**)&c.ix[a], Ni * 8);
      P.add((void**)&c.ip[a], Ni * 8);
    }
    P.add((void**)&c.ialive, Ni);
    P.add((void**)&c.icount, ncell * 4);
  }
  if (c.sort_every > 0) {  // second SoA buffer and sort scratch
    for (int a = 0; a < 3; ++a) {
      if (a < g.dims) P.add(&c.x2[a], N * rs);
      P.add(&c.p2[a], N * rs);
    }
    P.add((void**)&c.tau2, N * 8);
    if (fp) P.add((void**)&c.taub2, N * 8);
    P.add((void**)&c.w2, N * 8);
    P.add((void**)&c.id2, N * 4);
    P.add((void**)&c.skey, N * 4);
    P.add((void**)&c.scount, (size_t)c.nkeys * 4);
    P.add((void**)&c.soffset, (size_t)c.nkeys * 4);
    P.add((void**)&c.scursor, ((size_t)c.nkeys + sort_scratch_words(c.nkeys)) * 4);
  }
  P.add((void**)&c.n_active, 16);  // live count, count being built, count before the last sort
  const size_t pc = (size_t)(c.pcap > 0 ? c.pcap : 1);
  for (int a = 0; a < 3; ++a) {
    P.add(&c.px[a], pc * rs);
    P.add(&c.pk[a], pc * rs);
  }
  P.add(&c.pe, pc * rs);
  P.add((void**)&c.pw, pc * 8);
  P.add((void**)&c.pstep, pc * 4);
  P.add((void**)&c.ppar, pc * 4);
  P.add((void**)&c.pproc, pc * 4);
  P.add((void**)&c.pcount, 8);
  P.add((void**)&c.pfull, 4);   // a line of its own: read by every chunk, written once
  P.add((void**)&c.spec, (size_t)kSpecCopies * 2 * PIC_SPECTRUM_BINS * 8);
  if (c.cfg.flags & (PIC_BW | PIC_BH)) {  // photons in flight, pair records
    for (int a = 0; a < 3; ++a) P.add(&c.gx[a], pc * rs);
    P.add((void**)&c.gtau, pc * 8);
    P.add((void**)&c.gst, pc);
    const size_t rc = (size_t)(c.rcap > 0 ? c.rcap : 1);
    for (int a = 0; a < 3; ++a) {
      P.add(&c.rx[a], rc * rs);
      P.add(&c.rk[a], rc * rs);
    }
    P.add(&c.rem, rc * rs);
    P.add(&c.rep, rc * rs);
    P.add((void**)&c.rw, rc * 8);
    P.add((void**)&c.rstep, rc * 4);
    P.add((void**)&c.rpar, rc * 4);
    P.add((void**)&c.rpst, rc * 4);
    P.add((void**)&c.rproc, rc * 4);
    P.add((void**)&c.rcount, 8);
    P.add((void**)&c.rfull, 4);
    P.add((void**)&c.rev, 16);
    P.add((void**)&c.resum, 16);
  }
  const size_t nsl = (size_t)(c.nslots > 0 ? c.nslots : 1);
  P.add((void**)&c.slot_cnt, nsl * kSlotCnt * 8);
  P.add((void**)&c.slot_sum, nsl * kSlotSum * 8);
  P.add((void**)&c.red_cnt, (size_t)reduce_scratch_cnt() * 8);
  P.add((void**)&c.red_sum, (size_t)reduce_scratch_sum() * 8);
  P.add(&c.cold, std::max(sizeof(StepCold<double>), sizeof(StepCold<float>)));
  // tables: FP64 and FP32 copies of the standard-size tables
  const size_t tb = (256 + 256 + 256 * 256 + 128 + 128 * 64);
  P.total += tb * 12 + 10 * 256 + 4 * (((256 + 128) * (kGuide + 1) + 255) & ~(size_t)255);
  return P;
}

// Transverse profile of the laser source (host, once): amplitude, cos and
// -sin of the focusing phase of a Gaussian beam at the source plane.
void source_profile(const pic_config& cfg, const Grid& g, std::vector<double>& A,
                    std::vector<double>& C, std::vector<double>& S) {
  const int ny = g.nsrc_y, nz = g.nsrc_z;
  A.assign((size_t)ny * nz, 1.0);
  C.assign((size_t)ny * nz, 1.0);
  S.assign((size_t)ny * nz, 0.0);
  if (g.dims == 1 || !(cfg.w0_lambda > 0.0)) return;
  const double twopi = 2.0 * M_PI;
  const double w0n = cfg.w0_lambda * twopi;
  const double xs = (double)g.i_src * g.dx[0];
  const double xf = cfg.focus_x_lambda * twopi;
  const double zz = xs - xf;
  const double zR = 0.5 * w0n * w0n;
  const double wz = w0n * sqrt(1.0 + (zz / zR) * (zz / zR));
  const double Rinv = zz / (zz * zz + zR * zR);
  const double psi = atan(zz / zR);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      const size_t m = (size_t)j + (size_t)ny * k;
      const double yr = ((double)j + 0.5) * g.dx[1] - 0.5 * g.L[1];
      double r2 = yr * yr;
      double amp, ph;
      if (g.dims == 3) {
        const double zr = (double)k * g.dx[2] - 0.5 * g.L[2];
        r2 = r2 + zr * zr;
        amp = (w0n / wz) * exp(-r2 / (wz * wz));
        ph = 0.5 * r2 * Rinv - psi;
      } else {
        amp = sqrt(w0n / wz) * exp(-r2 / (wz * wz));
        ph = 0.5 * r2 * Rinv - 0.5 * psi;
      }
      A[m] = amp;
      C[m] = cos(ph);
      S[m] = -sin(ph);
    }
}

// a0 env(t) sin t and a0 env(t) cos t at the source time of step n, (n+1/2) dt.
void laser_scalars(const Ctx& c, uint64_t step, double* ls, double* lc) {
  const double t = ((double)step + 0.5) * c.g.dt;
  const double TL = c.cfg.duration_cycles * (2.0 * M_PI);
  double env = 0.0;
  if (t >= 0.0 && t <= TL) {
    if (c.cfg.envelope == PIC_ENV_FLAT) {
      env = 1.0;  // constant over the pulse (Sec. III)
    } else {
      env = sin(M_PI * t / TL);
      env = env * env;
    }
  }
  *ls = c.cfg.a0 * env * sin(t);
  *lc = c.cfg.a0 * env * cos(t);
}

template <class R>
void fill_step_params(Ctx& c, StepParams<R>& P) {
  const Grid& g = c.g;
  P.N = c.N;
  P.step = (uint32_t)c.step;
  P.key0 = c.key0;
  P.key1 = c.key1;
  P.flags = c.cfg.flags;
  P.cold = (const StepCold<R>*)c.cold;
  P.dt = g.dt;
  P.tn = (double)c.step * g.dt;
  for (int a = 0; a < 3; ++a) {
    P.x[a] = (R*)c.x[a];
    P.p[a] = (R*)c.p[a];
    P.F[a] = (const R*)c.E[a];
    // the push gathers B^n, which the B pass leaves in En (free until the E step)
    P.F[3 + a] = (const R*)((c.cfg.flags & PIC_FIELDS_FROZEN) ? c.B[a] : c.En[a]);
    P.J[a] = c.J[a];
    P.n[a] = g.n[a];
    P.gg[a] = g.gg[a];
    P.sz[a] = g.sz[a];
    P.idx[a] = g.idx[a];
    P.L[a] = g.L[a];
    P.dxdt[a] = g.dx[a] / g.dt;
  }
  P.tau = c.tau;
  P.taub = c.taub;
  P.w = c.w;
  P.id = c.id;
  P.invV = g.invV;
  P.ni = c.ni;
  P.iES = c.iES;
  P.K_N = c.K_N;
  P.K_BR = c.K_BR;
  const DevTables& t = c.t;
  P.n_eta = t.n_eta; P.n_T = t.n_T;
  P.ln_eta0 = t.ln_eta0; P.idln_eta = t.idln_eta; P.ln_T0 = t.ln_T0; P.idln_T = t.idln_T;
  P.k_cut = t.k_cut;
  P.eta_skip = t.n_eta > 0 ? exp(t.ln_eta0) * (1.0 - 1e-6) : 0.0;
  if (sizeof(R) == 8) {
    P.h = (const R*)t.h;
    P.sig = (const R*)t.sig;
  } else {
    P.h = (const R*)t.hf;
    P.sig = (const R*)t.sigf;
  }
  P.n_active = c.n_active;
  P.lds_nodes = c.lds_nodes;
  P.jbits = c.jbits;
  for (int a = 0; a < 3; ++a) {
    P.fb[a] = g.fb[a];
    P.iqs[a] = (float)ldexp(1.0, -g.fb[a]);
    P.iqd[a] = (float)(g.dx[a] * ldexp(1.0, -g.fb[a]));
    P.mvq[a] = (float)(g.dt * g.idx[a] * ldexp(1.0, g.fb[a]));
  }
}

template <class R>
void fill_step_cold(const Ctx& c, StepCold<R>& C) {
  C.frozen_kind = c.cfg.frozen_kind;
  for (int a = 0; a < 3; ++a) {
    C.fE[a] = c.cfg.frozen_E[a];
    C.fB[a] = c.cfg.frozen_B[a];
    C.px[a] = (R*)c.px[a];
    C.pk[a] = (R*)c.pk[a];
  }
  C.fa = c.cfg.frozen_a;
  C.photon_cut = c.cfg.photon_cut_mc2;
  const DevTables& t = c.t;
  C.n_xi = t.n_xi;
  C.n_y = t.n_y;
  C.iny1 = t.iny1;
  C.lnk = t.lnk;
  if (sizeof(R) == 8) {
    C.ncs = (const R*)t.ncs; C.lnxi = (const R*)t.lnxi; C.br = (const R*)t.br;
    C.gncs = t.gncs; C.gbr = t.gbr;
  } else {
    C.ncs = (const R*)t.ncsf; C.lnxi = (const R*)t.lnxif; C.br = (const R*)t.brf;
    C.gncs = t.gncsf; C.gbr = t.gbrf;
  }
  C.pcap = c.pcap;
  C.pe = (R*)c.pe;
  C.pw = c.pw;
  C.pstep = c.pstep;
  C.ppar = c.ppar;
  C.pproc = c.pproc;
  C.pcount = c.pcount;
  C.pfull = c.pfull;
  C.spec = c.spec;
  C.slot_cnt = c.slot_cnt;
  C.slot_sum = c.slot_sum;
}

// (Re)write the device copy of the cold block; called at creation and when
// tables are loaded (the stream is drained first: kernels may be reading it).
pic_status upload_cold(Ctx& c) {
  HIPCHK(c, hipStreamSynchronize(c.stream));
  if (c.fp32) {
    StepCold<float> C{};
    fill_step_cold(c, C);
    HIPCHK(c, hipMemcpy(c.cold, &C, sizeof(C), hipMemcpyHostToDevice));
  } else {
    StepCold<double> C{};
    fill_step_cold(c, C);
    HIPCHK(c, hipMemcpy(c.cold, &C, sizeof(C), hipMemcpyHostToDevice));
  }
  return PIC_OK;
}

bool sort_due(const Ctx& c) { return c.sort_every > 0 && c.step % (uint64_t)c.sort_every == 0; }

// Sort of the electron SoA into the second buffer set (swap_sorted then
// makes the sorted copy current).
SortArgs sort_args(const Ctx& c) {
  SortArgs A{};
  A.N = c.N;
  A.dims = c.g.dims;
  for (int a = 0; a < 3; ++a) {
    A.n[a] = c.g.n[a];
    A.tile[a] = c.tile[a];
    A.idx[a] = c.g.idx[a];
    A.fb[a] = c.g.fb[a];
    A.x[a] = c.x[a]; A.p[a] = c.p[a]; A.x2[a] = c.x2[a]; A.p2[a] = c.p2[a];
  }
  A.nkeys = c.nkeys;
  A.mbits = c.key_mbits;
  for (int a = 0; a < 3; ++a) A.hb[a] = c.key_hb[a];
  A.tau = c.tau; A.w = c.w; A.id = c.id;
  A.tau2 = c.tau2; A.w2 = c.w2; A.id2 = c.id2;
  A.taub = c.taub; A.taub2 = c.taub2;
  A.key = c.skey; A.count = c.scount; A.offset = c.soffset; A.cursor = c.scursor;
  A.n_active = c.n_active;
  return A;
}

void swap_sorted(Ctx& c) {
  for (int a = 0; a < 3; ++a) { std::swap(c.x[a], c.x2[a]); std::swap(c.p[a], c.p2[a]); }
  std::swap(c.tau, c.tau2); std::swap(c.w, c.w2); std::swap(c.id, c.id2);
  std::swap(c.taub, c.taub2);
}

pic_status step_ready(Ctx& c, int32_t nsteps) {
  if (nsteps < 0) FAIL(c, PIC_ERR_INVALID, "nsteps < 0");
  if ((c.cfg.flags & (PIC_NCS | PIC_BREM)) && !c.tables_loaded)
    FAIL(c, PIC_ERR_STATE, "emission enabled but no tables loaded");
  if ((c.cfg.flags & (PIC_BW | PIC_BH)) && !c.pair_tables_loaded)
    FAIL(c, PIC_ERR_STATE, "pair production enabled but no pair tables loaded");
  if (c.step + (uint64_t)nsteps >= 0xFFFFFFFFull) FAIL(c, PIC_ERR_INVALID, "step counter exhausted");
  return PIC_OK;
}

pic_status check_ctx(pic_ctx* ctx) {
  if (!ctx) return PIC_ERR_INVALID;
  if (ctx->c.broken) return PIC_ERR_DEVICE;
  return PIC_OK;
}

}  // namespace

namespace {
template <class R>
pic_status copy_real(Ctx& c, const void* dev, size_t n, std::vector<double>& out) {
  std::vector<R> tmp(n);
  HIPCHK(c, hipMemcpyAsync(tmp.data(), dev, n * sizeof(R), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  out.resize(n);
  for (size_t i = 0; i < n; ++i) out[i] = (double)tmp[i];
  return PIC_OK;
}
pic_status copy_any(Ctx& c, const void* dev, size_t n, std::vector<double>& out) {
  return c.fp32 ? copy_real<float>(c, dev, n, out) : copy_real<double>(c, dev, n, out);
}
}  // namespace

// Staging of the per-run parameter tables of pic_step_many: built on the host
// for the whole call, uploaded with one copy, read by the batched kernels.
struct pic_batch {
  hipStream_t stream = nullptr;
  std::string err;
  unsigned char* host = nullptr;   // pinned
  size_t host_cap = 0;
  unsigned char* dev = nullptr;
  size_t dev_cap = 0;
  hipEvent_t uploaded = nullptr;   // the last upload has left the pinned buffer
  bool pending = false;
  std::vector<unsigned char> stage;
  ~pic_batch() {
    (void)hipStreamSynchronize(stream);  // kernels may still read the tables
    if (pending && uploaded) (void)hipEventSynchronize(uploaded);
    if (uploaded) (void)hipEventDestroy(uploaded);
    if (host) (void)hipHostFree(host);
    if (dev) (void)hipFree(dev);
  }
};

namespace {

struct BatchLaunch {
  int kind;          // 0 sort, 1 both B half steps + clear J, 2 electron step, 4 E step,
                     // 5 ion density, 6 ion step, 7 photons in flight (one run each)
  int dims = 0;
  bool fp32 = false;
  size_t tab = 0, first = 0;
  int njobs = 0;
  uint32_t total = 0;
  int lds_nodes = 0;
  SortArgs sort{};
  IonArgs ion{};
  PhotonArgs ph{};
  hipStream_t stream = nullptr;
};

size_t stage_put(std::vector<unsigned char>& st, const void* src, size_t n) {
  const size_t off = (st.size() + 255) & ~(size_t)255;
  st.resize(off + n);
  std::memcpy(st.data() + off, src, n);
  return off;
}

template <class R>
void stage_step_group(std::vector<unsigned char>& st, std::vector<BatchLaunch>& L,
                      std::vector<Ctx*>& jobs, int dims) {
  std::vector<StepParams<R>> tab;
  std::vector<uint32_t> first{0u};
  int lds = 0;
  for (Ctx* c : jobs) {
    if (c->g.dims != dims || c->fp32 != (sizeof(R) == 4) || c->N <= 0) continue;
    StepParams<R> P{};
    fill_step_params(*c, P);
    tab.push_back(P);
    const int64_t per_chunk = chunk_electrons(c->fp32, dims);
    first.push_back(first.back() + (uint32_t)((c->N + per_chunk - 1) / per_chunk));
    lds = std::max(lds, c->lds_nodes);
  }
  if (tab.empty()) return;
  BatchLaunch b{};
  b.kind = 2;
  b.dims = dims;
  b.fp32 = sizeof(R) == 4;
  b.tab = stage_put(st, tab.data(), tab.size() * sizeof(StepParams<R>));
  b.first = stage_put(st, first.data(), first.size() * sizeof(uint32_t));
  b.njobs = (int)tab.size();
  b.total = first.back();
  b.lds_nodes = lds;
  L.push_back(b);
}

}  // namespace

extern "C" {

const char* pic_last_error(const pic_ctx* ctx) {
  if (!ctx) return g_create_err.c_str();
  return ctx->c.err.c_str();
}

pic_status pic_memory_required(const pic_config* cfg, uint64_t* bytes) {
  if (!cfg || !bytes) return PIC_ERR_INVALID;
  Ctx tmp;
  tmp.cfg = *cfg;
  const std::string e = derive(*cfg, tmp);
  if (!e.empty()) {
    g_create_err = e;
    return PIC_ERR_INVALID;
  }
  *bytes = make_plan(tmp).total;
  return PIC_OK;
}

pic_status pic_create(const pic_config* cfg, pic_ctx** out) {
  if (!cfg || !out) {
    g_create_err = "null argument";
    return PIC_ERR_INVALID;
  }
  pic_ctx* ctx = new (std::nothrow) pic_ctx;
  if (!ctx) {
    g_create_err = "host allocation failed";
    return PIC_ERR_NOMEM;
  }
  Ctx& c = ctx->c;
  c.cfg = *cfg;
  const std::string e = derive(*cfg, c);
  if (!e.empty()) {
    g_create_err = e;
    delete ctx;
    return PIC_ERR_INVALID;
  }
  c.stream = (hipStream_t)cfg->stream;
  Plan P = make_plan(c);
  for (auto& it : P.items) {
    void* p = nullptr;
    const hipError_t he = hipMalloc(&p, it.bytes);
    if (he != hipSuccess) {
      g_create_err = std::string("hipMalloc failed: ") + hipGetErrorString(he);
      (void)hipGetLastError();
      delete ctx;
      return he == hipErrorOutOfMemory ? PIC_ERR_NOMEM : PIC_ERR_DEVICE;
    }
    c.allocs.push_back(p);
    *it.dst = p;
  }
  // zero fields, J, counters, slots (plain stream-ordered memsets at set-up)
  for (auto& it : P.items) {
    const hipError_t he = hipMemsetAsync(*it.dst, 0, it.bytes, c.stream);
    if (he != hipSuccess) {
      g_create_err = std::string("hipMemsetAsync: ") + hipGetErrorString(he);
      delete ctx;
      return PIC_ERR_DEVICE;
    }
  }
  std::vector<double> A, C, S;
  source_profile(c.cfg, c.g, A, C, S);
  const size_t ns = A.size() * sizeof(double);
  hipError_t he = hipMemcpyAsync(c.srcA, A.data(), ns, hipMemcpyHostToDevice, c.stream);
  if (he == hipSuccess) he = hipMemcpyAsync(c.srcC, C.data(), ns, hipMemcpyHostToDevice, c.stream);
  if (he == hipSuccess) he = hipMemcpyAsync(c.srcS, S.data(), ns, hipMemcpyHostToDevice, c.stream);
  const uint32_t n_act[4] = {(uint32_t)c.N, (uint32_t)c.N, (uint32_t)c.N, 0u};
  if (he == hipSuccess) he = hipMemcpyAsync(c.n_active, n_act, 16, hipMemcpyHostToDevice, c.stream);
  if (he == hipSuccess) {
    launch_init_electrons(c, c.stream);
    if (c.Ni > 0) {
      IonArgs A{};
      fill_ion_args(c, A);
      launch_ion_init(A, c.stream);
    }
    he = hipGetLastError();
  }
  if (he == hipSuccess) he = hipStreamSynchronize(c.stream);
  if (he != hipSuccess) {
    g_create_err = std::string("initialisation: ") + hipGetErrorString(he);
    delete ctx;
    return PIC_ERR_DEVICE;
  }
  if (upload_cold(c) != PIC_OK) {
    g_create_err = c.err;
    delete ctx;
    return PIC_ERR_DEVICE;
  }
  *out = ctx;
  return PIC_OK;
}

void pic_destroy(pic_ctx* ctx) {
  if (!ctx) return;
  if (!ctx->c.broken) (void)hipStreamSynchronize(ctx->c.stream);
  delete ctx;
}

pic_status pic_load_tables(pic_ctx* ctx, const pic_tables* t) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!t) FAIL(c, PIC_ERR_INVALID, "null tables");
  if (t->version != PIC_TABLES_VERSION) FAIL(c, PIC_ERR_TABLES, "tables version %u != %u", t->version, PIC_TABLES_VERSION);
  if (t->Z != c.cfg.Z) FAIL(c, PIC_ERR_TABLES, "tables built for Z=%u, config has Z=%u", t->Z, c.cfg.Z);
  if (t->n_eta != 256 || t->n_xi != 256 || t->n_T != 128 || t->n_y != 64)
    FAIL(c, PIC_ERR_TABLES, "table sizes must be 256x256 (NCS) and 128x64 (brem)");
  if (!t->h || !t->ln_xi || !t->ncs_cdf || !t->sigma || !t->br_cdf) FAIL(c, PIC_ERR_TABLES, "null table array");
  if (!(t->k_cut_mc2 > 0.0) || !is_fin(t->k_cut_mc2)) FAIL(c, PIC_ERR_TABLES, "k_cut must be > 0");
  if (!(t->dln_eta > 0.0) || !(t->dln_T > 0.0) || !is_fin(t->ln_eta0) || !is_fin(t->ln_T0))
    FAIL(c, PIC_ERR_TABLES, "bad table grid");
  for (int i = 0; i < t->n_eta; ++i)
    if (!(t->h[i] >= 0.0) || !is_fin(t->h[i])) FAIL(c, PIC_ERR_TABLES, "h[%d] invalid", i);
  for (int j = 0; j < t->n_xi; ++j) {
    if (!is_fin(t->ln_xi[j]) || (j > 0 && !(t->ln_xi[j] > t->ln_xi[j - 1])))
      FAIL(c, PIC_ERR_TABLES, "ln_xi must be finite and increasing");
  }
  for (int i = 0; i < t->n_eta; ++i) {
    const double* r = t->ncs_cdf + (size_t)i * t->n_xi;
    if (!(r[0] > 0.0) || r[t->n_xi - 1] != 1.0) FAIL(c, PIC_ERR_TABLES, "NCS CDF row %d must start > 0 and end at 1", i);
    for (int j = 1; j < t->n_xi; ++j)
      if (!(r[j] >= r[j - 1]) || !is_fin(r[j])) FAIL(c, PIC_ERR_TABLES, "NCS CDF row %d not monotone", i);
  }
  if (t->checksum != 0 && tables_checksum(*t) != t->checksum)
    FAIL(c, PIC_ERR_TABLES, "table checksum mismatch (arrays altered after they were built)");
  for (int i = 0; i < t->n_T; ++i) {
    if (!(t->sigma[i] >= 0.0) || !is_fin(t->sigma[i])) FAIL(c, PIC_ERR_TABLES, "sigma[%d] invalid", i);
    const double* r = t->br_cdf + (size_t)i * t->n_y;
    if (r[0] != 0.0 || r[t->n_y - 1] != 1.0) FAIL(c, PIC_ERR_TABLES, "brem CDF row %d must run 0..1", i);
    for (int j = 1; j < t->n_y; ++j)
      if (!(r[j] >= r[j - 1]) || !is_fin(r[j])) FAIL(c, PIC_ERR_TABLES, "brem CDF row %d not monotone", i);
  }
  DevTables& d = c.t;
  auto upload = [&](double** dd, float** df, const double* src, size_t n) -> hipError_t {
    if (!*dd) {
      hipError_t e = hipMalloc((void**)dd, n * 8);
      if (e != hipSuccess) return e;
      c.allocs.push_back(*dd);
      e = hipMalloc((void**)df, n * 4);
      if (e != hipSuccess) return e;
      c.allocs.push_back(*df);
    }
    std::vector<float> f(n);
    for (size_t i = 0; i < n; ++i) f[i] = (float)src[i];
    hipError_t e = hipMemcpy(*dd, src, n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(*df, f.data(), n * 4, hipMemcpyHostToDevice);
    return e;
  };
  HIPCHK(c, hipStreamSynchronize(c.stream));
  HIPCHK(c, upload(&d.h, &d.hf, t->h, t->n_eta));
  HIPCHK(c, upload(&d.lnxi, &d.lnxif, t->ln_xi, t->n_xi));
  HIPCHK(c, upload(&d.ncs, &d.ncsf, t->ncs_cdf, (size_t)t->n_eta * t->n_xi));
  HIPCHK(c, upload(&d.sig, &d.sigf, t->sigma, t->n_T));
  HIPCHK(c, upload(&d.br, &d.brf, t->br_cdf, (size_t)t->n_T * t->n_y));
  // row guides of the two CDF tables, from the values each precision compares
  auto guides = [&](uint8_t** gd, uint8_t** gf, const double* rows, int nrow, int n) -> hipError_t {
    const size_t ng = (size_t)nrow * (kGuide + 1);
    if (!*gd) {
      hipError_t e = hipMalloc((void**)gd, ng);
      if (e != hipSuccess) return e;
      c.allocs.push_back(*gd);
      e = hipMalloc((void**)gf, ng);
      if (e != hipSuccess) return e;
      c.allocs.push_back(*gf);
    }
    std::vector<uint8_t> g8(ng), g4(ng);
    for (int r = 0; r < nrow; ++r) {
      const double* v = rows + (size_t)r * n;
      int jd = 0, jf = 0;  // largest j <= n-2 with v[j] <= b/kGuide, as b grows
      for (int b = 0; b <= kGuide; ++b) {
        const double th = (double)b / kGuide;
        while (jd + 1 <= n - 2 && v[jd + 1] <= th) ++jd;
        while (jf + 1 <= n - 2 && (float)v[jf + 1] <= (float)th) ++jf;
        g8[(size_t)r * (kGuide + 1) + b] = (uint8_t)jd;
        g4[(size_t)r * (kGuide + 1) + b] = (uint8_t)jf;
      }
    }
    hipError_t e = hipMemcpy(*gd, g8.data(), ng, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(*gf, g4.data(), ng, hipMemcpyHostToDevice);
    return e;
  };
  HIPCHK(c, guides(&d.gncs, &d.gncsf, t->ncs_cdf, t->n_eta, t->n_xi));
  HIPCHK(c, guides(&d.gbr, &d.gbrf, t->br_cdf, t->n_T, t->n_y));
  d.n_eta = t->n_eta; d.n_xi = t->n_xi; d.n_T = t->n_T; d.n_y = t->n_y;
  d.ln_eta0 = t->ln_eta0; d.idln_eta = 1.0 / t->dln_eta;
  d.ln_T0 = t->ln_T0; d.idln_T = 1.0 / t->dln_T;
  d.k_cut = t->k_cut_mc2; d.lnk = fp_log(t->k_cut_mc2); d.iny1 = 1.0 / (double)(t->n_y - 1);
  st = upload_cold(c);
  if (st) return st;
  c.tables_loaded = true;
  return PIC_OK;
}

pic_status pic_load_pair_tables(pic_ctx* ctx, const pic_pair_tables* t) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!(c.cfg.flags & (PIC_BW | PIC_BH))) FAIL(c, PIC_ERR_STATE, "run has no pair production");
  if (!t) FAIL(c, PIC_ERR_INVALID, "null tables");
  if (t->version != PIC_PAIR_TABLES_VERSION)
    FAIL(c, PIC_ERR_TABLES, "pair tables version %u != %u", t->version, PIC_PAIR_TABLES_VERSION);
  if (t->Z != c.cfg.Z) FAIL(c, PIC_ERR_TABLES, "pair tables built for Z=%u, config has Z=%u", t->Z, c.cfg.Z);
  if (t->n_chi != 128 || t->n_xp != 128 || t->n_k != 128 || t->n_s != 64)
    FAIL(c, PIC_ERR_TABLES, "pair table sizes must be 128x128 (Breit-Wheeler) and 128x64 (Bethe-Heitler)");
  if (!t->bw_lnT || !t->bw_cdf || !t->bh_sigma || !t->bh_cdf) FAIL(c, PIC_ERR_TABLES, "null table array");
  if (!(t->dln_chi > 0.0) || !(t->dln_k > 0.0) || !is_fin(t->ln_chi0) || !is_fin(t->ln_k0))
    FAIL(c, PIC_ERR_TABLES, "bad pair table grid");
  for (int i = 0; i < t->n_chi; ++i)
    if (!is_fin(t->bw_lnT[i])) FAIL(c, PIC_ERR_TABLES, "bw_lnT[%d] not finite", i);
  for (int i = 0; i < t->n_k; ++i)
    if (!(t->bh_sigma[i] >= 0.0) || !is_fin(t->bh_sigma[i])) FAIL(c, PIC_ERR_TABLES, "bh_sigma[%d] invalid", i);
  auto rows_ok = [](const double* C, int nrow, int n) {
    for (int i = 0; i < nrow; ++i) {
      const double* r = C + (size_t)i * n;
      if (r[0] != 0.0 || r[n - 1] != 1.0) return false;
      for (int j = 1; j < n; ++j)
        if (!(r[j] >= r[j - 1]) || !std::isfinite(r[j])) return false;
    }
    return true;
  };
  if (!rows_ok(t->bw_cdf, t->n_chi, t->n_xp) || !rows_ok(t->bh_cdf, t->n_k, t->n_s))
    FAIL(c, PIC_ERR_TABLES, "pair CDF rows must rise from 0 to exactly 1");
  if (t->checksum != 0 && pair_tables_checksum(*t) != t->checksum)
    FAIL(c, PIC_ERR_TABLES, "pair table checksum mismatch (arrays altered after they were built)");
  DevTables& d = c.t;
  auto upload = [&](double** dd, float** df, const double* src, size_t n) -> hipError_t {
    if (!*dd) {
      hipError_t e = hipMalloc((void**)dd, n * 8);
      if (e != hipSuccess) return e;
      c.allocs.push_back(*dd);
      e = hipMalloc((void**)df, n * 4);
      if (e != hipSuccess) return e;
      c.allocs.push_back(*df);
    }
    std::vector<float> f(n);
    for (size_t i = 0; i < n; ++i) f[i] = (float)src[i];
    hipError_t e = hipMemcpy(*dd, src, n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(*df, f.data(), n * 4, hipMemcpyHostToDevice);
    return e;
  };
  HIPCHK(c, hipStreamSynchronize(c.stream));
  HIPCHK(c, upload(&d.bwT, &d.bwTf, t->bw_lnT, t->n_chi));
  HIPCHK(c, upload(&d.bwC, &d.bwCf, t->bw_cdf, (size_t)t->n_chi * t->n_xp));
  HIPCHK(c, upload(&d.bhS, &d.bhSf, t->bh_sigma, t->n_k));
  HIPCHK(c, upload(&d.bhC, &d.bhCf, t->bh_cdf, (size_t)t->n_k * t->n_s));
  d.n_chi = t->n_chi; d.n_xp = t->n_xp; d.n_k = t->n_k; d.n_s = t->n_s;
  d.ln_chi0 = t->ln_chi0; d.idln_chi = 1.0 / t->dln_chi;
  d.ln_k0 = t->ln_k0; d.idln_k = 1.0 / t->dln_k;
  c.pair_tables_loaded = true;
  return PIC_OK;
}

pic_status pic_step(pic_ctx* ctx, int32_t nsteps) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  st = step_ready(c, nsteps);
  if (st) return st;
  const bool frozen = (c.cfg.flags & PIC_FIELDS_FROZEN) != 0;
  auto mark = [&](int kind) {
    if (!c.prof) return;
    hipEvent_t ev = c.prof_event();
    if (ev) {
      c.ev_kind.push_back(kind);
      (void)hipEventRecord(ev, c.stream);
    }
  };
  for (int32_t it = 0; it < nsteps; ++it) {
    if (sort_due(c)) {
      mark(2);
      launch_sort(sort_args(c), c.fp32, c.stream);
      swap_sorted(c);
      mark(2);
    }
    mark(1);
    if (!frozen) launch_b_both(c, c.stream);  // B^n (into En), B^{n+1/2}, J <- 0
    mark(1);
    IonArgs IA{};
    if (c.Ni > 0) {
      fill_ion_args(c, IA);
      mark(3);
      launch_ion_density(IA, c.stream);       // n of Eq. (4) from the ions at x^n
      mark(3);
    }
    mark(0);
    if (c.fp32) {
      StepParams<float> P{};
      fill_step_params(c, P);
      launch_step(c.g.dims, true, &P, c.stream);
    } else {
      StepParams<double> P{};
      fill_step_params(c, P);
      launch_step(c.g.dims, false, &P, c.stream);
    }
    mark(0);
    if (c.Ni > 0) {
      mark(3);
      launch_ion_step(IA, c.stream);
      mark(3);
    }
    if (c.cfg.flags & (PIC_BW | PIC_BH)) {     // photons in flight: E^n, B^n, n at x^n
      mark(4);
      PhotonArgs PA{};
      fill_photon_args(c, PA);
      launch_photon_step(PA, c.fp32, c.stream);
      mark(4);
    }
    mark(1);
    if (!frozen) {
      double ls, lc;
      laser_scalars(c, c.step, &ls, &lc);
      launch_e_full(c, ls, lc, c.stream);          // E^n -> E^{n+1}
    }
    mark(1);
    c.step++;
  }
  HIPCHK(c, hipGetLastError());
  return PIC_OK;
}

pic_status pic_emission_stats(pic_ctx* ctx, pic_stats* out) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!out) FAIL(c, PIC_ERR_INVALID, "null output");
  unsigned long long cnt[kRedCnt];
  double sum[kRedSum];
  unsigned long long pcount = 0, rcount = 0, rev[2] = {0, 0};
  double resum[2] = {0.0, 0.0};
  pic_stats s{};
  launch_stats_reduce(c, cnt, sum, c.stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(&pcount, c.pcount, 8, hipMemcpyDeviceToHost, c.stream));
  std::vector<unsigned long long> spec((size_t)kSpecCopies * 2 * PIC_SPECTRUM_BINS);
  HIPCHK(c, hipMemcpyAsync(spec.data(), c.spec, spec.size() * 8, hipMemcpyDeviceToHost, c.stream));
  if (c.rcount) {
    HIPCHK(c, hipMemcpyAsync(&rcount, c.rcount, 8, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipMemcpyAsync(rev, c.rev, 16, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipMemcpyAsync(resum, c.resum, 16, hipMemcpyDeviceToHost, c.stream));
  }
  HIPCHK(c, hipStreamSynchronize(c.stream));
  s.steps = c.step;
  for (size_t q = 0; q < spec.size(); ++q) (&s.spectrum[0][0])[q % (2 * PIC_SPECTRUM_BINS)] += spec[q];
  s.electrons_live = cnt[kSlotCnt];
  s.electron_steps = cnt[SC_ESTEPS];
  s.events[0] = cnt[SC_EV_NCS];
  s.events[1] = cnt[SC_EV_BR];
  s.kept[0] = cnt[SC_KEPT_NCS];
  s.kept[1] = cnt[SC_KEPT_BR];
  s.dropped_ncs = cnt[SC_DROPPED];
  s.brem_clamped = cnt[SC_CLAMPED];
  s.untiled_steps = cnt[SC_UNTILED];
  // the device stops reserving slots once the buffer is full, so the
  // counter can fall short of the kept photons: overflow = kept - stored
  s.photons_stored = pcount < c.pcap ? pcount : c.pcap;
  s.overflow = s.kept[0] + s.kept[1] + ctx->injected - s.photons_stored;
  s.e_rad_kept[0] = sum[0];
  s.e_rad_kept[1] = sum[1];
  s.e_rad_dropped = sum[2];
  s.e_kin_e = sum[3];
  s.e_field = 0.5 * sum[4] * (1.0 / c.g.invV);
  s.ions_live = cnt[kSlotCnt + 1];
  s.e_kin_i = sum[5];
  s.pairs[0] = rev[0];
  s.pairs[1] = rev[1];
  s.pairs_stored = rcount < c.rcap ? rcount : c.rcap;
  s.pairs_overflow = rev[0] + rev[1] - s.pairs_stored;
  s.e_pair[0] = resum[0];
  s.e_pair[1] = resum[1];
  *out = s;
  return s.overflow ? PIC_ERR_OVERFLOW : PIC_OK;
}

pic_status pic_batch_create(void* stream, pic_batch** out) {
  if (!out) return PIC_ERR_INVALID;
  *out = nullptr;
  pic_batch* b = new (std::nothrow) pic_batch;
  if (!b) return PIC_ERR_NOMEM;
  b->stream = (hipStream_t)stream;
  if (hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming) != hipSuccess) {
    g_create_err = "hipEventCreate failed";
    delete b;
    return PIC_ERR_DEVICE;
  }
  *out = b;
  return PIC_OK;
}

void pic_batch_destroy(pic_batch* b) { delete b; }

const char* pic_batch_last_error(const pic_batch* b) { return b ? b->err.c_str() : ""; }

pic_status pic_step_many(pic_batch* b, pic_ctx* const* ctxs, const int32_t* nsteps, int32_t njobs) {
  if (!b) return PIC_ERR_INVALID;
  if (njobs < 0 || (njobs > 0 && (!ctxs || !nsteps))) {
    b->err = "bad job list";
    return PIC_ERR_INVALID;
  }
  // validate everything before any run's state moves
  int32_t S = 0;
  std::vector<Ctx*> all;
  for (int32_t j = 0; j < njobs; ++j) {
    pic_status st = check_ctx(ctxs[j]);
    if (st) {
      b->err = "job " + std::to_string(j) + ": null or broken context";
      return st;
    }
    Ctx& c = ctxs[j]->c;
    st = step_ready(c, nsteps[j]);
    if (st) {
      b->err = "job " + std::to_string(j) + ": " + c.err;
      return st;
    }
    if (c.stream != b->stream) {
      b->err = "job " + std::to_string(j) + ": context stream differs from the batch stream";
      return PIC_ERR_INVALID;
    }
    for (Ctx* o : all)
      if (o == &c) {
        b->err = "job " + std::to_string(j) + ": context listed twice";
        return PIC_ERR_INVALID;
      }
    all.push_back(&c);
    S = std::max(S, nsteps[j]);
  }
  if (S == 0) return PIC_OK;

  // host pass: the launches of every step, with the parameter tables staged
  std::vector<unsigned char>& st = b->stage;
  st.clear();
  std::vector<BatchLaunch> L;
  std::vector<Ctx*> act;
  for (int32_t s = 0; s < S; ++s) {
    act.clear();
    for (int32_t j = 0; j < njobs; ++j)
      if (nsteps[j] > s) act.push_back(all[j]);
    for (Ctx* c : act)
      if (sort_due(*c)) {
        BatchLaunch l{};
        l.kind = 0;
        l.fp32 = c->fp32;
        l.sort = sort_args(*c);
        L.push_back(l);
        swap_sorted(*c);
      }
    BatchLaunch fl[2];
    bool have_f[2] = {false, false};
    for (int f = 0; f < 2; ++f) {
      std::vector<FieldJob> tab;
      std::vector<uint32_t> first{0u};
      for (Ctx* c : act) {
        if ((c->cfg.flags & PIC_FIELDS_FROZEN) || c->fp32 != (f == 1)) continue;
        double ls, lc;
        laser_scalars(*c, c->step, &ls, &lc);
        FieldJob F{};
        fill_field_job(*c, ls, lc, F);
        tab.push_back(F);
        first.push_back(first.back() + field_blocks(*c));
      }
      if (tab.empty()) continue;
      fl[f].fp32 = f == 1;
      fl[f].tab = stage_put(st, tab.data(), tab.size() * sizeof(FieldJob));
      fl[f].first = stage_put(st, first.data(), first.size() * sizeof(uint32_t));
      fl[f].njobs = (int)tab.size();
      fl[f].total = first.back();
      have_f[f] = true;
    }
    for (int f = 0; f < 2; ++f)
      if (have_f[f]) { BatchLaunch l = fl[f]; l.kind = 1; L.push_back(l); }
    std::vector<BatchLaunch> ion_steps;
    for (Ctx* c : act)
      if (c->Ni > 0) {
        BatchLaunch l{};
        fill_ion_args(*c, l.ion);
        l.kind = 5;
        L.push_back(l);
        l.kind = 6;
        ion_steps.push_back(l);
      }
    for (int d = 1; d <= 3; ++d) {
      stage_step_group<float>(st, L, act, d);
      stage_step_group<double>(st, L, act, d);
    }
    for (const BatchLaunch& l : ion_steps) L.push_back(l);
    for (Ctx* c : act)
      if (c->cfg.flags & (PIC_BW | PIC_BH)) {
        BatchLaunch l{};
        fill_photon_args(*c, l.ph);
        l.kind = 7;
        l.fp32 = c->fp32;
        L.push_back(l);
      }
    for (int f = 0; f < 2; ++f)
      if (have_f[f]) { BatchLaunch l = fl[f]; l.kind = 4; L.push_back(l); }
    for (Ctx* c : act) {
      if (!(c->cfg.flags & PIC_FIELDS_FROZEN))
        for (int d = 0; d < 3; ++d) std::swap(c->E[d], c->En[d]);
      c->step++;
    }
  }

  // one upload of every table, then the launches in order
  auto fail = [&](const char* what, hipError_t e) {
    b->err = std::string(what) + ": " + hipGetErrorString(e);
    for (Ctx* c : all) { c->broken = true; c->err = b->err; }
    return PIC_ERR_DEVICE;
  };
  hipError_t e = hipSuccess;
  if (b->pending) {
    e = hipEventSynchronize(b->uploaded);
    if (e != hipSuccess) return fail("hipEventSynchronize", e);
    b->pending = false;
  }
  const size_t need = st.size();
  if (need > b->host_cap) {
    if (b->host) (void)hipHostFree(b->host);
    b->host = nullptr;
    b->host_cap = 0;
    e = hipHostMalloc((void**)&b->host, need * 2, hipHostMallocDefault);
    if (e != hipSuccess) return fail("hipHostMalloc", e);
    b->host_cap = need * 2;
  }
  if (need > b->dev_cap) {
    if (b->dev) {
      e = hipStreamSynchronize(b->stream);  // earlier launches may still read it
      if (e != hipSuccess) return fail("hipStreamSynchronize", e);
      (void)hipFree(b->dev);
    }
    b->dev = nullptr;
    b->dev_cap = 0;
    e = hipMalloc((void**)&b->dev, need * 2);
    if (e != hipSuccess) return fail("hipMalloc", e);
    b->dev_cap = need * 2;
  }
  std::memcpy(b->host, st.data(), need);
  e = hipMemcpyAsync(b->dev, b->host, need, hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return fail("hipMemcpyAsync", e);
  e = hipEventRecord(b->uploaded, b->stream);
  if (e != hipSuccess) return fail("hipEventRecord", e);
  b->pending = true;
  unsigned char* D = b->dev;
  for (const BatchLaunch& l : L) {
    switch (l.kind) {
      case 0: launch_sort(l.sort, l.fp32, b->stream); break;
      case 5: launch_ion_density(l.ion, b->stream); break;
      case 6: launch_ion_step(l.ion, b->stream); break;
      case 7: launch_photon_step(l.ph, l.fp32, b->stream); break;
      case 1:
        launch_b_both_batch(l.fp32, (const FieldJob*)(D + l.tab), (const uint32_t*)(D + l.first),
                            l.njobs, l.total, b->stream);
        break;
      case 2:
        launch_step_batch(l.dims, l.fp32, D + l.tab, (const uint32_t*)(D + l.first), l.njobs, l.total,
                          l.lds_nodes, b->stream);
        break;
      default:
        launch_e_full_batch(l.fp32, (const FieldJob*)(D + l.tab), (const uint32_t*)(D + l.first),
                            l.njobs, l.total, b->stream);
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess) return fail("launch", e);
  return PIC_OK;
}

pic_status pic_synchronize(pic_ctx* ctx) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  HIPCHK(c, hipStreamSynchronize(c.stream));
  HIPCHK(c, hipGetLastError());
  return PIC_OK;
}

pic_status pic_counts(pic_ctx* ctx, uint64_t* electrons, uint64_t* stored, uint64_t* kept) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  unsigned long long pc = 0;
  // kept photons from the per-wave counts: the device's slot counter stops
  // once the buffer is full
  unsigned long long cnt[kRedCnt];
  double sum[kRedSum];
  if (kept) {
    launch_stats_reduce(c, cnt, sum, c.stream);
    HIPCHK(c, hipGetLastError());
  }
  HIPCHK(c, hipMemcpyAsync(&pc, c.pcount, 8, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  if (electrons) *electrons = (uint64_t)c.N;
  if (stored) *stored = pc < c.pcap ? pc : c.pcap;
  if (kept) *kept = cnt[SC_KEPT_NCS] + cnt[SC_KEPT_BR];
  return PIC_OK;
}


pic_status pic_get_buffers(pic_ctx* ctx, pic_buffers* out) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!out) FAIL(c, PIC_ERR_INVALID, "null output");
  uint64_t stored = 0;
  if ((st = pic_counts(ctx, nullptr, &stored, nullptr))) return st;
  pic_buffers b{};
  b.precision = c.cfg.precision;
  b.dims = (uint32_t)c.g.dims;
  b.electrons = (uint64_t)c.N;
  b.photons_stored = stored;
  b.field_size = (uint64_t)c.g.nfield;
  for (int a = 0; a < 3; ++a) {
    b.fb[a] = c.fp32 ? c.g.fb[a] : 0;
    b.x[a] = a < c.g.dims ? c.x[a] : nullptr;
    b.p[a] = c.p[a];
    b.E[a] = c.E[a];
    b.B[a] = c.B[a];
    b.J[a] = (int64_t*)c.J[a];
    b.photon_x[a] = c.px[a];
    b.photon_k[a] = c.pk[a];
  }
  b.tau = c.tau;
  b.taub = c.taub;
  b.w = c.w;
  b.id = c.id;
  b.photon_eps = c.pe;
  b.photon_w = c.pw;
  b.photon_step = c.pstep;
  b.photon_parent = c.ppar;
  b.photon_proc = c.pproc;
  *out = b;
  return PIC_OK;
}

pic_status pic_copy_electrons(pic_ctx* ctx, double* x, double* p, double* tau, double* w,
                              uint32_t* id, uint8_t* alive) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  const size_t N = (size_t)c.N;
  std::vector<uint32_t> ids(N);
  if (N) {
    HIPCHK(c, hipMemcpyAsync(ids.data(), c.id, N * 4, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
  }
  std::vector<double> v, t8(N), w8(N);
  for (int a = 0; a < 3; ++a) {
    if (x) {
      if (a < c.g.dims && c.fp32) {  // fixed point -> absolute position
        std::vector<int32_t> qv(N);
        HIPCHK(c, hipMemcpyAsync(qv.data(), c.x[a], N * 4, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(c, hipStreamSynchronize(c.stream));
        v.resize(N);
        const double s = ldexp(1.0, -c.g.fb[a]) * c.g.dx[a];
        for (size_t e = 0; e < N; ++e) v[e] = (double)qv[e] * s;
      } else if (a < c.g.dims) {
        if ((st = copy_any(c, c.x[a], N, v))) return st;
      } else {
        v.assign(N, 0.0);
      }
      for (size_t e = 0; e < N; ++e) x[3 * (ids[e] & ~kDead) + a] = v[e];
    }
    if (p) {
      if ((st = copy_any(c, c.p[a], N, v))) return st;
      for (size_t e = 0; e < N; ++e) p[3 * (ids[e] & ~kDead) + a] = v[e];
    }
  }
  if (N) {
    HIPCHK(c, hipMemcpyAsync(t8.data(), c.tau, N * 8, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipMemcpyAsync(w8.data(), c.w, N * 8, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
  }
  for (size_t e = 0; e < N; ++e) {
    const uint32_t i = ids[e] & ~kDead;
    if (tau) tau[i] = t8[e];
    if (w) w[i] = w8[e];
    if (id) id[i] = i;
    if (alive) alive[i] = (ids[e] & kDead) ? 0 : 1;
  }
  return PIC_OK;
}

pic_status pic_set_electrons(pic_ctx* ctx, const double* x, const double* p, const double* tau) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!x || !p || !tau) FAIL(c, PIC_ERR_INVALID, "null argument");
  const size_t N = (size_t)c.N;
  if (!N) return PIC_OK;
  std::vector<uint32_t> ids(N);
  HIPCHK(c, hipMemcpyAsync(ids.data(), c.id, N * 4, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  for (size_t e = 0; e < N; ++e) {
    for (int a = 0; a < 3; ++a)
      if (!is_fin(x[3 * e + a]) || !is_fin(p[3 * e + a])) FAIL(c, PIC_ERR_INVALID, "non-finite electron state");
    if (!is_fin(tau[e])) FAIL(c, PIC_ERR_INVALID, "non-finite optical depth");
    // the gather and deposit stencils assume every live electron is inside the box
    for (int a = 0; a < c.g.dims; ++a)
      if (!(x[3 * e + a] >= 0.0 && x[3 * e + a] < c.g.L[a]))
        FAIL(c, PIC_ERR_INVALID, "electron %zu outside the box on axis %d", e, a);
  }
  auto put = [&](void* dev, const double* src, int stride, int a) -> pic_status {
    if (c.fp32) {
      std::vector<float> f(N);
      for (size_t e = 0; e < N; ++e) f[e] = (float)src[(size_t)stride * (ids[e] & ~kDead) + a];
      HIPCHK(c, hipMemcpyAsync(dev, f.data(), N * 4, hipMemcpyHostToDevice, c.stream));
      HIPCHK(c, hipStreamSynchronize(c.stream));
    } else {
      std::vector<double> d(N);
      for (size_t e = 0; e < N; ++e) d[e] = src[(size_t)stride * (ids[e] & ~kDead) + a];
      HIPCHK(c, hipMemcpyAsync(dev, d.data(), N * 8, hipMemcpyHostToDevice, c.stream));
      HIPCHK(c, hipStreamSynchronize(c.stream));
    }
    return PIC_OK;
  };
  for (int a = 0; a < 3; ++a) {
    if (a < c.g.dims && c.fp32) {  // absolute position -> fixed point in cells
      std::vector<int32_t> qv(N);
      const double s = ldexp(1.0, c.g.fb[a]) * c.g.idx[a];
      const double qmax = ldexp((double)c.g.n[a], c.g.fb[a]) - 1.0;
      for (size_t e = 0; e < N; ++e)
        qv[e] = (int32_t)std::min(qmax, (double)llrint(x[3 * (size_t)(ids[e] & ~kDead) + a] * s));
      HIPCHK(c, hipMemcpyAsync(c.x[a], qv.data(), N * 4, hipMemcpyHostToDevice, c.stream));
      HIPCHK(c, hipStreamSynchronize(c.stream));
    } else if (a < c.g.dims && (st = put(c.x[a], x, 3, a))) {
      return st;
    }
    if ((st = put(c.p[a], p, 3, a))) return st;
  }
  std::vector<double> t8(N);
  for (size_t e = 0; e < N; ++e) t8[e] = tau[ids[e] & ~kDead];
  HIPCHK(c, hipMemcpyAsync(c.tau, t8.data(), N * 8, hipMemcpyHostToDevice, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  return PIC_OK;
}

pic_status pic_ion_count(pic_ctx* ctx, uint64_t* ions) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!ions) FAIL(c, PIC_ERR_INVALID, "null output");
  *ions = (uint64_t)c.Ni;
  return PIC_OK;
}

pic_status pic_copy_ions(pic_ctx* ctx, double* x, double* p, uint8_t* alive) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (c.Ni <= 0) FAIL(c, PIC_ERR_INVALID, "run has no mobile ions");
  const size_t N = (size_t)c.Ni;
  std::vector<double> v(N);
  for (int a = 0; a < 3; ++a) {
    if (x) {
      if (a < c.g.dims) {
        HIPCHK(c, hipMemcpyAsync(v.data(), c.ix[a], N * 8, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(c, hipStreamSynchronize(c.stream));
      } else {
        std::fill(v.begin(), v.end(), 0.0);
      }
      for (size_t e = 0; e < N; ++e) x[3 * e + a] = v[e];
    }
    if (p) {
      HIPCHK(c, hipMemcpyAsync(v.data(), c.ip[a], N * 8, hipMemcpyDeviceToHost, c.stream));
      HIPCHK(c, hipStreamSynchronize(c.stream));
      for (size_t e = 0; e < N; ++e) p[3 * e + a] = v[e];
    }
  }
  if (alive) {
    HIPCHK(c, hipMemcpyAsync(alive, c.ialive, N, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
  }
  return PIC_OK;
}

pic_status pic_set_ions(pic_ctx* ctx, const double* x, const double* p) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (c.Ni <= 0) FAIL(c, PIC_ERR_INVALID, "run has no mobile ions");
  if (!x || !p) FAIL(c, PIC_ERR_INVALID, "null argument");
  const size_t N = (size_t)c.Ni;
  std::vector<uint8_t> al(N);
  HIPCHK(c, hipMemcpyAsync(al.data(), c.ialive, N, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  for (size_t e = 0; e < N; ++e) {
    for (int a = 0; a < 3; ++a)
      if (!is_fin(x[3 * e + a]) || !is_fin(p[3 * e + a])) FAIL(c, PIC_ERR_INVALID, "non-finite ion state");
    // the gather and deposit stencils assume every live ion is inside the box
    if (al[e])
      for (int a = 0; a < c.g.dims; ++a)
        if (!(x[3 * e + a] >= 0.0 && x[3 * e + a] < c.g.L[a]))
          FAIL(c, PIC_ERR_INVALID, "ion %zu outside the box on axis %d", e, a);
  }
  std::vector<double> v(N);
  for (int a = 0; a < 3; ++a) {
    if (a < c.g.dims) {
      for (size_t e = 0; e < N; ++e) v[e] = x[3 * e + a];
      HIPCHK(c, hipMemcpyAsync(c.ix[a], v.data(), N * 8, hipMemcpyHostToDevice, c.stream));
      HIPCHK(c, hipStreamSynchronize(c.stream));
    }
    for (size_t e = 0; e < N; ++e) v[e] = p[3 * e + a];
    HIPCHK(c, hipMemcpyAsync(c.ip[a], v.data(), N * 8, hipMemcpyHostToDevice, c.stream));
    HIPCHK(c, hipStreamSynchronize(c.stream));
  }
  IonArgs A{};
  fill_ion_args(c, A);
  launch_ion_recount(A, c.stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c.stream));
  return PIC_OK;
}

pic_status pic_pair_counts(pic_ctx* ctx, uint64_t* stored, uint64_t* created) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!c.rcount) FAIL(c, PIC_ERR_STATE, "run has no pair production");
  unsigned long long rc = 0, ev[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(&rc, c.rcount, 8, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipMemcpyAsync(ev, c.rev, 16, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  if (stored) *stored = rc < c.rcap ? rc : c.rcap;
  if (created) *created = ev[0] + ev[1];
  return PIC_OK;
}

pic_status pic_copy_pairs(pic_ctx* ctx, uint64_t off, uint64_t n, double* x, double* k,
                          double* e_minus, double* e_plus, double* w, uint32_t* step,
                          uint32_t* parent, uint32_t* pstep, uint32_t* proc) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  uint64_t stored = 0;
  if ((st = pic_pair_counts(ctx, &stored, nullptr))) return st;
  if (off > stored || n > stored - off) FAIL(c, PIC_ERR_INVALID, "pair range beyond the stored records");
  if (!n) return PIC_OK;
  std::vector<double> v;
  for (int a = 0; a < 3; ++a) {
    if (x) {
      if ((st = copy_any(c, (const char*)c.rx[a] + off * real_size(c.cfg), n, v))) return st;
      for (uint64_t i = 0; i < n; ++i) x[3 * i + a] = v[i];
    }
    if (k) {
      if ((st = copy_any(c, (const char*)c.rk[a] + off * real_size(c.cfg), n, v))) return st;
      for (uint64_t i = 0; i < n; ++i) k[3 * i + a] = v[i];
    }
  }
  if (e_minus) {
    if ((st = copy_any(c, (const char*)c.rem + off * real_size(c.cfg), n, v))) return st;
    std::copy(v.begin(), v.end(), e_minus);
  }
  if (e_plus) {
    if ((st = copy_any(c, (const char*)c.rep + off * real_size(c.cfg), n, v))) return st;
    std::copy(v.begin(), v.end(), e_plus);
  }
  if (w) HIPCHK(c, hipMemcpyAsync(w, c.rw + off, n * 8, hipMemcpyDeviceToHost, c.stream));
  if (step) HIPCHK(c, hipMemcpyAsync(step, c.rstep + off, n * 4, hipMemcpyDeviceToHost, c.stream));
  if (parent) HIPCHK(c, hipMemcpyAsync(parent, c.rpar + off, n * 4, hipMemcpyDeviceToHost, c.stream));
  if (pstep) HIPCHK(c, hipMemcpyAsync(pstep, c.rpst + off, n * 4, hipMemcpyDeviceToHost, c.stream));
  if (proc) HIPCHK(c, hipMemcpyAsync(proc, c.rproc + off, n * 4, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  return PIC_OK;
}

pic_status pic_copy_flight(pic_ctx* ctx, uint64_t off, uint64_t n, double* x, double* tau,
                           uint8_t* state) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!c.gst) FAIL(c, PIC_ERR_STATE, "run has no pair production");
  unsigned long long pc = 0;
  HIPCHK(c, hipMemcpyAsync(&pc, c.pcount, 8, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  const uint64_t stored = pc < c.pcap ? pc : c.pcap;
  if (off > stored || n > stored - off) FAIL(c, PIC_ERR_INVALID, "photon range beyond the stored records");
  if (!n) return PIC_OK;
  std::vector<double> v;
  if (x)
    for (int a = 0; a < 3; ++a) {
      if ((st = copy_any(c, (const char*)c.gx[a] + off * real_size(c.cfg), n, v))) return st;
      for (uint64_t i = 0; i < n; ++i) x[3 * i + a] = v[i];
    }
  if (tau) HIPCHK(c, hipMemcpyAsync(tau, c.gtau + off, n * 8, hipMemcpyDeviceToHost, c.stream));
  if (state) HIPCHK(c, hipMemcpyAsync(state, c.gst + off, n, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  return PIC_OK;
}

pic_status pic_add_photons(pic_ctx* ctx, uint64_t n, const double* x, const double* k,
                           const double* eps, const double* w, const uint32_t* parent) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!c.gst) FAIL(c, PIC_ERR_STATE, "run has no pair production");
  if (n && (!x || !k || !eps || !w || !parent)) FAIL(c, PIC_ERR_INVALID, "null argument");
  for (uint64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a)
      if (!is_fin(x[3 * i + a]) || !is_fin(k[3 * i + a])) FAIL(c, PIC_ERR_INVALID, "non-finite photon");
    if (!(eps[i] > 0.0) || !is_fin(eps[i]) || !is_fin(w[i])) FAIL(c, PIC_ERR_INVALID, "bad photon energy or weight");
    for (int a = 0; a < c.g.dims; ++a)
      if (!(x[3 * i + a] >= 0.0 && x[3 * i + a] < c.g.L[a]))
        FAIL(c, PIC_ERR_INVALID, "photon %llu outside the box", (unsigned long long)i);
  }
  unsigned long long pc = 0;
  HIPCHK(c, hipMemcpyAsync(&pc, c.pcount, 8, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  if (pc > c.pcap || n > c.pcap - pc) {
    c.err = "photon buffer cannot take the photons";
    return PIC_ERR_OVERFLOW;
  }
  if (!n) return PIC_OK;
  const size_t rs = real_size(c.cfg);
  std::vector<unsigned char> buf(n * 8);
  auto put_real = [&](void* dev, const double* src, int stride, int a) -> hipError_t {
    for (uint64_t i = 0; i < n; ++i) {
      const double v = src[(size_t)stride * i + a];
      if (rs == 4) { const float f = (float)v; std::memcpy(&buf[i * 4], &f, 4); }
      else std::memcpy(&buf[i * 8], &v, 8);
    }
    hipError_t e = hipMemcpyAsync((char*)dev + pc * rs, buf.data(), n * rs, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    return e;
  };
  for (int a = 0; a < 3; ++a) {
    HIPCHK(c, put_real(c.px[a], x, 3, a));
    HIPCHK(c, put_real(c.pk[a], k, 3, a));
  }
  HIPCHK(c, put_real(c.pe, eps, 1, 0));
  std::vector<uint32_t> stp(n, (uint32_t)c.step), prc(n, 0u);
  HIPCHK(c, hipMemcpyAsync(c.pw + pc, w, n * 8, hipMemcpyHostToDevice, c.stream));
  HIPCHK(c, hipMemcpyAsync(c.pstep + pc, stp.data(), n * 4, hipMemcpyHostToDevice, c.stream));
  HIPCHK(c, hipMemcpyAsync(c.ppar + pc, parent, n * 4, hipMemcpyHostToDevice, c.stream));
  HIPCHK(c, hipMemcpyAsync(c.pproc + pc, prc.data(), n * 4, hipMemcpyHostToDevice, c.stream));
  const unsigned long long np = pc + n;
  HIPCHK(c, hipMemcpyAsync(c.pcount, &np, 8, hipMemcpyHostToDevice, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  ctx->injected += n;
  return PIC_OK;
}

pic_status pic_copy_brem_depth(pic_ctx* ctx, double* out) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!(c.cfg.flags & PIC_BREM_FREEPATH)) FAIL(c, PIC_ERR_STATE, "run has no free-path bremsstrahlung");
  if (!out) FAIL(c, PIC_ERR_INVALID, "null argument");
  const size_t N = (size_t)c.N;
  if (!N) return PIC_OK;
  std::vector<uint32_t> ids(N);
  std::vector<double> t8(N);
  HIPCHK(c, hipMemcpyAsync(ids.data(), c.id, N * 4, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipMemcpyAsync(t8.data(), c.taub, N * 8, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  for (size_t e = 0; e < N; ++e) out[ids[e] & ~kDead] = t8[e];
  return PIC_OK;
}

pic_status pic_set_brem_depth(pic_ctx* ctx, const double* in) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!(c.cfg.flags & PIC_BREM_FREEPATH)) FAIL(c, PIC_ERR_STATE, "run has no free-path bremsstrahlung");
  if (!in) FAIL(c, PIC_ERR_INVALID, "null argument");
  const size_t N = (size_t)c.N;
  if (!N) return PIC_OK;
  for (size_t e = 0; e < N; ++e)
    if (!is_fin(in[e])) FAIL(c, PIC_ERR_INVALID, "non-finite optical depth");
  std::vector<uint32_t> ids(N);
  HIPCHK(c, hipMemcpyAsync(ids.data(), c.id, N * 4, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  std::vector<double> t8(N);
  for (size_t e = 0; e < N; ++e) t8[e] = in[ids[e] & ~kDead];
  HIPCHK(c, hipMemcpyAsync(c.taub, t8.data(), N * 8, hipMemcpyHostToDevice, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  return PIC_OK;
}

pic_status pic_copy_photons(pic_ctx* ctx, uint64_t off, uint64_t n, double* x, double* k,
                            double* eps, double* w, uint32_t* step, uint32_t* parent,
                            uint32_t* proc) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  uint64_t stored = 0;
  if ((st = pic_counts(ctx, nullptr, &stored, nullptr))) return st;
  if (off > stored || n > stored - off) FAIL(c, PIC_ERR_INVALID, "photon range [%llu, +%llu) beyond %llu stored",
                                             (unsigned long long)off, (unsigned long long)n, (unsigned long long)stored);
  if (n == 0) return PIC_OK;
  const size_t rs = c.fp32 ? 4 : 8;
  std::vector<double> v;
  for (int a = 0; a < 3; ++a) {
    if (x) {
      if ((st = copy_any(c, (const char*)c.px[a] + off * rs, n, v))) return st;
      for (uint64_t i = 0; i < n; ++i) x[3 * i + a] = v[i];
    }
    if (k) {
      if ((st = copy_any(c, (const char*)c.pk[a] + off * rs, n, v))) return st;
      for (uint64_t i = 0; i < n; ++i) k[3 * i + a] = v[i];
    }
  }
  if (eps) {
    if ((st = copy_any(c, (const char*)c.pe + off * rs, n, v))) return st;
    memcpy(eps, v.data(), n * 8);
  }
  if (w) HIPCHK(c, hipMemcpyAsync(w, c.pw + off, n * 8, hipMemcpyDeviceToHost, c.stream));
  if (step) HIPCHK(c, hipMemcpyAsync(step, c.pstep + off, n * 4, hipMemcpyDeviceToHost, c.stream));
  if (parent) HIPCHK(c, hipMemcpyAsync(parent, c.ppar + off, n * 4, hipMemcpyDeviceToHost, c.stream));
  if (proc) HIPCHK(c, hipMemcpyAsync(proc, c.pproc + off, n * 4, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  return PIC_OK;
}

pic_status pic_field_size(pic_ctx* ctx, uint64_t* size) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  if (!size) return PIC_ERR_INVALID;
  *size = (uint64_t)ctx->c.g.nfield;
  return PIC_OK;
}

pic_status pic_copy_fields(pic_ctx* ctx, double* out) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!out) FAIL(c, PIC_ERR_INVALID, "null output");
  const size_t nf = (size_t)c.g.nfield;
  std::vector<double> v;
  for (int a = 0; a < 3; ++a) {
    if ((st = copy_any(c, c.E[a], nf, v))) return st;
    memcpy(out + (size_t)a * nf, v.data(), nf * 8);
    if ((st = copy_any(c, c.B[a], nf, v))) return st;
    memcpy(out + (size_t)(3 + a) * nf, v.data(), nf * 8);
  }
  return PIC_OK;
}

pic_status pic_profile(pic_ctx* ctx, int32_t enable) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  HIPCHK(c, hipStreamSynchronize(c.stream));
  c.prof = enable != 0;
  c.ev_used = 0;
  c.ev_kind.clear();
  return PIC_OK;
}

pic_status pic_profile_read(pic_ctx* ctx, double* ms2, uint64_t* n2) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!ms2 || !n2) FAIL(c, PIC_ERR_INVALID, "null output");
  HIPCHK(c, hipStreamSynchronize(c.stream));
  for (int k = 0; k < 5; ++k) {
    ms2[k] = 0.0;
    n2[k] = 0;
  }
  for (size_t i = 0; i + 1 < c.ev_used; i += 2) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c.ev_pool[i], c.ev_pool[i + 1]));
    const int k = c.ev_kind[i];
    ms2[k] += ms;
    n2[k] += 1;
  }
  return PIC_OK;
}

pic_status pic_copy_current(pic_ctx* ctx, int64_t* out) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  Ctx& c = ctx->c;
  if (!out) FAIL(c, PIC_ERR_INVALID, "null output");
  const size_t nf = (size_t)c.g.nfield;
  for (int a = 0; a < 3; ++a)
    HIPCHK(c, hipMemcpyAsync(out + (size_t)a * nf, c.J[a], nf * 8, hipMemcpyDeviceToHost, c.stream));
  HIPCHK(c, hipStreamSynchronize(c.stream));
  return PIC_OK;
}

pic_status pic_derived(pic_ctx* ctx, double* o) {
  pic_status st = check_ctx(ctx);
  if (st) return st;
  if (!o) return PIC_ERR_INVALID;
  const Ctx& c = ctx->c;
  o[0] = c.g.dx[0]; o[1] = c.g.dx[1]; o[2] = c.g.dx[2]; o[3] = c.g.dt;
  o[4] = c.E_S; o[5] = c.K_N; o[6] = c.K_BR; o[7] = c.n_c;
  return PIC_OK;
}

// ---- Philox without device allocation --------------------------------------
// Staging for pic_philox_noalloc: counters in the first half, outputs in the
// second, kPhiloxScratchMax counters of 16 bytes each per half (2 MiB in all).
// A file-scope device array: every GPU the library runs on holds its own
// copy, for the life of the process.  In host code `scratch` is a host-side
// stand-in, never a device address: kernels and copies get the address
// hipGetSymbolAddress returns, fetched once per device.
constexpr uint64_t kPhiloxScratchMax = 1ull << 16;
static __device__ __align__(256) uint32_t scratch[2 * 4 * kPhiloxScratchMax];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};  // per device ordinal

// Device address of this device's scratch array (set up on the device's
// first call); nullptr with *err set on failure.
uint32_t* scratch_ptr(std::string* err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= 64) {
    *err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return static_cast<uint32_t*>(g_scratch_ptr[dev]);
}
}  // namespace

pic_status pic_philox_noalloc(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n) {
  if (!ctr || !key || !out) {
    g_create_err = "pic_philox_noalloc: null argument";
    return PIC_ERR_INVALID;
  }
  if (n == 0) return PIC_OK;
  if (n > kPhiloxScratchMax) {
    g_create_err = "pic_philox_noalloc: n = " + std::to_string(n) + " exceeds the staging capacity of " +
                   std::to_string(kPhiloxScratchMax) + " counters";
    return PIC_ERR_INVALID;
  }
  uint32_t* base = scratch_ptr(&g_create_err);
  if (!base) return PIC_ERR_DEVICE;
  uint32_t* dc = base;                            // counters
  uint32_t* doo = base + 4 * kPhiloxScratchMax;   // outputs
  hipError_t e = hipMemcpy(dc, ctr, n * 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_philox(dc, key[0], key[1], doo, n, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out, doo, n * 16, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    g_create_err = std::string("pic_philox_noalloc: ") + hipGetErrorString(e);
    return PIC_ERR_DEVICE;
  }
  return PIC_OK;
}

pic_status pic_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n) {
  if (!ctr || !key || !out) return PIC_ERR_INVALID;
  if (n == 0) return PIC_OK;
  if (n > (1ull << 28)) return PIC_ERR_INVALID;
  uint32_t *dc = nullptr, *doo = nullptr;
  if (hipMalloc(&dc, n * 16) != hipSuccess) return PIC_ERR_NOMEM;
  if (hipMalloc(&doo, n * 16) != hipSuccess) {
    (void)!hipFree(dc);
    return PIC_ERR_NOMEM;
  }
  hipError_t e = hipMemcpy(dc, ctr, n * 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_philox(dc, key[0], key[1], doo, n, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out, doo, n * 16, hipMemcpyDeviceToHost);
  (void)!hipFree(dc);
  (void)!hipFree(doo);
  return e == hipSuccess ? PIC_OK : PIC_ERR_DEVICE;
}

}  // extern "C"
