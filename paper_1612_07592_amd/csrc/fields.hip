// Supporting kernels: Yee field solve (B half step, E full step with
// first-order Mur faces), the current-sheet laser source, electron and ion
// loading, and the fixed-order reductions behind pic_emission_stats.
#include "pic_internal.hpp"
#include "philox.hpp"
#include "fpmath.hpp"

namespace pic {


// Multiplier and shift for division by d of any n < 2^31: s = 31 + ceil(log2
// d), mg = floor(2^s / d) + 1 < 2^32.  With mg d = 2^s + e, 0 < e <= d,
// n mg / 2^s = n / d + n e / (d 2^s) and n e / (d 2^s) < 2^31 / 2^s <= 1 / d,
// which never reaches the next multiple of 1 / d above n / d, so the floor is
// floor(n / d) (division by invariant integers, Granlund and Montgomery 1994).
static void div_magic(uint32_t d, uint32_t& mg, int& sh) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  sh = 31 + l;
  mg = (uint32_t)((1ull << sh) / d + 1);
}

static FieldArgs field_args(const Grid& g) {
  FieldArgs a{};
  for (int d = 0; d < 3; ++d) {
    a.n[d] = g.n[d]; a.act[d] = g.act[d]; a.gg[d] = g.gg[d]; a.sz[d] = g.sz[d];
    a.hd[d] = g.hd[d]; a.cd[d] = g.cd[d]; a.cm[d] = g.cm[d];
  }
  a.dt = g.dt;
  a.srcfac = -2.0 / g.dx[0];
  a.i_src = g.i_src;
  a.nsrc_y = g.nsrc_y;
  a.nfield = g.nfield;
  div_magic((uint32_t)g.sz[0], a.mg0, a.sh0);
  div_magic((uint32_t)g.sz[1], a.mg1, a.sh1);
  return a;
}

// (32-bit arithmetic: the field arrays hold fewer than 2^31 nodes)
__device__ inline int64_t fidx(const FieldArgs& A, int i, int j, int k) {
  return (int64_t)((i + A.gg[0]) + A.sz[0] * ((j + A.gg[1]) + A.sz[1] * (k + A.gg[2])));
}

__device__ inline void decode(const FieldArgs& A, int64_t m, int& i, int& j, int& k) {
  const uint32_t mm = (uint32_t)m;
  const uint32_t r = (uint32_t)(((uint64_t)mm * A.mg0) >> A.sh0);
  const uint32_t q = (uint32_t)(((uint64_t)r * A.mg1) >> A.sh1);
  i = (int)(mm - r * (uint32_t)A.sz[0]) - A.gg[0];
  j = (int)(r - q * (uint32_t)A.sz[1]) - A.gg[1];
  k = (int)q - A.gg[2];
}

// half-integer stagger of E_c / B_c along axis a
__device__ inline int estag(int c, int a) { return c == a; }
__device__ inline int bstag(int c, int a) { return c != a; }

// valid node of component c (isB: magnetic) on the Yee lattice
__device__ inline bool in_range(const FieldArgs& A, bool isB, int c, int i, int j, int k) {
  const int ijk[3] = {i, j, k};
  for (int a = 0; a < 3; ++a) {
    if (!A.act[a]) { if (ijk[a] != 0) return false; continue; }
    const bool half = isB ? bstag(c, a) : estag(c, a);
    const int hi = half ? A.n[a] : A.n[a] + 1;
    if (ijk[a] < 0 || ijk[a] >= hi) return false;
  }
  return true;
}

// Both B half steps of a step, which use the same E^n, in one pass over the
// nodes: B^n = B^{n-1/2} - (dt/2) curl E^n into Bn (the field the push
// gathers) and B^{n+1/2} = B^n - (dt/2) curl E^n back into B (the field the E
// step uses).  Each is formed exactly as a separate half step forms it.  Bn
// gets every node (invalid B nodes copy B, which never changes there).  J is
// cleared for the step's deposit.
template <class R>
__device__ __forceinline__ void b_both_node(const FieldArgs& A, const R* __restrict__ Ex,
                                            const R* __restrict__ Ey, const R* __restrict__ Ez,
                                            R* Bx, R* By, R* Bz, R* Bnx, R* Bny, R* Bnz,
                                            unsigned long long* Jx, unsigned long long* Jy,
                                            unsigned long long* Jz, const int64_t m) {
  if (m >= A.nfield) return;
  int i, j, k;
  decode(A, m, i, j, k);
  const int64_t s1 = A.sz[0], s2 = (int64_t)A.sz[0] * A.sz[1];  // +1 along y, z
  Jx[m] = 0ull; Jy[m] = 0ull; Jz[m] = 0ull;
  {  // dBx/dt = -dEz/dy + dEy/dz
    const R b = Bx[m];
    if (in_range(A, true, 0, i, j, k)) {
      const R ty = A.act[1] ? R(A.hd[1]) * (Ez[m + s1] - Ez[m]) : R(0);
      const R tz = A.act[2] ? R(A.hd[2]) * (Ey[m + s2] - Ey[m]) : R(0);
      R b1 = b;
      if (A.act[1]) b1 = b1 - ty;
      if (A.act[2]) b1 = b1 + tz;
      R b2 = b1;
      if (A.act[1]) b2 = b2 - ty;
      if (A.act[2]) b2 = b2 + tz;
      Bnx[m] = b1;
      Bx[m] = b2;
    } else {
      Bnx[m] = b;
    }
  }
  {  // dBy/dt = -dEx/dz + dEz/dx
    const R b = By[m];
    if (in_range(A, true, 1, i, j, k)) {
      const R tz = A.act[2] ? R(A.hd[2]) * (Ex[m + s2] - Ex[m]) : R(0);
      const R tx = R(A.hd[0]) * (Ez[m + 1] - Ez[m]);
      R b1 = b;
      if (A.act[2]) b1 = b1 - tz;
      b1 = b1 + tx;
      R b2 = b1;
      if (A.act[2]) b2 = b2 - tz;
      b2 = b2 + tx;
      Bny[m] = b1;
      By[m] = b2;
    } else {
      Bny[m] = b;
    }
  }
  {  // dBz/dt = -dEy/dx + dEx/dy
    const R b = Bz[m];
    if (in_range(A, true, 2, i, j, k)) {
      const R tx = R(A.hd[0]) * (Ey[m + 1] - Ey[m]);
      const R ty = A.act[1] ? R(A.hd[1]) * (Ex[m + s1] - Ex[m]) : R(0);
      R b1 = b - tx;
      if (A.act[1]) b1 = b1 + ty;
      R b2 = b1 - tx;
      if (A.act[1]) b2 = b2 + ty;
      Bnz[m] = b1;
      Bz[m] = b2;
    } else {
      Bnz[m] = b;
    }
  }
}


// Ampere update of E_c at an interior node (old E, B^{n+1/2}, J^{n+1/2}).
template <class R>
__device__ inline R e_interior(const FieldArgs& A, const EPtrs& P, int c, int i, int j, int k,
                               int64_t m, double lsin, double lcos) {
  const int64_t s1 = A.sz[0], s2 = (int64_t)A.sz[0] * A.sz[1];  // -1 along y, z
  const R* Bx = (const R*)P.B[0];
  const R* By = (const R*)P.B[1];
  const R* Bz = (const R*)P.B[2];
  R e = ((const R*)P.E[c])[m];
  double jj = (double)(long long)P.J[c][m] * kJInv;
  if (c == 0) {        // dEx/dt = dBz/dy - dBy/dz - Jx
    if (A.act[1]) e = e + R(A.cd[1]) * (Bz[m] - Bz[m - s1]);
    if (A.act[2]) e = e - R(A.cd[2]) * (By[m] - By[m - s2]);
  } else if (c == 1) { // dEy/dt = dBx/dz - dBz/dx - Jy
    if (A.act[2]) e = e + R(A.cd[2]) * (Bx[m] - Bx[m - s2]);
    e = e - R(A.cd[0]) * (Bz[m] - Bz[m - 1]);
    if (i == A.i_src) {
      const int64_t s = j + (int64_t)A.nsrc_y * k;
      const double v = lsin * P.srcC[s] + lcos * P.srcS[s];
      jj = jj + A.srcfac * (P.srcA[s] * v);
    }
  } else {             // dEz/dt = dBy/dx - dBx/dy - Jz
    e = e + R(A.cd[0]) * (By[m] - By[m - 1]);
    if (A.act[1]) e = e - R(A.cd[1]) * (Bx[m] - Bx[m - s1]);
  }
  return e - R(A.dt * jj);
}

// E^{n+1} into En: interior nodes by Ampere, tangential face nodes by Mur
// (the interior neighbour's new value is recomputed here, bit-identically),
// edge/corner nodes and guards 0.
template <class R>
__device__ __forceinline__ void e_full_node(const FieldArgs& A, const EPtrs& P, double lsin,
                                            double lcos, const int c, const int64_t m) {
  if (m >= A.nfield) return;
  int i, j, k;
  decode(A, m, i, j, k);
  R* Fn = (R*)P.En[c];
  const R* Fo = (const R*)P.E[c];
  if (!in_range(A, false, c, i, j, k)) { Fn[m] = R(0); return; }
  const int ijk[3] = {i, j, k};
  int nb = 0, ax = -1;
  for (int a = 0; a < 3; ++a)
    if (A.act[a] && !estag(c, a) && (ijk[a] == 0 || ijk[a] == A.n[a])) { ++nb; ax = a; }
  if (nb == 0) { Fn[m] = e_interior<R>(A, P, c, i, j, k, m, lsin, lcos); return; }
  if (nb > 1) { Fn[m] = R(0); return; }
  int in[3] = {i, j, k};
  in[ax] += (ijk[ax] == 0) ? 1 : -1;
  const int64_t mi = fidx(A, in[0], in[1], in[2]);
  const R fin = e_interior<R>(A, P, c, in[0], in[1], in[2], mi, lsin, lcos);
  Fn[m] = Fo[mi] + R(A.cm[ax]) * (fin - Fo[m]);
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_b_both(FieldArgs A, const R* __restrict__ Ex,
                                                   const R* __restrict__ Ey, const R* __restrict__ Ez,
                                                   R* Bx, R* By, R* Bz, R* Bnx, R* Bny, R* Bnz,
                                                   unsigned long long* Jx, unsigned long long* Jy,
                                                   unsigned long long* Jz) {
  b_both_node<R>(A, Ex, Ey, Ez, Bx, By, Bz, Bnx, Bny, Bnz, Jx, Jy, Jz,
                 (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

// Every E component of node (i, j, k) is an interior Ampere node: 1 <= index
// <= n - 1 on each active axis (no tangential face, no guard), 0 on the others.
__device__ inline bool e_inner(const FieldArgs& A, int i, int j, int k) {
  const int ijk[3] = {i, j, k};
  bool in = true;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    in = in && (A.act[a] ? (ijk[a] >= 1 && ijk[a] <= A.n[a] - 1) : ijk[a] == 0);
  return in;
}

// E^{n+1} at all three components of a node.  At an interior node (nearly
// every node) the loads of all three updates are issued before the first
// store, so a thread waits on memory once rather than once per component and
// term; each value is e_interior's, in its operation order.  Other nodes take
// e_full_node per component.
template <class R>
__device__ __forceinline__ void e_full_all(const FieldArgs& A, const EPtrs& P, double lsin,
                                           double lcos, const int64_t m) {
  if (m >= A.nfield) return;
  int i, j, k;
  decode(A, m, i, j, k);
  if (!e_inner(A, i, j, k)) {
#pragma unroll
    for (int c = 0; c < 3; ++c) e_full_node<R>(A, P, lsin, lcos, c, m);
    return;
  }
  const int64_t s1 = A.sz[0], s2 = (int64_t)A.sz[0] * A.sz[1];  // -1 along y, z
  const bool ay = A.act[1] != 0, az = A.act[2] != 0;
  const R* Bx = (const R*)P.B[0];
  const R* By = (const R*)P.B[1];
  const R* Bz = (const R*)P.B[2];
  const R e0 = ((const R*)P.E[0])[m], e1 = ((const R*)P.E[1])[m], e2 = ((const R*)P.E[2])[m];
  const long long j0 = (long long)P.J[0][m], j1 = (long long)P.J[1][m], j2 = (long long)P.J[2][m];
  const R bx = Bx[m], by = By[m], bz = Bz[m];
  const R by_x = By[m - 1], bz_x = Bz[m - 1];
  R bx_y = R(0), bz_y = R(0), bx_z = R(0), by_z = R(0);
  if (ay) { bx_y = Bx[m - s1]; bz_y = Bz[m - s1]; }
  if (az) { bx_z = Bx[m - s2]; by_z = By[m - s2]; }
  // dEx/dt = dBz/dy - dBy/dz - Jx
  R x = e0;
  if (ay) x = x + R(A.cd[1]) * (bz - bz_y);
  if (az) x = x - R(A.cd[2]) * (by - by_z);
  x = x - R(A.dt * ((double)j0 * kJInv));
  // dEy/dt = dBx/dz - dBz/dx - Jy, plus the laser sheet
  R y = e1;
  if (az) y = y + R(A.cd[2]) * (bx - bx_z);
  y = y - R(A.cd[0]) * (bz - bz_x);
  double jy = (double)j1 * kJInv;
  if (i == A.i_src) {
    const int64_t s = j + (int64_t)A.nsrc_y * k;
    const double v = lsin * P.srcC[s] + lcos * P.srcS[s];
    jy = jy + A.srcfac * (P.srcA[s] * v);
  }
  y = y - R(A.dt * jy);
  // dEz/dt = dBy/dx - dBx/dy - Jz
  R z = e2;
  z = z + R(A.cd[0]) * (by - by_x);
  if (ay) z = z - R(A.cd[1]) * (bx - bx_y);
  z = z - R(A.dt * ((double)j2 * kJInv));
  ((R*)P.En[0])[m] = x;
  ((R*)P.En[1])[m] = y;
  ((R*)P.En[2])[m] = z;
}

// One thread updates the three components of its node, so each B value is
// fetched by the threads of one pass instead of two component passes.
template <class R>
__global__ __launch_bounds__(kBlock) void k_e_full(FieldArgs A, EPtrs P, double lsin, double lcos) {
  e_full_all<R>(A, P, lsin, lcos, (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

// Batched forms: the workgroups of every run laid end to end (run j owns
// blocks [first[j], first[j+1])); each run is updated exactly as alone.
__device__ inline int batch_job(const uint32_t* __restrict__ first, int njobs, uint32_t b) {
  int lo = 0, hi = njobs - 1;  // largest j with first[j] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_b_both_batch(const FieldJob* __restrict__ tab,
                                                         const uint32_t* __restrict__ first,
                                                         int njobs) {
  const int j = batch_job(first, njobs, blockIdx.x);
  const FieldJob& F = tab[j];
  b_both_node<R>(F.A, (const R*)F.P.E[0], (const R*)F.P.E[1], (const R*)F.P.E[2], (R*)F.Bw[0],
                 (R*)F.Bw[1], (R*)F.Bw[2], (R*)F.P.En[0], (R*)F.P.En[1], (R*)F.P.En[2], F.Jw[0],
                 F.Jw[1], F.Jw[2], (int64_t)(blockIdx.x - first[j]) * kBlock + threadIdx.x);
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_e_full_batch(const FieldJob* __restrict__ tab,
                                                         const uint32_t* __restrict__ first,
                                                         int njobs) {
  const int j = batch_job(first, njobs, blockIdx.x);
  const FieldJob& F = tab[j];
  e_full_all<R>(F.A, F.P, F.lsin, F.lcos, (int64_t)(blockIdx.x - first[j]) * kBlock + threadIdx.x);
}

uint32_t field_blocks(const Ctx& c) { return (uint32_t)((c.g.nfield + kBlock - 1) / kBlock); }

void fill_field_job(const Ctx& c, double lsin, double lcos, FieldJob& F) {
  F.A = field_args(c.g);
  for (int d = 0; d < 3; ++d) {
    F.P.E[d] = c.E[d]; F.P.En[d] = c.En[d]; F.P.B[d] = c.B[d]; F.P.J[d] = c.J[d];
    F.Bw[d] = c.B[d]; F.Jw[d] = c.J[d];
  }
  F.P.srcA = c.srcA; F.P.srcC = c.srcC; F.P.srcS = c.srcS;
  F.lsin = lsin;
  F.lcos = lcos;
}

void launch_b_both_batch(bool fp32, const FieldJob* tab, const uint32_t* first, int njobs,
                         uint32_t total, hipStream_t s) {
  if (njobs <= 0 || total == 0) return;
  if (fp32) hipLaunchKernelGGL(k_b_both_batch<float>, dim3(total), dim3(kBlock), 0, s, tab, first, njobs);
  else hipLaunchKernelGGL(k_b_both_batch<double>, dim3(total), dim3(kBlock), 0, s, tab, first, njobs);
}

void launch_e_full_batch(bool fp32, const FieldJob* tab, const uint32_t* first, int njobs,
                         uint32_t total, hipStream_t s) {
  if (njobs <= 0 || total == 0) return;
  if (fp32) hipLaunchKernelGGL(k_e_full_batch<float>, dim3(total), dim3(kBlock), 0, s, tab, first, njobs);
  else hipLaunchKernelGGL(k_e_full_batch<double>, dim3(total), dim3(kBlock), 0, s, tab, first, njobs);
}

// B^n goes into the E step's output buffer En, which is free until the E step
void launch_b_both(const Ctx& c, hipStream_t s) {
  const FieldArgs A = field_args(c.g);
  const unsigned blocks = (unsigned)((A.nfield + kBlock - 1) / kBlock);
  if (c.fp32)
    hipLaunchKernelGGL(k_b_both<float>, dim3(blocks), dim3(kBlock), 0, s, A, (const float*)c.E[0],
                       (const float*)c.E[1], (const float*)c.E[2], (float*)c.B[0], (float*)c.B[1],
                       (float*)c.B[2], (float*)c.En[0], (float*)c.En[1], (float*)c.En[2], c.J[0], c.J[1],
                       c.J[2]);
  else
    hipLaunchKernelGGL(k_b_both<double>, dim3(blocks), dim3(kBlock), 0, s, A, (const double*)c.E[0],
                       (const double*)c.E[1], (const double*)c.E[2], (double*)c.B[0], (double*)c.B[1],
                       (double*)c.B[2], (double*)c.En[0], (double*)c.En[1], (double*)c.En[2], c.J[0],
                       c.J[1], c.J[2]);
}

void launch_e_full(Ctx& c, double lsin, double lcos, hipStream_t s) {
  const FieldArgs A = field_args(c.g);
  EPtrs P{};
  for (int d = 0; d < 3; ++d) {
    P.E[d] = c.E[d]; P.En[d] = c.En[d]; P.B[d] = c.B[d]; P.J[d] = c.J[d];
  }
  P.srcA = c.srcA; P.srcC = c.srcC; P.srcS = c.srcS;
  const unsigned blocks = (unsigned)((A.nfield + kBlock - 1) / kBlock);
  if (c.fp32)
    hipLaunchKernelGGL(k_e_full<float>, dim3(blocks), dim3(kBlock), 0, s, A, P, lsin, lcos);
  else
    hipLaunchKernelGGL(k_e_full<double>, dim3(blocks), dim3(kBlock), 0, s, A, P, lsin, lcos);
  for (int d = 0; d < 3; ++d) { void* t = c.E[d]; c.E[d] = c.En[d]; c.En[d] = t; }
}

// ---- loading ----------------------------------------------------------------
struct InitArgs {
  int64_t N;
  int dims, ppc, nslab, i0, ny;
  double dx[3], wgt;
  uint32_t key0, key1;
  void* x[3];
  void* p[3];
  double* tau;
  double* taub;  // free-path bremsstrahlung only
  double* w;
  uint32_t* id;
  double* ni;
  int64_t ncell;
  int nx, nyc;
  double nion;
  int i1;
  int fb[3];
};

// Electron e of the slab cell with rank e/ppc; cold, uniform in the cell;
// tau_0 = -ln u (Philox counter (id, 0xFFFFFFFF, 0, 0)); the first collision
// optical depth of free-path bremsstrahlung, -ln u of word 0 of counter
// (id, 0xFFFFFFFF, 1, 0).
template <class R>
__global__ __launch_bounds__(kBlock) void k_init_electrons(InitArgs A) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= A.N) return;
  const int64_t rank = e / A.ppc;
  const int ii = (int)(rank % A.nslab) + A.i0;
  const int64_t r2 = rank / A.nslab;
  const int jj = A.dims >= 2 ? (int)(r2 % A.ny) : 0;
  const int kk = A.dims >= 3 ? (int)(r2 / A.ny) : 0;
  const U4 r = philox4x32_10((uint32_t)e, 0xFFFFFFFFu, 0u, 0u, A.key0, A.key1);
  if constexpr (sizeof(R) == 4) {  // fixed point in cells, fb fraction bits
    const int c3[3] = {ii, jj, kk};
    for (int a = 0; a < A.dims; ++a)
      ((int*)A.x[a])[e] = (c3[a] << A.fb[a]) + (int)(unif32(r.v[a]) * ldexp(1.0, A.fb[a]));
  } else {
    ((R*)A.x[0])[e] = (R)(((double)ii + unif32(r.v[0])) * A.dx[0]);
    if (A.dims >= 2) ((R*)A.x[1])[e] = (R)(((double)jj + unif32(r.v[1])) * A.dx[1]);
    if (A.dims >= 3) ((R*)A.x[2])[e] = (R)(((double)kk + unif32(r.v[2])) * A.dx[2]);
  }
  for (int a = 0; a < 3; ++a) ((R*)A.p[a])[e] = R(0);
  A.tau[e] = -fp_log(unif32(r.v[3]));
  if (A.taub) {
    const U4 rb = philox4x32_10((uint32_t)e, 0xFFFFFFFFu, 1u, 0u, A.key0, A.key1);
    A.taub[e] = -fp_log(unif32(rb.v[0]));
  }
  A.w[e] = A.wgt;
  A.id[e] = (uint32_t)e;
}

__global__ __launch_bounds__(kBlock) void k_init_ions(InitArgs A) {
  const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (m >= A.ncell) return;
  const int i = (int)(m % A.nx);
  A.ni[m] = (i >= A.i0 && i < A.i1) ? A.nion : 0.0;
}

void launch_init_electrons(const Ctx& c, hipStream_t s) {
  InitArgs A{};
  A.N = c.N;
  A.dims = c.g.dims;
  A.ppc = c.cfg.ppc;
  A.nslab = c.i1 - c.i0;
  A.i0 = c.i0;
  A.i1 = c.i1;
  A.ny = c.g.n[1];
  for (int d = 0; d < 3; ++d) {
    A.dx[d] = c.g.dx[d]; A.x[d] = c.x[d]; A.p[d] = c.p[d]; A.fb[d] = c.g.fb[d];
  }
  A.wgt = c.wgt;
  A.key0 = c.key0; A.key1 = c.key1;
  A.tau = c.tau; A.taub = c.taub; A.w = c.w; A.id = c.id; A.ni = c.ni;
  A.ncell = (int64_t)c.g.n[0] * c.g.n[1] * c.g.n[2];
  A.nx = c.g.n[0];
  A.nion = c.cfg.ne_over_nc / (double)c.cfg.charge_state;
  if (A.N > 0) {
    const unsigned blocks = (unsigned)((A.N + kBlock - 1) / kBlock);
    if (c.fp32) hipLaunchKernelGGL(k_init_electrons<float>, dim3(blocks), dim3(kBlock), 0, s, A);
    else hipLaunchKernelGGL(k_init_electrons<double>, dim3(blocks), dim3(kBlock), 0, s, A);
  }
  const unsigned cb = (unsigned)((A.ncell + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_init_ions, dim3(cb), dim3(kBlock), 0, s, A);
}

// ---- reductions -------------------------------------------------------------
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

__device__ inline void neu_add(double& s, double& c, double v) {
  const double t = s + v;
  if (fabs(s) >= fabs(v)) c += (s - t) + v;
  else c += (v - t) + s;
  s = t;
}

// fixed-order tree over a block: (s, c) pairs and u64 counters
template <int NS, int NC>
__device__ inline void block_reduce(double (&s)[NS], double (&c)[NS], unsigned long long (&n)[NC]) {
  __shared__ double ss[NS][kRedThreads], sc[NS][kRedThreads];
  __shared__ unsigned long long sn[NC][kRedThreads];
  const int t = threadIdx.x;
  for (int q = 0; q < NS; ++q) { ss[q][t] = s[q]; sc[q][t] = c[q]; }
  for (int q = 0; q < NC; ++q) sn[q][t] = n[q];
  __syncthreads();
  for (int h = kRedThreads / 2; h >= 1; h >>= 1) {
    if (t < h) {
      for (int q = 0; q < NS; ++q) {
        double a = ss[q][t], b = sc[q][t];
        neu_add(a, b, ss[q][t + h]);
        b += sc[q][t + h];
        ss[q][t] = a; sc[q][t] = b;
      }
      for (int q = 0; q < NC; ++q) sn[q][t] += sn[q][t + h];
    }
    __syncthreads();
  }
  for (int q = 0; q < NS; ++q) { s[q] = ss[q][0]; c[q] = sc[q][0]; }
  for (int q = 0; q < NC; ++q) n[q] = sn[q][0];
}

// Pass 1: per-block partial sums of the wave slots, the electrons' and mobile
// ions' kinetic energy and live counts, and the field energy.  Contiguous
// chunks per block.
struct RedArgs {
  const unsigned long long* scnt;
  const double* ssum;
  int64_t nslots;
  const void* p[3];
  const double* w;
  const uint32_t* id;
  int64_t N;
  const void* F[6];
  int64_t nfield;
  const double* ip[3];
  const uint8_t* ialive;
  int64_t Ni;
  double iwm;   // ion weight times mass (electron masses)
  unsigned long long* out_cnt;
  double* out_sum;
};

template <class R>
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(const RedArgs A) {
  constexpr int NS = kRedSum;   // kept0, kept1, dropped, e_kin, field, e_kin ions
  constexpr int NC = kRedCnt;
  double s[NS], c[NS];
  for (int q = 0; q < NS; ++q) { s[q] = 0.0; c[q] = 0.0; }
  unsigned long long n[NC];
  for (int q = 0; q < NC; ++q) n[q] = 0ull;
  const int b = blockIdx.x, t = threadIdx.x;
  // slots
  {
    const int64_t per = (A.nslots + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)b * per, hi = min(A.nslots, lo + per);
    for (int64_t q = lo + t; q < hi; q += kRedThreads) {
      for (int z = 0; z < kSlotCnt; ++z) n[z] += A.scnt[q * kSlotCnt + z];
      for (int z = 0; z < 3; ++z) {
        neu_add(s[z], c[z], A.ssum[q * kSlotSum + 2 * z]);
        c[z] += A.ssum[q * kSlotSum + 2 * z + 1];
      }
    }
  }
  // electrons
  {
    const R* px = (const R*)A.p[0];
    const R* py = (const R*)A.p[1];
    const R* pz = (const R*)A.p[2];
    const int64_t per = (A.N + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)b * per, hi = min(A.N, lo + per);
    for (int64_t e = lo + t; e < hi; e += kRedThreads) {
      if (A.id[e] & kDead) continue;
      const double a = (double)px[e], bb = (double)py[e], cc = (double)pz[e];
      const double g = sqrt(1.0 + (a * a + bb * bb + cc * cc));
      neu_add(s[3], c[3], A.w[e] * (g - 1.0));
      n[kSlotCnt] += 1ull;
    }
  }
  // mobile ions
  {
    const int64_t per = (A.Ni + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)b * per, hi = min(A.Ni, lo + per);
    for (int64_t e = lo + t; e < hi; e += kRedThreads) {
      if (!A.ialive[e]) continue;
      const double a = A.ip[0][e], bb = A.ip[1][e], cc = A.ip[2][e];
      const double g = sqrt(1.0 + (a * a + bb * bb + cc * cc));
      neu_add(s[5], c[5], A.iwm * (g - 1.0));
      n[kSlotCnt + 1] += 1ull;
    }
  }
  // fields
  {
    const R* const* F = (const R* const*)A.F;
    const int64_t per = (A.nfield + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)b * per, hi = min(A.nfield, lo + per);
    for (int64_t m = lo + t; m < hi; m += kRedThreads) {
      double v = 0.0;
      for (int q = 0; q < 6; ++q) v += (double)F[q][m] * (double)F[q][m];
      neu_add(s[4], c[4], v);
    }
  }
  block_reduce<NS, NC>(s, c, n);
  if (t == 0) {
    for (int q = 0; q < NC; ++q) A.out_cnt[(int64_t)b * NC + q] = n[q];
    for (int q = 0; q < NS; ++q) {
      A.out_sum[(int64_t)b * 2 * NS + 2 * q] = s[q];
      A.out_sum[(int64_t)b * 2 * NS + 2 * q + 1] = c[q];
    }
  }
}

// Pass 2: one block folds the partials in block order.
__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const unsigned long long* in_cnt,
                                                              const double* in_sum, int nblk,
                                                              unsigned long long* out_cnt,
                                                              double* out_sum) {
  constexpr int NS = kRedSum;
  constexpr int NC = kRedCnt;
  double s[NS], c[NS];
  for (int q = 0; q < NS; ++q) { s[q] = 0.0; c[q] = 0.0; }
  unsigned long long n[NC];
  for (int q = 0; q < NC; ++q) n[q] = 0ull;
  const int t = threadIdx.x;
  const int per = (nblk + kRedThreads - 1) / kRedThreads;
  for (int b = t * per; b < min(nblk, (t + 1) * per); ++b) {
    for (int q = 0; q < NC; ++q) n[q] += in_cnt[(int64_t)b * NC + q];
    for (int q = 0; q < NS; ++q) {
      neu_add(s[q], c[q], in_sum[(int64_t)b * 2 * NS + 2 * q]);
      c[q] += in_sum[(int64_t)b * 2 * NS + 2 * q + 1];
    }
  }
  block_reduce<NS, NC>(s, c, n);
  if (t == 0) {
    for (int q = 0; q < NC; ++q) out_cnt[q] = n[q];
    for (int q = 0; q < NS; ++q) out_sum[q] = s[q] + c[q];
  }
}

int reduce_scratch_cnt() { return kRedBlocks * kRedCnt + kRedCnt; }
int reduce_scratch_sum() { return kRedBlocks * 2 * kRedSum + kRedSum; }

void launch_stats_reduce(const Ctx& c, unsigned long long* cnt_out, double* sum_out, hipStream_t s) {
  RedArgs A{};
  A.scnt = c.slot_cnt;
  A.ssum = c.slot_sum;
  A.nslots = c.nslots;
  A.w = c.w;
  A.id = c.id;
  A.N = c.N;
  for (int a = 0; a < 3; ++a) {
    A.p[a] = c.p[a];
    A.F[a] = c.E[a];
    A.F[3 + a] = c.B[a];
    A.ip[a] = c.ip[a];
  }
  A.nfield = c.g.nfield;
  A.ialive = c.ialive;
  A.Ni = c.Ni;
  A.iwm = c.iw * c.imass;
  A.out_cnt = c.red_cnt;
  A.out_sum = c.red_sum;
  unsigned long long* fc = c.red_cnt + kRedBlocks * kRedCnt;
  double* fs = c.red_sum + kRedBlocks * 2 * kRedSum;
  if (c.fp32) hipLaunchKernelGGL(k_reduce_partial<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, s, A);
  else hipLaunchKernelGGL(k_reduce_partial<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, s, A);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, s, c.red_cnt, c.red_sum,
                     kRedBlocks, fc, fs);
  hipMemcpyAsync(cnt_out, fc, sizeof(unsigned long long) * kRedCnt, hipMemcpyDeviceToHost, s);
  hipMemcpyAsync(sum_out, fs, sizeof(double) * kRedSum, hipMemcpyDeviceToHost, s);
}

// ---- Philox exposure -------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1,
                                                   uint32_t* out, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const U4 r = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
  for (int q = 0; q < 4; ++q) out[4 * i + q] = r.v[q];
}

void launch_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, uint64_t n,
                   hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, ctr,
                     k0, k1, out, n);
}

}  // namespace pic
