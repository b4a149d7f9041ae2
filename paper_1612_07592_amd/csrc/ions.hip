// Mobile ions of the laser-solid runs (Wan et al., Sec. III, where the ions'
// share of the absorbed laser energy is reported): loading, the relativistic
// Boris push with charge q and mass M, the charge-conserving deposit of
// +q w, absorbing walls, and the ion density of every cell that the
// bremsstrahlung collision test of Eq. (4) reads as n.
//
// Ions are fewer than the electrons and slow, so they are kept simple: FP64
// in both precisions of the run (the fields are read in the run's precision),
// one thread per ion in id order, never re-sorted (heavy ions stay near the
// cells they were loaded in, in cell order); gathers read the Yee arrays
// through the caches; current and cell counts accumulate in LDS over each
// workgroup's box of nodes (64-bit integers in units of 2^-40, as the
// electrons' FP64 path) and reach memory once per touched node.
//
// Density: the push that moves an ion to x^{n+1} also counts it in its new
// cell; at the start of the next step one pass turns the counts into
// n = count w / V and clears them.  n of step n is thus the count at x^n, as
// the method needs (the collision test of step n happens before the ions
// move).
#include "particle.hpp"

namespace pic {

void fill_ion_args(const Ctx& c, IonArgs& A) {
  const Grid& g = c.g;
  A.Ni = c.Ni;
  A.dims = g.dims;
  A.ion_ppc = c.cfg.ion_ppc;
  A.nslab = c.i1 - c.i0;
  A.i0 = c.i0;
  A.ny = g.n[1];
  A.flags = c.cfg.flags;
  A.frozen_kind = c.cfg.frozen_kind;
  A.key0 = c.key0;
  A.key1 = c.key1;
  A.fp32 = c.fp32 ? 1 : 0;
  for (int a = 0; a < 3; ++a) {
    A.n[a] = g.n[a];
    A.gg[a] = g.gg[a];
    A.sz[a] = g.sz[a];
    A.dx[a] = g.dx[a];
    A.idx[a] = g.idx[a];
    A.L[a] = g.L[a];
    A.dxdt[a] = g.dx[a] / g.dt;
    A.fE[a] = c.cfg.frozen_E[a];
    A.fB[a] = c.cfg.frozen_B[a];
    A.F[a] = c.E[a];
    // B^n: the B pass leaves it in En until the E step (prescribed fields: B)
    A.F[3 + a] = (c.cfg.flags & PIC_FIELDS_FROZEN) ? c.B[a] : c.En[a];
    A.J[a] = c.J[a];
    A.x[a] = c.ix[a];
    A.p[a] = c.ip[a];
  }
  A.fa = c.cfg.frozen_a;
  A.invV = g.invV;
  A.dt = g.dt;
  A.hq = 0.5 * g.dt * (c.iq / c.imass);
  A.qw = -(c.iq * c.iw);
  A.iwv = c.iw * g.invV;
  A.tn = (double)c.step * g.dt;
  A.alive = c.ialive;
  A.count = c.icount;
  A.ni = c.ni;
  A.ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
}

namespace {

// cell of a position (nearest cell, clamped to the box), linear index
__device__ inline int64_t ion_cell(const IonArgs& A, const double* x) {
  int ci[3] = {0, 0, 0};
  for (int a = 0; a < A.dims; ++a) {
    int q = (int)floor(x[a] * A.idx[a]);
    q = q < 0 ? 0 : (q > A.n[a] - 1 ? A.n[a] - 1 : q);
    ci[a] = q;
  }
  return ci[0] + (int64_t)A.n[0] * (ci[1] + (int64_t)A.n[1] * ci[2]);
}

// Ion j of the slab cell with rank j / ion_ppc (the electrons' rank order),
// at rest, uniform in the cell: Philox counter (j, 0xFFFFFFFE, 0, 0).
__global__ __launch_bounds__(kBlock) void k_ion_init(const IonArgs A) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= A.Ni) return;
  const int64_t rank = e / A.ion_ppc;
  const int c3[3] = {(int)(rank % A.nslab) + A.i0, A.dims >= 2 ? (int)((rank / A.nslab) % A.ny) : 0,
                     A.dims >= 3 ? (int)((rank / A.nslab) / A.ny) : 0};
  const U4 r = philox4x32_10((uint32_t)e, 0xFFFFFFFEu, 0u, 0u, A.key0, A.key1);
  double x[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < A.dims; ++a) {
    x[a] = ((double)c3[a] + unif32(r.v[a])) * A.dx[a];
    A.x[a][e] = x[a];
  }
  for (int a = 0; a < 3; ++a) A.p[a][e] = 0.0;
  A.alive[e] = 1;
  atomicAdd(A.count + ion_cell(A, x), 1u);
}

__global__ __launch_bounds__(kBlock) void k_ion_clear(const IonArgs A) {
  const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (m < A.ncell) A.count[m] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_ion_count(const IonArgs A) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= A.Ni || !A.alive[e]) return;
  double x[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < A.dims; ++a) x[a] = A.x[a][e];
  atomicAdd(A.count + ion_cell(A, x), 1u);
}

__global__ __launch_bounds__(kBlock) void k_ion_density(const IonArgs A) {
  const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (m >= A.ncell) return;
  A.ni[m] = (double)A.count[m] * A.iwv;
  A.count[m] = 0u;
}

// Yee component as FP64, from arrays of the run's precision
template <class FT>
struct IonField {
  const FT* const* F;
  Idx<double> I;
  __device__ inline double operator()(int c, int i, int j, int k) const {
    return (double)F[c][I(i, j, k)];
  }
};

// Workgroup = 256 consecutive ions (the loading order is cell order and
// heavy ions stay near their cells, so a chunk covers a few cells).  As in
// the electron kernel, lanes take the chunk's ions with a stride, the
// chunk's box of nodes is reduced first and, when it fits, the current and
// the cell counts accumulate in LDS and go to memory once per touched node;
// otherwise straight to global memory.
constexpr int kIonBoxNodes = 1024;

template <int D>
struct IonDeal {
  static constexpr uint32_t value = D == 2 ? 4u : (D == 3 ? 8u : 16u);
};

// one ion: gather E^n, B^n at x^n; relativistic Boris push of the momentum
// per unit mass with (dt/2)(q/M); x^{n+1} = x^n + v dt; deposit; walls; count
template <int D, class FT>
__global__ __launch_bounds__(kBlock) void k_ion_step(const IonArgs A) {
  __shared__ int s_lo[3], s_hi[3];
  __shared__ unsigned long long sJ[3 * kIonBoxNodes];
  __shared__ uint32_t sC[kIonBoxNodes];
  constexpr uint32_t kDeal = IonDeal<D>::value;
  constexpr uint32_t kRow = kBlock / kDeal;
  const uint32_t t = threadIdx.x;
  const int64_t e = (int64_t)blockIdx.x * kBlock + (int64_t)((t % kRow) * kDeal + t / kRow);
  const bool live = e < A.Ni && A.alive[e] != 0;
  const bool frozen = (A.flags & PIC_FIELDS_FROZEN) != 0;
  double x[3] = {0.0, 0.0, 0.0};
  int bb[3] = {0, 0, 0};
  if (live) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      x[a] = A.x[a][e];
      bb[a] = (int)floor(x[a] * A.idx[a]) - 1;
    }
  }
  // the chunk's box: deposit windows [bb, bb + 3] (cells of x^{n+1} lie in
  // [bb, bb + 2], inside it)
  if (t < 3) { s_lo[t] = 0x7fffffff; s_hi[t] = -0x7fffffff; }
  __syncthreads();
  if (live) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      atomicMin(&s_lo[a], bb[a]);
      atomicMax(&s_hi[a], bb[a] + 3);
    }
  }
  __syncthreads();
  int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
  int nodes = 0;
  if (s_lo[0] <= s_hi[0]) {
    nodes = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      lo[a] = s_lo[a];
      ext[a] = s_hi[a] - s_lo[a] + 1;
      nodes *= ext[a];
    }
  }
  const bool tiled = nodes > 0 && nodes <= kIonBoxNodes;
  if (tiled) {
    for (int l = t; l < nodes; l += kBlock) {
      sJ[l] = 0ull;
      sJ[nodes + l] = 0ull;
      sJ[2 * nodes + l] = 0ull;
      sC[l] = 0u;
    }
  }
  __syncthreads();
  const Idx<double> I{A.gg[0], A.gg[1], A.gg[2], A.sz[0], A.sz[1]};
  if (live) {
    double px = A.p[0][e], py = A.p[1][e], pz = A.p[2][e];
    double E[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0};
    if (frozen) {
      if (A.frozen_kind == PIC_FROZEN_UNIFORM) {
        for (int a = 0; a < 3; ++a) { E[a] = A.fE[a]; B[a] = A.fB[a]; }
      } else {
        const double phi = A.tn - x[0];
        if (phi > 0.0) {
          const double v = A.fa * sin(phi);
          E[1] = v;
          B[2] = v;
        }
      }
    } else {
      const IonField<FT> f{(const FT* const*)A.F, I};
      double g[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < D; ++a) g[a] = x[a] * A.idx[a];
      E[0] = gather<double, D, 1, 0, 0>(f, 0, g);
      E[1] = gather<double, D, 0, 1, 0>(f, 1, g);
      E[2] = gather<double, D, 0, 0, 1>(f, 2, g);
      B[0] = gather<double, D, 0, 1, 1>(f, 3, g);
      B[1] = gather<double, D, 1, 0, 1>(f, 4, g);
      B[2] = gather<double, D, 1, 1, 0>(f, 5, g);
    }
    // Boris: half electric kick, magnetic rotation, half electric kick
    const double hq = A.hq;
    const double umx = px + hq * E[0], umy = py + hq * E[1], umz = pz + hq * E[2];
    const double gm = sqrt(1.0 + (umx * umx + umy * umy + umz * umz));
    const double fq = hq / gm;
    const double tx = fq * B[0], ty = fq * B[1], tz = fq * B[2];
    const double sf = 2.0 / (1.0 + (tx * tx + ty * ty + tz * tz));
    const double sx = sf * tx, sy = sf * ty, sz = sf * tz;
    const double upx = umx + (umy * tz - umz * ty);
    const double upy = umy + (umz * tx - umx * tz);
    const double upz = umz + (umx * ty - umy * tx);
    const double uqx = umx + (upy * sz - upz * sy);
    const double uqy = umy + (upz * sx - upx * sz);
    const double uqz = umz + (upx * sy - upy * sx);
    px = uqx + hq * E[0];
    py = uqy + hq * E[1];
    pz = uqz + hq * E[2];
    const double gamma = sqrt(1.0 + (px * px + py * py + pz * pz));
    A.p[0][e] = px;
    A.p[1][e] = py;
    A.p[2][e] = pz;
    const double ig = 1.0 / gamma;
    const double v[3] = {px * ig, py * ig, pz * ig};
    double x1[3] = {x[0], x[1], x[2]};
#pragma unroll
    for (int a = 0; a < D; ++a) x1[a] = x[a] + v[a] * A.dt;
    if (!frozen) {
      if (tiled) {
        const LdsCurrent J{sJ, lo[0], lo[1], lo[2], ext[0], ext[1], nodes};
        deposit<double, D>(A, J, x, x1, v, A.qw);
      } else {
        const GlobalCurrent J{{A.J[0], A.J[1], A.J[2]}, I};
        deposit<double, D>(A, J, x, x1, v, A.qw);
      }
    }
    bool out = false;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      A.x[a][e] = x1[a];
      if (x1[a] < 0.0 || x1[a] >= A.L[a]) out = true;
    }
    if (out) {
      A.alive[e] = 0;
    } else if (tiled) {
      int ci[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < D; ++a) ci[a] = (int)floor(x1[a] * A.idx[a]);
      atomicAdd(sC + (ci[0] - lo[0]) + ext[0] * ((ci[1] - lo[1]) + ext[1] * (ci[2] - lo[2])), 1u);
    } else {
      atomicAdd(A.count + ion_cell(A, x1), 1u);
    }
  }
  if (!tiled) return;  // block-uniform
  __syncthreads();
  for (int l = t; l < nodes; l += kBlock) {
    const int q0 = l % ext[0], r0 = l / ext[0];
    const int i = q0 + lo[0];
    const int j = (D >= 2 ? r0 % ext[1] : 0) + lo[1];
    const int k = (D == 3 ? r0 / ext[1] : 0) + lo[2];
    const int64_t m = I(i, j, k);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const unsigned long long q = sJ[c * nodes + l];
      if (q != 0ull) atomicAdd(A.J[c] + m, q);
    }
    const uint32_t n = sC[l];  // nonzero only at cells inside the box of the grid
    if (n != 0u) atomicAdd(A.count + i + (int64_t)A.n[0] * (j + (int64_t)A.n[1] * k), n);
  }
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <class FT>
void launch_step_ft(const IonArgs& A, hipStream_t s) {
  if (A.dims == 1) hipLaunchKernelGGL((k_ion_step<1, FT>), dim3(grid_of(A.Ni)), dim3(kBlock), 0, s, A);
  else if (A.dims == 2) hipLaunchKernelGGL((k_ion_step<2, FT>), dim3(grid_of(A.Ni)), dim3(kBlock), 0, s, A);
  else hipLaunchKernelGGL((k_ion_step<3, FT>), dim3(grid_of(A.Ni)), dim3(kBlock), 0, s, A);
}

}  // namespace

void launch_ion_init(const IonArgs& A, hipStream_t s) {
  if (A.Ni <= 0) return;
  hipLaunchKernelGGL(k_ion_clear, dim3(grid_of(A.ncell)), dim3(kBlock), 0, s, A);
  hipLaunchKernelGGL(k_ion_init, dim3(grid_of(A.Ni)), dim3(kBlock), 0, s, A);
}

void launch_ion_recount(const IonArgs& A, hipStream_t s) {
  if (A.Ni <= 0) return;
  hipLaunchKernelGGL(k_ion_clear, dim3(grid_of(A.ncell)), dim3(kBlock), 0, s, A);
  hipLaunchKernelGGL(k_ion_count, dim3(grid_of(A.Ni)), dim3(kBlock), 0, s, A);
}

void launch_ion_density(const IonArgs& A, hipStream_t s) {
  if (A.Ni <= 0) return;
  hipLaunchKernelGGL(k_ion_density, dim3(grid_of(A.ncell)), dim3(kBlock), 0, s, A);
}

void launch_ion_step(const IonArgs& A, hipStream_t s) {
  if (A.Ni <= 0) return;
  if (A.fp32) launch_step_ft<float>(A, s);
  else launch_step_ft<double>(A, s);
}

}  // namespace pic
