// The per-electron step on gfx950: one thread per electron, wave64.
//
// Per electron, in the order of the method (Wan et al., Sec. II):
//   Philox draw keyed by (id, step) -> gather E^n, B^n -> Boris push ->
//   eta -> NCS optical-depth decrement and inverse-CDF photon draw ->
//   bremsstrahlung test of Eq. (4) against the cell's ion density and the
//   R2 photon-energy draw -> recoil -> photon append -> move -> current deposit.
// Photon append: one ballot per process and wave, one atomic per wave on the
// photon counter (none once the buffer is full), lane offsets from mbcnt (no
// per-lane atomics).
// Statistics: per-wave slots (exact u64 counts, FP64 Neumaier pairs), reduced
// in a fixed order on demand.
// Current: each contribution rounded to 2^-40 and added as a 64-bit integer,
// so the sum is independent of the order electrons are visited in.
//
// The FP64 instantiation evaluates every expression in the same order as the
// written method (no contraction: built with -ffp-contract=off).  The FP32
// instantiation keeps the optical depth, weights, the 52-bit brem draw
// comparison and the energy sums in FP64.
#include "particle.hpp"
#include <algorithm>
#include <type_traits>

namespace pic {

// The cold parameter block, read through the constant address space so the
// compiler issues scalar loads at the point of use.
template <class R>
using ColdPtr = const __attribute__((address_space(4))) StepCold<R>*;
template <class R>
__device__ inline ColdPtr<R> cold(const StepParams<R>& P) { return (ColdPtr<R>)P.cold; }

// FP32 path: contribution -> multiple of 2^-jbits in float arithmetic.
__device__ inline int q32(float v, float scale) { return (int)rintf(v * scale); }

// a b rounded to the nearest integer (ties to even) in one rounding: the fma
// adds 1.5 2^23, whose unit in the last place is 1, and the integer is read
// from the low bits.  Exact for |a b| < 2^22, which the current quantum
// guarantees for every contribution (one chunk's sum at a node stays below
// 2^30, 256 contributions of at most 2^22 each).
__device__ inline int round_prod(float a, float b) {
  return __float_as_int(__builtin_fmaf(a, b, 12582912.0f)) - 0x4B400000;
}

// The FP32 accessors also offer a linear form: lin(i, j, k) gives a node's
// index once, neighbours are lin + 1, lin + s1, lin + s2 (32-bit indices; the
// field arrays hold fewer than 2^31 nodes).
struct GlobalCurrent32 {
  unsigned long long* J[3];
  Idx<float> I;
  float scale;
  int shift;  // 40 - jbits
  __device__ inline void operator()(int c, int i, int j, int k, float v) const {
    const int q = q32(v, scale);
    if (q != 0) atomicAdd(J[c] + I(i, j, k), (unsigned long long)((long long)q << shift));
  }
  __device__ inline int lin(int i, int j, int k) const { return (int)I(i, j, k); }
  __device__ inline int s1() const { return I.sz0; }
  __device__ inline int s2() const { return I.sz0 * I.sz1; }
  __device__ inline void add(int c, int l, float v) const {
    const int q = q32(v, scale);
    if (q != 0) atomicAdd(J[c] + l, (unsigned long long)((long long)q << shift));
  }
  // v already in units of the quantum
  __device__ inline float qscale() const { return scale; }
  __device__ inline void addq(int c, int l, float v) const {
    const int q = (int)rintf(v);
    if (q != 0) atomicAdd(J[c] + l, (unsigned long long)((long long)q << shift));
  }
  __device__ inline void addq2(int c, int l, float a, float b) const {
    const int q = round_prod(a, b);
    if (q != 0) atomicAdd(J[c] + l, (unsigned long long)((long long)q << shift));
  }
};

struct LdsCurrent32 {
  int* T;
  int lo0, lo1, lo2, e0, e1, nodes;
  float scale;
  __device__ inline void operator()(int c, int i, int j, int k, float v) const {
    // unconditional: adding 0 is harmless and keeps the wave convergent
    atomicAdd(T + c * nodes + (i - lo0) + e0 * ((j - lo1) + e1 * (k - lo2)), q32(v, scale));
  }
  __device__ inline int lin(int i, int j, int k) const { return (i - lo0) + e0 * ((j - lo1) + e1 * (k - lo2)); }
  __device__ inline int s1() const { return e0; }
  __device__ inline int s2() const { return e0 * e1; }
  __device__ inline void add(int c, int l, float v) const { atomicAdd(T + c * nodes + l, q32(v, scale)); }
  __device__ inline float qscale() const { return scale; }
  // zero contributions are skipped: a wave whose lanes all carry zero for a
  // node (electrons that did not move along the flux's axis) issues no LDS
  // atomic at all
  __device__ inline void addq(int c, int l, float v) const {
    const int q = (int)rintf(v);
    if (q != 0) atomicAdd(T + c * nodes + l, q);
  }
  __device__ inline void addq2(int c, int l, float a, float b) const {
    const int q = round_prod(a, b);
    if (q != 0) atomicAdd(T + c * nodes + l, q);
  }
};

// FP32 path: the same interpolation from fixed-point positions q (cell units,
// fb fraction bits); node index and in-cell fraction come from integer
// arithmetic, so they are as fine far from the origin as near it.
__device__ inline void split_q(int q, int S, int fb, float iqs, int& i, float& f) {
  const int qs = q - (S << (fb - 1));    // half-integer stagger: shift by half a cell
  i = qs >> fb;                          // floor (arithmetic shift)
  f = (float)(qs & ((1 << fb) - 1)) * iqs;
}

// The node/fraction pairs of one position for both staggers of every axis.
struct Splits {
  int i[3][2];
  float f[3][2];
};

template <int D>
__device__ inline Splits make_splits(const int* q, const int* fb, const float* iqs) {
  Splits s{};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    split_q(q[a], 0, fb[a], iqs[a], s.i[a][0], s.f[a][0]);
    split_q(q[a], 1, fb[a], iqs[a], s.i[a][1], s.f[a][1]);
  }
  return s;
}

// linear interpolation a + f (b - a) as one subtraction and one explicit fma
// (the FP32 path only; its rounding is judged statistically)
__device__ inline float lerp_f(float a, float b, float f) { return __builtin_fmaf(f, b - a, a); }

template <int D, int SX, int SY, int SZ, class F>
__device__ inline float gather_q(const F& f, int c, const Splits& s) {
  const float f0 = s.f[0][SX];
  const int l = f.lin(s.i[0][SX], D >= 2 ? s.i[1][SY] : 0, D == 3 ? s.i[2][SZ] : 0);
  if (D == 1) return lerp_f(f.at(c, l), f.at(c, l + 1), f0);
  const float f1 = s.f[1][SY];
  const int s1 = f.s1();
  const float v0 = lerp_f(f.at(c, l), f.at(c, l + 1), f0);
  const float v1 = lerp_f(f.at(c, l + s1), f.at(c, l + s1 + 1), f0);
  const float a2 = lerp_f(v0, v1, f1);
  if (D == 2) return a2;
  const float f2 = s.f[2][SZ];
  const int s2 = f.s2();
  const float w0 = lerp_f(f.at(c, l + s2), f.at(c, l + s2 + 1), f0);
  const float w1 = lerp_f(f.at(c, l + s2 + s1), f.at(c, l + s2 + s1 + 1), f0);
  const float b2 = lerp_f(w0, w1, f1);
  return lerp_f(a2, b2, f2);
}

// 3D FP32 gather in two rounds: the eight nodes of the three E components
// are loaded before any is interpolated, then those of B, so that twelve
// node-pair loads of an electron are in flight together (interleaved with
// the interpolation, the compiler waited for each component's loads in
// turn; all six components at once need 81 VGPRs).  Measured on the 3D gold
// slab: 3.24 -> 2.83 ms per launch before the laser arrives, 8.45 -> 8.12 ms
// at its peak.  The interpolation is gather_q's, in the same order.
template <int SX, int SY, int SZ, class F>
__device__ inline void gather_load8(const F& f, int c, const Splits& s, float v[8]) {
  const int l = f.lin(s.i[0][SX], s.i[1][SY], s.i[2][SZ]);
  const int s1 = f.s1(), s2 = f.s2();
  v[0] = f.at(c, l);
  v[1] = f.at(c, l + 1);
  v[2] = f.at(c, l + s1);
  v[3] = f.at(c, l + s1 + 1);
  v[4] = f.at(c, l + s2);
  v[5] = f.at(c, l + s2 + 1);
  v[6] = f.at(c, l + s2 + s1);
  v[7] = f.at(c, l + s2 + s1 + 1);
}

template <int SX, int SY, int SZ>
__device__ inline float interp8(const float v[8], const Splits& s) {
  const float f0 = s.f[0][SX], f1 = s.f[1][SY], f2 = s.f[2][SZ];
  const float a2 = lerp_f(lerp_f(v[0], v[1], f0), lerp_f(v[2], v[3], f0), f1);
  const float b2 = lerp_f(lerp_f(v[4], v[5], f0), lerp_f(v[6], v[7], f0), f1);
  return lerp_f(a2, b2, f2);
}

// Inverse of one bremsstrahlung cumulative row: scaled coordinate in [0,1].
template <class R>
__device__ inline R brem_inverse(const R* __restrict__ S, int n, R u, R iny1,
                                const uint8_t* __restrict__ G) {
  const int b = (int)(u * R(kGuide));
  int lo = G[b], hi = min((int)G[b + 1] + 1, n - 1);
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (S[mid] <= u) lo = mid; else hi = mid;
  }
  const R t = m_div(u - S[lo], S[lo + 1] - S[lo]);
  return (R(lo) + t) * iny1;
}

// node weights of a point on a 3-node window starting at m (m = lower of the
// two cells of the move, so the window holds both supports)
__device__ inline void shape3(int cell, float f, int m, float S[3]) {
  const int o = cell - m;  // 0 or 1
  S[0] = o == 0 ? 1.f - f : 0.f;
  S[1] = o == 0 ? f : 1.f - f;
  S[2] = o == 0 ? 0.f : f;
}

// FP32 form of the charge-conserving deposit on the 3-node windows that the
// move actually touches (the fourth node of the general window carries zero).
template <int D, class Acc>
__device__ inline void deposit3(const StepParams<float>& P, const Acc& J, const int* q0,
                                const int* q1, const float* v, double w) {
  // contributions in units of the current quantum
  const float c0 = (float)(-w * P.invV) * J.qscale();
  float S0[3][3], S1[3][3];
  int m[3] = {0, 0, 0};
  int i0s[3] = {0, 0, 0}, i1s[3] = {0, 0, 0};
  float f0s[3] = {0.f, 0.f, 0.f}, f1s[3] = {0.f, 0.f, 0.f};
  bool cross = false;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    split_q(q0[a], 0, P.fb[a], P.iqs[a], i0s[a], f0s[a]);
    split_q(q1[a], 0, P.fb[a], P.iqs[a], i1s[a], f1s[a]);
    cross = cross || i0s[a] != i1s[a];
  }
  // 2D and 3D: the form is chosen per wave.  A wave whose lanes took both
  // forms would issue the atomics of both (8 + 21 in 2D, 12 + 54 in 3D).  For
  // a move that stays in its cell the general form below yields exactly the
  // single-cell form's contributions: a position has at most 24 fraction
  // bits, so every node weight 1 - f is exact, the first face flux
  // -q ((1 - f1) - (1 - f0)) is q (f1 - f0) and the second is exactly 0.  An
  // electron's current therefore does not depend on which electrons share
  // its wave.
  const bool fast = D >= 2 ? __ballot(cross) == 0ull : !cross;
  if (fast) {
    // The move stays inside one cell on every axis: every node weight is
    // linear between the same two nodes, so the flux through the window's
    // second face vanishes and the third node carries nothing.  Only the
    // nodes {m, m+1} of each axis receive current: 4 of the 8 (1D), 8 of the
    // 21 (2D), 12 of the 54 (3D) contributions of the general form.  Each
    // axis's first-face flux is qa (f1 - f0) exactly, with no cancellation
    // of rounded node weights.
    const int base = J.lin(i0s[0], i0s[1], i0s[2]);
    const int s1 = J.s1(), s2 = J.s2();
    float A0[3], A1[3], B0[3], B1[3];  // node weights at x0 and x1 on {m, m+1}
#pragma unroll
    for (int a = 0; a < D; ++a) {
      A0[a] = 1.f - f0s[a]; A1[a] = f0s[a];
      B0[a] = 1.f - f1s[a]; B1[a] = f1s[a];
    }
    if (D == 1) {
      const float qx = c0 * (float)P.dxdt[0];
      J.addq2(0, base, qx, f1s[0] - f0s[0]);
      const float cy = 0.5f * c0 * v[1], cz = 0.5f * c0 * v[2];
      const float s0 = A0[0] + B0[0], s1w = A1[0] + B1[0];
      J.addq2(1, base, cy, s0);
      J.addq2(1, base + 1, cy, s1w);
      J.addq2(2, base, cz, s0);
      J.addq2(2, base + 1, cz, s1w);
    } else if (D == 2) {
      const float qx = 0.5f * c0 * (float)P.dxdt[0], qy = 0.5f * c0 * (float)P.dxdt[1];
      const float cz = c0 * v[2] * (1.f / 6.f);
      const float Fx = qx * (f1s[0] - f0s[0]), Fy = qy * (f1s[1] - f0s[1]);
      J.addq2(0, base, Fx, A0[1] + B0[1]);
      J.addq2(0, base + s1, Fx, A1[1] + B1[1]);
      J.addq2(1, base, Fy, A0[0] + B0[0]);
      J.addq2(1, base + 1, Fy, A1[0] + B1[0]);
      const float G0 = cz * __builtin_fmaf(2.f, A0[0], B0[0]), H0 = cz * __builtin_fmaf(2.f, B0[0], A0[0]);
      const float G1 = cz * __builtin_fmaf(2.f, A1[0], B1[0]), H1 = cz * __builtin_fmaf(2.f, B1[0], A1[0]);
      J.addq(2, base, __builtin_fmaf(G0, A0[1], H0 * B0[1]));
      J.addq(2, base + 1, __builtin_fmaf(G1, A0[1], H1 * B0[1]));
      J.addq(2, base + s1, __builtin_fmaf(G0, A1[1], H0 * B1[1]));
      J.addq(2, base + s1 + 1, __builtin_fmaf(G1, A1[1], H1 * B1[1]));
    } else {
      if (q0[0] == q1[0] && q0[1] == q1[1] && q0[2] == q1[2]) return;  // no move: no current
      float G[3][2], H[3][2], F[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        F[a] = c0 * (float)P.dxdt[a] * (f1s[a] - f0s[a]);
        G[a][0] = (1.f / 6.f) * __builtin_fmaf(2.f, A0[a], B0[a]);
        H[a][0] = (1.f / 6.f) * __builtin_fmaf(2.f, B0[a], A0[a]);
        G[a][1] = (1.f / 6.f) * __builtin_fmaf(2.f, A1[a], B1[a]);
        H[a][1] = (1.f / 6.f) * __builtin_fmaf(2.f, B1[a], A1[a]);
      }
      const float Z0[3] = {A0[0], A0[1], A0[2]}, Z1[3] = {A1[0], A1[1], A1[2]};
      const float Y0[3] = {B0[0], B0[1], B0[2]}, Y1[3] = {B1[0], B1[1], B1[2]};
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const float sa0 = k ? Z1[2] : Z0[2], sa1 = k ? Y1[2] : Y0[2];
          J.addq2(0, base + j * s1 + k * s2, F[0], __builtin_fmaf(G[1][j], sa0, H[1][j] * sa1));
        }
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float sa0 = k ? Z1[2] : Z0[2], sa1 = k ? Y1[2] : Y0[2];
          J.addq2(1, base + i + k * s2, F[1], __builtin_fmaf(G[0][i], sa0, H[0][i] * sa1));
        }
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float sa0 = j ? Z1[1] : Z0[1], sa1 = j ? Y1[1] : Y0[1];
          J.addq2(2, base + i + j * s1, F[2], __builtin_fmaf(G[0][i], sa0, H[0][i] * sa1));
        }
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    m[a] = min(i0s[a], i1s[a]);
    shape3(i0s[a], f0s[a], m[a], S0[a]);
    shape3(i1s[a], f1s[a], m[a], S1[a]);
  }
  // node (m0 + i, m1 + j, m2 + k) is base + i + j s1 + k s2
  const int base = J.lin(m[0], m[1], m[2]);
  const int s1 = J.s1(), s2 = J.s2();
  // Per axis a: the flux through the first two window faces, F[a][i] = -q_a
  // (d_0 + ... + d_i) with d = S1 - S0 (the Esirkepov prefix sum), and the
  // factors G = (2 S0 + S1) / 6, H = (S0 + 2 S1) / 6, with which the mixed
  // weight (S0a S0b + S1a S1b) / 3 + (S0a S1b + S1a S0b) / 6 of two axes is
  // G[a] S0[b] + H[a] S1[b].
  if (D == 1) {
    const float qx = c0 * (float)P.dxdt[0];
    const float F0 = -qx * (S1[0][0] - S0[0][0]);
    const float F1 = F0 - qx * (S1[0][1] - S0[0][1]);
    J.addq(0, base, F0);
    J.addq(0, base + 1, F1);
    const float cy = 0.5f * c0 * v[1], cz = 0.5f * c0 * v[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float sa = S0[0][i] + S1[0][i];
      J.addq2(1, base + i, cy, sa);
      J.addq2(2, base + i, cz, sa);
    }
  } else if (D == 2) {
    const float qx = 0.5f * c0 * (float)P.dxdt[0], qy = 0.5f * c0 * (float)P.dxdt[1];
    const float cz = c0 * v[2] * (1.f / 6.f);
    float Fx[2], Fy[2], sx[3], sy[3], G[3], H[3];
    Fx[0] = -qx * (S1[0][0] - S0[0][0]);
    Fx[1] = Fx[0] - qx * (S1[0][1] - S0[0][1]);
    Fy[0] = -qy * (S1[1][0] - S0[1][0]);
    Fy[1] = Fy[0] - qy * (S1[1][1] - S0[1][1]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sx[i] = S0[0][i] + S1[0][i];
      sy[i] = S0[1][i] + S1[1][i];
      G[i] = cz * __builtin_fmaf(2.f, S0[0][i], S1[0][i]);
      H[i] = cz * __builtin_fmaf(2.f, S1[0][i], S0[0][i]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 2; ++i) J.addq2(0, base + i + j * s1, Fx[i], sy[j]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) J.addq2(1, base + i + j * s1, Fy[j], sx[i]);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        J.addq(2, base + i + j * s1, __builtin_fmaf(G[i], S0[1][j], H[i] * S1[1][j]));
  } else {
    float F[3][2], G[3][3], H[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float qa = c0 * (float)P.dxdt[a];
      F[a][0] = -qa * (S1[a][0] - S0[a][0]);
      F[a][1] = F[a][0] - qa * (S1[a][1] - S0[a][1]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        G[a][i] = (1.f / 6.f) * __builtin_fmaf(2.f, S0[a][i], S1[a][i]);
        H[a][i] = (1.f / 6.f) * __builtin_fmaf(2.f, S1[a][i], S0[a][i]);
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float T = __builtin_fmaf(G[1][j], S0[2][k], H[1][j] * S1[2][k]);
#pragma unroll
        for (int i = 0; i < 2; ++i) J.addq2(0, base + i + j * s1 + k * s2, F[0][i], T);
      }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float T = __builtin_fmaf(G[0][i], S0[2][k], H[0][i] * S1[2][k]);
#pragma unroll
        for (int j = 0; j < 2; ++j) J.addq2(1, base + i + j * s1 + k * s2, F[1][j], T);
      }
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float T = __builtin_fmaf(G[0][i], S0[1][j], H[0][i] * S1[1][j]);
#pragma unroll
        for (int k = 0; k < 2; ++k) J.addq2(2, base + i + j * s1 + k * s2, F[2][k], T);
      }
  }
}

__device__ inline void neumaier(double* s, double* c, double v) {
  const double t = *s + v;
  if (fabs(*s) >= fabs(v)) *c += (*s - t) + v;
  else *c += (v - t) + *s;
  *s = t;
}

// Sum over the 64 lanes in a fixed order: DPP row shifts and broadcasts
// collect it in lane 63 (the halves of each double moved together), from
// where it is read as a wave-uniform value.  Call with every lane active.
template <int kCtrl, int kRows>
__device__ inline double dpp_add(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, kRows, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, kRows, 0xf, false);
  return v + __hiloint2double(hi, lo);
}

__device__ inline double wave_sum(double v) {
  v = dpp_add<0x111, 0xf>(v);  // row_shr:1
  v = dpp_add<0x112, 0xf>(v);  // row_shr:2
  v = dpp_add<0x114, 0xf>(v);  // row_shr:4
  v = dpp_add<0x118, 0xf>(v);  // row_shr:8
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}

__device__ inline uint32_t lane_offset(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Whether the step kernel stages the box's fields in LDS.  In 3D it does not:
// fields are gathered from global memory through the caches and only the
// current lives in LDS, which fits a three times larger box (2048 nodes) in
// the same LDS.  Measured on the 3D gold slab (134M electrons): 7.2e9 vs
// 6.6e9 electron-steps/s at the best staged-field box (1024 nodes).  In 2D
// the staged fields win (8.9e9 vs 8.6e9 on the 2D gold slab).
template <class R, int D>
struct FieldsInLds {
  static constexpr bool value = D != 3;
};

template <class R, int D>
constexpr size_t lds_bytes_per_node() {
  return (FieldsInLds<R, D>::value ? 6 * sizeof(R) : 0) +
         3 * (sizeof(R) == 4 ? sizeof(int) : sizeof(unsigned long long));
}

// Electrons per step-kernel workgroup: one per thread.  (Two per thread,
// in two passes, raised the FP32 2D kernel from 67 to 87 VGPRs and ran 15%
// slower.)
int chunk_electrons(bool fp32, int dims) {
  (void)fp32;
  (void)dims;
  return kBlock;
}

// Spectrum bin of a photon energy eps (mc^2): with eps = m 2^e, 1 <= m < 2,
// bin 4 (e + 2) + [m >= 2^(1/4)] + [m >= 2^(1/2)] + [m >= 2^(3/4)], clamped
// to [0, 64).  Exact comparisons with the rounded constants: the same bin
// in every implementation that rounds them the same way.
template <class R>
__device__ inline int spectrum_bin(R eps) {
  int e;
  const R m = R(2) * (sizeof(R) == 4 ? (R)frexpf((float)eps, &e) : (R)frexp((double)eps, &e));
  e -= 1;
  int b = 4 * (e + 2);
  if constexpr (sizeof(R) == 4) {
    b += (m >= 0x1.306fe0p+0f) + (m >= 0x1.6a09e6p+0f) + (m >= 0x1.ae89fap+0f);
  } else {
    b += (m >= 0x1.306fe0a31b715p+0) + (m >= 0x1.6a09e667f3bcdp+0) + (m >= 0x1.ae89f995ad3adp+0);
  }
  return b < 0 ? 0 : (b > PIC_SPECTRUM_BINS - 1 ? PIC_SPECTRUM_BINS - 1 : b);
}

// Per-electron results the block-level stages (append, statistics) need.
template <class R>
struct Emit {
  bool ev_ncs = false, ev_br = false, keep_ncs = false, clamped = false;
  R e[2] = {R(0), R(0)};
  R k[2][3] = {{R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
  R xo[3] = {R(0), R(0), R(0)};
};

// Per-electron state carried from the push to the move (registers).
template <class R>
struct Lane {
  R x[3] = {R(0), R(0), R(0)};   // absolute position (FP32: for records and the frozen plane wave)
  R px = R(0), py = R(0), pz = R(0), gamma = R(1);
  U4 r;                           // Philox words of (id, step), once drawn
  bool have_r = false;
  double taub = 0.0;              // collision optical depth at the start of the step
};

// The move of one electron, kept for the current deposit, which runs after
// the wave's photon records and statistics are out (so that these inputs are
// all the deposit holds in registers).
template <class R>
struct Move {
  int q0[3] = {0, 0, 0}, q1[3] = {0, 0, 0};  // FP32: fixed-point positions before and after
  R x0[3] = {R(0), R(0), R(0)};              // FP64: positions before and after
  R x1[3] = {R(0), R(0), R(0)};
  R v[3] = {R(0), R(0), R(0)};               // velocity of the move
};

// Inverse of the two NCS cumulative rows around eta at the same uniform u:
// ln(xi) of each row, linear in its bracket (the largest j <= n - 2 with
// C[j] <= u, found between the row guide's entries), and below the row's
// first point the small-xi form of the row, C proportional to xi^(1/3).  The two searches
// run side by side so that their dependent table loads overlap.
template <class R>
__device__ inline void ncs_inverse2(const R* __restrict__ Ca, const R* __restrict__ Cb,
                                    const R* __restrict__ lnxi, int n, R u, const uint8_t* __restrict__ Ga,
                                    const uint8_t* __restrict__ Gb, R& la, R& lb) {
  const int b = (int)(u * R(kGuide));
  const R ca0 = Ca[0], cb0 = Cb[0];
  int loa = Ga[b], hia = min((int)Ga[b + 1] + 1, n - 1);
  int lob = Gb[b], hib = min((int)Gb[b + 1] + 1, n - 1);
  while (hia - loa > 1 || hib - lob > 1) {
    if (hia - loa > 1) {
      const int mid = (loa + hia) >> 1;
      if (Ca[mid] <= u) loa = mid; else hia = mid;
    }
    if (hib - lob > 1) {
      const int mid = (lob + hib) >> 1;
      if (Cb[mid] <= u) lob = mid; else hib = mid;
    }
  }
  if (u < ca0) {
    la = lnxi[0] + R(3) * m_log(m_div(u, ca0));
  } else {
    const R t = m_div(u - Ca[loa], Ca[loa + 1] - Ca[loa]);
    la = lnxi[loa] + t * (lnxi[loa + 1] - lnxi[loa]);
  }
  if (u < cb0) {
    lb = lnxi[0] + R(3) * m_log(m_div(u, cb0));
  } else {
    const R t = m_div(u - Cb[lob], Cb[lob + 1] - Cb[lob]);
    lb = lnxi[lob] + t * (lnxi[lob + 1] - lnxi[lob]);
  }
}

// Photon energy of an NCS emission: each of the two rows around eta inverted
// at the uniform, blended in ln eta, xi = exp(.), eps = xi gamma capped at the
// kinetic energy.
template <class R>
__device__ inline R ncs_eps(const StepParams<R>& P, int i, R f, R u2, R gamma) {
  const ColdPtr<R> C = cold(P);
  const int nxi = C->n_xi;
  const R* ncs = C->ncs;
  const R* lnxi = C->lnxi;
  const uint8_t* gn = C->gncs;
  R la, lb;
  ncs_inverse2<R>(ncs + (int64_t)i * nxi, ncs + (int64_t)(i + 1) * nxi, lnxi, nxi, u2,
                  gn + i * (kGuide + 1), gn + (i + 1) * (kGuide + 1), la, lb);
  const R lx = la + f * (lb - la);
  const R xi = m_exp(lx);
  R eps = xi * gamma;
  if (eps > gamma - R(1)) eps = gamma - R(1);
  return eps;
}

// An NCS emission of energy eps: photon direction along p, the record cut,
// recoil along p (energy conserving), and the next optical depth.
template <class R>
__device__ inline void ncs_finish(const StepParams<R>& P, int64_t e, Lane<R>& L, R eps, double tau_new,
                                  Emit<R>& out) {
  const R pm = m_sqrt(L.px * L.px + L.py * L.py + L.pz * L.pz);
  out.ev_ncs = true;
  out.e[0] = eps;
  out.k[0][0] = m_div(L.px, pm); out.k[0][1] = m_div(L.py, pm); out.k[0][2] = m_div(L.pz, pm);
  out.keep_ncs = (double)eps >= cold(P)->photon_cut;
  if (!(P.flags & PIC_NO_RECOIL)) {
    const R gn = L.gamma - eps;
    const R pn = m_sqrt((gn - R(1)) * (gn + R(1)));
    const R sc = m_div(pn, pm);
    L.px = L.px * sc; L.py = L.py * sc; L.pz = L.pz * sc;
    L.gamma = gn;
  }
  P.tau[e] = tau_new;
}

// First half of one electron's step: gather, Boris push, eta, the NCS
// optical-depth decrement and, on an emission, the photon draw and recoil.
template <class R, int D, class FA>
__device__ inline void electron_push(const StepParams<R>& P, int64_t e, uint32_t idv, const R* xin,
                                     const int* qin, const R* pin, double tau_in, const FA& fld,
                                     Lane<R>& L, Emit<R>& out) {
  constexpr bool kF32 = sizeof(R) == 4;
  const uint32_t n = P.step;
  // absolute position (FP32 path: from the fixed point, for records and the
  // prescribed plane wave only; gather, cells and moves use the integers)
  L.x[0] = xin[0]; L.x[1] = xin[1]; L.x[2] = xin[2];
  if constexpr (kF32) {
#pragma unroll
    for (int a = 0; a < D; ++a) L.x[a] = (float)qin[a] * P.iqd[a];
  }
  out.xo[0] = L.x[0]; out.xo[1] = L.x[1]; out.xo[2] = L.x[2];
  // 3D: state prefetched by the caller; 1D/2D: loaded here, at first use
  R px, py, pz;
  if constexpr (D == 3) { px = pin[0]; py = pin[1]; pz = pin[2]; }
  else { px = P.p[0][e]; py = P.p[1][e]; pz = P.p[2][e]; }
  // free-path collision depth: loaded here so that its latency overlaps the
  // gather and the push (measured on the 2D gold slab: a load at the test
  // costs 7 us per launch)
  L.taub = (P.flags & PIC_BREM_FREEPATH) ? P.taub[e] : 0.0;

  // ---- gather E^n, B^n at x^n ----------------------------------------------
  R E0, E1, E2, B0, B1, B2;
  if (P.flags & PIC_FIELDS_FROZEN) {
    const ColdPtr<R> C = cold(P);
    if (C->frozen_kind == PIC_FROZEN_UNIFORM) {
      E0 = R(C->fE[0]); E1 = R(C->fE[1]); E2 = R(C->fE[2]);
      B0 = R(C->fB[0]); B1 = R(C->fB[1]); B2 = R(C->fB[2]);
    } else {
      E0 = R(0); E1 = R(0); E2 = R(0); B0 = R(0); B1 = R(0); B2 = R(0);
      const R phi = R(P.tn) - L.x[0];
      if (phi > R(0)) {
        const R v = R(C->fa) * m_sin(phi);
        E1 = v;
        B2 = v;
      }
    }
  } else if constexpr (kF32) {
    const Splits sp = make_splits<D>(qin, P.fb, P.iqs);
    if constexpr (D == 3) {
      float nv[6][8];
      gather_load8<1, 0, 0>(fld, 0, sp, nv[0]);
      gather_load8<0, 1, 0>(fld, 1, sp, nv[1]);
      gather_load8<0, 0, 1>(fld, 2, sp, nv[2]);
      E0 = interp8<1, 0, 0>(nv[0], sp);
      E1 = interp8<0, 1, 0>(nv[1], sp);
      E2 = interp8<0, 0, 1>(nv[2], sp);
      gather_load8<0, 1, 1>(fld, 3, sp, nv[3]);
      gather_load8<1, 0, 1>(fld, 4, sp, nv[4]);
      gather_load8<1, 1, 0>(fld, 5, sp, nv[5]);
      B0 = interp8<0, 1, 1>(nv[3], sp);
      B1 = interp8<1, 0, 1>(nv[4], sp);
      B2 = interp8<1, 1, 0>(nv[5], sp);
    } else {
      E0 = gather_q<D, 1, 0, 0>(fld, 0, sp);
      E1 = gather_q<D, 0, 1, 0>(fld, 1, sp);
      E2 = gather_q<D, 0, 0, 1>(fld, 2, sp);
      B0 = gather_q<D, 0, 1, 1>(fld, 3, sp);
      B1 = gather_q<D, 1, 0, 1>(fld, 4, sp);
      B2 = gather_q<D, 1, 1, 0>(fld, 5, sp);
    }
  } else {
    R g[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) g[a] = L.x[a] * R(P.idx[a]);
    E0 = gather<R, D, 1, 0, 0>(fld, 0, g);
    E1 = gather<R, D, 0, 1, 0>(fld, 1, g);
    E2 = gather<R, D, 0, 0, 1>(fld, 2, g);
    B0 = gather<R, D, 0, 1, 1>(fld, 3, g);
    B1 = gather<R, D, 1, 0, 1>(fld, 4, g);
    B2 = gather<R, D, 1, 1, 0>(fld, 5, g);
  }

  // ---- relativistic Boris push (q = -1, m = 1) ------------------------------
  const R hq = R(-0.5 * P.dt);
  const R umx = px + hq * E0, umy = py + hq * E1, umz = pz + hq * E2;
  const R gm = m_fsqrt(R(1) + (umx * umx + umy * umy + umz * umz));
  const R fq = m_div(hq, gm);
  const R tx = fq * B0, ty = fq * B1, tz = fq * B2;
  const R sf = m_div(R(2), R(1) + (tx * tx + ty * ty + tz * tz));
  const R sx = sf * tx, sy = sf * ty, sz = sf * tz;
  const R upx = umx + (umy * tz - umz * ty);
  const R upy = umy + (umz * tx - umx * tz);
  const R upz = umz + (umx * ty - umy * tx);
  const R uqx = umx + (upy * sz - upz * sy);
  const R uqy = umy + (upz * sx - upx * sz);
  const R uqz = umz + (upx * sy - upy * sx);
  L.px = uqx + hq * E0;
  L.py = uqy + hq * E1;
  L.pz = uqz + hq * E2;
  L.gamma = m_fsqrt(R(1) + (L.px * L.px + L.py * L.py + L.pz * L.pz));

  // ---- quantum parameter eta (Lorentz invariant, Sec. II.A) -----------------
  // eta^2 E_S^2 = |gamma E + p x B|^2 - (p.E)^2 (units m c = 1).  For
  // |p| >= 1 FP32 writes the same invariant as gamma^2 |F_perp|^2 + F_par^2,
  // F = E + v x B split across and along p: the difference of the two
  // squares cancels when p is nearly parallel to the force (its FP32 error
  // grows like gamma^4 relative to eta^2, noise that the clip at zero turns
  // into excess emission); the split form has no such cancellation.  Below
  // |p| = 1 (gamma < 1.42) the difference loses little, and the split form's
  // 1/p^2 is not safe (a denormal p^2 has an infinite hardware reciprocal).
  // FP64 keeps the difference.
  const R cx = L.gamma * E0 + (L.py * B2 - L.pz * B1);
  const R cy = L.gamma * E1 + (L.pz * B0 - L.px * B2);
  const R cz = L.gamma * E2 + (L.px * B1 - L.py * B0);
  const R pe = L.px * E0 + L.py * E1 + L.pz * E2;
  R q2 = (cx * cx + cy * cy + cz * cz) - pe * pe;
  if (q2 < R(0)) q2 = R(0);
  if constexpr (kF32) {
    const R pp = L.px * L.px + L.py * L.py + L.pz * L.pz;
    if (pp >= R(1)) {
      const R ig = m_div(R(1), L.gamma);
      const R Fx = E0 + ig * (L.py * B2 - L.pz * B1);
      const R Fy = E1 + ig * (L.pz * B0 - L.px * B2);
      const R Fz = E2 + ig * (L.px * B1 - L.py * B0);
      const R Fp = Fx * L.px + Fy * L.py + Fz * L.pz;
      const R sp = m_div(Fp, pp);  // F.p / p^2
      const R ux = Fx - sp * L.px, uy = Fy - sp * L.py, uz = Fz - sp * L.pz;
      q2 = L.gamma * L.gamma * (ux * ux + uy * uy + uz * uz) + Fp * sp;
    }
  }
  const R eta = m_fsqrt(q2) * R(P.iES);

  // ---- nonlinear Compton: optical depth + inverse-CDF draw ------------------
  // eta clearly below the first table point: no decrement (same decision as
  // the logarithm test below, without evaluating it)
  if ((P.flags & PIC_NCS) && (double)eta >= P.eta_skip) {
    const R sl = (m_log(eta) - R(P.ln_eta0)) * R(P.idln_eta);
    if (sl >= R(0)) {
      int i;
      R f;
      if (sl >= R(P.n_eta - 1)) { i = P.n_eta - 2; f = R(1); }
      else { i = (int)sl; f = sl - R(i); }
      const R h = P.h[i] + f * (P.h[i + 1] - P.h[i]);
      const R dtau = m_div(R(P.K_N) * eta, L.gamma) * h * R(P.dt);
      const double tau = (D == 3 ? tau_in : P.tau[e]) - (double)dtau;
      if (tau <= 0.0) {
        L.r = philox4x32_10(idv, n, 0u, 0u, P.key0, P.key1);
        L.have_r = true;
        const R eps = ncs_eps<R>(P, i, f, unif<R>(L.r.v[2]), L.gamma);
        // next optical depth -ln u: FP64 series on the FP64 path (bit parity);
        // the FP32 path takes the logarithm of its 23-bit uniform in FP32
        const double tau_new = kF32 ? -(double)m_log(unif<R>(L.r.v[3])) : -fp_log(unif32(L.r.v[3]));
        ncs_finish<R>(P, e, L, eps, tau_new, out);
      } else {
        P.tau[e] = tau;
      }
    }
  }
}

// Second half: bremsstrahlung test of Eq. (4) with the R2 energy draw, recoil,
// move, absorbing walls.  The current of the move is deposited later
// (electron_deposit).
template <class R, int D>
__device__ inline void electron_move(const StepParams<R>& P, int64_t e, uint32_t idv, const int* qin,
                                     Lane<R>& L, Emit<R>& out, Move<R>& mv) {
  constexpr bool kF32 = sizeof(R) == 4;
  const uint32_t n = P.step;
  const bool fpath = (P.flags & PIC_BREM_FREEPATH) != 0;
  R px = L.px, py = L.py, pz = L.pz, gamma = L.gamma;
  const R* x = L.x;

  // ---- bremsstrahlung: Eq. (4) test, R2 energy draw (Sec. II.B) -------------
  if (P.flags & PIC_BREM) {
    const R T = gamma - R(1);
    if ((double)T >= P.k_cut) {
      int ci[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < D; ++a) {
        int q;
        if constexpr (kF32) q = qin[a] >> P.fb[a];
        else q = (int)m_floor(x[a] * R(P.idx[a]));
        q = q < 0 ? 0 : (q > P.n[a] - 1 ? P.n[a] - 1 : q);
        ci[a] = q;
      }
      // the density n_i of the cell and the two sigma(T) rows are loaded
      // together: neither address depends on the other load
      const double ni = P.ni[ci[0] + (int64_t)P.n[0] * (ci[1] + (int64_t)P.n[1] * ci[2])];
      const R lt = m_log(T);
      const R sl = (lt - R(P.ln_T0)) * R(P.idln_T);
      int i = 0;
      R f = R(0);
      const bool top = sl >= R(P.n_T - 1);
      if (top) { i = P.n_T - 2; f = R(1); }
      else if (sl >= R(0)) { i = (int)sl; f = sl - R(i); }
      const R sg0 = P.sig[i], sg1 = P.sig[i + 1];
      if (ni > 0.0) {
        if (sl >= R(0)) {
          if (top) out.clamped = true;
          const R sig = sg0 + f * (sg1 - sg0);
          if (sig > R(0)) {
            const R pm = m_sqrt(px * px + py * py + pz * pz);
            const R v = m_div(pm, gamma);
            const R X = R(P.K_BR) * R(ni) * sig * v * R(P.dt);
            bool hit;
            double tb = 0.0;
            if (fpath) {
              // free path: X is the step's path in mean free paths; collide
              // when the electron's remaining depth runs out (no draw until then)
              tb = L.taub - (double)X;
              hit = tb <= 0.0;
            } else {
              const R Pb = -m_expm1(-X);
              if (!L.have_r) { L.r = philox4x32_10(idv, n, 0u, 0u, P.key0, P.key1); L.have_r = true; }
              hit = unif52(L.r.v[0], L.r.v[1]) < (double)Pb;
            }
            if (!hit) {
              if (fpath) P.taub[e] = tb;
            } else {
              const U4 r2 = philox4x32_10(idv, n, 1u, 0u, P.key0, P.key1);
              // next free path from word 1 of the energy draw's counter
              if (fpath)
                P.taub[e] = kF32 ? -(double)m_log(unif<R>(r2.v[1])) : -fp_log(unif32(r2.v[1]));
              const R u = unif<R>(r2.v[0]);
              const ColdPtr<R> C = cold(P);
              const int ny = C->n_y;
              const R* br = C->br;
              const R iny1 = R(C->iny1);
              const uint8_t* gb = C->gbr;
              const R sa = brem_inverse<R>(br + (int64_t)i * ny, ny, u, iny1, gb + i * (kGuide + 1));
              const R sb = brem_inverse<R>(br + (int64_t)(i + 1) * ny, ny, u, iny1,
                                           gb + (i + 1) * (kGuide + 1));
              const R sv = sa + f * (sb - sa);
              const R lk = R(C->lnk);
              R eps = m_exp(lk + sv * (lt - lk));
              if (eps > T) eps = T;
              out.ev_br = true;
              out.e[1] = eps;
              out.k[1][0] = m_div(px, pm); out.k[1][1] = m_div(py, pm); out.k[1][2] = m_div(pz, pm);
              if (!(P.flags & PIC_NO_RECOIL)) {
                const R gn = gamma - eps;
                const R pn = m_sqrt((gn - R(1)) * (gn + R(1)));
                const R sc = m_div(pn, pm);
                px = px * sc; py = py * sc; pz = pz * sc;
                gamma = gn;
              }
            }
          }
        }
      }
    }
  }

  // ---- move, absorbing walls -----------------------------------------------
  P.p[0][e] = px; P.p[1][e] = py; P.p[2][e] = pz;
  const R ig = m_div(R(1), gamma);
  mv.v[0] = px * ig; mv.v[1] = py * ig; mv.v[2] = pz * ig;
  bool outside = false;
  if constexpr (kF32) {
    // fixed-point move: displacement rounded to 2^-fb cell; the deposit sees
    // exactly the stored move, so charge is conserved on the stored positions
#pragma unroll
    for (int a = 0; a < 3; ++a) { mv.q0[a] = qin[a]; mv.q1[a] = qin[a]; }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      mv.q1[a] = qin[a] + (int)rintf(mv.v[a] * P.mvq[a]);
      if (mv.q1[a] < 0 || mv.q1[a] >= (P.n[a] << P.fb[a])) outside = true;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) reinterpret_cast<int*>(P.x[a])[e] = mv.q1[a];
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) { mv.x0[a] = x[a]; mv.x1[a] = x[a]; }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      mv.x1[a] = x[a] + mv.v[a] * R(P.dt);
      if (mv.x1[a] < R(0) || mv.x1[a] >= R(P.L[a])) outside = true;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) P.x[a][e] = mv.x1[a];
  }
  if (outside) P.id[e] = idv | kDead;
}

// Charge-conserving current of the move x^n -> x^{n+1} of one electron.
template <class R, int D, class JA>
__device__ inline void electron_deposit(const StepParams<R>& P, const JA& cur, const Move<R>& mv,
                                        double wgt) {
  if (P.flags & PIC_FIELDS_FROZEN) return;
  if constexpr (sizeof(R) == 4) deposit3<D>(P, cur, mv.q0, mv.q1, mv.v, wgt);
  else deposit<R, D>(P, cur, mv.x0, mv.x1, mv.v, wgt);
}

// Minimum over the 64 lanes of two packed 16-bit integers per lane (DPP row
// shifts and broadcasts; the result is read from lane 63).  Call with every
// lane of the wave active.
__device__ inline uint32_t wave_min_pk16(uint32_t v) {
  typedef short S2 __attribute__((ext_vector_type(2)));
  auto mn = [](uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(S2, a), __builtin_bit_cast(S2, b)));
  };
  constexpr int kId = 0x7fff7fff;
  v = mn(v, (uint32_t)__builtin_amdgcn_update_dpp(kId, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = mn(v, (uint32_t)__builtin_amdgcn_update_dpp(kId, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = mn(v, (uint32_t)__builtin_amdgcn_update_dpp(kId, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = mn(v, (uint32_t)__builtin_amdgcn_update_dpp(kId, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = mn(v, (uint32_t)__builtin_amdgcn_update_dpp(kId, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = mn(v, (uint32_t)__builtin_amdgcn_update_dpp(kId, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ inline uint32_t pk16(int lo, int hi) { return ((uint32_t)lo & 0xffffu) | ((uint32_t)hi << 16); }
__device__ inline int lo16(uint32_t w) { return (int)(short)(w & 0xffffu); }
__device__ inline int hi16(uint32_t w) { return (int)(short)(w >> 16); }

// One workgroup = one chunk of 256 consecutive electrons of the (tile-sorted)
// SoA (chunk_of_block spreads the chunks over the XCDs); lane t of the
// workgroup takes electron t of the chunk.
// When the chunk's cells fit the LDS box, the fields of the box are staged in
// LDS and the current is accumulated there (FP64: int64 in units of 2^-40;
// FP32: int32 in units of 2^-jbits); otherwise both go to global memory.
template <class R, int D>
__device__ __forceinline__ void step_chunk(const StepParams<R>& P, const uint32_t chunk,
                                           unsigned char* smem, uint32_t* s_box, uint32_t* s_spec) {
  constexpr bool kF32 = sizeof(R) == 4;
  using JT = typename std::conditional<kF32, int, unsigned long long>::type;
  const uint32_t t = threadIdx.x;
  // Consecutive lanes take consecutive electrons, so every state load and
  // store of a wave covers whole cache lines.  (Dealing electrons to lanes
  // with a stride, so that a wave's lanes came from many cells and rarely hit
  // the same LDS current node at once, made each wave touch four times the
  // lines; with the deposit holding only its inputs in registers it lost:
  // 3D gold slab 4.94 -> 3.31 ms per launch before the laser arrives and
  // 9.64 -> 8.46 ms at its peak against stride 8; 2D gold slab 4-5% against
  // stride 4; 1D unchanged.)
  const int64_t e = (int64_t)chunk * kBlock + (int64_t)t;
  const int64_t n_act = (int64_t)*P.n_active;
  // whether the photon buffer is known to be full: a flag on a line of its
  // own, set by the first reservation that reached the capacity (reading the
  // counter itself, which every wave's atomic targets, doubled the launch
  // time while the buffer was filling; a stale 0 only costs an unneeded
  // reservation).  A relaxed load, first used at the append: a volatile
  // load here made every wave wait for it before issuing anything else.
  const uint32_t full_flag = __hip_atomic_load(cold(P)->pfull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const bool frozen = (P.flags & PIC_FIELDS_FROZEN) != 0;
  uint32_t idv = kDead;
  R x[3] = {R(0), R(0), R(0)};
  int q[3] = {0, 0, 0};
  int bb[3] = {0, 0, 0};
  // 3D: the rest of the state is loaded up front, so its latency overlaps the
  // box reduction and the zeroing of the LDS current (measured: 3D gold slab
  // 11.2 -> 9.9 ms per launch; in 2D it costs 3 us, so 2D loads it later)
  constexpr bool kEarly = D == 3;
  R pin[3] = {R(0), R(0), R(0)};
  double tau_in = 0.0, wgt = 0.0;
  // The state is loaded together with the id, not after it: every index
  // below n_act holds an electron (an absorbed one's state is read and not
  // used), so the loads need not wait for the id's round trip.
  if (e < n_act) {
    idv = P.id[e];
    if constexpr (kEarly) {
#pragma unroll
      for (int a = 0; a < 3; ++a) pin[a] = P.p[a][e];
      tau_in = P.tau[e];
      wgt = P.w[e];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if constexpr (kF32) q[a] = reinterpret_cast<const int*>(P.x[a])[e];
      else x[a] = P.x[a][e];
    }
  }
  const bool live = (idv & kDead) == 0;
  if (live) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      if constexpr (kF32) bb[a] = (q[a] >> P.fb[a]) - 1;
      else bb[a] = (int)m_floor(x[a] * R(P.idx[a])) - 1;
    }
  }
  // ---- the chunk's box of nodes (deposit windows cover the gathers) --------
  // Per lane the window [bb, bb + 3] of each axis; the minimum of bb and of
  // -(bb + 3) over the chunk give the box.  Each wave reduces them as packed
  // 16-bit pairs (one word per two values) and leaves its words in LDS; the
  // chunk's box is the minimum over the four waves' words.  A cell index
  // beyond +-32000 (grids that large) widens the box to the whole 16-bit
  // range, which no LDS box holds: such a chunk takes the global path.
  if (t < 2 * PIC_SPECTRUM_BINS) s_spec[t] = 0u;
  {
    constexpr int kW = (2 * D + 1) / 2;  // packed words: 1 (1D), 2 (2D), 3 (3D)
    int v[6] = {32767, 32767, 32767, 32767, 32767, 32767};
    if (live && !frozen) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const bool in = bb[a] >= -32000 && bb[a] <= 32000;
        v[a] = in ? bb[a] : -32768;             // lower end
        v[D + a] = in ? -(bb[a] + 3) : -32767;  // minus the upper end
      }
    }
    const uint32_t wv = t >> 6;
#pragma unroll
    for (int k = 0; k < kW; ++k) {
      const uint32_t m = wave_min_pk16(pk16(v[2 * k], v[2 * k + 1]));
      if ((t & 63u) == 0u) s_box[4 * k + wv] = m;
    }
  }
  __syncthreads();
  int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
  int nodes = 0;
  bool tiled = false;
  {
    typedef short S2 __attribute__((ext_vector_type(2)));
    auto mn = [](uint32_t a, uint32_t b) {
      return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(S2, a), __builtin_bit_cast(S2, b)));
    };
    constexpr int kW = (2 * D + 1) / 2;
    int u[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kW; ++k) {
      const uint4 w4 = *reinterpret_cast<const uint4*>(s_box + 4 * k);
      const uint32_t m = mn(mn(w4.x, w4.y), mn(w4.z, w4.w));
      u[2 * k] = lo16(m);
      u[2 * k + 1] = hi16(m);
    }
    // u[a] = lowest bb, -u[D + a] = highest bb + 3 (empty chunk: lo > hi)
    if (!frozen && P.lds_nodes > 0 && u[0] <= -u[D]) {
      int64_t nn = 1;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        lo[a] = u[a];
        ext[a] = -u[D + a] - u[a] + 1;
        nn *= ext[a];
      }
      tiled = nn <= P.lds_nodes;
      nodes = (int)(nn < (1 << 30) ? nn : (1 << 30));
    }
  }
  constexpr bool kFL = FieldsInLds<R, D>::value;
  // 1D/2D boxes too large for fields + current may still fit the current
  // alone in the same allocation (three times the nodes): fields are then
  // gathered from global memory, the current still accumulates in LDS
  bool jtiled = false;
  if constexpr (kFL) {
    const int jcap = (int)((size_t)P.lds_nodes * lds_bytes_per_node<R, D>() / (3 * sizeof(JT)));
    jtiled = !tiled && nodes > 0 && nodes <= jcap;
  }
  R* sF = reinterpret_cast<R*>(smem);
  JT* sJ = reinterpret_cast<JT*>(smem + (kFL && tiled ? (size_t)6 * P.lds_nodes * sizeof(R) : 0));
  const Idx<R> I{P.gg[0], P.gg[1], P.gg[2], P.sz[0], P.sz[1]};
  // node l of the box -> (i, j, k); exact float-reciprocal division (l < 2^20)
  const float r0 = 1.0f / (float)ext[0], r1 = 1.0f / (float)ext[1];
  auto decode = [&](int l, int& i, int& j, int& k) {
    const int q0 = (int)(((float)l + 0.5f) * r0);
    i = l - q0 * ext[0] + lo[0];
    if (D == 1) { j = 0; k = 0; return; }
    const int q1 = (int)(((float)q0 + 0.5f) * r1);
    j = q0 - q1 * ext[1] + lo[1];
    k = (D == 3 ? q1 : 0) + lo[2];
  };
  if (tiled) {
    for (int l = t; l < nodes; l += kBlock) {
      int i, j, k;
      decode(l, i, j, k);
      const int64_t m = I(i, j, k);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (kFL) {
          sF[c * nodes + l] = P.F[c][m];
          sF[(3 + c) * nodes + l] = P.F[3 + c][m];
        }
        sJ[c * nodes + l] = JT(0);
      }
    }
  } else if (jtiled) {
    for (int l = t; l < 3 * nodes; l += kBlock) sJ[l] = JT(0);
  }
  __syncthreads();

  Emit<R> out;
  Lane<R> L;
  Move<R> mv;
  if (live) {
    if constexpr (!kEarly) wgt = P.w[e];
    if constexpr (kFL) {
      if (tiled) {
        const LdsField<R> fa{sF, lo[0], lo[1], lo[2], ext[0], ext[1], nodes};
        electron_push<R, D>(P, e, idv, x, q, pin, tau_in, fa, L, out);
      } else {
        electron_push<R, D>(P, e, idv, x, q, pin, tau_in, GlobalField<R>{P.F, I}, L, out);
      }
    } else {
      electron_push<R, D>(P, e, idv, x, q, pin, tau_in, GlobalField<R>{P.F, I}, L, out);
    }
    electron_move<R, D>(P, e, idv, q, L, out, mv);
  }
  // ---- photon records: one slot reservation per wave ----------------------
  // NCS and bremsstrahlung records of the wave take consecutive slots from
  // one atomic on the buffer's counter.  Once a reservation has reached the
  // capacity (a flag read as the chunk starts), no slot can be had and the
  // reservation is skipped: every such record is an overflow, and the
  // overflow count is the kept count (per-wave statistics) minus the
  // capacity.  (Every wave of the grid hammering the one counter after the
  // buffer filled cost 4.9 ms of a 14.7 ms launch on the 3D gold slab in the
  // interaction.)
  const uint32_t lane = __lane_id();
  const bool rec0 = out.ev_ncs && out.keep_ncs;
  const bool rec1 = out.ev_br;
  const unsigned long long mr0 = __ballot(rec0), mr1 = __ballot(rec1);
  // spectrum of every kept photon, stored or not (quarter-octave bins): LDS
  // counts of the chunk, added at the chunk's end to one of kSpecCopies
  // copies in memory (per-lane atomics on a few global bins cost 14 ms of a
  // 24 ms launch on the 3D gold slab at the laser peak)
  if (rec0) atomicAdd(s_spec + spectrum_bin<R>(out.e[0]), 1u);
  if (rec1) atomicAdd(s_spec + PIC_SPECTRUM_BINS + spectrum_bin<R>(out.e[1]), 1u);
  if ((mr0 | mr1) != 0ull && full_flag == 0u) {  // wave-uniform
    const ColdPtr<R> C = cold(P);
    unsigned long long base = 0;
    if (lane == 0) {
      const unsigned long long nr = (unsigned long long)(__popcll(mr0) + __popcll(mr1));
      base = atomicAdd(C->pcount, nr);
      if (base + nr >= C->pcap) __hip_atomic_store(C->pfull, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    base = __shfl(base, 0, 64);
#pragma unroll
    for (int proc = 0; proc < 2; ++proc) {
      const bool rec = proc == 0 ? rec0 : rec1;
      if (!rec) continue;
      const unsigned long long slot =
          proc == 0 ? base + lane_offset(mr0) : base + (unsigned long long)__popcll(mr0) + lane_offset(mr1);
      if (slot < C->pcap) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          C->px[a][slot] = out.xo[a];
          C->pk[a][slot] = out.k[proc][a];
        }
        C->pe[slot] = out.e[proc];
        C->pw[slot] = wgt;
        C->pstep[slot] = P.step;
        C->ppar[slot] = idv;
        C->pproc[slot] = (uint32_t)proc;
      }
    }
  }

  // ---- per-wave statistics slot --------------------------------------------
  const unsigned long long m_live = __ballot(live);
  if (m_live != 0ull) {  // wave-uniform
    const int64_t slot = (int64_t)chunk * (kBlock / 64) + (t >> 6);
    const unsigned long long m_ncs = __ballot(out.ev_ncs);
    const unsigned long long m_br = __ballot(out.ev_br);
    const unsigned long long m_cl = __ballot(out.clamped);
    unsigned long long* C = cold(P)->slot_cnt + slot * kSlotCnt;
    // the slot is this wave's alone; the counts go in as atomics whose result
    // is not used, so the wave does not wait for a read of the old value
    auto bump = [&](int k, unsigned long long v) { if (v) atomicAdd(C + k, v); };
    if (lane == 0) {
      bump(SC_ESTEPS, (unsigned long long)__popcll(m_live));
      if (!tiled && !jtiled && !frozen) bump(SC_UNTILED, (unsigned long long)__popcll(m_live));
    }
    if ((m_ncs | m_br | m_cl) != 0ull) {  // wave-uniform
      const unsigned long long m_keep = __ballot(rec0);
      const double e_keep0 = rec0 ? wgt * (double)out.e[0] : 0.0;
      const double e_drop = (out.ev_ncs && !out.keep_ncs) ? wgt * (double)out.e[0] : 0.0;
      const double e_keep1 = out.ev_br ? wgt * (double)out.e[1] : 0.0;
      const double s0 = wave_sum(e_keep0), s1 = wave_sum(e_keep1), s2 = wave_sum(e_drop);
      if (lane == 0) {
        bump(SC_EV_NCS, (unsigned long long)__popcll(m_ncs));
        bump(SC_EV_BR, (unsigned long long)__popcll(m_br));
        bump(SC_KEPT_NCS, (unsigned long long)__popcll(m_keep));
        bump(SC_KEPT_BR, (unsigned long long)__popcll(m_br));
        bump(SC_DROPPED, (unsigned long long)__popcll(m_ncs & ~m_keep));
        bump(SC_CLAMPED, (unsigned long long)__popcll(m_cl));
        double* Sm = cold(P)->slot_sum + slot * kSlotSum;
        if (m_keep) neumaier(Sm + 0, Sm + 1, s0);
        if (m_br) neumaier(Sm + 2, Sm + 3, s1);
        if (m_ncs & ~m_keep) neumaier(Sm + 4, Sm + 5, s2);
      }
    }
  }

  // ---- current deposit: last, so that its inputs are all that is live -----
  if (live) {
    if (tiled || jtiled) {
      if constexpr (kF32) {
        const LdsCurrent32 ja{reinterpret_cast<int*>(sJ), lo[0], lo[1], lo[2], ext[0], ext[1], nodes,
                              (float)ldexp(1.0, P.jbits)};
        electron_deposit<R, D>(P, ja, mv, wgt);
      } else {
        const LdsCurrent ja{reinterpret_cast<unsigned long long*>(sJ), lo[0], lo[1], lo[2], ext[0], ext[1], nodes};
        electron_deposit<R, D>(P, ja, mv, wgt);
      }
    } else {
      if constexpr (kF32) {
        const GlobalCurrent32 ja{{P.J[0], P.J[1], P.J[2]}, {P.gg[0], P.gg[1], P.gg[2], P.sz[0], P.sz[1]},
                                 (float)ldexp(1.0, P.jbits), 40 - P.jbits};
        electron_deposit<R, D>(P, ja, mv, wgt);
      } else {
        const GlobalCurrent ja{{P.J[0], P.J[1], P.J[2]}, {P.gg[0], P.gg[1], P.gg[2], P.sz[0], P.sz[1]}};
        electron_deposit<R, D>(P, ja, mv, wgt);
      }
    }
  }
  const int any_rec = __syncthreads_or((int)(rec0 || rec1));
  if (tiled || jtiled) {  // flush the LDS current: one global atomic per touched node
    for (int l = t; l < nodes; l += kBlock) {
      const JT qs[3] = {sJ[l], sJ[nodes + l], sJ[2 * nodes + l]};
      if ((qs[0] | qs[1] | qs[2]) == JT(0)) continue;  // untouched node: no index needed
      int i, j, k;
      decode(l, i, j, k);
      const int64_t m = I(i, j, k);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (qs[c] != JT(0)) {
          if constexpr (kF32) atomicAdd(P.J[c] + m, (unsigned long long)((long long)qs[c] << (40 - P.jbits)));
          else atomicAdd(P.J[c] + m, qs[c]);
        }
      }
    }
  }
  if (any_rec && t < 2 * PIC_SPECTRUM_BINS) {  // block-uniform
    const uint32_t v = s_spec[t];
    if (v)
      atomicAdd(cold(P)->spec + (size_t)(chunk % kSpecCopies) * (2 * PIC_SPECTRUM_BINS) + t,
                (unsigned long long)v);
  }
}

// Workgroup -> chunk.  The hardware deals workgroups to the 8 XCDs round
// robin (blockIdx % 8).  Groups of kXcdGroup consecutive chunks go to one XCD
// and successive groups to successive XCDs, so each XCD's L2 sees runs of
// neighbouring chunks while every XCD gets a share of every region of the
// grid.  Giving each XCD one contiguous eighth of the grid made the XCD that
// holds the laser-plasma interaction the straggler: on the 2D gold slab,
// groups of 16 run at 76.2 us per launch against 82.0 us for eighths (groups
// of 1: 76.0; of 128: 79.0); the 3D gold slab, with 524K chunks, runs at
// 9.89 ms against 9.82 ms.  The grid is a multiple of kGridQuantum.
__device__ inline uint32_t chunk_of_block(uint32_t b) {
  const uint32_t x = b & 7u, t = b >> 3;
  return ((t / kXcdGroup) * 8u + x) * kXcdGroup + (t % kXcdGroup);
}

// The 3D FP32 kernel runs at most 6 workgroups per CU (its LDS box), so it
// is compiled for 6 waves per SIMD: 80 VGPRs, room for the gather's loads
// to be in flight together.
template <class R, int D>
constexpr int kStepMinWaves = (sizeof(R) == 4 && D == 3) ? 6 : 1;

template <class R, int D>
__global__ __launch_bounds__(kBlock, (kStepMinWaves<R, D>)) void k_electron_step(const StepParams<R> P) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ __align__(16) uint32_t s_box[12];
  __shared__ uint32_t s_spec[2 * PIC_SPECTRUM_BINS];
  step_chunk<R, D>(P, chunk_of_block(blockIdx.x), smem, s_box, s_spec);
}

// Batched form for several runs: the chunks of every run are laid end to end
// (run j owns [first[j], first[j+1])) and one launch covers them all, with the
// same spread over the XCDs as the single-run kernel.  A chunk is processed
// exactly as the single-run kernel processes it, so a run's results do not
// depend on what else is in the batch.  (One chunk per workgroup: a
// grid-stride loop over chunks raises the kernel from 68 to 106 VGPRs and
// drops occupancy from 7 to 4 waves per SIMD.)
template <class R, int D>
__global__ __launch_bounds__(kBlock, (kStepMinWaves<R, D>)) void k_electron_step_batch(const StepParams<R>* __restrict__ tab,
                                                                const uint32_t* __restrict__ first,
                                                                int njobs) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ __align__(16) uint32_t s_box[12];
  __shared__ uint32_t s_spec[2 * PIC_SPECTRUM_BINS];
  const uint32_t w = chunk_of_block(blockIdx.x);
  if (w >= first[njobs]) return;  // padding of the grid to a multiple of kGridQuantum
  int lo = 0, hi = njobs - 1;     // largest j with first[j] <= w
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= w) lo = mid; else hi = mid - 1;
  }
  step_chunk<R, D>(tab[lo], w - first[lo], smem, s_box, s_spec);
}

template <class R, int D>
static void launch_one(const void* params, hipStream_t s) {
  const StepParams<R>& P = *static_cast<const StepParams<R>*>(params);
  if (P.N <= 0) return;
  constexpr int per_chunk = kBlock;
  int64_t blocks = (P.N + per_chunk - 1) / per_chunk;
  blocks = (blocks + kGridQuantum - 1) / kGridQuantum * kGridQuantum;  // see chunk_of_block
  const size_t lds = (size_t)P.lds_nodes * lds_bytes_per_node<R, D>();
  hipLaunchKernelGGL((k_electron_step<R, D>), dim3((unsigned)blocks), dim3(kBlock), lds, s, P);
}

template <class R, int D>
static void launch_batch(const void* tab, const uint32_t* first, int njobs, uint32_t total,
                         int lds_nodes, hipStream_t s) {
  if (njobs <= 0 || total == 0) return;
  const size_t lds = (size_t)lds_nodes * lds_bytes_per_node<R, D>();
  const int64_t blocks = ((int64_t)total + kGridQuantum - 1) / kGridQuantum * kGridQuantum;
  hipLaunchKernelGGL((k_electron_step_batch<R, D>), dim3((unsigned)blocks), dim3(kBlock), lds, s,
                     static_cast<const StepParams<R>*>(tab), first, njobs);
}

void launch_step_batch(int dims, bool fp32, const void* tab, const uint32_t* first, int njobs,
                       uint32_t total, int lds_nodes, hipStream_t s) {
  if (fp32) {
    if (dims == 1) launch_batch<float, 1>(tab, first, njobs, total, lds_nodes, s);
    else if (dims == 2) launch_batch<float, 2>(tab, first, njobs, total, lds_nodes, s);
    else launch_batch<float, 3>(tab, first, njobs, total, lds_nodes, s);
  } else {
    if (dims == 1) launch_batch<double, 1>(tab, first, njobs, total, lds_nodes, s);
    else if (dims == 2) launch_batch<double, 2>(tab, first, njobs, total, lds_nodes, s);
    else launch_batch<double, 3>(tab, first, njobs, total, lds_nodes, s);
  }
}

void launch_step(int dims, bool fp32, const void* params, hipStream_t s) {
  if (fp32) {
    if (dims == 1) launch_one<float, 1>(params, s);
    else if (dims == 2) launch_one<float, 2>(params, s);
    else launch_one<float, 3>(params, s);
  } else {
    if (dims == 1) launch_one<double, 1>(params, s);
    else if (dims == 2) launch_one<double, 2>(params, s);
    else launch_one<double, 3>(params, s);
  }
}

}  // namespace pic
