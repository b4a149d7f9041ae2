// Device building blocks shared by the electron and the ion step kernels:
// working-precision maths, grid indexing, field and current accessors, the
// linear field gather and the charge-conserving (Esirkepov) current deposit.
#pragma once
#include "pic_internal.hpp"
#include "philox.hpp"
#include "fpmath.hpp"

namespace pic {

// FP64: the fixed-order series of fpmath.hpp (the same bits as the oracle).
// FP32: the hardware's transcendental unit (v_sqrt_f32, v_log_f32 and
// v_exp_f32, each within a few ulp), a few instructions where the
// correctly rounded library forms take 11-24; the FP32 path's results are
// judged statistically against the FP64 path.  expm1 keeps its relative
// accuracy for small arguments (the per-step bremsstrahlung probability
// 1 - exp(-X)) with four terms of its series below 2^-7 (relative error
// under x^3/120 < 4e-9).
__device__ inline double m_sqrt(double v) { return sqrt(v); }
__device__ inline float m_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ inline double m_log(double v) { return fp_log(v); }
__device__ inline float m_log(float v) { return __logf(v); }
__device__ inline double m_exp(double v) { return fp_exp(v); }
__device__ inline float m_exp(float v) { return __expf(v); }
__device__ inline double m_expm1(double v) { return fp_expm1(v); }
__device__ inline float m_expm1(float v) {
  if (fabsf(v) < 0.0078125f)
    return v * __builtin_fmaf(v, __builtin_fmaf(v, __builtin_fmaf(v, 1.f / 24.f, 1.f / 6.f), 0.5f), 1.f);
  return __expf(v) - 1.f;
}
__device__ inline double m_floor(double v) { return floor(v); }
__device__ inline float m_floor(float v) { return floorf(v); }
__device__ inline double m_sin(double v) { return sin(v); }
__device__ inline float m_sin(float v) { return sinf(v); }
// divisions and square roots: IEEE in FP64 (bit parity), hardware rate in FP32
__device__ inline double m_div(double a, double b) { return a / b; }
__device__ inline float m_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double m_fsqrt(double v) { return sqrt(v); }
__device__ inline float m_fsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }

template <class R>
__device__ inline R unif(uint32_t r);
template <>
__device__ inline double unif<double>(uint32_t r) { return unif32(r); }
template <>
__device__ inline float unif<float>(uint32_t r) { return unif23f(r); }

template <class R>
struct Idx {
  int gg0, gg1, gg2, sz0, sz1;
  __device__ inline int64_t operator()(int i, int j, int k) const {
    return (int64_t)(i + gg0) + (int64_t)sz0 * ((int64_t)(j + gg1) + (int64_t)sz1 * (int64_t)(k + gg2));
  }
};

// Field access: straight from the Yee arrays, or from the block's LDS box.
template <class R>
struct GlobalField {
  const R* const* F;
  Idx<R> I;
  __device__ inline R operator()(int c, int i, int j, int k) const { return F[c][I(i, j, k)]; }
  __device__ inline int lin(int i, int j, int k) const { return (int)I(i, j, k); }
  __device__ inline int s1() const { return I.sz0; }
  __device__ inline int s2() const { return I.sz0 * I.sz1; }
  __device__ inline R at(int c, int l) const { return F[c][l]; }
};

template <class R>
struct LdsField {
  const R* T;
  int lo0, lo1, lo2, e0, e1, nodes;
  __device__ inline R operator()(int c, int i, int j, int k) const {
    return T[c * nodes + (i - lo0) + e0 * ((j - lo1) + e1 * (k - lo2))];
  }
  __device__ inline int lin(int i, int j, int k) const { return (i - lo0) + e0 * ((j - lo1) + e1 * (k - lo2)); }
  __device__ inline int s1() const { return e0; }
  __device__ inline int s2() const { return e0 * e1; }
  __device__ inline R at(int c, int l) const { return T[c * nodes + l]; }
};

// Current accumulation in 2^-40 fixed point: global atomics, or LDS atomics
// (ds_add_u64) on the block's box, flushed once per node afterwards.
struct GlobalCurrent {
  unsigned long long* J[3];
  Idx<double> I;
  __device__ inline void operator()(int c, int i, int j, int k, double v) const {
    const long long q = __double2ll_rn(v * kJScale);
    if (q != 0) atomicAdd(J[c] + I(i, j, k), (unsigned long long)q);
  }
};

struct LdsCurrent {
  unsigned long long* T;
  int lo0, lo1, lo2, e0, e1, nodes;
  __device__ inline void operator()(int c, int i, int j, int k, double v) const {
    const long long q = __double2ll_rn(v * kJScale);
    if (q != 0) atomicAdd(T + c * nodes + (i - lo0) + e0 * ((j - lo1) + e1 * (k - lo2)), (unsigned long long)q);
  }
};

// Linear interpolation of Yee component c (stagger S* = 1: half-integer).
template <class R, int D, int SX, int SY, int SZ, class F>
__device__ inline R gather(const F& f, int c, const R* g) {
  int i0 = 0, i1 = 0, i2 = 0;
  R f0 = R(0), f1 = R(0), f2 = R(0);
  {
    const R ga = g[0] - R(0.5) * R(SX);
    const R fl = m_floor(ga);
    i0 = (int)fl;
    f0 = ga - fl;
  }
  if (D == 1) return (R(1) - f0) * f(c, i0, 0, 0) + f0 * f(c, i0 + 1, 0, 0);
  {
    const R ga = g[1] - R(0.5) * R(SY);
    const R fl = m_floor(ga);
    i1 = (int)fl;
    f1 = ga - fl;
  }
  if (D == 3) {
    const R ga = g[2] - R(0.5) * R(SZ);
    const R fl = m_floor(ga);
    i2 = (int)fl;
    f2 = ga - fl;
  }
  const R v0 = (R(1) - f0) * f(c, i0, i1, i2) + f0 * f(c, i0 + 1, i1, i2);
  const R v1 = (R(1) - f0) * f(c, i0, i1 + 1, i2) + f0 * f(c, i0 + 1, i1 + 1, i2);
  const R a2 = (R(1) - f1) * v0 + f1 * v1;
  if (D == 2) return a2;
  const R w0 = (R(1) - f0) * f(c, i0, i1, i2 + 1) + f0 * f(c, i0 + 1, i1, i2 + 1);
  const R w1 = (R(1) - f0) * f(c, i0, i1 + 1, i2 + 1) + f0 * f(c, i0 + 1, i1 + 1, i2 + 1);
  const R b2 = (R(1) - f1) * w0 + f1 * w1;
  return (R(1) - f2) * a2 + f2 * b2;
}

// node weights of a point on a 4-node window starting at base
template <class R>
__device__ inline void shape4(R g, int base, R S[4]) {
  const R fl = m_floor(g);
  const int i = (int)fl;
  const R f = g - fl;
  S[0] = R(0); S[1] = R(0); S[2] = R(0); S[3] = R(0);
  const int o = i - base;  // 0, 1 or 2 (|move| < one cell)
  if (o == 0) { S[0] = R(1) - f; S[1] = f; }
  else if (o == 1) { S[1] = R(1) - f; S[2] = f; }
  else { S[2] = R(1) - f; S[3] = f; }
}

// Charge-conserving (Esirkepov) current of one macro-particle moving x0 -> x1
// at velocity v: contributions of charge density c0 = -w / V (an electron of
// weight w; an ion of charge q and weight w passes w = -q w)
template <class R, int D, class Acc, class PP>
__device__ inline void deposit(const PP& P, const Acc& J, const R* x0, const R* x1,
                               const R* v, double w) {
  const R c0 = R(-w * P.invV);
  R S0[3][4], S1[3][4];
  int b[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const R g0 = x0[a] * R(P.idx[a]);
    const R g1 = x1[a] * R(P.idx[a]);
    b[a] = (int)m_floor(g0) - 1;
    shape4<R>(g0, b[a], S0[a]);
    shape4<R>(g1, b[a], S1[a]);
  }
  if (D == 1) {
    const R qx = c0 * R(P.dxdt[0]);
    R acc = R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      acc = acc - qx * (S1[0][i] - S0[0][i]);
      J(0, b[0] + i, 0, 0, acc);
    }
    const R cy = c0 * v[1], cz = c0 * v[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const R sa = R(0.5) * (S0[0][i] + S1[0][i]);
      J(1, b[0] + i, 0, 0, cy * sa);
      J(2, b[0] + i, 0, 0, cz * sa);
    }
  } else if (D == 2) {
    const R qx = c0 * R(P.dxdt[0]), qy = c0 * R(P.dxdt[1]), cz = c0 * v[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      R acc = R(0);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const R W = R(0.5) * (S1[0][i] - S0[0][i]) * (S0[1][j] + S1[1][j]);
        acc = acc - qx * W;
        J(0, b[0] + i, b[1] + j, 0, acc);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R acc = R(0);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const R W = R(0.5) * (S0[0][i] + S1[0][i]) * (S1[1][j] - S0[1][j]);
        acc = acc - qy * W;
        J(1, b[0] + i, b[1] + j, 0, acc);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const R W = (S0[0][i] * S0[1][j] + S1[0][i] * S1[1][j]) * R(1.0 / 3.0) +
                    (S0[0][i] * S1[1][j] + S1[0][i] * S0[1][j]) * R(1.0 / 6.0);
        J(2, b[0] + i, b[1] + j, 0, cz * W);
      }
  } else {
    const R qx = c0 * R(P.dxdt[0]), qy = c0 * R(P.dxdt[1]), qz = c0 * R(P.dxdt[2]);
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j) {
        R acc = R(0);
        for (int i = 0; i < 3; ++i) {
          const R T = (S0[1][j] * S0[2][k] + S1[1][j] * S1[2][k]) * R(1.0 / 3.0) +
                      (S1[1][j] * S0[2][k] + S0[1][j] * S1[2][k]) * R(1.0 / 6.0);
          acc = acc - qx * ((S1[0][i] - S0[0][i]) * T);
          J(0, b[0] + i, b[1] + j, b[2] + k, acc);
        }
      }
    for (int k = 0; k < 4; ++k)
      for (int i = 0; i < 4; ++i) {
        R acc = R(0);
        for (int j = 0; j < 3; ++j) {
          const R T = (S0[0][i] * S0[2][k] + S1[0][i] * S1[2][k]) * R(1.0 / 3.0) +
                      (S1[0][i] * S0[2][k] + S0[0][i] * S1[2][k]) * R(1.0 / 6.0);
          acc = acc - qy * ((S1[1][j] - S0[1][j]) * T);
          J(1, b[0] + i, b[1] + j, b[2] + k, acc);
        }
      }
    for (int j = 0; j < 4; ++j)
      for (int i = 0; i < 4; ++i) {
        R acc = R(0);
        for (int k = 0; k < 3; ++k) {
          const R T = (S0[0][i] * S0[1][j] + S1[0][i] * S1[1][j]) * R(1.0 / 3.0) +
                      (S1[0][i] * S0[1][j] + S0[0][i] * S1[1][j]) * R(1.0 / 6.0);
          acc = acc - qz * ((S1[2][k] - S0[2][k]) * T);
          J(2, b[0] + i, b[1] + j, b[2] + k, acc);
        }
      }
  }
}

}  // namespace pic
