// Photons in flight and pair production (PIC_BW, PIC_BH): the pair channels
// the paper names beside NCS and bremsstrahlung (Sec. I and II.A for
// Breit-Wheeler in the laser field; Sec. II.B for Bethe-Heitler on the
// nuclei, "similar to the bremsstrahlung").
//
// Every stored photon record of at least 2 mc^2 travels on along its
// direction at c from the step after its emission.  Per step, in the fields
// E^n, B^n the electrons see and with the ion density of the collision test:
//   Breit-Wheeler: the pair optical depth (-ln u at the start) drops by
//     dt alpha (m c^2/hbar) (chi/eps) T(chi), chi = eps |E_perp + k x B| / E_S
//     (the electron's invariant with p = eps k, gamma = eps), ln T linear in
//     ln chi between table points, nothing below the first point; the photon
//     converts when the depth runs out;
//   Bethe-Heitler (if it did not): the Eq. (4) trial with the pair
//     cross-section, P = 1 - exp(-n sigma_BH(eps) c dt), against the 52-bit
//     uniform of the step's draw;
//   on a conversion the pair's energies come from the inverse-CDF rows of
//   the electron share (Breit-Wheeler) or positron share (Bethe-Heitler),
//   the two rows around chi or eps blended in the logarithm; both members
//   keep at least mc^2; the pair is recorded and the photon stops; the
//   others move x += k dt and are absorbed at the walls.
// Random numbers: Philox counter (parent, emission step, 2 + process, n) per
// step, (.., 0xFFFFFFFF) for the initial depth: independent of the record's
// slot in the buffer, which the device's append order decides.
//
// One grid-stride pass over the stored records per step; records that
// converted, left the box or cannot convert cost one byte read.  The FP64
// instantiation evaluates every expression in the written order (no
// contraction), the FP32 one keeps the optical depth and the 52-bit
// comparison in FP64.
#include "particle.hpp"

namespace pic {

void fill_photon_args(const Ctx& c, PhotonArgs& A) {
  const Grid& g = c.g;
  A.dims = g.dims;
  A.flags = c.cfg.flags;
  A.frozen_kind = c.cfg.frozen_kind;
  A.step = (uint32_t)c.step;
  A.key0 = c.key0;
  A.key1 = c.key1;
  for (int a = 0; a < 3; ++a) {
    A.n[a] = g.n[a];
    A.gg[a] = g.gg[a];
    A.sz[a] = g.sz[a];
    A.idx[a] = g.idx[a];
    A.L[a] = g.L[a];
    A.fE[a] = c.cfg.frozen_E[a];
    A.fB[a] = c.cfg.frozen_B[a];
    A.F[a] = c.E[a];
    A.F[3 + a] = (c.cfg.flags & PIC_FIELDS_FROZEN) ? c.B[a] : c.En[a];
    A.px[a] = c.px[a];
    A.pk[a] = c.pk[a];
    A.gx[a] = c.gx[a];
    A.rx[a] = c.rx[a];
    A.rk[a] = c.rk[a];
  }
  A.dt = g.dt;
  A.tn = (double)c.step * g.dt;
  A.iES = c.iES;
  A.K_P = 7.2973525693e-3 * c.E_S;
  A.K_BR = c.K_BR;
  A.fa = c.cfg.frozen_a;
  A.ni = c.ni;
  A.pcount = c.pcount;
  A.pcap = c.pcap;
  A.pe = c.pe;
  A.pw = c.pw;
  A.pstep = c.pstep;
  A.ppar = c.ppar;
  A.pproc = c.pproc;
  A.gtau = c.gtau;
  A.gst = c.gst;
  const DevTables& t = c.t;
  A.n_chi = t.n_chi; A.n_xp = t.n_xp; A.n_k = t.n_k; A.n_s = t.n_s;
  A.ln_chi0 = t.ln_chi0; A.idln_chi = t.idln_chi; A.ln_k0 = t.ln_k0; A.idln_k = t.idln_k;
  if (c.fp32) {
    A.bwT = t.bwTf; A.bwC = t.bwCf; A.bhS = t.bhSf; A.bhC = t.bhCf;
  } else {
    A.bwT = t.bwT; A.bwC = t.bwC; A.bhS = t.bhS; A.bhC = t.bhC;
  }
  A.rcap = c.rcap;
  A.rcount = c.rcount;
  A.rfull = c.rfull;
  A.rem = c.rem;
  A.rep = c.rep;
  A.rw = c.rw;
  A.rstep = c.rstep;
  A.rpar = c.rpar;
  A.rpst = c.rpst;
  A.rproc = c.rproc;
  A.ev = c.rev;
  A.esum = c.resum;
}

namespace {

constexpr int kPhotonBlocks = 2048;

// Share of a uniform-grid CDF row on [0, 1] at u (bisection, linear between
// points).
template <class R>
__device__ inline R share_inv(const R* __restrict__ C, int n, R u) {
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (C[mid] <= u) lo = mid; else hi = mid;
  }
  const R t = m_div(u - C[lo], C[lo + 1] - C[lo]);
  return m_div(R(lo) + t, R(n - 1));
}

template <class R, int D>
__global__ __launch_bounds__(kBlock) void k_photon_step(const PhotonArgs A) {
  constexpr bool kF32 = sizeof(R) == 4;
  const uint64_t cnt = *A.pcount;
  const uint64_t nst = cnt < A.pcap ? cnt : A.pcap;
  const uint32_t n = A.step;
  const bool frozen = (A.flags & PIC_FIELDS_FROZEN) != 0;
  const R* pe = (const R*)A.pe;
  for (uint64_t q = (uint64_t)blockIdx.x * kBlock + threadIdx.x; q < nst;
       q += (uint64_t)gridDim.x * kBlock) {
    uint8_t st = A.gst[q];
    if (st >= 2) continue;
    const uint32_t par = A.ppar[q], pst = A.pstep[q], pr = A.pproc[q];
    const R eps = pe[q];
    R x[3];
    if (st == 0) {
      if (pst == n) continue;  // emitted in this step
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        x[a] = ((const R*)A.px[a])[q];
        ((R*)A.gx[a])[q] = x[a];
      }
      if ((double)eps >= 2.0) {
        const U4 r0 = philox4x32_10(par, pst, 2u + pr, 0xFFFFFFFFu, A.key0, A.key1);
        A.gtau[q] = kF32 ? -(double)m_log(unif<R>(r0.v[0])) : -fp_log(unif32(r0.v[0]));
        st = 1;
      } else {
        st = 4;
      }
      A.gst[q] = st;
      if (st != 1) continue;
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) x[a] = ((const R*)A.gx[a])[q];
    }
    R k[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) k[a] = ((const R*)A.pk[a])[q];
    int conv = -1, bi = 0, ki = 0;
    R bf = R(0), kf = R(0);
    U4 r;
    bool have_r = false;
    // ---- Breit-Wheeler: the pair optical depth ----------------------------
    if (A.flags & PIC_BW) {
      R E[3] = {R(0), R(0), R(0)}, B[3] = {R(0), R(0), R(0)};
      if (frozen) {
        if (A.frozen_kind == PIC_FROZEN_UNIFORM) {
          for (int a = 0; a < 3; ++a) { E[a] = R(A.fE[a]); B[a] = R(A.fB[a]); }
        } else {
          const R phi = R(A.tn) - x[0];
          if (phi > R(0)) {
            const R v = R(A.fa) * m_sin(phi);
            E[1] = v;
            B[2] = v;
          }
        }
      } else {
        const GlobalField<R> f{(const R* const*)A.F, {A.gg[0], A.gg[1], A.gg[2], A.sz[0], A.sz[1]}};
        R g[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int a = 0; a < D; ++a) g[a] = x[a] * R(A.idx[a]);
        E[0] = gather<R, D, 1, 0, 0>(f, 0, g);
        E[1] = gather<R, D, 0, 1, 0>(f, 1, g);
        E[2] = gather<R, D, 0, 0, 1>(f, 2, g);
        B[0] = gather<R, D, 0, 1, 1>(f, 3, g);
        B[1] = gather<R, D, 1, 0, 1>(f, 4, g);
        B[2] = gather<R, D, 1, 1, 0>(f, 5, g);
      }
      const R cx = E[0] + (k[1] * B[2] - k[2] * B[1]);
      const R cy = E[1] + (k[2] * B[0] - k[0] * B[2]);
      const R cz = E[2] + (k[0] * B[1] - k[1] * B[0]);
      const R ke = k[0] * E[0] + k[1] * E[1] + k[2] * E[2];
      R q2 = (cx * cx + cy * cy + cz * cz) - ke * ke;
      if (q2 < R(0)) q2 = R(0);
      const R chi = eps * m_fsqrt(q2) * R(A.iES);
      if (chi > R(0)) {
        const R sl = (m_log(chi) - R(A.ln_chi0)) * R(A.idln_chi);
        if (sl >= R(0)) {
          if (sl >= R(A.n_chi - 1)) { bi = A.n_chi - 2; bf = R(1); }
          else { bi = (int)sl; bf = sl - R(bi); }
          const R* T = (const R*)A.bwT;
          const R lT = T[bi] + bf * (T[bi + 1] - T[bi]);
          const R dtau = m_div(R(A.K_P) * chi, eps) * m_exp(lT) * R(A.dt);
          const double tau = A.gtau[q] - (double)dtau;
          A.gtau[q] = tau;
          if (tau <= 0.0) conv = 0;
        }
      }
    }
    // ---- Bethe-Heitler: Eq. (4) with the pair cross-section ---------------
    if (conv < 0 && (A.flags & PIC_BH)) {
      int ci[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < D; ++a) {
        int qq = (int)m_floor(x[a] * R(A.idx[a]));
        qq = qq < 0 ? 0 : (qq > A.n[a] - 1 ? A.n[a] - 1 : qq);
        ci[a] = qq;
      }
      const double ni = A.ni[ci[0] + (int64_t)A.n[0] * (ci[1] + (int64_t)A.n[1] * ci[2])];
      const R sl = (m_log(eps) - R(A.ln_k0)) * R(A.idln_k);
      if (ni > 0.0 && sl >= R(0)) {
        if (sl >= R(A.n_k - 1)) { ki = A.n_k - 2; kf = R(1); }
        else { ki = (int)sl; kf = sl - R(ki); }
        const R* S = (const R*)A.bhS;
        const R sig = S[ki] + kf * (S[ki + 1] - S[ki]);
        if (sig > R(0)) {
          const R X = R(A.K_BR) * R(ni) * sig * R(A.dt);
          const R P = -m_expm1(-X);
          r = philox4x32_10(par, pst, 2u + pr, n, A.key0, A.key1);
          have_r = true;
          if (unif52(r.v[0], r.v[1]) < (double)P) conv = 1;
        }
      }
    }
    if (conv >= 0) {
      if (!have_r) r = philox4x32_10(par, pst, 2u + pr, n, A.key0, A.key1);
      R em, ep;
      if (conv == 0) {  // electron share xi
        const R* C = (const R*)A.bwC;
        const R u = kF32 ? unif<R>(r.v[2]) : R(unif32(r.v[2]));
        const R xa = share_inv<R>(C + (int64_t)bi * A.n_xp, A.n_xp, u);
        const R xb = share_inv<R>(C + (int64_t)(bi + 1) * A.n_xp, A.n_xp, u);
        R xi = xa + bf * (xb - xa);
        const R lo = m_div(R(1), eps), hi = R(1) - lo;
        if (xi < lo) xi = lo;
        if (xi > hi) xi = hi;
        em = xi * eps;
        ep = eps - em;
      } else {          // positron share x on s = (x - 1/k) / (1 - 2/k)
        const R* C = (const R*)A.bhC;
        const R u = kF32 ? unif<R>(r.v[3]) : R(unif32(r.v[3]));
        const R sa = share_inv<R>(C + (int64_t)ki * A.n_s, A.n_s, u);
        const R sb = share_inv<R>(C + (int64_t)(ki + 1) * A.n_s, A.n_s, u);
        const R sv = sa + kf * (sb - sa);
        const R lo = m_div(R(1), eps);
        const R xp = lo + sv * (R(1) - R(2) * lo);
        ep = xp * eps;
        em = eps - ep;
      }
      const double we = A.pw[q];
      atomicAdd(A.ev + conv, 1ull);
      atomicAdd(A.esum + conv, we * (double)eps);
      // one slot per pair; none once a reservation has reached the capacity
      if (*(volatile const uint32_t*)A.rfull == 0u) {
        const unsigned long long slot = atomicAdd(A.rcount, 1ull);
        if (slot + 1 >= A.rcap) *(volatile uint32_t*)A.rfull = 1u;
        if (slot < A.rcap) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            ((R*)A.rx[a])[slot] = x[a];
            ((R*)A.rk[a])[slot] = k[a];
          }
          ((R*)A.rem)[slot] = em;
          ((R*)A.rep)[slot] = ep;
          A.rw[slot] = we;
          A.rstep[slot] = n;
          A.rpar[slot] = par;
          A.rpst[slot] = pst;
          A.rproc[slot] = pr | ((uint32_t)conv << 1);
        }
      }
      A.gst[q] = 2;
      continue;
    }
    // ---- move on; absorbed at the walls -----------------------------------
    bool out = false;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      x[a] = x[a] + k[a] * R(A.dt);
      if (x[a] < R(0) || x[a] >= R(A.L[a])) out = true;
      ((R*)A.gx[a])[q] = x[a];
    }
    if (out) A.gst[q] = 3;
  }
}

template <class R>
void launch_r(const PhotonArgs& A, hipStream_t s) {
  if (A.dims == 1) hipLaunchKernelGGL((k_photon_step<R, 1>), dim3(kPhotonBlocks), dim3(kBlock), 0, s, A);
  else if (A.dims == 2) hipLaunchKernelGGL((k_photon_step<R, 2>), dim3(kPhotonBlocks), dim3(kBlock), 0, s, A);
  else hipLaunchKernelGGL((k_photon_step<R, 3>), dim3(kPhotonBlocks), dim3(kBlock), 0, s, A);
}

}  // namespace

void launch_photon_step(const PhotonArgs& A, bool fp32, hipStream_t s) {
  if (A.pcap == 0) return;
  if (fp32) launch_r<float>(A, s);
  else launch_r<double>(A, s);
}

}  // namespace pic
