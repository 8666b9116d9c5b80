// Device kernels of the lattice Boltzmann hot path for gfx950 (MI355X).
//
// One thread per lattice node, 256-thread tiles of consecutive nodes (x
// fastest).  Distributions live in one in-place array per lattice, blocked by
// x-row: element (q, row, x) at (row Q + q) nx + x, so that all Q populations
// of a row form one contiguous block (for DRAM page locality; each population
// is still contiguous along x for coalesced access).  The array is updated
// with the A-A pattern: on even steps a
// node reads its own slots and writes its post-collision values into the
// opposite slots (no data movement between nodes); on odd steps it gathers
// from its neighbours' opposite slots and scatters into its neighbours' slots.
// Each slot is read and written by the same thread within a step, so the
// update is race-free in place.  Halfway bounce-back only changes which slot a
// link reads / writes; boundary nodes are described by compact per-row
// records so that bulk rows pay no extra memory traffic.
//
// All quantities inside the kernels are dimensionless: velocities in units of
// c = dx/dt, body force as a dt / c, magnetic field as B / (c sqrt(mu)).
#include <type_traits>

#include "device.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// local physics
// ---------------------------------------------------------------------------
template <class T>
struct Macro {
  T drho, rho, irho;
  T J[3];   // momentum sum e d
  T Je[3];  // rho u^eq formed from J: J + lEq rho A
  T U[3], A[3], V[3], Ue[3], UF[3];
  T pi[6];  // Pi^neq / c^2: xx, yy, zz, xy, xz, yz
  T tau, itau, C;
  T b[3];
};

// MHD couplings (template parameter MHD): 0 none; 1 magnetic stress in the
// equilibrium (Eq. 10, the paper's approach); 2 Lorentz force through the
// force term with a hydrodynamic equilibrium (the third approach of Section 4).
//
// Moments (Section 2), model velocities, Pi^neq (cheap form after Eq. 9,
// with the Maxwell stress of Eq. 11 under coupling 1), Smagorinsky tau.
// Under coupling 1 the stored deviations are taken from w rho0 + phi(B0)
// (the rest equilibrium in the uniform field); db = b - b0 is the induced
// field and lam (coupling 2) the antisymmetric first moment of the induction
// distributions, lam_i = eps_ilm sum_k e_kl h_km.
//
// RAW (16-bit formats, interior nodes): d holds the values in their stored
// units (d_q / isc_q); a direction and its opposite share the factor isc_q,
// so each pair's sum and difference are scaled once.
template <class L, class T, int MHD, bool NEED_PI, bool RAW = false>
__device__ __forceinline__ void macro(const T (&d)[L::Q], const Phys& p, T Ax, T Ay, T Az, const T (&db)[3],
                                      const T (&lam)[3], Macro<T>& m) {
  // Moments from sums and differences of opposite populations (q odd, q + 1):
  // s = d_q + d_q+1 carries the even moments (rho, second moments), t = d_q -
  // d_q+1 the odd ones (momentum).  Pairing values of like size first keeps
  // the rounding of these sums small; the equilibrium below re-injects it
  // every step.
  T ps[(L::Q - 1) / 2], pt[(L::Q - 1) / 2];
#pragma unroll
  for (int k = 0; k < (L::Q - 1) / 2; ++k) {
    ps[k] = d[2 * k + 1] + d[2 * k + 2];
    pt[k] = d[2 * k + 1] - d[2 * k + 2];
    if (RAW) {
      ps[k] *= (T)p.inv_scale[2 * k + 1];
      pt[k] *= (T)p.inv_scale[2 * k + 1];
    }
  }
  T drho = RAW ? d[0] * (T)p.inv_scale[0] : d[0], jx = ZERO<T>, jy = ZERO<T>, jz = ZERO<T>;
#pragma unroll
  for (int k = 0; k < (L::Q - 1) / 2; ++k) {
    const int q = 2 * k + 1;
    drho += ps[k];
    if (L::ex(q) > 0) jx += pt[k];
    if (L::ex(q) < 0) jx -= pt[k];
    if (L::ey(q) > 0) jy += pt[k];
    if (L::ey(q) < 0) jy -= pt[k];
    if (L::ez(q) > 0) jz += pt[k];
    if (L::ez(q) < 0) jz -= pt[k];
  }
  m.drho = drho;
  m.rho = par<T>(p.rho0, p.f.rho0) + drho;
  m.irho = rcp(m.rho);
  m.J[0] = jx;
  m.J[1] = jy;
  m.J[2] = jz;
  m.U[0] = jx * m.irho;
  m.U[1] = jy * m.irho;
  m.U[2] = jz * m.irho;
  // porous resistance -sigma v, v = U + A / 2 with A including it:
  // A = (A_ext - sigma dt U) / (1 + sigma dt / 2) (exactly A_ext without it)
  const T ds = par<T>(p.darcy_s, p.f.darcy_s), di = par<T>(p.darcy_inv, p.f.darcy_inv);
  m.A[0] = (Ax - ds * m.U[0]) * di;
  m.A[1] = (Ay - ds * m.U[1]) * di;
  m.A[2] = (Az - ds * m.U[2]) * di;
#pragma unroll
  for (int k = 0; k < 3; ++k) m.b[k] = par<T>(p.b0[k], p.f.b0[k]) + db[k];
  if (MHD == 2) {
    // Lorentz force J x B / rho.  The induction moment's non-equilibrium
    // part gives curl b (first order Chapman-Enskog); with the velocity's own
    // half-force the current solves [tau_m theta I + (b^2 I - b b^T) / rho] J
    // = r, r = -lam + 2 U* x b, U* = U + A_ext / 2 (dimensionless), and the
    // force needs only J x b = (r x b) / (tau_m theta + b^2 / rho).
    const T* b = m.b;
    const T us[3] = {m.U[0] + T(0.5) * m.A[0], m.U[1] + T(0.5) * m.A[1], m.U[2] + T(0.5) * m.A[2]};
    const T r[3] = {-lam[0] + T(2) * (us[1] * b[2] - us[2] * b[1]), -lam[1] + T(2) * (us[2] * b[0] - us[0] * b[2]),
                    -lam[2] + T(2) * (us[0] * b[1] - us[1] * b[0])};
    const T ia = rcp(m.rho * par<T>(p.tm_theta, p.f.tm_theta) + (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
    m.A[0] += (r[1] * b[2] - r[2] * b[1]) * ia;
    m.A[1] += (r[2] * b[0] - r[0] * b[2]) * ia;
    m.A[2] += (r[0] * b[1] - r[1] * b[0]) * ia;
  }
  const T lEq = par<T>(p.lEq, p.f.lEq);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    m.V[k] = m.U[k] + T(0.5) * m.A[k];
    m.Ue[k] = m.U[k] + lEq * m.A[k];
    m.Je[k] = m.J[k] + lEq * m.rho * m.A[k];
  }
  m.tau = par<T>(p.tau0, p.f.tau0);
  m.itau = par<T>(p.inv_tau0, p.f.inv_tau0);
  if (NEED_PI || p.les_K > 0.0) {
    T sxx = ZERO<T>, syy = ZERO<T>, szz = ZERO<T>, sxy = ZERO<T>, sxz = ZERO<T>, syz = ZERO<T>;
#pragma unroll
    for (int k = 0; k < (L::Q - 1) / 2; ++k) {
      const int q = 2 * k + 1;  // e_q e_q is the same for q and its opposite
      if (L::ex(q) != 0) sxx += ps[k];
      if (L::ey(q) != 0) syy += ps[k];
      if (L::ez(q) != 0) szz += ps[k];
      if (L::ex(q) * L::ey(q) > 0) sxy += ps[k];
      if (L::ex(q) * L::ey(q) < 0) sxy -= ps[k];
      if (L::ex(q) * L::ez(q) > 0) sxz += ps[k];
      if (L::ex(q) * L::ez(q) < 0) sxz -= ps[k];
      if (L::ey(q) * L::ez(q) > 0) syz += ps[k];
      if (L::ey(q) * L::ez(q) < 0) syz -= ps[k];
    }
    const T third = drho * T(1.0 / 3.0);
    const T rho = m.rho * par<T>(p.quad, p.f.quad);  // the Stokes equilibrium has no rho u u part
    m.pi[0] = sxx - third - rho * m.Ue[0] * m.Ue[0];
    m.pi[1] = syy - third - rho * m.Ue[1] * m.Ue[1];
    m.pi[2] = L::D == 3 ? szz - third - rho * m.Ue[2] * m.Ue[2] : T(0);
    m.pi[3] = sxy - rho * m.Ue[0] * m.Ue[1];
    m.pi[4] = L::D == 3 ? sxz - rho * m.Ue[0] * m.Ue[2] : T(0);
    m.pi[5] = L::D == 3 ? syz - rho * m.Ue[1] * m.Ue[2] : T(0);
    if (MHD == 1) {
      // the stored second moment lacks L(b0); subtract L(b) - L(b0),
      // L_ij = b^2 delta_ij / 2 - b_i b_j, formed from db to keep precision
      const T bs[3] = {m.b[0] + par<T>(p.b0[0], p.f.b0[0]), m.b[1] + par<T>(p.b0[1], p.f.b0[1]), m.b[2] + par<T>(p.b0[2], p.f.b0[2])};  // b + b0
      const T b2h = T(0.5) * (db[0] * bs[0] + db[1] * bs[1] + db[2] * bs[2]);      // (b^2 - b0^2)/2
      // b_i b_j - b0_i b0_j = (db_i bs_j + bs_i db_j) / 2
      m.pi[0] -= b2h - db[0] * bs[0];
      m.pi[1] -= b2h - db[1] * bs[1];
      m.pi[2] -= b2h - db[2] * bs[2];
      m.pi[3] += T(0.5) * (db[0] * bs[1] + bs[0] * db[1]);
      m.pi[4] += T(0.5) * (db[0] * bs[2] + bs[0] * db[2]);
      m.pi[5] += T(0.5) * (db[1] * bs[2] + bs[1] * db[2]);
    }
    if (p.les_K > 0.0) {
      // nu_eff = nu0 + (Cs dx)^2 sqrt(2 S:S), S from Eq. (9) at tau_eff:
      // positive root of tau^2 - tau0 tau - 9 sqrt(2) Cs^2 |Pi|/(2 rho) = 0
      // (dimensionless form; dx / (c dt) = 1).
      const T pp = m.pi[0] * m.pi[0] + m.pi[1] * m.pi[1] + m.pi[2] * m.pi[2] +
                   T(2) * (m.pi[3] * m.pi[3] + m.pi[4] * m.pi[4] + m.pi[5] * m.pi[5]);
      const T qn = vsqrt(pp);
      const T t0 = par<T>(p.tau0, p.f.tau0);
      m.tau = T(0.5) * (t0 + vsqrt(t0 * t0 + par<T>(p.les_K, p.f.les_K) * qn * m.irho));
      m.itau = rcp(m.tau);
    }
  }
  m.C = T(1) - par<T>(p.cG, p.f.cG) * T(0.5) * m.itau;
  const T lF = par<T>(p.lF0, p.f.lF0) + par<T>(p.lF1, p.f.lF1) * m.tau;
  const T kF = par<T>(p.kF, p.f.kF);
#pragma unroll
  for (int k = 0; k < 3; ++k) m.UF[k] = kF * m.U[k] + lF * m.A[k];
}

// Relaxation of Eq. (2) with the equilibrium of Eq. (1) (+ magnetic part of
// Eq. 10) and the force term of Section 2 / Eq. (3); d is replaced by d_rel.
//
// Rounding design (FP32 arithmetic, FP32 or 16-bit storage).  In a steady or
// slowly varying flow every rounding below repeats with the same sign at
// each step, so a rounding that is large compared with the per-step changes
// (the force increment rho a dt ~ 1e-7 beside f ~ 1e-2) accumulates like a
// bias.  The equilibrium is therefore split into
//   a large part at the node's own velocity u = j / rho from the rounded
//   moments, whose difference with d (the small non-equilibrium part) is
//   formed first, and
//   a small part holding the shift u -> u^eq = u + lEq dt a and the
//   magnetic term,
// so that small quantities are never rounded at the scale of large ones.  The
// weights 1/9, 1/18, 1/36 are applied as hi + lo parts so that the large
// part's moments are not scaled by the weights' own rounding, and with
// FP32 storage (CLOSE) the mass and momentum of its non-equilibrium part are
// closed exactly (below; under 16-bit storage, at boundary nodes, the
// format's rounding is far coarser and the closure is left out).
// sink(q, value) receives each post-collision value as soon as it is formed,
// so that it can be stored at once and its register freed.
//
// (16-bit formats at interior nodes use collide_raw below.)
template <class L, class T, int MHD, class Sink, bool CLOSE>
__device__ __forceinline__ void collide(const T (&d)[L::Q], const Macro<T>& m, const T (&db)[3], const Phys& p,
                                        Sink&& sink) {
  const T rho = m.rho;
  const T lEq = par<T>(p.lEq, p.f.lEq);
  const T usq = T(1.5) * (m.U[0] * m.U[0] + m.U[1] * m.U[1] + m.U[2] * m.U[2]);
  const T ua = m.U[0] * m.A[0] + m.U[1] * m.A[1] + m.U[2] * m.A[2];
  const T aa = m.A[0] * m.A[0] + m.A[1] * m.A[1] + m.A[2] * m.A[2];
  const T ufa = m.UF[0] * m.A[0] + m.UF[1] * m.A[1] + m.UF[2] * m.A[2];
  const T cr = m.C * rho;
  const T itau = m.itau;
  const T rl = rho * lEq, rl2 = rho * lEq * lEq;
  const T quad = par<T>(p.quad, p.f.quad);  // 0 for the Stokes equilibrium
  const T rq = rho * quad, rlq = rl * quad, rl2q = rl2 * quad;
  T bs[3] = {T(0), T(0), T(0)}, db2 = T(0);
  if (MHD == 1) {
#pragma unroll
    for (int k = 0; k < 3; ++k) bs[k] = m.b[k] + par<T>(p.b0[k], p.f.b0[k]);  // b + b0
    db2 = db[0] * bs[0] + db[1] * bs[1] + db[2] * bs[2];     // b^2 - b0^2
  }
  const T last = (MHD == 1 && L::D == 3) ? db2 * T(1.0 / 6.0) : T(0);  // no -b^2 / 6 in two dimensions
  // The increment is formed first and added to d once: adding the small
  // force term F to an already rounded d + (neq + w Rs) / tau would round it
  // away in the same direction at every step (a drift of momentum and mass in
  // slowly varying flows).
  //
  // Parts of direction q and its opposite q + 1 (q odd, e_{q+1} = -e_q): the
  // parts even in e are formed once, the odd ones change sign.
  struct PairTerms {
    T Eb, Ob, Es, Os, EF, OF;
  };
  auto pair_terms = [&](int q) __attribute__((always_inline)) {
    PairTerms t;
    const T w = (T)L::w(q);
    const T eu = edot<L>(q, m.U[0], m.U[1], m.U[2]);
    const T ej = edot<L>(q, m.J[0], m.J[1], m.J[2]);
    const T ea = edot<L>(q, m.A[0], m.A[1], m.A[2]);
    const T euf = edot<L>(q, m.UF[0], m.UF[1], m.UF[2]);
    // large part: w [drho + 3 e.j + rho (9/2 (e.u)^2 - 3/2 u.u)]
    t.Eb = m.drho + rq * (T(4.5) * eu * eu - usq);
    t.Ob = T(3) * ej;
    // small part: the u^eq shift
    //   rho [(e.ue)^2 9/2 - ue.ue 3/2] - (same at u) + 3 e.(rho lEq A),
    // and the magnetic term phi(b) - phi(b0)
    t.Es = rlq * (T(9) * eu * ea - T(3) * ua) + rl2q * (T(4.5) * ea * ea - T(1.5) * aa);
    if (MHD == 1) {
      // (e.b)^2 - (e.b0)^2 = (e.db)(e.(b + b0))
      const T edb = edot<L>(q, db[0], db[1], db[2]);
      const T ebs = edot<L>(q, bs[0], bs[1], bs[2]);
      t.Es += T(4.5) * (T(0.5) * db2 * (T)L::e2(q) - edb * ebs - last);
    }
    t.Os = rl * (T(3) * ea);
    // force term C rho w [3 (e - u^F).a + 9 (e.u^F)(e.a)]
    const T cw = cr * w;
    t.EF = cw * (T(9) * euf * ea - T(3) * ufa);
    t.OF = cw * (T(3) * ea);
    return t;
  };
  // rest direction (e = 0): small part and force term
  T Rs0 = rlq * (T(-3) * ua) + rl2q * (T(-1.5) * aa);
  if (MHD == 1) Rs0 += T(-4.5) * last;
  const T F0 = cr * (T)L::w(0) * (T(-3) * ufa);
  if constexpr (CLOSE) {
    // FP32.  The large part's rounding (about one unit of the last place of
    // f per direction) would change the mass and momentum of the
    // non-equilibrium part neq = w Rb - d, which relaxation never removes:
    // in slowly varying flows it repeats with the same sign every step.  So
    // its conserved moments are closed exactly: the pairs with two nonzero
    // components come first and their sums are kept; each axis pair then
    // takes the odd part that makes the momentum of neq zero along its axis,
    // and the rest direction the value that makes its mass zero (all sums
    // at the size of neq, far below that of f).  In exact arithmetic these
    // are the values the formulas give.  (Measured on the 256x128x128 duct:
    // the same mean step time as the formulas in direction order; closing
    // with the last pairs instead, stored in direction order, 1 % slower.)
    T Mn = ZERO<T>, Jn[3] = {ZERO<T>, ZERO<T>, ZERO<T>};
#pragma unroll
    for (int k = 0; k < (L::Q - 1) / 2; ++k) {
      const int q = 2 * k + 1;
      if (L::e2(q) != 2) continue;
      const PairTerms t = pair_terms(q);
      const T w = (T)L::w(q);
      const T wlo = (T)(L::w(q) - (double)w);
      const T Rp = t.Eb + t.Ob, Rm = t.Eb - t.Ob;
      const T np = (w * Rp + wlo * Rp) - d[q];
      const T nm = (w * Rm + wlo * Rm) - d[q + 1];
      Mn += np + nm;
      const T od = np - nm;
      if (L::ex(q) > 0) Jn[0] += od;
      if (L::ex(q) < 0) Jn[0] -= od;
      if (L::ey(q) > 0) Jn[1] += od;
      if (L::ey(q) < 0) Jn[1] -= od;
      if (L::ez(q) > 0) Jn[2] += od;
      if (L::ez(q) < 0) Jn[2] -= od;
      sink(q, d[q] + ((np + w * (t.Es + t.Os)) * itau + (t.EF + t.OF)));
      sink(q + 1, d[q + 1] + ((nm + w * (t.Es - t.Os)) * itau + (t.EF - t.OF)));
    }
#pragma unroll
    for (int k = 0; k < (L::Q - 1) / 2; ++k) {
      const int q = 2 * k + 1;
      if (L::e2(q) != 1) continue;
      const PairTerms t = pair_terms(q);
      const T w = (T)L::w(q);
      const T wlo = (T)(L::w(q) - (double)w);
      // axis of q (+1 along it; its opposite -1)
      const int ax = L::ex(q) != 0 ? 0 : (L::ey(q) != 0 ? 1 : 2);
      const T E2 = T(2) * t.Eb;
      const T ev = (w * E2 + wlo * E2) - (d[q] + d[q + 1]);  // neq_q + neq_q+1
      const T od = -Jn[ax];                                  // neq_q - neq_q+1
      const T np = T(0.5) * (ev + od), nm = T(0.5) * (ev - od);
      Mn += ev;
      sink(q, d[q] + ((np + w * (t.Es + t.Os)) * itau + (t.EF + t.OF)));
      sink(q + 1, d[q + 1] + ((nm + w * (t.Es - t.Os)) * itau + (t.EF - t.OF)));
    }
    sink(0, d[0] + ((-Mn + (T)L::w(0) * Rs0) * itau + F0));
  } else {
    // rest direction (e = 0)
    {
      const T w = (T)L::w(0);
      const T wlo = (T)(L::w(0) - (double)w);
      const T Rb = m.drho - rq * usq;
      const T neq = (w * Rb + wlo * Rb) - d[0];
      sink(0, d[0] + ((neq + w * Rs0) * itau + F0));
    }
#pragma unroll
    for (int k = 0; k < (L::Q - 1) / 2; ++k) {
      const int q = 2 * k + 1;
      const PairTerms t = pair_terms(q);
      const T w = (T)L::w(q);
      const T wlo = (T)(L::w(q) - (double)w);
      {
        const T Rb = t.Eb + t.Ob;
        const T neq = (w * Rb + wlo * Rb) - d[q];
        sink(q, d[q] + ((neq + w * (t.Es + t.Os)) * itau + (t.EF + t.OF)));
      }
      {
        const T Rb = t.Eb - t.Ob;
        const T neq = (w * Rb + wlo * Rb) - d[q + 1];
        sink(q + 1, d[q + 1] + ((neq + w * (t.Es - t.Os)) * itau + (t.EF - t.OF)));
      }
    }
  }
}

// The same relaxation in the stored units of a 16-bit format at interior
// nodes (no MHD): v = K d / w with K = 2^10 (FP16) or 1 (BF16).  Eq. (1) and
// the force term of Eq. (3) are both quadratic in e, so
//   w R(e) = f^eq - w rho0,  R(e) = drho + rho [3 e.ue + quad (9/2 (e.ue)^2 - 3/2 ue.ue)],
//   F(e) = w C rho [3 (e - uF).a + 9 (e.uF)(e.a)],
// and the relaxed value d + (w R - d) / tau + F becomes, in stored units,
//   v' = v (1 - 1/tau) + K P(e),  P(e) = R(e) / tau + F(e) / w = a0 + b.e + e.Cm.e,
// whose ten coefficients are formed once per node; a direction and its
// opposite then share the even part a0 + e.Cm.e and differ in the sign of
// b.e.  The format's rounding (2^-11 or 2^-8 relative) is far coarser than
// that of this FP32 form, so the splitting of the FP32 path is not needed.
template <class L, int P, class Sink>
__device__ __forceinline__ void collide_raw(const float (&v)[L::Q], const Macro<float>& m, const Phys& p,
                                            Sink&& sink) {
  using T = float;
  constexpr T K = P == S_F16 ? T(1024) : T(1);
  const T rho = m.rho, itau = m.itau;
  const T kq = K * rho * par<T>(p.quad, p.f.quad);  // K rho quad
  const T kc = K * m.C * rho;                        // K C rho
  const T kt = kq * itau;
  const T* ue = m.Ue;
  const T* uf = m.UF;
  const T* A = m.A;
  const T uu = ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2];
  const T ufa = uf[0] * A[0] + uf[1] * A[1] + uf[2] * A[2];
  const T a0 = (K * m.drho - T(1.5) * kq * uu) * itau - T(3) * kc * ufa;
  T b[3], Cm[3], Cd[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    b[i] = T(3) * (K * rho * itau * ue[i] + kc * A[i]);
    Cm[i] = T(4.5) * kt * ue[i] * ue[i] + T(9) * kc * uf[i] * A[i];
    Cd[i] = a0 + Cm[i];
  }
  // twice the off-diagonal coefficients, xy, xz, yz
  const int ci[3] = {0, 0, 1}, cj[3] = {1, 2, 2};
  T C2[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int i = ci[c], j = cj[c];
    C2[c] = T(9) * kt * ue[i] * ue[j] + T(9) * kc * (uf[i] * A[j] + uf[j] * A[i]);
  }
  const T om = T(1) - itau;
  sink(0, v[0] * om + a0);
#pragma unroll
  for (int k = 0; k < (L::Q - 1) / 2; ++k) {
    const int q = 2 * k + 1;
    const int e[3] = {L::ex(q), L::ey(q), L::ez(q)};
    T E, O;
    if (L::e2(q) == 1) {
      const int i = e[0] != 0 ? 0 : (e[1] != 0 ? 1 : 2);
      E = Cd[i];
      O = e[i] > 0 ? b[i] : -b[i];
    } else {
      // two nonzero components i < j
      const int i = e[0] != 0 ? 0 : 1;
      const int j = e[2] != 0 ? 2 : 1;
      const int c = i == 0 ? (j == 1 ? 0 : 1) : 2;
      const T base = Cd[i] + Cm[j];  // a0 + Cm_ii + Cm_jj
      E = e[i] * e[j] > 0 ? base + C2[c] : base - C2[c];
      O = (e[i] > 0 ? b[i] : -b[i]) + (e[j] > 0 ? b[j] : -b[j]);
    }
    sink(q, v[q] * om + (E + O));
    sink(q + 1, v[q + 1] * om + (E - O));
  }
}

// Induction lattice: g^eq_{k,i} = W_k [b_i + (e_kj / theta)(V_j b_i - b_j V_i)],
// stored as deviations from W_k b0_i; relaxation with 1/tau_m.
// db: the induced field B - B0 as summed from the distributions.  The
// equilibrium's field term takes it directly: B - B0 formed from the total
// field in FP32 would round it to the last place of B0 (3e-8 at B0 = 0.25,
// against induced fields of 1e-6 and less), a relative error of a few
// percent in every step's induction relaxation.
template <class L, class T>
__device__ __forceinline__ void collide_g(T (&h)[Ind<L>::K][Ind<L>::NB], const Macro<T>& m, const T (&db)[3],
                                          const Phys& p) {
  using I = Ind<L>;
  const T itm = par<T>(p.inv_tau_m, p.f.inv_tau_m);
  const T b[3] = {m.b[0], m.b[1], m.b[2]};
  const T V[3] = {m.V[0], m.V[1], m.V[2]};
#pragma unroll
  for (int k = 0; k < I::K; ++k) {
    const T w = (T)I::w(k);
    const int ax = (k - 1) >> 1;           // axis of direction k (k >= 1)
    const T sgn = (k & 1) ? T(1) : T(-1);  // +1 for odd k
#pragma unroll
    for (int i = 0; i < I::NB; ++i) {
      T heq = w * db[i];
      if (k > 0) heq += w * sgn * T(1.0 / I::theta) * (V[ax] * b[i] - b[ax] * V[i]);
      h[k][i] = h[k][i] + (heq - h[k][i]) * itm;
    }
  }
}

// Induced field db = sum_k h_k and the antisymmetric first moment
// lam_i = eps_ilm Lambda_lm, Lambda_lm = sum_k e_kl h_km = h_{+l,m} - h_{-l,m}.
template <class L, class T>
__device__ __forceinline__ void ind_moments(const T (&h)[Ind<L>::K][Ind<L>::NB], T (&db)[3], T (&lam)[3]) {
  constexpr int NB = Ind<L>::NB;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T s = ZERO<T>;
    if (i < NB) {
#pragma unroll
      for (int k = 0; k < Ind<L>::K; ++k) s += h[k][i < NB ? i : 0];
    }
    db[i] = s;
  }
  if constexpr (NB == 3) {
    lam[0] = (h[3][2] - h[4][2]) - (h[5][1] - h[6][1]);
    lam[1] = (h[5][0] - h[6][0]) - (h[1][2] - h[2][2]);
    lam[2] = (h[1][1] - h[2][1]) - (h[3][0] - h[4][0]);
  } else {
    lam[0] = T(0);
    lam[1] = T(0);
    lam[2] = (h[1][1] - h[2][1]) - (h[3][0] - h[4][0]);
  }
}

// ---------------------------------------------------------------------------
// the fused step
// ---------------------------------------------------------------------------
// Directions with e_x != 0, numbered in order (the x-shifted ones of odd steps).
template <class L>
__host__ __device__ constexpr int xshift_count() {
  int c = 0;
  for (int q = 0; q < L::Q; ++q) c += L::ex(q) != 0;
  return c;
}
template <class L>
__host__ __device__ constexpr int xshift_index(int q) {
  int c = 0;
  for (int p = 0; p < q; ++p) c += L::ex(p) != 0;
  return c;
}

// Shear stress sigma = 2 rho nu S (Eq. 8) and strain rate
// S = -3 / (2 tau dt c^2 rho) (Pi^neq [+ E]) (Eq. 9) of the node's pre-step
// state, in physical units, stored as FP32 [NC][N] (2D: xx, xy, yy; 3D: xx,
// yy, zz, xy, xz, yz).  m.pi holds Pi^neq / c^2 and tau the closure's.  The
// artefact term E / c^2 = tau rho [quad (ue_i A_j + ue_j A_i) - thC C (uF_i A_j
// + uF_j A_i)] (Eq. 9 with Theta of Eq. 4; the Stokes form has no ue A part).
template <class L, class T>
__device__ __forceinline__ void store_stress(const StepArgs& a, uint32_t n, const Macro<T>& m) {
  T Pn[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) Pn[c] = m.pi[c];
  if (a.st_artefact) {
    const int ci[6] = {0, 1, 2, 0, 0, 1}, cj[6] = {0, 1, 2, 1, 2, 2};
    const T quad = par<T>(a.p.quad, a.p.f.quad);
    const T thc = par<T>(a.p.thC, a.p.f.thC) * m.C;
    const T tr = m.tau * m.rho;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int i = ci[c], j = cj[c];
      Pn[c] += tr * (quad * (m.Ue[i] * m.A[j] + m.Ue[j] * m.A[i]) - thc * (m.UF[i] * m.A[j] + m.UF[j] * m.A[i]));
    }
  }
  // sigma = -c^2 (1 - 1 / (2 tau)) Pn, S = -(3 / (2 dt)) Pn / (tau rho)
  const T cs = -(T)a.st_c2 * (T(1) - T(0.5) * m.itau);
  const T cS = -(T)a.st_hdt * m.itau * m.irho;
  const int map2[3] = {0, 3, 1};
  const uint64_t N = a.geo.N;
#pragma unroll
  for (int c = 0; c < L::NC; ++c) {
    const T v = Pn[L::D == 2 ? map2[c] : c];
    if (a.sig) __builtin_nontemporal_store((float)(cs * v), a.sig + (c * N + n));
    if (a.strain) __builtin_nontemporal_store((float)(cS * v), a.strain + (c * N + n));
  }
}

// XS (odd steps, tiles of whole rows without boundary links, buffer
// addressing): the x-shifted directions go through LDS.  The tile loads the
// source row of such a direction at its own x (aligned, coalesced), and each
// node takes its element x + e_x(opp q) from LDS; outputs are placed in LDS at
// x + e_x(q) and the tile stores the destination row at its own x.  A tile
// holds whole rows and x wraps inside a row, so every slot it loads or stores
// still belongs to one of its own nodes.  Every thread of the tile takes this
// path (the choice is per tile), so the two barriers are reached uniformly.
// DG: diagnostics of the step, 0 none, 1 the momentum exchange of the wall
// links only, 2 that and the balance sums.  ST: the step also stores the
// stress and strain rate of the pre-step state.
// lds: the tile's shared buffer, for the x staging (XS) or, in tiles that a
// wall group meets, the wall-link sums of each thread (DG): swall[j][tid],
// j = slot NWALL + quantity, each thread adding only to its own column (no
// barrier; quantity-major, so that a wavefront's accesses are conflict-free).
template <class L, int P, int MHD, int PAR, int DG, bool MAC, bool BND, class AD, bool XS = false, bool ST = false,
          bool IB = false>
__device__ __forceinline__ void node_update(const StepArgs& a, uint32_t n, const AD& Af, const AD& Ag, const uint4& rec,
                                            typename Stor<P>::T (&bal)[NBAL], typename Stor<P>::T* lds,
                                            uint32_t bgrp, uint32_t x = 0,
                                            const typename Stor<P>::T* uwl = nullptr) {
  using S = Stor<P>;
  using T = typename S::T;
  // 16-bit formats at interior nodes work in the stored units
  constexpr bool RAW = (P == S_F16 || P == S_BF16) && !BND && MHD == 0 && !XS;
  const Geom& g = a.geo;
  const uint32_t mask = rec.x;
  T d[L::Q];
  constexpr int NS = xshift_count<L>();
  [[maybe_unused]] T (*xs_out)[NTHREADS] = nullptr;
  [[maybe_unused]] uint32_t rb = 0;
  if constexpr (XS) {
    static_assert(PAR == 1 && !BND && MHD == 0, "x staging is for odd steps of interior tiles");
    T (*xs_in)[NTHREADS] = (T(*)[NTHREADS])lds;
    xs_out = xs_in + NS;
    const uint32_t tid = threadIdx.x;
    rb = tid - x;  // first thread of this node's row in the tile
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const int qb = opp(q);
      if (L::ex(qb) == 0)
        d[q] = Af.template ld<L, P>(nullptr, qb, qb);
      else
        xs_in[xshift_index<L>(q)][tid] = Af.template ldx<L, P>(qb, qb);
    }
    __syncthreads();
    const uint32_t nx = g.nx;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const int dx = L::ex(opp(q));
      if (dx != 0) {
        const uint32_t xs = dx > 0 ? (x + 1 == nx ? 0 : x + 1) : (x == 0 ? nx - 1 : x - 1);
        d[q] = xs_in[xshift_index<L>(q)][rb + xs];
      }
      if (P == S_F16 || P == S_BF16) d[q] *= (T)a.p.inv_scale[q];
    }
  } else {
    read_f<L, P, PAR, BND, AD, !RAW>((const typename S::E*)a.f, Af, mask, a.p, d);
  }
  if constexpr (BND && IB) {
    // Links to walls that are not halfway with q < 1/2 (interpolated
    // bounce-back, see k_ibb): the previous step of this call left
    // 2q f_rel_a(x) + ladd in the returning slot; the value streamed in along
    // a, f_rel_a(x - e_a), completes it (x - e_a fluid).
    const uint32_t ix = a.ibb_in ? rec.w >> 12 : 0u;
    if (ix) {
      const double* qp = a.ibq + (uint64_t)(ix - 1) * L::Q;
#pragma unroll
      for (int q = 1; q < L::Q; ++q) {
        const int qb = opp(q);
        if (((mask >> q) & 1u) && !((mask >> qb) & 1u)) {
          const double qv = qp[q];
          if (qv < 0.5) d[qb] += (T)(1.0 - 2.0 * qv) * d[q];
        }
      }
    }
  }
  T Ax, Ay, Az;
  if (a.afield) {
    const T s = par<T>(a.p.afield_scale, a.p.f.afield_scale);
    Ax = (T)a.afield[n] * s;
    Ay = (T)a.afield[g.N + n] * s;
    Az = L::D == 3 ? (T)a.afield[2 * (uint64_t)g.N + n] * s : T(0);
  } else {
    Ax = par<T>(a.p.A[0], a.p.f.A[0]);
    Ay = par<T>(a.p.A[1], a.p.f.A[1]);
    Az = par<T>(a.p.A[2], a.p.f.A[2]);
  }
  T h[Ind<L>::K][Ind<L>::NB];
  T db[3] = {T(0), T(0), T(0)}, lam[3] = {T(0), T(0), T(0)};
  if (MHD) {
    read_g<L, P, PAR, BND>((const typename S::E*)a.g, Ag, mask, h);
    ind_moments<L, T>(h, db, lam);  // B - B0 = sum_k (g_k - W_k B0)
  }
  Macro<T> m;
  macro<L, T, MHD, ST, RAW>(d, a.p, Ax, Ay, Az, db, lam, m);
  if constexpr (ST) store_stress<L, T>(a, n, m);
  if (MAC) {
    // density and velocity of the pre-step state, for the adjoint
    T* mo = (T*)a.mac;
    mo[n] = m.rho;
    mo[g.N + n] = m.U[0];
    mo[2 * (uint64_t)g.N + n] = m.U[1];
    mo[3 * (uint64_t)g.N + n] = m.U[2];
  }
  if (DG == 2) {
    bal[0] += m.drho;
    bal[1] += m.rho * m.U[0];
    bal[2] += m.rho * m.U[1];
    bal[3] += m.rho * m.U[2];
    bal[4] += m.rho * m.A[0];
    bal[5] += m.rho * m.A[1];
    bal[6] += m.rho * m.A[2];
  }
  typename S::E* fo = (typename S::E*)a.f;
  // emit(q, v, vo): store the relaxed value v of direction q (vo: that of
  // its opposite, which the interpolated bounce-back needs)
  [[maybe_unused]] const uint32_t ixo = (BND && IB && a.ibb_out) ? rec.w >> 12 : 0u;
  auto emit = [&](int q, T v, [[maybe_unused]] T vo) __attribute__((always_inline)) {
    if (BND && q > 0 && ((mask >> q) & 1u)) {
      // halfway bounce-back link: the returning population is d_rel plus the
      // moving-wall term 6 w rho (e_opp . u_w) / c^2; the Eq. (25) momentum
      // exchange per link is proportional to e_q (2 d_rel + ladd) beyond the
      // constant rest-state part, which the host adds from link counts.
      const uint32_t gr = nibble(rec, q);
      const T ux = uwl[3 * gr], uy = uwl[3 * gr + 1], uz = uwl[3 * gr + 2];  // u_w / c, from LDS
      const T ladd = T(-6) * (T)L::w(q) * m.rho * edot<L>(q, ux, uy, uz);
      const T out = v;
      v = out + ladd;
      if (IB && ixo) {
        // wall at fraction qv of the link (steps before the last of a call;
        // the last one returns the halfway value and k_ibb interpolates,
        // with the wall-force sums, which are formed on that step only)
        const double qv = a.ibq[(uint64_t)(ixo - 1) * L::Q + q];
        if (qv < 0.5) {
          if (!((mask >> opp(q)) & 1u)) v = (T)(2.0 * qv) * out + ladd;
        } else if (qv > 0.5) {
          v = (out + (T)(2.0 * qv - 1.0) * vo + ladd) * (T)(0.5 / qv);
        }
      }
      if (DG) {
        const T cq = out + v;
        T* sw = lds + threadIdx.x;
#pragma unroll
        for (int s = 0; s < MAXBG; ++s) {
          if (((bgrp >> (4 * s)) & 15u) == gr) {
            sw[(s * NWALL + 0) * NTHREADS] += (T)L::ex(q) * cq;
            sw[(s * NWALL + 1) * NTHREADS] += (T)L::ey(q) * cq;
            sw[(s * NWALL + 2) * NTHREADS] += (T)L::ez(q) * cq;
            sw[(s * NWALL + 3) * NTHREADS] += ladd;
          }
        }
      }
    }
    if constexpr (XS) {
      T s = v;
      if (P == S_F16 || P == S_BF16) s *= (T)a.p.scale[q];
      if (L::ex(q) == 0) {
        Af.template st<L, P>(nullptr, q, q, s);
      } else {
        const uint32_t nx = g.nx;
        const uint32_t xd = L::ex(q) > 0 ? (x + 1 == nx ? 0 : x + 1) : (x == 0 ? nx - 1 : x - 1);
        xs_out[xshift_index<L>(q)][rb + xd] = s;
      }
    } else {
      write_f1<L, P, PAR, BND, AD, !RAW>(fo, Af, mask, a.p, q, v);
    }
  };
  // The relaxation hands over a direction q (odd) and its opposite q + 1
  // one after the other; at boundary nodes the first is held until the
  // second arrives, so that each wall link sees its opposite's value.
  [[maybe_unused]] T held = T(0);
  auto sink = [&](int q, T v) __attribute__((always_inline)) {
    if constexpr (BND && IB) {
      if (q & 1) {
        held = v;
        return;
      }
      if (q > 0) {
        emit(q - 1, held, v);
        emit(q, v, held);
        return;
      }
    }
    emit(q, v, v);
  };
  if constexpr (RAW)
    collide_raw<L, P>(d, m, a.p, sink);
  else
    collide<L, T, MHD, decltype(sink)&, P == S_F32>(d, m, db, a.p, sink);
  if constexpr (XS) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
      if (L::ex(q) != 0) Af.template stx<L, P>(q, q, xs_out[xshift_index<L>(q)][threadIdx.x]);
  }
  if (MHD) {
    collide_g<L, T>(h, m, db, a.p);
    if (BND) {
      // insulating walls: anti-bounce-back to B = B0 (zero deviation)
#pragma unroll
      for (int k = 1; k < Ind<L>::K; ++k)
        if ((mask >> k) & 1u) {
#pragma unroll
          for (int i = 0; i < Ind<L>::NB; ++i) h[k][i] = -h[k][i];
        }
    }
    write_g<L, P, PAR, BND>((typename S::E*)a.g, Ag, mask, h);
  }
}

// Tile of a workgroup on odd steps.  Workgroups are dealt to the eight XCDs
// in turn (workgroup b to XCD b mod 8), each with its own L2.  When a row
// spans k > 1 tiles, the odd step's x-shifted loads and stores at the tiles'
// ends share 128-byte lines with the neighbouring tile of the same row; the
// mapping gives the k tiles of a row to consecutive workgroups of one XCD, so
// that these lines meet in one L2 (even steps, without x-shifted accesses,
// keep the identity).  Groups of 8 k workgroups: j-th workgroup of a
// group -> row (j mod 8) of the group's 8 rows, piece j / 8; the remainder
// of the grid (fewer than 8 k tiles) keeps the identity.
constexpr uint32_t NXCD = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t ntiles, uint32_t nx) {
  const uint32_t k = (nx > NTHREADS && nx % NTHREADS == 0) ? nx / NTHREADS : 1u;
  if (k == 1u) return b;
  const uint32_t chunk = NXCD * k;
  const uint32_t c = b / chunk;
  if ((c + 1) * chunk > ntiles) return b;
  const uint32_t j = b - c * chunk;
  return c * chunk + (j % NXCD) * k + j / NXCD;
}

// RU: 0 generic addressing; 1 row-uniform pointers; 2 row-uniform pointers
// for rows with boundary links and buffer resources for the other rows
// (arrays below 4 GiB).
// IB: links to walls that are not halfway are interpolated inside the step
// (a.ibb_in, a.ibb_out); only the row-uniform buffer form without MHD or the
// density record has this variant, so the others keep their registers.
// PLD: interior rows read with plain (cached) loads (AddrBP) instead of
// non-temporal ones; instantiated for FP32 odd steps without diagnostics,
// chosen by the host for states far beyond the last-level cache.
template <class L, int P, int MHD, int PAR, int DG, int RU, bool MAC = false, bool ST = false, bool IB = false,
          bool PLD = false>
__global__ __launch_bounds__(NTHREADS) void k_step(const StepArgs a) {
  using T = typename Stor<P>::T;
  const Geom& g = a.geo;
  // tiles with boundary rows (slower) first, so that they do not form the
  // tail of the launch (the host's order, one per parity, the odd one
  // XCD-aware); else the XCD-aware order of odd steps
  const uint32_t tile = a.tperm ? a.tperm[(PAR == 1 ? gridDim.x : 0u) + blockIdx.x]
                                : (PAR == 1 ? xcd_tile(blockIdx.x, gridDim.x, g.nx) : blockIdx.x);
  const uint32_t n = tile * NTHREADS + threadIdx.x;
  const bool active = n < g.N;
  T bal[NBAL];
  if (DG == 2) {
#pragma unroll
    for (int k = 0; k < NBAL; ++k) bal[k] = T(0);
  }
  // LDS x-staging on odd steps: FP32 (odd step -5 %) and FP64 (odd step
  // -7 %, 40 KB of LDS per tile); the 2-byte formats and the diagnostic
  // variant (register pressure) measured slower with it
  constexpr bool XS_OK = RU == 2 && MHD == 0 && PAR == 1 && !MAC && DG != 2 && (P == S_F32 || P == S_F64);
  const uint32_t bgrp = a.blkgrp[tile];
  // one shared buffer: the x staging of interior tiles, or the per-thread
  // wall-link sums of tiles that a wall group meets (never both in a tile)
  constexpr int NXS = xshift_count<L>();
  constexpr uint32_t LDS_XS = XS_OK ? 2 * NXS * NTHREADS : 0;
  constexpr uint32_t LDS_W = DG ? MAXBG * NWALL * NTHREADS : 0;
  constexpr uint32_t LDS_N = LDS_XS > LDS_W ? LDS_XS : (LDS_W > 0 ? LDS_W : 1);
  __shared__ T lds[LDS_N];
  if (DG && (bgrp >> 28)) {
#pragma unroll
    for (int j = 0; j < MAXBG * NWALL; ++j) lds[j * NTHREADS + threadIdx.x] = T(0);
  }
  // Tiles that a wall group meets (uniform per tile) put the wall velocities
  // in LDS: each wall link reads its group's velocity behind its own branch,
  // and from memory those reads would wait one link after the other.
  __shared__ T suw[3 * MAXG];
  if (bgrp >> 28) {
    if (threadIdx.x < 3 * MAXG) suw[threadIdx.x] = (T)a.uw[threadIdx.x];
    __syncthreads();
  }
  if (active) {
    uint32_t x, y, z, r;
    coords(g, n, x, y, z, r);
    if (RU) {
      // every lane of the wavefront is in the same row
      r = __builtin_amdgcn_readfirstlane(r);
      y = __builtin_amdgcn_readfirstlane(y);
      z = __builtin_amdgcn_readfirstlane(z);
    }
    const int rr = a.rowrec[r];
    const uint4 rec = rr < 0 ? make_uint4(0u, 0u, 0u, 0u) : a.rec[rr + x];
    if (!(rec.x >> 31)) {
      if (RU == 2 && rr < 0) {
        using E = typename Stor<P>::E;
        constexpr uint32_t GP = MHD ? Ind<L>::K * Ind<L>::NB : L::Q;
        using AFT = std::conditional_t<PLD, AddrBP, AddrB>;
        AFT Af;
        static_cast<AddrB&>(Af) = addr_b<E>(g, x, y, z, L::Q, a.f, (uint32_t)((uint64_t)g.N * L::Q * sizeof(E)));
        AFT Ag = Af;
        if constexpr (MHD != 0)
          static_cast<AddrB&>(Ag) = addr_b<E>(g, x, y, z, GP, a.g, (uint32_t)((uint64_t)g.N * GP * sizeof(E)));
        if constexpr (XS_OK) {
          if ((bgrp >> 27) & 1u) {
            // tile of whole rows without boundary links (uniform per tile)
            node_update<L, P, MHD, PAR, DG, MAC, false, AFT, true, ST>(a, n, Af, Ag, rec, bal, lds, bgrp, x);
          } else {
            node_update<L, P, MHD, PAR, DG, MAC, false, decltype(Af), false, ST>(a, n, Af, Ag, rec, bal, lds, bgrp);
          }
        } else {
          node_update<L, P, MHD, PAR, DG, MAC, false, decltype(Af), false, ST>(a, n, Af, Ag, rec, bal, lds, bgrp);
        }
      } else if (RU) {
        const AddrR Af = addr_r(g, x, y, z, L::Q);
        const AddrR Ag = addr_r(g, x, y, z, MHD ? Ind<L>::K * Ind<L>::NB : L::Q);
        if (rr < 0)
          node_update<L, P, MHD, PAR, DG, MAC, false, decltype(Af), false, ST>(a, n, Af, Ag, rec, bal, lds, bgrp);
        else
          node_update<L, P, MHD, PAR, DG, MAC, true, decltype(Af), false, ST, IB>(a, n, Af, Ag, rec, bal, lds, bgrp, 0u,
                                                                                 suw);
      } else {
        const AddrG Af = addr_g(g, x, y, z, r, L::Q);
        const AddrG Ag = addr_g(g, x, y, z, r, MHD ? Ind<L>::K * Ind<L>::NB : L::Q);
        if (rr < 0)
          node_update<L, P, MHD, PAR, DG, MAC, false, decltype(Af), false, ST>(a, n, Af, Ag, rec, bal, lds, bgrp);
        else
          node_update<L, P, MHD, PAR, DG, MAC, true, decltype(Af), false, ST>(a, n, Af, Ag, rec, bal, lds, bgrp, 0u, suw);
      }
    }
  }
  if (DG == 1 && (bgrp >> 28)) {
    // wall-link sums of this tile into the step's slot of the per-step ring
    // (compact tile index, quantity-major)
    double v[MAXBG * NWALL];
#pragma unroll
    for (int j = 0; j < MAXBG * NWALL; ++j) v[j] = (double)lds[j * NTHREADS + threadIdx.x];
    tile_sum_store<MAXBG * NWALL>(v, a.hist + a.wtile[tile], a.nwt);
  }
  if (DG == 2) {
    if (bgrp >> 28) {
      double v[NPART];
#pragma unroll
      for (int k = 0; k < NBAL; ++k) v[k] = (double)bal[k];
#pragma unroll
      for (int j = 0; j < MAXBG * NWALL; ++j) v[NBAL + j] = (double)lds[j * NTHREADS + threadIdx.x];
      tile_sum_store<NPART>(v, a.part + tile, gridDim.x);
    } else {
      // no wall group meets this tile (uniform per tile): its wall slots are
      // never read, only the balance sums are formed
      double v[NBAL];
#pragma unroll
      for (int k = 0; k < NBAL; ++k) v[k] = (double)bal[k];
      tile_sum_store<NBAL>(v, a.part + tile, gridDim.x);
    }
  }
}

// Magnetic part of the rest equilibrium in the uniform field b0 (Eq. 10; in
// two dimensions without -b^2 / 6); zero unless the equilibrium carries it.
template <class L, int MHD>
__device__ __forceinline__ double mhd_phi0(int q, const Phys& p) {
  if (MHD != 1) return 0.0;
  const double* b0 = p.b0;
  const double eb = edot<L>(q, b0[0], b0[1], b0[2]);
  const double b2 = b0[0] * b0[0] + b0[1] * b0[1] + b0[2] * b0[2];
  return 4.5 * L::w(q) * (0.5 * b2 * L::e2(q) - eb * eb - (L::D == 3 ? b2 / 6.0 : 0.0));
}

// ---------------------------------------------------------------------------
// diagnostics of the current state (read only)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool node_solid(const DiagArgs& a, uint32_t n) {
  uint32_t x, y, z, r;
  coords(a.geo, n, x, y, z, r);
  const int rr = a.rowrec[r];
  return rr >= 0 && (a.rec[rr + x].x >> 31);
}

// All diagnostic arithmetic is FP64, applied to the stored values.
template <class L, int P, int MHD, int PAR>
__global__ __launch_bounds__(NTHREADS) void k_diag(const DiagArgs a) {
  using S = Stor<P>;
  using T = double;
  using TS = typename S::T;
  const Geom& g = a.geo;
  const uint32_t n = blockIdx.x * NTHREADS + threadIdx.x;
  double part[NDIAGPART] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (n < g.N) {
    uint32_t x, y, z, r;
    coords(g, n, x, y, z, r);
    const AddrG Af = addr_g(g, x, y, z, r, L::Q);
    const AddrG Ag = addr_g(g, x, y, z, r, Ind<L>::K * Ind<L>::NB);
    const Offs on = offsets(g, x, y, z, (uint64_t)g.nx);  // node-index offsets
    const int rr = a.rowrec[r];
    const uint4 rec = rr >= 0 ? a.rec[rr + x] : make_uint4(0u, 0u, 0u, 0u);
    const bool solid = rec.x >> 31;
    T d[L::Q] = {};
    T h[Ind<L>::K][Ind<L>::NB] = {};
    T b[3] = {T(0), T(0), T(0)};
    T db[3] = {T(0), T(0), T(0)}, lam[3] = {T(0), T(0), T(0)};
    Macro<T> m = {};
    if (!solid) {
      TS ds[L::Q];
      read_f<L, P, PAR, true>((const typename S::E*)a.f, Af, rec.x, a.p, ds);
#pragma unroll
      for (int q = 0; q < L::Q; ++q) d[q] = (T)ds[q];
      T Ax, Ay, Az;
      if (a.afield) {
        const T s = par<T>(a.p.afield_scale, a.p.f.afield_scale);
        Ax = (T)a.afield[n] * s;
        Ay = (T)a.afield[g.N + n] * s;
        Az = L::D == 3 ? (T)a.afield[2 * (uint64_t)g.N + n] * s : T(0);
      } else {
        Ax = par<T>(a.p.A[0], a.p.f.A[0]);
        Ay = par<T>(a.p.A[1], a.p.f.A[1]);
        Az = par<T>(a.p.A[2], a.p.f.A[2]);
      }
      if (MHD) {
        TS hs[Ind<L>::K][Ind<L>::NB];
        read_g<L, P, PAR, true>((const typename S::E*)a.g, Ag, rec.x, hs);
#pragma unroll
        for (int k = 0; k < Ind<L>::K; ++k)
#pragma unroll
          for (int i = 0; i < Ind<L>::NB; ++i) h[k][i] = (T)hs[k][i];
        ind_moments<L, T>(h, db, lam);
      }
      macro<L, T, MHD, true>(d, a.p, Ax, Ay, Az, db, lam, m);
#pragma unroll
      for (int i = 0; i < 3; ++i) b[i] = m.b[i];
    }
    if (a.state) {
#pragma unroll
      for (int q = 0; q < L::Q; ++q) {
        double v = (double)d[q];
        v += mhd_phi0<L, MHD>(q, a.p);  // back to f - w rho0
        a.state[(uint64_t)q * g.N + n] = solid ? 0.0 : v;
      }
    }
    if (a.gstate) {
      // absolute g in units of B (the host rescales by c sqrt(mu))
#pragma unroll
      for (int k = 0; k < Ind<L>::K; ++k)
#pragma unroll
        for (int i = 0; i < Ind<L>::NB; ++i)
          a.gstate[(uint64_t)(Ind<L>::NB * k + i) * g.N + n] =
              solid ? 0.0 : (double)h[k][i] + Ind<L>::w(k) * a.p.b0[i];
    }
    if (a.rho) a.rho[n] = solid ? 0.0 : (double)m.rho;
    if (a.vel) {
#pragma unroll
      for (int k = 0; k < L::D; ++k) a.vel[(uint64_t)k * g.N + n] = solid ? 0.0 : (double)m.V[k] * a.c;
    }
    if (a.B) {
#pragma unroll
      for (int k = 0; k < 3; ++k) a.B[(uint64_t)k * g.N + n] = solid ? 0.0 : (double)b[k];
    }
    // stress and strain rate, Eqs. (8)-(9)
    double sig[6] = {0, 0, 0, 0, 0, 0}, str[6] = {0, 0, 0, 0, 0, 0};
    if (!solid) {
      T Pn[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) Pn[c] = m.pi[c];
      if (a.artefact) {
        // E / c^2 = tau rho [(Ue_i A_j + Ue_j A_i) - C (UF_i A_j + UF_j A_i)] (Eq. 9 with Eq. 4)
        const int ci[6] = {0, 1, 2, 0, 0, 1}, cj[6] = {0, 1, 2, 1, 2, 2};
        const T thc = par<T>(a.p.thC, a.p.f.thC) * m.C;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const int i = ci[c], j = cj[c];
          // (no u^eq a part with the Stokes equilibrium, whose M^eq has no rho u u)
          Pn[c] += m.tau * m.rho *
                   (par<T>(a.p.quad, a.p.f.quad) * (m.Ue[i] * m.A[j] + m.Ue[j] * m.A[i]) - thc * (m.UF[i] * m.A[j] + m.UF[j] * m.A[i]));
        }
      }
      const double cS = -3.0 / (2.0 * (double)m.tau * a.dt * (double)m.rho);
      const double cs = -(1.0 - 0.5 / (double)m.tau) * a.c * a.c;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        str[c] = cS * (double)Pn[c];
        sig[c] = cs * (double)Pn[c];
      }
    }
    // output order: 2D xx, xy, yy; 3D xx, yy, zz, xy, xz, yz
    const int map2[3] = {0, 3, 1};
#pragma unroll
    for (int c = 0; c < L::NC; ++c) {
      const int src = L::D == 2 ? map2[c] : c;
      if (a.sigma) a.sigma[(uint64_t)c * g.N + n] = sig[src];
      if (a.strain) a.strain[(uint64_t)c * g.N + n] = str[src];
    }
    if (a.part && !solid) {
      part[0] = (double)m.drho;
      part[1] = (double)(m.rho * m.U[0]);
      part[2] = (double)(m.rho * m.U[1]);
      part[3] = (double)(m.rho * m.U[2]);
      // plane-wall stress integral: weights 3/2 (first layer) and -1/2
      // (second layer) extrapolate (-p I + sigma) n to the halfway wall
      const uint32_t pos[3] = {x, y, z};
      const uint32_t ext[3] = {g.nx, g.ny, g.nz};
      const int64_t ax_off_p[3] = {on.xp, on.yp, on.zp}, ax_off_m[3] = {on.xm, on.ym, on.zm};
      const double p_iso = (double)m.rho * a.c * a.c / 3.0;
      double T3[3][3];
      const int fi[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) T3[i][j] = (i < L::D && j < L::D) ? sig[fi[i][j]] - (i == j ? p_iso : 0.0) : 0.0;
      for (int ax = 0; ax < L::D; ++ax) {
        if (ext[ax] < 2) continue;
        for (int side = 0; side < 2; ++side) {
          if (!(side == 0 ? a.wall_lo[ax] : a.wall_hi[ax])) continue;
          const uint32_t l0 = side == 0 ? 0u : ext[ax] - 1, l1 = side == 0 ? 1u : ext[ax] - 2;
          double wgt = 0.0;
          uint32_t partner = n;  // node index of the other extrapolation layer
          if (pos[ax] == l0) {
            wgt = 1.5;
            partner = (uint32_t)((int64_t)n + (side == 0 ? ax_off_p[ax] : ax_off_m[ax]));
          } else if (pos[ax] == l1) {
            wgt = -0.5;
            partner = (uint32_t)((int64_t)n + (side == 0 ? ax_off_m[ax] : ax_off_p[ax]));
          }
          if (wgt == 0.0 || node_solid(a, partner)) continue;
          const double nrm = side == 0 ? 1.0 : -1.0;
#pragma unroll
          for (int i = 0; i < 3; ++i) part[4 + i] += wgt * a.area * T3[i][ax] * nrm;
        }
      }
    }
  }
  if (a.part) tile_sum_store<NDIAGPART>(part, a.part + blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// initial state / upload
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// interpolated bounce-back (walls that are not halfway between nodes)
// ---------------------------------------------------------------------------
// The linear interpolation of Bouzidi, Firdaouss and Lallemand (2001) for a
// wall at fraction q of the link a returns into x, as direction opp(a):
//   q <  1/2: 2q f_rel_a(x) + (1 - 2q) f_rel_a(x - e_a) + ladd
//             (f_rel_a(x - e_a) is the value that streamed into x along a;
//             halfway when x - e_a is not a fluid node),
//   q >= 1/2: [f_rel_a(x) + (2q - 1) f_rel_opp(a)(x) + ladd] / (2q).
// The steps before the last of a call do this themselves: the q >= 1/2 form
// at once (both values are the node's own), the q < 1/2 form in two parts,
// 2q f_rel_a(x) + ladd in the step and the streamed part when the next step
// reads the node.  The last step of a call returns the halfway value
// f_rel_a(x) + ladd into the node's own slot for direction opp(a), and this
// pass, run after it on the nodes with such links, replaces it with the
// interpolated value and forms the changes the wall force needs.
// f_rel(x, t) is read back as for the half-step distribution; the moving-wall
// term ladd = -6 w rho(x, t) e_a.u_w needs rho(x, t), recovered by mass
// conservation of the relaxation.  One thread per node: every slot it reads
// belongs to links of its own node or to regular streamed values that no
// other thread of this pass writes.
// One wavefront per block: the list is short (boundary nodes only) and its
// gathers are scattered, so spreading it over as many compute units as
// possible is what shortens the pass.  The pass is bound by the latency of
// its chains of dependent loads, so it keeps them short: the list carries
// each node's boundary record (no lookup through the row table), and the
// wall velocities, indexed by each link's group, are read from LDS (a load
// per wall link, each behind its own branch, would otherwise wait for memory
// one link after the other).
constexpr int IBB_THREADS = 64;
static_assert(IBB_THREADS >= 3 * MAXG, "one thread per wall-velocity component");

template <class L, int P, int PAR>
__global__ __launch_bounds__(IBB_THREADS) void k_ibb(const IbbArgs a) {
  using S = Stor<P>;
  using E = typename S::E;
  using TS = typename S::T;
  const Geom& g = a.geo;
  __shared__ double suw[MAXG][3];
  if (threadIdx.x < 3 * MAXG) (&suw[0][0])[threadIdx.x] = (&a.uw[0][0])[threadIdx.x];
  __syncthreads();
  const uint32_t i = blockIdx.x * IBB_THREADS + threadIdx.x;
  if (i >= a.M) return;
  // every read comes before the first store (the stores could alias the
  // other arrays as far as the compiler knows, which would serialise them)
  double qv[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) qv[q] = a.qf[(uint64_t)i * L::Q + q];
  const uint32_t n = a.node[i];
  const uint4 rec = a.nrec[i];
  uint32_t x, y, z, r;
  coords(g, n, x, y, z, r);
  const AddrG Af = addr_g(g, x, y, z, r, L::Q);
  const uint32_t mask = rec.x;
  E* f = (E*)a.f;
  TS d1[L::Q];
  read_f<L, P, PAR, true>(f, Af, mask, a.p, d1);  // incoming values f(x, t + dt)
  double V[L::Q];
  double sV = 0.0, K = 0.0;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const bool wall = q > 0 && ((mask >> q) & 1u);
    const E* ptr = (PAR == 1 || wall) ? Af.template ptr<L>((const E*)f, opp(q), -1) : Af.template ptr<L>((const E*)f, q, q);
    double v = (double)S::ld(ptr);
    if (P == S_F16 || P == S_BF16) v *= (double)a.p.inv_scale[q];
    V[q] = v;
    sV += v;
    if (wall) {
      const uint32_t gr = nibble(rec, q);
      K += 6.0 * L::w(q) * edot<L>(q, suw[gr][0], suw[gr][1], suw[gr][2]);
    }
  }
  const double rho_t = (a.p.rho0 + sV) / (1.0 - K);
  // f_rel(x, t) of each direction (the moving-wall term removed again)
  double R[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    R[q] = V[q];
    if (q > 0 && ((mask >> q) & 1u)) {
      const uint32_t gr = nibble(rec, q);
      R[q] += 6.0 * L::w(q) * rho_t * edot<L>(q, suw[gr][0], suw[gr][1], suw[gr][2]);
    }
  }
  double dnew[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    dnew[q] = V[q];  // halfway value as the step returned it
    if (q == 0 || !((mask >> q) & 1u) || qv[q] == 0.5) continue;
    const int qb = opp(q);
    const uint32_t gr = nibble(rec, q);
    const double ladd = -6.0 * L::w(q) * rho_t * edot<L>(q, suw[gr][0], suw[gr][1], suw[gr][2]);
    if (qv[q] < 0.5) {
      if (!((mask >> qb) & 1u)) dnew[q] = 2.0 * qv[q] * R[q] + (1.0 - 2.0 * qv[q]) * (double)d1[q] + ladd;
    } else {
      dnew[q] = (R[q] + (2.0 * qv[q] - 1.0) * R[qb] + ladd) / (2.0 * qv[q]);
    }
  }
#pragma unroll
  for (int q = 1; q < L::Q; ++q) {
    if (!((mask >> q) & 1u)) continue;
    if (qv[q] != 0.5) {
      double sv = dnew[q];
      if (P == S_F16 || P == S_BF16) sv *= (double)a.p.scale[q];
      S::st(Af.template ptr<L>(f, opp(q), -1), (TS)sv);
    }
    if (a.delta) a.delta[(uint64_t)i * L::Q + q] = dnew[q] - V[q];
  }
  if (a.half) {
#pragma unroll
    for (int q = 0; q < L::Q; ++q) a.half[(uint64_t)i * L::Q + q] = V[q];
  }
}

// Wall-force corrections of the interpolated links: per block of 256 list
// entries (node, direction) the sums of e_k delta (k < 3) and delta (k = 3)
// of each group g < G into part[block][4 g + k]; k_colsum then adds the
// blocks' rows.  Both deterministic.
template <class L>
__global__ __launch_bounds__(NTHREADS) void k_ibb_part(const double* __restrict__ delta, const uint8_t* __restrict__ grp,
                                                       uint64_t entries, int G, double* __restrict__ part) {
  const uint64_t e = (uint64_t)blockIdx.x * NTHREADS + threadIdx.x;
  const int q = (int)(e % L::Q);
  const bool live = e < entries && q > 0;
  const uint32_t ge = live ? grp[e] : 0xFFu;
  const double dv = (live && ge != 0xFFu) ? delta[e] : 0.0;
  for (int gr = 0; gr < G; ++gr) {
    const double s = ge == (uint32_t)gr ? dv : 0.0;
    double v[4] = {L::ex(q) * s, L::ey(q) * s, L::ez(q) * s, s};
    tile_sum_store<4>(v, part + ((uint64_t)blockIdx.x * G + gr) * 4);
  }
}

__global__ __launch_bounds__(NTHREADS) void k_colsum(const double* __restrict__ part, uint32_t rows, uint32_t cols,
                                                     double* __restrict__ out) {
  const uint32_t c = blockIdx.x;
  double s = 0.0;
  for (uint32_t r = threadIdx.x; r < rows; r += NTHREADS) s += part[(uint64_t)r * cols + c];
  double v[1] = {s};
  tile_sum_store<1>(v, out + c);
}

// ---------------------------------------------------------------------------
// half-step distribution of the last step (Section 5, Eqs. 27-28)
// ---------------------------------------------------------------------------
// f_bar = (f_rel(x, t) + f(x, t + dt)) / 2.  f(t + dt) is the current state.
// f_rel(x, t) is read back from where the last step put it: in a node's own
// opposite slot after an even step (next parity odd), at the neighbour
// x + e after an odd step; a bounce-back link's value came back to the node
// with the moving-wall term added, which is removed again.  That term needs
// rho(x, t), recovered from mass conservation of the relaxation:
// rho = rho0 + sum_a f_rel_a = rho0 + sum_a V_a + rho K, with V the values as
// read and K = sum over wall links of 6 w (e.u_w).  Induction distributions
// likewise (anti-bounce-back: the stored value is the negated relaxed one).
// At a node with links to walls that are not halfway, the interpolation
// replaced the halfway values of the last step in the node's own slots; the
// pass after that step kept them (ibb_half), and they stand in for the slots'
// contents here, so that f_rel(x, t) and rho(x, t) come back the same way.
template <class L, int P, int MHD, int PAR>
__global__ __launch_bounds__(NTHREADS) void k_half(const HalfArgs a) {
  using S = Stor<P>;
  using E = typename S::E;
  using TS = typename S::T;
  const Geom& g = a.geo;
  // wall velocities by group, read per wall link from LDS
  __shared__ double suw[MAXG][3];
  if (threadIdx.x < 3 * MAXG) (&suw[0][0])[threadIdx.x] = (&a.uw[0][0])[threadIdx.x];
  __syncthreads();
  const uint32_t n = blockIdx.x * NTHREADS + threadIdx.x;
  if (n >= g.N) return;
  uint32_t x, y, z, r;
  coords(g, n, x, y, z, r);
  const AddrG Af = addr_g(g, x, y, z, r, L::Q);
  const AddrG Ag = addr_g(g, x, y, z, r, Ind<L>::K * Ind<L>::NB);
  const int rr = a.rowrec[r];
  const uint4 rec = rr >= 0 ? a.rec[rr + x] : make_uint4(0u, 0u, 0u, 0u);
  const uint32_t mask = rec.x;
  const bool solid = mask >> 31;
  double db[L::Q];
  double Bh[3] = {0.0, 0.0, 0.0};  // (B(t) + B(t + dt)) / 2 - B0
  if (!solid) {
    TS d1[L::Q];
    read_f<L, P, PAR, true>((const E*)a.f, Af, mask, a.p, d1);
    double V[L::Q];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const bool wall = q > 0 && ((mask >> q) & 1u);
      const E* ptr = (PAR == 1 || wall) ? Af.template ptr<L>((const E*)a.f, opp(q), -1)
                                        : Af.template ptr<L>((const E*)a.f, q, q);
      double v = (double)S::ld(ptr);
      if (P == S_F16 || P == S_BF16) v *= (double)a.p.inv_scale[q];
      V[q] = v;
    }
    // nodes with interpolated links: their wall slots' halfway values, as
    // the last step returned them (after the loads above, so that those are
    // not held behind a per-direction branch)
    const uint32_t ix = a.ibb_half ? rec.w >> 12 : 0u;
    if (ix) {
#pragma unroll
      for (int q = 1; q < L::Q; ++q)
        if ((mask >> q) & 1u) V[q] = a.ibb_half[(uint64_t)(ix - 1) * L::Q + q];
    }
    double sV = 0.0, K = 0.0;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      const bool wall = q > 0 && ((mask >> q) & 1u);
      sV += V[q];
      if (wall) {
        const uint32_t gr = nibble(rec, q);
        K += 6.0 * L::w(q) * edot<L>(q, suw[gr][0], suw[gr][1], suw[gr][2]);
      }
    }
    const double rho_t = (a.p.rho0 + sV) / (1.0 - K);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      double rel = V[q];
      if (q > 0 && ((mask >> q) & 1u)) {
        const uint32_t gr = nibble(rec, q);
        rel += 6.0 * L::w(q) * rho_t * edot<L>(q, suw[gr][0], suw[gr][1], suw[gr][2]);
      }
      db[q] = 0.5 * (rel + (double)d1[q]);
    }
    if (MHD) {
      constexpr int NB = Ind<L>::NB;
      TS h1[Ind<L>::K][NB];
      read_g<L, P, PAR, true>((const E*)a.g, Ag, mask, h1);
#pragma unroll
      for (int k = 0; k < Ind<L>::K; ++k) {
        const bool wall = k > 0 && ((mask >> k) & 1u);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const E* ptr = (PAR == 1 || wall) ? Ag.template ptr<L>((const E*)a.g, NB * opp(k) + i, -1)
                                            : Ag.template ptr<L>((const E*)a.g, NB * k + i, k);
          double hr = (double)S::ld(ptr);
          if (wall) hr = -hr;
          Bh[i] += 0.5 * (hr + (double)h1[k][i]);
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < L::Q; ++q) db[q] = 0.0;
  }
  if (a.fbar) {
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
      double v = db[q];
      if (!solid) v += mhd_phi0<L, MHD>(q, a.p);  // back to f - w rho0
      a.fbar[(uint64_t)q * g.N + n] = v;
    }
  }
  double srho = 0.0, j[3] = {0.0, 0.0, 0.0};
  double m2[6] = {0, 0, 0, 0, 0, 0};  // sum e e d_bar: xx, yy, zz, xy, xz, yz
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const double v = db[q];
    const int ex = L::ex(q), ey = L::ey(q), ez = L::ez(q);
    srho += v;
    j[0] += ex * v;
    j[1] += ey * v;
    j[2] += ez * v;
    m2[0] += ex * ex * v;
    m2[1] += ey * ey * v;
    m2[2] += ez * ez * v;
    m2[3] += ex * ey * v;
    m2[4] += ex * ez * v;
    m2[5] += ey * ez * v;
  }
  const double rho = a.p.rho0 + srho;
  const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  if (a.rho) a.rho[n] = solid ? 0.0 : rho;
  if (a.vel) {
#pragma unroll
    for (int k = 0; k < L::D; ++k) a.vel[(uint64_t)k * g.N + n] = solid ? 0.0 : u[k] * a.c;
  }
  if (a.sigma) {
    // -sum e e f_bar + p_bar delta + rho_bar u u (+ L(B_bar) when the
    // equilibrium carries it); the stored deviations exclude w rho0 (and then
    // phi(B0), whose second moment is L(B0))
    const int ci[6] = {0, 1, 2, 0, 0, 1}, cj[6] = {0, 1, 2, 1, 2, 2};
    double sg[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int i = ci[c], k = cj[c];
      double v = -m2[c] + (i == k ? srho / 3.0 : 0.0) + a.p.quad * rho * u[i] * u[k];
      if (MHD == 1) {
        // L(b) - L(b0) with b = b0 + Bh, L_ij = b^2 delta_ij / 2 - b_i b_j
        const double* b0 = a.p.b0;
        const double bs[3] = {2.0 * b0[0] + Bh[0], 2.0 * b0[1] + Bh[1], 2.0 * b0[2] + Bh[2]};  // b + b0
        const double b2h = 0.5 * (Bh[0] * bs[0] + Bh[1] * bs[1] + Bh[2] * bs[2]);
        v += (i == k ? b2h : 0.0) - 0.5 * (Bh[i] * bs[k] + bs[i] * Bh[k]);
      }
      sg[c] = solid ? 0.0 : v * a.c * a.c;
    }
    const int map2[3] = {0, 3, 1};
#pragma unroll
    for (int c = 0; c < L::NC; ++c) a.sigma[(uint64_t)c * g.N + n] = sg[L::D == 2 ? map2[c] : c];
  }
}

template <class L, int P, int MHD>
__global__ __launch_bounds__(NTHREADS) void k_init(const InitArgs a) {
  using S = Stor<P>;
  using T = typename S::T;
  const Geom& g = a.geo;
  const uint32_t n = blockIdx.x * NTHREADS + threadIdx.x;
  if (n >= g.N) return;
  uint32_t x, y, z, r;
  coords(g, n, x, y, z, r);
  const int rr = a.rowrec[r];
  const bool solid = rr >= 0 && (a.rec[rr + x].x >> 31);
  typename S::E* f = (typename S::E*)a.f;
  double U[3] = {0, 0, 0};
  if (a.u0 && !solid)
    for (int k = 0; k < L::D; ++k) U[k] = a.u0[(uint64_t)k * g.N + n] * a.inv_c;
  const double* b0 = a.p.b0;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    double v = 0.0;
    if (!solid) {
      if (a.state) {
        v = a.state[(uint64_t)q * g.N + n];
        v -= mhd_phi0<L, MHD>(q, a.p);  // stored relative to the rest equilibrium in B0
      } else {
        // f^eq(rho0, u0) (+ phi(B0), which the stored deviation excludes)
        const double w = L::w(q);
        const double eu = edot<L>(q, U[0], U[1], U[2]);
        const double usq = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
        v = w * a.p.rho0 * (3.0 * eu + a.p.quad * (4.5 * eu * eu - 1.5 * usq));
      }
    }
    T s = (T)v;
    if (P == S_F16 || P == S_BF16) s = (T)(v * (double)a.p.scale[q]);
    S::st(f + ((uint64_t)r * (L::Q * g.nx) + x) + q * g.nx, s);
  }
  if (MHD) {
    using I = Ind<L>;
    typename S::E* gg = (typename S::E*)a.g;
    for (int k = 0; k < I::K; ++k) {
      const int ax = (k - 1) >> 1;
      const double sgn = (k & 1) ? 1.0 : -1.0;
      for (int i = 0; i < I::NB; ++i) {
        double hv = 0.0;
        if (!solid && k > 0) hv = I::w(k) * sgn * (1.0 / I::theta) * (U[ax] * b0[i] - b0[ax] * U[i]);
        S::st(gg + ((uint64_t)r * (I::K * I::NB * g.nx) + x) + (I::NB * k + i) * g.nx, (T)hv);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// deterministic reductions of per-tile partial sums
// ---------------------------------------------------------------------------
// mode 0: step partials [NPART][ntiles] -> out[NBAL + MAXG * NWALL]
// mode 1: diagnostic partials [NDIAGPART][ntiles] -> out[NDIAGPART]
// (partials are quantity-major, so that a block's loads are coalesced; fixed
// order, deterministic).  The reduction is bound by the latency of its
// loads, so each thread keeps 8 or 16 independent loads in flight, and a wall
// group's sums visit only the tiles it meets: wlist holds, per group g, the
// entries wlist[wlist[g]] .. wlist[wlist[g + 1] - 1], each a tile index
// (bits 0-27) and the group's slot in that tile (bits 28-31), in tile order.
__global__ __launch_bounds__(NTHREADS) void k_reduce(const double* __restrict__ part, const uint32_t* __restrict__ wlist,
                                                     uint32_t ntiles, int mode, int G, double* __restrict__ out) {
  const int o = blockIdx.x;
  if (mode == 0 && o >= NBAL && (o - NBAL) / NWALL >= G) {
    // a group that is not in use (uniform per block)
    if (threadIdx.x == 0) out[o] = 0.0;
    return;
  }
  double acc[16] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (mode == 1 || o < NBAL) {
    // a whole row: sixteen loads in flight per thread
    const double* row = part + (uint64_t)o * ntiles;
    uint32_t t = threadIdx.x;
    for (; t + 15 * NTHREADS < ntiles; t += 16 * NTHREADS) {
      double v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = row[t + j * NTHREADS];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] += v[j];
    }
    for (; t < ntiles; t += NTHREADS) acc[0] += row[t];
  } else {
    const uint32_t grp = (o - NBAL) / NWALL, k = (o - NBAL) % NWALL;
    const uint32_t b = wlist[grp], e = wlist[grp + 1];
    uint32_t i = b + threadIdx.x;
    for (; i + 7 * NTHREADS < e; i += 8 * NTHREADS) {
      uint32_t en[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) en[j] = wlist[i + j * NTHREADS];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        acc[j] += part[(uint64_t)(NBAL + (en[j] >> 28) * NWALL + k) * ntiles + (en[j] & 0x0FFFFFFFu)];
    }
    for (; i < e; i += NTHREADS) {
      const uint32_t en = wlist[i];
      acc[0] += part[(uint64_t)(NBAL + (en >> 28) * NWALL + k) * ntiles + (en & 0x0FFFFFFFu)];
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] += acc[j + 8];
  const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  double v[1] = {s};
  tile_sum_store<1>(v, out + o);
}

// Per-step wall-force record: ring [steps][MAXBG NWALL][nwt] of compact-tile
// partial sums (nwt tiles that a wall group meets) -> out[step][MAXG NWALL]
// (group-major, the layout of the step record's wall part).  Block (step s,
// quantity o = g NWALL + k) sums the tiles of group g from the compact list
// wlc (entries wlc[wlc[g]] ... wlc[wlc[g + 1] - 1]: compact tile index in
// bits 0-27, the group's slot in that tile in bits 28-31), in list order:
// deterministic.  Groups not in use give 0.
__global__ __launch_bounds__(NTHREADS) void k_hist_reduce(const double* __restrict__ ring,
                                                          const uint32_t* __restrict__ wlc, uint32_t nwt, int G,
                                                          double* __restrict__ out) {
  const uint32_t s = blockIdx.x, o = blockIdx.y;
  const uint32_t grp = o / NWALL, k = o % NWALL;
  double acc = 0.0;
  if ((int)grp < G) {
    const double* r = ring + (uint64_t)s * MAXBG * NWALL * nwt;
    for (uint32_t i = wlc[grp] + threadIdx.x; i < wlc[grp + 1]; i += NTHREADS) {
      const uint32_t en = wlc[i];
      acc += r[(uint64_t)((en >> 28) * NWALL + k) * nwt + (en & 0x0FFFFFFFu)];
    }
  }
  double v[1] = {acc};
  tile_sum_store<1>(v, out + (uint64_t)s * MAXG * NWALL + o);
}

// ---------------------------------------------------------------------------
// launchers (called by the host library)
// ---------------------------------------------------------------------------
template <class L, int P, int MHD, int PAR, int RU, bool ST>
static void launch_step_dg(const StepArgs& a, int dg, uint32_t nb, hipStream_t st) {
  if constexpr (P == S_F32 && MHD == 0 && PAR == 1 && RU == 2 && !ST) {
    if (dg == 0 && a.plain_loads) {
      k_step<L, P, 0, 1, 0, 2, false, false, false, true><<<nb, NTHREADS, 0, st>>>(a);
      return;
    }
  }
  if (dg == 2)
    k_step<L, P, MHD, PAR, 2, RU, false, ST><<<nb, NTHREADS, 0, st>>>(a);
  else if (dg == 1)
    k_step<L, P, MHD, PAR, 1, RU, false, ST><<<nb, NTHREADS, 0, st>>>(a);
  else
    k_step<L, P, MHD, PAR, 0, RU, false, ST><<<nb, NTHREADS, 0, st>>>(a);
}

template <class L, int P, int MHD, int RU, bool ST>
static void launch_step_ru_st(const StepArgs& a, int parity, int dg, uint32_t nb, hipStream_t st) {
  if constexpr (RU == 2 && MHD == 0) {
    if (a.ibb_in || a.ibb_out) {
      // interpolated links inside the step (never with diagnostics mode 1)
      if (parity == 0) {
        if (dg == 2) k_step<L, P, 0, 0, 2, 2, false, ST, true><<<nb, NTHREADS, 0, st>>>(a);
        else k_step<L, P, 0, 0, 0, 2, false, ST, true><<<nb, NTHREADS, 0, st>>>(a);
      } else {
        if (dg == 2) k_step<L, P, 0, 1, 2, 2, false, ST, true><<<nb, NTHREADS, 0, st>>>(a);
        else k_step<L, P, 0, 1, 0, 2, false, ST, true><<<nb, NTHREADS, 0, st>>>(a);
      }
      return;
    }
  }
  if (parity == 0)
    launch_step_dg<L, P, MHD, 0, RU, ST>(a, dg, nb, st);
  else
    launch_step_dg<L, P, MHD, 1, RU, ST>(a, dg, nb, st);
}

// Steps that store the stress and strain rate (a.sig or a.strain set) run
// their own instantiation, so that the other steps keep their registers.
template <class L, int P, int MHD, int RU>
static void launch_step_ru(const StepArgs& a, int parity, int dg, uint32_t nb, hipStream_t st) {
  if (a.sig || a.strain)
    launch_step_ru_st<L, P, MHD, RU, true>(a, parity, dg, nb, st);
  else
    launch_step_ru_st<L, P, MHD, RU, false>(a, parity, dg, nb, st);
}

template <class L, int P, int MHD>
static bool buffer_form(const Geom& g) {
  using E = typename Stor<P>::E;
  const uint64_t fb = (uint64_t)g.N * L::Q * sizeof(E);
  const uint64_t gb = MHD ? (uint64_t)g.N * Ind<L>::K * Ind<L>::NB * sizeof(E) : 0;
  return g.nx % 64 == 0 && fb < (1ull << 32) && gb < (1ull << 32);
}

template <class L, int P, int MHD>
static hipError_t launch_step_t(const StepArgs& a, int parity, int dg, hipStream_t st) {
  const uint32_t nb = (a.geo.N + NTHREADS - 1) / NTHREADS;
  if ((a.ibb_in || a.ibb_out) && (MHD != 0 || !buffer_form<L, P, MHD>(a.geo) || dg == 1))
    return hipErrorInvalidValue;
  // buffer form (measured: FP32 -1 %, FP16 and BF16 -6 to -8 %; FP64 +2 %
  // alone, but it carries the LDS staging of odd steps, and with it -4 %)
  if (buffer_form<L, P, MHD>(a.geo))
    launch_step_ru<L, P, MHD, 2>(a, parity, dg, nb, st);
  else if (a.geo.nx % 64 == 0)
    launch_step_ru<L, P, MHD, 1>(a, parity, dg, nb, st);
  else
    launch_step_ru<L, P, MHD, 0>(a, parity, dg, nb, st);
  return hipGetLastError();
}

// Forward step that also records rho and U of the pre-step state (adjoint
// recompute, or the recorded run's tape): F32 / F64 storage, no MHD.
template <class L, int P>
static hipError_t launch_step_mac_t(const StepArgs& a, int parity, bool diag, hipStream_t st) {
  const uint32_t nb = (a.geo.N + NTHREADS - 1) / NTHREADS;
  const bool ru = a.geo.nx % 64 == 0;
#define LBM_MAC(PAR, DG, RU) k_step<L, P, 0, PAR, DG, RU, true><<<nb, NTHREADS, 0, st>>>(a)
  if (buffer_form<L, P, 0>(a.geo)) {
    // buffer addressing of rows without boundary links, as the plain steps
    // (the same arithmetic: bit-identical states)
    if (parity == 0) {
      if (diag) LBM_MAC(0, 2, 2); else LBM_MAC(0, 0, 2);
    } else {
      if (diag) LBM_MAC(1, 2, 2); else LBM_MAC(1, 0, 2);
    }
  } else if (ru) {
    if (parity == 0) {
      if (diag) LBM_MAC(0, 2, 1); else LBM_MAC(0, 0, 1);
    } else {
      if (diag) LBM_MAC(1, 2, 1); else LBM_MAC(1, 0, 1);
    }
  } else {
    if (parity == 0) {
      if (diag) LBM_MAC(0, 2, 0); else LBM_MAC(0, 0, 0);
    } else {
      if (diag) LBM_MAC(1, 2, 0); else LBM_MAC(1, 0, 0);
    }
  }
#undef LBM_MAC
  return hipGetLastError();
}

template <class L, int P, int MHD>
static hipError_t launch_diag_t(const DiagArgs& a, hipStream_t st) {
  const uint32_t nb = (a.geo.N + NTHREADS - 1) / NTHREADS;
  if (a.parity == 0)
    k_diag<L, P, MHD, 0><<<nb, NTHREADS, 0, st>>>(a);
  else
    k_diag<L, P, MHD, 1><<<nb, NTHREADS, 0, st>>>(a);
  return hipGetLastError();
}

template <class L, int P, int MHD>
static hipError_t launch_ibb_t(const IbbArgs& a, hipStream_t st) {
  const uint32_t nb = (a.M + IBB_THREADS - 1) / IBB_THREADS;
  if (a.parity == 0)
    k_ibb<L, P, 0><<<nb, IBB_THREADS, 0, st>>>(a);
  else
    k_ibb<L, P, 1><<<nb, IBB_THREADS, 0, st>>>(a);
  return hipGetLastError();
}

template <class L, int P, int MHD>
static hipError_t launch_half_t(const HalfArgs& a, hipStream_t st) {
  const uint32_t nb = (a.geo.N + NTHREADS - 1) / NTHREADS;
  if (a.parity == 0)
    k_half<L, P, MHD, 0><<<nb, NTHREADS, 0, st>>>(a);
  else
    k_half<L, P, MHD, 1><<<nb, NTHREADS, 0, st>>>(a);
  return hipGetLastError();
}

template <class L, int P, int MHD>
static hipError_t launch_init_t(const InitArgs& a, hipStream_t st) {
  const uint32_t nb = (a.geo.N + NTHREADS - 1) / NTHREADS;
  k_init<L, P, MHD><<<nb, NTHREADS, 0, st>>>(a);
  return hipGetLastError();
}

// mhd: 0 none, 1 magnetic stress in the equilibrium, 2 Lorentz force through
// the force term (F64 / F32 storage only under MHD).
#define LBM_DISPATCH(FN, lattice, prec, mhd, ...)                                          \
  do {                                                                                       \
    if (mhd) {                                                                               \
      const bool d64 = prec == S_F64;                                                        \
      if (lattice == 0) {                                                                    \
        if (mhd == 1) return d64 ? FN<D2Q9, S_F64, 1>(__VA_ARGS__) : FN<D2Q9, S_F32, 1>(__VA_ARGS__); \
        return d64 ? FN<D2Q9, S_F64, 2>(__VA_ARGS__) : FN<D2Q9, S_F32, 2>(__VA_ARGS__);      \
      }                                                                                      \
      if (mhd == 1) return d64 ? FN<D3Q19, S_F64, 1>(__VA_ARGS__) : FN<D3Q19, S_F32, 1>(__VA_ARGS__); \
      return d64 ? FN<D3Q19, S_F64, 2>(__VA_ARGS__) : FN<D3Q19, S_F32, 2>(__VA_ARGS__);      \
    }                                                                                        \
    if (lattice == 0) {                                                                      \
      switch (prec) {                                                                        \
        case S_F64: return FN<D2Q9, S_F64, 0>(__VA_ARGS__);                                  \
        case S_F32: return FN<D2Q9, S_F32, 0>(__VA_ARGS__);                                  \
        case S_F16: return FN<D2Q9, S_F16, 0>(__VA_ARGS__);                                  \
        default: return FN<D2Q9, S_BF16, 0>(__VA_ARGS__);                                    \
      }                                                                                      \
    } else {                                                                                 \
      switch (prec) {                                                                        \
        case S_F64: return FN<D3Q19, S_F64, 0>(__VA_ARGS__);                                 \
        case S_F32: return FN<D3Q19, S_F32, 0>(__VA_ARGS__);                                 \
        case S_F16: return FN<D3Q19, S_F16, 0>(__VA_ARGS__);                                 \
        default: return FN<D3Q19, S_BF16, 0>(__VA_ARGS__);                                   \
      }                                                                                      \
    }                                                                                        \
  } while (0)

// dg: 0 no diagnostics, 1 the wall links' momentum exchange into the
// per-step ring (a.hist), 2 all diagnostics of the last step of a call.
hipError_t launch_step(int lattice, int prec, int mhd, const StepArgs& a, int parity, int dg, hipStream_t st) {
  LBM_DISPATCH(launch_step_t, lattice, prec, mhd, a, parity, dg, st);
}

template <class L, int P, int MHD>
static bool in_step_ibb_t(const Geom& g) {
  return MHD == 0 && buffer_form<L, P, MHD>(g);
}

bool step_interpolates_in_step(int lattice, int prec, int mhd, const Geom& g) {
  if (mhd) return false;
  if (lattice == 0) {
    switch (prec) {
      case S_F64: return in_step_ibb_t<D2Q9, S_F64, 0>(g);
      case S_F32: return in_step_ibb_t<D2Q9, S_F32, 0>(g);
      case S_F16: return in_step_ibb_t<D2Q9, S_F16, 0>(g);
      default: return in_step_ibb_t<D2Q9, S_BF16, 0>(g);
    }
  }
  switch (prec) {
    case S_F64: return in_step_ibb_t<D3Q19, S_F64, 0>(g);
    case S_F32: return in_step_ibb_t<D3Q19, S_F32, 0>(g);
    case S_F16: return in_step_ibb_t<D3Q19, S_F16, 0>(g);
    default: return in_step_ibb_t<D3Q19, S_BF16, 0>(g);
  }
}

hipError_t launch_step_mac(int lattice, int prec, const StepArgs& a, int parity, bool diag, hipStream_t st) {
  if (prec != S_F32 && prec != S_F64) return hipErrorInvalidValue;
  if (lattice == 0)
    return prec == S_F64 ? launch_step_mac_t<D2Q9, S_F64>(a, parity, diag, st)
                         : launch_step_mac_t<D2Q9, S_F32>(a, parity, diag, st);
  return prec == S_F64 ? launch_step_mac_t<D3Q19, S_F64>(a, parity, diag, st)
                       : launch_step_mac_t<D3Q19, S_F32>(a, parity, diag, st);
}

hipError_t launch_diag(int lattice, int prec, int mhd, const DiagArgs& a, hipStream_t st) {
  LBM_DISPATCH(launch_diag_t, lattice, prec, mhd, a, st);
}

hipError_t launch_half(int lattice, int prec, int mhd, const HalfArgs& a, hipStream_t st) {
  LBM_DISPATCH(launch_half_t, lattice, prec, mhd, a, st);
}

hipError_t launch_ibb(int lattice, int prec, const IbbArgs& a, hipStream_t st) {
  if (a.M == 0) return hipSuccess;
  LBM_DISPATCH(launch_ibb_t, lattice, prec, 0, a, st);
}

hipError_t launch_ibb_reduce(int lattice, const double* delta, const uint8_t* grp, uint32_t M, int G, double* part,
                             double* out, hipStream_t st) {
  const uint64_t entries = (uint64_t)M * (lattice == 0 ? 9 : 19);
  const uint32_t nb = (uint32_t)((entries + NTHREADS - 1) / NTHREADS);
  if (lattice == 0)
    k_ibb_part<D2Q9><<<nb, NTHREADS, 0, st>>>(delta, grp, entries, G, part);
  else
    k_ibb_part<D3Q19><<<nb, NTHREADS, 0, st>>>(delta, grp, entries, G, part);
  k_colsum<<<G * 4, NTHREADS, 0, st>>>(part, nb, (uint32_t)G * 4, out);
  return hipGetLastError();
}

hipError_t launch_init(int lattice, int prec, int mhd, const InitArgs& a, hipStream_t st) {
  LBM_DISPATCH(launch_init_t, lattice, prec, mhd, a, st);
}

hipError_t launch_hist_reduce(const double* ring, const uint32_t* wlc, uint32_t nwt, int G, uint32_t nsteps,
                              double* out, hipStream_t st) {
  if (nsteps == 0) return hipSuccess;
  k_hist_reduce<<<dim3(nsteps, MAXG * NWALL), NTHREADS, 0, st>>>(ring, wlc, nwt, G, out);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* part, const uint32_t* wlist, uint32_t ntiles, int mode, int G, int nout, double* out,
                         hipStream_t st) {
  k_reduce<<<nout, NTHREADS, 0, st>>>(part, wlist, ntiles, mode, G, out);
  return hipGetLastError();
}

}  // namespace lbm
