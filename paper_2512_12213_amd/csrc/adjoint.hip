// Adjoint (reverse-mode) step kernels for gfx950: the transpose of one forward
// step (relaxation of Eq. 2 with the equilibrium of Eq. 1 and the force term
// of Section 2 / Eq. 3, then A-A propagation with halfway bounce-back and the
// moving-wall term), used to differentiate the Eq. (25) wall force with
// respect to the per-node body force and the wall velocities.  The paper does
// not differentiate its method; this is the discrete adjoint of the forward
// kernels' arithmetic.
//
// In-place A-A storage of the adjoint state.  A forward step reads a node's
// populations from a set of slots and writes its relaxed values into the same
// set of slots (the A-A property, bounce-back links included).  The
// transposed step therefore reads the cotangents of the relaxed values from
// the slots the forward step wrote and writes the cotangents of the pre-step
// populations into the slots the forward step read, one thread per node and
// race-free in place, with the parity of the forward step it reverses.
//
// Per node, with nu = 1/tau, u^eq = U + lEq A, u^F = kF U + lF A and the
// cotangents mu_q of the relaxed values, everything reduces to the weighted
// moments m0 = sum w mu, m1 = sum w mu e, m2 = sum w mu e e:
//   rho-cotangent  M_rho = nu [m0 + 3 m1.ue + 9/2 ue.m2.ue - 3/2 ue.ue m0]
//                        + C [3 m1.A - 3 (uF.A) m0 + 9 uF.m2.A]
//                        + sum over wall links of mu_q (-6 w_q e_q.u_w)
//   G_ue = nu rho (3 m1 + 9 m2 ue - 3 ue m0),  G_uF = C rho (9 m2 A - 3 A m0)
//   U-cotangent    M_U = G_ue + kF G_uF
//   A-cotangent    g_A = lEq G_ue + lF G_uF + C rho (3 m1 - 3 uF m0 + 9 m2 uF)
// (the quadratic terms carry the factor quad, 0 for the Stokes equilibrium; a
// porous resistance A = (A_ext - s U) / (1 + s/2) adds -s/(1 + s/2) g_A to
// M_U and scales the external force's cotangent by 1/(1 + s/2))
//   lambda_p = (1 - nu) mu_p + M_rho + M_U.(e_p - U) / rho
// and the wall velocity of a link's group gets mu_q (-6 w_q rho e_q).  rho
// and U of the forward state come from the recompute pass (4 values per node
// instead of Q), in the forward storage precision PS; the adjoint state and
// its arithmetic use precision PL.  PL = F64 with an FP32 forward keeps the
// small anisotropic parts of lambda (differences of nearly equal values, e.g.
// the shear sensitivity at a distant wall) that FP32 storage of lambda rounds
// away.
#include "device.hpp"

namespace lbm {

// pu: this thread's column of the wall-velocity cotangents in LDS,
// [MAXBG][3] with stride NTHREADS.
template <class L, int PS, int PL, int PAR, bool SEED, bool BND, class AD>
__device__ __forceinline__ void adj_node(const AdjArgs& a, uint32_t n, const AD& Al, const uint4& rec,
                                         double* pu, uint32_t bgrp) {
  using S = Stor<PL>;
  using T = typename S::T;
  using E = typename S::E;
  const Geom& g = a.geo;
  const Phys& p = a.p;
  const uint32_t mask = rec.x;
  E* lam = (E*)a.lam;

  // objective of the last forward step: sum over the links of one group of
  // e_axis (2 d_rel + ladd), i.e. 2 e_axis on the cotangent of d_rel and
  // e_axis on that of ladd (the link's seed e_axis below)
  auto seed_of = [&](int q) __attribute__((always_inline)) -> T {
    if (SEED && BND && q > 0 && ((mask >> q) & 1u) && (int)nibble(rec, q) == a.seed_group)
      return T(a.seed_axis == 0 ? L::ex(q) : (a.seed_axis == 1 ? L::ey(q) : L::ez(q)));
    return T(0);
  };

  // cotangents of the relaxed values: read where the forward step wrote them
  // (on the last forward step they hold what the transposed interpolation
  // pass left there, zero without walls that are not halfway)
  T mu[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const int qb = opp(q);
    if constexpr (BND && PAR == 1) {
      mu[q] = S::ld(pick((mask >> q) & 1u, Al.template ptr<L>(lam, qb, -1), Al.template ptr<L>(lam, q, q)));
    } else if constexpr (PAR == 0) {
      mu[q] = Al.template ld<L, PL>(lam, qb, -1);
    } else {
      mu[q] = Al.template ld<L, PL>(lam, q, q);
    }
    if (SEED) mu[q] += T(2) * seed_of(q);
  }

  // forward state of this node and its body force
  using M = typename Stor<PS>::T;
  const M* mac = (const M*)a.mac;
  const T rho = (T)mac[n];
  const T U[3] = {(T)mac[g.N + n], (T)mac[2 * (uint64_t)g.N + n], (T)mac[3 * (uint64_t)g.N + n]};
  T A[3];
  if (a.afield) {
    const T sc = (T)p.afield_scale;
    A[0] = (T)a.afield[n] * sc;
    A[1] = (T)a.afield[g.N + n] * sc;
    A[2] = L::D == 3 ? (T)a.afield[2 * (uint64_t)g.N + n] * sc : T(0);
  } else {
    A[0] = (T)p.A[0];
    A[1] = (T)p.A[1];
    A[2] = (T)p.A[2];
  }
  // porous resistance: the force the node applies is A = (A_ext - s U) di
  const T ds = (T)p.darcy_s, di = (T)p.darcy_inv;
#pragma unroll
  for (int k = 0; k < 3; ++k) A[k] = (A[k] - ds * U[k]) * di;
  const T quad = (T)p.quad;
  const T nu = (T)p.inv_tau0;
  const T lEq = (T)p.lEq, kF = (T)p.kF;
  const T lF = (T)(p.lF0 + p.lF1 * p.tau0);
  const T C = (T)(1.0 - p.cG * 0.5 * p.inv_tau0);
  T ue[3], uf[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ue[k] = U[k] + lEq * A[k];
    uf[k] = kF * U[k] + lF * A[k];
  }

  // weighted moments of mu
  T m0 = ZERO<T>, m1[3] = {ZERO<T>, ZERO<T>, ZERO<T>};
  T mxx = ZERO<T>, myy = ZERO<T>, mzz = ZERO<T>, mxy = ZERO<T>, mxz = ZERO<T>, myz = ZERO<T>;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const T wm = (T)L::w(q) * mu[q];
    const int ex = L::ex(q), ey = L::ey(q), ez = L::ez(q);
    m0 += wm;
    if (ex) m1[0] += ex > 0 ? wm : -wm;
    if (ey) m1[1] += ey > 0 ? wm : -wm;
    if (ez) m1[2] += ez > 0 ? wm : -wm;
    if (ex) mxx += wm;
    if (ey) myy += wm;
    if (ez) mzz += wm;
    if (ex * ey) mxy += ex * ey > 0 ? wm : -wm;
    if (ex * ez) mxz += ex * ez > 0 ? wm : -wm;
    if (ey * ez) myz += ey * ez > 0 ? wm : -wm;
  }
  auto m2v = [&](const T (&v)[3], T (&r)[3]) __attribute__((always_inline)) {
    r[0] = mxx * v[0] + mxy * v[1] + mxz * v[2];
    r[1] = mxy * v[0] + myy * v[1] + myz * v[2];
    r[2] = mxz * v[0] + myz * v[1] + mzz * v[2];
  };
  T m2ue[3], m2A[3], m2uf[3];
  m2v(ue, m2ue);
  m2v(A, m2A);
  m2v(uf, m2uf);
  const T m1ue = m1[0] * ue[0] + m1[1] * ue[1] + m1[2] * ue[2];
  const T m1A = m1[0] * A[0] + m1[1] * A[1] + m1[2] * A[2];
  const T uem2ue = ue[0] * m2ue[0] + ue[1] * m2ue[1] + ue[2] * m2ue[2];
  const T ufm2A = uf[0] * m2A[0] + uf[1] * m2A[1] + uf[2] * m2A[2];
  const T ueue = ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2];
  const T ufA = uf[0] * A[0] + uf[1] * A[1] + uf[2] * A[2];

  T Mrho = nu * (m0 + T(3) * m1ue + quad * (T(4.5) * uem2ue - T(1.5) * ueue * m0)) +
           C * (T(3) * m1A - T(3) * ufA * m0 + T(9) * ufm2A);
  T MU[3], gA[3];
  const T nr = nu * rho, cr = C * rho;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T Gue = nr * (T(3) * m1[k] + quad * (T(9) * m2ue[k] - T(3) * ue[k] * m0));
    const T Guf = cr * (T(9) * m2A[k] - T(3) * A[k] * m0);
    // cotangent of the applied force, then through A = (A_ext - s U) di:
    // to U (-s di) and to the external force (di)
    const T gAt = lEq * Gue + lF * Guf + cr * (T(3) * m1[k] - T(3) * uf[k] * m0 + T(9) * m2uf[k]);
    MU[k] = Gue + kF * Guf - ds * di * gAt;
    gA[k] = di * gAt;
  }

  // moving-wall terms of the bounce-back links: -6 w_q rho (e_q . u_w)
  if (BND) {
#pragma unroll
    for (int q = 1; q < L::Q; ++q) {
      if ((mask >> q) & 1u) {
        const uint32_t gr = nibble(rec, q);
        const T ux = (T)a.uw[3 * gr], uy = (T)a.uw[3 * gr + 1], uz = (T)a.uw[3 * gr + 2];
        const T muL = SEED ? mu[q] - seed_of(q) : mu[q];
        const T c6 = T(-6) * (T)L::w(q) * muL;
        Mrho += c6 * edot<L>(q, ux, uy, uz);
        const T cr6 = c6 * rho;
#pragma unroll
        for (int s = 0; s < MAXBG; ++s) {
          if (((bgrp >> (4 * s)) & 15u) == gr) {
            pu[(3 * s + 0) * NTHREADS] += (double)(cr6 * (T)L::ex(q));
            pu[(3 * s + 1) * NTHREADS] += (double)(cr6 * (T)L::ey(q));
            pu[(3 * s + 2) * NTHREADS] += (double)(cr6 * (T)L::ez(q));
          }
        }
      }
    }
  }

  // cotangents of the pre-step populations: written where the forward step read them
  const T irho = T(1) / rho;
  const T MUU = (MU[0] * U[0] + MU[1] * U[1] + MU[2] * U[2]) * irho;
  const T keep = T(1) - nu;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const int qb = opp(q);
    const T lq = keep * mu[q] + Mrho + edot<L>(q, MU[0], MU[1], MU[2]) * irho - MUU;
    if constexpr (BND && PAR == 1) {
      S::st(pick((mask >> qb) & 1u, Al.template ptr<L>(lam, q, -1), Al.template ptr<L>(lam, qb, qb)), lq);
    } else if constexpr (PAR == 0) {
      Al.template st<L, PL>(lam, q, -1, lq);
    } else {
      Al.template st<L, PL>(lam, qb, qb, lq);
    }
  }

  // body-force gradient, accumulated over the steps
  if (a.grad_a) {
    const double sc = a.ga_scale;
    if (a.grad_f64) {
      double* ga = (double*)a.grad_a;
#pragma unroll
      for (int k = 0; k < L::D; ++k) ga[(uint64_t)k * g.N + n] += sc * (double)gA[k];
    } else {
      float* ga = (float*)a.grad_a;
#pragma unroll
      for (int k = 0; k < L::D; ++k) ga[(uint64_t)k * g.N + n] += (float)(sc * (double)gA[k]);
    }
  }
}

// Register budget of three wavefronts per SIMD (at most 168 VGPRs; the FP64
// adjoint state otherwise takes 205-211 and runs two): measured 3.5 % faster
// per backward pass with two spilled registers; a budget of four spills 40-56
// and is 18 % slower.
template <class L, int PS, int PL, int PAR, bool SEED, bool RU>
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_adj(const AdjArgs a) {
  using T = typename Stor<PL>::T;
  const Geom& g = a.geo;
  // tiles with boundary rows (slower) first, so that they do not form the
  // tail of the launch
  const uint32_t tile = a.tperm ? a.tperm[blockIdx.x] : blockIdx.x;
  const uint32_t n = tile * NTHREADS + threadIdx.x;
  const uint32_t bgrp = a.blkgrp[tile];
  // wall-velocity cotangents of this thread's links, in its own column of
  // LDS (FP64; no barrier: a thread touches only its column) rather than in
  // twelve registers held through the whole node update
  __shared__ double spu[MAXBG * 3 * NTHREADS];
  double* pu = spu + threadIdx.x;
  if (bgrp >> 28) {
#pragma unroll
    for (int j = 0; j < MAXBG * 3; ++j) pu[j * NTHREADS] = 0.0;
  }
  if (n < g.N) {
    uint32_t x, y, z, r;
    coords(g, n, x, y, z, r);
    if (RU) {
      r = __builtin_amdgcn_readfirstlane(r);
      y = __builtin_amdgcn_readfirstlane(y);
      z = __builtin_amdgcn_readfirstlane(z);
    }
    const int rr = a.rowrec[r];
    const uint4 rec = rr < 0 ? make_uint4(0u, 0u, 0u, 0u) : a.rec[rr + x];
    if (!(rec.x >> 31)) {
      if (RU) {
        using E = typename Stor<PL>::E;
        if (rr < 0 && (uint64_t)g.N * L::Q * sizeof(E) < (1ull << 32)) {
          // rows without boundary links, state below 4 GiB: buffer
          // addressing (no 64-bit per-lane addresses)
          const AddrB Ab = addr_b<E>(g, x, y, z, L::Q, a.lam, (uint32_t)((uint64_t)g.N * L::Q * sizeof(E)));
          adj_node<L, PS, PL, PAR, SEED, false>(a, n, Ab, rec, pu, bgrp);
        } else {
          const AddrR Al = addr_r(g, x, y, z, L::Q);
          if (rr < 0)
            adj_node<L, PS, PL, PAR, SEED, false>(a, n, Al, rec, pu, bgrp);
          else
            adj_node<L, PS, PL, PAR, SEED, true>(a, n, Al, rec, pu, bgrp);
        }
      } else {
        const AddrG Al = addr_g(g, x, y, z, r, L::Q);
        if (rr < 0)
          adj_node<L, PS, PL, PAR, SEED, false>(a, n, Al, rec, pu, bgrp);
        else
          adj_node<L, PS, PL, PAR, SEED, true>(a, n, Al, rec, pu, bgrp);
      }
    }
  }
  // wall-velocity cotangents of this tile, in the wall slots of the tile's
  // partial-sum record (block-uniform condition: the tile has wall links)
  if (bgrp >> 28) {
    double v[MAXBG * NWALL];
#pragma unroll
    for (int s = 0; s < MAXBG; ++s) {
      v[s * NWALL + 0] = pu[(3 * s + 0) * NTHREADS];
      v[s * NWALL + 1] = pu[(3 * s + 1) * NTHREADS];
      v[s * NWALL + 2] = pu[(3 * s + 2) * NTHREADS];
      v[s * NWALL + 3] = 0.0;
    }
    tile_sum_store<MAXBG * NWALL, true>(v, a.part + (uint64_t)NBAL * gridDim.x + tile, gridDim.x);
  }
}

template <class L, int PS, int PL, bool RU>
static void launch_adj_ru(const AdjArgs& a, int parity, bool seed, uint32_t nb, hipStream_t st) {
  if (parity == 0) {
    if (seed)
      k_adj<L, PS, PL, 0, true, RU><<<nb, NTHREADS, 0, st>>>(a);
    else
      k_adj<L, PS, PL, 0, false, RU><<<nb, NTHREADS, 0, st>>>(a);
  } else {
    if (seed)
      k_adj<L, PS, PL, 1, true, RU><<<nb, NTHREADS, 0, st>>>(a);
    else
      k_adj<L, PS, PL, 1, false, RU><<<nb, NTHREADS, 0, st>>>(a);
  }
}

template <class L, int PS, int PL>
static hipError_t launch_adj_t(const AdjArgs& a, int parity, bool seed, hipStream_t st) {
  const uint32_t nb = (a.geo.N + NTHREADS - 1) / NTHREADS;
  if (a.geo.nx % 64 == 0)
    launch_adj_ru<L, PS, PL, true>(a, parity, seed, nb, st);
  else
    launch_adj_ru<L, PS, PL, false>(a, parity, seed, nb, st);
  return hipGetLastError();
}

template <class L>
static hipError_t launch_adj_l(int prec, int adj_prec, const AdjArgs& a, int parity, bool seed, hipStream_t st) {
  if (prec == S_F64 && adj_prec == S_F64) return launch_adj_t<L, S_F64, S_F64>(a, parity, seed, st);
  if (prec == S_F32 && adj_prec == S_F64) return launch_adj_t<L, S_F32, S_F64>(a, parity, seed, st);
  if (prec == S_F32 && adj_prec == S_F32) return launch_adj_t<L, S_F32, S_F32>(a, parity, seed, st);
  return hipErrorInvalidValue;
}

hipError_t launch_adj(int lattice, int prec, int adj_prec, const AdjArgs& a, int parity, bool seed, hipStream_t st) {
  if (lattice == 0) return launch_adj_l<D2Q9>(prec, adj_prec, a, parity, seed, st);
  return launch_adj_l<D3Q19>(prec, adj_prec, a, parity, seed, st);
}

// ---------------------------------------------------------------------------
// Transposed interpolation pass (walls that are not halfway)
// ---------------------------------------------------------------------------
// With walls that are not halfway the recorded forward step is P o K: K the
// step with every wall link halfway, P the interpolation pass after it
// (Bouzidi, Firdaouss and Lallemand 2001), which at each listed node x
// replaces the value returned along opp(a) by a wall link a at fraction q:
//   q <  1/2: 2q V_a + (1 - 2q) D_a + (2q - 1) 6 w_a rho_t e_a.u_w
//             (D_a the value that streamed into x along a; V_a unchanged
//             when x - e_a is not a fluid node),
//   q >= 1/2: [V_a + (2q - 1) (V_opp(a) + 6 w_opp(a) rho_t e_opp(a).u_w)] / (2q)
//             (the last term only when opp(a) is a wall link too),
// with V the values node x wrote, rho_t = (rho0 + sum V) / (1 - K) and
// K = sum over the wall links of 6 w e.u_w.  Its transpose runs before each
// k_adj, on the adjoint state in the same layout.  Pass 1 (one thread per
// listed node) takes the cotangents of the replaced values and writes the
// cotangents of the node's own values V in place: those slots belong to that
// node alone.  The D_a slots are values written by the upstream node, which
// that node's own pass-1 thread updates when it is listed too, so pass 1
// leaves their contributions in dd1 and pass 2 adds them after it.  The
// wall-velocity cotangents of each link (along e_q, in the link's group) are
// accumulated per link over the steps and summed once at the end.
// On the last forward step the objective includes the interpolated links'
// change of the returned value, e_axis (new - V), for the links of its group.
constexpr int IBA_THREADS = 64;
static_assert(IBA_THREADS >= 3 * MAXG, "one thread per wall-velocity component");

template <class L, int PS, int PL, int PAR>
__global__ __launch_bounds__(IBA_THREADS) void k_ibb_adj1(const IbbAdjArgs a) {
  using S = Stor<PL>;
  using E = typename S::E;
  using T = typename S::T;
  using M = typename Stor<PS>::T;
  __shared__ double suw[MAXG][3];
  if (threadIdx.x < 3 * MAXG) (&suw[0][0])[threadIdx.x] = (&a.uw[0][0])[threadIdx.x];
  __syncthreads();
  const uint32_t i = blockIdx.x * IBA_THREADS + threadIdx.x;
  if (i >= a.M) return;
  const Geom& g = a.geo;
  // every load before the first store (the stores could alias the loads as
  // far as the compiler knows, which would serialise them)
  double qv[L::Q], sacc[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    qv[q] = a.qf[(uint64_t)i * L::Q + q];
    sacc[q] = a.sacc[(uint64_t)i * L::Q + q];
  }
  const uint32_t n = a.node[i];
  const uint4 rec = a.nrec[i];
  uint32_t x, y, z, r;
  coords(g, n, x, y, z, r);
  const AddrG Al = addr_g(g, x, y, z, r, L::Q);
  const uint32_t mask = rec.x;
  E* lam = (E*)a.lam;
  const double rho = (double)((const M*)a.mac)[n];
  double eu[L::Q];
  double K = 0.0;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    eu[q] = 0.0;
    if (q > 0 && ((mask >> q) & 1u)) {
      const uint32_t gr = nibble(rec, q);
      eu[q] = edot<L>(q, suw[gr][0], suw[gr][1], suw[gr][2]);
      K += 6.0 * L::w(q) * eu[q];
    }
  }
  // mu: cotangents of the replaced values; out: of the values V the pass read
  double mu[L::Q], out[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const bool wall = q > 0 && ((mask >> q) & 1u);
    const bool wr = wall && qv[q] != 0.5;
    const E* ptr = (PAR == 1 || wall) ? Al.template ptr<L>((const E*)lam, opp(q), -1)
                                      : Al.template ptr<L>((const E*)lam, q, q);
    const double v = (double)S::ld(ptr);
    mu[q] = wr ? v : 0.0;
    out[q] = wr ? 0.0 : v;
    if (wr && (int)nibble(rec, q) == a.seed_group) {
      const double ek = a.seed_axis == 0 ? L::ex(q) : (a.seed_axis == 1 ? L::ey(q) : L::ez(q));
      mu[q] += ek;
      out[q] -= ek;
    }
  }
  double srho = 0.0;  // cotangent of rho_t
  double s[L::Q], d1c[L::Q];
#pragma unroll
  for (int q = 0; q < L::Q; ++q) s[q] = d1c[q] = 0.0;
#pragma unroll
  for (int q = 1; q < L::Q; ++q) {
    if (!((mask >> q) & 1u) || qv[q] == 0.5) continue;
    const int qb = opp(q);
    const double t2 = 2.0 * qv[q];
    if (qv[q] < 0.5) {
      if ((mask >> qb) & 1u) {
        out[q] += mu[q];
      } else {
        out[q] += t2 * mu[q];
        d1c[q] = (1.0 - t2) * mu[q];
        const double c6 = (t2 - 1.0) * 6.0 * L::w(q) * mu[q];
        srho += c6 * eu[q];
        s[q] += c6 * rho;
      }
    } else {
      const double a2 = mu[q] * (t2 - 1.0) / t2;
      out[q] += mu[q] / t2;
      out[qb] += a2;
      if ((mask >> qb) & 1u) {
        const double c6 = a2 * 6.0 * L::w(qb);
        srho += c6 * eu[qb];
        s[qb] += c6 * rho;
      }
    }
  }
  // rho_t: through every V, and through K to the wall velocities
  const double sr = srho / (1.0 - K);
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    const bool wall = q > 0 && ((mask >> q) & 1u);
    E* ptr = (PAR == 1 || wall) ? Al.template ptr<L>(lam, opp(q), -1) : Al.template ptr<L>(lam, q, q);
    S::st(ptr, (T)(out[q] + sr));
    if (wall) s[q] += sr * rho * 6.0 * L::w(q);
    a.dd1[(uint64_t)i * L::Q + q] = d1c[q];
    a.sacc[(uint64_t)i * L::Q + q] = sacc[q] + s[q];  // 0 for links that are not wall links
  }
}

template <class L, int PL, int PAR>
__global__ __launch_bounds__(IBA_THREADS) void k_ibb_adj2(const IbbAdjArgs a) {
  using S = Stor<PL>;
  using E = typename S::E;
  using T = typename S::T;
  const uint32_t i = blockIdx.x * IBA_THREADS + threadIdx.x;
  if (i >= a.M) return;
  const Geom& g = a.geo;
  const uint32_t n = a.node[i];
  const uint32_t mask = a.nrec[i].x;
  uint32_t x, y, z, r;
  coords(g, n, x, y, z, r);
  const AddrG Al = addr_g(g, x, y, z, r, L::Q);
  E* lam = (E*)a.lam;
  // loads first, then the stores (as in pass 1)
  double v[L::Q], d[L::Q];
  uint32_t sel = 0;  // links with q < 1/2 and a fluid node behind
#pragma unroll
  for (int q = 1; q < L::Q; ++q) {
    const int qb = opp(q);
    d[q] = a.dd1[(uint64_t)i * L::Q + q];
    v[q] = 0.0;
    if (!((mask >> q) & 1u) || ((mask >> qb) & 1u) || !(a.qf[(uint64_t)i * L::Q + q] < 0.5)) continue;
    sel |= 1u << q;
    // where the next step reads the value streamed into x along q
    v[q] = (double)S::ld(PAR == 0 ? Al.template ptr<L>(lam, q, -1) : Al.template ptr<L>(lam, qb, qb));
  }
#pragma unroll
  for (int q = 1; q < L::Q; ++q) {
    const int qb = opp(q);
    if ((sel >> q) & 1u)
      S::st(PAR == 0 ? Al.template ptr<L>(lam, q, -1) : Al.template ptr<L>(lam, qb, qb), (T)(v[q] + d[q]));
  }
}

template <class L, int PS, int PL>
static void launch_ibb_adj_t(const IbbAdjArgs& a, hipStream_t st) {
  const uint32_t nb = (a.M + IBA_THREADS - 1) / IBA_THREADS;
  if (a.parity == 0) {
    k_ibb_adj1<L, PS, PL, 0><<<nb, IBA_THREADS, 0, st>>>(a);
    k_ibb_adj2<L, PL, 0><<<nb, IBA_THREADS, 0, st>>>(a);
  } else {
    k_ibb_adj1<L, PS, PL, 1><<<nb, IBA_THREADS, 0, st>>>(a);
    k_ibb_adj2<L, PL, 1><<<nb, IBA_THREADS, 0, st>>>(a);
  }
}

template <class L>
static hipError_t launch_ibb_adj_l(int prec, int adj_prec, const IbbAdjArgs& a, hipStream_t st) {
  if (prec == S_F64 && adj_prec == S_F64)
    launch_ibb_adj_t<L, S_F64, S_F64>(a, st);
  else if (prec == S_F32 && adj_prec == S_F64)
    launch_ibb_adj_t<L, S_F32, S_F64>(a, st);
  else if (prec == S_F32 && adj_prec == S_F32)
    launch_ibb_adj_t<L, S_F32, S_F32>(a, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_ibb_adj(int lattice, int prec, int adj_prec, const IbbAdjArgs& a, hipStream_t st) {
  if (a.M == 0) return hipSuccess;
  if (lattice == 0) return launch_ibb_adj_l<D2Q9>(prec, adj_prec, a, st);
  return launch_ibb_adj_l<D3Q19>(prec, adj_prec, a, st);
}

}  // namespace lbm
