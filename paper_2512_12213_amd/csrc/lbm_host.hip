// Host side of the C ABI declared in include/lbm.h: validation, geometry ->
// boundary records, buffer management, step loop, and assembly of the
// wall-force and balance records in FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "kernels.hpp"
#include "lattice.hpp"

namespace lbm {
hipError_t launch_step(int lattice, int prec, int mhd, const StepArgs& a, int parity, int dg, hipStream_t st);
bool step_interpolates_in_step(int lattice, int prec, int mhd, const Geom& g);
hipError_t launch_hist_reduce(const double* ring, const uint32_t* wlc, uint32_t nwt, int G, uint32_t nsteps,
                              double* out, hipStream_t st);
hipError_t launch_diag(int lattice, int prec, int mhd, const DiagArgs& a, hipStream_t st);
hipError_t launch_init(int lattice, int prec, int mhd, const InitArgs& a, hipStream_t st);
hipError_t launch_reduce(const double* part, const uint32_t* wlist, uint32_t ntiles, int mode, int G, int nout, double* out,
                         hipStream_t st);
hipError_t launch_step_mac(int lattice, int prec, const StepArgs& a, int parity, bool diag, hipStream_t st);
hipError_t launch_half(int lattice, int prec, int mhd, const HalfArgs& a, hipStream_t st);
hipError_t launch_ibb(int lattice, int prec, const IbbArgs& a, hipStream_t st);
hipError_t launch_ibb_reduce(int lattice, const double* delta, const uint8_t* grp, uint32_t M, int G, double* part,
                             double* out, hipStream_t st);
hipError_t launch_adj(int lattice, int prec, int adj_prec, const AdjArgs& a, int parity, bool seed, hipStream_t st);
hipError_t launch_ibb_adj(int lattice, int prec, int adj_prec, const IbbAdjArgs& a, hipStream_t st);
}  // namespace lbm

using namespace lbm;

// Fixed scratch for lbm_step_noalloc: a file-scope device array, one copy on
// each GPU the library runs on, held until the process ends.  In host code
// its name is not a device address: the address is looked up once per device
// (with that device current, device_scratch below) and only that pointer is
// ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[LBM_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, b ? b : 1);
    if (e == hipSuccess) bytes = b;
    return e;
  }
};

// lattice-generic helpers on the host
int lat_Q(int lat) { return lat == 0 ? 9 : 19; }
int lat_D(int lat) { return lat == 0 ? 2 : 3; }
void lat_e(int lat, int q, int* e) {
  if (lat == 0) {
    e[0] = D2Q9::ex(q);
    e[1] = D2Q9::ey(q);
    e[2] = 0;
  } else {
    e[0] = D3Q19::ex(q);
    e[1] = D3Q19::ey(q);
    e[2] = D3Q19::ez(q);
  }
}
double lat_w(int lat, int q) { return lat == 0 ? D2Q9::w(q) : D3Q19::w(q); }

}  // namespace

struct lbm_ctx {
  int lattice, D, Q, NC;
  int nx, ny, nz;
  uint32_t N;
  double tau, dx, dt, c;
  int model;
  int prec = S_F32;
  double rho0 = 1.0;
  int wall[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};
  std::vector<uint8_t> solid;  // 0 fluid, 1 + group
  double uw[MAXG][3] = {};
  double a[3] = {0, 0, 0};
  const float* afield = nullptr;
  double cs = 0;
  int stokes = 0;
  double darcy = 0;
  int artefact = 0;
  // stress and strain rate written by the steps themselves (borrowed device
  // buffers [NC][N] FP32) every st_every steps, or none
  float* st_sig = nullptr;
  float* st_strain = nullptr;
  int st_every = 0;
  bool mhd = false;
  bool lorentz = false;  // MHD coupling: Lorentz force through the force term
  double B0[3] = {0, 0, 0}, mu = 1, tau_m = 1;
  int device = 0;
  hipStream_t own = nullptr, stream = nullptr;

  // geometry
  bool geom_ok = false;
  int G = 1;
  uint32_t ntiles = 0;
  uint32_t nfluid = 0;
  std::vector<long> nlink;  // [MAXG][Q]

  DevBuf f, g, rec, rowrec, blkgrp, wlist, uwdev, part, red, dpart, dred, tmp;
  // per-step wall-force record: the tiles a wall group meets get a compact
  // index (wtile, -1 elsewhere; nwt of them) and per group a compact tile
  // list (wlc, the layout of wlist); steps other than a call's last sum their
  // wall links into a ring of hist_ring_steps slots, reduced into hist_out
  bool hist_on = false;
  uint32_t nwt = 0;
  DevBuf wtile, wlc, hist_ring, hist_out;
  DevBuf tperm;  // launch order of the step's tiles (those with boundary rows first), when used
  bool use_tperm = false;
  std::vector<double> hist;  // [steps of the last call][MAXG NWALL]
  long hist_steps = 0;
  // walls that are not halfway: link fractions (host, [Q][N]) and the list of
  // nodes whose links are interpolated after each step
  std::vector<double> qlink;
  DevBuf ibb_node, ibb_rec, ibb_q, ibb_grp, ibb_delta, ibb_part, ibb_red;
  DevBuf ibb_half;  // [nibb][Q] halfway values of the last step (half-step distribution)
  DevBuf ibb_hist;  // [steps - 1][MAXG][4] interpolated links' force changes of each step (per-step record)
  uint32_t nibb = 0;
  double* hred = nullptr;  // pinned [NBAL + MAXG * NWALL]
  void* scratch = nullptr;  // this device's fixed scratch array (lbm_step_noalloc), or null
  bool uw_dirty = true;
  bool have_state = false;
  long steps = 0;
  int parity = 0;
  bool have_step = false;
  double last[NBAL + MAXG * NWALL] = {};
  double last_uw[MAXG][3] = {};
  // adjoint: the recorded forward run (checkpoints every tape_K steps) and
  // the buffers of the backward pass
  DevBuf ckpt, replay, lam, mac, adjpart, adjred;
  DevBuf ibb_dd1, ibb_sacc;  // [nibb][Q] transposed interpolation pass (walls that are not halfway)
  bool tape = false;
  int adj_prec = S_F64;  // precision of the adjoint state and arithmetic
  int tape_T = 0, tape_K = 0, tape_group = 0, tape_axis = 0, tape_par0 = 0;
  // optional per-launch timing of lbm_step (HIP events on the context stream)
  bool timing = false;
  std::vector<hipEvent_t> ev;
  double tim[6] = {};  // mean even-parity step, mean odd-parity step, diagnostic step, reduce+copy, launches, call
};

namespace {

// MHD coupling as the kernels take it: 0 none, 1 equilibrium, 2 Lorentz force.
int mhd_mode(const lbm_ctx* h) { return h->mhd ? (h->lorentz ? 2 : 1) : 0; }

// Induction planes per node: D3Q7 x 3 components, or 5 x 2 in two dimensions.
int ind_planes(const lbm_ctx* h) { return h->lattice == LBM_D2Q9 ? 10 : 21; }


Phys make_phys(const lbm_ctx* h) {
  Phys p = {};
  p.rho0 = h->rho0;
  p.tau0 = h->tau;
  p.inv_tau0 = 1.0 / h->tau;
  for (int k = 0; k < 3; ++k) p.A[k] = h->a[k] * h->dt / h->c;
  p.afield_scale = h->dt / h->c;
  // force-model table: u^F = kF u + (lF0 + lF1 tau) dt a, u^eq = u + lEq dt a,
  // C = 1 - cG / (2 tau); thC = 1 when Theta follows Eq. (4).
  switch (h->model) {
    case LBM_FORCE_HE: p.kF = 0; p.lF0 = 0; p.lF1 = 0; p.lEq = 0; p.cG = 0; p.thC = 0; break;
    case LBM_FORCE_LUO: p.kF = 1; p.lF0 = 0; p.lF1 = 0; p.lEq = 0; p.cG = 0; p.thC = 1; break;
    case LBM_FORCE_SHANCHEN: p.kF = 1; p.lF0 = 0; p.lF1 = 0.5; p.lEq = 0; p.cG = 0; p.thC = 1; break;
    case LBM_FORCE_EDM: p.kF = 1; p.lF0 = 0.5; p.lF1 = 0; p.lEq = 0; p.cG = 0; p.thC = 1; break;
    default: p.kF = 1; p.lF0 = 0.5; p.lF1 = 0; p.lEq = 0.5; p.cG = 1; p.thC = 1; break;
  }
  p.les_K = 18.0 * std::sqrt(2.0) * h->cs * h->cs;
  p.quad = h->stokes ? 0.0 : 1.0;
  p.darcy_s = h->darcy * h->dt;
  p.darcy_inv = 1.0 / (1.0 + 0.5 * h->darcy * h->dt);
  const double bs = h->mhd ? 1.0 / (h->c * std::sqrt(h->mu)) : 0.0;
  for (int k = 0; k < 3; ++k) p.b0[k] = h->B0[k] * bs;
  p.inv_tau_m = h->mhd ? 1.0 / h->tau_m : 0.0;
  p.tm_theta = h->mhd ? 0.25 * h->tau_m : 0.0;
  for (int q = 0; q < 19; ++q) {
    double s = 1.0;
    if (q < h->Q) {
      if (h->prec == S_F16) s = 1024.0 / lat_w(h->lattice, q);
      if (h->prec == S_BF16) s = 1.0 / lat_w(h->lattice, q);
    }
    p.scale[q] = (float)s;
    p.inv_scale[q] = (float)(1.0 / s);
  }
  p.f.rho0 = (float)p.rho0;
  p.f.tau0 = (float)p.tau0;
  p.f.inv_tau0 = (float)p.inv_tau0;
  for (int k = 0; k < 3; ++k) {
    p.f.A[k] = (float)p.A[k];
    p.f.b0[k] = (float)p.b0[k];
  }
  p.f.afield_scale = (float)p.afield_scale;
  p.f.kF = (float)p.kF;
  p.f.lF0 = (float)p.lF0;
  p.f.lF1 = (float)p.lF1;
  p.f.lEq = (float)p.lEq;
  p.f.cG = (float)p.cG;
  p.f.thC = (float)p.thC;
  p.f.les_K = (float)p.les_K;
  p.f.quad = (float)p.quad;
  p.f.darcy_s = (float)p.darcy_s;
  p.f.darcy_inv = (float)p.darcy_inv;
  p.f.inv_tau_m = (float)p.inv_tau_m;
  p.f.tm_theta = (float)p.tm_theta;
  return p;
}

Geom make_geom(const lbm_ctx* h) {
  Geom g = {};
  g.nx = h->nx;
  g.ny = h->ny;
  g.nz = h->nz;
  g.N = h->N;
  g.mnx = h->nx > 1 ? UINT64_MAX / (uint64_t)h->nx + 1 : 0;
  g.mny = h->ny > 1 ? UINT64_MAX / (uint64_t)h->ny + 1 : 0;
  return g;
}

size_t elem_bytes(int prec) { return prec == S_F64 ? 8 : (prec == S_F32 ? 4 : 2); }

// Where does the link from (x,y,z) along e end?  0 = fluid node, 1 = wall or
// solid (group returned).  Corner links belong to the lowest axis.
int link_end(const lbm_ctx* h, int x, int y, int z, const int* e, int* grp) {
  int p[3] = {x + e[0], y + e[1], z + e[2]};
  const int n[3] = {h->nx, h->ny, h->nz};
  for (int k = 0; k < 3; ++k) {
    if (p[k] < 0 || p[k] >= n[k]) {
      const int side = p[k] < 0 ? 0 : 1;
      if (h->wall[k][side] >= 0) {
        *grp = h->wall[k][side];
        return 1;
      }
      p[k] = (p[k] + n[k]) % n[k];
    }
  }
  const uint8_t s = h->solid[((size_t)p[2] * h->ny + p[1]) * h->nx + p[0]];
  if (s) {
    *grp = s - 1;
    return 1;
  }
  return 0;
}

int build_geometry(lbm_ctx* h) {
  if (h->geom_ok) return LBM_OK;
  const int Q = h->Q;
  const size_t rows = (size_t)h->ny * h->nz;
  std::vector<int> rowrec(rows, -1);
  std::vector<uint4> recs;
  std::vector<uint4> rowbuf(h->nx);
  h->nlink.assign((size_t)MAXG * Q, 0);
  h->ntiles = (h->N + NTHREADS - 1) / NTHREADS;
  std::vector<uint32_t> tilegrp(h->ntiles, 0);
  std::vector<uint32_t> tilemask(h->ntiles, 0);  // bit per group present in the tile
  int gmax = 0;
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s) gmax = std::max(gmax, h->wall[a][s]);
  for (size_t i = 0; i < h->solid.size(); ++i)
    if (h->solid[i]) gmax = std::max(gmax, (int)h->solid[i] - 1);
  h->G = gmax + 1;
  h->nfluid = 0;
  for (int z = 0; z < h->nz; ++z)
    for (int y = 0; y < h->ny; ++y) {
      bool any = false;
      for (int x = 0; x < h->nx; ++x) {
        const size_t n = ((size_t)z * h->ny + y) * h->nx + x;
        uint4 r = make_uint4(0u, 0u, 0u, 0u);
        if (h->solid[n]) {
          r.x = 1u << 31;
          any = true;
        } else {
          ++h->nfluid;
          for (int q = 1; q < Q; ++q) {
            int e[3], grp;
            lat_e(h->lattice, q, e);
            if (link_end(h, x, y, z, e, &grp)) {
              r.x |= 1u << q;
              uint32_t* wv = q < 8 ? &r.y : (q < 16 ? &r.z : &r.w);
              *wv |= (uint32_t)grp << (4 * (q & 7));
              h->nlink[(size_t)grp * Q + q]++;
              tilemask[n / NTHREADS] |= 1u << grp;
              any = true;
            }
          }
        }
        rowbuf[x] = r;
      }
      if (any) {
        rowrec[(size_t)z * h->ny + y] = (int)recs.size();
        recs.insert(recs.end(), rowbuf.begin(), rowbuf.end());
      }
    }
  if (recs.size() > (size_t)INT32_MAX) return fail(LBM_EINVAL, "too many boundary rows");
  // nodes with links to walls that are not halfway
  std::vector<uint32_t> inode;
  std::vector<double> iq;
  std::vector<uint8_t> igrp;
  std::vector<uint4> irec;
  if (!h->qlink.empty()) {
    for (size_t row = 0; row < rows; ++row) {
      if (rowrec[row] < 0) continue;
      for (int x = 0; x < h->nx; ++x) {
        const uint4 r = recs[(size_t)rowrec[row] + x];
        if (r.x >> 31) continue;
        const size_t n = row * h->nx + x;
        bool any = false;
        for (int q = 1; q < Q; ++q)
          if (((r.x >> q) & 1u) && h->qlink[(size_t)q * h->N + n] != 0.5) any = true;
        if (!any) continue;
        // the record carries 1 + the node's index in this list
        if (inode.size() + 1 >= (1u << 20))
          return fail(LBM_EINVAL, "more than %u nodes with links to walls that are not halfway", (1u << 20) - 2);
        recs[(size_t)rowrec[row] + x].w |= (uint32_t)(inode.size() + 1) << 12;
        inode.push_back((uint32_t)n);
        irec.push_back(recs[(size_t)rowrec[row] + x]);
        for (int q = 0; q < Q; ++q) {
          const bool wall = q > 0 && ((r.x >> q) & 1u);
          const uint32_t wv = q < 8 ? r.y : (q < 16 ? r.z : r.w);
          iq.push_back(wall ? h->qlink[(size_t)q * h->N + n] : 0.5);
          igrp.push_back(wall ? (uint8_t)((wv >> (4 * (q & 7))) & 15u) : (uint8_t)0xFF);
        }
      }
    }
  }
  h->nibb = (uint32_t)inode.size();
  for (uint32_t t = 0; t < h->ntiles; ++t) {
    uint32_t cnt = 0, packed = 0;
    for (int gr = 0; gr < MAXG; ++gr)
      if (tilemask[t] >> gr & 1u) {
        if (cnt == MAXBG)
          return fail(LBM_EINVAL, "more than %d wall groups meet within one tile of %d nodes (tile %u)", MAXBG,
                      NTHREADS, t);
        packed |= (uint32_t)gr << (4 * cnt);
        ++cnt;
      }
    tilegrp[t] = packed | (cnt << 28);
    // bit 27: the tile holds whole rows, all nodes, and no row with boundary
    // links (odd steps may then stage their x-shifted directions in LDS)
    const uint64_t n0 = (uint64_t)t * NTHREADS;
    if (NTHREADS % h->nx == 0 && n0 + NTHREADS <= (uint64_t)h->N) {
      bool interior = true;
      for (uint64_t r = n0 / h->nx; r < (n0 + NTHREADS) / h->nx; ++r)
        if (rowrec[r] >= 0) interior = false;
      if (interior) tilegrp[t] |= 1u << 27;
    }
  }
  // per wall group, the tiles it meets with its slot there, in tile order
  // (offsets of the MAXG lists first): the reduction of the group's sums
  // visits only these tiles
  std::vector<uint32_t> wlist(MAXG + 1, 0);
  for (int gr = 0; gr < MAXG; ++gr) {
    wlist[gr] = (uint32_t)wlist.size();
    for (uint32_t t = 0; t < h->ntiles; ++t) {
      const uint32_t cnt = tilegrp[t] >> 28;
      for (uint32_t sl = 0; sl < cnt; ++sl)
        if (((tilegrp[t] >> (4 * sl)) & 15u) == (uint32_t)gr) wlist.push_back(t | (sl << 28));
    }
  }
  wlist[MAXG] = (uint32_t)wlist.size();
  // compact indices of the tiles a wall group meets, and the same per-group
  // lists with those indices
  std::vector<int> wtile(h->ntiles, -1);
  uint32_t nwt = 0;
  for (uint32_t t = 0; t < h->ntiles; ++t)
    if (tilegrp[t] >> 28) wtile[t] = (int)nwt++;
  std::vector<uint32_t> wlc(wlist.size());
  for (int gr = 0; gr <= MAXG; ++gr) wlc[gr] = wlist[gr];
  for (size_t i = MAXG + 1; i < wlist.size(); ++i)
    wlc[i] = (uint32_t)wtile[wlist[i] & 0x0FFFFFFFu] | (wlist[i] & 0xF0000000u);
  h->nwt = nwt;
  // Launch order of the step: the tiles holding a row with boundary links
  // first (when some but not all tiles have such rows); [0, T) for even
  // steps, [T, 2T) for odd ones.  Rows longer than a tile keep the odd
  // steps' XCD-aware order (kernel xcd_tile) over the rows in this order:
  // each group of 8 k workgroups takes 8 rows, row j mod 8, piece j / 8, so
  // that the k tiles of a row still meet in one L2 (even steps, without
  // x-shifted accesses, measured 3 % slower in that order).
  {
    const uint32_t T = h->ntiles;
    const uint32_t k = (h->nx > NTHREADS && h->nx % NTHREADS == 0) ? h->nx / NTHREADS : 1u;
    std::vector<uint32_t> first, rest;  // tiles in row order, boundary rows first
    for (uint32_t t = 0; t < T; t += k) {
      const uint64_t n0 = (uint64_t)t * NTHREADS;
      const uint64_t n1 = std::min<uint64_t>(n0 + (uint64_t)k * NTHREADS, (uint64_t)h->N) - 1;
      bool bnd = false;
      for (uint64_t r = n0 / h->nx; r <= n1 / h->nx && !bnd; ++r) bnd = rowrec[r] >= 0;
      for (uint32_t i = t; i < std::min(T, t + k); ++i) (bnd ? first : rest).push_back(i);
    }
    h->use_tperm = !first.empty() && !rest.empty();
    if (h->use_tperm) {
      first.insert(first.end(), rest.begin(), rest.end());
      std::vector<uint32_t> perm(2 * (size_t)T);
      const uint32_t chunk = 8u * k;
      for (uint32_t b = 0; b < T; ++b) {
        uint32_t j = b;
        if (k > 1u) {
          const uint32_t c = b / chunk;
          if ((uint64_t)(c + 1) * chunk <= T) j = c * chunk + ((b - c * chunk) % 8u) * k + (b - c * chunk) / 8u;
        }
        perm[b] = first[b];
        perm[T + b] = first[j];
      }
      HIPCHK(h->tperm.ensure(perm.size() * sizeof(uint32_t)));
      HIPCHK(hipMemcpy(h->tperm.p, perm.data(), perm.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    }
  }
  HIPCHK(h->wtile.ensure(wtile.size() * sizeof(int)));
  HIPCHK(hipMemcpy(h->wtile.p, wtile.data(), wtile.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(h->wlc.ensure(wlc.size() * sizeof(uint32_t)));
  HIPCHK(hipMemcpy(h->wlc.p, wlc.data(), wlc.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  HIPCHK(h->wlist.ensure(wlist.size() * sizeof(uint32_t)));
  HIPCHK(hipMemcpy(h->wlist.p, wlist.data(), wlist.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  HIPCHK(h->rowrec.ensure(rows * sizeof(int)));
  HIPCHK(h->rec.ensure(std::max<size_t>(recs.size(), 1) * sizeof(uint4)));
  HIPCHK(h->blkgrp.ensure((size_t)h->ntiles * sizeof(uint32_t)));
  HIPCHK(hipMemcpy(h->rowrec.p, rowrec.data(), rows * sizeof(int), hipMemcpyHostToDevice));
  if (!recs.empty()) HIPCHK(hipMemcpy(h->rec.p, recs.data(), recs.size() * sizeof(uint4), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(h->blkgrp.p, tilegrp.data(), (size_t)h->ntiles * sizeof(uint32_t), hipMemcpyHostToDevice));
  HIPCHK(h->part.ensure((size_t)h->ntiles * NPART * sizeof(double)));
  HIPCHK(h->dpart.ensure((size_t)h->ntiles * NDIAGPART * sizeof(double)));
  HIPCHK(h->red.ensure((NBAL + MAXG * NWALL) * sizeof(double)));
  HIPCHK(h->dred.ensure(NDIAGPART * sizeof(double)));
  HIPCHK(h->uwdev.ensure(MAXG * 3 * sizeof(double)));
  if (h->nibb) {
    HIPCHK(h->ibb_node.ensure(inode.size() * sizeof(uint32_t)));
    HIPCHK(h->ibb_rec.ensure(irec.size() * sizeof(uint4)));
    HIPCHK(h->ibb_q.ensure(iq.size() * sizeof(double)));
    HIPCHK(h->ibb_grp.ensure(igrp.size()));
    HIPCHK(h->ibb_delta.ensure(iq.size() * sizeof(double)));
    HIPCHK(h->ibb_half.ensure(iq.size() * sizeof(double)));
    HIPCHK(h->ibb_red.ensure(MAXG * 4 * sizeof(double)));
    HIPCHK(h->ibb_part.ensure(((iq.size() + NTHREADS - 1) / NTHREADS) * MAXG * 4 * sizeof(double)));
    HIPCHK(hipMemcpy(h->ibb_node.p, inode.data(), inode.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->ibb_rec.p, irec.data(), irec.size() * sizeof(uint4), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->ibb_q.p, iq.data(), iq.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->ibb_grp.p, igrp.data(), igrp.size(), hipMemcpyHostToDevice));
  }
  h->uw_dirty = true;
  h->geom_ok = true;
  return LBM_OK;
}

int alloc_state(lbm_ctx* h) {
  const size_t eb = elem_bytes(h->prec);
  HIPCHK(h->f.ensure((size_t)h->Q * h->N * eb));
  if (h->mhd) HIPCHK(h->g.ensure((size_t)ind_planes(h) * h->N * eb));
  return LBM_OK;
}

StepArgs step_args(lbm_ctx* h) {
  StepArgs a = {};
  // FP32 states beyond 1 GiB, far larger than the 256 MB last-level cache:
  // odd steps read with plain loads (measured 3 % faster there; 4.5 %
  // slower on a 318 MB state, which partly stays in that cache)
  a.plain_loads = h->prec == S_F32 && (uint64_t)h->Q * h->N * 4 > (1ull << 30);
  a.tperm = h->use_tperm ? (const uint32_t*)h->tperm.p : nullptr;
  a.f = h->f.p;
  a.g = h->mhd ? h->g.p : nullptr;
  a.afield = h->afield;
  a.rec = (const uint4*)h->rec.p;
  a.rowrec = (const int*)h->rowrec.p;
  a.blkgrp = (const uint32_t*)h->blkgrp.p;
  a.uw = (const double*)h->uwdev.p;
  a.part = (double*)h->part.p;
  a.geo = make_geom(h);
  a.p = make_phys(h);
  return a;
}

DiagArgs diag_args(lbm_ctx* h) {
  DiagArgs a = {};
  a.f = h->f.p;
  a.g = h->mhd ? h->g.p : nullptr;
  a.afield = h->afield;
  a.rec = (const uint4*)h->rec.p;
  a.rowrec = (const int*)h->rowrec.p;
  a.geo = make_geom(h);
  a.p = make_phys(h);
  a.parity = h->parity;
  a.artefact = h->artefact;
  a.c = h->c;
  a.dt = h->dt;
  for (int k = 0; k < 3; ++k) {
    a.wall_lo[k] = h->wall[k][0] >= 0;
    a.wall_hi[k] = h->wall[k][1] >= 0;
  }
  a.area = h->D == 2 ? h->dx : h->dx * h->dx;
  return a;
}

double vol(const lbm_ctx* h) { return h->D == 2 ? h->dx * h->dx : h->dx * h->dx * h->dx; }

int check_ready(lbm_ctx* h) {
  if (!h) return fail(LBM_EINVAL, "null context");
  if (!h->have_state) return fail(LBM_ESTATE, "no state: call lbm_init_equilibrium or lbm_set_state first");
  return LBM_OK;
}

int setup_guard(lbm_ctx* h) {
  if (!h) return fail(LBM_EINVAL, "null context");
  if (h->have_state) return fail(LBM_ESTATE, "geometry and storage must be set before the state is initialised");
  return LBM_OK;
}

// Device scratch of the step (per-tile partial sums, the reduced records, the
// interpolated-wall changes and their sums), from the context's own buffers
// or carved from the fixed array below.
struct Scratch {
  double* part;       // [NPART][ntiles]
  double* red;        // [NBAL + MAXG NWALL]
  double* ibb_delta;  // [nibb Q]
  double* ibb_part;   // [ceil(nibb Q / NTHREADS)][MAXG][4]
  double* ibb_red;    // [MAXG][4]
};

Scratch own_scratch(lbm_ctx* h) {
  return Scratch{(double*)h->part.p, (double*)h->red.p, (double*)h->ibb_delta.p, (double*)h->ibb_part.p,
                 (double*)h->ibb_red.p};
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Address of the current device's array (looked up on the first call for the
// device), or null with the HIP error.
void* device_scratch(int dev, hipError_t* err) {
  *err = hipSuccess;
  if (dev < 0 || dev >= MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// The step's scratch carved from the fixed array; bytes needed in *need.
Scratch fixed_scratch(const lbm_ctx* h, size_t* need) {
  char* base = (char*)h->scratch;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    char* p = base + off;
    off += round256(bytes);
    return (double*)p;
  };
  Scratch sc = {};
  sc.part = carve((size_t)h->ntiles * NPART * sizeof(double));
  sc.red = carve((NBAL + MAXG * NWALL) * sizeof(double));
  if (h->nibb) {
    const size_t entries = (size_t)h->nibb * h->Q;
    sc.ibb_delta = carve(entries * sizeof(double));
    sc.ibb_part = carve(((entries + NTHREADS - 1) / NTHREADS) * MAXG * 4 * sizeof(double));
    sc.ibb_red = carve(MAXG * 4 * sizeof(double));
  }
  *need = off;
  return sc;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

lbm_ctx* lbm_create(int lattice, int nx, int ny, int nz, double tau, double dx, double dt, int force_model) {
  if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) {
    fail(LBM_EINVAL, "lattice must be LBM_D2Q9 or LBM_D3Q19");
    return nullptr;
  }
  if (nx < 1 || ny < 1 || nz < 1 || nx > 65536 || ny > 65536 || nz > 65536) {
    fail(LBM_EINVAL, "sizes must be in [1, 65536]");
    return nullptr;
  }
  if (lattice == LBM_D2Q9 && nz != 1) {
    fail(LBM_EINVAL, "D2Q9 requires nz == 1");
    return nullptr;
  }
  if (!(tau > 0.5) || !std::isfinite(tau)) {
    fail(LBM_EINVAL, "tau must be > 1/2 (tau = %g)", tau);
    return nullptr;
  }
  if (!(dx > 0) || !(dt > 0) || !std::isfinite(dx) || !std::isfinite(dt)) {
    fail(LBM_EINVAL, "dx and dt must be positive");
    return nullptr;
  }
  if (force_model < 0 || force_model > 4) {
    fail(LBM_EINVAL, "force model must be in [0, 4]");
    return nullptr;
  }
  const uint64_t N = (uint64_t)nx * ny * nz;
  if (N >= (1ull << 31)) {
    fail(LBM_EINVAL, "lattice too large: %llu nodes (limit 2^31)", (unsigned long long)N);
    return nullptr;
  }
  lbm_ctx* h = new lbm_ctx();
  h->lattice = lattice;
  h->D = lat_D(lattice);
  h->Q = lat_Q(lattice);
  h->NC = lattice == 0 ? 3 : 6;
  h->nx = nx;
  h->ny = ny;
  h->nz = nz;
  h->N = (uint32_t)N;
  h->tau = tau;
  h->dx = dx;
  h->dt = dt;
  h->c = dx / dt;
  h->model = force_model;
  h->solid.assign(N, 0);
  if (hipGetDevice(&h->device) != hipSuccess || hipStreamCreate(&h->own) != hipSuccess) {
    fail(LBM_EHIP, "no HIP device / stream");
    delete h;
    return nullptr;
  }
  h->stream = h->own;
  {
    // the fixed scratch of lbm_step_noalloc: its address on this device
    // (a failed lookup only disables that entry point)
    hipError_t e;
    h->scratch = device_scratch(h->device, &e);
  }
  if (hipHostMalloc((void**)&h->hred, (2 * (NBAL + MAXG * NWALL) + NDIAGPART + MAXG * 4) * sizeof(double)) !=
      hipSuccess) {
    fail(LBM_ENOMEM, "pinned host buffer");
    (void)hipStreamDestroy(h->own);
    delete h;
    return nullptr;
  }
  return h;
}

void lbm_destroy(lbm_ctx* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->hred) (void)hipHostFree(h->hred);
  if (h->own) (void)hipStreamDestroy(h->own);
  delete h;
}

int lbm_set_storage(lbm_ctx* h, int precision) {
  int rc = setup_guard(h);
  if (rc) return rc;
  if (precision < LBM_F64 || precision > LBM_BF16) return fail(LBM_EINVAL, "unknown storage precision %d", precision);
  if (h->mhd && (precision == LBM_F16 || precision == LBM_BF16))
    return fail(LBM_EINVAL, "MHD supports F32 and F64 storage only");
  h->prec = precision;
  h->f.release();
  h->g.release();
  return LBM_OK;
}

int lbm_set_rho0(lbm_ctx* h, double rho0) {
  int rc = setup_guard(h);
  if (rc) return rc;
  if (!(rho0 > 0) || !std::isfinite(rho0)) return fail(LBM_EINVAL, "rho0 must be positive");
  h->rho0 = rho0;
  return LBM_OK;
}

int lbm_add_plane_walls(lbm_ctx* h, int axis, int glo, int ghi) {
  int rc = setup_guard(h);
  if (rc) return rc;
  if (axis < 0 || axis >= h->D) return fail(LBM_EINVAL, "axis %d out of range", axis);
  if (glo < -1 || glo >= MAXG || ghi < -1 || ghi >= MAXG) return fail(LBM_EINVAL, "group out of range");
  h->wall[axis][0] = glo;
  h->wall[axis][1] = ghi;
  h->geom_ok = false;
  return LBM_OK;
}

int lbm_add_solid_mask(lbm_ctx* h, const unsigned char* mask, int group) {
  int rc = setup_guard(h);
  if (rc) return rc;
  if (!mask) return fail(LBM_EINVAL, "null mask");
  if (group < 0 || group >= MAXG) return fail(LBM_EINVAL, "group out of range");
  for (uint32_t i = 0; i < h->N; ++i)
    if (mask[i]) h->solid[i] = (uint8_t)(1 + group);
  h->geom_ok = false;
  return LBM_OK;
}

int lbm_set_wall_velocity(lbm_ctx* h, int group, double ux, double uy, double uz) {
  if (!h) return fail(LBM_EINVAL, "null context");
  h->tape = false;
  if (group < 0 || group >= MAXG) return fail(LBM_EINVAL, "group out of range");
  if (!std::isfinite(ux) || !std::isfinite(uy) || !std::isfinite(uz)) return fail(LBM_EINVAL, "non-finite velocity");
  h->uw[group][0] = ux;
  h->uw[group][1] = uy;
  h->uw[group][2] = h->D == 3 ? uz : 0.0;
  h->uw_dirty = true;
  return LBM_OK;
}

int lbm_set_body_force(lbm_ctx* h, double ax, double ay, double az) {
  if (!h) return fail(LBM_EINVAL, "null context");
  h->tape = false;
  if (!std::isfinite(ax) || !std::isfinite(ay) || !std::isfinite(az)) return fail(LBM_EINVAL, "non-finite force");
  h->a[0] = ax;
  h->a[1] = ay;
  h->a[2] = h->D == 3 ? az : 0.0;
  return LBM_OK;
}

int lbm_set_body_force_field(lbm_ctx* h, const void* dev_ptr) {
  if (!h) return fail(LBM_EINVAL, "null context");
  h->tape = false;
  h->afield = (const float*)dev_ptr;
  return LBM_OK;
}

int lbm_set_les(lbm_ctx* h, double cs) {
  if (!h) return fail(LBM_EINVAL, "null context");
  h->tape = false;
  if (!(cs >= 0) || !std::isfinite(cs)) return fail(LBM_EINVAL, "C_s must be >= 0");
  h->cs = cs;
  return LBM_OK;
}

int lbm_set_link_fractions(lbm_ctx* h, const double* q) {
  int rc = setup_guard(h);
  if (rc) return rc;
  if (!q) {
    h->qlink.clear();
  } else {
    std::vector<double> v((size_t)h->Q * h->N);
    for (size_t i = 0; i < v.size(); ++i) {
      if (!(q[i] > 0.0 && q[i] <= 1.0)) return fail(LBM_EINVAL, "link fraction %g outside (0, 1] at %zu", q[i], i);
      v[i] = q[i];
    }
    h->qlink.swap(v);
  }
  h->geom_ok = false;
  return LBM_OK;
}

int lbm_set_equilibrium(lbm_ctx* h, int kind) {
  int rc = setup_guard(h);
  if (rc) return rc;
  if (kind != LBM_EQ_NS && kind != LBM_EQ_STOKES) return fail(LBM_EINVAL, "unknown equilibrium %d", kind);
  h->stokes = kind == LBM_EQ_STOKES;
  return LBM_OK;
}

int lbm_set_darcy(lbm_ctx* h, double sigma) {
  if (!h) return fail(LBM_EINVAL, "null context");
  if (!(sigma >= 0) || !std::isfinite(sigma)) return fail(LBM_EINVAL, "sigma must be >= 0");
  if (sigma > 0 && h->lorentz) return fail(LBM_EINVAL, "porous resistance is not combined with the Lorentz-force coupling");
  h->darcy = sigma;
  h->tape = false;
  return LBM_OK;
}

int lbm_set_step_stress(lbm_ctx* h, void* sigma_dev, void* strain_dev, int every) {
  if (!h) return fail(LBM_EINVAL, "null context");
  if (!sigma_dev && !strain_dev) {
    h->st_sig = h->st_strain = nullptr;
    h->st_every = 0;
    return LBM_OK;
  }
  if (every < 1) return fail(LBM_EINVAL, "every must be >= 1 (got %d)", every);
  const size_t bytes = (size_t)h->NC * h->N * sizeof(float);
  if (sigma_dev) HIPCHK(hipMemsetAsync(sigma_dev, 0, bytes, h->stream));
  if (strain_dev) HIPCHK(hipMemsetAsync(strain_dev, 0, bytes, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->st_sig = (float*)sigma_dev;
  h->st_strain = (float*)strain_dev;
  h->st_every = every;
  return LBM_OK;
}

int lbm_set_artefact(lbm_ctx* h, int on) {
  if (!h) return fail(LBM_EINVAL, "null context");
  h->artefact = on ? 1 : 0;
  return LBM_OK;
}

int lbm_set_mhd(lbm_ctx* h, double B0x, double B0y, double B0z, double mu, double tau_m) {
  int rc = setup_guard(h);
  if (rc) return rc;
  if (h->lattice == LBM_D2Q9 && B0z != 0.0) return fail(LBM_EINVAL, "two-dimensional MHD needs B0z = 0");
  if (h->prec == S_F16 || h->prec == S_BF16) return fail(LBM_EINVAL, "MHD supports F32 and F64 storage only");
  if (!(mu > 0) || !(tau_m > 0.5)) return fail(LBM_EINVAL, "need mu > 0 and tau_m > 1/2");
  h->mhd = true;
  h->B0[0] = B0x;
  h->B0[1] = B0y;
  h->B0[2] = B0z;
  h->mu = mu;
  h->tau_m = tau_m;
  return LBM_OK;
}

int lbm_set_mhd_coupling(lbm_ctx* h, int kind) {
  int rc = setup_guard(h);
  if (rc) return rc;
  if (!h->mhd) return fail(LBM_ESTATE, "MHD is not enabled");
  if (kind != LBM_MHD_EQUILIBRIUM && kind != LBM_MHD_LORENTZ_FORCE) return fail(LBM_EINVAL, "unknown coupling %d", kind);
  if (kind == LBM_MHD_LORENTZ_FORCE && h->darcy > 0)
    return fail(LBM_EINVAL, "porous resistance is not combined with the Lorentz-force coupling");
  h->lorentz = kind == LBM_MHD_LORENTZ_FORCE;
  return LBM_OK;
}

int lbm_set_stream(lbm_ctx* h, void* s) {
  if (!h) return fail(LBM_EINVAL, "null context");
  h->stream = s ? (hipStream_t)s : h->own;
  return LBM_OK;
}

int lbm_init_equilibrium(lbm_ctx* h, const double* u0) {
  if (!h) return fail(LBM_EINVAL, "null context");
  h->tape = false;
  int rc = build_geometry(h);
  if (rc) return rc;
  rc = alloc_state(h);
  if (rc) return rc;
  InitArgs a = {};
  a.f = h->f.p;
  a.g = h->mhd ? h->g.p : nullptr;
  a.rec = (const uint4*)h->rec.p;
  a.rowrec = (const int*)h->rowrec.p;
  a.geo = make_geom(h);
  a.p = make_phys(h);
  a.inv_c = 1.0 / h->c;
  if (u0) {
    HIPCHK(h->tmp.ensure((size_t)h->D * h->N * sizeof(double)));
    HIPCHK(hipMemcpyAsync(h->tmp.p, u0, (size_t)h->D * h->N * sizeof(double), hipMemcpyHostToDevice, h->stream));
    a.u0 = (const double*)h->tmp.p;
  }
  HIPCHK(launch_init(h->lattice, h->prec, mhd_mode(h), a, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->have_state = true;
  h->steps = 0;
  h->parity = 0;
  h->have_step = false;
  h->hist_steps = 0;
  return LBM_OK;
}

int lbm_set_state(lbm_ctx* h, const double* d) {
  if (!h) return fail(LBM_EINVAL, "null context");
  h->tape = false;
  if (!d) return fail(LBM_EINVAL, "null state");
  int rc = build_geometry(h);
  if (rc) return rc;
  rc = alloc_state(h);
  if (rc) return rc;
  InitArgs a = {};
  a.f = h->f.p;
  a.g = h->mhd ? h->g.p : nullptr;
  a.rec = (const uint4*)h->rec.p;
  a.rowrec = (const int*)h->rowrec.p;
  a.geo = make_geom(h);
  a.p = make_phys(h);
  a.inv_c = 1.0 / h->c;
  HIPCHK(h->tmp.ensure((size_t)h->Q * h->N * sizeof(double)));
  HIPCHK(hipMemcpyAsync(h->tmp.p, d, (size_t)h->Q * h->N * sizeof(double), hipMemcpyHostToDevice, h->stream));
  a.state = (const double*)h->tmp.p;
  HIPCHK(launch_init(h->lattice, h->prec, mhd_mode(h), a, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->have_state = true;
  h->steps = 0;
  h->parity = 0;
  h->have_step = false;
  h->hist_steps = 0;
  return LBM_OK;
}

static int run_diag(lbm_ctx* h, DiagArgs& a) {
  HIPCHK(launch_diag(h->lattice, h->prec, mhd_mode(h), a, h->stream));
  return LBM_OK;
}

int lbm_get_state(lbm_ctx* h, double* d) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!d) return fail(LBM_EINVAL, "null buffer");
  const size_t bytes = (size_t)h->Q * h->N * sizeof(double);
  HIPCHK(h->tmp.ensure(bytes));
  DiagArgs a = diag_args(h);
  a.state = (double*)h->tmp.p;
  rc = run_diag(h, a);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(d, h->tmp.p, bytes, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_get_induction(lbm_ctx* h, double* gout) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->mhd) return fail(LBM_ESTATE, "MHD is not enabled");
  if (!gout) return fail(LBM_EINVAL, "null buffer");
  const size_t bytes = (size_t)ind_planes(h) * h->N * sizeof(double);
  HIPCHK(h->tmp.ensure(bytes));
  DiagArgs a = diag_args(h);
  a.gstate = (double*)h->tmp.p;
  rc = run_diag(h, a);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(gout, h->tmp.p, bytes, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const double s = h->c * std::sqrt(h->mu);
  for (size_t i = 0; i < (size_t)ind_planes(h) * h->N; ++i) gout[i] *= s;
  return LBM_OK;
}

static int upload_uw(lbm_ctx* h) {
  if (h->uw_dirty) {
    double t[MAXG * 3];
    for (int gr = 0; gr < MAXG; ++gr)
      for (int k = 0; k < 3; ++k) t[3 * gr + k] = h->uw[gr][k] / h->c;
    HIPCHK(hipMemcpy(h->uwdev.p, t, sizeof(t), hipMemcpyHostToDevice));
    h->uw_dirty = false;
  }
  return LBM_OK;
}

// n >= 1 steps; the last one with diagnostics.  With ckpt_every > 0 the state
// before step i is copied to checkpoint i / ckpt_every whenever
// i % ckpt_every == 0; with a tape, every step also records rho and U of its
// pre-step state at tape + i * 4 N values.  sc: the scratch buffers of the
// step (the context's own when null); timing events are recorded only with
// the context's own buffers (creating events may allocate).  With hist, the
// steps before the last also record the momentum exchange of the wall links
// (reduced in chunks of the ring's size into hist_out).
constexpr int HIST_RING = 256;  // steps per ring (one reduction per chunk)
static int step_loop(lbm_ctx* h, int n, int ckpt_every, void* tape = nullptr, const Scratch* scp = nullptr,
                     bool hist = false) {
  int rc = upload_uw(h);
  if (rc) return rc;
  const Scratch sc = scp ? *scp : own_scratch(h);
  const bool timing = h->timing && !scp;
  StepArgs a = step_args(h);
  a.part = sc.part;
  a.wtile = (const int*)h->wtile.p;
  a.nwt = h->nwt;
  const size_t slot = (size_t)MAXBG * NWALL * std::max<uint32_t>(h->nwt, 1);  // doubles per ring slot
  const int ring = std::min(HIST_RING, std::max(n - 1, 1));
  if (hist) {
    HIPCHK(h->hist_ring.ensure((size_t)ring * slot * sizeof(double)));
    HIPCHK(h->hist_out.ensure((size_t)std::max(n - 1, 1) * MAXG * NWALL * sizeof(double)));
    if (h->nibb) HIPCHK(h->ibb_hist.ensure((size_t)std::max(n - 1, 1) * MAXG * 4 * sizeof(double)));
  }
  int chunk0 = 0;  // first step of the ring's current chunk
  const size_t mbytes = (size_t)4 * h->N * elem_bytes(h->prec);
  IbbArgs ib = {};
  if (h->nibb) {
    ib.f = h->f.p;
    ib.node = (const uint32_t*)h->ibb_node.p;
    ib.qf = (const double*)h->ibb_q.p;
    ib.grp = (const uint8_t*)h->ibb_grp.p;
    ib.nrec = (const uint4*)h->ibb_rec.p;
    for (int gr = 0; gr < MAXG; ++gr)
      for (int k = 0; k < 3; ++k) ib.uw[gr][k] = h->uw[gr][k] / h->c;
    ib.M = h->nibb;
    ib.geo = a.geo;
    ib.p = a.p;
  }
  const size_t sbytes = (size_t)h->Q * h->N * elem_bytes(h->prec);
  if (timing) {
    while (h->ev.size() < (size_t)n + 2) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      h->ev.push_back(e);
    }
  }
  const int par0 = h->parity;
  if (timing) HIPCHK(hipEventRecord(h->ev[0], h->stream));
  a.ibq = h->nibb ? (const double*)h->ibb_q.p : nullptr;
  // (a recorded run keeps the pass after every step: its checkpoints then
  // hold whole states, and the adjoint reverses the pass step by step)
  const bool in_step = h->nibb && !tape && !hist && ckpt_every == 0 &&
                       step_interpolates_in_step(h->lattice, h->prec, mhd_mode(h), a.geo);
  a.st_c2 = (float)(h->c * h->c);
  a.st_hdt = (float)(1.5 / h->dt);
  a.st_artefact = h->artefact;
  for (int i = 0; i < n; ++i) {
    const bool st = h->st_every > 0 && (h->steps + i) % h->st_every == 0;
    a.sig = st ? h->st_sig : nullptr;
    a.strain = st ? h->st_strain : nullptr;
    if (ckpt_every > 0 && i % ckpt_every == 0)
      HIPCHK(hipMemcpyAsync((char*)h->ckpt.p + (size_t)(i / ckpt_every) * sbytes, h->f.p, sbytes,
                            hipMemcpyDeviceToDevice, h->stream));
    const bool diag = i == n - 1;
    // interpolated links: in the step except on the last one of the call,
    // whose halfway values the pass after it replaces (row-uniform buffer
    // form without MHD; otherwise the pass runs after every step)
    a.ibb_in = in_step && i > 0;
    a.ibb_out = in_step && !diag;
    if (tape) {
      a.mac = (char*)tape + (size_t)i * mbytes;
      HIPCHK(launch_step_mac(h->lattice, h->prec, a, h->parity, diag, h->stream));
    } else {
      const int dg = diag ? 2 : (hist ? 1 : 0);
      a.hist = dg == 1 ? (double*)h->hist_ring.p + (size_t)(i - chunk0) * slot : nullptr;
      HIPCHK(launch_step(h->lattice, h->prec, mhd_mode(h), a, h->parity, dg, h->stream));
      if (hist && !diag && (i - chunk0 + 1 == ring || i == n - 2)) {
        HIPCHK(launch_hist_reduce((const double*)h->hist_ring.p, (const uint32_t*)h->wlc.p, h->nwt, h->G,
                                  (uint32_t)(i - chunk0 + 1),
                                  (double*)h->hist_out.p + (size_t)chunk0 * MAXG * NWALL, h->stream));
        chunk0 = i + 1;
      }
    }
    if (h->nibb && (diag || !in_step)) {
      ib.parity = h->parity ^ 1;
      ib.delta = (diag || hist) ? sc.ibb_delta : nullptr;
      ib.half = diag ? (double*)h->ibb_half.p : nullptr;
      HIPCHK(launch_ibb(h->lattice, h->prec, ib, h->stream));
      if (hist && !diag)
        // this step's changes of the returning values, for its record
        HIPCHK(launch_ibb_reduce(h->lattice, sc.ibb_delta, (const uint8_t*)h->ibb_grp.p, h->nibb, h->G, sc.ibb_part,
                                 (double*)h->ibb_hist.p + (size_t)i * MAXG * 4, h->stream));
    }
    if (timing) HIPCHK(hipEventRecord(h->ev[i + 1], h->stream));
    h->parity ^= 1;
  }
  HIPCHK(launch_reduce(sc.part, (const uint32_t*)h->wlist.p, h->ntiles, 0, h->G, NBAL + MAXG * NWALL, sc.red,
                       h->stream));
  HIPCHK(hipMemcpyAsync(h->hred, sc.red, (NBAL + MAXG * NWALL) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  double* ibb_host = h->hred + 2 * (NBAL + MAXG * NWALL) + NDIAGPART;
  if (h->nibb) {
    HIPCHK(launch_ibb_reduce(h->lattice, sc.ibb_delta, (const uint8_t*)h->ibb_grp.p, h->nibb, h->G, sc.ibb_part,
                             sc.ibb_red, h->stream));
    HIPCHK(hipMemcpyAsync(ibb_host, sc.ibb_red, (size_t)h->G * 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  }
  if (timing) HIPCHK(hipEventRecord(h->ev[n + 1], h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (timing) {
    double se = 0, so = 0;
    int ne = 0, no = 0;
    for (int i = 0; i < n; ++i) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]));
      if (i == n - 1) {
        h->tim[2] = ms * 1e-3;
      } else if (((par0 + i) & 1) == 0) {
        se += ms * 1e-3;
        ++ne;
      } else {
        so += ms * 1e-3;
        ++no;
      }
    }
    float ms = 0, tot = 0;
    HIPCHK(hipEventElapsedTime(&ms, h->ev[n], h->ev[n + 1]));
    HIPCHK(hipEventElapsedTime(&tot, h->ev[0], h->ev[n + 1]));
    h->tim[0] = ne ? se / ne : 0;
    h->tim[1] = no ? so / no : 0;
    h->tim[3] = ms * 1e-3;
    h->tim[4] = n;
    h->tim[5] = tot * 1e-3;
  }
  std::memcpy(h->last, h->hred, sizeof(h->last));
  // interpolated links: the returning values changed after the step's own sums
  for (int gr = 0; h->nibb && gr < h->G; ++gr)
    for (int k = 0; k < NWALL; ++k) h->last[NBAL + gr * NWALL + k] += ibb_host[gr * 4 + k];
  if (hist) {
    // the steps before the last from the ring's reductions, the last from the
    // call's own record
    h->hist.assign((size_t)n * MAXG * NWALL, 0.0);
    if (n > 1)
      HIPCHK(hipMemcpy(h->hist.data(), h->hist_out.p, (size_t)(n - 1) * MAXG * NWALL * sizeof(double),
                       hipMemcpyDeviceToHost));
    if (n > 1 && h->nibb) {
      // interpolated links: each step's changes of the returning values
      std::vector<double> ih((size_t)(n - 1) * MAXG * 4);
      HIPCHK(hipMemcpy(ih.data(), h->ibb_hist.p, ih.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (int st = 0; st < n - 1; ++st)
        for (int gr = 0; gr < h->G; ++gr)
          for (int k = 0; k < NWALL; ++k)
            h->hist[((size_t)st * MAXG + gr) * NWALL + k] += ih[((size_t)st * MAXG + gr) * 4 + k];
    }
    std::memcpy(h->hist.data() + (size_t)(n - 1) * MAXG * NWALL, h->last + NBAL, MAXG * NWALL * sizeof(double));
    h->hist_steps = n;
  } else {
    h->hist_steps = 0;
  }
  std::memcpy(h->last_uw, h->uw, sizeof(h->last_uw));
  h->steps += n;
  h->have_step = true;
  if (!std::isfinite(h->last[0])) return fail(LBM_EUNSTABLE, "total mass is not finite after step %ld", h->steps);
  return LBM_OK;
}

int lbm_step(lbm_ctx* h, int n) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (n < 0) return fail(LBM_EINVAL, "negative step count");
  if (n == 0) return LBM_OK;
  h->tape = false;
  return step_loop(h, n, 0, nullptr, nullptr, h->hist_on);
}

int lbm_step_noalloc(lbm_ctx* h, int n) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (n < 0) return fail(LBM_EINVAL, "negative step count");
  if (!h->scratch) return fail(LBM_EHIP, "the fixed scratch array of this device could not be located");
  if (h->hist_on) return fail(LBM_EINVAL, "lbm_step_noalloc does not record the per-step wall-force history");
  size_t need = 0;
  const Scratch sc = fixed_scratch(h, &need);
  if (need > (size_t)LBM_SCRATCH_BYTES)
    return fail(LBM_EINVAL, "lbm_step_noalloc: this lattice needs %zu bytes of step scratch, above the fixed %d",
                need, (int)LBM_SCRATCH_BYTES);
  if (n == 0) return LBM_OK;
  h->tape = false;
  return step_loop(h, n, 0, nullptr, &sc);
}

int lbm_get_macro(lbm_ctx* h, double* rho, double* v) {
  int rc = check_ready(h);
  if (rc) return rc;
  const size_t N = h->N;
  HIPCHK(h->tmp.ensure((1 + (size_t)h->D) * N * sizeof(double)));
  DiagArgs a = diag_args(h);
  double* base = (double*)h->tmp.p;
  a.rho = rho ? base : nullptr;
  a.vel = v ? base + N : nullptr;
  rc = run_diag(h, a);
  if (rc) return rc;
  if (rho) HIPCHK(hipMemcpyAsync(rho, base, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (v) HIPCHK(hipMemcpyAsync(v, base + N, (size_t)h->D * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_get_field_B(lbm_ctx* h, double* B) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->mhd) return fail(LBM_ESTATE, "MHD is not enabled");
  const size_t N = h->N;
  HIPCHK(h->tmp.ensure(3 * N * sizeof(double)));
  DiagArgs a = diag_args(h);
  a.B = (double*)h->tmp.p;
  rc = run_diag(h, a);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(B, h->tmp.p, 3 * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const double s = h->c * std::sqrt(h->mu);
  for (size_t i = 0; i < 3 * N; ++i) B[i] *= s;
  return LBM_OK;
}

int lbm_stress(lbm_ctx* h, double* sigma, double* strain) {
  int rc = check_ready(h);
  if (rc) return rc;
  const size_t N = h->N, nc = h->NC;
  HIPCHK(h->tmp.ensure(2 * nc * N * sizeof(double)));
  DiagArgs a = diag_args(h);
  double* base = (double*)h->tmp.p;
  a.sigma = sigma ? base : nullptr;
  a.strain = strain ? base + nc * N : nullptr;
  rc = run_diag(h, a);
  if (rc) return rc;
  if (sigma) HIPCHK(hipMemcpyAsync(sigma, base, nc * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (strain) HIPCHK(hipMemcpyAsync(strain, base + nc * N, nc * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_stress_device(lbm_ctx* h, double* sigma, double* strain) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!sigma && !strain) return LBM_OK;
  DiagArgs a = diag_args(h);
  a.sigma = sigma;
  a.strain = strain;
  return run_diag(h, a);
}

// The half-step kernel's arguments for the last step, outputs left null.
static HalfArgs half_args(lbm_ctx* h) {
  HalfArgs a = {};
  a.f = h->f.p;
  a.g = h->mhd ? h->g.p : nullptr;
  a.rec = (const uint4*)h->rec.p;
  a.rowrec = (const int*)h->rowrec.p;
  a.ibb_half = h->nibb ? (const double*)h->ibb_half.p : nullptr;
  for (int gr = 0; gr < MAXG; ++gr)
    for (int k = 0; k < 3; ++k) a.uw[gr][k] = h->last_uw[gr][k] / h->c;
  a.geo = make_geom(h);
  a.p = make_phys(h);
  a.parity = h->parity;
  a.c = h->c;
  return a;
}

int lbm_halfstep_device(lbm_ctx* h, double* fbar, double* rho_bar, double* u_bar, double* sigma_bar) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->have_step) return fail(LBM_ESTATE, "no step taken since the state was set");
  if (!fbar && !rho_bar && !u_bar && !sigma_bar) return LBM_OK;
  HalfArgs a = half_args(h);
  a.fbar = fbar;
  a.rho = rho_bar;
  a.vel = u_bar;
  a.sigma = sigma_bar;
  HIPCHK(launch_half(h->lattice, h->prec, mhd_mode(h), a, h->stream));
  return LBM_OK;
}

int lbm_halfstep(lbm_ctx* h, double* fbar, double* rho_bar, double* u_bar, double* sigma_bar) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->have_step) return fail(LBM_ESTATE, "no step taken since the state was set");
  const size_t N = h->N, Q = h->Q, D = h->D, nc = h->NC;
  const size_t total = (fbar ? Q : 0) + (rho_bar ? 1 : 0) + (u_bar ? D : 0) + (sigma_bar ? nc : 0);
  if (!total) return LBM_OK;
  HIPCHK(h->tmp.ensure(total * N * sizeof(double)));
  HalfArgs a = half_args(h);
  double* base = (double*)h->tmp.p;
  size_t off = 0;
  if (fbar) { a.fbar = base + off; off += Q * N; }
  if (rho_bar) { a.rho = base + off; off += N; }
  if (u_bar) { a.vel = base + off; off += D * N; }
  if (sigma_bar) { a.sigma = base + off; off += nc * N; }
  HIPCHK(launch_half(h->lattice, h->prec, mhd_mode(h), a, h->stream));
  if (fbar) HIPCHK(hipMemcpyAsync(fbar, a.fbar, Q * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (rho_bar) HIPCHK(hipMemcpyAsync(rho_bar, a.rho, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (u_bar) HIPCHK(hipMemcpyAsync(u_bar, a.vel, D * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (sigma_bar) HIPCHK(hipMemcpyAsync(sigma_bar, a.sigma, nc * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

// Wall-force variants per group from the last step's FP64 sums plus the
// constant per-link parts (rest-state pressure, Maxwell stress at B0).
static void wall_variants(const lbm_ctx* h, int gr, double out[4][3], const double* sums = nullptr) {
  const double fscale = vol(h) * h->c / h->dt;  // (dx^D / dt) c
  const double* s = (sums ? sums : h->last + NBAL) + gr * NWALL;
  double raw[3], mf[3], mx[3] = {0, 0, 0};
  double stat[3] = {0, 0, 0};
  const double b = h->mhd ? 1.0 / (h->c * std::sqrt(h->mu)) : 0.0;
  const double bb[3] = {h->B0[0] * b, h->B0[1] * b, h->B0[2] * b};
  const double b2 = bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2];
  for (int q = 1; q < h->Q; ++q) {
    const long nl = h->nlink[(size_t)gr * h->Q + q];
    if (!nl) continue;
    int e[3];
    lat_e(h->lattice, q, e);
    const double w = lat_w(h->lattice, q);
    double phi = 0.0;
    if (h->mhd && !h->lorentz) {
      // magnetic part of the equilibrium at the wall field B0 (Eq. 10; two
      // dimensions without -b^2 / 6); with the Lorentz force in the force
      // term the equilibrium has none and P carries no Maxwell stress
      const double eb = e[0] * bb[0] + e[1] * bb[1] + e[2] * bb[2];
      const double e2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
      phi = 4.5 * w * (0.5 * b2 * e2 - eb * eb - (h->D == 3 ? b2 / 6.0 : 0.0));
    }
    for (int k = 0; k < 3; ++k) {
      // rest-state part of 2 f_out: 2 (w rho0 + phi(B0)) per link (the stored
      // deviations exclude both)
      stat[k] += (double)nl * 2.0 * (w * h->rho0 + phi) * e[k];
      mx[k] += -(double)nl * 2.0 * e[k] * phi;
    }
  }
  for (int k = 0; k < 3; ++k) {
    raw[k] = fscale * (s[k] + stat[k]);
    mf[k] = fscale * (h->last_uw[gr][k] / h->c) * s[3];
    mx[k] *= fscale;
    out[0][k] = raw[k];
    out[1][k] = raw[k] + mf[k];
    out[2][k] = raw[k] + mx[k];
    out[3][k] = raw[k] + mf[k] + mx[k];
  }
}

int lbm_wall_force(lbm_ctx* h, double* out) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->have_step) return fail(LBM_ESTATE, "no step taken yet");
  if (!out) return fail(LBM_EINVAL, "null buffer");
  for (int gr = 0; gr < h->G; ++gr) {
    double v[4][3];
    wall_variants(h, gr, v);
    for (int var = 0; var < 4; ++var)
      for (int k = 0; k < 3; ++k) out[(gr * 4 + var) * 3 + k] = v[var][k];
  }
  return LBM_OK;
}

int lbm_set_wall_force_history(lbm_ctx* h, int on) {
  if (!h) return fail(LBM_EINVAL, "null context");
  if (on && !h->geom_ok) {
    int rc = build_geometry(h);
    if (rc) return rc;
  }
  h->hist_on = on != 0;
  return LBM_OK;
}

int lbm_wall_force_history(lbm_ctx* h, double* out, int max_steps, int* nsteps) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!out || !nsteps) return fail(LBM_EINVAL, "null buffer");
  if (max_steps < 0) return fail(LBM_EINVAL, "negative max_steps");
  if (!h->have_step || !h->hist_steps) return fail(LBM_ESTATE, "no call with the history on since the state was set");
  const int n = (int)std::min<long>(h->hist_steps, max_steps);
  for (int st = 0; st < n; ++st)
    for (int gr = 0; gr < h->G; ++gr) {
      double v[4][3];
      wall_variants(h, gr, v, h->hist.data() + (size_t)st * MAXG * NWALL);
      for (int var = 0; var < 4; ++var)
        for (int k = 0; k < 3; ++k) out[(((size_t)st * h->G + gr) * 4 + var) * 3 + k] = v[var][k];
    }
  *nsteps = n;
  return LBM_OK;
}

int lbm_force_balance(lbm_ctx* h, double* out) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->have_step) return fail(LBM_ESTATE, "no step taken yet");
  if (!out) return fail(LBM_EINVAL, "null buffer");
  DiagArgs a = diag_args(h);
  a.part = (double*)h->dpart.p;
  rc = run_diag(h, a);
  if (rc) return rc;
  HIPCHK(launch_reduce((const double*)h->dpart.p, nullptr, h->ntiles, 1, 0, NDIAGPART, (double*)h->dred.p, h->stream));
  double* dr = h->hred + NBAL + MAXG * NWALL;
  HIPCHK(hipMemcpyAsync(dr, h->dred.p, NDIAGPART * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const double V = vol(h), c = h->c, dt = h->dt;
  const double M1 = V * ((double)h->nfluid * h->rho0 + dr[0]);
  const double M0 = V * ((double)h->nfluid * h->rho0 + h->last[0]);
  std::memset(out, 0, sizeof(double) * LBM_NREC);
  double Fraw[3] = {0, 0, 0}, Fmf[3] = {0, 0, 0}, Fmx[3] = {0, 0, 0};
  for (int gr = 0; gr < h->G; ++gr) {
    double v[4][3];
    wall_variants(h, gr, v);
    for (int k = 0; k < 3; ++k) {
      Fraw[k] += v[0][k];
      Fmf[k] += v[1][k] - v[0][k];
      Fmx[k] += v[2][k] - v[0][k];
    }
  }
  for (int k = 0; k < 3; ++k) {
    const double bt = V * c / dt * h->last[4 + k];
    const double dP = V * c * (dr[1 + k] - h->last[1 + k]) / dt;
    out[0 + k] = Fraw[k];
    out[3 + k] = bt;
    out[6 + k] = dP;
    out[9 + k] = bt - Fraw[k] - dP;
    out[12 + k] = Fmx[k];
    out[15 + k] = Fmf[k];
    out[18 + k] = dr[4 + k];
  }
  out[21] = M1;
  out[22] = V * (dr[0] - h->last[0]);
  out[23] = (double)h->steps;
  (void)M0;
  return LBM_OK;
}

int lbm_num_groups(lbm_ctx* h) {
  if (!h) return fail(LBM_EINVAL, "null context");
  if (!h->geom_ok) {
    int rc = build_geometry(h);
    if (rc) return rc;
  }
  return h->G;
}

long lbm_link_count(lbm_ctx* h, int group) {
  if (!h) return fail(LBM_EINVAL, "null context");
  if (!h->geom_ok) {
    int rc = build_geometry(h);
    if (rc) return rc;
  }
  long s = 0;
  for (int gr = 0; gr < MAXG; ++gr) {
    if (group >= 0 && gr != group) continue;
    for (int q = 0; q < h->Q; ++q) s += h->nlink[(size_t)gr * h->Q + q];
  }
  return s;
}

static int adjoint_supported(lbm_ctx* h) {
  if (h->prec != S_F32 && h->prec != S_F64) return fail(LBM_EINVAL, "the adjoint needs F32 or F64 storage");
  if (h->mhd) return fail(LBM_EINVAL, "the adjoint does not cover the MHD equilibrium");
  if (h->cs > 0) return fail(LBM_EINVAL, "the adjoint does not cover the Smagorinsky closure");
  return LBM_OK;
}

int lbm_adjoint_forward(lbm_ctx* h, int T, int ckpt_every, int group, int axis, double* J) {
  int rc = check_ready(h);
  if (rc) return rc;
  rc = adjoint_supported(h);
  if (rc) return rc;
  if (T < 1) return fail(LBM_EINVAL, "T must be >= 1");
  if (ckpt_every < 0) return fail(LBM_EINVAL, "ckpt_every must be >= 0");
  if (group < 0 || group >= h->G) return fail(LBM_EINVAL, "group %d is not a wall group in use", group);
  if (axis < 0 || axis >= h->D) return fail(LBM_EINVAL, "axis %d out of range", axis);
  if (!J) return fail(LBM_EINVAL, "null J");
  h->tape = false;
  const int par0 = h->parity;
  if (ckpt_every > 0) {
    const int nseg = (T + ckpt_every - 1) / ckpt_every;
    const size_t sbytes = (size_t)h->Q * h->N * elem_bytes(h->prec);
    HIPCHK(h->ckpt.ensure((size_t)nseg * sbytes));
    rc = step_loop(h, T, ckpt_every);
  } else {
    HIPCHK(h->mac.ensure((size_t)T * 4 * h->N * elem_bytes(h->prec)));
    rc = step_loop(h, T, 0, h->mac.p);
  }
  if (rc) return rc;
  double v[4][3];
  wall_variants(h, group, v);
  *J = v[0][axis];
  h->tape = true;
  h->tape_T = T;
  h->tape_K = ckpt_every;
  h->tape_group = group;
  h->tape_axis = axis;
  h->tape_par0 = par0;
  return LBM_OK;
}

int lbm_adjoint_backward(lbm_ctx* h, double gJ, void* grad_a_dev, int grad_f64, double* grad_uw) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->tape) return fail(LBM_ESTATE, "no recorded run: call lbm_adjoint_forward first (set-up changes and steps discard it)");
  if (!std::isfinite(gJ)) return fail(LBM_EINVAL, "non-finite gJ");
  const int T = h->tape_T, K = h->tape_K;
  const int nseg = K > 0 ? (T + K - 1) / K : 1;
  const size_t eb = elem_bytes(h->prec);
  const size_t sbytes = (size_t)h->Q * h->N * eb;
  const size_t mbytes = (size_t)4 * h->N * eb;
  const int ap = h->prec == S_F64 ? S_F64 : h->adj_prec;
  if (K > 0) {
    HIPCHK(h->replay.ensure(sbytes));
    HIPCHK(h->mac.ensure((size_t)std::min(K, T) * mbytes));
  }
  HIPCHK(h->lam.ensure((size_t)h->Q * h->N * elem_bytes(ap)));
  HIPCHK(h->adjpart.ensure((size_t)h->ntiles * NPART * sizeof(double)));
  HIPCHK(h->adjred.ensure((NBAL + MAXG * NWALL) * sizeof(double)));
  rc = upload_uw(h);
  if (rc) return rc;
  const size_t gbytes = (size_t)3 * h->N * (grad_f64 ? sizeof(double) : sizeof(float));
  if (grad_a_dev) HIPCHK(hipMemsetAsync(grad_a_dev, 0, gbytes, h->stream));
  HIPCHK(hipMemsetAsync(h->adjpart.p, 0, (size_t)h->ntiles * NPART * sizeof(double), h->stream));
  // the objective's step adds its seed to what the adjoint state holds
  HIPCHK(hipMemsetAsync(h->lam.p, 0, (size_t)h->Q * h->N * elem_bytes(ap), h->stream));
  const size_t ibytes = (size_t)h->nibb * h->Q * sizeof(double);
  IbbArgs ib = {};
  IbbAdjArgs ia = {};
  if (h->nibb) {
    HIPCHK(h->ibb_dd1.ensure(ibytes));
    HIPCHK(h->ibb_sacc.ensure(ibytes));
    HIPCHK(hipMemsetAsync(h->ibb_sacc.p, 0, ibytes, h->stream));
    ib.f = h->replay.p;
    ib.node = ia.node = (const uint32_t*)h->ibb_node.p;
    ib.qf = ia.qf = (const double*)h->ibb_q.p;
    ib.grp = (const uint8_t*)h->ibb_grp.p;
    ib.nrec = ia.nrec = (const uint4*)h->ibb_rec.p;
    for (int gr = 0; gr < MAXG; ++gr)
      for (int k = 0; k < 3; ++k) ib.uw[gr][k] = ia.uw[gr][k] = h->uw[gr][k] / h->c;
    ib.M = ia.M = h->nibb;
    ia.lam = h->lam.p;
    ia.dd1 = (double*)h->ibb_dd1.p;
    ia.sacc = (double*)h->ibb_sacc.p;
    ia.seed_axis = h->tape_axis;
  }
  const double fscale = vol(h) * h->c / h->dt;  // force units of the unit-seed objective
  StepArgs sa = step_args(h);
  sa.f = h->replay.p;
  AdjArgs aa = {};
  aa.lam = h->lam.p;
  aa.afield = h->afield;
  aa.rec = (const uint4*)h->rec.p;
  aa.rowrec = (const int*)h->rowrec.p;
  aa.blkgrp = (const uint32_t*)h->blkgrp.p;
  aa.uw = (const double*)h->uwdev.p;
  aa.grad_a = grad_a_dev;
  aa.grad_f64 = grad_f64 ? 1 : 0;
  aa.part = (double*)h->adjpart.p;
  aa.ga_scale = gJ * fscale * h->dt / h->c;
  aa.seed_group = h->tape_group;
  aa.seed_axis = h->tape_axis;
  aa.tperm = h->use_tperm ? (const uint32_t*)h->tperm.p : nullptr;  // the even steps' order
  aa.geo = sa.geo;
  aa.p = sa.p;
  ib.geo = ia.geo = sa.geo;
  ib.p = sa.p;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int t0 = K > 0 ? seg * K : 0, t1 = K > 0 ? std::min(T, t0 + K) : T;
    if (K > 0) {
      // recompute the segment from its checkpoint, recording rho and U
      HIPCHK(hipMemcpyAsync(h->replay.p, (char*)h->ckpt.p + (size_t)seg * sbytes, sbytes, hipMemcpyDeviceToDevice,
                            h->stream));
      for (int t = t0; t < t1; ++t) {
        sa.mac = (char*)h->mac.p + (size_t)(t - t0) * mbytes;
        HIPCHK(launch_step_mac(h->lattice, h->prec, sa, (h->tape_par0 + t) & 1, false, h->stream));
        if (h->nibb) {
          ib.parity = ((h->tape_par0 + t) & 1) ^ 1;
          HIPCHK(launch_ibb(h->lattice, h->prec, ib, h->stream));
        }
      }
    }
    // then reverse its steps (the interpolation pass first, then the step)
    for (int t = t1 - 1; t >= t0; --t) {
      aa.mac = (const char*)h->mac.p + (size_t)(t - t0) * mbytes;
      if (h->nibb) {
        ia.mac = aa.mac;
        ia.parity = ((h->tape_par0 + t) & 1) ^ 1;
        ia.seed_group = t == T - 1 ? h->tape_group : -1;
        HIPCHK(launch_ibb_adj(h->lattice, h->prec, ap, ia, h->stream));
      }
      HIPCHK(launch_adj(h->lattice, h->prec, ap, aa, (h->tape_par0 + t) & 1, t == T - 1, h->stream));
    }
  }
  double* hr = h->hred + NBAL + MAXG * NWALL + NDIAGPART;
  HIPCHK(launch_reduce((const double*)h->adjpart.p, (const uint32_t*)h->wlist.p, h->ntiles, 0, h->G, NBAL + MAXG * NWALL,
                       (double*)h->adjred.p, h->stream));
  HIPCHK(hipMemcpyAsync(hr, h->adjred.p, (NBAL + MAXG * NWALL) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  // the interpolation pass's wall-velocity cotangents, per link along e_q
  double* ir = hr + NBAL + MAXG * NWALL;
  if (h->nibb) {
    HIPCHK(launch_ibb_reduce(h->lattice, (const double*)h->ibb_sacc.p, (const uint8_t*)h->ibb_grp.p, h->nibb, h->G,
                             (double*)h->ibb_part.p, (double*)h->ibb_red.p, h->stream));
    HIPCHK(hipMemcpyAsync(ir, h->ibb_red.p, (size_t)h->G * 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  if (grad_uw) {
    const double su = gJ * fscale / h->c;
    for (int gr = 0; gr < h->G; ++gr)
      for (int k = 0; k < 3; ++k)
        grad_uw[3 * gr + k] =
            k < h->D ? su * (hr[NBAL + gr * NWALL + k] + (h->nibb ? ir[gr * 4 + k] : 0.0)) : 0.0;
  }
  return LBM_OK;
}

int lbm_set_adjoint_precision(lbm_ctx* h, int precision) {
  if (!h) return fail(LBM_EINVAL, "null context");
  if (precision != LBM_F64 && precision != LBM_F32) return fail(LBM_EINVAL, "adjoint precision must be LBM_F64 or LBM_F32");
  if (precision == LBM_F32 && h->prec == S_F64) return fail(LBM_EINVAL, "an FP64 lattice keeps an FP64 adjoint");
  h->adj_prec = precision;
  return LBM_OK;
}

int lbm_set_timing(lbm_ctx* h, int on) {
  if (!h) return fail(LBM_EINVAL, "null context");
  h->timing = on != 0;
  return LBM_OK;
}

int lbm_step_timings(lbm_ctx* h, double* out) {
  if (!h) return fail(LBM_EINVAL, "null context");
  if (!out) return fail(LBM_EINVAL, "null buffer");
  for (int k = 0; k < 6; ++k) out[k] = h->tim[k];
  return LBM_OK;
}

long lbm_steps_taken(lbm_ctx* h) {
  if (!h) return fail(LBM_EINVAL, "null context");
  return h->steps;
}

}  // extern "C"
