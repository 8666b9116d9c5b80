// Kernel argument blocks shared by the host library and the device kernels.
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

namespace lbm {

enum { S_F64 = 0, S_F32 = 1, S_F16 = 2, S_BF16 = 3 };
constexpr int MAXG = 16;   // wall groups per context
constexpr int MAXBG = 4;   // distinct wall groups inside one 256-node tile
constexpr int NTHREADS = 256;
constexpr int NBAL = 7;                    // sum drho, sum rho U (3), sum rho A (3)
constexpr int NWALL = 4;                   // sum e (2 d_rel + ladd) (3), sum ladd
constexpr int NPART = NBAL + MAXBG * NWALL;  // per-tile partial sums on diagnostic steps
constexpr int NDIAGPART = 8;               // sum drho, sum rho U (3), stress integral (3), pad

// Index geometry.  Nodes are numbered n = (z ny + y) nx + x = row nx + x; an
// array with P planes stores element (q, row, x) at (row P + q) nx + x.
struct Geom {
  uint32_t nx, ny, nz, N;
  uint64_t mnx, mny;  // ceil(2^64 / d) for exact division by nx, ny (unused when d == 1)
};

// Physical parameters, all dimensionless (velocities in units of c).
struct Phys {
  double rho0;
  double tau0, inv_tau0;
  double A[3];         // uniform a dt / c
  double afield_scale; // dt / c, applied to the per-node field a
  double kF, lF0, lF1, lEq, cG, thC;  // force-model table (see host)
  double les_K;        // 18 sqrt(2) C_s^2, 0 = no closure
  double quad;         // 1: equilibrium of Eq. (1); 0: Stokes form (no quadratic velocity terms)
  double darcy_s;      // porous resistance sigma dt (0 = none)
  double darcy_inv;    // 1 / (1 + sigma dt / 2)
  double b0[3];        // MHD B0 / (c sqrt(mu))
  double inv_tau_m;
  double tm_theta;     // tau_m theta of the induction lattice (Lorentz-force coupling)
  float scale[19], inv_scale[19];  // storage scaling per direction
  // the same parameters rounded to FP32 by the host, so that FP32 kernels
  // read them from scalar registers instead of converting them per thread
  struct {
    float rho0, tau0, inv_tau0, A[3], afield_scale, kF, lF0, lF1, lEq, cG, thC, les_K, quad, darcy_s, darcy_inv;
    float b0[3], inv_tau_m, tm_theta;
  } f;
};

struct StepArgs {
  void* f;                 // distributions, row-blocked [ny nz][Q][nx]
  void* g;                 // induction deviations, row-blocked [ny nz][K NB][nx] (MHD) or null
  const float* afield;     // [3][N] or null
  const uint4* rec;        // boundary records: x = solid-link mask (bit 31: node solid), y..w = group nibbles;
                           // w >> 12: 1 + index in the list of nodes with interpolated links (0: none)
  const int* rowrec;       // per row: index of the row's first record, or -1
  const uint32_t* blkgrp;  // per tile: up to MAXBG group labels, 4 bits each, + count in bits 28..31
  const double* uw;        // [MAXG][3] wall velocity / c
  double* part;            // [ntiles][NPART] on diagnostic steps
  void* mac;               // [4][N] rho, U of the pre-step state (adjoint recompute), or null
  float* sig;              // [NC][N] stress of the pre-step state (Eq. 8), FP32, or null
  float* strain;           // [NC][N] strain rate (Eq. 9), FP32, or null
  float st_c2, st_hdt;     // c^2 and 3 / (2 dt) of the stress and strain outputs
  int st_artefact;         // include the artefact term E in them
  double* hist;            // per-step ring slot [MAXBG NWALL][nwt] of the wall-link sums (diagnostics mode 1)
  const int* wtile;        // per tile: compact index among the tiles a wall group meets, or -1
  uint32_t nwt;            // number of such tiles
  // links to walls that are not halfway (nodes with rec.w >> 12 != 0)
  const double* ibq;       // [M][Q] wall distance / link length of each listed node
  int ibb_in;              // the state holds 2q f_rel + ladd at their q < 1/2 links: complete it at the read
  int ibb_out;             // interpolate at their links in the step (q < 1/2: the part known at x)
  int plain_loads;         // FP32 odd steps read interior rows with plain (cached) loads
  const uint32_t* tperm;   // [2][ntiles] tile of each workgroup, even / odd steps (boundary rows first), or null
  Geom geo;
  Phys p;
};

// Arguments of the adjoint step kernel (reverse of one forward step).
struct AdjArgs {
  void* lam;               // adjoint state, same type and layout as the distributions
  const void* mac;         // [4][N] rho, U of the forward state before this step
  const float* afield;     // [3][N] or null
  const uint4* rec;
  const int* rowrec;
  const uint32_t* blkgrp;
  const double* uw;        // [MAXG][3] wall velocity / c
  void* grad_a;            // [3][N] float or double (grad_f64), accumulated; or null
  double* part;            // [ntiles][NPART], wall-velocity cotangents accumulated in the wall slots
  double ga_scale;         // factor from the node's force cotangent to grad_a
  int grad_f64;
  int seed_group, seed_axis;  // objective (last forward step only)
  const uint32_t* tperm;   // [ntiles] tile of each workgroup (tiles with boundary rows first), or null
  Geom geo;
  Phys p;
};

// Arguments of the read-only diagnostic kernel.
struct DiagArgs {
  const void* f;
  const void* g;
  const float* afield;
  const uint4* rec;
  const int* rowrec;
  double* rho;     // [N] or null
  double* vel;     // [D][N] or null (v = u + dt a / 2, physical units)
  double* sigma;   // [NC][N] or null
  double* strain;  // [NC][N] or null
  double* B;       // [3][N] or null
  double* state;   // [Q][N] natural-layout deviations or null
  double* gstate;  // [21][N] absolute induction distributions or null
  double* part;    // [ntiles][NDIAGPART] or null
  Geom geo;
  Phys p;
  int parity;
  int artefact;
  double c, dt;
  int wall_lo[3], wall_hi[3];  // plane walls present per axis end (stress integral)
  double area;                 // dx^(D-1)
};

// Interpolated bounce-back after a step, for walls that are not halfway: one
// entry per fluid node with such links.
struct IbbArgs {
  void* f;                 // state at t + dt, in the layout the next step reads
  const uint32_t* node;    // [M] node index
  const double* qf;        // [M][Q] wall distance / link length (1/2: halfway, left as is)
  const uint8_t* grp;      // [M][Q] wall group of each link
  double* delta;           // [M][Q] change of the returning value (diagnostic steps), or null
  double* half;            // [M][Q] the halfway values the step returned (last step of a call), or null
  const uint4* nrec;       // [M] boundary record of each listed node (wall mask, group nibbles)
  double uw[MAXG][3];      // wall velocities / c of the step
  uint32_t M;
  Geom geo;
  Phys p;
  int parity;              // parity of the next step
};

// Transposed interpolation pass of the adjoint (walls that are not halfway).
struct IbbAdjArgs {
  void* lam;               // adjoint state, type and layout of AdjArgs::lam
  const void* mac;         // [4][N] rho, U of the forward step being reversed (rho read)
  const uint32_t* node;    // [M] node index
  const double* qf;        // [M][Q] wall distance / link length
  const uint4* nrec;       // [M] boundary record of each listed node
  double* dd1;             // [M][Q] cotangents of the streamed values the q < 1/2 links read
  double* sacc;            // [M][Q] wall-velocity cotangent of each link along e_q, accumulated
  double uw[MAXG][3];      // wall velocities / c
  uint32_t M;
  Geom geo;
  int parity;              // parity of the step after the reversed one (that of the forward pass)
  int seed_group, seed_axis;  // objective on the last forward step; seed_group < 0 on the others
};

// Half-step distribution of the last step (Section 5, Eq. 27).
struct HalfArgs {
  const void* f;        // state at t + dt, in the layout the next step reads
  const void* g;
  const uint4* rec;
  const int* rowrec;
  double* fbar;         // [Q][N] f_bar - w rho0, or null
  double* rho;          // [N] or null
  double* vel;          // [D][N] u_bar (physical), or null
  double* sigma;        // [NC][N] -sum e e f_bar + Mbar^eq (physical), or null
  const double* ibb_half;  // [M][Q] halfway values of the last step at nodes with interpolated links, or null
  double uw[MAXG][3];   // wall velocities / c of the last step
  Geom geo;
  Phys p;
  int parity;           // parity of the next step
  double c;
};

// Initial-state / upload kernel arguments.
struct InitArgs {
  void* f;
  void* g;
  const double* u0;    // [D][N] physical u, or null
  const double* state; // [Q][N] deviations to upload, or null
  const uint4* rec;
  const int* rowrec;
  Geom geo;
  Phys p;
  double inv_c;
};

}  // namespace lbm
