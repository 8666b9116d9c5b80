/*
 * Plain CPU reference ("oracle") for the LBM hot path of arXiv 2512.12213.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product library.
 *
 * Straightforward two-array push scheme in double precision (or double complex
 * for complex-step derivatives), one node at a time, in the order of the
 * paper's Section 2:
 *   moments -> model velocities -> (Smagorinsky tau) -> equilibrium (Eq. 1 /
 *   Eq. 10) -> force term (Section 2 / Eq. 3) -> relaxation (Eq. 2) ->
 *   propagation with halfway bounce-back -> momentum exchange (Eq. 25).
 * Distributions are held as deviations d = f - w*rho0 (a change of variable
 * only; it keeps FP64 round-off small when f is close to w*rho0).
 *
 * Every function is a direct transcription of the formula it cites; there is
 * no blocking, fusion or reordering beyond per-row partial sums that make the
 * reductions independent of the thread count.
 *
 * Parity status: pinned by the closed-form and invariant tests in the test
 * suite (moment identities, model equivalences, exact-bounce-back channel
 * profiles, the 1D class-sum recurrence, momentum and mass balances, Maxwell
 * per-link sums, Hartmann channel, Smagorinsky fixed point, finite differences
 * for the complex-step build).
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORC_COMPLEX
#include <complex.h>
typedef double complex real;
#define RSQRT(x) csqrt(x)
#define RE(x) creal(x)
#define IM(x) cimag(x)
#define MK(re, im) ((re) + (im) * I)
#else
typedef double real;
#define RSQRT(x) sqrt(x)
#define RE(x) (x)
#define IM(x) (0.0 * (x))
#define MK(re, im) (re)
#endif

#define MAXG 16
#define NREC 24

struct orc {
  int lat, D, Q;
  int nx, ny, nz;
  long N;
  double tau, dx, dt, c;
  int model;
  double rho0;
  int e[19][3]; /* unit lattice vectors; the lattice velocity is c * e */
  double w[19];
  int opp[19];
  int wall[3][2];       /* group of the plane wall at the low / high end of an axis; -1 periodic */
  unsigned char* solid; /* per node: 0 fluid, 1 + group for a solid node */
  int G;                /* number of link groups in use */
  real uw[MAXG][3];
  real a[3];
  real* afield; /* [3][N] or NULL */
  double cs;
  int stokes;   /* 1: equilibrium without the quadratic velocity terms (text after Eq. 11) */
  double darcy; /* porous resistance sigma: body force -sigma v added to a (Brinkman) */
  int artefact;
  int mhd;
  int lorentz;  /* MHD coupling: 0 magnetic stress in the equilibrium (Eq. 10), 1 Lorentz force as a body force */
  int K;        /* induction directions: 7 (D3Q7) or 5 (its planar restriction) */
  double B0[3], mu, tau_m;
  real *g, *gn; /* induction distributions less W_k B0, [K][3][N] */
  real *d, *dn; /* [Q][N] deviations f - w rho0 (- phi(B0) under the MHD equilibrium) */
  real* rel;     /* [Q][N] relaxed values f_rel(x, t) of the last step, before propagation */
  real* rho_t;   /* [N] density of the last step's pre-step state */
  double* qlink; /* [Q][N] wall distance / link length for wall links, or NULL (all 1/2) */
  real* Bt;      /* [3][N] B(x, t) - B0 before the last step (MHD) */
  /* records of the last executed step */
  real wf[MAXG][3][3]; /* per group: raw, momentum-flux correction, Maxwell correction */
  real M_t, P_t[3], rho_a[3];
  long step;
  int have_step;
};

/* ---------------------------------------------------------------------------
 * Lattices (Section 2; velocity sets and weights of Qian, d'Humieres and
 * Lallemand 1992).  Direction order is the documented state-exchange order.
 * ------------------------------------------------------------------------- */
static void set_lattice(orc* o) {
  static const int e9[9][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
  static const int e19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                 {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                 {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                 {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  memset(o->e, 0, sizeof(o->e));
  if (o->lat == 0) {
    o->D = 2;
    o->Q = 9;
    for (int q = 0; q < 9; ++q) {
      o->e[q][0] = e9[q][0];
      o->e[q][1] = e9[q][1];
      int s = abs(e9[q][0]) + abs(e9[q][1]);
      o->w[q] = s == 0 ? 4.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  } else {
    o->D = 3;
    o->Q = 19;
    for (int q = 0; q < 19; ++q) {
      int s = 0;
      for (int k = 0; k < 3; ++k) {
        o->e[q][k] = e19[q][k];
        s += abs(e19[q][k]);
      }
      o->w[q] = s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
  }
  for (int q = 0; q < o->Q; ++q)
    for (int p = 0; p < o->Q; ++p)
      if (o->e[p][0] == -o->e[q][0] && o->e[p][1] == -o->e[q][1] && o->e[p][2] == -o->e[q][2]) o->opp[q] = p;
}

/* D3Q7 lattice of the induction solver: weights 1/4 (rest) and 1/8, so that
 * sum_k W_k e_k e_k = theta c^2 I with theta = 1/4.  Two-dimensional flows use
 * its restriction to the plane (directions 0-4): the two z links fold into
 * the rest direction, weights 1/2 and 1/8, the same theta and therefore the
 * same magnetic diffusivity eta = theta c^2 dt (tau_m - 1/2). */
static const int e7[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const int opp7[7] = {0, 2, 1, 4, 3, 6, 5};
static double w7(const orc* o, int k) { return k == 0 ? (o->lat == 0 ? 0.5 : 0.25) : 0.125; }
#define THETA7 0.25

orc* orc_create(int lattice, int nx, int ny, int nz, double tau, double dx, double dt, int model) {
  if (lattice != 0 && lattice != 1) return NULL;
  if (nx < 1 || ny < 1 || nz < 1) return NULL;
  if (lattice == 0 && nz != 1) return NULL;
  if (!(tau > 0.5) || !(dx > 0) || !(dt > 0)) return NULL;
  if (model < 0 || model > 6) return NULL;
  orc* o = (orc*)calloc(1, sizeof(orc));
  o->lat = lattice;
  set_lattice(o);
  o->nx = nx;
  o->ny = ny;
  o->nz = nz;
  o->N = (long)nx * ny * nz;
  o->tau = tau;
  o->dx = dx;
  o->dt = dt;
  o->c = dx / dt;
  o->model = model;
  o->rho0 = 1.0;
  for (int k = 0; k < 3; ++k) o->wall[k][0] = o->wall[k][1] = -1;
  o->G = 1;
  o->solid = (unsigned char*)calloc(o->N, 1);
  o->d = (real*)calloc((size_t)o->Q * o->N, sizeof(real));
  o->dn = (real*)calloc((size_t)o->Q * o->N, sizeof(real));
  o->rel = (real*)calloc((size_t)o->Q * o->N, sizeof(real));
  o->Bt = (real*)calloc((size_t)3 * o->N, sizeof(real));
  o->rho_t = (real*)calloc((size_t)o->N, sizeof(real));
  return o;
}

void orc_destroy(orc* o) {
  if (!o) return;
  free(o->solid);
  free(o->d);
  free(o->dn);
  free(o->rel);
  free(o->Bt);
  free(o->rho_t);
  free(o->qlink);
  free(o->afield);
  free(o->g);
  free(o->gn);
  free(o);
}

int orc_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int orc_set_rho0(orc* o, double rho0) {
  if (!(rho0 > 0)) return -1;
  o->rho0 = rho0;
  return 0;
}

static void note_group(orc* o, int g) {
  if (g + 1 > o->G) o->G = g + 1;
}

int orc_set_walls(orc* o, int axis, int glo, int ghi) {
  if (axis < 0 || axis >= o->D) return -1;
  if (glo >= MAXG || ghi >= MAXG || glo < -1 || ghi < -1) return -1;
  o->wall[axis][0] = glo;
  o->wall[axis][1] = ghi;
  if (glo >= 0) note_group(o, glo);
  if (ghi >= 0) note_group(o, ghi);
  return 0;
}

int orc_set_solid(orc* o, const unsigned char* mask, int group) {
  if (group < 0 || group >= MAXG) return -1;
  for (long i = 0; i < o->N; ++i)
    if (mask[i]) o->solid[i] = (unsigned char)(1 + group);
  note_group(o, group);
  return 0;
}

int orc_set_wall_velocity(orc* o, int group, const double* u, const double* u_im) {
  if (group < 0 || group >= MAXG) return -1;
  /* a two-dimensional lattice has no z component */
  for (int k = 0; k < 3; ++k) o->uw[group][k] = k < o->D ? MK(u[k], u_im ? u_im[k] : 0.0) : 0.0;
  note_group(o, group);
  return 0;
}

int orc_set_body_force(orc* o, const double* a, const double* a_im) {
  for (int k = 0; k < 3; ++k) o->a[k] = k < o->D ? MK(a[k], a_im ? a_im[k] : 0.0) : 0.0;
  return 0;
}

int orc_set_body_force_field(orc* o, const double* a, const double* a_im) {
  free(o->afield);
  o->afield = NULL;
  if (!a) return 0;
  o->afield = (real*)malloc(sizeof(real) * 3 * o->N);
  for (long i = 0; i < 3 * o->N; ++i) o->afield[i] = MK(a[i], a_im ? a_im[i] : 0.0);
  return 0;
}

int orc_set_les(orc* o, double cs) {
  if (cs < 0) return -1;
  o->cs = cs;
  return 0;
}

/* Wall position per link for interpolated bounce-back: q[a][n] is the
 * distance from fluid node n to the wall along link a, as a fraction of the
 * link; 1/2 is the halfway wall.  Values of non-wall links are ignored. */
int orc_set_link_fraction(orc* o, const double* q) {
  if (!q) {
    free(o->qlink);
    o->qlink = NULL;
    return 0;
  }
  if (!o->qlink) o->qlink = (double*)malloc(sizeof(double) * o->Q * o->N);
  for (long i = 0; i < (long)o->Q * o->N; ++i) {
    if (!(q[i] > 0.0 && q[i] <= 1.0)) return -1;
    o->qlink[i] = q[i];
  }
  return 0;
}

static double link_fraction(const orc* o, int q, long idx) { return o->qlink ? o->qlink[(long)q * o->N + idx] : 0.5; }

int orc_set_equilibrium(orc* o, int stokes) {
  o->stokes = stokes ? 1 : 0;
  return 0;
}

int orc_set_darcy(orc* o, double sigma) {
  if (!(sigma >= 0) || (sigma > 0 && o->lorentz)) return -1;
  o->darcy = sigma;
  return 0;
}

int orc_set_artefact(orc* o, int on) {
  o->artefact = on ? 1 : 0;
  return 0;
}

int orc_set_mhd(orc* o, double B0x, double B0y, double B0z, double mu, double tau_m) {
  if (!(mu > 0) || !(tau_m > 0.5)) return -1;
  if (o->lat == 0 && B0z != 0.0) return -1; /* planar field in two dimensions */
  o->mhd = 1;
  o->K = o->lat == 0 ? 5 : 7;
  o->B0[0] = B0x;
  o->B0[1] = B0y;
  o->B0[2] = B0z;
  o->mu = mu;
  o->tau_m = tau_m;
  free(o->g);
  free(o->gn);
  o->g = (real*)calloc((size_t)3 * o->K * o->N, sizeof(real));
  o->gn = (real*)calloc((size_t)3 * o->K * o->N, sizeof(real));
  return 0;
}

/* 1: the Lorentz force enters through the force term and the equilibrium
 * stays hydrodynamic (the third approach of Section 4; the text after Eq. 36
 * gives its balance); 0: the paper's approach, magnetic stress in f^eq. */
int orc_set_lorentz_force(orc* o, int on) {
  if (!o->mhd || (on && o->darcy > 0)) return -1;
  o->lorentz = on ? 1 : 0;
  return 0;
}

/* ---------------------------------------------------------------------------
 * Local formulas
 * ------------------------------------------------------------------------- */
static real edot(const orc* o, int q, const real* v) {
  real s = 0;
  for (int k = 0; k < o->D; ++k) s += (real)(o->c * o->e[q][k]) * v[k];
  return s;
}

/* Equilibrium of Eq. (1), as a deviation from w*rho0; drho = rho - rho0.
 * The Stokes form (text after Eq. 11) keeps only the linear term
 * rho w [1 + 3 e.u / c^2]. */
static real feq_dev(const orc* o, int q, real rho, real drho, const real* u) {
  const double c2 = o->c * o->c;
  real eu = edot(o, q, u);
  if (o->stokes) return o->w[q] * (drho + rho * 3.0 * eu / c2);
  real uu = 0;
  for (int k = 0; k < o->D; ++k) uu += u[k] * u[k];
  return o->w[q] * (drho + rho * (3.0 * eu / c2 + 4.5 * eu * eu / (c2 * c2) - 1.5 * uu / c2));
}

/* Magnetic part of the MHD equilibrium, Eq. (10); two-dimensional flows
 * leave out its -c^2 B^2 / 6 term (the text after Eq. 10). */
static real phi_mhd(const orc* o, int q, const real* B) {
  const double c2 = o->c * o->c;
  real ee = 0, eB = 0, B2 = 0;
  for (int k = 0; k < 3; ++k) {
    ee += (real)(c2 * o->e[q][k] * o->e[q][k]);
    eB += (real)(o->c * o->e[q][k]) * B[k];
    B2 += B[k] * B[k];
  }
  real last = o->lat == 1 ? c2 * B2 / 6.0 : 0.0;
  return 9.0 * o->w[q] / (2.0 * c2 * c2 * o->mu) * (0.5 * B2 * ee - eB * eB - last);
}

/* Is the magnetic stress carried by the equilibrium (Eq. 10)? */
static int mhd_eq(const orc* o) { return o->mhd && !o->lorentz; }


/* The rest state in the uniform field B0 is kept outside the stored
 * variables, a change of variable only (as the deviation from w rho0): the
 * distributions are held as f - w rho0 - phi(B0) under the MHD equilibrium,
 * and the induction distributions as g_k - W_k B0, so that the small induced
 * parts are never rounded at the size of B0.  phi0 is that magnetic part of
 * the rest equilibrium (zero unless the equilibrium carries Eq. 10). */
static real phi0(const orc* o, int q) {
  if (!mhd_eq(o)) return 0.0;
  real B0[3] = {o->B0[0], o->B0[1], o->B0[2]};
  return phi_mhd(o, q, B0);
}

/* phi(B0 + b) - phi(B0) of Eq. (10), expanded in the induced field b: with
 * s = 2 B0 + b, B^2 - B0^2 = b.s and (e.B)^2 - (e.B0)^2 = (e.b)(e.s). */
static real phi_change(const orc* o, int q, const real* b) {
  const double c2 = o->c * o->c;
  real ee = 0, eb = 0, es = 0, bs = 0;
  for (int k = 0; k < 3; ++k) {
    real sk = 2.0 * o->B0[k] + b[k];
    ee += (real)(c2 * o->e[q][k] * o->e[q][k]);
    eb += (real)(o->c * o->e[q][k]) * b[k];
    es += (real)(o->c * o->e[q][k]) * sk;
    bs += b[k] * sk;
  }
  real last = o->lat == 1 ? c2 * bs / 6.0 : 0.0;
  return 9.0 * o->w[q] / (2.0 * c2 * c2 * o->mu) * (0.5 * bs * ee - eb * es - last);
}

/* L(B0 + b) - L(B0) of the Maxwell stress after Eq. (11),
 * L_ij(B) = (B^2 delta_ij / 2 - B_i B_j) / mu, expanded in b:
 * B^2 - B0^2 = b.s and B_i B_j - B0_i B0_j = (b_i s_j + s_i b_j) / 2, s = 2 B0 + b. */
static real maxwell_change(const orc* o, int i, int j, const real* b) {
  real s[3], bs = 0;
  for (int k = 0; k < 3; ++k) {
    s[k] = 2.0 * o->B0[k] + b[k];
    bs += b[k] * s[k];
  }
  return ((i == j ? 0.5 * bs : 0.0) - 0.5 * (b[i] * s[j] + s[i] * b[j])) / o->mu;
}

static real body_force(const orc* o, long idx, int k) {
  if (o->afield) return o->afield[(long)k * o->N + idx];
  return o->a[k];
}

/* Per-node state needed by the collision and by the diagnostics. */
typedef struct {
  real rho, drho, u[3], v[3], a[3], ueq[3], uF[3], B[3];
  real b[3];   /* induced field B - B0 */
  real C;      /* force-term coefficient */
  real tau;    /* relaxation time in use (Smagorinsky or molecular) */
  real Pi[3][3]; /* non-equilibrium second moment, Pi^neq */
  real F[19];  /* force term per direction */
  real E[3][3];  /* artefact term E_ij of Eq. (9) */
} node_t;

/* Lorentz force per unit mass a_L = J x B / rho, J = curl B / mu, when it
 * enters through the force term.  curl B comes from the first moment of the
 * induction distributions, Lambda_lm = sum_k c e_kl g_km, whose equilibrium
 * part is v_l B_m - B_l v_m and whose non-equilibrium part is, to first
 * order in the Chapman-Enskog expansion (as Pi^neq for the flow),
 * -tau_m dt theta c^2 d_l B_m.  With lambda_i = eps_ilm Lambda_lm and
 * kappa = tau_m dt theta c^2 this reads mu kappa J = -lambda + 2 v x B.  The
 * velocity v = u* + dt a_L / 2 (u* = u + dt a_ext / 2) holds J itself, which
 * makes it the linear system
 *   [mu kappa I + (dt / rho) (B^2 I - B B^T)] J = -lambda + 2 u* x B,
 * solved here by Gaussian elimination with partial pivoting. */
static void lorentz_accel(const orc* o, real rho, const real* ustar, const real* B, const real* lam, real* aL) {
  const double kappa = o->tau_m * o->dt * THETA7 * o->c * o->c;
  real B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  real A[3][4];
  real uxB[3] = {ustar[1] * B[2] - ustar[2] * B[1], ustar[2] * B[0] - ustar[0] * B[2], ustar[0] * B[1] - ustar[1] * B[0]};
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) A[i][j] = (i == j ? o->mu * kappa + o->dt / rho * B2 : 0.0) - o->dt / rho * B[i] * B[j];
    A[i][3] = -lam[i] + 2.0 * uxB[i];
  }
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (fabs(RE(A[r][col])) > fabs(RE(A[piv][col]))) piv = r;
    if (piv != col)
      for (int j = 0; j < 4; ++j) {
        real t = A[col][j];
        A[col][j] = A[piv][j];
        A[piv][j] = t;
      }
    for (int r = col + 1; r < 3; ++r) {
      real f = A[r][col] / A[col][col];
      for (int j = col; j < 4; ++j) A[r][j] -= f * A[col][j];
    }
  }
  real J[3];
  for (int i = 2; i >= 0; --i) {
    real v = A[i][3];
    for (int j = i + 1; j < 3; ++j) v -= A[i][j] * J[j];
    J[i] = v / A[i][i];
  }
  aL[0] = (J[1] * B[2] - J[2] * B[1]) / rho;
  aL[1] = (J[2] * B[0] - J[0] * B[2]) / rho;
  aL[2] = (J[0] * B[1] - J[1] * B[0]) / rho;
}

/* Moments, model velocities, Pi^neq, Smagorinsky tau, force term.  gl: the
 * node's induction distributions [K][3] (MHD) or NULL.  a_node, when not
 * NULL, replaces the node's body force (used to differentiate with respect
 * to it). */
static void node_setup(const orc* o, const real* dl, long idx, const real (*gl)[3], const real* a_node, node_t* s) {
  const int D = o->D, Q = o->Q;
  const double c = o->c, c2 = c * c, dt = o->dt;
  memset(s, 0, sizeof(*s));
  /* rho = sum f, rho u = sum e f (Section 2); with f = d + w rho0 and
   * sum w = 1, rho - rho0 = sum d exactly, which is kept as such */
  real drho = 0, j[3] = {0, 0, 0};
  for (int q = 0; q < Q; ++q) {
    drho += dl[q];
    for (int k = 0; k < D; ++k) j[k] += (real)(c * o->e[q][k]) * dl[q];
  }
  real rho = o->rho0 + drho;
  s->rho = rho;
  s->drho = drho;
  for (int k = 0; k < 3; ++k) {
    s->b[k] = 0;
    if (gl)
      for (int m = 0; m < o->K; ++m) s->b[k] += gl[m][k]; /* B - B0 = sum_k (g_k - W_k B0) */
    s->B[k] = (gl ? o->B0[k] : 0.0) + s->b[k];
  }
  for (int k = 0; k < 3; ++k) {
    s->u[k] = k < D ? j[k] / rho : 0;
    s->a[k] = k < D ? (a_node ? a_node[k] : body_force(o, idx, k)) : 0;
    /* porous resistance -sigma v with v = u + dt a / 2, a including it:
     * a = (a_ext - sigma u) / (1 + sigma dt / 2) */
    if (o->darcy > 0) s->a[k] = (s->a[k] - o->darcy * s->u[k]) / (1.0 + 0.5 * o->darcy * dt);
  }
  if (o->mhd && o->lorentz && gl) {
    real Lam[3][3] = {{0}}, lam[3], us[3], aL[3];
    for (int m = 0; m < o->K; ++m)
      for (int l = 0; l < 3; ++l)
        for (int n = 0; n < 3; ++n) Lam[l][n] += (real)(c * e7[m][l]) * gl[m][n];
    lam[0] = Lam[1][2] - Lam[2][1];
    lam[1] = Lam[2][0] - Lam[0][2];
    lam[2] = Lam[0][1] - Lam[1][0];
    for (int k = 0; k < 3; ++k) us[k] = s->u[k] + 0.5 * dt * s->a[k];
    lorentz_accel(o, rho, us, s->B, lam, aL);
    for (int k = 0; k < D; ++k) s->a[k] += aL[k];
  }
  for (int k = 0; k < 3; ++k) s->v[k] = s->u[k] + 0.5 * dt * s->a[k]; /* v = u + dt a / 2 for all models */
  /* u^eq per model (Section 2): [e] uses v, the original Shan-Chen form uses
   * u + tau dt a, all others use u. */
  for (int k = 0; k < 3; ++k) {
    if (o->model == 4)
      s->ueq[k] = s->v[k];
    else if (o->model == 5)
      s->ueq[k] = s->u[k] + o->tau * dt * s->a[k];
    else
      s->ueq[k] = s->u[k];
  }
  /* Pi^neq = sum e e f - (p delta + rho u^eq u^eq + L) (cheap form after
   * Eq. 9, with the Maxwell stress that Eq. 11 puts in M^eq_ij).  The stored
   * second moment lacks that of phi(B0), which is L(B0), so L(B) - L(B0) is
   * subtracted. */
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k) {
      real m = 0;
      for (int q = 0; q < Q; ++q) m += (real)(c2 * o->e[q][i] * o->e[q][k]) * dl[q];
      real eqm = (i == k ? drho * c2 / 3.0 : 0.0) + (o->stokes ? 0.0 : rho * s->ueq[i] * s->ueq[k]);
      if (mhd_eq(o)) eqm += maxwell_change(o, i, k, s->b);
      s->Pi[i][k] = m - eqm;
    }
  /* Smagorinsky closure (C_s > 0): nu_eff = nu0 + (C_s dx)^2 |S| with
   * |S| = sqrt(2 S:S) and S from Eq. (9) at the same tau_eff; with
   * nu = dt c^2 (tau - 1/2) / 3 this is the quadratic
   *   tau^2 - tau0 tau - 9 sqrt(2) (C_s dx)^2 Q / (2 rho c^4 dt^2) = 0,
   * Q = sqrt(Pi:Pi), whose positive root is taken. */
  s->tau = o->tau;
  if (o->cs > 0) {
    real PP = 0;
    for (int i = 0; i < D; ++i)
      for (int k = 0; k < D; ++k) PP += s->Pi[i][k] * s->Pi[i][k];
    real Qn = RSQRT(PP);
    double l2 = (o->cs * o->dx) * (o->cs * o->dx);
    s->tau = 0.5 * (o->tau + RSQRT(o->tau * o->tau + 18.0 * sqrt(2.0) * l2 * Qn / (rho * c2 * c2 * dt * dt)));
  }
  /* u^F and C per model (Section 2) */
  s->C = 1.0;
  for (int k = 0; k < 3; ++k) {
    switch (o->model) {
      case 1: s->uF[k] = s->u[k]; break;                                   /* [b] */
      case 2: s->uF[k] = s->u[k] + 0.5 * s->tau * dt * s->a[k]; break;   /* [c] */
      case 3: s->uF[k] = s->v[k]; break;                                   /* [d] */
      case 4: s->uF[k] = s->v[k]; break;                                   /* [e] */
      default: s->uF[k] = 0; break;
    }
  }
  if (o->model == 4) s->C = 1.0 - 1.0 / (2.0 * s->tau);
  /* force term */
  for (int q = 0; q < Q; ++q) {
    real ea = edot(o, q, s->a);
    if (o->model == 0) {
      /* [a] He et al.: F = rho w 3 e.a dt / c^2 */
      s->F[q] = rho * o->w[q] * 3.0 * ea * dt / c2;
    } else if (o->model >= 1 && o->model <= 4) {
      /* Eq. (3): F = C rho w [3 (e - u^F)/c^2 + 9 (e.u^F) e / c^4] . a dt */
      real uFa = 0;
      for (int k = 0; k < D; ++k) uFa += s->uF[k] * s->a[k];
      real euF = edot(o, q, s->uF);
      s->F[q] = s->C * rho * o->w[q] * (3.0 * (ea - uFa) / c2 + 9.0 * euF * ea / (c2 * c2)) * dt;
    } else if (o->model == 6) {
      /* original exact-difference form: F = feq(rho, u + dt a) - feq(rho, u) */
      real us[3];
      for (int k = 0; k < 3; ++k) us[k] = s->u[k] + dt * s->a[k];
      s->F[q] = feq_dev(o, q, rho, drho, us) - feq_dev(o, q, rho, drho, s->u);
    } else {
      s->F[q] = 0; /* original Shan-Chen: no force term */
    }
  }
  /* artefact term of Eq. (9): E = tau dt (u^eq_i rho a_j + u^eq_j rho a_i) - tau Theta_ij,
   * Theta_ij = sum e_i e_j F (Eq. 4) */
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k) {
      real th = 0;
      for (int q = 0; q < Q; ++q) th += (real)(c2 * o->e[q][i] * o->e[q][k]) * s->F[q];
      /* with the Stokes equilibrium M^eq has no rho u u part, whose time
       * derivative gives the u^eq a terms */
      real ua = o->stokes ? 0.0 : s->tau * dt * (s->ueq[i] * rho * s->a[k] + s->ueq[k] * rho * s->a[i]);
      s->E[i][k] = ua - s->tau * th;
    }
}

/* Where does the link from node (x,y,z) along direction e end?
 * Returns 0 and the target index for a fluid target (periodic wrap), or 1 and
 * the link group for a link that ends in a wall or solid node.  A link that
 * crosses plane walls of two axes (a corner) belongs to the lowest such axis. */
static int link_target(const orc* o, int x, int y, int z, const int* e, long* tidx, int* grp) {
  int p[3] = {x + e[0], y + e[1], z + e[2]};
  int n[3] = {o->nx, o->ny, o->nz};
  for (int k = 0; k < 3; ++k) {
    if (p[k] < 0 || p[k] >= n[k]) {
      int side = p[k] < 0 ? 0 : 1;
      if (o->wall[k][side] >= 0) {
        *grp = o->wall[k][side];
        return 1;
      }
      p[k] = (p[k] + n[k]) % n[k];
    }
  }
  long t = ((long)p[2] * o->ny + p[1]) * o->nx + p[0];
  if (o->solid[t]) {
    *grp = o->solid[t] - 1;
    return 1;
  }
  *tidx = t;
  return 0;
}

/* ---------------------------------------------------------------------------
 * Initial state
 * ------------------------------------------------------------------------- */
int orc_init_equilibrium(orc* o, const double* u0) {
  const long N = o->N;
  for (long i = 0; i < N; ++i) {
    real u[3] = {0, 0, 0};
    if (u0)
      for (int k = 0; k < o->D; ++k) u[k] = u0[(long)k * N + i];
    /* f^eq(rho0, u0) (+ phi(B0), outside the stored deviation) and
     * g^eq(B0, u0) less W B0 */
    real B[3] = {o->B0[0], o->B0[1], o->B0[2]};
    for (int q = 0; q < o->Q; ++q) o->d[(long)q * N + i] = o->solid[i] ? 0 : feq_dev(o, q, o->rho0, 0.0, u);
    if (o->mhd) {
      for (int k = 0; k < o->K; ++k)
        for (int c = 0; c < 3; ++c) {
          real geq = 0;
          if (!o->solid[i])
            for (int m = 0; m < 3; ++m)
              geq += w7(o, k) * (e7[k][m] / (THETA7 * o->c)) * (u[m] * B[c] - B[m] * u[c]);
          o->g[((long)k * 3 + c) * N + i] = geq;
        }
    }
  }
  o->step = 0;
  o->have_step = 0;
  return 0;
}

/* States are exchanged as f - w rho0 [Q][N] (phi(B0) included; solid
 * nodes as given). */
int orc_set_state(orc* o, const double* d, const double* d_im) {
  for (long i = 0; i < (long)o->Q * o->N; ++i)
    o->d[i] = MK(d[i], d_im ? d_im[i] : 0.0) - (o->solid[i % o->N] ? 0.0 : phi0(o, (int)(i / o->N)));
  o->have_step = 0;
  return 0;
}

/* Replace the state without forgetting the records of the last step. */
int orc_replace_state(orc* o, const double* d) {
  for (long i = 0; i < (long)o->Q * o->N; ++i)
    o->d[i] = MK(d[i], 0.0) - (o->solid[i % o->N] ? 0.0 : phi0(o, (int)(i / o->N)));
  return 0;
}

int orc_get_state(const orc* o, double* d, double* d_im) {
  for (long i = 0; i < (long)o->Q * o->N; ++i) {
    d[i] = RE(o->d[i] + (o->solid[i % o->N] ? 0.0 : phi0(o, (int)(i / o->N))));
    if (d_im) d_im[i] = IM(o->d[i]);
  }
  return 0;
}

/* Absolute induction distributions g [K][3][N] (solid nodes read 0). */
int orc_get_induction(const orc* o, double* g) {
  if (!o->mhd) return -1;
  for (int k = 0; k < o->K; ++k)
    for (int m = 0; m < 3; ++m)
      for (long i = 0; i < o->N; ++i) {
        long j = ((long)k * 3 + m) * o->N + i;
        g[j] = o->solid[i] ? 0.0 : RE(o->g[j] + w7(o, k) * o->B0[m]);
      }
  return 0;
}

/* ---------------------------------------------------------------------------
 * One time step
 * ------------------------------------------------------------------------- */
/* per-row partial sums: [G][3][3] wall force, then M, P[3], rho_a[3], then
 * [G][Q] the number of wall links of each group and direction */
static int part_size(const orc* o) { return o->G * 9 + 7 + o->G * o->Q; }
static int count_slot(const orc* o, int grp, int q) { return o->G * 9 + 7 + grp * o->Q + q; }

/* Eq. (25) with f = d + c_a, c_a = w_a rho0 + phi_a(B0) the rest-state
 * populations: each link contributes e_a (f_out + f_in) = e_a (d_out + d_in)
 * + 2 e_a c_a (c_a is the same for a and its opposite).  The deviation parts
 * are summed link by link; the rest-state parts, large next to the force on
 * a body and cancelling between its sides, are summed exactly as integer
 * link counts per direction and its opposite, then weighted (an FP64 sum of
 * the absolute populations loses about 1e-12 of the force on a small
 * sphere).  The momentum-flux term has no rest-state part (f_out - f_in =
 * d_out - d_in). */
static void add_rest_state_part(const orc* o, const real* tot, real* wf_raw, int grp) {
  const double vol = o->lat == 0 ? o->dx * o->dx : o->dx * o->dx * o->dx;
  for (int q = 1; q < o->Q; ++q) {
    const int qb = o->opp[q];
    if (qb < q) continue;
    const real n = tot[count_slot(o, grp, q)] - tot[count_slot(o, grp, qb)];
    if (n == 0) continue;
    const real ca = o->w[q] * o->rho0 + phi0(o, q);
    for (int k = 0; k < 3; ++k) wf_raw[k] += vol / o->dt * 2.0 * (o->c * o->e[q][k]) * ca * n;
  }
}

/* Everything of one node's update before propagation: node_setup, then the
 * relaxation of Eq. (2), drel = d + (d^eq - d)/tau + F, with the equilibrium
 * of Eq. (1) (+ the magnetic term of Eq. 10). */
static void node_relax(const orc* o, const real* dl, long idx, const real (*gl)[3], const real* a_node, node_t* s,
                       real* drel) {
  node_setup(o, dl, idx, gl, a_node, s);
  for (int q = 0; q < o->Q; ++q) {
    real deq = feq_dev(o, q, s->rho, s->drho, s->ueq);
    if (mhd_eq(o)) deq += phi_change(o, q, s->b); /* phi(B) less the stored phi(B0) */
    drel[q] = dl[q] + (deq - dl[q]) / s->tau + s->F[q];
  }
}

/* Moving wall (halfway bounce-back, Ladd): the population returning along
 * opp(q) gains 6 w_q rho (e_opp(q) . u_w) / c^2. */
static real moving_wall_term(const orc* o, int q, real rho, const real* uw) {
  return 6.0 * o->w[q] * rho * edot(o, o->opp[q], uw) / (o->c * o->c);
}

static void update_node(orc* o, int x, int y, int z, real* part) {
  const int D = o->D, Q = o->Q;
  const long N = o->N;
  const double c = o->c, c2 = c * c, dt = o->dt;
  const double vol = o->lat == 0 ? o->dx * o->dx : o->dx * o->dx * o->dx; /* dx^D */
  const long idx = ((long)z * o->ny + y) * o->nx + x;
  real dl[19], drel[19];
  for (int q = 0; q < Q; ++q) dl[q] = o->d[(long)q * N + idx];
  real gl[7][3];
  if (o->mhd)
    for (int k = 0; k < o->K; ++k)
      for (int m = 0; m < 3; ++m) gl[k][m] = o->g[((long)k * 3 + m) * N + idx];
  node_t s;
  node_relax(o, dl, idx, o->mhd ? (const real(*)[3])gl : NULL, NULL, &s, drel);
  /* kept for the half-step distribution of Eq. (27) and for interpolated
   * bounce-back */
  for (int q = 0; q < Q; ++q) o->rel[(long)q * N + idx] = drel[q];
  o->rho_t[idx] = s.rho;
  for (int k = 0; k < 3; ++k) o->Bt[(long)k * N + idx] = s.b[k];

  /* balance partials at time t (Eq. 32): mass, momentum, body force */
  real* pb = part + o->G * 9;
  pb[0] += vol * s.rho;
  for (int k = 0; k < 3; ++k) {
    pb[1 + k] += vol * s.rho * s.u[k];
    pb[4 + k] += vol * s.rho * s.a[k];
  }

  /* propagation with halfway bounce-back and momentum exchange */
  for (int q = 0; q < Q; ++q) {
    long t;
    int grp;
    if (!link_target(o, x, y, z, o->e[q], &t, &grp)) {
      o->dn[(long)q * N + t] = drel[q];
      continue;
    }
    /* a wall that is not halfway: bounce-back by interpolation after all
     * nodes have relaxed (interpolated_bounce_back) */
    if (link_fraction(o, q, idx) != 0.5) continue;
    const int qb = o->opp[q];
    real ladd = moving_wall_term(o, q, s.rho, o->uw[grp]);
    o->dn[(long)qb * N + idx] = drel[q] + ladd;
    /* Eq. (25): outgoing f_bar = f_rel(x_f, t), incoming f_bar = f(x_f, t + dt),
     * as deviations (rest-state part: add_rest_state_part) */
    real dout = drel[q];
    real din = dout + ladd;
    real* pw = part + grp * 9;
    for (int k = 0; k < 3; ++k) {
      double ek = c * o->e[q][k], ebk = c * o->e[qb][k];
      pw[k] += vol / dt * (ek * dout - ebk * din);          /* raw momentum exchange */
      pw[3 + k] += -vol / dt * o->uw[grp][k] * (dout - din); /* minus momentum flux */
    }
    part[count_slot(o, grp, q)] += 1;
    if (mhd_eq(o)) {
      /* minus Maxwell stress: the magnetic part of the equilibrium at the wall
       * field carried by both populations of the link */
      real Bw[3] = {o->B0[0], o->B0[1], o->B0[2]};
      real ph = phi_mhd(o, q, Bw);
      for (int k = 0; k < 3; ++k) pw[6 + k] += -vol / dt * 2.0 * (c * o->e[q][k]) * ph;
    }
  }

  /* induction lattice (D3Q7 vector distributions, B Dirichlet on walls) */
  if (o->mhd) {
    for (int k = 0; k < o->K; ++k) {
      real grel[3];
      for (int m = 0; m < 3; ++m) {
        /* g^eq_k(B, v) = W_k [B + (e_k / (theta c)).(v B - B v)], less W_k B0 */
        real geq = w7(o, k) * s.b[m];
        for (int j = 0; j < 3; ++j)
          geq += w7(o, k) * (e7[k][j] / (THETA7 * c)) * (s.v[j] * s.B[m] - s.B[j] * s.v[m]);
        grel[m] = gl[k][m] + (geq - gl[k][m]) / o->tau_m;
      }
      long t;
      int grp;
      if (!link_target(o, x, y, z, e7[k], &t, &grp)) {
        for (int m = 0; m < 3; ++m) o->gn[((long)k * 3 + m) * N + t] = grel[m];
      } else {
        /* anti-bounce-back imposing B = B0 at the halfway wall:
         * g_kb(x_f, t + dt) = -g_rel_k(x_f, t) + 2 W_k B0; less W_kb B0 = W_k B0
         * on both sides this is -(g_rel_k - W_k B0) */
        int kb = opp7[k];
        for (int m = 0; m < 3; ++m) o->gn[((long)kb * 3 + m) * N + idx] = -grel[m];
      }
    }
  }
  (void)D;
}

/* Linearly interpolated bounce-back (Bouzidi, Firdaouss and Lallemand 2001)
 * for a wall at fraction qv of link a from fluid node x (a value of 1/2 is the
 * halfway wall of Section 5, handled in update_node):
 *   qv <  1/2: f_opp(a)(x, t+dt) = 2qv f_rel_a(x) + (1 - 2qv) f_rel_a(x - e_a)
 *              (+ the moving-wall term), halfway bounce-back when x - e_a is
 *              not a fluid node;
 *   qv >= 1/2: f_opp(a)(x, t+dt) = f_rel_a(x) / (2qv) + (2qv - 1)/(2qv) f_rel_opp(a)(x)
 *              (+ the moving-wall term / (2qv)).
 * Deviations from w rho0 obey the same formulas (the weights sum to one).  The
 * momentum exchange of Eq. (25) uses the values that leave and return at x,
 * so its result is the stress at x + e_a dt / 2 (Section 5), not at the wall.
 * Adds the links' wall-force contributions to tot (layout of part_size). */
static void interpolated_bounce_back(orc* o, real* tot) {
  const int Q = o->Q;
  const long N = o->N;
  const double c = o->c, dt = o->dt;
  const double vol = o->lat == 0 ? o->dx * o->dx : o->dx * o->dx * o->dx;
  for (int z = 0; z < o->nz; ++z)
    for (int y = 0; y < o->ny; ++y)
      for (int x = 0; x < o->nx; ++x) {
        const long idx = ((long)z * o->ny + y) * o->nx + x;
        if (o->solid[idx]) continue;
        for (int q = 1; q < Q; ++q) {
          long t;
          int grp;
          if (!link_target(o, x, y, z, o->e[q], &t, &grp)) continue;
          const double qv = link_fraction(o, q, idx);
          if (qv == 0.5) continue;
          const int qb = o->opp[q];
          const real rq = o->rel[(long)q * N + idx];
          const real ladd = moving_wall_term(o, q, o->rho_t[idx], o->uw[grp]);
          real din;
          if (qv < 0.5) {
            int back[3] = {-o->e[q][0], -o->e[q][1], -o->e[q][2]};
            long tu;
            int gu;
            if (!link_target(o, x, y, z, back, &tu, &gu))
              din = 2.0 * qv * rq + (1.0 - 2.0 * qv) * o->rel[(long)q * N + tu] + ladd;
            else
              din = rq + ladd;
          } else {
            din = rq / (2.0 * qv) + (2.0 * qv - 1.0) / (2.0 * qv) * o->rel[(long)qb * N + idx] + ladd / (2.0 * qv);
          }
          o->dn[(long)qb * N + idx] = din;
          /* deviations (rest-state part: add_rest_state_part) */
          real* pw = tot + grp * 9;
          for (int k = 0; k < 3; ++k) {
            double ek = c * o->e[q][k], ebk = c * o->e[qb][k];
            pw[k] += vol / dt * (ek * rq - ebk * din);
            pw[3 + k] += -vol / dt * o->uw[grp][k] * (rq - din);
          }
          tot[count_slot(o, grp, q)] += 1;
          if (mhd_eq(o)) {
            /* minus Maxwell stress, per link as at a halfway wall: both
             * populations of the link carry the magnetic part of the
             * equilibrium at the wall field B0 */
            real Bw[3] = {o->B0[0], o->B0[1], o->B0[2]};
            real ph = phi_mhd(o, q, Bw);
            for (int k = 0; k < 3; ++k) pw[6 + k] += -vol / dt * 2.0 * (c * o->e[q][k]) * ph;
          }
        }
      }
}

int orc_step(orc* o, int n) {
  if (n < 0) return -1;
  const int P = part_size(o);
  const long rows = (long)o->ny * o->nz;
  real* part = (real*)malloc(sizeof(real) * P * rows);
  for (int it = 0; it < n; ++it) {
    memset(part, 0, sizeof(real) * P * rows);
#pragma omp parallel for schedule(static)
    for (long r = 0; r < rows; ++r) {
      int y = (int)(r % o->ny), z = (int)(r / o->ny);
      real* pr = part + r * P;
      for (int x = 0; x < o->nx; ++x) {
        long idx = ((long)z * o->ny + y) * o->nx + x;
        if (o->solid[idx]) continue;
        update_node(o, x, y, z, pr);
      }
    }
    /* row partials summed in row order */
    real tot[MAXG * 9 + 7 + MAXG * 19];
    memset(tot, 0, sizeof(tot));
    for (long r = 0; r < rows; ++r)
      for (int k = 0; k < P; ++k) tot[k] += part[r * P + k];
    if (o->qlink) interpolated_bounce_back(o, tot);
    for (int gr = 0; gr < o->G; ++gr) add_rest_state_part(o, tot, tot + gr * 9, gr);
    for (int gr = 0; gr < o->G; ++gr)
      for (int v = 0; v < 3; ++v)
        for (int k = 0; k < 3; ++k) o->wf[gr][v][k] = tot[gr * 9 + v * 3 + k];
    o->M_t = tot[o->G * 9];
    for (int k = 0; k < 3; ++k) {
      o->P_t[k] = tot[o->G * 9 + 1 + k];
      o->rho_a[k] = tot[o->G * 9 + 4 + k];
    }
    real* t = o->d;
    o->d = o->dn;
    o->dn = t;
    if (o->mhd) {
      t = o->g;
      o->g = o->gn;
      o->gn = t;
    }
    o->step++;
    o->have_step = 1;
  }
  free(part);
  return 0;
}

/* ---------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------- */
/* Induced field B - B0 = sum_k (g_k - W_k B0) of a node. */
static void node_b(const orc* o, long idx, real* b) {
  b[0] = b[1] = b[2] = 0;
  if (!o->mhd) return;
  for (int k = 0; k < o->K; ++k)
    for (int m = 0; m < 3; ++m) b[m] += o->g[((long)k * 3 + m) * o->N + idx];
}

/* The node's induction distributions [K][3]; NULL without MHD. */
static const real (*load_g(const orc* o, long idx, real gl[7][3]))[3] {
  if (!o->mhd) return NULL;
  for (int k = 0; k < o->K; ++k)
    for (int m = 0; m < 3; ++m) gl[k][m] = o->g[((long)k * 3 + m) * o->N + idx];
  return (const real(*)[3])gl;
}

static void load_node(const orc* o, long idx, real* dl) {
  for (int q = 0; q < o->Q; ++q) dl[q] = o->d[(long)q * o->N + idx];
}

int orc_get_macro(const orc* o, double* rho, double* v, double* B) {
  for (long i = 0; i < o->N; ++i) {
    if (o->solid[i]) {
      rho[i] = 0;
      for (int k = 0; k < o->D; ++k) v[(long)k * o->N + i] = 0;
      if (B)
        for (int k = 0; k < 3; ++k) B[(long)k * o->N + i] = 0;
      continue;
    }
    real dl[19], gl[7][3];
    load_node(o, i, dl);
    node_t s;
    node_setup(o, dl, i, load_g(o, i, gl), NULL, &s);
    rho[i] = RE(s.rho);
    for (int k = 0; k < o->D; ++k) v[(long)k * o->N + i] = RE(s.v[k]);
    if (B)
      for (int k = 0; k < 3; ++k) B[(long)k * o->N + i] = RE(s.B[k]);
  }
  return 0;
}

/* Eq. (8)-(9): S = -3 / (2 tau dt c^2 rho) (Pi^neq [+ E]),  sigma = 2 rho nu S
 * with nu = dt c^2 (tau - 1/2) / 3, tau the relaxation time in use. */
static void node_stress(const orc* o, const node_t* s, real sig[3][3], real S[3][3]) {
  const double c2 = o->c * o->c, dt = o->dt;
  real nu = dt * c2 * (s->tau - 0.5) / 3.0;
  for (int i = 0; i < o->D; ++i)
    for (int k = 0; k < o->D; ++k) {
      real P = s->Pi[i][k] + (o->artefact ? s->E[i][k] : 0.0);
      S[i][k] = -3.0 / (2.0 * s->tau * dt * c2 * s->rho) * P;
      sig[i][k] = 2.0 * s->rho * nu * S[i][k];
    }
}

static const int comp2[3][2] = {{0, 0}, {0, 1}, {1, 1}};
static const int comp3[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};

int orc_stress(const orc* o, double* sigma, double* strain) {
  const int nc = o->D == 2 ? 3 : 6;
  for (long i = 0; i < o->N; ++i) {
    real sig[3][3], S[3][3];
    memset(sig, 0, sizeof(sig));
    memset(S, 0, sizeof(S));
    if (!o->solid[i]) {
      real dl[19], gl[7][3];
      load_node(o, i, dl);
      node_t s;
      node_setup(o, dl, i, load_g(o, i, gl), NULL, &s);
      node_stress(o, &s, sig, S);
    }
    for (int m = 0; m < nc; ++m) {
      int a = o->D == 2 ? comp2[m][0] : comp3[m][0];
      int b = o->D == 2 ? comp2[m][1] : comp3[m][1];
      if (sigma) sigma[(long)m * o->N + i] = RE(sig[a][b]);
      if (strain) strain[(long)m * o->N + i] = RE(S[a][b]);
    }
  }
  return 0;
}

int orc_wall_force(const orc* o, double* out, double* out_im, int G) {
  for (int gr = 0; gr < G; ++gr) {
    for (int k = 0; k < 3; ++k) {
      real raw = gr < o->G ? o->wf[gr][0][k] : 0;
      real mf = gr < o->G ? o->wf[gr][1][k] : 0;
      real mx = gr < o->G ? o->wf[gr][2][k] : 0;
      real v[4] = {raw, raw + mf, raw + mx, raw + mf + mx};
      for (int var = 0; var < 4; ++var) {
        out[(gr * 4 + var) * 3 + k] = RE(v[var]);
        if (out_im) out_im[(gr * 4 + var) * 3 + k] = IM(v[var]);
      }
    }
  }
  return 0;
}

long orc_link_count(const orc* o, int group) {
  long n = 0;
  for (int z = 0; z < o->nz; ++z)
    for (int y = 0; y < o->ny; ++y)
      for (int x = 0; x < o->nx; ++x) {
        long idx = ((long)z * o->ny + y) * o->nx + x;
        if (o->solid[idx]) continue;
        for (int q = 0; q < o->Q; ++q) {
          long t;
          int grp;
          if (link_target(o, x, y, z, o->e[q], &t, &grp) && (group < 0 || grp == group)) ++n;
        }
      }
  return n;
}

/* Surface sum of (-p delta + sigma) n over the plane walls, with p and sigma
 * extrapolated linearly from the first two fluid layers to the halfway wall
 * (the stress form of the wall force, Eqs. 26, 28 and 33). */
static void stress_integral(const orc* o, real* F) {
  const double c2 = o->c * o->c;
  const double area = o->lat == 0 ? o->dx : o->dx * o->dx;
  int n[3] = {o->nx, o->ny, o->nz};
  F[0] = F[1] = F[2] = 0;
  for (int ax = 0; ax < o->D; ++ax) {
    if (n[ax] < 2) continue;
    for (int side = 0; side < 2; ++side) {
      if (o->wall[ax][side] < 0) continue;
      int l0 = side == 0 ? 0 : n[ax] - 1, l1 = side == 0 ? 1 : n[ax] - 2;
      double nrm = side == 0 ? 1.0 : -1.0; /* inward normal component along ax */
      for (int z = 0; z < o->nz; ++z)
        for (int y = 0; y < o->ny; ++y)
          for (int x = 0; x < o->nx; ++x) {
            int p[3] = {x, y, z};
            if (p[ax] != l0) continue;
            long i0 = ((long)z * o->ny + y) * o->nx + x;
            p[ax] = l1;
            long i1 = ((long)p[2] * o->ny + p[1]) * o->nx + p[0];
            if (o->solid[i0] || o->solid[i1]) continue;
            real T[2][3][3];
            long ids[2] = {i0, i1};
            for (int l = 0; l < 2; ++l) {
              real dl[19], gl[7][3], sig[3][3], S[3][3];
              load_node(o, ids[l], dl);
              node_t s;
              node_setup(o, dl, ids[l], load_g(o, ids[l], gl), NULL, &s);
              memset(sig, 0, sizeof(sig));
              node_stress(o, &s, sig, S);
              for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k) T[l][i][k] = sig[i][k] - (i == k && i < o->D ? s.rho * c2 / 3.0 : 0.0);
            }
            for (int i = 0; i < o->D; ++i) F[i] += area * (1.5 * T[0][i][ax] - 0.5 * T[1][i][ax]) * nrm;
          }
    }
  }
}

int orc_force_balance(const orc* o, double* out) {
  memset(out, 0, sizeof(double) * NREC);
  const double vol = o->lat == 0 ? o->dx * o->dx : o->dx * o->dx * o->dx;
  /* moments of the current state, time t + dt */
  real M1 = 0, P1[3] = {0, 0, 0};
  for (long i = 0; i < o->N; ++i) {
    if (o->solid[i]) continue;
    real rho = o->rho0, j[3] = {0, 0, 0};
    for (int q = 0; q < o->Q; ++q) {
      real dq = o->d[(long)q * o->N + i];
      rho += dq;
      for (int k = 0; k < o->D; ++k) j[k] += (real)(o->c * o->e[q][k]) * dq;
    }
    M1 += vol * rho;
    for (int k = 0; k < 3; ++k) P1[k] += vol * j[k];
  }
  real Fsi[3];
  stress_integral(o, Fsi);
  for (int k = 0; k < 3; ++k) {
    real raw = 0, mx = 0, mf = 0;
    for (int gr = 0; gr < o->G; ++gr) {
      raw += o->wf[gr][0][k];
      mf += o->wf[gr][1][k];
      mx += o->wf[gr][2][k];
    }
    real dP = o->have_step ? (P1[k] - o->P_t[k]) / o->dt : 0;
    out[0 + k] = RE(raw);
    out[3 + k] = RE(o->rho_a[k]);
    out[6 + k] = RE(dP);
    out[9 + k] = RE(o->rho_a[k] - raw - dP);
    out[12 + k] = RE(mx);
    out[15 + k] = RE(mf);
    out[18 + k] = RE(Fsi[k]);
  }
  out[21] = RE(M1);
  out[22] = o->have_step ? RE(M1 - o->M_t) : 0;
  out[23] = (double)o->step;
  return 0;
}

/* ---------------------------------------------------------------------------
 * Half-step distribution (Section 5, Eqs. 27-28)
 * ---------------------------------------------------------------------------
 * fbar = (f_rel(x, t) + f(x, t + dt)) / 2 of the last step (Eq. 27), as a
 * deviation from w rho0; its density, velocity and the stress of Eq. (28):
 *   sigma_bar_ij = -sum_a e_ai e_aj fbar_a + Mbar^eq_ij,
 *   Mbar^eq_ij = pbar delta_ij + rhobar ubar_i ubar_j (+ L_ij(Bbar) under MHD),
 * pbar = rhobar c^2 / 3, Bbar = (B(t) + B(t + dt)) / 2 (the induction
 * distributions interpolated the same way; relaxation conserves B).
 * Any output may be NULL; solid nodes read 0.  -1 before the first step. */
int orc_halfstep(const orc* o, double* fbar, double* rho_bar, double* u_bar, double* sigma_bar) {
  if (!o->have_step) return -1;
  const int D = o->D, Q = o->Q;
  const long N = o->N;
  const double c = o->c, c2 = c * c;
  const int nc = D == 2 ? 3 : 6;
  const int (*comp)[2] = D == 2 ? comp2 : comp3;
  for (long i = 0; i < N; ++i) {
    real db[19];
    for (int q = 0; q < Q; ++q) db[q] = o->solid[i] ? 0 : 0.5 * (o->rel[(long)q * N + i] + o->d[(long)q * N + i]);
    if (fbar)
      for (int q = 0; q < Q; ++q) fbar[(long)q * N + i] = o->solid[i] ? 0.0 : RE(db[q] + phi0(o, q));
    if (o->solid[i]) {
      if (rho_bar) rho_bar[i] = 0;
      if (u_bar)
        for (int k = 0; k < D; ++k) u_bar[(long)k * N + i] = 0;
      if (sigma_bar)
        for (int m = 0; m < nc; ++m) sigma_bar[(long)m * N + i] = 0;
      continue;
    }
    real drho = 0, j[3] = {0, 0, 0};
    for (int q = 0; q < Q; ++q) {
      drho += db[q];
      for (int k = 0; k < D; ++k) j[k] += (real)(c * o->e[q][k]) * db[q];
    }
    real rho = o->rho0 + drho, u[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) u[k] = j[k] / rho;
    if (rho_bar) rho_bar[i] = RE(rho);
    if (u_bar)
      for (int k = 0; k < D; ++k) u_bar[(long)k * N + i] = RE(u[k]);
    if (sigma_bar) {
      real bbar[3] = {0, 0, 0}; /* Bbar - B0 */
      if (o->mhd) {
        real bn[3];
        node_b(o, i, bn);
        for (int k = 0; k < 3; ++k) bbar[k] = 0.5 * (o->Bt[(long)k * N + i] + bn[k]);
      }
      for (int m = 0; m < nc; ++m) {
        const int a = comp[m][0], b = comp[m][1];
        /* -sum e_a e_b fbar with fbar = d_bar + w rho0 (+ phi(B0)): the w rho0
         * part gives -rho0 c^2/3 delta_ab, which joins pbar delta_ab of
         * Mbar^eq as (rhobar - rho0) c^2 / 3 (as in Pi^neq); phi(B0) gives
         * -L(B0), which joins L(Bbar) as L(Bbar) - L(B0) */
        real mom = 0;
        for (int q = 0; q < Q; ++q) mom += (real)(c2 * o->e[q][a] * o->e[q][b]) * db[q];
        real meq = (a == b ? drho * c2 / 3.0 : 0.0) + (o->stokes ? 0.0 : rho * u[a] * u[b]);
        if (mhd_eq(o)) meq += maxwell_change(o, a, b, bbar);
        real val = -mom + meq;
        sigma_bar[(long)m * N + i] = RE(val);
      }
    }
  }
  return 0;
}

/* ---------------------------------------------------------------------------
 * Reverse-mode gradient of a wall-force objective (complex-step build only)
 * ---------------------------------------------------------------------------
 * J = component `axis` of the raw momentum-exchange force (Eq. 25) on the
 * links of wall group `group` during the last of T steps.  The map from the
 * state at step n to the state at step n + 1 is relaxation (node-local) then
 * propagation with bounce-back (a permutation of the relaxed values plus the
 * moving-wall term).  Its transpose is applied backwards in time:
 *   - propagation: the cotangent of a relaxed value is the cotangent of the
 *     slot it was written to (and the same for the moving-wall term added to a
 *     bounce-back slot);
 *   - relaxation: the node's Jacobian with respect to its Q distributions, its
 *     body force and (through the moving-wall term) the wall velocity, each
 *     column taken by a complex step of node_relax itself (exact to rounding,
 *     no hand-derived formula), multiplied by the cotangents.
 * All T pre-step states are kept (no checkpointing).  MHD is not supported. */
#ifdef ORC_COMPLEX
int orc_adjoint(orc* o, int T, int group, int axis, double* J, double* grad_a, double* grad_uw) {
  if (T < 1 || o->mhd || o->qlink || group < 0 || group >= o->G || axis < 0 || axis >= o->D) return -1;
  const int Q = o->Q, D = o->D, G = o->G;
  const long N = o->N;
  const long QN = (long)Q * N;
  const double c = o->c, dt = o->dt;
  const double vol = o->lat == 0 ? o->dx * o->dx : o->dx * o->dx * o->dx;
  const double h = 1e-30; /* complex step */
  double* states = (double*)malloc(sizeof(double) * QN * T);
  double* lam = (double*)calloc(QN, sizeof(double));
  double* lamn = (double*)calloc(QN, sizeof(double));
  const long rows = (long)o->ny * o->nz;
  double* uwpart = (double*)calloc((size_t)rows * G * 3, sizeof(double));
  if (!states || !lam || !lamn || !uwpart) {
    free(states);
    free(lam);
    free(lamn);
    free(uwpart);
    return -2;
  }
  /* forward, keeping the state before each step */
  for (int n = 0; n < T; ++n) {
    for (long i = 0; i < QN; ++i) states[(long)n * QN + i] = RE(o->d[i]);
    orc_step(o, 1);
  }
  *J = RE(o->wf[group][0][axis]);
  memset(grad_a, 0, sizeof(double) * 3 * N);
  /* backward */
  for (int n = T - 1; n >= 0; --n) {
    const double* sn = states + (long)n * QN;
    memset(lamn, 0, sizeof(double) * QN);
#pragma omp parallel for schedule(static)
    for (long r = 0; r < rows; ++r) {
      const int y = (int)(r % o->ny), z = (int)(r / o->ny);
      double* pu = uwpart + r * G * 3;
      for (int x = 0; x < o->nx; ++x) {
        const long idx = ((long)z * o->ny + y) * o->nx + x;
        if (o->solid[idx]) continue;
        /* cotangents of the relaxed values (muR) and of the moving-wall terms (muL) */
        double muR[19], muL[19];
        int wall[19], grp[19];
        for (int q = 0; q < Q; ++q) {
          long t;
          int g;
          wall[q] = link_target(o, x, y, z, o->e[q], &t, &g);
          grp[q] = wall[q] ? g : -1;
          if (!wall[q]) {
            muR[q] = lam[(long)q * N + t];
            muL[q] = 0;
          } else {
            muR[q] = muL[q] = lam[(long)o->opp[q] * N + idx];
          }
        }
        if (n == T - 1) {
          /* J = sum over the group's links of (dx^D/dt)(e_q f_out - e_opp f_in)_axis,
           * f_out = drel + w rho0, f_in = f_out + moving-wall term */
          for (int q = 0; q < Q; ++q)
            if (wall[q] && grp[q] == group) {
              const double ek = c * o->e[q][axis];
              muR[q] += 2.0 * vol / dt * ek;
              muL[q] += vol / dt * ek;
            }
        }
        real dl[19], drel[19];
        node_t s;
        for (int q = 0; q < Q; ++q) dl[q] = sn[(long)q * N + idx];
        /* distributions */
        for (int p = 0; p < Q; ++p) {
          const real keep = dl[p];
          dl[p] = keep + MK(0.0, h);
          node_relax(o, dl, idx, NULL, NULL, &s, drel);
          double acc = 0;
          for (int q = 0; q < Q; ++q) {
            acc += muR[q] * (IM(drel[q]) / h);
            if (wall[q]) {
              real uw[3] = {RE(o->uw[grp[q]][0]), RE(o->uw[grp[q]][1]), RE(o->uw[grp[q]][2])};
              acc += muL[q] * (IM(moving_wall_term(o, q, s.rho, uw)) / h);
            }
          }
          lamn[(long)p * N + idx] = acc;
          dl[p] = keep;
        }
        /* body force of this node */
        for (int k = 0; k < D; ++k) {
          real an[3] = {0, 0, 0};
          for (int m = 0; m < D; ++m) an[m] = RE(body_force(o, idx, m));
          an[k] += MK(0.0, h);
          node_relax(o, dl, idx, NULL, an, &s, drel);
          double acc = 0;
          for (int q = 0; q < Q; ++q) acc += muR[q] * (IM(drel[q]) / h);
          grad_a[(long)k * N + idx] += acc;
        }
        /* wall velocities (through the moving-wall term only) */
        node_relax(o, dl, idx, NULL, NULL, &s, drel);
        for (int q = 0; q < Q; ++q) {
          if (!wall[q]) continue;
          for (int k = 0; k < D; ++k) {
            real uw[3] = {RE(o->uw[grp[q]][0]), RE(o->uw[grp[q]][1]), RE(o->uw[grp[q]][2])};
            uw[k] += MK(0.0, h);
            pu[grp[q] * 3 + k] += muL[q] * (IM(moving_wall_term(o, q, s.rho, uw)) / h);
          }
        }
      }
    }
    double* t = lam;
    lam = lamn;
    lamn = t;
  }
  memset(grad_uw, 0, sizeof(double) * G * 3);
  for (long r = 0; r < rows; ++r)
    for (int k = 0; k < G * 3; ++k) grad_uw[k] += uwpart[r * G * 3 + k];
  free(states);
  free(lam);
  free(lamn);
  free(uwpart);
  return 0;
}
#else
int orc_adjoint(orc* o, int T, int group, int axis, double* J, double* grad_a, double* grad_uw) {
  (void)o, (void)T, (void)group, (void)axis, (void)J, (void)grad_a, (void)grad_uw;
  return -3; /* needs the complex-step build */
}
#endif
