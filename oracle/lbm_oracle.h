/*
 * Plain CPU reference ("oracle") for the lattice Boltzmann hot path of
 * J. Li, "Shear Stress and Fluid-Wall Interaction Force in LBM Simulations of
 * Hydrodynamic and MHD Flows" (arXiv 2512.12213).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the GPU path.
 *
 * Two builds come from one source file:
 *   liboracle.so     real = double          (the FP64 reference)
 *   liboracle_cs.so  real = double complex  (complex-step derivatives: run with
 *                    an input perturbed by i*h*delta and the imaginary part of
 *                    any output divided by h is its exact directional derivative,
 *                    Squire & Trapp, SIAM Review 40 (1998))
 * Every function takes the imaginary parts of complex inputs as separate
 * arrays (may be NULL) and returns imaginary parts the same way; the double
 * build ignores / zero-fills them.
 *
 * Conventions (shared by contract with the GPU library's public header, not by
 * code): state arrays are structure-of-arrays [Q][nz][ny][nx], x fastest; the
 * stored quantity is the deviation d = f - w*rho0; the direction order is
 *   D2Q9 : 0 rest; 1 +x; 2 -x; 3 +y; 4 -y; 5 (+x,+y); 6 (-x,-y); 7 (+x,-y); 8 (-x,+y)
 *   D3Q19: 0 rest; 1,2 +-x; 3,4 +-y; 5,6 +-z; 7,8 +-(x+y); 9,10 +-(x-y);
 *          11,12 +-(x+z); 13,14 +-(x-z); 15,16 +-(y+z); 17,18 +-(y-z)
 *   D3Q7 (induction): 0 rest; 1,2 +-x; 3,4 +-y; 5,6 +-z
 *   D2Q5 (induction, two dimensions): directions 0-4 of D3Q7
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc orc;

/* lattice: 0 = D2Q9, 1 = D3Q19.  model: 0..4 = [a] He, [b] Luo, [c] Shan-Chen
 * (reformulated), [d] EDM (reformulated), [e] Guo; 5 = Shan-Chen original
 * (shifted u^eq, no force term), 6 = EDM original (F = feq(u+dt a) - feq(u)).
 * Returns NULL on invalid arguments. */
orc* orc_create(int lattice, int nx, int ny, int nz, double tau, double dx, double dt, int model);
void orc_destroy(orc* o);
int orc_threads(int n);                     /* set OpenMP threads, returns threads in use */

int orc_set_rho0(orc* o, double rho0);
int orc_set_walls(orc* o, int axis, int group_lo, int group_hi);   /* -1,-1 = periodic */
int orc_set_solid(orc* o, const unsigned char* mask, int group);   /* [nz][ny][nx], nonzero = solid */
int orc_set_wall_velocity(orc* o, int group, const double* u, const double* u_im);      /* u[3] */
int orc_set_body_force(orc* o, const double* a, const double* a_im);                    /* a[3] */
int orc_set_body_force_field(orc* o, const double* a, const double* a_im);              /* [3][N] or NULL */
int orc_set_les(orc* o, double cs);
int orc_set_equilibrium(orc* o, int stokes);   /* 0: Eq. (1); 1: Stokes form (text after Eq. 11) */
int orc_set_darcy(orc* o, double sigma);
/* Interpolated bounce-back: q [Q][N] = wall distance / link length per link
 * (1/2 = halfway wall, values of non-wall links ignored), or NULL for all
 * halfway.  -1 if a value is outside (0, 1]. */
int orc_set_link_fraction(orc* o, const double* q);       /* porous resistance: adds -sigma v to the body force */
int orc_set_artefact(orc* o, int on);
/* MHD: D3Q19 with D3Q7 induction, or D2Q9 with D2Q5 induction (B0z = 0) */
int orc_set_mhd(orc* o, double B0x, double B0y, double B0z, double mu, double tau_m);
/* after orc_set_mhd: 1 = Lorentz force through the force term, f^eq hydrodynamic */
int orc_set_lorentz_force(orc* o, int on);

int orc_init_equilibrium(orc* o, const double* u0);   /* u0 [D][N] or NULL */
int orc_set_state(orc* o, const double* d, const double* d_im);   /* [Q][N] deviations */
int orc_get_state(const orc* o, double* d, double* d_im);
int orc_replace_state(orc* o, const double* d);            /* keeps the last-step records */
int orc_get_induction(const orc* o, double* g);                   /* [K][3][N], K = 7 or 5 */

int orc_step(orc* o, int n);

/* rho [N], v [D][N]; B [3][N] may be NULL */
int orc_get_macro(const orc* o, double* rho, double* v, double* B);
/* sigma, strain: [ncomp][N], ncomp = 3 (xx, xy, yy) in 2D, 6 (xx, yy, zz, xy, xz, yz) in 3D */
int orc_stress(const orc* o, double* sigma, double* strain);
/* out [G][4][3]: raw, minus momentum flux, minus Maxwell, minus both; last step */
int orc_wall_force(const orc* o, double* out, double* out_im, int G);
/* out [24]: force balance record of the last step */
int orc_force_balance(const orc* o, double* out);
long orc_link_count(const orc* o, int group);

/* Half-step distribution of the last step (Section 5, Eq. 27) and its moments:
 * fbar [Q][N] = (f_rel(x,t) + f(x,t+dt))/2 - w rho0; rho_bar [N]; u_bar [D][N]
 * (sum e fbar / rho_bar); sigma_bar [ncomp][N] = -sum e e fbar + Mbar^eq (Eq. 28).
 * Any may be NULL.  -1 before the first step. */
int orc_halfstep(const orc* o, double* fbar, double* rho_bar, double* u_bar, double* sigma_bar);

/* Reverse-mode gradient (complex-step build only; -3 from the double build).
 * From the current state, runs T steps and returns J = component `axis` of
 * the raw wall force on group `group` during the last step, grad_a [3][N]
 * = dJ/da per node (physical units; components beyond D are 0) and
 * grad_uw [G][3] = dJ/du_w per wall group.  Leaves the state at step T.
 * Parameters must carry no imaginary parts. */
int orc_adjoint(orc* o, int T, int group, int axis, double* J, double* grad_a, double* grad_uw);

#ifdef __cplusplus
}
#endif
#endif
