/*
 * lbm.h - C ABI of the MI355X lattice Boltzmann hot path.
 *
 * Method: J. Li, "Shear Stress and Fluid-Wall Interaction Force in LBM
 * Simulations of Hydrodynamic and MHD Flows", arXiv 2512.12213.
 *
 * One context = one lattice on one GPU (the current HIP device when
 * lbm_create is called).  The library owns every device buffer it allocates;
 * host buffers passed in are owned by the caller and only read / written
 * during the call; device pointers passed in are borrowed and must outlive
 * their use.  A context is not thread-safe: call it from one host thread.
 *
 * Every int-returning call returns LBM_OK (0) or a negative error code and
 * then sets a thread-local message readable with lbm_last_error().
 *
 * Units are physical: lattice spacing dx, time step dt, lattice speed
 * c = dx/dt, kinematic viscosity nu = dt c^2 (tau - 1/2) / 3 (Section 2).
 * Forces are per unit depth in 2D.
 *
 * Array layouts (all x fastest, "[a][b]" = a slowest):
 *   scalar field   [nz][ny][nx]
 *   vector field   [D][nz][ny][nx]   (D = 2 for D2Q9, 3 for D3Q19)
 *   distributions  [Q][nz][ny][nx], deviations d = f - w * rho0, in the
 *                  direction order below
 *   stress tensor  [ncomp][nz][ny][nx]: ncomp = 3 (xx, xy, yy) in 2D,
 *                  6 (xx, yy, zz, xy, xz, yz) in 3D
 * Direction order:
 *   D2Q9 : 0 rest; 1 +x; 2 -x; 3 +y; 4 -y; 5 (+x,+y); 6 (-x,-y); 7 (+x,-y); 8 (-x,+y)
 *   D3Q19: 0 rest; 1,2 +-x; 3,4 +-y; 5,6 +-z; 7,8 +-(x+y); 9,10 +-(x-y);
 *          11,12 +-(x+z); 13,14 +-(x-z); 15,16 +-(y+z); 17,18 +-(y-z)
 *   D3Q7 (induction): 0 rest; 1,2 +-x; 3,4 +-y; 5,6 +-z
 *   D2Q5 (induction, two dimensions): directions 0-4 of D3Q7
 */
#ifndef LBM_H
#define LBM_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
/* Body-force models of Section 2: [a] He et al., [b] Martys-Shan-Chen / Luo
 * (Eq. 3), [c] Shan-Chen reformulated, [d] exact-difference reformulated,
 * [e] Guo. */
enum { LBM_FORCE_HE = 0, LBM_FORCE_LUO = 1, LBM_FORCE_SHANCHEN = 2, LBM_FORCE_EDM = 3, LBM_FORCE_GUO = 4 };
/* Storage precision of the distributions (arithmetic is FP32 for the
 * reduced formats, FP64 for LBM_F64). */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2, LBM_BF16 = 3 };
/* Equilibrium form: Eq. (1), or the Stokes form rho w [1 + 3 e.u^eq / c^2]
 * (text after Eq. 11: M^eq = c^2 rho I / 3, no convection term). */
enum { LBM_EQ_NS = 0, LBM_EQ_STOKES = 1 };
enum { LBM_OK = 0, LBM_EINVAL = -1, LBM_ENOMEM = -2, LBM_EHIP = -3, LBM_ESTATE = -4, LBM_EUNSTABLE = -5 };
enum { LBM_MAX_GROUPS = 16, LBM_NREC = 24 };
/* Bytes of the fixed device scratch array of lbm_step_noalloc (8 MiB). */
enum { LBM_SCRATCH_BYTES = 8 << 20 };

/* Create a lattice.  Section 2: uniform grid with spacing dx, time step dt,
 * relaxation time tau (tau > 1/2), D2Q9 (nz must be 1) or D3Q19.  All axes
 * are periodic until walls are added.  Storage defaults to LBM_F32, rho0 to 1.
 * Limits: every axis <= 65536 nodes and fewer than 2^31 nodes in total.
 * Returns NULL on error (lbm_last_error() explains). */
lbm_ctx* lbm_create(int lattice, int nx, int ny, int nz, double tau, double dx, double dt, int force_model);

/* Free every device buffer of the context; NULL is accepted. */
void lbm_destroy(lbm_ctx* ctx);

/* Thread-local message of the last failing call on this thread. */
const char* lbm_last_error(void);

/* ---- set-up (before the first lbm_init_equilibrium / lbm_set_state unless noted) ---- */

/* Storage precision, one of LBM_F64/F32/F16/BF16.  16-bit formats store
 * d/w scaled by 2^10 (F16) or d/w (BF16), rounded to nearest even. */
int lbm_set_storage(lbm_ctx* ctx, int precision);

/* Reference density rho0 > 0 (the deviation origin and the initial density). */
int lbm_set_rho0(lbm_ctx* ctx, double rho0);

/* Halfway bounce-back plane walls half a spacing beyond the first and last
 * node along `axis` (0 = x, 1 = y, 2 = z); all nodes stay fluid
 * (Section 5, Eq. 25: wall a half grid away from the fluid node).  A group
 * is a label in [0, 16) under which wall forces are summed; -1 leaves that
 * end periodic.  A link crossing two walls (a corner) belongs to the
 * lower-numbered axis. */
int lbm_add_plane_walls(lbm_ctx* ctx, int axis, int group_lo, int group_hi);

/* Solid nodes: mask_host [nz][ny][nx], nonzero = solid, links from fluid
 * nodes into them are halfway bounce-back links of `group`. */
int lbm_add_solid_mask(lbm_ctx* ctx, const unsigned char* mask_host, int group);

/* Walls that are not halfway between nodes (Section 5: the momentum exchange
 * then gives the stress half a link from the fluid node, not at the wall).
 * q_host [Q][nz][ny][nx]: for each fluid node and each link that ends in a
 * wall or solid node, the distance to the wall as a fraction of the link, in
 * (0, 1]; 1/2 keeps halfway bounce-back; entries of other links are ignored
 * but must also lie in (0, 1]; NULL returns to halfway walls everywhere.
 * Links with q != 1/2 are bounced back by linear interpolation (Bouzidi,
 * Firdaouss and Lallemand 2001), inside the step (in a pass after the last
 * step of each call), with the moving-wall term: q < 1/2: 2q f_rel_a(x) + (1 - 2q) f_rel_a(x - e_a) (halfway
 * when x - e_a is not fluid); q >= 1/2: [f_rel_a(x) + (2q - 1) f_rel_opp(a)(x)]
 * / (2q).  The wall force uses the values that leave and return at the node;
 * lbm_halfstep averages f_rel(x, t) with the interpolated f(x, t + dt).  At
 * most 1,048,574 fluid nodes with such links (LBM_EINVAL beyond).  Under
 * MHD the induction distributions keep halfway anti-bounce-back (B = B0
 * half a link from the fluid node), each wall link keeps its Maxwell-stress
 * correction, and the pass runs after every step.  A run recorded by
 * lbm_adjoint_forward also runs the pass after every step, and its adjoint
 * reverses it; so does a call with the per-step wall-force record, whose
 * every step then includes the interpolated links' changes.  Set-up only. */
int lbm_set_link_fractions(lbm_ctx* ctx, const double* q_host);

/* Wall velocity of a group (moving-wall bounce-back adds
 * 6 w rho (e.u_w)/c^2 to the returning population).  May change between
 * steps. */
int lbm_set_wall_velocity(lbm_ctx* ctx, int group, double ux, double uy, double uz);

/* Uniform body force per unit mass a.  May change between steps. */
int lbm_set_body_force(lbm_ctx* ctx, double ax, double ay, double az);

/* Per-node body force: borrowed device pointer to float [3][nz][ny][nx]
 * (e.g. a torch tensor's data_ptr), or NULL to return to the uniform force.
 * May change between steps; must stay valid while steps run. */
int lbm_set_body_force_field(lbm_ctx* ctx, const void* dev_ptr);

/* Smagorinsky constant C_s >= 0 for the eddy viscosity built from the
 * strain rate of Eq. (9); 0 disables it. */
int lbm_set_les(lbm_ctx* ctx, double cs);

/* Equilibrium form, LBM_EQ_NS (default) or LBM_EQ_STOKES.  Set-up only.
 * With the Stokes form the stress of Eq. (9) and the half-step stress use
 * M^eq = p I, and the artefact term loses its u^eq a part. */
int lbm_set_equilibrium(lbm_ctx* ctx, int kind);

/* Porous resistance (Brinkman; text after Eq. 11): the body force becomes
 * a - sigma v with v = u + dt a / 2 the velocity of Section 2, i.e. each node
 * applies (a - sigma u) / (1 + sigma dt / 2).  sigma >= 0 in 1/time (nu / K
 * for permeability K); 0 disables it.  May change between steps; wall forces,
 * the balance record and the adjoint include it. */
int lbm_set_darcy(lbm_ctx* ctx, double sigma);

/* Include the artefact term E_ij of Eq. (9) in the stress and strain
 * outputs (0 = off, the default).  Any time. */
int lbm_set_artefact(lbm_ctx* ctx, int include_Eij);

/* Stress and strain rate written by the steps themselves (Eqs. 8-9, the
 * values lbm_stress gives, with the artefact term when lbm_set_artefact is
 * on): during lbm_step, each step whose index i (steps taken since the state
 * was set, before that step) is a multiple of `every` >= 1 writes sigma and
 * S of the state f(t_i) it starts from, as FP32 in physical units, into the
 * borrowed device buffers sigma_dev and strain_dev (float [ncomp][nz][ny][nx],
 * component order of lbm_stress; either may be NULL), at 4 ncomp bytes per
 * node and buffer on top of the step's own traffic.  The buffers are zeroed
 * by this call (solid nodes keep 0) and must stay valid while steps run.
 * Both NULL turns it off.  Any time. */
int lbm_set_step_stress(lbm_ctx* ctx, void* sigma_dev, void* strain_dev, int every);

/* MHD (Section 4; F32/F64 storage) with a vector-distribution induction
 * lattice (relaxation time tau_m > 1/2, magnetic diffusivity
 * dt c^2 (tau_m - 1/2) / 4): D3Q7 with three field components on D3Q19; on
 * D2Q9 its planar restriction (rest weight 1/2, 1/8 per axis link) with the
 * two in-plane components, which needs B0z = 0.  All walls are insulating:
 * B = B0 on them.  mu is the magnetic permeability.  The coupling is the
 * paper's by default (magnetic stress in the equilibrium, Eq. 10; in two
 * dimensions without its -c^2 B^2 / 6 term); see lbm_set_mhd_coupling. */
int lbm_set_mhd(lbm_ctx* ctx, double B0x, double B0y, double B0z, double mu, double tau_m);

/* MHD coupling (Section 4 names three approaches; two are provided):
 *   LBM_MHD_EQUILIBRIUM   the Lorentz force as minus the divergence of the
 *                         Maxwell stress in f^eq (Eq. 10); P of Eq. (25)
 *                         then holds -L, which the Maxwell variant of
 *                         lbm_wall_force removes;
 *   LBM_MHD_LORENTZ_FORCE f^eq hydrodynamic and the Lorentz force J x B
 *                         added to the body force of the force model; P
 *                         holds no -L and the balance record's body force
 *                         includes the Lorentz force (text after Eq. 36).
 * J = curl B / mu comes from the non-equilibrium part of the induction
 * distributions' first moment (-tau_m dt theta c^2 grad B to first order),
 * with the velocity's own half-force solved for in closed form.  After
 * lbm_set_mhd; set-up only; not with lbm_set_darcy (LBM_EINVAL). */
enum { LBM_MHD_EQUILIBRIUM = 0, LBM_MHD_LORENTZ_FORCE = 1 };
int lbm_set_mhd_coupling(lbm_ctx* ctx, int kind);

/* HIP stream (hipStream_t) on which all later work of the context is
 * enqueued, e.g. torch.cuda.current_stream().cuda_stream; NULL = the
 * context's own stream.  Any time. */
int lbm_set_stream(lbm_ctx* ctx, void* hip_stream);

/* ---- state ---- */

/* f = f^eq(rho0, u0) (Eq. 1; plus the magnetic term of Eq. 10 with B0 under
 * MHD).  u0_host: [D][nz][ny][nx] doubles, the velocity u = sum(e f)/rho, or
 * NULL for rest.  Resets the step counter. */
int lbm_init_equilibrium(lbm_ctx* ctx, const double* u0_host);

/* Upload / download deviations [Q][nz][ny][nx] (doubles, caller-owned),
 * in the direction order above.  lbm_set_state resets the step counter. */
int lbm_set_state(lbm_ctx* ctx, const double* d_host);
int lbm_get_state(lbm_ctx* ctx, double* d_host);

/* Induction distributions g [K][NB][nz][ny][nx] (absolute values; K = 7,
 * NB = 3 on D3Q19, K = 5, NB = 2 on D2Q9).  MHD only. */
int lbm_get_induction(lbm_ctx* ctx, double* g_host);

/* ---- the hot path ---- */

/* Advance n >= 0 steps of Eq. (2): f(x + dt e, t + dt) = f + (f^eq - f)/tau + F,
 * with streaming in place, bounce-back, the force model and (if enabled)
 * Smagorinsky closure and the MHD equilibrium.  All steps are enqueued on
 * the stream with no host synchronisation between them; the last step also
 * produces the wall-force and balance records.  The call ends with one
 * stream synchronisation and a finiteness check of the total mass:
 * LBM_EUNSTABLE if it is NaN or infinite. */
int lbm_step(lbm_ctx* ctx, int n);

/* lbm_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same steps and records as lbm_step(ctx, n), with the step's scratch (the
 * per-tile partial sums of the last step, the reduced records, and with walls
 * that are not halfway the changes of their returning values and their sums)
 * taken from a fixed array of LBM_SCRATCH_BYTES bytes in device memory, one
 * copy per GPU, held until the process ends; it calls no hipMalloc, hipFree
 * or allocating routine (the context's own buffers are allocated by its
 * set-up and state calls).  Fits lattices whose scratch is at most that size,
 * about 184 bytes per 256 nodes plus 152 bytes per node with links to walls
 * that are not halfway (e.g. 11 M nodes with halfway walls); larger ones
 * give LBM_EINVAL before any work.  Every call on one GPU uses that GPU's
 * single array and leaves its contents there; nothing in it has to start at
 * zero (each step writes every entry it later reads).  Calls that overlap on
 * one GPU (contexts used from several host threads or on streams that run
 * concurrently) race on the array.  Per-launch timing (lbm_set_timing) is
 * not recorded. */
int lbm_step_noalloc(lbm_ctx* ctx, int n);

/* Density rho [nz][ny][nx] and flow velocity v = u + dt a / 2 [D][nz][ny][nx]
 * (Section 2) of the current state, into caller-owned host buffers (either
 * may be NULL).  Solid nodes read 0. */
int lbm_get_macro(lbm_ctx* ctx, double* rho, double* v);

/* Magnetic field B = sum_k g_k [3][nz][ny][nx] of the current state (MHD). */
int lbm_get_field_B(lbm_ctx* ctx, double* B);

/* Shear stress sigma = 2 rho nu S (Eq. 8) and strain rate
 * S = -3 / (2 tau dt c^2 rho) (Pi^neq [+ E]) (Eq. 9) of the current state,
 * with Pi^neq = sum(e e f) - (p I + rho u^eq u^eq [+ L]) and tau the
 * Smagorinsky-effective relaxation time when LES is on.  Caller-owned host
 * buffers [ncomp][nz][ny][nx]; either may be NULL.  Solid nodes read 0. */
int lbm_stress(lbm_ctx* ctx, double* sigma, double* strain);

/* The same stress and strain rate (Eqs. 8-9) into caller-owned DEVICE
 * buffers of the same layout (FP64), with no copy to the host: one kernel
 * enqueued on the context's stream (lbm_set_stream); the outputs are
 * complete when that stream reaches this point.  Either may be NULL; the
 * buffers must stay valid until then and must not overlap. */
int lbm_stress_device(lbm_ctx* ctx, double* sigma, double* strain);

/* Half-step distribution of the last step (Section 5, Eq. 27):
 * f_bar = (f_rel(x, t) + f(x, t + dt)) / 2, the relaxed value before
 * propagation averaged with the propagated one, and its moments: density
 * rho_bar = sum f_bar, velocity u_bar = sum e f_bar / rho_bar, and the stress
 * of Eq. (28), sigma_bar = -sum e e f_bar + Mbar^eq with
 * Mbar^eq = p_bar I + rho_bar u_bar u_bar (+ the Maxwell stress of
 * B_bar = (B(t) + B(t + dt)) / 2 under MHD), p_bar = rho_bar c^2 / 3.  At a
 * steady state sigma_bar equals the Eq. (9) stress up to the force term's
 * second moment (Eq. 30).  Caller-owned host buffers: fbar [Q][nz][ny][nx] as
 * f_bar - w rho0, rho_bar [nz][ny][nx], u_bar [D][nz][ny][nx] (physical),
 * sigma_bar [ncomp][nz][ny][nx] (physical, component order of lbm_stress); any
 * may be NULL; solid nodes read 0.  LBM_ESTATE unless a step has been taken
 * since the state was last set.  The wall velocities of the last step are
 * used, even if they have been changed since.  At links to walls that are
 * not halfway (lbm_set_link_fractions), f(x, t + dt) is the interpolated
 * returning value. */
int lbm_halfstep(lbm_ctx* ctx, double* fbar, double* rho_bar, double* u_bar, double* sigma_bar);

/* The same half-step distribution and moments (Section 5, Eqs. 27-28) into
 * caller-owned DEVICE buffers of the same layouts (FP64), with no copy to
 * the host: one kernel enqueued on the context's stream (lbm_set_stream);
 * the outputs are complete when that stream reaches this point.  Any may be
 * NULL; the buffers must stay valid until then and must not overlap.
 * LBM_ESTATE unless a step has been taken since the state was last set. */
int lbm_halfstep_device(lbm_ctx* ctx, double* fbar, double* rho_bar, double* u_bar, double* sigma_bar);

/* Momentum-exchange force on the walls of each group during the last step
 * (Eq. 25, the populations leaving at t and returning at t + dt, per link
 * (dx^D / dt)(e_out f_out - e_in f_in)).  out [G][4][3], G = lbm_num_groups:
 * variant 0 raw; 1 minus the moving-boundary momentum flux
 * -(dx^D/dt) u_w (f_out - f_in); 2 minus the Maxwell stress carried by the
 * MHD equilibrium, -(dx^D/dt) 2 e_out phi_out(B0); 3 minus both.  z = 0 in 2D.
 * LBM_ESTATE before the first step. */
int lbm_wall_force(lbm_ctx* ctx, double* out);

/* Per-step wall-force record (Eq. 25 for every step, not only the last):
 * with on != 0, the steps of later lbm_step calls also sum the momentum
 * exchange of their wall links (only the 256-node tiles that a wall group
 * meets do any extra work), and lbm_wall_force_history returns, for each step
 * of the most recent such call in order, the four variants of lbm_wall_force:
 * out[n][G][4][3], G = lbm_num_groups, n = min(steps of that call,
 * max_steps), written to *nsteps.  The last entry equals lbm_wall_force.
 * With walls that are not halfway (lbm_set_link_fractions) the interpolation
 * runs as a pass after every step of such a call, and each step's record
 * includes its interpolated links' changes.  Not recorded by
 * lbm_step_noalloc (LBM_EINVAL while on) or lbm_adjoint_forward.  Device
 * buffers of about 64 bytes per such tile and recorded step (and 128 bytes
 * per recorded step with interpolated links) are allocated on the first
 * call.  LBM_ESTATE when no call has recorded it since the state
 * was set. */
int lbm_set_wall_force_history(lbm_ctx* ctx, int on);
int lbm_wall_force_history(lbm_ctx* ctx, double* out, int max_steps, int* nsteps);

/* Global balance of the last step (Eq. 32), out[24] doubles:
 *  0-2  F_wall raw (all groups)          3-5  sum rho a dx^D at t
 *  6-8  (P(t+dt) - P(t)) / dt, P = sum rho u dx^D
 *  9-11 residual (3-5) - (0-2) - (6-8)   (exactly 0 up to rounding)
 * 12-14 total Maxwell correction        15-17 total momentum-flux correction
 * 18-20 stress-integral force over plane walls: sum of (-p I + sigma) n dA
 *       with p, sigma extrapolated linearly from the first two fluid layers
 *       (Eqs. 26, 33), of the current state
 * 21 mass M(t+dt) = sum rho dx^D    22 M(t+dt) - M(t)    23 steps taken
 * LBM_ESTATE before the first step. */
int lbm_force_balance(lbm_ctx* ctx, double* out);

/* Number of wall groups (1 + largest group label in use). */
int lbm_num_groups(lbm_ctx* ctx);

/* Number of bounce-back links of a group (-1 = all groups). */
long lbm_link_count(lbm_ctx* ctx, int group);

/* Steps taken since the last initialisation. */
long lbm_steps_taken(lbm_ctx* ctx);

/* ---- differentiation (the discrete adjoint of the step; the paper does not
 * differentiate its method) ---- */

/* Record a differentiable run: from the current state, advance T >= 1 steps
 * exactly as lbm_step(T) does, keeping a device copy of the state every
 * ckpt_every >= 1 steps (ceil(T / ckpt_every) copies of Q N values, owned by
 * the context; the backward pass recomputes each segment), or, with
 * ckpt_every = 0, recording density and velocity of every step instead
 * (T x 4 N values; no recompute in the backward pass), and return in *J the
 * objective: component `axis` (0 = x,
 * 1 = y, 2 = z; < D) of the raw Eq. (25) force on wall group `group` during
 * the last step, i.e. lbm_wall_force variant 0.  Needs LBM_F32 or LBM_F64
 * storage, no MHD and no Smagorinsky closure (LBM_EINVAL otherwise).  The run
 * stays recorded for lbm_adjoint_backward until the next lbm_step,
 * lbm_adjoint_forward, state upload or change of wall velocities, body force
 * or closure; the body-force field's device memory must not change meanwhile.
 * With walls that are not halfway (lbm_set_link_fractions) every recorded
 * step runs the interpolation as a pass after it (the same values as inside
 * the step, up to rounding order), and J includes the interpolated links'
 * changes of the returning values. */
int lbm_adjoint_forward(lbm_ctx* ctx, int T, int ckpt_every, int group, int axis, double* J);

/* Gradient of gJ * J for the recorded run, by the adjoint of every step in
 * reverse order: each checkpoint segment is first recomputed forward (also
 * recording density and velocity per node and step), then its adjoint steps
 * run backwards (with ckpt_every = 0 the recorded densities and velocities
 * are used directly).  grad_a_dev: device buffer [3][nz][ny][nx], float
 * (grad_f64 = 0) or double (grad_f64 = 1), overwritten with gJ dJ/da per
 * node in physical units (the z plane is 0 in 2D), or NULL.  grad_uw: host
 * buffer [G][3], G = lbm_num_groups, overwritten with gJ dJ/du_w per wall
 * group (physical units), or NULL.  Work buffers (with checkpoints: two
 * state copies and min(ckpt_every, T) x 4 N values; one state copy without)
 * are allocated on first use and kept.  The
 * context's state is not changed and the run stays recorded.  LBM_ESTATE
 * without a recorded run.  The recompute runs in the storage precision, the
 * adjoint steps in the adjoint precision (lbm_set_adjoint_precision).  With
 * walls that are not halfway each adjoint step is preceded by the transpose
 * of the interpolation pass (FP64 arithmetic), and dJ/du_w includes the
 * moving-wall terms of the interpolated links. */
int lbm_adjoint_backward(lbm_ctx* ctx, double gJ, void* grad_a_dev, int grad_f64, double* grad_uw);

/* Precision of the adjoint state and its arithmetic: LBM_F64 (the default;
 * the only choice for LBM_F64 storage) or LBM_F32 (LBM_F32 storage only:
 * half the adjoint's memory traffic, but FP32 rounding of the adjoint state
 * loses the small differences between nearly equal sensitivities, e.g. the
 * gradient with respect to the velocity of a distant wall).  Any time. */
int lbm_set_adjoint_precision(lbm_ctx* ctx, int precision);

/* Per-launch timing of lbm_step with HIP events recorded on the context's
 * stream between consecutive launches (on = 1; adds one event per launch).
 * lbm_step_timings fills out[6] for the most recent timed call, in seconds:
 * 0 mean duration of an even-parity step launch, 1 of an odd-parity one
 * (both excluding the call's last, diagnostic, step), 2 the diagnostic step,
 * 3 the reduction and 568-byte copy that follow it, 4 launches in the call,
 * 5 the whole call from the first launch to the end of the copy. */
int lbm_set_timing(lbm_ctx* ctx, int on);
int lbm_step_timings(lbm_ctx* ctx, double* out);

#ifdef __cplusplus
}
#endif
#endif
