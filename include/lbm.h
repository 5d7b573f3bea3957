/*
 * lbm.h - C ABI of the MI355X lattice Boltzmann particle-resolved library.
 *
 * The library advances a D3Q19 multiple-relaxation-time lattice Boltzmann
 * flow on one GPU, with the two no-slip treatments for moving resolved
 * spheres compared in Peng, Ayala, Brandle de Motta & Wang (arXiv 1906.05448):
 * interpolated bounce-back with refilling, and the immersed boundary method
 * with a 4-point delta. Section references below are to that paper.
 *
 * Conventions (every entry point):
 *  - Return an int status: LBM_OK (0) or a negative lbm_status. Nothing
 *    throws, aborts or exits across this boundary; lbm_strerror() gives text.
 *  - Device memory is owned by the caller: one workspace of
 *    lbm_workspace_size() bytes, 256-byte aligned, handed to lbm_init() and
 *    kept alive until lbm_destroy(). The library never allocates device
 *    memory itself.
 *  - All GPU work is ordered on the HIP stream given to lbm_init() (with
 *    lbm_set_overlap() on, part of a step runs on a second stream of the
 *    context, forked from and joined back into that stream within the
 *    step). Calls marked "async" return before the work finishes; calls
 *    marked "sync" wait for the stream and report errors latched by earlier
 *    async calls.
 *  - Host pointers are read or written before the call returns and are
 *    never retained.
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Lattice arrays are laid out [component][z][y][x], x fastest; node
 *    (x, y, z) sits at coordinate (x, y, z); N = nx*ny*nz. The box is
 *    periodic in all three directions (Sec. 2.1, Sec. 3.1).
 *  - Units are lattice units: dx = dt = 1, reference density 1.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_E_ARG = -1,      /* invalid argument or configuration              */
  LBM_E_HIP = -2,      /* a HIP runtime call failed                       */
  LBM_E_SIZE = -3,     /* workspace too small, or a capacity exceeded     */
  LBM_E_STATE = -4,    /* call not valid in the context's current state   */
  LBM_E_UNSTABLE = -5, /* non-finite density/velocity or |u| above 0.35   */
  LBM_E_OVERLAP = -6   /* two particles overlap by more than half a radius*/
} lbm_status;

/* No-slip treatment on particle surfaces and walls (Sec. 2.1, Sec. 3.1). */
enum { LBM_BC_NONE = 0, LBM_BC_IBB = 1, LBM_BC_IBM = 2 };
/* Population storage: FP32 or IEEE half of the shifted value f_i - w_i.
 * Collision arithmetic is FP32 in both cases. */
enum { LBM_STORE_F32 = 0, LBM_STORE_F16S = 1 };
/* Static wall: none, or a pipe with its axis along z (Sec. 2.1). */
enum { LBM_WALL_NONE = 0, LBM_WALL_PIPE_Z = 1 };
/* Lattice. D3Q19 MRT (Sec. 3.1) runs every configuration. D3Q27 is the
 * turbulent-pipe solver (Sec. 2.2): one relaxation parameter for every
 * moment (BGK) plus an optional separate relaxation time for the energy mode
 * (the bulk-viscosity knob the paper describes), Guo forcing, FP32 storage;
 * a periodic box (LBM_BC_NONE) or the pipe wall with linear interpolated
 * bounce-back (LBM_BC_IBB, LBM_WALL_PIPE_Z, ibb_max_order 1); no particles. */
enum { LBM_LATTICE_D3Q19 = 0, LBM_LATTICE_D3Q27 = 1 };

typedef struct {
  int32_t nx, ny, nz;        /* lattice size, each >= 4                      */
  double tau;                /* shear relaxation time, > 0.5;
                                nu = (tau - 1/2)/3, rate s_nu = 1/tau        */
  double s_e, s_eps, s_q, s_pi, s_m; /* remaining d'Humieres MRT rates,
                                each in (0, 2); Sec. 3.1 names the model,
                                usual values 1.19, 1.4, 1.2, 1.4, 1.98.
                                s_e sets the bulk viscosity (Sec. 2.2.2)     */
  double body_force[3];      /* rho*g per unit volume (Sec. 2.1)             */
  int32_t bc;                /* LBM_BC_*                                      */
  int32_t ibb_max_order;     /* 2: quadratic with fallback chain, 1: linear  */
  double ibm_retraction;     /* r_d in lattice units: 0 (Uhlmann), 0.4
                                (Breugem), Sec. 2.1 and Sec. 3.1             */
  int32_t ibm_iters;         /* forcing passes after the first prediction;
                                the paper uses 2 (Sec. 2.1)                  */
  int32_t store;             /* LBM_STORE_*                                  */
  int32_t wall;              /* LBM_WALL_*; with LBM_BC_IBM the wall carries
                                static ring markers and no particles may be
                                set                                          */
  double pipe_radius, pipe_cx, pipe_cy; /* pipe wall, lattice units         */
  int32_t max_particles;     /* capacity reserved in the workspace           */
  double max_radius;         /* largest sphere radius that will be set       */
  double coll_restitution;   /* soft-sphere normal restitution (Sec. 3.1)    */
  double coll_tc_steps;      /* soft-sphere contact duration, time steps     */
  int32_t lattice;           /* LBM_LATTICE_*                                 */
  double tau_bulk;           /* D3Q27: relaxation time of the energy mode,
                                > 0.5, or 0 for tau (one parameter). The
                                mode's viscosity nu_b = (tau_bulk - 1/2)/3
                                gives the bulk viscosity 2 rho nu_b / 3.
                                Must be 0 with D3Q19 (s_e plays that role) */
} lbm_config;

/* Fills *cfg with defaults: 32^3, tau 0.6, the usual d'Humieres rates, no
 * force, no boundary, FP32 storage, ibm_iters 2, restitution 0.97, contact
 * time 8 steps, D3Q19. */
void lbm_config_default(lbm_config* cfg);

/* Bytes of device workspace a context with this configuration needs.
 * Errors: LBM_E_ARG for an invalid configuration; LBM_E_SIZE if
 * N = nx*ny*nz exceeds 2^31 - 1, or 2^30 with FP32 storage (one population
 * array must stay within 4 GiB). */
int lbm_workspace_size(const lbm_config* cfg, size_t* bytes);

/* Creates a context on the current HIP device. workspace: device pointer,
 * 256-byte aligned, >= lbm_workspace_size() bytes, owned by the caller.
 * stream: a hipStream_t (NULL = default stream). The context creates one
 * stream and two events of its own (released by lbm_destroy). The lattice
 * starts at rest with density 1. Errors: LBM_E_ARG, LBM_E_SIZE, LBM_E_HIP. */
int lbm_init(const lbm_config* cfg, void* workspace, size_t bytes,
             void* stream, lbm_ctx** out);

/* Sets every node to the equilibrium of (rho, u): u host [3][N] FP32,
 * rho host [N] FP32 or NULL for 1. Resets the step counter. Sync. */
int lbm_set_fields(lbm_ctx* ctx, const float* u, const float* rho);

/* Same, from device pointers on the context's stream. Async. */
int lbm_set_fields_device(lbm_ctx* ctx, const float* u_dev, const float* rho_dev);

/* Advances nsteps time steps (Sec. 2.1, Sec. 3.1): pull streaming fused
 * with MRT collision and body/boundary forcing, the no-slip treatment and
 * the particle update. Async; instability latches and is reported by the
 * next sync call. Errors: LBM_E_ARG if nsteps < 0. */
int lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* Density and half-force velocity u = (sum_i c_i f_i + F/2)/rho of the
 * current step at every node, to host [N] and [3][N] FP32 (either may be
 * NULL). At nodes inside an interpolated-bounce-back particle the values
 * are undefined. Sync. */
int lbm_get_fields(lbm_ctx* ctx, float* u, float* rho);

/* Same, into device buffers on the context's stream. Async. */
int lbm_get_fields_device(lbm_ctx* ctx, float* u_dev, float* rho_dev);

/* Waits for the stream; returns the first latched error, if any. */
int lbm_sync(lbm_ctx* ctx);

/* Number of completed time steps since the last lbm_set_fields(). */
int lbm_step_count(const lbm_ctx* ctx, int64_t* step);

/* ---- Checkpoint and restart ---------------------------------------------
 * The paper starts one pipe run from the velocity field of another to save
 * computing time (Sec. 2.2.1). A state blob holds everything later steps
 * depend on: the populations of the current step, the step counter, the
 * particle state in FP64 (centres, velocities, angular velocities, radii,
 * densities, motion mode), the momentum of the nodes covered or uncovered
 * in the previous step, the Kempe inner momentum, the forces of the last
 * update and, with the immersed boundary, the support and spread force of
 * the last collision (the velocity extraction of the current step reads
 * them). The boundary geometry is rebuilt from the centres on restore, with
 * the kernels the step uses, so a restored context continues bit for bit as
 * the original would. Not in the blob: the pipe budget sums, an attached
 * corrector, profiling counters, latched errors. The blob is host memory in
 * the library's own layout (native byte order), valid only for a context
 * with the same configuration.
 *
 * lbm_state_size: bytes of the current state (depends on the particle count
 *   and, with the immersed boundary, the support size). Sync.
 * lbm_get_state: copies the state to host (bytes >= lbm_state_size()).
 *   Sync. Errors: LBM_E_ARG (NULL), LBM_E_SIZE (bytes too small).
 * lbm_set_state: restores a blob of lbm_get_state() from a context with an
 *   identical configuration (another or the same context). Sync. Errors:
 *   LBM_E_ARG (NULL, not a state blob, another configuration, a particle
 *   block that lbm_set_particles would reject), LBM_E_SIZE (bytes shorter
 *   than the blob); the context is unchanged on these errors. */
int lbm_state_size(lbm_ctx* ctx, size_t* bytes);
int lbm_get_state(lbm_ctx* ctx, void* host, size_t bytes);
int lbm_set_state(lbm_ctx* ctx, const void* host, size_t bytes);

/* lbm_set_particles() modes. LBM_RELEASE follows Sec. 3.1: each particle
 * starts with the fluid velocity averaged over its volume (weighted by the
 * cell solid fraction) and zero angular velocity, and the populations at its
 * nodes are reset once to the equilibrium of the local density and that
 * velocity. LBM_SET_STATE takes u and omega as given. LBM_SET_RIGID takes
 * them as given and resets the populations at the particle's nodes once to
 * the equilibrium of the local density and the rigid-body velocity
 * U + Omega x (x - X) (the rigid interior of Sec. 3.1 with a given motion). */
enum { LBM_SET_STATE = 0, LBM_RELEASE = 1, LBM_SET_RIGID = 2 };
/* Particle motion: free (equations of motion with hydrodynamic and contact
 * forces), fixed in place, or prescribed (centres advance with the given
 * constant velocities). Forces are evaluated in every mode. */
enum { LBM_MOTION_FREE = 0, LBM_MOTION_FIXED = 1, LBM_MOTION_PRESCRIBED = 2 };

/* Places np rigid spheres (Sec. 3.1). Host arrays: x, u, omega [np][3]
 * (u, omega may be NULL for zero), radius [np], rho_p [np] (NULL for 1).
 * Centres are wrapped into the box. Requires bc = LBM_BC_IBB or LBM_BC_IBM,
 * np <= max_particles, 0 < radius <= max_radius, 2*radius + 8 <= min(nx,
 * ny, nz), no pipe wall; the immersed boundary needs one common radius.
 * Rebuilds the boundary geometry. Sync. Errors: LBM_E_ARG, LBM_E_SIZE. */
int lbm_set_particles(lbm_ctx* ctx, int32_t np, const double* x, const double* u, const double* omega,
                      const double* radius, const double* rho_p, int32_t mode, int32_t motion);

/* Number of particles set (lbm_set_particles, lbm_set_state). */
int lbm_particle_count(const lbm_ctx* ctx, int32_t* np);

/* Current particle state to host [np][3] arrays (any may be NULL). Sync. */
int lbm_get_particles(lbm_ctx* ctx, double* x, double* u, double* omega);

/* Hydrodynamic force and torque that entered the last particle update, and
 * the contact force, to host [np][3] (any may be NULL). Interpolated
 * bounce-back: sum of the link forces (Wen et al. momentum exchange) plus
 * the momentum of nodes covered/uncovered in the previous step. Immersed
 * boundary: minus the sum of the marker forces plus the change of the inner
 * fluid momentum (Kempe et al.). Sync. */
int lbm_forces(lbm_ctx* ctx, double* F, double* T, double* F_contact);

/* Number of boundary links of the current geometry (spheres and wall). Sync. */
int lbm_link_count(lbm_ctx* ctx, int64_t* n);

/* Copies up to cap links to host arrays: fluid node (x, y, z) [cap][3],
 * lattice direction c (towards the solid) [cap][3], owning particle [cap]
 * (-1 for the wall), wall fraction q [cap], scheme [cap] (2 quadratic,
 * 1 linear, 0 single-node). *n gets the number copied. Sync. */
int lbm_get_links(lbm_ctx* ctx, int64_t cap, int32_t* node, int32_t* dir, int32_t* particle, float* q,
                  int32_t* scheme, int64_t* n);

/* Sizes of the current geometry: nodes inside solids (spheres and wall,
 * interpolated bounce-back) and boundary links; either pointer may be NULL.
 * Sync. */
int lbm_geometry_counts(lbm_ctx* ctx, int64_t* solid_nodes, int64_t* links);

/* Immersed boundary: nodes of the current support set (the union of the
 * marker stencils and of the Kempe cells of every sphere, Sec. 2.1 and
 * Sec. 3.1; with a pipe wall its marker stencils too) and the nodes that
 * more than one sphere's support holds. Zero for other boundaries. Sync. */
int lbm_ibm_support(lbm_ctx* ctx, int64_t* support_nodes, int64_t* shared_nodes);

/* Statistics of the current snapshot (Sec. 3.2). Every sum is FP64, reduced
 * in a fixed order (bit-reproducible). Means are over all N nodes (raw and
 * masked) or over the N_f fluid nodes (*_fluid, bulk_u). A node is inside
 * sphere p iff its periodic minimum-image squared distance to X_p is below
 * r_p^2 (lowest index wins); inside the pipe wall iff
 * (x - cx)^2 + (y - cy)^2 >= R^2 (the wall wins).
 *   ke = 1/2 <|u|^2>; eps = 2 nu <s_ij s_ij>, nu = (tau - 1/2)/3, with
 *   s_ij = (d_i u_j + d_j u_i)/2 by periodic central differences
 *   (Sec. 3.2.1; the paper evaluates them spectrally).
 *   masked: u replaced by U_p + Omega_p x (x - X_p) inside particles and by
 *   0 inside the wall; raw: the lattice field as it is (not a physical field
 *   inside bounce-back solids).
 *   umax: max |u| over fluid nodes; bulk_u: <u_z> over fluid nodes (pipe).
 *   particle_ke = 1/2 sum m |U|^2, particle_ke_rot = 1/2 sum I |Omega|^2,
 *   m = rho_p 4/3 pi r^3, I = 2/5 m r^2 (Sec. 3.2.2). */
typedef struct {
  int64_t step;
  int64_t n_nodes, n_fluid;
  double mass;          /* sum of rho over fluid nodes   */
  double momentum[3];   /* sum of rho u over fluid nodes */
  double ke_raw, ke_masked, ke_fluid;
  double eps_raw, eps_masked, eps_fluid;
  double umax, bulk_u;
  double particle_ke, particle_ke_rot;
  double eps_fluid_corrected;  /* eps_fluid with the corrector's gradients at
                                  its cells (= eps_fluid without one)     */
  int64_t n_corrected;         /* cells the corrector handled             */
} lbm_stats_t;

#define LBM_STATS_MAX_BINS 256

/* Computes the statistics of the current field and particle state. Local
 * profiles (Sec. 3.2.1): fluid node x falls in bin floor(d / bin_width) of
 * d = min(min_p |x - X_p| - r_p, R - |x_perp - c| with a pipe), if that bin
 * is below nbins. hist (host, [6][nbins], may be NULL; ignored if nbins is
 * 0) receives per bin the node count and the sums of 1/2 |u|^2, eps (of the
 * masked field), u_z, u_z^2 and the corrected eps. With a corrector attached
 * (lbm_corrector_set), eps at its interface cells is recomputed from the
 * corrected gradient (eps_fluid_corrected, hist row 5). Uses the idle
 * population buffer as scratch. Sync. Errors: LBM_E_ARG (nbins outside
 * 0 .. LBM_STATS_MAX_BINS, bin_width <= 0, out NULL), LBM_E_SIZE (corrector
 * zone larger than the lattice, or more interface cells than scratch). */
int lbm_stats(lbm_ctx* ctx, int32_t nbins, double bin_width, lbm_stats_t* out, double* hist);

#define LBM_PIPE_BUDGET_MOMENTS 38
#define LBM_PIPE_BUDGET_TERMS 13
#define LBM_PIPE_BUDGET_MAX_BINS 1024

/* Component-wise budget of the turbulent kinetic energy in the pipe, in
 * cylindrical coordinates (Sec. 2.2, Eq. (1a)-(1c)), averaged over radial
 * bins [k w, (k + 1) w) of the fluid nodes (r^2 < R^2) and over the snapshots
 * added since the last reset. Needs a pipe wall (LBM_WALL_PIPE_Z).
 *
 * Per node, from the masked field (as lbm_stats: zero in the wall, rigid
 * motion inside spheres) and its central-difference gradient
 * G_ij = d_j u_i, with e_r = (x_perp - c) / r (e_x on the axis) and
 * e_theta = e_z x e_r: u_r, u_theta, u_z; p = rho / 3; L_ab = e_a . G . e_b
 * (the physical cylindrical components of the velocity gradient, e.g.
 * L_r,theta = (1/r) du_r/dtheta - u_theta/r); s_ab = (L_ab + L_ba) / 2.
 *
 * lbm_pipe_budget_reset: clears the sums and sets the bin width w > 0
 * (ceil(R / w) <= LBM_PIPE_BUDGET_MAX_BINS bins). Sync. Errors: LBM_E_STATE
 * (no pipe wall), LBM_E_ARG (width).
 * lbm_pipe_budget_add: adds the current snapshot's sums (FP64, fixed order:
 * reproducible). Uses the idle population buffer as scratch. Sync. Errors:
 * LBM_E_STATE (not reset), LBM_E_SIZE (scratch too small).
 * lbm_pipe_budget_read: *nbins, *snapshots; moments (host,
 * [LBM_PIPE_BUDGET_MOMENTS][nbins], may be NULL): the sums, in the order
 *   count, u_r, u_t, u_z, p, s_rr, s_rt, s_rz, s_tt, s_tz, s_zz,
 *   L_zr, L_zt, L_zz, L_rr, L_rt, L_rz, L_tt, L_tr, L_tz,
 *   u_z u_r, u_r u_r, u_t u_r, u_z u_z, u_t u_t,
 *   p u_r, p L_zz, p L_rr, p L_tt, u_z s_zr, u_r s_rr, u_t s_tr,
 *   s_zr L_zr + s_zt L_zt + s_zz L_zz, s_rr L_rr + s_rt L_rt + s_rz L_rz,
 *   s_tt L_tt + s_tr L_tr + s_tz L_tz, u_z u_z u_r, u_r u_r u_r, u_t u_t u_r
 * (t = theta); terms (host, [LBM_PIPE_BUDGET_TERMS][nbins], may be NULL):
 *   E_Oz, E_Tz, E_Pz, E_Vz, E_Dz, E_Tr, E_Pr, E_Vr, E_Dr,
 *   E_Ttheta, E_Ptheta, E_Vtheta, E_Dtheta
 * of Eq. (1) from the bin means, with a' = a - <a> (so <a'b'> = <ab> -
 * <a><b>, <a'a'b'> = <a^2 b> - 2<a><ab> - <b><a^2> + 2<a>^2<b>), d/dr by
 * central differences over the bin centres (k + 1/2) w (one-sided at the
 * first and last bin), nu = (tau - 1/2) / 3; empty bins give NaN. Sync.
 * Errors: LBM_E_STATE (not reset), LBM_E_ARG (nbins or snapshots NULL). */
int lbm_pipe_budget_reset(lbm_ctx* ctx, double bin_width);
int lbm_pipe_budget_add(lbm_ctx* ctx);
int lbm_pipe_budget_read(lbm_ctx* ctx, int32_t* nbins, int64_t* snapshots, double* moments, double* terms);

#define LBM_SPECTRUM_MAX_SHELL 4096

/* Three-dimensional spectra of the kinetic energy and of its dissipation
 * rate of the current field (Sec. 3.2.1). With
 * u^(k) = (1/N) sum_x u(x) exp(-2 pi i k.x / L), k in integer wavenumbers of
 * the periodic box (k_max = n/2 along an axis of n nodes),
 *   E[s] = 1/2 sum over round(|k|) = s of |u^(k)|^2,  D[s] = 2 nu s^2 E[s],
 * for s = 0 .. kmax, so that the sum of E over all shells is 1/2 <|u|^2>
 * over the N nodes (Parseval). masked != 0 replaces the velocity inside each
 * sphere by its rigid-body motion U + Omega x (x - X) and zeroes the pipe
 * wall, as the masked statistics do; with interpolated bounce-back the
 * interior holds no fluid, so only the masked spectrum is meaningful there.
 * E (host, [kmax + 1]) is required, D (host, [kmax + 1]) may be NULL;
 * shells above kmax are not reported. FP32 transform, FP64 shell sums in a
 * fixed order (reproducible). Uses the idle population buffer as scratch.
 * Sync. Errors: LBM_E_ARG (E NULL, kmax outside 0 .. LBM_SPECTRUM_MAX_SHELL,
 * a lattice side not a power of two or above 1024). */
int lbm_spectrum(lbm_ctx* ctx, int32_t masked, int32_t kmax, double* E, double* D);

/* ---- Gradient-corrector network ----------------------------------------
 * The paper finds the immersed boundary smears near-surface velocity
 * gradients, so the local dissipation next to particles differs from the
 * bounce-back result (Sec. 3.2.1, Sec. 4). The corrector maps the
 * neighbourhood of an interface cell to its velocity gradient: a multilayer
 * perceptron 85 -> 64 -> 64 -> 9 with SiLU activations,
 *   z1 = W1 x + b1, h1 = silu(z1), z2 = W2 h1 + b2, h2 = silu(z2),
 *   y = W3 h2 + b3,
 * trained on the mean squared error with Adam. Parameters are one FP32
 * vector of LBM_MLP_PARAMS: W1 (64x85, [out][in]), b1, W2 (64x64), b2,
 * W3 (9x64), b3. Matrix products run on the matrix cores with BF16 weights
 * and activations and FP32 accumulation; the master parameters and the
 * Adam moments are FP32.
 * Features: device BF16 rows of LBM_MLP_IN_STRIDE (entries 85..95 zero).
 * Targets and outputs: device FP32 rows of LBM_MLP_OUT_STRIDE (9 used). */
#define LBM_MLP_IN 85
#define LBM_MLP_IN_STRIDE 96
#define LBM_MLP_OUT 9
#define LBM_MLP_OUT_STRIDE 16
#define LBM_MLP_PARAMS 10249

typedef struct lbm_mlp lbm_mlp;

/* Bytes of the device workspace of one network (parameters, Adam moments,
 * gradient and reduction partials). */
size_t lbm_mlp_workspace_size(void);

/* Binds a network to a caller-allocated device workspace (256-byte aligned,
 * at least lbm_mlp_workspace_size() bytes, outliving the handle) and the
 * caller's hipStream_t; copies the host parameters and zeroes the Adam
 * state. Sync. Errors: LBM_E_ARG, LBM_E_SIZE. */
int lbm_mlp_init(void* workspace, size_t bytes, const float* params_host, void* hip_stream, lbm_mlp** out);

/* Replaces the parameters (host) and resets the Adam state. Sync. */
int lbm_mlp_set_params(lbm_mlp* mlp, const float* params_host);

/* Current parameters to host. Sync. */
int lbm_mlp_get_params(lbm_mlp* mlp, float* params_host);

/* Device address of the FP32 parameter vector (for lbm_corrector_set). */
const float* lbm_mlp_device_params(const lbm_mlp* mlp);

/* y[n][16] = network(x[n][96]) for n >= 0 samples (device buffers, both
 * 16-byte aligned, else LBM_E_ARG). Async. */
int lbm_mlp_forward(lbm_mlp* mlp, const uint16_t* x_dev, int64_t n, float* y_dev);

/* Gradient of L = mean over the n samples and 9 outputs of (y - t)^2 at the
 * current parameters, kept for lbm_mlp_adam_step. If loss or grad (host,
 * LBM_MLP_PARAMS) is non-NULL the call syncs and returns them. Errors:
 * LBM_E_ARG (n <= 0). */
int lbm_mlp_gradient(lbm_mlp* mlp, const uint16_t* x_dev, const float* t_dev, int64_t n, double* loss,
                     float* grad_host);

/* The gradient of lbm_mlp_gradient without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * training or serving loops, harnesses that forbid allocation): no network
 * handle or workspace; the parameters (device FP32, LBM_MLP_PARAMS, e.g.
 * lbm_mlp_device_params()), the n features x and targets t (device, as for
 * lbm_mlp_gradient) are inputs, grad (device FP32, LBM_MLP_PARAMS) receives
 * the gradient of the mean loss and loss_sum (device FP64, one value) the
 * sum over the n samples and 9 outputs of (y - t)^2 (the mean loss is
 * loss_sum / (9 n)); both equal what lbm_mlp_gradient computes for the same
 * inputs. The per-workgroup partial sums go to a scratch array of fixed size
 * (256 x LBM_MLP_PARAMS FP32 plus 256 FP64, 10.5 MB) that the library holds
 * on each GPU it runs on until the process ends; every call on a GPU uses
 * that GPU's array, so calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller. Enqueued on stream
 * (a hipStream_t, NULL for the default stream) on the current device; async.
 * Errors: LBM_E_ARG (a NULL pointer, n <= 0), LBM_E_SIZE (n above
 * LBM_MLP_NOALLOC_MAX_SAMPLES), LBM_E_HIP. */
#define LBM_MLP_NOALLOC_MAX_SAMPLES (1ll << 30)
int lbm_mlp_gradient_noalloc(const float* theta_dev, const uint16_t* x_dev, const float* t_dev, int64_t n,
                             float* grad_dev, double* loss_sum_dev, void* hip_stream);

/* One Adam step (Kingma & Ba) with the last gradient:
 *   m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 *   theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * Async. Errors: LBM_E_ARG (no gradient yet, or rates out of range). */
int lbm_mlp_adam_step(lbm_mlp* mlp, double lr, double beta1, double beta2, double eps);

/* Waits for the network's stream. */
int lbm_mlp_sync(lbm_mlp* mlp);

/* Releases the handle (not the workspace). NULL is ignored. */
void lbm_mlp_destroy(lbm_mlp* mlp);

/* ---- Corrector on a lattice ---------------------------------------------
 * Interface cells of sphere p: fluid nodes with r_p <= |x - X_p| <
 * r_p - r_d + 2 (r_d = ibm_retraction: the marker radius plus the reach of
 * the 4-point delta) and d = |x - X_p| - r_p in [d_min, d_max]; a cell falls
 * back to the plain central difference when another sphere q has
 * |x - X_q| < r_q - r_d + 2 + sqrt(3) (its band or interior within the 3x3x3
 * stencil, or a gap below two spacings). Distances are periodic minimum-image,
 * squared as ((dx dx + dy dy) + dz dz) and compared squared.
 * Features (85): for the 27 offsets o (z slowest, x fastest, each -1, 0, 1)
 * and components c, (u_c(x + o) - [U_p + Omega_p x (x + o - X_p)]_c) / u_rms
 * of the lattice field; then d; then (x - X_p) / |x - X_p|. Labels (9):
 * G_ij / u_rms = (d_j u_i) / u_rms, row-major in (i, j), by central
 * differences of the masked field (as lbm_stats). The network predicts the
 * correction of the plain immersed-boundary gradient, y = (G_ref - G_plain) /
 * u_rms with G_ref from a paired bounce-back run: its training targets are
 * the bounce-back labels minus the immersed-boundary labels at the same
 * cells, and the corrected gradient is G_plain + u_rms y. All three calls
 * require 2 (max_radius - r_d + 2 + sqrt(3)) + 3 <= min(nx, ny, nz)
 * (LBM_E_SIZE otherwise). */

/* Interface cells of the current state in ascending node order: node index
 * (x + nx (y + ny z)) and sphere of up to cap cells into device int32
 * arrays, and, if x_dev (device, 16-byte aligned, [cap][96] BF16) is not
 * NULL, their features. *n gets the number of cells; LBM_E_SIZE if it
 * exceeds cap (nothing beyond cap is written). Sync. */
int lbm_corrector_cells(lbm_ctx* ctx, double d_min, double d_max, double u_rms, int64_t cap, int32_t* node_dev,
                        int32_t* particle_dev, uint16_t* x_dev, int64_t* n);

/* Labels at n given nodes (device int32): the masked central-difference
 * gradient of this lattice's field / u_rms, written to t_dev ([n][16] FP32,
 * entries 9..15 zero), or subtracted from its entries if subtract != 0 (the
 * reference labels minus this lattice's: a training target). Sync. */
int lbm_corrector_labels(lbm_ctx* ctx, const int32_t* node_dev, int64_t n, double u_rms, int32_t subtract,
                         float* t_dev);

/* Attaches a network for lbm_stats (params_dev: lbm_mlp_device_params(), must
 * stay valid while attached; NULL detaches) with the training range of d and
 * the velocity scale of the features. */
int lbm_corrector_set(lbm_ctx* ctx, const float* params_dev, double d_min, double d_max, double u_rms);

/* Kernel classes for lbm_profile_read(). */
enum {
  LBM_K_STREAM_COLLIDE = 0, /* fused pull-stream + MRT collision, all nodes  */
  LBM_K_GEOMETRY = 1,       /* solid mask, boundary links, support sets      */
  LBM_K_IBB_LINKS = 2,      /* interpolated bounce-back + link forces        */
  LBM_K_REFILL = 3,         /* refilling of uncovered nodes                  */
  LBM_K_IBM_PREPASS = 4,    /* density/velocity at immersed-boundary support */
  LBM_K_IBM_FORCING = 5,    /* interpolate / spread passes                   */
  LBM_K_PARTICLE = 6,       /* per-particle reductions, motion, contacts     */
  LBM_K_STATS = 7,          /* statistics                                    */
  LBM_K_CORRECTOR = 8,      /* learned gradient corrector                    */
  LBM_NPROF = 9
};

/* Overlap (on != 0; off after lbm_init): in every step with particles the
 * particle stage and the next step's geometry (owner map and links, or the
 * immersed-boundary support) run on a second stream of the context, at the
 * default priority, beside the stream-collide kernel, which reads and
 * writes none of their data; the step joins that stream back into the
 * context's stream before its last kernel. Results are bit-identical with
 * and without overlap. At 512^3 with 6250 spheres it shortens a step by
 * about 5% (bounce-back) and 3% (immersed boundary); the stream-collide
 * kernel, sharing the device, takes longer by itself. Takes effect at the
 * next lbm_step(). Errors: LBM_E_ARG (null context). */
int lbm_set_overlap(lbm_ctx* ctx, int32_t on);

/* Enables (on != 0) or disables per-kernel timing: every kernel that
 * lbm_step() launches is bracketed by HIP events on the context's stream,
 * grouped by the classes above. Timing adds event overhead; leave it off
 * for throughput runs. */
int lbm_profile_enable(lbm_ctx* ctx, int32_t on);

/* Sync. Writes, per class, the summed kernel time in milliseconds and the
 * number of timed launches since the last read (arrays of LBM_NPROF), then
 * resets the counters. Either pointer may be NULL. */
int lbm_profile_read(lbm_ctx* ctx, double* ms, int64_t* launches);

/* Releases the context (not the caller's workspace). NULL is ignored. */
void lbm_destroy(lbm_ctx* ctx);

/* Static text for a status code. */
const char* lbm_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
