/*
 * lbfreeze -- coupled lattice-Boltzmann solver for N-phase flow with
 * liquid-solid phase change on one AMD MI355X (gfx950).
 *
 * Method: Huang, Zhan, Chai, Huang, Liu, "A diffuse-interface model for
 * N-phase flows with liquid-solid phase change", arXiv:2603.22902.  One time
 * step couples (Sec. 3)
 *   - N conservative phase-field LBs g_{i,p} (conservative Allen-Cahn
 *     equation, eq. (eq_ph), with the pairwise source R_p),
 *   - the pressure-based flow LB f_i with the surface force F_s, the solid
 *     penalty force and the volume-change source of eq. (fluid2),
 *   - the total-enthalpy LB h_i with the enthalpy inversion of eq. (H),
 * on D2Q9 (2D) or D3Q19 (3D).  Lateral axes are periodic; the wall-normal
 * axis (y in 2D, z in 3D) ends in two faces, each a no-slip wall or an open
 * (zero-pressure) face, with a Dirichlet or adiabatic thermal condition.
 *
 * Calling conventions
 *   - Every function returns an lbf_status; nothing throws across the ABI.
 *   - The caller owns every host array and the device buffer given to
 *     lbf_create (size from lbf_state_bytes).  The library owns only the
 *     opaque context, never allocates device memory and never frees caller
 *     memory.
 *   - Host arrays are float64 in C order [field][z][y][x] (nz = 1 in 2D),
 *     whatever the device precision.
 *   - lbf_step is asynchronous on the stream bound at lbf_create.  The
 *     lbf_get_*, lbf_diagnostics and lbf_save_state calls synchronise that
 *     stream before returning.
 *   - A call that fails leaves the context unchanged unless stated otherwise;
 *     lbf_last_error() then holds a message.
 *   - Calls on one context must not overlap (one host thread at a time).
 */
#ifndef LBFREEZE_H
#define LBFREEZE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBF_OK = 0,
  LBF_EINVAL = -1,  /* invalid argument or parameter set            */
  LBF_ENOMEM = -2,  /* buffer too small / size overflow            */
  LBF_EDEVICE = -3, /* HIP runtime error                           */
  LBF_ENOTSUP = -4, /* valid but unsupported combination           */
  LBF_ENAN = -5,    /* non-finite state found by lbf_diagnostics   */
  LBF_ESTATE = -6   /* call out of order (e.g. step before init)   */
} lbf_status;

enum { LBF_FP32 = 0, LBF_FP64 = 1, LBF_MIXED = 2 };
enum { LBF_BC_WALL = 0, LBF_BC_OPEN = 1 };
enum { LBF_TBC_DIRICHLET = 0, LBF_TBC_ADIABATIC = 1 };

#define LBF_MAXP 4

/* Problem definition, lattice units (dx = dt = 1, c_s^2 = 1/3).
 * Phase p is described by liquid and solid values (eq. (eq2) mixes them
 * with the solid fraction f_s).  A phase with freezes[p] = 0 must have equal
 * liquid and solid values and zero latent heat.  Index [0] of the face
 * arrays is the low face (coordinate 0, the substrate), [1] the high face. */
typedef struct lbf_params {
  int dim;             /* 2 (D2Q9) or 3 (D3Q19)                                   */
  int nx, ny, nz;      /* cells; nz is ignored (taken as 1) in 2D                 */
  int nphase;          /* N, 1..LBF_MAXP                                         */
  int precision;       /* LBF_FP32: float32 storage and arithmetic; LBF_FP64:
                          float64 throughout; LBF_MIXED: float32 storage,
                          float64 arithmetic                                     */
  int flow_bc[2];      /* LBF_BC_WALL / LBF_BC_OPEN per wall-normal face          */
  int therm_bc[2];     /* LBF_TBC_DIRICHLET / LBF_TBC_ADIABATIC                   */
  double T_face[2];    /* temperature of Dirichlet faces                          */
  double rho_l[LBF_MAXP], rho_s[LBF_MAXP]; /* densities                            */
  double mu_l[LBF_MAXP], mu_s[LBF_MAXP];   /* dynamic viscosities                  */
  double lam_l[LBF_MAXP], lam_s[LBF_MAXP]; /* thermal conductivities               */
  double cp_l[LBF_MAXP], cp_s[LBF_MAXP];   /* specific heats                       */
  double latent[LBF_MAXP];                 /* latent heat L_p                      */
  int freezes[LBF_MAXP];                   /* 1 if phase p can solidify            */
  double sigma[LBF_MAXP][LBF_MAXP];        /* pairwise surface tension, symmetric  */
  double cos_theta[LBF_MAXP][LBF_MAXP];    /* wetting at the low wall, cos of the
                                              angle measured inside p; antisymmetric */
  double eps;          /* interface width parameter epsilon (> 0)                 */
  double tau_g;        /* phase-field relaxation time, mobility (tau_g-1/2)/3     */
  double T_melt;       /* solidus = liquidus temperature                          */
  double E_ref;        /* rho_ref C_p,ref of the enthalpy equilibrium (> 0)        */
  double gravity[3];   /* body force G = rho g                                    */
} lbf_params;

typedef struct lbf_ctx lbf_ctx;

/* Moment selection for lbf_get_moments; fields are written in this order,
 * each as one [nz][ny][nx] plane (PHI: N planes, U: dim planes). */
#define LBF_M_PHI (1u << 0)  /* order parameters phi_p                          */
#define LBF_M_RHOH (1u << 1) /* total enthalpy rho H                            */
#define LBF_M_T (1u << 2)    /* temperature                                     */
#define LBF_M_FL (1u << 3)   /* liquid fraction f_l                             */
#define LBF_M_RHO (1u << 4)  /* mixture density                                 */
#define LBF_M_U (1u << 5)    /* velocity u                                      */
#define LBF_M_P (1u << 6)    /* pressure                                        */
#define LBF_M_MDOT (1u << 7) /* volume-change source mdot of eq. (fluid2)       */
#define LBF_M_ALL 0xffu

/* Validate a parameter set without touching any device (host only).  Checks
 * sizes, N, relaxation times tau_f = 3 mu/rho + 1/2, tau_h = 3 lambda/E_ref
 * + 1/2 and tau_g all above 1/2 in every phase state, positive densities and
 * heat capacities, rho C_p >= (1 - w_0) E_ref (non-negative rest weight of
 * the enthalpy equilibrium), consistency of non-freezing phases, symmetric
 * sigma and antisymmetric cos_theta.  msg (may be NULL) receives the reason. */
lbf_status lbf_check_params(const lbf_params* prm, char* msg, size_t msg_len);

/* Device bytes the caller must provide to lbf_create for this problem:
 * two population buffers ((N+2) Q values per cell), two lagged-field
 * buffers (N + dim + 3 values per cell), one float64 staging plane and the
 * reduction scratch of lbf_diagnostics. */
lbf_status lbf_state_bytes(const lbf_params* prm, size_t* bytes);

/* Bind a context to caller-owned device memory dev_buf (at least
 * lbf_state_bytes, 256-byte aligned) on the current HIP device, and to the
 * HIP stream hip_stream (a hipStream_t; NULL = default stream).  The state
 * is undefined until lbf_init_fields. */
lbf_status lbf_create(const lbf_params* prm, void* dev_buf, size_t bytes, void* hip_stream,
                      lbf_ctx** out);

/* Initial fields (Sec. 3, equilibrium start).  phi: [N][cells] with
 * sum_p phi_p = 1 within 1e-12 and phi_p >= -1e-12; T: [cells]; u: [dim][cells]
 * or NULL for rest; p: [cells] or NULL for zero.  Cells with T > T_melt start
 * liquid, the rest solid; rho H follows from eq. (H); every population starts
 * at its equilibrium.  Clears the sticky LBF_ENAN state. */
lbf_status lbf_init_fields(lbf_ctx* ctx, const double* phi, const double* T, const double* u,
                           const double* p);

/* Advance nsteps >= 0 time steps, Sec. 3.  Each step is two kernel launches
 * on the context's stream: a moments pass (phi_p, f_s of every cell from its
 * populations) and a collide pass (finite differences, interface and flow
 * sources, the three collisions, push streaming and boundary rules). */
lbf_status lbf_step(lbf_ctx* ctx, int nsteps);

/* lbf_step with per-kernel timing: the same launches, bracketed by HIP events
 * on the context's stream.  On return (the stream has been synchronised)
 * ms[0] and ms[1] hold the average duration per step, in milliseconds, of
 * the moments and the collide launch.  1 <= nsteps <= 4096 (LBF_EINVAL
 * otherwise); ms must point to 2 doubles.  The state advances exactly as
 * with lbf_step. */
lbf_status lbf_step_timed(lbf_ctx* ctx, int nsteps, double* ms);

/* Macroscopic fields at the current time level (moments of the current
 * populations, inversion, and the flow macros u, p, mdot of Sec. 3), for the
 * fields selected by mask, into out (float64, planes in LBF_M_* order). */
lbf_status lbf_get_moments(lbf_ctx* ctx, unsigned mask, double* out);

/* Current populations as float64 [(N+2)*Q][cells]: lattice 0 = f,
 * 1..N = g_p, N+1 = h; direction order of the lattice tables in DESIGN notes
 * (D2Q9: rest, +x, +y, -x, -y, then the four diagonals (+,+), (-,+), (-,-),
 * (+,-); D3Q19: rest, +-x, +-y, +-z, then xy, xz, yz pairs). */
lbf_status lbf_get_populations(lbf_ctx* ctx, double* out);

/* Lagged fields as float64 [N + dim + 3][cells]: phi_p^{n-1}, f_s^{n-1},
 * u^{n-1}, the velocity divergence D^{n-1} and (rho C_p T D)^{n-1}. */
lbf_status lbf_get_aux(lbf_ctx* ctx, double* out);

/* Conservation diagnostics at the current time level, float64:
 * out[0..N) phase masses sum phi_p [f_s rho_p^s + (1-f_s) rho_p^l],
 * out[N..2N) solid volumes sum f_s phi_p, out[2N..3N) volumes sum phi_p,
 * out[3N] sum rho H, out[3N+1] max |sum_p phi_p - 1|, out[3N+2] front
 * position sum f_s psi / (cells per wall layer) with psi the freezing
 * phases' fraction, out[3N+3] 1 if any phi or rho H is non-finite.
 * Returns LBF_ENAN (sticky until lbf_init_fields/lbf_load_state) if so. */
lbf_status lbf_diagnostics(lbf_ctx* ctx, double* out);

/* lbf_diagnostics for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops): the same values and
 * status, with the reduction's per-block partials and result kept in a
 * static device array of LBF_DIAG_MAX_BLOCKS * LBF_DIAG_MAX_VALUES +
 * LBF_DIAG_MAX_VALUES doubles (131 KB, one copy per device, held until the
 * process ends) instead of the context's buffer.  Calls no allocating
 * routine.  Calls that overlap on one device share that array and race:
 * serialise them (one stream, or host synchronisation).  LBF_EINVAL if the
 * reduction would need more than the array holds (never for N <= 4). */
#define LBF_DIAG_MAX_BLOCKS 1024
#define LBF_DIAG_MAX_VALUES 16
lbf_status lbf_diagnostics_noalloc(lbf_ctx* ctx, double* out);

/* Opaque snapshot of the whole state (populations, lagged fields, step
 * count).  bytes must equal lbf_snapshot_bytes. */
lbf_status lbf_snapshot_bytes(const lbf_ctx* ctx, size_t* bytes);
lbf_status lbf_save_state(lbf_ctx* ctx, void* host, size_t bytes);
lbf_status lbf_load_state(lbf_ctx* ctx, const void* host, size_t bytes);

/* Device-side state copies (for checkpointing on the GPU).  A device state
 * is the populations followed by the lagged fields, in the storage type,
 * lbf_state_device_bytes long.  lbf_state_to_device copies the current state
 * to dst (asynchronous on the context's stream); lbf_state_from_device makes
 * src the current state and sets the step count to steps (clears LBF_ENAN). */
lbf_status lbf_state_device_bytes(const lbf_ctx* ctx, size_t* bytes);
lbf_status lbf_state_to_device(lbf_ctx* ctx, void* dst);
lbf_status lbf_state_from_device(lbf_ctx* ctx, const void* src, long long steps);
/* One time step from device state src to device state dst (distinct, each
 * lbf_state_device_bytes), asynchronous on the context's stream; the
 * context's own state and step count are not touched (recomputation of a
 * checkpoint window straight into its tape). */
lbf_status lbf_step_states(lbf_ctx* ctx, const void* src, void* dst);

/* ---- Reverse mode: the discrete adjoint of the Sec. 3 step ----------------
 * Gradient of an objective of the final state (lbf_adjoint_seed_objective:
 * the frozen fraction of the freezing material, J = sum_x f_s psi / sum_x psi
 * with psi the sum of the freezing phases' phi_p, or the front position),
 * f_s and phi_p the moments of the final state, with respect to
 * T_face[2], latent[4] and cos_theta[4][4] (each entry independent), through
 * every step of the run and the equilibrium start (lbf_init_fields with u
 * and p zero).  Built for dim = 2 with LBF_FP32 or LBF_FP64 (LBF_ENOTSUP
 * otherwise), for grids whose largest adjoint buffer spans less than 2 GiB
 * (lbf_adjoint_bytes returns LBF_EINVAL beyond: about 3 150^2 cells in
 * float32 with N = 4).  The inversion of eq. (H) and the regularised norm of the
 * pairwise normals are piecewise smooth: the derivative of the branch taken
 * is used.
 *
 * Use: run the forward steps keeping device states x^0..x^K (or checkpoints
 * and recomputation); with x^K current, lbf_adjoint_seed; then for
 * n = K-1 .. 0, lbf_adjoint_step with x^n (and x^{n+1}); then
 * lbf_adjoint_finish with x^0 and lbf_adjoint_gradient.  All calls are
 * asynchronous on the context's stream except seed and gradient, which
 * synchronise it.  The adjoint
 * context reads the forward context's parameters and stream; it must not
 * outlive it.  The caller allocates lbf_adjoint_bytes of device memory
 * (256-byte aligned) and keeps it for the adjoint context's lifetime. */
typedef struct lbf_adj lbf_adj;
lbf_status lbf_adjoint_bytes(const lbf_params* prm, size_t* bytes);
lbf_status lbf_adjoint_create(lbf_ctx* ctx, void* dev_buf, size_t bytes, lbf_adj** out);
/* Objectives of the final state x^K (psi = the freezing phases' fraction,
 * f_s the solid fraction of eq. (H)'s inversion):
 *   LBF_OBJ_FROZEN_FRACTION  J = sum f_s psi / sum psi, the frozen fraction
 *                            of the freezing material;
 *   LBF_OBJ_FRONT            J = sum f_s psi / (cells per wall layer), the
 *                            front position as a volume-equivalent solid
 *                            thickness (out[3N+2] of lbf_diagnostics). */
#define LBF_OBJ_FROZEN_FRACTION 0
#define LBF_OBJ_FRONT 1
/* The objective of the context's current state into *J (may be NULL);
 * resets the gradient and sets the adjoint state to dJ/dx^K.  LBF_EINVAL
 * for an unknown objective, or for the frozen fraction of a state that
 * holds no freezing material. */
lbf_status lbf_adjoint_seed_objective(lbf_adj* adj, int objective, double* J);
/* lbf_adjoint_seed_objective with LBF_OBJ_FROZEN_FRACTION. */
lbf_status lbf_adjoint_seed(lbf_adj* adj, double* J);
/* One reverse step: state = device state x^n (layout of lbf_state_to_device)
 * of the step whose output's adjoint is current; afterwards the adjoint of
 * x^n is current and the step's parameter terms are added.  next = the
 * device state x^{n+1} = step(x^n), or NULL: its lagged fields hold the
 * moments of x^n, which are otherwise recomputed (one more pass). */
lbf_status lbf_adjoint_step(lbf_adj* adj, const void* state, const void* next);
/* Adds the dependence of the equilibrium start x^0 on the latent heats. */
lbf_status lbf_adjoint_finish(lbf_adj* adj, const void* state0);
/* grad[22] (float64): [0..1] dJ/dT_face, [2..5] dJ/dlatent,
 * [6..21] dJ/dcos_theta[p][q] row-major. */
lbf_status lbf_adjoint_gradient(lbf_adj* adj, double* grad);
/* Current adjoint state as float64, in the layouts of lbf_get_populations
 * and lbf_get_aux. */
lbf_status lbf_adjoint_state(lbf_adj* adj, double* pops, double* aux);
/* Release the adjoint context (not its buffer).  NULL is a no-op. */
lbf_status lbf_adjoint_destroy(lbf_adj* adj);

/* ---- Batched cases ---------------------------------------------------------
 * Many independent 2D cases (any grid sizes, parameters and phase counts;
 * one precision, one device) advance together: per time step, one moments
 * launch and one collide launch over all cases of each phase count N.  Each
 * case's result is bitwise that of lbf_step on its own context.  A batch
 * needs a non-default HIP stream (it is captured into a graph); it orders its
 * launches after nothing else, so the caller synchronises the members'
 * streams before batch calls.  Members must not be stepped on their own while
 * in the batch (LBF_ESTATE); lbf_batch_step and lbf_batch_replay update their
 * states and step counts.  The caller allocates lbf_batch_bytes of device
 * memory (256-byte aligned; the case tables and their block-to-case maps)
 * for the batch's lifetime. */
typedef struct lbf_batch lbf_batch;
lbf_status lbf_batch_bytes(lbf_ctx* const* ctxs, int n, size_t* bytes);
lbf_status lbf_batch_create(lbf_ctx* const* ctxs, int n, void* dev_buf, size_t bytes, void* hip_stream,
                            lbf_batch** out);
/* Row tile per phase count: tile[N-1] in {64, 128, 256}, 0 keeps the current
 * one (the default is 128).  This and lbf_batch_tune rewrite the case tables
 * and drop a captured graph: lbf_batch_replay then returns LBF_ESTATE until
 * the next lbf_batch_capture. */
lbf_status lbf_batch_set_tiles(lbf_batch* b, const int* tile);
/* Autotuner: for each phase count, time trial_steps passes with each row tile
 * (passes that read the current states and write only the scratch buffers,
 * so the states do not change) and keep the fastest; tile[4] receives the
 * choice (0 where the batch has no case of that N); tile may be NULL. */
lbf_status lbf_batch_tune(lbf_batch* b, int trial_steps, int* tile);
/* How the batched passes are launched (lbf_batch_create sets
 * LBF_BATCH_CONCURRENT when the batch holds more than one phase count, and
 * nothing else):
 * LBF_BATCH_PERSISTENT launches each pass with a fixed number of blocks,
 * each block striding over the pass's work items (moment blocks; collide
 * tiles with their layer chunk) instead of one block per item: grid blocks
 * (a positive multiple of 8), or with grid = 0 as many as the GPU holds at
 * once (the kernel's occupancy times the compute units), never more than
 * the items.  LBF_BATCH_CONCURRENT runs the phase-count groups on streams of
 * their own, forked from and joined back to the batch's stream (parallel
 * branches of a captured graph); the batched reverse steps
 * (lbf_batch_adjoint_step) follow it too.  The states and gradients are
 * bitwise the same in every mode.  Drops a captured graph; LBF_EINVAL for
 * unknown flags or a grid that is negative or not a multiple of 8,
 * LBF_EDEVICE if the side streams cannot be created. */
#define LBF_BATCH_PERSISTENT 1u
#define LBF_BATCH_CONCURRENT 2u
lbf_status lbf_batch_set_launch(lbf_batch* b, unsigned flags, int grid);
/* nsteps batched steps, launched one by one (asynchronous on the batch's
 * stream). */
lbf_status lbf_batch_step(lbf_batch* b, int nsteps);
/* Capture two batched steps into a HIP graph (replacing a previous one);
 * lbf_batch_replay launches it times times (2 * times steps). */
lbf_status lbf_batch_capture(lbf_batch* b);
lbf_status lbf_batch_replay(lbf_batch* b, int times);
/* Release the batch (not the contexts or the buffer).  NULL is a no-op. */
lbf_status lbf_batch_destroy(lbf_batch* b);

/* Packed batch states (checkpoints and the tape of a batched reverse
 * sweep): every case's device state (layout of lbf_state_to_device) in the
 * order of the contexts given to lbf_batch_create, each at a 256-byte
 * aligned offset; lbf_batch_state_bytes is the size of one.  The caller owns
 * the device memory (256-byte aligned).  lbf_batch_state_to_device copies
 * the members' current states; lbf_batch_step_states advances every case
 * by one step from src to dst (distinct) in one launch per pass and phase
 * count, with the bitwise result of lbf_step_states per case; neither
 * touches the members' own states.  Asynchronous on the batch's stream. */
lbf_status lbf_batch_state_bytes(const lbf_batch* b, size_t* bytes);
lbf_status lbf_batch_state_to_device(lbf_batch* b, void* dst);
/* The reverse copy: every member's current state becomes its slice of the
 * packed state src (as lbf_state_from_device does per context), and its
 * step count advances by advance (how many steps src is ahead of the
 * members' current states).  Asynchronous on the batch's stream;
 * LBF_EINVAL for a NULL or unaligned src or a negative advance. */
lbf_status lbf_batch_state_from_device(lbf_batch* b, const void* src, long long advance);
lbf_status lbf_batch_step_states(lbf_batch* b, const void* src, void* dst);

/* Batched reverse step (2D, float32 or float64; the objectives and the
 * gradient of the single-case reverse step, per case).  The two per-step
 * passes run as one launch each per phase count over all cases; each case
 * keeps its single-case block decomposition and gradient rows, so its J and
 * gradient are bitwise those of a single-case sweep over the same states.
 * Sweep: lbf_batch_adjoint_seed with the packed final state x^K; for
 * n = K-1 .. 0, lbf_batch_adjoint_step with the packed x^n and x^{n+1}
 * (both required); lbf_batch_adjoint_finish with the packed x^0;
 * lbf_batch_adjoint_gradient.  The caller allocates lbf_batch_adjoint_bytes
 * of device memory (256-byte aligned: case tables and each case's adjoint
 * buffer) for the object's lifetime, which must not exceed the batch's.
 * All calls run on the batch's stream; seed and gradient synchronise it.
 * LBF_ENOTSUP if a member has no reverse step (3D, or float32 storage with
 * float64 arithmetic). */
typedef struct lbf_batch_adj lbf_batch_adj;
lbf_status lbf_batch_adjoint_bytes(const lbf_batch* b, size_t* bytes);
lbf_status lbf_batch_adjoint_create(lbf_batch* b, void* dev_buf, size_t bytes, lbf_batch_adj** out);
/* objective: LBF_OBJ_FROZEN_FRACTION or LBF_OBJ_FRONT; J (may be NULL)
 * receives one value per case, in caller order. */
lbf_status lbf_batch_adjoint_seed(lbf_batch_adj* adj, int objective, const void* state, double* J);
lbf_status lbf_batch_adjoint_step(lbf_batch_adj* adj, const void* state, const void* next);
lbf_status lbf_batch_adjoint_finish(lbf_batch_adj* adj, const void* state0);
/* grad[ncase][22], caller order, each row as lbf_adjoint_gradient. */
lbf_status lbf_batch_adjoint_gradient(lbf_batch_adj* adj, double* grad);
/* Release the object (not the buffer).  NULL is a no-op. */
lbf_status lbf_batch_adjoint_destroy(lbf_batch_adj* adj);

/* Steps taken since lbf_init_fields (restored by lbf_load_state). */
lbf_status lbf_step_count(const lbf_ctx* ctx, long long* steps);

/* Release the context (not the caller's device buffer). NULL is a no-op. */
lbf_status lbf_destroy(lbf_ctx* ctx);

/* Last error message of this context ("" if none); valid until the next call. */
const char* lbf_last_error(const lbf_ctx* ctx);
const char* lbf_status_string(lbf_status s);

/* HBM bandwidth probe, context for the kernels' roofline: the best rate of a
 * float4 grid-stride copy a -> b and of a float4 read-only sweep of a, over
 * a few launch shapes, each timed over reps launches with HIP events on
 * hip_stream (synchronises it).  a and b: caller-owned device buffers of
 * `bytes` each (16-byte aligned, distinct; the last 16 bytes of b are
 * scratch).  Rates in bytes per second (copy counts read + write).
 * LBF_EINVAL for bad arguments, LBF_EDEVICE on a HIP error. */
lbf_status lbf_bandwidth_probe(void* a, void* b, size_t bytes, void* hip_stream, int reps, double* copy_bytes_per_s,
                               double* read_bytes_per_s);

#ifdef __cplusplus
}
#endif
#endif /* LBFREEZE_H */
