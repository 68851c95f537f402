/*
 * lbm.h -- C ABI of the MI355X (gfx950) multi-component pseudo-potential lattice
 * Boltzmann step.
 *
 * Model: Peng, Ayala & Ayala, "A thermodynamically consistent pseudo-potential
 * lattice Boltzmann model for multi-component, multiphase, partially miscible
 * mixtures" (arXiv 1909.12390).  One step, in the order of Sec. 3.4:
 *   mixture Peng-Robinson pressure  (Sec. 3.2, Eq. MCPengRobinson + randommixingrule)
 *   pseudo-potential psi            (Sec. 3.1, Eq. psicorrected)
 *   total interaction force         (Sec. 3.3, Eq. coupledMCforce)
 *   split into components           (Sec. 3.1, Eqs. forcedistribution, distributionforce)
 *   collision with forcing          (Sec. 2.1, Eq. LBE with Eq. equilibrium; or the
 *                                    exact-difference method; BGK or MRT)
 *   streaming                       (Sec. 2.1, left side of Eq. LBE)
 *
 * Conventions shared by every entry point
 *   - Every call returns an lbm_status; nothing throws or aborts across the ABI.
 *     lbm_last_error() returns a thread-local message for the last failure.
 *   - Units are lattice units (dx = dt = 1, c_s^2 = 1/3) for the step; the thermo
 *     calls (lbm_critical, lbm_fugacity, lbm_flash, lbm_bubble_pressure,
 *     lbm_dew_pressure) accept any consistent unit system through lbm_mixture.R.
 *   - All thermodynamics and psi are float64.
 *   - Field layout on the device: structure of arrays, x fastest:
 *       cell = (z * ny + y) * nx + x,   cells = nx * ny * nz   (nz = 1 in 2-D)
 *       scalar field [cells]; per-component field [nc][cells];
 *       vector field [D][cells]; populations [nc][Q][cells].
 *   - "dev" pointers are device (HBM) pointers owned by the caller; "host" pointers
 *     are host memory, borrowed for the duration of the call.
 *   - Boundaries are periodic in every direction (Sec. 4 uses periodic domains),
 *     except where lbm_set_solid or lbm_box.solid installs solid walls (halfway
 *     bounce-back, see lbm_set_solid).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,          /* invalid argument (checked on the host before any launch)   */
  LBM_ERR_DOMAIN = -2,       /* EOS / psi left its domain on the device: b_m*rho~ >= 1,
                                negative argument of the square root in Eq. psicorrected,
                                sum_i gamma_i rbar_i <= 0, or a non-finite value           */
  LBM_ERR_HIP = -3,          /* a HIP runtime call failed                                    */
  LBM_ERR_NOCONVERGE = -4,   /* an iterative thermo solve did not converge                   */
  LBM_ERR_SINGLEPHASE = -5,  /* flash found one phase (trivial K or vapor fraction outside (0,1)) */
  LBM_ERR_UNSUPPORTED = -6   /* combination not built into this library                      */
} lbm_status;

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
enum { LBM_BGK = 0, LBM_MRT = 1 };
enum { LBM_GUO = 0, LBM_EDM = 1 };
/* Population storage.  F64: plain float64 populations, float64 collision.
 * F32_OFS / F16_OFS: per cell and component a float32 base b and Q offsets
 * r_a = f_a / b0 - w_a stored in float32 / float16 (round to nearest even), with
 * b0 = sum_a |f_a| carrying the sign of the cell's mass of the component, and b
 * rescaled after rounding so that the decoded populations
 * sum to the component's mass; decode f_a = b (w_a + r_a).  Collision in float32;
 * EOS, psi, the force stencil and the masses stay float64.  In the workspace the
 * offset formats keep the components of a cell side by side (offsets
 * [Q][cells][nc], bases [cells][nc]), float64 keeps [nc][Q][cells];
 * lbm_get_populations / lbm_set_populations convert from / to the float64
 * [nc][Q][cells] layout of the conventions above. */
enum { LBM_F64 = 0, LBM_F32_OFS = 1, LBM_F16_OFS = 2 };
/* Kernel schedule of one step (identical results).
 * TWO_PASS: a density/EOS/psi pass over the whole box, then a collide pass.
 * BLOCKED : the same two passes slab by slab along the slowest axis (y in 2-D, z in
 *           3-D): psi on the slab plus one plane each side, then the collide pass of
 *           the slab, so the collide pass re-reads populations the psi pass has just
 *           brought into the last-level cache.  Slab height lbm_params.slab_planes
 *           (0 = sized for about 64 MiB of population input per slab).
 * OVERLAP : the density/EOS/psi pass slab by slab on a second stream the library
 *           creates (default priority), each slab's collide pass on the context's
 *           stream as soon as the psi of its slab and of the two neighbouring slabs
 *           is done, so the memory-bound psi pass of later slabs runs beside the
 *           arithmetic-bound collide pass of earlier ones.  Slab height as BLOCKED
 *           (0 = one eighth of the planes). */
enum { LBM_SCHED_TWO_PASS = 0, LBM_SCHED_BLOCKED = 1, LBM_SCHED_OVERLAP = 2 };

#define LBM_MAX_NC 4
#define LBM_MAX_Q 19

/* Component data (Sec. 3.2).  a_i, b_i per mole with gas constant R; molar mass
 * M_i converts the cell-volume (mass) densities of the populations to molar
 * densities; k = binary interaction coefficients zeta_ij (symmetric, zero diagonal). */
typedef struct {
  int nc;                    /* 1..4                                            */
  double R;
  double a[LBM_MAX_NC], b[LBM_MAX_NC], omega[LBM_MAX_NC], M[LBM_MAX_NC];
  double k[LBM_MAX_NC][LBM_MAX_NC];
} lbm_mixture;

typedef struct {
  int lattice;               /* LBM_D2Q9 | LBM_D3Q19                            */
  int nx, ny, nz;            /* nz must be 1 for D2Q9                           */
  int collision;             /* LBM_BGK | LBM_MRT                               */
  int forcing;               /* LBM_GUO | LBM_EDM                               */
  int storage;               /* LBM_F64 | LBM_F32_OFS | LBM_F16_OFS             */
  int schedule;              /* LBM_SCHED_TWO_PASS | LBM_SCHED_BLOCKED | LBM_SCHED_OVERLAP */
  int slab_planes;           /* BLOCKED: planes per slab (0 = automatic)        */
  double T;                  /* temperature                                     */
  double tau;                /* relaxation time, > 0.5 (Sec. 2.1)               */
  double G;                  /* interaction strength, < 0 (Sec. 4.1: only its sign matters) */
  double beta;               /* blending parameter of Eq. coupledMCforce        */
  double gamma[LBM_MAX_NC];  /* volatility coefficients, Eq. distributionforce, each in (0, 1];
                                all zero: taken from lbm_flash at (T, p_flash, z_flash) */
  double mrt_s[LBM_MAX_Q];   /* MRT: relaxation rate of each moment row (rows of the orthogonal
                                Lallemand-Luo D2Q9 / d'Humieres D3Q19 bases, in their order) */
  double accel[3];           /* uniform body acceleration g; adds rbar_sigma g to F_sigma */
  double p_flash;            /* gamma all zero: pressure and overall composition of the   */
  double z_flash[LBM_MAX_NC];/* two-phase flash whose gamma (Eq. gamma) is used           */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Result of a two-phase flash at (T, p, z) (Sec. 3.2 iso-fugacity; Sec. 2.2 relations). */
typedef struct {
  double V;                          /* vapor mole fraction                       */
  double x[LBM_MAX_NC], y[LBM_MAX_NC], K[LBM_MAX_NC];
  double Zl, Zv;                     /* compressibility factors                   */
  double rho_l, rho_v;               /* molar densities of the phases             */
  double rbar_l[LBM_MAX_NC];         /* cell-volume (mass) densities, liquid: rho_l x_i M_i */
  double rbar_v[LBM_MAX_NC];         /* ... vapor: rho_v y_i M_i                  */
  double gamma[LBM_MAX_NC];          /* Eq. gamma against the least volatile component */
  double fug_l[LBM_MAX_NC], fug_v[LBM_MAX_NC];
  double residual;                   /* Eq. error                                  */
  int iterations;
} lbm_flash_result;

/* ---------------------------------------------------------------------------
 * Time stepping (device)
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace lbm_init needs for (mix, prm): two population copies
 * (ping-pong) in the chosen storage, the psi field (two-pass schedule), reduction
 * partials and an error flag.  Pure host computation. */
lbm_status lbm_workspace_bytes(const lbm_mixture* mix, const lbm_params* prm, size_t* bytes);

/* Validate (mix, prm) on the host, bind the caller-owned device workspace
 * (dev, >= lbm_workspace_bytes, 256-byte aligned, must outlive the context) and
 * set the populations to equilibrium f_a = f^eq_a(rbar_sigma, u) (Eq. equilibrium a)
 * of the initial cell-volume densities rho_bar0 (dev, float64 [nc][cells]) and the
 * velocity u0 (dev, float64 [D][cells], or NULL for rest).  All work is enqueued
 * on `stream` (a hipStream_t; NULL = default stream).  Host-side rejections:
 * nc outside 1..4, tau <= 0.5, G >= 0, gamma outside (0, 1], non-positive a, b, M,
 * box sides < 1, nz != 1 for D2Q9, unknown enums -> LBM_ERR_ARG.  With gamma all
 * zero the flash at (T, p_flash, z_flash) supplies it (Sec. 3.1 Eq. gamma on the
 * phases of Sec. 3.2); its failures (LBM_ERR_SINGLEPHASE, LBM_ERR_NOCONVERGE, or
 * LBM_ERR_ARG for a bad p_flash / z_flash) are returned as they are.  For nc = 1
 * gamma does not enter the split; pass 1. */
lbm_status lbm_init(const lbm_mixture* mix, const lbm_params* prm, void* workspace_dev,
                    size_t workspace_bytes, const double* rho_bar0_dev, const double* u0_dev,
                    void* stream, lbm_ctx** out);

/* Capture `steps` time steps (rounded up to even, so the population buffers end
 * where they started) once per buffer parity in a HIP graph; lbm_step then
 * replays it for every full `steps` and launches the rest one by one.  0 (the
 * default) launches every kernel.  Needs a non-default stream (LBM_ERR_ARG
 * otherwise); the OVERLAP schedule keeps plain launches.  lbm_set_gamma and
 * lbm_set_solid drop captured graphs (their values are kernel arguments). */
lbm_status lbm_set_graph_steps(lbm_ctx* ctx, int steps);

/* Enqueue nsteps time steps (Sec. 3.4 order) on the context's stream.
 * Asynchronous: device domain errors are recorded in a device flag and reported by
 * the next lbm_moments or lbm_check. */
lbm_status lbm_step(lbm_ctx* ctx, int nsteps);

/* Macroscopic fields of the current state, each output optional (NULL = skip):
 *   rho_bar_dev [nc][cells]  cell-volume densities rbar_sigma (Sec. 2.1)
 *   u_dev       [D][cells]   physical velocity (sum_sigma j_sigma + F_total/2)/rho
 *   p_dev       [cells]      p_EOS (= hydrodynamic pressure of Eq. hydropressure)
 *   psi_dev     [cells]      pseudo-potential, Eq. psicorrected
 *   totals_host [2*nc + 2*D] mass of each component, total momentum sum(j + F_total/2),
 *                            net interaction force sum(F), as float64 sums in a fixed
 *                            (deterministic) order, then per component the number of
 *                            fluid cells where its cell-volume density is negative (the
 *                            scheme does not keep partial densities positive and nothing
 *                            is clamped: a trace component can cross zero in a phase
 *                            where it is nearly absent; the counts report it).
 * Synchronises the stream when totals_host != NULL; returns LBM_ERR_DOMAIN if the
 * device error flag is set. */
lbm_status lbm_moments(lbm_ctx* ctx, double* rho_bar_dev, double* u_dev, double* p_dev,
                       double* psi_dev, double* totals_host);

/* lbm_moments for callers that cannot allocate device memory or use a workspace
 * beyond the context's (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same outputs, bitwise, from the same kernels, but the
 * per-block partial sums and the totals live in a static device array of the library
 * (1 MiB per GPU, held until the process ends) instead of the context's workspace.
 * Allocates nothing.  Boxes whose partial sums exceed the array (more than
 * floor((1 MiB - 256) / (8 (2 nc + 2 D))) * 256 cells rounded to the launch grid:
 * about 2.4 M cells for D3Q19 with nc = 4) are rejected with LBM_ERR_ARG.  Every call
 * on a GPU uses that GPU's one array: calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  Synchronises the stream
 * when totals_host != NULL, like lbm_moments. */
lbm_status lbm_moments_noalloc(lbm_ctx* ctx, double* rho_bar_dev, double* u_dev, double* p_dev,
                               double* psi_dev, double* totals_host);

/* Export / import the populations of the current state as float64 [nc][Q][cells]
 * (dev), post-streaming (the f of Eq. LBE at time t), velocity order:
 *   D2Q9 : (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
 *   D3Q19: (0,0,0) (+-1,0,0) (0,+-1,0) (0,0,+-1) (+-1,+-1,0) (+-1,0,+-1) (0,+-1,+-1)
 *          each group with the sign pattern (+,+) (-,+) (+,-) (-,-) for pairs.
 * Import encodes into the context's storage (rounding for reduced precision). */
lbm_status lbm_get_populations(lbm_ctx* ctx, double* f_dev);
lbm_status lbm_set_populations(lbm_ctx* ctx, const double* f_dev);

/* lbm_step with HIP events recorded on the context's stream around every kernel
 * launch: kernel_ms_host[0] receives the summed duration (ms) of the density/psi
 * launches, kernel_ms_host[1] that of the collide launches.  Synchronises the
 * stream at the end.  Used by the benchmark to price the dominant kernel against
 * the roofline. */
lbm_status lbm_step_timed(lbm_ctx* ctx, int nsteps, double* kernel_ms_host);

/* Synchronise the stream and report the device error flag (LBM_OK / LBM_ERR_DOMAIN). */
lbm_status lbm_check(lbm_ctx* ctx);

/* Replace the volatility coefficients gamma_i of Eq. (gamma) used by the force split
 * (host, nc values in (0, 1]); the next enqueued step uses them.  The paper's gamma
 * depends on (T, p, z) (Sec. 3.1); this lets a caller re-flash at the evolving bulk
 * state and update it during a run. */
lbm_status lbm_set_gamma(lbm_ctx* ctx, const double* gamma_host);

/* Clear the device error flag. */
lbm_status lbm_clear_error(lbm_ctx* ctx);

/* Solid walls (porous media, the application that motivates the model in Sec. 1;
 * the paper defines no boundary, so this is a design of its own).
 * solid_host: one byte per cell in the field order of lbm_moments (x fastest),
 * nonzero = solid; NULL removes every wall.  psi_wall (finite, >= 0): the value of
 * psi on solid cells in the force stencil of Eq. (coupledMCforce) -- a wetting
 * parameter: above the fluid's psi the wall attracts it, below repels it.
 * Streaming uses halfway bounce-back: a population that would arrive at a fluid
 * cell from a solid one is the cell's own post-collision population of the
 * opposite direction.  Solid cells hold no fluid: no collision, zero populations,
 * zero density / velocity / pressure in lbm_moments, psi = psi_wall.
 * The call converts the current state: the canonical populations (lbm_get_populations)
 * of cells that stay fluid are kept, new solid cells are emptied (a cell that stops
 * being solid starts empty, outside the EOS domain, until lbm_set_populations fills
 * it).  It allocates the per-cell mask (4 bytes per cell, kept until lbm_destroy)
 * and a temporary of nc * Q * cells doubles, synchronises the stream, and is not
 * meant for graph capture.  Every schedule and the adjoint (lbm_step_adjoint,
 * lbm_adjoint: solid cells carry no adjoint) support walls. */
lbm_status lbm_set_solid(lbm_ctx* ctx, const unsigned char* solid_host, double psi_wall);

/* Release the context (not the caller's workspace). NULL is accepted. */
void lbm_destroy(lbm_ctx* ctx);

/* Thread-local text of the last error (never NULL). */
const char* lbm_last_error(void);

/* Streaming copy of `bytes` (a multiple of 16; dst and src dev, 16-byte aligned,
 * not overlapping) with 16-byte non-temporal loads and stores on `stream`, `grid`
 * workgroups of 256 threads (0 = 2048).  Not part of the model: it measures the
 * HBM bandwidth a kernel that reads and writes every byte once reaches, the
 * ceiling the step's kernels are compared with.  Asynchronous. */
lbm_status lbm_stream_copy(void* dst_dev, const void* src_dev, size_t bytes, int grid, void* stream);

/* ---------------------------------------------------------------------------
 * Thermodynamics (host, float64)
 * ------------------------------------------------------------------------- */

/* Critical constants implied by a_i, b_i (inverting the Sec. 3.2 definitions):
 * Tc_i = (Omega_b/Omega_a) a_i / (b_i R), pc_i = Omega_b R Tc_i / b_i. Outputs [nc]. */
lbm_status lbm_critical(const lbm_mixture* mix, double* Tc_host, double* pc_host);

/* State of nstates homogeneous cells given molar densities n (host, [nstates][nc]):
 * p from Eq. MCPengRobinson, Z = p / (rho~ R T) (no root choice), ln(phi_i) from
 * Eq. fugacitycoeff2 at the local composition, fugacity f_i = phi_i c_i p
 * (Eq. fugacity).  Outputs (host, any may be NULL): p [nstates], Z [nstates],
 * lnphi [nstates][nc], fug [nstates][nc]. */
lbm_status lbm_fugacity(const lbm_mixture* mix, double T, int nstates, const double* n_host,
                        double* p_host, double* Z_host, double* lnphi_host, double* fug_host);

/* Two-phase flash at (T, p, z) (z host [nc]): Wilson start, successive substitution
 * on K with the Gibbs-energy root choice of Eq. solutionselection, Rachford-Rice for
 * the vapor fraction.  LBM_ERR_SINGLEPHASE if no two-phase split exists. */
lbm_status lbm_flash(const lbm_mixture* mix, double T, double p, const double* z_host,
                     lbm_flash_result* out);

/* Bubble- and dew-point pressures of composition z at T (successive substitution). */
lbm_status lbm_bubble_pressure(const lbm_mixture* mix, double T, const double* z_host, double* p_out);
lbm_status lbm_dew_pressure(const lbm_mixture* mix, double T, const double* z_host, double* p_out);


/* ---------------------------------------------------------------------------
 * Batched boxes: many independent periodic boxes, each with its own mixture,
 * temperature and volatility coefficients (e.g. a sweep of flash states), advanced
 * together: each pass of a step (density/EOS/psi, then force/split/collide/store)
 * is one persistent launch over the (box, tile) work list; K steps can be captured
 * once in a HIP graph and replayed.  The per-box arithmetic is the single-box one.
 * Concatenated layouts: fields [box][nc_b][cells_b], populations [box][nc_b][Q][cells_b].
 * ------------------------------------------------------------------------- */
typedef struct {
  lbm_mixture mix;           /* the box's components (nc 1..4)                    */
  int nx, ny, nz;            /* nz = 1 for D2Q9; periodic                         */
  double T, tau, G, beta;
  double gamma[LBM_MAX_NC];  /* each in (0, 1]                                    */
  const unsigned char* solid;  /* host, one byte per cell (x fastest), nonzero =
                                  solid; NULL = no walls.  Same wall model as
                                  lbm_set_solid; read during lbm_batch_init only. */
  double psi_wall;           /* psi of the box's solid cells (finite, >= 0)       */
} lbm_box;

typedef struct {
  int lattice, collision, forcing, storage;   /* shared by every box              */
  int tile;                  /* cells per work-list tile: 64, 128 or 256 (0 = 256); the
                                collide pass runs nc_max x tile threads per workgroup */
  int graph_steps;           /* steps per captured HIP graph (rounded up to even; 0 = none).
                                Capture needs a non-default stream.               */
  int grid;                  /* workgroups of the persistent launch (0 = all resident) */
  double mrt_s[LBM_MAX_Q];
  double accel[3];
  int fused;                 /* 0: two launches per step (psi pass, collide pass).
                                1: one launch per step: each workgroup computes psi
                                for its tile's cells and their neighbours into LDS
                                (rows padded with their periodic images), then
                                collides from the pull it kept; populations equal the
                                two-launch step's bit for bit.  D2Q9 with float32 / float16 offset storage
                                and boxes with nx <= LBM_FUSED_MAX_NX only, else
                                lbm_batch_layout / lbm_batch_init return LBM_ERR_ARG. */
} lbm_batch_params;

#define LBM_FUSED_MAX_NX 2048

typedef struct lbm_batch lbm_batch;

/* Workspace bytes and the element counts of the concatenated field and population
 * layouts (any output may be NULL).  Host validation as for lbm_init, per box. */
lbm_status lbm_batch_layout(const lbm_box* boxes_host, int nboxes, const lbm_batch_params* prm,
                            size_t* workspace_bytes, size_t* field_elems, size_t* pop_elems);

/* Bind the caller's workspace (dev, 256-byte aligned), upload the box table and the
 * work list, and set every box to rest-equilibrium of rho0 (dev, float64, concatenated
 * [box][nc_b][cells_b]).  Synchronises `stream` once (host tables are uploaded). */
lbm_status lbm_batch_init(const lbm_box* boxes_host, int nboxes, const lbm_batch_params* prm,
                          void* workspace_dev, size_t workspace_bytes, const double* rho0_dev,
                          void* stream, lbm_batch** out);

/* Enqueue nsteps steps of every box (asynchronous; graph replays when configured). */
lbm_status lbm_batch_step(lbm_batch* b, int nsteps);

/* Export cell-volume densities (dev, concatenated [box][nc_b][cells_b]) and/or the
 * canonical float64 populations (dev, [box][nc_b][Q][cells_b]); either may be NULL. */
lbm_status lbm_batch_fields(lbm_batch* b, double* rho_bar_dev, double* f_dev);

/* Synchronise and report the device error flag of the batch. */
lbm_status lbm_batch_check(lbm_batch* b);

/* Synchronise and copy the per-box error flags (host int [nboxes], 1 = the box left
 * the EOS domain or produced a non-finite value) so a sweep can tell which states failed. */
lbm_status lbm_batch_box_errors(lbm_batch* b, int* flags_host);

/* Replace gamma of one box (host, nc_b values in (0, 1]); written to the device box
 * table in stream order; synchronises the stream.  Captured graphs read the table,
 * so later replays use the new values. */
lbm_status lbm_batch_set_gamma(lbm_batch* b, int box, const double* gamma_host);

/* Release the batch (not the caller's workspace); NULL is accepted. */
void lbm_batch_destroy(lbm_batch* b);

/* ---------------------------------------------------------------------------
 * Discrete adjoint (reverse-mode derivative of the step).  The paper does not
 * differentiate its model; these calls give the exact derivative of the discrete
 * step of Sec. 3.4 (the transpose of its Jacobian), evaluated in float64 at the
 * stored states, for every collision (BGK, MRT), forcing (exact difference, Guo),
 * storage, lattice and nc.
 * Parameters: the EOS tables aa_ij = sqrt(a_i alpha_i a_j alpha_j)(1 - k_ij) and
 * b_i of Eq. (randommixingrule) / Eq. (MCPengRobinson), chained to (k_ij, a_i, b_i)
 * with alpha_i following a_i and b_i through Tc_i (Sec. 3.2).
 * ------------------------------------------------------------------------- */

/* Device workspace bytes of lbm_adjoint for `nsteps` steps with a checkpoint every
 * `checkpoint_every` steps: two float64 adjoint population arrays, per-cell scratch,
 * ceil(nsteps/K) checkpoints and K - 1 recomputed states in the context's storage.
 * lbm_step_adjoint needs lbm_adjoint_workspace(ctx, 1, 1). */
lbm_status lbm_adjoint_workspace(const lbm_ctx* ctx, int nsteps, int checkpoint_every, size_t* bytes);

/* One reverse step at the context's current state f(t) (the state is not changed):
 *   h_next_dev [nc][Q][cells] float64: dL/d(post-streaming populations after the step)
 *   h_out_dev  [nc][Q][cells] float64: receives dL/d f(t) (must not alias h_next_dev)
 *   d_aa_host  [nc*nc] += dL/d aa_ij over ordered pairs (i, j) (aa_ij and aa_ji counted
 *              as separate entries);   d_b_host [nc] += dL/d b_i through the EOS.
 * Synchronises the stream; LBM_ERR_DOMAIN if the state is outside the EOS domain. */
lbm_status lbm_step_adjoint(lbm_ctx* ctx, const double* h_next_dev, double* h_out_dev, double* d_aa_host,
                            double* d_b_host, void* workspace_dev, size_t workspace_bytes);

/* Gradient run.  Advances the context by nsteps (as lbm_step), keeping a checkpoint
 * every checkpoint_every steps in the workspace; evaluates
 *   L = sum_i (x_i - x_target_i)^2,  x_i = N_i / sum_j N_j,  N_i = sum_{mask} rbar_i / M_i
 * over the cells with mask_dev[cell] != 0 (uint8 [cells]) of the final state; then
 * runs the adjoint back to the starting state, recomputing each segment's states
 * from its checkpoint.  Outputs (host): *loss_host, x_liq_host [nc] (may be NULL),
 * d_k_host [nc*nc] (symmetric; entry (i,j) = (j,i) = dL/dk_ij for the symmetric
 * parameter, diagonal 0), d_a_host [nc], d_b_host [nc].  Synchronises the stream. */
lbm_status lbm_adjoint(lbm_ctx* ctx, int nsteps, int checkpoint_every, const unsigned char* mask_dev,
                       const double* x_target_host, void* workspace_dev, size_t workspace_bytes,
                       double* loss_host, double* x_liq_host, double* d_k_host, double* d_a_host,
                       double* d_b_host);

/* Host chain rule from the EOS-table derivatives (d_aa over ordered pairs, d_b_direct
 * through the EOS) to d_k (as in lbm_adjoint), d_a and d_b, with alpha_i following
 * a_i and b_i through Tc_i (Sec. 3.2).  All arrays host float64. */
lbm_status lbm_eos_param_grad(const lbm_mixture* mix, double T, const double* d_aa_host,
                              const double* d_b_direct_host, double* d_k_host, double* d_a_host,
                              double* d_b_host);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
