/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the Euler-Lagrange bubble-column method of
 * Agarwal, Ravindra & Prakash, "Development of algorithm to model dispersed gas-liquid flow
 * using lattice Boltzmann method" (arXiv 1710.07073).
 *
 * The liquid is a D3Q19 BGK lattice-Boltzmann fluid with a per-cell body force (Sec. 2.2,
 * eq. (5)-(16)); bubbles are Lagrangian point particles (Sec. 2.1, eq. (1)-(4), Table 1) coupled
 * both ways through the clipped fourth-order polynomial mapping kernel (Sec. 3.2, eq. (18)-(21)).
 * One method step of Algorithm 1 is bubbles_step() followed by lbm_step(ctx, 1).
 *
 * Conventions
 *   - Lattice units: dx = dt_l = 1, liquid reference density 1. Cell (i, j, k) has its centre at
 *     (i, j, k); a non-periodic wall lies half a cell outside the outermost cells. Gravity acts
 *     along -z. Bubble sub-step dt_b = 1 / n_sub.
 *   - Populations are stored shifted by their weights, g_q = f_q - w_q, q in the paper's
 *     velocity order of eq. (7): the six axis directions (+x, -x, +y, -y, +z, -z), the twelve
 *     face diagonals (+x+y, -x+y, +x-y, -x-y, +x+z, -x+z, +x-z, -x-z, +y+z, -y+z, +y-z, -y-z) and
 *     the rest particle. Population buffers are plane-blocked, pop[z][q][y][x] (x fastest: the
 *     19 populations of a z-plane are 19 consecutive planes), or plain structure of arrays
 *     pop[q][z][y][x] with LBM_FLAG_PLAIN_SOA. Exported populations (lbm_populations) are always
 *     pop[q][z][y][x]. Vector fields are vec[a][z][y][x], a = x, y, z. Field element type is
 *     float for LBM_FP32_SHIFTED and double for LBM_FP64_SHIFTED.
 *   - Memory: every buffer is caller-owned device memory (hipMalloc / torch allocations). The
 *     library never allocates or frees device memory; the context itself is host memory owned by
 *     the library and released by lbm_destroy(). The one device array the library holds, the
 *     workspace of bubbles_step_static_work(), is a static array of its code object.
 *   - Streams: every call enqueues its kernels on the stream given to lbm_init() (or
 *     lbm_set_stream()) and returns without waiting, except where stated. NULL = default stream.
 *   - Errors: argument errors are detected on the host and returned at once as LBM_EINVAL,
 *     without enqueuing anything. Launch failures return LBM_EDEVICE. Errors raised inside
 *     kernels (a bubble too large for the stencil limit) are recorded in device memory and
 *     reported by the next synchronising call (moments() with sums, lbm_check()).
 *   - Threading: a context is not thread-safe; calls on one context must be serialised.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,       /* bad argument */
  LBM_EUNSUPPORTED = -2, /* valid request outside what this build supports */
  LBM_EDEVICE = -3,      /* HIP runtime or launch error */
  LBM_EDIVERGED = -4     /* non-finite global sums: the BGK step went unstable */
} lbm_status;

typedef enum { LBM_FP32_SHIFTED = 1, LBM_FP64_SHIFTED = 2 } lbm_precision;

/* Face conditions (Sec. 3.3): half-way bounce-back no-slip wall, free-slip (specular) wall,
 * periodic (both faces of an axis must then be periodic). */
typedef enum { LBM_BC_BOUNCE_BACK = 0, LBM_BC_FREE_SLIP = 1, LBM_BC_PERIODIC = 2 } lbm_bc;

/* Behaviour flags of lbm_desc.flags. */
enum {
  /* Read the force field in every cell on every step and never clear it (a user-supplied
   * steady body force, e.g. a driven channel). Not allowed together with bubbles_step(). */
  LBM_FLAG_STATIC_FORCE = 1,
  /* Write the collision velocity U in every cell, not only near bubbles. */
  LBM_FLAG_WRITE_U_ALL = 2,
  /* population buffers in plain structure-of-arrays order (19, nz, ny, nx) instead of the
   * default plane-blocked order (nz, 19, ny, nx) */
  LBM_FLAG_PLAIN_SOA = 4
};

typedef struct {
  int32_t nx, ny, nz;  /* lattice extent, each >= 1 */
  int32_t precision;   /* lbm_precision */
  double omega;        /* BGK relaxation frequency 1/tau, 0 < omega < 2 (eq. (5), (9)) */
  int32_t bc[6];       /* faces -x, +x, -y, +y, -z, +z (lbm_bc) */
  int32_t flags;       /* LBM_FLAG_* */
  int32_t reserved;    /* must be 0 */
} lbm_desc;

/* Bubble-phase constants (Table 1, Table 3), all in lattice units. */
typedef struct {
  double g;             /* gravity magnitude (acts along -z) */
  double rho_l;         /* liquid density used by the force closures */
  double rho_b;         /* bubble density */
  double sigma;         /* surface tension (Eotvos number) */
  double c_a;           /* added-mass coefficient C_A (Table 1: 0.5) */
  double drag_scale;    /* multiplier of the drag force */
  double lift_scale;    /* multiplier of the lift force */
  double kernel_factor; /* half-width of the mapping window in diameters (Sec. 3.2: 1.5) */
  double cd_k;          /* k in C_D = 24/Re (1 + k Re^0.687) */
  double lift_f0;       /* constant term of the lift polynomial f(Eo_d) */
  int32_t n_sub;        /* bubble sub-steps per liquid step, dt_b = 1/n_sub (Table 2: 10) */
  int32_t coupling;     /* LBM_COUPLING_* / LBM_REACTION_* bits; 0 = the default readings */
} bubble_params;

/* Coupling variants (bubble_params.coupling). The paper states the reaction spread into the
 * liquid twice (Sec. 3.2: minus the sum of the forces on the bubble; Algorithm 1: -(F_D + F_L)
 * from the updated velocity), the mapping weights as cell integrals of the kernel (eq. (19)),
 * and leaves the time level of the forward coupling open. Default (0): -(F_D + F_L) at the
 * velocity after the sub-steps, cell-integral weights, and the liquid velocity of the previous
 * collision (the velocity field U the liquid step writes).
 *   reaction (bits 0-1): LBM_REACTION_SUBSTEP_MEAN, the mean of -(F_D + F_L) over the sub-steps
 *     (the impulse those forces gave the bubble in the liquid step); LBM_REACTION_NET_FORCE,
 *     minus the mean over the sub-steps of the net force m_b du_b/dt of eq. (1);
 *   LBM_COUPLING_POINT_KERNEL: weights Z(x_j - x_b) at cell centres, renormalised to a sum of one
 *     on every axis (instead of cell integrals);
 *   LBM_COUPLING_EXACT_TIME: the forward coupling interpolates the velocity of the current state
 *     f^n (eq. (10), no force term), recomputed from the populations on the stencil, instead of
 *     U. Single lattices only (lbm_batch_step returns LBM_EUNSUPPORTED).
 * lbm_adjoint_bubbles differentiates the default only (LBM_EUNSUPPORTED otherwise). Other bits,
 * or a reaction value of 3, give LBM_EINVAL. */
#define LBM_REACTION_MASK 3
#define LBM_REACTION_SUBSTEP_MEAN 1
#define LBM_REACTION_NET_FORCE 2
#define LBM_COUPLING_POINT_KERNEL 4
#define LBM_COUPLING_EXACT_TIME 8

/* Bubble state, structure of arrays of length nb in device memory (double precision).
 * state: 0 = inactive (reached the top layer, Algorithm 1 stop test), 1 = active without a
 * previous interpolated liquid velocity (first step), 2 = active. ul* hold the liquid velocity
 * interpolated at the previous step (for the material derivative of u_l). psi* (optional) receive
 * the reaction spread into the liquid: -(F_D + F_L), or what bubble_params.coupling selects (0 for
 * an inactive bubble). */
typedef struct {
  double *x, *y, *z;
  double *ux, *uy, *uz;
  double *d;
  double *ulx, *uly, *ulz;
  int32_t *state;
  double *psix, *psiy, *psiz; /* nullable: receives the reaction spread in the last step */
  double *work;               /* device scratch of nb * LBM_BUBBLE_WORK doubles */
} bubble_soa;

/* Doubles of per-bubble device scratch that bubbles_step() needs in bubble_soa.work (the
 * interpolated liquid velocity and vorticity, the start position, the reaction of the step and
 * the stencil weights at the start position, passed between its kernels). Its contents need no
 * initialisation. */
#define LBM_BUBBLE_WORK 216

typedef struct lbm_ctx lbm_ctx;

/* Largest bubble the stencil kernels accept: the mapping window may span at most this many
 * cells per axis (window half-width n = kernel_factor * d, so d <= about 20 at factor 1.5). */
#define LBM_MAX_STENCIL 64

/* Sizes, in bytes, of one population buffer (19 x cells), of one vector field (3 x cells:
 * force or velocity) and of the scratch buffer (tile masks and reduction partials). */
lbm_status lbm_bytes_required(const lbm_desc* desc, size_t* pop_buffer_bytes,
                              size_t* field_bytes, size_t* scratch_bytes);

/* Create a context over caller-owned device buffers and initialise them on the stream:
 * both population buffers to g = 0 (f = w, liquid at rest, rho = 1: Algorithm 1
 * initialisation), force and velocity to 0, scratch to its initial state. The buffers must stay
 * valid and unaliased until lbm_destroy(). stream is a hipStream_t or NULL. */
lbm_status lbm_init(const lbm_desc* desc, void* pops_a, void* pops_b, void* force, void* vel,
                    void* scratch, void* stream, lbm_ctx** out);

/* Change the stream later calls enqueue on. */
lbm_status lbm_set_stream(lbm_ctx* ctx, void* stream);

/* Launch shape of the liquid step (the tuning knob of the autotuner; results do not depend on
 * it): vec = cells per thread along x (1, 2 or 4, must divide nx), block_x = threads per 256-thread
 * workgroup along x (16, 32, 64, 128 or 256). lbm_init() picks a default. */
lbm_status lbm_set_launch(lbm_ctx* ctx, int32_t vec, int32_t block_x);

/* Occupancy of the liquid-step launches (a tuning knob; results do not depend on it): at most
 * workgroups_per_cu of their workgroups run on one compute unit at a time (each launch requests
 * unused LDS to that end), 0 = no cap, at most 32. lbm_init() picks 5 for FP32 lattices and 3 for
 * FP64. LBM_EINVAL while a bubble half is pending. */
lbm_status lbm_set_step_occupancy(lbm_ctx* ctx, int32_t workgroups_per_cu);
lbm_status lbm_get_step_occupancy(lbm_ctx* ctx, int32_t* workgroups_per_cu);
lbm_status lbm_get_launch(lbm_ctx* ctx, int32_t* vec, int32_t* block_x);

/* Overlap of the bubble kernels with the liquid step, available when no face is periodic,
 * the launch shape has one cell per thread and the population buffer is below 4 GiB; on by
 * default for lattices of 2^22 cells or more, where the liquid step outlasts the bubble kernels
 * (it costs a region launch and two cross-stream waits). With it,
 * bubbles_step() marks the region of this step (the 8^3 tiles within the bubbles' stencil windows
 * widened by the curl ring and two cells), runs the bubble kernels on a library-owned side stream
 * while the liquid update of every other tile (the bulk) runs on the caller's stream, and makes the
 * caller's stream wait for the bubble kernels; lbm_step() then updates the region. Within
 * lbm_run() each overlapped step also marks the region of the next one on the side stream. Work
 * enqueued on the caller's stream after bubbles_step() sees the bubble results. Results are identical to the
 * serial step bit for bit. A bubble that moves more than two cells in one step would leave the region; that
 * is reported by lbm_check() / moments() with sums as LBM_EUNSUPPORTED. Not allowed while a
 * bubble half awaits its lbm_step(). available (nullable) reports whether the current
 * configuration can overlap. */
lbm_status lbm_set_overlap(lbm_ctx* ctx, int32_t enable);
lbm_status lbm_get_overlap(lbm_ctx* ctx, int32_t* enabled, int32_t* available);

/* Timing hook for profiling: start and end (hipEvent_t, each nullable) are recorded on the
 * caller's stream immediately before and after the next liquid launch that updates the lattice
 * away from the bubbles (the bulk launch of an overlapped step, made by bubbles_step(), else the
 * whole liquid step). One-shot: the events are forgotten after that launch. The caller owns the events. */
lbm_status lbm_time_next_step(lbm_ctx* ctx, void* start, void* end);

/* Cells in the region of the last overlapped step (0 if none since the last serial step); the bulk
 * launch of that step updated the other N - cells. Synchronises the stream. */
lbm_status lbm_region_cells(lbm_ctx* ctx, int64_t* cells);

/* nsteps liquid steps (Sec. 2.2, eq. (13)-(16) with the face conditions of Sec. 3.3): first
 * forcing (13), BGK collision (14), Guo forcing (12), (15), streaming (16). Each step reads the
 * force field where bubbles have spread force (or everywhere with LBM_FLAG_STATIC_FORCE),
 * writes the collision velocity U of eq. (13) there (or everywhere with LBM_FLAG_WRITE_U_ALL)
 * and clears the force it used. */
lbm_status lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* Bubble half of one step of Algorithm 1 for nb bubbles (forward coupling eq. (20) of the
 * liquid velocity and its curl with the weights of eq. (19); force closures of Table 1 and
 * eq. (3); n_sub explicit sub-steps of eq. (4); backward coupling eq. (21) of the reaction
 * -(F_D + F_L) into the force field). Uses the velocity field of the previous lbm_step() (the
 * current state's with LBM_COUPLING_EXACT_TIME; params->coupling selects the variants). With
 * several bubbles each cell sums their forces in bubble order: the force field is
 * bit-reproducible. Call exactly once before each lbm_step(ctx, 1). soa: host struct of device
 * pointers. LBM_EINVAL for invalid params (n_sub < 1, unknown coupling bits, non-positive
 * kernel_factor, sigma or rho_l) or a missing array. */
lbm_status bubbles_step(lbm_ctx* ctx, const bubble_params* params, const bubble_soa* soa,
                        int32_t nb);

/* Macroscopic fields of the current state (eq. (10)): rho = sum_q f_q and u = sum_q c_q f_q / rho
 * per cell (device buffers of N and 3 x N elements of the lattice type, each nullable), and
 * sums_out (host, 4 doubles, nullable) = (sum rho, sum rho u_x, sum rho u_y, sum rho u_z)
 * accumulated in double precision. With sums_out the call synchronises the stream and returns
 * LBM_EDIVERGED if a sum is not finite (the BGK step went unstable, Sec. 4.3; this takes precedence
 * over the kernel error the bubbles of a diverged liquid then raise), else a pending kernel error
 * (cleared, as by lbm_check()); sums_out is written in every case but LBM_EDEVICE. */
lbm_status moments(lbm_ctx* ctx, void* rho_out, void* u_out, double* sums_out);

/* Write the current pre-collision populations g = f - w (19 x N, lattice type, plain order
 * pop[q][z][y][x] whatever the buffer layout) into the device buffer out. */
lbm_status lbm_populations(lbm_ctx* ctx, void* out);

/* Pointer of the buffer holding the current state (post-collision, awaiting streaming), in the
 * context's population layout. */
lbm_status lbm_state_buffer(lbm_ctx* ctx, void** out);

/* Checkpoint and resume at a step boundary: everything the method carries from one step to the
 * next besides the caller's bubble arrays is the post-collision buffer and the velocity field of
 * the last collision (Algorithm 1; the force field is zero between steps). lbm_checkpoint copies
 * them (19 x N and 3 x N elements of the lattice type, the buffer in the library's layout) into
 * caller-owned device buffers, lbm_restore copies them back into a lattice of the same
 * description, asynchronously on the context's stream; the caller saves and restores the bubble
 * arrays itself. A restored lattice continues bit for bit as the one checkpointed. LBM_EINVAL
 * while a bubble half awaits its lbm_step(), or for a NULL buffer. */
lbm_status lbm_checkpoint(lbm_ctx* ctx, void* state_out, void* vel_out);
lbm_status lbm_restore(lbm_ctx* ctx, const void* state, const void* vel);

/* Rebind the context to other caller-owned buffers (each nullable: keep the current one). state:
 * a population buffer (layout of the context) that already holds the current state; next_state:
 * the buffer the next liquid step writes into (then the current state); vel: the velocity field
 * the bubble half reads and the liquid step writes. Used by checkpointed recomputation to write
 * each step's state straight into its own buffer. Not allowed while a bubble half awaits its
 * lbm_step(); state and next_state must differ. Drops the captured lbm_run() graph. */
lbm_status lbm_bind_buffers(lbm_ctx* ctx, void* state, void* next_state, void* vel);

/* Synchronise the stream and report a pending kernel error (LBM_EINVAL for a bubble beyond the
 * stencil limit, with a non-finite position, or whose point-sampled window holds no cell centre;
 * LBM_EUNSUPPORTED for a bubble that left the region of an overlapped step), then clear it. Such
 * a bubble is skipped for the step (no force, state unchanged). */
lbm_status lbm_check(lbm_ctx* ctx);

/* nsteps method steps (bubbles_step then lbm_step(ctx, 1), Algorithm 1) with the launches of
 * graph_steps consecutive steps captured once into a HIP graph and replayed; the graph is kept
 * while params, soa and nb stay the same. graph_steps must be even (the step alternates two
 * population buffers), 0 runs every step eagerly. Graph capture needs a non-NULL stream. */
lbm_status lbm_run(lbm_ctx* ctx, const bubble_params* params, const bubble_soa* soa, int32_t nb,
                   int32_t nsteps, int32_t graph_steps);

/* Release the context (not the caller's buffers). NULL is accepted. */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* ---------------------------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): bubbles_step() with its per-bubble workspace held by
 * the library instead of the caller.
 * ------------------------------------------------------------------------------------------- */

/* Bubbles bubbles_step_static_work() accepts: its workspace array holds this many bubbles'
 * LBM_BUBBLE_WORK doubles (1.7 MiB per GPU). */
#define LBM_STATIC_WORK_BUBBLES 1024

/* As bubbles_step(), with the nb x LBM_BUBBLE_WORK doubles of per-bubble workspace taken from a
 * fixed device array inside the library; soa->work is ignored and may be NULL. The call allocates
 * nothing: the array exists on every GPU the library runs on and is held until the process ends
 * (its address on a device is resolved once, by the first lbm_init() on that device). The caller
 * still passes the context's buffers and the bubble arrays. nb > LBM_STATIC_WORK_BUBBLES (or
 * negative): LBM_EINVAL, nothing enqueued. LBM_EDEVICE if the array's address could not be
 * resolved on the context's device. Every call on one GPU uses the same array and leaves its
 * contents there; each call writes every entry before reading it, so nothing needs clearing, but
 * bubble halves that may run at the same time on one GPU (contexts stepping on different streams
 * with no ordering between them) race on it and must not be issued. lbm_bubble_record() stage 1
 * reads soa->work and so cannot follow this call; arm lbm_record_next_bubble_half() instead. */
lbm_status bubbles_step_static_work(lbm_ctx* ctx, const bubble_params* params,
                                    const bubble_soa* soa, int32_t nb);

/* ---------------------------------------------------------------------------------------------
 * Adjoint (reverse-mode derivative) of one method step, for gradients of a loss on bubble
 * trajectories with respect to drag_scale, lift_scale and omega. The caller keeps the forward
 * data of the step (a checkpoint-and-recompute schedule) and walks the steps backwards.
 * grad (device, 4 doubles, accumulated): [0] dL/domega, through the collision (lbm_adjoint_liquid)
 * and through the bubble closures (lbm_adjoint_bubbles adds dL/dnu dnu/domega, nu = (1/omega - 1/2)/3,
 * eq. (9)); [1] dL/d drag_scale, [2] dL/d lift_scale; [3] dL/dnu of the closures alone (already
 * contained in [0]).
 * ------------------------------------------------------------------------------------------- */

/* Doubles per bubble in a step record: [0, 21) x[3] u_b[3] u_l,prev[3] state u_l[3] w_l[3] psi[3]
 * valid d, taken before the step (x, u_b, u_l,prev, state, d) and after its bubble half (u_l, w_l,
 * psi, valid = the first LBM_BUBBLE_WORK slots 0-5, 9-12 of bubble_soa.work); [21] 1 if the
 * sub-steps below were recorded, else 0; [24, 123) the velocity u_b at the start of each sub-step
 * k = 0..n_sub (k = n_sub: after the last), 3 doubles each; [123, 126) the clamp flags of the
 * sub-steps (bit 3 k + a of the 96-bit word held as three 32-bit integers in doubles: component a
 * clamped at a wall in sub-step k). */
#define LBM_BUBBLE_RECORD 128
/* Doubles per bubble of adjoint state: dL/dx[3], dL/du_b[3], dL/du_l,prev[3], unused[3]. */
#define LBM_BUBBLE_ADJ 12

/* Fill the step record (nb x LBM_BUBBLE_RECORD doubles, device) from the bubble arrays: stage 0,
 * called before the step's bubble half, writes x, u_b, u_l,prev, state and d (and marks the
 * sub-steps as not recorded); stage 1, called after it, writes u_l, w_l, psi and valid from
 * soa->work. */
lbm_status lbm_bubble_record(lbm_ctx* ctx, const bubble_soa* soa, int32_t nb, int32_t stage,
                             double* record);

/* Trajectory recording for callers that run many steps without returning to the host between
 * them (lbm_run, graph replays): from this call on, every bubble half writes each bubble's position
 * after its update into the next row of traj (device, rows x 3 x nb doubles, row-major, a row
 * component-major [a * nb + b]; inactive bubbles keep their position) until rows rows are written;
 * the row counter is device memory and starts at 0 here. traj = NULL (rows 0) disarms. Drops the
 * captured lbm_run() graph. LBM_EINVAL while a bubble half awaits its lbm_step(). */
lbm_status lbm_record_positions(lbm_ctx* ctx, double* traj, int32_t rows);

/* One-shot: the next bubbles_step() writes the whole step record of every bubble into record (nb x
 * LBM_BUBBLE_RECORD doubles, device, caller-owned), the sub-steps included when n_sub <= 32, from
 * inside the bubble update (no launch of its own; the same values as the two stages of
 * lbm_bubble_record). record = NULL disarms. lbm_run() returns LBM_EINVAL while a record is
 * armed. */
lbm_status lbm_record_next_bubble_half(lbm_ctx* ctx, double* record);

/* Adjoint of the liquid step (eq. (12)-(16), Sec. 3.3). state: the post-collision buffer before the
 * step (19 x N); force: the force field of the step (3 x N); lam_next: dL/d(state after the step);
 * lam_prev (out, every element written): dL/d(state before); lam_u (in/out): dL/dU of the step's
 * velocity field, read and cleared; lam_f (out): dL/dF. Device buffers of the lattice type. */
lbm_status lbm_adjoint_liquid(lbm_ctx* ctx, const void* state, const void* force,
                              const void* lam_next, void* lam_prev, void* lam_u, void* lam_f,
                              double* grad);

/* Tile mask of a step (the tiles its liquid step forces or writes the velocity in, Algorithm 1's
 * coupling windows): *ntiles (out) = number of tiles, ceil(nx/8) ceil(ny/8) ceil(nz/8); with
 * tiles != NULL (device, *ntiles bytes, caller-owned) the mask the last bubbles_step() flagged is
 * copied there, asynchronously on the context's stream, entry ((z/8) ceil(ny/8) + y/8) ceil(nx/8)
 * + x/8 nonzero for a flagged tile. Call it between the step's bubbles_step() and its lbm_step(),
 * which reads the mask and clears it for a later step. */
lbm_status lbm_step_tiles(lbm_ctx* ctx, uint8_t* tiles, int64_t* ntiles);

/* lbm_adjoint_liquid() with the step's tile mask from lbm_step_tiles() (NULL: every tile). Outside
 * the flagged tiles the step's force and the velocity adjoint lam_u are zero (the step neither
 * forced nor wrote the velocity there, and lbm_adjoint_bubbles() scatters only into the velocity
 * windows the step flagged), so those cells take them as zero without reading them and leave
 * lam_u and lam_f unwritten (lam_f there keeps what it held): the same lam_prev and grad as
 * lbm_adjoint_liquid(), from 228 instead of 276 bytes per FP32 cell. A lattice with
 * LBM_FLAG_STATIC_FORCE ignores the mask. */
lbm_status lbm_adjoint_liquid_tiles(lbm_ctx* ctx, const void* state, const void* force,
                                    const void* lam_next, void* lam_prev, void* lam_u, void* lam_f,
                                    const uint8_t* tiles, double* grad);

/* Timing hook for profiling the adjoint liquid step (the transposed step above, no equation of
 * its own): start and end (hipEvent_t, each nullable) are recorded on the caller's stream
 * immediately before and after the next launch of the adjoint liquid kernel made by
 * lbm_adjoint_liquid() / lbm_adjoint_liquid_tiles(); the clearing and the final sum of the
 * dL/domega bins stay outside. One-shot: the events are forgotten after that launch. The caller
 * owns the events. */
lbm_status lbm_time_next_adjoint_liquid(lbm_ctx* ctx, void* start, void* end);

/* Adjoint of the bubble half (eq. (18)-(21), Table 1, eq. (1)-(4)). record: nb x
 * LBM_BUBBLE_RECORD doubles of the step; vel_prev: velocity field the step interpolated;
 * lam_f: dL/dF from lbm_adjoint_liquid; lam_u (out, accumulated): dL/d(vel_prev); lam: nb x
 * LBM_BUBBLE_ADJ adjoint bubble state, dL/d(state after the step) in, dL/d(state before) out;
 * lam_x (may be NULL): the loss's own dL/dx of the positions after the step, 3 x nb doubles
 * (component-major, [a * nb + b]), added to lam's dL/dx first (so a loss on every step's
 * positions needs no separate addition). grad[1..3] accumulate dL/d(drag_scale),
 * dL/d(lift_scale), dL/dnu, and grad[0] dL/dnu dnu/domega. n_sub may be at most 32. */
lbm_status lbm_adjoint_bubbles(lbm_ctx* ctx, const bubble_params* params, const double* record,
                               const void* vel_prev, const void* lam_f, void* lam_u, double* lam,
                               const double* lam_x, int32_t nb, double* grad);

/* Host evaluation of the arithmetic the adjoint kernels run (double precision), for checks:
 * one cell's collision (eq. (13)-(15)) and, if lam/lam_u/mu/lam_f/domega are given, its
 * transposed Jacobian; */
lbm_status lbm_host_collide(const double* p, const double* F, double omega, const double* lam,
                            const double* lam_u, double* out, double* u, double* mu, double* lam_f,
                            double* domega);
/* the weights of one axis (LBM_MAX_STENCIL + 2 entries from cell lo - 1), their curl
 * counterparts and both derivatives in the bubble coordinate; s_lo, s_hi: -1 bounce-back, +1
 * free slip; */
lbm_status lbm_host_axis_weights(double x, double n, int32_t ext, int32_t periodic, double s_lo,
                                 double s_hi, int32_t* lo, double* w, double* dw, double* wx,
                                 double* dwx);
/* one step of the bubble ODE, and its reverse sweep: out = dL/d(x[3], u_b[3], u_l[3], w_l[3],
 * D_t u_l[3]), dL/d drag_scale, dL/d lift_scale, dL/dnu. */
lbm_status lbm_host_bubble_ode(const bubble_params* params, double nu, double d, const double* x0,
                               const double* ub0, const double* ul, const double* wl,
                               const double* dul, const int32_t* ext, const int32_t* periodic,
                               double* x, double* ub, double* psi);
lbm_status lbm_host_bubble_ode_adjoint(const bubble_params* params, double nu, double d,
                                       const double* x0, const double* ub0, const double* ul,
                                       const double* wl, const double* dul, const int32_t* ext,
                                       const int32_t* periodic, const double* lx,
                                       const double* lub, const double* lpsi, double* out);

/* ---------------------------------------------------------------------------------------------
 * Batched columns: many independent lattices (uneven extents, each with its own omega and faces)
 * stepped together, as in the paper's grid-independence and stability sweeps (Sec. 4.2, 4.3).
 * All columns share the precision and the bubble constants except that a column may carry its own
 * gravity and surface tension in lattice units (one physical setup resolved at several grid
 * spacings, App. A: g and sigma scale with the spacing); column c owns bubbles
 * [bubble_begin, bubble_begin + nb) of one shared bubble_soa, ranges consecutive in column order.
 * Every buffer lives in one caller-owned pool and one caller-owned scratch block.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz;
  int32_t bubble_begin, nb;
  int32_t bc[6];
  int32_t reserved;  /* 0 */
  double omega;
  /* this column's bubbles' g and sigma (bubble_params units); 0: the batch's bubble_params value */
  double g, sigma;
} lbm_column;

typedef struct lbm_batch lbm_batch;

lbm_status lbm_batch_bytes_required(const lbm_column* cols, int32_t ncols, int32_t precision,
                                    size_t* pool_bytes, size_t* scratch_bytes);
/* Lay the columns out in pool, initialise every population to g = 0 and the fields to 0. The call
 * synchronises the stream once (it uploads the column table). */
lbm_status lbm_batch_init(const lbm_column* cols, int32_t ncols, int32_t precision, int32_t flags,
                          void* pool, void* scratch, void* stream, lbm_batch** out);
/* Cells per work item of each column in the batched liquid step (multiple of 256, at most 65536):
 * the tuning knob of the batch autotuner; results do not depend on it. */
lbm_status lbm_batch_set_items(lbm_batch* batch, const int32_t* item_cells);
lbm_status lbm_batch_get_items(lbm_batch* batch, int32_t* item_cells);
/* Occupancy of the batched liquid step (as lbm_set_step_occupancy): at most workgroups_per_cu of
 * its workgroups per compute unit, 0 = no cap, at most 32. lbm_batch_init() picks 3 for FP32 and 0
 * for FP64 (held to 3 by registers). */
lbm_status lbm_batch_set_step_occupancy(lbm_batch* batch, int32_t workgroups_per_cu);
lbm_status lbm_batch_get_step_occupancy(lbm_batch* batch, int32_t* workgroups_per_cu);
/* Persistent launches (the sweep of Sec. 4.2-4.3 as one kernel per run of steps): with enable,
 * lbm_batch_step runs its nsteps method steps as one kernel and lbm_batch_run captures one such
 * kernel of graph_steps steps per graph. The kernel holds as many workgroups as stay resident
 * together (at most the batch occupancy cap per compute unit) and separates the phases of each step
 * (bubble half, force gather, liquid step) by grid-wide barriers; results are those of the
 * per-step launches. Should the workgroups not all be resident (other work on the device), its
 * barriers time out after about a second, the launch ends early and lbm_batch_check() returns
 * LBM_EDEVICE. grid (nullable) receives the workgroups of the last persistent launch. */
lbm_status lbm_batch_set_persistent(lbm_batch* batch, int32_t enable);
lbm_status lbm_batch_get_persistent(lbm_batch* batch, int32_t* enabled, int32_t* grid);
/* nsteps method steps of every column (eager launches). nb must equal the total bubble count. */
lbm_status lbm_batch_step(lbm_batch* batch, const bubble_params* params, const bubble_soa* soa,
                          int32_t nb, int32_t nsteps);
/* As lbm_batch_step, with graph_steps steps captured into a HIP graph and replayed (see lbm_run). */
lbm_status lbm_batch_run(lbm_batch* batch, const bubble_params* params, const bubble_soa* soa,
                         int32_t nb, int32_t nsteps, int32_t graph_steps);
/* Pre-collision populations g = f - w of column col (19 x N, lattice type) into device buffer out. */
lbm_status lbm_batch_populations(lbm_batch* batch, int32_t col, void* out);
/* Per-column global sums of the current state (eq. (10)): sums (host, ncols x 4 doubles) =
 * (sum rho, sum rho u_x, sum rho u_y, sum rho u_z) of each column, accumulated in double
 * precision in a fixed order. Synchronises the stream. Returns LBM_EDIVERGED when a sum is not
 * finite (the BGK step of that column went unstable; the other columns' sums are valid). */
lbm_status lbm_batch_sums(lbm_batch* batch, double* sums);
/* Device pointers of column col: current state buffer, force field, velocity field. */
lbm_status lbm_batch_column(lbm_batch* batch, int32_t col, void** state, void** force, void** vel);
/* Synchronise and report a pending kernel error (as lbm_check). */
lbm_status lbm_batch_check(lbm_batch* batch);
lbm_status lbm_batch_destroy(lbm_batch* batch);

/* Static description of a status code. */
const char* lbm_status_string(lbm_status status);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
