/*
 * lbm.h - C ABI of the MI355X (gfx950) D3Q39 13-moment double-distribution
 * lattice Boltzmann library.
 *
 * Method: Latt, Coreixas, Beny, Parmigiani, "Efficient supersonic flows
 * through high-order guided equilibrium with lattice Boltzmann" (2019).
 *   - lattice: Sec. 3, D3Q39 (E_{3,7}^{39});
 *   - equilibrium: Sec. 2, Eq. (eq:discrete-equilibrium), the exponential of
 *     13 monomials whose multipliers match the 13 Maxwell-Boltzmann moments of
 *     Eq. (eq:13constraints), found by Newton-Raphson warm-started from the
 *     previous step (Sec. 5, algorithm table);
 *   - second population: Eq. (eq:discrete-equilibrium-poly);
 *   - collide-and-stream with BGK for f and g, Pr = 1: Sec. 3;
 *   - Knudsen-dependent relaxation time: Eq. (eq:DeltaAvg) and Eq. (eq:alpha);
 *   - boundary conditions of the NACA0012 set-up (Sec. 4): free-stream
 *     equilibrium faces, first-order Neumann outlet, half-way bounce-back.
 *
 * Conventions shared by every call:
 *   - All functions return an lbm_status (0 = success, negative = error) or,
 *     where stated, a non-negative count.  No C++ exception, abort or exit
 *     crosses the ABI.  lbm_last_error() describes the last failure.
 *   - Cells are numbered x fastest: cell = x + nx*(y + ny*z).  Host field
 *     arrays are structure-of-arrays in that order.
 *   - Velocity i of the lattice is returned by lbm_velocities(); for every odd
 *     i, velocity i+1 is its opposite; velocity 0 is the rest velocity.
 *   - Multiplier k multiplies basis function phi_k of the exponent, with
 *     phi = (1, xi_x, xi_y, xi_z, xi_x^2, xi_y^2, xi_z^2, xi_x xi_y, xi_x xi_z,
 *     xi_y xi_z, xi_x |xi|^2, xi_y |xi|^2, xi_z |xi|^2).
 *   - Device memory is the caller's: lbm_create() sub-allocates everything it
 *     needs inside a caller-provided device arena and never calls hipMalloc.
 *     The arena must stay allocated until lbm_destroy().
 *   - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL = the null stream).  Calls on one context are not
 *     thread-safe; distinct contexts are independent.
 */
#ifndef LBM13_LBM_H
#define LBM13_LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_E_INVAL = -1,          /* invalid argument or parameter */
    LBM_E_NOMEM = -2,          /* arena smaller than lbm_required_bytes() */
    LBM_E_DEVICE = -3,         /* a HIP call failed, or the library was built for another GPU */
    LBM_E_NONREALIZABLE = -4,  /* a reference or initial state has no 13-moment equilibrium */
    LBM_E_NEWTON = -5,         /* at least one cell's Newton solve did not converge (state stays defined) */
    LBM_E_NONFINITE = -6       /* a moment is NaN or infinite */
} lbm_status;

/* The shifted modes stop Newton at 1e-5 of the largest target (FP32
 * arithmetic) and then remove the five collision-invariant residuals that
 * stop leaves (mass, momentum, energy) by scaling each equilibrium
 * population by 1 + x . (1, xi_i, |xi_i|^2), with x solving the 5x5 system of
 * the equilibrium's own moments.  The correction is proportional to each
 * population, so the smallest equilibria of a supersonic stream (1e-11 and
 * below) keep their relative accuracy and the Knudsen sensor of
 * Eq. (eq:DeltaAvg) stays at the FP64 value within the arithmetic's bound.
 * Storage as deviations from the rest weights rounds the smallest
 * populations of a fast stream to the spacing of their (much larger)
 * weights; shift_ref = 1 stores them near exactly. */
typedef enum {
    LBM_STORE_FP64 = 0,          /* populations and multipliers in FP64, arithmetic in FP64 */
    LBM_STORE_FP32_SHIFTED = 1,  /* populations stored in FP32 as deviations from shift weights, FP32 arithmetic */
    LBM_STORE_FP16_SHIFTED = 2   /* deviations stored in FP16 (power-of-two scaled per velocity), FP32 arithmetic */
} lbm_storage;

typedef enum {
    LBM_FACE_PERIODIC = 0,     /* wrap around (both faces of an axis must be periodic) */
    LBM_FACE_EQUILIBRIUM = 1,  /* three outer layers frozen at the equilibrium of their initial state */
    LBM_FACE_NEUMANN = 2       /* three outer layers read as copies of the nearest interior layer */
} lbm_face;

/* Problem statement.  Every field is read during lbm_create() only; the
 * pointers may be freed afterwards.  Zero/NULL selects the default noted. */
typedef struct {
    int32_t nx, ny, nz;        /* cells (>= 1; a non-periodic axis needs >= 7); nx*ny*nz < 2^28 in FP64,
                                  2^29 in FP32, 2^30 in FP16 (the gathers' 32-bit offsets), and the
                                  footprint of lbm_required_bytes must fit the arena */
    int32_t storage;           /* lbm_storage */
    int32_t shift_ref;         /* shifted storage only: 0 = rest-state equilibrium at (rho_ref, T_ref),
                                  1 = equilibrium of the reference stream (rho_ref, u_ref, T_ref); with 1
                                  opposite velocities have unequal weights, and a bounce-back moves the
                                  gathered deviation onto the other weight (FP16: one more rounding) */
    int32_t kn_relax;          /* 1: tau(eps) = tau * alpha(eps), Eq. (eq:alpha); 0: plain BGK */
    int32_t newton_maxit;      /* cap on Newton updates per cell and step (0: 20); a cold restart, where
                                  allowed, has a cap of max(newton_maxit, 100) */
    int32_t faces[6];          /* lbm_face for -x, +x, -y, +y, -z, +z */
    double gamma;              /* heat-capacity ratio, 1 < gamma <= 5/3 (C_v = 1/(gamma-1), D = 3) */
    double mach;               /* |u_ref| / sqrt(gamma T_ref) */
    double reynolds;           /* |u_ref| L_ref / nu, nu = K(T_ref) (tau - 1/2) (used when tau <= 0) */
    double length_ref;         /* L_ref in cells (used when tau <= 0) */
    double rho_ref, T_ref;     /* reference (free-stream) state; 0 selects 1 and 0.5 */
    double u_dir[3];           /* direction of u_ref (normalised here; zero vector with mach = 0 is allowed) */
    double tau;                /* > 0: relaxation time as given; <= 0: derived from reynolds */
    double newton_tol;         /* stopping bound on max_k |G_k|/rho relative to max(1, max_k |M_k|/rho)
                                  (0: 1e-12 in FP64 as in Sec. 5, 1e-5 in FP32 arithmetic).  A solve also
                                  stops at the arithmetic's round-off floor: when the full Newton step does
                                  not lower ||G||_2 while max_k |G_k| before and after it is within 8 times
                                  the bound, the step is taken (this fires in FP32 arithmetic; in FP64 the
                                  floor lies far below the bound) */
    const uint8_t *solid;      /* nx*ny*nz obstacle flags (nonzero = solid) or NULL */
    const double *init_rho;    /* initial fields (N, 3N as ux|uy|uz, N) or NULL for the reference state */
    const double *init_u;
    const double *init_T;
    int32_t root_finder;       /* multipliers found by 0: Newton-Raphson (Sec. 3, the algorithm table of
                                  Sec. 5); 1: a secant method that never evaluates the Jacobian of G, the
                                  gradient-free side of the choice Sec. 6 leaves open (FP64 storage only;
                                  not in the pool): limited-memory BFGS on the convex dual whose gradient
                                  is G, memory 3, started from the inverse of a model Jacobian (the rest
                                  Jacobian at T_ref, scaled to the cell's T and shifted to its u); same
                                  stopping rule, floor stop, stall and failure handling as Newton; a step is
                                  accepted when it lowers ||G||_2 or, along a descent direction, the dual by
                                  1e-4 t G.d; newton_maxit 0 selects 100 for it */
} lbm_params;

/* Per-call statistics of lbm_step(), summed over fluid cells and steps. */
typedef struct {
    int64_t cell_updates;      /* fluid cells x steps */
    int64_t iterations;        /* accepted Newton updates */
    int64_t max_iterations;    /* largest count of one cell in one step */
    int64_t failed;            /* cell-steps whose Newton did not converge */
    int64_t cold_restarts;     /* cell-steps whose warm start failed and that were restarted cold */
    int64_t alpha_hist[4];     /* cell-steps per branch of Eq. (eq:alpha) */
    int64_t wave_iterations;   /* sum over wave-steps of the largest count in the wave (64 cells) */
    int64_t waves;             /* wave-steps (a wave runs as many Newton updates as its slowest cell) */
} lbm_step_stats;

/* Values derived by lbm_create(). */
typedef struct {
    double tau;                /* relaxation time in use */
    double u_ref[3];           /* reference velocity */
    double shear_response;     /* K(T_ref): nu = K (tau - 1/2) */
    double delta;              /* 2 C_v - D, the factor of g^eq = delta T f^eq */
    int64_t cells;             /* nx*ny*nz */
    int64_t fluid_cells;       /* cells updated by a step */
    int64_t steps_done;        /* steps taken since creation or the last lbm_set_state() */
    int64_t arena_bytes_used;
} lbm_info;

/* Library version (major*10000 + minor*100 + patch). */
int32_t lbm_version(void);

/* Writes the 39 lattice velocities (39 x 3 int32, row i = velocity i). */
int lbm_velocities(int32_t *out);

/* Bytes of device arena that lbm_create() needs for these parameters, or a
 * negative lbm_status if they are invalid.  This is the admission footprint:
 * two ping-pong buffers of the 2 x 39 populations per cell (f and g of
 * Sec. 3, Eq. (eq:discrete-equilibrium-poly)), the 13 multipliers per cell
 * that warm-start the next solve (Sec. 5 algorithm table), the obstacle's
 * link masks and the reduction scratch. */
int64_t lbm_required_bytes(const lbm_params *params);

/* The problem of Sec. 4: a polyatomic gas of ratio gamma (Sec. 2, C_v =
 * 1/(gamma-1), g^eq of Eq. (eq:discrete-equilibrium-poly)) at Mach and
 * Reynolds numbers, with an obstacle under half-way bounce-back and
 * free-stream equilibrium or Neumann faces.  Validates the parameters,
 * sub-allocates the arena (device pointer, 256-byte aligned, at least
 * lbm_required_bytes()), uploads the obstacle and initial fields and writes
 * the initial state: every cell at the equilibrium of its initial (rho, u, T)
 * (Eq. (eq:discrete-equilibrium) with the targets of Eq. (eq:13constraints)),
 * multipliers from a cold-started Newton solve.  Blocks until the initial
 * state is written.  On success *out owns the context; on
 * failure *out is NULL, no host memory is kept and lbm_last_error(NULL) holds
 * the message. */
int lbm_create(const lbm_params *params, void *dev_arena, int64_t arena_bytes, void *hip_stream, lbm_ctx **out);

/* Advances nsteps >= 0 time steps (fused pull-stream and collide, Sec. 3).
 * Asynchronous on the stream when stats is NULL; otherwise synchronises and
 * fills *stats.  A fluid cell whose 13 multipliers are not found (warm start,
 * then cold start) is not collided in that step: its gathered populations are
 * stored unchanged and its multipliers kept, so every moment of the cell is
 * conserved; multiplier 0 is replaced by NaN as the mark of that failure.  In
 * its next step a marked cell starts from its other 12 multipliers (lambda_0
 * normalising) and is not restarted cold, which bounds the cost of a cell
 * without equilibrium to one capped attempt per step.  A Newton attempt also
 * ends when its line search finds no step length (down to 2^-39) that lowers
 * ||G||_2.  With stats, returns LBM_E_NEWTON when a cell failed (the number
 * of such cell updates is stats->failed); the state stays defined. */
int lbm_step(lbm_ctx *ctx, int32_t nsteps, lbm_step_stats *stats);

/* Macroscopic fields of the current state, in FP64: rho, u and T of the
 * populations (Sec. 3; T from the total energy sum_i f_i |xi_i|^2 + g_i with
 * E = |u|^2/2 + C_v T, Sec. 2).  Collision conserves them, so after n steps
 * they are those of the stored post-collision state.  out_host (nullable):
 * 5*N doubles, SoA rho | ux | uy | uz | T; NaN at solid cells; Neumann
 * boundary cells report the interior cell they copy.  totals (nullable):
 * mass, momentum x, y, z and total energy (sum over i of (f_i |xi_i|^2 +
 * g_i) / 2), summed over fluid cells in a fixed order.  Synchronises.  Returns
 * LBM_E_NONFINITE if any fluid-cell moment is not finite. */
int lbm_moments(lbm_ctx *ctx, double *out_host, double *totals);

/* For callers that cannot allocate device memory at the point of the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * it): lbm_moments with the per-cell fields written to caller-owned device
 * memory, dev_out (5*N doubles, SoA as lbm_moments, required), and the
 * reduction scratch (block partials and totals) in a static array of the
 * library instead of the context's arena; totals (nullable, host) as
 * lbm_moments.  Grids of at most 524288 cells (larger ones: LBM_E_INVAL).
 * Calls no allocating routine.  Every call on one GPU shares that GPU's
 * scratch: calls that overlap on one GPU (two threads, two streams) race.
 * Synchronises the context's stream. */
int lbm_moments_noalloc(lbm_ctx *ctx, double *dev_out, double *totals);

/* Per-cell diagnostics of the next step, from the current state, which is
 * left unchanged: the Knudsen sensor eps of Eq. (eq:DeltaAvg), whose maps
 * Sec. 4 shows for the airfoil (Fig. fig:naca-knudsen), and the number of
 * Newton iterations the cell's solve takes (warm start; the cold restart's
 * count when that is used).  eps_out (nullable): N doubles, NaN outside fluid
 * cells and where the solve fails, +inf where an equilibrium population
 * underflows in the arithmetic (branch alpha = 1/tau of Eq. (eq:alpha));
 * iters_out (nullable): N int32, -1 outside
 * fluid cells, the iteration cap where the solve fails.  Uses the moments
 * scratch of the arena.  Synchronises. */
int lbm_diagnostics(lbm_ctx *ctx, double *eps_out, int32_t *iters_out);

/* Copies the state to host FP64 arrays (each nullable): f and g as [39][N],
 * multipliers as [13][N] (multiplier 0 is NaN for a cell whose last solve
 * failed, see lbm_step).  Shifted storage is decoded.  Synchronises. */
int lbm_get_state(lbm_ctx *ctx, double *f, double *g, double *lam);

/* Replaces the state (all three arrays required, layouts as above; shifted
 * storage is encoded with rounding to nearest).  Writes both ping-pong
 * buffers, so boundary and solid cells take the given values too.  Resets
 * steps_done.  Synchronises. */
int lbm_set_state(lbm_ctx *ctx, const double *f, const double *g, const double *lam);

int lbm_get_info(const lbm_ctx *ctx, lbm_info *info);

/* Releases the context (not the caller's arena).  Synchronises the stream. */
int lbm_destroy(lbm_ctx *ctx);

/* Message of the last failure on ctx, or of the calling thread's last failed
 * call that had no context (ctx = NULL).  Never NULL. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* ------------------------------------------------------------------------
 * Serving pool: many independent solves resident in one device arena and
 * advanced together.  Not a construct of the paper; it batches the step of
 * Sec. 3 across solves.  Every solve is one slot; a round advances the slots
 * the scheduling policy picks by one launch of a captured HIP graph of
 * graph_steps launches of the fused step kernel, whose persistent grid strides
 * over the row blocks of every picked slot (a slot table in device memory
 * tells each launch which slots to advance and from which buffer).  Solves may
 * differ in grid, parameters and step count but share the storage mode.  A
 * slot's arithmetic is exactly that of the same solve run alone with
 * lbm_step(), whatever the other slots are.
 *
 * Streams: rounds run on the pool's stream; admission (lbm_create of the
 * slot), moments and release run on a second stream the pool owns, so they
 * overlap a round in flight.  A round waits for the last admission.
 * One host thread drives a pool; calls on one pool must not overlap.
 * ------------------------------------------------------------------------ */
typedef struct lbm_pool lbm_pool;

typedef enum {
    LBM_SCHED_ALL = 0,   /* every slot with steps left runs in every round */
    LBM_SCHED_SRPT = 1,  /* slots by least remaining work (fluid cells x steps
                            left); the first always, further ones while the
                            cells per step stay within the first's cells plus
                            fill_cells; the rest wait for a later round */
    LBM_SCHED_VFT = 2    /* as SRPT, ordered by virtual finish time: admission
                            time + remaining work / throughput of recent full
                            rounds (small solves first, large ones not passed
                            indefinitely) */
} lbm_sched;

typedef struct {
    int32_t max_slots;         /* capacity of the slot table */
    int32_t active;            /* admitted solves not yet released */
    int32_t running;           /* active solves with steps left */
    int32_t graph_steps;       /* steps per round */
    int32_t sched;             /* lbm_sched */
    int32_t in_flight;         /* 1 between lbm_pool_launch and lbm_pool_wait */
    int64_t fill_cells;        /* SRPT cells-per-step bound in effect */
    int64_t arena_bytes;       /* caller's arena */
    int64_t free_bytes;        /* total free bytes of the slot heap */
    int64_t largest_free;      /* largest admissible footprint right now */
} lbm_pool_info;

/* Device bytes the pool itself needs besides its slots (slot table). */
int64_t lbm_pool_overhead_bytes(int32_t max_slots);

/* Creates a pool over a caller-owned device arena (256-byte aligned).  The
 * slots' footprints (lbm_required_bytes) are carved from the arena beyond the
 * pool overhead.  storage: lbm_storage shared by all slots.  graph_steps in
 * [1, 4096].  sched: lbm_sched.  fill_cells: SRPT/VFT bound, 0 = four row blocks
 * per resident workgroup of the persistent grid.  hip_stream NULL: the pool
 * creates its own stream.  Captures the graph.  LBM_E_NOMEM when the arena
 * cannot hold the overhead. */
int lbm_pool_create(int32_t storage, int32_t max_slots, int32_t graph_steps, int32_t sched, int64_t fill_cells,
                    void *dev_arena, int64_t arena_bytes, void *hip_stream, lbm_pool **out);

/* Admits a solve of nsteps steps: sub-allocates its footprint (first fit),
 * creates it in place on the admission stream (initial state written, as
 * lbm_create) and returns its slot index.  Allowed while a round is in flight.
 * LBM_E_NOMEM when no slot or no free range fits (nothing is changed); other
 * errors as lbm_create.  A slot admitted with nsteps = 0 never runs.  The
 * pool's graph runs one kernel for all slots: LBM_E_INVAL for
 * params->root_finder != 0 and for grids of 2^28 cells or more. */
int lbm_pool_admit(lbm_pool *pool, const lbm_params *params, int32_t nsteps, int32_t *slot_out);

/* Starts a round without waiting: picks the slots (policy), uploads the slot
 * table and launches the graph; each picked slot advances by
 * min(graph_steps, its steps left).  *nlaunched (nullable): slots picked, 0
 * when nothing has steps left (then nothing is launched).  LBM_E_INVAL when a
 * round is already in flight. */
int lbm_pool_launch(lbm_pool *pool, int32_t *nlaunched);

/* Waits for the round in flight (no-op without one) and books its steps.
 * finished (nullable, max_slots entries) receives the slots that reached
 * their step count in this round, *nfinished their number. */
int lbm_pool_wait(lbm_pool *pool, int32_t *finished, int32_t *nfinished);

/* lbm_pool_launch followed by lbm_pool_wait. */
int lbm_pool_run(lbm_pool *pool, int32_t *finished, int32_t *nfinished);

/* Steps taken and steps still to run of a slot.  The slot-level calls below
 * return LBM_E_INVAL for a slot that is not admitted, with the message on the
 * pool. */
int lbm_pool_slot_progress(const lbm_pool *pool, int32_t slot, int64_t *steps_done, int64_t *steps_left);

/* Moments of a slot, as lbm_moments().  LBM_E_INVAL for a slot of the round
 * in flight. */
int lbm_pool_moments(lbm_pool *pool, int32_t slot, double *out_host, double *totals);

/* Releases a slot and its arena range.  LBM_E_INVAL for a slot of the round
 * in flight. */
int lbm_pool_release(lbm_pool *pool, int32_t slot);

int lbm_pool_get_info(const lbm_pool *pool, lbm_pool_info *info);

/* Waits for everything the pool launched, releases every slot, the graph,
 * the admission stream and the pool (not the caller's arena). */
int lbm_pool_destroy(lbm_pool *pool);

/* Message of the last failure on pool, or of the calling thread's last
 * failed pool call that had no pool (pool = NULL).  Never NULL. */
const char *lbm_pool_last_error(const lbm_pool *pool);

#ifdef __cplusplus
}
#endif

#endif /* LBM13_LBM_H */
