/*
 * pdbm.h -- C ABI of libpdbm, a gfx950 (MI355X) implementation of the
 * per-timestep update of the polar-coordinate lattice Boltzmann kinetic model
 * of detonation of Lin, Xu, Zhang and Li (arXiv:1308.0653).
 *
 * One time step of one solve (Sec. II.C and III.A of the paper):
 *   1. moments rho, u, T (p = rho T) of the 33 discrete distributions f_ki
 *      of the D2V33 velocity set (Sec. II.B);
 *   2. f^eq rebuilt from the moment-matched weights F_k(T) (Sec. II.B);
 *   3. BGK relaxation solved analytically over dt, plus the chemical term
 *      M_ki dt (Sec. II.A-B) driven by Cochran's rate
 *      R = w1 p^m (1-lambda) + w2 p^n lambda (1-lambda), active where
 *      T > T_th (Sec. III.A);
 *   4. first-order upwind advection of f_ki in r and theta with Courant
 *      numbers C_r = v_kir dt/dr, C_theta = v_kitheta dt/(r dtheta) (the
 *      geometric 1/r term), a periodic theta halo and radial boundaries
 *      (Sec. II.C-D); the reaction progress lambda is integrated in closed
 *      form and advected upwind by the cell's own u (Sec. III.A).
 * All four run in one fused kernel launch per step on the caller's stream
 * (full-annulus solves: one launch per two steps, see pdbm_step).
 *
 * Conventions
 *   - Every entry point returns 0 (PDBM_OK) or a negative PDBM_E* code;
 *     pdbm_last_error() gives a message for the calling thread's last error.
 *   - Host buffers passed in are read during the call and not retained.
 *     Buffers passed out are written during the call.
 *   - `stream` is a hipStream_t (for example torch.cuda.current_stream()
 *     .cuda_stream); NULL means the default stream.  All device work of a
 *     solver is enqueued on its stream.
 *   - Grids are cell-centred: r_i = r_min + (i + 1/2) dr, dr = (r_max -
 *     r_min)/nr; theta_j = (j + 1/2) dtheta, dtheta = sector*pi/4 / ntheta.
 *   - Field arrays exchanged with the caller are float64, C order, no
 *     padding: [F][nr][ntheta].
 *   - A solver is driven from one host thread at a time.  The server entry
 *     points are thread-safe.
 *
 * Environment (read once per process; for measurement and tuning)
 *   PDBM_FUSE=0            every launch (single solves, batches, servers)
 *                          takes a single step.
 *   PDBM_ROWS_PER_WAVE=n   r rows per wavefront of single solves (created
 *                          after it is set); above 16 disables two-step
 *                          launches.
 *   PDBM_BATCH_ROWS=n      r rows per wavefront of packed grids of more
 *                          than one column (16); above 16 disables
 *                          two-step launches.
 */
#ifndef PDBM_H
#define PDBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes -- */
enum {
    PDBM_OK = 0,
    PDBM_EINVAL = -1,   /* invalid argument or parameter                     */
    PDBM_ECFL = -2,     /* |C_r| + |C_theta| > 1 somewhere (donor cell bound) */
    PDBM_ENOMEM = -3,   /* device or host allocation failed / buffer too small */
    PDBM_EHIP = -4,     /* a HIP runtime call failed                          */
    PDBM_EAGAIN = -5,   /* request not finished yet                           */
    PDBM_ENOENT = -6,   /* unknown request id                                 */
    PDBM_ENONPHYS = -7, /* non-finite value, rho <= 0 or T <= 0 was detected  */
    PDBM_ENOSYS = -8    /* no usable gfx950 device                            */
};

enum { PDBM_FP64 = 0, PDBM_FP32 = 1 };                        /* precision   */
enum { PDBM_QUEUED = 0, PDBM_RUNNING = 1, PDBM_DONE = 2, PDBM_FAILED = 3 }; /* request */
enum { PDBM_ALLOW_CFL = 1, PDBM_TAU_FIELD = 2 };               /* flags       */

/* Problem statement of one solve (Sec. II.D and III of the paper).
 *   nr, ntheta   cells in r and theta (>= 1, nr * ntheta <= 2^24, and one
 *                f buffer, 33 * nr * pitch elements of 8 or 4 bytes with
 *                pitch = ntheta rounded up to a multiple of 64, or 2 for
 *                ntheta = 1, below 4 GiB: float64 grids up to about
 *                4034 x 4000 cells, float32 up to 2^24 cells)
 *   sector       azimuthal extent s*pi/4, s in 1..8 (8 = full annulus).  The
 *                periodic theta halo rotates the direction index by s:
 *                f_{k,i}(j=-1) = f_{k,(i+s)%8}(ntheta-1),
 *                f_{k,i}(j=ntheta) = f_{k,(i-s)%8}(0).
 *   precision    PDBM_FP64: f stored and updated in float64.
 *                PDBM_FP32: f stored and updated in float32; F_k(T), the
 *                reaction rate, lambda and all reductions stay float64.
 *   m, n         integer pressure exponents of Cochran's rate (>= 0)
 *   diag_every   record the drift diagnostics every this many steps (0: off)
 *   flags        PDBM_ALLOW_CFL skips the Courant-number check;
 *                PDBM_TAU_FIELD gives the solve a per-cell relaxation time
 *                (see pdbm_set_tau; single solves only)
 *   r_min,r_max  0 <= r_min < r_max.  r_min > 0: annulus with zero-gradient
 *                ghost cells at both radial ends.  r_min = 0: disc, whose
 *                centre uses the paper's ghost rule
 *                f(-1, j, k, i) = f(0, j, k, (i+4)%8) (Sec. II.D), the
 *                image of the cell across the centre; a disc needs sector
 *                1, 2 or 4, where that image is this rule (PDBM_EINVAL
 *                otherwise).
 *   dt, tau      time step and BGK relaxation time (> 0; tau may be +inf;
 *                with PDBM_TAU_FIELD, the value every cell starts with)
 *   w1, w2       Cochran rate constants (>= 0)
 *   Q            heat release per unit mass (>= 0)
 *   T_th         ignition temperature: reaction only where T > T_th       */
typedef struct pdbm_params {
    int32_t nr, ntheta;
    int32_t sector;
    int32_t precision;
    int32_t m, n;
    int32_t diag_every;
    int32_t flags;
    double r_min, r_max;
    double dt, tau;
    double w1, w2;
    double Q, T_th;
} pdbm_params;

/* Two-region initial state (Sec. III.B-D).  A cell whose centre radius is
 * below r_split takes `inner`, every other cell `outer`; each tuple is
 * (rho, T, u_r, u_theta, lambda) in the paper's order.  Uniform noise is
 * added to the pressure of every cell: p = rho*T + p_noise*(2U - 1) with
 * U = (splitmix64(seed ^ (c * 0x9E3779B97F4A7C15)) >> 11) * 2^-53, c =
 * i*ntheta + j, and T = p / rho.  f starts at f^eq of that state. */
typedef struct pdbm_ic {
    double r_split;
    double inner[5];
    double outer[5];
    double p_noise;
    uint64_t seed;
} pdbm_ic;

/* Drift report of one state: area-weighted (r_i dr dtheta) float64 sums of
 * mass rho, total energy rho T + rho |u|^2/2 and unreleased chemical energy
 * rho Q (1 - lambda); counts of cells holding a non-finite value and of
 * cells with rho <= 0 or T <= 0.  `step` is the step count of the state. */
typedef struct pdbm_diag {
    int64_t step;
    double mass, energy, chem;
    int64_t n_nonfinite, n_nonphys;
} pdbm_diag;

typedef struct pdbm_solver pdbm_solver;
typedef struct pdbm_batch pdbm_batch;
typedef struct pdbm_server pdbm_server;

/* --------------------------------------------------------- host helpers -- */
const char *pdbm_strerror(int code);
/* Message of the calling thread's most recent error ("" if none). */
const char *pdbm_last_error(void);
int pdbm_version(void);

/* Checks a problem statement (and an initial state, which may be NULL)
 * without touching a GPU.  PDBM_EINVAL for bad values (see pdbm_params and
 * pdbm_ic: rho > 0, T > 0, finite values), PDBM_ECFL when the largest
 * |C_r| + |C_theta| over the grid for the fastest speed exceeds 1 and
 * PDBM_ALLOW_CFL is not set.  `cfl` (may be NULL) receives that largest
 * Courant sum. */
int pdbm_validate(const pdbm_params *p, const pdbm_ic *ic, double *cfl);

/* Device bytes of one solve's state (two f buffers, two lambda buffers,
 * tables and reduction scratch) for the given parameters. */
int pdbm_state_bytes(const pdbm_params *p, size_t *bytes);

/* The once-computed moment-inversion matrix (Sec. II.B): the weights are
 * F_k(T) = sum_{n=1..4} A[(k-1)*4 + (n-1)] T^n for k = 1..4, obtained on the
 * host in float64 by inverting sum_k 8 F_k v_k^(2n) = 2^n n! T^n; F_0 =
 * 1 - 8 sum_k F_k.  A must hold 16 doubles. */
int pdbm_fk_matrix(double *A);

/* ------------------------------------------------------------ one solve -- */
/* Creates a solve and enqueues its initial state on `stream`.
 *   ic          two-region initial state, or NULL for a state of rho = 1,
 *               T = 1, u = 0, lambda = 0 (to be replaced by pdbm_set_fields
 *               or pdbm_write_f)
 *   workspace   device memory of at least pdbm_state_bytes() bytes owned by
 *               the caller (never freed by the library), or NULL for the
 *               library to allocate its own
 * Errors: PDBM_EINVAL / PDBM_ECFL as pdbm_validate, PDBM_ENOMEM if the
 * workspace is too small or allocation fails, PDBM_ENOSYS without a gfx950
 * device, PDBM_EHIP. */
int pdbm_create(const pdbm_params *p, const pdbm_ic *ic, void *workspace, size_t workspace_bytes, void *stream,
                pdbm_solver **out);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): pdbm_create without any
 * allocation, device or host.  The caller's device buffer `state` holds the
 * solve's state only (two f buffers and two lambda buffers); everything else
 * a solve keeps on the device (solve description, theta table, drift
 * partial sums and records, the moments reduction's partials and counter)
 * lives in a static array of PDBM_SCRATCH_BYTES in the library, one per
 * device, and the handle itself is that device's static slot.
 *   state == NULL   *state_bytes receives the bytes the state needs (the
 *                   parameters are validated; no device is touched)
 *   state != NULL   at least that many bytes, 256-byte aligned, owned by the
 *                   caller and never freed by the library
 * The solver works with every single-solve entry point and ends with
 * pdbm_destroy, which frees the device's slot.  At most one such solver
 * exists per device at a time: PDBM_EAGAIN while another holds the slot.
 * The static array keeps what the previous solver left; everything that must
 * start at zero is cleared here, on the solver's stream.
 * Errors: as pdbm_create; PDBM_ENOMEM if the state buffer is too small or
 * the solve needs more than PDBM_SCRATCH_BYTES of auxiliary memory (about
 * 2048 x 2048 cells). */
enum { PDBM_SCRATCH_BYTES = 16 << 20 };
int pdbm_create_noalloc(const pdbm_params *p, const pdbm_ic *ic, void *state, size_t *state_bytes, void *stream,
                        pdbm_solver **out);
void pdbm_destroy(pdbm_solver *s);

/* Sets the state to f = f^eq of host fields [5][nr][ntheta] = (rho, T, u_r,
 * u_theta, lambda) and the step count to 0.  Synchronous. */
int pdbm_set_fields(pdbm_solver *s, const double *fields);

/* Per-cell relaxation time.  The paper (Sec. IV, point (ii)) notes that tau
 * should depend on the local state (density, temperature), and so vary in
 * space and time, without giving a form; these calls let the caller supply
 * it.  The solve must have been created with PDBM_TAU_FIELD (PDBM_EINVAL
 * otherwise); its cells then relax over each step with their own
 * exp(-dt / tau[i][j]) in place of the parameters' tau, and nothing else
 * in the step changes.  The field holds until it is set again, so a caller
 * can update it between calls of pdbm_step.
 *   pdbm_set_tau        host tau [nr][ntheta] float64, each > 0 (+inf: no
 *                       relaxation in that cell; PDBM_EINVAL otherwise), or
 *                       NULL for the parameters' tau everywhere.
 *                       Synchronous.
 *   pdbm_set_tau_async  the same from device memory [nr][ntheta] float64,
 *                       enqueued on the solver's stream; the values are not
 *                       checked (a value <= 0 or NaN gives non-physical
 *                       states).  The buffer must stay valid until the
 *                       stream reaches the call. */
int pdbm_set_tau(pdbm_solver *s, const double *tau);
int pdbm_set_tau_async(pdbm_solver *s, const void *tau_device);

/* Enqueues `nsteps` time steps on the solver's stream and returns without
 * waiting.  Every diag_every-th step also records the drift report of the
 * state it starts from.  Solves of the full annulus with ntheta > 1, in
 * either precision, take the steps two per launch (one pass over f for both;
 * the result equals that of single steps to rounding), and an odd count ends
 * with a single step; solves with a single theta column take up to 8 steps
 * per launch.  The states after every call are those of Sec. II.C's scheme
 * either way. */
int pdbm_step(pdbm_solver *s, int64_t nsteps);

/* Number of steps taken so far (host-side counter). */
int64_t pdbm_step_count(const pdbm_solver *s);

/* Writes host fields [6][nr][ntheta] = (rho, u_r, u_theta, T, p, lambda) of
 * the current state (out may be NULL) and its drift report (diag may be
 * NULL).  Synchronises the stream.  Returns PDBM_ENONPHYS (after filling the
 * outputs) if the state holds non-finite values or rho <= 0 or T <= 0. */
int pdbm_moments(pdbm_solver *s, double *out, pdbm_diag *diag);

/* As pdbm_moments, but enqueued on the stream into caller-owned device
 * memory [6][nr][ntheta] float64 without synchronising. */
int pdbm_moments_async(pdbm_solver *s, void *out_device);

/* Non-equilibrium measures of Sec. II.E ("non-equilibrium characteristics"):
 * Delta*_m = M*_m(f) - M*_m(f^eq), the central moments about the cell's own
 * u of f minus those of its equilibrium, in polar components of the cell's
 * frame (e_r, e_theta at theta_j):
 *   M*_2     = sum f v* v*              M*_3     = sum f v* v* v*
 *   M*_{3,1} = sum 1/2 f (v*.v*) v*     M*_{4,2} = sum 1/2 f (v*.v*) v* v*
 * with v* = v - u, computed in float64 (also for an FP32 solver).  `out`:
 * host [PDBM_NONEQ_N][nr][ntheta] float64, components in the order of the
 * enum below.  Synchronises the stream. */
enum {
    PDBM_NONEQ_D2_RR, PDBM_NONEQ_D2_RT, PDBM_NONEQ_D2_TT,
    PDBM_NONEQ_D3_RRR, PDBM_NONEQ_D3_RRT, PDBM_NONEQ_D3_RTT, PDBM_NONEQ_D3_TTT,
    PDBM_NONEQ_D31_R, PDBM_NONEQ_D31_T,
    PDBM_NONEQ_D42_RR, PDBM_NONEQ_D42_RT, PDBM_NONEQ_D42_TT,
    PDBM_NONEQ_N
};
int pdbm_noneq(pdbm_solver *s, double *out);
/* As pdbm_noneq, enqueued on the stream into caller-owned device memory
 * [PDBM_NONEQ_N][nr][ntheta] float64 without synchronising. */
int pdbm_noneq_async(pdbm_solver *s, void *out_device);

/* Copies up to `cap` of the most recent drift reports recorded while
 * stepping (oldest first) into `out`; *n receives how many.  At most 4096
 * are kept.  Synchronises the stream. */
int pdbm_diag_history(pdbm_solver *s, pdbm_diag *out, int32_t cap, int32_t *n);

/* Raw state in float64, host memory: f as [33][nr][ntheta] with velocity
 * index q = 0 (rest) or 1 + 8(k-1) + i (speed k = 1..4, direction i*pi/4,
 * i = 0..7, directions fixed in the Cartesian frame), lambda as
 * [nr][ntheta].  Either pointer may be NULL.  Synchronous.  Writing sets the
 * step count to `step`; an FP32 solver rounds f to float32. */
int pdbm_read_f(pdbm_solver *s, double *f, double *lam);
int pdbm_write_f(pdbm_solver *s, const double *f, const double *lam, int64_t step);

/* Checkpoint of the full state (f in the solver's precision, lambda, step
 * count) as an opaque host blob.  With buf == NULL, *bytes receives the
 * size.  pdbm_set_state accepts only a blob of a solve with the same nr,
 * ntheta and precision.  Synchronous. */
int pdbm_get_state(pdbm_solver *s, void *buf, size_t *bytes);
int pdbm_set_state(pdbm_solver *s, const void *buf, size_t bytes);

/* -------------------------------------------------------- packed batch -- */
enum { PDBM_MAX_CHUNK = 64 }; /* most steps captured in one graph */

/* A fixed set of independent solves (each with its own grid, parameters and
 * initial state; all of one precision) advanced together: one launch takes
 * every member with ntheta > 1 two steps (one step where a count is odd),
 * and one launch of another kernel takes every single theta column up to 8
 * steps.  Runs of `chunk_steps` steps are captured once in a HIP graph and
 * replayed (chunk_steps = 0: plain launches; at most PDBM_MAX_CHUNK, else
 * PDBM_EINVAL).  Graphs need a stream other than the null stream: with
 * stream = NULL and chunk_steps > 1 the batch creates a stream of its own.
 * Each member's fields are bitwise those it would have alone in a batch of
 * its own.  Errors as pdbm_create, for any member. */
int pdbm_batch_create(int32_t n, const pdbm_params *params, const pdbm_ic *ics, int32_t chunk_steps, void *stream,
                      pdbm_batch **out);
void pdbm_batch_destroy(pdbm_batch *b);
/* Enqueues nsteps steps of every member; returns without waiting. */
int pdbm_batch_step(pdbm_batch *b, int64_t nsteps);
int64_t pdbm_batch_step_count(const pdbm_batch *b, int32_t i);
/* As pdbm_moments, for member i. */
int pdbm_batch_moments(pdbm_batch *b, int32_t i, double *out, pdbm_diag *diag);
/* As pdbm_noneq, for member i. */
int pdbm_batch_noneq(pdbm_batch *b, int32_t i, double *out);

/* ------------------------------------------------- continuous batching -- */
/* A request server: submitted solves wait in a first-come-first-served queue
 * and are admitted, between chunks of `chunk_steps` (1 to PDBM_MAX_CHUNK)
 * steps, while fewer than `max_slots` run and the device memory of the
 * running ones stays within `hbm_cap_bytes` (a packed solve takes its
 * pdbm_state_bytes up to the drift partial-sum ring, which scales with its
 * number of wavefronts and so with the packed row blocks).  All running solves advance together
 * in packed, graph-captured launches on the server's stream (NULL: a stream
 * of its own) driven by a scheduler thread; a solve leaves at the chunk
 * boundary after it reaches its step count.  Submit and poll are
 * thread-safe. */
enum { PDBM_KEEP_FIELDS = 1 }; /* submit flag: keep the final fields for pdbm_poll */

typedef struct pdbm_server_stats {
    int64_t submitted, queued, running, done, failed;
    int64_t steps_launched; /* chunks run x chunk_steps                      */
    size_t hbm_in_use, hbm_cap;
    double cell_updates;    /* grid cells x steps of the solves that finished */
    double elapsed;         /* seconds since the server was created            */
} pdbm_server_stats;

int pdbm_server_create(size_t hbm_cap_bytes, int32_t max_slots, int32_t chunk_steps, void *stream,
                       pdbm_server **out);
/* Stops admitting, fails queued requests and those still running after the
 * chunk in progress, joins the scheduler and frees everything. */
void pdbm_server_destroy(pdbm_server *s);
/* Queues a solve of `nsteps` steps and returns its id without waiting.
 * PDBM_EINVAL / PDBM_ECFL as pdbm_validate; PDBM_ENOMEM if the solve alone
 * exceeds the memory cap. */
int pdbm_submit(pdbm_server *s, const pdbm_params *p, const pdbm_ic *ic, int64_t nsteps, uint32_t flags,
                uint64_t *req_id);
/* State of a request (PDBM_QUEUED / RUNNING / DONE / FAILED).  Returns
 * PDBM_EAGAIN while it has not finished; once finished, fills `diag` (drift
 * report of the final state) and, if it was submitted with
 * PDBM_KEEP_FIELDS, `out` ([6][nr][ntheta] as pdbm_moments).  A request
 * fails when its state turns non-finite or non-physical; the others are
 * unaffected.  PDBM_ENOENT for an unknown id. */
int pdbm_poll(pdbm_server *s, uint64_t req_id, int32_t *state, double *out, pdbm_diag *diag);
/* Seconds since server creation at submit, admission and completion
 * (-1 where it has not happened): times[3]. */
int pdbm_request_times(pdbm_server *s, uint64_t req_id, double *times);
/* Forgets a finished request and its kept fields. */
int pdbm_release(pdbm_server *s, uint64_t req_id);
/* Waits until no request is queued or running (timeout_s < 0: no limit);
 * PDBM_EAGAIN on timeout. */
int pdbm_server_wait(pdbm_server *s, double timeout_s);
int pdbm_server_get_stats(pdbm_server *s, pdbm_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* PDBM_H */
