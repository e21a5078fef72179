// Internal declarations shared by the host code and the HIP kernels of
// libpdbm.  Not part of the public ABI (include/pdbm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdbm.h"

namespace pdbm {

constexpr int NQ = 33;          // D2V33: rest particle + 4 speeds x 8 directions
constexpr int BLOCK = 256;      // threads per workgroup of the cell kernels
constexpr int HIST_CAP = 4096;  // drift reports kept per solve
constexpr int PART_RING = PDBM_MAX_CHUNK;  // records whose partial sums may wait to be added up
constexpr int NXCD = 8;         // accelerator complex dies of an MI355X
constexpr int NONEQ = PDBM_NONEQ_N;  // components of the non-equilibrium measures
constexpr int STRIP = 64;       // theta columns stored per wavefront, one per lane
constexpr int FUSE_ROWS = 16;   // most rows per wavefront of the two-step kernel (its edge cells sit in LDS)
constexpr int COL_K = 8;                  // steps per launch of the single-column kernel, at most
constexpr int COL_W = STRIP - 2 * COL_K;  // rows a wavefront owns in a single-column solve (48)

// Layout of f within one r row (33 * pitch elements): the rest particle's
// plane [pitch], then the 16 pairs of opposite directions of each speed, pair
// c = 4 (k - 1) + (i mod 4) holding directions i and i + 4 interleaved per
// column ([pitch][2]).  The pair of a cell is one 16-byte (float64) or
// 8-byte (float32) access, and the two members are updated together.
__host__ __device__ constexpr int pair_of(int q) { return 4 * ((q - 1) / 8) + ((q - 1) & 3); }
__host__ __device__ constexpr int member_of(int q) { return ((q - 1) & 7) >> 2; }
// Element offset of velocity q, column col, from the start of its r row.
__host__ __device__ constexpr int64_t elem_of(int q, int64_t col, int64_t pitch)
{
    return q == 0 ? col : pitch + 2 * pitch * pair_of(q) + 2 * col + member_of(q);
}

// Per-solve state in device memory written by the host.
struct SolveState {
    int64_t rec_from;  // drift records are produced for steps >= rec_from only
};

// Everything a kernel needs to know about one solve.  The step kernel reads
// it from device memory (one entry, or a table of entries for a packed
// launch over many solves); the cell kernels take it by value.
struct SolveDesc {
    void *f[2];         // float or double, r rows of NQ * pitch elements in the layout of elem_of
    double *lam[2];     // [nr][pitch]
    const double2 *cs;  // [ntheta] (cos theta_j, sin theta_j)
    SolveState *state;
    double *wpart;      // [PART_RING][nwaves][5] per-wavefront drift partial sums, slot (record % PART_RING)
    pdbm_diag *hist;    // [HIST_CAP] drift reports, record k for step k * diag_every
    int32_t nr, nt, pitch, sector;
    int32_t m, n, disc, reacts;          // disc: r_min == 0; reacts: w1+w2 > 0
    int32_t rows, nwaves, nstrip, diag_every;  // rows marched by one wavefront; its wavefronts
    int64_t plane;    // elements of the rest particle's plane (= pitch; a pair takes 2 * plane)
    int64_t rstride;  // elements between consecutive r rows of f (= NQ * pitch)
    int64_t nsteps;   // the solve stops advancing once it has taken this many steps
    double r_min, dr, dth;
    double dt_dr, dt_dth;  // dt/dr, dt/dtheta
    double omega;          // exp(-dt/tau) of the parameters' tau
    double w1, w2, Q, T_th, dt;
    double A[16];  // F_k(T) = sum_n A[(k-1)*4+n-1] T^n
    void *omegaf;  // float or double [nr][pitch] per-cell exp(-dt/tau) (PDBM_TAU_FIELD), else NULL
};

// Block-level drift reduction of the cell kernels (moments).
struct DiagCtl {
    double *partials;  // [nblocks][5]
    pdbm_diag *out;    // where the final record goes
    int64_t step;      // step count of the reduced state
};

// Kernel launchers (pdbm_step.hip, pdbm_step2.hip, pdbm_cells.hip).  All enqueue on `st` and return the
// hipError_t of the launch.
//
// One step of every solve listed: `descs` is a device array of solve
// descriptions; `tiles` maps each wavefront tile of the launch to (solve,
// tile of that solve), or is NULL for a single solve (descs[0], tiles
// 0..ntiles-1).  All solves share the precision; `rot` selects the variant
// for sectors other than the full annulus, `tauf` the variant that relaxes
// each cell with its own exp(-dt/tau) from SolveDesc::omegaf.
// The step a solve takes is bases[solve] + step_off (bases NULL: step_off);
// a solve whose step is at or beyond its nsteps is left alone.  A step that
// makes a drift record leaves partial sums that launch_records adds up.
// The state of step s of solve i lives in buffer (s + flip_i) & 1, flip_i =
// flips[i] ^ flip (flips NULL: flip), the parity its two-step launches have
// left.
hipError_t launch_step(const SolveDesc *descs, const uint2 *tiles, int ntiles, const int64_t *bases, int64_t step_off,
                       const int *flips, int flip, bool fp32, bool rot, bool tauf, hipStream_t st);
// Up to COL_K steps (nk) of single-column solves (ntheta = 1) in one launch
// of k_column; tiles, bases, step_off, flips and flip as launch_step.  Solve
// i takes min(nk, steps it has left) steps from buffer (s + flip_i) & 1 into
// the other one, so the caller toggles flip_i when that count is even.
hipError_t launch_column(const SolveDesc *descs, const uint2 *tiles, int ntiles, const int64_t *bases,
                         int64_t step_off, const int *flips, int flip, int nk, bool fp32, bool tauf, hipStream_t st);
// Steps s and s + 1 of every solve of the launch in one pass (tiles, bases,
// step_off, flips and flip as launch_step): reads buffer (s + flip_i) & 1 and
// writes the other one, so the caller toggles flip_i.  A solve with one step
// left, or every solve with `single`, takes one step and keeps its parity.
// ntheta > 1, rows per wavefront at most FUSE_ROWS; `rot` selects the
// variant for sectors other than the full annulus (discs included).  Makes the drift
// records of the steps it takes as launch_step does; `tauf` as launch_step.
hipError_t launch_step2(const SolveDesc *descs, const uint2 *tiles, int ntiles, const int64_t *bases,
                        int64_t step_off, const int *flips, int flip, bool single, bool fp32, bool tauf, bool rot,
                        hipStream_t st);
// Per-cell relaxation factors omegaf[i][j] = exp(-dt / tau[i * nt + j]) from
// a dense float64 tau field in device memory, or all equal to `uniform`
// with tau NULL; stored in the solve's precision.
hipError_t launch_omega(const SolveDesc &d, bool fp32, const double *tau, double uniform, hipStream_t st);
// Non-equilibrium measures (Sec. II.E) of the state in buffer `cur` into
// device memory out [NONEQ][nr][nt] float64.
hipError_t launch_noneq(const SolveDesc &d, int cur, bool fp32, double *out, hipStream_t st);
// bases[i] += by for i < n.  With flips (after `by` steps taken as two-step
// launches, a single launch closing an odd count): flips[i] toggles when
// solve i took an odd number of two-step launches, min(left, by) / 2 of them
// with left = max(nsteps - bases[i], 0).  With flips and column_k > 0 (the
// steps taken as k_column launches of min(column_k, steps of the run left)):
// flips[i] toggles for each launch in which solve i took an even number of
// steps.
hipError_t launch_advance(const SolveDesc *descs, int *flips, int64_t *bases, int n, int64_t by, int column_k,
                          hipStream_t st);
// Drift records of steps [base + lo, base + hi) of solves descs[0..n), base =
// bases[i] (0 if bases is NULL); at most PART_RING steps per call, and the
// steps must have been launched before on the same stream.
hipError_t launch_records(const SolveDesc *descs, int n, const int64_t *bases, int64_t lo, int64_t hi,
                          hipStream_t st);
// Cell kernels on buffer `cur` of one solve.
hipError_t launch_init_ic(const SolveDesc &d, int cur, bool fp32, const pdbm_ic &ic, hipStream_t st);
hipError_t launch_init_fields(const SolveDesc &d, int cur, bool fp32, const double *fields, hipStream_t st);
hipError_t launch_moments(const SolveDesc &d, int cur, bool fp32, double *out, const DiagCtl &dc, hipStream_t st);
int cell_blocks(int nr, int nt);
// Wavefront tiles of a solve marched `rows` rows at a time.
int solve_waves(int nr, int nt, int rows);
// Rows per wavefront of the step kernel for a solve that has the GPU to itself.
int rows_per_wave(const pdbm_params &p);

}  // namespace pdbm
