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
constexpr int NXCD = 8;         // accelerator complex dies of an MI355X
constexpr int STRIP = 62;       // theta columns stored per wavefront (64 lanes minus 2 halo lanes)

// Everything a kernel needs to know about one solve.  Passed by value as a
// kernel argument (one solve per launch) or read from a device table (packed
// launches over many solves).
struct SolveDesc {
    const void *f_in;  // [nr][NQ][pitch] of float or double: the 33 velocity rows of one r row are adjacent
    void *f_out;
    const double *lam_in;  // [nr][pitch]
    double *lam_out;
    const double2 *cs;  // [ntheta] (cos theta_j, sin theta_j)
    int32_t nr, nt, pitch, sector;
    int32_t m, n, disc, reacts;  // disc: r_min == 0; reacts: w1+w2 > 0
    int32_t rows, pad_;          // rows marched by one wavefront per step
    int64_t plane;               // elements between the rows of consecutive velocities (= pitch)
    int64_t rstride;             // elements between consecutive r rows of f (= NQ * pitch)
    double r_min, dr, dth;
    double dt_dr, dt_dth;  // dt/dr, dt/dtheta
    double omega;          // exp(-dt/tau)
    double w1, w2, Q, T_th, dt;
    double A[16];  // F_k(T) = sum_n A[(k-1)*4+n-1] T^n
};

// The two f and lambda buffers of one step (they swap every step).
struct StepBufs {
    const void *f_in;
    void *f_out;
    const double *lam_in;
    double *lam_out;
};

// Drift-report reduction state of one solve.
struct DiagCtl {
    double *partials;    // [nblocks][5]
    unsigned *counter;   // blocks finished, reset by the last one
    pdbm_diag *out;      // where the final record goes
    int64_t step;        // step count of the reduced state
    int32_t enabled;
    int32_t pad;
};

// Kernel launchers (pdbm_kernels.hip).  All enqueue on `st` and return the
// hipError_t of the launch.
// The step kernel reads the solve's description from device memory
// (dev_desc, a copy of d); d's buffer pointers give this step's buffers.
hipError_t launch_step(const SolveDesc &d, const SolveDesc *dev_desc, bool fp32, const DiagCtl &dc, hipStream_t st);
hipError_t launch_init_ic(const SolveDesc &d, bool fp32, const pdbm_ic &ic, hipStream_t st);
hipError_t launch_init_fields(const SolveDesc &d, bool fp32, const double *fields, hipStream_t st);
hipError_t launch_moments(const SolveDesc &d, bool fp32, double *out, const DiagCtl &dc, hipStream_t st);
int cell_blocks(const SolveDesc &d);
int step_blocks(const SolveDesc &d);
// Rows per wavefront of the step kernel for an nr x nt grid.
int rows_per_wave(int nr, int nt, bool fp32);

}  // namespace pdbm
