// Host-side internals shared by the single-solve, batch and server parts of
// libpdbm.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "pdbm_internal.h"

namespace pdbm {

// Records `msg` as the calling thread's last error and returns `code`.
int fail(int code, const std::string &msg);

#define PDBM_HIPCHK(call)                                                                                      \
    do {                                                                                                       \
        hipError_t e_ = (call);                                                                                \
        if (e_ != hipSuccess) return ::pdbm::fail(PDBM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device memory of one solve, in this order (all offsets 256-byte aligned):
// the state (two f buffers, two lambda buffers, the per-cell relaxation
// factors of a solve with PDBM_TAU_FIELD), then the auxiliary part
// (theta table, description, step state, drift partial sums and records,
// moments reduction scratch).
struct Layout {
    size_t f, lam, omega, cs, desc, state, wpart, hist, cpart, total;  // omega: per-cell relaxation factors (0 without PDBM_TAU_FIELD)
    size_t state_total, aux_total;  // total = state_total + aux_total
    int pitch, rows, nwaves, cblocks;
    size_t esz;
};

Layout layout_of(const pdbm_params &p, int rows);
class Solve;
// Non-equilibrium measures of the current state into host `out`
// [NONEQ][nr][ntheta] (staged in the idle f buffer; synchronises st).
int noneq_to_host(const Solve &s, double *out, hipStream_t st);
int check_device();

// One solve resident on the GPU: its buffers, the description its kernels
// read and a host mirror of its step counter.
class Solve {
  public:
    pdbm_params p{};
    Layout L{};
    bool fp32 = false, own = false;
    char *ws = nullptr;
    SolveDesc hd{};           // host copy, pointers filled in
    SolveDesc *dd = nullptr;  // device copy read by the step kernel
    double *cpart = nullptr;  // moments-kernel reduction scratch
    int64_t step = 0;      // steps taken (never beyond hd.nsteps)
    int flip = 0;          // the current state is in buffer (step + flip) & 1 (two-step launches toggle it)
    int64_t rec_from = 0;  // drift records are valid from this step on
    int64_t red_to = 0;    // records of steps before this one have been added up
    SolveState zero_state{};  // staging of the step-state upload (kept until the next sync)

    // Lays out the solve in `workspace` (or a fresh allocation), uploads its
    // description and enqueues its initial state on `st`.  `rows`: rows per
    // wavefront; `nsteps`: step count after which the solve stops advancing.
    // With `aux`, the workspace holds the state only (L.state_total bytes)
    // and the auxiliary part goes to `aux` (L.aux_total bytes, 256-byte
    // aligned).  Allocates device memory only when workspace is NULL and no
    // host memory at all.
    int init(const pdbm_params &p, const pdbm_ic *ic, void *workspace, size_t bytes, int rows, int64_t nsteps,
             hipStream_t st, char *aux = nullptr);
    void release();  // frees an owned workspace (the stream must be idle)

    int cur() const { return (int)((step + flip) & 1); }
    // Whether two steps may go in one launch: ntheta > 1 and row blocks of
    // at most FUSE_ROWS rows (either precision, any sector; PDBM_FUSE=0
    // turns it off).
    bool fusable() const;
    // Whether a launch may take up to COL_K steps: a single theta column
    // (PDBM_FUSE=0 turns it off: one step per launch, k_step).
    bool columnar() const;
    int waves() const { return L.nwaves; }
    bool rot() const { return p.sector != 8; }
    bool tauf() const { return hd.omegaf != nullptr; }  // relaxes with a per-cell tau
    // Sets the step count on host and device (stream must be idle).
    int set_step(int64_t s, hipStream_t st);
    // Enqueues the adding up of the drift partial sums of steps [red_to,
    // step), at most PART_RING steps (single-solve launches only).
    int reduce_records(hipStream_t st);
    // Fields [6][nr][ntheta] of the current state into device memory `out`
    // and the drift report into `diag_dev` (both enqueued on st).
    int moments(double *out, pdbm_diag *diag_dev, hipStream_t st) const;
};

// Ends a solver made by pdbm_create_noalloc: frees its device's static
// scratch for the next one (pdbm_noalloc.hip).
void release_scratch_solver(int dev);

}  // namespace pdbm

// Handle of one solve (the opaque pdbm_solver of the ABI).
struct pdbm_solver {
    pdbm::Solve s;
    hipStream_t st = nullptr;
    int scratch_dev = -1;  // device whose static scratch holds the auxiliary part (pdbm_create_noalloc), or -1
};
