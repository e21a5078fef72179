// One time step per launch (k_step): every solve of the launch, float64 or
// float32, full annulus or rotated sector, wavefront strips of 64 theta
// columns or, for a single column, wavefronts of 64 rows; and the kernels
// that add up the drift records (k_records) and move packed solves' step
// bases on (k_advance).
#include "pdbm_device.h"

namespace pdbm {
namespace {

// One step of the rows of a solve with a single theta column (ntheta = 1,
// the quasi-one-dimensional runs of Sec. III) in packed launches: lane l
// holds row COL_W blk + l and owns it for l < COL_W (the rows a wavefront
// owns are those of k_column, so that the two keep the same per-wavefront
// drift partial sums).  Radial neighbours come from the adjacent lanes (DPP
// shifts) and, for lanes 0 and 63, from gathers of the rows below and above
// the block, which apply the radial ghost rules of Sec. II.D.  The azimuthal
// neighbours of a cell are the cell itself with directions turned by the
// sector (periodic halo, f_{k,i}(j-1) = f_{k,(i+s)%8}(j) and f_{k,i}(j+1) =
// f_{k,(i-s)%8}(j)); they are read back from the wavefront's LDS slot.
// The arithmetic per cell is that of update_row.
template <typename real, bool TAUF>
__device__ __forceinline__ void radial_block(DescPtr dp, const StepBufs &bufs, int blk, real (*slot)[64],
                                             double red[5], bool diag)
{
    const int lane = threadIdx.x & 63;
    const int nr = dp->nr, sec = dp->sector;
    const bool store = lane < COL_W && blk * COL_W + lane < nr;
    const __amdgpu_buffer_rsrc_t fin = rsrc_of(bufs.f_in), fout = rsrc_of(bufs.f_out);
    const __amdgpu_buffer_rsrc_t lin = rsrc_of(bufs.lam_in), lout = rsrc_of(bufs.lam_out);
    const RowBytes b = row_bytes_of(dp->rstride, dp->pitch, (int)sizeof(real));
    const uint32_t rb = b.rest, pb = b.pair;  // rest plane, one pair (column 0)
    // the lane's row, and gathers of the row below the block (ghost of row 0
    // at r_min: a copy, or at the disc centre row 0 with directions turned
    // by 4) and of the row above it (clamped: the zero-gradient copy of the
    // last row)
    const RadialOffsets o = radial_offsets(nr, dp->pitch, dp->disc, (int)sizeof(real), b, blk, lane);
    const int re = o.re;
    const uint32_t vo = o.vo, vol = o.vol;

    real fc[NQ];
    double lc;
    bload(fc[0], fin, vo, 0u);
#pragma unroll
    for (int c = 0; c < 16; ++c)
        bload2(fc[1 + 8 * (c >> 2) + (c & 3)], fc[5 + 8 * (c >> 2) + (c & 3)], fin, vo, rb + (uint32_t)c * pb);
    bload(lc, lin, vol, 0u);
    real hf[2];
    double hlam;
    bload(hf[0], fin, o.vh1, 0u);
    bload(hf[1], fin, o.vh2, 0u);
    bload(hlam, lin, o.vhl, 0u);

    // (1)-(3) moments, weights, f^eq polynomial, BGK and chemical factors
    const Cell<real> C(dp, fc, lc, omega_at<real, TAUF>(dp, o.om, 0u));
    const real rho = C.rho, e = C.e, ux = C.ux, uy = C.uy, u2 = C.u2, T = C.T;
    const real beta = C.beta, omega = C.omega, keep = C.keep, Bz = C.Bz;
    const double Td = C.Td;
    const real *F = C.F;
    const EqPoly<real> &EP = C.EP;

    // polar components of directions dd = 0..3 at theta_0 (dd+4 is the negative)
    const double2 cs = dp->cs[0];
    const real cth = (real)cs.x, sth = (real)cs.y;
    const real crv[4] = {cth, (real)SQH * (cth + sth), sth, (real)SQH * (sth - cth)};
    const real ctv[4] = {-sth, (real)SQH * (cth - sth), cth, (real)SQH * (cth + sth)};
    const double ri = dp->r_min + ((double)re + 0.5) * dp->dr;
    const real kr = (real)dp->dt_dr, kt = (real)(dp->dt_dth / ri);
    real acr[4], act[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        acr[dd] = fabs(crv[dd]) * kr;
        act[dd] = fabs(ctv[dd]) * kt;
    }
    // the cell's distributions, for its rotated azimuthal neighbours
#pragma unroll
    for (int q = 0; q < NQ; ++q) slot[q][lane] = fc[q];

    const real rest = rho * F[0] * EP.c0 * (keep + beta * (u2 - (real)2 * T)) + omega * fc[0];
    if (store) bstore(rest, fout, vo, 0u);
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
        const real v = (real)speed(k);
        const real rF = rho * F[k];
        const real rA = rF * (keep + beta * (v * v + u2 - (real)2 * T)), rB = rF * Bz;
        const int base = 1 + 8 * (k - 1);
        real o[8];
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            real E, O;
            pair_coll(EP, v * EP.w(dd), rA, rB, E, O);
            const real s = omega - v * (acr[dd] + act[dd]);
#pragma unroll
            for (int sgn = 0; sgn < 2; ++sgn) {
                const int q = base + dd + 4 * sgn;
                const real x = fc[q];
                // radial upwind (C_r >= 0 takes the row below); every lane
                // takes both shifts, then selects
                const real sl = from_left(x), sr = from_right(x);
                const real hl = halo_left(hf, q), hr = halo_right(hf, q);
                const real lower = lane == 0 ? hl : sl;
                const real upper = lane == 63 ? hr : sr;
                const bool below = sgn == 0 ? crv[dd] >= (real)0 : crv[dd] < (real)0;
                const real nbr = below ? lower : upper;
                // azimuthal upwind (C_theta >= 0 takes j-1): this cell with
                // the direction index turned by +s (j-1) or -s (j+1)
                const bool left = sgn == 0 ? ctv[dd] >= (real)0 : ctv[dd] < (real)0;
                const int dir = dd + 4 * sgn;
                const real nbt = slot[base + ((dir + (left ? sec : 8 - sec)) & 7)][lane];
                o[dd + 4 * sgn] = dir_new(sgn == 0 ? E + O : E - O, s, x, v, acr[dd], act[dd], nbr, nbt);
            }
        }
        if (store) {
#pragma unroll
            for (int dd = 0; dd < 4; ++dd) bstore2(o[dd], o[dd + 4], fout, vo, rb + (uint32_t)(4 * (k - 1) + dd) * pb);
        }
    }

    // (4) lambda: closed-form Cochran step, then upwind by own-cell u (the
    // azimuthal neighbour of the single column is the cell itself)
    const double uxd = (double)ux, uyd = (double)uy;
    const double urp = uxd * cs.x + uyd * cs.y;
    const double lreac = C.reacted(dp, lc);
    const double sll = from_left(lc), slr = from_right(lc);
    const double hll = lane_value(hlam, 0), hlr = lane_value(hlam, 1);
    const double llow = lane == 0 ? hll : sll;
    const double lup = lane == 63 ? hlr : slr;
    const double lr = urp >= 0.0 ? llow : lup;
    const double lnew = lreac - fabs(urp) * dp->dt_dr * (lc - lr);
    if (store) bstore(lnew, lout, vol, 0u);

    if (diag && store) diag_cell(red, (double)rho, uxd, uyd, Td, (double)e, lc, ri * dp->dr * dp->dth, dp->Q);
}

// Up to COL_K steps of a single-column solve in one launch (the
// quasi-one-dimensional runs of Sec. III, single solves): wavefront t holds
// rows r0 - COL_K .. r0 + 63 - COL_K, r0 = COL_W t, one per lane, and owns
// rows r0 .. r0 + COL_W - 1 (column_offsets).  Each step updates every lane
// from the lanes beside it (DPP shifts; lanes 0 and 63 read nothing from
// outside and go wrong), so a wrong value moves in by one lane per step:
// after k steps lanes k .. 63 - k still hold the true state, the owned lanes
// after all COL_K.  Rows outside the grid hold the radial ghosts of
// Sec. II.D: they are loaded from the boundary row and set from it again
// before every step (a zero-gradient copy; at the disc centre row 0 with
// directions turned by 4, lambda copied).  The azimuthal neighbours are the
// cell itself with directions turned by the sector, as in radial_block, and
// the arithmetic per cell is the same.  Drift partial sums of each recorded
// step come from the owned lanes' state at the start of that step.
// Packed launches as k_step's (tiles, bases, step_off, flips, flip): solve i
// takes steps bases[i] + step_off on, min(nk, its steps left) of them, from
// buffer (step + flip_i) & 1 into the other one.
template <typename real, bool TAUF>
__global__ __launch_bounds__(BLOCK, 1) void k_column(const SolveDesc *descs, const uint2 *tiles, int ntiles,
                                                     const int64_t *bases, int64_t step_off, const int *flips,
                                                     int flip, int nk_most)
{
    const int nb = gridDim.x;
    const int tg = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, nb) * (BLOCK / 64) + (threadIdx.x >> 6));
    if (tg >= ntiles) return;
    int solve = 0, t = tg;
    if (tiles) {
        const uint2 e = tiles[tg];
        solve = __builtin_amdgcn_readfirstlane((int)e.x);
        t = __builtin_amdgcn_readfirstlane((int)e.y);
    }
    const DescPtr dp = (DescPtr)(descs + solve);
    const int64_t step0 = (bases ? bases[solve] : 0) + step_off;
    if (step0 >= dp->nsteps) return;
    const int nk = (int)min((int64_t)nk_most, dp->nsteps - step0);
    __shared__ real slots[BLOCK / 64][NQ][64];
    real(*slot)[64] = slots[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int nr = dp->nr, sec = dp->sector;
    const int cur = (int)((step0 + ((flips ? flips[solve] : 0) ^ flip)) & 1);
    const __amdgpu_buffer_rsrc_t fin = rsrc_of(dp->f[cur]), fout = rsrc_of(dp->f[cur ^ 1]);
    const __amdgpu_buffer_rsrc_t lin = rsrc_of(dp->lam[cur]), lout = rsrc_of(dp->lam[cur ^ 1]);
    const RowBytes b = row_bytes_of(dp->rstride, dp->pitch, (int)sizeof(real));
    const ColumnOffsets o = column_offsets(nr, b, t, lane);
    const bool below = o.row < 0, above = o.row >= nr;
    const bool disc = dp->disc;
    // lanes of the first and the last row of the grid, where the wavefront holds them
    const int r_first = t * COL_W - COL_K;
    const int l_first = -r_first, l_last = nr - 1 - r_first;
    const bool has_below = r_first < 0, has_above = r_first + 63 >= nr;

    // the state at step0 (rows below the grid: row 0, its pairs' members
    // exchanged at the disc centre, which turns each direction by 4)
    real fc[NQ];
    double lc;
    bload(fc[0], fin, o.vo, 0u);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        real a, bb;
        bload2(a, bb, fin, o.vo, b.rest + (uint32_t)c * b.pair);
        const int q = 1 + 8 * (c >> 2) + (c & 3);
        const bool turn = below && disc;
        fc[q] = turn ? bb : a;
        fc[q + 4] = turn ? a : bb;
    }
    bload(lc, lin, o.vol, 0u);
    const real om = omega_at<real, TAUF>(dp, o.om, 0u);

    // polar components of directions dd = 0..3 at theta_0 (dd+4 is the negative)
    const double2 cs = dp->cs[0];
    const real cth = (real)cs.x, sth = (real)cs.y;
    const real crv[4] = {cth, (real)SQH * (cth + sth), sth, (real)SQH * (sth - cth)};
    const real ctv[4] = {-sth, (real)SQH * (cth - sth), cth, (real)SQH * (cth + sth)};
    const double ri = dp->r_min + ((double)o.re + 0.5) * dp->dr;
    const real kr = (real)dp->dt_dr, kt = (real)(dp->dt_dth / ri);
    real acr[4], act[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        acr[dd] = fabs(crv[dd]) * kr;
        act[dd] = fabs(ctv[dd]) * kt;
    }
    const double w_area = ri * dp->dr * dp->dth;

    for (int j = 0; j < nk; ++j) {
        const int64_t step = step0 + j;
        if (j > 0 && has_below) {
            // rows below the grid: the ghost of row 0 (lane l_first)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int qs = (q == 0 || !disc) ? q : 1 + 8 * ((q - 1) >> 3) + ((((q - 1) & 7) + 4) & 7);
                const real g = lane_value(fc[qs], l_first);
                fc[q] = below ? g : fc[q];
            }
            const double g = lane_value(lc, l_first);
            lc = below ? g : lc;
        }
        if (j > 0 && has_above) {
            // rows above the grid: the copy of row nr - 1 (lane l_last)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const real g = lane_value(fc[q], l_last);
                fc[q] = above ? g : fc[q];
            }
            const double g = lane_value(lc, l_last);
            lc = above ? g : lc;
        }

        const Cell<real> C(dp, fc, lc, om);
        if (records(dp, step)) {
            double red[5] = {0, 0, 0, 0, 0};
            if (o.own)
                diag_cell(red, (double)C.rho, (double)C.ux, (double)C.uy, C.Td, (double)C.e, lc, w_area, dp->Q);
            double v[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) v[i] = wave_sum(red[i]);
            double *part = dp->wpart + (((size_t)((step / dp->diag_every) % PART_RING)) * dp->nwaves + t) * 5;
            if (lane == 0)
#pragma unroll
                for (int i = 0; i < 5; ++i) part[i] = v[i];
        }

        // the cell's distributions, for its rotated azimuthal neighbours
#pragma unroll
        for (int q = 0; q < NQ; ++q) slot[q][lane] = fc[q];
        real fn[NQ];
        fn[0] = C.rest(fc[0]);
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            const real v = (real)speed(k);
            const real rF = C.rho * C.F[k];
            const real rA = rF * (C.keep + C.beta * (v * v + C.u2 - (real)2 * C.T)), rB = rF * C.Bz;
            const int base = 1 + 8 * (k - 1);
#pragma unroll
            for (int dd = 0; dd < 4; ++dd) {
                real E, O;
                pair_coll(C.EP, v * C.EP.w(dd), rA, rB, E, O);
                const real s = C.omega - v * (acr[dd] + act[dd]);
#pragma unroll
                for (int sgn = 0; sgn < 2; ++sgn) {
                    const int q = base + dd + 4 * sgn;
                    const real x = fc[q];
                    // radial upwind (C_r >= 0 takes the row below, lane - 1)
                    const real lower = from_left(x), upper = from_right(x);
                    const bool lo = sgn == 0 ? crv[dd] >= (real)0 : crv[dd] < (real)0;
                    const real nbr = lo ? lower : upper;
                    // azimuthal upwind: this cell, direction turned by +s or -s
                    const bool left = sgn == 0 ? ctv[dd] >= (real)0 : ctv[dd] < (real)0;
                    const int dir = dd + 4 * sgn;
                    const real nbt = slot[base + ((dir + (left ? sec : 8 - sec)) & 7)][lane];
                    fn[q] = dir_new(sgn == 0 ? E + O : E - O, s, x, v, acr[dd], act[dd], nbr, nbt);
                }
            }
        }
        // lambda: closed-form Cochran step, then upwind by own-cell u_r
        const double uxd = (double)C.ux, uyd = (double)C.uy;
        const double urp = uxd * cs.x + uyd * cs.y;
        const double lreac = C.reacted(dp, lc);
        const double llow = from_left(lc), lup = from_right(lc);
        const double lr = urp >= 0.0 ? llow : lup;
        lc = lreac - fabs(urp) * dp->dt_dr * (lc - lr);
#pragma unroll
        for (int q = 0; q < NQ; ++q) fc[q] = fn[q];
    }

    if (o.own) {
        bstore(fc[0], fout, o.vo, 0u);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int q = 1 + 8 * (c >> 2) + (c & 3);
            bstore2(fc[q], fc[q + 4], fout, o.vo, b.rest + (uint32_t)c * b.pair);
        }
        bstore(lc, lout, o.vol, 0u);
    }
}

// Occupancy: float32 rows fit two wavefronts per SIMD; float64 rows take
// the whole register file of one (the next row in flight is 66 VGPRs).
template <typename real>
struct StepOcc {
    static constexpr int waves = sizeof(real) == 4 ? 2 : 1;
};

// One time step of every solve of the launch.  Wavefront w of the grid takes
// tile t = (its block's XCD-ordered index) * 4 + w, which the tile table maps
// to (solve, tile of that solve); a solve's tile lt is row block lt / nstrip,
// strip lt % nstrip.  Each wavefront works on its own: no barriers and no
// atomics.  A drift-report step leaves per-wavefront partial sums in its
// slot of the solve's partial-sum ring; k_records adds them up later.
template <typename real, bool ROT, bool TAUF>
__global__ __launch_bounds__(BLOCK, StepOcc<real>::waves) void k_step(const SolveDesc *descs, const uint2 *tiles,
                                                                       int ntiles, const int64_t *bases,
                                                                       int64_t step_off, const int *flips,
                                                                       int flip)
{
    const int nb = gridDim.x;
    const int blk = xcd_tile(blockIdx.x, nb);
    // wave-uniform by construction; tell the compiler so that the row loop
    // and the offsets derived from it live in scalar registers
    const int t = __builtin_amdgcn_readfirstlane(blk * (BLOCK / 64) + (threadIdx.x >> 6));
    if (t >= ntiles) return;
    int solve = 0, lt = t;
    if (tiles) {
        const uint2 e = tiles[t];
        solve = __builtin_amdgcn_readfirstlane((int)e.x);
        lt = __builtin_amdgcn_readfirstlane((int)e.y);
    }
    const DescPtr dp = (DescPtr)(descs + solve);
    const int64_t step = (bases ? bases[solve] : 0) + step_off;
    if (step >= dp->nsteps) return;
    const bool diag = records(dp, step);
    const int cur = (int)((step + ((flips ? flips[solve] : 0) ^ flip)) & 1);
    const StepBufs bufs{dp->f[cur], dp->f[cur ^ 1], dp->lam[cur], dp->lam[cur ^ 1]};
    __shared__ real prev[BLOCK / 64][NQ][64];
    double red[5] = {0, 0, 0, 0, 0};
    // row-block major: the strips of one row block sit side by side in the
    // same XCD and share their halo columns in its L2; odd row blocks march
    // inward so that the rows bounding two blocks are read by both at once.
    if (dp->nt == 1) {
        // one theta column: lanes along r
        radial_block<real, TAUF>(dp, bufs, lt, prev[threadIdx.x >> 6], red, diag);
    } else {
        const int rows = dp->rows, nstrip = dp->nstrip;
        const int rb = lt / nstrip, strip = lt - rb * nstrip;
        const int i0 = rb * rows;
        const int i1 = min(i0 + rows, dp->nr);
        march<real, ROT, TAUF>(dp, bufs, strip, i0, i1, (rb & 1) != 0, prev[threadIdx.x >> 6], red, diag);
    }
    if (diag) {
        const int64_t slot = (step / dp->diag_every) % PART_RING;
        double *part = dp->wpart + ((size_t)slot * dp->nwaves + lt) * 5;
        double v[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] = wave_sum(red[i]);
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int i = 0; i < 5; ++i) part[i] = v[i];
    }
}

__global__ void k_advance(const SolveDesc *descs, int *flips, int64_t *bases, int n, int64_t by, int column_k)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (flips && column_k > 0) {
        // launches of up to column_k steps: one of nk steps toggles the
        // parity when nk is even
        int64_t left = max(descs[i].nsteps - bases[i], (int64_t)0);
        int f = flips[i];
        for (int64_t done = 0; done < by && left > 0;) {
            const int64_t nk = min(min((int64_t)column_k, by - done), left);
            f ^= (int)((nk + 1) & 1);
            left -= nk;
            done += min((int64_t)column_k, by - done);
        }
        flips[i] = f;
    } else if (flips) {
        // two-step launches of solve i in these `by` steps: min(left, by) / 2
        const int64_t left = max(descs[i].nsteps - bases[i], (int64_t)0);
        flips[i] ^= (int)((min(left, by) / 2) & 1);
    }
    bases[i] += by;
}

// Drift records of the steps [base + lo, base + hi) of each solve, where base
// is bases[solve] (0 without bases): block (solve, r) adds up the partial sums
// of the r-th record in that range, one wavefront, in a fixed order, so the
// record does not depend on the order in which wavefronts finished.
__global__ __launch_bounds__(64) void k_records(const SolveDesc *descs, const int64_t *bases, int64_t lo, int64_t hi)
{
    const DescPtr dp = (DescPtr)(descs + blockIdx.x);
    const int64_t de = dp->diag_every;
    if (de <= 0) return;
    const int64_t base = bases ? bases[blockIdx.x] : 0;
    const int64_t s0 = max(base + lo, dp->state->rec_from);
    const int64_t s1 = min(base + hi, dp->nsteps);
    const int64_t k = (s0 + de - 1) / de + blockIdx.y;  // record k is step k * de
    if (s0 >= s1 || k * de >= s1) return;
    const int lane = threadIdx.x;
    const double *part = dp->wpart + (size_t)(k % PART_RING) * dp->nwaves * 5;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int w = lane; w < dp->nwaves; w += 64)
#pragma unroll
        for (int i = 0; i < 5; ++i) acc[i] += part[5 * (size_t)w + i];
#pragma unroll
    for (int i = 0; i < 5; ++i) acc[i] = wave_sum(acc[i]);
    if (lane == 0) {
        pdbm_diag r;
        r.step = k * de;
        r.mass = acc[0];
        r.energy = acc[1];
        r.chem = acc[2];
        r.n_nonfinite = (int64_t)acc[3];
        r.n_nonphys = (int64_t)acc[4];
        dp->hist[k % HIST_CAP] = r;
    }
}

}  // namespace

int solve_waves(int nr, int nt, int rows)
{
    if (nt == 1) return (nr + COL_W - 1) / COL_W;  // lanes along r: COL_W rows per wavefront
    return (int)((int64_t)((nr + rows - 1) / rows) * ((nt + STRIP - 1) / STRIP));
}

template <typename real, bool ROT, bool TAUF>
static void launch_k_step(int nb, hipStream_t st, const SolveDesc *descs, const uint2 *tiles, int ntiles,
                          const int64_t *bases, int64_t step_off, const int *flips, int flip)
{
    hipLaunchKernelGGL((k_step<real, ROT, TAUF>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases, step_off,
                       flips, flip);
}

hipError_t launch_step(const SolveDesc *descs, const uint2 *tiles, int ntiles, const int64_t *bases, int64_t step_off,
                       const int *flips, int flip, bool fp32, bool rot, bool tauf, hipStream_t st)
{
    const int nb = (ntiles + BLOCK / 64 - 1) / (BLOCK / 64);
    if (nb == 0) return hipSuccess;
    using L = void (*)(int, hipStream_t, const SolveDesc *, const uint2 *, int, const int64_t *, int64_t, const int *,
                       int);
    // [fp32][rot][tauf]
    static const L table[2][2][2] = {
        {{launch_k_step<double, false, false>, launch_k_step<double, false, true>},
         {launch_k_step<double, true, false>, launch_k_step<double, true, true>}},
        {{launch_k_step<float, false, false>, launch_k_step<float, false, true>},
         {launch_k_step<float, true, false>, launch_k_step<float, true, true>}}};
    table[fp32][rot][tauf](nb, st, descs, tiles, ntiles, bases, step_off, flips, flip);
    return hipGetLastError();
}

hipError_t launch_column(const SolveDesc *descs, const uint2 *tiles, int ntiles, const int64_t *bases,
                         int64_t step_off, const int *flips, int flip, int nk, bool fp32, bool tauf, hipStream_t st)
{
    const int nb = (ntiles + BLOCK / 64 - 1) / (BLOCK / 64);
    if (nb == 0 || nk <= 0) return hipSuccess;
    if (fp32) {
        if (tauf)
            hipLaunchKernelGGL((k_column<float, true>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases,
                               step_off, flips, flip, nk);
        else
            hipLaunchKernelGGL((k_column<float, false>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases,
                               step_off, flips, flip, nk);
    } else {
        if (tauf)
            hipLaunchKernelGGL((k_column<double, true>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases,
                               step_off, flips, flip, nk);
        else
            hipLaunchKernelGGL((k_column<double, false>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases,
                               step_off, flips, flip, nk);
    }
    return hipGetLastError();
}

hipError_t launch_advance(const SolveDesc *descs, int *flips, int64_t *bases, int n, int64_t by, int column_k,
                          hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_advance, dim3((n + 255) / 256), dim3(256), 0, st, descs, flips, bases, n, by, column_k);
    return hipGetLastError();
}

hipError_t launch_records(const SolveDesc *descs, int n, const int64_t *bases, int64_t lo, int64_t hi, hipStream_t st)
{
    if (n <= 0 || hi <= lo) return hipSuccess;
    const int nrec = (int)std::min<int64_t>(hi - lo, PART_RING);
    hipLaunchKernelGGL(k_records, dim3(n, nrec), dim3(64), 0, st, descs, bases, lo, hi);
    return hipGetLastError();
}

}  // namespace pdbm
