// HIP kernels of libpdbm for gfx950 (MI355X).
//
// One cell per lane.  Within an r row, f holds the rest particle's plane and
// the 16 pairs of opposite directions interleaved per column (elem_of), so
// that a wavefront of 64 consecutive theta cells reads one contiguous block
// per plane or pair, one 8- or 16-byte access per lane for a pair.
// The collision is evaluated in the Cartesian frame: f^eq depends on v.u and
// |u|^2 only, which are the same in polar and Cartesian components, so the
// 33 velocities are compile-time constants (speeds 0, 1.5, 3.5, 7.5, 12.5 of
// Sec. II.B, directions i*pi/4 fixed in the Cartesian frame).  Polar
// components are needed only for the Courant numbers and for u_r, u_theta.
#include <math.h>

#include "pdbm_internal.h"

namespace pdbm {
namespace {

constexpr double SQH = 0.70710678118654752440;  // cos(pi/4) = sin(pi/4)

__device__ __forceinline__ constexpr double speed(int k)
{
    return k == 1 ? 1.5 : k == 2 ? 3.5 : k == 3 ? 7.5 : 12.5;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Renumber them so that each XCD walks one contiguous range of
// tiles: neighbouring rows of the stencil then meet in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb)
{
    const int q = nb / NXCD, r = nb % NXCD;
    const int x = bid % NXCD, s = bid / NXCD;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

__device__ __forceinline__ double ipow(double x, int e)
{
    double y = 1.0;
    for (int i = 0; i < e; ++i) y *= x;
    return y;
}

// F_k(T), k = 0..4, from the moment-inversion matrix (Horner in T, float64).
template <typename real>
__device__ __forceinline__ void weights(const double *A, double T, real F[5])
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = T * (A[4 * k] + T * (A[4 * k + 1] + T * (A[4 * k + 2] + T * A[4 * k + 3])));
        F[k + 1] = (real)v;
        s += v;
    }
    F[0] = (real)(1.0 - 8.0 * s);
}

// rho, rho*u (Cartesian), and e = sum f |v|^2 / 2 of one cell.
template <typename real>
__device__ __forceinline__ void raw_moments(const real f[NQ], real &rho, real &jx, real &jy, real &e)
{
    rho = f[0];
    jx = 0;
    jy = 0;
    e = 0;
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
        const real *g = f + 1 + 8 * (k - 1);
        const real v = (real)speed(k);
        const real ring = ((g[0] + g[4]) + (g[2] + g[6])) + ((g[1] + g[5]) + (g[3] + g[7]));
        const real a15 = g[1] - g[5], a37 = g[3] - g[7];
        const real X = (g[0] - g[4]) + (real)SQH * (a15 - a37);
        const real Y = (g[2] - g[6]) + (real)SQH * (a15 + a37);
        rho += ring;
        jx += v * X;
        jy += v * Y;
        e += (real)(0.5 * speed(k) * speed(k)) * ring;
    }
}

// Coefficients of the f^eq polynomial in z = v.u / T (Sec. II.B):
// P(z) = (1 - a + a^2/2) + z (1 - a) + z^2 (1 - a)/2 + z^3/6 + z^4/24, a = u^2/(2T)
template <typename real>
struct EqPoly {
    real c0, c1, c2, wx, wy;
    EqPoly() = default;
    __device__ __forceinline__ EqPoly(real ux, real uy, real u2, real T)
    {
        const real iT = (real)1 / T;
        const real a = (real)0.5 * u2 * iT;
        c0 = (real)1 - a + (real)0.5 * a * a;
        c1 = (real)1 - a;
        c2 = (real)0.5 * c1;
        wx = ux * iT;
        wy = uy * iT;
    }
    // projection of direction d (0..3) on u, divided by T; d+4 is its negative
    __device__ __forceinline__ real w(int d) const
    {
        return d == 0 ? wx : d == 1 ? (real)SQH * (wx + wy) : d == 2 ? wy : (real)SQH * (wy - wx);
    }
    // P(z) and P(-z) from the even and odd parts
    __device__ __forceinline__ void eval(real z, real &pp, real &pm) const
    {
        const real z2 = z * z;
        const real ev = c0 + z2 * (c2 + z2 * (real)(1.0 / 24.0));
        const real od = z * (c1 + z2 * (real)(1.0 / 6.0));
        pp = ev + od;
        pm = ev - od;
    }
};

template <typename real>
__device__ __forceinline__ void equilibrium(const double *A, real rho, real ux, real uy, real T, real f[NQ])
{
    real F[5];
    weights(A, (double)T, F);
    const real u2 = ux * ux + uy * uy;
    const EqPoly<real> P(ux, uy, u2, T);
    f[0] = rho * F[0] * P.c0;
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
        const real rF = rho * F[k];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            real pp, pm;
            P.eval((real)speed(k) * P.w(d), pp, pm);
            f[1 + 8 * (k - 1) + d] = rF * pp;
            f[1 + 8 * (k - 1) + d + 4] = rF * pm;
        }
    }
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Sums v[0..4] over the workgroup; the result is valid in thread 0.
__device__ __forceinline__ void block_sum5(double v[5])
{
    __shared__ double lds[BLOCK / 64][5];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 5; ++i) v[i] = wave_sum(v[i]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) lds[w][i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            double s = lds[0][i];
            for (int j = 1; j < BLOCK / 64; ++j) s += lds[j][i];
            v[i] = s;
        }
}

// Per-block partial sums, then the last block to finish adds the partials in
// a fixed order (deterministic, no floating-point atomics) and writes the
// record.  Must be reached by every thread of every block.
__device__ void diag_reduce(const DiagCtl &dc, double v[5], int tile, int nb)
{
    __shared__ int last;
    block_sum5(v);
    if (threadIdx.x == 0) {
        double *p = dc.partials + 5 * (size_t)tile;
#pragma unroll
        for (int i = 0; i < 5; ++i) p[i] = v[i];
        __threadfence();
        const unsigned done = atomicAdd(dc.counter, 1u);
        last = done == (unsigned)(nb - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += BLOCK)
#pragma unroll
        for (int i = 0; i < 5; ++i)
            acc[i] += __hip_atomic_load(dc.partials + 5 * (size_t)b + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    block_sum5(acc);
    if (threadIdx.x == 0) {
        pdbm_diag r;
        r.step = dc.step;
        r.mass = acc[0];
        r.energy = acc[1];
        r.chem = acc[2];
        r.n_nonfinite = (int64_t)acc[3];
        r.n_nonphys = (int64_t)acc[4];
        *dc.out = r;
        __hip_atomic_store(dc.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Contribution of one cell to the drift report.
__device__ __forceinline__ void diag_cell(double v[5], double rho, double ux, double uy, double T, double e, double lam,
                                          double w, double Q)
{
    const bool finite = isfinite(rho) && isfinite(T) && isfinite(ux) && isfinite(uy) && isfinite(lam);
    if (!finite) {
        v[3] += 1.0;
        return;
    }
    if (rho <= 0.0 || T <= 0.0) v[4] += 1.0;
    v[0] += rho * w;
    v[1] += e * w;
    v[2] += rho * Q * (1.0 - lam) * w;
}

// ------------------------------------------------------------------ step --
// Cross-lane moves within a wavefront (DPP wave shifts): the value held by
// lane-1 (from_left) and by lane+1 (from_right).  Lanes 0 / 63 receive 0 and
// take their neighbours from the halo gathers instead.  Call these only where
// every lane of the wavefront is active (never inside a divergent branch).
// bound_ctrl set: the lane shifted in from outside the wavefront reads 0, so
// the instruction needs no prior value of its destination.
__device__ __forceinline__ int dpp_shr1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_shl1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_shr1(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_shl1(__float_as_int(v))); }
__device__ __forceinline__ double from_left(double v)
{
    return __hiloint2double(dpp_shr1(__double2hiint(v)), dpp_shr1(__double2loint(v)));
}
__device__ __forceinline__ double from_right(double v)
{
    return __hiloint2double(dpp_shl1(__double2hiint(v)), dpp_shl1(__double2loint(v)));
}

// The same shifts with the value lane 0 (from_left_or) or lane 63
// (from_right_or) receives from outside the wavefront given as `edge`
// (bound_ctrl clear: a lane without a source lane keeps the old value).
__device__ __forceinline__ int dpp_shr1_or(int edge, int v)
{
    return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_shl1_or(int edge, int v)
{
    return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ float from_left_or(float edge, float v)
{
    return __int_as_float(dpp_shr1_or(__float_as_int(edge), __float_as_int(v)));
}
__device__ __forceinline__ float from_right_or(float edge, float v)
{
    return __int_as_float(dpp_shl1_or(__float_as_int(edge), __float_as_int(v)));
}
__device__ __forceinline__ double from_left_or(double edge, double v)
{
    return __hiloint2double(dpp_shr1_or(__double2hiint(edge), __double2hiint(v)),
                            dpp_shr1_or(__double2loint(edge), __double2loint(v)));
}
__device__ __forceinline__ double from_right_or(double edge, double v)
{
    return __hiloint2double(dpp_shl1_or(__double2hiint(edge), __double2hiint(v)),
                            dpp_shl1_or(__double2loint(edge), __double2loint(v)));
}

// The step kernel reads the solve description through the constant address
// space: it is never written while a step runs, so the loads are scalar.  The
// kernel parameter stays a plain pointer (host and device must see the same
// kernel signature) and is cast inside device code.
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) SolveDesc *DescPtr;
#else
typedef const SolveDesc *DescPtr;
#endif

// The two f and lambda buffers of one step (they swap every step).
struct StepBufs {
    const void *f_in;
    void *f_out;
    const double *lam_in;
    double *lam_out;
};

// Raw buffer access to the f and lambda arrays: the lane's column offset is a
// loop-invariant VGPR, the row and velocity-plane offsets a scalar register
// (arrays stay below 4 GiB, which create() checks).
typedef int i32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void *p)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)0xFFFFFFFF, 0x00020000);
}
__device__ __forceinline__ void bload(float &v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    v = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ __forceinline__ void bload(double &v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    const i32x2 t = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
    v = __hiloint2double(t.y, t.x);
}
// Stores are non-temporal (cache policy nt): the new state is not read again
// in this step, and keeping it out of the caches leaves them to the lines
// the adjacent strips and row blocks read twice (halo columns, block
// boundary rows).
constexpr int STORE_NT = 2;
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, vo, so, STORE_NT);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    i32x2 t;
    t.x = __double2loint(v);
    t.y = __double2hiint(v);
    __builtin_amdgcn_raw_buffer_store_b64(t, r, vo, so, STORE_NT);
}
// Both members of a pair of opposite directions (see elem_of): one 8-byte
// (float32) or 16-byte (float64) access per lane.
typedef int i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void bload2(float &a, float &b, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    const i32x2 t = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
    a = __int_as_float(t.x);
    b = __int_as_float(t.y);
}
__device__ __forceinline__ void bload2(double &a, double &b, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    const i32x4 t = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0);
    a = __hiloint2double(t.y, t.x);
    b = __hiloint2double(t.w, t.z);
}
__device__ __forceinline__ void bstore2(float a, float b, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    i32x2 t;
    t.x = __float_as_int(a);
    t.y = __float_as_int(b);
    __builtin_amdgcn_raw_buffer_store_b64(t, r, vo, so, STORE_NT);
}
__device__ __forceinline__ void bstore2(double a, double b, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so)
{
    i32x4 t;
    t.x = __double2loint(a);
    t.y = __double2hiint(a);
    t.z = __double2loint(b);
    t.w = __double2hiint(b);
    __builtin_amdgcn_raw_buffer_store_b128(t, r, vo, so, STORE_NT);
}

// Keeps a scalar offset opaque to the optimiser, so that the 33 plane offsets
// are re-derived by one scalar add each instead of being hoisted out of the
// row loop (where they would not fit in scalar registers).
__device__ __forceinline__ uint32_t opaque(uint32_t x)
{
    asm volatile("" : "+s"(x));
    return x;
}

// A wavefront owns a strip of 64 consecutive theta columns, one per lane, and
// marches outward (or inward) over a block of rows.  The row being computed
// and the next two in marching order are held in registers, the row behind
// in a lane-private LDS slot: radial neighbours come from there, azimuthal
// ones from the adjacent lanes, so each f value is read from memory once per
// step (plus the two rows bounding the block).  The azimuthal neighbours of
// lanes 0 and 63 (the halo columns, owned by the adjacent strips) come from
// three gathered loads per row, lane q of which fetches one (plane, side)
// pair, and are moved into lane 0 or 63 by readlane.  Strips start on
// 64-column boundaries and rows are padded to a multiple of 64, so every
// store of a plane or pair covers whole cache lines; lanes past the last
// column own a padding column.  The second row ahead is requested a whole row
// of compute before it is first needed.
template <typename real, bool ROT>
struct Strip {
    DescPtr dp;
    __amdgpu_buffer_rsrc_t fin, fout, lin, lout;
    uint32_t vo, vo2, vol;   // byte offsets of this lane's column: rest plane, pair, lambda
    uint32_t vos, vos2, vols;  // ... of the lane's own column (the padding for periodic images)
    uint32_t vh1, vh2, vhl;  // byte offsets of this lane's halo gathers (plane and column)
    uint32_t row_bytes, lrow_bytes, rest_bytes, pair_bytes;
    uint32_t poff[4];     // rotated sectors: byte offset of the pair holding this lane's directions dd, dd + 4
    bool pswap[4];        // ... and whether its members come in the other order
    int lane, pc, rot;    // physical column, direction shift of this lane's data
    bool useful;

    // memory plane of velocity q for data whose direction index is shifted by r
    static __device__ __forceinline__ int plane_of(int q, int r)
    {
        return q == 0 ? 0 : 1 + 8 * ((q - 1) / 8) + ((((q - 1) % 8) + r) & 7);
    }

    __device__ __forceinline__ Strip(DescPtr dp_, const StepBufs &b, int strip) : dp(dp_)
    {
        fin = rsrc_of(b.f_in);
        fout = rsrc_of(b.f_out);
        lin = rsrc_of(b.lam_in);
        lout = rsrc_of(b.lam_out);
        const int nt = dp->nt, sec = dp->sector;
        lane = threadIdx.x & 63;
        const int c0 = strip * STRIP;
        const int col = c0 + lane;
        // lanes past the last column hold periodic images of the first ones
        const int wraps = col / nt;
        pc = col - wraps * nt;
        rot = ROT ? ((-wraps * sec) & 7) : 0;
        useful = col < nt;
        vo = (uint32_t)pc * (uint32_t)sizeof(real);
        vo2 = 2u * vo;
        vol = (uint32_t)pc * 8u;
        vos = (uint32_t)col * (uint32_t)sizeof(real);
        vos2 = 2u * vos;
        vols = (uint32_t)col * 8u;
        row_bytes = (uint32_t)dp->rstride * (uint32_t)sizeof(real);
        lrow_bytes = (uint32_t)dp->pitch * 8u;
        rest_bytes = (uint32_t)dp->plane * (uint32_t)sizeof(real);
        pair_bytes = 2u * rest_bytes;
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            // direction dd of this lane's data is direction (dd + rot) % 8
            poff[dd] = vo2 + rest_bytes + (uint32_t)((dd + rot) & 3) * pair_bytes;
            pswap[dd] = ((dd + rot) & 4) != 0;
        }
        // halo columns: c0 - 1 (0 <= c0 < nt) and c0 + 64, as periodic images
        const int cl = c0 == 0 ? nt - 1 : c0 - 1;
        const int rl = ROT && c0 == 0 ? (sec & 7) : 0;
        const int wr = (c0 + STRIP) / nt;
        const int cr = c0 + STRIP - wr * nt;
        const int rr = ROT ? ((-wr * sec) & 7) : 0;
        // gather 1: lanes 0..32 left halo of planes 0..32, lanes 33..63 right
        // halo of planes 0..30; gather 2: lanes 0, 1 right halo of planes 31,
        // 32; lambda gather: lane 0 left, lane 1 right (other lanes repeat a
        // valid address)
        const int es = (int)sizeof(real);
        const int64_t pt = dp->pitch;
        vh1 = lane <= 32 ? (uint32_t)elem_of(plane_of(lane, rl), cl, pt) * es
                         : (uint32_t)elem_of(plane_of(lane - 33, rr), cr, pt) * es;
        vh2 = lane < 2 ? (uint32_t)elem_of(plane_of(31 + lane, rr), cr, pt) * es : (uint32_t)cl * es;
        vhl = lane == 1 ? (uint32_t)cr * 8u : (uint32_t)cl * 8u;
    }

    __device__ __forceinline__ void load_row(int row, real f[NQ], double &lam) const
    {
        uint32_t so = (uint32_t)row * row_bytes;
        bload(f[0], fin, vo, so);
        if (ROT) {
            // this lane's data of direction dir lives in direction (dir + rot) % 8
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t sk = so + (uint32_t)k * 4u * pair_bytes;
#pragma unroll
                for (int dd = 0; dd < 4; ++dd) {
                    real a, b;
                    bload2(a, b, fin, poff[dd], sk);
                    f[1 + 8 * k + dd] = pswap[dd] ? b : a;
                    f[5 + 8 * k + dd] = pswap[dd] ? a : b;
                }
            }
        } else {
            so = opaque(so + rest_bytes);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                bload2(f[1 + 8 * (c >> 2) + (c & 3)], f[5 + 8 * (c >> 2) + (c & 3)], fin, vo2, so);
                so = opaque(so + pair_bytes);
            }
        }
        bload(lam, lin, vol, (uint32_t)row * lrow_bytes);
    }

    // The halo values of row `row`: h[0], h[1] for f, h[2] for lambda.
    __device__ __forceinline__ void load_halo(int row, real h[2], double &hl) const
    {
        const uint32_t so = (uint32_t)row * row_bytes;
        bload(h[0], fin, vh1, so);
        bload(h[1], fin, vh2, so);
        bload(hl, lin, vhl, (uint32_t)row * lrow_bytes);
    }
};

// Wave-uniform copy of lane l of v.
__device__ __forceinline__ float lane_value(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
// Halo of plane q from the two f gathers: left neighbour of lane 0, right
// neighbour of lane 63.
template <typename real>
__device__ __forceinline__ real halo_left(const real h[2], int q)
{
    return lane_value(h[0], q);
}
template <typename real>
__device__ __forceinline__ real halo_right(const real h[2], int q)
{
    return q <= 30 ? lane_value(h[0], 33 + q) : lane_value(h[1], q - 31);
}

// Per-cell quantities of one update (Sec. II.B-C): moments, F_k(T), the f^eq
// polynomial and the BGK / chemical factors (the Cochran rate gated by the
// ignition temperature, in float64; M dt = f^eq beta (|v - u|^2 - 2T) with
// beta = Q R dt / (2 T^2), D = 2).
template <typename real>
struct Cell {
    real rho, e, ux, uy, u2, T, beta, omega, keep, Bz;
    double Td, a, b;
    bool on;
    real F[5];
    EqPoly<real> EP;

    Cell() = default;
    __device__ __forceinline__ Cell(DescPtr dp, const real x[NQ], double lc)
    {
        real jx, jy;
        raw_moments(x, rho, jx, jy, e);
        init_moments(dp, jx, jy, lc);
    }
    // from rho, e (members) and the momentum jx, jy
    __device__ __forceinline__ void init_moments(DescPtr dp, real jx, real jy, double lc)
    {
        const real irho = (real)1 / rho;
        ux = jx * irho;
        uy = jy * irho;
        u2 = ux * ux + uy * uy;
        T = e * irho - (real)0.5 * u2;
        Td = (double)T;
        weights(dp->A, Td, F);
        EP = EqPoly<real>(ux, uy, u2, T);
        a = 0.0;
        b = 0.0;
        double R = 0.0;
        on = dp->reacts && Td > dp->T_th;
        if (on) {
            const double p = (double)rho * Td;
            a = dp->w1 * ipow(p, dp->m);
            b = dp->w2 * ipow(p, dp->n);
            R = (1.0 - lc) * (a + b * lc);
        }
        beta = (real)(dp->Q * R * dp->dt / (2.0 * Td * Td));
        omega = (real)dp->omega;
        keep = (real)1 - omega;
        Bz = (real)-2 * beta * T;
    }
    // the rest particle after collision (it does not stream)
    __device__ __forceinline__ real rest(real x0) const
    {
        return rho * F[0] * EP.c0 * (keep + beta * (u2 - (real)2 * T)) + omega * x0;
    }
    // lambda after the closed-form Cochran step
    __device__ __forceinline__ double reacted(DescPtr dp, double lc) const
    {
        if (on && a + b > 0.0) {
            const double q1 = (1.0 - lc) * exp(-(a + b) * dp->dt);
            return 1.0 - (a + b) * q1 / ((a + b * lc) + b * q1);
        }
        return lc;
    }
};

// One row of one strip: moments, F_k(T), f^eq, BGK + chemical term, Cochran
// lambda, donor-cell fluxes of f and lambda.  fc: row i.  Marching outward
// (down = false): prev (LDS, this lane's column) holds row i-1 and fn row
// i+1; marching inward the roles swap.  prev is replaced by row i as it is
// consumed.  mr[dd] / mt[dd]: which side is upwind for direction dd (its
// opposite dd+4 takes the other side).
template <typename real, bool ROT>
__device__ __forceinline__ void update_row(const Strip<real, ROT> &S, int ir, real (*prev)[64], const real fc[NQ],
                                           const real fn[NQ], const real hf[2], double hlam, double lbehind,
                                           double lc, double lahead,
                                           const bool mr[4], const bool mt[4], const real acr[4], const real ctv[4],
                                           bool lr_behind, double csx, double csy, double red[5], bool diag)
{
    const DescPtr dp = S.dp;
    // (1)-(3) moments, weights, f^eq polynomial, BGK and chemical factors
    const Cell<real> C(dp, fc, lc);
    const real rho = C.rho, e = C.e, ux = C.ux, uy = C.uy, u2 = C.u2, T = C.T;
    const real beta = C.beta, omega = C.omega, keep = C.keep, Bz = C.Bz;
    const double Td = C.Td;
    const real *F = C.F;
    const EqPoly<real> &EP = C.EP;

    // azimuthal Courant magnitudes of this row (the geometric 1/r term)
    const double ri = dp->r_min + ((double)ir + 0.5) * dp->dr;
    const real kt = (real)(dp->dt_dth / ri);
    real act[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) act[dd] = fabs(ctv[dd]) * kt;

    const bool store = S.useful;
    const int lane = S.lane;
    // pair c of this row sits at rowoff + rest plane + c * pb (pb re-derived
    // per row so the 16 products stay scalar arithmetic inside the loop)
    const uint32_t rowoff = (uint32_t)ir * S.row_bytes;
    const uint32_t pb = opaque(S.pair_bytes);
    const uint32_t pairs = rowoff + S.rest_bytes;

    // rest particle: no streaming
    // every lane stores, periodic images into their own column of the row
    // padding (see stage_row)
    const real rest = rho * F[0] * EP.c0 * (keep + beta * (u2 - (real)2 * T)) + omega * fc[0];
    bstore(rest, S.fout, S.vos, rowoff);

#pragma unroll
    for (int k = 1; k <= 4; ++k) {
        const real v = (real)speed(k);
        const real rF = rho * F[k];
        const real Ak = keep + beta * (v * v + u2 - (real)2 * T);
        const int base = 1 + 8 * (k - 1);
        // the ring's new values, stored together under one lane mask (in
        // halves where the rotated sector's per-lane plane offsets already
        // hold registers)
        constexpr int G = ROT ? 2 : 4;  // directions dd per store group
        real o[8];
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            const real z = v * EP.w(dd);
            real pp, pm;
            EP.eval(z, pp, pm);
            const real bz = Bz * z;
#pragma unroll
            for (int sgn = 0; sgn < 2; ++sgn) {
                const int q = base + dd + 4 * sgn;
                const real x = fc[q];
                const real coll = sgn == 0 ? rF * pp * (Ak + bz) + omega * x : rF * pm * (Ak - bz) + omega * x;
                // upwind neighbours: C >= 0 takes the lower one (Sec. II.C)
                const real behind = prev[q][lane];
                prev[q][lane] = x;
                const bool rb = sgn == 0 ? mr[dd] : !mr[dd];
                const real nbr = rb ? behind : fn[q];
                // both shifts and both halo values are taken by every lane
                // (a DPP read of a lane switched off by a branch would return
                // 0), then selected; lanes 0 and 63 take the halo columns
                const real sl = from_left(x), sr = from_right(x);
                const real hl = halo_left(hf, q), hr = halo_right(hf, q);
                const real left = lane == 0 ? hl : sl;
                const real right = lane == 63 ? hr : sr;
                const bool tl = sgn == 0 ? mt[dd] : !mt[dd];
                const real nbt = tl ? left : right;
                o[dd + 4 * sgn] = coll - v * (acr[dd] * (x - nbr) + act[dd] * (x - nbt));
            }
            // lanes holding rotated sector images store into the padding
            // too (their values are never read)
            if (dd % G == G - 1) {
#pragma unroll
                for (int e = dd + 1 - G; e <= dd; ++e)
                    bstore2(o[e], o[e + 4], S.fout, S.vos2, pairs + (uint32_t)(4 * (k - 1) + e) * pb);
            }
        }
    }

    // (4) lambda: closed-form Cochran step, then upwind by own-cell u
    const double uxd = (double)ux, uyd = (double)uy;
    const double urp = uxd * csx + uyd * csy;
    const double utp = -uxd * csy + uyd * csx;
    const double lreac = C.reacted(dp, lc);
    const double sll = from_left(lc), slr = from_right(lc);
    const double hll = lane_value(hlam, 0), hlr = lane_value(hlam, 1);
    const double lleft = lane == 0 ? hll : sll;
    const double lright = lane == 63 ? hlr : slr;
    const double lr = (urp >= 0.0) == lr_behind ? lbehind : lahead;
    const double lt = utp >= 0.0 ? lleft : lright;
    const double lnew = lreac - fabs(urp) * dp->dt_dr * (lc - lr) - fabs(utp) * (dp->dt_dth / ri) * (lc - lt);
    bstore(lnew, S.lout, S.vols, (uint32_t)ir * S.lrow_bytes);

    if (diag && store) diag_cell(red, (double)rho, uxd, uyd, Td, (double)e, lc, ri * dp->dr * dp->dth, dp->Q);
}

// Row `row` of the strip into f, or a ghost row outside [0, nr): below r_min
// the zero-gradient copy of row 0 or the disc-centre rule f(-1, j, k, i) =
// f(0, j, k, (i+4)%8) (Sec. II.D); above r_max the zero-gradient copy of row
// nr-1.  `edge` holds the boundary row the ghost copies.
template <typename real, bool ROT>
__device__ __forceinline__ void row_or_ghost(const Strip<real, ROT> &S, int row, real f[NQ], double &lam,
                                             const real edge[NQ], double ledge)
{
    if (row >= 0 && row < S.dp->nr) {
        S.load_row(row, f, lam);
        return;
    }
    const bool disc = row < 0 && S.dp->disc;
    f[0] = edge[0];
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        const int base = 1 + 8 * ((q - 1) / 8), dir = (q - 1) % 8;
        f[q] = disc ? edge[base + ((dir + 4) & 7)] : edge[q];
    }
    lam = ledge;
}

// Work of one wavefront: strip `strip`, rows [i0, i1), marched outward or,
// with `down`, inward.  prev: this wavefront's [NQ][64] LDS slots.
template <typename real, bool ROT>
__device__ __forceinline__ void march(DescPtr dp, const StepBufs &bufs, int strip, int i0, int i1, bool down,
                                      real (*prev)[64], double red[5], bool diag)
{
    const Strip<real, ROT> S(dp, bufs, strip);
    const int lane = S.lane;
    const double2 cs = dp->cs[S.pc];
    const real cth = (real)cs.x, sth = (real)cs.y;
    // polar components of directions dd = 0..3 at theta_j (dd+4 is the negative):
    // v_r = v (cos(dd pi/4) cos th + sin(dd pi/4) sin th),
    // v_theta = v (sin(dd pi/4) cos th - cos(dd pi/4) sin th)
    const real crv[4] = {cth, (real)SQH * (cth + sth), sth, (real)SQH * (sth - cth)};
    const real ctv[4] = {-sth, (real)SQH * (cth - sth), cth, (real)SQH * (cth + sth)};
    const real kr = (real)dp->dt_dr;
    real acr[4];
    bool mr[4], mt[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        acr[dd] = fabs(crv[dd]) * kr;
        mr[dd] = (crv[dd] >= (real)0) != down;  // true: the upwind radial neighbour is the row behind
        mt[dd] = ctv[dd] >= (real)0;            // true: the upwind azimuthal neighbour is lane-1
    }
    const int step = down ? -1 : 1;
    const int first = down ? i1 - 1 : i0;
    const int count = i1 - i0;
    // halos of a row are gathered right after its main loads, when the
    // adjacent strips fetch the same lines (they then hit in L2)
    real fc[NQ], fn[NQ], fnn[NQ], hc[2], hn[2], hnn[2];
    double lp, lc, ln, lnn, hlc, hln, hlnn;
    S.load_row(first, fc, lc);
    S.load_halo(first, hc, hlc);
    row_or_ghost(S, first + step, fn, ln, fc, lc);
    if (count > 1) S.load_halo(first + step, hn, hln);
    row_or_ghost(S, first - step, fnn, lp, fc, lc);  // the row behind the first
#pragma unroll
    for (int q = 0; q < NQ; ++q) prev[q][lane] = fnn[q];
    int ir = first;
    for (int n = 0; n < count; ++n, ir += step) {
        // the second row ahead is the radial neighbour of the next row
        // computed, if there is one; rows computed are never ghosts
        if (n + 1 < count) row_or_ghost(S, ir + 2 * step, fnn, lnn, fn, ln);
        if (n + 2 < count) S.load_halo(ir + 2 * step, hnn, hlnn);
        update_row<real, ROT>(S, ir, prev, fc, fn, hc, hlc, lp, lc, ln, mr, mt, acr, ctv, !down, cs.x, cs.y, red,
                              diag);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            fc[q] = fn[q];
            fn[q] = fnn[q];
        }
        hc[0] = hn[0];
        hc[1] = hn[1];
        hlc = hln;
        hn[0] = hnn[0];
        hn[1] = hnn[1];
        hln = hlnn;
        lp = lc;
        lc = ln;
        ln = lnn;
        // Compiler-only barrier: the LDS slots must not be promoted to
        // registers across iterations (they exist to free those registers).
        asm volatile("" ::: "memory");
    }
}

// Memory plane of velocity q whose direction index is shifted by r.
__device__ __forceinline__ int shifted_plane(int q, int r)
{
    return q == 0 ? 0 : 1 + 8 * ((q - 1) / 8) + ((((q - 1) % 8) + r) & 7);
}

// One step of 64 consecutive rows of a solve with a single theta column
// (ntheta = 1, the quasi-one-dimensional runs of Sec. III): lane l owns row
// 64 blk + l.  Radial neighbours come from the adjacent lanes (DPP shifts)
// and, for lanes 0 and 63, from gathers of the rows below and above the
// block, which apply the radial ghost rules of Sec. II.D.  The azimuthal
// neighbours of a cell are the cell itself with directions turned by the
// sector (periodic halo, f_{k,i}(j-1) = f_{k,(i+s)%8}(j) and f_{k,i}(j+1) =
// f_{k,(i-s)%8}(j)); they are read back from the wavefront's LDS slot.
// The arithmetic per cell is that of update_row.
template <typename real>
__device__ __forceinline__ void radial_block(DescPtr dp, const StepBufs &bufs, int blk, real (*slot)[64],
                                             double red[5], bool diag)
{
    const int lane = threadIdx.x & 63;
    const int nr = dp->nr, sec = dp->sector;
    const int r0 = blk * 64;
    const int row = r0 + lane;
    const int re = min(row, nr - 1);  // lanes past the last row hold its zero-gradient image
    const bool store = row < nr;
    const __amdgpu_buffer_rsrc_t fin = rsrc_of(bufs.f_in), fout = rsrc_of(bufs.f_out);
    const __amdgpu_buffer_rsrc_t lin = rsrc_of(bufs.lam_in), lout = rsrc_of(bufs.lam_out);
    const uint32_t es = (uint32_t)sizeof(real);
    const uint32_t rowb = (uint32_t)dp->rstride * es;
    const uint32_t rb = (uint32_t)dp->plane * es, pb = 2u * rb;  // rest plane, one pair (column 0)
    const int64_t pt = dp->pitch;
    const uint32_t lrowb = (uint32_t)dp->pitch * 8u;
    const uint32_t vo = (uint32_t)re * rowb, vol = (uint32_t)re * lrowb;

    real fc[NQ];
    double lc;
    bload(fc[0], fin, vo, 0u);
#pragma unroll
    for (int c = 0; c < 16; ++c)
        bload2(fc[1 + 8 * (c >> 2) + (c & 3)], fc[5 + 8 * (c >> 2) + (c & 3)], fin, vo, rb + (uint32_t)c * pb);
    bload(lc, lin, vol, 0u);
    // gathers of the row below the block (ghost of row 0 at r_min: a copy,
    // or at the disc centre row 0 with directions turned by 4) and of the
    // row above it (clamped: the zero-gradient copy of the last row)
    const int rlo = r0 == 0 ? 0 : r0 - 1;
    const int tlo = r0 == 0 && dp->disc ? 4 : 0;
    const int rhi = min(r0 + 64, nr - 1);
    const uint32_t vh1 = lane <= 32 ? (uint32_t)rlo * rowb + (uint32_t)elem_of(shifted_plane(lane, tlo), 0, pt) * es
                                    : (uint32_t)rhi * rowb + (uint32_t)elem_of(lane - 33, 0, pt) * es;
    const uint32_t vh2 = lane < 2 ? (uint32_t)rhi * rowb + (uint32_t)elem_of(31 + lane, 0, pt) * es
                                  : (uint32_t)rlo * rowb;
    const uint32_t vhl = lane == 1 ? (uint32_t)rhi * lrowb : (uint32_t)rlo * lrowb;
    real hf[2];
    double hlam;
    bload(hf[0], fin, vh1, 0u);
    bload(hf[1], fin, vh2, 0u);
    bload(hlam, lin, vhl, 0u);

    // (1)-(3) moments, weights, f^eq polynomial, BGK and chemical factors
    const Cell<real> C(dp, fc, lc);
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
        const real Ak = keep + beta * (v * v + u2 - (real)2 * T);
        const int base = 1 + 8 * (k - 1);
        real o[8];
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            const real z = v * EP.w(dd);
            real pp, pm;
            EP.eval(z, pp, pm);
            const real bz = Bz * z;
#pragma unroll
            for (int sgn = 0; sgn < 2; ++sgn) {
                const int q = base + dd + 4 * sgn;
                const real x = fc[q];
                const real coll = sgn == 0 ? rF * pp * (Ak + bz) + omega * x : rF * pm * (Ak - bz) + omega * x;
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
                o[dd + 4 * sgn] = coll - v * (acr[dd] * (x - nbr) + act[dd] * (x - nbt));
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

// Occupancy: float32 rows fit two wavefronts per SIMD; float64 rows take
// the whole register file of one (the next row in flight is 66 VGPRs).
template <typename real>
struct StepOcc {
    static constexpr int waves = sizeof(real) == 4 ? 2 : 1;
};

// Whether step `s` of a solve makes a drift record.
__device__ __forceinline__ bool records(DescPtr dp, int64_t s)
{
    return dp->diag_every > 0 && s >= dp->state->rec_from && s % dp->diag_every == 0;
}

// One time step of every solve of the launch.  Wavefront w of the grid takes
// tile t = (its block's XCD-ordered index) * 4 + w, which the tile table maps
// to (solve, tile of that solve); a solve's tile lt is row block lt / nstrip,
// strip lt % nstrip.  Each wavefront works on its own: no barriers and no
// atomics.  A drift-report step leaves per-wavefront partial sums in its
// slot of the solve's partial-sum ring; k_records adds them up later.
template <typename real, bool ROT>
__global__ __launch_bounds__(BLOCK, StepOcc<real>::waves) void k_step(const SolveDesc *descs, const uint2 *tiles,
                                                                       int ntiles, const int64_t *bases,
                                                                       int64_t step_off, int flip)
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
    const int cur = (int)((step + flip) & 1);
    const StepBufs bufs{dp->f[cur], dp->f[cur ^ 1], dp->lam[cur], dp->lam[cur ^ 1]};
    __shared__ real prev[BLOCK / 64][NQ][64];
    double red[5] = {0, 0, 0, 0, 0};
    // row-block major: the strips of one row block sit side by side in the
    // same XCD and share their halo columns in its L2; odd row blocks march
    // inward so that the rows bounding two blocks are read by both at once.
    if (dp->nt == 1) {
        // one theta column: lanes along r
        radial_block<real>(dp, bufs, lt, prev[threadIdx.x >> 6], red, diag);
    } else {
        const int rows = dp->rows, nstrip = dp->nstrip;
        const int rb = lt / nstrip, strip = lt - rb * nstrip;
        const int i0 = rb * rows;
        const int i1 = min(i0 + rows, dp->nr);
        march<real, ROT>(dp, bufs, strip, i0, i1, (rb & 1) != 0, prev[threadIdx.x >> 6], red, diag);
    }
    if (diag) {
        const int64_t slot = (step / dp->diag_every) % PART_RING;
        double *part = dp->wpart + ((size_t)slot * dp->nwaves + lt) * 5;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const double v = wave_sum(red[i]);
            if ((threadIdx.x & 63) == 0) part[i] = v;
        }
    }
}

// ------------------------------------------------------ two steps per pass --
// Steps s and s + 1 in one pass over f.  Stage A computes the state after
// step s (g) one row ahead of stage B, which computes the state after step
// s + 1 from g and stores it: g never leaves the wavefront.  Stage B's
// azimuthal neighbours of lanes 0 and 63 are g at the columns bordering the
// strip; the wavefront computes those cells itself at the start
// (edge_cells), as the adjacent strips do in their own stage A.  A block of
// R rows runs stage A on R + 2 rows and reads R + 4 rows of f, so each f
// value is read about 1.3 times (block boundaries, edge-cell gathers) and
// written once per two steps.

// Azimuthal neighbours of lanes 0 and 63 for stage A: the three gathered
// loads of a row of the input state, written to an LDS row and read back by
// every lane (hb[q] left halo of plane q, hb[33 + q] right halo; hl[0], hl[1]
// lambda).
template <typename real>
struct LdsHalo {
    const real *hb;
    const double *hl;
    __device__ __forceinline__ real left(int q) const { return hb[q]; }
    __device__ __forceinline__ real right(int q) const { return hb[33 + q]; }
    __device__ __forceinline__ double lleft() const { return hl[0]; }
    __device__ __forceinline__ double lright() const { return hl[1]; }
};
// The gathered halo registers of one row (see Strip::load_halo).
template <typename real>
struct GatherHalo {
    real h[2];
    double hl;
};

// ... and from the edge cells of the intermediate state in LDS (stage B).  Of
// each pair of opposite directions an edge cell keeps only the one lane 0
// (left side) or lane 63 (right side) takes from that side, in slot
// 4 (k - 1) + (direction mod 4).
template <typename real>
struct EdgeHalo {
    const real *L, *R;
    double ll, lr;
    static __device__ __forceinline__ int slot(int q) { return ((q - 1) >> 3) * 4 + ((q - 1) & 3); }
    __device__ __forceinline__ real left(int q) const { return L[slot(q)]; }
    __device__ __forceinline__ real right(int q) const { return R[slot(q)]; }
    __device__ __forceinline__ double lleft() const { return ll; }
    __device__ __forceinline__ double lright() const { return lr; }
};

// One row of one of the two steps: the arithmetic of update_row, with the
// azimuthal halo from H.  Radial neighbours: the row behind in compact LDS
// slots (of each opposite pair of directions only the one that takes its
// upwind value from behind, slot 4 (k - 1) + (direction mod 4); replaced by
// this row's as they are read), the row ahead in `fn` (stage A) or in the
// full LDS row `ga` (stage B).  STAGEA: the new row goes to `ga` and `lout`,
// for every lane (stage B reads the periodic images too); otherwise it is
// stored, for the strip's own columns.
template <typename real, bool STAGEA, class Halo>
__device__ __forceinline__ void stage_row(const Strip<real, false> &S, int ir, real (*behind)[64], const real fc[NQ],
                                          const real *fn, real (*ga)[64], const Halo &H, double lbehind, double lc,
                                          double lahead, const bool mr[4], const bool mt[4], const real acr[4],
                                          const real ctv[4], bool lr_behind, double csx, double csy, double &lout,
                                          double red[5], bool diag)
{
    const DescPtr dp = S.dp;
    const Cell<real> C(dp, fc, lc);
    const double ri = dp->r_min + ((double)ir + 0.5) * dp->dr;
    const real kt = (real)(dp->dt_dth / ri);
    real act[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) act[dd] = fabs(ctv[dd]) * kt;

    const bool store = S.useful;
    const int lane = S.lane;
    const uint32_t rowoff = (uint32_t)ir * S.row_bytes;
    const uint32_t pb = opaque(S.pair_bytes);
    const uint32_t pairs = rowoff + S.rest_bytes;

    // stage B stores from every lane, periodic images into their own
    // column of the row padding (nothing reads it): no store sits under a
    // lane mask, which keeps the exec-mask branches and their registers out
    // of the row loop
    const real rest = C.rest(fc[0]);
    if (STAGEA)
        ga[0][lane] = rest;
    else
        bstore(rest, S.fout, S.vos, rowoff);
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
        const real v = (real)speed(k);
        const real rF = C.rho * C.F[k];
        const real Ak = C.keep + C.beta * (v * v + C.u2 - (real)2 * C.T);
        const int base = 1 + 8 * (k - 1);
        real o[8];
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            const real z = v * C.EP.w(dd);
            real pp, pm;
            C.EP.eval(z, pp, pm);
            const real bz = C.Bz * z;
            const int c = 4 * (k - 1) + dd;
            const real back = behind[c][lane];
            behind[c][lane] = mr[dd] ? fc[base + dd] : fc[base + dd + 4];
#pragma unroll
            for (int sgn = 0; sgn < 2; ++sgn) {
                const int q = base + dd + 4 * sgn;
                const real x = fc[q];
                const real coll =
                    sgn == 0 ? rF * pp * (Ak + bz) + C.omega * x : rF * pm * (Ak - bz) + C.omega * x;
                const bool rb = sgn == 0 ? mr[dd] : !mr[dd];
                real ahead;
                if constexpr (STAGEA)
                    ahead = fn[q];
                else
                    ahead = ga[q][lane];
                const real nbr = rb ? back : ahead;
                // every lane takes both shifts (lanes 0 and 63 the halo
                // values), then selects
                const real left = from_left_or(H.left(q), x);
                const real right = from_right_or(H.right(q), x);
                const bool tl = sgn == 0 ? mt[dd] : !mt[dd];
                const real nbt = tl ? left : right;
                o[dd + 4 * sgn] = coll - v * (acr[dd] * (x - nbr) + act[dd] * (x - nbt));
            }
        }
        if (STAGEA) {
#pragma unroll
            for (int i = 0; i < 8; ++i) ga[base + i][lane] = o[i];
        } else {
#pragma unroll
            for (int dd = 0; dd < 4; ++dd)
                bstore2(o[dd], o[dd + 4], S.fout, S.vos2, pairs + (uint32_t)(4 * (k - 1) + dd) * pb);
        }
    }

    const double uxd = (double)C.ux, uyd = (double)C.uy;
    const double urp = uxd * csx + uyd * csy;
    const double utp = -uxd * csy + uyd * csx;
    const double lreac = C.reacted(dp, lc);
    const double lleft = from_left_or(H.lleft(), lc);
    const double lright = from_right_or(H.lright(), lc);
    const double lr = (urp >= 0.0) == lr_behind ? lbehind : lahead;
    const double lt = utp >= 0.0 ? lleft : lright;
    const double lnew = lreac - fabs(urp) * dp->dt_dr * (lc - lr) - fabs(utp) * (dp->dt_dth / ri) * (lc - lt);
    if (STAGEA)
        lout = lnew;
    else
        bstore(lnew, S.lout, S.vols, (uint32_t)ir * S.lrow_bytes);

    if (diag && store) diag_cell(red, (double)C.rho, uxd, uyd, C.Td, (double)C.e, lc, ri * dp->dr * dp->dth, dp->Q);
}

// The value the other lane of a lane pair (lanes 2m, 2m + 1) holds.
__device__ __forceinline__ float pair_swap(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xf, 0xf, false));
}
__device__ __forceinline__ double pair_swap(double v)
{
    return __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xf, 0xf, false),
                            __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xf, 0xf, false));
}

// The intermediate state at the columns bordering strip `strip`, c0 - 1
// (left) and c0 + 64 (right) as periodic images, for the rows [i0, i1) of the
// block.  Two lanes take one cell: lane 32 side + 2 e + h takes row i0 + e of
// its side, h = 0 the speeds 1 and 2 (and the rest particle), h = 1 the
// speeds 3 and 4.  Each lane gathers its pairs of the cell and of the cell's
// upwind neighbours (radial ghost rules of Sec. II.D included), one access
// per pair; the two lanes add up their partial moments, and each updates its
// pairs as stage A of the strip owning the column does.  Of each opposite
// pair of directions it keeps the one that lane 0 (left side) or lane 63
// (right side) takes from there; the first lane of the two keeps lambda.
// Every lane runs every instruction up to the final stores (the moment
// exchange is a lane shift).
template <typename real>
__device__ __forceinline__ void edge_cells(const Strip<real, false> &S, int strip, int i0, int i1,
                                           real (*ef)[FUSE_ROWS][16], double (*el)[FUSE_ROWS])
{
    const DescPtr dp = S.dp;
    const int lane = S.lane, side = lane >> 5, e = (lane >> 1) & 15, h = lane & 1;
    const int count = i1 - i0;
    const int nr = dp->nr, nt = dp->nt;
    const int r = i0 + min(e, count - 1);  // lanes past the block repeat its last row
    const int c0 = strip * STRIP;
    const int pc = side == 0 ? (c0 + nt - 1) % nt : (c0 + STRIP) % nt;
    const int pl = (pc + nt - 1) % nt, pr = (pc + 1) % nt;
    const int pk = (side == 0 ? c0 : c0 + STRIP - 1) % nt;  // column of lane 0 / lane 63
    const double2 cs = dp->cs[pc], ck = dp->cs[pk];
    const real cth = (real)cs.x, sth = (real)cs.y;
    const real crv[4] = {cth, (real)SQH * (cth + sth), sth, (real)SQH * (sth - cth)};
    const real ctv[4] = {-sth, (real)SQH * (cth - sth), cth, (real)SQH * (cth + sth)};
    const real kcth = (real)ck.x, ksth = (real)ck.y;
    const real kctv[4] = {-ksth, (real)SQH * (kcth - ksth), kcth, (real)SQH * (kcth + ksth)};

    const uint32_t es = (uint32_t)sizeof(real), rowb = S.row_bytes, lrowb = S.lrow_bytes;
    // radial neighbours: below row 0 the copy of row 0 (disc centre: with
    // directions turned by 4, i.e. the members of each pair swapped), above
    // row nr - 1 the copy of row nr - 1
    const int rlo = max(r - 1, 0), rhi = min(r + 1, nr - 1);
    const bool turn = r == 0 && dp->disc;
    const uint32_t orow = (uint32_t)r * rowb, olo = (uint32_t)rlo * rowb, ohi = (uint32_t)rhi * rowb;
    const uint32_t cc = 2u * (uint32_t)pc * es, cl = 2u * (uint32_t)pl * es, cr = 2u * (uint32_t)pr * es;
    // this lane's pairs 8 h .. 8 h + 7 (speeds 2 h + 1, 2 h + 2): directions
    // dd of pair i in x[i], dd + 4 in x[i + 8]
    real x[16], nbr[16], nbt[16], x0;
    bload(x0, S.fin, orow + (uint32_t)pc * es, 0u);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t po = S.rest_bytes + (uint32_t)(8 * h + i) * S.pair_bytes;
        const int dd = i & 3;
        real lo0, lo1, hi0, hi1, l0, l1, r0, r1;
        bload2(x[i], x[i + 8], S.fin, orow + cc + po, 0u);
        bload2(lo0, lo1, S.fin, olo + cc + po, 0u);
        bload2(hi0, hi1, S.fin, ohi + cc + po, 0u);
        bload2(l0, l1, S.fin, orow + cl + po, 0u);
        bload2(r0, r1, S.fin, orow + cr + po, 0u);
        const real t0 = turn ? lo1 : lo0, t1 = turn ? lo0 : lo1;
        const bool mr = crv[dd] >= (real)0, mt = ctv[dd] >= (real)0;
        // direction dd takes the lower row if mr and the left column if mt,
        // dd + 4 the other ones
        nbr[i] = mr ? t0 : hi0;
        nbr[i + 8] = mr ? hi1 : t1;
        nbt[i] = mt ? l0 : r0;
        nbt[i + 8] = mt ? r1 : l1;
    }
    double lc, lb, la, lL, lR;
    bload(lc, S.lin, (uint32_t)r * lrowb + (uint32_t)pc * 8u, 0u);
    bload(lb, S.lin, (uint32_t)rlo * lrowb + (uint32_t)pc * 8u, 0u);
    bload(la, S.lin, (uint32_t)rhi * lrowb + (uint32_t)pc * 8u, 0u);
    bload(lL, S.lin, (uint32_t)r * lrowb + (uint32_t)pl * 8u, 0u);
    bload(lR, S.lin, (uint32_t)r * lrowb + (uint32_t)pr * 8u, 0u);

    // moments: this lane's two rings (summed as raw_moments does), then the
    // other lane's added
    const real va = h == 0 ? (real)speed(1) : (real)speed(3), vb = h == 0 ? (real)speed(2) : (real)speed(4);
    real rho = h == 0 ? x0 : (real)0, jx = 0, jy = 0, en = 0;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        const real *g = x + 4 * kk;  // directions 0..3 at g[0..3], 4..7 at g[8..11]
        const real v = kk == 0 ? va : vb;
        const real ring = ((g[0] + g[8]) + (g[2] + g[10])) + ((g[1] + g[9]) + (g[3] + g[11]));
        const real a15 = g[1] - g[9], a37 = g[3] - g[11];
        const real X = (g[0] - g[8]) + (real)SQH * (a15 - a37);
        const real Y = (g[2] - g[10]) + (real)SQH * (a15 + a37);
        rho += ring;
        jx += v * X;
        jy += v * Y;
        en += (real)0.5 * v * v * ring;
    }
    Cell<real> C;
    C.rho = rho + pair_swap(rho);
    C.e = en + pair_swap(en);
    C.init_moments(dp, jx + pair_swap(jx), jy + pair_swap(jy), lc);

    const double ri = dp->r_min + ((double)r + 0.5) * dp->dr;
    const real kr = (real)dp->dt_dr, kt = (real)(dp->dt_dth / ri);
    real g[16];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        const real v = kk == 0 ? va : vb;
        const real Fk = h == 0 ? C.F[1 + kk] : C.F[3 + kk];
        const real rF = C.rho * Fk;
        const real Ak = C.keep + C.beta * (v * v + C.u2 - (real)2 * C.T);
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            const int i = 4 * kk + dd;
            const real z = v * C.EP.w(dd);
            real pp, pm;
            C.EP.eval(z, pp, pm);
            const real bz = C.Bz * z;
            const real acr = fabs(crv[dd]) * kr, act = fabs(ctv[dd]) * kt;
            const real c0v = rF * pp * (Ak + bz) + C.omega * x[i];
            const real c1v = rF * pm * (Ak - bz) + C.omega * x[i + 8];
            g[i] = c0v - v * (acr * (x[i] - nbr[i]) + act * (x[i] - nbt[i]));
            g[i + 8] = c1v - v * (acr * (x[i + 8] - nbr[i + 8]) + act * (x[i + 8] - nbt[i + 8]));
        }
    }
    const double uxd = (double)C.ux, uyd = (double)C.uy;
    const double urp = uxd * cs.x + uyd * cs.y;
    const double utp = -uxd * cs.y + uyd * cs.x;
    const double lr = urp >= 0.0 ? lb : la;
    const double lt = utp >= 0.0 ? lL : lR;
    const double lnew =
        C.reacted(dp, lc) - fabs(urp) * dp->dt_dr * (lc - lr) - fabs(utp) * (dp->dt_dth / ri) * (lc - lt);
    if (e < count) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int dd = i & 3;
            const bool first = (kctv[dd] >= (real)0) != (side == 1);  // keep direction dd, else dd + 4
            ef[side][e][8 * h + i] = first ? g[i] : g[i + 8];
        }
        if (h == 0) el[side][e] = lnew;
    }
}

// Orders this wavefront's LDS writes before its reads of what other lanes
// wrote (a wavefront's LDS operations complete in order; this keeps the
// compiler from moving them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Plane q of the ghost row beyond the grid made from row `src`: the copy of
// the boundary row, with directions turned by 4 below the disc centre.
__device__ __forceinline__ int ghost_plane(int q, bool turn)
{
    if (q == 0 || !turn) return q;
    const int base = 1 + 8 * ((q - 1) / 8), dir = (q - 1) % 8;
    return base + ((dir + 4) & 7);
}

// Fills the compact slots of the row behind (see stage_row) from a full row.
template <typename real>
__device__ __forceinline__ void fill_behind(real (*behind)[64], const real x[NQ], const bool mr[4], int lane)
{
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) behind[4 * k + dd][lane] = mr[dd] ? x[1 + 8 * k + dd] : x[5 + 8 * k + dd];
}

// Work of one wavefront of the two-step kernel: strip `strip`, rows [i0, i1)
// (at most FUSE_ROWS), marched outward or, with `down`, inward.  Positions p
// count rows in marching order from the first row of the block (p = 0);
// stage A runs on positions -1 .. R where they are grid rows, stage B on
// 0 .. R - 1, one position behind stage A.  LDS per wavefront: the compact
// rows behind of f (fb) and of g (gb), the full row of g just computed (ga),
// the edge cells (ef, el) and the gathered halo values of stage A's row
// (hb, hbl).
template <typename real>
__device__ __forceinline__ void march2(DescPtr dp, const StepBufs &bufs, int strip, int i0, int i1, bool down,
                                       real (*fb)[64], real (*gb)[64], real (*ga)[64], real (*ef)[FUSE_ROWS][16],
                                       double (*el)[FUSE_ROWS], real *hb, double *hbl, double redA[5],
                                       double redB[5], bool diagA, bool diagB)
{
    const Strip<real, false> S(dp, bufs, strip);
    edge_cells<real>(S, strip, i0, i1, ef, el);
    wave_lds_sync();

    const int lane = S.lane;
    const double2 cs = dp->cs[S.pc];
    const real cth = (real)cs.x, sth = (real)cs.y;
    const real crv[4] = {cth, (real)SQH * (cth + sth), sth, (real)SQH * (sth - cth)};
    const real ctv[4] = {-sth, (real)SQH * (cth - sth), cth, (real)SQH * (cth + sth)};
    const real kr = (real)dp->dt_dr;
    real acr[4];
    bool mr[4], mt[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        acr[dd] = fabs(crv[dd]) * kr;
        mr[dd] = (crv[dd] >= (real)0) != down;
        mt[dd] = ctv[dd] >= (real)0;
    }
    const int nr = dp->nr;
    const int step = down ? -1 : 1;
    const int first = down ? i1 - 1 : i0;
    const int count = i1 - i0;
    const int rbefore = first - step, rafter = first + count * step;  // rows of positions -1 and R
    const bool vlo = rbefore >= 0 && rbefore < nr, vhi = rafter >= 0 && rafter < nr;
    const bool turn_lo = rbefore < 0 && dp->disc, turn_hi = rafter < 0 && dp->disc;

    // f at positions p (fc) and p + 1 (fn) in registers; f(p + 2) is loaded
    // into fc once stage A has used it, and the two swap at the end of the
    // pass (the loop is not unrolled: one pass is already half the
    // instruction cache)
    real fc[NQ], fn[NQ];
    double lp, lc, ln, lx = 0.0;             // lambda of f at positions p-1, p, p+1, p+2
    double glp = 0.0, glc = 0.0, gln = 0.0;  // lambda of g at positions p-2, p-1, p
    GatherHalo<real> hc, hn, hx;
    int p0;
    {
        real t[NQ];
        if (vlo) {
            // stage A starts at position -1: behind it position -2 (a ghost
            // beyond the grid), centre -1, ahead 0
            S.load_row(rbefore, fc, lc);
            S.load_halo(rbefore, hc.h, hc.hl);
            S.load_row(first, fn, ln);
            S.load_halo(first, hn.h, hn.hl);
            row_or_ghost(S, rbefore - step, t, lp, fc, lc);
            p0 = -1;
        } else {
            S.load_row(first, fc, lc);
            S.load_halo(first, hc.h, hc.hl);
            row_or_ghost(S, first + step, fn, ln, fc, lc);
            if (count > 1 || vhi) S.load_halo(first + step, hn.h, hn.hl);
            row_or_ghost(S, rbefore, t, lp, fc, lc);
            p0 = 0;
        }
        fill_behind(fb, t, mr, lane);
    }

    for (int p = p0; p <= count; ++p) {
        const int ir = first + p * step;
        // g(p - 1), centre of stage B, before stage A replaces it in ga
        real gc[NQ];
        if (p >= 1) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) gc[q] = ga[q][lane];
        } else if (p == 0 && vlo) {
            // g(-1), computed by stage A at position -1, is the row behind
            // stage B's first row
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int dd = 0; dd < 4; ++dd)
                    gb[4 * k + dd][lane] = mr[dd] ? ga[1 + 8 * k + dd][lane] : ga[5 + 8 * k + dd][lane];
        }
        // (A) first step at position p, or the ghost beyond the grid
        if (p < count || vhi) {
            // the row's gathered halo values into LDS, read back by every lane
            hb[lane] = hc.h[0];
            if (lane < 2) {
                hb[64 + lane] = hc.h[1];
                hbl[lane] = hc.hl;
            }
            wave_lds_sync();
            const LdsHalo<real> H{hb, hbl};
            stage_row<real, true>(S, ir, fb, fc, fn, ga, H, lp, lc, ln, mr, mt, acr, ctv, !down, cs.x, cs.y, gln,
                                  redA, diagA && p >= 0 && p < count);
        } else {
#pragma unroll
            for (int q = 0; q < NQ; ++q) ga[q][lane] = turn_hi ? gc[ghost_plane(q, true)] : gc[q];
            gln = glc;
        }
        // f at position p + 2 (the row ahead of the next stage A) replaces f(p)
        if (p + 1 < count || (p + 1 == count && vhi)) row_or_ghost(S, ir + 2 * step, fc, lx, fn, ln);
        if (p + 2 < count || (p + 2 == count && vhi)) S.load_halo(ir + 2 * step, hx.h, hx.hl);
        // (B) second step at position p - 1
        if (p == 0 && !vlo) {
            // the row behind stage B's first row is the ghost of g(0)
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int dd = 0; dd < 4; ++dd) {
                    const real a = ga[ghost_plane(1 + 8 * k + dd, turn_lo)][lane];
                    const real b = ga[ghost_plane(5 + 8 * k + dd, turn_lo)][lane];
                    gb[4 * k + dd][lane] = mr[dd] ? a : b;
                }
            glc = gln;
        } else if (p > 0) {
            const int e = ir - step - i0;
            const EdgeHalo<real> H{ef[0][e], ef[1][e], el[0][e], el[1][e]};
            double unused;
            stage_row<real, false>(S, ir - step, gb, gc, nullptr, ga, H, glp, glc, gln, mr, mt, acr, ctv, !down,
                                   cs.x, cs.y, unused, redB, diagB);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const real t = fc[q];
            fc[q] = fn[q];
            fn[q] = t;
        }
        hc = hn;
        hn = hx;
        lp = lc;
        lc = ln;
        ln = lx;
        glp = glc;
        glc = gln;
        // Compiler-only barrier: the LDS rows must not be promoted to
        // registers across passes.
        asm volatile("" ::: "memory");
    }
}

// Steps `step` and step + 1 of one solve (descs[0]); tiles as k_step's.  One
// wavefront per SIMD in both precisions (the two steps' rows fill the
// register file and the LDS rows of four wavefronts most of a CU's LDS).
template <typename real>
__global__ __launch_bounds__(BLOCK, 1) void k_step2(const SolveDesc *descs, int ntiles,
                                                                       int64_t step, int flip)
{
    const int nb = gridDim.x;
    const int blk = xcd_tile(blockIdx.x, nb);
    const int t = __builtin_amdgcn_readfirstlane(blk * (BLOCK / 64) + (threadIdx.x >> 6));
    if (t >= ntiles) return;
    const DescPtr dp = (DescPtr)descs;
    const bool diagA = records(dp, step), diagB = records(dp, step + 1);
    const int cur = (int)((step + flip) & 1);
    const StepBufs bufs{dp->f[cur], dp->f[cur ^ 1], dp->lam[cur], dp->lam[cur ^ 1]};
    __shared__ real fb[BLOCK / 64][16][64];
    __shared__ real gb[BLOCK / 64][16][64];
    __shared__ real ga[BLOCK / 64][NQ][64];
    __shared__ real ef[BLOCK / 64][2][FUSE_ROWS][16];
    __shared__ double el[BLOCK / 64][2][FUSE_ROWS];
    __shared__ real hb[BLOCK / 64][66];
    __shared__ double hbl[BLOCK / 64][2];
    const int w = threadIdx.x >> 6;
    double redA[5] = {0, 0, 0, 0, 0}, redB[5] = {0, 0, 0, 0, 0};
    const int rows = dp->rows, nstrip = dp->nstrip;
    const int rb = t / nstrip, strip = t - rb * nstrip;
    const int i0 = rb * rows;
    const int i1 = min(i0 + rows, dp->nr);
    march2<real>(dp, bufs, strip, i0, i1, (rb & 1) != 0, fb[w], gb[w], ga[w], ef[w], el[w], hb[w], hbl[w], redA,
                 redB, diagA, diagB);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        if (!(s == 0 ? diagA : diagB)) continue;
        const int64_t slot = ((step + s) / dp->diag_every) % PART_RING;
        double *part = dp->wpart + ((size_t)slot * dp->nwaves + t) * 5;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const double v = wave_sum(s == 0 ? redA[i] : redB[i]);
            if ((threadIdx.x & 63) == 0) part[i] = v;
        }
    }
}

__global__ void k_advance(int64_t *bases, int n, int64_t by)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bases[i] += by;
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

// -------------------------------------------------------------- moments --
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_moments(SolveDesc d, int cur, double *out, DiagCtl dc)
{
    const int nb = gridDim.x;
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    const int ncell = d.nr * d.nt;
    double red[5] = {0, 0, 0, 0, 0};
    if (c < ncell) {
        const int ir = c / d.nt;
        const int jt = c - ir * d.nt;
        const real *fin = (const real *)d.f[cur];
        const int64_t idx = (int64_t)ir * d.pitch + jt;
        const int64_t frow = (int64_t)ir * d.rstride;
        real f[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) f[q] = fin[frow + elem_of(q, jt, d.pitch)];
        real rho, jx, jy, e;
        raw_moments(f, rho, jx, jy, e);
        const double rd = (double)rho;
        const double ux = (double)(jx / rho), uy = (double)(jy / rho);
        const double T = (double)(e / rho - (real)0.5 * ((jx / rho) * (jx / rho) + (jy / rho) * (jy / rho)));
        const double2 cs = d.cs[jt];
        const double lam = d.lam[cur][idx];
        if (out) {
            out[c] = rd;
            out[(size_t)ncell + c] = ux * cs.x + uy * cs.y;
            out[2 * (size_t)ncell + c] = -ux * cs.y + uy * cs.x;
            out[3 * (size_t)ncell + c] = T;
            out[4 * (size_t)ncell + c] = rd * T;
            out[5 * (size_t)ncell + c] = lam;
        }
        const double ri = d.r_min + ((double)ir + 0.5) * d.dr;
        diag_cell(red, rd, ux, uy, T, (double)e, lam, ri * d.dr * d.dth, d.Q);
    }
    diag_reduce(dc, red, blockIdx.x, nb);
}

// ----------------------------------------------------- non-equilibrium --
// Delta*_m = M*_m(f) - M*_m(f^eq) of every cell (Sec. II.E): central moments
// about the cell's u in its polar frame (e_r, e_theta at theta_j), taken as
// the moments of f - f^eq.  Float64 throughout.  out: [NONEQ][nr][nt] in the
// order M*_2 rr, r theta, theta theta; M*_3 rrr, rr theta, r theta theta,
// theta theta theta; M*_{3,1} r, theta; M*_{4,2} rr, r theta, theta theta.
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_noneq(SolveDesc d, int cur, double *out)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    const int ncell = d.nr * d.nt;
    if (c >= ncell) return;
    const int ir = c / d.nt;
    const int jt = c - ir * d.nt;
    const real *fin = (const real *)d.f[cur];
    const int64_t frow = (int64_t)ir * d.rstride;
    double f[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) f[q] = (double)fin[frow + elem_of(q, jt, d.pitch)];
    double rho, jx, jy, e;
    raw_moments(f, rho, jx, jy, e);
    const double ux = jx / rho, uy = jy / rho;
    const double T = e / rho - 0.5 * (ux * ux + uy * uy);
    double g[NQ];
    equilibrium<double>(d.A, rho, ux, uy, T, g);
#pragma unroll
    for (int q = 0; q < NQ; ++q) g[q] = f[q] - g[q];
    const double2 cs = d.cs[jt];
    const double ur = ux * cs.x + uy * cs.y, ut = -ux * cs.y + uy * cs.x;
    // cos and sin of the directions i pi/4
    constexpr double DX[8] = {1.0, SQH, 0.0, -SQH, -1.0, -SQH, 0.0, SQH};
    constexpr double DY[8] = {0.0, SQH, 1.0, SQH, 0.0, -SQH, -1.0, -SQH};
    double m[NONEQ];
#pragma unroll
    for (int k = 0; k < NONEQ; ++k) m[k] = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double vr = 0.0, vt = 0.0;
        if (q > 0) {
            const int k = 1 + (q - 1) / 8, i = (q - 1) % 8;
            vr = speed(k) * (DX[i] * cs.x + DY[i] * cs.y);  // v cos(i pi/4 - theta)
            vt = speed(k) * (DY[i] * cs.x - DX[i] * cs.y);  // v sin(i pi/4 - theta)
        }
        const double cr = vr - ur, ct = vt - ut;
        const double h = 0.5 * (cr * cr + ct * ct);
        const double grr = g[q] * cr, gtt = g[q] * ct;
        m[0] += grr * cr;
        m[1] += grr * ct;
        m[2] += gtt * ct;
        m[3] += grr * cr * cr;
        m[4] += grr * cr * ct;
        m[5] += grr * ct * ct;
        m[6] += gtt * ct * ct;
        m[7] += h * grr;
        m[8] += h * gtt;
        m[9] += h * grr * cr;
        m[10] += h * grr * ct;
        m[11] += h * gtt * ct;
    }
#pragma unroll
    for (int k = 0; k < NONEQ; ++k) out[(size_t)k * ncell + c] = m[k];
}

// ------------------------------------------------------------ initial state
// Pressure with noise, rounded exactly as written (no contraction): the
// same bits as any IEEE implementation of the formula.
__device__ __attribute__((noinline)) double noisy_pressure(double rho, double T, double amp, uint64_t h)
{
#pragma clang fp contract(off)
    const double U = (double)(h >> 11) * 0x1.0p-53;
    const double p = rho * T;
    return p + amp * (2.0 * U - 1.0);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename real>
__device__ __forceinline__ void store_eq(const SolveDesc &d, int cur, int64_t idx, int jt, double rho, double T,
                                         double ur, double ut)
{
    const double2 cs = d.cs[jt];
    const double ux = ur * cs.x - ut * cs.y, uy = ur * cs.y + ut * cs.x;
    real f[NQ];
    equilibrium<real>(d.A, (real)rho, (real)ux, (real)uy, (real)T, f);
    real *fo = (real *)d.f[cur] + (idx / d.pitch) * d.rstride;
#pragma unroll
    for (int q = 0; q < NQ; ++q) fo[elem_of(q, jt, d.pitch)] = f[q];
}

template <typename real>
__global__ __launch_bounds__(BLOCK) void k_init_ic(SolveDesc d, int cur, pdbm_ic ic)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= d.nr * d.nt) return;
    const int ir = c / d.nt;
    const int jt = c - ir * d.nt;
    const int64_t idx = (int64_t)ir * d.pitch + jt;
    const double ri = d.r_min + ((double)ir + 0.5) * d.dr;
    const double *st = ri < ic.r_split ? ic.inner : ic.outer;
    const uint64_t h = splitmix64(ic.seed ^ ((uint64_t)c * 0x9E3779B97F4A7C15ull));
    const double p = noisy_pressure(st[0], st[1], ic.p_noise, h);
    store_eq<real>(d, cur, idx, jt, st[0], p / st[0], st[2], st[3]);
    d.lam[cur][idx] = st[4];
}

// fields: [5][nr][ntheta] = rho, T, u_r, u_theta, lambda
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_init_fields(SolveDesc d, int cur, const double *fields)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    const int ncell = d.nr * d.nt;
    if (c >= ncell) return;
    const int ir = c / d.nt;
    const int jt = c - ir * d.nt;
    const int64_t idx = (int64_t)ir * d.pitch + jt;
    store_eq<real>(d, cur, idx, jt, fields[c], fields[(size_t)ncell + c], fields[2 * (size_t)ncell + c],
                   fields[3 * (size_t)ncell + c]);
    d.lam[cur][idx] = fields[4 * (size_t)ncell + c];
}

}  // namespace

int cell_blocks(int nr, int nt) { return (int)(((int64_t)nr * nt + BLOCK - 1) / BLOCK); }

int solve_waves(int nr, int nt, int rows)
{
    if (nt == 1) return (nr + STRIP - 1) / STRIP;  // lanes along r: 64 rows per wavefront
    return (int)((int64_t)((nr + rows - 1) / rows) * ((nt + STRIP - 1) / STRIP));
}

hipError_t launch_step(const SolveDesc *descs, const uint2 *tiles, int ntiles, const int64_t *bases, int64_t step_off,
                       int flip, bool fp32, bool rot, hipStream_t st)
{
    const int nb = (ntiles + BLOCK / 64 - 1) / (BLOCK / 64);
    if (nb == 0) return hipSuccess;
    if (fp32) {
        if (rot)
            hipLaunchKernelGGL((k_step<float, true>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases,
                               step_off, flip);
        else
            hipLaunchKernelGGL((k_step<float, false>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases,
                               step_off, flip);
    } else {
        if (rot)
            hipLaunchKernelGGL((k_step<double, true>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases,
                               step_off, flip);
        else
            hipLaunchKernelGGL((k_step<double, false>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases,
                               step_off, flip);
    }
    return hipGetLastError();
}

hipError_t launch_step2(const SolveDesc *descs, int ntiles, int64_t step, int flip, hipStream_t st)
{
    const int nb = (ntiles + BLOCK / 64 - 1) / (BLOCK / 64);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_step2<double>, dim3(nb), dim3(BLOCK), 0, st, descs, ntiles, step, flip);
    return hipGetLastError();
}

hipError_t launch_noneq(const SolveDesc &d, int cur, bool fp32, double *out, hipStream_t st)
{
    const int nb = cell_blocks(d.nr, d.nt);
    if (fp32)
        hipLaunchKernelGGL(k_noneq<float>, dim3(nb), dim3(BLOCK), 0, st, d, cur, out);
    else
        hipLaunchKernelGGL(k_noneq<double>, dim3(nb), dim3(BLOCK), 0, st, d, cur, out);
    return hipGetLastError();
}

hipError_t launch_advance(int64_t *bases, int n, int64_t by, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_advance, dim3((n + 255) / 256), dim3(256), 0, st, bases, n, by);
    return hipGetLastError();
}

hipError_t launch_records(const SolveDesc *descs, int n, const int64_t *bases, int64_t lo, int64_t hi, hipStream_t st)
{
    if (n <= 0 || hi <= lo) return hipSuccess;
    const int nrec = (int)std::min<int64_t>(hi - lo, PART_RING);
    hipLaunchKernelGGL(k_records, dim3(n, nrec), dim3(64), 0, st, descs, bases, lo, hi);
    return hipGetLastError();
}

hipError_t launch_moments(const SolveDesc &d, int cur, bool fp32, double *out, const DiagCtl &dc, hipStream_t st)
{
    const int nb = cell_blocks(d.nr, d.nt);
    if (fp32)
        hipLaunchKernelGGL(k_moments<float>, dim3(nb), dim3(BLOCK), 0, st, d, cur, out, dc);
    else
        hipLaunchKernelGGL(k_moments<double>, dim3(nb), dim3(BLOCK), 0, st, d, cur, out, dc);
    return hipGetLastError();
}

hipError_t launch_init_ic(const SolveDesc &d, int cur, bool fp32, const pdbm_ic &ic, hipStream_t st)
{
    const int nb = cell_blocks(d.nr, d.nt);
    if (fp32)
        hipLaunchKernelGGL(k_init_ic<float>, dim3(nb), dim3(BLOCK), 0, st, d, cur, ic);
    else
        hipLaunchKernelGGL(k_init_ic<double>, dim3(nb), dim3(BLOCK), 0, st, d, cur, ic);
    return hipGetLastError();
}

hipError_t launch_init_fields(const SolveDesc &d, int cur, bool fp32, const double *fields, hipStream_t st)
{
    const int nb = cell_blocks(d.nr, d.nt);
    if (fp32)
        hipLaunchKernelGGL(k_init_fields<float>, dim3(nb), dim3(BLOCK), 0, st, d, cur, fields);
    else
        hipLaunchKernelGGL(k_init_fields<double>, dim3(nb), dim3(BLOCK), 0, st, d, cur, fields);
    return hipGetLastError();
}

}  // namespace pdbm
