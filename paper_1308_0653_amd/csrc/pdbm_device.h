// Device code shared by the kernels of libpdbm for gfx950 (MI355X): the
// per-cell arithmetic of the method, wavefront reductions, lane shifts, raw
// buffer access and the wavefront strip over the paired f layout.  It sits
// in an unnamed namespace on purpose: each kernel source compiles its own
// internal copy, and no device symbol is shared between the sources.
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

#pragma once

#include <math.h>

#include "pdbm_internal.h"
#include "pdbm_offsets.h"

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

// F_k(T), k = 0..4, from the moment-inversion matrix, in float64: the
// powers T .. T^4 once, then each F_k as a sum of A_kn T^n.  (In Horner form
// each step adds a coefficient, which sits in a scalar register; the
// compiler's multiply-add takes its addend in the destination register, so
// every coefficient first took two moves into vector registers.  Here the
// coefficients are multiplicands, read from the scalar registers directly.)
template <typename real>
__device__ __forceinline__ void weights(const double *A, double T, real F[5])
{
    const double T2 = T * T, T3 = T2 * T, T4 = T2 * T2;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = A[4 * k] * T;
        v = fma(A[4 * k + 1], T2, v);
        v = fma(A[4 * k + 2], T3, v);
        v = fma(A[4 * k + 3], T4, v);
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

// 1/x: in float32 the hardware reciprocal (within 1 ulp) and one Newton step
// r + r (1 - x r), three instructions instead of a correctly rounded
// division's ten, within about half an ulp; in float64 the division.
__device__ __forceinline__ float inv(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double inv(double x) { return 1.0 / x; }

// Coefficients of the f^eq polynomial in z = v.u / T (Sec. II.B):
// P(z) = (1 - a + a^2/2) + z (1 - a) + z^2 (1 - a)/2 + z^3/6 + z^4/24, a = u^2/(2T)
template <typename real>
struct EqPoly {
    real c0, c1, c2, wx, wy;
    EqPoly() = default;
    __device__ __forceinline__ EqPoly(real ux, real uy, real u2, real T)
    {
        const real iT = inv(T);
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
    // the even and odd parts of P: P(z) = ev + od, P(-z) = ev - od
    __device__ __forceinline__ void parts(real z, real &ev, real &od) const
    {
        const real z2 = z * z;
        ev = c0 + z2 * (c2 + z2 * (real)(1.0 / 24.0));
        od = z * (c1 + z2 * (real)(1.0 / 6.0));
    }
    // P(z) and P(-z)
    __device__ __forceinline__ void eval(real z, real &pp, real &pm) const
    {
        real ev, od;
        parts(z, ev, od);
        pp = ev + od;
        pm = ev - od;
    }
};

// One step of an opposite pair of directions (Sec. II.C): direction q,
// whose velocity projects on u as z = v.u/T, and its opposite (-z).  With
// f^eq = rho F_k P(+-z), P = ev +- od, and the BGK + chemical factor
// A_k +- Bz z of the two (A_k = 1 - omega + beta (v^2 + u^2 - 2T),
// Bz = -2 beta T; Sec. II.B, II.C):
//   f^coll = rho F_k (ev +- od)(A_k +- Bz z) + omega f = (E +- O) + omega f,
//   E = rA ev + rb od,  O = rA od + rb ev,  rA = rho F_k A_k,  rb = rho F_k Bz z.
// The donor-cell fluxes -v acr (f - f_r) - v act (f - f_theta) (|C_r| =
// v acr, |C_theta| = v act for both directions of the pair) join the f term:
//   f^new = (E +- O) + s f + v (acr f_r + act f_theta),  s = omega - v (acr + act),
// with f_r, f_theta the radial and azimuthal upwind neighbours.
template <typename real>
__device__ __forceinline__ void pair_coll(const EqPoly<real> &EP, real z, real rA, real rB, real &E, real &O)
{
    real ev, od;
    EP.parts(z, ev, od);
    const real rb = rB * z;
    E = ev * rA + od * rb;
    O = od * rA + ev * rb;
}
// f^new of one direction from its collision part c = E +- O.  (acr, act and
// v enter as they are, not as the products v acr, v act: acr is the same in
// every row of a strip, and the compiler would keep the sixteen products in
// registers through the march.)
template <typename real>
__device__ __forceinline__ real dir_new(real c, real s, real x, real v, real acr, real act, real nbr, real nbt)
{
    return c + s * x + v * (acr * nbr + act * nbt);
}

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

// Sum of x over the wavefront (every lane must be active), in a fixed order:
// pairs, quads, half rows and rows of 16 lanes by DPP (after which every
// lane of a row holds the row's sum), then rows 1 and 3 add rows 0 and 2 by
// broadcast of lanes 15 and 47, and rows 2 and 3 the first half by
// broadcast of lane 31.  Lane 63 ends with the total, which is returned to
// every lane.  The moves stay in the VALU: the LDS permutes of a butterfly
// cost six dependent LDS round trips per value at the end of each
// wavefront's work.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double x)
{
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xf, false);
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xf, false);
    return x + __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double x)
{
    x = dpp_add<0xB1, 0xf>(x);   // quad_perm [1, 0, 3, 2]
    x = dpp_add<0x4E, 0xf>(x);   // quad_perm [2, 3, 0, 1]
    x = dpp_add<0x141, 0xf>(x);  // row_half_mirror
    x = dpp_add<0x140, 0xf>(x);  // row_mirror
    x = dpp_add<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x = dpp_add<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), 63),
                            __builtin_amdgcn_readlane(__double2loint(x), 63));
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

// Per-block partial sums of the drift report, written to dc.partials[tile];
// a second launch (k_diag_final) adds them up.  Must be reached by every
// thread of every block.  (A version in one kernel, where the last block to
// finish added the partials, needed a device-wide release per block, which
// on this GPU writes back the L2 of the block's die: the moments of a
// 1024 x 1024 float64 state took 268 us there, 64 + 7 us in two launches.)
__device__ __forceinline__ void diag_partial(const DiagCtl &dc, double v[5], int tile)
{
    block_sum5(v);
    if (threadIdx.x == 0) {
        double *p = dc.partials + 5 * (size_t)tile;
#pragma unroll
        for (int i = 0; i < 5; ++i) p[i] = v[i];
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

// ------------------------------------------------- wavefront strips --
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

// Has the value of a load made before a row loop arrive before the loop
// starts.  Used in the loop without that, the value makes the compiler wait
// there for every load in flight, including those of the rows ahead that the
// pass has just requested.
template <typename T>
__device__ __forceinline__ void settle(T &v)
{
    asm volatile("" : "+v"(v));
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
    bool turned;          // rotated sectors: some lane of the wavefront holds turned data (wave-uniform)

    __device__ __forceinline__ Strip(DescPtr dp_, const StepBufs &b, int strip) : dp(dp_)
    {
        fin = rsrc_of(b.f_in);
        fout = rsrc_of(b.f_out);
        lin = rsrc_of(b.lam_in);
        lout = rsrc_of(b.lam_out);
        lane = threadIdx.x & 63;
        const RowBytes rb = row_bytes_of(dp->rstride, dp->pitch, (int)sizeof(real));
        row_bytes = rb.row;
        lrow_bytes = rb.lrow;
        rest_bytes = rb.rest;
        pair_bytes = rb.pair;
        const StripOffsets o = strip_offsets(dp->nt, dp->pitch, dp->sector, ROT, (int)sizeof(real), rb, strip, lane);
        pc = o.pc;
        rot = o.rot;
        useful = o.useful;
        vo = o.vo;
        vo2 = o.vo2;
        vol = o.vol;
        vos = o.vos;
        vos2 = o.vos2;
        vols = o.vols;
        vh1 = o.vh1;
        vh2 = o.vh2;
        vhl = o.vhl;
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            poff[dd] = o.poff[dd];
            pswap[dd] = o.pswap[dd];
        }
        turned = ROT && __builtin_amdgcn_ballot_w64(rot != 0) != 0;
    }

    __device__ __forceinline__ void load_row(int row, real f[NQ], double &lam) const
    {
        uint32_t so = (uint32_t)row * row_bytes;
        bload(f[0], fin, vo, so);
        if (ROT && sizeof(real) == 8 && !turned) {
            // float64, no lane of the strip holding turned data (every strip
            // but one with periodic images past the last column): plain pair
            // loads, half as many as the member loads below (a 1024 x 512
            // float64 half annulus took 45.9 against 48.4 us per step with
            // member loads throughout)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t sk = so + (uint32_t)k * 4u * pair_bytes;
#pragma unroll
                for (int dd = 0; dd < 4; ++dd) bload2(f[1 + 8 * k + dd], f[5 + 8 * k + dd], fin, poff[dd], sk);
            }
        } else if (ROT && sizeof(real) == 8) {
            // this lane's data of direction dir lives in direction (dir + rot) % 8;
            // float64: each member loaded on its own, straight into its
            // register (with a pair load and a select, the one wavefront of
            // the SIMD waited for each load as it was made: 104.1 against
            // 63.0 us per step of a 1024 x 512 half annulus)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t sk = so + (uint32_t)k * 4u * pair_bytes;
#pragma unroll
                for (int dd = 0; dd < 4; ++dd) {
                    const uint32_t m = pswap[dd] ? (uint32_t)sizeof(real) : 0u;
                    bload(f[1 + 8 * k + dd], fin, poff[dd] + m, sk);
                    bload(f[5 + 8 * k + dd], fin, (poff[dd] + (uint32_t)sizeof(real)) - m, sk);
                }
            }
        } else if (ROT) {
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

// (cos, sin) of an angle turned by m pi / 4: the angle of a periodic image
// of a rotated sector, m sector widths on, from that of its physical column.
__device__ __forceinline__ double2 turn_cs(double2 cs, int m)
{
    double c = cs.x, s = cs.y;
    if (m & 1) {
        const double c1 = SQH * (c - s), s1 = SQH * (c + s);
        c = c1;
        s = s1;
    }
    if (m & 2) {
        const double c1 = -s;
        s = c;
        c = c1;
    }
    if (m & 4) {
        c = -c;
        s = -s;
    }
    return make_double2(c, s);
}

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
    // om: the cell's relaxation factor exp(-dt/tau)
    __device__ __forceinline__ Cell(DescPtr dp, const real x[NQ], double lc, real om)
    {
        real jx, jy;
        raw_moments(x, rho, jx, jy, e);
        init_moments(dp, jx, jy, lc, om);
    }
    // from rho, e (members) and the momentum jx, jy
    __device__ __forceinline__ void init_moments(DescPtr dp, real jx, real jy, double lc, real om)
    {
        const real irho = inv(rho);
        ux = jx * irho;
        uy = jy * irho;
        u2 = ux * ux + uy * uy;
        T = e * irho - (real)0.5 * u2;
        Td = (double)T;
        weights(dp->A, Td, F);
        EP = EqPoly<real>(ux, uy, u2, T);
        a = 0.0;
        b = 0.0;
        beta = (real)0;  // no reaction: R = 0
        on = dp->reacts && Td > dp->T_th;
        if (on) {
            const double p = (double)rho * Td;
            a = dp->w1 * ipow(p, dp->m);
            b = dp->w2 * ipow(p, dp->n);
            const double R = (1.0 - lc) * (a + b * lc);
            beta = (real)(dp->Q * R * dp->dt / (2.0 * Td * Td));
        }
        omega = om;
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

// Relaxation factor exp(-dt/tau) of a cell: the solve's own, or with TAUF
// the cell's entry of the per-cell field (Sec. IV, point (ii): tau may
// depend on the local state; the field is the caller's), stored in the
// solve's precision as [nr][pitch], so that cell (i, j) sits at byte
// (i pitch + j) sizeof(real) = vo + so as the rest particle's plane does
// within a row of f.
template <typename real, bool TAUF>
__device__ __forceinline__ real omega_at(DescPtr dp, uint32_t vo, uint32_t so)
{
    if constexpr (TAUF) {
        real v;
        bload(v, rsrc_of(dp->omegaf), vo, so);
        return v;
    } else {
        return (real)dp->omega;
    }
}

// Row `row` of the strip into f, or a ghost row outside [0, nr): below r_min
// the zero-gradient copy of row 0 or the disc-centre rule f(-1, j, k, i) =
// f(0, j, k, (i+4)%8) (Sec. II.D; discs are sectors 1, 2 or 4, so only the
// rotated-sector variant meets one at run time); above r_max the
// zero-gradient copy of row nr-1.  `edge` holds the boundary row the ghost
// copies.
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

// One row of one strip: moments, F_k(T), f^eq, BGK + chemical term, Cochran
// lambda, donor-cell fluxes of f and lambda.  fc: row i.  Marching outward
// (down = false): prev (LDS, this lane's column) holds row i-1 and fn row
// i+1; marching inward the roles swap.  prev is replaced by row i as it is
// consumed.  mr[dd] / mt[dd]: which side is upwind for direction dd (its
// opposite dd+4 takes the other side).
template <typename real, bool ROT, bool TAUF>
__device__ __forceinline__ void update_row(const Strip<real, ROT> &S, int ir, real (*prev)[64], const real fc[NQ],
                                           const real fn[NQ], const real hf[2], double hlam, double lbehind,
                                           double lc, double lahead,
                                           const bool mr[4], const bool mt[4], const real acr[4], const real ctv[4],
                                           bool lr_behind, double csx, double csy, real om, double red[5],
                                           bool diag)
{
    const DescPtr dp = S.dp;
    // the cell's exp(-dt/tau): with TAUF `om`, loaded by march a row ahead
    real omc;
    if constexpr (TAUF)
        omc = om;
    else
        omc = omega_at<real, TAUF>(dp, S.vo, (uint32_t)ir * S.rest_bytes);
    // (1)-(3) moments, weights, f^eq polynomial, BGK and chemical factors
    const Cell<real> C(dp, fc, lc, omc);
    const real rho = C.rho, e = C.e, ux = C.ux, uy = C.uy, u2 = C.u2, T = C.T;
    const real beta = C.beta, omega = C.omega, keep = C.keep, Bz = C.Bz;
    const double Td = C.Td;
    const real *F = C.F;
    const EqPoly<real> &EP = C.EP;

    // azimuthal Courant magnitudes of this row (the geometric 1/r term)
    const double ri = dp->r_min + ((double)ir + 0.5) * dp->dr;
    const real kt = (real)(dp->dt_dth / ri);
    real act[4], aa[4];
#pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
        act[dd] = fabs(ctv[dd]) * kt;
        aa[dd] = acr[dd] + act[dd];
    }

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
        const real rA = rF * (keep + beta * (v * v + u2 - (real)2 * T)), rB = rF * Bz;
        const int base = 1 + 8 * (k - 1);
        // the ring's new values, stored together under one lane mask (in
        // halves where the rotated sector's per-lane plane offsets already
        // hold registers)
        constexpr int G = ROT ? 2 : 4;  // directions dd per store group
        real o[8];
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            real E, O;
            pair_coll(EP, v * EP.w(dd), rA, rB, E, O);
            const real s = omega - v * aa[dd];
#pragma unroll
            for (int sgn = 0; sgn < 2; ++sgn) {
                const int q = base + dd + 4 * sgn;
                const real x = fc[q];
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
                o[dd + 4 * sgn] = dir_new(sgn == 0 ? E + O : E - O, s, x, v, acr[dd], act[dd], nbr, nbt);
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

// Work of one wavefront: strip `strip`, rows [i0, i1), marched outward or,
// with `down`, inward.  prev: this wavefront's [NQ][64] LDS slots.
template <typename real, bool ROT, bool TAUF>
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
    // TAUF: exp(-dt/tau) of the row computed (oc) and of the next (on),
    // loaded a row ahead so that the wavefront does not wait for it
    real oc = (real)0, on = (real)0;
    if constexpr (TAUF) oc = omega_at<real, true>(dp, S.vo, (uint32_t)first * S.rest_bytes);
    S.load_row(first, fc, lc);
    S.load_halo(first, hc, hlc);
    row_or_ghost(S, first + step, fn, ln, fc, lc);
    if (count > 1) S.load_halo(first + step, hn, hln);
    row_or_ghost(S, first - step, fnn, lp, fc, lc);  // the row behind the first
#pragma unroll
    for (int q = 0; q < NQ; ++q) prev[q][lane] = fnn[q];
    if constexpr (TAUF) settle(oc);
    int ir = first;
    for (int n = 0; n < count; ++n, ir += step) {
        // the second row ahead is the radial neighbour of the next row
        // computed, if there is one; rows computed are never ghosts
        if (n + 1 < count) row_or_ghost(S, ir + 2 * step, fnn, lnn, fn, ln);
        if (n + 2 < count) S.load_halo(ir + 2 * step, hnn, hlnn);
        if constexpr (TAUF) {
            if (n + 1 < count) on = omega_at<real, true>(dp, S.vo, (uint32_t)(ir + step) * S.rest_bytes);
        }
        update_row<real, ROT, TAUF>(S, ir, prev, fc, fn, hc, hlc, lp, lc, ln, mr, mt, acr, ctv, !down, cs.x, cs.y, oc,
                                    red, diag);
        oc = on;
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


// Whether step `s` of a solve makes a drift record.
__device__ __forceinline__ bool records(DescPtr dp, int64_t s)
{
    return dp->diag_every > 0 && s >= dp->state->rec_from && s % dp->diag_every == 0;
}

}  // namespace
}  // namespace pdbm
