// Byte offsets of the raw buffer accesses of the step kernels: plain integer
// arithmetic, shared by the kernels (pdbm_device.h, pdbm_step.hip,
// pdbm_step2.hip) and by the host bounds check (tests/host/offsets_check.cpp,
// built with g++ from this header), which evaluates the same functions for
// every lane, strip and row of a grid and checks each access against its
// buffer.
//
// A buffer access reads or writes at base + so + vo, so = a scalar (row)
// offset, vo = a per-lane offset, both 32-bit: each f buffer stays below
// 4 GiB (checked at create).
#pragma once

#include <stdint.h>

#include "pdbm_internal.h"

namespace pdbm {

constexpr int ROT_NONE = 0;

// Memory plane of velocity q for data whose direction index is shifted by r.
__host__ __device__ constexpr int plane_of(int q, int r)
{
    return q == 0 ? 0 : 1 + 8 * ((q - 1) / 8) + ((((q - 1) % 8) + r) & 7);
}

// Row strides of one solve, in bytes.
struct RowBytes {
    uint32_t row;   // one r row of f: NQ planes of pitch values
    uint32_t lrow;  // one r row of lambda: pitch doubles
    uint32_t rest;  // the rest particle's plane (pitch values); also one row of the per-cell tau field
    uint32_t pair;  // one pair of opposite directions (2 pitch values)
};
__host__ __device__ inline RowBytes row_bytes_of(int64_t rstride, int64_t pitch, int esz)
{
    RowBytes b;
    b.row = (uint32_t)rstride * (uint32_t)esz;
    b.lrow = (uint32_t)pitch * 8u;
    b.rest = (uint32_t)pitch * (uint32_t)esz;
    b.pair = 2u * b.rest;
    return b;
}

// Per-lane offsets of a wavefront strip (see Strip in pdbm_device.h): lane
// `lane` of strip `strip` owns column c0 + lane, c0 = 64 strip, or its
// periodic image (the data of physical column pc, directions turned by
// `rot` in a rotated sector).
struct StripOffsets {
    uint32_t vo, vo2, vol;     // this lane's physical column: rest plane, pair, lambda
    uint32_t vos, vos2, vols;  // ... of its own column (the padding for periodic images)
    uint32_t vh1, vh2, vhl;    // halo gathers (plane and column)
    uint32_t poff[4];          // rotated sectors: pair holding this lane's directions dd, dd + 4
    bool pswap[4];             // ... and whether its members come in the other order
    int pc, rot;
    bool useful;               // the lane holds a grid column (not an image)
};
__host__ __device__ inline StripOffsets strip_offsets(int nt, int64_t pitch, int sector, bool rotated, int esz,
                                                      const RowBytes &b, int strip, int lane)
{
    StripOffsets o;
    const int c0 = strip * STRIP;
    const int col = c0 + lane;
    // lanes past the last column hold periodic images of the first ones
    const int wraps = col / nt;
    o.pc = col - wraps * nt;
    o.rot = rotated ? ((-wraps * sector) & 7) : ROT_NONE;
    o.useful = col < nt;
    o.vo = (uint32_t)o.pc * (uint32_t)esz;
    o.vo2 = 2u * o.vo;
    o.vol = (uint32_t)o.pc * 8u;
    o.vos = (uint32_t)col * (uint32_t)esz;
    o.vos2 = 2u * o.vos;
    o.vols = (uint32_t)col * 8u;
    for (int dd = 0; dd < 4; ++dd) {
        // direction dd of this lane's data is direction (dd + rot) % 8
        o.poff[dd] = o.vo2 + b.rest + (uint32_t)((dd + o.rot) & 3) * b.pair;
        o.pswap[dd] = ((dd + o.rot) & 4) != 0;
    }
    // halo columns: c0 - 1 (0 <= c0 < nt) and c0 + 64, as periodic images
    const int cl = c0 == 0 ? nt - 1 : c0 - 1;
    const int rl = rotated && c0 == 0 ? (sector & 7) : 0;
    const int wr = (c0 + STRIP) / nt;
    const int cr = c0 + STRIP - wr * nt;
    const int rr = rotated ? ((-wr * sector) & 7) : 0;
    // gather 1: lanes 0..32 left halo of planes 0..32, lanes 33..63 right
    // halo of planes 0..30; gather 2: lanes 0, 1 right halo of planes 31,
    // 32; lambda gather: lane 0 left, lane 1 right (other lanes repeat a
    // valid address)
    o.vh1 = lane <= 32 ? (uint32_t)elem_of(plane_of(lane, rl), cl, pitch) * (uint32_t)esz
                       : (uint32_t)elem_of(plane_of(lane - 33, rr), cr, pitch) * (uint32_t)esz;
    o.vh2 = lane < 2 ? (uint32_t)elem_of(plane_of(31 + lane, rr), cr, pitch) * (uint32_t)esz
                     : (uint32_t)cl * (uint32_t)esz;
    o.vhl = lane == 1 ? (uint32_t)cr * 8u : (uint32_t)cl * 8u;
    return o;
}

// floor(c / n) for n > 0: the periodic image a strip column c belongs to.
__host__ __device__ constexpr int wraps_of(int c, int n) { return c >= 0 ? c / n : -((n - 1 - c) / n); }

// Cells of the two-step kernel's strip edges (edge_cells in pdbm_step2.hip):
// lane 32 side + 2 e + h takes row r of the column bordering strip `strip`
// on `side` (0: left, 1: right) and gathers the cell (row r, column pc), its
// radial neighbours (rows rlo, rhi: zero-gradient ghosts at the ends) and
// its azimuthal neighbours (columns pl, pr).  Those columns, in the strip's
// own numbering, may be periodic images: in a rotated sector their data has
// its directions turned (tc, tl, tr, as `rot` in strip_offsets), and the
// cell's and lane 0 / 63's angles are those of the physical columns pc and
// pk turned by the sector (tc, tk).
struct EdgeOffsets {
    int pc, pl, pr, pk;            // the cell's column, its left and right neighbours, the column of lane 0 / 63
    int tc, tl, tr, tk;            // direction shifts of the data of those columns in the strip's frame
    int rlo, rhi;                  // rows of its radial neighbours
    uint32_t orow, olo, ohi;       // row offsets of f: the cell's row and its radial neighbours
    uint32_t cc, cl, cr;           // pair-column offsets of f: pc, pl, pr
    uint32_t x0;                   // the rest particle of the cell
    uint32_t lc, lb, la, lL, lR;   // lambda: the cell, below, above, left, right
    uint32_t om;                   // the cell's entry of the per-cell tau field
};
__host__ __device__ inline EdgeOffsets edge_offsets(int nr, int nt, int sector, bool rotated, int esz,
                                                    const RowBytes &b, int strip, int side, int r)
{
    EdgeOffsets o;
    const int c0 = strip * STRIP;
    if (!rotated) {
        o.pc = side == 0 ? (c0 + nt - 1) % nt : (c0 + STRIP) % nt;
        o.pl = (o.pc + nt - 1) % nt;
        o.pr = (o.pc + 1) % nt;
        o.pk = (side == 0 ? c0 : c0 + STRIP - 1) % nt;
        o.tc = o.tl = o.tr = o.tk = ROT_NONE;
    } else {
        const int c = side == 0 ? c0 - 1 : c0 + STRIP, k = side == 0 ? c0 : c0 + STRIP - 1;  // strip numbering
        const int wc = wraps_of(c, nt), wl = wraps_of(c - 1, nt), wr = wraps_of(c + 1, nt), wk = wraps_of(k, nt);
        o.pc = c - wc * nt;
        o.pl = (c - 1) - wl * nt;
        o.pr = (c + 1) - wr * nt;
        o.pk = k - wk * nt;
        o.tc = (-wc * sector) & 7;
        o.tl = (-wl * sector) & 7;
        o.tr = (-wr * sector) & 7;
        o.tk = (-wk * sector) & 7;
    }
    o.rlo = r - 1 < 0 ? 0 : r - 1;
    o.rhi = r + 1 > nr - 1 ? nr - 1 : r + 1;
    const uint32_t es = (uint32_t)esz;
    o.orow = (uint32_t)r * b.row;
    o.olo = (uint32_t)o.rlo * b.row;
    o.ohi = (uint32_t)o.rhi * b.row;
    o.cc = 2u * (uint32_t)o.pc * es;
    o.cl = 2u * (uint32_t)o.pl * es;
    o.cr = 2u * (uint32_t)o.pr * es;
    o.x0 = o.orow + (uint32_t)o.pc * es;
    o.lc = (uint32_t)r * b.lrow + (uint32_t)o.pc * 8u;
    o.lb = (uint32_t)o.rlo * b.lrow + (uint32_t)o.pc * 8u;
    o.la = (uint32_t)o.rhi * b.lrow + (uint32_t)o.pc * 8u;
    o.lL = (uint32_t)r * b.lrow + (uint32_t)o.pl * 8u;
    o.lR = (uint32_t)r * b.lrow + (uint32_t)o.pr * 8u;
    o.om = (uint32_t)o.pc * es + (uint32_t)r * b.rest;
    return o;
}
// Offset of pair i (0..15) within a row of f (column 0).
__host__ __device__ inline uint32_t pair_in_row(const RowBytes &b, int i) { return b.rest + (uint32_t)i * b.pair; }

// The one-step single-column kernel (radial_block in pdbm_step.hip): lane l
// of block blk holds row re = min(COL_W blk + l, nr - 1) of column 0 (it
// owns the rows of lanes below COL_W) and gathers the row below the block
// (rlo, directions turned by `tlo` at the disc centre) and the row 64 above
// its first (rhi).
struct RadialOffsets {
    int re, rlo, rhi;
    uint32_t vo, vol;     // the lane's row: f and lambda
    uint32_t vh1, vh2, vhl;  // gathers of the rows bounding the block
    uint32_t om;             // the lane's entry of the per-cell tau field
};
__host__ __device__ inline RadialOffsets radial_offsets(int nr, int64_t pitch, bool disc, int esz, const RowBytes &b,
                                                        int blk, int lane)
{
    RadialOffsets o;
    const int r0 = blk * COL_W;
    const int row = r0 + lane;
    o.re = row < nr - 1 ? row : nr - 1;  // lanes past the last row hold its zero-gradient image
    o.rlo = r0 == 0 ? 0 : r0 - 1;
    o.rhi = r0 + 64 < nr - 1 ? r0 + 64 : nr - 1;
    const int tlo = r0 == 0 && disc ? 4 : 0;
    const uint32_t es = (uint32_t)esz;
    o.vo = (uint32_t)o.re * b.row;
    o.vol = (uint32_t)o.re * b.lrow;
    o.vh1 = lane <= 32 ? (uint32_t)o.rlo * b.row + (uint32_t)elem_of(plane_of(lane, tlo), 0, pitch) * es
                       : (uint32_t)o.rhi * b.row + (uint32_t)elem_of(lane - 33, 0, pitch) * es;
    o.vh2 = lane < 2 ? (uint32_t)o.rhi * b.row + (uint32_t)elem_of(31 + lane, 0, pitch) * es
                     : (uint32_t)o.rlo * b.row;
    o.vhl = lane == 1 ? (uint32_t)o.rhi * b.lrow : (uint32_t)o.rlo * b.lrow;
    o.om = (uint32_t)o.re * b.rest;
    return o;
}

// The multi-step single-column kernel (k_column in pdbm_step.hip): lane l
// of wavefront t holds row r0 - COL_K + l, r0 = COL_W t, whose data it
// loads from row re (the row clamped to the grid: rows outside it start as
// their radial ghosts), and owns it if it is one of rows r0 .. r0 + COL_W - 1
// of the grid (then it stores the new state there).
struct ColumnOffsets {
    int row, re;
    bool own;
    uint32_t vo, vol, om;  // f (rest plane of the row; pairs follow), lambda, the per-cell tau field
};
__host__ __device__ inline ColumnOffsets column_offsets(int nr, const RowBytes &b, int t, int lane)
{
    ColumnOffsets o;
    const int r0 = t * COL_W;
    o.row = r0 - COL_K + lane;
    o.re = o.row < 0 ? 0 : o.row > nr - 1 ? nr - 1 : o.row;
    o.own = lane >= COL_K && lane < COL_K + COL_W && o.row < nr;
    o.vo = (uint32_t)o.re * b.row;
    o.vol = (uint32_t)o.re * b.lrow;
    o.om = (uint32_t)o.re * b.rest;
    return o;
}

}  // namespace pdbm
