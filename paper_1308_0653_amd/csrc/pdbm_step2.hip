// Two time steps per launch, in one pass over f (k_step2): solves with more
// than one theta column, full annuli and rotated sectors (annuli and discs),
// single or packed, in float64 (one wavefront per SIMD) and float32 (two).
#include "pdbm_device.h"

namespace pdbm {
namespace {

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

// Drift sums of one step (mass, energy, chemical energy, non-finite and
// non-physical cells; see diag_cell), kept per lane over the whole march and
// added across the wavefront at the end.  In float32 they take 20 of the
// kernel's 256 registers; summing each row across the wavefront at once
// instead (a DPP reduction per row, no registers held) took 1.9 % more time.
struct LaneDiag {
    double red[5] = {0, 0, 0, 0, 0};
    __device__ __forceinline__ void add(bool valid, double rho, double ux, double uy, double T, double e, double lam,
                                        double w, double Q)
    {
        if (valid) diag_cell(red, rho, ux, uy, T, e, lam, w, Q);
    }
    __device__ __forceinline__ double total(int i) const { return wave_sum(red[i]); }
};

// One row of one of the two steps: the arithmetic of update_row, with the
// azimuthal halo from H.  Radial neighbours: the row behind in compact LDS
// slots (of each opposite pair of directions only the one that takes its
// upwind value from behind, slot 4 (k - 1) + (direction mod 4); replaced by
// this row's as they are read), the row ahead in `fn` (stage A) or in the
// full LDS row `ga` (stage B).  STAGEA: the new row goes to `ga` and `lout`,
// for every lane (stage B reads the periodic images too), and the row it
// replaces in `ga` to `gold`, plane by plane, so that the registers of the
// old row fill as those of fc empty; otherwise it is stored, for the strip's
// own columns.
template <typename real, bool STAGEA, bool TAUF, bool ROT, class Halo, class Diag>
__device__ __forceinline__ void stage_row(const Strip<real, ROT> &S, int ir, real (*behind)[64], const real fc[NQ],
                                          const real *fn, real (*ga)[64], real *gold, const Halo &H, double lbehind,
                                          double lc,
                                          double lahead, const bool mr[4], const bool mt[4], const real acr[4],
                                          const real ctv[4], bool lr_behind, double csx, double csy, double &lout,
                                          real om, Diag &D, bool diag)
{
    const DescPtr dp = S.dp;
    // the cell's exp(-dt/tau): with TAUF `om`, loaded by march2 a pass ahead
    real omega;
    if constexpr (TAUF)
        omega = om;
    else
        omega = omega_at<real, TAUF>(dp, S.vo, (uint32_t)ir * S.rest_bytes);
    const Cell<real> C(dp, fc, lc, omega);
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
    const uint32_t rowoff = (uint32_t)ir * S.row_bytes;
    const uint32_t pb = opaque(S.pair_bytes);
    const uint32_t pairs = rowoff + S.rest_bytes;

    // stage B stores from every lane, periodic images into their own
    // column of the row padding (nothing reads it): no store sits under a
    // lane mask, which keeps the exec-mask branches and their registers out
    // of the row loop
    const real rest = C.rest(fc[0]);
    if (STAGEA) {
        gold[0] = ga[0][lane];
        ga[0][lane] = rest;
    } else {
        bstore(rest, S.fout, S.vos, rowoff);
    }
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
        const real v = (real)speed(k);
        const real rF = C.rho * C.F[k];
        const real rA = rF * (C.keep + C.beta * (v * v + C.u2 - (real)2 * C.T)), rB = rF * C.Bz;
        const int base = 1 + 8 * (k - 1);
        real o[8];
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            real E, O;
            pair_coll(C.EP, v * C.EP.w(dd), rA, rB, E, O);
            const real s = C.omega - v * aa[dd];
            const int c = 4 * (k - 1) + dd;
            const real back = behind[c][lane];
            behind[c][lane] = mr[dd] ? fc[base + dd] : fc[base + dd + 4];
#pragma unroll
            for (int sgn = 0; sgn < 2; ++sgn) {
                const int q = base + dd + 4 * sgn;
                const real x = fc[q];
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
                o[dd + 4 * sgn] = dir_new(sgn == 0 ? E + O : E - O, s, x, v, acr[dd], act[dd], nbr, nbt);
            }
        }
        if (STAGEA) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                gold[base + i] = ga[base + i][lane];
                ga[base + i][lane] = o[i];
            }
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

    if (diag) D.add(store, (double)C.rho, uxd, uyd, C.Td, (double)C.e, lc, ri * dp->dr * dp->dth, dp->Q);
}

// The value lane l ^ x holds, x = 1 or 2 (a permutation within each group of
// four lanes).
template <int X>
__device__ __forceinline__ float lane_xor(float v)
{
    constexpr int ctl = X == 1 ? 0xB1 : 0x4E;  // quad_perm [1,0,3,2] or [2,3,0,1]
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctl, 0xf, 0xf, false));
}
template <int X>
__device__ __forceinline__ double lane_xor(double v)
{
    constexpr int ctl = X == 1 ? 0xB1 : 0x4E;
    return __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), ctl, 0xf, 0xf, false),
                            __builtin_amdgcn_mov_dpp(__double2loint(v), ctl, 0xf, 0xf, false));
}
// The sum of v over the LPC lanes of a cell (2 or 4 adjacent lanes).
template <int LPC, typename T>
__device__ __forceinline__ T cell_sum(T v)
{
    v += lane_xor<1>(v);
    if constexpr (LPC == 4) v += lane_xor<2>(v);
    return v;
}

// The intermediate state at the columns bordering strip `strip`, c0 - 1
// (left) and c0 + 64 (right) as periodic images, for the rows [i0, i1) of the
// block.  LPC lanes (2, or 4 for blocks of at most 8 rows) take one cell:
// lane 32 side + LPC e + h takes row i0 + e of its side and the speeds
// 4 h / LPC + 1 .. 4 (h + 1) / LPC (h = 0 also the rest particle).  Of each
// opposite pair of directions only the one that lane 0 (left side) or lane
// 63 (right side) takes from there is kept.  Each lane gathers its pairs of
// the cell (one access per pair) and, for the kept direction of each, its
// two upwind neighbours (radial ghost rules of Sec. II.D included); the
// lanes of a cell add up their partial moments, and each updates its kept
// directions as stage A of the strip owning the column does.  The first
// lane of a cell keeps lambda.  Every lane runs every instruction up to the
// final stores (the moment exchange is a lane permutation).
template <typename real, bool TAUF, int LPC, bool ROT>
__device__ __forceinline__ void edge_cells(const Strip<real, ROT> &S, int strip, int i0, int i1,
                                           real (*ef)[FUSE_ROWS][16], double (*el)[FUSE_ROWS])
{
    static_assert(LPC == 2 || LPC == 4, "two or four lanes per cell");
    constexpr int NP = 16 / LPC;  // pairs per lane
    constexpr int NS = 4 / LPC;   // speeds per lane
    const DescPtr dp = S.dp;
    const int lane = S.lane, side = lane >> 5, e = (lane & 31) / LPC, h = lane & (LPC - 1);
    const int count = i1 - i0;
    const int nr = dp->nr, nt = dp->nt;
    const int r = i0 + min(e, count - 1);  // lanes past the block repeat its last row
    const RowBytes rb{S.row_bytes, S.lrow_bytes, S.rest_bytes, S.pair_bytes};
    // the cell, its radial neighbours (below row 0 the copy of row 0, or at
    // a disc centre row 0 with its directions turned by 4; above row nr - 1
    // the copy of row nr - 1) and its azimuthal neighbours
    const EdgeOffsets o = edge_offsets(nr, nt, dp->sector, ROT, (int)sizeof(real), rb, strip, side, r);
    double2 cs = dp->cs[o.pc], ck = dp->cs[o.pk];
    if constexpr (ROT) {
        // periodic images of a rotated sector: the angles turned by the sector
        cs = turn_cs(cs, (8 - o.tc) & 7);
        ck = turn_cs(ck, (8 - o.tk) & 7);
    }
    const real cth = (real)cs.x, sth = (real)cs.y;
    const real crv[4] = {cth, (real)SQH * (cth + sth), sth, (real)SQH * (sth - cth)};
    const real ctv[4] = {-sth, (real)SQH * (cth - sth), cth, (real)SQH * (cth + sth)};
    const real kcth = (real)ck.x, ksth = (real)ck.y;
    const real kctv[4] = {-ksth, (real)SQH * (kcth - ksth), kcth, (real)SQH * (kcth + ksth)};

    // this lane's pairs NP h .. NP h + NP - 1: directions dd of pair i in
    // x[i], dd + 4 in x[i + NP].  Of each pair only one direction is kept
    // (the one lane 0 or 63 takes from this side: dd + 4 where `second`), so
    // only its upwind neighbours are gathered, one value each: from the lower
    // row if its C_r >= 0, from the left column if its C_theta >= 0
    // (direction dd + 4 has the opposite signs of dd).
    real x[2 * NP], nbr[NP], nbt[NP], x0;
    bool second[NP];
    bload(x0, S.fin, o.x0, 0u);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const uint32_t po = pair_in_row(rb, NP * h + i);
        const int dd = i & 3;
        if constexpr (ROT) {
            second[i] = (kctv[dd] >= (real)0) == (side == 1);
            const bool low = (crv[dd] >= (real)0) != second[i], left = (ctv[dd] >= (real)0) != second[i];
            // each column's data has its directions turned by its shift t:
            // direction dd (dd + 4) of this strip's frame is in the pair of
            // (dd + t) % 4 of the same speed, the members swapped where
            // (dd + t) % 8 >= 4
            const int kb = (NP * h + i) & ~3;
            const uint32_t pc = pair_in_row(rb, kb + ((dd + o.tc) & 3));
            const uint32_t pl = pair_in_row(rb, kb + ((dd + o.tl) & 3));
            const uint32_t pr = pair_in_row(rb, kb + ((dd + o.tr) & 3));
            const bool sc = ((dd + o.tc) & 4) != 0, sl = ((dd + o.tl) & 4) != 0, sr = ((dd + o.tr) & 4) != 0;
            real a, b;
            bload2(a, b, S.fin, o.orow + o.cc + pc, 0u);
            x[i] = sc ? b : a;
            x[i + NP] = sc ? a : b;
            // the radial neighbour's member: below row 0 of a disc the
            // ghost is row 0 with every direction turned by 4
            const bool mc = second[i] != sc, mlr = left ? second[i] != sl : second[i] != sr;
            const bool mlo = mc != (dp->disc && r == 0);
            if constexpr (sizeof(real) == 4) {
                bload(nbr[i], S.fin, (low ? o.olo : o.ohi) + o.cc + pc + ((low ? mlo : mc) ? (uint32_t)sizeof(real) : 0u),
                      0u);
                bload(nbt[i], S.fin, o.orow + (left ? o.cl + pl : o.cr + pr) + (mlr ? (uint32_t)sizeof(real) : 0u),
                      0u);
            } else {
                real lo0, lo1, hi0, hi1, l0, l1, r0, r1;
                bload2(lo0, lo1, S.fin, o.olo + o.cc + pc, 0u);
                bload2(hi0, hi1, S.fin, o.ohi + o.cc + pc, 0u);
                bload2(l0, l1, S.fin, o.orow + o.cl + pl, 0u);
                bload2(r0, r1, S.fin, o.orow + o.cr + pr, 0u);
                nbr[i] = low ? (mlo ? lo1 : lo0) : (mc ? hi1 : hi0);
                nbt[i] = left ? (mlr ? l1 : l0) : (mlr ? r1 : r0);
            }
            continue;
        }
        bload2(x[i], x[i + NP], S.fin, o.orow + o.cc + po, 0u);
        second[i] = (kctv[dd] >= (real)0) == (side == 1);
        const bool low = (crv[dd] >= (real)0) != second[i], left = (ctv[dd] >= (real)0) != second[i];
        if constexpr (sizeof(real) == 4) {
            const uint32_t mo = second[i] ? (uint32_t)sizeof(real) : 0u;  // the member within the pair
            bload(nbr[i], S.fin, (low ? o.olo : o.ohi) + o.cc + po + mo, 0u);
            bload(nbt[i], S.fin, o.orow + (left ? o.cl : o.cr) + po + mo, 0u);
        } else {
            // float64 (one wavefront per SIMD, nothing else to issue while
            // the gathers are in flight): the four neighbour pairs from
            // addresses known up front took less time than two from
            // addresses chosen per lane
            real lo0, lo1, hi0, hi1, l0, l1, r0, r1;
            bload2(lo0, lo1, S.fin, o.olo + o.cc + po, 0u);
            bload2(hi0, hi1, S.fin, o.ohi + o.cc + po, 0u);
            bload2(l0, l1, S.fin, o.orow + o.cl + po, 0u);
            bload2(r0, r1, S.fin, o.orow + o.cr + po, 0u);
            nbr[i] = second[i] ? (low ? lo1 : hi1) : (low ? lo0 : hi0);
            nbt[i] = second[i] ? (left ? l1 : r1) : (left ? l0 : r0);
        }
    }
    double lc, lb, la, lL, lR;
    bload(lc, S.lin, o.lc, 0u);
    bload(lb, S.lin, o.lb, 0u);
    bload(la, S.lin, o.la, 0u);
    bload(lL, S.lin, o.lL, 0u);
    bload(lR, S.lin, o.lR, 0u);

    // moments: this lane's rings (summed as raw_moments does), then the
    // other lanes' added
    real vk[NS];  // this lane's speeds
#pragma unroll
    for (int kk = 0; kk < NS; ++kk) {
        if constexpr (LPC == 2)
            vk[kk] = h == 0 ? (real)speed(1 + kk) : (real)speed(3 + kk);
        else
            vk[kk] = h == 0 ? (real)speed(1) : h == 1 ? (real)speed(2) : h == 2 ? (real)speed(3) : (real)speed(4);
    }
    real rho = h == 0 ? x0 : (real)0, jx = 0, jy = 0, en = 0;
#pragma unroll
    for (int kk = 0; kk < NS; ++kk) {
        const real *g = x + 4 * kk;  // directions 0..3 at g[0..3], 4..7 at g[NP..NP + 3]
        const real v = vk[kk];
        const real ring = ((g[0] + g[NP]) + (g[2] + g[NP + 2])) + ((g[1] + g[NP + 1]) + (g[3] + g[NP + 3]));
        const real a15 = g[1] - g[NP + 1], a37 = g[3] - g[NP + 3];
        const real X = (g[0] - g[NP]) + (real)SQH * (a15 - a37);
        const real Y = (g[2] - g[NP + 2]) + (real)SQH * (a15 + a37);
        rho += ring;
        jx += v * X;
        jy += v * Y;
        en += (real)0.5 * v * v * ring;
    }
    Cell<real> C;
    C.rho = cell_sum<LPC>(rho);
    C.e = cell_sum<LPC>(en);
    C.init_moments(dp, cell_sum<LPC>(jx), cell_sum<LPC>(jy), lc, omega_at<real, TAUF>(dp, o.om, 0u));

    const double ri = dp->r_min + ((double)r + 0.5) * dp->dr;
    const real kr = (real)dp->dt_dr, kt = (real)(dp->dt_dth / ri);
    real g[NP];
#pragma unroll
    for (int kk = 0; kk < NS; ++kk) {
        const real v = vk[kk];
        real Fk;
        if constexpr (LPC == 2)
            Fk = h == 0 ? C.F[1 + kk] : C.F[3 + kk];
        else
            Fk = h == 0 ? C.F[1] : h == 1 ? C.F[2] : h == 2 ? C.F[3] : C.F[4];
        const real rF = C.rho * Fk;
        const real rA = rF * (C.keep + C.beta * (v * v + C.u2 - (real)2 * C.T)), rB = rF * C.Bz;
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) {
            const int i = 4 * kk + dd;
            // the same arithmetic as stage A of the strip owning the column
            const real acr = fabs(crv[dd]) * kr, act = fabs(ctv[dd]) * kt;
            real E, O;
            pair_coll(C.EP, v * C.EP.w(dd), rA, rB, E, O);
            const real s = C.omega - v * (acr + act);
            g[i] = dir_new(second[i] ? E - O : E + O, s, second[i] ? x[i + NP] : x[i], v, acr, act, nbr[i], nbt[i]);
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
        for (int i = 0; i < NP; ++i) ef[side][e][NP * h + i] = g[i];
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

// Fills the compact slots of the row behind (see stage_row) from a full row.
template <typename real>
__device__ __forceinline__ void fill_behind(real (*behind)[64], const real x[NQ], const bool mr[4], int lane)
{
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int dd = 0; dd < 4; ++dd) behind[4 * k + dd][lane] = mr[dd] ? x[1 + 8 * k + dd] : x[5 + 8 * k + dd];
}

// Exchanges two float32 rows of f in registers at the end of a pass.
// Written as plain copies, the loop-carried exchange became three moves per
// value (through a temporary, in three places of the loop); one v_swap_b32
// per value does it (33 instructions instead of 99 per pass).  The s_nop
// gives the two wait states a DPP read of a VGPR needs after a VALU write of
// it, which the compiler does not insert after inline asm.
__device__ __forceinline__ void swap_rows(float (&a)[NQ], float (&b)[NQ])
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) asm("v_swap_b32 %0, %1" : "+v"(a[q]), "+v"(b[q]));
    asm volatile("s_nop 1");
}

// Work of one wavefront of the two-step kernel: strip `strip`, rows [i0, i1)
// (at most FUSE_ROWS), marched outward or, with `down`, inward.  Positions p
// count rows in marching order from the first row of the block (p = 0);
// stage A runs on positions -1 .. R where they are grid rows, stage B on
// 0 .. R - 1, one position behind stage A.  LDS per wavefront: the compact
// rows behind of f (fb) and of g (gb), the full row of g just computed (ga),
// the edge cells (ef, el) and the gathered halo values of stage A's row
// (hb, hbl).
template <typename real, bool TAUF, bool ROT, class Diag>
__device__ __forceinline__ void march2(DescPtr dp, const StepBufs &bufs, int strip, int i0, int i1, bool down,
                                       real (*fb)[64], real (*gb)[64], real (*ga)[64], real (*ef)[FUSE_ROWS][16],
                                       double (*el)[FUSE_ROWS], real *hb, double *hbl, Diag &DA, Diag &DB,
                                       bool diagA, bool diagB)
{
    const Strip<real, ROT> S(dp, bufs, strip);
    const int lane = S.lane;
    double2 cs = dp->cs[S.pc];
    // a periodic image of a rotated sector (its data turned by S.rot): the
    // angle turned by the sector, so that its stage-A row, which stage B of
    // the lanes beside it reads, is in the strip's frame
    if constexpr (ROT) cs = turn_cs(cs, (8 - S.rot) & 7);
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

    // f at positions p (fc) and p + 1 (fn) in registers; f(p + 2) is loaded
    // into fc once stage A has used it, and the two swap at the end of the
    // pass (the loop is not unrolled: a second copy of the pass, which would
    // take the swap away, ran slower, 168 against 157 us per float64 launch
    // and 106 against 103 in float32)
    real fc[NQ], fn[NQ];
    double lp, lc, ln, lx = 0.0;             // lambda of f at positions p-1, p, p+1, p+2
    double glp = 0.0, glc = 0.0, gln = 0.0;  // lambda of g at positions p-2, p-1, p
    GatherHalo<real> hc, hn, hx;
    int p0;
    real t[NQ];  // the row behind stage A's first row
    auto load_first_rows = [&]() {
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
    };
    // the edge cells first: issuing the first rows' loads before their
    // gathers, to wait for memory once, took more time in both precisions
    // (97.7 against 95.1 us per float32 launch), the rows held through the
    // edge cells
    // float32 blocks of up to 8 rows: four lanes per edge cell, so that the
    // 2 x 8 cells keep all 64 lanes busy (93.9 against 95.3 us per launch);
    // float64 keeps two (its 16-row blocks fill the lanes with two; with
    // both forms compiled into its kernel it ran 2 us per launch slower)
    if (sizeof(real) == 4 && i1 - i0 <= 8)
        edge_cells<real, TAUF, 4, ROT>(S, strip, i0, i1, ef, el);
    else
        edge_cells<real, TAUF, 2, ROT>(S, strip, i0, i1, ef, el);
    // TAUF: exp(-dt/tau) of stage A's row (oa), loaded a pass ahead, and of
    // stage B's (ob), the row stage A had a pass before (loaded at the point
    // of use, the field cost 7.2 us per float64 launch and 4.2 us per float32
    // one; loaded ahead, 0.8 and 2.3 us)
    real oa = (real)0, ob = (real)0;
    if constexpr (TAUF)
        oa = omega_at<real, true>(dp, S.vo, (uint32_t)(vlo ? rbefore : first) * S.rest_bytes);
    load_first_rows();
    fill_behind(fb, t, mr, lane);
    if constexpr (TAUF) settle(oa);
    wave_lds_sync();

    for (int p = p0; p <= count; ++p) {
        const int ir = first + p * step;
        // g(p - 1), centre of stage B: stage A hands it over as it replaces
        // it in ga
        real gc[NQ];
        if (p == 0 && vlo) {
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
            stage_row<real, true, TAUF>(S, ir, fb, fc, fn, ga, gc, H, lp, lc, ln, mr, mt, acr, ctv, !down, cs.x, cs.y,
                                        gln, oa, DA, diagA && p >= 0 && p < count);
        } else {
            // beyond the last grid row: the zero-gradient ghost of g (at a
            // disc centre, row 0 with every direction turned by 4)
            if constexpr (ROT) {
                const bool turn = dp->disc && rafter < 0;
                gc[0] = ga[0][lane];
#pragma unroll
                for (int q = 1; q < NQ; ++q) gc[q] = ga[turn ? (((q - 1) ^ 4) + 1) : q][lane];
            } else {
#pragma unroll
                for (int q = 0; q < NQ; ++q) gc[q] = ga[q][lane];
            }
            gln = glc;
        }
        // f at position p + 2 (the row ahead of the next stage A) replaces f(p)
        if (p + 1 < count || (p + 1 == count && vhi)) row_or_ghost(S, ir + 2 * step, fc, lx, fn, ln);
        if (p + 2 < count || (p + 2 == count && vhi)) S.load_halo(ir + 2 * step, hx.h, hx.hl);
        // the next stage A's exp(-dt/tau), where that stage runs on a grid row
        const real oa_used = oa;
        if constexpr (TAUF) {
            if (p + 1 < count || (p + 1 == count && vhi))
                oa = omega_at<real, true>(dp, S.vo, (uint32_t)(ir + step) * S.rest_bytes);
        }
        // (B) second step at position p - 1
        if (p == 0 && !vlo) {
            // the row behind stage B's first row is the (zero-gradient)
            // ghost of g(0) (at a disc centre with every direction turned by
            // 4: the slot of direction dd takes g(0)'s direction dd + 4)
            if constexpr (ROT) {
                const bool turn = dp->disc && rbefore < 0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int dd = 0; dd < 4; ++dd)
                        gb[4 * k + dd][lane] = mr[dd] != turn ? ga[1 + 8 * k + dd][lane] : ga[5 + 8 * k + dd][lane];
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int dd = 0; dd < 4; ++dd)
                        gb[4 * k + dd][lane] = mr[dd] ? ga[1 + 8 * k + dd][lane] : ga[5 + 8 * k + dd][lane];
            }
            glc = gln;
        } else if (p > 0) {
            const int e = ir - step - i0;
            const EdgeHalo<real> H{ef[0][e], ef[1][e], el[0][e], el[1][e]};
            double unused;
            stage_row<real, false, TAUF>(S, ir - step, gb, gc, nullptr, ga, nullptr, H, glp, glc, gln, mr, mt, acr, ctv,
                                         !down, cs.x, cs.y, unused, ob, DB, diagB);
        }
        if constexpr (sizeof(real) == 4) {
            swap_rows(fc, fn);
        } else {
            // float64: one 64-bit move per copy (the same exchange moved into
            // a function came out with 90 more AGPR moves per pass)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const real t = fc[q];
                fc[q] = fn[q];
                fn[q] = t;
            }
        }
        ob = oa_used;
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

// Wavefronts per SIMD of the two-step kernel: one in float64, whose two
// steps' rows fill the register file, two in float32.
template <typename real>
struct Step2Occ {
    static constexpr int waves = sizeof(real) == 4 ? 2 : 1;
};

// Steps s and s + 1 of every solve of the launch in one pass over f.  Tiles,
// step bases and step_off as k_step's (a single solve passes no tile table,
// so wavefront t takes its tile t, and no bases, so s = step_off).  The state
// of step s of solve i is in buffer (s + flip_i) & 1 with flip_i = flips[i]
// ^ flip (flips may be NULL); a two-step launch leaves it in the other
// buffer, so the caller toggles flip_i after it.  A solve with one step left,
// or every solve when `single` is set, takes one step instead (the one-step
// march), which keeps the parity.  One wavefront per SIMD in float64, where
// the two steps' rows fill the register file and the LDS rows of four
// wavefronts most of a CU's LDS; two in float32, whose rows take half the
// LDS.  ROT: solves of rotated sectors, discs included, whose periodic
// images have their directions and angles turned by the sector.
template <typename real, bool TAUF, bool ROT>
__global__ __launch_bounds__(BLOCK, Step2Occ<real>::waves) void k_step2(const SolveDesc *descs, const uint2 *tiles,
                                                                       int ntiles, const int64_t *bases,
                                                                       int64_t step_off, const int *flips, int flip,
                                                                       int single)
{
    const int nb = gridDim.x;
    const int blk = xcd_tile(blockIdx.x, nb);
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
    const int cur = (int)((step + ((flips ? flips[solve] : 0) ^ flip)) & 1);
    const StepBufs bufs{dp->f[cur], dp->f[cur ^ 1], dp->lam[cur], dp->lam[cur ^ 1]};
    __shared__ real fb[BLOCK / 64][16][64];
    __shared__ real gb[BLOCK / 64][16][64];
    __shared__ real ga[BLOCK / 64][NQ][64];
    __shared__ real ef[BLOCK / 64][2][FUSE_ROWS][16];
    __shared__ double el[BLOCK / 64][2][FUSE_ROWS];
    __shared__ real hb[BLOCK / 64][66];
    __shared__ double hbl[BLOCK / 64][2];
    const int w = threadIdx.x >> 6;
    const int rows = dp->rows, nstrip = dp->nstrip;
    const int rb = lt / nstrip, strip = lt - rb * nstrip;
    const int i0 = rb * rows;
    const int i1 = min(i0 + rows, dp->nr);
    if (single || step + 1 >= dp->nsteps) {
        // one step, with the row behind in the LDS row of g
        const bool diag = records(dp, step);
        double red[5] = {0, 0, 0, 0, 0};
        march<real, ROT, TAUF>(dp, bufs, strip, i0, i1, (rb & 1) != 0, ga[w], red, diag);
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
        return;
    }
    const bool diagA = records(dp, step), diagB = records(dp, step + 1);
    LaneDiag DA, DB;
    march2<real, TAUF, ROT>(dp, bufs, strip, i0, i1, (rb & 1) != 0, fb[w], gb[w], ga[w], ef[w], el[w], hb[w], hbl[w],
                            DA, DB, diagA, diagB);
    // both steps' totals first (independent DPP chains the compiler can
    // interleave), then one lane stores them
    double v[2][5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        v[0][i] = diagA ? DA.total(i) : 0.0;
        v[1][i] = diagB ? DB.total(i) : 0.0;
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!(s == 0 ? diagA : diagB)) continue;
            const int64_t slot = ((step + s) / dp->diag_every) % PART_RING;
            double *part = dp->wpart + ((size_t)slot * dp->nwaves + lt) * 5;
#pragma unroll
            for (int i = 0; i < 5; ++i) part[i] = v[s][i];
        }
    }
}

}  // namespace

template <typename real, bool TAUF, bool ROT>
static void launch_k_step2(int nb, hipStream_t st, const SolveDesc *descs, const uint2 *tiles, int ntiles,
                           const int64_t *bases, int64_t step_off, const int *flips, int flip, bool single)
{
    hipLaunchKernelGGL((k_step2<real, TAUF, ROT>), dim3(nb), dim3(BLOCK), 0, st, descs, tiles, ntiles, bases, step_off,
                       flips, flip, (int)single);
}

hipError_t launch_step2(const SolveDesc *descs, const uint2 *tiles, int ntiles, const int64_t *bases,
                        int64_t step_off, const int *flips, int flip, bool single, bool fp32, bool tauf, bool rot,
                        hipStream_t st)
{
    const int nb = (ntiles + BLOCK / 64 - 1) / (BLOCK / 64);
    if (nb == 0) return hipSuccess;
    auto *fn = fp32 ? (rot ? (tauf ? &launch_k_step2<float, true, true> : &launch_k_step2<float, false, true>)
                           : (tauf ? &launch_k_step2<float, true, false> : &launch_k_step2<float, false, false>))
                    : (rot ? (tauf ? &launch_k_step2<double, true, true> : &launch_k_step2<double, false, true>)
                           : (tauf ? &launch_k_step2<double, true, false> : &launch_k_step2<double, false, false>));
    fn(nb, st, descs, tiles, ntiles, bases, step_off, flips, flip, single);
    return hipGetLastError();
}

}  // namespace pdbm
