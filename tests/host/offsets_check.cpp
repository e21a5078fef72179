// Host bounds check of the step kernels' buffer accesses (the PDBM_CHECK
// build): for a list of grids, evaluates the kernels' own offset functions
// (pdbm_offsets.h) for every strip, lane and row, as the one-step kernel,
// the two-step kernel (with its strip-edge cells) and the single-column
// kernel form them, and checks that every access -- the 32-bit sum of its
// scalar and per-lane offsets plus its width -- lies inside its buffer (two
// f buffers of 33 x nr x pitch values, lambda of nr x pitch doubles, the
// per-cell tau field of nr x pitch values) and that no 32-bit offset product
// wraps.  Rows outside [0, nr) are never loaded (the kernels build ghost
// rows from the boundary row in registers), so rows 0 .. nr - 1 cover every
// access.  Exit status 0 when every access is in bounds.
//
//   offsets_check                 the built-in list (the largest grids of
//                                 each kind, the strip-edge test widths,
//                                 the benchmark workloads)
//   offsets_check NR NT SECTOR ESZ  one grid
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pdbm_offsets.h"

using namespace pdbm;

namespace {

long long n_checked = 0;
int n_failed = 0;

struct Grid {
    int nr, nt, sector, esz;
};

// One access of `width` bytes at so + vo in a buffer of `bytes` bytes; so
// and vo are the kernel's 32-bit operands, so64 the same scalar offset in
// 64-bit arithmetic.
void access(const Grid &g, const char *what, uint64_t so64, uint32_t so, uint32_t vo, uint32_t width, uint64_t bytes,
            int a, int b)
{
    ++n_checked;
    const uint64_t start = so64 + vo;
    if (so64 != so || start >= (uint64_t(1) << 32) || start + width > bytes) {
        if (n_failed++ < 20)
            std::fprintf(stderr, "OUT OF BOUNDS %s: grid %dx%d sector %d esz %d (%d, %d): so=%llu vo=%u width=%u, buffer %llu\n",
                         what, g.nr, g.nt, g.sector, g.esz, a, b, (unsigned long long)so64, vo, width,
                         (unsigned long long)bytes);
    }
}

void check_grid(const Grid &g)
{
    const int64_t pitch = g.nt == 1 ? 2 : (g.nt + STRIP - 1) / STRIP * STRIP;
    const int64_t rstride = (int64_t)NQ * pitch;
    const uint64_t F = (uint64_t)g.nr * rstride * g.esz, L = (uint64_t)g.nr * pitch * 8,
                   OM = (uint64_t)g.nr * pitch * g.esz;
    const RowBytes b = row_bytes_of(rstride, pitch, g.esz);
    const uint32_t es = (uint32_t)g.esz;
    const bool rotated = g.sector != 8;
    if (g.nt == 1) {
        // single column, several steps per launch (k_column): every lane
        // loads its row clamped to the grid, owned lanes store there, and
        // every row is owned exactly once
        std::vector<int> owners(g.nr, 0);
        for (int t = 0; t * COL_W < g.nr; ++t)
            for (int lane = 0; lane < 64; ++lane) {
                const ColumnOffsets o = column_offsets(g.nr, b, t, lane);
                if (o.own && o.row >= 0 && o.row < g.nr) ++owners[o.row];
            }
        for (int r = 0; r < g.nr; ++r) {
            ++n_checked;
            if (owners[r] != 1 && n_failed++ < 20) std::fprintf(stderr, "column row %d owned %d times\n", r, owners[r]);
        }
        for (int t = 0; t * COL_W < g.nr; ++t)
            for (int lane = 0; lane < 64; ++lane) {
                const ColumnOffsets o = column_offsets(g.nr, b, t, lane);
                access(g, "column rest", 0, 0, o.vo, es, F, t, lane);
                for (int c = 0; c < 16; ++c)
                    access(g, "column pair", b.rest + (uint64_t)c * b.pair, b.rest + (uint32_t)c * b.pair, o.vo,
                           2 * es, F, t, lane);
                access(g, "column lambda", 0, 0, o.vol, 8, L, t, lane);
                access(g, "column tau field", 0, 0, o.om, es, OM, t, lane);
                if (o.own && (o.row < 0 || o.row >= g.nr)) {
                    if (n_failed++ < 20) std::fprintf(stderr, "column lane %d of wavefront %d owns row %d\n", lane, t, o.row);
                }
            }
        // single column, one step per launch in packs: lanes along r (radial_block)
        const bool disc = false;
        for (int blk = 0; blk * COL_W < g.nr; ++blk)
            for (int lane = 0; lane < 64; ++lane) {
                const RadialOffsets o = radial_offsets(g.nr, pitch, disc, g.esz, b, blk, lane);
                access(g, "radial rest", 0, 0, o.vo, es, F, blk, lane);
                for (int c = 0; c < 16; ++c)
                    access(g, "radial pair", b.rest + (uint64_t)c * b.pair, b.rest + (uint32_t)c * b.pair, o.vo,
                           2 * es, F, blk, lane);
                access(g, "radial lambda", 0, 0, o.vol, 8, L, blk, lane);
                access(g, "radial gather 1", 0, 0, o.vh1, es, F, blk, lane);
                access(g, "radial gather 2", 0, 0, o.vh2, es, F, blk, lane);
                access(g, "radial lambda gather", 0, 0, o.vhl, 8, L, blk, lane);
                access(g, "radial tau field", 0, 0, o.om, es, OM, blk, lane);
                // stores: the lane's own row (lanes past the last row do not store)
            }
        return;
    }
    const int nstrip = (int)((g.nt + STRIP - 1) / STRIP);
    for (int strip = 0; strip < nstrip; ++strip)
        for (int lane = 0; lane < 64; ++lane) {
            const StripOffsets o = strip_offsets(g.nt, pitch, g.sector, rotated, g.esz, b, strip, lane);
            for (int row = 0; row < g.nr; ++row) {
                const uint64_t so64 = (uint64_t)row * b.row;
                const uint32_t so = (uint32_t)row * b.row;
                const uint64_t lso64 = (uint64_t)row * b.lrow;
                const uint32_t lso = (uint32_t)row * b.lrow;
                // load_row
                access(g, "rest", so64, so, o.vo, es, F, strip, lane);
                for (int c = 0; c < 16; ++c) {
                    if (rotated) {
                        const int k = c >> 2, dd = c & 3;
                        access(g, "rotated pair", so64 + (uint64_t)k * 4 * b.pair, so + (uint32_t)k * 4u * b.pair,
                               o.poff[dd], 2 * es, F, strip, lane);
                    } else {
                        access(g, "pair", so64 + b.rest + (uint64_t)c * b.pair, so + b.rest + (uint32_t)c * b.pair,
                               o.vo2, 2 * es, F, strip, lane);
                    }
                }
                access(g, "lambda", lso64, lso, o.vol, 8, L, strip, lane);
                // load_halo
                access(g, "halo gather 1", so64, so, o.vh1, es, F, strip, lane);
                access(g, "halo gather 2", so64, so, o.vh2, es, F, strip, lane);
                access(g, "lambda halo", lso64, lso, o.vhl, 8, L, strip, lane);
                // stores of the new state (every lane: images into their own padding column)
                access(g, "rest store", so64, so, o.vos, es, F, strip, lane);
                for (int c = 0; c < 16; ++c)
                    access(g, "pair store", so64 + b.rest + (uint64_t)c * b.pair, so + b.rest + (uint32_t)c * b.pair,
                           o.vos2, 2 * es, F, strip, lane);
                access(g, "lambda store", lso64, lso, o.vols, 8, L, strip, lane);
                // per-cell tau field
                access(g, "tau field", (uint64_t)row * b.rest, (uint32_t)row * b.rest, o.vo, es, OM, strip, lane);
            }
        }
    // the two-step kernel's edge cells (rotated sectors: the pair of each
    // column's turned directions, one of the 16 checked here)
    for (int strip = 0; strip < nstrip; ++strip)
        for (int side = 0; side < 2; ++side)
            for (int r = 0; r < g.nr; ++r) {
                const EdgeOffsets o = edge_offsets(g.nr, g.nt, g.sector, rotated, g.esz, b, strip, side, r);
                for (int t : {o.tc, o.tl, o.tr, o.tk})
                    if ((t < 0 || t > 7) && n_failed++ < 20)
                        std::fprintf(stderr, "edge direction shift %d: strip %d row %d\n", t, strip, r);
                for (int pcol : {o.pc, o.pl, o.pr, o.pk})
                    if ((pcol < 0 || pcol >= g.nt) && n_failed++ < 20)
                        std::fprintf(stderr, "edge column %d outside the grid: strip %d row %d\n", pcol, strip, r);
                access(g, "edge rest", 0, 0, o.x0, es, F, strip, r);
                for (int i = 0; i < 16; ++i) {
                    const uint32_t po = pair_in_row(b, i);
                    access(g, "edge pair", 0, 0, o.orow + o.cc + po, 2 * es, F, strip, r);
                    // one member (either) of the upwind neighbours' pairs
                    for (uint32_t mo : {0u, es}) {
                        access(g, "edge member below", 0, 0, o.olo + o.cc + po + mo, es, F, strip, r);
                        access(g, "edge member above", 0, 0, o.ohi + o.cc + po + mo, es, F, strip, r);
                        access(g, "edge member left", 0, 0, o.orow + o.cl + po + mo, es, F, strip, r);
                        access(g, "edge member right", 0, 0, o.orow + o.cr + po + mo, es, F, strip, r);
                    }
                    // the per-lane sums above must not wrap either
                    const uint64_t far = (uint64_t)o.ohi + o.cc + po + es;
                    access(g, "edge sum", far, (uint32_t)far, 0, es, F, strip, r);
                }
                for (uint32_t lo : {o.lc, o.lb, o.la, o.lL, o.lR}) access(g, "edge lambda", 0, 0, lo, 8, L, strip, r);
                access(g, "edge tau field", 0, 0, o.om, es, OM, strip, r);
            }
}

}  // namespace

int main(int argc, char **argv)
{
    std::vector<Grid> grids;
    if (argc == 5) {
        grids.push_back({std::atoi(argv[1]), std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4])});
    } else {
        // the largest grid of each kind: float64 4034 x 4000 (f 1 MB under
        // 4 GiB, ragged last strip), float32 4096 x 4096 (2^24 cells),
        // float64 single column of 8134407 rows (400 bytes under 4 GiB)
        grids.push_back({4034, 4000, 8, 8});
        grids.push_back({4096, 4096, 8, 4});
        grids.push_back({8134407, 1, 8, 8});
        // the strip-edge test widths, each row count, both precisions, and
        // the rotated sectors they run
        for (int nt : {1, 2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 200})
            for (int nr : {1, 2, 5, 33})
                for (int esz : {4, 8}) grids.push_back({nr, nt, 8, esz});
        for (int esz : {4, 8}) {
            grids.push_back({6, 65, 1, esz});
            grids.push_back({6, 130, 3, esz});
            grids.push_back({6, 17, 5, esz});
            grids.push_back({6, 64, 2, esz});
        }
        // the benchmark's workloads: the outward 1024^2 detonation, the
        // sweep's largest member, the serving stream's largest request
        for (int esz : {4, 8}) grids.push_back({1024, 1024, 8, esz});
        grids.push_back({986, 462, 8, 4});
        grids.push_back({2015, 1935, 8, 4});
    }
    for (const Grid &g : grids) check_grid(g);
    std::printf("%lld accesses on %zu grids, %d out of bounds\n", n_checked, grids.size(), n_failed);
    return n_failed ? 1 : 0;
}
