// Buffer parity of packed solves over a chunk of steps (host side).  The
// state of step s of a solve lives in buffer (s + flip) & 1.  A launch that
// takes a member k steps reads that buffer and leaves the state in the other
// one, so the member's flip toggles when k is even.  The device's k_advance
// applies the same rules to its copy of the flips.
#pragma once

#include <algorithm>
#include <cstdint>

namespace pdbm {

// Two steps per launch over a chunk of n steps (an odd n ends with one
// step): a member with `left` steps to go takes min(left, n) of them, and
// every two-step launch toggles its flip.
inline int pair_chunk_toggle(int64_t left, int64_t n)
{
    return (int)((std::min(std::max<int64_t>(left, 0), n) / 2) & 1);
}

// Launches of min(k, steps of the chunk left) steps over a chunk of n steps
// (single columns, k = COL_K): a member with `left` steps to go takes
// min(k, its steps left) of each launch it is still running in.
inline int column_chunk_toggle(int64_t left, int64_t n, int k)
{
    int t = 0;
    for (int64_t done = 0; done < n && left > 0;) {
        const int64_t run = std::min<int64_t>(k, n - done);
        const int64_t nk = std::min(run, left);
        t ^= (int)((nk + 1) & 1);
        left -= nk;
        done += run;
    }
    return t;
}

}  // namespace pdbm
