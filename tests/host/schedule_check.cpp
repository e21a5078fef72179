// Checks the host's buffer-parity rules for packed chunks (pdbm_schedule.h)
// against a step-by-step model of the launches a chunk enqueues: at every
// launch the buffer a kernel reads, (step + (flip_i ^ launch flip)) & 1, must
// hold the member's state, and after the chunk the state must sit in
// (new step + new flip) & 1.  A launch that takes a member any number of
// steps reads its buffer and leaves the state in the other one.
#include <cstdio>
#include <cstdlib>

#include "pdbm_schedule.h"

using pdbm::column_chunk_toggle;
using pdbm::pair_chunk_toggle;

static int failures = 0;

static void check(bool ok, const char *what, long base, long nsteps, int flip, long n, int k)
{
    if (!ok && failures++ < 20)
        std::printf("FAIL %s: base %ld nsteps %ld flip %d n %ld k %d\n", what, base, nsteps, flip, n, k);
}

// Launches of up to k steps, each with launch flip pf, which toggles after a
// launch of even length (the column launches of a chunk).
static void column_case(long base, long nsteps, int flip, long n, int k)
{
    int buf = (int)((base + flip) & 1);
    int pf = 0;
    for (long done = 0; done < n;) {
        const long nk = std::min<long>(k, n - done);
        const long s0 = base + done;
        if (s0 < nsteps) {
            check(((s0 + (flip ^ pf)) & 1) == buf, "column launch reads the state", base, nsteps, flip, n, k);
            buf ^= 1;
        }
        pf ^= (int)((nk + 1) & 1);
        done += nk;
    }
    const long left = nsteps > base ? nsteps - base : 0;
    const int nf = flip ^ column_chunk_toggle(left, n, k);
    const long ns = std::min(base + n, std::max(nsteps, base));
    check(((ns + nf) & 1) == buf, "column chunk leaves the parity", base, nsteps, flip, n, k);
}

// Two-step launch i with launch flip i & 1 (a member with one step left
// takes one), and an odd n ending with a launch of single steps.
static void pair_case(long base, long nsteps, int flip, long n)
{
    int buf = (int)((base + flip) & 1);
    for (long i = 0; 2 * i + 1 < n; ++i) {
        const long s0 = base + 2 * i;
        if (s0 < nsteps) {
            check(((s0 + (flip ^ (int)(i & 1))) & 1) == buf, "pair launch reads the state", base, nsteps, flip, n, 2);
            buf ^= 1;
        }
    }
    if (n & 1) {
        const long s0 = base + n - 1;
        if (s0 < nsteps) {
            check(((s0 + (flip ^ (int)((n / 2) & 1))) & 1) == buf, "last single step reads the state", base, nsteps,
                  flip, n, 2);
            buf ^= 1;
        }
    }
    const long left = nsteps > base ? nsteps - base : 0;
    const int nf = flip ^ pair_chunk_toggle(left, n);
    const long ns = std::min(base + n, std::max(nsteps, base));
    check(((ns + nf) & 1) == buf, "pair chunk leaves the parity", base, nsteps, flip, n, 2);
}

int main()
{
    long cases = 0;
    for (long base = 0; base < 4; ++base)
        for (long nsteps = base; nsteps < base + 80; ++nsteps)
            for (int flip = 0; flip < 2; ++flip)
                for (long n = 1; n <= 64; ++n) {
                    for (int k = 1; k <= 8; ++k, ++cases) column_case(base, nsteps, flip, n, k);
                    pair_case(base, nsteps, flip, n);
                    ++cases;
                }
    if (failures) {
        std::printf("%d failures in %ld cases\n", failures, cases);
        return 1;
    }
    std::printf("schedule ok: %ld cases\n", cases);
    return 0;
}
