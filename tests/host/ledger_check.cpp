// CPU unit test of the request server's admission accounting (pdbm_ledger.h):
// memory in use, request counts and state moves, including the paths that
// reach a request twice (a set-up failure followed by a scheduler error,
// shutdown after retirement).  Exit status 0 when every check holds.
#include <cstdio>

#include "pdbm_ledger.h"

static int fails = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #c); \
            fails++;                                                    \
        }                                                               \
    } while (0)

static bool balanced(const pdbm::Ledger &L)
{
    const pdbm_server_stats &s = L.stats;
    return s.queued >= 0 && s.running >= 0 && s.submitted == s.queued + s.running + s.done + s.failed;
}

int main()
{
    pdbm::Ledger L;
    L.cap = 100;
    int32_t a, b, c, d;
    L.submit(a);
    L.submit(b);
    L.submit(c);
    L.submit(d);
    CHECK(a == PDBM_QUEUED && L.stats.submitted == 4 && L.stats.queued == 4);

    // admission by footprint, first come first served
    CHECK(L.fits(60) && L.admit(a, 60));
    CHECK(!L.fits(50));
    CHECK(L.fits(40) && L.admit(b, 40));
    CHECK(L.in_use == 100 && L.stats.running == 2 && L.stats.queued == 2 && balanced(L));
    CHECK(!L.admit(a, 60));  // already running: refused, nothing changes
    CHECK(L.in_use == 100 && L.stats.running == 2);

    // b's set-up fails: retired as failed, then a scheduler error fails every
    // admitted request again; the second retirement is refused
    CHECK(L.retire(b, 40, false, 0.0));
    CHECK(b == PDBM_FAILED && L.in_use == 60 && L.stats.failed == 1 && L.stats.running == 1);
    CHECK(!L.retire(b, 40, false, 0.0));
    CHECK(b == PDBM_FAILED && L.in_use == 60 && L.stats.failed == 1 && L.stats.running == 1 && balanced(L));

    // a finishes: its cell-updates count, memory comes back once
    CHECK(L.retire(a, 60, true, 1.5e6));
    CHECK(!L.retire(a, 60, false, 0.0));
    CHECK(a == PDBM_DONE && L.in_use == 0 && L.stats.done == 1 && L.stats.cell_updates == 1.5e6);
    CHECK(L.stats.failed == 1 && L.stats.running == 0 && balanced(L));

    // c runs, d is dropped from the queue at shutdown; dropping c (running)
    // or d again changes nothing; a queued request cannot be retired
    CHECK(L.admit(c, 100));
    CHECK(!L.retire(d, 5, true, 1.0));
    CHECK(L.drop(d) && d == PDBM_FAILED && L.stats.queued == 0);
    CHECK(!L.drop(d) && !L.drop(c));
    CHECK(L.retire(c, 100, false, 0.0) && L.in_use == 0);
    CHECK(L.stats.submitted == 4 && L.stats.done == 1 && L.stats.failed == 3 && balanced(L));
    if (fails == 0) std::printf("ledger ok\n");
    return fails ? 1 : 0;
}
