// Admission accounting of the request server: the memory in use, the
// request counts and each request's state moves.  Host-only C++ with no
// device calls, so that it is unit-tested on the CPU; the server calls it
// with its mutex held.
#pragma once

#include <cstddef>
#include <cstdint>

#include "pdbm.h"

namespace pdbm {

struct Ledger {
    size_t cap = 0, in_use = 0;
    pdbm_server_stats stats{};

    // A request joins the queue.
    void submit(int32_t &state)
    {
        state = PDBM_QUEUED;
        stats.submitted++;
        stats.queued++;
    }
    // Whether a request of `bytes` fits beside the running ones.
    bool fits(size_t bytes) const { return in_use + bytes <= cap; }
    // QUEUED -> RUNNING, holding `bytes`.  False (nothing changes) from any
    // other state.
    bool admit(int32_t &state, size_t bytes)
    {
        if (state != PDBM_QUEUED) return false;
        state = PDBM_RUNNING;
        in_use += bytes;
        stats.queued--;
        stats.running++;
        return true;
    }
    // RUNNING -> DONE or FAILED, giving back `bytes`; a finished request
    // adds its cell-updates.  False (nothing changes) from any other state,
    // so a request is retired at most once whatever path reaches it twice.
    bool retire(int32_t &state, size_t bytes, bool ok, double cell_updates)
    {
        if (state != PDBM_RUNNING) return false;
        state = ok ? PDBM_DONE : PDBM_FAILED;
        in_use -= bytes;
        stats.running--;
        if (ok) {
            stats.done++;
            stats.cell_updates += cell_updates;
        } else {
            stats.failed++;
        }
        return true;
    }
    // QUEUED -> FAILED (shutdown, or the scheduler stopped on an error).
    bool drop(int32_t &state)
    {
        if (state != PDBM_QUEUED) return false;
        state = PDBM_FAILED;
        stats.queued--;
        stats.failed++;
        return true;
    }
};

}  // namespace pdbm
