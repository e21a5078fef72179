// Packed launches over many independent solves: a fixed batch (pdbm_batch)
// and continuous batching of a request stream (pdbm_server).
//
// Every member keeps its own state resident in HBM.  One launch of the step
// kernel advances all members by one step: its wavefront tiles are the
// concatenation of the members' tiles, mapped back to (member, tile) by a
// device table.  Member i takes step bases[i] + (the launch's place in the
// chunk); a small kernel at the end of a chunk adds up the chunk's drift
// records and advances bases[] by the chunk, so a chunk of launches is
// captured once in a hipGraph and replayed; membership changes only between
// chunks.  Members never read each other's data, so a solve's fields are the
// same bit for bit alone or in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pdbm_host.h"
#include "pdbm_ledger.h"
#include "pdbm_schedule.h"

using namespace pdbm;

#define HIPCHK PDBM_HIPCHK

namespace {

// A set of solves of one precision stepped together.
class Pack {
  public:
    bool fp32 = false;
    std::vector<Solve *> members;
    bool dirty = true;

    ~Pack() { destroy(); }

    // Uploads the description, step-base, buffer-parity and tile tables of
    // the current members and drops the captured graph.  The tables hold the
    // grids of more than one column first (nwide of them, nwt tiles), then
    // the single columns (Solve::columnar).  The wide ones step in pairs when
    // every one of them may (Solve::fusable), with the variant for rotated
    // sectors when one is, else one step per launch; the columns up to COL_K
    // steps per launch of their own kernel.  Synchronises st.
    int rebuild(hipStream_t st)
    {
        drop_graph();
        rot = false;
        pairs = true;
        std::vector<SolveDesc> descs;
        std::vector<uint2> tiles;
        bases_host.clear();
        flips_host.clear();
        nwide = nwt = 0;
        for (int pass = 0; pass < 2; ++pass) {
            for (Solve *m : members) {
                if (m->columnar() != (pass == 1)) continue;
                const unsigned i = (unsigned)descs.size();
                descs.push_back(m->hd);
                bases_host.push_back(m->step);
                flips_host.push_back(m->flip);
                if (pass == 0) {
                    rot = rot || m->rot();
                    pairs = pairs && m->fusable();
                }
                for (int t = 0; t < m->waves(); ++t) tiles.push_back(make_uint2(i, (unsigned)t));
            }
            if (pass == 0) {
                nwide = (int)descs.size();
                nwt = (int)tiles.size();
            }
        }
        ntiles = (int)tiles.size();
        int rc = grow((void **)&ddescs, cap_descs, descs.size() * sizeof(SolveDesc));
        if (rc == PDBM_OK) rc = grow((void **)&dtiles, cap_tiles, tiles.size() * sizeof(uint2));
        if (rc == PDBM_OK) rc = grow((void **)&dbases, cap_bases, bases_host.size() * sizeof(int64_t));
        if (rc == PDBM_OK) rc = grow((void **)&dflips, cap_flips, flips_host.size() * sizeof(int));
        if (rc) return rc;
        if (!descs.empty()) {
            HIPCHK(hipMemcpyAsync(ddescs, descs.data(), descs.size() * sizeof(SolveDesc), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(dbases, bases_host.data(), bases_host.size() * sizeof(int64_t),
                                  hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(dflips, flips_host.data(), flips_host.size() * sizeof(int), hipMemcpyHostToDevice,
                                  st));
            HIPCHK(hipMemcpyAsync(dtiles, tiles.data(), tiles.size() * sizeof(uint2), hipMemcpyHostToDevice, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        dirty = false;
        return PDBM_OK;
    }

    // Enqueues `steps` steps of every member (a member stops at its own
    // step limit): whole chunks by replaying the captured graph, the rest as
    // plain launches.  chunk <= PART_RING.
    int run(int64_t steps, int chunk, hipStream_t st)
    {
        if (members.empty() || steps <= 0) return PDBM_OK;
        if (chunk > 1 && steps >= chunk) {
            if (!exec || graph_steps != chunk) {
                int rc = capture(chunk, st);
                if (rc) return rc;
            }
            for (; steps >= chunk; steps -= chunk) {
                HIPCHK(hipGraphLaunch(exec, st));
                advance(chunk);
            }
        }
        while (steps > 0) {
            const int n = (int)std::min<int64_t>(steps, PART_RING);
            HIPCHK(enqueue_steps(n, st));
            advance(n);
            steps -= n;
        }
        return PDBM_OK;
    }

    void destroy()
    {
        drop_graph();
        if (ddescs) (void)hipFree(ddescs);
        if (dtiles) (void)hipFree(dtiles);
        if (dbases) (void)hipFree(dbases);
        if (dflips) (void)hipFree(dflips);
        ddescs = nullptr;
        dtiles = nullptr;
        dbases = nullptr;
        dflips = nullptr;
        cap_descs = cap_tiles = cap_bases = cap_flips = 0;
    }

  private:
    bool rot = false;
    SolveDesc *ddescs = nullptr;
    uint2 *dtiles = nullptr;
    int64_t *dbases = nullptr;  // step of each member at the start of the next chunk
    int *dflips = nullptr;      // buffer parity of each member (Solve::flip) at that step
    bool pairs = false;         // the wide members step two steps per launch
    int nwide = 0, nwt = 0;     // wide members (the first in the tables) and their tiles
    std::vector<int64_t> bases_host;
    std::vector<int> flips_host;
    size_t cap_descs = 0, cap_tiles = 0, cap_bases = 0, cap_flips = 0;
    int ntiles = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_steps = 0;

    static int grow(void **p, size_t &cap, size_t need)
    {
        if (need <= cap) return PDBM_OK;
        const size_t n = std::max<size_t>(need, 2 * cap + 4096);
        if (*p) (void)hipFree(*p);
        *p = nullptr;
        cap = 0;
        if (hipMalloc(p, n) != hipSuccess) return fail(PDBM_ENOMEM, "hipMalloc of a launch table failed");
        cap = n;
        return PDBM_OK;
    }

    int capture(int chunk, hipStream_t st)
    {
        drop_graph();
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const hipError_t e = enqueue_steps(chunk, st);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(st, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(PDBM_EHIP, std::string("graph capture failed: ") +
                                       hipGetErrorString(e != hipSuccess ? e : e2));
        }
        graph = g;
        HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        graph_steps = chunk;
        return PDBM_OK;
    }

    // n <= PART_RING steps of every member, their drift records, and the
    // advance of the step bases (and, in pairs and for the columns, of the
    // buffer parities).  The wide members: in pairs, two-step launch i takes
    // steps 2i and 2i + 1 with parity flips ^ (i & 1) (every member still
    // running has taken the i launches before), and an odd n ends with a
    // launch of single steps; otherwise one step per launch.  The columns:
    // launches of nk = min(COL_K, steps of the chunk left) steps; each
    // toggles the parity of the members still running when nk is even.
    hipError_t enqueue_steps(int n, hipStream_t st)
    {
        const int nm = (int)members.size(), ncol = nm - nwide;
        hipError_t e = hipSuccess;
        if (nwide > 0) {
            if (pairs) {
                for (int i = 0; 2 * i + 1 < n && e == hipSuccess; ++i)
                    e = launch_step2(ddescs, dtiles, nwt, dbases, 2 * i, dflips, i & 1, false, fp32, false, rot, st);
                if (e == hipSuccess && (n & 1))
                    e = launch_step2(ddescs, dtiles, nwt, dbases, n - 1, dflips, (n / 2) & 1, true, fp32, false, rot,
                                     st);
            } else {
                for (int i = 0; i < n && e == hipSuccess; ++i)
                    e = launch_step(ddescs, dtiles, nwt, dbases, i, dflips, 0, fp32, rot, false, st);
            }
        }
        if (ncol > 0) {
            int pf = 0;
            for (int done = 0; done < n && e == hipSuccess;) {
                const int nk = std::min(COL_K, n - done);
                e = launch_column(ddescs, dtiles + nwt, ntiles - nwt, dbases, done, dflips, pf, nk, fp32, false, st);
                pf ^= (nk + 1) & 1;
                done += nk;
            }
        }
        if (e == hipSuccess) e = launch_records(ddescs, nm, dbases, 0, n, st);
        if (e == hipSuccess && nwide > 0)
            e = launch_advance(ddescs, pairs ? dflips : nullptr, dbases, nwide, n, 0, st);
        if (e == hipSuccess && ncol > 0)
            e = launch_advance(ddescs + nwide, dflips + nwide, dbases + nwide, ncol, n, COL_K, st);
        return e;
    }

    // Host copy of what the device tables go through in n steps.
    void advance(int64_t n)
    {
        for (Solve *m : members) {
            const int64_t left = std::max<int64_t>(m->hd.nsteps - m->step, 0);
            if (m->columnar())
                m->flip ^= column_chunk_toggle(left, n, COL_K);
            else if (pairs)
                m->flip ^= pair_chunk_toggle(left, n);
            m->step = std::min(m->step + n, m->hd.nsteps);
        }
    }

    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_steps = 0;
    }
};

// Rows per wavefront of a packed solve of more than one column: FUSE_ROWS,
// the longest blocks the two-step kernel takes, which recompute the fewest
// rows; PDBM_BATCH_ROWS overrides it (tuning).  A single column's
// wavefronts hold COL_W rows whatever this is.
int batch_rows(const pdbm_params &p)
{
    static const int env = [] {
        const char *e = std::getenv("PDBM_BATCH_ROWS");
        return e ? std::atoi(e) : 0;
    }();
    if (env > 0) return env;
    return FUSE_ROWS;
}

// Fields [6][nr][ntheta] (host, may be NULL) and drift report of a member.
int fetch_result(const Solve &s, double *out, pdbm_diag *diag, hipStream_t st)
{
    double *stage = out ? (double *)s.hd.f[s.cur() ^ 1] : nullptr;
    pdbm_diag *dslot = s.hd.hist + HIST_CAP;
    int rc = s.moments(stage, dslot, st);
    if (rc) return rc;
    pdbm_diag d;
    if (out)
        HIPCHK(hipMemcpyAsync(out, stage, (size_t)6 * s.p.nr * s.p.ntheta * sizeof(double), hipMemcpyDeviceToHost,
                              st));
    HIPCHK(hipMemcpyAsync(&d, dslot, sizeof d, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    d.step = s.step;
    if (diag) *diag = d;
    return PDBM_OK;
}

}  // namespace

// ------------------------------------------------------------------ batch --
struct pdbm_batch {
    std::vector<std::unique_ptr<Solve>> solves;
    Pack pack;
    hipStream_t st = nullptr;
    bool own_stream = false;  // graphs cannot be captured on the null stream
    int chunk = 0;
};

extern "C" {

int pdbm_batch_create(int32_t n, const pdbm_params *ps, const pdbm_ic *ics, int32_t chunk_steps, void *stream,
                      pdbm_batch **out)
{
    if (!out || n < 1 || !ps || chunk_steps < 0 || chunk_steps > PART_RING) return fail(PDBM_EINVAL, "bad argument");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        int rc = pdbm_validate(ps + i, ics ? ics + i : nullptr, nullptr);
        if (rc) return rc;
        if (ps[i].precision != ps[0].precision) return fail(PDBM_EINVAL, "all solves of a batch share the precision");
        if (ps[i].flags & PDBM_TAU_FIELD) return fail(PDBM_EINVAL, "a per-cell tau field is for single solves only");
    }
    int rc = check_device();
    if (rc) return rc;
    pdbm_batch *b = new (std::nothrow) pdbm_batch;
    if (!b) return fail(PDBM_ENOMEM, "host allocation failed");
    b->st = (hipStream_t)stream;
    if (!b->st && chunk_steps > 1) {
        if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return fail(PDBM_EHIP, "hipStreamCreateWithFlags failed");
        }
        b->own_stream = true;
    }
    b->chunk = chunk_steps;
    b->pack.fp32 = ps[0].precision == PDBM_FP32;
    for (int i = 0; i < n && rc == PDBM_OK; ++i) {
        b->solves.emplace_back(new Solve);
        rc = b->solves.back()->init(ps[i], ics ? ics + i : nullptr, nullptr, 0, batch_rows(ps[i]), INT64_MAX, b->st);
        if (rc == PDBM_OK && hipStreamSynchronize(b->st) != hipSuccess) rc = fail(PDBM_EHIP, "initialisation failed");
        b->pack.members.push_back(b->solves.back().get());
    }
    if (rc == PDBM_OK) rc = b->pack.rebuild(b->st);
    if (rc) {
        pdbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PDBM_OK;
}

void pdbm_batch_destroy(pdbm_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->st);
    b->pack.destroy();
    for (auto &s : b->solves) s->release();
    if (b->own_stream) (void)hipStreamDestroy(b->st);
    delete b;
}

int pdbm_batch_step(pdbm_batch *b, int64_t nsteps)
{
    if (!b || nsteps < 0) return fail(PDBM_EINVAL, "bad batch or step count");
    return b->pack.run(nsteps, b->chunk, b->st);
}

int64_t pdbm_batch_step_count(const pdbm_batch *b, int32_t i)
{
    if (!b || i < 0 || i >= (int32_t)b->solves.size()) return -1;
    return b->solves[i]->step;
}

int pdbm_batch_moments(pdbm_batch *b, int32_t i, double *out, pdbm_diag *diag)
{
    if (!b || i < 0 || i >= (int32_t)b->solves.size()) return fail(PDBM_EINVAL, "bad batch index");
    pdbm_diag d;
    int rc = fetch_result(*b->solves[i], out, &d, b->st);
    if (rc) return rc;
    if (diag) *diag = d;
    if (d.n_nonfinite || d.n_nonphys) return fail(PDBM_ENONPHYS, "non-finite or non-physical state");
    return PDBM_OK;
}

int pdbm_batch_noneq(pdbm_batch *b, int32_t i, double *out)
{
    if (!b || i < 0 || i >= (int32_t)b->solves.size() || !out) return fail(PDBM_EINVAL, "bad batch index or NULL");
    return noneq_to_host(*b->solves[i], out, b->st);
}

}  // extern "C"

// ----------------------------------------------------------------- server --
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id = 0;
    pdbm_params p{};
    pdbm_ic ic{};
    int64_t nsteps = 0;
    uint32_t flags = 0;
    int32_t state = PDBM_QUEUED;
    size_t bytes = 0;
    std::unique_ptr<Solve> solve;
    std::vector<double> fields;
    pdbm_diag diag{};
    double t_submit = -1, t_admit = -1, t_done = -1;
};

}  // namespace

struct pdbm_server {
    int max_slots = 0, chunk = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;    // wakes the scheduler
    std::condition_variable done;  // wakes pollers waiting for completion
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_id = 1;
    Ledger led;  // memory in use, request counts and state moves (guarded by mu)
    bool stop = false;
    int sched_error = 0;

    // scheduler-thread state
    std::vector<Request *> running;
    Pack pack[2];  // by precision: PDBM_FP64, PDBM_FP32
    std::thread thr;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void loop();
    int admit_and_step(std::vector<Request *> &admitted);
    void retire(Request *r, int err);
};

void pdbm_server::retire(Request *r, int err)
{
    {
        // a request is retired once (the ledger refuses a second time too)
        std::lock_guard<std::mutex> g(mu);
        if (r->state != PDBM_RUNNING) return;
    }
    pdbm_diag d{};
    bool ok = err == 0;
    if (ok && r->solve) {
        std::vector<double> f;
        if (r->flags & PDBM_KEEP_FIELDS) f.resize((size_t)6 * r->p.nr * r->p.ntheta);
        if (fetch_result(*r->solve, f.empty() ? nullptr : f.data(), &d, st) != PDBM_OK) ok = false;
        if (d.n_nonfinite || d.n_nonphys) ok = false;
        r->fields.swap(f);
    }
    if (r->solve) {
        (void)hipStreamSynchronize(st);
        r->solve->release();
        r->solve.reset();
    }
    std::lock_guard<std::mutex> g(mu);
    r->diag = d;
    r->t_done = now();
    led.retire(r->state, r->bytes, ok, (double)r->p.nr * r->p.ntheta * (double)r->nsteps);
    done.notify_all();
}

void pdbm_server::loop()
{
    for (;;) {
        std::vector<Request *> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                while (!queue.empty() && (int)(running.size() + admitted.size()) < max_slots) {
                    Request *r = reqs[queue.front()].get();
                    if (!led.fits(r->bytes)) break;  // first come, first served
                    queue.pop_front();
                    led.admit(r->state, r->bytes);
                    r->t_admit = now();
                    admitted.push_back(r);
                }
                if (stop) break;
                if (!admitted.empty() || !running.empty()) break;
                cv.wait(lk);
            }
        }
        bool quit;
        {
            std::lock_guard<std::mutex> g(mu);
            quit = stop;
        }
        const int rc = quit ? PDBM_OK : admit_and_step(admitted);
        if (quit || rc) {
            // shutting down, or a HIP error left the device state unknown:
            // every solve still held fails (admitted ones whose set-up
            // failed were retired already and are left alone)
            if (rc) {
                std::lock_guard<std::mutex> g(mu);
                sched_error = rc;
            }
            for (Request *r : admitted)
                if (std::find(running.begin(), running.end(), r) == running.end()) running.push_back(r);
            for (Request *r : running) retire(r, PDBM_EHIP);
            running.clear();
            for (auto &k : pack) k.members.clear();
            if (rc) {
                std::lock_guard<std::mutex> g(mu);
                stop = true;
                for (uint64_t id : queue) led.drop(reqs[id]->state);
                queue.clear();
                done.notify_all();
            }
            return;
        }
    }
}

int pdbm_server::admit_and_step(std::vector<Request *> &admitted)
{
    for (Request *r : admitted) {
        r->solve.reset(new Solve);
        int rc = r->solve->init(r->p, &r->ic, nullptr, 0, batch_rows(r->p), r->nsteps, st);
        if (rc == PDBM_OK && hipStreamSynchronize(st) != hipSuccess) rc = PDBM_EHIP;
        if (rc) {
            retire(r, rc);
            continue;
        }
        running.push_back(r);
        pack[r->p.precision].members.push_back(r->solve.get());
        pack[r->p.precision].dirty = true;
    }
    for (int k = 0; k < 2; ++k)
        if (pack[k].dirty) {
            int rc = pack[k].rebuild(st);
            if (rc) return rc;
        }
    // one chunk of steps for every member (members that reach their step
    // count stop advancing inside the chunk)
    for (int k = 0; k < 2; ++k) {
        int rc = pack[k].run(chunk, chunk, st);
        if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(st));
    {
        std::lock_guard<std::mutex> g(mu);
        led.stats.steps_launched += chunk;
    }
    std::vector<Request *> still;
    for (size_t i = 0; i < running.size(); ++i) {
        Request *r = running[i];
        if (r->solve->step >= r->nsteps) {
            auto &m = pack[r->p.precision].members;
            m.erase(std::find(m.begin(), m.end(), r->solve.get()));
            pack[r->p.precision].dirty = true;
            retire(r, 0);
        } else {
            still.push_back(r);
        }
    }
    running.swap(still);
    return PDBM_OK;
}

extern "C" {

int pdbm_server_create(size_t hbm_cap_bytes, int32_t max_slots, int32_t chunk_steps, void *stream,
                       pdbm_server **out)
{
    if (!out || hbm_cap_bytes == 0 || max_slots < 1 || chunk_steps < 1 || chunk_steps > PART_RING)
        return fail(PDBM_EINVAL, "bad argument");
    *out = nullptr;
    int rc = check_device();
    if (rc) return rc;
    pdbm_server *s = new (std::nothrow) pdbm_server;
    if (!s) return fail(PDBM_ENOMEM, "host allocation failed");
    s->led.cap = hbm_cap_bytes;
    s->max_slots = max_slots;
    s->chunk = chunk_steps;
    s->t0 = Clock::now();
    s->led.stats.hbm_cap = hbm_cap_bytes;
    s->pack[PDBM_FP64].fp32 = false;
    s->pack[PDBM_FP32].fp32 = true;
    if (stream) {
        s->st = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return fail(PDBM_EHIP, "hipStreamCreateWithFlags failed");
        }
        s->own_stream = true;
    }
    s->thr = std::thread([s] { s->loop(); });
    *out = s;
    return PDBM_OK;
}

void pdbm_server_destroy(pdbm_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        // requests not finished fail: queued ones now, running ones after
        // the chunk in progress
        for (uint64_t id : s->queue) s->led.drop(s->reqs[id]->state);
        s->queue.clear();
    }
    s->cv.notify_all();
    if (s->thr.joinable()) s->thr.join();
    (void)hipStreamSynchronize(s->st);
    for (auto &k : s->pack) k.destroy();
    for (auto &kv : s->reqs)
        if (kv.second->solve) kv.second->solve->release();
    if (s->own_stream) (void)hipStreamDestroy(s->st);
    delete s;
}

int pdbm_submit(pdbm_server *s, const pdbm_params *p, const pdbm_ic *ic, int64_t nsteps, uint32_t flags,
                uint64_t *req_id)
{
    if (!s || !p || !ic || !req_id || nsteps < 0 || (flags & ~PDBM_KEEP_FIELDS)) return fail(PDBM_EINVAL, "bad argument");
    int rc = pdbm_validate(p, ic, nullptr);
    if (rc) return rc;
    if (p->flags & PDBM_TAU_FIELD) return fail(PDBM_EINVAL, "a per-cell tau field is for single solves only");
    std::unique_ptr<Request> r(new (std::nothrow) Request);
    if (!r) return fail(PDBM_ENOMEM, "host allocation failed");
    r->p = *p;
    r->ic = *ic;
    r->nsteps = nsteps;
    r->flags = flags;
    r->bytes = layout_of(*p, batch_rows(*p)).total;
    if (r->bytes > s->led.cap) return fail(PDBM_ENOMEM, "request larger than the server's memory cap");
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(PDBM_EINVAL, "server is shutting down");
    r->id = s->next_id++;
    r->t_submit = s->now();
    *req_id = r->id;
    s->led.submit(r->state);
    s->queue.push_back(r->id);
    s->reqs[r->id] = std::move(r);
    s->cv.notify_all();
    return PDBM_OK;
}

int pdbm_poll(pdbm_server *s, uint64_t req_id, int32_t *state, double *out, pdbm_diag *diag)
{
    if (!s) return fail(PDBM_EINVAL, "NULL server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return fail(PDBM_ENOENT, "no such request");
    Request *r = it->second.get();
    if (state) *state = r->state;
    if (r->state == PDBM_QUEUED || r->state == PDBM_RUNNING) return PDBM_EAGAIN;
    if (diag) *diag = r->diag;
    if (out) {
        if (r->fields.empty()) return fail(PDBM_EINVAL, "fields were not kept (submit with PDBM_KEEP_FIELDS)");
        std::memcpy(out, r->fields.data(), r->fields.size() * sizeof(double));
    }
    return PDBM_OK;
}

int pdbm_request_times(pdbm_server *s, uint64_t req_id, double *times)
{
    if (!s || !times) return fail(PDBM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return fail(PDBM_ENOENT, "no such request");
    times[0] = it->second->t_submit;
    times[1] = it->second->t_admit;
    times[2] = it->second->t_done;
    return PDBM_OK;
}

int pdbm_release(pdbm_server *s, uint64_t req_id)
{
    if (!s) return fail(PDBM_EINVAL, "NULL server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return fail(PDBM_ENOENT, "no such request");
    if (it->second->state == PDBM_QUEUED || it->second->state == PDBM_RUNNING) return fail(PDBM_EAGAIN, "not finished");
    s->reqs.erase(it);
    return PDBM_OK;
}

int pdbm_server_wait(pdbm_server *s, double timeout_s)
{
    if (!s) return fail(PDBM_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(
                                          timeout_s < 0 ? 1e9 : timeout_s));
    while (s->led.stats.queued > 0 || s->led.stats.running > 0) {
        if (s->sched_error) return fail(s->sched_error, "scheduler stopped on an error");
        if (s->done.wait_until(lk, until) == std::cv_status::timeout) return PDBM_EAGAIN;
    }
    return s->sched_error ? fail(s->sched_error, "scheduler stopped on an error") : PDBM_OK;
}

int pdbm_server_get_stats(pdbm_server *s, pdbm_server_stats *out)
{
    if (!s || !out) return fail(PDBM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->led.stats;
    out->hbm_in_use = s->led.in_use;
    out->elapsed = s->now();
    return PDBM_OK;
}

}  // extern "C"
