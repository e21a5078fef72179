// pdbm_create_noalloc: a single solve that allocates no memory.  Its
// auxiliary device memory (description, theta table, drift partial sums and
// records, moments reduction scratch) lives in a static device array, one per
// device; the caller brings the state buffer.  The kernels are those of every
// other solve: they take the auxiliary buffers through the solve description.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "pdbm_host.h"

using namespace pdbm;

namespace {

constexpr int MAX_DEVICES = 16;

// Each device holds its own copy; host code reaches it only through the
// address hipGetSymbolAddress gives for that device (scratch_ptr).
static __device__ __align__(256) char scratch[PDBM_SCRATCH_BYTES];

std::mutex g_mu;
char *g_ptr[MAX_DEVICES];           // device address of `scratch` on each device
bool g_busy[MAX_DEVICES];           // a solver holds that device's scratch
pdbm_solver g_slot[MAX_DEVICES];    // the handle of that solver

// Address of this device's copy of the scratch array (looked up once per
// device, with the device current).  Call with g_mu held.
int scratch_ptr(int dev, char **out)
{
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PDBM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = (char *)p;
    }
    *out = g_ptr[dev];
    return PDBM_OK;
}

}  // namespace

void pdbm::release_scratch_solver(int dev)
{
    std::lock_guard<std::mutex> g(g_mu);
    g_slot[dev].s = Solve();
    g_slot[dev].st = nullptr;
    g_slot[dev].scratch_dev = -1;
    g_busy[dev] = false;
}

extern "C" int pdbm_create_noalloc(const pdbm_params *p, const pdbm_ic *ic, void *state, size_t *state_bytes,
                                   void *stream, pdbm_solver **out)
{
    if (!state_bytes) return fail(PDBM_EINVAL, "state_bytes is NULL");
    int rc = pdbm_validate(p, ic, nullptr);
    if (rc) return rc;
    const int rows = rows_per_wave(*p);
    const Layout L = layout_of(*p, rows);
    if (!state) {
        *state_bytes = L.state_total;
        return PDBM_OK;
    }
    if (!out) return fail(PDBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (L.aux_total > (size_t)PDBM_SCRATCH_BYTES) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "this grid needs %zu bytes of auxiliary memory; the static scratch holds %d",
                      L.aux_total, (int)PDBM_SCRATCH_BYTES);
        return fail(PDBM_ENOMEM, buf);
    }
    if ((rc = check_device())) return rc;
    int dev = 0;
    PDBM_HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PDBM_EINVAL, "device index beyond the static slots");
    char *aux = nullptr;
    pdbm_solver *h = &g_slot[dev];
    {
        std::lock_guard<std::mutex> g(g_mu);
        if ((rc = scratch_ptr(dev, &aux))) return rc;
        if (g_busy[dev]) return fail(PDBM_EAGAIN, "another solver holds this device's static scratch");
        g_busy[dev] = true;
        h->scratch_dev = dev;
    }
    h->st = (hipStream_t)stream;
    rc = h->s.init(*p, ic, state, *state_bytes, rows, INT64_MAX, h->st, aux);
    if (rc == PDBM_OK && hipStreamSynchronize(h->st) != hipSuccess) rc = fail(PDBM_EHIP, "initialisation failed");
    if (rc) {
        (void)hipStreamSynchronize(h->st);
        release_scratch_solver(dev);
        return rc;
    }
    *out = h;
    return PDBM_OK;
}
