// Host side of libpdbm: parameter validation, the moment-inversion matrix,
// device memory layout, and the C ABI of one solve (include/pdbm.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pdbm_internal.h"

using namespace pdbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail(PDBM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr double SPEEDS[5] = {0.0, 1.5, 3.5, 7.5, 12.5};  // Sec. II.B
constexpr int64_t MAX_CELLS = int64_t(1) << 24;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int pitch_of(int nt) { return nt <= 16 ? nt : (nt + 31) / 32 * 32; }

// Device memory of one solve, in this order.
struct Layout {
    size_t f, lam, cs, desc, partials, counter, hist, total;
    int pitch, nblocks;
    size_t esz;
};

int blocks_of(const pdbm_params &p)
{
    const int64_t cellb = ((int64_t)p.nr * p.ntheta + BLOCK - 1) / BLOCK;
    const int rows = rows_per_wave(p.nr, p.ntheta, p.precision == PDBM_FP32);
    const int64_t waves = (int64_t)((p.nr + rows - 1) / rows) * ((p.ntheta + STRIP - 1) / STRIP);
    const int64_t stepb = (waves + BLOCK / 64 - 1) / (BLOCK / 64);
    return (int)(cellb > stepb ? cellb : stepb);
}

Layout layout_of(const pdbm_params &p)
{
    Layout L;
    L.esz = p.precision == PDBM_FP32 ? sizeof(float) : sizeof(double);
    L.pitch = pitch_of(p.ntheta);
    const size_t cells_p = (size_t)p.nr * L.pitch;
    L.nblocks = blocks_of(p);
    L.f = align256((size_t)NQ * cells_p * L.esz);
    L.lam = align256(cells_p * sizeof(double));
    L.cs = align256((size_t)p.ntheta * sizeof(double2));
    L.desc = align256(sizeof(SolveDesc));
    L.partials = align256((size_t)L.nblocks * 5 * sizeof(double));
    L.counter = 256;
    L.hist = align256((size_t)(HIST_CAP + 1) * sizeof(pdbm_diag));
    L.total = 2 * L.f + 2 * L.lam + L.cs + L.desc + L.partials + L.counter + L.hist;
    return L;
}

bool is_fin(double x) { return std::isfinite(x); }

}  // namespace

// Rows per wavefront: just enough wavefronts for one resident wave of the
// whole grid (256 CUs x 4 SIMDs x the step kernel's occupancy: 1 wavefront
// per SIMD in float64, 2 in float32), so that every wavefront marches the
// longest possible column and none waits for a second round.
// PDBM_ROWS_PER_WAVE overrides it (tuning).
int pdbm::rows_per_wave(int nr, int nt, bool fp32)
{
    static const int env = [] {
        const char *e = std::getenv("PDBM_ROWS_PER_WAVE");
        return e ? std::atoi(e) : 0;
    }();
    if (env > 0) return env;
    const int64_t slots = 256 * 4 * (fp32 ? 2 : 1);
    const int64_t strips = (nt + STRIP - 1) / STRIP;
    int64_t rows = ((int64_t)nr * strips + slots - 1) / slots;
    if (rows < 2) rows = 2;
    while (strips * ((nr + rows - 1) / rows) > slots) ++rows;
    return (int)rows;
}

// Largest |C_r| + |C_theta| over the grid for the fastest speed: the
// innermost row has the largest azimuthal Courant number.
static double max_courant(const pdbm_params &p)
{
    const double dr = (p.r_max - p.r_min) / p.nr;
    const double dth = p.sector * M_PI / 4.0 / p.ntheta;
    const double r0 = p.r_min + 0.5 * dr;
    const double v = SPEEDS[4] * p.dt;
    double worst = 0.0;
    for (int j = 0; j < p.ntheta; ++j) {
        const double th = (j + 0.5) * dth;
        for (int i = 0; i < 8; ++i) {
            const double a = i * M_PI / 4.0 - th;
            const double c = v * (std::fabs(std::cos(a)) / dr + std::fabs(std::sin(a)) / (r0 * dth));
            if (c > worst) worst = c;
        }
    }
    return worst;
}

extern "C" {

const char *pdbm_strerror(int code)
{
    switch (code) {
    case PDBM_OK: return "ok";
    case PDBM_EINVAL: return "invalid argument";
    case PDBM_ECFL: return "Courant number above 1";
    case PDBM_ENOMEM: return "out of memory or buffer too small";
    case PDBM_EHIP: return "HIP runtime error";
    case PDBM_EAGAIN: return "not finished yet";
    case PDBM_ENOENT: return "no such request";
    case PDBM_ENONPHYS: return "non-finite or non-physical state";
    case PDBM_ENOSYS: return "no usable gfx950 device";
    default: return "unknown error";
    }
}

const char *pdbm_last_error(void) { return g_err.c_str(); }

int pdbm_version(void) { return 1; }

int pdbm_validate(const pdbm_params *p, const pdbm_ic *ic, double *cfl)
{
    if (!p) return fail(PDBM_EINVAL, "params is NULL");
    if (p->nr < 1 || p->ntheta < 1) return fail(PDBM_EINVAL, "nr and ntheta must be >= 1");
    if ((int64_t)p->nr * p->ntheta > MAX_CELLS) return fail(PDBM_EINVAL, "grid larger than 2^24 cells");
    if (p->sector < 1 || p->sector > 8) return fail(PDBM_EINVAL, "sector must be in 1..8");
    {
        const size_t esz = p->precision == PDBM_FP32 ? 4 : 8;
        if ((size_t)NQ * p->nr * pitch_of(p->ntheta) * esz >= ((size_t)1 << 32))
            return fail(PDBM_EINVAL, "f array of one solve must stay below 4 GiB");
    }
    if (p->precision != PDBM_FP64 && p->precision != PDBM_FP32) return fail(PDBM_EINVAL, "unknown precision");
    if (p->m < 0 || p->n < 0 || p->m > 64 || p->n > 64) return fail(PDBM_EINVAL, "m, n must be in 0..64");
    if (p->diag_every < 0) return fail(PDBM_EINVAL, "diag_every must be >= 0");
    if (p->flags & ~PDBM_ALLOW_CFL) return fail(PDBM_EINVAL, "unknown flags");
    if (!is_fin(p->r_min) || !is_fin(p->r_max) || p->r_min < 0.0 || !(p->r_max > p->r_min))
        return fail(PDBM_EINVAL, "need 0 <= r_min < r_max");
    if (!is_fin(p->dt) || !(p->dt > 0.0)) return fail(PDBM_EINVAL, "dt must be finite and > 0");
    if (std::isnan(p->tau) || !(p->tau > 0.0)) return fail(PDBM_EINVAL, "tau must be > 0");
    if (!is_fin(p->w1) || !is_fin(p->w2) || p->w1 < 0.0 || p->w2 < 0.0)
        return fail(PDBM_EINVAL, "w1, w2 must be finite and >= 0");
    if (!is_fin(p->Q) || p->Q < 0.0) return fail(PDBM_EINVAL, "Q must be finite and >= 0");
    if (!is_fin(p->T_th)) return fail(PDBM_EINVAL, "T_th must be finite");
    if (ic) {
        if (!is_fin(ic->r_split)) return fail(PDBM_EINVAL, "r_split must be finite");
        if (!is_fin(ic->p_noise) || ic->p_noise < 0.0) return fail(PDBM_EINVAL, "p_noise must be finite and >= 0");
        for (const double *s : {ic->inner, ic->outer}) {
            for (int i = 0; i < 5; ++i)
                if (!is_fin(s[i])) return fail(PDBM_EINVAL, "initial state must be finite");
            if (!(s[0] > 0.0) || !(s[1] > 0.0)) return fail(PDBM_EINVAL, "initial rho and T must be > 0");
            if (!(s[0] * s[1] - ic->p_noise > 0.0)) return fail(PDBM_EINVAL, "p_noise must keep p > 0");
        }
    }
    const double c = max_courant(*p);
    if (cfl) *cfl = c;
    if (c > 1.0 && !(p->flags & PDBM_ALLOW_CFL)) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "max |C_r|+|C_theta| = %.4g > 1", c);
        return fail(PDBM_ECFL, buf);
    }
    return PDBM_OK;
}

int pdbm_state_bytes(const pdbm_params *p, size_t *bytes)
{
    if (!p || !bytes) return fail(PDBM_EINVAL, "NULL argument");
    if (p->nr < 1 || p->ntheta < 1 || (int64_t)p->nr * p->ntheta > MAX_CELLS ||
        (p->precision != PDBM_FP64 && p->precision != PDBM_FP32))
        return fail(PDBM_EINVAL, "bad grid or precision");
    *bytes = layout_of(*p).total;
    return PDBM_OK;
}

// F_k(T) from the moment constraints sum_k 8 F_k x_k^n = 2^n n! T^n, x_k =
// v_k^2, n = 1..4.  With G_k = 8 x_k F_k this is a Vandermonde system in x_k
// whose inverse rows are the coefficients of the Lagrange polynomials
// L_k(x) = prod_{l != k} (x - x_l) / (x_k - x_l).
int pdbm_fk_matrix(double *A)
{
    if (!A) return fail(PDBM_EINVAL, "NULL argument");
    const double cn[5] = {1.0, 2.0, 8.0, 48.0, 384.0};  // 2^n n!
    for (int k = 0; k < 4; ++k) {
        const double xk = SPEEDS[k + 1] * SPEEDS[k + 1];
        double c[4] = {1.0, 0.0, 0.0, 0.0};
        double den = 1.0;
        int deg = 0;
        for (int l = 0; l < 4; ++l) {
            if (l == k) continue;
            const double xl = SPEEDS[l + 1] * SPEEDS[l + 1];
            for (int j = deg + 1; j >= 1; --j) c[j] = c[j - 1] - xl * c[j];
            c[0] = -xl * c[0];
            ++deg;
            den *= xk - xl;
        }
        for (int j = 0; j < 4; ++j) A[4 * k + j] = c[j] / den * cn[j + 1] / (8.0 * xk);
    }
    return PDBM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ solver --
struct pdbm_solver {
    pdbm_params p;
    hipStream_t st = nullptr;
    Layout L;
    bool fp32 = false, own = false;
    char *ws = nullptr;
    void *f[2] = {nullptr, nullptr};
    double *lam[2] = {nullptr, nullptr};
    double2 *cs = nullptr;
    SolveDesc *ddesc = nullptr;  // device copy read by the step kernel
    double *partials = nullptr;
    unsigned *counter = nullptr;
    pdbm_diag *hist = nullptr;  // [HIST_CAP] ring + 1 slot for pdbm_moments
    int cur = 0;
    int64_t step = 0, nrec = 0;
    double A[16];

    SolveDesc desc(int from) const
    {
        SolveDesc d;
        std::memset(&d, 0, sizeof d);
        d.f_in = f[from];
        d.f_out = f[from ^ 1];
        d.lam_in = lam[from];
        d.lam_out = lam[from ^ 1];
        d.cs = cs;
        d.nr = p.nr;
        d.nt = p.ntheta;
        d.pitch = L.pitch;
        d.sector = p.sector;
        d.m = p.m;
        d.n = p.n;
        d.disc = p.r_min == 0.0;
        d.reacts = (p.w1 > 0.0 || p.w2 > 0.0) ? 1 : 0;
        d.rows = rows_per_wave(p.nr, p.ntheta, p.precision == PDBM_FP32);
        d.plane = L.pitch;
        d.rstride = (int64_t)NQ * L.pitch;
        d.dr = (p.r_max - p.r_min) / p.nr;
        d.dth = p.sector * M_PI / 4.0 / p.ntheta;
        d.r_min = p.r_min;
        d.dt_dr = p.dt / d.dr;
        d.dt_dth = p.dt / d.dth;
        d.omega = std::exp(-p.dt / p.tau);
        d.w1 = p.w1;
        d.w2 = p.w2;
        d.Q = p.Q;
        d.T_th = p.T_th;
        d.dt = p.dt;
        std::memcpy(d.A, A, sizeof A);
        return d;
    }
    DiagCtl diag(pdbm_diag *out, bool on) const
    {
        DiagCtl c;
        c.partials = partials;
        c.counter = counter;
        c.out = out;
        c.step = step;
        c.enabled = on ? 1 : 0;
        c.pad = 0;
        return c;
    }
};

static int check_device()
{
    int dev = 0, n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(PDBM_ENOSYS, "no HIP device");
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PDBM_ENOSYS, std::string("device is ") + prop.gcnArchName + ", need gfx950");
    return PDBM_OK;
}

extern "C" {

int pdbm_create(const pdbm_params *p, const pdbm_ic *ic, void *workspace, size_t workspace_bytes, void *stream,
                pdbm_solver **out)
{
    if (!out) return fail(PDBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = pdbm_validate(p, ic, nullptr);
    if (rc) return rc;
    if ((rc = check_device())) return rc;

    pdbm_solver *s = new (std::nothrow) pdbm_solver;
    if (!s) return fail(PDBM_ENOMEM, "host allocation failed");
    s->p = *p;
    s->st = (hipStream_t)stream;
    s->L = layout_of(*p);
    s->fp32 = p->precision == PDBM_FP32;
    pdbm_fk_matrix(s->A);
    if (workspace) {
        if (workspace_bytes < s->L.total || ((uintptr_t)workspace & 255)) {
            delete s;
            return fail(PDBM_ENOMEM, "workspace smaller than pdbm_state_bytes() or not 256-byte aligned");
        }
        s->ws = (char *)workspace;
    } else {
        if (hipMalloc((void **)&s->ws, s->L.total) != hipSuccess) {
            delete s;
            return fail(PDBM_ENOMEM, "hipMalloc of the solve state failed");
        }
        s->own = true;
    }
    char *q = s->ws;
    s->f[0] = q;
    q += s->L.f;
    s->f[1] = q;
    q += s->L.f;
    s->lam[0] = (double *)q;
    q += s->L.lam;
    s->lam[1] = (double *)q;
    q += s->L.lam;
    s->cs = (double2 *)q;
    q += s->L.cs;
    s->ddesc = (SolveDesc *)q;
    q += s->L.desc;
    s->partials = (double *)q;
    q += s->L.partials;
    s->counter = (unsigned *)q;
    q += s->L.counter;
    s->hist = (pdbm_diag *)q;

    // theta table and zeroed counter, then the initial state
    std::vector<double2> cs(p->ntheta);
    const double dth = p->sector * M_PI / 4.0 / p->ntheta;
    for (int j = 0; j < p->ntheta; ++j) cs[j] = make_double2(std::cos((j + 0.5) * dth), std::sin((j + 0.5) * dth));
    const unsigned zero = 0;
    pdbm_ic uni;
    if (!ic) {
        std::memset(&uni, 0, sizeof uni);
        for (double *t : {uni.inner, uni.outer}) {
            t[0] = 1.0;
            t[1] = 1.0;
        }
        ic = &uni;
    }
    hipError_t e = hipMemcpyAsync(s->cs, cs.data(), cs.size() * sizeof(double2), hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipMemcpyAsync(s->counter, &zero, sizeof zero, hipMemcpyHostToDevice, s->st);
    const SolveDesc hd = s->desc(0);
    if (e == hipSuccess) e = hipMemcpyAsync(s->ddesc, &hd, sizeof hd, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) {
        // the initial state goes to buffer 0: a desc reading 1 writes 0
        e = launch_init_ic(s->desc(1), s->fp32, *ic, s->st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) {
        std::string m = std::string("initialisation failed: ") + hipGetErrorString(e);
        pdbm_destroy(s);
        return fail(PDBM_EHIP, m);
    }
    s->cur = 0;
    *out = s;
    return PDBM_OK;
}

void pdbm_destroy(pdbm_solver *s)
{
    if (!s) return;
    if (s->st || s->ws) (void)hipStreamSynchronize(s->st);
    if (s->own && s->ws) (void)hipFree(s->ws);
    delete s;
}

int pdbm_set_fields(pdbm_solver *s, const double *fields)
{
    if (!s || !fields) return fail(PDBM_EINVAL, "NULL argument");
    const size_t n = (size_t)5 * s->p.nr * s->p.ntheta;
    // stage the fields in the idle f buffer (at least 132 bytes per cell)
    double *stage = (double *)s->f[s->cur ^ 1];
    HIPCHK(hipMemcpyAsync(stage, fields, n * sizeof(double), hipMemcpyHostToDevice, s->st));
    HIPCHK(launch_init_fields(s->desc(s->cur ^ 1), s->fp32, stage, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    s->step = 0;
    s->nrec = 0;
    return PDBM_OK;
}

int pdbm_step(pdbm_solver *s, int64_t nsteps)
{
    if (!s || nsteps < 0) return fail(PDBM_EINVAL, "bad solver or step count");
    for (int64_t i = 0; i < nsteps; ++i) {
        const bool rec = s->p.diag_every > 0 && s->step % s->p.diag_every == 0;
        pdbm_diag *slot = s->hist + (s->nrec % HIST_CAP);
        HIPCHK(launch_step(s->desc(s->cur), s->ddesc, s->fp32, s->diag(slot, rec), s->st));
        s->cur ^= 1;
        s->step++;
        if (rec) s->nrec++;
    }
    return PDBM_OK;
}

int64_t pdbm_step_count(const pdbm_solver *s) { return s ? s->step : -1; }

static int moments_into(pdbm_solver *s, double *dev_out)
{
    HIPCHK(launch_moments(s->desc(s->cur), s->fp32, dev_out, s->diag(s->hist + HIST_CAP, true), s->st));
    return PDBM_OK;
}

int pdbm_moments(pdbm_solver *s, double *out, pdbm_diag *diag)
{
    if (!s) return fail(PDBM_EINVAL, "NULL solver");
    double *stage = out ? (double *)s->f[s->cur ^ 1] : nullptr;  // idle buffer holds 6 doubles per cell
    int rc = moments_into(s, stage);
    if (rc) return rc;
    pdbm_diag d;
    if (out)
        HIPCHK(hipMemcpyAsync(out, stage, (size_t)6 * s->p.nr * s->p.ntheta * sizeof(double), hipMemcpyDeviceToHost,
                              s->st));
    HIPCHK(hipMemcpyAsync(&d, s->hist + HIST_CAP, sizeof d, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    d.step = s->step;
    if (diag) *diag = d;
    if (d.n_nonfinite || d.n_nonphys) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "step %lld: %lld non-finite cells, %lld cells with rho<=0 or T<=0",
                      (long long)s->step, (long long)d.n_nonfinite, (long long)d.n_nonphys);
        return fail(PDBM_ENONPHYS, buf);
    }
    return PDBM_OK;
}

int pdbm_moments_async(pdbm_solver *s, void *out_device)
{
    if (!s || !out_device) return fail(PDBM_EINVAL, "NULL argument");
    return moments_into(s, (double *)out_device);
}

int pdbm_diag_history(pdbm_solver *s, pdbm_diag *out, int32_t cap, int32_t *n)
{
    if (!s || !n || cap < 0 || (cap > 0 && !out)) return fail(PDBM_EINVAL, "bad argument");
    HIPCHK(hipStreamSynchronize(s->st));
    const int64_t have = s->nrec < HIST_CAP ? s->nrec : HIST_CAP;
    const int64_t take = have < cap ? have : cap;
    const int64_t first = s->nrec - take;  // oldest record returned
    for (int64_t i = 0; i < take; ++i)
        HIPCHK(hipMemcpy(out + i, s->hist + ((first + i) % HIST_CAP), sizeof(pdbm_diag), hipMemcpyDeviceToHost));
    *n = (int32_t)take;
    return PDBM_OK;
}

// f on the device is [nr][NQ][pitch]; host arrays are [NQ][nr][ntheta].
static hipError_t f_to_host(pdbm_solver *s, void *host)
{
    const int nr = s->p.nr, nt = s->p.ntheta;
    const size_t esz = s->L.esz, pitch = s->L.pitch;
    for (int q = 0; q < NQ; ++q) {
        hipError_t e = hipMemcpy2D((char *)host + (size_t)q * nr * nt * esz, nt * esz,
                                   (const char *)s->f[s->cur] + q * pitch * esz, NQ * pitch * esz, nt * esz, nr,
                                   hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static hipError_t f_to_device(pdbm_solver *s, const void *host)
{
    const int nr = s->p.nr, nt = s->p.ntheta;
    const size_t esz = s->L.esz, pitch = s->L.pitch;
    for (int q = 0; q < NQ; ++q) {
        hipError_t e = hipMemcpy2D((char *)s->f[s->cur] + q * pitch * esz, NQ * pitch * esz,
                                   (const char *)host + (size_t)q * nr * nt * esz, nt * esz, nt * esz, nr,
                                   hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int pdbm_read_f(pdbm_solver *s, double *f, double *lam)
{
    if (!s) return fail(PDBM_EINVAL, "NULL solver");
    const int nr = s->p.nr, nt = s->p.ntheta, pitch = s->L.pitch;
    const size_t ncell = (size_t)nr * nt;
    HIPCHK(hipStreamSynchronize(s->st));
    if (f) {
        if (s->fp32) {
            std::vector<float> tmp((size_t)NQ * ncell);
            HIPCHK(f_to_host(s, tmp.data()));
            for (size_t i = 0; i < tmp.size(); ++i) f[i] = tmp[i];
        } else {
            HIPCHK(f_to_host(s, f));
        }
    }
    if (lam)
        HIPCHK(hipMemcpy2D(lam, nt * sizeof(double), s->lam[s->cur], pitch * sizeof(double), nt * sizeof(double), nr,
                           hipMemcpyDeviceToHost));
    return PDBM_OK;
}

int pdbm_write_f(pdbm_solver *s, const double *f, const double *lam, int64_t step)
{
    if (!s || step < 0) return fail(PDBM_EINVAL, "bad argument");
    const int nr = s->p.nr, nt = s->p.ntheta, pitch = s->L.pitch;
    const size_t ncell = (size_t)nr * nt;
    HIPCHK(hipStreamSynchronize(s->st));
    if (f) {
        if (s->fp32) {
            std::vector<float> tmp((size_t)NQ * ncell);
            for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (float)f[i];
            HIPCHK(f_to_device(s, tmp.data()));
        } else {
            HIPCHK(f_to_device(s, f));
        }
    }
    if (lam)
        HIPCHK(hipMemcpy2D(s->lam[s->cur], pitch * sizeof(double), lam, nt * sizeof(double), nt * sizeof(double), nr,
                           hipMemcpyHostToDevice));
    s->step = step;
    s->nrec = 0;
    return PDBM_OK;
}

namespace {
struct BlobHeader {
    uint64_t magic;
    int32_t version, nr, ntheta, precision;
    int64_t step;
};
constexpr uint64_t BLOB_MAGIC = 0x3130455441545344ull;  // "DSTATE01"
}  // namespace

int pdbm_get_state(pdbm_solver *s, void *buf, size_t *bytes)
{
    if (!s || !bytes) return fail(PDBM_EINVAL, "NULL argument");
    const int nr = s->p.nr, nt = s->p.ntheta, pitch = s->L.pitch;
    const size_t fb = (size_t)NQ * nr * nt * s->L.esz, lb = (size_t)nr * nt * sizeof(double);
    const size_t need = sizeof(BlobHeader) + fb + lb;
    if (!buf) {
        *bytes = need;
        return PDBM_OK;
    }
    if (*bytes < need) return fail(PDBM_ENOMEM, "checkpoint buffer too small");
    BlobHeader h{BLOB_MAGIC, 1, nr, nt, s->p.precision, s->step};
    std::memcpy(buf, &h, sizeof h);
    char *fdst = (char *)buf + sizeof h;
    HIPCHK(hipStreamSynchronize(s->st));
    HIPCHK(f_to_host(s, fdst));
    HIPCHK(hipMemcpy2D(fdst + fb, nt * sizeof(double), s->lam[s->cur], pitch * sizeof(double), nt * sizeof(double),
                       nr, hipMemcpyDeviceToHost));
    *bytes = need;
    return PDBM_OK;
}

int pdbm_set_state(pdbm_solver *s, const void *buf, size_t bytes)
{
    if (!s || !buf || bytes < sizeof(BlobHeader)) return fail(PDBM_EINVAL, "bad argument");
    BlobHeader h;
    std::memcpy(&h, buf, sizeof h);
    const int nr = s->p.nr, nt = s->p.ntheta, pitch = s->L.pitch;
    const size_t fb = (size_t)NQ * nr * nt * s->L.esz, lb = (size_t)nr * nt * sizeof(double);
    if (h.magic != BLOB_MAGIC || h.version != 1 || h.nr != nr || h.ntheta != nt || h.precision != s->p.precision ||
        h.step < 0 || bytes < sizeof h + fb + lb)
        return fail(PDBM_EINVAL, "checkpoint does not match this solve");
    const char *src = (const char *)buf + sizeof h;
    HIPCHK(hipStreamSynchronize(s->st));
    HIPCHK(f_to_device(s, src));
    HIPCHK(hipMemcpy2D(s->lam[s->cur], pitch * sizeof(double), src + fb, nt * sizeof(double), nt * sizeof(double),
                       nr, hipMemcpyHostToDevice));
    s->step = h.step;
    s->nrec = 0;
    return PDBM_OK;
}

}  // extern "C"
