// Host side of libpdbm: parameter validation, the moment-inversion matrix,
// the device memory of one solve, and the C ABI of a single solve
// (include/pdbm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pdbm_host.h"

using namespace pdbm;

namespace {

thread_local std::string g_err;

constexpr double SPEEDS[5] = {0.0, 1.5, 3.5, 7.5, 12.5};  // Sec. II.B
constexpr int64_t MAX_CELLS = int64_t(1) << 24;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Padded row length: whole 64-column strips, so that a wavefront's loads and
// stores of a velocity plane or pair cover whole cache lines; a single
// column gets a pitch of 2, which keeps the pairs of the f layout 16-byte
// aligned.
int pitch_of(int nt) { return nt == 1 ? 2 : (nt + STRIP - 1) / STRIP * STRIP; }

bool is_fin(double x) { return std::isfinite(x); }

}  // namespace

#define HIPCHK PDBM_HIPCHK

int pdbm::fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

Layout pdbm::layout_of(const pdbm_params &p, int rows)
{
    Layout L;
    L.esz = p.precision == PDBM_FP32 ? sizeof(float) : sizeof(double);
    L.pitch = pitch_of(p.ntheta);
    L.rows = rows;
    L.nwaves = solve_waves(p.nr, p.ntheta, rows);
    L.cblocks = cell_blocks(p.nr, p.ntheta);
    const size_t cells_p = (size_t)p.nr * L.pitch;
    L.f = align256((size_t)NQ * cells_p * L.esz);
    L.lam = align256(cells_p * sizeof(double));
    L.omega = (p.flags & PDBM_TAU_FIELD) ? align256(cells_p * L.esz) : 0;
    L.cs = align256((size_t)p.ntheta * sizeof(double2));
    L.desc = align256(sizeof(SolveDesc));
    L.state = align256(sizeof(SolveState));
    L.wpart = align256((size_t)PART_RING * L.nwaves * 5 * sizeof(double));
    L.hist = align256((size_t)(HIST_CAP + 1) * sizeof(pdbm_diag));
    L.cpart = align256((size_t)L.cblocks * 5 * sizeof(double));
    L.state_total = 2 * L.f + 2 * L.lam + L.omega;
    L.aux_total = L.cs + L.desc + L.state + L.wpart + L.hist + L.cpart;
    L.total = L.state_total + L.aux_total;
    return L;
}

// Rows per wavefront: just enough wavefronts for one resident wave of the
// whole grid (256 CUs x 4 SIMDs x the step kernels' occupancy: 1 wavefront
// per SIMD in float64, 2 in float32), so that every wavefront marches the
// longest possible column and none waits for a second round; at most
// FUSE_ROWS (the two-step kernel's limit), so grids of more than 16 rows per
// SIMD run several rounds.  PDBM_ROWS_PER_WAVE overrides it (tuning).
int pdbm::rows_per_wave(const pdbm_params &p)
{
    const int nr = p.nr, nt = p.ntheta;
    static const int env = [] {
        const char *e = std::getenv("PDBM_ROWS_PER_WAVE");
        return e ? std::atoi(e) : 0;
    }();
    if (env > 0) return env;
    // one round of wavefronts: one per SIMD in float64, two in float32
    const int64_t slots = 256 * 4 * (p.precision == PDBM_FP32 ? 2 : 1);
    const int64_t strips = (nt + STRIP - 1) / STRIP;
    int64_t rows = ((int64_t)nr * strips + slots - 1) / slots;
    if (rows < 2) rows = 2;
    while (strips * ((nr + rows - 1) / rows) > slots) ++rows;
    // short enough for the two-step kernel (large grids then run more than
    // one round of wavefronts)
    return (int)std::min<int64_t>(rows, FUSE_ROWS);
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
    if (p->flags & ~(PDBM_ALLOW_CFL | PDBM_TAU_FIELD)) return fail(PDBM_EINVAL, "unknown flags");
    if (!is_fin(p->r_min) || !is_fin(p->r_max) || p->r_min < 0.0 || !(p->r_max > p->r_min))
        return fail(PDBM_EINVAL, "need 0 <= r_min < r_max");
    // The disc-centre ghost is the cell's image across the centre, at theta + pi.  The paper's rule
    // f(-1, j, k, i) = f(0, j, k, (i+4)%8) (Sec. II.D) is that image when the periodic sector divides a
    // half turn (rotating by the sector angle s pi/4 turns the direction index by s); on any other sector
    // it would impose a symmetry the solution need not have.
    if (p->r_min == 0.0 && p->sector != 1 && p->sector != 2 && p->sector != 4)
        return fail(PDBM_EINVAL, "a disc (r_min = 0) needs sector 1, 2 or 4 (the centre rule takes the image "
                                 "across the centre, which lies on the grid only when the sector divides a half turn)");
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
    *bytes = layout_of(*p, rows_per_wave(*p)).total;
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


// ------------------------------------------------------------------- solve --
int pdbm::check_device()
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

int Solve::init(const pdbm_params &pp, const pdbm_ic *ic, void *workspace, size_t bytes, int rows, int64_t nsteps,
                hipStream_t st, char *aux)
{
    p = pp;
    L = layout_of(p, rows);
    fp32 = p.precision == PDBM_FP32;
    if (workspace) {
        if (bytes < (aux ? L.state_total : L.total) || ((uintptr_t)workspace & 255))
            return fail(PDBM_ENOMEM, aux ? "state buffer smaller than its size query or not 256-byte aligned"
                                         : "workspace smaller than pdbm_state_bytes() or not 256-byte aligned");
        ws = (char *)workspace;
        own = false;
    } else {
        if (hipMalloc((void **)&ws, L.total) != hipSuccess) {
            ws = nullptr;
            return fail(PDBM_ENOMEM, "hipMalloc of the solve state failed");
        }
        own = true;
    }
    char *q = ws;
    auto take = [&q](size_t n) {
        char *r = q;
        q += n;
        return r;
    };
    std::memset(&hd, 0, sizeof hd);
    hd.f[0] = take(L.f);
    hd.f[1] = take(L.f);
    hd.lam[0] = (double *)take(L.lam);
    hd.lam[1] = (double *)take(L.lam);
    hd.omegaf = L.omega ? (void *)take(L.omega) : nullptr;
    if (aux) q = aux;  // the auxiliary part lives apart from the state
    hd.cs = (const double2 *)take(L.cs);
    dd = (SolveDesc *)take(L.desc);
    hd.state = (SolveState *)take(L.state);
    hd.wpart = (double *)take(L.wpart);
    hd.hist = (pdbm_diag *)take(L.hist);
    cpart = (double *)take(L.cpart);

    hd.nr = p.nr;
    hd.nt = p.ntheta;
    hd.pitch = L.pitch;
    hd.sector = p.sector;
    hd.m = p.m;
    hd.n = p.n;
    hd.disc = p.r_min == 0.0;
    hd.reacts = (p.w1 > 0.0 || p.w2 > 0.0) ? 1 : 0;
    hd.rows = rows;
    hd.nwaves = L.nwaves;
    hd.nstrip = (p.ntheta + STRIP - 1) / STRIP;
    hd.diag_every = p.diag_every;
    hd.plane = L.pitch;
    hd.rstride = (int64_t)NQ * L.pitch;
    hd.nsteps = nsteps;
    hd.dr = (p.r_max - p.r_min) / p.nr;
    hd.dth = p.sector * M_PI / 4.0 / p.ntheta;
    hd.r_min = p.r_min;
    hd.dt_dr = p.dt / hd.dr;
    hd.dt_dth = p.dt / hd.dth;
    hd.omega = std::exp(-p.dt / p.tau);
    hd.w1 = p.w1;
    hd.w2 = p.w2;
    hd.Q = p.Q;
    hd.T_th = p.T_th;
    hd.dt = p.dt;
    pdbm_fk_matrix(hd.A);

    // theta table (in pieces through a buffer on the stack, each copy
    // waited for before the buffer is refilled), description, zeroed
    // counters, then the initial state.  Host sources of the asynchronous
    // copies (hd, zero_state) must outlive them: the caller synchronises st
    // before returning to its own caller.
    const double dth = hd.dth;
    double2 piece[256];
    for (int j0 = 0; j0 < p.ntheta; j0 += 256) {
        const int n = std::min(256, p.ntheta - j0);
        for (int j = 0; j < n; ++j)
            piece[j] = make_double2(std::cos((j0 + j + 0.5) * dth), std::sin((j0 + j + 0.5) * dth));
        HIPCHK(hipMemcpyAsync((void *)(hd.cs + j0), piece, n * sizeof(double2), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    zero_state = SolveState{0};
    HIPCHK(hipMemcpyAsync(dd, &hd, sizeof hd, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(hd.state, &zero_state, sizeof zero_state, hipMemcpyHostToDevice, st));
    pdbm_ic uni;
    if (!ic) {
        std::memset(&uni, 0, sizeof uni);
        for (double *t : {uni.inner, uni.outer}) {
            t[0] = 1.0;
            t[1] = 1.0;
        }
        ic = &uni;
    }
    HIPCHK(launch_init_ic(hd, 0, fp32, *ic, st));
    if (hd.omegaf) HIPCHK(launch_omega(hd, fp32, nullptr, hd.omega, st));  // every cell starts with the parameters' tau
    step = 0;
    flip = 0;
    rec_from = 0;
    red_to = 0;
    return PDBM_OK;
}

void Solve::release()
{
    if (own && ws) (void)hipFree(ws);
    ws = nullptr;
    own = false;
}

int Solve::set_step(int64_t s, hipStream_t st)
{
    zero_state = SolveState{s};
    HIPCHK(hipMemcpyAsync(hd.state, &zero_state, sizeof zero_state, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    step = s;
    flip = 0;
    rec_from = s;
    red_to = s;
    return PDBM_OK;
}

// PDBM_FUSE=0: every launch takes a single step (read once per process).
static bool fuse_off()
{
    static const bool off = [] {
        const char *e = std::getenv("PDBM_FUSE");
        return e && e[0] == '0';
    }();
    return off;
}

bool Solve::fusable() const { return !fuse_off() && p.ntheta > 1 && L.rows <= FUSE_ROWS; }

bool Solve::columnar() const { return !fuse_off() && p.ntheta == 1; }

int Solve::reduce_records(hipStream_t st)
{
    // a solve that makes no records has no partial sums to add up
    if (step > red_to && p.diag_every > 0) HIPCHK(launch_records(dd, 1, nullptr, red_to, step, st));
    red_to = step;
    return PDBM_OK;
}

int Solve::moments(double *out, pdbm_diag *diag_dev, hipStream_t st) const
{
    DiagCtl c;
    c.partials = cpart;
    c.out = diag_dev;
    c.step = step;
    HIPCHK(launch_moments(hd, cur(), fp32, out, c, st));
    return PDBM_OK;
}

int pdbm::noneq_to_host(const Solve &s, double *out, hipStream_t st)
{
    // the idle f buffer (at least 33 x 4 bytes per cell) stages the 12 float64 values
    double *stage = (double *)s.hd.f[s.cur() ^ 1];
    HIPCHK(launch_noneq(s.hd, s.cur(), s.fp32, stage, st));
    HIPCHK(hipMemcpyAsync(out, stage, (size_t)NONEQ * s.p.nr * s.p.ntheta * sizeof(double), hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipStreamSynchronize(st));
    return PDBM_OK;
}

// ------------------------------------------------------------ one solve ABI --
extern "C" {

int pdbm_create(const pdbm_params *p, const pdbm_ic *ic, void *workspace, size_t workspace_bytes, void *stream,
                pdbm_solver **out)
{
    if (!out) return fail(PDBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = pdbm_validate(p, ic, nullptr);
    if (rc) return rc;
    if ((rc = check_device())) return rc;
    pdbm_solver *h = new (std::nothrow) pdbm_solver;
    if (!h) return fail(PDBM_ENOMEM, "host allocation failed");
    h->st = (hipStream_t)stream;
    rc = h->s.init(*p, ic, workspace, workspace_bytes, rows_per_wave(*p), INT64_MAX, h->st);
    if (rc == PDBM_OK && hipStreamSynchronize(h->st) != hipSuccess) rc = fail(PDBM_EHIP, "initialisation failed");
    if (rc) {
        (void)hipStreamSynchronize(h->st);
        h->s.release();
        delete h;
        return rc;
    }
    *out = h;
    return PDBM_OK;
}

void pdbm_destroy(pdbm_solver *h)
{
    if (!h) return;
    if (h->s.ws) (void)hipStreamSynchronize(h->st);
    h->s.release();
    if (h->scratch_dev >= 0)
        release_scratch_solver(h->scratch_dev);  // the handle is that device's static slot
    else
        delete h;
}

int pdbm_set_fields(pdbm_solver *h, const double *fields)
{
    if (!h || !fields) return fail(PDBM_EINVAL, "NULL argument");
    Solve &s = h->s;
    const size_t n = (size_t)5 * s.p.nr * s.p.ntheta;
    HIPCHK(hipStreamSynchronize(h->st));
    // stage the fields in buffer 1 (at least 132 bytes per cell), build the
    // state in buffer 0, and restart the step count
    double *stage = (double *)s.hd.f[1];
    HIPCHK(hipMemcpyAsync(stage, fields, n * sizeof(double), hipMemcpyHostToDevice, h->st));
    HIPCHK(launch_init_fields(s.hd, 0, s.fp32, stage, h->st));
    return s.set_step(0, h->st);
}

int pdbm_set_tau(pdbm_solver *h, const double *tau)
{
    if (!h) return fail(PDBM_EINVAL, "NULL solver");
    Solve &s = h->s;
    if (!s.tauf()) return fail(PDBM_EINVAL, "the solve was created without PDBM_TAU_FIELD");
    HIPCHK(hipStreamSynchronize(h->st));
    if (!tau) {
        HIPCHK(launch_omega(s.hd, s.fp32, nullptr, s.hd.omega, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        return PDBM_OK;
    }
    const size_t n = (size_t)s.p.nr * s.p.ntheta;
    for (size_t c = 0; c < n; ++c)
        if (!(tau[c] > 0.0)) return fail(PDBM_EINVAL, "tau must be > 0 (or +inf) in every cell");
    // the idle f buffer (at least 132 bytes per cell) stages the field
    double *stage = (double *)s.hd.f[s.cur() ^ 1];
    HIPCHK(hipMemcpyAsync(stage, tau, n * sizeof(double), hipMemcpyHostToDevice, h->st));
    HIPCHK(launch_omega(s.hd, s.fp32, stage, 0.0, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return PDBM_OK;
}

int pdbm_set_tau_async(pdbm_solver *h, const void *tau_device)
{
    if (!h || !tau_device) return fail(PDBM_EINVAL, "NULL argument");
    if (!h->s.tauf()) return fail(PDBM_EINVAL, "the solve was created without PDBM_TAU_FIELD");
    HIPCHK(launch_omega(h->s.hd, h->s.fp32, (const double *)tau_device, 0.0, h->st));
    return PDBM_OK;
}

int pdbm_step(pdbm_solver *h, int64_t nsteps)
{
    if (!h || nsteps < 0) return fail(PDBM_EINVAL, "bad solver or step count");
    Solve &s = h->s;
    const bool pairs = s.fusable();
    const bool column = s.columnar();
    const int most = column ? COL_K : 2;  // steps of one launch, at most
    for (int64_t i = 0; i < nsteps;) {
        if (column) {
            // a single column: up to COL_K steps per launch; the state moves
            // to the other buffer, which toggles the parity unless nk is odd
            const int nk = (int)std::min<int64_t>(COL_K, nsteps - i);
            HIPCHK(launch_column(s.dd, nullptr, s.waves(), nullptr, s.step, nullptr, s.flip, nk, s.fp32, s.tauf(),
                                 h->st));
            s.step += nk;
            s.flip ^= (nk + 1) & 1;
            i += nk;
        } else if (pairs && nsteps - i >= 2) {
            HIPCHK(launch_step2(s.dd, nullptr, s.waves(), nullptr, s.step, nullptr, s.flip, false, s.fp32, s.tauf(),
                                s.rot(), h->st));
            s.step += 2;
            s.flip ^= 1;
            i += 2;
        } else {
            HIPCHK(launch_step(s.dd, nullptr, s.waves(), nullptr, s.step, nullptr, s.flip, s.fp32, s.rot(), s.tauf(),
                               h->st));
            s.step += 1;
            i += 1;
        }
        // the partial-sum ring holds PART_RING records: add them up before
        // the next launch (at most `most` steps) could overwrite one
        if (s.step - s.red_to > PART_RING - most) {
            int rc = s.reduce_records(h->st);
            if (rc) return rc;
        }
    }
    return PDBM_OK;
}

int64_t pdbm_step_count(const pdbm_solver *h) { return h ? h->s.step : -1; }

int pdbm_moments(pdbm_solver *h, double *out, pdbm_diag *diag)
{
    if (!h) return fail(PDBM_EINVAL, "NULL solver");
    Solve &s = h->s;
    double *stage = out ? (double *)s.hd.f[s.cur() ^ 1] : nullptr;  // idle buffer holds 6 doubles per cell
    pdbm_diag *dslot = s.hd.hist + HIST_CAP;
    int rc = s.moments(stage, dslot, h->st);
    if (rc) return rc;
    pdbm_diag d;
    if (out)
        HIPCHK(hipMemcpyAsync(out, stage, (size_t)6 * s.p.nr * s.p.ntheta * sizeof(double), hipMemcpyDeviceToHost,
                              h->st));
    HIPCHK(hipMemcpyAsync(&d, dslot, sizeof d, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    d.step = s.step;
    if (diag) *diag = d;
    if (d.n_nonfinite || d.n_nonphys) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "step %lld: %lld non-finite cells, %lld cells with rho<=0 or T<=0",
                      (long long)s.step, (long long)d.n_nonfinite, (long long)d.n_nonphys);
        return fail(PDBM_ENONPHYS, buf);
    }
    return PDBM_OK;
}

int pdbm_moments_async(pdbm_solver *h, void *out_device)
{
    if (!h || !out_device) return fail(PDBM_EINVAL, "NULL argument");
    return h->s.moments((double *)out_device, h->s.hd.hist + HIST_CAP, h->st);
}

int pdbm_noneq(pdbm_solver *h, double *out)
{
    if (!h || !out) return fail(PDBM_EINVAL, "NULL argument");
    Solve &s = h->s;
    return noneq_to_host(s, out, h->st);
}

int pdbm_noneq_async(pdbm_solver *h, void *out_device)
{
    if (!h || !out_device) return fail(PDBM_EINVAL, "NULL argument");
    HIPCHK(launch_noneq(h->s.hd, h->s.cur(), h->s.fp32, (double *)out_device, h->st));
    return PDBM_OK;
}

int pdbm_diag_history(pdbm_solver *h, pdbm_diag *out, int32_t cap, int32_t *n)
{
    if (!h || !n || cap < 0 || (cap > 0 && !out)) return fail(PDBM_EINVAL, "bad argument");
    Solve &s = h->s;
    int rc = s.reduce_records(h->st);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->st));
    *n = 0;
    const int64_t de = s.p.diag_every;
    if (de <= 0 || s.step <= s.rec_from) return PDBM_OK;
    // records k cover steps k*de in [rec_from, step); the ring keeps HIST_CAP
    int64_t k1 = (s.step - 1) / de + 1;          // one past the last record
    int64_t k0 = (s.rec_from + de - 1) / de;     // first record since the reset
    if (k1 - k0 > HIST_CAP) k0 = k1 - HIST_CAP;
    if (k1 - k0 > cap) k0 = k1 - cap;
    for (int64_t k = k0; k < k1; ++k)
        HIPCHK(hipMemcpy(out + (k - k0), s.hd.hist + (k % HIST_CAP), sizeof(pdbm_diag), hipMemcpyDeviceToHost));
    *n = (int32_t)(k1 - k0);
    return PDBM_OK;
}

}  // extern "C"

// f on the device: r rows of 33 * pitch elements in the paired layout of
// elem_of; host arrays are [NQ][nr][ntheta].  Whole buffers are copied and
// rearranged on the host.
static hipError_t f_to_host(const Solve &s, void *host)
{
    const int nr = s.p.nr, nt = s.p.ntheta;
    const size_t esz = s.L.esz, pitch = s.L.pitch, rstride = (size_t)NQ * pitch;
    std::vector<char> raw((size_t)nr * rstride * esz);
    hipError_t e = hipMemcpy(raw.data(), s.hd.f[s.cur()], raw.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    for (int q = 0; q < NQ; ++q)
        for (int ir = 0; ir < nr; ++ir)
            for (int jt = 0; jt < nt; ++jt)
                std::memcpy((char *)host + (((size_t)q * nr + ir) * nt + jt) * esz,
                            raw.data() + (ir * rstride + elem_of(q, jt, pitch)) * esz, esz);
    return hipSuccess;
}

static hipError_t f_to_device(const Solve &s, int buf, const void *host)
{
    const int nr = s.p.nr, nt = s.p.ntheta;
    const size_t esz = s.L.esz, pitch = s.L.pitch, rstride = (size_t)NQ * pitch;
    std::vector<char> raw((size_t)nr * rstride * esz, 0);
    for (int q = 0; q < NQ; ++q)
        for (int ir = 0; ir < nr; ++ir)
            for (int jt = 0; jt < nt; ++jt)
                std::memcpy(raw.data() + (ir * rstride + elem_of(q, jt, pitch)) * esz,
                            (const char *)host + (((size_t)q * nr + ir) * nt + jt) * esz, esz);
    return hipMemcpy(s.hd.f[buf], raw.data(), raw.size(), hipMemcpyHostToDevice);
}

extern "C" {

int pdbm_read_f(pdbm_solver *h, double *f, double *lam)
{
    if (!h) return fail(PDBM_EINVAL, "NULL solver");
    const Solve &s = h->s;
    const int nr = s.p.nr, nt = s.p.ntheta, pitch = s.L.pitch;
    const size_t ncell = (size_t)nr * nt;
    HIPCHK(hipStreamSynchronize(h->st));
    if (f) {
        if (s.fp32) {
            std::vector<float> tmp((size_t)NQ * ncell);
            HIPCHK(f_to_host(s, tmp.data()));
            for (size_t i = 0; i < tmp.size(); ++i) f[i] = tmp[i];
        } else {
            HIPCHK(f_to_host(s, f));
        }
    }
    if (lam)
        HIPCHK(hipMemcpy2D(lam, nt * sizeof(double), s.hd.lam[s.cur()], pitch * sizeof(double), nt * sizeof(double),
                           nr, hipMemcpyDeviceToHost));
    return PDBM_OK;
}

int pdbm_write_f(pdbm_solver *h, const double *f, const double *lam, int64_t step)
{
    if (!h || step < 0) return fail(PDBM_EINVAL, "bad argument");
    Solve &s = h->s;
    const int nr = s.p.nr, nt = s.p.ntheta, pitch = s.L.pitch;
    const size_t ncell = (size_t)nr * nt;
    HIPCHK(hipStreamSynchronize(h->st));
    const int cur = s.cur(), buf = (int)(step & 1);
    if (cur != buf) {  // the state must end up in the buffer of the new step's parity
        if (!f || !lam) {
            HIPCHK(hipMemcpy(s.hd.f[buf], s.hd.f[cur], s.L.f, hipMemcpyDeviceToDevice));
            HIPCHK(hipMemcpy(s.hd.lam[buf], s.hd.lam[cur], s.L.lam, hipMemcpyDeviceToDevice));
        }
    }
    if (f) {
        if (s.fp32) {
            std::vector<float> tmp((size_t)NQ * ncell);
            for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (float)f[i];
            HIPCHK(f_to_device(s, buf, tmp.data()));
        } else {
            HIPCHK(f_to_device(s, buf, f));
        }
    }
    if (lam)
        HIPCHK(hipMemcpy2D(s.hd.lam[buf], pitch * sizeof(double), lam, nt * sizeof(double), nt * sizeof(double), nr,
                           hipMemcpyHostToDevice));
    return s.set_step(step, h->st);
}

namespace {
struct BlobHeader {
    uint64_t magic;
    int32_t version, nr, ntheta, precision;
    int64_t step;
};
constexpr uint64_t BLOB_MAGIC = 0x3130455441545344ull;  // "DSTATE01"
}  // namespace

int pdbm_get_state(pdbm_solver *h, void *buf, size_t *bytes)
{
    if (!h || !bytes) return fail(PDBM_EINVAL, "NULL argument");
    const Solve &s = h->s;
    const int nr = s.p.nr, nt = s.p.ntheta, pitch = s.L.pitch;
    const size_t fb = (size_t)NQ * nr * nt * s.L.esz, lb = (size_t)nr * nt * sizeof(double);
    const size_t need = sizeof(BlobHeader) + fb + lb;
    if (!buf) {
        *bytes = need;
        return PDBM_OK;
    }
    if (*bytes < need) return fail(PDBM_ENOMEM, "checkpoint buffer too small");
    BlobHeader hh{BLOB_MAGIC, 1, nr, nt, s.p.precision, s.step};
    std::memcpy(buf, &hh, sizeof hh);
    char *fdst = (char *)buf + sizeof hh;
    HIPCHK(hipStreamSynchronize(h->st));
    HIPCHK(f_to_host(s, fdst));
    HIPCHK(hipMemcpy2D(fdst + fb, nt * sizeof(double), s.hd.lam[s.cur()], pitch * sizeof(double), nt * sizeof(double),
                       nr, hipMemcpyDeviceToHost));
    *bytes = need;
    return PDBM_OK;
}

int pdbm_set_state(pdbm_solver *h, const void *buf, size_t bytes)
{
    if (!h || !buf || bytes < sizeof(BlobHeader)) return fail(PDBM_EINVAL, "bad argument");
    Solve &s = h->s;
    BlobHeader hh;
    std::memcpy(&hh, buf, sizeof hh);
    const int nr = s.p.nr, nt = s.p.ntheta, pitch = s.L.pitch;
    const size_t fb = (size_t)NQ * nr * nt * s.L.esz, lb = (size_t)nr * nt * sizeof(double);
    if (hh.magic != BLOB_MAGIC || hh.version != 1 || hh.nr != nr || hh.ntheta != nt || hh.precision != s.p.precision ||
        hh.step < 0 || bytes < sizeof hh + fb + lb)
        return fail(PDBM_EINVAL, "checkpoint does not match this solve");
    const char *src = (const char *)buf + sizeof hh;
    const int b = (int)(hh.step & 1);
    HIPCHK(hipStreamSynchronize(h->st));
    HIPCHK(f_to_device(s, b, src));
    HIPCHK(hipMemcpy2D(s.hd.lam[b], pitch * sizeof(double), src + fb, nt * sizeof(double), nt * sizeof(double), nr,
                       hipMemcpyHostToDevice));
    return s.set_step(hh.step, h->st);
}

}  // extern "C"
