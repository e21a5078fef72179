/*
 * A plain C consumer of libpdbm's ABI (include/pdbm.h), with no Python and
 * no torch in the process: the boundary works for any C caller.
 *
 *   pdbm_c_client cpu            host-side entry points; creating a solve
 *                                must fail cleanly when no GPU is usable
 *   pdbm_c_client gpu OUT.bin    a single solve (64 x 64 annulus, 50 steps,
 *                                fields written to OUT.bin as float64
 *                                [6][64][64]), a packed batch and the
 *                                request server, end to end
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pdbm.h"

static int fails = 0;

#define CHECK(cond, ...)                                                  \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "FAILED %s:%d: ", __FILE__, __LINE__);        \
            fprintf(stderr, __VA_ARGS__);                                 \
            fprintf(stderr, " [last error: %s]\n", pdbm_last_error());    \
            fails++;                                                      \
        }                                                                 \
    } while (0)

/* The 64 x 64 annulus r in [0.1, 1]: ignition disc r < 0.2 at rho = 1.5,
 * p = 20, burnt; unburnt rho = p = 1 at rest outside. */
static pdbm_params small_params(int precision)
{
    pdbm_params p;
    memset(&p, 0, sizeof p);
    p.nr = 64;
    p.ntheta = 64;
    p.sector = 8;
    p.precision = precision;
    p.m = 2;
    p.n = 2;
    p.diag_every = 10;
    p.r_min = 0.1;
    p.r_max = 1.0;
    p.dt = 1e-5;
    p.tau = 2e-5;
    p.w1 = 2.0;
    p.w2 = 2.0;
    p.Q = 1.0;
    p.T_th = 1.1;
    return p;
}

static pdbm_ic small_ic(uint64_t seed)
{
    pdbm_ic ic;
    const double inner[5] = {1.5, 20.0 / 1.5, 0.0, 0.0, 1.0};
    const double outer[5] = {1.0, 1.0, 0.0, 0.0, 0.0};
    memset(&ic, 0, sizeof ic);
    ic.r_split = 0.2;
    memcpy(ic.inner, inner, sizeof inner);
    memcpy(ic.outer, outer, sizeof outer);
    ic.p_noise = 1e-6;
    ic.seed = seed;
    return ic;
}

static int cpu_checks(void)
{
    static const int codes[] = {PDBM_OK, PDBM_EINVAL, PDBM_ECFL, PDBM_ENOMEM, PDBM_EHIP,
                                PDBM_EAGAIN, PDBM_ENOENT, PDBM_ENONPHYS, PDBM_ENOSYS};
    for (size_t i = 0; i < sizeof codes / sizeof codes[0]; ++i)
        CHECK(pdbm_strerror(codes[i]) && pdbm_strerror(codes[i])[0], "strerror(%d)", codes[i]);
    CHECK(pdbm_version() > 0, "version");

    pdbm_params p = small_params(PDBM_FP64);
    pdbm_ic ic = small_ic(0);
    double cfl = -1.0;
    CHECK(pdbm_validate(&p, &ic, &cfl) == PDBM_OK && cfl > 0.0 && cfl < 1.0, "validate ok (cfl %g)", cfl);
    pdbm_params bad = p;
    bad.nr = 0;
    CHECK(pdbm_validate(&bad, &ic, NULL) == PDBM_EINVAL, "nr = 0");
    bad = p;
    bad.sector = 9;
    CHECK(pdbm_validate(&bad, &ic, NULL) == PDBM_EINVAL, "sector = 9");
    bad = p;
    bad.dt = 1e-2;
    CHECK(pdbm_validate(&bad, &ic, NULL) == PDBM_ECFL, "Courant bound");
    bad.flags = PDBM_ALLOW_CFL;
    CHECK(pdbm_validate(&bad, &ic, NULL) == PDBM_OK, "Courant override");
    pdbm_ic badic = ic;
    badic.inner[1] = -1.0;
    CHECK(pdbm_validate(&p, &badic, NULL) == PDBM_EINVAL, "negative T");

    /* the weights from the matrix meet the moment constraints they invert */
    double A[16];
    CHECK(pdbm_fk_matrix(A) == PDBM_OK, "fk_matrix");
    const double v[4] = {1.5, 3.5, 7.5, 12.5}, T = 1.7;
    double F[4];
    for (int k = 0; k < 4; ++k) {
        F[k] = 0.0;
        for (int n = 0; n < 4; ++n) F[k] += A[4 * k + n] * pow(T, n + 1);
    }
    double fact = 1.0;
    for (int n = 1; n <= 4; ++n) {
        fact *= n;
        double lhs = 0.0;
        for (int k = 0; k < 4; ++k) lhs += 8.0 * F[k] * pow(v[k], 2 * n);
        const double rhs = pow(2.0, n) * fact * pow(T, n);
        CHECK(fabs(lhs - rhs) <= 1e-12 * rhs, "moment %d: %g vs %g", n, lhs, rhs);
    }

    size_t bytes = 0;
    CHECK(pdbm_state_bytes(&p, &bytes) == PDBM_OK && bytes >= 2 * 33 * 64 * 64 * sizeof(double), "state bytes");

    pdbm_solver *s = NULL;
    const int rc = pdbm_create(&p, &ic, NULL, 0, NULL, &s);
    CHECK((rc == PDBM_ENOSYS || rc == PDBM_EHIP) && s == NULL, "create without a GPU gave %d", rc);
    if (!fails) printf("cpu ok\n");
    return fails != 0;
}

static int gpu_run(const char *out_path)
{
    /* one solve */
    pdbm_params p = small_params(PDBM_FP64);
    pdbm_ic ic = small_ic(0);
    pdbm_solver *s = NULL;
    int rc = pdbm_create(&p, &ic, NULL, 0, NULL, &s);
    CHECK(rc == PDBM_OK, "create: %d", rc);
    if (rc) return 1;
    CHECK(pdbm_step(s, 50) == PDBM_OK, "step");
    CHECK(pdbm_step_count(s) == 50, "step count");
    const size_t n = (size_t)6 * p.nr * p.ntheta;
    double *out = (double *)malloc(n * sizeof(double));
    pdbm_diag d;
    CHECK(pdbm_moments(s, out, &d) == PDBM_OK && d.step == 50, "moments");
    FILE *f = fopen(out_path, "wb");
    CHECK(f && fwrite(out, sizeof(double), n, f) == n, "write %s", out_path);
    if (f) fclose(f);
    pdbm_diag hist[8];
    int32_t nh = 0;
    CHECK(pdbm_diag_history(s, hist, 8, &nh) == PDBM_OK && nh == 5 && hist[0].step == 0 && hist[4].step == 40,
          "history (%d records)", nh);
    for (int i = 1; i < nh; ++i) CHECK(fabs(hist[i].mass / hist[0].mass - 1.0) < 1e-2, "mass drift");
    pdbm_destroy(s);

    /* a packed batch of two FP32 solves, graph chunks of 5 steps */
    pdbm_params bp[2] = {small_params(PDBM_FP32), small_params(PDBM_FP32)};
    bp[1].nr = 40;
    bp[1].ntheta = 100;
    pdbm_ic bic[2] = {small_ic(1), small_ic(2)};
    pdbm_batch *b = NULL;
    CHECK(pdbm_batch_create(2, bp, bic, 5, NULL, &b) == PDBM_OK, "batch create");
    if (b) {
        CHECK(pdbm_batch_step(b, 23) == PDBM_OK && pdbm_batch_step_count(b, 1) == 23, "batch step");
        double *bo = (double *)malloc((size_t)6 * 40 * 100 * sizeof(double));
        CHECK(pdbm_batch_moments(b, 1, bo, &d) == PDBM_OK && d.n_nonfinite == 0 && d.n_nonphys == 0, "batch moments");
        free(bo);
        pdbm_batch_destroy(b);
    }

    /* the request server: three requests, two slots */
    pdbm_server *srv = NULL;
    CHECK(pdbm_server_create((size_t)1 << 30, 2, 5, NULL, &srv) == PDBM_OK, "server create");
    if (srv) {
        uint64_t id[3];
        for (int i = 0; i < 3; ++i) {
            pdbm_params rp = small_params(i == 1 ? PDBM_FP64 : PDBM_FP32);
            pdbm_ic ric = small_ic(10 + i);
            CHECK(pdbm_submit(srv, &rp, &ric, 20 + 5 * i, PDBM_KEEP_FIELDS, &id[i]) == PDBM_OK, "submit %d", i);
        }
        CHECK(pdbm_server_wait(srv, 60.0) == PDBM_OK, "wait");
        for (int i = 0; i < 3; ++i) {
            int32_t state = -1;
            CHECK(pdbm_poll(srv, id[i], &state, out, &d) == PDBM_OK && state == PDBM_DONE, "poll %d", i);
            CHECK(d.step == 20 + 5 * i, "request %d step %lld", i, (long long)d.step);
            double t[3];
            CHECK(pdbm_request_times(srv, id[i], t) == PDBM_OK && 0 <= t[0] && t[0] <= t[1] && t[1] <= t[2],
                  "times %d", i);
            CHECK(pdbm_release(srv, id[i]) == PDBM_OK, "release %d", i);
        }
        int32_t state;
        CHECK(pdbm_poll(srv, id[0], &state, NULL, NULL) == PDBM_ENOENT, "released id is gone");
        pdbm_server_stats st;
        CHECK(pdbm_server_get_stats(srv, &st) == PDBM_OK && st.done == 3 && st.failed == 0, "stats");
        pdbm_server_destroy(srv);
    }
    free(out);
    if (!fails) printf("gpu ok\n");
    return fails != 0;
}

int main(int argc, char **argv)
{
    if (argc >= 2 && !strcmp(argv[1], "cpu")) return cpu_checks();
    if (argc >= 3 && !strcmp(argv[1], "gpu")) return gpu_run(argv[2]);
    fprintf(stderr, "usage: %s cpu | gpu OUT.bin\n", argv[0]);
    return 2;
}
