/*
 * pdbm_oracle.c -- plain, slow CPU oracle of the polar-coordinate lattice
 * Boltzmann kinetic model of detonation (Lin, Xu, Zhang, Li, arXiv:1308.0653).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU path.
 *
 * It is written to be checked against the paper by eye, not to be fast:
 *   - array-of-structures state f[ir][jt][q], q = 0 (rest) or 1+8(k-1)+i;
 *   - discrete velocities in the paper's polar components
 *     v_kir = v_k cos(i pi/4 - theta), v_kitheta = v_k sin(i pi/4 - theta)
 *     (Sec. II.B, velocity-model equation);
 *   - every quantity evaluated literally from its defining formula, in the
 *     order the paper gives it.  The only speed-up is an OpenMP loop over
 *     cells (each cell reads time-t arrays only, so the order is irrelevant).
 *
 * Arithmetic type: `real`, double by default.  Building with
 * -DORA_REAL="long double" gives an extended-precision copy used to bound the
 * oracle's own rounding drift.
 *
 * Readings of points where the paper is silent, ambiguous or misprinted
 * (each is listed with its justification in the design notes of the repo):
 *   R1  F_k weights: the T-linear term enters with -1/4 (Sec. II.B).  Only
 *       that sign satisfies the moment constraints sum_k 8 F_k v_k^2n =
 *       2^n n! T^n, n=1..4, that the weights exist to meet.
 *   R2  v_ki = v_kir e_r + v_kitheta e_theta (the printed "v_kir e_theta" is
 *       a typo; the two components are given right after it).
 *   R3  The upwind fluxes f*_r, f*_theta of the LB evolution equation are
 *       SUBTRACTED (the lambda fluxes carry the minus sign explicitly; adding
 *       them would be anti-diffusive).
 *   R4  Cochran closed form (Sec. III.A): the denominator term is
 *       +b(1-lambda), the exact solution of dlambda/dt = (1-lambda)(a+b
 *       lambda); the printed "+a(1-lambda)" violates lambda(dt=0)=lambda.
 *   R5  gamma = 2 is fixed by the model (D = 2, T = 2E/(D rho)).
 *   R6  The reaction (rate R in the chemical term M and in lambda) acts only
 *       where the own-cell temperature at time t is strictly above T_th.
 *   R7  M uses R(lambda^t, P^t) explicitly.
 *   R8  Unsplit update: collision, M and both fluxes all use time-t values.
 *   R9  C_r, C_theta use r, theta of the updated cell.
 *   R10 Cell-centred grid r_i = r_min + (i+1/2) dr, theta_j = (j+1/2) dtheta.
 *   R11 Azimuthal domain is a sector of s*pi/4 (s = 1..8); the periodic halo
 *       rotates the velocity index: f_{k,i}(-1) = f_{k,(i+s)%8}(Ntheta-1),
 *       f_{k,i}(Ntheta) = f_{k,(i-s)%8}(0).  s = 8 is the full annulus.
 *   R12 Radial "inflow/outflow" boundaries: zero-gradient ghost cells.
 *   R13 Disc centre (r_min = 0): the paper's ghost rule
 *       f(-1, j, k, i) = f(0, j, k, (i+4)%8); lambda is mirrored.
 *   R14 Initial f = f^eq of the initial macroscopic state.
 *   R15 Initial-state noise: p = rho T + p_noise (2U-1),
 *       U = (splitmix64(seed ^ (cell * 0x9E3779B97F4A7C15)) >> 11) 2^-53,
 *       cell = ir*Ntheta + jt; rho unchanged, T = p / rho.
 *   R16 P^m with integer m by repeated multiplication.
 *   R17 lambda is not clamped.
 *   R18 If the reaction is gated off or a+b = 0: lambda_reac = lambda.
 *
 * Drift report (ora_diag): the paper defines none.  The sums are taken over
 * the cells with the area weight r_i dr dtheta of the cell-centred grid:
 * mass rho, energy rho T + rho |u|^2 / 2, chemical energy rho Q (1 - lambda);
 * cells with a non-finite moment or lambda are counted and left out of the
 * sums, and cells with rho <= 0 or T <= 0 are counted.
 *
 * Per-cell relaxation time (Sec. IV, point (ii)): the paper says tau should
 * depend on the local state but gives no form, so the oracle takes a field
 * tau[ir][jt] as an input (ora_set_tau) and relaxes each cell with its own
 * exp(-dt/tau); without a field every cell uses the parameters' tau.
 *
 * Parity unpinned: readings R7, R8 and R12.  The tests pin every other part
 * of this file to values the paper or the mathematics fix.  Nothing the
 * paper prints separates these three choices from their alternatives: the
 * explicit rate R inside M against an effective rate taken from the
 * closed-form lambda step (R7), the unsplit update against a split one
 * (R8), and the zero-gradient radial ghosts beyond the invariance of a
 * uniform state (R12).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>

#ifndef ORA_REAL
#define ORA_REAL double
#endif
typedef ORA_REAL real;

#define NQ 33
#define DIM 2 /* D, the spatial dimension (Sec. II.A) */

/* Problem parameters, mirrored by oracle.py. */
typedef struct {
    int32_t nr, ntheta, sector, m, n, pad_;
    double r_min, r_max, dt, tau, w1, w2, Q, T_th;
} ora_params;

typedef struct {
    ora_params p;
    real dr, dth;
    real *f, *fn;     /* [nr][ntheta][NQ] */
    real *lam, *lamn; /* [nr][ntheta]     */
    real *vr, *vt;    /* [ntheta][NQ]: polar velocity components per column */
    real *tau;        /* [nr][ntheta] per-cell relaxation time, or NULL: p.tau in every cell */
    long long step;
} ora_state;

/* Speeds of the D2V33 model (Sec. II.B): v0 = 0, v1..v4. */
static const double VK[5] = {0.0, 1.5, 3.5, 7.5, 12.5};

static real pi_(void) { return acos((real)-1); }

static int k_of(int q) { return q == 0 ? 0 : 1 + (q - 1) / 8; }
static int i_of(int q) { return q == 0 ? 0 : (q - 1) % 8; }
static int q_of(int k, int i) { return k == 0 ? 0 : 1 + 8 * (k - 1) + i; }

/* Velocity-set equation (Sec. II.B): polar components at azimuth theta. */
static void velocities(real theta, real vr[NQ], real vt[NQ])
{
    vr[0] = 0;
    vt[0] = 0;
    for (int k = 1; k <= 4; ++k)
        for (int i = 0; i < 8; ++i) {
            real ang = (real)i * pi_() / 4 - theta;
            vr[q_of(k, i)] = (real)VK[k] * cos(ang);
            vt[q_of(k, i)] = (real)VK[k] * sin(ang);
        }
}

/* Weighting coefficients F_k(T) (Sec. II.B, below the f^eq equation).
 * Index k+l wraps to k+l-4 when above 4.  Reading R1: -1/4 v^2 v^2 v^2 T. */
static void weights(real T, real F[5])
{
    real sum = 0;
    for (int k = 1; k <= 4; ++k) {
        int k1 = k + 1 > 4 ? k + 1 - 4 : k + 1;
        int k2 = k + 2 > 4 ? k + 2 - 4 : k + 2;
        int k3 = k + 3 > 4 ? k + 3 - 4 : k + 3;
        real a = (real)VK[k] * (real)VK[k];
        real b = (real)VK[k1] * (real)VK[k1];
        real c = (real)VK[k2] * (real)VK[k2];
        real d = (real)VK[k3] * (real)VK[k3];
        real den = a * (a - b) * (a - c) * (a - d);
        real num = 48 * T * T * T * T - 6 * (b + c + d) * T * T * T + (b * c + c * d + d * b) * T * T -
                   (real)0.25 * b * c * d * T;
        F[k] = num / den;
        sum += F[k];
    }
    F[0] = 1 - 8 * sum;
}

/* Equilibrium distribution, the f^eq equation of Sec. II.B. */
static void equilibrium(real rho, real ur, real ut, real T, const real vr[NQ], const real vt[NQ], real feq[NQ])
{
    real F[5];
    weights(T, F);
    real u2 = ur * ur + ut * ut;
    for (int q = 0; q < NQ; ++q) {
        real vu = vr[q] * ur + vt[q] * ut; /* v_ki,eps u_eps */
        real term0 = 1 - u2 / (2 * T) + u2 * u2 / (8 * T * T);
        real term1 = vu / T * (1 - u2 / (2 * T));
        real term2 = vu * vu / (2 * T * T) * (1 - u2 / (2 * T));
        real term3 = vu * vu * vu / (6 * T * T * T);
        real term4 = vu * vu * vu * vu / (24 * T * T * T * T);
        feq[q] = rho * F[k_of(q)] * (term0 + term1 + term2 + term3 + term4);
    }
}

/* Macroscopic quantities (Sec. II.B, text above the f^eq equation). */
static void moments(const real f[NQ], const real vr[NQ], const real vt[NQ], real *rho, real *ur, real *ut, real *T)
{
    real s0 = 0, sr = 0, st = 0;
    for (int q = 0; q < NQ; ++q) {
        s0 += f[q];
        sr += f[q] * vr[q];
        st += f[q] * vt[q];
    }
    *rho = s0;
    *ur = sr / s0;
    *ut = st / s0;
    real e = 0;
    for (int q = 0; q < NQ; ++q) {
        real cr = vr[q] - *ur, ct = vt[q] - *ut;
        e += (real)0.5 * f[q] * (cr * cr + ct * ct);
    }
    *T = e / s0;
}

/* Integer power (reading R16). */
static real ipow(real x, int e)
{
    real y = 1;
    for (int i = 0; i < e; ++i) y *= x;
    return y;
}

/* Cochran's closed-form lambda update (Sec. III.A, reading R4). */
static real cochran(real lam, real a, real b, real dt)
{
    if (a + b == 0) return lam; /* R18 */
    real E = exp((a + b) * dt);
    return ((a + b * lam) * E - a * (1 - lam)) / ((a + b * lam) * E + b * (1 - lam));
}

/* Collision of one cell: BGK relaxation with the cell's relaxation time tau
 * solved analytically over dt, plus the chemical term M dt (LB evolution
 * equation of Sec. II.C without the fluxes).  Returns moments and reaction
 * coefficients through the out-pointers. */
static void collide(const ora_params *p, const real f[NQ], real lam, const real vr[NQ], const real vt[NQ], real tau,
                    real out[NQ], real mom[4], real *a_out, real *b_out, int *react)
{
    real rho, ur, ut, T;
    moments(f, vr, vt, &rho, &ur, &ut, &T);
    real P = rho * T; /* P = rho T (m = 1, T = 2E/(D rho)) */
    real feq[NQ];
    equilibrium(rho, ur, ut, T, vr, vt, feq);

    /* Cochran rate (Sec. III.A), gated by the ignition temperature (R6). */
    real a = 0, b = 0, R = 0;
    int on = T > (real)p->T_th;
    if (on) {
        a = (real)p->w1 * ipow(P, p->m);
        b = (real)p->w2 * ipow(P, p->n);
        R = a * (1 - lam) + b * lam * (1 - lam);
    }
    real relax = exp(-(real)p->dt / tau);
    for (int q = 0; q < NQ; ++q) {
        real cr = vr[q] - ur, ct = vt[q] - ut;
        /* M_ki = f^eq (-D T + (v-u)^2) / (2 T^2) * (2Q/D) R (Sec. II.B) */
        real M = feq[q] * (-DIM * T + (cr * cr + ct * ct)) / (2 * T * T) * (2 * (real)p->Q / DIM) * R;
        out[q] = feq[q] + (f[q] - feq[q]) * relax + M * (real)p->dt;
    }
    if (mom) {
        mom[0] = rho;
        mom[1] = ur;
        mom[2] = ut;
        mom[3] = T;
    }
    if (a_out) *a_out = a;
    if (b_out) *b_out = b;
    if (react) *react = on;
}

/* ---------------------------------------------------------------- state --- */

static real *F_AT(ora_state *s, real *arr, int ir, int jt) { return arr + ((size_t)ir * s->p.ntheta + jt) * NQ; }

/* f_q at (ir, jt) including ghost cells (readings R11-R13). */
static real fget(ora_state *s, int ir, int jt, int q)
{
    int k = k_of(q), i = i_of(q);
    int nt = s->p.ntheta, sec = s->p.sector;
    if (jt < 0) { /* R11 */
        jt += nt;
        if (k > 0) i = (i + sec) % 8;
    } else if (jt >= nt) {
        jt -= nt;
        if (k > 0) i = ((i - sec) % 8 + 8) % 8;
    }
    if (ir < 0) {
        ir = 0;
        if (s->p.r_min == 0 && k > 0) i = (i + 4) % 8; /* R13: disc centre */
    } else if (ir >= s->p.nr) {
        ir = s->p.nr - 1; /* R12 */
    }
    return F_AT(s, s->f, ir, jt)[q_of(k, i)];
}

static real lget(ora_state *s, int ir, int jt)
{
    int nt = s->p.ntheta;
    if (jt < 0) jt += nt;
    if (jt >= nt) jt -= nt;
    if (ir < 0) ir = 0;
    if (ir >= s->p.nr) ir = s->p.nr - 1;
    return s->lam[(size_t)ir * nt + jt];
}

ora_state *ora_create(const ora_params *p)
{
    if (p->nr < 1 || p->ntheta < 1 || p->sector < 1 || p->sector > 8) return NULL;
    ora_state *s = (ora_state *)calloc(1, sizeof(ora_state));
    s->p = *p;
    s->dr = ((real)p->r_max - (real)p->r_min) / p->nr;
    s->dth = (real)p->sector * pi_() / 4 / p->ntheta;
    size_t nc = (size_t)p->nr * p->ntheta;
    s->f = (real *)calloc(nc * NQ, sizeof(real));
    s->fn = (real *)calloc(nc * NQ, sizeof(real));
    s->lam = (real *)calloc(nc, sizeof(real));
    s->lamn = (real *)calloc(nc, sizeof(real));
    s->vr = (real *)calloc((size_t)p->ntheta * NQ, sizeof(real));
    s->vt = (real *)calloc((size_t)p->ntheta * NQ, sizeof(real));
    for (int jt = 0; jt < p->ntheta; ++jt) velocities(((real)jt + (real)0.5) * s->dth, s->vr + jt * NQ, s->vt + jt * NQ);
    return s;
}

void ora_destroy(ora_state *s)
{
    if (!s) return;
    free(s->f);
    free(s->fn);
    free(s->lam);
    free(s->lamn);
    free(s->vr);
    free(s->vt);
    free(s->tau);
    free(s);
}

/* splitmix64 output function (Steele, Lea, Flood, OOPSLA 2014). */
static uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Two-region initial state with pressure noise (readings R14, R15).
 * inner/outer = (rho, T, u_r, u_theta, lambda), the paper's tuple order. */
void ora_init_ic(ora_state *s, double r_split, const double inner[5], const double outer[5], double p_noise,
                 uint64_t seed)
{
    int nr = s->p.nr, nt = s->p.ntheta;
    for (int ir = 0; ir < nr; ++ir) {
        double r = s->p.r_min + ((double)ir + 0.5) * (double)s->dr;
        const double *st = r < r_split ? inner : outer;
        for (int jt = 0; jt < nt; ++jt) {
            uint64_t cell = (uint64_t)ir * (uint64_t)nt + (uint64_t)jt;
            uint64_t h = splitmix64(seed ^ (cell * 0x9E3779B97F4A7C15ull));
            double U = (double)(h >> 11) * 0x1.0p-53;
            double pr = st[0] * st[1];
            pr = pr + p_noise * (2.0 * U - 1.0); /* built with -ffp-contract=off */
            double T = pr / st[0];
            equilibrium((real)st[0], (real)st[2], (real)st[3], (real)T, s->vr + jt * NQ, s->vt + jt * NQ,
                        F_AT(s, s->f, ir, jt));
            s->lam[(size_t)ir * nt + jt] = (real)st[4];
        }
    }
    s->step = 0;
}

/* Initial state from given macroscopic fields [5][nr][ntheta] = rho, T, u_r,
 * u_theta, lambda (reading R14, no noise added). */
void ora_init_fields(ora_state *s, const double *fields)
{
    size_t nc = (size_t)s->p.nr * s->p.ntheta;
    for (int ir = 0; ir < s->p.nr; ++ir)
        for (int jt = 0; jt < s->p.ntheta; ++jt) {
            size_t c = (size_t)ir * s->p.ntheta + jt;
            equilibrium((real)fields[c], (real)fields[2 * nc + c], (real)fields[3 * nc + c], (real)fields[nc + c],
                        s->vr + jt * NQ, s->vt + jt * NQ, F_AT(s, s->f, ir, jt));
            s->lam[c] = (real)fields[4 * nc + c];
        }
    s->step = 0;
}

/* Raw state access: f as [nr][ntheta][33], lambda as [nr][ntheta]. */
void ora_set_state(ora_state *s, const double *f, const double *lam, long long step)
{
    size_t nc = (size_t)s->p.nr * s->p.ntheta;
    for (size_t i = 0; i < nc * NQ; ++i) s->f[i] = (real)f[i];
    for (size_t i = 0; i < nc; ++i) s->lam[i] = (real)lam[i];
    s->step = step;
}

void ora_get_state(ora_state *s, double *f, double *lam)
{
    size_t nc = (size_t)s->p.nr * s->p.ntheta;
    for (size_t i = 0; i < nc * NQ; ++i) f[i] = (double)s->f[i];
    for (size_t i = 0; i < nc; ++i) lam[i] = (double)s->lam[i];
}

long long ora_step_count(ora_state *s) { return s->step; }

/* Per-cell relaxation time field [nr][ntheta] (Sec. IV, point (ii)), or NULL
 * for the parameters' tau everywhere. */
void ora_set_tau(ora_state *s, const double *tau)
{
    size_t nc = (size_t)s->p.nr * s->p.ntheta;
    if (!tau) {
        free(s->tau);
        s->tau = NULL;
        return;
    }
    if (!s->tau) s->tau = (real *)calloc(nc, sizeof(real));
    for (size_t i = 0; i < nc; ++i) s->tau[i] = (real)tau[i];
}

/* One time step of every cell: the LB evolution equation of Sec. II.C with
 * the fluxes f*_r, f*_theta, and the lambda update of Sec. III.A. */
static void step_once(ora_state *s)
{
    const ora_params *p = &s->p;
    int nr = p->nr, nt = p->ntheta;
    real dt = (real)p->dt, dr = s->dr, dth = s->dth;
#pragma omp parallel for schedule(static)
    for (int ir = 0; ir < nr; ++ir) {
        real r = (real)p->r_min + ((real)ir + (real)0.5) * dr;
        for (int jt = 0; jt < nt; ++jt) {
            const real *vr = s->vr + jt * NQ, *vt = s->vt + jt * NQ;
            real *fc = F_AT(s, s->f, ir, jt);
            real lam = s->lam[(size_t)ir * nt + jt];
            real tau = s->tau ? s->tau[(size_t)ir * nt + jt] : (real)p->tau;
            real coll[NQ], mom[4], a, b;
            int on;
            collide(p, fc, lam, vr, vt, tau, coll, mom, &a, &b, &on);

            real *fo = F_AT(s, s->fn, ir, jt);
            for (int q = 0; q < NQ; ++q) {
                real Cr = vr[q] * dt / dr;        /* C_r = v_kir dt / dr */
                real Ct = vt[q] * dt / (r * dth); /* C_theta = v_kitheta dt / (r dtheta) */
                real fs_r, fs_t;
                if (Cr >= 0)
                    fs_r = Cr * (fc[q] - fget(s, ir - 1, jt, q));
                else
                    fs_r = Cr * (fget(s, ir + 1, jt, q) - fc[q]);
                if (Ct >= 0)
                    fs_t = Ct * (fc[q] - fget(s, ir, jt - 1, q));
                else
                    fs_t = Ct * (fget(s, ir, jt + 1, q) - fc[q]);
                fo[q] = coll[q] - fs_r - fs_t; /* reading R3 */
            }

            /* lambda: analytic reaction plus upwind advection with own-cell u */
            real ur = mom[1], ut = mom[2];
            real lreac = on ? cochran(lam, a, b, dt) : lam;
            real ls_r, ls_t;
            if (ur >= 0)
                ls_r = -ur * (lam - lget(s, ir - 1, jt)) / dr * dt;
            else
                ls_r = -ur * (lget(s, ir + 1, jt) - lam) / dr * dt;
            if (ut >= 0)
                ls_t = -ut * (lam - lget(s, ir, jt - 1)) / (r * dth) * dt;
            else
                ls_t = -ut * (lget(s, ir, jt + 1) - lam) / (r * dth) * dt;
            s->lamn[(size_t)ir * nt + jt] = lreac + ls_r + ls_t;
        }
    }
    real *t = s->f;
    s->f = s->fn;
    s->fn = t;
    t = s->lam;
    s->lam = s->lamn;
    s->lamn = t;
    s->step++;
}

void ora_step(ora_state *s, long long nsteps)
{
    for (long long n = 0; n < nsteps; ++n) step_once(s);
}

/* Macroscopic fields [6][nr][ntheta]: rho, u_r, u_theta, T, p, lambda. */
void ora_fields(ora_state *s, double *out)
{
    int nr = s->p.nr, nt = s->p.ntheta;
    size_t nc = (size_t)nr * nt;
    for (int ir = 0; ir < nr; ++ir)
        for (int jt = 0; jt < nt; ++jt) {
            size_t c = (size_t)ir * nt + jt;
            real rho, ur, ut, T;
            moments(F_AT(s, s->f, ir, jt), s->vr + jt * NQ, s->vt + jt * NQ, &rho, &ur, &ut, &T);
            out[c] = (double)rho;
            out[nc + c] = (double)ur;
            out[2 * nc + c] = (double)ut;
            out[3 * nc + c] = (double)T;
            out[4 * nc + c] = (double)(rho * T);
            out[5 * nc + c] = (double)s->lam[c];
        }
}

/* Central moments of a distribution g about the velocity u (Sec. II.E),
 * in the polar components of the cell's frame, v* = v - u:
 *   M*_2     = sum g v* v*               -> out[0..2]  = rr, r theta, theta theta
 *   M*_3     = sum g v* v* v*            -> out[3..6]  = rrr, rr theta, r theta theta, theta theta theta
 *   M*_{3,1} = sum 1/2 g (v*.v*) v*      -> out[7..8]  = r, theta
 *   M*_{4,2} = sum 1/2 g (v*.v*) v* v*   -> out[9..11] = rr, r theta, theta theta */
static void central_moments(const real g[NQ], const real vr[NQ], const real vt[NQ], real ur, real ut, real out[12])
{
    for (int m = 0; m < 12; ++m) out[m] = 0;
    for (int q = 0; q < NQ; ++q) {
        real cr = vr[q] - ur, ct = vt[q] - ut;
        real h = (real)0.5 * (cr * cr + ct * ct);
        out[0] += g[q] * cr * cr;
        out[1] += g[q] * cr * ct;
        out[2] += g[q] * ct * ct;
        out[3] += g[q] * cr * cr * cr;
        out[4] += g[q] * cr * cr * ct;
        out[5] += g[q] * cr * ct * ct;
        out[6] += g[q] * ct * ct * ct;
        out[7] += g[q] * h * cr;
        out[8] += g[q] * h * ct;
        out[9] += g[q] * h * cr * cr;
        out[10] += g[q] * h * cr * ct;
        out[11] += g[q] * h * ct * ct;
    }
}

/* Non-equilibrium manifestations Delta*_m = M*_m(f) - M*_m(f^eq) of every
 * cell (Sec. II.E), u and f^eq from the cell's own moments; out is
 * [12][nr][ntheta] in the component order of central_moments. */
void ora_noneq(ora_state *s, double *out)
{
    int nr = s->p.nr, nt = s->p.ntheta;
    size_t nc = (size_t)nr * nt;
    for (int ir = 0; ir < nr; ++ir)
        for (int jt = 0; jt < nt; ++jt) {
            const real *vr = s->vr + jt * NQ, *vt = s->vt + jt * NQ;
            const real *f = F_AT(s, s->f, ir, jt);
            real rho, ur, ut, T, feq[NQ], mf[12], me[12];
            moments(f, vr, vt, &rho, &ur, &ut, &T);
            equilibrium(rho, ur, ut, T, vr, vt, feq);
            central_moments(f, vr, vt, ur, ut, mf);
            central_moments(feq, vr, vt, ur, ut, me);
            for (int m = 0; m < 12; ++m) out[m * nc + (size_t)ir * nt + jt] = (double)(mf[m] - me[m]);
        }
}

/* Global drift report: area-weighted sums over cells (weight r_i dr dtheta)
 * of mass rho, total energy rho T + rho u^2 / 2 and unreleased chemical
 * energy rho Q (1 - lambda); counts of cells with a non-finite value and of
 * cells with rho <= 0 or T <= 0. */
void ora_diag(ora_state *s, double out[3], long long counts[2])
{
    int nr = s->p.nr, nt = s->p.ntheta;
    real m = 0, e = 0, c = 0;
    long long nonfinite = 0, nonphys = 0;
    for (int ir = 0; ir < nr; ++ir) {
        real r = (real)s->p.r_min + ((real)ir + (real)0.5) * s->dr;
        real w = r * s->dr * s->dth;
        for (int jt = 0; jt < nt; ++jt) {
            real rho, ur, ut, T;
            moments(F_AT(s, s->f, ir, jt), s->vr + jt * NQ, s->vt + jt * NQ, &rho, &ur, &ut, &T);
            real lam = s->lam[(size_t)ir * nt + jt];
            if (!isfinite(rho) || !isfinite(T) || !isfinite(ur) || !isfinite(ut) || !isfinite(lam)) {
                nonfinite++;
                continue;
            }
            if (rho <= 0 || T <= 0) nonphys++;
            m += rho * w;
            e += (rho * T + (real)0.5 * rho * (ur * ur + ut * ut)) * w;
            c += rho * (real)s->p.Q * (1 - lam) * w;
        }
    }
    out[0] = (double)m;
    out[1] = (double)e;
    out[2] = (double)c;
    counts[0] = nonfinite;
    counts[1] = nonphys;
}

/* ------------------------------------------- single-cell entry points --- */

void ora_weights(double T, double F[5])
{
    real Fr[5];
    weights((real)T, Fr);
    for (int k = 0; k < 5; ++k) F[k] = (double)Fr[k];
}

void ora_velocities(double theta, double vr[NQ], double vt[NQ])
{
    real a[NQ], b[NQ];
    velocities((real)theta, a, b);
    for (int q = 0; q < NQ; ++q) {
        vr[q] = (double)a[q];
        vt[q] = (double)b[q];
    }
}

void ora_equilibrium(double rho, double ur, double ut, double T, double theta, double feq[NQ])
{
    real vr[NQ], vt[NQ], out[NQ];
    velocities((real)theta, vr, vt);
    equilibrium((real)rho, (real)ur, (real)ut, (real)T, vr, vt, out);
    for (int q = 0; q < NQ; ++q) feq[q] = (double)out[q];
}

void ora_moments(const double f[NQ], double theta, double out[4])
{
    real vr[NQ], vt[NQ], fr[NQ], rho, ur, ut, T;
    velocities((real)theta, vr, vt);
    for (int q = 0; q < NQ; ++q) fr[q] = (real)f[q];
    moments(fr, vr, vt, &rho, &ur, &ut, &T);
    out[0] = (double)rho;
    out[1] = (double)ur;
    out[2] = (double)ut;
    out[3] = (double)T;
}

/* Collision of one cell; out[33] = post-collision f, info = (rho, u_r,
 * u_theta, T, a, b, reacting). */
void ora_collide(const ora_params *p, const double f[NQ], double lam, double theta, double out[NQ], double info[7])
{
    real vr[NQ], vt[NQ], fr[NQ], o[NQ], mom[4], a, b;
    int on;
    velocities((real)theta, vr, vt);
    for (int q = 0; q < NQ; ++q) fr[q] = (real)f[q];
    collide(p, fr, (real)lam, vr, vt, (real)p->tau, o, mom, &a, &b, &on);
    for (int q = 0; q < NQ; ++q) out[q] = (double)o[q];
    for (int i = 0; i < 4; ++i) info[i] = (double)mom[i];
    info[4] = (double)a;
    info[5] = (double)b;
    info[6] = on;
}

double ora_cochran(double lam, double a, double b, double dt) { return (double)cochran(lam, a, b, dt); }

/* Central moments (Sec. II.E) of g[33] about (u_r, u_theta) at azimuth theta. */
void ora_central_moments(const double g[NQ], double theta, double ur, double ut, double out[12])
{
    real vr[NQ], vt[NQ], gr[NQ], o[12];
    velocities((real)theta, vr, vt);
    for (int q = 0; q < NQ; ++q) gr[q] = (real)g[q];
    central_moments(gr, vr, vt, (real)ur, (real)ut, o);
    for (int m = 0; m < 12; ++m) out[m] = (double)o[m];
}

uint64_t ora_splitmix64(uint64_t x) { return splitmix64(x); }

int ora_real_bytes(void) { return (int)sizeof(real); }
