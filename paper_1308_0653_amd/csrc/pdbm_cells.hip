// Kernels off the time-step path: the output moments and drift report
// (k_moments), the non-equilibrium measures (k_noneq), the initial state
// (k_init_ic, k_init_fields) and the per-cell relaxation factors (k_omega).
#include "pdbm_device.h"

namespace pdbm {
namespace {

// -------------------------------------------------------------- moments --
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_moments(SolveDesc d, int cur, double *out, DiagCtl dc)
{
    const int nb = gridDim.x;
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    const int ncell = d.nr * d.nt;
    double red[5] = {0, 0, 0, 0, 0};
    if (c < ncell) {
        const int ir = c / d.nt;
        const int jt = c - ir * d.nt;
        const real *fin = (const real *)d.f[cur];
        const int64_t idx = (int64_t)ir * d.pitch + jt;
        const int64_t frow = (int64_t)ir * d.rstride;
        real f[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) f[q] = fin[frow + elem_of(q, jt, d.pitch)];
        real rho, jx, jy, e;
        raw_moments(f, rho, jx, jy, e);
        const double rd = (double)rho;
        const double ux = (double)(jx / rho), uy = (double)(jy / rho);
        const double T = (double)(e / rho - (real)0.5 * ((jx / rho) * (jx / rho) + (jy / rho) * (jy / rho)));
        const double2 cs = d.cs[jt];
        const double lam = d.lam[cur][idx];
        if (out) {
            out[c] = rd;
            out[(size_t)ncell + c] = ux * cs.x + uy * cs.y;
            out[2 * (size_t)ncell + c] = -ux * cs.y + uy * cs.x;
            out[3 * (size_t)ncell + c] = T;
            out[4 * (size_t)ncell + c] = rd * T;
            out[5 * (size_t)ncell + c] = lam;
        }
        const double ri = d.r_min + ((double)ir + 0.5) * d.dr;
        diag_cell(red, rd, ux, uy, T, (double)e, lam, ri * d.dr * d.dth, d.Q);
    }
    diag_partial(dc, red, blockIdx.x);
}

// The drift record of k_moments: one block adds the nb per-block partial
// sums in a fixed order (deterministic, no floating-point atomics).
__global__ __launch_bounds__(BLOCK) void k_diag_final(DiagCtl dc, int nb)
{
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += BLOCK)
#pragma unroll
        for (int i = 0; i < 5; ++i) acc[i] += dc.partials[5 * (size_t)b + i];
    block_sum5(acc);
    if (threadIdx.x == 0) {
        pdbm_diag r;
        r.step = dc.step;
        r.mass = acc[0];
        r.energy = acc[1];
        r.chem = acc[2];
        r.n_nonfinite = (int64_t)acc[3];
        r.n_nonphys = (int64_t)acc[4];
        *dc.out = r;
    }
}

// ----------------------------------------------------- non-equilibrium --
// Delta*_m = M*_m(f) - M*_m(f^eq) of every cell (Sec. II.E): central moments
// about the cell's u in its polar frame (e_r, e_theta at theta_j), taken as
// the moments of f - f^eq.  Float64 throughout.  out: [NONEQ][nr][nt] in the
// order M*_2 rr, r theta, theta theta; M*_3 rrr, rr theta, r theta theta,
// theta theta theta; M*_{3,1} r, theta; M*_{4,2} rr, r theta, theta theta.
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_noneq(SolveDesc d, int cur, double *out)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    const int ncell = d.nr * d.nt;
    if (c >= ncell) return;
    const int ir = c / d.nt;
    const int jt = c - ir * d.nt;
    const real *fin = (const real *)d.f[cur];
    const int64_t frow = (int64_t)ir * d.rstride;
    double f[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) f[q] = (double)fin[frow + elem_of(q, jt, d.pitch)];
    double rho, jx, jy, e;
    raw_moments(f, rho, jx, jy, e);
    const double ux = jx / rho, uy = jy / rho;
    const double T = e / rho - 0.5 * (ux * ux + uy * uy);
    double g[NQ];
    equilibrium<double>(d.A, rho, ux, uy, T, g);
#pragma unroll
    for (int q = 0; q < NQ; ++q) g[q] = f[q] - g[q];
    const double2 cs = d.cs[jt];
    const double ur = ux * cs.x + uy * cs.y, ut = -ux * cs.y + uy * cs.x;
    // cos and sin of the directions i pi/4
    constexpr double DX[8] = {1.0, SQH, 0.0, -SQH, -1.0, -SQH, 0.0, SQH};
    constexpr double DY[8] = {0.0, SQH, 1.0, SQH, 0.0, -SQH, -1.0, -SQH};
    double m[NONEQ];
#pragma unroll
    for (int k = 0; k < NONEQ; ++k) m[k] = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double vr = 0.0, vt = 0.0;
        if (q > 0) {
            const int k = 1 + (q - 1) / 8, i = (q - 1) % 8;
            vr = speed(k) * (DX[i] * cs.x + DY[i] * cs.y);  // v cos(i pi/4 - theta)
            vt = speed(k) * (DY[i] * cs.x - DX[i] * cs.y);  // v sin(i pi/4 - theta)
        }
        const double cr = vr - ur, ct = vt - ut;
        const double h = 0.5 * (cr * cr + ct * ct);
        const double grr = g[q] * cr, gtt = g[q] * ct;
        m[0] += grr * cr;
        m[1] += grr * ct;
        m[2] += gtt * ct;
        m[3] += grr * cr * cr;
        m[4] += grr * cr * ct;
        m[5] += grr * ct * ct;
        m[6] += gtt * ct * ct;
        m[7] += h * grr;
        m[8] += h * gtt;
        m[9] += h * grr * cr;
        m[10] += h * grr * ct;
        m[11] += h * gtt * ct;
    }
#pragma unroll
    for (int k = 0; k < NONEQ; ++k) out[(size_t)k * ncell + c] = m[k];
}

// ------------------------------------------------------------ initial state
// Pressure with noise, rounded exactly as written (no contraction): the
// same bits as any IEEE implementation of the formula.
__device__ __attribute__((noinline)) double noisy_pressure(double rho, double T, double amp, uint64_t h)
{
#pragma clang fp contract(off)
    const double U = (double)(h >> 11) * 0x1.0p-53;
    const double p = rho * T;
    return p + amp * (2.0 * U - 1.0);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename real>
__device__ __forceinline__ void store_eq(const SolveDesc &d, int cur, int64_t idx, int jt, double rho, double T,
                                         double ur, double ut)
{
    const double2 cs = d.cs[jt];
    const double ux = ur * cs.x - ut * cs.y, uy = ur * cs.y + ut * cs.x;
    real f[NQ];
    equilibrium<real>(d.A, (real)rho, (real)ux, (real)uy, (real)T, f);
    real *fo = (real *)d.f[cur] + (idx / d.pitch) * d.rstride;
#pragma unroll
    for (int q = 0; q < NQ; ++q) fo[elem_of(q, jt, d.pitch)] = f[q];
}

template <typename real>
__global__ __launch_bounds__(BLOCK) void k_init_ic(SolveDesc d, int cur, pdbm_ic ic)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= d.nr * d.nt) return;
    const int ir = c / d.nt;
    const int jt = c - ir * d.nt;
    const int64_t idx = (int64_t)ir * d.pitch + jt;
    const double ri = d.r_min + ((double)ir + 0.5) * d.dr;
    const double *st = ri < ic.r_split ? ic.inner : ic.outer;
    const uint64_t h = splitmix64(ic.seed ^ ((uint64_t)c * 0x9E3779B97F4A7C15ull));
    const double p = noisy_pressure(st[0], st[1], ic.p_noise, h);
    store_eq<real>(d, cur, idx, jt, st[0], p / st[0], st[2], st[3]);
    d.lam[cur][idx] = st[4];
}

// fields: [5][nr][ntheta] = rho, T, u_r, u_theta, lambda
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_init_fields(SolveDesc d, int cur, const double *fields)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    const int ncell = d.nr * d.nt;
    if (c >= ncell) return;
    const int ir = c / d.nt;
    const int jt = c - ir * d.nt;
    const int64_t idx = (int64_t)ir * d.pitch + jt;
    store_eq<real>(d, cur, idx, jt, fields[c], fields[(size_t)ncell + c], fields[2 * (size_t)ncell + c],
                   fields[3 * (size_t)ncell + c]);
    d.lam[cur][idx] = fields[4 * (size_t)ncell + c];
}

// ---------------------------------------------- per-cell relaxation time --
// omegaf[i][j] = exp(-dt / tau[i nt + j]) (tau = +inf gives 1: no
// relaxation), or `uniform` everywhere when tau is NULL; evaluated in
// float64, stored in the solve's precision.
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_omega(SolveDesc d, const double *tau, double uniform)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    if (c >= d.nr * d.nt) return;
    const int ir = c / d.nt;
    const int jt = c - ir * d.nt;
    ((real *)d.omegaf)[(int64_t)ir * d.pitch + jt] = (real)(tau ? exp(-d.dt / tau[c]) : uniform);
}

}  // namespace

int cell_blocks(int nr, int nt) { return (int)(((int64_t)nr * nt + BLOCK - 1) / BLOCK); }

hipError_t launch_omega(const SolveDesc &d, bool fp32, const double *tau, double uniform, hipStream_t st)
{
    const int nb = cell_blocks(d.nr, d.nt);
    if (fp32)
        hipLaunchKernelGGL(k_omega<float>, dim3(nb), dim3(BLOCK), 0, st, d, tau, uniform);
    else
        hipLaunchKernelGGL(k_omega<double>, dim3(nb), dim3(BLOCK), 0, st, d, tau, uniform);
    return hipGetLastError();
}

hipError_t launch_noneq(const SolveDesc &d, int cur, bool fp32, double *out, hipStream_t st)
{
    const int nb = cell_blocks(d.nr, d.nt);
    if (fp32)
        hipLaunchKernelGGL(k_noneq<float>, dim3(nb), dim3(BLOCK), 0, st, d, cur, out);
    else
        hipLaunchKernelGGL(k_noneq<double>, dim3(nb), dim3(BLOCK), 0, st, d, cur, out);
    return hipGetLastError();
}

hipError_t launch_moments(const SolveDesc &d, int cur, bool fp32, double *out, const DiagCtl &dc, hipStream_t st)
{
    const int nb = cell_blocks(d.nr, d.nt);
    if (fp32)
        hipLaunchKernelGGL(k_moments<float>, dim3(nb), dim3(BLOCK), 0, st, d, cur, out, dc);
    else
        hipLaunchKernelGGL(k_moments<double>, dim3(nb), dim3(BLOCK), 0, st, d, cur, out, dc);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(BLOCK), 0, st, dc, nb);
    return hipGetLastError();
}

hipError_t launch_init_ic(const SolveDesc &d, int cur, bool fp32, const pdbm_ic &ic, hipStream_t st)
{
    const int nb = cell_blocks(d.nr, d.nt);
    if (fp32)
        hipLaunchKernelGGL(k_init_ic<float>, dim3(nb), dim3(BLOCK), 0, st, d, cur, ic);
    else
        hipLaunchKernelGGL(k_init_ic<double>, dim3(nb), dim3(BLOCK), 0, st, d, cur, ic);
    return hipGetLastError();
}

hipError_t launch_init_fields(const SolveDesc &d, int cur, bool fp32, const double *fields, hipStream_t st)
{
    const int nb = cell_blocks(d.nr, d.nt);
    if (fp32)
        hipLaunchKernelGGL(k_init_fields<float>, dim3(nb), dim3(BLOCK), 0, st, d, cur, fields);
    else
        hipLaunchKernelGGL(k_init_fields<double>, dim3(nb), dim3(BLOCK), 0, st, d, cur, fields);
    return hipGetLastError();
}

}  // namespace pdbm
