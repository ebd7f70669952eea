// art_rtchem.hip -- one radiative step coupled to the chemistry and energy
// update (Appendix D iteration; fields of the diffuse recombination
// radiation from Sect. 2.2).  Entry points and model in include/art_chem.h.
//
// The iteration is driven from the host: each pass builds kappa and S from
// the latest state (one thread per cell, double precision, rounded to the
// float32 fields the sweep takes), loads them into the mesh, sweeps, adds the
// point sources' rates, advances the start state by dt with art_chem_step,
// and counts the cells whose n_e or
// u moved by more than the tolerance; the count is read back to decide
// whether to stop.  Every step is an existing library call or a plain
// per-cell kernel; the convergence count is the only atomic, and it is an
// integer sum (the same on every run).
#include <algorithm>
#include <cmath>
#include <string>

#include "../../include/art.h"
#include "../../include/art_chem.h"
#include "../../include/art_point.h"
#include "art_internal.h"

#pragma clang fp contract(off)

namespace {

struct RtcArgs {
    float sigma[ART_MAX_BINS], src[ART_MAX_BINS];
    const double *dalpha;
    int nT;
    double lt0, dlt, T_per_u, x_floor;
};

// Linear interpolation in log10 T, held at the ends (the chemistry's tables).
__device__ double rtc_tab(const double *__restrict__ t, const RtcArgs &a, double T)
{
    const double s = (log10(fmax(T, 1e-300)) - a.lt0) / a.dlt;
    if (s <= 0.0) return t[0];
    if (s >= (double)(a.nT - 1)) return t[a.nT - 1];
    const int i = (int)floor(s);
    const double f = s - (double)i;
    return t[i] * (1.0 - f) + t[i + 1] * f;
}

__global__ __launch_bounds__(256) void rtc_fields_kernel(long long n, int nb, const double *__restrict__ nH_,
                                                         const double *__restrict__ x_,
                                                         const double *__restrict__ u_, RtcArgs a,
                                                         float *__restrict__ kappa, float *__restrict__ S,
                                                         float *__restrict__ nabs)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double nh = nH_[c];
    if (!(nh > 0.0)) {
        for (int b = 0; b < nb; ++b) {
            kappa[b * n + c] = 0.0f;
            S[b * n + c] = 0.0f;
        }
        nabs[c] = 0.0f;
        return;
    }
    const double x = x_[c];
    const double nHI = nh * fmax(x, a.x_floor);
    nabs[c] = (float)nHI;                                    // absorber density of the point-source rates
    const double ne = nh * (1.0 - x);                        // = n_HII
    const double T = a.T_per_u * u_[c] / (1.0 + ne / nh);
    const double da = rtc_tab(a.dalpha, a, T);
    for (int b = 0; b < nb; ++b) {
        kappa[b * n + c] = (float)((double)a.sigma[b] * nHI);
        S[b * n + c] = (float)((double)a.src[b] * da * ne * ne / nHI);
    }
}

// Cells (n_H > 0) that have not converged: |n_e' - n_e| > eps n_e' or
// |u' - u| > eps u' (also when either is NaN).
__global__ __launch_bounds__(256) void rtc_check_kernel(long long n, const double *__restrict__ nH_,
                                                        const double *__restrict__ xn,
                                                        const double *__restrict__ un,
                                                        const double *__restrict__ xp,
                                                        const double *__restrict__ up, double eps,
                                                        unsigned int *__restrict__ count)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (c < n) {
        const double nh = nH_[c];
        if (nh > 0.0) {
            const double en = nh * (1.0 - xn[c]), ep = nh * (1.0 - xp[c]);
            bad = !(fabs(en - ep) <= eps * en && fabs(un[c] - up[c]) <= eps * un[c]);
        }
    }
    const int k = __syncthreads_count(bad);
    if (threadIdx.x == 0 && k > 0) atomicAdd(count, (unsigned int)k);
}

__global__ void rtc_zero_kernel(unsigned int *p) { *p = 0u; }

// Gamma += Gp, Heat += Hp (Heat may be absent).
__global__ __launch_bounds__(256) void rtc_add_kernel(long long n, const float *__restrict__ Gp,
                                                      const float *__restrict__ Hp, float *__restrict__ G,
                                                      float *__restrict__ H)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    G[c] += Gp[c];
    if (Hp) H[c] += Hp[c];
}

// Minimum of v over [0, n): per-block minima, then one block over those.
__global__ __launch_bounds__(256) void rtc_min_kernel(const double *__restrict__ v, long long n,
                                                      double *__restrict__ out)
{
    __shared__ double red[256];
    double m = INFINITY;
    for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < n; c += (long long)gridDim.x * 256)
        m = fmin(m, v[c]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

constexpr int RTC_MIN_BLOCKS = 1024;

struct Layout {
    size_t kappa, S, G, H, xa, ua, xb, ub, dtc, nabs, Gp, Hp, cnt, mn, total;
};

Layout layout(long long n, int nb)
{
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = up(o + bytes);
        return at;
    };
    L.kappa = take((size_t)nb * n * 4);
    L.S = take((size_t)nb * n * 4);
    L.G = take((size_t)n * 4);
    L.H = take((size_t)n * 4);
    L.xa = take((size_t)n * 8);
    L.ua = take((size_t)n * 8);
    L.xb = take((size_t)n * 8);
    L.ub = take((size_t)n * 8);
    L.dtc = take((size_t)n * 8);
    L.nabs = take((size_t)n * 4);
    L.Gp = take((size_t)n * 4);
    L.Hp = take((size_t)n * 4);
    L.cnt = take(4);
    L.mn = take((RTC_MIN_BLOCKS + 1) * 8);
    L.total = o;
    return L;
}

int rtc_fail(int code, const std::string &m) { return art_set_error(code, m.c_str()); }

int hip_fail(const char *what, hipError_t e)
{
    return rtc_fail(ART_E_HIP, std::string("art_rt_chem_step: ") + what + ": " + hipGetErrorString(e));
}

bool finite_nonneg(const float *v, int nb)
{
    for (int b = 0; b < nb; ++b)
        if (!(v[b] >= 0.0f) || !std::isfinite(v[b])) return false;
    return true;
}

bool finite_or_null(const float *v, int nb)
{
    if (!v) return true;
    for (int b = 0; b < nb; ++b)
        if (!std::isfinite(v[b])) return false;
    return true;
}

long long mesh_cells(const art_mesh *mesh)
{
    int dims[3] = {0, 0, 0}, nb = 0;
    double h = 0.0;
    const float2 *f = nullptr;
    art_mesh_fields(mesh, dims, &nb, &h, &f);
    return (long long)dims[0] * dims[1] * dims[2];
}

}  // namespace

extern "C" long long art_rt_chem_workspace(const art_mesh *mesh, int nbins)
{
    if (!mesh || nbins < 1 || nbins > ART_MAX_BINS) return -1;
    return (long long)layout(mesh_cells(mesh), nbins).total;
}

namespace {

// One coupled step; keep_start leaves x_HI and u as they came in (the step of
// length 0 that gives the chemical timestep of the start state).
int rt_chem_step(art_mesh *mesh, const art_rt_chem_params *rp, const art_chem_params *cp, const double *n_H,
                 const double *rho, double *x_HI, double *u, double dt, void *work, long long work_bytes,
                 float *Gamma, float *Heat, art_rt_chem_result *res, void *hip_stream, bool keep_start)
{
    if (!mesh || !rp || !cp || !res) return rtc_fail(ART_E_INVAL, "art_rt_chem_step: null mesh, parameters or result");
    if (!n_H || !rho || !x_HI || !u || !work)
        return rtc_fail(ART_E_INVAL, "art_rt_chem_step: null cell array or workspace");
    const int nb = rp->nbins;
    if (nb < 1 || nb > ART_MAX_BINS) return rtc_fail(ART_E_INVAL, "art_rt_chem_step: nbins must be 1..4");
    if (!rp->sigma || !rp->src_coef || !finite_nonneg(rp->sigma, nb) || !finite_nonneg(rp->src_coef, nb))
        return rtc_fail(ART_E_INVAL, "art_rt_chem_step: sigma and src_coef must be finite and >= 0");
    if (!finite_or_null(rp->gamma_w, nb) || !finite_or_null(rp->heat_in, nb) || !finite_or_null(rp->heat_src, nb))
        return rtc_fail(ART_E_INVAL, "art_rt_chem_step: non-finite rate weight");
    if (!rp->dalpha) return rtc_fail(ART_E_INVAL, "art_rt_chem_step: null dalpha table");
    if (rp->nside < 1) return rtc_fail(ART_E_INVAL, "art_rt_chem_step: nside must be >= 1");
    if (!(rp->x_floor > 0.0) || !(rp->x_floor <= 1.0))
        return rtc_fail(ART_E_INVAL, "art_rt_chem_step: x_floor must be in (0, 1]");
    if (rp->max_iter < 1) return rtc_fail(ART_E_INVAL, "art_rt_chem_step: max_iter must be >= 1");
    if (rp->nsrc < 0 || (rp->nsrc > 0 && (!rp->src_pos || !rp->src_Q)))
        return rtc_fail(ART_E_INVAL, "art_rt_chem_step: nsrc must be >= 0, with positions and photon rates");
    // the chemistry parameters and dt, checked by the chemistry entry point itself
    if (int rc = art_chem_step(0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, dt, cp, nullptr,
                               nullptr, hip_stream))
        return rc;
    const long long n = mesh_cells(mesh);
    const Layout L = layout(n, nb);
    if (work_bytes < (long long)L.total)
        return rtc_fail(ART_E_INVAL, "art_rt_chem_step: workspace smaller than art_rt_chem_workspace()");

    hipStream_t st = (hipStream_t)hip_stream;
    char *w = (char *)work;
    float *kap = (float *)(w + L.kappa), *S = (float *)(w + L.S);
    art_outputs o{};
    o.Gamma = Gamma ? Gamma : (float *)(w + L.G);
    o.Heat = Heat ? Heat : (float *)(w + L.H);
    double *bx[2] = {(double *)(w + L.xa), (double *)(w + L.xb)};
    double *bu[2] = {(double *)(w + L.ua), (double *)(w + L.ub)};
    double *dtc = (double *)(w + L.dtc), *mn = (double *)(w + L.mn);
    float *nabs = (float *)(w + L.nabs), *Gp = (float *)(w + L.Gp), *Hp = (float *)(w + L.Hp);
    unsigned int *cnt = (unsigned int *)(w + L.cnt);

    RtcArgs a{};
    for (int b = 0; b < nb; ++b) {
        a.sigma[b] = rp->sigma[b];
        a.src[b] = rp->src_coef[b];
    }
    a.dalpha = rp->dalpha;
    a.nT = cp->nT;
    a.lt0 = cp->logT_min;
    a.dlt = cp->dlogT;
    a.T_per_u = cp->T_per_u;
    a.x_floor = rp->x_floor;
    const unsigned nblk = (unsigned)((n + 255) / 256);

    const double *xp = x_HI, *up = u;                          // iteration 0: the start state
    int it = 0, conv = 0;
    for (it = 1; it <= rp->max_iter; ++it) {
        hipLaunchKernelGGL(rtc_fields_kernel, dim3(nblk), dim3(256), 0, st, n, nb, n_H, xp, up, a, kap, S, nabs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail("fields", e);
        if (int rc = art_set_fields(mesh, nb, kap, S, 1, hip_stream)) return rc;
        if (int rc = art_set_heating(mesh, rp->heat_in, rp->heat_src)) return rc;
        if (int rc = art_sweep(mesh, rp->nside, rp->gamma_w, 0.0f, &o, hip_stream)) return rc;
        if (rp->nsrc > 0) {
            if (int rc = art_point_sources(mesh, rp->nsrc, rp->src_pos, rp->src_Q, rp->src_e, nabs, Gp,
                                           rp->src_e ? Hp : nullptr, nullptr, hip_stream))
                return rc;
            hipLaunchKernelGGL(rtc_add_kernel, dim3(nblk), dim3(256), 0, st, n, Gp, rp->src_e ? Hp : nullptr,
                               o.Gamma, o.Heat);
            e = hipGetLastError();
            if (e != hipSuccess) return hip_fail("point-source rates", e);
        }
        double *xn = bx[(it - 1) & 1], *un = bu[(it - 1) & 1];
        e = hipMemcpyAsync(xn, x_HI, (size_t)n * 8, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(un, u, (size_t)n * 8, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail("state copy", e);
        if (int rc = art_chem_step(n, n_H, rho, o.Gamma, o.Heat, xn, un, dt, cp, dtc, nullptr, hip_stream))
            return rc;
        hipLaunchKernelGGL(rtc_zero_kernel, dim3(1), dim3(1), 0, st, cnt);
        hipLaunchKernelGGL(rtc_check_kernel, dim3(nblk), dim3(256), 0, st, n, n_H, xn, un, xp, up, cp->eps, cnt);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail("convergence count", e);
        unsigned int hc = 0;
        e = hipMemcpyAsync(&hc, cnt, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail("convergence count", e);
        xp = xn;
        up = un;
        if (hc == 0) {
            conv = 1;
            break;
        }
    }
    if (it > rp->max_iter) it = rp->max_iter;
    hipError_t e = hipSuccess;
    if (!keep_start) {
        e = hipMemcpyAsync(x_HI, xp, (size_t)n * 8, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(u, up, (size_t)n * 8, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail("state copy", e);
    }
    const unsigned nmb = nblk < (unsigned)RTC_MIN_BLOCKS ? nblk : (unsigned)RTC_MIN_BLOCKS;
    hipLaunchKernelGGL(rtc_min_kernel, dim3(nmb), dim3(256), 0, st, dtc, n, mn);
    hipLaunchKernelGGL(rtc_min_kernel, dim3(1), dim3(256), 0, st, mn, (long long)nmb, mn + RTC_MIN_BLOCKS);
    e = hipGetLastError();
    double dmin = INFINITY;
    if (e == hipSuccess) e = hipMemcpyAsync(&dmin, mn + RTC_MIN_BLOCKS, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail("timestep minimum", e);
    res->iterations = it;
    res->converged = conv;
    res->dt_chem_min = dmin;
    return ART_OK;
}

}  // namespace

extern "C" int art_rt_chem_step(art_mesh *mesh, const art_rt_chem_params *rp, const art_chem_params *cp,
                                const double *n_H, const double *rho, double *x_HI, double *u, double dt,
                                void *work, long long work_bytes, float *Gamma, float *Heat,
                                art_rt_chem_result *res, void *hip_stream)
{
    return rt_chem_step(mesh, rp, cp, n_H, rho, x_HI, u, dt, work, work_bytes, Gamma, Heat, res, hip_stream,
                        false);
}

extern "C" int art_rt_chem_advance(art_mesh *mesh, const art_rt_chem_params *rp, const art_chem_params *cp,
                                   const double *n_H, const double *rho, double *x_HI, double *u,
                                   double t_end, double F, int max_steps, void *work, long long work_bytes,
                                   float *Gamma, float *Heat, art_rt_chem_run *run, void *hip_stream)
{
    if (!run) return rtc_fail(ART_E_INVAL, "art_rt_chem_advance: null result");
    if (!(t_end >= 0.0) || !std::isfinite(t_end))
        return rtc_fail(ART_E_INVAL, "art_rt_chem_advance: t_end must be finite and >= 0");
    if (!(F > 0.0) || !std::isfinite(F)) return rtc_fail(ART_E_INVAL, "art_rt_chem_advance: F must be finite and > 0");
    if (max_steps < 1) return rtc_fail(ART_E_INVAL, "art_rt_chem_advance: max_steps must be >= 1");
    art_rt_chem_result r{};
    // the chemical timestep of the start state: a step of length 0
    if (int rc = rt_chem_step(mesh, rp, cp, n_H, rho, x_HI, u, 0.0, work, work_bytes, Gamma, Heat, &r,
                              hip_stream, true))
        return rc;
    double dcm = r.dt_chem_min, t = 0.0;
    int steps = 0, its = 0, unconv = 0;
    while (t < t_end && steps < max_steps) {
        const double rest = t_end - t;
        const double dt = std::isfinite(dcm) ? std::min(F * dcm, rest) : rest;
        if (!(dt > 0.0))   // a chemical timestep of 0 would never reach t_end
            return rtc_fail(ART_E_STATE, "art_rt_chem_advance: the chemical timestep fell to 0");
        if (int rc = art_rt_chem_step(mesh, rp, cp, n_H, rho, x_HI, u, dt, work, work_bytes, Gamma, Heat, &r,
                                      hip_stream))
            return rc;
        dcm = r.dt_chem_min;
        t = dt < rest ? t + dt : t_end;
        ++steps;
        its += r.iterations;
        unconv += r.converged ? 0 : 1;
    }
    run->steps = steps;
    run->iterations = its;
    run->unconverged = unconv;
    run->t = t;
    run->dt_chem_min = dcm;
    return ART_OK;
}
