// art_chem.hip -- chemistry and energy update of a radiative step
// (Appendices B, C and D; entry point and model in include/art_chem.h).
//
// One thread per cell, double precision throughout: the update is a handful
// of scalar recurrences per cell with data-dependent sub-step and iteration
// counts, a per-cell latency-bound job with no reuse between cells, so it is
// written as plain vector code (no LDS, no matrix cores).  The four rate
// tables live in device memory and are read through the scalar cache (all
// lanes read the same small table).  Multiply-add contraction is off in this
// file so that each expression rounds as written.
#include <cmath>
#include <string>

#include "../../include/art.h"
#include "../../include/art_chem.h"
#include "art_internal.h"

#pragma clang fp contract(off)

namespace {

struct ChemArgs {
    const double *tab[4];   // alpha, k_ci, cool_I, cool_II
    int nT;
    double lt0, dlt;
    double T_per_u, eps, eps_e, eps_HI;
    int max_iter, max_sub;
};

// Linear interpolation in log10 T, held at the ends: the position in the
// grid once per temperature, then the value of each table at it.
struct TabPos {
    int i;        // lower node (or the end node where held)
    double f;     // weight of node i + 1 (0 where held)
};

__device__ TabPos tab_pos(const ChemArgs &a, double T)
{
    const double s = (log10(fmax(T, 1e-300)) - a.lt0) / a.dlt;
    if (s <= 0.0) return TabPos{0, 0.0};
    if (s >= (double)(a.nT - 1)) return TabPos{a.nT - 1, 0.0};
    const int i = (int)floor(s);
    return TabPos{i, s - (double)i};
}

__device__ double tab_val(const double *__restrict__ t, const ChemArgs &a, TabPos p)
{
    if (p.i >= a.nT - 1) return t[a.nT - 1];
    if (p.f == 0.0 && p.i == 0) return t[0];
    return t[p.i] * (1.0 - p.f) + t[p.i + 1] * p.f;
}

__device__ double temp_of(const ChemArgs &a, double u, double xe) { return a.T_per_u * u / (1.0 + xe); }

// Chemical timestep of Appendix D at a state (n_HI of n_H, energy u).
__device__ double dt_chem_of(const ChemArgs &a, double nH, double nHI, double u, double G)
{
    const double nII = nH - nHI;
    const TabPos tp = tab_pos(a, temp_of(a, u, nII / nH));
    const double al = tab_val(a.tab[0], a, tp), kc = tab_val(a.tab[1], a, tp);
    const double rHI = al * nII * nII - (kc * nII + G) * nHI;   // dn_HI/dt; dn_e/dt = -rHI
    const double te = rHI == 0.0 ? INFINITY : a.eps_e * fabs(nII / rHI);
    const double th = rHI == 0.0 ? INFINITY : a.eps_HI * fabs(nHI / rHI);
    return te + th;
}

// n_HI' of the backward-difference update at fixed coefficients: the root in
// [0, n_H] of (kc + al) h y^2 - (1 + (kc + 2 al) h n_H + G h) y + al h n_H^2 +
// n_HI0 = 0, taken as 2c / (b + sqrt(b^2 - 4 q c)) (no cancellation).
__device__ double hi_new(double nH, double nHI0, double h, double al, double kc, double G)
{
    const double q = (kc + al) * h;
    const double b = 1.0 + (kc + 2.0 * al) * h * nH + G * h;
    const double c = al * h * nH * nH + nHI0;
    const double disc = fmax(b * b - 4.0 * q * c, 0.0);
    const double y = 2.0 * c / (b + sqrt(disc));
    return fmin(fmax(y, 0.0), nH);
}

// u' of the implicit energy equation for fixed species (bisection).
__device__ double u_new(const ChemArgs &a, double u0, double h, double H, double nH, double nHI,
                        double rho)
{
    const double nII = nH - nHI, xe = nII / nH;
    const double ufl = pow(10.0, a.lt0) / a.T_per_u;
    auto resid = [&](double uu) {
        const TabPos tp = tab_pos(a, temp_of(a, uu, xe));
        const double lam = nII * (tab_val(a.tab[2], a, tp) * nHI + tab_val(a.tab[3], a, tp) * nII);
        return uu - u0 - h * (H * nHI - lam) / rho;
    };
    double lo = ufl, hi = fmax(ufl, u0 + h * H * nHI / rho);
    if (resid(lo) >= 0.0) return lo;
    for (int k = 0; k < 64; ++k) {
        const double mid = 0.5 * (lo + hi);
        // lo and hi adjacent (or equal): every further halving leaves
        // 0.5 (lo + hi) where it is, so stopping returns the same value
        if (mid == lo || mid == hi) break;
        if (resid(mid) >= 0.0) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

__global__ __launch_bounds__(256) void art_chem_kernel(long long n, const double *__restrict__ nH_,
                                                       const double *__restrict__ rho_,
                                                       const float *__restrict__ G_,
                                                       const float *__restrict__ H_,
                                                       double *__restrict__ x_, double *__restrict__ u_,
                                                       double dt, ChemArgs a,
                                                       double *__restrict__ dtc_, int *__restrict__ ns_)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double nH = nH_[c];
    if (!(nH > 0.0)) {
        if (dtc_) dtc_[c] = INFINITY;
        if (ns_) ns_[c] = 0;
        return;
    }
    const double rho = rho_[c], G = (double)G_[c], H = (double)H_[c];
    double nHI = x_[c] * nH, u = u_[c];
    double t = 0.0;
    int sub = 0;
    while (t < dt) {
        const double rest = dt - t;
        const double h = sub >= a.max_sub ? rest : fmin(dt_chem_of(a, nH, nHI, u, G), rest);
        // one sub-step: species and energy at the advanced time, iterated
        double nHIi = nHI, ui = u, ne_prev = nH - nHI;
        for (int it = 0; it < a.max_iter; ++it) {
            const TabPos tp = tab_pos(a, temp_of(a, ui, (nH - nHIi) / nH));
            const double al = tab_val(a.tab[0], a, tp), kc = tab_val(a.tab[1], a, tp);
            const double yn = hi_new(nH, nHI, h, al, kc, G);
            const double un = u_new(a, u, h, H, nH, yn, rho);
            const double ne = nH - yn;
            const bool done = fabs(ne - ne_prev) <= a.eps * ne && fabs(un - ui) <= a.eps * un;
            nHIi = yn;
            ui = un;
            ne_prev = ne;
            if (done) break;
        }
        nHI = nHIi;
        u = ui;
        t = h < rest ? t + h : dt;
        ++sub;
    }
    x_[c] = nHI / nH;
    u_[c] = u;
    if (dtc_) dtc_[c] = dt_chem_of(a, nH, nHI, u, G);
    if (ns_) ns_[c] = sub;
}

int chem_fail(int code, const std::string &m) { return art_set_error(code, m.c_str()); }

}  // namespace

extern "C" int art_chem_step(long long ncell, const double *n_H, const double *rho, const float *Gamma,
                             const float *Heat, double *x_HI, double *u, double dt,
                             const art_chem_params *p, double *dt_chem, int *nsub, void *hip_stream)
{
    if (ncell < 0) return chem_fail(ART_E_INVAL, "art_chem_step: ncell < 0");
    if (!p) return chem_fail(ART_E_INVAL, "art_chem_step: null parameters");
    if (ncell > 0 && (!n_H || !rho || !Gamma || !Heat || !x_HI || !u))
        return chem_fail(ART_E_INVAL, "art_chem_step: null cell array");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return chem_fail(ART_E_INVAL, "art_chem_step: dt must be finite and >= 0");
    if (p->nT < 2 || !(p->dlogT > 0.0) || !std::isfinite(p->logT_min) || !std::isfinite(p->dlogT))
        return chem_fail(ART_E_INVAL, "art_chem_step: the table grid needs nT >= 2 and dlogT > 0");
    if (!p->alpha || !p->k_ci || !p->cool_I || !p->cool_II)
        return chem_fail(ART_E_INVAL, "art_chem_step: null rate table");
    if (!(p->T_per_u > 0.0) || !std::isfinite(p->T_per_u) || !(p->eps > 0.0) || !(p->eps_e >= 0.0) ||
        !(p->eps_HI >= 0.0) || !(p->eps_e + p->eps_HI > 0.0) || !std::isfinite(p->eps_e + p->eps_HI))
        return chem_fail(ART_E_INVAL, "art_chem_step: T_per_u and eps must be > 0, eps_e and eps_HI >= 0 and not both 0");
    if (p->max_iter < 1 || p->max_sub < 0) return chem_fail(ART_E_INVAL, "art_chem_step: max_iter >= 1, max_sub >= 0");
    if (ncell == 0) return ART_OK;
    ChemArgs a{};
    a.tab[0] = p->alpha;
    a.tab[1] = p->k_ci;
    a.tab[2] = p->cool_I;
    a.tab[3] = p->cool_II;
    a.nT = p->nT;
    a.lt0 = p->logT_min;
    a.dlt = p->dlogT;
    a.T_per_u = p->T_per_u;
    a.eps = p->eps;
    a.eps_e = p->eps_e;
    a.eps_HI = p->eps_HI;
    a.max_iter = p->max_iter;
    a.max_sub = p->max_sub;
    const long long nblk = (ncell + 255) / 256;
    if (nblk > 0x7fffffffll) return chem_fail(ART_E_UNSUPPORTED, "art_chem_step: too many cells");
    hipLaunchKernelGGL(art_chem_kernel, dim3((unsigned)nblk), dim3(256), 0, (hipStream_t)hip_stream, ncell,
                       n_H, rho, Gamma, Heat, x_HI, u, dt, a, dt_chem, nsub);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return chem_fail(ART_E_HIP, std::string("art_chem_step: ") + hipGetErrorString(e));
    return ART_OK;
}
