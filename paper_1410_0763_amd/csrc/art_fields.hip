// art_fields.hip -- field layout, normalisation / rates, exit sums.
//
// Layout (at set_fields): kappa and S arrive as [bin][cell]; the march wants
// all bins of a cell in one place, so each cell gets nb float2 records
// {kappa h, S} (kappa h is the optical depth per cell length), once with cells
// x fastest and once with y fastest, then z, then x (read by the directions
// whose dominant axis is x, whose tiles span y and z).
//
// Normalisation (Sect. 2.2, eq mean_intensity, and eq gamma_diff):
//   J_in = A1 / N_d,  J = J_in + S,  J_exact = J_in + S A2 / N_d,
//   Gamma = sum_b g_b (J_in_b + S_b),
// where A1, A2 are summed over the per-bucket accumulator copies in a fixed
// order (deterministic).  Copies of empty buckets are skipped.
//
// Exit sums: after a sweep every ray's state slot holds the intensity with
// which it left the mesh; one workgroup per direction adds up I_exit - I_bc
// over the rays that cross the mesh (photon-balance diagnostics).  Rays that
// only touch the mesh (chords of rounding size) are never marched; the state
// buffer is filled with I_bc before such a sweep so that they add nothing.
#include <algorithm>

#include "art_internal.h"

namespace {

// Validation pass (before anything is written): bad[0] = 1 if some kappa is
// negative or not finite, or some S is not finite.
__global__ __launch_bounds__(256) void art_check_kernel(const float *__restrict__ kappa,
                                                        const float *__restrict__ S, long long n,
                                                        int *__restrict__ bad)
{
    bool ok = true;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float k = kappa[i], s = S[i];
        ok = ok && (k >= 0.0f) && isfinite(k) && isfinite(s);
    }
    if (!ok) *bad = 1;
}

__global__ __launch_bounds__(256) void art_layout_kernel(const float *__restrict__ kappa,
                                                         const float *__restrict__ S,
                                                         long long ncell, int nb, float h,
                                                         int nx, int ny, int nz,
                                                         float2 *__restrict__ fields,
                                                         float2 *__restrict__ fields_t)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const long long x = c % nx, y = (c / nx) % ny, z = c / ((long long)nx * ny);
    const long long ct = (x * nz + z) * ny + y;           // y fastest, then z, then x
    for (int b = 0; b < nb; ++b) {
        const float k = kappa[(long long)b * ncell + c];
        const float s = S[(long long)b * ncell + c];
        const float kh = k * h;
        fields[c * nb + b] = make_float2(kh, s);
        fields_t[ct * nb + b] = make_float2(kh, s);
    }
}

__global__ __launch_bounds__(256) void art_fill_kernel(float *__restrict__ p, long long n, float v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

struct GW {
    float g[4];                 // rate weights of eq gamma_diff
    float hin[4], hsrc[4];      // heating weights of eq heat_diff (J_in and S terms)
};

__global__ __launch_bounds__(256) void art_normalize_kernel(
    const float *__restrict__ acc, const int *__restrict__ bucket_start, int nbuckets,
    const float2 *__restrict__ fields, long long ncell, int nb, float inv_nd, GW gw,
    float *__restrict__ J_in, float *__restrict__ J, float *__restrict__ J_exact,
    float *__restrict__ Gamma, float *__restrict__ Heat, float *__restrict__ A1raw,
    float *__restrict__ A2raw)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    float gam = 0.0f, heat = 0.0f;
    for (int b = 0; b < nb; ++b) {
        float a1 = 0.0f, a2 = 0.0f;
        for (int k = 0; k < nbuckets; ++k) {
            if (bucket_start[k + 1] == bucket_start[k]) continue;
            const float *base = acc + ((long long)k * nb + b) * 2 * ncell;
            a1 += base[c];
            a2 += base[ncell + c];
        }
        const long long bc = (long long)b * ncell + c;
        if (A1raw) A1raw[bc] = a1;
        if (A2raw) A2raw[bc] = a2;
        const float s = fields[c * nb + b].y;
        const float jin = a1 * inv_nd;
        if (J_in) J_in[bc] = jin;
        if (J) J[bc] = jin + s;
        if (J_exact) J_exact[bc] = fmaf(s, a2 * inv_nd, jin);
        gam = fmaf(gw.g[b], jin + s, gam);
        heat = fmaf(gw.hin[b], jin, fmaf(gw.hsrc[b], s, heat));
    }
    if (Gamma) Gamma[c] = gam;
    if (Heat) Heat[c] = heat;
}

__global__ __launch_bounds__(256) void art_exit_sum_kernel(const ArtDir *__restrict__ dirs,
                                                           const float *__restrict__ state, int nx,
                                                           int ny, int nz, int nb, float I_bc,
                                                           float *__restrict__ exit_sum)
{
    __shared__ float red[4][256];
    const int d = blockIdx.x;
    const ArtDir D = dirs[d];
    float sum[4] = {0.f, 0.f, 0.f, 0.f};
    if (D.bucket >= 0) {
        const double N[3] = {(double)nx, (double)ny, (double)nz};
        const int nr = D.nj * D.nk;
        for (int r = threadIdx.x; r < nr; r += blockDim.x) {
            const int j = D.j0 + (D.kfast ? r / D.nk : r % D.nj);
            const int k = D.k0 + (D.kfast ? r % D.nk : r / D.nj);
            double lo = -INFINITY, hi = INFINITY;
            bool ok = true;
            for (int q = 0; q < 3; ++q) {
                const double x0 = q == D.a ? D.alpha_a : (q == D.b ? j + 0.5 : k + 0.5);
                if (D.beta[q] == 0.0) {
                    ok = ok && (x0 > 0.0 && x0 < N[q]);
                } else {
                    const double t0 = (0.0 - x0) * D.rbeta[q], t1 = (N[q] - x0) * D.rbeta[q];
                    lo = fmax(lo, fmin(t0, t1));
                    hi = fmin(hi, fmax(t0, t1));
                }
            }
            if (!ok || !(hi > lo)) continue;
            const long long sidx = D.state_off + ((long long)r) * nb;
            for (int b = 0; b < nb; ++b) sum[b] += state[sidx + b] - I_bc;
        }
    }
    for (int b = 0; b < 4; ++b) red[b][threadIdx.x] = sum[b];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int b = 0; b < 4; ++b) red[b][threadIdx.x] += red[b][threadIdx.x + w];
        __syncthreads();
    }
    if ((int)threadIdx.x < nb) exit_sum[(long long)d * nb + threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

hipError_t art_launch_check(const float *kappa, const float *S, long long n, int *bad_flag,
                            hipStream_t stream)
{
    const long long blocks = std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192));
    hipLaunchKernelGGL(art_check_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, kappa, S, n,
                       bad_flag);
    return hipGetLastError();
}

hipError_t art_launch_layout(const float *kappa, const float *S, int nx, int ny, int nz, int nb,
                             double h, float2 *fields, float2 *fields_t, hipStream_t stream)
{
    const long long ncell = (long long)nx * ny * nz;
    const long long nblk = (ncell + 255) / 256;
    hipLaunchKernelGGL(art_layout_kernel, dim3((unsigned)nblk), dim3(256), 0, stream, kappa, S,
                       ncell, nb, (float)h, nx, ny, nz, fields, fields_t);
    return hipGetLastError();
}

hipError_t art_launch_fill(float *p, long long n, float v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const long long blocks = std::min<long long>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(art_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t art_launch_normalize(const float *acc, const int *bucket_start, int nbuckets,
                                const float2 *fields, long long ncell, int nb, int nd,
                                const float *gw4, const float *hw8, float *J_in, float *J,
                                float *J_exact, float *Gamma, float *Heat, float *A1raw,
                                float *A2raw, hipStream_t stream)
{
    GW gw;
    for (int b = 0; b < 4; ++b) {
        gw.g[b] = gw4[b];
        gw.hin[b] = hw8 ? hw8[b] : 0.0f;
        gw.hsrc[b] = hw8 ? hw8[4 + b] : 0.0f;
    }
    const long long nblk = (ncell + 255) / 256;
    hipLaunchKernelGGL(art_normalize_kernel, dim3((unsigned)nblk), dim3(256), 0, stream, acc,
                       bucket_start, nbuckets, fields, ncell, nb, 1.0f / (float)nd, gw, J_in, J,
                       J_exact, Gamma, Heat, A1raw, A2raw);
    return hipGetLastError();
}

hipError_t art_launch_exit_sum(const ArtDir *dirs, int nd, const float *state, int nx, int ny,
                               int nz, int nb, float I_bc, float *exit_sum, hipStream_t stream)
{
    hipLaunchKernelGGL(art_exit_sum_kernel, dim3(nd), dim3(256), 0, stream, dirs, state, nx, ny,
                       nz, nb, I_bc, exit_sum);
    return hipGetLastError();
}
