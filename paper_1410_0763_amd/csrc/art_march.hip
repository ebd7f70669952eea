// art_march.hip -- the ray march of the diffuse sweep (Sect. 2.2, 3.1).
//
// Work decomposition (block wavefronts).  The mesh is cut into blocks of
// bx*by*bz cells.  Directions are grouped by octant of travel, as in the
// multiple-wave-front scheme the paper uses between nodes (Sect. 3.3), and
// each octant is split into `subsets` buckets.  A workgroup owns one
// (block, bucket) pair: it marches every ray of the bucket's directions
// through its block, one ray per lane, accumulating the per-cell sums in LDS,
// and finally stores the block into the bucket's own accumulator copy with
// plain stores: no other workgroup ever writes those cells of that copy, so
// no global atomics are needed (the single-writer property that Sect. 3.1
// obtains with ray groups).  A ray's intensity crosses block faces through a
// per-ray state slot: the blocks of octant o on wavefront w (the sum of the
// block indices counted along o's travel directions) only receive rays from
// wavefronts < w, which earlier launches on the same stream have finished.
//
// Per segment of length dL (in cells) and depth step ds = dL |n_a|, for each
// frequency bin (eq rt and eq path_averaged_intensity):
//   x = kappa h dL,  e1 = 1 - e^{-x},  phi = e1 / x,
//   A1 += ds * I * phi        (sum_j dtau_j Ibar_in,j / sum_j dtau_j per direction)
//   A2 += ds * (1 - phi)      (exact path average of the source term)
//   I  <- I + (S - I) e1      (= I e^{-x} + S (1 - e^{-x}))
// For x < 1/8, e1, phi and 1 - phi come from the Taylor series of
// (x - 1 + e^{-x}) / x^2 so that none of them cancels; above, from v_exp_f32.
// Geometry (entry points, plane crossings) is double precision and derived
// from the lattice indices, never accumulated; transfer is single precision.
#include "art_internal.h"

#define ART_MAX_NB 4
#define ART_LOG2E 1.4426950408889634f

namespace {

__device__ __forceinline__ void lds_add(float *p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Depth interval of x0 + beta s inside [lo, hi] for one axis.
__device__ __forceinline__ bool clip1(double x0, double beta, double rbeta, double lo, double hi,
                                      double &tlo, double &thi)
{
    if (beta == 0.0) {
        tlo = -INFINITY;
        thi = INFINITY;
        return lo < x0 && x0 < hi;
    }
    const double t0 = (lo - x0) * rbeta, t1 = (hi - x0) * rbeta;
    tlo = fmin(t0, t1);
    thi = fmax(t0, t1);
    return true;
}

// Next plane crossing along one axis from cell m.
__device__ __forceinline__ double next_cross(int m, double x0, double beta, double rbeta)
{
    if (beta > 0.0) return ((double)(m + 1) - x0) * rbeta;
    if (beta < 0.0) return ((double)m - x0) * rbeta;
    return INFINITY;
}

__device__ __forceinline__ int entry_cell(bool via_face, double beta, int lo, int hi, double x)
{
    int m = via_face ? (beta > 0.0 ? lo : hi - 1) : (int)floor(x);
    return min(max(m, lo), hi - 1);
}

__global__ __launch_bounds__(1024) void art_march_kernel(const ArtItem *__restrict__ items,
                                                         const ArtMeshDesc *__restrict__ meshes)
{
    extern __shared__ float lds[];
    const ArtItem it = items[blockIdx.x];
    const ArtMeshDesc M = meshes[it.mesh];
    const int dbeg = M.bucket_start[it.bucket], dend = M.bucket_start[it.bucket + 1];
    if (dbeg == dend) return;

    const int nb = M.nb;
    const int V = M.bx * M.by * M.bz;
    for (int i = threadIdx.x; i < nb * 2 * V; i += blockDim.x) lds[i] = 0.0f;
    __syncthreads();

    const int bxi = it.block % M.nbx;
    const int byi = (it.block / M.nbx) % M.nby;
    const int bzi = it.block / (M.nbx * M.nby);
    const int lo0 = bxi * M.bx, lo1 = byi * M.by, lo2 = bzi * M.bz;
    const int hi0 = min(lo0 + M.bx, M.nx), hi1 = min(lo1 + M.by, M.ny), hi2 = min(lo2 + M.bz, M.nz);
    const int maxit = (hi0 - lo0) + (hi1 - lo1) + (hi2 - lo2) + 3;

    for (int q = dbeg; q < dend; ++q) {
        const ArtDir D = M.dirs[M.order[q]];
        const float invw_f = (float)D.invw;
        const float w_f = (float)D.w;
        // Depth range of the block along the dominant axis, then the lattice
        // indices whose rays can meet the block (one spare index each side).
        const double ba = D.beta[D.a];
        const double la = D.a == 0 ? lo0 : (D.a == 1 ? lo1 : lo2);
        const double ha = D.a == 0 ? hi0 : (D.a == 1 ? hi1 : hi2);
        const double sa0 = fmin((la - D.alpha_a) * ba, (ha - D.alpha_a) * ba);
        const double sa1 = fmax((la - D.alpha_a) * ba, (ha - D.alpha_a) * ba);
        const double tb = D.beta[D.b], tc = D.beta[D.c];
        const double lb = D.b == 0 ? lo0 : lo1, hb = D.b == 0 ? hi0 : hi1;
        const double lc = D.c == 1 ? lo1 : lo2, hc = D.c == 1 ? hi1 : hi2;
        int jlo = (int)floor(lb - 0.5 - fmax(tb * sa0, tb * sa1)) - 1;
        int jhi = (int)ceil(hb - 0.5 - fmin(tb * sa0, tb * sa1)) + 1;
        int klo = (int)floor(lc - 0.5 - fmax(tc * sa0, tc * sa1)) - 1;
        int khi = (int)ceil(hc - 0.5 - fmin(tc * sa0, tc * sa1)) + 1;
        jlo = max(jlo, D.j0); jhi = min(jhi, D.j0 + D.nj - 1);
        klo = max(klo, D.k0); khi = min(khi, D.k0 + D.nk - 1);
        const int cj = jhi - jlo + 1, ck = khi - klo + 1;
        if (cj <= 0 || ck <= 0) continue;
        const int ncand = cj * ck;

        for (int r = threadIdx.x; r < ncand; r += blockDim.x) {
            const int j = jlo + r % cj, k = klo + r / cj;
            // ray origin per world axis
            const double ax0 = D.a == 0 ? D.alpha_a : (D.b == 0 ? j + 0.5 : k + 0.5);
            const double ax1 = D.a == 1 ? D.alpha_a : (D.b == 1 ? j + 0.5 : k + 0.5);
            const double ax2 = D.a == 2 ? D.alpha_a : k + 0.5;   // axis 2 is never b
            double t0l, t0h, t1l, t1h, t2l, t2h;
            if (!clip1(ax0, D.beta[0], D.rbeta[0], lo0, hi0, t0l, t0h)) continue;
            if (!clip1(ax1, D.beta[1], D.rbeta[1], lo1, hi1, t1l, t1h)) continue;
            if (!clip1(ax2, D.beta[2], D.rbeta[2], lo2, hi2, t2l, t2h)) continue;
            const double slo = fmax(t0l, fmax(t1l, t2l));
            const double shi = fmin(t0h, fmin(t1h, t2h));
            if (!(shi > slo)) continue;
            // where the ray enters the whole mesh: the boundary intensity applies
            double u0l, u0h, u1l, u1h, u2l, u2h;
            clip1(ax0, D.beta[0], D.rbeta[0], 0.0, (double)M.nx, u0l, u0h);
            clip1(ax1, D.beta[1], D.rbeta[1], 0.0, (double)M.ny, u1l, u1h);
            clip1(ax2, D.beta[2], D.rbeta[2], 0.0, (double)M.nz, u2l, u2h);
            const double sdom = fmax(u0l, fmax(u1l, u2l));

            const long long sidx = D.state_off + ((long long)(k - D.k0) * D.nj + (j - D.j0)) * nb;
            float I[ART_MAX_NB];
#pragma unroll
            for (int b = 0; b < ART_MAX_NB; ++b)
                if (b < nb) I[b] = (slo == sdom) ? M.I_bc : M.state[sidx + b];

            int m0 = entry_cell(t0l == slo && D.beta[0] != 0.0, D.beta[0], lo0, hi0, ax0 + D.beta[0] * slo);
            int m1 = entry_cell(t1l == slo && D.beta[1] != 0.0, D.beta[1], lo1, hi1, ax1 + D.beta[1] * slo);
            int m2 = entry_cell(t2l == slo && D.beta[2] != 0.0, D.beta[2], lo2, hi2, ax2 + D.beta[2] * slo);
            double s0 = next_cross(m0, ax0, D.beta[0], D.rbeta[0]);
            double s1 = next_cross(m1, ax1, D.beta[1], D.rbeta[1]);
            double s2 = next_cross(m2, ax2, D.beta[2], D.rbeta[2]);
            const int st0 = D.beta[0] < 0.0 ? -1 : 1;
            const int st1 = D.beta[1] < 0.0 ? -1 : 1;
            const int st2 = D.beta[2] < 0.0 ? -1 : 1;
            double s = slo;

            for (int iter = 0; iter < maxit; ++iter) {
                const double sn = fmin(s0, fmin(s1, s2));
                const float ds = (float)(sn - s);
                const float dl = ds * invw_f;
                const long long cell = ((long long)m2 * M.ny + m1) * M.nx + m0;
                const int lcell = ((m2 - lo2) * M.by + (m1 - lo1)) * M.bx + (m0 - lo0);
                const float4 *f = M.fields + cell * nb;
#pragma unroll
                for (int b = 0; b < ART_MAX_NB; ++b) {
                    if (b < nb) {
                        const float4 F = f[b];
                        const float x = F.x * dl;
                        // large-x branch
                        const float e = __builtin_amdgcn_exp2f(-x * ART_LOG2E);
                        const float e1l = 1.0f - e;
                        const float lphil = e1l * (F.y * w_f);
                        const float lpsil = ds - lphil;
                        // small-x branch: q = (x - 1 + e^{-x}) / x^2
                        const float qq = fmaf(x, fmaf(x, fmaf(x, fmaf(x, 1.0f / 720.0f, -1.0f / 120.0f),
                                                              1.0f / 24.0f), -1.0f / 6.0f), 0.5f);
                        const float xq = x * qq;
                        const float lpsis = ds * xq;
                        const float lphis = ds - lpsis;
                        const float e1s = fmaf(-x, xq, x);
                        const bool small = x < 0.125f;
                        const float e1 = small ? e1s : e1l;
                        const float lphi = small ? lphis : lphil;
                        const float lpsi = small ? lpsis : lpsil;
                        lds_add(&lds[(2 * b) * V + lcell], I[b] * lphi);
                        lds_add(&lds[(2 * b + 1) * V + lcell], lpsi);
                        I[b] = fmaf(F.z - I[b], e1, I[b]);
                    }
                }
                s = sn;
                bool out = false;
                if (s0 == sn) {
                    m0 += st0;
                    out |= (m0 < lo0) | (m0 >= hi0);
                    s0 = next_cross(m0, ax0, D.beta[0], D.rbeta[0]);
                }
                if (s1 == sn) {
                    m1 += st1;
                    out |= (m1 < lo1) | (m1 >= hi1);
                    s1 = next_cross(m1, ax1, D.beta[1], D.rbeta[1]);
                }
                if (s2 == sn) {
                    m2 += st2;
                    out |= (m2 < lo2) | (m2 >= hi2);
                    s2 = next_cross(m2, ax2, D.beta[2], D.rbeta[2]);
                }
                if (out) break;
            }
#pragma unroll
            for (int b = 0; b < ART_MAX_NB; ++b)
                if (b < nb) M.state[sidx + b] = I[b];
        }
    }
    __syncthreads();

    // Flush: this workgroup is the only writer of its block in this bucket's copy.
    float *dst = M.acc + (long long)it.bucket * nb * 2 * M.ncell;
    const int ex = hi0 - lo0, ey = hi1 - lo1;
    const int nrow = nb * 2 * M.bz * M.by;
    for (int row = threadIdx.x / 64; row < nrow; row += blockDim.x / 64) {
        const int comp = row / (M.bz * M.by);
        const int ly = row % M.by, lz = (row / M.by) % M.bz;
        if (ly >= ey || lo2 + lz >= hi2) continue;
        const long long gbase = comp * M.ncell + ((long long)(lo2 + lz) * M.ny + (lo1 + ly)) * M.nx + lo0;
        const float *src = lds + comp * V + (lz * M.by + ly) * M.bx;
        for (int lx = threadIdx.x % 64; lx < ex; lx += 64) dst[gbase + lx] = src[lx];
    }
}

}  // namespace

int art_march_max_lds_bytes() { return 160 * 1024; }

hipError_t art_launch_march(const ArtItem *items, int nitems, const ArtMeshDesc *meshes,
                            int lds_floats, int threads, hipStream_t stream)
{
    if (nitems <= 0) return hipSuccess;
    const size_t bytes = (size_t)lds_floats * sizeof(float);
    static int configured = 0;
    if (!configured) {
        hipError_t e = hipFuncSetAttribute((const void *)art_march_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           art_march_max_lds_bytes());
        if (e != hipSuccess) return e;
        configured = 1;
    }
    hipLaunchKernelGGL(art_march_kernel, dim3(nitems), dim3(threads), bytes, stream, items, meshes);
    return hipGetLastError();
}
