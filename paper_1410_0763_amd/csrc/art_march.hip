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
// Inside a workgroup the lanes are persistent: the candidate rays of all the
// bucket's directions form one index range, and a lane whose ray has left the
// block takes the next candidate, so lanes do not idle while the longest ray
// of their wave finishes.  Idle lanes are refilled together once enough of
// them are waiting, which amortises the divergent set-up.
//
// Per segment of length dL (in cells) and depth step ds = dL |n_a|, for each
// frequency bin (eq rt and eq path_averaged_intensity):
//   x = kappa h dL,  e1 = 1 - e^{-x},  phi = e1 / x,
//   A1 += ds * I * phi        (sum_j dtau_j Ibar_in,j / sum_j dtau_j per direction)
//   A2 += ds * (1 - phi)      (exact path average of the source term)
//   I  <- I + (S - I) e1      (= I e^{-x} + S (1 - e^{-x}))
// For x < 1/8, e1, phi and 1 - phi come from the Taylor series of
// (x - 1 + e^{-x}) / x^2 so that none of them cancels; above, from v_exp_f32.
// Geometry (entry points, plane crossings) is double precision; transfer is
// single precision.
#include "art_internal.h"

#define ART_MAX_NB 4
#define ART_DIR_CHUNK 64
#define ART_LOG2E 1.4426950408889634f

namespace {

// One direction of the bucket, with its candidate rays for this block.
struct DirRow {
    double beta[3];       // dx_i/ds
    double rbeta[3];      // 1/beta_i or 0
    double alpha_a;       // x_a at depth 0
    long long state_off;
    float invw, w;
    int a, b;             // dominant axis, first transverse axis (c = 3 - a - b)
    int jlo, cj, klo, ck; // candidate lattice rectangle for this block
    int pre;              // exclusive prefix of cj * ck over the chunk
    int j0, nj, k0;
    int pad[4];
};
static_assert(sizeof(DirRow) == 128, "DirRow layout");

__device__ __forceinline__ void lds_add(float *p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ double pick3(int i, double v0, double v1, double v2)
{
    return i == 0 ? v0 : (i == 1 ? v1 : v2);
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

// Entry cell along one axis and the depth of its next plane crossing.
__device__ __forceinline__ void enter_axis(bool via_face, double x0, double beta, double rbeta,
                                           int lo, int hi, double slo, int &m, double &snext,
                                           double &dstep, int &st)
{
    int mm = via_face ? (beta > 0.0 ? lo : hi - 1) : (int)floor(x0 + beta * slo);
    mm = min(max(mm, lo), hi - 1);
    m = mm;
    if (beta > 0.0) {
        snext = ((double)(mm + 1) - x0) * rbeta;
        dstep = rbeta;
        st = 1;
    } else if (beta < 0.0) {
        snext = ((double)mm - x0) * rbeta;
        dstep = -rbeta;
        st = -1;
    } else {
        snext = INFINITY;
        dstep = 0.0;
        st = 0;
    }
}

// Global-address-space views: pointers read from the mesh descriptor are
// generic, and generic (flat) loads would share the LDS wait counter.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v4f g_f4;
typedef __attribute__((address_space(1))) float g_f;

template <int NB>
__global__ __launch_bounds__(1024) void art_march_kernel(const ArtItem *__restrict__ items,
                                                         const ArtMeshDesc *__restrict__ meshes,
                                                         int refill,
                                                         unsigned int *__restrict__ seg_count)
{
    extern __shared__ __align__(16) float lds[];
    const ArtItem it = items[blockIdx.x];
    const ArtMeshDesc M = meshes[it.mesh];
    const int dbeg = M.bucket_start[it.bucket], dend = M.bucket_start[it.bucket + 1];
    if (dbeg == dend) {
        if (threadIdx.x == 0) seg_count[blockIdx.x] = 0u;
        return;
    }

    constexpr int nb = NB;
    const int PX = M.bx + 1;              // odd row pitch: strided lanes hit distinct banks
    const int PXY = PX * M.by;
    const int Vp = PXY * M.bz;
    const int nacc = ((nb * 2 * Vp + 31) / 32) * 32;
    float *accl = lds;
    DirRow *tab = reinterpret_cast<DirRow *>(lds + nacc);
    for (int i = threadIdx.x; i < nb * 2 * Vp; i += blockDim.x) accl[i] = 0.0f;

    const int bxi = it.block % M.nbx;
    const int byi = (it.block / M.nbx) % M.nby;
    const int bzi = it.block / (M.nbx * M.nby);
    const int lo0 = bxi * M.bx, lo1 = byi * M.by, lo2 = bzi * M.bz;
    const int hi0 = min(lo0 + M.bx, M.nx), hi1 = min(lo1 + M.by, M.ny), hi2 = min(lo2 + M.bz, M.nz);
    const int nxny = M.nx * M.ny;
    g_f4 *fields = (g_f4 *)M.fields;
    g_f *state = (g_f *)M.state;
    const float I_bc = M.I_bc;
    const int T = blockDim.x;
    const int lane = threadIdx.x & 63;
    const int maxit = (hi0 - lo0) + (hi1 - lo1) + (hi2 - lo2) + 3;   // steps of one ray, with margin
    unsigned int nseg = 0;   // segments of positive length marched by this lane

    for (int chunk = dbeg; chunk < dend; chunk += ART_DIR_CHUNK) {
        const int K = min(ART_DIR_CHUNK, dend - chunk);
        __syncthreads();   // the previous chunk's table is no longer read
        if ((int)threadIdx.x < K) {
            const ArtDir D = M.dirs[M.order[chunk + threadIdx.x]];
            DirRow R;
            for (int q = 0; q < 3; ++q) {
                R.beta[q] = D.beta[q];
                R.rbeta[q] = D.rbeta[q];
            }
            R.alpha_a = D.alpha_a;
            R.state_off = D.state_off;
            R.invw = (float)D.invw;
            R.w = (float)D.w;
            R.a = D.a;
            R.b = D.b;
            R.j0 = D.j0; R.nj = D.nj; R.k0 = D.k0;
            // depth range of the block along a, then the lattice indices whose
            // rays can meet the block (one spare index each side)
            const double ba = pick3(D.a, D.beta[0], D.beta[1], D.beta[2]);
            const double la = D.a == 0 ? lo0 : (D.a == 1 ? lo1 : lo2);
            const double ha = D.a == 0 ? hi0 : (D.a == 1 ? hi1 : hi2);
            const double sa0 = fmin((la - D.alpha_a) * ba, (ha - D.alpha_a) * ba);
            const double sa1 = fmax((la - D.alpha_a) * ba, (ha - D.alpha_a) * ba);
            const double tb = pick3(D.b, D.beta[0], D.beta[1], D.beta[2]);
            const double tc = pick3(D.c, D.beta[0], D.beta[1], D.beta[2]);
            const double lb = D.b == 0 ? lo0 : lo1, hb = D.b == 0 ? hi0 : hi1;
            const double lc = D.c == 1 ? lo1 : lo2, hc = D.c == 1 ? hi1 : hi2;
            int jlo = (int)floor(lb - 0.5 - fmax(tb * sa0, tb * sa1)) - 1;
            int jhi = (int)ceil(hb - 0.5 - fmin(tb * sa0, tb * sa1)) + 1;
            int klo = (int)floor(lc - 0.5 - fmax(tc * sa0, tc * sa1)) - 1;
            int khi = (int)ceil(hc - 0.5 - fmin(tc * sa0, tc * sa1)) + 1;
            jlo = max(jlo, D.j0); jhi = min(jhi, D.j0 + D.nj - 1);
            klo = max(klo, D.k0); khi = min(khi, D.k0 + D.nk - 1);
            R.jlo = jlo; R.cj = max(jhi - jlo + 1, 0);
            R.klo = klo; R.ck = max(khi - klo + 1, 0);
            R.pre = 0;
            R.pad[0] = R.pad[1] = R.pad[2] = R.pad[3] = 0;
            tab[threadIdx.x] = R;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int q = 0; q < K; ++q) {
                tab[q].pre = acc;
                acc += tab[q].cj * tab[q].ck;
            }
            tab[ART_DIR_CHUNK].pre = acc;   // spare row holds the chunk's total
        }
        __syncthreads();
        const int total = tab[ART_DIR_CHUNK].pre;

        // ---- persistent lanes ------------------------------------------
        int r = (int)threadIdx.x - T;
        int q = 0;                 // this lane's row in the table (non-decreasing)
        bool active = false, done = false;
        // ray state
        double s = 0.0, sn0 = 0.0, sn1 = 0.0, sn2 = 0.0, dd0 = 0.0, dd1 = 0.0, dd2 = 0.0;
        int m0 = 0, m1 = 0, m2 = 0, st0 = 0, st1 = 0, st2 = 0, cell = 0, lcell = 0, nstep = 0;
        float invw = 0.f, wdir = 0.f;
        long long sidx = 0;
        float I[NB];
        v4f F[NB];   // fields of the current cell, loaded one step ahead
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            I[b] = 0.f;
            F[b] = v4f{0.f, 0.f, 0.f, 0.f};
        }

        while (true) {
            const unsigned long long waiting = __ballot(!active && !done);
            const unsigned long long busy = __ballot(active);
            if (!waiting && !busy) break;
            if (waiting && (!busy || __popcll(waiting) >= refill) && !active && !done) {
                // take candidates until one meets the block or none are left
                while (true) {
                    r += T;
                    if (r >= total) {
                        done = true;
                        break;
                    }
                    while (q + 1 < K && tab[q + 1].pre <= r) ++q;
                    const DirRow &R = tab[q];
                    const int loc = r - R.pre;
                    const int j = R.jlo + loc % R.cj, k = R.klo + loc / R.cj;
                    const int ra = R.a, rb = R.b;
                    const double aa = R.alpha_a;
                    const double ax0 = ra == 0 ? aa : (rb == 0 ? j + 0.5 : k + 0.5);
                    const double ax1 = ra == 1 ? aa : (rb == 1 ? j + 0.5 : k + 0.5);
                    const double ax2 = ra == 2 ? aa : k + 0.5;   // axis 2 is never b
                    const double b0 = R.beta[0], b1 = R.beta[1], b2 = R.beta[2];
                    const double r0 = R.rbeta[0], r1 = R.rbeta[1], r2 = R.rbeta[2];
                    double t0l, t0h, t1l, t1h, t2l, t2h;
                    if (!clip1(ax0, b0, r0, lo0, hi0, t0l, t0h)) continue;
                    if (!clip1(ax1, b1, r1, lo1, hi1, t1l, t1h)) continue;
                    if (!clip1(ax2, b2, r2, lo2, hi2, t2l, t2h)) continue;
                    const double slo = fmax(t0l, fmax(t1l, t2l));
                    const double shi = fmin(t0h, fmin(t1h, t2h));
                    if (!(shi > slo)) continue;
                    // where the ray enters the whole mesh the boundary intensity applies
                    double u0l, u0h, u1l, u1h, u2l, u2h;
                    clip1(ax0, b0, r0, 0.0, (double)M.nx, u0l, u0h);
                    clip1(ax1, b1, r1, 0.0, (double)M.ny, u1l, u1h);
                    clip1(ax2, b2, r2, 0.0, (double)M.nz, u2l, u2h);
                    const double sdom = fmax(u0l, fmax(u1l, u2l));
                    sidx = R.state_off + ((long long)(k - R.k0) * R.nj + (j - R.j0)) * nb;
                    const bool fresh = (slo == sdom);
#pragma unroll
                    for (int b = 0; b < NB; ++b) I[b] = fresh ? I_bc : state[sidx + b];
                    enter_axis(t0l == slo && b0 != 0.0, ax0, b0, r0, lo0, hi0, slo, m0, sn0, dd0, st0);
                    enter_axis(t1l == slo && b1 != 0.0, ax1, b1, r1, lo1, hi1, slo, m1, sn1, dd1, st1);
                    enter_axis(t2l == slo && b2 != 0.0, ax2, b2, r2, lo2, hi2, slo, m2, sn2, dd2, st2);
                    s = slo;
                    cell = (m2 * M.ny + m1) * M.nx + m0;
                    lcell = (m2 - lo2) * PXY + (m1 - lo1) * PX + (m0 - lo0);
#pragma unroll
                    for (int b = 0; b < NB; ++b) F[b] = fields[(long long)cell * NB + b];
                    invw = R.invw;
                    wdir = R.w;
                    nstep = 0;
                    active = true;
                    break;
                }
            }
            if (active) {
                const double sn = fmin(sn0, fmin(sn1, sn2));
                const float ds = (float)(sn - s);
                const float dl = ds * invw;
                nseg += ds > 0.0f ? 1u : 0u;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const float x = F[b].x * dl;
                    // large-x branch
                    const float e = __builtin_amdgcn_exp2f(-x * ART_LOG2E);
                    const float e1l = 1.0f - e;
                    const float lphil = e1l * (F[b].y * wdir);
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
                    lds_add(&accl[(2 * b) * Vp + lcell], I[b] * lphi);
                    lds_add(&accl[(2 * b + 1) * Vp + lcell], lpsi);
                    I[b] = fmaf(F[b].z - I[b], e1, I[b]);
                }
                s = sn;
                const bool x0 = sn0 == sn, x1 = sn1 == sn, x2 = sn2 == sn;
                const int d0 = x0 ? st0 : 0, d1 = x1 ? st1 : 0, d2 = x2 ? st2 : 0;
                m0 += d0; m1 += d1; m2 += d2;
                sn0 = x0 ? sn0 + dd0 : sn0;
                sn1 = x1 ? sn1 + dd1 : sn1;
                sn2 = x2 ? sn2 + dd2 : sn2;
                cell += d0 + d1 * M.nx + d2 * nxny;
                lcell += d0 + d1 * PX + d2 * PXY;
                // a ray leaves the block within maxit steps; the cap only guards the loop
                const bool out = (m0 < lo0) | (m0 >= hi0) | (m1 < lo1) | (m1 >= hi1) |
                                 (m2 < lo2) | (m2 >= hi2) | (++nstep >= maxit);
                if (out) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) state[sidx + b] = I[b];
                    active = false;
                } else {
                    // next cell's fields: in flight while the wave does other work
#pragma unroll
                    for (int b = 0; b < NB; ++b) F[b] = fields[(long long)cell * NB + b];
                }
            }
        }
    }
    // workgroup total of marched segments (work accounting)
    for (int off = 32; off > 0; off >>= 1) nseg += __shfl_down(nseg, off, 64);
    __syncthreads();
    unsigned int *wg_count = reinterpret_cast<unsigned int *>(&tab[ART_DIR_CHUNK].pad[0]);
    if (threadIdx.x == 0) *wg_count = 0u;
    __syncthreads();
    if (lane == 0) atomicAdd(wg_count, nseg);
    __syncthreads();
    if (threadIdx.x == 0) seg_count[blockIdx.x] = *wg_count;

    // Flush: this workgroup is the only writer of its block in this bucket's copy.
    g_f *dst = (g_f *)M.acc + (long long)it.bucket * nb * 2 * M.ncell;
    const int ex = hi0 - lo0, ey = hi1 - lo1;
    const int nrow = nb * 2 * M.bz * M.by;
    for (int row = threadIdx.x / 64; row < nrow; row += T / 64) {
        const int comp = row / (M.bz * M.by);
        const int ly = row % M.by, lz = (row / M.by) % M.bz;
        if (ly >= ey || lo2 + lz >= hi2) continue;
        const long long gbase = comp * M.ncell + ((long long)(lo2 + lz) * M.ny + (lo1 + ly)) * M.nx + lo0;
        const float *src = accl + comp * Vp + lz * PXY + ly * PX;
        for (int lx = lane; lx < ex; lx += 64) dst[gbase + lx] = src[lx];
    }
}

}  // namespace

int art_march_max_lds_bytes() { return 160 * 1024; }

// LDS floats of one workgroup: padded accumulators plus the direction table.
int art_march_lds_floats(int bx, int by, int bz, int nb)
{
    const int acc = nb * 2 * (bx + 1) * by * bz;
    return ((acc + 31) / 32) * 32 + (ART_DIR_CHUNK + 1) * (int)(sizeof(DirRow) / sizeof(float));
}

hipError_t art_launch_march(const ArtItem *items, int nitems, const ArtMeshDesc *meshes, int nb,
                            int lds_floats, int threads, unsigned int *seg_count,
                            hipStream_t stream)
{
    if (nitems <= 0) return hipSuccess;
    const size_t bytes = (size_t)lds_floats * sizeof(float);
    static size_t configured[5] = {0, 64 * 1024, 64 * 1024, 64 * 1024, 64 * 1024};
    if (nb < 1 || nb > 4) return hipErrorInvalidValue;
    if (bytes > configured[nb]) {
        const void *fn = nb == 1 ? (const void *)art_march_kernel<1>
                       : nb == 2 ? (const void *)art_march_kernel<2>
                       : nb == 3 ? (const void *)art_march_kernel<3>
                                 : (const void *)art_march_kernel<4>;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        configured[nb] = bytes;
    }
    const int refill = 16;
    switch (nb) {
    case 1: hipLaunchKernelGGL(art_march_kernel<1>, dim3(nitems), dim3(threads), bytes, stream, items, meshes, refill, seg_count); break;
    case 2: hipLaunchKernelGGL(art_march_kernel<2>, dim3(nitems), dim3(threads), bytes, stream, items, meshes, refill, seg_count); break;
    case 3: hipLaunchKernelGGL(art_march_kernel<3>, dim3(nitems), dim3(threads), bytes, stream, items, meshes, refill, seg_count); break;
    case 4: hipLaunchKernelGGL(art_march_kernel<4>, dim3(nitems), dim3(threads), bytes, stream, items, meshes, refill, seg_count); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
