// art_march.hip -- the ray march of the diffuse sweep (Sect. 2.2, 3.1).
//
// Work decomposition.  Directions are grouped by dominant axis a and octant
// of travel (the eight direction groups of the multiple-wave-front scheme the
// paper uses between nodes, Sect. 3.3), and each group is split into
// `subsets` buckets.  For dominant axis a the mesh is cut into blocks of
// 8 x 8 columns (transverse axes b, c) by `depth` slabs along a.  A workgroup
// owns one (block, bucket) pair; each of its waves takes whole directions of
// the bucket and sweeps the block slab by slab.  Blocks of one group on
// wavefront w (the sum of block indices counted along the group's travel
// directions) only receive rays from wavefronts < w, which earlier launches on
// the same stream have finished; a ray's intensity crosses block faces through
// its state slot.  Each workgroup stores its block into its bucket's own
// accumulator copy with plain stores: no other workgroup writes those cells of
// that copy, so no global atomics are needed (the single-writer property that
// Sect. 3.1 obtains with ray groups).
//
// Slab sweep.  Lane (col, row) of a wave owns column (lo_b + col, lo_c + row).
// Ray (j,k) sits at transverse position (j + 1/2 + t_b s, k + 1/2 + t_c s) at
// depth s, so at the top of slab i it is in column (j + B_b(i), k + B_c(i)),
// B(i) = floor(1/2 + t i): the lattice shift is the same for every ray.  Hence
// the whole wave shares one segment pattern per slab: at most one b- and one
// c-plane crossing, at depth fractions f_b, f_c, splitting the slab into up to
// three segments.  At a crossing every ray moves to the neighbouring column,
// i.e. the intensities move one lane over (ds_bpermute); edge lanes hand rays
// to and from the neighbouring blocks through the state buffer.  A lane thus
// reads its own cell's fields once per slab and adds its contributions to its
// own cell once per slab.
//
// Per segment of depth length ds (path length dL = ds / |n_a| cells), per bin
// (eq rt and eq path_averaged_intensity):
//   x = kappa h dL,  e1 = 1 - e^{-x},  phi = e1 / x,
//   A1 += ds * I * phi        (sum_j dtau_j Ibar_in,j / sum_j dtau_j per direction)
//   A2 += ds * (1 - phi)      (exact path average of the source term)
//   I  <- I + (S - I) e1      (= I e^{-x} + S (1 - e^{-x}))
// For x < 1/8, e1, phi and 1 - phi come from the Taylor series of
// (x - 1 + e^{-x}) / x^2 so that none of them cancels; above, from v_exp_f32.
// Slab geometry is double precision; transfer is single precision.
#include "art_internal.h"

#define ART_LOG2E 1.4426950408889634f

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
// Global-address-space views: pointers read from the descriptor are generic,
// and generic (flat) loads would share the LDS wait counter.
typedef __attribute__((address_space(1))) const v4f g_f4;
typedef __attribute__((address_space(1))) float g_f;

__device__ __forceinline__ void lds_add(float *p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Value of `v` in lane `src` of the wave (src in [0, 64)); all lanes active.
__device__ __forceinline__ float lane_get(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// One segment of depth length ds in the lane's cell, for every bin.
template <int NB>
__device__ __forceinline__ void segment(const v4f *F, float ds, float invw, float w, float *I,
                                        float *a1, float *a2)
{
    const float dl = ds * invw;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const float x = F[b].x * dl;
        // large-x branch
        const float e = __builtin_amdgcn_exp2f(-x * ART_LOG2E);
        const float e1l = 1.0f - e;
        const float lphil = e1l * (F[b].y * w);
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
        a1[b] = fmaf(I[b], lphi, a1[b]);
        a2[b] += lpsi;
        I[b] = fmaf(F[b].z - I[b], e1, I[b]);
    }
}

// Lane shift along b by one column (within each row of 8): row_shr:1 /
// row_shl:1 of DPP move a value from the lane before / after; the lanes of
// column 0 / 7, whose value comes from outside the row, are overwritten by
// the caller.
__device__ __forceinline__ float shift_prev(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, false));
}
__device__ __forceinline__ float shift_next(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xF, 0xF, false));
}

typedef __attribute__((address_space(4))) const v4f c_f4;
typedef __attribute__((address_space(4))) const ArtDir c_dir;
typedef __attribute__((address_space(4))) const int c_int;

template <int NB, int K>
__global__ __launch_bounds__(512) void art_march_kernel(const ArtItem *__restrict__ items,
                                                         const ArtMeshDesc *__restrict__ meshes,
                                                         unsigned int *__restrict__ seg_count)
{
    extern __shared__ __align__(16) float lds[];
    const ArtItem it = items[blockIdx.x];
    const ArtMeshDesc &M = meshes[it.mesh];
    const int dbeg = M.bucket_start[it.bucket], dend = M.bucket_start[it.bucket + 1];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwave = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    if (dbeg == dend) {
        if (threadIdx.x == 0) seg_count[blockIdx.x] = 0u;
        return;
    }
    const int subsets = M.subsets;
    const int cls = it.bucket / (8 * subsets);            // dominant axis of the bucket
    const int oct = (it.bucket / subsets) % 8;
    const int ab = cls == 0 ? 1 : 0, ac = cls == 2 ? 1 : 2;
    const int Na = cls == 0 ? M.nx : (cls == 1 ? M.ny : M.nz);
    const int Nb = ab == 0 ? M.nx : M.ny;
    const int Nc = ac == 1 ? M.ny : M.nz;
    const int depth = M.depth;
    const int nbb = (Nb + 7) / 8, nbc = (Nc + 7) / 8;
    const int pb = it.block % nbb, pc = (it.block / nbb) % nbc, pa = it.block / (nbb * nbc);
    const int lo_b = pb * 8, lo_c = pc * 8, lo_a = pa * depth;
    const int hi_a = min(lo_a + depth, Na);
    const int sig_neg = (oct >> cls) & 1;                 // rays travel towards -x_a
    const int d0 = sig_neg ? Na - hi_a : lo_a;            // depth range of the block
    const int nslab = hi_a - lo_a;

    // strides of the world cell index along a, b, c
    const long long sa = cls == 0 ? 1 : (cls == 1 ? M.nx : (long long)M.nx * M.ny);
    const long long sb = ab == 0 ? 1 : M.nx;
    const long long sc = ac == 1 ? M.nx : (long long)M.nx * M.ny;

    const int col = lane & 7, row = lane >> 3;
    const int gb = lo_b + col, gc = lo_c + row;
    const bool in_dom = gb < Nb && gc < Nc;
    const int V = depth * 64;                             // cells of one block
    float *accl = lds;
    for (int i = threadIdx.x; i < NB * 2 * V; i += blockDim.x) accl[i] = 0.0f;
    __syncthreads();

    g_f4 *fields = (g_f4 *)M.fields;
    g_f *state = (g_f *)M.state;
    c_f4 *geo = (c_f4 *)M.geo;
    c_dir *dirs = (c_dir *)M.dirs;
    c_int *order = (c_int *)M.order;
    const int gstride = M.geo_stride;
    const float I_bc = M.I_bc;
    const long long xa0 = sig_neg ? Na - 1 - d0 : d0;
    const long long cell0 = xa0 * sa + gb * sb + gc * sc;
    const long long dcell = sig_neg ? -sa : sa;
    unsigned int nseg = 0;

    // A wave marches K directions of the bucket together: q0 + m * nwave, m < K.
    for (int q0 = dbeg + wave; q0 < dend; q0 += nwave * K) {
        bool act[K];
        int dix[K], Bb[K], Bc[K], j0[K], nj[K], k0[K];
        long long soff[K];
        float invw[K], wdir[K];
        float I[K][NB];
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int q = q0 + m * nwave;
            act[m] = q < dend;
            dix[m] = act[m] ? order[q] : order[q0];
            const c_dir &D = dirs[dix[m]];
            const double tb = ab == 0 ? D.beta[0] : D.beta[1];
            const double tc = ac == 1 ? D.beta[1] : D.beta[2];
            Bb[m] = (int)floor(fma(tb, (double)d0, 0.5));
            Bc[m] = (int)floor(fma(tc, (double)d0, 0.5));
            j0[m] = D.j0; nj[m] = D.nj; k0[m] = D.k0;
            soff[m] = D.state_off;
            invw[m] = (float)D.invw;
            wdir[m] = (float)D.w;
#pragma unroll
            for (int b = 0; b < NB; ++b) I[m][b] = I_bc;
            if (act[m] && in_dom && d0 > 0) {
                const long long sl = soff[m] + ((long long)(gc - Bc[m] - k0[m]) * nj[m] + (gb - Bb[m] - j0[m])) * NB;
#pragma unroll
                for (int b = 0; b < NB; ++b) I[m][b] = state[sl + b];
            }
        }
        v4f F[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) F[b] = v4f{0.f, 0.f, 0.f, 0.f};
        if (in_dom) {
#pragma unroll
            for (int b = 0; b < NB; ++b) F[b] = fields[cell0 * NB + b];
        }
        long long cell = cell0;

        for (int t = 0; t < nslab; ++t) {
            const int i = d0 + t;
            // prefetch the next slab's fields
            v4f Fn[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) Fn[b] = v4f{0.f, 0.f, 0.f, 0.f};
            if (in_dom && t + 1 < nslab) {
#pragma unroll
                for (int b = 0; b < NB; ++b) Fn[b] = fields[(cell + dcell) * NB + b];
            }
            float a1[NB], a2[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) a1[b] = a2[b] = 0.0f;
            unsigned int ns = 0;

#pragma unroll
            for (int m = 0; m < K; ++m) {
                if (!act[m]) continue;
                const v4f g = geo[(long long)dix[m] * gstride + i];   // wave-uniform
                const int shb = (int)g.z, shc = (int)g.w;
                const float fb = g.x, fc = g.y;
                const bool b_first = fb <= fc;
                auto slot = [&](int Bb_, int Bc_) -> long long {
                    return soff[m] + ((long long)(gc - Bc_ - k0[m]) * nj[m] + (gb - Bb_ - j0[m])) * NB;
                };
                // Rays arriving from outside this tile at the crossings.
                const int srcb = col - shb, srcc = row - shc;
                const bool b_mesh = gb - shb >= 0 && gb - shb < Nb;
                const bool c_mesh = gc - shc >= 0 && gc - shc < Nc;
                const bool b_tile = srcb >= 0 && srcb <= 7;
                const bool c_tile = srcc >= 0 && srcc <= 7;
                float inb[NB], inc[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b) inb[b] = inc[b] = I_bc;
                if (shb && in_dom && b_mesh && !b_tile) {
                    const long long sl = slot(Bb[m] + shb, b_first ? Bc[m] : Bc[m] + shc);
#pragma unroll
                    for (int b = 0; b < NB; ++b) inb[b] = state[sl + b];
                }
                if (shc && in_dom && c_mesh && !c_tile) {
                    const long long sl = slot(b_first ? Bb[m] + shb : Bb[m], Bc[m] + shc);
#pragma unroll
                    for (int b = 0; b < NB; ++b) inc[b] = state[sl + b];
                }
                float *Im = I[m];
                // crossing of a b-plane: every ray moves from column gb to gb + shb
                auto cross_b = [&]() {
                    const bool leaves = col + shb < 0 || col + shb > 7 || gb + shb < 0 || gb + shb >= Nb;
                    if (in_dom && leaves) {
                        const long long sl = slot(Bb[m], Bc[m]);
#pragma unroll
                        for (int b = 0; b < NB; ++b) state[sl + b] = Im[b];
                    }
                    const bool take = b_tile && b_mesh;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float moved = shb > 0 ? shift_prev(Im[b]) : shift_next(Im[b]);
                        Im[b] = take ? moved : inb[b];
                    }
                    Bb[m] += shb;
                };
                // crossing of a c-plane: every ray moves from row gc to gc + shc
                auto cross_c = [&]() {
                    const bool leaves = row + shc < 0 || row + shc > 7 || gc + shc < 0 || gc + shc >= Nc;
                    if (in_dom && leaves) {
                        const long long sl = slot(Bb[m], Bc[m]);
#pragma unroll
                        for (int b = 0; b < NB; ++b) state[sl + b] = Im[b];
                    }
                    const int src = (min(7, max(0, srcc)) << 3) + col;
                    const bool take = c_tile && c_mesh;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float moved = lane_get(Im[b], src);
                        Im[b] = take ? moved : inc[b];
                    }
                    Bc[m] += shc;
                };
                if (shb && shc) {
                    const float f1 = fminf(fb, fc), f2 = fmaxf(fb, fc);
                    segment<NB>(F, f1, invw[m], wdir[m], Im, a1, a2);
                    if (b_first) cross_b(); else cross_c();
                    segment<NB>(F, f2 - f1, invw[m], wdir[m], Im, a1, a2);
                    if (b_first) cross_c(); else cross_b();
                    segment<NB>(F, 1.0f - f2, invw[m], wdir[m], Im, a1, a2);
                    ns += (f1 > 0.f) + (f2 - f1 > 0.f) + (1.0f - f2 > 0.f);
                } else if (shb || shc) {
                    const float f1 = shb ? fb : fc;
                    segment<NB>(F, f1, invw[m], wdir[m], Im, a1, a2);
                    if (shb) cross_b(); else cross_c();
                    segment<NB>(F, 1.0f - f1, invw[m], wdir[m], Im, a1, a2);
                    ns += (f1 > 0.f) + (1.0f - f1 > 0.f);
                } else {
                    segment<NB>(F, 1.0f, invw[m], wdir[m], Im, a1, a2);
                    ns += 1;
                }
            }
            if (in_dom) {
                nseg += ns;
                const int la = (sig_neg ? Na - 1 - i : i) - lo_a;
                const int lc = la * 64 + lane;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    lds_add(&accl[(2 * b) * V + lc], a1[b]);
                    lds_add(&accl[(2 * b + 1) * V + lc], a2[b]);
                }
            }
            cell += dcell;
#pragma unroll
            for (int b = 0; b < NB; ++b) F[b] = Fn[b];
        }
        // rays leave through the block's far face (into the next block or out of the mesh)
#pragma unroll
        for (int m = 0; m < K; ++m) {
            if (act[m] && in_dom) {
                const long long sl = soff[m] + ((long long)(gc - Bc[m] - k0[m]) * nj[m] + (gb - Bb[m] - j0[m])) * NB;
#pragma unroll
                for (int b = 0; b < NB; ++b) state[sl + b] = I[m][b];
            }
        }
    }

    // workgroup total of marched segments of positive length (work accounting)
    for (int off = 32; off > 0; off >>= 1) nseg += __shfl_down(nseg, off, 64);
    unsigned int *wg_count = reinterpret_cast<unsigned int *>(lds + NB * 2 * V);
    if (threadIdx.x == 0) *wg_count = 0u;
    __syncthreads();
    if (lane == 0) atomicAdd(wg_count, nseg);
    __syncthreads();
    if (threadIdx.x == 0) seg_count[blockIdx.x] = *wg_count;

    // Flush: this workgroup is the only writer of its block in this bucket's copy.
    g_f *dst = (g_f *)M.acc + (long long)it.bucket * NB * 2 * M.ncell;
    for (int idx = threadIdx.x; idx < NB * 2 * V; idx += blockDim.x) {
        const int comp = idx / V, rem = idx - comp * V;
        const int la = rem >> 6, l = rem & 63;
        const int cb = lo_b + (l & 7), cc = lo_c + (l >> 3);
        if (la >= nslab || cb >= Nb || cc >= Nc) continue;
        const long long wc = (lo_a + la) * sa + cb * sb + cc * sc;
        dst[comp * M.ncell + wc] = accl[idx];
    }
}

}  // namespace

int art_march_max_lds_bytes() { return 160 * 1024; }

// LDS floats of one workgroup: accumulators of depth * 64 cells plus a counter.
int art_march_lds_floats(int depth, int nb) { return nb * 2 * depth * 64 + 32; }


template <int NB, int K>
hipError_t launch_nbk(const ArtItem *items, int nitems, const ArtMeshDesc *meshes, size_t bytes,
                      int threads, unsigned int *seg_count, hipStream_t stream)
{
    static size_t configured = 64 * 1024;   // up to 64 KiB needs no opt-in
    if (bytes > configured) {
        hipError_t e = hipFuncSetAttribute((const void *)art_march_kernel<NB, K>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        configured = bytes;
    }
    if (nitems <= 0) return hipSuccess;   // a call without items only configures the kernel
    hipLaunchKernelGGL((art_march_kernel<NB, K>), dim3(nitems), dim3(threads), bytes, stream, items,
                       meshes, seg_count);
    return hipGetLastError();
}

template <int NB>
hipError_t launch_nb(const ArtItem *items, int nitems, const ArtMeshDesc *meshes, int K, size_t bytes,
                     int threads, unsigned int *seg_count, hipStream_t stream)
{
    switch (K) {
    case 1: return launch_nbk<NB, 1>(items, nitems, meshes, bytes, threads, seg_count, stream);
    case 2: return launch_nbk<NB, 2>(items, nitems, meshes, bytes, threads, seg_count, stream);
    case 4: return launch_nbk<NB, 4>(items, nitems, meshes, bytes, threads, seg_count, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t art_launch_march(const ArtItem *items, int nitems, const ArtMeshDesc *meshes, int nb,
                            int interleave, int lds_floats, int threads, unsigned int *seg_count,
                            hipStream_t stream)
{
    const size_t bytes = (size_t)lds_floats * sizeof(float);
    switch (nb) {
    case 1: return launch_nb<1>(items, nitems, meshes, interleave, bytes, threads, seg_count, stream);
    case 2: return launch_nb<2>(items, nitems, meshes, interleave, bytes, threads, seg_count, stream);
    case 3: return launch_nb<3>(items, nitems, meshes, interleave, bytes, threads, seg_count, stream);
    case 4: return launch_nb<4>(items, nitems, meshes, interleave, bytes, threads, seg_count, stream);
    default: return hipErrorInvalidValue;
    }
}
