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
typedef float v3f __attribute__((ext_vector_type(3)));   // 16-byte stride, 12-byte loads
// Global-address-space views: pointers read from the descriptor are generic,
// and generic (flat) loads would share the LDS wait counter.  The field
// records are read as three floats: a dead fourth register would be reused
// at once and force a wait for the whole load (write-after-write).
typedef __attribute__((address_space(1))) const v3f g_f3;
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
__device__ __forceinline__ void segment(const v3f *F, float ds, float invw, float w, float *I,
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

typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const v4u c_u4;
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
    // What a lane does when all rays move one column (b) or row (c) forward
    // (+1) or back (-1): its ray leaves the tile or the mesh (store the
    // state), it takes the neighbour lane's ray, or it loads a ray arriving
    // from the next tile (otherwise a fresh ray enters the mesh with I_bc).
    const bool lbp = col == 7 || gb + 1 >= Nb, tbp = col >= 1, ibp = col == 0 && gb >= 1;
    const bool lbm = col == 0, tbm = col <= 6 && gb + 1 < Nb, ibm = col == 7 && gb + 1 < Nb;
    const bool lcp = row == 7 || gc + 1 >= Nc, tcp = row >= 1, icp = row == 0 && gc >= 1;
    const bool lcm = row == 0, tcm = row <= 6 && gc + 1 < Nc, icm = row == 7 && gc + 1 < Nc;

    const int V = depth * 64;                             // cells of one block
    float *accl = lds;
    for (int i = threadIdx.x; i < NB * 2 * V; i += blockDim.x) accl[i] = 0.0f;
    __syncthreads();

    g_f3 *fields = (g_f3 *)M.fields;
    g_f *state = (g_f *)M.state;
    c_u4 *geo = (c_u4 *)M.geo;
    c_dir *dirs = (c_dir *)M.dirs;
    c_int *order = (c_int *)M.order;
    const int gstride = M.geo_stride;
    const float I_bc = M.I_bc;
    const long long xa0 = sig_neg ? Na - 1 - d0 : d0;
    const long long cell0 = xa0 * sa + gb * sb + gc * sc;
    const long long dcell = sig_neg ? -sa : sa;
    unsigned int sseg = 0;   // segments of positive length per in-mesh lane (wave-uniform)

    // A wave marches K directions of the bucket together: q0 + m * nwave, m < K.
    // Software pipeline: at the top of slab t every load slab t+1 needs is
    // issued (its fields, the rays that enter the tile during it, and the
    // crossing table of slab t+2); they land while slab t is marched and are
    // rotated into place at its end.  All of these loads are issued by every
    // lane from a valid address (lanes that need no value read the
    // direction's first state slot or cell 0): a load under a branch, or a
    // dead register of a vector load, makes the compiler wait for it at once.
    for (int q0 = dbeg + wave; q0 < dend; q0 += nwave * K) {
        bool act[K];
        int dix[K], njm[K];
        long long cur[K];       // state slot of the lane's current ray
        long long soff[K];      // first state slot of the direction
        float invw[K], wdir[K];
        float I[K][NB];
        float ib[K][NB], ic[K][NB];   // rays entering the tile during the current slab
        bool needb[K], needc[K];
        v4u gA[K], gB[K];             // crossing tables of the current and the next slab
        // Rays entering the tile during the slab with crossing table g, for a
        // lane whose ray is in slot `at` at the top of that slab.
        auto load_incoming = [&](int m, const v4u &g, long long at, float *jb, float *jc,
                                 bool &nbm, bool &ncm) {
            const unsigned code = g.w;
            const int shb = (int)(code & 3u) - 1, shc = (int)((code >> 2) & 3u) - 1;
            const bool b_first = (code >> 4) & 1u;
            const long long dB = (long long)shb * NB;
            const long long dC = (long long)shc * njm[m] * NB;
            nbm = shb && in_dom && (shb > 0 ? ibp : ibm);
            ncm = shc && in_dom && (shc > 0 ? icp : icm);
            const long long slb = nbm ? at - (b_first ? 0 : dC) - dB : soff[m];
            const long long slc = ncm ? at - (b_first ? dB : 0) - dC : soff[m];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                jb[b] = state[slb + b];
                jc[b] = state[slc + b];
            }
        };
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int q = q0 + m * nwave;
            act[m] = q < dend;
            dix[m] = act[m] ? order[q] : order[q0];
            const c_dir &D = dirs[dix[m]];
            const double tb = ab == 0 ? D.beta[0] : D.beta[1];
            const double tc = ac == 1 ? D.beta[1] : D.beta[2];
            const int Bb = (int)floor(fma(tb, (double)d0, 0.5));
            const int Bc = (int)floor(fma(tc, (double)d0, 0.5));
            njm[m] = D.nj;
            soff[m] = D.state_off;
            cur[m] = D.state_off + ((long long)(gc - Bc - D.k0) * D.nj + (gb - Bb - D.j0)) * NB;
            invw[m] = (float)D.invw;
            wdir[m] = (float)D.w;
            // rays entering through the top face come from the block above
            const bool from_above = in_dom && d0 > 0;
            const long long s0 = from_above ? cur[m] : soff[m];
#pragma unroll
            for (int b = 0; b < NB; ++b) I[m][b] = state[s0 + b];
#pragma unroll
            for (int b = 0; b < NB; ++b) I[m][b] = from_above ? I[m][b] : I_bc;
            const long long gbase = (long long)dix[m] * gstride;
            gA[m] = geo[gbase + d0];
            gB[m] = geo[gbase + min(d0 + 1, Na - 1)];
            load_incoming(m, gA[m], cur[m], ib[m], ic[m], needb[m], needc[m]);
        }
        // lanes outside the mesh read cell 0 (their results are never stored)
        v3f F[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) F[b] = fields[(in_dom ? cell0 : 0) * NB + b];
        long long cell = cell0;

        for (int t = 0; t < nslab; ++t) {
            const int i = d0 + t;
            // prefetch for slab t+1 (past the last slab: harmless repeats)
            const long long ncell = in_dom ? (t + 1 < nslab ? cell + dcell : cell) : 0;
            v3f Fn[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) Fn[b] = fields[ncell * NB + b];
            float ibn[K][NB], icn[K][NB];
            bool needbn[K], needcn[K];
            v4u gC[K];
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const unsigned code = gA[m].w;
                const long long at = cur[m] - (long long)((int)(code & 3u) - 1) * NB -
                                     (long long)((int)((code >> 2) & 3u) - 1) * njm[m] * NB;
                load_incoming(m, gB[m], at, ibn[m], icn[m], needbn[m], needcn[m]);
                gC[m] = geo[(long long)dix[m] * gstride + min(i + 2, Na - 1)];
            }
            float a1[NB], a2[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) a1[b] = a2[b] = 0.0f;

#pragma unroll
            for (int m = 0; m < K; ++m) {
                if (!act[m]) continue;
                const v4u g = gA[m];
                const unsigned code = g.w;
                const int shb = (int)(code & 3u) - 1, shc = (int)((code >> 2) & 3u) - 1;
                const bool b_first = (code >> 4) & 1u;
                const float s1 = __uint_as_float(g.x), s2 = __uint_as_float(g.y),
                            s3 = __uint_as_float(g.z);
                sseg += code >> 5;
                const long long dB = (long long)shb * NB;
                const long long dC = (long long)shc * njm[m] * NB;
                float *Im = I[m];
                // crossing of a b-plane: every ray moves from column gb to gb + shb
                auto cross_b = [&]() {
                    if (in_dom && (shb > 0 ? lbp : lbm)) {
#pragma unroll
                        for (int b = 0; b < NB; ++b) state[cur[m] + b] = Im[b];
                    }
                    const bool take = shb > 0 ? tbp : tbm;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float moved = shb > 0 ? shift_prev(Im[b]) : shift_next(Im[b]);
                        Im[b] = take ? moved : (needb[m] ? ib[m][b] : I_bc);
                    }
                    cur[m] -= dB;
                };
                // crossing of a c-plane: every ray moves from row gc to gc + shc
                auto cross_c = [&]() {
                    if (in_dom && (shc > 0 ? lcp : lcm)) {
#pragma unroll
                        for (int b = 0; b < NB; ++b) state[cur[m] + b] = Im[b];
                    }
                    const bool take = shc > 0 ? tcp : tcm;
                    const int src = (min(7, max(0, row - shc)) << 3) + col;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float moved = lane_get(Im[b], src);
                        Im[b] = take ? moved : (needc[m] ? ic[m][b] : I_bc);
                    }
                    cur[m] -= dC;
                };
                segment<NB>(F, s1, invw[m], wdir[m], Im, a1, a2);
                if (shb && shc) {
                    if (b_first) cross_b(); else cross_c();
                    segment<NB>(F, s2, invw[m], wdir[m], Im, a1, a2);
                    if (b_first) cross_c(); else cross_b();
                    segment<NB>(F, s3, invw[m], wdir[m], Im, a1, a2);
                } else if (shb || shc) {
                    if (shb) cross_b(); else cross_c();
                    segment<NB>(F, s2, invw[m], wdir[m], Im, a1, a2);
                }
            }
            if (in_dom) {
                const int la = (sig_neg ? Na - 1 - i : i) - lo_a;
                const int lc = la * 64 + lane;
                if (nwave == 1) {
                    // a single wave owns the block: plain read-modify-write
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        accl[(2 * b) * V + lc] += a1[b];
                        accl[(2 * b + 1) * V + lc] += a2[b];
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        lds_add(&accl[(2 * b) * V + lc], a1[b]);
                        lds_add(&accl[(2 * b + 1) * V + lc], a2[b]);
                    }
                }
            }
            // rotate the pipeline
            cell += dcell;
#pragma unroll
            for (int b = 0; b < NB; ++b) F[b] = Fn[b];
#pragma unroll
            for (int m = 0; m < K; ++m) {
                gA[m] = gB[m];
                gB[m] = gC[m];
                needb[m] = needbn[m];
                needc[m] = needcn[m];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    ib[m][b] = ibn[m][b];
                    ic[m][b] = icn[m][b];
                }
            }
        }
        // rays leave through the block's far face (into the next block or out of the mesh)
#pragma unroll
        for (int m = 0; m < K; ++m) {
            if (act[m] && in_dom) {
#pragma unroll
                for (int b = 0; b < NB; ++b) state[cur[m] + b] = I[m][b];
            }
        }
    }

    // workgroup total of marched segments of positive length (work accounting)
    const unsigned int nseg = sseg * (unsigned)__popcll(__ballot(in_dom));
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
