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
// c-plane crossing, splitting the slab into up to three segments.  At a
// crossing every ray moves to the neighbouring column, i.e. the intensities
// move one lane over (DPP row shift along b, ds_bpermute along c); edge lanes
// hand rays to and from the neighbouring blocks through the state buffer.  A
// lane reads its own cell's fields once per slab and adds its contributions to
// its own cell once per slab.  The per-(direction, slab) pattern comes from a
// table built once per sweep and is read with scalar loads, so every branch on
// it is a scalar branch (its segment lengths stay in vector registers).
//
// A wave marches K directions at once and orders a slab's work by phase: the
// first segment of every direction, then the first crossing and second
// segment of every direction, then the second crossing and third segment.
// The rays that enter the tile during the slab are loaded at its top and are
// first needed after the K first segments; the next slab's fields are loaded
// one slab ahead.
//
// Memory is addressed through buffer descriptors with 32-bit byte offsets
// (wave-uniform bases in scalar registers): a direction's state region, and
// the block's field records.  A lane that must not store (it is not at the
// tile edge the rays leave through, or outside the mesh) stores to an offset
// beyond the descriptor's range, which the hardware drops.  Each direction's
// state region starts with a boundary slot holding I_bc, read by every lane
// whose ray enters through a mesh face (and by lanes that need no ray).
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

typedef float v3f __attribute__((ext_vector_type(3)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef __attribute__((address_space(1))) float g_f;
typedef __attribute__((address_space(1))) const u32x4 g_u4;
typedef __attribute__((address_space(4))) const ArtDir c_dir;
typedef __attribute__((address_space(4))) const int c_int;

// Buffer descriptor of `bytes` bytes at p (word 3 as for every gfx9 part:
// 32-bit data format, no swizzle).  Accesses at offsets >= bytes read 0 and
// write nothing.
__device__ __forceinline__ rsrc_t make_rsrc(const void *p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

// A byte offset no descriptor here reaches (every range is below 2^31 bytes).
#define ART_OOB 0x80000000u

// The NB floats of a ray-state slot.
template <int NB>
__device__ __forceinline__ void load_slot(rsrc_t r, unsigned off, float *v)
{
    if constexpr (NB == 4) {
        const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        v[0] = __uint_as_float(x.x); v[1] = __uint_as_float(x.y);
        v[2] = __uint_as_float(x.z); v[3] = __uint_as_float(x.w);
    } else if constexpr (NB == 3) {
        const u32x3 x = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
        v[0] = __uint_as_float(x.x); v[1] = __uint_as_float(x.y); v[2] = __uint_as_float(x.z);
    } else if constexpr (NB == 2) {
        const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        v[0] = __uint_as_float(x.x); v[1] = __uint_as_float(x.y);
    } else {
        v[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
}

template <int NB>
__device__ __forceinline__ void store_slot(rsrc_t r, unsigned off, const float *v)
{
    if constexpr (NB == 4) {
        const u32x4 x = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                         __float_as_uint(v[3])};
        __builtin_amdgcn_raw_buffer_store_b128(x, r, off, 0, 0);
    } else if constexpr (NB == 3) {
        const u32x3 x = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2])};
        __builtin_amdgcn_raw_buffer_store_b96(x, r, off, 0, 0);
    } else if constexpr (NB == 2) {
        const u32x2 x = {__float_as_uint(v[0]), __float_as_uint(v[1])};
        __builtin_amdgcn_raw_buffer_store_b64(x, r, off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[0]), r, off, 0, 0);
    }
}

// Field record {kappa h, 1/(kappa h), S} of one (cell, bin): 12 bytes of a
// 16-byte record (a dead fourth register would be reused at once and force a
// wait for the whole load).
__device__ __forceinline__ v3f load_field(rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(v3f, __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, 0));
}

// A wave-uniform value kept in a vector register: per-direction constants
// that only feed vector arithmetic would otherwise occupy scalar registers,
// which the K interleaved directions exhaust.
__device__ __forceinline__ float in_vgpr(float x)
{
    float v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
    return v;
}
__device__ __forceinline__ unsigned in_vgpr(unsigned x)
{
    unsigned v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
    return v;
}

__device__ __forceinline__ void lds_add(float *p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Value of `v` in lane `src` of the wave (src in [0, 64)); all lanes active.
__device__ __forceinline__ float lane_get(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
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

// One segment of depth length ds in the lane's cell, for every bin; fw[b] is
// |n_a| / (kappa_b h) of the cell.
template <int NB>
__device__ __forceinline__ void segment(const v3f *F, const float *fw, float ds, float invw,
                                        float *I, float *a1, float *a2)
{
    const float dl = ds * invw;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const float x = F[b].x * dl;
        // large-x branch
        const float e = __builtin_amdgcn_exp2f(-x * ART_LOG2E);
        const float e1l = 1.0f - e;
        const float lphil = e1l * fw[b];
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

template <int NB, int K>
__global__ __launch_bounds__(512) void art_march_kernel(const ArtItem *__restrict__ items,
                                                        const ArtMeshDesc *__restrict__ meshes,
                                                        unsigned int *__restrict__ seg_count)
{
    extern __shared__ __align__(16) float lds[];
    const ArtItem it = items[blockIdx.x];
    const ArtMeshDesc &M = meshes[it.mesh];
    // (read through a generic pointer, which the compiler cannot prove uniform)
    const int dbeg = __builtin_amdgcn_readfirstlane(M.bucket_start[it.bucket]);
    const int dend = __builtin_amdgcn_readfirstlane(M.bucket_start[it.bucket + 1]);
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
    // All directions of the bucket share its octant, so along b the rays only
    // ever move one way (sgb = +1 or -1, towards larger or smaller b), and so
    // along c.  When all rays move one column (b) or row (c): the lane's ray
    // leaves the tile or the mesh (store its state: Lb / Lc), the lane takes
    // the neighbour lane's ray (Tb / Tc), or it loads a ray arriving from the
    // next tile (Nb / Nc; otherwise a fresh ray enters the mesh with I_bc).
    const bool bneg = (oct >> ab) & 1, cneg = (oct >> ac) & 1;
    const bool Lb = in_dom && (bneg ? col == 0 : (col == 7 || gb + 1 >= Nb));
    const bool Tb = bneg ? (col <= 6 && gb + 1 < Nb) : col >= 1;
    const bool Nb_ = in_dom && (bneg ? (col == 7 && gb + 1 < Nb) : (col == 0 && gb >= 1));
    const bool Lc = in_dom && (cneg ? row == 0 : (row == 7 || gc + 1 >= Nc));
    const bool Tc = cneg ? (row <= 6 && gc + 1 < Nc) : row >= 1;
    const bool Nc_ = in_dom && (cneg ? (row == 7 && gc + 1 < Nc) : (row == 0 && gc >= 1));
    const int csrc = (min(7, max(0, row + (cneg ? 1 : -1))) << 3) + col;   // lane a c-move takes from

    // LDS accumulators: per cell of the block, {A1, A2} of every bin.
    const int V = depth * 64;                             // cells of one block
    float *accl = lds;
    for (int i = threadIdx.x; i < NB * 2 * V; i += blockDim.x) accl[i] = 0.0f;
    __syncthreads();

    // Field records of the block: base at its lowest cell, lane offset fixed,
    // slab offset in the scalar offset.
    const long long base_cell = (long long)lo_a * sa + (long long)lo_b * sb + (long long)lo_c * sc;
    const long long rec_left = (M.ncell - base_cell) * NB * 16;
    const rsrc_t rF = make_rsrc((const float4 *)M.fields + base_cell * NB,
                                (unsigned)min(rec_left, 0x7fffffffll));
    const unsigned foff = in_dom ? (unsigned)((col * sb + row * sc) * NB * 16) : 0u;
    auto slab_soff = [&](int t) {     // byte offset of the t-th slab swept
        const int la = sig_neg ? nslab - 1 - t : t;
        return (unsigned)(la * sa * NB * 16);
    };
    g_u4 *geo = (g_u4 *)M.geo;
    c_dir *dirs = (c_dir *)M.dirs;
    c_int *order = (c_int *)M.order;
    const int gstride = M.geo_stride;
    // The bucket's ray states are one contiguous range (boundary slot of its
    // first direction up to the last ray of its last direction).
    const long long sbase = dirs[order[dbeg]].state_off - NB;
    const c_dir &Dl = dirs[order[dend - 1]];
    const rsrc_t rS = make_rsrc(M.state + sbase,
                                (unsigned)((Dl.state_off + (long long)Dl.nj * Dl.nk * NB - sbase) * 4));
    unsigned int sseg = 0;   // segments of positive length per in-mesh lane (wave-uniform)

    for (int q0 = dbeg + wave; q0 < dend; q0 += nwave * K) {
        bool act[K];
        int gbase[K];
        unsigned cstride[K];    // bytes between rays of neighbouring c (nj slots)
        unsigned dbase[K];      // byte offset of the direction's boundary slot in rS
        unsigned cur[K];        // byte offset of the lane's current ray in rS
        float invw[K], wdir[K];
        float I[K][NB];
        float ib[K][NB], ic[K][NB];   // rays entering the tile during the current slab
        u32x4 gcur[K], gnext[K];      // crossing table entries of the current and next slab
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const int q = q0 + m * nwave;
            act[m] = q < dend;
            const int d = act[m] ? order[q] : order[q0];
            const c_dir &D = dirs[d];
            const double tb = ab == 0 ? D.beta[0] : D.beta[1];
            const double tc = ac == 1 ? D.beta[1] : D.beta[2];
            const int Bb = (int)floor(fma(tb, (double)d0, 0.5));
            const int Bc = (int)floor(fma(tc, (double)d0, 0.5));
            gbase[m] = d * gstride;
            const unsigned db = (unsigned)((D.state_off - NB - sbase) * 4);
            cur[m] = db + (unsigned)((1 + (gc - Bc - D.k0) * D.nj + (gb - Bb - D.j0)) * NB * 4);
            cstride[m] = in_vgpr((unsigned)(D.nj * NB * 4));
            dbase[m] = in_vgpr(db);
            invw[m] = in_vgpr((float)D.invw);
            wdir[m] = in_vgpr((float)D.w);
            // rays entering through the top face come from the block above
            load_slot<NB>(rS, (in_dom && d0 > 0) ? cur[m] : dbase[m], I[m]);
            gcur[m] = geo[gbase[m] + d0];
            gnext[m] = geo[gbase[m] + min(d0 + 1, Na - 1)];
        }
        v3f F[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) F[b] = load_field(rF, foff + 16 * b, slab_soff(0));

        for (int t = 0; t < nslab; ++t) {
            const int i = d0 + t;
            // next slab's fields (past the last slab: a harmless repeat)
            const unsigned so_next = slab_soff(t + 1 < nslab ? t + 1 : t);
            v3f Fn[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) Fn[b] = load_field(rF, foff + 16 * b, so_next);
            // the table entry is the same in every lane: its code word goes to a
            // scalar register, so that every branch on it is a scalar branch
            unsigned codes[K];
#pragma unroll
            for (int m = 0; m < K; ++m) codes[m] = __builtin_amdgcn_readfirstlane(gcur[m].w);
            // rays entering the tile during this slab; the table two slabs ahead
            u32x4 gnext2[K];
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const unsigned code = codes[m];
                const int shb = (int)(code & 3u) - 1, shc = (int)((code >> 2) & 3u) - 1;
                const bool b_first = (code >> 4) & 1u;
                const int dB = shb * NB * 4;
                const int dC = shc * (int)cstride[m];
                load_slot<NB>(rS, (shb && Nb_) ? cur[m] - (b_first ? 0 : dC) - dB : dbase[m], ib[m]);
                load_slot<NB>(rS, (shc && Nc_) ? cur[m] - (b_first ? dB : 0) - dC : dbase[m], ic[m]);
                gnext2[m] = geo[gbase[m] + min(i + 2, Na - 1)];
            }
            float fw[K][NB];
#pragma unroll
            for (int m = 0; m < K; ++m)
#pragma unroll
                for (int b = 0; b < NB; ++b) fw[m][b] = F[b].y * wdir[m];
            float a1[NB], a2[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) a1[b] = a2[b] = 0.0f;

            // crossing of a b-plane: every ray moves from column gb to gb + shb
            auto cross_b = [&](int m, int shb) {
                store_slot<NB>(rS, Lb ? cur[m] : ART_OOB, I[m]);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const float moved = bneg ? shift_next(I[m][b]) : shift_prev(I[m][b]);
                    I[m][b] = Tb ? moved : ib[m][b];
                }
                cur[m] -= shb * NB * 4;
            };
            // crossing of a c-plane: every ray moves from row gc to gc + shc
            auto cross_c = [&](int m, int shc) {
                store_slot<NB>(rS, Lc ? cur[m] : ART_OOB, I[m]);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const float moved = lane_get(I[m][b], csrc);
                    I[m][b] = Tc ? moved : ic[m][b];
                }
                cur[m] -= shc * (int)cstride[m];
            };

            // phase 1: first segment of every direction
#pragma unroll
            for (int m = 0; m < K; ++m) {
                if (!act[m]) continue;
                sseg += codes[m] >> 5;
                segment<NB>(F, fw[m], __uint_as_float(gcur[m].x), invw[m], I[m], a1, a2);
            }
            // phase 2: first crossing and second segment
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const unsigned code = codes[m];
                const int shb = (int)(code & 3u) - 1, shc = (int)((code >> 2) & 3u) - 1;
                if (!act[m] || !(shb || shc)) continue;
                const bool b_first = (code >> 4) & 1u;
                if (shb && (b_first || !shc)) cross_b(m, shb); else cross_c(m, shc);
                segment<NB>(F, fw[m], __uint_as_float(gcur[m].y), invw[m], I[m], a1, a2);
            }
            // phase 3: second crossing and third segment
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const unsigned code = codes[m];
                const int shb = (int)(code & 3u) - 1, shc = (int)((code >> 2) & 3u) - 1;
                if (!act[m] || !(shb && shc)) continue;
                const bool b_first = (code >> 4) & 1u;
                if (b_first) cross_c(m, shc); else cross_b(m, shb);
                segment<NB>(F, fw[m], __uint_as_float(gcur[m].z), invw[m], I[m], a1, a2);
            }

            if (in_dom) {
                const int la = (sig_neg ? Na - 1 - i : i) - lo_a;
                float *cellacc = accl + (la * 64 + lane) * (2 * NB);
                if (nwave == 1) {
                    // a single wave owns the block: plain read-modify-write
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        cellacc[2 * b] += a1[b];
                        cellacc[2 * b + 1] += a2[b];
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        lds_add(&cellacc[2 * b], a1[b]);
                        lds_add(&cellacc[2 * b + 1], a2[b]);
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) F[b] = Fn[b];
#pragma unroll
            for (int m = 0; m < K; ++m) {
                gcur[m] = gnext[m];
                gnext[m] = gnext2[m];
            }
        }
        // rays leave through the block's far face (into the next block or out of the mesh)
#pragma unroll
        for (int m = 0; m < K; ++m)
            store_slot<NB>(rS, (act[m] && in_dom) ? cur[m] : ART_OOB, I[m]);
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
        const int comp = idx % (2 * NB), cl = idx / (2 * NB);
        const int la = cl >> 6, l = cl & 63;
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
