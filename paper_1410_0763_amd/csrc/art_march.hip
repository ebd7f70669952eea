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
// face buffers laid out by block face (a move's rays, or a tile's, are one
// contiguous run), and the intensity with which it leaves the mesh goes to
// its ray-state slot.  Each workgroup stores its block into its bucket's own
// accumulator copy with plain stores: no other workgroup writes those cells of
// that copy, so no global atomics are needed (the single-writer property that
// Sect. 3.1 obtains with ray groups).
//
// Slab sweep.  Each lane of a wave owns one column of the 8 x 8 tile.  Ray
// (j,k) sits at transverse position (j + 1/2 + t_b s, k + 1/2 + t_c s) at
// depth s, so at the top of slab i it is in column (j + B_b(i), k + B_c(i)),
// B(i) = floor(1/2 + t i): the lattice shift is the same for every ray.  Hence
// the whole wave shares one segment pattern per slab: at most one b- and one
// c-plane crossing, splitting the slab into up to three segments.  At a
// crossing every ray moves to the neighbouring column.  All directions of a
// bucket travel the same way along b and c, so the lane-to-column map is
// mirrored per bucket such that a move always hands lane l - 1's ray to lane
// l along b (a DPP row shift) and lane l - 8's ray along c (ds_bpermute); edge
// lanes hand rays to and from the neighbouring blocks through the face
// buffers.  A lane reads its own cell's fields once per slab and adds its
// contributions to its own cell once per slab.  The per-(direction, slab)
// pattern comes from a table built once per sweep (segment lengths and a code
// word naming the moves in order); the code word goes to a scalar register, so
// every branch on it is a scalar branch.
//
// A wave marches K directions at once and orders a slab's work by phase: the
// first segment of every direction; the first move of every direction, then
// their second segments; the second moves, then the third segments.  The rays
// that enter the tile during the slab are loaded at its top and are first
// needed after the K first segments; the next slab's fields and table
// entries are loaded one slab ahead.
//
// Memory is addressed through buffer descriptors with 32-bit byte offsets
// (wave-uniform bases in scalar registers): the bucket's face buffers and
// ray-state region, the block's field records and the table.  A lane that must
// not store (it is not at the tile edge the rays leave through, or outside the
// mesh) stores to an offset beyond the descriptor's range, which the hardware
// drops; a load there returns 0 without touching memory.  Lanes whose ray
// enters through a mesh face, and lanes that need no ray in a slab, read out
// of range and take I_bc from a register.
//
// Field records are {kappa h, S} per (cell, bin), 8 bytes, all bins of a cell
// together; directions whose dominant axis is x read a second copy with y
// fastest, so that for every axis the lanes of a tile row read consecutive
// records.  |n_a| / (kappa h) comes from v_rcp_f32 once per slab and bin.
//
// Per segment of depth length ds (path length dL = ds / |n_a| cells), per bin
// (eq rt and eq path_averaged_intensity):
//   x = kappa h dL,  phi = (1 - e^{-x}) / x,
//   A1 += ds * I * phi        (sum_j dtau_j Ibar_in,j / sum_j dtau_j per direction)
//   A2 += ds * (1 - phi)      (exact path average of the source term)
//   I  <- I e^{-x} + S x phi  (x phi = 1 - e^{-x}; two positive terms)
// e^{-x} comes from v_exp_f32.  For x >= 1/8, phi ds = (1 - e^{-x}) |n_a| /
// (kappa h); for x < 1/8, (1 - phi) ds = x q(x) ds with q(x) = (x - 1 +
// e^{-x}) / x^2 from a degree-2 polynomial (relative error below 1.2e-6), so
// that neither phi nor 1 - phi cancels.  In both branches
// S x phi = (phi ds) (S kappa h / |n_a|), the factor formed once per slab.
// Slab geometry is double precision; transfer is single precision.
#include "art_internal.h"

namespace {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef __attribute__((address_space(1))) float g_f;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) f32x4 g_f32x4;
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

// The NB floats of a ray (a ray-state slot or a face-buffer entry) at byte
// offset off + soff (soff wave-uniform).
template <int NB>
__device__ __forceinline__ void load_slot(rsrc_t r, unsigned off, float *v, unsigned soff = 0)
{
    if constexpr (NB == 4) {
        const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0);
        v[0] = __uint_as_float(x.x); v[1] = __uint_as_float(x.y);
        v[2] = __uint_as_float(x.z); v[3] = __uint_as_float(x.w);
    } else if constexpr (NB == 3) {
        const u32x3 x = __builtin_amdgcn_raw_buffer_load_b96(r, off, soff, 0);
        v[0] = __uint_as_float(x.x); v[1] = __uint_as_float(x.y); v[2] = __uint_as_float(x.z);
    } else if constexpr (NB == 2) {
        const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0);
        v[0] = __uint_as_float(x.x); v[1] = __uint_as_float(x.y);
    } else {
        v[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    }
}

// Rays handed to another block are read again only by a later launch, so
// they are stored with the non-temporal cache policy (bit 1 of the policy
// operand, `nt`).
#define ART_STATE_STORE_POLICY 2

template <int NB>
__device__ __forceinline__ void store_slot(rsrc_t r, unsigned off, const float *v, unsigned soff = 0)
{
    if constexpr (NB == 4) {
        const u32x4 x = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                         __float_as_uint(v[3])};
        __builtin_amdgcn_raw_buffer_store_b128(x, r, off, soff, ART_STATE_STORE_POLICY);
    } else if constexpr (NB == 3) {
        const u32x3 x = {__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2])};
        __builtin_amdgcn_raw_buffer_store_b96(x, r, off, soff, ART_STATE_STORE_POLICY);
    } else if constexpr (NB == 2) {
        const u32x2 x = {__float_as_uint(v[0]), __float_as_uint(v[1])};
        __builtin_amdgcn_raw_buffer_store_b64(x, r, off, soff, ART_STATE_STORE_POLICY);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[0]), r, off, soff, ART_STATE_STORE_POLICY);
    }
}

// Field records {kappa h, S} of all NB bins of one cell (8 bytes per bin,
// two bins per 16-byte load).
template <int NB>
__device__ __forceinline__ void load_fields(rsrc_t r, unsigned voff, unsigned soff, float *kh, float *S)
{
    if constexpr (NB == 1) {
        const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        kh[0] = __uint_as_float(a.x); S[0] = __uint_as_float(a.y);
    } else {
        const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        kh[0] = __uint_as_float(a.x); S[0] = __uint_as_float(a.y);
        kh[1] = __uint_as_float(a.z); S[1] = __uint_as_float(a.w);
        if constexpr (NB == 3) {
            const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, voff + 16, soff, 0);
            kh[2] = __uint_as_float(b.x); S[2] = __uint_as_float(b.y);
        } else if constexpr (NB == 4) {
            const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0);
            kh[2] = __uint_as_float(b.x); S[2] = __uint_as_float(b.y);
            kh[3] = __uint_as_float(b.z); S[3] = __uint_as_float(b.w);
        }
    }
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

// Small x in y = -x log2(e): x q(x) = y R(y), q(x) = (x - 1 + e^{-x}) / x^2,
// R of degree 2 fitted for the least maximum relative error over x in
// [0, 1/8] (fit_small_x.py beside this file): 9.1e-7 in exact arithmetic,
// 1.15e-6 evaluated in float32.  (The Taylor series of q to third order,
// 7e-7, costs one more multiply-add per segment and bin.)
#define ART_LN2 0.69314718055994531
#define ART_R0 (-0.3465732746531325f)
#define ART_R1 (-0.08004055512772128f)
#define ART_R2 (-0.013361410132475101f)
#define ART_YSMALL ((float)(-0.125 / ART_LN2))   // x < 1/8

template <int NB>
__device__ __forceinline__ void segment(const float *kh, const float *fw, const float *sfw,
                                        float invwl, float ds, float *I, float *a1, float *a2)
{
    const float dsl = ds * invwl;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const float y = kh[b] * dsl;                     // -x log2(e)
        const float e = __builtin_amdgcn_exp2f(y);      // e^{-x}
        // large-x branch: (1 - e^{-x}) |n_a| / (kappa h), one rounding
        const float lphil = fmaf(-e, fw[b], fw[b]);
        const float lpsil = ds - lphil;
        // small-x branch (relative error below 1.2e-6 for x < 1/8)
        const float r = fmaf(y, fmaf(y, ART_R2, ART_R1), ART_R0);
        const float lpsis = ds * (y * r);
        const float lphis = ds - lpsis;
        const bool small = y > ART_YSMALL;
        const float lphi = small ? lphis : lphil;
        const float lpsi = small ? lpsis : lpsil;
        a1[b] = fmaf(I[b], lphi, a1[b]);
        a2[b] += lpsi;
        // I e^{-x} + S (1 - e^{-x}), two positive terms (the form
        // I + (S - I)(1 - e^{-x}) cancels when a bright ray enters an opaque
        // cell), with S (1 - e^{-x}) = (phi ds) S kappa h / |n_a|
        I[b] = fmaf(I[b], e, lphi * sfw[b]);
    }
}

template <int NB, int K>
__global__ __launch_bounds__(512) void art_march_kernel(const ArtItem *__restrict__ items,
                                                        const ArtMeshDesc *__restrict__ meshes,
                                                        unsigned int *__restrict__ seg_count, int priv_acc)
{
    extern __shared__ __align__(16) float lds[];
    const int it_mesh = __builtin_amdgcn_readfirstlane(items[blockIdx.x].mesh);
    const int it_block = __builtin_amdgcn_readfirstlane(items[blockIdx.x].block);
    const int it_bucket = __builtin_amdgcn_readfirstlane(items[blockIdx.x].bucket);
    const ArtMeshDesc &M = meshes[it_mesh];
    // (read through a generic pointer, which the compiler cannot prove uniform)
    const int dbeg = __builtin_amdgcn_readfirstlane(M.bucket_start[it_bucket]);
    const int dend = __builtin_amdgcn_readfirstlane(M.bucket_start[it_bucket + 1]);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwave = blockDim.x >> 6;
    const int lane = threadIdx.x & 63;
    if (dbeg == dend) {
        if (threadIdx.x == 0) seg_count[blockIdx.x] = 0u;
        return;
    }
    const int subsets = M.subsets;
    const int cls = it_bucket / (8 * subsets);            // dominant axis of the bucket
    const int oct = (it_bucket / subsets) % 8;
    const int ab = cls == 0 ? 1 : 0, ac = cls == 2 ? 1 : 2;
    const int Na = cls == 0 ? M.nx : (cls == 1 ? M.ny : M.nz);
    const int Nb = ab == 0 ? M.nx : M.ny;
    const int Nc = ac == 1 ? M.ny : M.nz;
    const int depth = M.depth;
    const int nbb = (Nb + 7) / 8, nbc = (Nc + 7) / 8;
    const int pb = it_block % nbb, pc = (it_block / nbb) % nbc, pa = it_block / (nbb * nbc);
    const int lo_b = pb * 8, lo_c = pc * 8, lo_a = pa * depth;
    const int hi_a = min(lo_a + depth, Na);
    const int sig_neg = (oct >> cls) & 1;                 // rays travel towards -x_a
    const int d0 = sig_neg ? Na - hi_a : lo_a;            // depth range of the block
    const int nslab = hi_a - lo_a;

    // strides of the world cell index along a, b, c
    const long long sa = cls == 0 ? 1 : (cls == 1 ? M.nx : (long long)M.nx * M.ny);
    const long long sb = ab == 0 ? 1 : M.nx;
    const long long sc = ac == 1 ? M.nx : (long long)M.nx * M.ny;

    // All directions of the bucket share its octant, so along b every ray
    // moves the same way (towards smaller b if bneg), and so along c.  Lane
    // (cl, rw) owns tile column cl, or 7 - cl if bneg (row rw, or 7 - rw if
    // cneg): a b-move then always hands the ray of lane cl - 1 to lane cl (DPP
    // row shift), a c-move that of lane - 8 to the lane.  At a move the lane
    // stores its ray if it leaves the tile (Fb / Fc, to the face buffer) or
    // the mesh (Xb / Xc, to its ray-state slot), takes the neighbour lane's
    // ray (Tb / Tc), or loads a ray arriving from the neighbouring tile
    // (Nb / Nc; otherwise a ray entering the mesh, I_bc).
    const int cl = lane & 7, rw = lane >> 3;
    const bool bneg = (oct >> ab) & 1, cneg = (oct >> ac) & 1;
    const int gb = lo_b + (bneg ? 7 - cl : cl), gc = lo_c + (cneg ? 7 - rw : rw);
    const bool in_dom = gb < Nb && gc < Nc;
    const int gbs = bneg ? gb + 1 : gb - 1;               // column a b-move brings a ray from
    const int gcs = cneg ? gc + 1 : gc - 1;
    const bool Xb = in_dom && (bneg ? gb == 0 : gb + 1 >= Nb);   // leaves the mesh
    const bool Fb = in_dom && cl == 7 && !Xb;                      // leaves the tile
    const bool Tb = cl >= 1 && gbs < Nb;
    const bool Nb_ = in_dom && cl == 0 && gbs >= 0 && gbs < Nb;
    const bool Xc = in_dom && (cneg ? gc == 0 : gc + 1 >= Nc);
    const bool Fc = in_dom && rw == 7 && !Xc;
    const bool Tc = rw >= 1 && gcs < Nc;
    const bool Nc_ = in_dom && rw == 0 && gcs >= 0 && gcs < Nc;
    // blocks with lanes on the mesh's exit faces along b and c, and the last
    // block along a (wave-uniform)
    const bool edge_b = bneg ? lo_b == 0 : lo_b + 8 >= Nb;
    const bool edge_c = cneg ? lo_c == 0 : lo_c + 8 >= Nc;
    const bool last_a = d0 + nslab >= Na;
    const int csrc4 = (rw >= 1 ? lane - 8 : lane) << 2;   // ds_bpermute byte address

    // LDS accumulators: per cell of the block, {A1, A2} of every bin; with
    // priv_acc one region per wave (no atomics; the regions are added in wave
    // order at the flush, so the sums do not depend on timing), else one
    // region for the workgroup.
    const int V = depth * 64;                             // cells of one block
    const int region = NB * 2 * V;
    const bool priv = priv_acc != 0 && nwave > 1;
    const int nreg = priv ? nwave : 1;
    float *accl = lds + (priv ? wave * region : 0);
    for (int i = threadIdx.x; i < nreg * region; i += blockDim.x) lds[i] = 0.0f;
    __syncthreads();

    // Field records of the block: base at its lowest cell, lane offset fixed,
    // slab offset in the scalar offset.
    // (x-dominant directions read the y-fastest copy, so that the lanes of a
    // tile row read consecutive cells as for the other two axes)
    const float2 *fbase = cls == 0 ? M.fields_t : M.fields;
    const long long fsa = cls == 0 ? (long long)M.ny * M.nz : sa;
    const long long fsb = cls == 0 ? 1 : sb;
    const long long fsc = cls == 0 ? M.ny : sc;
    const long long base_cell = (long long)lo_a * fsa + (long long)lo_b * fsb + (long long)lo_c * fsc;
    const long long rec_left = (M.ncell - base_cell) * NB * 8;
    const rsrc_t rF = make_rsrc(fbase + base_cell * NB, (unsigned)min(rec_left, 0x7fffffffll));
    const unsigned foff = in_dom ? (unsigned)(((gb - lo_b) * fsb + (gc - lo_c) * fsc) * NB * 8) : 0u;
    auto slab_soff = [&](int t) {     // byte offset of the t-th slab swept
        const int la = sig_neg ? nslab - 1 - t : t;
        return (unsigned)(la * fsa * NB * 8);
    };
    // crossing table: one descriptor over all of it (rows past a direction's
    // last slab are read but never used; past the table they read 0)
    const rsrc_t rG = make_rsrc(M.geo, (unsigned)min((long long)M.geo_rows * 16, 0x7fffffffll));
    c_dir *dirs = (c_dir *)M.dirs;
    c_int *order = (c_int *)M.order;
    const int gstride = M.geo_stride;
    // The bucket's ray states (exit intensities) are one contiguous range
    // (boundary slot of its first direction up to the last ray of its last
    // direction).
    const long long sbase = dirs[order[dbeg]].state_off - NB;
    const c_dir &Dl = dirs[order[dend - 1]];
    const rsrc_t rS = make_rsrc(M.state + sbase,
                                (unsigned)((Dl.state_off + (long long)Dl.nj * Dl.nk * NB - sbase) * 4));
    unsigned int sseg = 0;   // segments of positive length per in-mesh lane (wave-uniform)
    const bool zero_bc = M.I_bc == 0.0f;
    const float Ibc = M.I_bc;

    // Face buffers.  A ray that crosses from this block into a neighbouring
    // one is handed over by block face: per direction of the bucket, b-faces
    // [a-parity][block][slab of the block][lane row], c-faces [a-parity]
    // [block][slab][lane column] and a-faces [block][lane], with blocks
    // numbered b + nbb c; the 8 rays of a move, and the 64 of a tile, are one
    // contiguous run.  The neighbour along b or c reads the entry in the next
    // launch, on the same slab, before the block two steps on along a
    // reuses it; the next block along a reads the a-face.  A ray that leaves
    // the mesh goes to its ray-state slot instead (its exit intensity).
    const unsigned es = NB * 4;                           // bytes of one ray
    const unsigned slab_b = 8 * es;                       // one slab of a block face
    const unsigned fb_sz = 2u * (unsigned)M.face_P * (unsigned)depth * slab_b;
    const unsigned fdir = (unsigned)(M.face_dir_floats * 4);
    const rsrc_t rX = make_rsrc(M.faces + (long long)it_bucket * M.face_bucket_dirs * M.face_dir_floats,
                                fdir * (unsigned)M.face_bucket_dirs);
    const int par = pa & 1;
    const int pb_n = bneg ? pb + 1 : pb - 1, pc_n = cneg ? pc + 1 : pc - 1;   // upstream neighbours
    const unsigned pbc = (unsigned)(pb + nbb * pc);
    const unsigned pbc_b = (unsigned)((pb_n >= 0 && pb_n < nbb ? pb_n : pb) + nbb * pc);
    const unsigned pbc_c = (unsigned)(pb + nbb * (pc_n >= 0 && pc_n < nbc ? pc_n : pc));
    const unsigned fbw = (par * (unsigned)M.face_P + pbc) * (unsigned)depth * slab_b;
    const unsigned fbr = (par * (unsigned)M.face_P + pbc_b) * (unsigned)depth * slab_b;
    const unsigned fcw = fb_sz + (par * (unsigned)M.face_P + pbc) * (unsigned)depth * slab_b;
    const unsigned fcr = fb_sz + (par * (unsigned)M.face_P + pbc_c) * (unsigned)depth * slab_b;
    const unsigned fa = 2u * fb_sz + pbc * 64u * es;
    const unsigned rwo = (unsigned)rw * es, clo = (unsigned)cl * es, lno = (unsigned)lane * es;

    for (int q0 = dbeg + wave; q0 < dend; q0 += nwave * K) {
        bool act[K];
        unsigned gvoff[K];      // byte offset of the direction's first table row
        unsigned dB[K], dC[K];  // state offset change of a b-move, a c-move
        unsigned dirb[K];       // byte offset of the direction's face buffers in rX
        unsigned cur[K];        // byte offset of the lane's current ray in rS
        float invw[K], invwl[K], wdir[K];
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
            gvoff[m] = in_vgpr((unsigned)(d * gstride * 16));
            const unsigned db = (unsigned)((D.state_off - NB - sbase) * 4);
            const int sj = D.kfast ? D.nk : 1, sk = D.kfast ? 1 : D.nj;   // slot strides of j, k
            cur[m] = db + (unsigned)((1 + (gc - Bc - D.k0) * sk + (gb - Bb - D.j0) * sj) * NB * 4);
            dB[m] = in_vgpr((unsigned)((bneg ? -1 : 1) * sj * NB * 4));
            dC[m] = in_vgpr((unsigned)((cneg ? -1 : 1) * sk * NB * 4));
            dirb[m] = (unsigned)((act[m] ? q : q0) - dbeg) * fdir;
            invw[m] = in_vgpr((float)D.invw);
            invwl[m] = in_vgpr((float)(-D.invw * 1.4426950408889634));
            wdir[m] = in_vgpr((float)D.w);
            // rays entering through the top face come from the block above
            // (its a-face entry), or from outside the mesh (I_bc)
            load_slot<NB>(rX, (in_dom && d0 > 0) ? lno : ART_OOB, I[m], dirb[m] + fa);
            if (!zero_bc)
#pragma unroll
                for (int b = 0; b < NB; ++b) I[m][b] = (in_dom && d0 > 0) ? I[m][b] : Ibc;
            gcur[m] = __builtin_amdgcn_raw_buffer_load_b128(rG, gvoff[m], (unsigned)(d0 * 16), 0);
        }
        float kh[NB], Sv[NB];
        load_fields<NB>(rF, foff, slab_soff(0), kh, Sv);

        for (int t = 0; t < nslab; ++t) {
            const int i = d0 + t;
            // next slab's fields (past the last slab: a harmless repeat)
            const unsigned so_next = slab_soff(t + 1 < nslab ? t + 1 : t);
            float khn[NB], Svn[NB];
            load_fields<NB>(rF, foff, so_next, khn, Svn);
            // the table entry is the same in every lane: its code word goes to a
            // scalar register, so that every branch on it is a scalar branch.
            // Code: bits 0-1 first move (0 none, 1 b, 2 c), bits 2-3 second
            // move, bits 5+ segments of positive length.
            unsigned codes[K];
#pragma unroll
            for (int m = 0; m < K; ++m) codes[m] = __builtin_amdgcn_readfirstlane(gcur[m].w);
            // rays entering the tile during this slab
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const unsigned c1 = codes[m] & 3u, c2 = (codes[m] >> 2) & 3u;
                const bool hb = c1 == 1u || c2 == 1u, hc = c1 == 2u || c2 == 2u;
                load_slot<NB>(rX, (hb && Nb_) ? rwo : ART_OOB, ib[m], dirb[m] + fbr + (unsigned)t * slab_b);
                load_slot<NB>(rX, (hc && Nc_) ? clo : ART_OOB, ic[m], dirb[m] + fcr + (unsigned)t * slab_b);
                if (!zero_bc) {     // rays entering the mesh
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        ib[m][b] = Nb_ ? ib[m][b] : Ibc;
                        ic[m][b] = Nc_ ? ic[m][b] : Ibc;
                    }
                }
                gnext[m] = __builtin_amdgcn_raw_buffer_load_b128(rG, gvoff[m], (unsigned)((i + 1) * 16), 0);
            }
            // |n_a| / (kappa h) per direction and bin (1/0 = inf: vacuum takes the
            // small-x branch, which does not use it)
            float rk[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) rk[b] = __builtin_amdgcn_rcpf(kh[b]);
            // |n_a| / (kappa h) and S kappa h / |n_a| per direction and bin
            float skh[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) skh[b] = Sv[b] * kh[b];
            float fw[K][NB], sfw[K][NB];
#pragma unroll
            for (int m = 0; m < K; ++m)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    fw[m][b] = rk[b] * wdir[m];
                    sfw[m][b] = skh[b] * invw[m];
                }
            float a1[NB], a2[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) a1[b] = a2[b] = -0.0f;   // -0 + v = v: the first add folds away

            // a b-move: every ray moves one column; lane cl takes lane cl - 1's ray
            auto cross_b = [&](int m) {
                store_slot<NB>(rX, Fb ? rwo : ART_OOB, I[m], dirb[m] + fbw + (unsigned)t * slab_b);
                if (edge_b) store_slot<NB>(rS, Xb ? cur[m] : ART_OOB, I[m]);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const float moved =
                        __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(I[m][b]), 0x111, 0xF, 0xF, true));
                    I[m][b] = Tb ? moved : ib[m][b];
                }
                cur[m] -= dB[m];
            };
            // a c-move: every ray moves one row; the lane takes lane - 8's ray
            auto cross_c = [&](int m) {
                store_slot<NB>(rX, Fc ? clo : ART_OOB, I[m], dirb[m] + fcw + (unsigned)t * slab_b);
                if (edge_c) store_slot<NB>(rS, Xc ? cur[m] : ART_OOB, I[m]);
                float moved[NB];
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    moved[b] = __int_as_float(__builtin_amdgcn_ds_bpermute(csrc4, __float_as_int(I[m][b])));
#pragma unroll
                for (int b = 0; b < NB; ++b) I[m][b] = Tc ? moved[b] : ic[m][b];
                cur[m] -= dC[m];
            };

            // phase 1: first segment of every direction
#pragma unroll
            for (int m = 0; m < K; ++m) {
                if (!act[m]) continue;
                sseg += codes[m] >> 5;
                segment<NB>(kh, fw[m], sfw[m], invwl[m], __uint_as_float(gcur[m].x), I[m], a1, a2);
            }
            // phase 2: first move of every direction, then its second segment
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const unsigned c1 = codes[m] & 3u;
                if (!act[m] || !c1) continue;
                if (c1 == 1u) cross_b(m); else cross_c(m);
            }
#pragma unroll
            for (int m = 0; m < K; ++m) {
                if (!act[m] || !(codes[m] & 3u)) continue;
                segment<NB>(kh, fw[m], sfw[m], invwl[m], __uint_as_float(gcur[m].y), I[m], a1, a2);
            }
            // phase 3: second move and third segment
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const unsigned c2 = (codes[m] >> 2) & 3u;
                if (!act[m] || !c2) continue;
                if (c2 == 1u) cross_b(m); else cross_c(m);
            }
#pragma unroll
            for (int m = 0; m < K; ++m) {
                if (!act[m] || !((codes[m] >> 2) & 3u)) continue;
                segment<NB>(kh, fw[m], sfw[m], invwl[m], __uint_as_float(gcur[m].z), I[m], a1, a2);
            }

            if (in_dom) {
                const int la = (sig_neg ? Na - 1 - i : i) - lo_a;
                float *cellacc = accl + (la * 64 + lane) * (2 * NB);
                if (nwave == 1 || priv) {
                    // the wave owns its region: plain read-modify-write
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
            for (int b = 0; b < NB; ++b) {
                kh[b] = khn[b];
                Sv[b] = Svn[b];
            }
#pragma unroll
            for (int m = 0; m < K; ++m) gcur[m] = gnext[m];
        }
        // rays leave through the block's far face: into the next block's
        // a-face entry, or out of the mesh into their ray-state slots
#pragma unroll
        for (int m = 0; m < K; ++m) {
            if (last_a)
                store_slot<NB>(rS, (act[m] && in_dom) ? cur[m] : ART_OOB, I[m]);
            else
                store_slot<NB>(rX, (act[m] && in_dom) ? lno : ART_OOB, I[m], dirb[m] + fa);
        }
    }

    // workgroup total of marched segments of positive length (work accounting)
    const unsigned int nseg = sseg * (unsigned)__popcll(__ballot(in_dom));
    unsigned int *wg_count = reinterpret_cast<unsigned int *>(lds + nreg * region);
    if (threadIdx.x == 0) *wg_count = 0u;
    __syncthreads();
    if (lane == 0) atomicAdd(wg_count, nseg);
    __syncthreads();
    if (threadIdx.x == 0) seg_count[blockIdx.x] = *wg_count;

    // Flush: this workgroup is the only writer of its block in this bucket's
    // copy.  The stores follow the copy's x-fastest order: for dominant axis y
    // or z a tile row runs along x, and four of its cells go out as one
    // 16-byte store where the copy is 16-byte aligned; for dominant axis x the
    // slabs of a column run along x, so consecutive threads take consecutive
    // slabs.  (Component-fastest or tile-row-fastest orders scatter each store
    // instruction over 8 or 64 cache lines and made the march 7-9% slower.)
    auto accv = [&](int x) {     // a block cell's sum over the regions
        float v = lds[x];
        for (int w = 1; w < nreg; ++w) v += lds[w * region + x];
        return v;
    };
    g_f *dst = (g_f *)M.acc + (long long)it_bucket * NB * 2 * M.ncell;
    if (cls != 0 && (M.ncell & 3) == 0 && (M.nx & 3) == 0) {
        const int ng = nslab * 16;                // groups of four cells per component
        for (int idx = threadIdx.x; idx < NB * 2 * ng; idx += blockDim.x) {
            const int comp = idx / ng, q = idx % ng;
            const int la = q >> 4, rw = (q >> 1) & 7, half = q & 1;
            const int cc = lo_c + rw;             // the tile row's c index
            if (cc >= Nc) continue;
            const int cb0 = lo_b + 4 * half;      // its first cell along b = x
            const int rwl = cneg ? 7 - rw : rw;   // the lane row holding it
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int cbk = 4 * half + k;
                v[k] = accv((la * 64 + rwl * 8 + (bneg ? 7 - cbk : cbk)) * (2 * NB) + comp);
            }
            const long long wc = (lo_a + la) * sa + (long long)cb0 * sb + (long long)cc * sc;
            if (cb0 + 3 < Nb) {
                *(g_f32x4 *)&dst[comp * M.ncell + wc] = f32x4{v[0], v[1], v[2], v[3]};
            } else {
                for (int k = 0; k < 4; ++k)
                    if (cb0 + k < Nb) dst[comp * M.ncell + wc + k] = v[k];
            }
        }
    } else if (cls == 0) {
        const int nq = nslab * 64;
        for (int idx = threadIdx.x; idx < NB * 2 * nq; idx += blockDim.x) {
            const int comp = idx / nq, q = idx % nq;
            const int l = q / nslab, la = q % nslab;
            const int cb = lo_b + (bneg ? 7 - (l & 7) : (l & 7));
            const int cc = lo_c + (cneg ? 7 - (l >> 3) : (l >> 3));
            if (cb >= Nb || cc >= Nc) continue;
            const long long wc = (lo_a + la) * sa + cb * sb + cc * sc;
            dst[comp * M.ncell + wc] = accv((la * 64 + l) * (2 * NB) + comp);
        }
    } else {
        for (int idx = threadIdx.x; idx < NB * 2 * V; idx += blockDim.x) {
            const int comp = idx / V, cell = idx % V;
            const int la = cell >> 6, l = cell & 63;
            const int cb = lo_b + (bneg ? 7 - (l & 7) : (l & 7));
            const int cc = lo_c + (cneg ? 7 - (l >> 3) : (l >> 3));
            if (la >= nslab || cb >= Nb || cc >= Nc) continue;
            const long long wc = (lo_a + la) * sa + cb * sb + cc * sc;
            dst[comp * M.ncell + wc] = accv(cell * (2 * NB) + comp);
        }
    }
}

}  // namespace

int art_march_max_lds_bytes() { return 160 * 1024; }

// LDS floats of one workgroup: accumulators of depth * 64 cells (one region,
// or one per wave with private accumulators) plus a counter.
int art_march_lds_floats(int depth, int nb, int regions) { return regions * nb * 2 * depth * 64 + 32; }


template <int NB, int K>
hipError_t launch_nbk(const ArtItem *items, int nitems, const ArtMeshDesc *meshes, size_t bytes,
                      int threads, unsigned int *seg_count, int priv, hipStream_t stream)
{
    // Up to 64 KiB of local memory needs no opt-in; beyond, one opt-in to the
    // whole of it, made once (a function-local static: thread-safe).
    static const hipError_t cfg = hipFuncSetAttribute((const void *)art_march_kernel<NB, K>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      art_march_max_lds_bytes());
    if (bytes > 64 * 1024 && cfg != hipSuccess) return cfg;
    if (nitems <= 0) return hipSuccess;   // a call without items only configures the kernel
    hipLaunchKernelGGL((art_march_kernel<NB, K>), dim3(nitems), dim3(threads), bytes, stream, items,
                       meshes, seg_count, priv);
    return hipGetLastError();
}

template <int NB>
hipError_t launch_nb(const ArtItem *items, int nitems, const ArtMeshDesc *meshes, int K, size_t bytes,
                     int threads, unsigned int *seg_count, int priv, hipStream_t stream)
{
    switch (K) {
    case 1: return launch_nbk<NB, 1>(items, nitems, meshes, bytes, threads, seg_count, priv, stream);
    case 2: return launch_nbk<NB, 2>(items, nitems, meshes, bytes, threads, seg_count, priv, stream);
    case 4: return launch_nbk<NB, 4>(items, nitems, meshes, bytes, threads, seg_count, priv, stream);
    case 3: return launch_nbk<NB, 3>(items, nitems, meshes, bytes, threads, seg_count, priv, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t art_launch_march(const ArtItem *items, int nitems, const ArtMeshDesc *meshes, int nb,
                            int interleave, int lds_floats, int threads, unsigned int *seg_count,
                            hipStream_t stream, int priv)
{
    const size_t bytes = (size_t)lds_floats * sizeof(float);
    switch (nb) {
    case 1: return launch_nb<1>(items, nitems, meshes, interleave, bytes, threads, seg_count, priv, stream);
    case 2: return launch_nb<2>(items, nitems, meshes, interleave, bytes, threads, seg_count, priv, stream);
    case 3: return launch_nb<3>(items, nitems, meshes, interleave, bytes, threads, seg_count, priv, stream);
    case 4: return launch_nb<4>(items, nitems, meshes, interleave, bytes, threads, seg_count, priv, stream);
    default: return hipErrorInvalidValue;
    }
}
