// art_internal.h -- data structures shared by the HIP kernels and the host
// side of libart.  Not part of the public interface (include/art.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

typedef struct art_mesh art_mesh;

// One direction of the HEALPix set with its parallel-ray lattice (Sect. 2.2,
// 2.3).  Ray (j,k) is the line x_i(s) = alpha_i + beta_i s over depth s in
// [0, N_a]: along the dominant axis a, alpha_a is the upstream face (0 or N_a)
// and beta_a = +-1; along the transverse axes b < c, alpha = j + 1/2 (or
// k + 1/2) and beta = n_b/|n_a| (n_c/|n_a|).  World axes are x = 0, y = 1, z = 2.
struct ArtDir {
    double n[3];          // unit direction
    double alpha_a;       // x_a at depth 0
    double beta[3];       // dx_i/ds per world axis
    double rbeta[3];      // 1/beta_i (0 where beta_i = 0)
    double w;             // |n_a|: one unit of depth is a path of 1/w cells
    double invw;          // 1/|n_a|
    int a, b, c;          // dominant axis, then the other two (b < c)
    int octant;           // bit i set: the rays travel towards decreasing x_i
    int j0, nj, k0, nk;   // lattice index ranges [j0, j0+nj) x [k0, k0+nk)
    long long state_off;  // first float of this direction's ray states
    int bucket;           // (a * 8 + octant) * subsets + subset; -1 outside the range
    int pad;
    int kfast;            // ray slots ordered k fastest (else j fastest)
    int pad2;
};

// Everything one workgroup of the march needs about its mesh.
struct ArtMeshDesc {
    const float2 *fields;      // [cell][nb] = {kappa h, S}, cells x fastest
    const float2 *fields_t;    // the same with y fastest, then z, then x
    float *state;              // ray intensities where rays leave the mesh
    float *faces;              // rays handed from block to block (block-face buffers)
    long long face_dir_floats; // face-buffer floats per direction
    int face_bucket_dirs;      // directions per bucket the face buffers hold
    int face_P;                // blocks of the largest cross-section (b x c)
    float *acc;                // [bucket][nb][2][cell] per-bucket direction sums
    const ArtDir *dirs;        // [N_d]
    const int *order;          // direction indices grouped by bucket
    const int *bucket_start;   // [nbuckets + 1]
    const uint4 *geo;          // [N_d][geo_stride] slab crossing table
    long long ncell;
    int geo_stride;            // max(nx, ny, nz)
    long long geo_rows;        // rows allocated for the crossing table (>= N_d * geo_stride)
    int interleave;            // directions marched together by one wave (1..4)
    int nx, ny, nz, nb;
    int depth;                 // block cells along the dominant axis
    int subsets;               // buckets per (dominant axis, octant) group
    float I_bc;
    int nbuckets;              // 24 * subsets
};

// Work item of one wavefront launch: (mesh, block, bucket).
struct ArtItem {
    int mesh;
    int block;                 // linear block index (x fastest)
    int bucket;
    int pad;
};

#define ART_CHECK_LAUNCH() (hipGetLastError())

// Kernel launchers (defined in the .hip files).
hipError_t art_launch_dirs(int nside, int nx, int ny, int nz, int nb, int d_begin, int d_end,
                           int subsets, ArtDir *dirs, int *order, int *bucket_start, uint4 *geo,
                           int geo_stride, float *state, float I_bc, hipStream_t stream);
// priv != 0 with more than one wave per workgroup: each wave accumulates in
// its own local-memory region (lds_floats must cover threads / 64 regions).
hipError_t art_launch_march(const ArtItem *items, int nitems, const ArtMeshDesc *meshes, int nb,
                            int interleave, int lds_floats, int threads, unsigned int *seg_count,
                            hipStream_t stream, int priv = 0);
hipError_t art_launch_check(const float *kappa, const float *S, long long n, int *bad_flag,
                            hipStream_t stream);
hipError_t art_launch_layout(const float *kappa, const float *S, int nx, int ny, int nz, int nb,
                             double h, float2 *fields, float2 *fields_t, hipStream_t stream);
hipError_t art_launch_normalize(const float *acc, const int *bucket_start, int nbuckets,
                                const float2 *fields, long long ncell, int nb, int nd,
                                const float *gw4, const float *hw8, float *J_in, float *J,
                                float *J_exact, float *Gamma, float *Heat, float *A1raw,
                                float *A2raw, hipStream_t stream);
// Heating weights of a mesh (art_set_heating): hin[4] then hsrc[4].
void art_mesh_heating(const art_mesh *mesh, float hw8[8]);
hipError_t art_launch_exit_sum(const ArtDir *dirs, int nd, const float *state, int nx, int ny,
                               int nz, int nb, float I_bc, float *exit_sum, hipStream_t stream);
hipError_t art_launch_fill(float *p, long long n, float v, hipStream_t stream);
int art_max_bucket_dirs(int nside, int subsets);
// Sets the thread-local error text returned by art_last_error; returns code.
int art_set_error(int code, const char *msg);
int art_march_max_lds_bytes();
int art_march_lds_floats(int depth, int nb, int regions = 1);
// Shape, bins, cell size and device field records ([cell][nb] {kappa h,
// 1/(kappa h), S, 0}; NULL before art_set_fields) of a mesh.
void art_mesh_fields(const art_mesh *mesh, int dims[3], int *nb, double *h, const float2 **fields);
// kappa h of every cell without S, ks floats per cell (ks = 1, 2 or 4 for 1,
// 2 or 3-4 bins; padding 0), built on first use after art_set_fields and
// kept until the next one.  ART_E_STATE without fields.
int art_mesh_kpack(art_mesh *mesh, hipStream_t stream, const float **kpack, int *ks);
hipError_t art_launch_kpack(const float2 *fields, long long ncell, int nb, int ks, float *kpack,
                            hipStream_t stream);

// float -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t art_bf16_rne(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Raw surrogate feature k of a value: the logarithm (floored at 1e-30) for
// k = 0 (J of the coarse sweep) and k = 1 (density), the value itself for
// k = 2 (neutral fraction, in [0, 1]).
__device__ __forceinline__ float art_feature_raw(int k, float v)
{
    return k < 2 ? logf(fmaxf(v, 1e-30f)) : v;
}

// Input record of the surrogate network for one cell, 16 bf16 channels:
// channel k < 3 is (raw feature k - mu[k]) * isd[k] for (J, n, x_HI), the
// other 13 are 0.
__device__ __forceinline__ void art_feature_store(float J, float n, float xhi, const float *mu,
                                                  const float *isd, uint16_t *x16)
{
    const float f[3] = {J, n, xhi};
    uint16_t h[3];
    for (int k = 0; k < 3; ++k) h[k] = art_bf16_rne((art_feature_raw(k, f[k]) - mu[k]) * isd[k]);
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    u4 *dst = reinterpret_cast<u4 *>(x16);
    dst[0] = u4{(unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2], 0u, 0u};
    dst[1] = u4{0u, 0u, 0u, 0u};
}
