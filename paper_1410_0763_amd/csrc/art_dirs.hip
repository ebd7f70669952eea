// art_dirs.hip -- direction set and ray-lattice generator.
//
// Directions are the centres of the 12 Nside^2 HEALPix pixels in RING order
// (Sect. 2.3; Gorski et al. 2005): rings i = 1 .. 4N-1 from north to south;
// polar-cap rings (i < N) hold 4i pixels at z = 1 - i^2/(3N^2), phi =
// pi/(2i) (j - 1/2); belt rings (N <= i <= 3N) hold 4N pixels at
// z = 4/3 - 2i/(3N), phi = pi/(2N) (j - s/2), s = (i - N + 1) mod 2 (pixels of
// rings with s = 0 numbered from phi = 0); the south cap mirrors the north.
//
// For each direction the generator fixes the parallel-ray lattice of Sect. 2.2
// (rays at the half-integer points of the upstream face of the dominant axis,
// unit spacing; ties of the dominant axis go to the lowest axis index within
// 1e-12; components below 1e-12 are zero), the octant of travel, the workgroup
// bucket (dominant axis x octant x subset) and the offset of its rays in the
// state buffer.
//
// One workgroup: every thread builds directions; wave 0 then assigns buckets
// and offsets with wave-wide prefix sums, so the result is deterministic.
#include <algorithm>
#include <cmath>

#include "art_internal.h"

#define ART_TIE 1e-12

namespace {

__host__ __device__ void healpix_ring(int nside, int d, double *n)
{
    const double N = (double)nside;
    const double PI = 3.14159265358979323846;
    int i = 1, start = 0;
    // walk the rings until the one holding pixel d
    for (;; ++i) {
        int npix = (i < nside) ? 4 * i : (i <= 3 * nside ? 4 * nside : 4 * (4 * nside - i));
        if (d < start + npix) break;
        start += npix;
    }
    const int j = d - start + 1;   // 1-based position in the ring
    double z, phi;
    if (i < nside) {
        z = 1.0 - (double)i * i / (3.0 * N * N);
        phi = PI / (2.0 * i) * (j - 0.5);
    } else if (i <= 3 * nside) {
        z = 4.0 / 3.0 - 2.0 * i / (3.0 * N);
        const int s = (i - nside + 1) % 2;
        phi = PI / (2.0 * N) * (s ? (j - 0.5) : (double)(j - 1));
    } else {
        const int ip = 4 * nside - i;
        z = -(1.0 - (double)ip * ip / (3.0 * N * N));
        phi = PI / (2.0 * ip) * (j - 0.5);
    }
    const double st = sqrt((1.0 - z) * (1.0 + z));
    n[0] = st * cos(phi);
    n[1] = st * sin(phi);
    n[2] = z;
    for (int q = 0; q < 3; ++q)
        if (fabs(n[q]) < ART_TIE) n[q] = 0.0;
}

__device__ void build_dir(int nside, int d, int nx, int ny, int nz, ArtDir *out)
{
    double n[3];
    healpix_ring(nside, d, n);
    const int N[3] = {nx, ny, nz};
    const double m = fmax(fabs(n[0]), fmax(fabs(n[1]), fabs(n[2])));
    const int a = fabs(n[0]) >= m - ART_TIE ? 0 : (fabs(n[1]) >= m - ART_TIE ? 1 : 2);
    const int b = (a == 0) ? 1 : 0;
    const int c = (a == 2) ? 1 : 2;
    const double w = fabs(n[a]);
    ArtDir D;
    D.n[0] = n[0]; D.n[1] = n[1]; D.n[2] = n[2];
    D.a = a; D.b = b; D.c = c;
    D.w = w;
    D.invw = 1.0 / w;
    const double sig = n[a] > 0.0 ? 1.0 : -1.0;
    D.alpha_a = sig > 0.0 ? 0.0 : (double)N[a];
    const double tb = n[b] / w, tc = n[c] / w;
    for (int q = 0; q < 3; ++q) {
        const double bq = (q == a) ? sig : (q == b ? tb : tc);
        D.beta[q] = bq;
        D.rbeta[q] = bq != 0.0 ? 1.0 / bq : 0.0;
    }
    D.octant = (D.beta[0] < 0.0 ? 1 : 0) | (D.beta[1] < 0.0 ? 2 : 0) | (D.beta[2] < 0.0 ? 4 : 0);
    // lattice: x_b = j + 1/2 + tb s must meet (0, N_b) for some s in [0, N_a]
    const double Na = (double)N[a];
    const int jlo = (int)floor(-0.5 - fmax(0.0, tb * Na));
    const int jhi = (int)ceil((double)N[b] - 0.5 - fmin(0.0, tb * Na));
    const int klo = (int)floor(-0.5 - fmax(0.0, tc * Na));
    const int khi = (int)ceil((double)N[c] - 0.5 - fmin(0.0, tc * Na));
    D.j0 = jlo; D.nj = jhi - jlo + 1;
    D.k0 = klo; D.nk = khi - klo + 1;
    // slot order: the lattice index that changes at the more frequent plane
    // crossing runs fastest, so that the rays a tile hands over at that
    // crossing (a tile edge along the other index) sit in consecutive slots
    D.kfast = fabs(tb) > fabs(tc) ? 1 : 0;
    D.state_off = 0;
    D.bucket = -1;
    D.pad = 0;
    *out = D;
}

__global__ __launch_bounds__(256) void art_dirs_kernel(int nside, int nx, int ny, int nz, int nb,
                                                       int d_begin, int d_end, int subsets,
                                                       ArtDir *__restrict__ dirs,
                                                       int *__restrict__ order,
                                                       int *__restrict__ bucket_start)
{
    const int nd = 12 * nside * nside;
    for (int d = threadIdx.x; d < nd; d += blockDim.x) build_dir(nside, d, nx, ny, nz, dirs + d);
    __syncthreads();
    if (threadIdx.x >= 64) return;

    // Wave 0: rank of each in-range direction within its group g = a * 8 +
    // octant (ballot prefix counts in index order), bucket = g * subsets +
    // rank % subsets, and the bucket-major order of the directions.
    const int lane = threadIdx.x;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int oct_count[24];
#pragma unroll
    for (int g = 0; g < 24; ++g) oct_count[g] = 0;
    for (int base = 0; base < nd; base += 64) {
        const int d = base + lane;
        const bool valid = d < nd && d >= d_begin && d < d_end;
        const int oct = (d < nd) ? dirs[d].a * 8 + dirs[d].octant : -1;
        int rank = 0;
#pragma unroll
        for (int o = 0; o < 24; ++o) {
            const unsigned long long msk = __ballot(valid && oct == o);
            if (valid && oct == o) rank = oct_count[o] + __popcll(msk & below);
            oct_count[o] += __popcll(msk);
        }
        if (d < nd) {
            dirs[d].bucket = valid ? oct * subsets + rank % subsets : -1;
            dirs[d].pad = valid ? rank / subsets : 0;   // position inside the bucket
        }
    }
    // Bucket sizes follow from the octant counts (identical in every lane),
    // so each lane derives the bucket offsets itself.
    auto bucket_size = [&](int bk) {
        const int o = bk / subsets, s = bk % subsets;
        return (oct_count[o] > s) ? (oct_count[o] - s + subsets - 1) / subsets : 0;
    };
    if (lane == 0) {
        int acc = 0;
        for (int bk = 0; bk < 24 * subsets; ++bk) {
            bucket_start[bk] = acc;
            acc += bucket_size(bk);
        }
        bucket_start[24 * subsets] = acc;
    }
    for (int d = lane; d < nd; d += 64) {
        const int bk = dirs[d].bucket;   // written by this lane above
        if (bk < 0) continue;
        int start = 0;
        for (int q = 0; q < bk; ++q) start += bucket_size(q);
        order[start + dirs[d].pad] = d;
    }
}


// State-buffer offsets in bucket-major order (prefix sums of nj nk nb over
// `order`), so that the directions of one bucket occupy one contiguous range.
// Each direction's region starts with a boundary slot holding I_bc: the march
// reads it for every ray that enters the mesh through a face.  One wave.
__global__ __launch_bounds__(64) void art_state_kernel(int nb, const int *__restrict__ bucket_start,
                                                       int nbuckets, const int *__restrict__ order,
                                                       ArtDir *__restrict__ dirs,
                                                       float *__restrict__ state, float I_bc)
{
    const int lane = threadIdx.x;
    const int n = bucket_start[nbuckets];
    long long off_base = 0;
    for (int base = 0; base < n; base += 64) {
        const int p = base + lane;
        const int d = p < n ? order[p] : -1;
        const long long mine = d >= 0 ? (long long)dirs[d].nj * dirs[d].nk * nb + nb : 0;
        long long incl = mine;
        for (int sh = 1; sh < 64; sh <<= 1) {
            const long long t = __shfl_up(incl, sh, 64);
            if (lane >= sh) incl += t;
        }
        if (d >= 0) {
            const long long first = off_base + incl - mine;
            dirs[d].state_off = first + nb;
            for (int b = 0; b < nb; ++b) state[first + b] = I_bc;
        }
        off_base += __shfl(incl, 63, 64);
    }
}

// Per-(direction, slab) crossing table used by the march.  For slab i of the
// depth axis the transverse lattice shift B(i) = floor(1/2 + t i) of every ray
// changes by sh = B(i+1) - B(i) in {-1, 0, 1}, at depth fraction
// f = (X - (1/2 + t i)) / t (X the plane crossed), per transverse axis.  The
// entry holds the lengths of the slab's (up to three) segments in crossing
// order and a code: bits 0-1 sh_b + 1, bits 2-3 sh_c + 1, bit 4 "b-plane
// crossed first", bits 5-6 number of segments of positive length.
__global__ __launch_bounds__(256) void art_geo_kernel(const ArtDir *__restrict__ dirs, int nx, int ny,
                                                      int nz, int stride, uint4 *__restrict__ geo)
{
    const int d = blockIdx.x;
    const ArtDir &D = dirs[d];
    if (D.bucket < 0) return;
    const int N[3] = {nx, ny, nz};
    const int Na = N[D.a];
    const double tb = D.beta[D.b], tc = D.beta[D.c];
    const double rtb = D.rbeta[D.b], rtc = D.rbeta[D.c];
    for (int i = threadIdx.x; i < Na; i += blockDim.x) {
        const double xb0 = fma(tb, (double)i, 0.5), xb1 = fma(tb, (double)(i + 1), 0.5);
        const double xc0 = fma(tc, (double)i, 0.5), xc1 = fma(tc, (double)(i + 1), 0.5);
        const int Bb = (int)floor(xb0), Bc = (int)floor(xc0);
        const int shb = max(-1, min(1, (int)floor(xb1) - Bb));
        const int shc = max(-1, min(1, (int)floor(xc1) - Bc));
        double fb = 2.0, fc = 2.0;
        if (shb) fb = fmin(1.0, fmax(0.0, ((double)(shb > 0 ? Bb + 1 : Bb) - xb0) * rtb));
        if (shc) fc = fmin(1.0, fmax(0.0, ((double)(shc > 0 ? Bc + 1 : Bc) - xc0) * rtc));
        const bool b_first = fb <= fc;
        // lengths differenced in double, then rounded: each carries a relative
        // error of one float rounding, also a sliver next to a crossing (a
        // float difference of rounded depths would carry an absolute 2^-24,
        // which a bright ray crossing the sliver turns into a large relative
        // error of the cell's sums)
        float s1, s2, s3;
        if (shb && shc) {
            const double f1 = fmin(fb, fc), f2 = fmax(fb, fc);
            s1 = (float)f1; s2 = (float)(f2 - f1); s3 = (float)(1.0 - f2);
        } else if (shb || shc) {
            const double f1 = shb ? fb : fc;
            s1 = (float)f1; s2 = (float)(1.0 - f1); s3 = 0.0f;
        } else {
            s1 = 1.0f; s2 = 0.0f; s3 = 0.0f;
        }
        // crossings within 1e-12 of each other or of the slab face are one
        // point in exact arithmetic (a ray through a cell edge): the sliver
        // between them is a contact of zero length, as in the oracle
        if (s1 < 1e-12f) s1 = 0.0f;
        if (s2 < 1e-12f) s2 = 0.0f;
        if (s3 < 1e-12f) s3 = 0.0f;
        const unsigned npos = (s1 > 0.f) + (s2 > 0.f) + (s3 > 0.f);
        // moves in slab order: 0 none, 1 a b-plane, 2 a c-plane
        const unsigned mv1 = shb && (b_first || !shc) ? 1u : (shc ? 2u : 0u);
        const unsigned mv2 = shb && shc ? (b_first ? 2u : 1u) : 0u;
        const unsigned code = mv1 | (mv2 << 2) | (npos << 5);
        geo[(long long)d * stride + i] =
            make_uint4(__float_as_uint(s1), __float_as_uint(s2), __float_as_uint(s3), code);
    }
}

}  // namespace

hipError_t art_launch_dirs(int nside, int nx, int ny, int nz, int nb, int d_begin, int d_end,
                           int subsets, ArtDir *dirs, int *order, int *bucket_start, uint4 *geo,
                           int geo_stride, float *state, float I_bc, hipStream_t stream)
{
    hipLaunchKernelGGL(art_dirs_kernel, dim3(1), dim3(256), 0, stream, nside, nx, ny, nz, nb,
                       d_begin, d_end, subsets, dirs, order, bucket_start);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(art_state_kernel, dim3(1), dim3(64), 0, stream, nb, bucket_start,
                       24 * subsets, order, dirs, state, I_bc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(art_geo_kernel, dim3(12 * nside * nside), dim3(256), 0, stream, dirs, nx, ny,
                       nz, geo_stride, geo);
    return hipGetLastError();
}

// Largest number of directions in one bucket for this direction set (the
// same classification as the generator, on the host).
int art_max_bucket_dirs(int nside, int subsets)
{
    int cnt[24] = {0};
    const int nd = 12 * nside * nside;
    for (int d = 0; d < nd; ++d) {
        double n[3];
        healpix_ring(nside, d, n);
        const double m = fmax(fabs(n[0]), fmax(fabs(n[1]), fabs(n[2])));
        const int a = fabs(n[0]) >= m - ART_TIE ? 0 : (fabs(n[1]) >= m - ART_TIE ? 1 : 2);
        const int oct = (n[0] < 0.0 ? 1 : 0) | (n[1] < 0.0 ? 2 : 0) | (n[2] < 0.0 ? 4 : 0);
        ++cnt[a * 8 + oct];
    }
    int worst = 0;
    for (int g = 0; g < 24; ++g) worst = std::max(worst, (cnt[g] + subsets - 1) / subsets);
    return worst;
}
