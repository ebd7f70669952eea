// art_point.hip -- rates from point radiation sources (Sect. 2.3; the
// photon-conserving form of Appendix A).  Entry point: include/art_point.h.
//
// One thread per target cell, a workgroup per 8 x 8 x 4 brick of cells, so
// that the lines of a wave towards one source run side by side through the
// same cells and their kappa reads share cache lines.  Per (source, cell) the
// thread intersects the line from the source through the cell's centre with
// the cell (slab method: r_in, r_out) and marches the line from the source to
// r_in with a three-axis cell walk: at each step the nearest of the three
// next plane crossings ends the current cell's segment; tau_b += (kappa h)_b
// dl.  Geometry and optical depths are double precision.  The walk reads a
// pack of kappa h alone (16 bytes per cell for 3-4 bins, one load per step),
// which the mesh builds from its {kappa h, S} records on first use after
// art_set_fields: half the cache lines and a quarter of the load instructions
// of reading the records bin by bin.  Sources arrive 64 per
// launch as kernel arguments; the first launch writes the outputs, later ones
// add to them.  The pack is read through a buffer descriptor with 32-bit
// byte offsets (a cell index outside the mesh reads 0 and never touches
// memory), and the walk takes exactly the |dx| + |dy| + |dz| cell moves
// between the source's cell and the target.
#include <cmath>
#include <string>

#include "../../include/art.h"
#include "../../include/art_point.h"
#include "art_internal.h"

namespace {

constexpr int PT_CHUNK = 64;
constexpr int PT_UNROLL = 4;   // walk steps whose loads are issued together

struct PtSource {
    double p[3];
    double Q[4];
};

// Kernel argument block (3624 bytes, below the 4 KiB argument limit).
struct PtChunk {
    PtSource s[PT_CHUNK];
    double e[4];
    int n;
    int has_e;
};

typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// One step of the cell walk: the segment from t to the nearest plane
// crossing (its cell and its length), then the move to the next cell across
// that plane (ties: x, y, z).  The next crossing of the axis crossed is
// t_n + 1 * dt and of the others t_n + 0 * dt, one multiply-add each with
// the same value as the sum or t_n itself (dt is finite: a direction
// without a component along an axis has t_n = inf and dt = 1e300 there).
__device__ __forceinline__ void walk_step(double &tnx, double &tny, double &tnz, double &t, int &cell,
                                          int dcx, int dcy, int dcz, double dtx, double dty,
                                          double dtz, int &cl, double &dl)
{
    const double tmin = fmin(tnx, fmin(tny, tnz));
    dl = tmin - t;
    cl = cell;
    t = tmin;
    const bool mx = tnx == tmin;
    const bool my = !mx && tny == tmin;
    cell += mx ? dcx : (my ? dcy : dcz);
    tnx = fma(mx ? 1.0 : 0.0, dtx, tnx);
    tny = fma(my ? 1.0 : 0.0, dty, tny);
    tnz = fma((!mx && !my) ? 1.0 : 0.0, dtz, tnz);
}

// kappa h of the NB bins of one cell from the pack (KS floats per cell);
// an index outside the pack reads 0.
template <int NB, int KS>
__device__ __forceinline__ void load_kh(rsrc_t kp, int cell, float *kh)
{
    const unsigned off = (unsigned)cell * (unsigned)(KS * 4);
    if constexpr (KS == 4) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(kp, off, 0, 0);
        const float a[4] = {__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                            __uint_as_float(v.w)};
#pragma unroll
        for (int b = 0; b < NB; ++b) kh[b] = a[b];
    } else if constexpr (KS == 2) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(kp, off, 0, 0);
        kh[0] = __uint_as_float(v.x);
        if constexpr (NB > 1) kh[1] = __uint_as_float(v.y);
    } else {
        kh[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(kp, off, 0, 0));
    }
}

template <int NB, int KS>
__global__ __launch_bounds__(256) void art_point_kernel(const float *__restrict__ kpack,
                                                        const float *__restrict__ n_abs, int nx,
                                                        int ny, int nz, double h, PtChunk src,
                                                        int first, float *__restrict__ Gamma,
                                                        float *__restrict__ Heat,
                                                        unsigned *__restrict__ segs)
{
    const int bx = (nx + 7) >> 3, by = (ny + 7) >> 3;
    int blk = blockIdx.x;
    const int gx = blk % bx;
    blk /= bx;
    const int gy = blk % by, gz = blk / by;
    const int cx = gx * 8 + (threadIdx.x & 7);
    const int cy = gy * 8 + ((threadIdx.x >> 3) & 7);
    const int cz = gz * 4 + (threadIdx.x >> 6);
    if (cx >= nx || cy >= ny || cz >= nz) return;
    const int cid = (cz * ny + cy) * nx + cx;
    const double na = (double)n_abs[cid];
    // the pack, KS floats per cell (below 2^31 bytes: checked by the host)
    const rsrc_t kp = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(kpack), (short)0,
                                                        (int)((unsigned)(nx * ny * nz) * (unsigned)(KS * 4)),
                                                        0x00020000);
    const double vol_c = (4.0 * M_PI / 3.0) * h * h * h;
    double g = 0.0, ht = 0.0;
    unsigned nseg = 0;

    for (int s = 0; s < src.n; ++s) {
        const double px = src.s[s].p[0], py = src.s[s].p[1], pz = src.s[s].p[2];
        double ux = cx + 0.5 - px, uy = cy + 0.5 - py, uz = cz + 0.5 - pz;
        const double dist = sqrt(ux * ux + uy * uy + uz * uz);
        if (dist > 0.0) {
            const double r = 1.0 / dist;
            ux *= r; uy *= r; uz *= r;
        } else {
            ux = 1.0; uy = 0.0; uz = 0.0;
        }
        // where the line enters and leaves the target cell (slab method)
        double tin = -INFINITY, tout = INFINITY;
        const double ix_ = ux != 0.0 ? 1.0 / ux : 0.0;
        const double iy_ = uy != 0.0 ? 1.0 / uy : 0.0;
        const double iz_ = uz != 0.0 ? 1.0 / uz : 0.0;
        if (ux != 0.0) {
            const double t0 = (cx - px) * ix_, t1 = (cx + 1.0 - px) * ix_;
            tin = fmax(tin, fmin(t0, t1));
            tout = fmin(tout, fmax(t0, t1));
        }
        if (uy != 0.0) {
            const double t0 = (cy - py) * iy_, t1 = (cy + 1.0 - py) * iy_;
            tin = fmax(tin, fmin(t0, t1));
            tout = fmin(tout, fmax(t0, t1));
        }
        if (uz != 0.0) {
            const double t0 = (cz - pz) * iz_, t1 = (cz + 1.0 - pz) * iz_;
            tin = fmax(tin, fmin(t0, t1));
            tout = fmin(tout, fmax(t0, t1));
        }
        tin = fmax(tin, 0.0);

        // cell walk from the source to r_in
        const int ix = min(max((int)floor(px), 0), nx - 1);
        const int iy = min(max((int)floor(py), 0), ny - 1);
        const int iz = min(max((int)floor(pz), 0), nz - 1);
        int cell = (iz * ny + iy) * nx + ix;
        const int dcx = ux > 0.0 ? 1 : -1, dcy = uy > 0.0 ? nx : -nx;
        const int dcz = uz > 0.0 ? nx * ny : -(nx * ny);
        double tnx = ux > 0.0 ? (ix + 1.0 - px) * ix_ : (ux < 0.0 ? (ix - px) * ix_ : INFINITY);
        double tny = uy > 0.0 ? (iy + 1.0 - py) * iy_ : (uy < 0.0 ? (iy - py) * iy_ : INFINITY);
        double tnz = uz > 0.0 ? (iz + 1.0 - pz) * iz_ : (uz < 0.0 ? (iz - pz) * iz_ : INFINITY);
        const double dtx = fmin(fabs(ix_), 1e300), dty = fmin(fabs(iy_), 1e300), dtz = fmin(fabs(iz_), 1e300);
        double tau[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) tau[b] = 0.0;
        // The walk moves one axis at a time and never back, so it enters the
        // target after exactly nmove = |dix| + |diy| + |diz| moves; segment k
        // runs from the (k-1)-th to the k-th crossing, the last crossing being
        // r_in.  Groups of four steps of geometry, then their four loads, then
        // their sums, so that four loads are in flight per lane; the last
        // nmove mod 4 steps one by one.
        const int nmove = abs(cx - ix) + abs(cy - iy) + abs(cz - iz);
        double t = 0.0;
        int k = 0;
        for (; k + PT_UNROLL <= nmove; k += PT_UNROLL) {
            int cl[PT_UNROLL];
            double dl[PT_UNROLL];
#pragma unroll
            for (int u = 0; u < PT_UNROLL; ++u)
                walk_step(tnx, tny, tnz, t, cell, dcx, dcy, dcz, dtx, dty, dtz, cl[u], dl[u]);
            float kh[PT_UNROLL][NB];
#pragma unroll
            for (int u = 0; u < PT_UNROLL; ++u) load_kh<NB, KS>(kp, cl[u], kh[u]);
#pragma unroll
            for (int u = 0; u < PT_UNROLL; ++u)
#pragma unroll
                for (int b = 0; b < NB; ++b) tau[b] = fma((double)kh[u][b], dl[u], tau[b]);
        }
        for (; k < nmove; ++k) {                  // the last nmove mod 4 steps
            int cl;
            double dl;
            walk_step(tnx, tny, tnz, t, cell, dcx, dcy, dcz, dtx, dty, dtz, cl, dl);
            float kh[NB];
            load_kh<NB, KS>(kp, cl, kh);
#pragma unroll
            for (int b = 0; b < NB; ++b) tau[b] = fma((double)kh[b], dl, tau[b]);
        }
        nseg += (unsigned)nmove;
        ++nseg;                                   // the target cell itself
        if (na > 0.0) {
            // absorbers in the shell r_in..r_out; r_out^3 - r_in^3 factored
            const double inv_abs =
                1.0 / (na * vol_c * (tout - tin) * (tout * tout + tout * tin + tin * tin));
            float khc[NB];
            load_kh<NB, KS>(kp, cid, khc);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const double dtau = (double)khc[b] * (tout - tin);
                const double nabs_dot = src.s[s].Q[b] * exp(-tau[b]) * -expm1(-dtau);
                g += nabs_dot * inv_abs;
                ht += nabs_dot * src.e[b] * inv_abs;
            }
        }
    }
    if (first) {
        Gamma[cid] = (float)g;
        if (Heat) Heat[cid] = src.has_e ? (float)ht : 0.0f;
        if (segs) segs[cid] = nseg;
    } else {
        Gamma[cid] = (float)((double)Gamma[cid] + g);
        if (Heat && src.has_e) Heat[cid] = (float)((double)Heat[cid] + ht);
        if (segs) segs[cid] += nseg;
    }
}

int pt_fail(int code, const std::string &msg) { return art_set_error(code, msg.c_str()); }

template <int NB, int KS>
hipError_t launch_point(const float *kp, const float *n_abs, const int *dims, double h,
                        const PtChunk &chunk, int first, float *Gamma, float *Heat, unsigned *segs,
                        hipStream_t st)
{
    const int nblk = ((dims[0] + 7) / 8) * ((dims[1] + 7) / 8) * ((dims[2] + 3) / 4);
    hipLaunchKernelGGL((art_point_kernel<NB, KS>), dim3(nblk), dim3(256), 0, st, kp, n_abs, dims[0],
                       dims[1], dims[2], h, chunk, first, Gamma, Heat, segs);
    return hipGetLastError();
}

__global__ void art_kpack_kernel(const float2 *__restrict__ fields, long long ncell, int nb, int ks,
                                 float *__restrict__ kpack)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    for (int b = 0; b < ks; ++b) kpack[c * ks + b] = b < nb ? fields[c * nb + b].x : 0.0f;
}

}  // namespace

hipError_t art_launch_kpack(const float2 *fields, long long ncell, int nb, int ks, float *kpack,
                            hipStream_t stream)
{
    const long long nblk = (ncell + 255) / 256;
    hipLaunchKernelGGL(art_kpack_kernel, dim3((unsigned)nblk), dim3(256), 0, stream, fields, ncell, nb,
                       ks, kpack);
    return hipGetLastError();
}

// The entry point's work.  kpack_buf == NULL: the mesh's own kappa pack
// (built on first use, kept until the next art_set_fields); else the pack is
// rebuilt into kpack_buf (room for kpack_cap floats) on every call.
int art_point_impl(art_mesh *mesh, int nsrc, const double *pos, const double *Q, const double *e,
                   const float *n_abs, float *Gamma, float *Heat, unsigned *segs, void *hip_stream,
                   float *kpack_buf, long long kpack_cap)
{
    if (!mesh) return pt_fail(ART_E_INVAL, "art_point_sources: null mesh");
    int dims[3], nb;
    double h;
    const float2 *rec;
    art_mesh_fields(mesh, dims, &nb, &h, &rec);
    if (!rec) return pt_fail(ART_E_STATE, "art_point_sources: art_set_fields has not been called");
    if (nsrc < 0) return pt_fail(ART_E_INVAL, "art_point_sources: nsrc < 0");
    if (nsrc > 0 && (!pos || !Q)) return pt_fail(ART_E_INVAL, "art_point_sources: null pos or Q");
    if (!n_abs || !Gamma) return pt_fail(ART_E_INVAL, "art_point_sources: null n_abs or Gamma");
    if ((long long)dims[0] * dims[1] * dims[2] * nb >= 0x7fffffffll)
        return pt_fail(ART_E_UNSUPPORTED, "art_point_sources: more than 2^31 - 1 records");
    {
        const long long ks_ = nb == 1 ? 1 : (nb == 2 ? 2 : 4);
        if ((long long)dims[0] * dims[1] * dims[2] * ks_ * 4 >= 0x80000000ll)
            return pt_fail(ART_E_UNSUPPORTED, "art_point_sources: kappa pack of 2 GiB or more");
    }
    for (int s = 0; s < nsrc; ++s) {
        for (int ax = 0; ax < 3; ++ax) {
            const double v = pos[3 * s + ax];
            if (!(std::isfinite(v) && v >= 0.0 && v <= (double)dims[ax]))
                return pt_fail(ART_E_INVAL, "art_point_sources: source " + std::to_string(s) +
                                                " lies outside the box [0, n] of its axes");
        }
        for (int b = 0; b < nb; ++b)
            if (!(std::isfinite(Q[(long long)s * nb + b]) && Q[(long long)s * nb + b] >= 0.0))
                return pt_fail(ART_E_INVAL, "art_point_sources: photon rates must be finite and >= 0");
    }
    if (e)
        for (int b = 0; b < nb; ++b)
            if (!std::isfinite(e[b]))
                return pt_fail(ART_E_INVAL, "art_point_sources: heating energies must be finite");
    hipStream_t st = (hipStream_t)hip_stream;
    const float *kp;
    int ks;
    if (kpack_buf) {
        ks = nb == 1 ? 1 : (nb == 2 ? 2 : 4);
        const long long ncell = (long long)dims[0] * dims[1] * dims[2];
        if (ncell * ks > kpack_cap)
            return pt_fail(ART_E_UNSUPPORTED, "art_point_sources_noalloc: the kappa pack needs " +
                                                  std::to_string(ncell * ks) + " floats, above the " +
                                                  std::to_string(kpack_cap) + " of the static scratch");
        const hipError_t err = art_launch_kpack(rec, ncell, nb, ks, kpack_buf, st);
        if (err != hipSuccess)
            return pt_fail(ART_E_HIP, std::string("art_point_sources_noalloc: ") + hipGetErrorString(err));
        kp = kpack_buf;
    } else {
        int rc = art_mesh_kpack(mesh, st, &kp, &ks);
        if (rc != ART_OK) return rc;
    }
    int s0 = 0;
    do {
        PtChunk chunk{};
        chunk.n = nsrc - s0 < PT_CHUNK ? nsrc - s0 : PT_CHUNK;
        chunk.has_e = e ? 1 : 0;
        for (int b = 0; b < nb; ++b) chunk.e[b] = e ? e[b] : 0.0;
        for (int i = 0; i < chunk.n; ++i) {
            for (int ax = 0; ax < 3; ++ax) chunk.s[i].p[ax] = pos[3 * (s0 + i) + ax];
            for (int b = 0; b < nb; ++b) chunk.s[i].Q[b] = Q[(long long)(s0 + i) * nb + b];
        }
        hipError_t err;
        switch (nb) {
        case 1: err = launch_point<1, 1>(kp, n_abs, dims, h, chunk, s0 == 0, Gamma, Heat, segs, st); break;
        case 2: err = launch_point<2, 2>(kp, n_abs, dims, h, chunk, s0 == 0, Gamma, Heat, segs, st); break;
        case 3: err = launch_point<3, 4>(kp, n_abs, dims, h, chunk, s0 == 0, Gamma, Heat, segs, st); break;
        default: err = launch_point<4, 4>(kp, n_abs, dims, h, chunk, s0 == 0, Gamma, Heat, segs, st); break;
        }
        if (err != hipSuccess)
            return pt_fail(ART_E_HIP, std::string("art_point_sources: launch: ") + hipGetErrorString(err));
        s0 += chunk.n;
    } while (s0 < nsrc);
    return ART_OK;
}

extern "C" int art_point_sources(art_mesh *mesh, int nsrc, const double *pos, const double *Q,
                                 const double *e, const float *n_abs, float *Gamma, float *Heat,
                                 unsigned *segs, void *hip_stream)
{
    return art_point_impl(mesh, nsrc, pos, Q, e, n_abs, Gamma, Heat, segs, hip_stream, nullptr, 0);
}
