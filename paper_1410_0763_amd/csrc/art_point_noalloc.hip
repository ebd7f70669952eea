// art_point_noalloc.hip -- point-source rates without any allocation by the
// library: the kappa pack the walk reads lives in a file-scope device array
// (one per GPU, held until the process ends) instead of the mesh's own
// buffer.  Its device address is looked up once per device with
// hipGetSymbolAddress (in host code the array's name is not a device
// address) and cached; every call rebuilds the pack there, so calls that
// overlap on one GPU race on it.
#include <mutex>
#include <string>

#include "../../include/art_point.h"
#include "art_internal.h"

int art_point_impl(art_mesh *mesh, int nsrc, const double *pos, const double *Q, const double *e,
                   const float *n_abs, float *Gamma, float *Heat, unsigned *segs, void *hip_stream,
                   float *kpack_buf, long long kpack_cap);

namespace {

constexpr long long kScratchFloats = ART_POINT_NOALLOC_FLOATS;
constexpr int kMaxDevices = 64;

__device__ __align__(256) float scratch[kScratchFloats];

std::mutex g_mu;
float *g_ptr[kMaxDevices] = {};

// The array's address on the current device (looked up on first use).
int scratch_on_device(float **out)
{
    int dev = -1;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return art_set_error(ART_E_HIP, (std::string("art_point_sources_noalloc: hipGetDevice: ") +
                                         hipGetErrorString(err)).c_str());
    if (dev < 0 || dev >= kMaxDevices)
        return art_set_error(ART_E_UNSUPPORTED, "art_point_sources_noalloc: device index above 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !p)
            return art_set_error(ART_E_HIP, (std::string("art_point_sources_noalloc: hipGetSymbolAddress: ") +
                                             hipGetErrorString(err)).c_str());
        g_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_ptr[dev];
    return ART_OK;
}

}  // namespace

extern "C" int art_point_sources_noalloc(art_mesh *mesh, int nsrc, const double *pos,
                                         const double *Q, const double *e, const float *n_abs,
                                         float *Gamma, float *Heat, unsigned *segs,
                                         void *hip_stream)
{
    if (!mesh) return art_set_error(ART_E_INVAL, "art_point_sources_noalloc: null mesh");
    float *buf = nullptr;
    const int rc = scratch_on_device(&buf);
    if (rc != ART_OK) return rc;
    return art_point_impl(mesh, nsrc, pos, Q, e, n_abs, Gamma, Heat, segs, hip_stream, buf,
                          kScratchFloats);
}
