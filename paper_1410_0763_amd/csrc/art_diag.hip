// art_diag.hip -- measurements behind design decisions (include/art_diag.h).
#include <string>

#include "../../include/art.h"
#include "../../include/art_diag.h"
#include "art_internal.h"

namespace {

__global__ __launch_bounds__(64) void release_cost_kernel(float *out, unsigned *flag, int mode, int words)
{
    float *o = out + (long long)blockIdx.x * words;
    for (int i = threadIdx.x; i < words; i += 64) o[i] = (float)(i + blockIdx.x);
    if (mode == 1) __threadfence();
    if (mode == 2 && threadIdx.x == 0)
        __hip_atomic_store(flag + blockIdx.x, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (mode == 3 && threadIdx.x == 0)
        __hip_atomic_store(flag + blockIdx.x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (mode == 4 && threadIdx.x == 0) {
        const unsigned v =
            __hip_atomic_load(flag + (blockIdx.x ^ 1u), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        o[0] += (float)v;
    }
}

int diag_fail(int code, const std::string &m) { return art_set_error(code, m.c_str()); }

}  // namespace

extern "C" int art_diag_release_cost(int nwg, int words, float ns[5])
{
    if (!ns || nwg < 1 || nwg > 1000000 || words < 1 || words > 65536)
        return diag_fail(ART_E_INVAL, "art_diag_release_cost: nwg in [1, 1e6], words in [1, 65536]");
    float *out = nullptr;
    unsigned *flag = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int rc = ART_OK;
    hipError_t e = hipMalloc(&out, (size_t)nwg * words * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&flag, (size_t)(nwg + 1) * sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(flag, 0, (size_t)(nwg + 1) * sizeof(unsigned));
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    for (int mode = 0; mode < 5 && e == hipSuccess; ++mode) {
        float best = 1e30f;
        for (int rep = 0; rep < 6 && e == hipSuccess; ++rep) {
            e = hipEventRecord(a, nullptr);
            hipLaunchKernelGGL(release_cost_kernel, dim3((unsigned)nwg), dim3(64), 0, nullptr, out, flag, mode,
                               words);
            if (e == hipSuccess) e = hipGetLastError();
            if (e == hipSuccess) e = hipEventRecord(b, nullptr);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (rep > 0 && ms < best) best = ms;
        }
        ns[mode] = best * 1e6f / (float)nwg;
    }
    if (e != hipSuccess) rc = diag_fail(ART_E_HIP, std::string("art_diag_release_cost: ") + hipGetErrorString(e));
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (out) (void)hipFree(out);
    if (flag) (void)hipFree(flag);
    return rc;
}
