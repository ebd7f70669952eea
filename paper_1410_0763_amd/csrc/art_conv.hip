// art_conv.hip -- layers of the learned surrogate: 3-D convolution on the
// matrix cores (bf16 inputs, float32 sums), its input and weight gradients,
// ReLU gradient, mean-squared-error loss, AdamW, and the feature transforms.
//
// Forward (and input gradient, which is the same operation with mirrored
// taps and swapped channels): an implicit GEMM.  One wave computes four rows
// of 32 consecutive voxels along x times the 32 output channels as four
// 32 x 32 x 16 MFMA accumulators; the K loop runs over the 27 taps and the
// input channels in groups of 16, each input row and weight fragment loaded
// once per (dz, dx) and used by up to four MFMAs.  Each lane feeds 8 input channels of one
// voxel (one 16-byte load of the channels-last activations) and 8 input
// channels of one output channel's weights; neighbours outside the mesh are
// read through a buffer descriptor at an offset beyond its range, which
// returns zeros (the zero padding).  The accumulator tile goes through LDS so
// that every lane stores whole 16-byte runs of one voxel's channels.
//
// Weight gradient: dw[tap] = X_tap^T G is a reduction over voxels, so the
// voxels are the K dimension.  The operands are channels-first copies (one
// 16-byte load = 8 consecutive voxels of one channel); the x offset of a tap
// would misalign them, so the layer input is kept as three copies shifted by
// -1, 0, +1 along x.  Each wave reduces one (tap, chunk of rows) into a
// float32 partial; a second kernel sums the chunks in a fixed order.
#include <cstdint>

#include "../../include/art.h"
#include "../../include/art_nn.h"
#include "art_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;

#define NN_OOB 0x80000000u

__device__ __forceinline__ rsrc_t nn_rsrc(const void *p, long long bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0,
                                             (int)(bytes < 0x7fffffffll ? bytes : 0x7fffffffll),
                                             0x00020000);
}

__device__ __forceinline__ bf16x8 load8(rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

// Row of a 32 x 32 MFMA accumulator held in element r of a lane's 16 floats
// (the lane holds column lane % 32).
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// One workgroup of 8 waves: output rows y0 .. y0+15 (2 per wave) x 32 voxels
// along x at one z, 32 output channels.  For each dz and group of 16 input
// channels, that group of the input plane z + dz (rows y0-1 .. y0+16, voxels
// x0-1 .. x0+32; zero outside the mesh) and of the nine weight taps of that
// dz are staged in LDS once; each wave then takes its 4 input rows and the
// 3 weight fragments of every dx from LDS for 6 MFMAs.  Staged voxels are
// padded to 48 bytes against bank conflicts; 43 KB per workgroup lets three
// workgroups share a CU (6 waves per SIMD).
constexpr int CONV_ROWS = 18, CONV_COLS = 34;
constexpr int CONV_VS = 24;                                          // bf16 per staged voxel (16 + pad)
template <int CIN> constexpr int conv_lds_bytes() { return (CONV_ROWS * CONV_COLS + 9 * 32) * CONV_VS * 2; }

template <int CIN>
__global__ __launch_bounds__(512) void conv_fwd_kernel(const uint16_t *__restrict__ x,
                                                       const uint16_t *__restrict__ w,
                                                       const float *__restrict__ bias, int D,
                                                       int H, int W, int relu,
                                                       uint16_t *__restrict__ y,
                                                       float *__restrict__ y0)
{
    constexpr int R = 2, VS = CONV_VS;
    extern __shared__ __align__(16) uint16_t smem[];
    uint16_t *sx = smem;                                       // [18][34][VS]
    uint16_t *sw = smem + CONV_ROWS * CONV_COLS * VS;          // [9][32][VS]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ntw = W / 32, nty = (H + 15) / 16;
    const long long t = blockIdx.x;
    const int xt = (int)(t % ntw), ty = (int)((t / ntw) % nty), zz0 = (int)(t / ((long long)ntw * nty));
    const int yb = ty * 16, x0 = xt * 32;
    const int m = lane & 31, kh = lane >> 5;
    const long long V = (long long)D * H * W;
    const rsrc_t rX = nn_rsrc(x, V * CIN * 2);
    const rsrc_t rW = nn_rsrc(w, 27ll * 32 * CIN * 2);
    f32x16 acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = f32x16{};
    for (int dz = -1; dz <= 1; ++dz) {
        const int zz = zz0 + dz;
        if (zz < 0 || zz >= D) continue;                       // uniform over the workgroup
        for (int ks = 0; ks < CIN / 16; ++ks) {
            __syncthreads();                                   // the previous stage is consumed
            for (int c = threadIdx.x; c < CONV_ROWS * CONV_COLS * 2; c += 512) {
                const int q = c & 1, vox = c >> 1, col = vox % CONV_COLS, row = vox / CONV_COLS;
                const int yy = yb - 1 + row, xx = x0 - 1 + col;
                const bool ok = yy >= 0 && yy < H && xx >= 0 && xx < W;
                const unsigned off =
                    ok ? (unsigned)((((long long)zz * H + yy) * W + xx) * CIN * 2 + 32 * ks + 16 * q) : NN_OOB;
                *reinterpret_cast<u32x4 *>(sx + vox * VS + q * 8) = __builtin_amdgcn_raw_buffer_load_b128(rX, off, 0, 0);
            }
            for (int c = threadIdx.x; c < 9 * 32 * 2; c += 512) {
                const int q = c & 1, row = c >> 1;               // row = tap in dz * 32 + co
                const unsigned off = (unsigned)((((dz + 1) * 9 * 32 + row) * CIN) * 2 + 32 * ks + 16 * q);
                *reinterpret_cast<u32x4 *>(sw + row * VS + q * 8) = __builtin_amdgcn_raw_buffer_load_b128(rW, off, 0, 0);
            }
            __syncthreads();
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                bf16x8 a[R + 2];
#pragma unroll
                for (int r = 0; r < R + 2; ++r)
                    a[r] = *reinterpret_cast<const bf16x8 *>(sx + ((wave * R + r) * CONV_COLS + m + 1 + dx) * VS + 8 * kh);
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    const int tl = (dy + 1) * 3 + (dx + 1);
                    const bf16x8 bw = *reinterpret_cast<const bf16x8 *>(sw + (tl * 32 + m) * VS + 8 * kh);
#pragma unroll
                    for (int q = 0; q < R; ++q)
                        acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[q + dy + 1], bw, acc[q], 0, 0, 0);
                }
            }
        }
    }
    __syncthreads();                                           // LDS now holds the output tiles
    float (*tile)[32][33] = reinterpret_cast<float (*)[32][33]>(smem) + wave;
    const float bm = bias ? bias[m] : 0.0f;
    for (int q = 0; q < R; ++q) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float v = acc[q][r] + bm;
            if (relu) v = fmaxf(v, 0.0f);
            (*tile)[acc_row(r, lane)][m] = v;
        }
        __syncthreads();
        const int yq = yb + wave * R + q;
        if (yq < H) {
            const long long v0 = ((long long)zz0 * H + yq) * W + x0;
            if (y) {
                const int row = lane >> 1, c0 = (lane & 1) * 16;
                u32x4 p[2];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = c0 + 8 * h + 2 * e;
                        p[h][e] = (unsigned)f2bf((*tile)[row][c]) | ((unsigned)f2bf((*tile)[row][c + 1]) << 16);
                    }
                u32x4 *dst = reinterpret_cast<u32x4 *>(y + (v0 + row) * 32 + c0);
                dst[0] = p[0];
                dst[1] = p[1];
            }
            if (y0 && lane < 32) y0[v0 + lane] = (*tile)[lane][0];
        }
        __syncthreads();
    }
}

// One wave: the three taps dx = -1, 0, 1 of one (dz, dy) over one chunk of
// rows; the gradient operand is loaded once per K step for three MFMAs.
template <int CIN>
__global__ __launch_bounds__(256) void conv_bwdw_kernel(const uint16_t *__restrict__ xs,
                                                        const uint16_t *__restrict__ g, int D,
                                                        int H, int W, int nchunk,
                                                        float *__restrict__ partial)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long job = (long long)blockIdx.x * 4 + wave;
    if (job >= 9ll * nchunk) return;                       // whole wave
    const int zy = (int)(job % 9), chunk = (int)(job / 9);
    const int dz = zy / 3 - 1, dy = zy % 3 - 1;
    const int m = lane & 31, kh = lane >> 5;
    const long long V = (long long)D * H * W;
    const rsrc_t rX = nn_rsrc(xs, 3ll * CIN * V * 2);
    const rsrc_t rG = nn_rsrc(g, 32ll * V * 2);
    const long long gbase = (long long)m * V;
    const int rows = D * H / nchunk;
    f32x16 acc[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) acc[s] = f32x16{};
    for (int r = chunk * rows; r < (chunk + 1) * rows; ++r) {
        const int z = r / H, yv = r % H;
        const int zz = z + dz, yy = yv + dy;
        const bool ok = zz >= 0 && zz < D && yy >= 0 && yy < H && m < CIN;
        const long long arow = ((long long)zz * H + yy) * W + 8 * kh;   // within one copy
        const long long grow = gbase + (long long)r * W + 8 * kh;
        for (int x0 = 0; x0 < W; x0 += 16) {
            const bf16x8 b = load8(rG, (unsigned)((grow + x0) * 2));
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const long long aoff = ((long long)s * CIN + m) * V + arow + x0;
                const bf16x8 a = load8(rX, ok ? (unsigned)(aoff * 2) : NN_OOB);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[s], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int tap = zy * 3 + s;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int ci = acc_row(q, lane);
            if (ci < CIN) partial[(((long long)chunk * 27 + tap) * CIN + ci) * 32 + m] = acc[s][q];
        }
    }
}

__global__ void sum_chunks_kernel(const float *__restrict__ partial, int nchunk, int n,
                                  float *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += partial[(long long)c * n + i];
    out[i] = s;
}

// Per-chunk channel sums of a channels-first [32][V] bf16 array (fixed tree order).
__global__ __launch_bounds__(256) void bias_partial_kernel(const uint16_t *__restrict__ g,
                                                           long long V, int nchunk,
                                                           float *__restrict__ partial)
{
    __shared__ float red[256];
    const int chunk = blockIdx.x;
    const long long len = V / nchunk, v0 = chunk * len;
    for (int c = 0; c < 32; ++c) {
        float s = 0.0f;
        for (long long v = threadIdx.x; v < len; v += 256) s += bf2f(g[c * V + v0 + v]);
        red[threadIdx.x] = s;
        __syncthreads();
        for (int k = 128; k > 0; k >>= 1) {
            if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[chunk * 32 + c] = red[0];
        __syncthreads();
    }
}

// One thread per (voxel, group of 8 channels): a 16-byte load of the
// channels-last input, eight 2-byte stores into each channels-first copy.
__global__ void shift3_kernel(const uint16_t *__restrict__ x, int cin, int W, long long V,
                              uint16_t *__restrict__ xs)
{
    const int ng = cin / 8;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * ng) return;
    const long long v = t / ng;
    const int cg = (int)(t % ng);
    const int xx = (int)(v % W);
    for (int s = 0; s < 3; ++s) {
        const int sx = xx + s - 1;
        u32x4 d = {0u, 0u, 0u, 0u};
        if (sx >= 0 && sx < W) d = *reinterpret_cast<const u32x4 *>(x + (v + s - 1) * cin + 8 * cg);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const unsigned word = d[e >> 1];
            xs[((long long)s * cin + 8 * cg + e) * V + v] = (uint16_t)((e & 1) ? (word >> 16) : (word & 0xffffu));
        }
    }
}

// One thread per (voxel, group of 8 channels): 16-byte loads and store of the
// channels-last arrays, eight 2-byte stores into the channels-first copy.
__global__ void relu_grad_kernel(const uint16_t *__restrict__ dy, const uint16_t *__restrict__ y,
                                 long long V, uint16_t *__restrict__ g, uint16_t *__restrict__ gcf)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= V * 4) return;
    const long long v = t >> 2;
    const int cg = (int)(t & 3);
    u32x4 d = *reinterpret_cast<const u32x4 *>(dy + v * 32 + 8 * cg);
    if (y) {
        const u32x4 a = *reinterpret_cast<const u32x4 *>(y + v * 32 + 8 * cg);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned lo = bf2f((uint16_t)(a[k] & 0xffffu)) > 0.0f ? 0x0000ffffu : 0u;
            const unsigned hi = bf2f((uint16_t)(a[k] >> 16)) > 0.0f ? 0xffff0000u : 0u;
            d[k] &= lo | hi;
        }
    }
    *reinterpret_cast<u32x4 *>(g + v * 32 + 8 * cg) = d;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const unsigned word = d[e >> 1];
        gcf[(long long)(8 * cg + e) * V + v] = (uint16_t)((e & 1) ? (word >> 16) : (word & 0xffffu));
    }
}

__global__ void prep_weights_kernel(const float *__restrict__ w, int cin, uint16_t *__restrict__ wf,
                                    uint16_t *__restrict__ wb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // over 27 * 32 * 32
    if (i >= 27 * 32 * 32) return;
    const int t = i / 1024, a = (i / 32) % 32, b = i % 32;
    // forward: wf[t][co = a][ci = b] = w[t][ci][co]
    if (b < cin) wf[(t * 32 + a) * cin + b] = f2bf(w[(t * cin + b) * 32 + a]);
    // input gradient: wb[t][ci = a][co = b] = w[26 - t][ci][co] (zero for ci >= cin)
    wb[(t * 32 + a) * 32 + b] = a < cin ? f2bf(w[((26 - t) * cin + a) * 32 + b]) : (uint16_t)0;
}

__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ pred,
                                                  const float *__restrict__ target,
                                                  const float *__restrict__ weight, long long V,
                                                  float *__restrict__ partial,
                                                  uint16_t *__restrict__ dy)
{
    __shared__ float red[256];
    const long long len = (V + gridDim.x - 1) / gridDim.x;
    const long long v0 = blockIdx.x * len, v1 = v0 + len < V ? v0 + len : V;
    const float scale = 2.0f / (float)V;
    float s = 0.0f;
    for (long long v = v0 + threadIdx.x; v < v1; v += 256) {
        const float d = pred[v] - target[v];
        const float wv = weight ? weight[v] : 1.0f;
        s += wv * d * d;
        u32x4 *dst = reinterpret_cast<u32x4 *>(dy + v * 32);
        const u32x4 z = {0u, 0u, 0u, 0u};
        u32x4 first = z;
        first.x = (unsigned)f2bf(scale * wv * d);
        dst[0] = first;
        dst[1] = z;
        dst[2] = z;
        dst[3] = z;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void mse_final_kernel(const float *__restrict__ partial, int n, long long V,
                                 float *__restrict__ loss)
{
    if (threadIdx.x != 0) return;
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s += partial[i];
    loss[0] = s / (float)V;
}

// w = J^2 / mean(J^2): per-block partial sums, their total, the weights.
__global__ __launch_bounds__(256) void sq_partial_kernel(const float *__restrict__ J, long long V,
                                                         float *__restrict__ partial)
{
    __shared__ float red[256];
    const long long len = (V + gridDim.x - 1) / gridDim.x;
    const long long v0 = blockIdx.x * len, v1 = v0 + len < V ? v0 + len : V;
    float s = 0.0f;
    for (long long v = v0 + threadIdx.x; v < v1; v += 256) s += J[v] * J[v];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sq_total_kernel(float *__restrict__ partial, int n)
{
    if (threadIdx.x != 0) return;
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s += partial[i];
    partial[n] = s;
}

__global__ void sq_weight_kernel(const float *__restrict__ J, long long V, float lambda,
                                 const float *__restrict__ total, float *__restrict__ w)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float t = total[0];
    const float q = t > 0.0f ? J[v] * J[v] * ((float)V / t) : 1.0f;
    w[v] = (q + lambda) / (1.0f + lambda);
}

__global__ void adamw_kernel(float *__restrict__ w, const float *__restrict__ g,
                             float *__restrict__ m, float *__restrict__ v, int n, float lr,
                             float b1, float b2, float eps, float wd, float bc1, float bc2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    w[i] = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
}

struct F3 {
    float a[3];
};

__global__ void features_kernel(const float *__restrict__ J, const float *__restrict__ dens,
                                const float *__restrict__ xhi, long long V, F3 mu, F3 isd,
                                uint16_t *__restrict__ x)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    art_feature_store(J[v], dens[v], xhi[v], mu.a, isd.a, x + v * 16);
}

__global__ void expand_kernel(const float *__restrict__ Jc, const float *__restrict__ pred,
                              long long V, float *__restrict__ out)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    out[v] = Jc[v] * expf(pred[v]);
}

__global__ void log_ratio_kernel(const float *__restrict__ Jf, const float *__restrict__ Jc,
                                 long long V, float *__restrict__ t)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    t[v] = logf(fmaxf(Jf[v], 1e-30f)) - logf(fmaxf(Jc[v], 1e-30f));
}

// Voxels with any of the three feature channels outside [lo, hi].
__global__ __launch_bounds__(256) void ood_kernel(const uint16_t *__restrict__ x, long long V,
                                                  F3 lo, F3 hi, unsigned int *__restrict__ count)
{
    __shared__ unsigned int red;
    if (threadIdx.x == 0) red = 0u;
    __syncthreads();
    unsigned int c = 0;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < V;
         v += (long long)gridDim.x * blockDim.x) {
        bool out = false;
        for (int k = 0; k < 3; ++k) {
            const float f = bf2f(x[v * 16 + k]);
            out = out || !(f >= lo.a[k] && f <= hi.a[k]);
        }
        c += out ? 1u : 0u;
    }
    atomicAdd(&red, c);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(count, red);
}

int launch_status(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return ART_OK;
    return art_set_error(ART_E_HIP, (std::string(what) + ": " + hipGetErrorString(e)).c_str());
}

unsigned blocks_for(long long n, int per) { return (unsigned)((n + per - 1) / per); }

__global__ void art_fill_u32_kernel_entry(unsigned int *p) { *p = 0u; }

}  // namespace

extern "C" {

int art_conv3d_fwd(const void *x, int cin, const void *w_k, const float *bias, int D, int H,
                   int W, int relu, void *y, float *y0, void *hip_stream)
{
    if (!x || !w_k) return art_set_error(ART_E_INVAL, "art_conv3d_fwd: null input or weights");
    if (cin != 16 && cin != 32) return art_set_error(ART_E_INVAL, "art_conv3d_fwd: cin must be 16 or 32");
    if (D < 1 || H < 1 || W < 32 || W % 32)
        return art_set_error(ART_E_INVAL, "art_conv3d_fwd: W must be a positive multiple of 32");
    if ((long long)D * H * W * 64 >= (1ll << 31))
        return art_set_error(ART_E_UNSUPPORTED, "art_conv3d_fwd: activation tensor above 2 GiB");
    hipStream_t st = (hipStream_t)hip_stream;
    const long long tiles = (long long)D * ((H + 15) / 16) * (W / 32);
    const auto *xp = (const uint16_t *)x;
    const auto *wp = (const uint16_t *)w_k;
    static bool configured = false;   // LDS above the 64 KiB default needs an opt-in
    if (!configured) {
        hipError_t e = hipFuncSetAttribute((const void *)conv_fwd_kernel<16>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, conv_lds_bytes<16>());
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)conv_fwd_kernel<32>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, conv_lds_bytes<32>());
        if (e != hipSuccess)
            return art_set_error(ART_E_HIP, (std::string("art_conv3d_fwd: ") + hipGetErrorString(e)).c_str());
        configured = true;
    }
    if (cin == 16)
        hipLaunchKernelGGL(conv_fwd_kernel<16>, dim3((unsigned)tiles), dim3(512), conv_lds_bytes<16>(), st,
                           xp, wp, bias, D, H, W, relu, (uint16_t *)y, y0);
    else
        hipLaunchKernelGGL(conv_fwd_kernel<32>, dim3((unsigned)tiles), dim3(512), conv_lds_bytes<32>(), st,
                           xp, wp, bias, D, H, W, relu, (uint16_t *)y, y0);
    return launch_status("art_conv3d_fwd");
}

int art_conv3d_bwd_weight(const void *xs, int cin, const void *g, int D, int H, int W,
                          float *partial, int nchunk, float *dw, void *hip_stream)
{
    if (!xs || !g || !partial || !dw) return art_set_error(ART_E_INVAL, "art_conv3d_bwd_weight: null pointer");
    if (cin != 16 && cin != 32) return art_set_error(ART_E_INVAL, "art_conv3d_bwd_weight: cin must be 16 or 32");
    if (D < 1 || H < 1 || W < 16 || W % 16)
        return art_set_error(ART_E_INVAL, "art_conv3d_bwd_weight: W must be a positive multiple of 16");
    if (nchunk < 1 || (D * H) % nchunk)
        return art_set_error(ART_E_INVAL, "art_conv3d_bwd_weight: nchunk must divide D*H");
    if (3ll * cin * D * H * W * 2 >= (1ll << 31))
        return art_set_error(ART_E_UNSUPPORTED, "art_conv3d_bwd_weight: shifted copies above 2 GiB");
    hipStream_t st = (hipStream_t)hip_stream;
    const auto *xp = (const uint16_t *)xs;
    const auto *gp = (const uint16_t *)g;
    const unsigned nb = blocks_for(9ll * nchunk, 4);
    if (cin == 16)
        hipLaunchKernelGGL(conv_bwdw_kernel<16>, dim3(nb), dim3(256), 0, st, xp, gp, D, H, W, nchunk, partial);
    else
        hipLaunchKernelGGL(conv_bwdw_kernel<32>, dim3(nb), dim3(256), 0, st, xp, gp, D, H, W, nchunk, partial);
    int rc = launch_status("art_conv3d_bwd_weight");
    if (rc) return rc;
    const int n = 27 * cin * 32;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, partial, nchunk, n, dw);
    return launch_status("art_conv3d_bwd_weight (sum)");
}

int art_nn_bias_grad(const void *g, int V, float *partial, int nchunk, float *db, void *hip_stream)
{
    if (!g || !partial || !db || V < 1 || nchunk < 1 || V % nchunk)
        return art_set_error(ART_E_INVAL, "art_nn_bias_grad: bad arguments (nchunk must divide V)");
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(bias_partial_kernel, dim3(nchunk), dim3(256), 0, st, (const uint16_t *)g,
                       (long long)V, nchunk, partial);
    int rc = launch_status("art_nn_bias_grad");
    if (rc) return rc;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(1), dim3(32), 0, st, partial, nchunk, 32, db);
    return launch_status("art_nn_bias_grad (sum)");
}

int art_nn_shift3(const void *x, int cin, int D, int H, int W, void *xs, void *hip_stream)
{
    if (!x || !xs || (cin != 16 && cin != 32) || D < 1 || H < 1 || W < 1)
        return art_set_error(ART_E_INVAL, "art_nn_shift3: bad arguments (cin must be 16 or 32)");
    const long long V = (long long)D * H * W;
    hipLaunchKernelGGL(shift3_kernel, dim3(blocks_for(V * (cin / 8), 256)), dim3(256), 0, (hipStream_t)hip_stream,
                       (const uint16_t *)x, cin, W, V, (uint16_t *)xs);
    return launch_status("art_nn_shift3");
}

int art_nn_relu_grad(const void *dy, const void *y, int V, void *g, void *g_cf, void *hip_stream)
{
    if (!dy || !g || !g_cf || V < 1) return art_set_error(ART_E_INVAL, "art_nn_relu_grad: bad arguments");
    hipLaunchKernelGGL(relu_grad_kernel, dim3(blocks_for(4ll * V, 256)), dim3(256), 0, (hipStream_t)hip_stream,
                       (const uint16_t *)dy, (const uint16_t *)y, (long long)V, (uint16_t *)g,
                       (uint16_t *)g_cf);
    return launch_status("art_nn_relu_grad");
}

int art_nn_prep_weights(const float *w, int cin, void *w_fwd, void *w_bwd, void *hip_stream)
{
    if (!w || !w_fwd || !w_bwd || (cin != 16 && cin != 32))
        return art_set_error(ART_E_INVAL, "art_nn_prep_weights: bad arguments");
    hipLaunchKernelGGL(prep_weights_kernel, dim3(blocks_for(27 * 32 * 32, 256)), dim3(256), 0,
                       (hipStream_t)hip_stream, w, cin, (uint16_t *)w_fwd, (uint16_t *)w_bwd);
    return launch_status("art_nn_prep_weights");
}

int art_nn_mse(const float *pred, const float *target, const float *weight, int V, float *partial,
               float *loss, void *dy, void *hip_stream)
{
    if (!pred || !target || !partial || !loss || !dy || V < 1)
        return art_set_error(ART_E_INVAL, "art_nn_mse: bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(mse_kernel, dim3(256), dim3(256), 0, st, pred, target, weight, (long long)V,
                       partial, (uint16_t *)dy);
    int rc = launch_status("art_nn_mse");
    if (rc) return rc;
    hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(64), 0, st, partial, 256, (long long)V, loss);
    return launch_status("art_nn_mse (sum)");
}

int art_nn_adamw(float *w, const float *g, float *m, float *v, int n, float lr, float beta1,
                 float beta2, float eps, float wd, int step, void *hip_stream)
{
    if (!w || !g || !m || !v || n < 1 || step < 1)
        return art_set_error(ART_E_INVAL, "art_nn_adamw: bad arguments");
    const float bc1 = 1.0f - powf(beta1, (float)step), bc2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adamw_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)hip_stream,
                       w, g, m, v, n, lr, beta1, beta2, eps, wd, bc1, bc2);
    return launch_status("art_nn_adamw");
}

int art_nn_features(const float *J, const float *density, const float *x_hi, int V, const float *mu,
                    const float *inv_sd, void *x, void *hip_stream)
{
    if (!J || !density || !x_hi || !mu || !inv_sd || !x || V < 1)
        return art_set_error(ART_E_INVAL, "art_nn_features: bad arguments");
    F3 m3, s3;
    for (int k = 0; k < 3; ++k) {
        m3.a[k] = mu[k];
        s3.a[k] = inv_sd[k];
    }
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(V, 256)), dim3(256), 0, (hipStream_t)hip_stream,
                       J, density, x_hi, (long long)V, m3, s3, (uint16_t *)x);
    return launch_status("art_nn_features");
}

int art_nn_expand(const float *J_coarse, const float *pred, int V, float *J_out, void *hip_stream)
{
    if (!J_coarse || !pred || !J_out || V < 1) return art_set_error(ART_E_INVAL, "art_nn_expand: bad arguments");
    hipLaunchKernelGGL(expand_kernel, dim3(blocks_for(V, 256)), dim3(256), 0, (hipStream_t)hip_stream,
                       J_coarse, pred, (long long)V, J_out);
    return launch_status("art_nn_expand");
}

int art_nn_sq_weights(const float *J, int V, float lambda, float *partial, float *w,
                      void *hip_stream)
{
    if (!J || !partial || !w || V < 1 || !(lambda >= 0.0f))
        return art_set_error(ART_E_INVAL, "art_nn_sq_weights: bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(sq_partial_kernel, dim3(256), dim3(256), 0, st, J, (long long)V, partial);
    int rc = launch_status("art_nn_sq_weights");
    if (rc) return rc;
    hipLaunchKernelGGL(sq_total_kernel, dim3(1), dim3(64), 0, st, partial, 256);
    if ((rc = launch_status("art_nn_sq_weights (sum)"))) return rc;
    hipLaunchKernelGGL(sq_weight_kernel, dim3(blocks_for(V, 256)), dim3(256), 0, st, J, (long long)V,
                       lambda, partial + 256, w);
    return launch_status("art_nn_sq_weights (weights)");
}

int art_nn_log_ratio(const float *J_fine, const float *J_coarse, int V, float *target,
                     void *hip_stream)
{
    if (!J_fine || !J_coarse || !target || V < 1)
        return art_set_error(ART_E_INVAL, "art_nn_log_ratio: bad arguments");
    hipLaunchKernelGGL(log_ratio_kernel, dim3(blocks_for(V, 256)), dim3(256), 0, (hipStream_t)hip_stream,
                       J_fine, J_coarse, (long long)V, target);
    return launch_status("art_nn_log_ratio");
}

int art_nn_ood_count(const void *x, int V, const float *lo, const float *hi, unsigned int *count,
                     void *hip_stream)
{
    if (!x || !lo || !hi || !count || V < 1) return art_set_error(ART_E_INVAL, "art_nn_ood_count: bad arguments");
    F3 l3, h3;
    for (int k = 0; k < 3; ++k) {
        l3.a[k] = lo[k];
        h3.a[k] = hi[k];
    }
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(art_fill_u32_kernel_entry, dim3(1), dim3(1), 0, st, count);
    int rc = launch_status("art_nn_ood_count (clear)");
    if (rc) return rc;
    hipLaunchKernelGGL(ood_kernel, dim3(1024), dim3(256), 0, st, (const uint16_t *)x, (long long)V,
                       l3, h3, count);
    return launch_status("art_nn_ood_count");
}

}  // extern "C"
