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
// voxels are the K dimension of the products; the channels-last operands
// are transposed into LDS as they are staged (see conv_bwdw_kernel), and
// the per-workgroup partials are added in a fixed order.
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
__global__ __launch_bounds__(512, 6) void conv_fwd_kernel(const uint16_t *__restrict__ x,
                                                       const uint16_t *__restrict__ w,
                                                       const float *__restrict__ bias, int D,
                                                       int H, int W, int relu,
                                                       const uint16_t *__restrict__ mask,
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
    // Stages (dz, group ks of 16 input channels), planes outside the mesh
    // skipped.  The input tile of the next stage is loaded into registers
    // while the current one is multiplied, so that its latency overlaps the
    // products.  A thread's 16-byte chunks c = tid + 512 j: chunk c is half q
    // = bit 4 of c of voxel 16 (c >> 5) + (c & 15), so that 16 consecutive
    // lanes write 16 different voxels (48 bytes apart: no two in one bank).
    constexpr int KS = CIN / 16, NVOX = CONV_ROWS * CONV_COLS, NXC = (NVOX + 15) / 16 * 32;
    auto stage_ok = [&](int sidx) { const int zz = zz0 + sidx / KS - 1; return zz >= 0 && zz < D; };
    u32x4 xr[(NXC + 511) / 512];
    auto xload = [&](int sidx) {
        const int zz = zz0 + sidx / KS - 1, ks = sidx % KS;
#pragma unroll
        for (int j = 0; j < (NXC + 511) / 512; ++j) {
            const int c = threadIdx.x + 512 * j;
            const int q = (c >> 4) & 1, vox = ((c >> 5) << 4) | (c & 15);
            const int col = vox % CONV_COLS, row = vox / CONV_COLS;
            const int yy = yb - 1 + row, xx = x0 - 1 + col;
            const bool ok = c < NXC && vox < NVOX && yy >= 0 && yy < H && xx >= 0 && xx < W;
            const unsigned off =
                ok ? (unsigned)((((long long)zz * H + yy) * W + xx) * CIN * 2 + 32 * ks + 16 * q) : NN_OOB;
            xr[j] = __builtin_amdgcn_raw_buffer_load_b128(rX, off, 0, 0);
        }
    };
    int sidx = 0;
    while (!stage_ok(sidx)) ++sidx;                            // dz = 0 always is
    xload(sidx);
    for (; sidx < 3 * KS; ++sidx) {
        if (!stage_ok(sidx)) continue;                         // uniform over the workgroup
        const int dz = sidx / KS - 1, ks = sidx % KS;
        __syncthreads();                                       // the previous stage is consumed
#pragma unroll
        for (int j = 0; j < (NXC + 511) / 512; ++j) {
            const int c = threadIdx.x + 512 * j;
            const int q = (c >> 4) & 1, vox = ((c >> 5) << 4) | (c & 15);
            if (c < NXC && vox < NVOX) *reinterpret_cast<u32x4 *>(sx + vox * VS + q * 8) = xr[j];
        }
        for (int c = threadIdx.x; c < 9 * 32 * 2; c += 512) {
            const int q = (c >> 4) & 1, row = ((c >> 5) << 4) | (c & 15);   // row = tap in dz * 32 + co
            const unsigned off = (unsigned)((((dz + 1) * 9 * 32 + row) * CIN) * 2 + 32 * ks + 16 * q);
            *reinterpret_cast<u32x4 *>(sw + row * VS + q * 8) = __builtin_amdgcn_raw_buffer_load_b128(rW, off, 0, 0);
        }
        __syncthreads();
        {
            int nx = sidx + 1;
            while (nx < 3 * KS && !stage_ok(nx)) ++nx;
            if (nx < 3 * KS) xload(nx);                        // in flight during the products
        }
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
                if (mask) {                                    // keep where mask > 0
                    const u32x4 *mk = reinterpret_cast<const u32x4 *>(mask + (v0 + row) * 32 + c0);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const u32x4 mm = mk[h];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const unsigned lo = bf2f((uint16_t)(mm[e] & 0xffffu)) > 0.0f ? 0x0000ffffu : 0u;
                            const unsigned hi = bf2f((uint16_t)(mm[e] >> 16)) > 0.0f ? 0xffff0000u : 0u;
                            p[h][e] &= lo | hi;
                        }
                    }
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

// Weight and bias gradients.  A workgroup owns one row of TX voxels along x
// (one y, one x tile) and marches over a chunk of z planes.  LDS holds the
// input rows y-1 .. y+1 of the planes z-1 .. z+2 (a ring of four slots, one
// voxel of halo at each end along x) and the gradient rows of planes z and
// z+1 (two buffers), transposed on the way in so that one 16-byte read gives a lane eight
// voxels of one channel: voxel x0 + k + j S (j = 0..7, S = TX / 8) is element
// j of group k.  The eight voxels of a group are S apart, so the x offset of
// a tap only moves to the neighbouring group (k - 1 or k + 1) and every read
// stays aligned; groups k = -1 and k = S hold the halo.  Nine waves, one per
// (dz, dy), keep their three dx taps in float32 accumulators for the whole
// march.  Each step writes the plane loaded during the previous step into
// the free slot, issues the loads of the plane after it, and runs the
// products of plane z: the loads have a whole step to arrive and one
// barrier per step suffices.  The bias gradient is summed from the staged
// gradient rows.  Each workgroup writes one float32 partial of all 27 taps
// and the bias; a second kernel adds the partials in a fixed order.
constexpr int BW_WAVES = 9, BW_THREADS = 64 * BW_WAVES, BW_SMAX = 16;
constexpr int BW_CSX = (3 * (BW_SMAX + 2)) | 1;   // 16-byte groups per channel of an input slot (odd)
constexpr int BW_CSG = BW_SMAX | 1;               // 16-byte groups per channel of the gradient row
// LDS: four input slots, two gradient buffers, the bias sums [32][S] (float)
template <int CIN> constexpr int bw_lds_bytes() { return (4 * CIN * BW_CSX + 2 * 32 * BW_CSG) * 16 + 32 * BW_SMAX * 4; }

// Keeps the loads of the next plane after the LDS writes of the previous one
// (both sets of registers live at once would spill).
__device__ __forceinline__ void bw_order()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Eight voxels (one 16-byte load each: eight channels) -> eight channels
// (one 16-byte group each: the eight voxels); one byte permute per dword
// (selector bytes 0-3 take the second operand, 4-7 the first).
__device__ __forceinline__ void bw_transpose(const u32x4 (&in)[8], u32x4 (&out)[8])
{
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            out[e][q] = __builtin_amdgcn_perm(in[2 * q + 1][e >> 1], in[2 * q][e >> 1],
                                              (e & 1) ? 0x07060302u : 0x05040100u);
}

// Wave roles.  Waves 0-8 each own the taps of one (dz, dy) = (w / 3 - 1,
// w % 3 - 1).  Staging: wave 1 stages the gradient row (and sums the bias),
// waves 2, 3, 6 and 7 the input rows; with the usual round-robin placement
// of waves on the four SIMDs (w % 4), the SIMD that holds three product
// waves (0, 4, 8) does no staging.
__device__ __forceinline__ int bw_xstager(int wave)
{
    return wave == 2 ? 0 : wave == 3 ? 1 : wave == 6 ? 2 : wave == 7 ? 3 : -1;
}

template <int CIN, int S>
__global__ __launch_bounds__(BW_THREADS) void conv_bwdw_kernel(const uint16_t *__restrict__ x,
                                                               const uint16_t *__restrict__ g, int D,
                                                               int H, int W, int ntx,
                                                               int planes, int nwg, int remap,
                                                               float *__restrict__ partial)
{
    extern __shared__ __align__(16) u32x4 lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, kh = lane >> 5;
    // workgroups that handle neighbouring rows share an XCD (and its L2)
    const int b = (int)blockIdx.x;
    const int L = remap ? (b & 7) * (nwg >> 3) + (b >> 3) : b;
    const int rows = H * ntx;
    const int row = L % rows, chunk = L / rows;
    const int y = row % H, x0 = (row / H) * (8 * S);
    const int z0 = chunk * planes, z1 = min(D, z0 + planes);
    const long long V = (long long)D * H * W;
    const rsrc_t rX = nn_rsrc(x, V * CIN * 2);
    const rsrc_t rG = nn_rsrc(g, V * 64);
    const int GB = 4 * CIN * BW_CSX;                          // first group of the gradient rows

    // this thread's staging task: a gradient group (kk < S, channels c8 ..
    // c8 + 7) or an input group (row r of a slot, kk in [0, S + 2)); the kind
    // is uniform over a wave
    const bool isg = wave == 1;
    const int xw = bw_xstager(wave);
    const int nxt = 3 * (S + 2) * (CIN / 8), per = (nxt + 3) / 4;
    const int task = isg ? lane : xw * per + lane;
    const bool has = isg ? lane < 4 * S : xw >= 0 && lane < per && task < nxt;
    int tr = 0, tkk = 0, tc8 = 0;
    if (isg) {
        tkk = task % S;
        tc8 = 8 * (task / S);
    } else {
        tkk = task % (S + 2);
        tr = (task / (S + 2)) % 3;
        tc8 = 8 * (task / (3 * (S + 2)));
    }
    // voxel x of element j: xj0 + j S; only j = 0 (left halo) and j = 7
    // (right halo) can leave the mesh
    const int xj0 = isg ? x0 + tkk : x0 + tkk - 1;
    const bool okl = xj0 >= 0, okr = xj0 + 7 * S < W;
    constexpr int CH = 32;                                    // channels of the gradient
    u32x4 ld[8];
    float *bacc = reinterpret_cast<float *>(lds + GB + 2 * 32 * BW_CSG);   // bias sums [32][S]
    if (isg && has)
#pragma unroll
        for (int e = 0; e < 8; ++e) bacc[(tc8 + e) * S + tkk] = 0.0f;

    auto load = [&](int p) {                                  // plane p of the task's array
        if (!has) return;
        const int yy = isg ? y : y + tr - 1;
        const bool inrow = p >= 0 && p < D && yy >= 0 && yy < H;
        const long long v0 = ((long long)p * H + yy) * W + xj0;
        if (isg) {
            const unsigned o = inrow ? (unsigned)((v0 * CH + tc8) * 2) : NN_OOB;
#pragma unroll
            for (int j = 0; j < 8; ++j) ld[j] = __builtin_amdgcn_raw_buffer_load_b128(rG, o + j * S * CH * 2, 0, 0);
        } else {
            const unsigned o = inrow ? (unsigned)((v0 * CIN + tc8) * 2) : NN_OOB;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool ok = j == 0 ? okl : j == 7 ? okr : true;
                ld[j] = __builtin_amdgcn_raw_buffer_load_b128(rX, ok ? o + j * S * CIN * 2 : NN_OOB, 0, 0);
            }
        }
    };
    auto store = [&](int slot) {                              // transpose into LDS (x slot or g buffer)
        if (!has) return;
        u32x4 t[8];
        bw_transpose(ld, t);
        if (isg) {
            u32x4 *dst = lds + GB + (slot * 32 + tc8) * BW_CSG + tkk;
            float *bs = bacc + tc8 * S + tkk;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                dst[e * BW_CSG] = t[e];
                float s4[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    s4[q] = __uint_as_float(t[e][q] << 16) + __uint_as_float(t[e][q] & 0xffff0000u);
                bs[e * S] += (s4[0] + s4[1]) + (s4[2] + s4[3]);
            }
        } else {
            u32x4 *dst = lds + (slot * CIN + tc8) * BW_CSX + tr * (S + 2) + tkk;
#pragma unroll
            for (int e = 0; e < 8; ++e) dst[e * BW_CSX] = t[e];
        }
    };
    auto slot_of = [&](int p) { return (p - z0 + 1) & 3; };
    auto gbuf_of = [&](int p) { return (p - z0) & 1; };

    // prologue: input planes z0 - 1 .. z0 + 1 and the gradient row of z0 in
    // LDS, the next plane (input z0 + 2, gradient z0 + 1) in registers
    if (isg) {
        load(z0);
        store(0);
    } else {
        for (int p = z0 - 1; p <= z0 + 1; ++p) {
            load(p);
            store(slot_of(p));
            bw_order();
        }
    }
    bw_order();
    if (z0 + 1 < z1) load(isg ? z0 + 1 : z0 + 2);
    __syncthreads();

    const int dz = wave / 3 - 1, dy = wave % 3 - 1;
    f32x16 acc[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) acc[s] = f32x16{};
    const bool lane_x = CIN == 32 || m < CIN;
    const bool row_ok = y + dy >= 0 && y + dy < H;
    for (int z = z0; z < z1; ++z) {
        // the slot of plane z - 2 and the gradient buffer of z - 1 are free
        if (z + 1 < z1) store(isg ? gbuf_of(z + 1) : slot_of(z + 2));
        bw_order();
        if (z + 2 < z1) load(isg ? z + 2 : z + 3);
        const int p = z + dz;
        if (row_ok && p >= 0 && p < D) {                      // uniform over the wave
            const u32x4 *xa = lds + (slot_of(p) * CIN + m) * BW_CSX + (dy + 1) * (S + 2) + kh;
            const u32x4 *ga = lds + GB + (gbuf_of(z) * 32 + m) * BW_CSG + kh;
#pragma unroll
            for (int kb = 0; kb < S; kb += 2) {
                const bf16x8 bv = __builtin_bit_cast(bf16x8, ga[kb]);
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    const bf16x8 av = lane_x ? __builtin_bit_cast(bf16x8, xa[kb + s]) : bf16x8{};
                    acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[s], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    const int nper = 27 * CIN * 32 + 32;
    float *out = partial + (long long)L * nper;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int tap = wave * 3 + s;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int ci = acc_row(q, lane);
            if (ci < CIN) out[(tap * CIN + ci) * 32 + m] = acc[s][q];
        }
    }
    // bias: the gradient tasks' sums, added over k in order (the loop's last
    // barrier has made them visible)
    if (threadIdx.x < 32) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < S; ++k) s += bacc[threadIdx.x * S + k];
        out[27 * CIN * 32 + threadIdx.x] = s;
    }
}

// out[i] = sum over the partials p of partial[p][i]: wave w adds p = w, w + 8,
// ... in order, then the eight wave sums are added pairwise.
__global__ __launch_bounds__(512) void bw_reduce_kernel(const float *__restrict__ partial, int np, int n,
                                                        int ndw, float *__restrict__ dw,
                                                        float *__restrict__ db)
{
    __shared__ float red[8][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (i < n) {
#pragma unroll 8
        for (int p = wave; p < np; p += 8) s += partial[(long long)p * n + i];
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && i < n) {
        const float t = ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane])) +
                        ((red[4][lane] + red[5][lane]) + (red[6][lane] + red[7][lane]));
        if (i < ndw) dw[i] = t;
        else if (db) db[i - ndw] = t;
    }
}

// Workgroup layout of the weight gradient: x tiles of TX = 128, 64, 32 or 16
// voxels (the largest dividing W), rows (y, x tile), and chunks of z planes
// so that about 256 workgroups (one per compute unit) run.
struct BwPlan {
    int S, ntx, planes, nwg;
};
BwPlan bw_plan(int D, int H, int W)
{
    BwPlan p{};
    const int tx = W % 128 == 0 ? 128 : W % 64 == 0 ? 64 : W % 32 == 0 ? 32 : 16;
    p.S = tx / 8;
    p.ntx = W / tx;
    const long long rows = (long long)H * p.ntx;
    long long zc = (256 + rows - 1) / rows;
    zc = zc < 1 ? 1 : zc > D ? D : zc;
    p.planes = (int)((D + zc - 1) / zc);
    zc = (D + p.planes - 1) / p.planes;
    p.nwg = (int)(rows * zc);
    return p;
}

// One thread per (voxel, group of 8 channels): 16-byte loads and store.
__global__ void relu_grad_kernel(const uint16_t *__restrict__ dy, const uint16_t *__restrict__ y,
                                 long long V, uint16_t *__restrict__ g)
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

// One instantiation per (cin, S); the LDS opt-in above 64 KiB is made once
// per instantiation.
template <int CIN, int S>
int bw_launch_s(const BwPlan &p, const uint16_t *x, const uint16_t *g, int D, int H, int W, float *work,
                hipStream_t st)
{
    // (a function-local static: initialised once, thread-safely)
    static const hipError_t cfg = hipFuncSetAttribute((const void *)conv_bwdw_kernel<CIN, S>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      bw_lds_bytes<CIN>());
    if (cfg != hipSuccess)
        return art_set_error(ART_E_HIP, (std::string("art_conv3d_bwd_weight: ") + hipGetErrorString(cfg)).c_str());
    hipLaunchKernelGGL((conv_bwdw_kernel<CIN, S>), dim3(p.nwg), dim3(BW_THREADS), bw_lds_bytes<CIN>(), st, x, g, D,
                       H, W, p.ntx, p.planes, p.nwg, (int)(p.nwg % 8 == 0), work);
    return ART_OK;
}

template <int CIN>
int bw_launch(const BwPlan &p, const uint16_t *x, const uint16_t *g, int D, int H, int W, float *work,
              hipStream_t st)
{
    switch (p.S) {
    case 2: return bw_launch_s<CIN, 2>(p, x, g, D, H, W, work, st);
    case 4: return bw_launch_s<CIN, 4>(p, x, g, D, H, W, work, st);
    case 8: return bw_launch_s<CIN, 8>(p, x, g, D, H, W, work, st);
    default: return bw_launch_s<CIN, 16>(p, x, g, D, H, W, work, st);
    }
}

__global__ void art_fill_u32_kernel_entry(unsigned int *p) { *p = 0u; }

}  // namespace

extern "C" {

int art_conv3d_fwd(const void *x, int cin, const void *w_k, const float *bias, int D, int H,
                   int W, int relu, const void *mask, void *y, float *y0, void *hip_stream)
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
    // the dynamic LDS opt-in, once (a function-local static initialises thread-safely)
    static const hipError_t cfg = [] {
        hipError_t e = hipFuncSetAttribute((const void *)conv_fwd_kernel<16>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, conv_lds_bytes<16>());
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)conv_fwd_kernel<32>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, conv_lds_bytes<32>());
        return e;
    }();
    if (cfg != hipSuccess)
        return art_set_error(ART_E_HIP, (std::string("art_conv3d_fwd: ") + hipGetErrorString(cfg)).c_str());
    if (cin == 16)
        hipLaunchKernelGGL(conv_fwd_kernel<16>, dim3((unsigned)tiles), dim3(512), conv_lds_bytes<16>(), st,
                           xp, wp, bias, D, H, W, relu, (const uint16_t *)mask, (uint16_t *)y, y0);
    else
        hipLaunchKernelGGL(conv_fwd_kernel<32>, dim3((unsigned)tiles), dim3(512), conv_lds_bytes<32>(), st,
                           xp, wp, bias, D, H, W, relu, (const uint16_t *)mask, (uint16_t *)y, y0);
    return launch_status("art_conv3d_fwd");
}

long long art_conv3d_bwd_weight_workspace(int cin, int D, int H, int W)
{
    if ((cin != 16 && cin != 32) || D < 1 || H < 1 || W < 16 || W % 16) return -1;
    const BwPlan p = bw_plan(D, H, W);
    return (long long)p.nwg * (27 * cin * 32 + 32);
}

int art_conv3d_bwd_weight(const void *x, int cin, const void *g, int D, int H, int W, float *work,
                          long long work_floats, float *dw, float *db, void *hip_stream)
{
    if (!x || !g || !work || !dw) return art_set_error(ART_E_INVAL, "art_conv3d_bwd_weight: null pointer");
    if (cin != 16 && cin != 32) return art_set_error(ART_E_INVAL, "art_conv3d_bwd_weight: cin must be 16 or 32");
    if (D < 1 || H < 1 || W < 16 || W % 16)
        return art_set_error(ART_E_INVAL, "art_conv3d_bwd_weight: W must be a positive multiple of 16");
    if ((long long)D * H * W * 64 >= (1ll << 31))
        return art_set_error(ART_E_UNSUPPORTED, "art_conv3d_bwd_weight: gradient tensor above 2 GiB");
    const BwPlan p = bw_plan(D, H, W);
    const int n = 27 * cin * 32 + 32;
    if (work_floats < (long long)p.nwg * n)
        return art_set_error(ART_E_INVAL, "art_conv3d_bwd_weight: workspace smaller than "
                                          "art_conv3d_bwd_weight_workspace()");
    hipStream_t st = (hipStream_t)hip_stream;
    const auto *xp = (const uint16_t *)x;
    const auto *gp = (const uint16_t *)g;
    int rc = cin == 16 ? bw_launch<16>(p, xp, gp, D, H, W, work, st) : bw_launch<32>(p, xp, gp, D, H, W, work, st);
    if (rc) return rc;
    rc = launch_status("art_conv3d_bwd_weight");
    if (rc) return rc;
    hipLaunchKernelGGL(bw_reduce_kernel, dim3(blocks_for(n, 64)), dim3(512), 0, st, work, p.nwg, n,
                       27 * cin * 32, dw, db);
    return launch_status("art_conv3d_bwd_weight (sum)");
}

int art_nn_relu_grad(const void *dy, const void *y, int V, void *g, void *hip_stream)
{
    if (!dy || !g || V < 1) return art_set_error(ART_E_INVAL, "art_nn_relu_grad: bad arguments");
    hipLaunchKernelGGL(relu_grad_kernel, dim3(blocks_for(4ll * V, 256)), dim3(256), 0, (hipStream_t)hip_stream,
                       (const uint16_t *)dy, (const uint16_t *)y, (long long)V, (uint16_t *)g);
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
