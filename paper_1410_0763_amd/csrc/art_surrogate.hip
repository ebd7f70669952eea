// art_surrogate.hip -- the learned surrogate of the fine sweep as a library
// object (include/art_surrogate.h).  This file owns the parameters, AdamW
// state and work buffers and sequences the layer kernels of art_conv.hip:
//
//   forward:   x -> conv(16->32)+ReLU -> 4 x conv(32->32)+ReLU -> conv(32->1) = p
//   backward:  loss gradient at p; per layer from the last: ReLU mask, the
//              shifted input copies, weight and bias gradients, and (except
//              for the first layer) the input gradient as a forward
//              convolution with mirrored taps and swapped channels
//   update:    AdamW on every weight and bias
//
// The gate of art_sweep_surrogate and the checkpoint format are host code
// here; the SHA-256 digest follows FIPS 180-4, with its round constants and
// initial hash derived from the primes as the standard defines them (integer
// cube and square roots), not tabulated.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/art.h"
#include "../../include/art_nn.h"
#include "../../include/art_surrogate.h"
#include "art_internal.h"

namespace {

constexpr int NL = 6;
constexpr int CIN[NL] = {16, 32, 32, 32, 32, 32};      // input channels as stored
constexpr int REAL_IN[NL] = {3, 32, 32, 32, 32, 32};   // channels that carry data
constexpr int REAL_OUT[NL] = {32, 32, 32, 32, 32, 1};
constexpr int RELU[NL] = {1, 1, 1, 1, 1, 0};
constexpr long long MAX_CELLS = 11184810;              // 3 * 32 * 2 bytes per cell < 2 GiB
constexpr char MAGIC[8] = {'A', 'R', 'T', 'S', 'G', 'C', 'K', '2'};   // features (log J, log n, x_HI)

int wcount(int l) { return 27 * CIN[l] * 32; }

int sg_fail(int code, const std::string &msg) { return art_set_error(code, msg.c_str()); }

#define SGCHK(expr)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return sg_fail(e_ == hipErrorOutOfMemory ? ART_E_NOMEM : ART_E_HIP,                  \
                           std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    } while (0)

#define RCCHK(expr)                                                                              \
    do {                                                                                         \
        int rc_ = (expr);                                                                        \
        if (rc_ != ART_OK) return rc_;                                                           \
    } while (0)

// ---------------------------------------------------------------- kernels

// Outputs of an accepted prediction: J_in = J_in,coarse e^p, J = J_in + S.
__global__ __launch_bounds__(256) void finish_kernel(const float *__restrict__ pred,
                                                     const float *__restrict__ Jinc,
                                                     const float *__restrict__ Jc,
                                                     const float *__restrict__ Jexc,
                                                     const float2 *__restrict__ rec, int nb,
                                                     float g0, float h_in, float h_src, long long V,
                                                     float *__restrict__ J,
                                                     float *__restrict__ J_in,
                                                     float *__restrict__ J_exact,
                                                     float *__restrict__ Gamma,
                                                     float *__restrict__ Heat)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float jin = Jinc[v] * expf(pred[v]), s = rec[v * nb].y;
    const float j = jin + s;
    if (J) J[v] = j;
    if (J_in) J_in[v] = jin;
    if (Heat) Heat[v] = fmaf(h_in, jin, h_src * s);
    if (J_exact) J_exact[v] = j + (Jexc[v] - Jc[v]);
    if (Gamma) Gamma[v] = g0 * j;
}

// Per-block sums, sums of squares (double), minima and maxima of the three
// raw features; out[block][k][4].
constexpr int STAT_BLOCKS = 256;
__global__ __launch_bounds__(256) void stats_kernel(const float *__restrict__ J,
                                                    const float *__restrict__ dens,
                                                    const float *__restrict__ xhi, long long V,
                                                    double *__restrict__ out)
{
    __shared__ double s1[3][256], s2[3][256];
    __shared__ float mn[3][256], mx[3][256];
    const int t = threadIdx.x;
    double a1[3] = {0.0, 0.0, 0.0}, a2[3] = {0.0, 0.0, 0.0};
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long long v = (long long)blockIdx.x * 256 + t; v < V; v += (long long)gridDim.x * 256) {
        const float f[3] = {J[v], dens[v], xhi[v]};
        for (int k = 0; k < 3; ++k) {
            const float l = art_feature_raw(k, f[k]);
            a1[k] += l;
            a2[k] += (double)l * l;
            lo[k] = fminf(lo[k], l);
            hi[k] = fmaxf(hi[k], l);
        }
    }
    for (int k = 0; k < 3; ++k) {
        s1[k][t] = a1[k];
        s2[k][t] = a2[k];
        mn[k][t] = lo[k];
        mx[k][t] = hi[k];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 3; ++k) {
                s1[k][t] += s1[k][t + w];
                s2[k][t] += s2[k][t + w];
                mn[k][t] = fminf(mn[k][t], mn[k][t + w]);
                mx[k][t] = fmaxf(mx[k][t], mx[k][t + w]);
            }
        __syncthreads();
    }
    if (t < 3) {
        double *o = out + ((long long)blockIdx.x * 3 + t) * 4;
        o[0] = s1[t][0];
        o[1] = s2[t][0];
        o[2] = mn[t][0];
        o[3] = mx[t][0];
    }
}

unsigned blocks_for(long long n, int per) { return (unsigned)((n + per - 1) / per); }

int launch_status(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return ART_OK;
    return sg_fail(ART_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- SHA-256

struct ShaConst {
    uint32_t k[64], h0[8];
    ShaConst()
    {
        int primes[64], n = 0;
        for (int p = 2; n < 64; ++p) {
            bool prime = true;
            for (int q = 2; q * q <= p; ++q)
                if (p % q == 0) { prime = false; break; }
            if (prime) primes[n++] = p;
        }
        typedef unsigned __int128 u128;
        for (int i = 0; i < 64; ++i) {
            // floor(cbrt(p) 2^32) = largest x with x^3 <= p 2^96; keep its low 32 bits
            const u128 target = (u128)primes[i] << 96;
            uint64_t lo = 0, hi = 1ull << 40;
            while (lo < hi) {
                const uint64_t mid = lo + (hi - lo + 1) / 2;
                if ((u128)mid * mid * mid <= target) lo = mid; else hi = mid - 1;
            }
            k[i] = (uint32_t)lo;
        }
        for (int i = 0; i < 8; ++i) {
            const u128 target = (u128)primes[i] << 64;   // floor(sqrt(p) 2^32)
            uint64_t lo = 0, hi = 1ull << 36;
            while (lo < hi) {
                const uint64_t mid = lo + (hi - lo + 1) / 2;
                if ((u128)mid * mid <= target) lo = mid; else hi = mid - 1;
            }
            h0[i] = (uint32_t)lo;
        }
    }
};

const ShaConst &sha_const()
{
    static const ShaConst c;
    return c;
}

inline uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

void sha_block(uint32_t h[8], const unsigned char *blk)
{
    const ShaConst &C = sha_const();
    uint32_t w[64];
    for (int t = 0; t < 16; ++t)
        w[t] = (uint32_t)blk[4 * t] << 24 | (uint32_t)blk[4 * t + 1] << 16 |
               (uint32_t)blk[4 * t + 2] << 8 | (uint32_t)blk[4 * t + 3];
    for (int t = 16; t < 64; ++t) {
        const uint32_t s0 = rotr(w[t - 15], 7) ^ rotr(w[t - 15], 18) ^ (w[t - 15] >> 3);
        const uint32_t s1 = rotr(w[t - 2], 17) ^ rotr(w[t - 2], 19) ^ (w[t - 2] >> 10);
        w[t] = s1 + w[t - 7] + s0 + w[t - 16];
    }
    uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
    for (int t = 0; t < 64; ++t) {
        const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
        const uint32_t ch = (e & f) ^ (~e & g);
        const uint32_t t1 = hh + S1 + ch + C.k[t] + w[t];
        const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
        const uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
        const uint32_t t2 = S0 + maj;
        hh = g; g = f; f = e; e = d + t1; d = c; c = b; b = a; a = t1 + t2;
    }
    h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
}

void sha256(const unsigned char *p, unsigned long long n, unsigned char out[32])
{
    uint32_t h[8];
    std::memcpy(h, sha_const().h0, sizeof h);
    unsigned long long i = 0;
    for (; i + 64 <= n; i += 64) sha_block(h, p + i);
    // padding: 0x80, zeros to 56 mod 64, then the bit length (big-endian)
    unsigned char tail[128] = {};
    const unsigned rem = (unsigned)(n - i);
    if (rem) std::memcpy(tail, p + i, rem);
    tail[rem] = 0x80;
    const unsigned len = rem + 1 + 8 <= 64 ? 64 : 128;
    const unsigned long long bits = n * 8ull;
    for (int b = 0; b < 8; ++b) tail[len - 1 - b] = (unsigned char)(bits >> (8 * b));
    for (unsigned o = 0; o < len; o += 64) sha_block(h, tail + o);
    for (int k = 0; k < 8; ++k)
        for (int b = 0; b < 4; ++b) out[4 * k + b] = (unsigned char)(h[k] >> (24 - 8 * b));
}

// ---------------------------------------------------------------- generator

// splitmix64 stream; normals by the Box-Muller transform.
struct Gen {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 1) * (1.0 / 9007199254740993.0); }   // (0, 1)
    bool have = false;
    double spare = 0.0;
    double normal()
    {
        if (have) { have = false; return spare; }
        const double r = std::sqrt(-2.0 * std::log(uniform())), th = 6.283185307179586 * uniform();
        spare = r * std::sin(th);
        have = true;
        return r * std::cos(th);
    }
};

}  // namespace

struct art_surrogate {
    int D = 0, H = 0, W = 0;
    long long V = 0;
    long long nwork = 0;
    int step = 0;
    float mu[3] = {0, 0, 0}, sd[3] = {1, 1, 1};
    float lo[3] = {-INFINITY, -INFINITY, -INFINITY}, hi[3] = {INFINITY, INFINITY, INFINITY};
    float val_err = NAN;
    bool prepped = false;
    float *w[NL] = {}, *b[NL] = {}, *mw[NL] = {}, *vw[NL] = {}, *mb[NL] = {}, *vb[NL] = {};
    float *dw[NL] = {}, *db[NL] = {};
    uint16_t *w_fwd[NL] = {}, *w_bwd[NL] = {};
    uint16_t *acts[NL - 1] = {}, *dy[2] = {}, *x = nullptr;
    float *pred = nullptr, *work = nullptr, *mpart = nullptr,
          *wpart = nullptr, *loss = nullptr;
    float *Jc = nullptr, *Jexc = nullptr, *Jinc = nullptr, *Jf = nullptr, *Jinf = nullptr;
    unsigned *count = nullptr;
    double *spart = nullptr;
    std::vector<void *> mem;
};

namespace {

template <class T>
int sg_alloc(art_surrogate *s, T **p, size_t count)
{
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess)
        return sg_fail(ART_E_NOMEM, "art_surrogate_create: hipMalloc of " +
                                        std::to_string(count * sizeof(T)) + " bytes: " +
                                        hipGetErrorString(e));
    s->mem.push_back(q);
    *p = (T *)q;
    SGCHK(hipMemset(q, 0, count * sizeof(T)));
    return ART_OK;
}

void release(art_surrogate *s)
{
    for (void *p : s->mem) (void)hipFree(p);
    s->mem.clear();
}

int prep(art_surrogate *s, hipStream_t st)
{
    if (s->prepped) return ART_OK;
    for (int l = 0; l < NL; ++l) RCCHK(art_nn_prep_weights(s->w[l], CIN[l], s->w_fwd[l], s->w_bwd[l], st));
    s->prepped = true;
    return ART_OK;
}

int forward(art_surrogate *s, const void *x, hipStream_t st)
{
    RCCHK(prep(s, st));
    for (int l = 0; l < NL; ++l) {
        const void *xin = l == 0 ? x : s->acts[l - 1];
        RCCHK(art_conv3d_fwd(xin, CIN[l], s->w_fwd[l], s->b[l], s->D, s->H, s->W, RELU[l], nullptr,
                             l < NL - 1 ? s->acts[l] : nullptr, l == NL - 1 ? s->pred : nullptr, st));
    }
    return ART_OK;
}

int check_mesh(const art_surrogate *s, const art_mesh *mesh, const float2 **rec, int *nb, double *h,
               const char *who)
{
    int dims[3];
    art_mesh_fields(mesh, dims, nb, h, rec);
    if (dims[0] != s->W || dims[1] != s->H || dims[2] != s->D)
        return sg_fail(ART_E_INVAL, std::string(who) + ": mesh shape differs from the surrogate's");
    if (!*rec) return sg_fail(ART_E_STATE, std::string(who) + ": mesh has no fields");
    if (*nb != 1) return sg_fail(ART_E_UNSUPPORTED, std::string(who) + ": the surrogate covers one bin");
    return ART_OK;
}

void put(std::vector<unsigned char> &b, const void *p, size_t n)
{
    const unsigned char *c = (const unsigned char *)p;
    b.insert(b.end(), c, c + n);
}

}  // namespace

extern "C" {

int art_surrogate_create(int nx, int ny, int nz, unsigned long long seed, art_surrogate **out)
{
    if (!out) return sg_fail(ART_E_INVAL, "art_surrogate_create: out is NULL");
    *out = nullptr;
    if (nx < 32 || nx % 32 || ny < 1 || nz < 1)
        return sg_fail(ART_E_INVAL, "art_surrogate_create: nx must be a positive multiple of 32, ny, nz >= 1");
    const long long V = (long long)nx * ny * nz;
    if (V > MAX_CELLS)
        return sg_fail(ART_E_UNSUPPORTED, "art_surrogate_create: more than 11184810 cells");
    art_surrogate *s = new (std::nothrow) art_surrogate;
    if (!s) return sg_fail(ART_E_NOMEM, "art_surrogate_create: host allocation");
    s->D = nz;
    s->H = ny;
    s->W = nx;
    s->V = V;
    s->nwork = art_conv3d_bwd_weight_workspace(32, nz, ny, nx);   // covers cin = 16 too
    int rc = ART_OK;
    auto A = [&](auto **p, size_t n) {
        if (rc == ART_OK) rc = sg_alloc(s, p, n);
    };
    for (int l = 0; l < NL; ++l) {
        A(&s->w[l], wcount(l)); A(&s->mw[l], wcount(l)); A(&s->vw[l], wcount(l)); A(&s->dw[l], wcount(l));
        A(&s->b[l], 32); A(&s->mb[l], 32); A(&s->vb[l], 32); A(&s->db[l], 32);
        A(&s->w_fwd[l], 27 * 32 * CIN[l]);
        A(&s->w_bwd[l], 27 * 32 * 32);
    }
    for (int l = 0; l < NL - 1; ++l) A(&s->acts[l], V * 32);
    A(&s->dy[0], V * 32); A(&s->dy[1], V * 32);
    A(&s->x, V * 16);
    A(&s->pred, V); A(&s->Jc, V); A(&s->Jexc, V); A(&s->Jinc, V); A(&s->Jf, V); A(&s->Jinf, V);
    A(&s->work, (size_t)s->nwork);
    A(&s->mpart, 256); A(&s->wpart, 257); A(&s->loss, 1); A(&s->count, 1);
    A(&s->spart, (size_t)STAT_BLOCKS * 12);
    if (rc == ART_OK) {
        Gen gen{seed * 0x2545f4914f6cdd1dull + 0x1234567ull};
        for (int l = 0; l < NL && rc == ART_OK; ++l) {
            std::vector<float> h((size_t)wcount(l), 0.0f);
            const double sdev = l < NL - 1 ? std::sqrt(2.0 / (27.0 * REAL_IN[l])) : 1e-3;
            for (int t = 0; t < 27; ++t)
                for (int ci = 0; ci < REAL_IN[l]; ++ci)
                    for (int co = 0; co < REAL_OUT[l]; ++co)
                        h[((size_t)t * CIN[l] + ci) * 32 + co] = (float)(sdev * gen.normal());
            const hipError_t e = hipMemcpy(s->w[l], h.data(), h.size() * 4, hipMemcpyHostToDevice);
            if (e != hipSuccess) rc = sg_fail(ART_E_HIP, std::string("art_surrogate_create: ") + hipGetErrorString(e));
        }
    }
    if (rc != ART_OK) {
        release(s);
        delete s;
        return rc;
    }
    *out = s;
    return ART_OK;
}

int art_surrogate_destroy(art_surrogate *s)
{
    if (!s) return ART_OK;
    (void)hipDeviceSynchronize();
    release(s);
    delete s;
    return ART_OK;
}

int art_surrogate_n_params(const art_surrogate *s)
{
    if (!s) return sg_fail(ART_E_INVAL, "art_surrogate_n_params: NULL surrogate");
    int n = 0;
    for (int l = 0; l < NL; ++l) n += 27 * REAL_IN[l] * REAL_OUT[l] + REAL_OUT[l];
    return n;
}

int art_surrogate_set_stats(art_surrogate *s, const float *mu, const float *sd, const float *lo,
                            const float *hi, float val_err)
{
    if (!s || !mu || !sd || !lo || !hi) return sg_fail(ART_E_INVAL, "art_surrogate_set_stats: NULL argument");
    for (int k = 0; k < 3; ++k)
        if (!(sd[k] > 0.0f) || !std::isfinite(sd[k]) || !std::isfinite(mu[k]) || std::isnan(lo[k]) ||
            std::isnan(hi[k]))
            return sg_fail(ART_E_INVAL, "art_surrogate_set_stats: sd must be positive and finite, mu finite");
    for (int k = 0; k < 3; ++k) {
        s->mu[k] = mu[k];
        s->sd[k] = sd[k];
        s->lo[k] = lo[k];
        s->hi[k] = hi[k];
    }
    s->val_err = val_err >= 0.0f ? val_err : NAN;
    return ART_OK;
}

int art_surrogate_get_stats(const art_surrogate *s, float *mu, float *sd, float *lo, float *hi,
                            float *val_err)
{
    if (!s) return sg_fail(ART_E_INVAL, "art_surrogate_get_stats: NULL surrogate");
    for (int k = 0; k < 3; ++k) {
        if (mu) mu[k] = s->mu[k];
        if (sd) sd[k] = s->sd[k];
        if (lo) lo[k] = s->lo[k];
        if (hi) hi[k] = s->hi[k];
    }
    if (val_err) *val_err = s->val_err;
    return ART_OK;
}

int art_surrogate_fit_stats(art_surrogate *s, int n, const float *const *J_coarse,
                            const float *const *density, const float *const *x_hi, float margin,
                            void *hip_stream)
{
    if (!s || n < 1 || !J_coarse || !density || !x_hi || !(margin >= 0.0f))
        return sg_fail(ART_E_INVAL, "art_surrogate_fit_stats: bad arguments");
    for (int i = 0; i < n; ++i)
        if (!J_coarse[i] || !density[i] || !x_hi[i])
            return sg_fail(ART_E_INVAL, "art_surrogate_fit_stats: NULL field");
    hipStream_t st = (hipStream_t)hip_stream;
    double sum[3] = {0, 0, 0}, sq[3] = {0, 0, 0};
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    std::vector<double> h((size_t)STAT_BLOCKS * 12);
    for (int i = 0; i < n; ++i) {
        hipLaunchKernelGGL(stats_kernel, dim3(STAT_BLOCKS), dim3(256), 0, st, J_coarse[i], density[i],
                           x_hi[i], s->V, s->spart);
        RCCHK(launch_status("art_surrogate_fit_stats"));
        SGCHK(hipMemcpyAsync(h.data(), s->spart, h.size() * 8, hipMemcpyDeviceToHost, st));
        SGCHK(hipStreamSynchronize(st));
        for (int b = 0; b < STAT_BLOCKS; ++b)
            for (int k = 0; k < 3; ++k) {
                const double *o = &h[((size_t)b * 3 + k) * 4];
                sum[k] += o[0];
                sq[k] += o[1];
                mn[k] = std::fmin(mn[k], o[2]);
                mx[k] = std::fmax(mx[k], o[3]);
            }
    }
    const double N = (double)n * (double)s->V;
    float mu[3], sd[3], lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        const double m = sum[k] / N;
        const double var = std::fmax(sq[k] / N - m * m, 0.0);
        double d = std::sqrt(var);
        if (!(d > 1e-12)) d = 1.0;    // a constant feature: no scaling
        mu[k] = (float)m;
        sd[k] = (float)d;
        lo[k] = (float)((mn[k] - m) / d - margin);
        hi[k] = (float)((mx[k] - m) / d + margin);
    }
    const float ve = s->val_err;
    RCCHK(art_surrogate_set_stats(s, mu, sd, lo, hi, 0.0f));
    s->val_err = ve;
    return ART_OK;
}

int art_surrogate_features(const art_surrogate *s, const float *J_coarse, const float *density,
                           const float *x_hi, void *x, void *hip_stream)
{
    if (!s || !J_coarse || !density || !x_hi || !x)
        return sg_fail(ART_E_INVAL, "art_surrogate_features: NULL argument");
    const float isd[3] = {1.0f / s->sd[0], 1.0f / s->sd[1], 1.0f / s->sd[2]};
    return art_nn_features(J_coarse, density, x_hi, (int)s->V, s->mu, isd, x, hip_stream);
}

int art_surrogate_make_pair(art_surrogate *s, art_mesh *mesh, int nside_coarse, int nside_fine,
                            float lambda, float *target, float *weight, float *J_coarse,
                            float *J_fine, void *hip_stream)
{
    if (!s || !mesh || !target || !J_coarse || !(lambda >= 0.0f))
        return sg_fail(ART_E_INVAL, "art_surrogate_make_pair: bad arguments");
    const float2 *rec;
    int nb;
    double h;
    RCCHK(check_mesh(s, mesh, &rec, &nb, &h, "art_surrogate_make_pair"));
    art_outputs oc{}, of{};
    oc.J = J_coarse;
    oc.J_in = s->Jinc;
    of.J = J_fine ? J_fine : s->Jf;
    of.J_in = s->Jinf;
    RCCHK(art_sweep(mesh, nside_coarse, nullptr, 0.0f, &oc, hip_stream));
    RCCHK(art_sweep(mesh, nside_fine, nullptr, 0.0f, &of, hip_stream));
    RCCHK(art_nn_log_ratio(s->Jinf, s->Jinc, (int)s->V, target, hip_stream));
    if (weight) RCCHK(art_nn_sq_weights(s->Jinc, (int)s->V, lambda, s->wpart, weight, hip_stream));
    return ART_OK;
}

int art_surrogate_gradients(art_surrogate *s, const void *x, const float *target,
                            const float *weight, float *loss, void *hip_stream)
{
    if (!s || !x || !target) return sg_fail(ART_E_INVAL, "art_surrogate_gradients: NULL argument");
    hipStream_t st = (hipStream_t)hip_stream;
    const int V = (int)s->V;
    RCCHK(forward(s, x, st));
    RCCHK(art_nn_mse(s->pred, target, weight, V, s->mpart, loss ? loss : s->loss, s->dy[0], st));
    // dy[cur] holds the gradient at layer l's pre-activation output: the loss
    // gradient for the last layer (no ReLU), else the input gradient of
    // layer l + 1 with layer l's ReLU mask applied by the convolution itself
    int cur = 0;
    for (int l = NL - 1; l >= 0; --l) {
        const void *xin = l == 0 ? x : s->acts[l - 1];
        RCCHK(art_conv3d_bwd_weight(xin, CIN[l], s->dy[cur], s->D, s->H, s->W, s->work, s->nwork,
                                    s->dw[l], s->db[l], st));
        if (l > 0) {
            RCCHK(art_conv3d_fwd(s->dy[cur], 32, s->w_bwd[l], nullptr, s->D, s->H, s->W, 0, s->acts[l - 1],
                                 s->dy[1 - cur], nullptr, st));
            cur = 1 - cur;
        }
    }
    return ART_OK;
}

int art_surrogate_train_step(art_surrogate *s, const void *x, const float *target,
                             const float *weight, float lr, float wd, float *loss,
                             void *hip_stream)
{
    if (!s || !(lr > 0.0f) || !(wd >= 0.0f)) return sg_fail(ART_E_INVAL, "art_surrogate_train_step: bad arguments");
    RCCHK(art_surrogate_gradients(s, x, target, weight, loss, hip_stream));
    const int step = s->step + 1;
    for (int l = 0; l < NL; ++l) {
        RCCHK(art_nn_adamw(s->w[l], s->dw[l], s->mw[l], s->vw[l], wcount(l), lr, 0.9f, 0.999f, 1e-8f, wd,
                           step, hip_stream));
        RCCHK(art_nn_adamw(s->b[l], s->db[l], s->mb[l], s->vb[l], 32, lr, 0.9f, 0.999f, 1e-8f, 0.0f,
                           step, hip_stream));
    }
    s->step = step;
    s->prepped = false;
    return ART_OK;
}

int art_surrogate_infer(art_surrogate *s, const void *x, float *pred, void *hip_stream)
{
    if (!s || !x || !pred) return sg_fail(ART_E_INVAL, "art_surrogate_infer: NULL argument");
    hipStream_t st = (hipStream_t)hip_stream;
    RCCHK(forward(s, x, st));
    SGCHK(hipMemcpyAsync(pred, s->pred, s->V * 4, hipMemcpyDeviceToDevice, st));
    return ART_OK;
}

int art_surrogate_param(art_surrogate *s, int layer, int what, float *buf, int write,
                        void *hip_stream)
{
    if (!s || !buf || layer < 0 || layer >= NL || what < ART_SG_W || what > ART_SG_DB)
        return sg_fail(ART_E_INVAL, "art_surrogate_param: bad arguments");
    if (write && what != ART_SG_W && what != ART_SG_B)
        return sg_fail(ART_E_INVAL, "art_surrogate_param: only weights and biases can be written");
    float *arr[4] = {s->w[layer], s->b[layer], s->dw[layer], s->db[layer]};
    const size_t n = (what == ART_SG_W || what == ART_SG_DW) ? (size_t)wcount(layer) : 32;
    hipStream_t st = (hipStream_t)hip_stream;
    if (write) {
        SGCHK(hipMemcpyAsync(arr[what], buf, n * 4, hipMemcpyDeviceToDevice, st));
        s->prepped = false;
    } else {
        SGCHK(hipMemcpyAsync(buf, arr[what], n * 4, hipMemcpyDeviceToDevice, st));
    }
    return ART_OK;
}

int art_surrogate_save(art_surrogate *s, const char *path, void *hip_stream)
{
    if (!s || !path) return sg_fail(ART_E_INVAL, "art_surrogate_save: NULL argument");
    SGCHK(hipStreamSynchronize((hipStream_t)hip_stream));
    std::vector<unsigned char> body;
    const int32_t head[4] = {s->D, s->H, s->W, s->step};
    put(body, head, sizeof head);
    put(body, s->mu, 12); put(body, s->sd, 12); put(body, s->lo, 12); put(body, s->hi, 12);
    put(body, &s->val_err, 4);
    for (float **group : {s->w, s->b, s->mw, s->vw, s->mb, s->vb})
        for (int l = 0; l < NL; ++l) {
            const size_t n = (group == s->w || group == s->mw || group == s->vw) ? (size_t)wcount(l) : 32;
            std::vector<float> h(n);
            SGCHK(hipMemcpy(h.data(), group[l], n * 4, hipMemcpyDeviceToHost));
            put(body, h.data(), n * 4);
        }
    unsigned char dig[32];
    sha256(body.data(), body.size(), dig);
    FILE *f = std::fopen(path, "wb");
    if (!f) return sg_fail(ART_E_INVAL, std::string("art_surrogate_save: cannot open ") + path);
    bool ok = std::fwrite(MAGIC, 1, 8, f) == 8 && std::fwrite(dig, 1, 32, f) == 32 &&
              std::fwrite(body.data(), 1, body.size(), f) == body.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return sg_fail(ART_E_INVAL, std::string("art_surrogate_save: write failed: ") + path);
    return ART_OK;
}

int art_surrogate_load(art_surrogate *s, const char *path, void *hip_stream)
{
    if (!s || !path) return sg_fail(ART_E_INVAL, "art_surrogate_load: NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return sg_fail(ART_E_INVAL, std::string("art_surrogate_load: cannot open ") + path);
    std::vector<unsigned char> data;
    unsigned char buf[65536];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) data.insert(data.end(), buf, buf + got);
    std::fclose(f);
    size_t payload = 0;
    for (int l = 0; l < NL; ++l) payload += 3 * (size_t)wcount(l) + 3 * 32;
    const size_t body_len = 16 + 4 * 13 + payload * 4;
    if (data.size() < 40 || std::memcmp(data.data(), MAGIC, 8) != 0)
        return sg_fail(ART_E_INVAL, "art_surrogate_load: not a surrogate checkpoint");
    if (data.size() != 40 + body_len)
        return sg_fail(ART_E_INVAL, "art_surrogate_load: checkpoint size does not match the network");
    unsigned char dig[32];
    sha256(data.data() + 40, body_len, dig);
    if (std::memcmp(dig, data.data() + 8, 32) != 0)
        return sg_fail(ART_E_INVAL, "art_surrogate_load: checksum mismatch");
    const unsigned char *p = data.data() + 40;
    int32_t head[4];
    std::memcpy(head, p, 16);
    if (head[0] != s->D || head[1] != s->H || head[2] != s->W)
        return sg_fail(ART_E_INVAL, "art_surrogate_load: mesh shape differs");
    SGCHK(hipStreamSynchronize((hipStream_t)hip_stream));
    const unsigned char *q = p + 16 + 4 * 13;
    for (float **group : {s->w, s->b, s->mw, s->vw, s->mb, s->vb})
        for (int l = 0; l < NL; ++l) {
            const size_t n = (group == s->w || group == s->mw || group == s->vw) ? (size_t)wcount(l) : 32;
            SGCHK(hipMemcpy(group[l], q, n * 4, hipMemcpyHostToDevice));
            q += n * 4;
        }
    s->step = head[3];
    std::memcpy(s->mu, p + 16, 12);
    std::memcpy(s->sd, p + 28, 12);
    std::memcpy(s->lo, p + 40, 12);
    std::memcpy(s->hi, p + 52, 12);
    std::memcpy(&s->val_err, p + 64, 4);
    s->prepped = false;
    return ART_OK;
}

int art_sweep_surrogate(art_mesh *mesh, art_surrogate *s, const float *density, const float *x_hi,
                        int nside_coarse, int nside_fine, const float *gamma_w, float err_bound,
                        const art_outputs *out, int *used_fallback, float *est_err, void *hip_stream)
{
    if (!mesh || !s || !out || !density || !x_hi)
        return sg_fail(ART_E_INVAL, "art_sweep_surrogate: NULL argument");
    if (out->exit_sum) return sg_fail(ART_E_INVAL, "art_sweep_surrogate: exit sums are not produced");
    if (gamma_w && !std::isfinite(gamma_w[0])) return sg_fail(ART_E_INVAL, "art_sweep_surrogate: gamma_w not finite");
    const float2 *rec;
    int nb;
    double h;
    RCCHK(check_mesh(s, mesh, &rec, &nb, &h, "art_sweep_surrogate"));
    hipStream_t st = (hipStream_t)hip_stream;
    const long long V = s->V;
    art_outputs oc{};
    oc.J = s->Jc;
    oc.J_in = s->Jinc;
    oc.J_exact = s->Jexc;
    RCCHK(art_sweep(mesh, nside_coarse, gamma_w, 0.0f, &oc, hip_stream));
    RCCHK(art_surrogate_features(s, s->Jc, density, x_hi, s->x, hip_stream));
    RCCHK(art_nn_ood_count(s->x, (int)V, s->lo, s->hi, s->count, hip_stream));
    RCCHK(forward(s, s->x, st));
    unsigned nout = 0;
    SGCHK(hipMemcpyAsync(&nout, s->count, 4, hipMemcpyDeviceToHost, st));
    SGCHK(hipStreamSynchronize(st));
    const float est = s->val_err + (float)((double)nout / (double)V);   // NaN if val_err unknown
    const bool accept = err_bound > 0.0f && est <= err_bound;
    if (est_err) *est_err = est;
    if (used_fallback) *used_fallback = accept ? 0 : 1;
    if (!accept) return art_sweep(mesh, nside_fine, gamma_w, 0.0f, out, hip_stream);
    float hw[8];
    art_mesh_heating(mesh, hw);
    hipLaunchKernelGGL(finish_kernel, dim3(blocks_for(V, 256)), dim3(256), 0, st, s->pred, s->Jinc, s->Jc,
                       s->Jexc, rec, nb, gamma_w ? gamma_w[0] : 1.0f, hw[0], hw[4], V, out->J,
                       out->J_in, out->J_exact, out->Gamma, out->Heat);
    return launch_status("art_sweep_surrogate (outputs)");
}

int art_sha256(const void *data, unsigned long long n, unsigned char *digest)
{
    if ((!data && n) || !digest) return sg_fail(ART_E_INVAL, "art_sha256: NULL argument");
    sha256((const unsigned char *)data, n, digest);
    return ART_OK;
}

}  // extern "C"
