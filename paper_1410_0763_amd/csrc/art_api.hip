// art_api.hip -- host side of libart: handles, validation, buffers, the
// block-wavefront schedule and the launch sequence of one sweep.
//
// Sweep = direction generator -> march launches, one per wavefront (all eight
// octants and all direction subsets of that wavefront in one launch) ->
// normalisation/rates -> optional exit sums.  Everything is queued on the
// caller's stream; nothing in a sweep synchronises the host.
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/art.h"
#include "art_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(e_ == hipErrorOutOfMemory ? ART_E_NOMEM : ART_E_HIP,           \
                        std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

template <class T>
int dev_alloc(T **p, size_t count, size_t *cap)
{
    if (*p && *cap >= count) return ART_OK;
    if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
        *cap = 0;
    }
    if (count == 0) return ART_OK;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ART_E_NOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                                     " bytes: " + hipGetErrorString(e));
    }
    *cap = count;
    return ART_OK;
}

}  // namespace

// Error text for the other translation units of the library.
int art_set_error(int code, const char *msg) { return fail(code, msg); }

struct art_mesh {
    int nx = 0, ny = 0, nz = 0;
    double h = 1.0;
    long long ncell = 0;
    int nb = 0;                         // bins loaded (0: no fields yet)
    art_tuning tune{6, 1, 1, 3};
    // No shape set by the caller (art_set_tuning, an autotuner): depth 8 for
    // 1-3 bins, 6 for 4, and per plain sweep min(3, directions per bucket)
    // directions per wave (march_k; a batch keeps 3).
    bool shape_auto = true;
    float heat[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // heating weights: J_in terms, then S terms
    int mbd = 0, mbd_key[2] = {-1, -1};   // largest bucket (directions) for (nside, subsets)

    float2 *fields = nullptr; size_t fields_cap = 0;
    float2 *fields_t = nullptr; size_t fields_t_cap = 0;   // y-fastest copy
    int *bad = nullptr; size_t bad_cap = 0;
    float *stage = nullptr; size_t stage_cap = 0;   // host-upload staging
    float *kpack = nullptr; size_t kpack_cap = 0;   // kappa h alone (point sources)
    bool kpack_ok = false;

    ArtDir *dirs = nullptr; size_t dirs_cap = 0;
    int *order = nullptr; size_t order_cap = 0;
    int *bucket_start = nullptr; size_t bs_cap = 0;
    float *state = nullptr; size_t state_cap = 0;
    float *faces = nullptr; size_t faces_cap = 0;
    uint4 *geo = nullptr; size_t geo_cap = 0;
    float *acc = nullptr; size_t acc_cap = 0;

    // schedule (depends on shape and tuning only)
    ArtItem *items = nullptr; size_t items_cap = 0;
    unsigned int *seg_count = nullptr; size_t seg_cap = 0;   // per work item
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // start, march start, march end, end
    bool timed = false;
    std::vector<int> wave_off;          // [W + 1]
    std::vector<ArtItem> items_host;    // the same items on the host
    int sched_key[6] = {0, 0, 0, 0, 0, 0};
    ArtMeshDesc *desc = nullptr; size_t desc_cap = 0;
    ArtMeshDesc desc_host{};
    bool desc_valid = false;

    // Direction tables (dirs, order, bucket_start, crossing table and the
    // boundary slots of the state buffer) depend only on this key; a sweep
    // whose key matches the tables on the device skips the generator.
    struct TableKey {
        int nside = 0, d_begin = 0, d_end = 0, subsets = 0, nb = 0;
        float I_bc = 0.0f;
        bool operator==(const TableKey &o) const
        {
            return nside == o.nside && d_begin == o.d_begin && d_end == o.d_end &&
                   subsets == o.subsets && nb == o.nb &&
                   std::memcmp(&I_bc, &o.I_bc, sizeof I_bc) == 0;
        }
    };
    TableKey tab{};
    bool tab_valid = false;
    // Live batches holding this mesh: its buffers are captured in their
    // graphs, so nothing may reallocate them, re-tune the mesh or free it.
    int batches = 0;
};

namespace {
// Directions one wave marches together in a sweep at this Nside: the tuned
// value, or, for a mesh without a set shape, one per direction of a bucket up
// to 3 (12 Nside^2 directions over 24 buckets: 1 at Nside 1, 2 at Nside 2).
int march_k(const art_mesh *m, int nside)
{
    if (!m->shape_auto) return m->tune.interleave;
    return nside == 1 ? 1 : (nside == 2 ? 2 : 3);
}
}  // namespace

void art_mesh_heating(const art_mesh *m, float hw8[8])
{
    for (int i = 0; i < 8; ++i) hw8[i] = m->heat[i];
}

int art_mesh_kpack(art_mesh *m, hipStream_t st, const float **kpack, int *ks)
{
    if (m->nb == 0) return fail(ART_E_STATE, "art_set_fields has not been called");
    const int k = m->nb == 1 ? 1 : (m->nb == 2 ? 2 : 4);
    if (!m->kpack_ok) {
        int rc = dev_alloc(&m->kpack, (size_t)m->ncell * k, &m->kpack_cap);
        if (rc) return rc;
        HIPCHK(art_launch_kpack(m->fields, m->ncell, m->nb, k, m->kpack, st));
        m->kpack_ok = true;
    }
    *kpack = m->kpack;
    *ks = k;
    return ART_OK;
}

void art_mesh_fields(const art_mesh *m, int dims[3], int *nb, double *h, const float2 **fields)
{
    dims[0] = m->nx;
    dims[1] = m->ny;
    dims[2] = m->nz;
    *nb = m->nb;
    *h = m->h;
    *fields = m->nb > 0 ? m->fields : nullptr;
}

namespace {

int nblocks(int n, int b) { return (n + b - 1) / b; }

int validate_tuning(const art_tuning &t, int nb)
{
    if (t.depth < 1 || t.depth > 256) return fail(ART_E_INVAL, "tuning: depth must be in [1, 256]");
    if (t.subsets < 1 || t.subsets > 64) return fail(ART_E_INVAL, "tuning: subsets must be in [1, 64]");
    if (t.waves < 1 || t.waves > 8) return fail(ART_E_INVAL, "tuning: waves must be in [1, 8]");
    if (t.interleave < 1 || t.interleave > 4)
        return fail(ART_E_INVAL, "tuning: interleave must be 1, 2, 3 or 4");
    const long long lds = (long long)art_march_lds_floats(t.depth, std::max(nb, 1)) * 4;
    if (lds > art_march_max_lds_bytes())
        return fail(ART_E_UNSUPPORTED, "tuning: block accumulators need " + std::to_string(lds) +
                                           " bytes of LDS, above the workgroup limit");
    return ART_OK;
}

// Work items of the block wavefronts.  For dominant axis a the blocks are
// 8 x 8 columns (axes b < c) by `depth` cells along a; launch w holds, for
// every (a, octant) group, the blocks whose indices counted along the group's
// travel directions sum to w, once per direction subset.  Host only.
void schedule_items(const int N[3], int depth, int subsets, std::vector<ArtItem> &flat,
                    std::vector<int> &wave_off)
{
    std::vector<std::vector<ArtItem>> waves;
    for (int a = 0; a < 3; ++a) {
        const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
        int nblk[3];
        nblk[a] = nblocks(N[a], depth);
        nblk[b] = nblocks(N[b], 8);
        nblk[c] = nblocks(N[c], 8);
        const int W = nblk[0] + nblk[1] + nblk[2] - 2;
        if ((int)waves.size() < W) waves.resize(W);
        for (int o = 0; o < 8; ++o)
            for (int pa = 0; pa < nblk[a]; ++pa)
                for (int pc = 0; pc < nblk[c]; ++pc)
                    for (int pb = 0; pb < nblk[b]; ++pb) {
                        int p[3];
                        p[a] = pa; p[b] = pb; p[c] = pc;
                        int wsum = 0;
                        for (int ax = 0; ax < 3; ++ax)
                            wsum += ((o >> ax) & 1) ? nblk[ax] - 1 - p[ax] : p[ax];
                        const int blk = (pa * nblk[c] + pc) * nblk[b] + pb;
                        for (int s = 0; s < subsets; ++s)
                            waves[wsum].push_back(ArtItem{0, blk, (a * 8 + o) * subsets + s, 0});
                    }
    }
    flat.clear();
    wave_off.assign(1, 0);
    for (auto &w : waves) {
        flat.insert(flat.end(), w.begin(), w.end());
        wave_off.push_back((int)flat.size());
    }
}

int build_schedule(art_mesh *m)
{
    const art_tuning &t = m->tune;
    const int key[6] = {m->nx, m->ny, m->nz, t.depth, t.subsets, 2};
    if (m->items && std::equal(key, key + 6, m->sched_key)) return ART_OK;
    const int N[3] = {m->nx, m->ny, m->nz};
    std::vector<ArtItem> flat;
    schedule_items(N, t.depth, t.subsets, flat, m->wave_off);
    HIPCHK(hipDeviceSynchronize());   // items of earlier sweeps may still be in use
    int rc = dev_alloc(&m->items, flat.size(), &m->items_cap);
    if (rc) return rc;
    if ((rc = dev_alloc(&m->seg_count, flat.size(), &m->seg_cap))) return rc;
    HIPCHK(hipMemcpy(m->items, flat.data(), flat.size() * sizeof(ArtItem), hipMemcpyHostToDevice));
    m->items_host = flat;
    std::copy(key, key + 6, m->sched_key);
    return ART_OK;
}

// Largest ray-slot count of one direction (the lattice covers the mesh's
// cross-section widened by the depth on both sides).
long long dir_slot_bound(const art_mesh *m)
{
    const long long N[3] = {m->nx, m->ny, m->nz};
    long long worst = 0;
    for (int a = 0; a < 3; ++a) {
        const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
        worst = std::max(worst, (N[b] + N[a] + 4) * (N[c] + N[a] + 4));
    }
    return worst;
}

// Blocks of the largest block cross-section over the three dominant axes.
long long face_blocks(const art_mesh *m)
{
    const long long N[3] = {m->nx, m->ny, m->nz};
    long long worst = 0;
    for (int a = 0; a < 3; ++a) {
        const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
        worst = std::max(worst, ((N[b] + 7) / 8) * ((N[c] + 7) / 8));
    }
    return worst;
}

// Face-buffer floats of one direction: b- and c-faces of two block layers
// along a (depth slabs x 8 rays per block), a-faces (64 rays per block).
long long face_dir_floats(const art_mesh *m)
{
    return (4ll * m->tune.depth * 8 + 64) * face_blocks(m) * m->nb;
}

long long state_bound(const art_mesh *m, int nd)
{
    const long long N[3] = {m->nx, m->ny, m->nz};
    long long worst = 0;
    for (int a = 0; a < 3; ++a) {
        const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
        worst = std::max(worst, (N[b] + N[a] + 4) * (N[c] + N[a] + 4));
    }
    return (worst + 1) * nd * m->nb;   // ray slots plus one boundary slot per direction
}

// Buffers and descriptor for a sweep at this nside (allocation is the only
// host-synchronous part, and happens only when sizes grow or tuning changes).
int prepare(art_mesh *m, int nside, float I_bc, hipStream_t st)
{
    const int nd = 12 * nside * nside;
    // the march addresses one bucket's ray states, one block's field records
    // and the crossing table with 32-bit byte offsets from wave-uniform bases
    // (a block spans at most depth - 1 + 7 + 7 steps of the largest cell
    // stride of either field copy: nx ny, or ny nz for the y-fastest copy)
    if (m->mbd_key[0] != nside || m->mbd_key[1] != m->tune.subsets) {
        m->mbd = art_max_bucket_dirs(nside, m->tune.subsets);
        m->mbd_key[0] = nside;
        m->mbd_key[1] = m->tune.subsets;
    }
    if ((long long)m->mbd * (dir_slot_bound(m) + 1) * m->nb * 4 >=
            (1ll << 31) ||
        (m->tune.depth + 14ll) * std::max((long long)m->nx * m->ny, (long long)m->ny * m->nz) * m->nb * 8 >=
            (1ll << 31) ||
        (long long)nd * std::max(m->nx, std::max(m->ny, m->nz)) * 16 >= (1ll << 31) ||
        (long long)m->mbd * face_dir_floats(m) * 4 >= (1ll << 31))
        return fail(ART_E_UNSUPPORTED, "mesh too large for 32-bit offsets within a bucket of directions or a block");
    const int nbk = 24 * m->tune.subsets;
    const int gstride = std::max(m->nx, std::max(m->ny, m->nz));
    const size_t need_state = (size_t)state_bound(m, nd), need_geo = (size_t)nd * gstride;
    const size_t need_acc = (size_t)nbk * m->nb * 2 * m->ncell;
    const size_t need_faces = (size_t)nbk * m->mbd * face_dir_floats(m);
    if (m->batches > 0 &&
        ((size_t)nd > m->dirs_cap || (size_t)nd > m->order_cap || (size_t)nbk + 1 > m->bs_cap ||
         need_state > m->state_cap || need_geo > m->geo_cap || need_acc > m->acc_cap ||
         need_faces > m->faces_cap))
        return fail(ART_E_STATE, "this sweep would reallocate buffers of a mesh held by a live batch "
                                 "(larger Nside than the batch's); destroy the batch first");
    const void *tab_bufs[5] = {m->dirs, m->order, m->bucket_start, m->state, m->geo};
    int rc;
    if ((rc = dev_alloc(&m->dirs, (size_t)nd, &m->dirs_cap))) return rc;
    if ((rc = dev_alloc(&m->order, (size_t)nd, &m->order_cap))) return rc;
    if ((rc = dev_alloc(&m->bucket_start, (size_t)nbk + 1, &m->bs_cap))) return rc;
    if ((rc = dev_alloc(&m->state, need_state, &m->state_cap))) return rc;
    if ((rc = dev_alloc(&m->geo, need_geo, &m->geo_cap))) return rc;
    if ((rc = dev_alloc(&m->acc, need_acc, &m->acc_cap))) return rc;
    if ((rc = dev_alloc(&m->faces, need_faces, &m->faces_cap))) return rc;
    if (tab_bufs[0] != m->dirs || tab_bufs[1] != m->order || tab_bufs[2] != m->bucket_start ||
        tab_bufs[3] != m->state || tab_bufs[4] != m->geo)
        m->tab_valid = false;   // new buffers hold no tables
    if ((rc = build_schedule(m))) return rc;
    ArtMeshDesc d{};
    d.fields = m->fields;
    d.fields_t = m->fields_t;
    d.state = m->state;
    d.faces = m->faces;
    d.face_dir_floats = face_dir_floats(m);
    d.face_bucket_dirs = m->mbd;
    d.face_P = (int)face_blocks(m);
    d.acc = m->acc;
    d.dirs = m->dirs;
    d.order = m->order;
    d.bucket_start = m->bucket_start;
    d.geo = m->geo;
    d.geo_stride = gstride;
    // the whole allocation, not this Nside's rows: switching between Nsides
    // that fit then leaves the descriptor (and the host) alone
    d.geo_rows = (long long)m->geo_cap;
    d.interleave = m->tune.interleave;
    d.ncell = m->ncell;
    d.nx = m->nx; d.ny = m->ny; d.nz = m->nz; d.nb = m->nb;
    d.depth = m->tune.depth;
    d.subsets = m->tune.subsets;
    d.I_bc = I_bc;
    d.nbuckets = nbk;
    if ((rc = dev_alloc(&m->desc, 1, &m->desc_cap))) return rc;
    if (!m->desc_valid || std::memcmp(&d, &m->desc_host, sizeof d) != 0) {
        // earlier sweeps queued on the stream may still read the old descriptor
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(m->desc, &d, sizeof d, hipMemcpyHostToDevice));
        m->desc_host = d;
        m->desc_valid = true;
    }
    return ART_OK;
}

art_mesh::TableKey table_key(const art_mesh *m, int nside, int d_begin, int d_end, float I_bc)
{
    art_mesh::TableKey k;
    k.nside = nside;
    k.d_begin = d_begin;
    k.d_end = d_end;
    k.subsets = m->tune.subsets;
    k.nb = m->nb;
    k.I_bc = I_bc;
    return k;
}

// Direction generator, state offsets with boundary slots, crossing table:
// queued on st unless the device already holds the tables of this key.
int ensure_tables(art_mesh *m, int nside, int d_begin, int d_end, float I_bc, hipStream_t st)
{
    const art_mesh::TableKey k = table_key(m, nside, d_begin, d_end, I_bc);
    if (m->tab_valid && m->tab == k) return ART_OK;
    m->tab_valid = false;
    HIPCHK(art_launch_dirs(nside, m->nx, m->ny, m->nz, m->nb, d_begin, d_end, m->tune.subsets,
                           m->dirs, m->order, m->bucket_start, m->geo, m->desc_host.geo_stride,
                           m->state, I_bc, st));
    m->tab = k;
    m->tab_valid = true;
    return ART_OK;
}

int run_sweep(art_mesh *m, int nside, int d_begin, int d_end, float I_bc, hipStream_t st,
              bool fill_state = false)
{
    int rc = prepare(m, nside, I_bc, st);
    if (rc) return rc;
    if (fill_state) HIPCHK(art_launch_fill(m->state, (long long)m->state_cap, I_bc, st));
    if (!m->ev[0])
        for (int i = 0; i < 4; ++i) HIPCHK(hipEventCreate(&m->ev[i]));
    HIPCHK(hipEventRecord(m->ev[0], st));
    if ((rc = ensure_tables(m, nside, d_begin, d_end, I_bc, st))) return rc;
    HIPCHK(hipEventRecord(m->ev[1], st));
    const int lds_floats = art_march_lds_floats(m->tune.depth, m->nb);
    for (size_t w = 0; w + 1 < m->wave_off.size(); ++w) {
        const int n = m->wave_off[w + 1] - m->wave_off[w];
        // The launches of the wavefront ramps hold few workgroups, and each
        // takes as long as one workgroup alone: there, with one wave per
        // workgroup tuned, 4 (or 2) waves share a workgroup's directions, each
        // with its own accumulators.  Fixed thresholds (a quarter and a half
        // of 3072 workgroups, the resident one-wave workgroups of 256 CUs), so
        // that which blocks take the multi-wave sums does not depend on the GPU.
        int waves = m->tune.waves, priv = 0, lf = lds_floats;
        if (waves == 1)
            for (int W : {4, 2})
                if (n * W <= 3072 &&
                    (long long)art_march_lds_floats(m->tune.depth, m->nb, W) * 4 <= art_march_max_lds_bytes()) {
                    waves = W;
                    priv = 1;
                    lf = art_march_lds_floats(m->tune.depth, m->nb, W);
                    break;
                }
        HIPCHK(art_launch_march(m->items + m->wave_off[w], n, m->desc, m->nb, march_k(m, nside), lf,
                                64 * waves, m->seg_count + m->wave_off[w], st, priv));
    }
    HIPCHK(hipEventRecord(m->ev[2], st));
    return ART_OK;
}

int check_mesh_ready(const art_mesh *m, int nside)
{
    if (!m) return fail(ART_E_INVAL, "mesh is NULL");
    if (m->nb == 0) return fail(ART_E_STATE, "art_set_fields has not been called");
    if (nside < 1 || nside > ART_MAX_NSIDE)
        return fail(ART_E_INVAL, "nside must be in [1, " + std::to_string(ART_MAX_NSIDE) + "]");
    return ART_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batched form: several meshes (each with its own shape, Nside, bins and
// tuning) marched by one captured graph.  Launch (w, nb, K) holds the
// wavefront-w items of every mesh with nb bins and K directions per wave;
// items index a descriptor array of all meshes.  The meshes of one (nb, K)
// form a chain (direction setup, their launches in wavefront order, their
// normalisations) on a stream of its own, forked from and joined to the
// capture stream, so that the replayed graph runs the chains side by side.
// The graph is captured once on an internal stream and replayed on the
// caller's stream.
// ---------------------------------------------------------------------------
struct art_batch {
    std::vector<art_mesh *> meshes;
    std::vector<int> nside;
    std::vector<art_outputs> outs;
    std::vector<std::array<float, 4>> gw;
    std::vector<std::array<float, 8>> hw;   // heating weights of each mesh at creation
    float I_bc = 0.0f;
    int waves = 8;
    ArtMeshDesc *descs = nullptr; size_t descs_cap = 0;
    ArtItem *items = nullptr; size_t items_cap = 0;
    unsigned int *seg_count = nullptr; size_t seg_cap = 0;
    struct Launch { int off, n, nb, lds, interleave, chain, waves, priv; };
    std::vector<Launch> launches;
    std::vector<int> mesh_chain;        // chain (stream of the captured graph) of each mesh
    int nchain = 1;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool launched = false;
    bool held = false;                  // the meshes count this batch in art_mesh::batches
};

namespace {

int batch_enqueue(art_batch *B, hipStream_t st)
{
    const int n = (int)B->meshes.size();
    // Meshes with different (bins, directions per wave) never share a launch:
    // each such chain runs on its own stream between a fork and a join, so
    // that the captured graph lets the chains overlap.
    std::vector<hipStream_t> side(B->nchain, st);
    std::vector<hipEvent_t> evs;
    auto cleanup = [&]() {
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
        for (hipStream_t s : side)
            if (s != st) (void)hipStreamDestroy(s);
    };
    auto chk = [&](hipError_t e) -> int {
        if (e != hipSuccess) { cleanup(); return fail(ART_E_HIP, std::string("batch capture: ") + hipGetErrorString(e)); }
        return ART_OK;
    };
    int rc;
    if (B->nchain > 1) {
        hipEvent_t fork;
        if ((rc = chk(hipEventCreateWithFlags(&fork, hipEventDisableTiming)))) return rc;
        evs.push_back(fork);
        if ((rc = chk(hipEventRecord(fork, st)))) return rc;
        for (int c = 0; c < B->nchain; ++c) {
            hipStream_t s;
            if ((rc = chk(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)))) return rc;
            side[c] = s;
            if ((rc = chk(hipStreamWaitEvent(s, fork, 0)))) return rc;
        }
    }
    // (the direction tables are not part of the graph: art_batch_create
    // builds them and art_batch_launch rebuilds those a plain sweep replaced)
    for (const auto &L : B->launches)
        if ((rc = chk(art_launch_march(B->items + L.off, L.n, B->descs, L.nb, L.interleave, L.lds,
                                       64 * L.waves, B->seg_count + L.off, side[L.chain], L.priv)))) return rc;
    for (int i = 0; i < n; ++i) {
        art_mesh *m = B->meshes[i];
        const art_outputs &o = B->outs[i];
        if ((rc = chk(art_launch_normalize(m->acc, m->bucket_start, 24 * m->tune.subsets, m->fields, m->ncell,
                                           m->nb, 12 * B->nside[i] * B->nside[i], B->gw[i].data(),
                                           B->hw[i].data(), o.J_in, o.J, o.J_exact, o.Gamma, o.Heat,
                                           nullptr, nullptr, side[B->mesh_chain[i]])))) return rc;
    }
    if (B->nchain > 1) {
        for (int c = 0; c < B->nchain; ++c) {
            hipEvent_t j;
            if ((rc = chk(hipEventCreateWithFlags(&j, hipEventDisableTiming)))) return rc;
            evs.push_back(j);
            if ((rc = chk(hipEventRecord(j, side[c])))) return rc;
            if ((rc = chk(hipStreamWaitEvent(st, j, 0)))) return rc;
        }
    }
    cleanup();
    return ART_OK;
}

void batch_free(art_batch *B)
{
    if (!B) return;
    if (B->held)
        for (art_mesh *m : B->meshes) --m->batches;
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    for (hipEvent_t e : B->ev)
        if (e) (void)hipEventDestroy(e);
    if (B->descs) (void)hipFree(B->descs);
    if (B->items) (void)hipFree(B->items);
    if (B->seg_count) (void)hipFree(B->seg_count);
    delete B;
}

}  // namespace

extern "C" {

const char *art_last_error(void) { return g_err.c_str(); }

int art_ndirs(int nside)
{
    if (nside < 1 || nside > ART_MAX_NSIDE) return fail(ART_E_INVAL, "nside out of range");
    return 12 * nside * nside;
}

int art_schedule(int nx, int ny, int nz, const art_tuning *t, int *items, long long cap,
                 long long *n, int *nwave)
{
    try {
        if (!t || !n) return fail(ART_E_INVAL, "schedule: null argument");
        if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
            return fail(ART_E_INVAL, "mesh sides must be in [1, 4096]");
        int rc = validate_tuning(*t, 1);
        if (rc) return rc;
        const int N[3] = {nx, ny, nz};
        std::vector<ArtItem> flat;
        std::vector<int> off;
        schedule_items(N, t->depth, t->subsets, flat, off);
        *n = (long long)flat.size();
        if (nwave) *nwave = (int)off.size() - 1;
        if (items) {
            if (cap < (long long)flat.size()) return fail(ART_E_INVAL, "schedule: cap below the item count");
            for (size_t w = 0; w + 1 < off.size(); ++w)
                for (int q = off[w]; q < off[w + 1]; ++q) {
                    items[3 * (size_t)q] = (int)w;
                    items[3 * (size_t)q + 1] = flat[q].block;
                    items[3 * (size_t)q + 2] = flat[q].bucket;
                }
        }
        g_err.clear();
        return ART_OK;
    } catch (const std::bad_alloc &) {
        return fail(ART_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ART_E_HIP, "unexpected exception");
    }
}

int art_create_mesh(int nx, int ny, int nz, double cell_size, art_mesh **out)
{
    try {
        if (!out) return fail(ART_E_INVAL, "out is NULL");
        if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
            return fail(ART_E_INVAL, "mesh sides must be in [1, 4096]");
        if (!(cell_size > 0.0) || !std::isfinite(cell_size))
            return fail(ART_E_INVAL, "cell_size must be positive and finite");
        art_mesh *m = new art_mesh;
        m->nx = nx; m->ny = ny; m->nz = nz;
        m->h = cell_size;
        m->ncell = (long long)nx * ny * nz;
        *out = m;
        g_err.clear();
        return ART_OK;
    } catch (const std::bad_alloc &) {
        return fail(ART_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ART_E_HIP, "unexpected exception");
    }
}

int art_destroy_mesh(art_mesh *m)
{
    if (!m) return ART_OK;
    if (m->batches > 0) return fail(ART_E_STATE, "mesh is held by a live batch; destroy the batch first");
    void *bufs[] = {m->fields, m->fields_t, m->bad, m->stage, m->dirs, m->order, m->bucket_start,
                    m->state, m->faces, m->geo, m->acc, m->items, m->desc, m->seg_count, m->kpack};
    for (hipEvent_t e : m->ev)
        if (e) (void)hipEventDestroy(e);
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    delete m;
    return ART_OK;
}

int art_set_fields(art_mesh *m, int nbins, const float *kappa, const float *S, int on_device,
                   void *hip_stream)
{
    try {
        if (!m || !kappa || !S) return fail(ART_E_INVAL, "null mesh or field pointer");
        if (nbins < 1 || nbins > ART_MAX_BINS)
            return fail(ART_E_UNSUPPORTED, "nbins must be in [1, " + std::to_string(ART_MAX_BINS) + "]");
        art_tuning tn = m->tune;
        if (m->shape_auto) tn.depth = nbins <= 3 ? 8 : 6;   // 4 bins at depth 8: 2 workgroups per SIMD
        int rc = validate_tuning(tn, nbins);
        if (rc) return rc;
        if (m->batches > 0 && nbins != m->nb)
            return fail(ART_E_STATE, "mesh is held by a live batch: its bin count cannot change");
        hipStream_t st = (hipStream_t)hip_stream;
        const size_t n = (size_t)m->ncell * nbins;
        if (m->batches > 0 && (n > m->fields_cap || n > m->fields_t_cap))
            return fail(ART_E_STATE, "mesh is held by a live batch: its field buffers cannot grow");
        if ((rc = dev_alloc(&m->bad, 1, &m->bad_cap))) return rc;
        const float *dk = kappa, *ds = S;
        if (!on_device) {
            if ((rc = dev_alloc(&m->stage, 2 * n, &m->stage_cap))) return rc;
            HIPCHK(hipMemcpyAsync(m->stage, kappa, n * sizeof(float), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(m->stage + n, S, n * sizeof(float), hipMemcpyHostToDevice, st));
            dk = m->stage;
            ds = m->stage + n;
        }
        // validate first: a rejected call leaves the mesh's fields as they were
        HIPCHK(art_launch_fill(reinterpret_cast<float *>(m->bad), 1, 0.0f, st));
        HIPCHK(art_launch_check(dk, ds, (long long)n, m->bad, st));
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, m->bad, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (bad) return fail(ART_E_INVAL, "kappa must be finite and >= 0 and S finite in every cell");
        m->kpack_ok = false;
        if ((rc = dev_alloc(&m->fields, n, &m->fields_cap))) return rc;
        if ((rc = dev_alloc(&m->fields_t, n, &m->fields_t_cap))) return rc;
        HIPCHK(art_launch_layout(dk, ds, m->nx, m->ny, m->nz, nbins, m->h, m->fields, m->fields_t, st));
        if (m->nb != nbins) {
            m->desc_valid = false;
            for (float &w : m->heat) w = 0.0f;   // weights belong to the old bins
        }
        m->nb = nbins;
        if (tn.depth != m->tune.depth) {
            m->tune = tn;
            m->desc_valid = false;
        }
        g_err.clear();
        return ART_OK;
    } catch (const std::bad_alloc &) {
        return fail(ART_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ART_E_HIP, "unexpected exception");
    }
}

int art_sweep(art_mesh *m, int nside, const float *gamma_w, float I_bc, const art_outputs *out,
              void *hip_stream)
{
    try {
        int rc = check_mesh_ready(m, nside);
        if (rc) return rc;
        if (!out) return fail(ART_E_INVAL, "outputs are NULL");
        if (!std::isfinite(I_bc)) return fail(ART_E_INVAL, "I_bc must be finite");
        float gw[4] = {1.f, 1.f, 1.f, 1.f};
        if (gamma_w)
            for (int b = 0; b < m->nb; ++b) {
                if (!std::isfinite(gamma_w[b])) return fail(ART_E_INVAL, "gamma_w must be finite");
                gw[b] = gamma_w[b];
            }
        hipStream_t st = (hipStream_t)hip_stream;
        const int nd = 12 * nside * nside;
        if ((rc = run_sweep(m, nside, 0, nd, I_bc, st, out->exit_sum != nullptr))) return rc;
        HIPCHK(art_launch_normalize(m->acc, m->bucket_start, 24 * m->tune.subsets, m->fields,
                                    m->ncell, m->nb, nd, gw, m->heat, out->J_in, out->J,
                                    out->J_exact, out->Gamma, out->Heat, nullptr, nullptr, st));
        HIPCHK(hipEventRecord(m->ev[3], st));
        m->timed = true;
        if (out->exit_sum)
            HIPCHK(art_launch_exit_sum(m->dirs, nd, m->state, m->nx, m->ny, m->nz, m->nb, I_bc,
                                       out->exit_sum, st));
        g_err.clear();
        return ART_OK;
    } catch (const std::bad_alloc &) {
        return fail(ART_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ART_E_HIP, "unexpected exception");
    }
}

int art_sweep_range(art_mesh *m, int nside, int d_begin, int d_end, float I_bc, float *A1,
                    float *A2, void *hip_stream)
{
    try {
        int rc = check_mesh_ready(m, nside);
        if (rc) return rc;
        const int nd = 12 * nside * nside;
        if (d_begin < 0 || d_end > nd || d_begin >= d_end)
            return fail(ART_E_INVAL, "direction range must satisfy 0 <= d_begin < d_end <= N_d");
        if (!A1) return fail(ART_E_INVAL, "A1 is NULL");
        if (!std::isfinite(I_bc)) return fail(ART_E_INVAL, "I_bc must be finite");
        hipStream_t st = (hipStream_t)hip_stream;
        if ((rc = run_sweep(m, nside, d_begin, d_end, I_bc, st))) return rc;
        const float ones[4] = {1.f, 1.f, 1.f, 1.f};
        HIPCHK(art_launch_normalize(m->acc, m->bucket_start, 24 * m->tune.subsets, m->fields,
                                    m->ncell, m->nb, nd, ones, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, nullptr, A1, A2, st));
        HIPCHK(hipEventRecord(m->ev[3], st));
        m->timed = true;
        g_err.clear();
        return ART_OK;
    } catch (const std::bad_alloc &) {
        return fail(ART_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ART_E_HIP, "unexpected exception");
    }
}

int art_autotune(art_mesh *m, int nside, const art_tuning *cand, int ncand, art_tuning *best,
                 float *best_ms, void *hip_stream)
{
    float *scratch = nullptr;
    size_t cap = 0;
    art_tuning saved{};
    bool saved_auto = true;
    if (m) {
        saved = m->tune;
        saved_auto = m->shape_auto;
    }
    auto done = [&](int rc) {
        if (scratch) (void)hipFree(scratch);
        if (rc != ART_OK && m) {
            m->tune = saved;
            m->shape_auto = saved_auto;
            m->desc_valid = false;
        }
        return rc;
    };
    try {
        int rc = check_mesh_ready(m, nside);
        if (rc) return rc;
        if (m->batches > 0) return fail(ART_E_STATE, "mesh is held by a live batch: it cannot be re-tuned");
        std::vector<art_tuning> list;
        if (cand) {
            if (ncand < 1) return fail(ART_E_INVAL, "autotune: ncand must be positive");
            list.assign(cand, cand + ncand);
        } else {
            for (int depth : {4, 6, 8, 12})
                for (int k : {2, 3, 4}) list.push_back(art_tuning{depth, 1, 1, k});
        }
        if ((rc = dev_alloc(&scratch, (size_t)m->ncell * m->nb, &cap))) return done(rc);
        const int nd = 12 * nside * nside;
        float best_t = INFINITY;
        art_tuning bt = saved;
        for (const art_tuning &t : list) {
            if (validate_tuning(t, m->nb) != ART_OK) continue;     // the mesh cannot run it
            m->tune = t;
            m->shape_auto = false;
            m->desc_valid = false;
            for (int rep = 0; rep < 2; ++rep)                        // warm-up, then timed
                if ((rc = art_sweep_range(m, nside, 0, nd, 0.0f, scratch, nullptr, hip_stream)))
                    return done(rc);
            float ms = 0.0f;
            hipError_t e = hipEventSynchronize(m->ev[3]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, m->ev[0], m->ev[3]);
            if (e != hipSuccess) return done(fail(ART_E_HIP, std::string("autotune: ") + hipGetErrorString(e)));
            if (ms < best_t) {
                best_t = ms;
                bt = t;
            }
        }
        if (!(best_t < INFINITY)) return done(fail(ART_E_INVAL, "autotune: no candidate can run on this mesh"));
        m->tune = bt;
        m->desc_valid = false;
        if (best) *best = bt;
        if (best_ms) *best_ms = best_t;
        g_err.clear();
        return done(ART_OK);
    } catch (const std::bad_alloc &) {
        return done(fail(ART_E_NOMEM, "host allocation failed"));
    } catch (...) {
        return done(fail(ART_E_HIP, "unexpected exception"));
    }
}

// Process-wide autotune cache keyed by shape class, Nside and bins.
namespace {
struct TuneEntry {
    art_tuning t;
    float ms;
};
std::mutex g_tune_mu;
std::map<std::array<int, 3>, TuneEntry> g_tune;

// Shape class: cells counted in factors of 4 (floor(log2(cells) / 2)), so that
// meshes within a factor of about 4 in size share their launch shape.
int shape_class(const art_mesh *m)
{
    int l = 0;
    for (long long c = m->ncell; c > 1; c >>= 1) ++l;
    return l / 2;
}
}  // namespace

int art_autotune_class(art_mesh *m, int nside, const art_tuning *cand, int ncand, art_tuning *best,
                       float *best_ms, int *cached, void *hip_stream)
{
    try {
        int rc = check_mesh_ready(m, nside);
        if (rc) return rc;
        if (m->batches > 0) return fail(ART_E_STATE, "mesh is held by a live batch: it cannot be re-tuned");
        const std::array<int, 3> key{shape_class(m), nside, m->nb};
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tune.find(key);
            if (it != g_tune.end() && validate_tuning(it->second.t, m->nb) == ART_OK) {
                m->tune = it->second.t;
                m->shape_auto = false;
                m->desc_valid = false;
                if (best) *best = it->second.t;
                if (best_ms) *best_ms = it->second.ms;
                if (cached) *cached = 1;
                g_err.clear();
                return ART_OK;
            }
        }
        art_tuning bt{};
        float ms = 0.0f;
        if ((rc = art_autotune(m, nside, cand, ncand, &bt, &ms, hip_stream))) return rc;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tune[key] = TuneEntry{bt, ms};
        }
        if (best) *best = bt;
        if (best_ms) *best_ms = ms;
        if (cached) *cached = 0;
        return ART_OK;
    } catch (const std::bad_alloc &) {
        return fail(ART_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ART_E_HIP, "unexpected exception");
    }
}

int art_tune_cache(int op, const char *path)
{
    try {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        if (op == 0) {
            g_tune.clear();
            return ART_OK;
        }
        if (!path) return fail(ART_E_INVAL, "tune cache: null path");
        if (op == 1) {
            FILE *f = std::fopen(path, "w");
            if (!f) return fail(ART_E_INVAL, std::string("tune cache: cannot write ") + path);
            std::fprintf(f, "art-tune-cache 1\n");
            for (const auto &kv : g_tune)
                std::fprintf(f, "%d %d %d %d %d %d %d %.6g\n", kv.first[0], kv.first[1], kv.first[2],
                             kv.second.t.depth, kv.second.t.subsets, kv.second.t.waves,
                             kv.second.t.interleave, (double)kv.second.ms);
            const bool ok = std::fclose(f) == 0;
            return ok ? ART_OK : fail(ART_E_INVAL, std::string("tune cache: cannot write ") + path);
        }
        if (op == 2) {
            FILE *f = std::fopen(path, "r");
            if (!f) return fail(ART_E_INVAL, std::string("tune cache: cannot read ") + path);
            char magic[32] = {0};
            int ver = 0;
            if (std::fscanf(f, "%31s %d", magic, &ver) != 2 || std::strcmp(magic, "art-tune-cache") != 0 ||
                ver != 1) {
                std::fclose(f);
                return fail(ART_E_INVAL, "tune cache: not a cache file");
            }
            std::map<std::array<int, 3>, TuneEntry> in;
            int c, ns, nb, d, sub, w, k;
            double ms;
            int n;
            while ((n = std::fscanf(f, "%d %d %d %d %d %d %d %lf", &c, &ns, &nb, &d, &sub, &w, &k, &ms)) == 8) {
                art_tuning t{d, sub, w, k};
                if (validate_tuning(t, nb) != ART_OK || ns < 1 || ns > ART_MAX_NSIDE || nb < 1 || nb > ART_MAX_BINS) {
                    std::fclose(f);
                    return fail(ART_E_INVAL, "tune cache: invalid entry");
                }
                in[{c, ns, nb}] = TuneEntry{t, (float)ms};
            }
            const bool clean_end = n == EOF;
            std::fclose(f);
            if (!clean_end) return fail(ART_E_INVAL, "tune cache: malformed line");
            for (const auto &kv : in) g_tune[kv.first] = kv.second;
            g_err.clear();
            return ART_OK;
        }
        return fail(ART_E_INVAL, "tune cache: op must be 0 (clear), 1 (save) or 2 (load)");
    } catch (const std::bad_alloc &) {
        return fail(ART_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(ART_E_HIP, "unexpected exception");
    }
}

int art_set_tuning(art_mesh *m, const art_tuning *t)
{
    if (!m || !t) return fail(ART_E_INVAL, "null argument");
    int rc = validate_tuning(*t, m->nb);
    if (rc) return rc;
    if (m->batches > 0) return fail(ART_E_STATE, "mesh is held by a live batch: it cannot be re-tuned");
    m->tune = *t;
    m->shape_auto = false;
    m->desc_valid = false;
    g_err.clear();
    return ART_OK;
}

int art_sweep_stats(art_mesh *m, long long *segments, float *march_ms, float *sweep_ms)
{
    try {
        if (!m) return fail(ART_E_INVAL, "mesh is NULL");
        if (!m->timed) return fail(ART_E_STATE, "no sweep has run on this mesh");
        HIPCHK(hipEventSynchronize(m->ev[3]));
        if (march_ms) HIPCHK(hipEventElapsedTime(march_ms, m->ev[1], m->ev[2]));
        if (sweep_ms) HIPCHK(hipEventElapsedTime(sweep_ms, m->ev[0], m->ev[3]));
        if (segments) {
            const size_t n = (size_t)m->wave_off.back();
            std::vector<unsigned int> h(n);
            HIPCHK(hipMemcpy(h.data(), m->seg_count, n * sizeof(unsigned int), hipMemcpyDeviceToHost));
            long long tot = 0;
            for (unsigned int v : h) tot += v;
            *segments = tot;
        }
        g_err.clear();
        return ART_OK;
    } catch (...) {
        return fail(ART_E_HIP, "unexpected exception");
    }
}

int art_get_tuning(const art_mesh *m, art_tuning *t)
{
    if (!m || !t) return fail(ART_E_INVAL, "null argument");
    *t = m->tune;
    return ART_OK;
}

int art_set_heating(art_mesh *m, const float *heat_in, const float *heat_src)
{
    if (!m) return fail(ART_E_INVAL, "null mesh");
    if (m->nb == 0) return fail(ART_E_STATE, "art_set_fields has not been called");
    float h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < m->nb; ++b) {
        h[b] = heat_in ? heat_in[b] : 0.0f;
        h[4 + b] = heat_src ? heat_src[b] : 0.0f;
        if (!std::isfinite(h[b]) || !std::isfinite(h[4 + b]))
            return fail(ART_E_INVAL, "heating weights must be finite");
    }
    for (int i = 0; i < 8; ++i) m->heat[i] = h[i];
    return ART_OK;
}


int art_batch_create(art_mesh *const *meshes, const int *nside, int n, const float *const *gamma_w,
                     float I_bc, const art_outputs *outs, int waves, art_batch **out, void *hip_stream)
{
    art_batch *B = nullptr;
    try {
        if (!meshes || !nside || !outs || !out || n < 1)
            return fail(ART_E_INVAL, "batch: null argument or n < 1");
        if (waves < 1 || waves > 8) return fail(ART_E_INVAL, "batch: waves must be in [1, 8]");
        if (!std::isfinite(I_bc)) return fail(ART_E_INVAL, "I_bc must be finite");
        hipStream_t st = (hipStream_t)hip_stream;
        B = new art_batch;
        B->I_bc = I_bc;
        B->waves = waves;
        std::vector<ArtMeshDesc> descs;
        // per (wavefront, nb): items of all meshes
        std::map<std::tuple<int, int, int>, std::vector<ArtItem>> groups;
        std::map<std::tuple<int, int, int>, int> lds;
        std::map<std::pair<int, int>, int> chains;   // (bins, directions per wave) -> chain
        for (int i = 0; i < n; ++i) {
            art_mesh *m = meshes[i];
            int rc = check_mesh_ready(m, nside[i]);
            if (rc) { batch_free(B); return rc; }
            for (int j = 0; j < i; ++j)
                if (meshes[j] == m) { batch_free(B); return fail(ART_E_INVAL, "batch: a mesh appears twice"); }
            if ((rc = prepare(m, nside[i], I_bc, st))) { batch_free(B); return rc; }
            const int ndi = 12 * nside[i] * nside[i];
            if ((rc = ensure_tables(m, nside[i], 0, ndi, I_bc, st))) { batch_free(B); return rc; }
            descs.push_back(m->desc_host);
            B->meshes.push_back(m);
            B->nside.push_back(nside[i]);
            B->outs.push_back(outs[i]);
            std::array<float, 4> g = {1.f, 1.f, 1.f, 1.f};
            if (gamma_w && gamma_w[i])
                for (int b = 0; b < m->nb; ++b) g[b] = gamma_w[i][b];
            B->gw.push_back(g);
            std::array<float, 8> h;
            for (int q = 0; q < 8; ++q) h[q] = m->heat[q];
            B->hw.push_back(h);
            const int lf = art_march_lds_floats(m->tune.depth, m->nb);
            // the tuned directions per wave; a mesh without a set shape keeps
            // 3 here at every Nside, since each (bins, directions per wave)
            // pair is a chain of its own and more chains than hardware queues
            // run slower (48 uneven meshes: 81.4 ms with 2 at Nside 2, 76.5
            // ms with 3)
            const int mk = m->tune.interleave;
            const auto ck = std::make_pair(m->nb, mk);
            if (!chains.count(ck)) {
                const int c = (int)chains.size();
                chains[ck] = c;
            }
            B->mesh_chain.push_back(chains[ck]);
            for (size_t w = 0; w + 1 < m->wave_off.size(); ++w) {
                auto key = std::make_tuple((int)w, m->nb, mk);
                auto &v = groups[key];
                for (int q = m->wave_off[w]; q < m->wave_off[w + 1]; ++q) {
                    ArtItem it = m->items_host[q];
                    it.mesh = i;
                    v.push_back(it);
                }
                lds[key] = std::max(lds[key], lf);
            }
        }
        std::vector<ArtItem> flat;
        for (auto &kv : groups) {
            art_batch::Launch L{(int)flat.size(), (int)kv.second.size(), std::get<1>(kv.first),
                                lds[kv.first], std::get<2>(kv.first),
                                chains[std::make_pair(std::get<1>(kv.first), std::get<2>(kv.first))],
                                waves, 0};
            // small launches: several waves per workgroup with per-wave
            // accumulators, as in the plain sweep (the regions sized for the
            // launch's deepest mesh)
            if (waves == 1)
                for (int W : {4, 2})
                    if (L.n * W <= 3072 && (long long)(W * (L.lds - 32) + 32) * 4 <= art_march_max_lds_bytes()) {
                        L.waves = W;
                        L.priv = 1;
                        L.lds = W * (L.lds - 32) + 32;
                        break;
                    }
            flat.insert(flat.end(), kv.second.begin(), kv.second.end());
            B->launches.push_back(L);
        }
        B->nchain = (int)chains.size();
        int rc;
        if ((rc = dev_alloc(&B->descs, descs.size(), &B->descs_cap))) { batch_free(B); return rc; }
        if ((rc = dev_alloc(&B->items, flat.size(), &B->items_cap))) { batch_free(B); return rc; }
        if ((rc = dev_alloc(&B->seg_count, flat.size(), &B->seg_cap))) { batch_free(B); return rc; }
        hipError_t e = hipMemcpy(B->descs, descs.data(), descs.size() * sizeof(ArtMeshDesc), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(B->items, flat.data(), flat.size() * sizeof(ArtItem), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&B->ev[0]);
        if (e == hipSuccess) e = hipEventCreate(&B->ev[1]);
        if (e != hipSuccess) { batch_free(B); return fail(ART_E_HIP, std::string("batch setup: ") + hipGetErrorString(e)); }
        // the march kernels may need more LDS than the default: set it before capture
        for (const auto &L : B->launches) {
            e = art_launch_march(nullptr, 0, nullptr, L.nb, L.interleave, L.lds, 64 * L.waves, nullptr, B->cap);
            if (e != hipSuccess) { batch_free(B); return fail(ART_E_HIP, hipGetErrorString(e)); }
        }
        e = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) { batch_free(B); return fail(ART_E_HIP, std::string("capture: ") + hipGetErrorString(e)); }
        rc = batch_enqueue(B, B->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(B->cap, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); batch_free(B); return rc; }
        if (e != hipSuccess) { batch_free(B); return fail(ART_E_HIP, std::string("capture end: ") + hipGetErrorString(e)); }
        B->graph = g;
        e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { batch_free(B); return fail(ART_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e)); }
        // the tables queued on the caller's stream are done before any replay
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) { batch_free(B); return fail(ART_E_HIP, std::string("batch setup: ") + hipGetErrorString(e)); }
        for (art_mesh *m : B->meshes) ++m->batches;
        B->held = true;
        *out = B;
        g_err.clear();
        return ART_OK;
    } catch (const std::bad_alloc &) {
        batch_free(B);
        return fail(ART_E_NOMEM, "host allocation failed");
    } catch (...) {
        batch_free(B);
        return fail(ART_E_HIP, "unexpected exception");
    }
}

int art_batch_launch(art_batch *B, void *hip_stream)
{
    if (!B || !B->exec) return fail(ART_E_INVAL, "batch is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    HIPCHK(hipEventRecord(B->ev[0], st));
    // tables that a plain sweep of a mesh replaced since the last replay
    for (size_t i = 0; i < B->meshes.size(); ++i) {
        const int ndi = 12 * B->nside[i] * B->nside[i];
        int rc = ensure_tables(B->meshes[i], B->nside[i], 0, ndi, B->I_bc, st);
        if (rc) return rc;
    }
    HIPCHK(hipGraphLaunch(B->exec, st));
    HIPCHK(hipEventRecord(B->ev[1], st));
    B->launched = true;
    g_err.clear();
    return ART_OK;
}

int art_batch_stats(art_batch *B, long long *segment_bins, float *ms)
{
    if (!B) return fail(ART_E_INVAL, "batch is NULL");
    if (!B->launched) return fail(ART_E_STATE, "batch has not been launched");
    HIPCHK(hipEventSynchronize(B->ev[1]));
    if (ms) HIPCHK(hipEventElapsedTime(ms, B->ev[0], B->ev[1]));
    if (segment_bins) {
        std::vector<unsigned int> h(B->seg_cap);
        HIPCHK(hipMemcpy(h.data(), B->seg_count, h.size() * sizeof(unsigned int), hipMemcpyDeviceToHost));
        long long tot = 0;
        for (const auto &L : B->launches)
            for (int q = L.off; q < L.off + L.n; ++q) tot += (long long)h[q] * L.nb;
        *segment_bins = tot;
    }
    g_err.clear();
    return ART_OK;
}

int art_batch_destroy(art_batch *B)
{
    batch_free(B);
    return ART_OK;
}

int art_sweep_batched(art_mesh *const *meshes, const int *nside, int n, const float *const *gamma_w,
                      const art_outputs *outs, art_graph **graph, void *hip_stream)
{
    if (!graph) return fail(ART_E_INVAL, "art_sweep_batched: graph is NULL");
    art_batch *B = nullptr;
    int rc = art_batch_create(meshes, nside, n, gamma_w, 0.0f, outs, 1, &B, hip_stream);
    if (rc) return rc;
    if ((rc = art_batch_launch(B, hip_stream))) {
        batch_free(B);
        return rc;
    }
    *graph = B;
    return ART_OK;
}

int art_graph_launch(art_graph *graph, void *hip_stream) { return art_batch_launch(graph, hip_stream); }

int art_graph_destroy(art_graph *graph) { return art_batch_destroy(graph); }

}  // extern "C"
