/*
 * art.h -- C interface of libart, the MI355X implementation of the diffuse-
 * radiation ray-tracing sweep of Tanaka, Yoshikawa, Okamoto & Hasegawa,
 * "A new ray-tracing scheme for 3D diffuse radiation transfer on highly
 * parallel architectures" (PASJ; arXiv:1410.0763), Sect. 2.2-2.3 and 3.1.
 *
 * The sweep: for each direction of a HEALPix set of 12 Nside^2 directions
 * (Sect. 2.3), a lattice of parallel rays with unit spacing crosses the mesh
 * cell by cell; across a segment of length dL the intensity becomes
 * I e^{-dtau} + S (1 - e^{-dtau}), dtau = kappa dL (eq rt); each cell collects
 * the optical-depth-weighted mean over the rays crossing it of the path-
 * averaged incoming intensity I (1 - e^{-dtau}) / dtau (eqs path_averaged_
 * intensity, averaged_intensity), and the equal-weight mean over directions is
 * J_in, with J = J_in + S (eq mean_intensity).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Mesh fields are float32 arrays in C order [bin][z][y][x] (x fastest).
 *   Cells are cubes of side cell_size; kappa is per unit length.
 * - Every call returns ART_OK (0) or a negative ART_E_* code; on error the
 *   outputs are left untouched and art_last_error() (thread-local) describes
 *   the failure.  No C++ exception and no abort crosses this interface.
 * - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *   Work is queued on it asynchronously unless stated otherwise; device
 *   pointers must stay valid until the stream has passed the call.
 * - One handle must not be used from two threads at once.
 * - The library owns every handle and the device memory behind it.
 */
#ifndef ART_H
#define ART_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ART_OK = 0,
    ART_E_INVAL = -1,        /* bad argument (null, size, range, non-finite field) */
    ART_E_NOMEM = -2,        /* device or host allocation failed */
    ART_E_HIP = -3,          /* a HIP runtime call failed */
    ART_E_STATE = -4,        /* call out of order (e.g. sweep before set_fields) */
    ART_E_UNSUPPORTED = -5   /* valid request the library does not handle */
};

#define ART_MAX_BINS 4       /* frequency bins per mesh (Sect. 2.2 multi-bin form) */
#define ART_MAX_NSIDE 64     /* 49152 directions */

typedef struct art_mesh art_mesh;

/* Caller-owned device output buffers of one sweep; any member may be NULL.
 * J_in, J, J_exact: [nbins][cells]; Gamma: [cells]; exit_sum: [N_d][nbins]. */
typedef struct {
    float *J_in;     /* (1/N_d) sum_d mean of path-averaged incoming intensity */
    float *J;        /* J_in + S  (eq mean_intensity) */
    float *J_exact;  /* J_in + S <1 - (1 - e^{-dtau})/dtau>: the exact path
                        average of the formal solution (eq rad_tr2) */
    float *Gamma;    /* sum_b gamma_w[b] (J_in_b + S_b): eq gamma_diff with its
                        frequency integral folded into the per-bin weights */
    float *exit_sum; /* per direction and bin: sum over rays of (I_exit - I_bc) */
    float *Heat;     /* sum_b heat_in[b] J_in_b + heat_src[b] S_b: eq heat_diff with
                        its frequency integrals folded into per-bin weights
                        (art_set_heating; all 0 unless set) */
} art_outputs;

/* Launch shape of the sweep.  For directions with dominant axis a the mesh is
 * cut into blocks of 8 x 8 columns (the two other axes) by `depth` cells
 * along a; one workgroup of `waves` 64-lane waves marches one block for one
 * bucket of directions (one of `subsets` parts of a dominant-axis x octant
 * group).  Until a shape is set (art_set_tuning, art_autotune,
 * art_autotune_class) the mesh chooses its own: depth 8 for 1-3 bins and 6 for
 * 4 (set when art_set_fields loads the bins), one subset and one wave, and
 * per sweep min(3, directions per bucket) directions per wave, i.e. 1 at
 * Nside 1, 2 at Nside 2 and 3 above (the 24 buckets share 12 Nside^2
 * directions).  Depth 6 with 3 directions per wave is the fastest shape
 * measured for a 256^3 mesh with 768 directions and 4 bins; with 1-3 bins
 * depth 8 is 2-7% faster (128^3 and 256^3, Nside 8 and 16), and at Nside 2
 * 2 directions per wave are 9% faster than 3.  art_get_tuning then reports interleave 3, and a batch
 * (art_sweep_batched, art_batch_create) marches such a mesh with 3 directions
 * per wave at every Nside. */
typedef struct {
    int depth;        /* cells of a block along the dominant axis, 1..256 */
    int subsets;      /* buckets per (dominant axis, octant) group, 1..64 */
    int waves;        /* waves per workgroup, 1..8 */
    int interleave;   /* directions marched together by one wave: 1, 2, 3 or 4 */
} art_tuning;

/* Create a mesh of nx*ny*nz cubic cells of side cell_size (> 0).
 * Ownership: *out is owned by the library until art_destroy_mesh. */
int art_create_mesh(int nx, int ny, int nz, double cell_size, art_mesh **out);

/* Release the mesh and all its device memory (NULL is accepted).
 * ART_E_STATE, and nothing is released, while a live batch holds the mesh. */
int art_destroy_mesh(art_mesh *mesh);

/* Load the absorption coefficient kappa (>= 0, finite) and source function S
 * (finite) of nbins frequency bins (1..ART_MAX_BINS), each [nbins][nz][ny][nx]
 * float32, from device memory (on_device = 1) or host memory (on_device = 0).
 * The library copies and re-lays out the data (Sect. 3: mesh data are moved to
 * the accelerator before the sweep); the caller keeps ownership of its arrays.
 * The values are checked before anything is written, and hip_stream is
 * synchronised to report invalid ones: ART_E_INVAL leaves the mesh with the
 * fields it had (a mesh with valid fields stays ready to sweep).  While a
 * live batch holds the mesh, a different bin count gives ART_E_STATE (new
 * values of the same bin count are fine: later replays use them). */
int art_set_fields(art_mesh *mesh, int nbins, const float *kappa, const float *S,
                   int on_device, void *hip_stream);

/* Weights of the diffuse photo-heating rate (eq heat_diff, Sect. 2.2): the
 * Heat output of later sweeps of this mesh (plain and batched; a batch takes
 * the weights at art_batch_create) is sum_b heat_in[b] J_in_b +
 * heat_src[b] S_b.  In the paper's monochromatic form, heat_in is
 * 4 pi int sigma (1 - nu_0 / nu) dnu over the bin and heat_src the factor
 * of the local recombination term (half the gamma_w of that term times
 * h dnu_th); with a nonparametric spectrum of rectangular bins both are
 * 4 pi int_bin sigma (1 - nu_i / nu) dnu.  heat_in, heat_src: host arrays
 * [nbins] (NULL: all 0), finite.  ART_E_STATE before art_set_fields; a new
 * bin count resets the weights to 0. */
int art_set_heating(art_mesh *mesh, const float *heat_in, const float *heat_src);

/* Full sweep over the 12 nside^2 HEALPix directions (Sect. 2.2-2.3).
 * gamma_w: host array [nbins] of rate weights (NULL = all 1).  I_bc: uniform
 * intensity entering the box (Sect. 3.1 casts rays from the boundaries).
 * out: caller-owned device buffers (see art_outputs).  The direction tables
 * of the last (nside, direction range, I_bc) are kept on the device and
 * reused.  Buffers grow on the first sweep at a larger Nside (this
 * synchronises the device); while a live batch holds the mesh such a sweep
 * gives ART_E_STATE instead.  Device memory beyond the fields and outputs:
 * per direction the ray-state slots (NB floats per lattice ray) and the
 * block-face buffers (NB floats x (32 depth + 64) per block of the largest
 * cross-section, depth the tuned block depth), and per bucket one
 * accumulator copy (2 NB floats per cell): about 3 + 3 + 13 GB at 256^3,
 * Nside 8, 4 bins.  ART_E_UNSUPPORTED when one bucket's slots or face
 * buffers would exceed 2 GiB. */
int art_sweep(art_mesh *mesh, int nside, const float *gamma_w, float I_bc,
              const art_outputs *out, void *hip_stream);

/* Raw direction sums over the HEALPix directions [d_begin, d_end) only (the
 * direction split of Sect. 3.2): A1[b][c] = sum_d mean of the path-averaged
 * incoming intensity, A2[b][c] = sum_d mean of (1 - (1 - e^{-dtau})/dtau),
 * both [nbins][cells] device float32 (A2 may be NULL).  J_in = A1 / N_d after
 * summing the ranges of all devices. */
int art_sweep_range(art_mesh *mesh, int nside, int d_begin, int d_end, float I_bc,
                    float *A1, float *A2, void *hip_stream);

/* Work and time of the last sweep of this mesh (synchronises with it):
 * segments = ray-cell segments of positive length marched (per bin; the work
 * unit of one bin is one segment update), march_ms = time from the first to
 * the end of the last march launch, sweep_ms = time from the direction
 * generator to the end of the rates; both from HIP events recorded on the
 * sweep's stream.  Any pointer may be NULL.
 * ART_E_STATE if no sweep has run. */
int art_sweep_stats(art_mesh *mesh, long long *segments, float *march_ms, float *sweep_ms);

/* Launch-shape control.  art_set_tuning validates and stores t for later
 * sweeps of this mesh (ART_E_INVAL if outside the limits, ART_E_UNSUPPORTED if
 * the block's accumulators exceed the workgroup's local memory, ART_E_STATE
 * while a live batch holds the mesh). */
int art_set_tuning(art_mesh *mesh, const art_tuning *t);
int art_get_tuning(const art_mesh *mesh, art_tuning *t);

/* Autotuner: for this mesh (fields set) and Nside, run a warm-up and a timed
 * sweep (HIP events around direction setup, march and normalisation) with
 * each candidate launch shape (candidates NULL: depth in {4, 6, 8, 12} x
 * interleave in {2, 3, 4}, one subset, one wave), keep the fastest on the mesh,
 * and return it in *best and its sweep time in *best_ms (either may be NULL).
 * Candidates the mesh cannot run (local-memory limit) are skipped; on error
 * the mesh keeps its previous tuning.  Synchronises hip_stream and holds a
 * scratch output of nbins x cells floats while it runs.  ART_E_STATE while a
 * live batch holds the mesh. */
int art_autotune(art_mesh *mesh, int nside, const art_tuning *candidates, int ncand,
                 art_tuning *best, float *best_ms, void *hip_stream);

/* Autotuner with a process-wide cache keyed by (shape class, Nside, bins),
 * the shape class being floor(log2(cells) / 2) (meshes within about a factor
 * of 4 in cell count share it): a cached shape is set on the mesh without
 * timing (*cached = 1), else art_autotune runs and its result is cached
 * (*cached = 0).  best, best_ms, cached may be NULL.  ART_E_STATE while a
 * live batch holds the mesh.  The cache is shared by all threads. */
int art_autotune_class(art_mesh *mesh, int nside, const art_tuning *candidates, int ncand,
                       art_tuning *best, float *best_ms, int *cached, void *hip_stream);

/* The autotune cache as a text file: op 0 clears it (path unused), 1 writes
 * it to path, 2 merges the entries of path into it (ART_E_INVAL, the cache
 * unchanged, for a file that is not a cache or holds an invalid entry). */
int art_tune_cache(int op, const char *path);

/* Batched form: one launch sequence for n distinct meshes (each already
 * holding fields, each with its own shape, Nside, bins and tuning), captured
 * once into a HIP graph.  Launch w of the sequence marches wavefront w of
 * every mesh.  nside[i], gamma_w[i] (host array of the mesh's bins, or NULL),
 * outs[i] (caller-owned device buffers, which must outlive the batch) as in
 * art_sweep; exit sums are not produced (outs[i].exit_sum is ignored).  waves:
 * waves per workgroup for all meshes, 1..8.  art_batch_create runs no sweep:
 * it builds each mesh's direction tables on hip_stream and synchronises it;
 * the graph holds the march launches and the normalisations.
 * art_batch_launch replays the graph on hip_stream (asynchronous), first
 * rebuilding the tables of any mesh that a plain sweep at another Nside,
 * range or I_bc has used since; art_batch_stats synchronises with the last
 * launch and returns the segment-bin updates it performed and its HIP-event
 * time.  The meshes' buffers are captured in the graph, so while the batch
 * exists each mesh refuses (ART_E_STATE) whatever would reallocate or
 * re-shape them: re-tuning, autotuning, a different bin count, a sweep at a
 * larger Nside, and art_destroy_mesh.  Work on one mesh queued on two streams
 * at once races. */
typedef struct art_batch art_batch;
int art_batch_create(art_mesh *const *meshes, const int *nside, int n, const float *const *gamma_w,
                     float I_bc, const art_outputs *outs, int waves, art_batch **out,
                     void *hip_stream);
int art_batch_launch(art_batch *batch, void *hip_stream);
int art_batch_stats(art_batch *batch, long long *segment_bins, float *ms);
int art_batch_destroy(art_batch *batch);

/* The batched form under the names of its graph: art_sweep_batched creates
 * the batch of n meshes (I_bc = 0, one wave per workgroup) as *graph and
 * replays it once on hip_stream; art_graph_launch replays it again;
 * art_graph_destroy releases it.  Same rules as art_batch_create. */
typedef struct art_batch art_graph;
int art_sweep_batched(art_mesh *const *meshes, const int *nside, int n,
                      const float *const *gamma_w, const art_outputs *outs, art_graph **graph,
                      void *hip_stream);
int art_graph_launch(art_graph *graph, void *hip_stream);
int art_graph_destroy(art_graph *graph);

/* The block-wavefront schedule a sweep of an nx x ny x nz mesh with launch
 * shape t runs (host only, no device work; Sect. 3.1 and 3.3: single writers
 * without atomics, each block after the blocks its rays come from).  Work
 * item q is (wavefront w, block, bucket): items[3q..3q+2].  Buckets are
 * (a * 8 + octant) * subsets + subset for dominant axis a (x = 0, y = 1,
 * z = 2) and octant bit i set when the rays travel towards decreasing x_i;
 * block = (pa * nbc + pc) * nbb + pb indexes the 8 x 8 x depth blocks along
 * (a, c, b), b < c the other two axes, nbb, nbc the block counts along b, c.
 * Launch w of a sweep runs the items of wavefront w.  *n = item count,
 * *nwave = wavefront count (may be NULL); items may be NULL to query n,
 * else it must hold cap >= n triples (ART_E_INVAL otherwise). */
int art_schedule(int nx, int ny, int nz, const art_tuning *t, int *items, long long cap,
                 long long *n, int *nwave);

/* Number of directions of an Nside (12 nside^2), or ART_E_INVAL. */
int art_ndirs(int nside);

/* Description of the last error on this thread ("" if none). */
const char *art_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ART_H */
