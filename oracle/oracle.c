/*
 * oracle.c -- plain FP64 CPU reference of the diffuse-radiation ray-tracing
 * sweep of Tanaka, Yoshikawa, Okamoto & Hasegawa, "A new ray-tracing scheme
 * for 3D diffuse radiation transfer on highly parallel architectures"
 * (PASJ; arXiv:1410.0763), Sect. 2.2 (eqs rt, path_averaged_intensity,
 * averaged_intensity, mean_intensity), Sect. 2.3 (HEALPix directions) and
 * Sect. 3.1 (ray grouping).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP implementation; the product
 * path never calls it.
 *
 * Everything is double precision and deliberately simple:
 *   - directions are HEALPix RING pixel centres written from the formulas of
 *     Gorski et al. (2005), the package the paper uses (Sect. 2.3);
 *   - a ray's cell segments are found by collecting every integer-plane
 *     crossing along the ray, sorting them, and taking the cell that contains
 *     the midpoint of each consecutive pair (no incremental stepping);
 *   - the per-(direction, cell) averages are normalised literally with the
 *     optical-depth weights of eq averaged_intensity, direction by direction;
 *   - OpenMP runs the rays of one ray group (Sect. 3.1) in parallel: rays of a
 *     group never share a cell, so the per-direction scratch needs no locks.
 *
 * Readings of points the paper leaves open:
 *   Q1 ray lattice: for direction n with dominant axis a (sign sig) and the
 *      other two axes b < c, ray (j,k) is the line
 *         x_a = s (sig>0) or N_a - s (sig<0),  x_b = j + 1/2 + t_b s,
 *         x_c = k + 1/2 + t_c s,   t_b = n_b/|n_a|, t_c = n_c/|n_a|,
 *      for depth s in [0, N_a], in cell units; every (j,k) whose chord through
 *      the box is positive is cast.  Ray spacing equals the cell size.
 *   Q2 dominant-axis ties: the lowest axis index among the components within
 *      1e-12 of the largest |n_i|.  Components below 1e-12 are set to zero.
 *   Q3 kappa = 0: the optical-depth weights are 0/0; the limit (path-length
 *      weights, phi(0) = 1) is used.
 *   Q4 the paper's J = J_in + S (eq mean_intensity) is returned, and in
 *      addition J_exact = J_in + S * <1 - phi>, the exact path average of the
 *      formal solution (eq rad_tr2) with constant S in a cell.
 *   Q5 Gamma = sum_b g_b (J_in_b + S_b) with caller weights g_b: the affine
 *      form of eq gamma_diff with the frequency integral folded into g_b.
 *   Q6 the intensity entering the box is a uniform I_bc.
 *
 * Point sources (Sect. 2.3 and Appendix A; oracle_point, oracle_point_pair
 * at the end of this file) use the same crossing-and-midpoint segment
 * finder along the line from the source to each cell's centre.  Readings:
 *   P1 one absorbing species, rates per absorber, frequency integrals as sums
 *      over the bins with per-bin photon rates Q_b and energies e_b;
 *   P2 the line runs from the source through the cell's centre; r_in = 0 when
 *      the source lies in the cell; a source at the centre takes +x;
 *   P3 the shell r_in..r_out holds n_c (4 pi / 3)(r_out^3 - r_in^3) h^3
 *      absorbers; tau runs from the source to r_in.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_TIE 1e-12
#define ORACLE_SLIVER 1e-12

/* ------------------------------------------------------------------------ */
/* Directions: HEALPix RING pixel centres (Sect. 2.3; Gorski et al. 2005).   */
/* Rings i = 1 .. 4N-1 from north to south; pixels j = 1 .. ring size.      */
/* ------------------------------------------------------------------------ */
int oracle_ndirs(int nside) { return 12 * nside * nside; }

int oracle_directions(int nside, double *n_out)
{
    if (nside < 1) return -1;
    const double N = (double)nside;
    int idx = 0;
    for (int i = 1; i <= 4 * nside - 1; ++i) {
        double z;
        int npix;
        double dphi, phi0;
        if (i < nside) {                      /* north polar cap */
            z = 1.0 - (double)i * i / (3.0 * N * N);
            npix = 4 * i;
            dphi = M_PI / (2.0 * i);
            phi0 = 0.5 * dphi;                /* phi = dphi (j - 1/2) */
        } else if (i <= 3 * nside) {          /* equatorial belt */
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * N);
            npix = 4 * nside;
            dphi = M_PI / (2.0 * N);
            /* phi = dphi (j - s/2) with s = (i - N + 1) mod 2; rings with s = 0
               are numbered from phi = 0 as in the HEALPix library */
            int s = (i - nside + 1) % 2;
            phi0 = s ? 0.5 * dphi : 0.0;
        } else {                              /* south polar cap: mirror */
            int ip = 4 * nside - i;
            z = -(1.0 - (double)ip * ip / (3.0 * N * N));
            npix = 4 * ip;
            dphi = M_PI / (2.0 * ip);
            phi0 = 0.5 * dphi;
        }
        double st = sqrt((1.0 - z) * (1.0 + z));
        for (int j = 0; j < npix; ++j) {
            double phi = phi0 + dphi * j;
            double v[3] = {st * cos(phi), st * sin(phi), z};
            for (int q = 0; q < 3; ++q)
                if (fabs(v[q]) < ORACLE_TIE) v[q] = 0.0;
            n_out[3 * idx + 0] = v[0];
            n_out[3 * idx + 1] = v[1];
            n_out[3 * idx + 2] = v[2];
            ++idx;
        }
    }
    return idx;
}

/* ------------------------------------------------------------------------ */
/* Parallel-ray lattice of one direction (Sect. 2.2, Fig. parallel_ray;      */
/* reading Q1/Q2 above).                                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int a, b, c;      /* dominant axis and the two others (b < c) */
    int sig;          /* +1: rays travel towards +x_a, -1: towards -x_a */
    double w;         /* |n_a|: unit depth is a path length of 1/w cells */
    double tb, tc;    /* transverse slopes n_b/|n_a|, n_c/|n_a| */
} odir_t;

static void dir_geom(const double *n, odir_t *g)
{
    double m = fmax(fabs(n[0]), fmax(fabs(n[1]), fabs(n[2])));
    int a = 0;
    while (fabs(n[a]) < m - ORACLE_TIE) ++a;
    int b = (a == 0) ? 1 : 0;
    int c = (a == 2) ? 1 : 2;
    g->a = a; g->b = b; g->c = c;
    g->sig = n[a] > 0.0 ? 1 : -1;
    g->w = fabs(n[a]);
    g->tb = n[b] / g->w;
    g->tc = n[c] / g->w;
}

/* Position of ray (j,k) at depth s, in world axes (cell units). */
static void ray_pos(const odir_t *g, const int *N, int j, int k, double s, double *p)
{
    p[g->a] = g->sig > 0 ? s : (double)N[g->a] - s;
    p[g->b] = j + 0.5 + g->tb * s;
    p[g->c] = k + 0.5 + g->tc * s;
}

/* Depth interval where x0 + t s lies in (0, L); returns 0 if empty. */
static int clip_axis(double x0, double t, double L, double *lo, double *hi)
{
    if (t == 0.0) {
        if (x0 > 0.0 && x0 < L) { *lo = -INFINITY; *hi = INFINITY; return 1; }
        return 0;
    }
    double s0 = (0.0 - x0) / t, s1 = (L - x0) / t;
    *lo = fmin(s0, s1);
    *hi = fmax(s0, s1);
    return 1;
}

/* Chord of ray (j,k) through the box, as a depth interval. */
static int ray_clip(const odir_t *g, const int *N, int j, int k, double *sin_, double *sout)
{
    double lo = 0.0, hi = (double)N[g->a], l, h;
    if (!clip_axis(j + 0.5, g->tb, (double)N[g->b], &l, &h)) return 0;
    lo = fmax(lo, l); hi = fmin(hi, h);
    if (!clip_axis(k + 0.5, g->tc, (double)N[g->c], &l, &h)) return 0;
    lo = fmax(lo, l); hi = fmin(hi, h);
    *sin_ = lo; *sout = hi;
    return hi > lo;
}

/* Conservative lattice index ranges [jlo, jhi] x [klo, khi]. */
static void lattice_range(const odir_t *g, const int *N, int *jlo, int *jhi, int *klo, int *khi)
{
    double Na = (double)N[g->a];
    *jlo = (int)floor(-0.5 - fmax(0.0, g->tb * Na)) - 1;
    *jhi = (int)ceil((double)N[g->b] - 0.5 - fmin(0.0, g->tb * Na)) + 1;
    *klo = (int)floor(-0.5 - fmax(0.0, g->tc * Na)) - 1;
    *khi = (int)ceil((double)N[g->c] - 0.5 - fmin(0.0, g->tc * Na)) + 1;
}

static int cmp_double(const void *x, const void *y)
{
    double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

/*
 * Cell segments of ray (j,k): every depth where the line crosses an integer
 * plane of any axis inside the chord, sorted; each consecutive pair with a
 * positive gap is one segment, in the cell that holds its midpoint.
 * Writes cell index (x fastest), path length (cell units times h) and the
 * segment's entry depth.  Returns the number of segments.
 */
static int ray_segments(const odir_t *g, const int *N, double h, int j, int k,
                        double *buf, int *cell, double *dl, double *s0)
{
    double si, so;
    if (!ray_clip(g, N, j, k, &si, &so)) return 0;
    int nb = 0;
    buf[nb++] = si;
    buf[nb++] = so;
    double p0[3], p1[3];
    ray_pos(g, N, j, k, si, p0);
    ray_pos(g, N, j, k, so, p1);
    for (int ax = 0; ax < 3; ++ax) {
        double lo = fmin(p0[ax], p1[ax]), hi = fmax(p0[ax], p1[ax]);
        for (double m = floor(lo) + 1.0; m < hi; m += 1.0) {
            double s;
            if (ax == g->a) s = g->sig > 0 ? m : (double)N[g->a] - m;
            else if (ax == g->b) s = (m - (j + 0.5)) / g->tb;
            else s = (m - (k + 0.5)) / g->tc;
            if (s > si && s < so) buf[nb++] = s;
        }
    }
    qsort(buf, nb, sizeof(double), cmp_double);
    int ns = 0;
    for (int q = 0; q + 1 < nb; ++q) {
        double sa = buf[q], sb = buf[q + 1];
        /* Crossings that coincide in exact arithmetic (a ray through a cell
           edge or corner) come out a few ulps apart; such slivers are contacts
           of zero length and are not segments. */
        if (!(sb - sa > ORACLE_SLIVER)) continue;
        double pm[3];
        ray_pos(g, N, j, k, 0.5 * (sa + sb), pm);
        int ci[3];
        for (int ax = 0; ax < 3; ++ax) {
            int v = (int)floor(pm[ax]);
            if (v < 0) v = 0;
            if (v > N[ax] - 1) v = N[ax] - 1;
            ci[ax] = v;
        }
        const int cid = (ci[2] * N[1] + ci[1]) * N[0] + ci[0];
        if (ns > 0 && cell[ns - 1] == cid) {
            /* the same cell on both sides of a dropped sliver: one visit */
            dl[ns - 1] = (sb - s0[ns - 1]) * h / g->w;
            continue;
        }
        cell[ns] = cid;
        dl[ns] = (sb - sa) * h / g->w;
        s0[ns] = sa;
        ++ns;
    }
    return ns;
}

static int max_crossings(const int *N) { return N[0] + N[1] + N[2] + 8; }

/* ------------------------------------------------------------------------ */
/* Exported geometry helpers (used by the brute-force tests).               */
/* ------------------------------------------------------------------------ */
int oracle_dir_geom(int nside, int d, double *out /* a,b,c,sig,w,tb,tc */)
{
    int nd = oracle_ndirs(nside);
    if (d < 0 || d >= nd) return -1;
    double *n = (double *)malloc(sizeof(double) * 3 * nd);
    oracle_directions(nside, n);
    odir_t g;
    dir_geom(n + 3 * d, &g);
    free(n);
    out[0] = g.a; out[1] = g.b; out[2] = g.c; out[3] = g.sig;
    out[4] = g.w; out[5] = g.tb; out[6] = g.tc;
    return 0;
}

int oracle_lattice(int nx, int ny, int nz, int nside, int d, int *range /* jlo,jhi,klo,khi */)
{
    int N[3] = {nx, ny, nz};
    double geo[7];
    if (oracle_dir_geom(nside, d, geo)) return -1;
    odir_t g = {(int)geo[0], (int)geo[1], (int)geo[2], (int)geo[3], geo[4], geo[5], geo[6]};
    lattice_range(&g, N, range, range + 1, range + 2, range + 3);
    return 0;
}

int oracle_ray_segments(int nx, int ny, int nz, double h, int nside, int d, int j, int k,
                        int *cell, double *dl, double *s0, int maxseg)
{
    int N[3] = {nx, ny, nz};
    double geo[7];
    if (oracle_dir_geom(nside, d, geo)) return -1;
    odir_t g = {(int)geo[0], (int)geo[1], (int)geo[2], (int)geo[3], geo[4], geo[5], geo[6]};
    int mc = max_crossings(N);
    if (maxseg < mc) return -2;
    double *buf = (double *)malloc(sizeof(double) * mc);
    int ns = ray_segments(&g, N, h, j, k, buf, cell, dl, s0);
    free(buf);
    return ns;
}

/* ------------------------------------------------------------------------ */
/* The sweep (Sect. 2.2), over the directions [d_begin, d_end).             */
/*                                                                          */
/* Outputs (any may be NULL), cells in x-fastest order, bins outermost:     */
/*   jin_sum[b][c] = sum_d  Ibar^{ave,in}_b(n_d, c)   (eq averaged_intensity) */
/*   ex_sum[b][c]  = sum_d  <1 - phi>_b(n_d, c)        (reading Q4)          */
/*   exit_sum[d][b] = sum over rays of (I_exit - I_bc)  (d indexes all N_d) */
/*   stats[0] = number of segments with positive length (one bin)           */
/*   stats[1] = max |w * sum_j dL_j / h - 1| over (direction, cell)         */
/*   stats[2] = max number of crossings of one cell by one ray group        */
/* Returns 0 on success.                                                    */
/* ------------------------------------------------------------------------ */
int oracle_sweep(int nx, int ny, int nz, double h, int nbins,
                 const double *kappa, const double *S,
                 int nside, int d_begin, int d_end, double I_bc,
                 double *jin_sum, double *ex_sum, double *exit_sum,
                 double *stats, int nthreads)
{
    const int N[3] = {nx, ny, nz};
    const int64_t ncell = (int64_t)nx * ny * nz;
    const int nd = oracle_ndirs(nside);
    if (nx < 1 || ny < 1 || nz < 1 || nbins < 1 || nside < 1 || !(h > 0.0)) return -1;
    if (d_begin < 0 || d_end > nd || d_begin > d_end) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double *n = (double *)malloc(sizeof(double) * 3 * nd);
    oracle_directions(nside, n);

    const int64_t nsc = ncell * nbins;
    double *num = (double *)malloc(sizeof(double) * nsc);   /* sum dtau * Ibar_in */
    double *den = (double *)malloc(sizeof(double) * nsc);   /* sum dtau */
    double *numL = (double *)malloc(sizeof(double) * nsc);  /* sum dL * Ibar_in  (Q3) */
    double *denL = (double *)malloc(sizeof(double) * ncell); /* sum dL */
    double *exL = (double *)malloc(sizeof(double) * nsc);   /* sum dL * (1 - phi) (Q4) */
    int *hits = (int *)malloc(sizeof(int) * ncell);         /* crossings per group */
    if (!n || !num || !den || !numL || !denL || !exL || !hits) {
        free(n); free(num); free(den); free(numL); free(denL); free(exL); free(hits);
        return -2;
    }
    if (jin_sum) memset(jin_sum, 0, sizeof(double) * nsc);
    if (ex_sum) memset(ex_sum, 0, sizeof(double) * nsc);
    if (exit_sum) memset(exit_sum, 0, sizeof(double) * (size_t)nd * nbins);
    double nseg_total = 0.0, inv_err = 0.0;
    int max_hits = 0;
    const int mc = max_crossings(N);

    for (int d = d_begin; d < d_end; ++d) {
        odir_t g;
        dir_geom(n + 3 * d, &g);
        memset(num, 0, sizeof(double) * nsc);
        memset(den, 0, sizeof(double) * nsc);
        memset(numL, 0, sizeof(double) * nsc);
        memset(denL, 0, sizeof(double) * ncell);
        memset(exL, 0, sizeof(double) * nsc);
        int jlo, jhi, klo, khi;
        lattice_range(&g, N, &jlo, &jhi, &klo, &khi);
        const int nj = jhi - jlo + 1, nk = khi - klo + 1;
        double *exit_d = exit_sum ? exit_sum + (size_t)d * nbins : NULL;

        /* Ray groups (Sect. 3.1): rays from 2x2-interleaved lattice points. */
        for (int grp = 0; grp < 4; ++grp) {
            const int pj = grp & 1, pk = grp >> 1;
            memset(hits, 0, sizeof(int) * ncell);
            double seg_grp = 0.0;
            int nrays = nj * nk;
#pragma omp parallel reduction(+ : seg_grp)
            {
                double *buf = (double *)malloc(sizeof(double) * mc);
                int *cell = (int *)malloc(sizeof(int) * mc);
                double *dl = (double *)malloc(sizeof(double) * mc);
                double *s0 = (double *)malloc(sizeof(double) * mc);
                double *I = (double *)malloc(sizeof(double) * nbins);
                double *exit_loc = (double *)calloc(nbins, sizeof(double));
#pragma omp for schedule(dynamic, 16)
                for (int r = 0; r < nrays; ++r) {
                    int j = jlo + r % nj, k = klo + r / nj;
                    if ((((j % 2) + 2) % 2) != pj || (((k % 2) + 2) % 2) != pk) continue;
                    int ns = ray_segments(&g, N, h, j, k, buf, cell, dl, s0);
                    if (ns == 0) continue;
                    for (int b = 0; b < nbins; ++b) I[b] = I_bc;
                    for (int q = 0; q < ns; ++q) {
                        const int64_t c = cell[q];
                        hits[c] += 1;   /* rays of one group never share a cell */
                        denL[c] += dl[q];
                        seg_grp += 1.0;
                        for (int b = 0; b < nbins; ++b) {
                            const int64_t bc = (int64_t)b * ncell + c;
                            const double dtau = kappa[bc] * dl[q];          /* eq rt */
                            const double one_m_e = -expm1(-dtau);           /* 1 - e^{-dtau} */
                            const double phi = dtau > 0.0 ? one_m_e / dtau : 1.0;
                            const double ibar_in = I[b] * phi;              /* path-averaged I_in */
                            num[bc] += dtau * ibar_in;                      /* eq averaged_intensity */
                            den[bc] += dtau;
                            numL[bc] += dl[q] * ibar_in;                    /* Q3 limit weights */
                            exL[bc] += dl[q] * (1.0 - phi);                 /* Q4 */
                            I[b] = I[b] * exp(-dtau) + S[bc] * one_m_e;     /* eq rt */
                        }
                    }
                    if (exit_d)
                        for (int b = 0; b < nbins; ++b) exit_loc[b] += I[b] - I_bc;
                }
                if (exit_d) {
#pragma omp critical
                    for (int b = 0; b < nbins; ++b) exit_d[b] += exit_loc[b];
                }
                free(buf); free(cell); free(dl); free(s0); free(I); free(exit_loc);
            }
            nseg_total += seg_grp;
            for (int64_t c = 0; c < ncell; ++c)
                if (hits[c] > max_hits) max_hits = hits[c];
        }

        /* Per-(direction, cell) averages, then the direction sum of eq mean_intensity. */
        double inv_loc = 0.0;
#pragma omp parallel for reduction(max : inv_loc)
        for (int64_t c = 0; c < ncell; ++c) {
            const double inv = fabs(denL[c] * g.w / h - 1.0);
            if (inv > inv_loc) inv_loc = inv;
            for (int b = 0; b < nbins; ++b) {
                const int64_t bc = (int64_t)b * ncell + c;
                double ave_in;
                if (den[bc] > 0.0) ave_in = num[bc] / den[bc];          /* eq averaged_intensity */
                else ave_in = denL[c] > 0.0 ? numL[bc] / denL[c] : 0.0; /* Q3 */
                if (jin_sum) jin_sum[bc] += ave_in;
                if (ex_sum && denL[c] > 0.0) ex_sum[bc] += exL[bc] / denL[c];
            }
        }
        if (inv_loc > inv_err) inv_err = inv_loc;
    }
    if (stats) {
        stats[0] = nseg_total;
        stats[1] = inv_err;
        stats[2] = (double)max_hits;
    }
    free(n); free(num); free(den); free(numL); free(denL); free(exL); free(hits);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The same sums as oracle_sweep, at chosen cells only (Sect. 2.2, eq       */
/* averaged_intensity; readings Q3/Q4): for each direction, the rays that   */
/* cross cell c are found by enumerating every lattice ray whose transverse */
/* position can reach the cell's box over the cell's depth interval, and    */
/* each is marched from its entry up to the cell.  This lets single cells   */
/* of a large mesh be checked without sweeping all of it.                   */
/*   jin_sum[b][i], ex_sum[b][i] for cells[i] (x-fastest cell index).       */
/* Returns 0 on success.                                                    */
/* ------------------------------------------------------------------------ */
int oracle_cells(int nx, int ny, int nz, double h, int nbins,
                 const double *kappa, const double *S,
                 int nside, int d_begin, int d_end, double I_bc,
                 const int64_t *cells, int ncells, double *jin_sum, double *ex_sum,
                 int nthreads)
{
    const int N[3] = {nx, ny, nz};
    const int64_t ncell = (int64_t)nx * ny * nz;
    const int nd = oracle_ndirs(nside);
    if (nx < 1 || ny < 1 || nz < 1 || nbins < 1 || nside < 1 || !(h > 0.0)) return -1;
    if (d_begin < 0 || d_end > nd || d_begin > d_end || ncells < 0) return -1;
    for (int i = 0; i < ncells; ++i)
        if (cells[i] < 0 || cells[i] >= ncell) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double *n = (double *)malloc(sizeof(double) * 3 * nd);
    if (!n) return -2;
    oracle_directions(nside, n);
    const int mc = max_crossings(N);
    int failed = 0;

#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
    for (int i = 0; i < ncells; ++i) {
        const int64_t cid = cells[i];
        const int cx[3] = {(int)(cid % nx), (int)((cid / nx) % ny), (int)(cid / ((int64_t)nx * ny))};
        double *buf = (double *)malloc(sizeof(double) * mc);
        int *cell = (int *)malloc(sizeof(int) * mc);
        double *dl = (double *)malloc(sizeof(double) * mc);
        double *s0 = (double *)malloc(sizeof(double) * mc);
        double *I = (double *)malloc(sizeof(double) * nbins);
        double *num = (double *)malloc(sizeof(double) * nbins);
        double *den = (double *)malloc(sizeof(double) * nbins);
        double *numL = (double *)malloc(sizeof(double) * nbins);
        double *exL = (double *)malloc(sizeof(double) * nbins);
        if (!buf || !cell || !dl || !s0 || !I || !num || !den || !numL || !exL) {
            failed = 1;
        } else {
            for (int b = 0; b < nbins; ++b) {
                if (jin_sum) jin_sum[(int64_t)b * ncells + i] = 0.0;
                if (ex_sum) ex_sum[(int64_t)b * ncells + i] = 0.0;
            }
            for (int d = d_begin; d < d_end; ++d) {
                odir_t g;
                dir_geom(n + 3 * d, &g);
                /* depth interval of the cell's slab along the dominant axis */
                double slo = g.sig > 0 ? cx[g.a] : (double)N[g.a] - cx[g.a] - 1.0;
                double shi = slo + 1.0;
                /* lattice rays whose transverse position can be inside the cell */
                const double b0 = g.tb * slo, b1 = g.tb * shi, c0 = g.tc * slo, c1 = g.tc * shi;
                const int jlo = (int)floor(cx[g.b] - 0.5 - fmax(b0, b1)) - 1;
                const int jhi = (int)ceil(cx[g.b] + 0.5 - fmin(b0, b1)) + 1;
                const int klo = (int)floor(cx[g.c] - 0.5 - fmax(c0, c1)) - 1;
                const int khi = (int)ceil(cx[g.c] + 0.5 - fmin(c0, c1)) + 1;
                double denL = 0.0;
                for (int b = 0; b < nbins; ++b) num[b] = den[b] = numL[b] = exL[b] = 0.0;
                for (int k = klo; k <= khi; ++k) {
                    for (int j = jlo; j <= jhi; ++j) {
                        const int ns = ray_segments(&g, N, h, j, k, buf, cell, dl, s0);
                        int hit = -1;
                        for (int q = 0; q < ns; ++q)
                            if (cell[q] == cid) { hit = q; break; }
                        if (hit < 0) continue;
                        for (int b = 0; b < nbins; ++b) I[b] = I_bc;
                        for (int q = 0; q <= hit; ++q) {
                            const int64_t c = cell[q];
                            for (int b = 0; b < nbins; ++b) {
                                const int64_t bc = (int64_t)b * ncell + c;
                                const double dtau = kappa[bc] * dl[q];          /* eq rt */
                                const double one_m_e = -expm1(-dtau);
                                const double phi = dtau > 0.0 ? one_m_e / dtau : 1.0;
                                if (q == hit) {                                 /* eq averaged_intensity */
                                    num[b] += dtau * I[b] * phi;
                                    den[b] += dtau;
                                    numL[b] += dl[q] * I[b] * phi;              /* Q3 */
                                    exL[b] += dl[q] * (1.0 - phi);              /* Q4 */
                                }
                                I[b] = I[b] * exp(-dtau) + S[bc] * one_m_e;     /* eq rt */
                            }
                        }
                        denL += dl[hit];
                    }
                }
                for (int b = 0; b < nbins; ++b) {
                    double ave_in;
                    if (den[b] > 0.0) ave_in = num[b] / den[b];
                    else ave_in = denL > 0.0 ? numL[b] / denL : 0.0;
                    if (jin_sum) jin_sum[(int64_t)b * ncells + i] += ave_in;
                    if (ex_sum && denL > 0.0) ex_sum[(int64_t)b * ncells + i] += exL[b] / denL;
                }
            }
        }
        free(buf); free(cell); free(dl); free(s0); free(I);
        free(num); free(den); free(numL); free(exL);
    }
    free(n);
    return failed ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Point sources (Sect. 2.3, RT from point radiation sources, and the       */
/* photon-conserving rates of Appendix A).                                  */
/*                                                                          */
/* Source at p (cell units, inside the closed box), target cell c with     */
/* centre q.  The light ray is the line from p through q, unit direction   */
/* u = (q - p) / |q - p| (reading P2: u = +x when p == q).  r_in and r_out  */
/* are the distances from p where the line enters and leaves cell c        */
/* (r_in = 0 when p lies in c).  tau_b sums kappa_b h dl over the cells the */
/* line crosses before c; dtau_b = kappa_b(c) h (r_out - r_in) is the       */
/* radial optical depth of the imaginary shell r_in..r_out.  The photons    */
/* the shell absorbs per unit time are Q_b e^{-tau_b} (1 - e^{-dtau_b})     */
/* (Q_b: photon rate of the source in bin b); divided by the absorbers in   */
/* the shell, n_c (4 pi / 3)(r_out^3 - r_in^3) h^3, they give the rate per  */
/* absorber (eq pc_gamma with one absorbing species, so that the species'   */
/* share of dtau is 1), and weighted by e_b (the energy per absorbed photon */
/* above threshold) the heating rate per absorber.  Sums over sources and   */
/* bins.  Cells with n_c <= 0 get 0.                                        */
/* ------------------------------------------------------------------------ */

/* Segments of the line from p towards cell c, up to where it enters c:
   every integer-plane crossing in (0, r_in) sorted; a gap longer than a
   sliver belongs to the cell holding its midpoint.  Writes the cells and
   lengths (cell units) of the segments before c, r_in and r_out; returns the
   number of segments. */
static int point_path(const int *N, const double *p, const int *c, double *buf, int *cell,
                      double *len, double *r_in, double *r_out)
{
    double q[3], u[3], dist = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        q[ax] = c[ax] + 0.5;
        u[ax] = q[ax] - p[ax];
        dist += u[ax] * u[ax];
    }
    dist = sqrt(dist);
    if (dist > 0.0) {
        for (int ax = 0; ax < 3; ++ax) u[ax] /= dist;
    } else {
        u[0] = 1.0; u[1] = 0.0; u[2] = 0.0;
    }
    /* slab intersection of the line with the cell's box */
    double tin = -INFINITY, tout = INFINITY;
    for (int ax = 0; ax < 3; ++ax) {
        if (u[ax] == 0.0) continue;       /* then p[ax] = q[ax] lies inside the slab */
        const double t0 = (c[ax] - p[ax]) / u[ax], t1 = (c[ax] + 1.0 - p[ax]) / u[ax];
        tin = fmax(tin, fmin(t0, t1));
        tout = fmin(tout, fmax(t0, t1));
    }
    if (tin < 0.0) tin = 0.0;
    *r_in = tin;
    *r_out = tout;
    int nb = 0;
    buf[nb++] = 0.0;
    buf[nb++] = tin;
    for (int ax = 0; ax < 3; ++ax) {
        if (u[ax] == 0.0) continue;
        const double x1 = p[ax] + u[ax] * tin;
        const double lo = fmin(p[ax], x1), hi = fmax(p[ax], x1);
        for (double m = floor(lo) + 1.0; m < hi; m += 1.0) {
            const double t = (m - p[ax]) / u[ax];
            if (t > 0.0 && t < tin) buf[nb++] = t;
        }
    }
    qsort(buf, nb, sizeof(double), cmp_double);
    int ns = 0;
    for (int k = 0; k + 1 < nb; ++k) {
        const double ta = buf[k], tb = buf[k + 1];
        if (!(tb - ta > ORACLE_SLIVER)) continue;
        int ci[3];
        for (int ax = 0; ax < 3; ++ax) {
            int v = (int)floor(p[ax] + u[ax] * 0.5 * (ta + tb));
            if (v < 0) v = 0;
            if (v > N[ax] - 1) v = N[ax] - 1;
            ci[ax] = v;
        }
        if (ci[0] == c[0] && ci[1] == c[1] && ci[2] == c[2]) continue;   /* rounding at r_in */
        cell[ns] = (ci[2] * N[1] + ci[1]) * N[0] + ci[0];
        len[ns] = tb - ta;
        ++ns;
    }
    return ns;
}

/* One (source, cell) pair: tau[b], dtau[b] (optical depths, h included),
   r_in, r_out (cell units).  Returns 0, or -1 for a bad argument. */
int oracle_point_pair(int nx, int ny, int nz, double h, int nbins, const double *kappa,
                      const double *p, int64_t cid, double *tau, double *dtau,
                      double *r_in, double *r_out)
{
    const int N[3] = {nx, ny, nz};
    const int64_t ncell = (int64_t)nx * ny * nz;
    if (nx < 1 || ny < 1 || nz < 1 || nbins < 1 || !(h > 0.0) || cid < 0 || cid >= ncell) return -1;
    for (int ax = 0; ax < 3; ++ax)
        if (!(p[ax] >= 0.0 && p[ax] <= N[ax])) return -1;
    const int c[3] = {(int)(cid % nx), (int)((cid / nx) % ny), (int)(cid / ((int64_t)nx * ny))};
    const int mc = max_crossings(N);
    double *buf = (double *)malloc(sizeof(double) * mc);
    double *len = (double *)malloc(sizeof(double) * mc);
    int *cell = (int *)malloc(sizeof(int) * mc);
    if (!buf || !len || !cell) { free(buf); free(len); free(cell); return -2; }
    const int ns = point_path(N, p, c, buf, cell, len, r_in, r_out);
    for (int b = 0; b < nbins; ++b) {
        double t = 0.0;
        for (int k = 0; k < ns; ++k) t += kappa[(int64_t)b * ncell + cell[k]] * h * len[k];
        tau[b] = t;
        dtau[b] = kappa[(int64_t)b * ncell + cid] * h * (*r_out - *r_in);
    }
    free(buf); free(len); free(cell);
    return 0;
}

/* Rates at cells[i] (all cells if cells is NULL, ncells = nx ny nz) from
   nsrc sources: pos [nsrc][3], Q [nsrc][nbins], e [nbins] (NULL: Heat not
   written); Gamma, Heat [ncells].  Returns 0, -1 (bad argument), -2. */
int oracle_point(int nx, int ny, int nz, double h, int nbins, const double *kappa,
                 const double *n_abs, int nsrc, const double *pos, const double *Q,
                 const double *e, const int64_t *cells, int ncells, double *Gamma,
                 double *Heat, int nthreads)
{
    const int N[3] = {nx, ny, nz};
    const int64_t ncell = (int64_t)nx * ny * nz;
    if (nx < 1 || ny < 1 || nz < 1 || nbins < 1 || !(h > 0.0) || nsrc < 0 || ncells < 0) return -1;
    if (!cells && ncells != ncell) return -1;
    for (int i = 0; cells && i < ncells; ++i)
        if (cells[i] < 0 || cells[i] >= ncell) return -1;
    for (int s = 0; s < nsrc; ++s)
        for (int ax = 0; ax < 3; ++ax)
            if (!(pos[3 * s + ax] >= 0.0 && pos[3 * s + ax] <= N[ax])) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    const int mc = max_crossings(N);
    const double four_pi_3 = 4.0 * M_PI / 3.0;
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : failed)
    for (int i = 0; i < ncells; ++i) {
        const int64_t cid = cells ? cells[i] : i;
        const int c[3] = {(int)(cid % nx), (int)((cid / nx) % ny), (int)(cid / ((int64_t)nx * ny))};
        double *buf = (double *)malloc(sizeof(double) * mc);
        double *len = (double *)malloc(sizeof(double) * mc);
        int *cell = (int *)malloc(sizeof(int) * mc);
        double g = 0.0, ht = 0.0;
        if (!buf || !len || !cell) {
            failed = 1;
        } else if (n_abs[cid] > 0.0) {
            for (int s = 0; s < nsrc; ++s) {
                double rin, rout;
                const int ns = point_path(N, pos + 3 * s, c, buf, cell, len, &rin, &rout);
                /* r_out^3 - r_in^3 in factored form (no cancellation) */
                const double vol = four_pi_3 * h * h * h * (rout - rin) *
                                   (rout * rout + rout * rin + rin * rin);
                const double absorbers = n_abs[cid] * vol;
                for (int b = 0; b < nbins; ++b) {
                    double tau = 0.0;
                    for (int k = 0; k < ns; ++k) tau += kappa[(int64_t)b * ncell + cell[k]] * h * len[k];
                    const double dtau = kappa[(int64_t)b * ncell + cid] * h * (rout - rin);
                    const double nabs_dot = Q[(int64_t)s * nbins + b] * exp(-tau) * -expm1(-dtau);
                    g += nabs_dot / absorbers;
                    if (e) ht += nabs_dot * e[b] / absorbers;
                }
            }
        }
        Gamma[i] = g;
        if (Heat) Heat[i] = e ? ht : 0.0;
        free(buf); free(len); free(cell);
    }
    return failed ? -2 : 0;
}
