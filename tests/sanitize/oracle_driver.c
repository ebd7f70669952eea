/* Drives every entry point of the oracle (oracle/oracle.c) on small ragged
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer:
 * any out-of-bounds access, use after free or undefined operation aborts.
 * Exit status 0 when every call returned 0 and every result is finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_ndirs(int nside);
int oracle_directions(int nside, double *n_out);
int oracle_dir_geom(int nside, int d, double *out);
int oracle_lattice(int nx, int ny, int nz, int nside, int d, int *range);
int oracle_ray_segments(int nx, int ny, int nz, double h, int nside, int d, int j, int k,
                        int *cell, double *dl, double *s0, int maxseg);
int oracle_sweep(int nx, int ny, int nz, double h, int nbins, const double *kappa, const double *S,
                 int nside, int d_begin, int d_end, double I_bc, double *jin_sum, double *ex_sum,
                 double *exit_sum, double *stats, int nthreads);
int oracle_cells(int nx, int ny, int nz, double h, int nbins, const double *kappa, const double *S,
                 int nside, int d_begin, int d_end, double I_bc, const int64_t *cells, int ncells,
                 double *jin_sum, double *ex_sum, int nthreads);
int oracle_point_pair(int nx, int ny, int nz, double h, int nbins, const double *kappa,
                      const double *p, int64_t cid, double *tau, double *dtau, double *r_in,
                      double *r_out);
int oracle_point(int nx, int ny, int nz, double h, int nbins, const double *kappa,
                 const double *n_abs, int nsrc, const double *pos, const double *Q, const double *e,
                 const int64_t *cells, int ncells, double *Gamma, double *Heat, int nthreads);

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static double urand(void)
{
    rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
    return (double)(rs >> 11) * (1.0 / 9007199254740992.0);
}

static int finite_all(const double *a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

#define CHECK(cond, what)                                            \
    do {                                                             \
        if (!(cond)) { fprintf(stderr, "FAIL: %s\n", what); return 1; } \
    } while (0)

int main(void)
{
    const int shapes[4][3] = {{5, 4, 6}, {1, 3, 2}, {7, 1, 1}, {3, 5, 4}};
    for (int si = 0; si < 4; ++si) {
        const int nx = shapes[si][0], ny = shapes[si][1], nz = shapes[si][2], nb = 2;
        const int64_t nc = (int64_t)nx * ny * nz;
        double *k = malloc(sizeof(double) * nb * nc), *S = malloc(sizeof(double) * nb * nc);
        for (int64_t i = 0; i < nb * nc; ++i) {
            k[i] = (i % 7 == 0) ? 0.0 : 3.0 * urand();   /* vacuum cells too */
            S[i] = urand();
        }
        for (int nside = 1; nside <= 4; nside *= 2) {
            const int nd = oracle_ndirs(nside);
            double *n = malloc(sizeof(double) * 3 * nd);
            CHECK(oracle_directions(nside, n) == nd, "directions");
            for (int d = 0; d < nd; ++d) {
                double g[7];
                int r[4];
                CHECK(oracle_dir_geom(nside, d, g) == 0, "dir_geom");
                CHECK(oracle_lattice(nx, ny, nz, nside, d, r) == 0, "lattice");
                const int maxseg = nx + ny + nz + 8;
                int *cell = malloc(sizeof(int) * maxseg);
                double *dl = malloc(sizeof(double) * maxseg), *s0 = malloc(sizeof(double) * maxseg);
                for (int j = r[0]; j <= r[1]; ++j)
                    for (int kk = r[2]; kk <= r[3]; ++kk)
                        CHECK(oracle_ray_segments(nx, ny, nz, 0.7, nside, d, j, kk, cell, dl, s0,
                                                  maxseg) >= 0, "ray_segments");
                free(cell); free(dl); free(s0);
            }
            double *jin = calloc(nb * nc, sizeof(double)), *ex = calloc(nb * nc, sizeof(double));
            double *exs = calloc((size_t)nd * nb, sizeof(double)), st[3];
            CHECK(oracle_sweep(nx, ny, nz, 0.7, nb, k, S, nside, 0, nd, 0.25, jin, ex, exs, st, 2) == 0,
                  "sweep");
            CHECK(finite_all(jin, nb * nc) && finite_all(ex, nb * nc) && finite_all(exs, nd * nb),
                  "sweep finite");
            int64_t cells[3] = {0, nc / 2, nc - 1};
            double cj[6], ce[6];
            CHECK(oracle_cells(nx, ny, nz, 0.7, nb, k, S, nside, 1, nd, 0.25, cells, 3, cj, ce, 2) == 0,
                  "cells");
            CHECK(finite_all(cj, 6) && finite_all(ce, 6), "cells finite");
            free(jin); free(ex); free(exs); free(n);
        }
        double *nab = malloc(sizeof(double) * nc);
        for (int64_t i = 0; i < nc; ++i) nab[i] = (i % 5 == 0) ? 0.0 : 1.0 + urand();
        double pos[9] = {0.0, 0.0, 0.0, nx * urand(), ny * urand(), nz * urand(), nx, ny, nz};
        pos[3] = nx * 0.5; pos[4] = ny * 0.5; pos[5] = nz * 0.5;   /* a cell centre when odd */
        double Q[6] = {1.0, 0.5, 2.0, 0.1, 0.3, 0.0}, e[2] = {0.2, 0.7};
        double *G = malloc(sizeof(double) * nc), *H = malloc(sizeof(double) * nc);
        CHECK(oracle_point(nx, ny, nz, 0.7, nb, k, nab, 3, pos, Q, e, NULL, (int)nc, G, H, 2) == 0, "point");
        CHECK(finite_all(G, nc) && finite_all(H, nc), "point finite");
        for (int64_t c = 0; c < nc; ++c) {
            double tau[2], dtau[2], ri, ro;
            CHECK(oracle_point_pair(nx, ny, nz, 0.7, nb, k, pos + 3, c, tau, dtau, &ri, &ro) == 0, "pair");
        }
        /* rejected arguments return codes without touching memory */
        CHECK(oracle_sweep(0, ny, nz, 0.7, nb, k, S, 1, 0, 12, 0.0, NULL, NULL, NULL, NULL, 1) != 0, "bad sweep");
        CHECK(oracle_point(nx, ny, nz, -1.0, nb, k, nab, 1, pos, Q, e, NULL, (int)nc, G, H, 1) != 0, "bad point");
        free(k); free(S); free(nab); free(G); free(H);
    }
    printf("oracle driver: ok\n");
    return 0;
}
