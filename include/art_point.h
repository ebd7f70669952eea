/*
 * art_point.h -- radiation from point sources (Tanaka et al., arXiv:1410.0763,
 * Sect. 2.3 "RT from point radiation sources", with the photon-conserving
 * rates of Appendix A).
 *
 * For every point source alpha and every target cell c the light ray is the
 * straight line from the source position p to the centre q of c.  It enters
 * c at distance r_in from p and leaves it at r_out (r_in = 0 when p lies in
 * c; when p equals q the line is taken along +x).  The optical depth tau_b
 * is the sum of kappa_b h dl over the cells the line crosses before c, and
 * dtau_b = kappa_b(c) h (r_out - r_in) is the radial optical depth of the
 * imaginary shell between r_in and r_out.  The shell absorbs
 *     Q_{alpha,b} e^{-tau_b} (1 - e^{-dtau_b})
 * photons per unit time (Q: the source's photon rate in bin b) out of
 * n_c (4 pi / 3)(r_out^3 - r_in^3) h^3 absorbers.  The rates per absorber,
 * summed over sources and bins, are
 *     Gamma_c = sum Q e^{-tau} (1 - e^{-dtau}) / (n_c V_shell)
 *     Heat_c  = sum Q e^{-tau} (1 - e^{-dtau}) e_b / (n_c V_shell)
 * with e_b the energy an absorbed photon of bin b leaves above the threshold
 * (the integrals over frequency of eq pc_gamma and the heating rate that
 * follows it, as sums over the mesh's bins, for one absorbing species).
 * Cells with n_c <= 0 get 0.
 *
 * The cost is one march per (source, cell) pair, O(N_m^{4/3} N_s) (Sect. 2.3).
 * Conventions as in art.h: ART_OK or a negative ART_E_* code, art_last_error
 * on failure, work queued on hip_stream.
 */
#ifndef ART_POINT_H
#define ART_POINT_H

#include "art.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Rates from nsrc point sources for the kappa fields loaded in mesh
 * (art_set_fields; S is not used).
 *   pos     host double [nsrc][3]: (x, y, z) in cell units, each finite and in
 *           [0, n_axis] (the closed box);
 *   Q       host double [nsrc][nbins]: photon rates, finite and >= 0;
 *   e       host double [nbins] or NULL: energy per absorbed photon above the
 *           threshold, finite (NULL: Heat, if given, is set to 0);
 *   n_abs   device float [nz][ny][nx]: absorber number density per cell;
 *   Gamma   device float [nz][ny][nx]: caller-owned output, overwritten;
 *   Heat    device float [nz][ny][nx] or NULL: caller-owned output;
 *   segs    device unsigned [nz][ny][nx] or NULL: cells each target's rays
 *           crossed, summed over sources (the cells before the target plus
 *           the target itself), for work accounting.
 * nsrc = 0 writes zeros.  Sources are taken 64 per launch; the host arrays
 * may be reused as soon as the call returns (they travel as launch
 * arguments).  ART_E_STATE before art_set_fields; ART_E_INVAL for a bad
 * argument, before any GPU work.
 */
int art_point_sources(art_mesh *mesh, int nsrc, const double *pos, const double *Q,
                      const double *e, const float *n_abs, float *Gamma, float *Heat,
                      unsigned *segs, void *hip_stream);

/* Room of the static scratch of art_point_sources_noalloc, in floats (64 MiB). */
#define ART_POINT_NOALLOC_FLOATS (16ll * 1024 * 1024)

/*
 * art_point_sources for callers that cannot allocate device memory (code
 * under HIP graph capture, tight time-step loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, but the library
 * calls no hipMalloc, hipFree or allocating routine.  The per-cell kappa
 * pack the walk reads (1, 2 or 4 floats per cell for 1, 2 or 3-4 bins) is
 * rebuilt on every call in a static device array of ART_POINT_NOALLOC_FLOATS
 * floats, one per GPU, which the GPU holds from the first call on it until
 * the process ends; a mesh whose pack does not fit gives ART_E_UNSUPPORTED
 * (about 128^3 cells with 4 bins fit).  The mesh's fields must be set
 * (art_set_fields) beforehand; the caller owns n_abs and the outputs.  All
 * calls on one GPU share the array: calls that overlap on one GPU (two
 * streams, two threads) race and give wrong results.
 */
int art_point_sources_noalloc(art_mesh *mesh, int nsrc, const double *pos, const double *Q,
                              const double *e, const float *n_abs, float *Gamma, float *Heat,
                              unsigned *segs, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ART_POINT_H */
