/*
 * art_chem.h -- the chemistry and energy update that follows a radiative-
 * transfer step (Tanaka et al., arXiv:1410.0763, Appendix B ionisation
 * balance, Appendix C photo-heating and radiative cooling, Appendix D
 * iteration and timestep control), for a hydrogen network (HI, HII, e).
 *
 * The paper cites its rate fits without printing them, so the caller supplies
 * the rate coefficients as tables on a uniform grid of log10 T; they are
 * interpolated linearly in log10 T and held at the end values outside the
 * grid.  Per cell, with n_e = n_HII = n_H - n_HI and T = T_per_u u / (1 + x_e),
 * x_e = n_HII / n_H:
 *
 *   dn_HI/dt = alpha(T) n_e n_HII - (k_ci(T) n_e + Gamma) n_HI
 *   du/dt    = (Heat n_HI - n_e (cool_I(T) n_HI + cool_II(T) n_HII)) / rho
 *
 * Gamma and Heat are the photo-ionisation and photo-heating rates per HI atom
 * from the transfer (art_sweep's Gamma and Heat, art_point_sources, or their
 * sum), constant over the step because the transfer equation is static.  The
 * step dt is divided into sub-steps h = min(dt_chem, rest of dt), dt_chem =
 * eps_e |n_e / (dn_e/dt)| + eps_HI |n_HI / (dn_HI/dt)| (a term whose rate is 0
 * is infinite; after max_sub sub-steps the rest is taken at once).  In a
 * sub-step the backward-difference update n_HI' = (C h + n_HI) / (1 + D h),
 * C = alpha n_e' n_HII', D = k_ci n_e' + Gamma at the advanced time, is solved
 * exactly for n_HI' (with hydrogen alone it is a quadratic at fixed T), then
 * u' = u + h (Heat n_HI' - Lambda(n', u')) / rho is solved for u' by 64
 * bisection halvings on [u_floor, max(u_floor, u + h Heat n_HI' / rho)],
 * u_floor = 10^logT_min / T_per_u; the two are iterated at most max_iter times
 * until |n_e^(i) - n_e^(i-1)| <= eps n_e^(i) and |u^(i) - u^(i-1)| <= eps
 * u^(i).  All arithmetic is double precision.
 *
 * Conventions as in art.h: ART_OK or a negative ART_E_* code, art_last_error
 * on failure, work queued on hip_stream, device pointers owned by the caller.
 */
#ifndef ART_CHEM_H
#define ART_CHEM_H

#include "art.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nT;                 /* table points, >= 2 */
    double logT_min;        /* log10 T of the first point */
    double dlogT;           /* spacing in log10 T, > 0 */
    const double *alpha;    /* device [nT]: radiative recombination of HII, per n_e n_HII */
    const double *k_ci;     /* device [nT]: collisional ionisation of HI, per n_e n_HI */
    const double *cool_I;   /* device [nT]: cooling per n_e n_HI (collisional ionisation and excitation) */
    const double *cool_II;  /* device [nT]: cooling per n_e n_HII (recombination, bremsstrahlung) */
    double T_per_u;         /* T = T_per_u u / (1 + x_e), > 0 */
    double eps;             /* convergence tolerance of the iteration (the paper: 1e-3), > 0 */
    double eps_e, eps_HI;   /* timestep factors (the paper: 0.2 and 0.002), >= 0, not both 0 */
    int max_iter;           /* iterations per sub-step, >= 1 */
    int max_sub;            /* sub-steps before the rest of dt is taken at once, >= 0 */
} art_chem_params;

/*
 * Advance ncell cells by dt (finite, >= 0).  n_H, rho: device double [ncell],
 * hydrogen number density and mass density (cells with n_H <= 0 are left as
 * they are, with dt_chem = +inf and nsub = 0); Gamma, Heat: device float
 * [ncell], per HI atom; x_HI (in [0, 1]) and u (>= 0): device double [ncell],
 * updated in place; dt_chem: device double [ncell] or NULL, the chemical
 * timestep at the final state (the radiative step of Appendix D is F times
 * its minimum); nsub: device int [ncell] or NULL, sub-steps taken.
 * ART_E_INVAL for a bad size, pointer or parameter, before any GPU work.
 */
int art_chem_step(long long ncell, const double *n_H, const double *rho, const float *Gamma,
                  const float *Heat, double *x_HI, double *u, double dt, const art_chem_params *p,
                  double *dt_chem, int *nsub, void *hip_stream);

/*
 * One radiative step coupled to the chemistry (Appendix D: the transfer
 * equation is static, so the diffuse radiation field and the rate and energy
 * equations are iterated until n_e and u converge in every cell).  The
 * fields of the diffuse recombination radiation follow from the chemical
 * state (Sect. 2.2): per bin b, kappa_b = sigma_b n_HI and the source
 * function S_b = src_coef_b dalpha(T) n_e n_HII / n_HI (the rectangular
 * recombination spectrum: src_coef = h nu_0 / (4 pi sigma dnu_th) in the
 * paper's units), dalpha = alpha_A - alpha_B a table on the chemistry's
 * log10 T grid, n_HI floored at x_floor n_H in both (a fully ionised cell
 * then absorbs next to nothing and emits dalpha n_e n_HII per unit volume,
 * the limit of the formal solution); cells with n_H <= 0 have kappa = S = 0.
 * The rates are Gamma = sum_b gamma_w_b (J_in_b + S_b) and Heat =
 * sum_b heat_in_b J_in_b + heat_src_b S_b (eqs gamma_diff, heat_diff; with
 * gamma_w_b src_coef_b = 1 the S part of Gamma is the on-the-spot term
 * dalpha n_e n_HII / n_HI).  Point sources (art_point.h: Sect. 2.3,
 * Appendix A) add their photon-conserving rates per absorber for the same
 * kappa, with the floored n_HI as the absorber density.
 */
typedef struct {
    int nbins;               /* 1..ART_MAX_BINS */
    const float *sigma;      /* host [nbins]: kappa_b = sigma_b n_HI (per unit length), finite, >= 0 */
    const float *src_coef;   /* host [nbins]: source-function coefficient, finite, >= 0 */
    const double *dalpha;    /* device [nT] (the chemistry's grid): alpha_A - alpha_B */
    const float *gamma_w;    /* host [nbins] or NULL (all 1) */
    const float *heat_in;    /* host [nbins] or NULL (all 0) */
    const float *heat_src;   /* host [nbins] or NULL (all 0) */
    int nside;               /* HEALPix resolution of the sweeps, >= 1 */
    double x_floor;          /* in (0, 1] */
    int max_iter;            /* transfer-chemistry iterations, >= 1 */
    int nsrc;                /* point sources (0: none); their rates are added each iteration */
    const double *src_pos;   /* host [nsrc][3], as art_point_sources */
    const double *src_Q;     /* host [nsrc][nbins], as art_point_sources */
    const double *src_e;     /* host [nbins] or NULL, as art_point_sources */
} art_rt_chem_params;

typedef struct {
    int iterations;          /* iterations run */
    int converged;           /* 1: the last iteration met the tolerance in every cell */
    double dt_chem_min;      /* minimum chemical timestep at the final state (+inf if none):
                                the next radiative step is F times it (the paper: F = 1-10) */
} art_rt_chem_result;

/* Bytes of workspace art_rt_chem_step needs on this mesh with nbins bins
 * (-1 for a NULL mesh or a bad bin count).  Host only. */
long long art_rt_chem_workspace(const art_mesh *mesh, int nbins);

/*
 * Advance every cell of the mesh by the radiative step dt.  Iteration i
 * (1 .. max_iter) loads the fields built from the state of iteration i - 1
 * (iteration 0: x_HI, u as given) into the mesh (art_set_fields, with the
 * heating weights), sweeps (art_sweep at nside, I_bc = 0), adds the point
 * sources' rates (art_point_sources), and advances the given state over dt
 * with those rates (art_chem_step with cp); it stops when
 * every cell with n_H > 0 has |n_e^(i) - n_e^(i-1)| <= eps n_e^(i) and
 * |u^(i) - u^(i-1)| <= eps u^(i) (eps = cp->eps).  Then x_HI and u hold the
 * last iteration's state.  n_H, rho, x_HI, u: device double [cells] (x
 * fastest); Gamma, Heat: device float [cells] or NULL, the last iteration's
 * rates.  work: device buffer of work_bytes >= art_rt_chem_workspace().
 * res: host, filled on success.  The call blocks the host: after each
 * iteration it waits for the stream to learn whether every cell converged.
 * It replaces the mesh's fields and heating weights.  ART_E_INVAL for a bad
 * argument (before any GPU work), or the code of the failing step.
 */
int art_rt_chem_step(art_mesh *mesh, const art_rt_chem_params *rp, const art_chem_params *cp,
                     const double *n_H, const double *rho, double *x_HI, double *u, double dt,
                     void *work, long long work_bytes, float *Gamma, float *Heat,
                     art_rt_chem_result *res, void *hip_stream);

typedef struct {
    int steps;               /* radiative steps taken */
    int iterations;          /* transfer-chemistry iterations, all steps */
    int unconverged;         /* steps that ended at max_iter without converging */
    double t;                /* time reached: t_end unless max_steps stopped first */
    double dt_chem_min;      /* minimum chemical timestep at the final state */
} art_rt_chem_run;

/*
 * Radiative steps from t = 0 to t_end (Appendix D): the chemical timestep of
 * the start state, with the rates of its own fields, is that of a step of
 * length 0 (which leaves x_HI and u as they are); then each step is art_rt_chem_step over dt = min(F dt_chem_min,
 * t_end - t), dt_chem_min from the end of the previous step (the rest at
 * once where it is infinite), until t_end or max_steps steps.  The paper
 * sets F = 1-10.  Arguments as art_rt_chem_step; t_end finite and >= 0,
 * F > 0 and finite, max_steps >= 1.  x_HI and u hold the final state;
 * Gamma and Heat (or NULL) the last iteration's rates.  run: host, filled on
 * success.  Blocks the host like art_rt_chem_step.  ART_E_INVAL for a bad
 * argument, ART_E_STATE if the chemical timestep falls to 0 before t_end
 * (the state then holds the steps taken), or the code of a failing step.
 */
int art_rt_chem_advance(art_mesh *mesh, const art_rt_chem_params *rp, const art_chem_params *cp,
                        const double *n_H, const double *rho, double *x_HI, double *u, double t_end,
                        double F, int max_steps, void *work, long long work_bytes, float *Gamma,
                        float *Heat, art_rt_chem_run *run, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ART_CHEM_H */
