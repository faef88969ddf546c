/*
 * CPU oracle for the ternary Cahn-Hilliard time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow FP64 implementation that
 * the tests, the smoke check and the benchmark's CPU-baseline leg use to check
 * the GPU library.  The product path never links it.  It shares no code with
 * the GPU library (only the seeded input generators on the Python side serve
 * both).
 *
 * What it computes (Bergermann et al., "Preconditioning for a Phase-Field
 * Model with Application to Morphology Evolution in Organic Semiconductors"):
 *   - P1 mass M and stiffness K (Section 3, the matrices of eq. chternary_space);
 *   - the right-hand side of the symmetric saddle-point system
 *     (eq. saddle_point_system) with the explicit potential term
 *     f_j = integral of f'(phi_h) * lambda_j;
 *   - the block-diagonal preconditioner of Algorithm 1 with the matching
 *     Schur approximation (Section 3, Lemma 1), its AMG solves realised by
 *     smoothed-aggregation V-cycles;
 *   - right-preconditioned flexible GMRES on each species' system;
 *   - the state update phi_s = 1 - phi_p - phi_n (Section 2) and an optional
 *     per-step solvent removal.
 */
#ifndef CHM_ORACLE_H
#define CHM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOCONV (-4)
#define ORC_ENAN (-5)
#define ORC_EDOMAIN (-6) /* the new state leaves [0, 1] (range_check) */

/* potentials */
#define ORC_POT_FLORY_HUGGINS 0
#define ORC_POT_POLYNOMIAL 1
#define ORC_POT_NONE 2

/* smoothers */
#define ORC_SMOOTH_CHEBYSHEV 0
#define ORC_SMOOTH_JACOBI 1

typedef struct {
    double tau;          /* time step */
    double eps[2];       /* interface parameter per species (0 = polymer, 1 = acceptor) */
    double mobility[2];  /* mobility per species; it multiplies tau */
    int32_t potential;   /* ORC_POT_* */
    double Np, Nn, Ns;   /* degrees of polymerisation */
    double chi_pn, chi_ps, chi_ns;
    double log_floor;    /* log arguments are clamped to at least this */
    double evap_ds;      /* solvent fraction removed after each step */
    int32_t evap_steps;  /* number of steps (counted from creation) that remove solvent */
    double rtol;         /* FGMRES relative residual tolerance (2-norm, relative to ||b||) */
    int32_t restart;     /* FGMRES restart length m */
    int32_t max_iters;   /* total FGMRES iterations allowed per solve */
    int32_t amg_cycles;  /* V-cycles per stationary AMG solve (mass solves); the cap when amg_tol > 0 */
    int32_t schur_pcg;   /* CG steps (one V-cycle each) per As solve; 0 = stationary;
                            -1 = chosen at creation (FGMRES only): 2 if the measured
                            contraction of one As V-cycle is at most 0.3, 4 up to
                            0.6, else 6 (orc_schur_info) */
    int32_t smoother;    /* ORC_SMOOTH_* */
    int32_t cheb_degree; /* As hierarchies: Chebyshev degree (pre and post) or Jacobi sweeps */
    double cheb_ratio;   /* As hierarchies: Chebyshev interval [rho/ratio, rho] */
    int32_t cheb_degree_mass; /* the same two for the mass hierarchy */
    double cheb_ratio_mass;
    int32_t coarse_max;  /* stop coarsening at or below this many rows */
    int32_t max_levels;  /* at most this many levels */
    /* boundary terms of eq. chternary:2 (Section 2), explicit in time: the
     * top facets (largest second coordinate) take the solvent evaporation as
     * an inflow k phi_i phi_s of polymer and acceptor, the bottom facets
     * (smallest second coordinate) the substrate flux d f_s / d phi_i =
     * p_i(x) (g_i + 2 h_i phi_i) of eq. surfenergy; elsewhere no flux */
    int32_t boundary;    /* 0: no flux everywhere; 1: the two terms above */
    double bc_k;         /* evaporation rate k */
    double bc_g[2], bc_h[2]; /* substrate coefficients g_i, h_i */
    int32_t bc_pattern;  /* 1: p_p, p_n alternate on sixths of the bottom (Section 4); 0: p = 1 */
    int32_t krylov;      /* ORC_KRYLOV_*: the Krylov method of each time step */
    /* Inner tolerance of the stationary AMG solves (the paper runs its AMG
     * preconditioner to a tolerance of 1e-4, Section 4): 0 gives exactly
     * amg_cycles V-cycles; amg_tol > 0 stops as soon as the 2-norm
     * residual of the block is at most amg_tol times the norm of its
     * right-hand side, after at least one and at most amg_cycles cycles. */
    double amg_tol;
    /* The mass block of Algorithm 1 (an approximation of M^-1, Section 3):
     * ORC_MASS_AMG, amg_cycles stationary V-cycles of the mass hierarchy;
     * ORC_MASS_CHEBYSHEV, the Chebyshev semi-iteration the paper names as
     * the alternative (Wathen and Rees): cheb_degree_mass steps on D^-1 M
     * over [rho/cheb_ratio_mass, rho] from zero, no coarse levels (the
     * mass hierarchy's fine-level smoother applied once). */
    int32_t mass_solver;
    /* As hierarchies: Chebyshev degree (or Jacobi sweeps) of the smoother on
     * the levels below the finest, each over [rho/cheb_ratio, rho] of its own
     * rho (the paper leaves the AMG smoother open); 0 = cheb_degree. */
    int32_t cheb_degree_coarse;
    /* The volume fractions are physical in [0, 1] (Section 2); a step whose
     * new state leaves that range at any vertex (the divergence the paper
     * records for eps = 1e-4, Section 4) is counted in orc_stats_t.outside;
     * with range_check = 1 it also fails with ORC_EDOMAIN and leaves the
     * state unchanged. */
    int32_t range_check;
} orc_params_t;

/* FGMRES (right preconditioned, any Algorithm 1), or preconditioned MINRES
 * as in the paper's experiments, which needs the symmetric positive
 * definite Algorithm 1 of stationary V-cycles (schur_pcg = 0) and stops on
 * the residual in the preconditioner's inverse norm relative to that of b */
#define ORC_KRYLOV_FGMRES 0
#define ORC_KRYLOV_MINRES 1
#define ORC_MASS_AMG 0
#define ORC_MASS_CHEBYSHEV 1

typedef struct {
    int32_t iters[2];
    double relres[2];
    int32_t status;
    int32_t clamped;
    int32_t outside; /* vertices whose phi_p, phi_n or phi_s lies outside [0, 1] after the step */
} orc_stats_t;

typedef struct orc_solver orc_solver_t;

/* element matrices of one simplex: xv = (dim+1) vertices x dim coords */
int orc_element_matrices(int dim, const double *xv, double *MT, double *KT, double *vol);
/* quadrature rule on the reference simplex: barycentric points [npts][dim+1], weights sum to 1
 * (dim 1: three-point Gauss-Legendre on an edge; 2, 3: degree 5) */
int orc_quadrature(int dim, int *npts, double *bary, double *w);
/* the boundary vector G of eq. chternary:2: G_j = integral over the top and
 * bottom facets of the flux g_i(phi_h) lambda_j, per species (gp, gn: n_vertices) */
int orc_boundary(orc_solver_t *s, const double *php, const double *phn, double *gp, double *gn);
/* potential and its derivatives at one point */
int orc_potential(const orc_params_t *p, double php, double phn, double *f, double *fp, double *fn);

int orc_create(int dim, int64_t nv, const double *coords, int64_t nc, const int32_t *cells,
               const orc_params_t *prm, orc_solver_t **out);
void orc_destroy(orc_solver_t *s);

int64_t orc_nnz(const orc_solver_t *s);
/* which: 0 = M, 1 = K, 2 = As of species 0, 3 = As of species 1 */
int orc_get_matrix(const orc_solver_t *s, int which, int32_t *rowptr, int32_t *col, double *val);

/* hierarchy id: 0 = mass, 1 = As of species 0, 2 = As of species 1 */
int orc_num_levels(const orc_solver_t *s, int hier);
int orc_level_info(const orc_solver_t *s, int hier, int lev, int64_t *n, int64_t *nnzA,
                   int64_t *nnzP, double *rho);
int orc_level_get(const orc_solver_t *s, int hier, int lev, int32_t *Arp, int32_t *Aci, double *Av,
                  int32_t *agg, int32_t *Prp, int32_t *Pci, double *Pv);
/* stationary AMG solve (amg_cycles V-cycles), one V-cycle, the As solve of Algorithm 1 */
int orc_amg_solve(const orc_solver_t *s, int hier, const double *b, double *x);
int orc_vcycle(const orc_solver_t *s, int hier, const double *b, double *x);
int orc_schur_solve(const orc_solver_t *s, int species, const double *b, double *x);
/* one application of the level's smoother to x (in place) */
int orc_smooth(const orc_solver_t *s, int hier, int lev, const double *b, double *x);

int orc_apply_saddle(const orc_solver_t *s, int species, const double *x, double *y);
int orc_apply_prec(const orc_solver_t *s, int species, const double *v, double *w);
int orc_rhs(orc_solver_t *s, const double *php, const double *phn, double *bp, double *bn);
int orc_fgmres(const orc_solver_t *s, int species, const double *b, double *x,
               int32_t *iters, double *relres);
/* preconditioned MINRES; relres = the true ||b - A x||_2 / ||b||_2 at the end */
int orc_minres(const orc_solver_t *s, int species, const double *b, double *x,
               int32_t *iters, double *relres);
int orc_step(orc_solver_t *s, double *php, double *phn, double *mup, double *mun,
             orc_stats_t *st);
double orc_energy(const orc_solver_t *s, const double *php, const double *phn);

/* The CG steps per As solve in use and the measured V-cycle contraction
 * (0 unless schur_pcg was -1). */
int orc_schur_info(const orc_solver_t *s, int32_t *schur_pcg, double *contraction);

/* Host threads of the solve's row loops (n > 0 sets them; returns the count in
 * use).  Results do not depend on it. */
int orc_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
