/*
 * chm.h -- C ABI of the MI355X library for the per-time-step solve of the
 * ternary Cahn-Hilliard model of Bergermann, Deibel, Herzog, MacKenzie,
 * Pietschmann and Stoll, "Preconditioning for a Phase-Field Model with
 * Application to Morphology Evolution in Organic Semiconductors".
 *
 * What one time step computes (paper Section 3):
 *   for each species i in {polymer, acceptor}, with tau' = tau * mobility_i,
 *   solve the symmetric saddle-point system (eq. saddle_point_system)
 *       [ M        tau' K          ] [phi^{k+1}]   [ M phi^k               ]
 *       [ tau' K   -(tau'/eps_i) M ] [ mu^{k+1}] = [ -(tau'/eps_i) f_i^k   ]
 *   where M, K are the P1 mass and stiffness matrices and
 *   f_i^k = integral of (d f / d phi_i)(phi_h^k) times each hat function
 *   (the explicit part of the IMEX scheme eq. chternary_space), by
 *   right-preconditioned flexible GMRES (or, as in the paper's experiments,
 *   MINRES: krylov) with the block-diagonal preconditioner of Algorithm 1
 *   (mass block by AMG or a Chebyshev semi-iteration: mass_solver; Schur
 *   block by the matching approximation
 *   (tau' K + sqrt(tau'/eps) M) M^-1 (tau' K + sqrt(tau'/eps) M) justified by
 *   Lemma 1), then set phi_s = 1 - phi_p - phi_n (Section 2).  Optional
 *   boundary terms of eq. chternary:2 (boundary) add to the first block of
 *   the right-hand side.  The AMG is smoothed aggregation with Chebyshev or
 *   Jacobi smoothing.
 *
 * Conventions
 *   - Every call returns CHM_OK (0) or a negative CHM_E* code; no exception
 *     or abort crosses the ABI.  chm_last_error() gives the message.
 *   - The caller owns every pointer it passes.  The library copies mesh and
 *     fields into device memory it allocates itself; chm_destroy frees it.
 *   - All GPU work is enqueued on the HIP stream given to chm_create (NULL =
 *     the default stream).  Calls that return host data synchronise it.
 *   - Fields are FP64, one value per mesh vertex, in vertex order.
 *   - "on_device" arguments: 1 = the pointers are device memory on the
 *     library's device, 0 = host memory.
 *   - A handle is not thread safe; separate handles are independent.
 */
#ifndef CHM_H
#define CHM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHM_OK 0
#define CHM_EINVAL (-1)   /* bad argument or unsupported configuration */
#define CHM_ENOMEM (-2)   /* device allocation failed */
#define CHM_EHIP (-3)     /* a HIP runtime call failed */
#define CHM_ENOCONV (-4)  /* the Krylov method did not reach rtol within max_iters */
#define CHM_ENAN (-5)     /* a non-finite value appeared */
#define CHM_EDOMAIN (-6)  /* the new state leaves [0, 1] (range_check = 1) */

#define CHM_POT_FLORY_HUGGINS 0 /* eq. logarithmicpotential (Section 2) */
#define CHM_POT_POLYNOMIAL 1    /* eq. polynomial_potential (Section 4) */
#define CHM_POT_NONE 2          /* f = 0: linear fourth-order problem */

#define CHM_SMOOTH_CHEBYSHEV 0
#define CHM_SMOOTH_JACOBI 1

/* Arithmetic of the block preconditioner (Algorithm 1).  FP32: V-cycles
 * (smoothing, residual, restriction, prolongation), the inner CG of the As
 * solves and the product with M run in FP32 on FP32 copies of the matrix
 * values; the coarsest-level inverse and all dot-product sums stay FP64, and
 * the preconditioner takes and returns FP64 vectors.  The Krylov method, the
 * saddle-point residual, the orthogonalisation and the right-hand side are
 * FP64 in both settings. */
#define CHM_PREC_FP64 0
#define CHM_PREC_FP32 1

/* Krylov method of the time step (Section 3).  FGMRES: restarted, with the
 * preconditioner applied on the right, stopped on the true 2-norm residual.
 * MINRES (the method of the paper's experiments): the symmetric saddle-point
 * matrix with Algorithm 1 as a symmetric positive definite preconditioner,
 * which needs schur_pcg = 0 (the As solves are then amg_cycles stationary
 * V-cycles, a fixed symmetric operator); it stops when the residual in the
 * P^-1 norm that its rotations give is at most rtol times the P^-1 norm of
 * b, and relres still reports the true 2-norm residual. */
#define CHM_KRYLOV_FGMRES 0
#define CHM_KRYLOV_MINRES 1

#define CHM_MASS_AMG 0
#define CHM_MASS_CHEBYSHEV 1

#define CHM_ORTHO_DCGS2 0
#define CHM_ORTHO_CGS2 1

typedef struct chm_solver chm_solver_t;

/* A conforming simplex mesh: triangles (dim 2) or tetrahedra (dim 3).
 * coords: host, n_vertices * dim doubles, vertex-major.
 * cells:  host, n_cells * (dim + 1) vertex indices, each in [0, n_vertices).
 * Cells must have non-zero volume.  The library copies both. */
typedef struct {
    int32_t dim;
    int64_t n_vertices;
    const double *coords;
    int64_t n_cells;
    const int32_t *cells;
} chm_mesh_t;

/* Model and solver parameters.  Model values of the paper (Section 4):
 * chi_pn = 1, chi_ps = chi_ns = 0.3, N_p = N_n = 20, N_s = 1, eps = 1e-3,
 * tau between 1e-7 and 1e-4.  Both species must share tau * mobility and
 * eps (they then share the As hierarchy); other combinations give
 * CHM_EINVAL. */
typedef struct {
    double tau;            /* time step */
    double eps[2];         /* interface parameter per species (0 polymer, 1 acceptor) */
    double mobility[2];    /* mobility per species; multiplies tau */
    int32_t potential;     /* CHM_POT_* */
    double Np, Nn, Ns;     /* degrees of polymerisation (Flory-Huggins) */
    double chi_pn, chi_ps, chi_ns; /* interaction parameters (Flory-Huggins) */
    double log_floor;      /* log arguments below this are clamped to it */
    double evap_ds;        /* solvent fraction removed per step (0 = off) */
    int32_t evap_steps;    /* steps, counted from creation, that remove solvent */
    double rtol;           /* FGMRES: ||b - A x||_2 <= rtol ||b||_2 per species (MINRES: see above) */
    int32_t restart;       /* FGMRES restart length m, 1..64 */
    int32_t max_iters;     /* Krylov iterations allowed per species and step */
    int32_t amg_cycles;    /* V-cycles per mass-matrix solve */
    int32_t schur_pcg;     /* CG steps (one V-cycle each) per As solve; 0 = amg_cycles V-cycles;
                              -1 = chosen at setup from the measured V-cycle contraction
                              (FGMRES only; see chm_schur_info) */
    int32_t smoother;      /* CHM_SMOOTH_* */
    int32_t cheb_degree;   /* As hierarchy: Chebyshev degree or Jacobi sweeps (1..31) */
    double cheb_ratio;     /* As hierarchy: Chebyshev interval [rho/ratio, rho] */
    int32_t cheb_degree_mass; /* mass hierarchy: the same two */
    double cheb_ratio_mass;
    int32_t coarse_max;    /* coarsen until a level has at most this many rows */
    int32_t max_levels;    /* at most this many levels (1..24) */
    int32_t use_graphs;    /* 1: each FGMRES iteration runs as a captured HIP graph
                              (the same kernels, bitwise the same results); 0: eager */
    int32_t precision;     /* CHM_PREC_*: arithmetic of the preconditioner */
    /* Boundary terms of eq. chternary:2 (Section 2, coefficients of Section
     * 4), explicit in time, added to the first block row of the right-hand
     * side times tau: on the top facets (all vertices at the largest second
     * coordinate) the solvent evaporation as an inflow bc_k phi_i phi_s of
     * polymer and acceptor; on the bottom facets (smallest second
     * coordinate) the substrate flux p_i(x) (bc_g[i] + 2 bc_h[i] phi_i),
     * p_p = 1 on the first, third and fifth sixth of the bottom in x and
     * p_n = 1 on the others when bc_pattern = 1, p = 1 otherwise; no flux
     * elsewhere.  boundary = 0: no flux everywhere (the other fields are
     * ignored). */
    int32_t boundary;
    double bc_k;
    double bc_g[2], bc_h[2];
    int32_t bc_pattern;
    int32_t krylov;        /* CHM_KRYLOV_* */
    /* Inner tolerance of the stationary AMG solves (Section 4 runs its AMG
     * preconditioner to 1e-4): 0 = exactly amg_cycles V-cycles; > 0 = per
     * species, stop at the first cycle whose residual norm is at most amg_tol
     * times the norm of the block's right-hand side (at least one cycle, at
     * most amg_cycles).  The preconditioner then varies slightly from one
     * application to the next; the cycle counts are decided on the host, so
     * these runs use no HIP graphs. */
    double amg_tol;
    /* The mass block of Algorithm 1, an approximation of M^-1 (Section 3
     * names AMG and, after Wathen and Rees, a Chebyshev semi-iteration):
     * CHM_MASS_AMG, amg_cycles stationary V-cycles of the mass hierarchy
     * (smoother degree cheb_degree_mass); CHM_MASS_CHEBYSHEV,
     * cheb_degree_mass Chebyshev steps on D^-1 M over
     * [rho/cheb_ratio_mass, rho] from zero, with no coarse levels (damped
     * Jacobi sweeps with the Jacobi smoother).  Both are fixed symmetric
     * positive definite operators. */
    int32_t mass_solver;
    /* Column indices of the SELL-64 matrices (one lane per row: the fine
     * levels and the products with M, K and As): 0, the default, stores each
     * column of a square matrix as a 16-bit offset from its row when every
     * offset of the matrix fits (|col - row| <= 32767; 2 B per entry instead
     * of 4 in the kernels' traffic); 1 keeps 32-bit columns everywhere.  The
     * results are bitwise the same. */
    int32_t wide_index;
    /* Batches (chm_create_batch): how many runs one lane of the SELL-64
     * kernels (fine-level smoothing and products, the saddle-point operator)
     * and of the coarsest-level solve serves: each matrix entry the lane
     * loads is used for that many runs, so a launch over R runs streams the
     * matrix ceil(R / runs_per_lane) times.  1, 2 or 4; 0 = 2.  Every run's
     * arithmetic is the same for any value (bitwise the same results); it
     * trades matrix traffic against registers per lane.  Ignored for one
     * run. */
    int32_t runs_per_lane;
    /* As hierarchy: Chebyshev degree (or Jacobi sweeps) of the smoother on
     * every level below the finest, over the same interval [rho/cheb_ratio,
     * rho] of each level's own rho; 0 = cheb_degree on every level. */
    int32_t cheb_degree_coarse;
    /* The volume fractions are physical in [0, 1] (Section 2).  Every step
     * counts the vertices at which its new state (after the solvent removal)
     * has phi_p, phi_n or phi_s outside that range (chm_stats_t.outside; the
     * paper records such a divergence for eps = 1e-4, Section 4).  1: such a
     * step fails with CHM_EDOMAIN and no run is advanced; 0: it is only
     * counted. */
    int32_t range_check;
    /* Orthogonalisation of the FGMRES basis (the Arnoldi process of the
     * Krylov method the paper solves the saddle-point system with, Section
     * 3).  CHM_ORTHO_DCGS2 (0, the default): classical Gram-Schmidt twice per
     * vector, the second pass delayed to the next iteration, where it shares
     * a sweep over the basis with the first pass of the next vector: two
     * sweeps per iteration.  The preconditioner then takes each basis vector
     * after its first pass, which FGMRES allows (the stored preconditioned
     * vectors define the solution space; the Hessenberg column of the
     * previous iteration is corrected for the second pass).
     * CHM_ORTHO_CGS2: both passes in the vector's own iteration, three
     * sweeps.  Both build the same Krylov space and differ by rounding. */
    int32_t ortho;
    /* 1: never use value tables (chm_value_table); the kernels read every
     * value.  0, the default: tables where they fit.  The results are
     * bitwise the same either way. */
    int32_t values_direct;
} chm_params_t;

/* Per-step statistics. */
typedef struct {
    int32_t iters[2];      /* Krylov iterations per species */
    double relres[2];      /* final true residual / ||b|| per species */
    int32_t status;        /* CHM_OK or the step's error code */
    int32_t clamped;       /* clamped log arguments in the right-hand side */
    double t_step_ms;      /* wall time of the step on the stream */
    int32_t guess_used[2]; /* CHM_GUESS_* (chm_net.h) of the start each species'
                              solve used: 0 the previous state */
    double res0[2];        /* relative residual of that start per species */
    int32_t outside;       /* vertices of the new state with a fraction outside [0, 1] */
} chm_stats_t;

/* Build the solver: upload the mesh, colour the cells, assemble M and K by
 * coloured scatter, form As = tau' K + sqrt(tau'/eps) M (Algorithm 1), build
 * the two smoothed-aggregation hierarchies (for M and for As) and allocate
 * the Krylov workspace.  `stream` is a hipStream_t (may be NULL).  The
 * initial state is phi = mu = 0.  On error *out is left NULL and the message
 * is available from chm_last_error(NULL). */
int chm_create(const chm_mesh_t *mesh, const chm_params_t *params, void *stream,
               chm_solver_t **out);

/* What may differ between the runs of a batch (chm_create_batch): the
 * interaction parameters of the Flory-Huggins energy and the solvent removal
 * (evap_ds per step for the first evap_steps steps). */
typedef struct {
    double chi_pn, chi_ps, chi_ns;
    double evap_ds;
    int32_t evap_steps;
} chm_run_t;

/* A batch of `runs` (1..64) independent runs on one mesh with one set of
 * parameters except for run[r] (NULL: every run takes params' values).  The
 * runs share the assembled matrices and both AMG hierarchies (none of them
 * depends on the per-run values) and advance together: every kernel launch
 * of a time step covers all runs, each with its own vectors, reductions,
 * Krylov control and convergence test, so each run takes the iterates it
 * would take alone.  chm_create is chm_create_batch with one run.  The
 * inspection calls below (chm_vcycle ... chm_rhs) work on run 0. */
int chm_create_batch(const chm_mesh_t *mesh, const chm_params_t *params, int32_t runs,
                     const chm_run_t *run, void *stream, chm_solver_t **out);

/* Number of runs of the solver (1 for chm_create). */
int chm_batch_size(const chm_solver_t *s);

/* Set the state (of run 0).  phi_p, phi_n: required, n_vertices values each.
 * mu_p, mu_n: optional (NULL = 0); they are only the first Krylov guess of
 * the next step. */
int chm_set_fields(chm_solver_t *s, const double *phi_p, const double *phi_n,
                   const double *mu_p, const double *mu_n, int32_t on_device);
/* The same for run `run` of a batch. */
int chm_set_fields_run(chm_solver_t *s, int32_t run, const double *phi_p, const double *phi_n,
                       const double *mu_p, const double *mu_n, int32_t on_device);

/* Advance nsteps time steps (eq. FE_systems for both species, then
 * phi_s = 1 - phi_p - phi_n and the optional solvent removal) of every run.
 * stats may be NULL or hold nsteps * runs entries (step-major: entry
 * k * runs + r for run r of step k).  On CHM_ENOCONV / CHM_ENAN (of any run)
 * every run is left at the last completed step and the failing step's stats
 * are filled; likewise on CHM_EDOMAIN (range_check = 1). */
int chm_step(chm_solver_t *s, int32_t nsteps, chm_stats_t *stats);

/* Advance several solvers (for example the batches of a parameter sweep,
 * one per mesh size) by nsteps time steps each, concurrently: one host thread
 * per solver, so that the launches of solvers on different HIP streams
 * overlap on the GPU (solvers that share a stream serialise on it).  The
 * handles must be distinct.  stats: NULL, or `count` pointers, each NULL or
 * room for nsteps * runs entries of that solver (as chm_step).  codes: NULL
 * or `count` entries receiving each solver's return code.  Returns CHM_OK, or
 * the code of the first failing solver in handle order (its chm_last_error
 * holds the message).  Each solver takes the iterates it takes in chm_step. */
int chm_step_many(chm_solver_t *const *solvers, int32_t count, int32_t nsteps,
                  chm_stats_t *const *stats, int32_t *codes);

/* Copy out the state (of run 0); any pointer may be NULL. */
int chm_get_fields(chm_solver_t *s, double *phi_p, double *phi_n, double *phi_s,
                   double *mu_p, double *mu_n, int32_t on_device);
/* The same for run `run` of a batch. */
int chm_get_fields_run(chm_solver_t *s, int32_t run, double *phi_p, double *phi_n, double *phi_s,
                       double *mu_p, double *mu_n, int32_t on_device);

/* Exact checkpoint and resume.  Besides the fields of chm_get_fields_run,
 * two things carry from one time step to the next: the history of solutions
 * of the solve that the extrapolating starts use (chm_set_guess in chm_net.h:
 * y1 = y_{n-1}, y2 = y_{n-2}, each a state vector of 4 n_vertices doubles in
 * the layout of chm_get_state, with `valid` = how many of them exist, 0..2),
 * and the run's count of completed time steps, which decides whether a step
 * removes solvent (evap_steps).  chm_get_history copies them out (y1, y2 may
 * be NULL; a vector past `valid` is left untouched).  chm_set_history,
 * called after chm_set_fields_run (which starts a history of one, the new
 * state), replaces them; a solver restored this way takes, from its next
 * chm_step on, the iterates the uninterrupted solver would take, bit for
 * bit.  y1 (valid >= 1) and y2 (valid = 2) are required by the set call;
 * steps_done >= 0.  on_device: as for the fields. */
int chm_get_history(chm_solver_t *s, int32_t run, double *y1, double *y2, int32_t *valid,
                    int64_t *steps_done, int32_t on_device);
int chm_set_history(chm_solver_t *s, int32_t run, const double *y1, const double *y2,
                    int32_t valid, int64_t steps_done, int32_t on_device);

int chm_destroy(chm_solver_t *s);

/* Message of the last failed call on s (s = NULL: of the last failed
 * chm_create on this thread).  Valid until the next call on s. */
const char *chm_last_error(const chm_solver_t *s);

/* ---- inspection (used by the parity tests; all synchronise the stream) ---- */

/* nnz of the shared pattern of M, K, As */
int64_t chm_nnz(const chm_solver_t *s);
/* which: 0 = M, 1 = K, 2 = As.  Host buffers rowptr[n+1], col[nnz], val[nnz]
 * (any may be NULL). */
int chm_get_matrix(chm_solver_t *s, int32_t which, int32_t *rowptr, int32_t *col, double *val);
/* hierarchy: 0 = mass, 1 = As */
int chm_num_levels(const chm_solver_t *s, int32_t hierarchy);
int chm_level_info(const chm_solver_t *s, int32_t hierarchy, int32_t level, int64_t *n,
                   int64_t *nnz_a, int64_t *nnz_p, double *rho);
/* How the solve kernels read a matrix: hierarchy 0 (mass) or 1 (As) with
 * its level's A, or hierarchy -1 for the solver's own M, K, As (one
 * pattern; level ignored).  *lanes_per_row: 0 for the SELL-64 layout (one
 * lane per row), else the lanes that share a CSR row; *index_bytes: bytes per
 * column index the kernels load, 2 for 16-bit offsets from the row (the
 * wide_index parameter), else 4.  Either pointer may be NULL. */
int chm_level_layout(const chm_solver_t *s, int32_t hierarchy, int32_t level,
                     int32_t *lanes_per_row, int32_t *index_bytes);
/* Value tables: where a SELL-64 matrix with 16-bit column offsets holds at
 * most 2048 distinct values (uniform meshes: 5 to 7 at 512 x 512, a few
 * hundred on the 3D box, where summation order splits equal sums), the
 * kernels read a 2-byte index per entry into the table of those values
 * instead of the value: the same value, so bitwise the same results, with
 * 2 bytes per entry instead of 8 (4 in FP32).  *values: the table size for
 * hierarchy 0 or 1 at `level` (its A), or hierarchy -1 with level 0 for M and
 * level 1 for K; 0 = no table (values read directly). */
int chm_value_table(const chm_solver_t *s, int32_t hierarchy, int32_t level, int32_t *values);
/* Host buffers; agg/P arrays are left untouched on the coarsest level. */
int chm_level_get(chm_solver_t *s, int32_t hierarchy, int32_t level, int32_t *a_rowptr,
                  int32_t *a_col, double *a_val, int32_t *agg, int32_t *p_rowptr,
                  int32_t *p_col, double *p_val);
/* Device pair vectors (double2[n]: species 0 in .x, 1 in .y).  These and
 * chm_apply_prec run in the configured precision (FP64 vectors in and out). */
int chm_vcycle(chm_solver_t *s, int32_t hierarchy, const double *b, double *x);
int chm_schur_solve(chm_solver_t *s, const double *b, double *x);
/* Device block vectors (double2[2n]: rows [0,n) phi block, [n,2n) mu block). */
int chm_apply_saddle(chm_solver_t *s, const double *x, double *y);
int chm_apply_prec(chm_solver_t *s, const double *v, double *w);
/* right-hand side of the current state into a device block vector b */
int chm_rhs(chm_solver_t *s, double *b);
/* the boundary vector G of the current state (run 0) into a device pair
 * vector g (double2[n]); zero without boundary terms */
int chm_boundary(chm_solver_t *s, double *g);

/* The CG steps per As solve chm_create settled on (with schur_pcg = -1:
 * 2 when one V-cycle of the As hierarchy contracts the As-norm error by at
 * most 0.3, 4 up to 0.6, else 6) and that contraction, measured at setup by
 * six steps of the power iteration e <- (I - V As) e from a seeded start
 * (SplitMix64 counters 2^32 + 2 i + s for row i and species s, mapped to
 * [-1, 1)), as the ratio of the As-norms of the last step (0 when schur_pcg
 * was given).  Either pointer may be NULL. */
int chm_schur_info(const chm_solver_t *s, int32_t *schur_pcg, double *contraction);

/* Host-only: the quadrature rule of the right-hand side (barycentric points
 * [npts][dim+1], weights summing to 1); bary and w hold at least 64 points. */
int chm_quadrature(int32_t dim, int32_t *npts, double *bary, double *w);

/* Per-launch timing of one kernel kind with HIP events on the solver's
 * stream (kind 0: fine-level Chebyshev step of the As hierarchy).  enable
 * resets the counters. */
int chm_timer_enable(chm_solver_t *s, int32_t kind, int32_t enable);
int chm_timer_read(chm_solver_t *s, int64_t *launches, double *total_ms, int64_t *bytes);
/* setup time of chm_create in ms and device bytes held */
int chm_setup_info(const chm_solver_t *s, double *setup_ms, int64_t *levels_m,
                   int64_t *levels_as);

#ifdef __cplusplus
}
#endif
#endif
