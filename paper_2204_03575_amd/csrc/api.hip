// C ABI of the library (declared in include/chm.h).  Argument checking,
// error capture and marshalling only; every step of the computation runs in
// the kernels of mesh_setup.hip, amg_setup.hip and solve.hip.
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

#include "chm_internal.h"

struct chm_solver {
    chm::Solver s;
};

namespace {

thread_local std::string g_create_error;

int fail(chm_solver *h, int code, const std::string &msg)
{
    if (h) {
        h->s.err.code = code;
        h->s.err.msg = msg;
    } else {
        g_create_error = msg;
    }
    return code;
}

template <class F> int guarded(chm_solver *h, F &&f)
{
    try {
        return f();
    } catch (const chm::Failure &e) {
        return fail(h, e.code, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(h, CHM_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(h, CHM_EINVAL, e.what());
    }
}

const char *check_params(const chm_params_t &p)
{
    if (!(p.tau > 0.0) || !std::isfinite(p.tau))
        return "tau must be positive";
    for (int s = 0; s < 2; ++s) {
        if (!(p.eps[s] > 0.0) || !(p.mobility[s] > 0.0))
            return "eps and mobility must be positive";
    }
    if (p.eps[0] != p.eps[1] || p.mobility[0] != p.mobility[1])
        return "both species must share eps and mobility (one As hierarchy)";
    if (p.potential < 0 || p.potential > 2)
        return "unknown potential";
    if (p.potential == CHM_POT_FLORY_HUGGINS &&
        (!(p.Np > 0) || !(p.Nn > 0) || !(p.Ns > 0) || !(p.log_floor > 0.0)))
        return "Flory-Huggins needs positive N_p, N_n, N_s and log_floor";
    if (!(p.rtol > 0.0) || p.restart < 1 || p.restart > chm::kMaxRestart || p.max_iters < 1)
        return "need rtol > 0, 1 <= restart <= 64, max_iters >= 1";
    if (p.amg_cycles < 1 || p.schur_pcg < -1 || p.schur_pcg > 39)
        return "need amg_cycles >= 1 and -1 <= schur_pcg <= 39";
    if (p.schur_pcg < 0 && p.krylov != CHM_KRYLOV_FGMRES)
        return "the automatic inner CG steps (schur_pcg = -1) need FGMRES";
    if (p.smoother != CHM_SMOOTH_CHEBYSHEV && p.smoother != CHM_SMOOTH_JACOBI)
        return "unknown smoother";
    if (p.cheb_degree < 1 || p.cheb_degree > 31 || p.cheb_degree_mass < 1 || p.cheb_degree_mass > 31)
        return "smoother degrees must be in 1..31";
    if (!(p.cheb_ratio > 1.0) || !(p.cheb_ratio_mass > 1.0))
        return "Chebyshev ratios must exceed 1";
    if (p.coarse_max < 1 || p.max_levels < 1 || p.max_levels > chm::kMaxLevels)
        return "need coarse_max >= 1 and 1 <= max_levels <= 24";
    if (p.evap_ds < 0.0 || p.evap_steps < 0)
        return "evaporation settings must be non-negative";
    if (p.precision != CHM_PREC_FP64 && p.precision != CHM_PREC_FP32)
        return "unknown precision";
    if (p.boundary != 0 && p.boundary != 1)
        return "boundary must be 0 or 1";
    if (p.boundary && (!(p.bc_k >= 0.0) || !std::isfinite(p.bc_k) || !std::isfinite(p.bc_g[0]) ||
                       !std::isfinite(p.bc_g[1]) || !std::isfinite(p.bc_h[0]) ||
                       !std::isfinite(p.bc_h[1]) || (p.bc_pattern != 0 && p.bc_pattern != 1)))
        return "bad boundary coefficients";
    if (p.krylov != CHM_KRYLOV_FGMRES && p.krylov != CHM_KRYLOV_MINRES)
        return "unknown Krylov method";
    if (!(p.amg_tol >= 0.0) || !std::isfinite(p.amg_tol))
        return "amg_tol must be finite and non-negative";
    if (p.mass_solver != CHM_MASS_AMG && p.mass_solver != CHM_MASS_CHEBYSHEV)
        return "unknown mass solver";
    if (p.wide_index != 0 && p.wide_index != 1)
        return "wide_index must be 0 or 1";
    if (p.runs_per_lane != 0 && p.runs_per_lane != 1 && p.runs_per_lane != 2 && p.runs_per_lane != 4)
        return "runs_per_lane must be 0, 1, 2 or 4";
    if (p.cheb_degree_coarse < 0 || p.cheb_degree_coarse > 31)
        return "cheb_degree_coarse must be in 0..31";
    if (p.range_check != 0 && p.range_check != 1)
        return "range_check must be 0 or 1";
    if (p.ortho != CHM_ORTHO_CGS2 && p.ortho != CHM_ORTHO_DCGS2)
        return "ortho must be CHM_ORTHO_CGS2 or CHM_ORTHO_DCGS2";
    if (p.values_direct != 0 && p.values_direct != 1)
        return "values_direct must be 0 or 1";
    if (p.krylov == CHM_KRYLOV_MINRES && p.schur_pcg != 0)
        return "MINRES needs a symmetric positive definite preconditioner: schur_pcg = 0";
    return nullptr;
}

// Automatic inner CG steps per As solve (schur_pcg = -1): the power
// iteration runs kContractionIters steps, and a V-cycle contracting by rho
// gets 2 CG steps up to kRhoTwo, 4 up to kRhoFour, else 6.
constexpr int kContractionIters = 6;
constexpr double kRhoTwo = 0.3, kRhoFour = 0.6;

int schur_steps_for(double rho) { return rho <= kRhoTwo ? 2 : (rho <= kRhoFour ? 4 : 6); }

// one field into component `comp` of a pair vector, and back out: comp 0
// or 1, or 2 for phi_s = 1 - phi_p - phi_n (Section 2)
__global__ void k_field_in(int n, const double *__restrict__ src, double2 *dst, int comp)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    double2 v = dst[i];
    if (comp == 0)
        v.x = src[i];
    else
        v.y = src[i];
    dst[i] = v;
}

__global__ void k_field_out(int n, const double2 *__restrict__ src, double *dst, int comp)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    const double2 v = src[i];
    dst[i] = comp == 0 ? v.x : (comp == 1 ? v.y : 1.0 - v.x - v.y);
}

inline int blocks256(int n) { return n > 0 ? (n + 255) / 256 : 1; }

// src: device or host (through the solver's staging vector)
void copy_field(chm::Solver &S, double2 *dst, int comp, const double *src, bool on_device)
{
    const int n = S.nv;
    if (!on_device) {
        CHM_HIP(hipMemcpyAsync(S.stage, src, sizeof(double) * n, hipMemcpyHostToDevice, S.stream));
        src = S.stage;
    }
    k_field_in<<<blocks256(n), 256, 0, S.stream>>>(n, src, dst, comp);
    CHM_HIP(hipGetLastError());
}

void get_field(chm::Solver &S, double *dst, const double2 *src, int comp, bool on_device)
{
    const int n = S.nv;
    double *out = on_device ? dst : S.stage;
    k_field_out<<<blocks256(n), 256, 0, S.stream>>>(n, src, out, comp);
    CHM_HIP(hipGetLastError());
    if (!on_device)
        CHM_HIP(hipMemcpyAsync(dst, S.stage, sizeof(double) * n, hipMemcpyDeviceToHost, S.stream));
}

}  // namespace

extern "C" {

int chm_create(const chm_mesh_t *mesh, const chm_params_t *params, void *stream,
               chm_solver_t **out)
{
    return chm_create_batch(mesh, params, 1, nullptr, stream, out);
}

int chm_create_batch(const chm_mesh_t *mesh, const chm_params_t *params, int32_t runs,
                     const chm_run_t *run_params, void *stream, chm_solver_t **out)
{
    if (out)
        *out = nullptr;
    if (!mesh || !params || !out)
        return fail(nullptr, CHM_EINVAL, "chm_create: NULL argument");
    if (runs < 1 || runs > chm::kMaxRuns)
        return fail(nullptr, CHM_EINVAL, "chm_create: runs must be in 1..64");
    if (run_params)
        for (int r = 0; r < runs; ++r)
            if (!(run_params[r].evap_ds >= 0.0) || run_params[r].evap_steps < 0 ||
                !std::isfinite(run_params[r].chi_pn) || !std::isfinite(run_params[r].chi_ps) ||
                !std::isfinite(run_params[r].chi_ns))
                return fail(nullptr, CHM_EINVAL, "chm_create: bad run parameters");
    if ((mesh->dim != 2 && mesh->dim != 3) || mesh->n_vertices < 1 || mesh->n_cells < 1 ||
        !mesh->coords || !mesh->cells || mesh->n_vertices > 0x3fffffff || mesh->n_cells > 0x1fffffff)
        return fail(nullptr, CHM_EINVAL, "chm_create: bad mesh dimensions or pointers");
    if (const char *why = check_params(*params))
        return fail(nullptr, CHM_EINVAL, std::string("chm_create: ") + why);
    const int nl = mesh->dim + 1;
    for (int64_t i = 0; i < mesh->n_cells * nl; ++i)
        if (mesh->cells[i] < 0 || mesh->cells[i] >= mesh->n_vertices)
            return fail(nullptr, CHM_EINVAL, "chm_create: cell vertex index out of range");
    for (int64_t i = 0; i < mesh->n_vertices * mesh->dim; ++i)
        if (!std::isfinite(mesh->coords[i]))
            return fail(nullptr, CHM_EINVAL, "chm_create: non-finite coordinate");

    chm_solver *h = new (std::nothrow) chm_solver;
    if (!h)
        return fail(nullptr, CHM_ENOMEM, "chm_create: host allocation failed");
    int rc = guarded(h, [&]() {
        chm::Solver &S = h->s;
        auto t0 = std::chrono::steady_clock::now();
        S.stream = static_cast<hipStream_t>(stream);
        S.prm = *params;
        S.nb = runs;
        S.nrun = 1;
        S.rb = params->runs_per_lane > 0 ? params->runs_per_lane : 2;
        S.runs.resize(runs);
        S.hist.assign(runs, 0);
        S.steps.assign(runs, 0);
        for (int r = 0; r < runs; ++r) {
            chm::RunPrm &P = S.runs[r];
            if (run_params) {
                P.chi_pn = run_params[r].chi_pn;
                P.chi_ps = run_params[r].chi_ps;
                P.chi_ns = run_params[r].chi_ns;
                P.evap_ds = run_params[r].evap_ds;
                P.evap_steps = run_params[r].evap_steps;
            } else {
                P.chi_pn = params->chi_pn;
                P.chi_ps = params->chi_ps;
                P.chi_ns = params->chi_ns;
                P.evap_ds = params->evap_ds;
                P.evap_steps = params->evap_steps;
            }
        }
        S.dim = mesh->dim;
        S.nv = (int)mesh->n_vertices;
        S.ncell = (int)mesh->n_cells;
        S.nl = nl;
        for (int s = 0; s < 2; ++s) {
            S.tau_s[s] = S.prm.tau * S.prm.mobility[s];
            S.te_s[s] = S.tau_s[s] / S.prm.eps[s];
        }
        S.coords = S.pool.get<double>((size_t)S.nv * S.dim);
        S.cells = S.pool.get<int>((size_t)S.ncell * nl);
        CHM_HIP(hipMemcpyAsync(S.coords, mesh->coords, sizeof(double) * S.nv * S.dim,
                               hipMemcpyHostToDevice, S.stream));
        CHM_HIP(hipMemcpyAsync(S.cells, mesh->cells, sizeof(int) * (size_t)S.ncell * nl,
                               hipMemcpyHostToDevice, S.stream));
        chm::mesh_setup(S);
        chm::boundary_setup(S);
        S.hM.degree = S.prm.cheb_degree_mass;
        S.hM.ratio = S.prm.cheb_ratio_mass;
        S.hM.jacobi = S.prm.smoother == CHM_SMOOTH_JACOBI;
        S.hA.degree = S.prm.cheb_degree;
        S.hA.degree_coarse = S.prm.cheb_degree_coarse;
        S.hA.ratio = S.prm.cheb_ratio;
        S.hA.jacobi = S.hM.jacobi;
        chm::amg_build(S, S.hM, S.M);
        chm::amg_build(S, S.hA, S.As);
        S.mixed = S.prm.precision == CHM_PREC_FP32;
        chm::prec_setup(S);
        chm::alloc_workspace(S);
        if (S.prm.schur_pcg < 0) {
            // automatic inner CG steps from the measured V-cycle contraction
            S.vc_rho = chm::vcycle_contraction(S, kContractionIters);
            S.prm.schur_pcg = schur_steps_for(S.vc_rho);
        }
        if (S.prm.krylov == CHM_KRYLOV_MINRES)
            chm::minres_alloc(S);
        CHM_HIP(hipStreamSynchronize(S.stream));
        S.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return CHM_OK;
    });
    if (rc != CHM_OK) {
        g_create_error = h->s.err.msg;
        (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (h->s.hctl)
            (void)hipHostFree(h->s.hctl);
        if (h->s.hmrctl)
            (void)hipHostFree(h->s.hmrctl);
        if (h->s.hamg_act)
            (void)hipHostFree(h->s.hamg_act);
        delete h;
        return rc;
    }
    *out = h;
    return CHM_OK;
}

int chm_set_fields(chm_solver_t *h, const double *phi_p, const double *phi_n, const double *mu_p,
                   const double *mu_n, int32_t on_device)
{
    return chm_set_fields_run(h, 0, phi_p, phi_n, mu_p, mu_n, on_device);
}

int chm_set_fields_run(chm_solver_t *h, int32_t run, const double *phi_p, const double *phi_n,
                       const double *mu_p, const double *mu_n, int32_t on_device)
{
    if (!h)
        return fail(nullptr, CHM_EINVAL, "chm_set_fields: NULL handle");
    if (!phi_p || !phi_n)
        return fail(h, CHM_EINVAL, "chm_set_fields: phi_p and phi_n are required");
    if (run < 0 || run >= h->s.nb)
        return fail(h, CHM_EINVAL, "chm_set_fields: run out of range");
    return guarded(h, [&]() {
        chm::Solver &S = h->s;
        const int n = S.nv;
        double2 *xr = S.x + (size_t)run * 2 * n;
        copy_field(S, xr, 0, phi_p, on_device);
        copy_field(S, xr, 1, phi_n, on_device);
        chm::fill_double(reinterpret_cast<double *>(xr + n), 0.0, 2 * (size_t)n, S.stream);
        if (mu_p)
            copy_field(S, xr + n, 0, mu_p, on_device);
        if (mu_n)
            copy_field(S, xr + n, 1, mu_n, on_device);
        // the new state starts this run's history of solutions
        CHM_HIP(hipMemcpyAsync(S.yh1 + (size_t)run * 2 * n, xr, sizeof(double2) * 2 * (size_t)n,
                               hipMemcpyDeviceToDevice, S.stream));
        S.hist[run] = 1;
        CHM_HIP(hipStreamSynchronize(S.stream));
        return CHM_OK;
    });
}

int chm_step(chm_solver_t *h, int32_t nsteps, chm_stats_t *stats)
{
    if (!h)
        return fail(nullptr, CHM_EINVAL, "chm_step: NULL handle");
    if (nsteps < 0)
        return fail(h, CHM_EINVAL, "chm_step: nsteps < 0");
    return guarded(h, [&]() {
        for (int k = 0; k < nsteps; ++k) {
            int rc = chm::step_once(h->s, stats ? stats + (size_t)k * h->s.nb : nullptr);
            if (rc != CHM_OK)
                return fail(h, rc, rc == CHM_ENOCONV
                                       ? "the Krylov method did not converge within max_iters"
                                       : rc == CHM_EDOMAIN
                                             ? "the new state leaves [0, 1] (" + h->s.nan_where + ")"
                                             : "non-finite value in the solve (" + h->s.nan_where + ")");
        }
        return CHM_OK;
    });
}

int chm_step_many(chm_solver_t *const *solvers, int32_t count, int32_t nsteps,
                  chm_stats_t *const *stats, int32_t *codes)
{
    if (!solvers || count < 1 || count > 1024 || nsteps < 0)
        return fail(nullptr, CHM_EINVAL, "chm_step_many: bad arguments");
    for (int i = 0; i < count; ++i) {
        if (!solvers[i])
            return fail(nullptr, CHM_EINVAL, "chm_step_many: NULL handle");
        for (int j = 0; j < i; ++j)
            if (solvers[j] == solvers[i])
                return fail(nullptr, CHM_EINVAL, "chm_step_many: a handle appears twice");
    }
    std::vector<int> rc(count, CHM_OK);
    std::vector<std::thread> pool;
    try {
        pool.reserve(count);
        for (int i = 0; i < count; ++i)
            pool.emplace_back([&, i]() { rc[i] = chm_step(solvers[i], nsteps, stats ? stats[i] : nullptr); });
    } catch (const std::exception &e) {
        for (std::thread &t : pool)
            t.join();
        return fail(nullptr, CHM_EINVAL, std::string("chm_step_many: cannot start threads: ") + e.what());
    }
    for (std::thread &t : pool)
        t.join();
    int first = CHM_OK;
    for (int i = 0; i < count; ++i) {
        if (codes)
            codes[i] = rc[i];
        if (first == CHM_OK && rc[i] != CHM_OK)
            first = rc[i];
    }
    return first;
}

int chm_get_fields(chm_solver_t *h, double *phi_p, double *phi_n, double *phi_s, double *mu_p,
                   double *mu_n, int32_t on_device)
{
    return chm_get_fields_run(h, 0, phi_p, phi_n, phi_s, mu_p, mu_n, on_device);
}

int chm_get_fields_run(chm_solver_t *h, int32_t run, double *phi_p, double *phi_n, double *phi_s,
                       double *mu_p, double *mu_n, int32_t on_device)
{
    if (!h)
        return fail(nullptr, CHM_EINVAL, "chm_get_fields: NULL handle");
    if (run < 0 || run >= h->s.nb)
        return fail(h, CHM_EINVAL, "chm_get_fields: run out of range");
    return guarded(h, [&]() {
        chm::Solver &S = h->s;
        const int n = S.nv;
        const double2 *xr = S.x + (size_t)run * 2 * n;
        if (phi_p)
            get_field(S, phi_p, xr, 0, on_device);
        if (phi_n)
            get_field(S, phi_n, xr, 1, on_device);
        if (phi_s)
            get_field(S, phi_s, xr, 2, on_device);
        if (mu_p)
            get_field(S, mu_p, xr + n, 0, on_device);
        if (mu_n)
            get_field(S, mu_n, xr + n, 1, on_device);
        CHM_HIP(hipStreamSynchronize(S.stream));
        return CHM_OK;
    });
}

int chm_get_history(chm_solver_t *h, int32_t run, double *y1, double *y2, int32_t *valid,
                    int64_t *steps_done, int32_t on_device)
{
    if (!h)
        return fail(nullptr, CHM_EINVAL, "chm_get_history: NULL handle");
    if (run < 0 || run >= h->s.nb)
        return fail(h, CHM_EINVAL, "chm_get_history: run out of range");
    return guarded(h, [&]() {
        chm::Solver &S = h->s;
        const size_t bytes = sizeof(double2) * 2 * (size_t)S.nv;
        const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        const int have = S.hist[run];
        if (y1 && have >= 1)
            CHM_HIP(hipMemcpyAsync(y1, S.yh1 + (size_t)run * 2 * S.nv, bytes, kind, S.stream));
        if (y2 && have >= 2)
            CHM_HIP(hipMemcpyAsync(y2, S.yh2 + (size_t)run * 2 * S.nv, bytes, kind, S.stream));
        if (valid)
            *valid = have;
        if (steps_done)
            *steps_done = S.steps[run];
        CHM_HIP(hipStreamSynchronize(S.stream));
        return CHM_OK;
    });
}

int chm_set_history(chm_solver_t *h, int32_t run, const double *y1, const double *y2,
                    int32_t valid, int64_t steps_done, int32_t on_device)
{
    if (!h)
        return fail(nullptr, CHM_EINVAL, "chm_set_history: NULL handle");
    if (run < 0 || run >= h->s.nb)
        return fail(h, CHM_EINVAL, "chm_set_history: run out of range");
    if (valid < 0 || valid > 2 || steps_done < 0 || (valid >= 1 && !y1) || (valid == 2 && !y2))
        return fail(h, CHM_EINVAL, "chm_set_history: need 0 <= valid <= 2 with y1 (and y2) "
                                   "given, and steps_done >= 0");
    return guarded(h, [&]() {
        chm::Solver &S = h->s;
        const size_t bytes = sizeof(double2) * 2 * (size_t)S.nv;
        const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        if (valid >= 1)
            CHM_HIP(hipMemcpyAsync(S.yh1 + (size_t)run * 2 * S.nv, y1, bytes, kind, S.stream));
        if (valid >= 2)
            CHM_HIP(hipMemcpyAsync(S.yh2 + (size_t)run * 2 * S.nv, y2, bytes, kind, S.stream));
        CHM_HIP(hipStreamSynchronize(S.stream));
        S.hist[run] = valid;
        S.steps[run] = steps_done;
        return CHM_OK;
    });
}

int chm_destroy(chm_solver_t *h)
{
    if (!h)
        return CHM_OK;
    (void)hipStreamSynchronize(h->s.stream);
    for (hipEvent_t e : h->s.timer.ev)
        (void)hipEventDestroy(e);
    for (hipGraphExec_t g : h->s.iter_graphs)
        if (g)
            (void)hipGraphExecDestroy(g);
    if (h->s.cap_stream)
        (void)hipStreamDestroy(h->s.cap_stream);
    if (h->s.hctl)
        (void)hipHostFree(h->s.hctl);
    if (h->s.hmrctl)
        (void)hipHostFree(h->s.hmrctl);
    if (h->s.hamg_act)
        (void)hipHostFree(h->s.hamg_act);
    delete h;
    return CHM_OK;
}

const char *chm_last_error(const chm_solver_t *h)
{
    if (!h)
        return g_create_error.c_str();
    return h->s.err.msg.c_str();
}

int64_t chm_nnz(const chm_solver_t *h) { return h ? h->s.M.nnz : -1; }

int chm_get_matrix(chm_solver_t *h, int32_t which, int32_t *rowptr, int32_t *col, double *val)
{
    if (!h || which < 0 || which > 2)
        return fail(h, CHM_EINVAL, "chm_get_matrix: bad arguments");
    return guarded(h, [&]() {
        chm::Solver &S = h->s;
        const chm::Csr &A = which == 0 ? S.M : which == 1 ? S.K : S.As;
        if (rowptr)
            CHM_HIP(hipMemcpy(rowptr, A.rp, sizeof(int) * (A.n + 1), hipMemcpyDeviceToHost));
        if (col)
            CHM_HIP(hipMemcpy(col, A.ci, sizeof(int) * A.nnz, hipMemcpyDeviceToHost));
        if (val)
            CHM_HIP(hipMemcpy(val, A.v, sizeof(double) * A.nnz, hipMemcpyDeviceToHost));
        return CHM_OK;
    });
}

static const chm::Hierarchy *hier_of(const chm_solver_t *h, int hier)
{
    if (!h || hier < 0 || hier > 1)
        return nullptr;
    return hier == 0 ? &h->s.hM : &h->s.hA;
}

int chm_num_levels(const chm_solver_t *h, int32_t hierarchy)
{
    const chm::Hierarchy *H = hier_of(h, hierarchy);
    return H ? H->nlev : CHM_EINVAL;
}

int chm_level_info(const chm_solver_t *h, int32_t hierarchy, int32_t level, int64_t *n,
                   int64_t *nnz_a, int64_t *nnz_p, double *rho)
{
    const chm::Hierarchy *H = hier_of(h, hierarchy);
    if (!H || level < 0 || level >= H->nlev)
        return CHM_EINVAL;
    const chm::Level &L = H->lev[level];
    if (n)
        *n = L.n;
    if (nnz_a)
        *nnz_a = L.A.nnz;
    if (nnz_p)
        *nnz_p = (level + 1 < H->nlev) ? L.P.nnz : 0;
    if (rho)
        *rho = L.rho;
    return CHM_OK;
}

int chm_level_layout(const chm_solver_t *h, int32_t hierarchy, int32_t level,
                     int32_t *lanes_per_row, int32_t *index_bytes)
{
    int lanes = 0;
    const int16_t *ocol = nullptr;
    if (h && hierarchy == -1) {
        ocol = h->s.sM.ocol;
    } else {
        const chm::Hierarchy *H = hier_of(h, hierarchy);
        if (!H || level < 0 || level >= H->nlev)
            return CHM_EINVAL;
        const chm::Level &L = H->lev[level];
        lanes = L.gsA;
        ocol = L.sA.ocol;
    }
    if (lanes_per_row)
        *lanes_per_row = lanes;
    if (index_bytes)
        *index_bytes = (lanes == 0 && ocol) ? 2 : 4;
    return CHM_OK;
}

int chm_value_table(const chm_solver_t *h, int32_t hierarchy, int32_t level, int32_t *values)
{
    if (!h || !values)
        return CHM_EINVAL;
    if (hierarchy == -1) {
        if (level != 0 && level != 1)
            return CHM_EINVAL;
        *values = level == 0 ? h->s.vtM.m : h->s.vtK.m;
        return CHM_OK;
    }
    const chm::Hierarchy *H = hier_of(h, hierarchy);
    if (!H || level < 0 || level >= H->nlev)
        return CHM_EINVAL;
    *values = H->lev[level].vtA.m;
    return CHM_OK;
}

int chm_level_get(chm_solver_t *h, int32_t hierarchy, int32_t level, int32_t *a_rowptr,
                  int32_t *a_col, double *a_val, int32_t *agg, int32_t *p_rowptr, int32_t *p_col,
                  double *p_val)
{
    const chm::Hierarchy *H = hier_of(h, hierarchy);
    if (!H || level < 0 || level >= H->nlev)
        return fail(h ? const_cast<chm_solver_t *>(h) : nullptr, CHM_EINVAL, "chm_level_get: bad level");
    return guarded(h, [&]() {
        const chm::Level &L = H->lev[level];
        CHM_HIP(hipStreamSynchronize(h->s.stream));
        if (a_rowptr)
            CHM_HIP(hipMemcpy(a_rowptr, L.A.rp, sizeof(int) * (L.n + 1), hipMemcpyDeviceToHost));
        if (a_col)
            CHM_HIP(hipMemcpy(a_col, L.A.ci, sizeof(int) * L.A.nnz, hipMemcpyDeviceToHost));
        if (a_val)
            CHM_HIP(hipMemcpy(a_val, L.A.v, sizeof(double) * L.A.nnz, hipMemcpyDeviceToHost));
        if (level + 1 < H->nlev) {
            if (agg)
                CHM_HIP(hipMemcpy(agg, L.agg, sizeof(int) * L.n, hipMemcpyDeviceToHost));
            if (p_rowptr)
                CHM_HIP(hipMemcpy(p_rowptr, L.P.rp, sizeof(int) * (L.n + 1), hipMemcpyDeviceToHost));
            if (p_col)
                CHM_HIP(hipMemcpy(p_col, L.P.ci, sizeof(int) * L.P.nnz, hipMemcpyDeviceToHost));
            if (p_val)
                CHM_HIP(hipMemcpy(p_val, L.P.v, sizeof(double) * L.P.nnz, hipMemcpyDeviceToHost));
        }
        return CHM_OK;
    });
}

int chm_vcycle(chm_solver_t *h, int32_t hierarchy, const double *b, double *x)
{
    if (!h || hierarchy < 0 || hierarchy > 1 || !b || !x)
        return fail(h, CHM_EINVAL, "chm_vcycle: bad arguments");
    return guarded(h, [&]() {
        chm::Solver &S = h->s;
        S.nrun = 1;   // run 0's buffers; the caller's vectors are one run's
        chm::vcycle(S, hierarchy, reinterpret_cast<const double2 *>(b),
                    reinterpret_cast<double2 *>(x));
        CHM_HIP(hipGetLastError());
        CHM_HIP(hipStreamSynchronize(S.stream));
        return CHM_OK;
    });
}

int chm_schur_solve(chm_solver_t *h, const double *b, double *x)
{
    if (!h || !b || !x)
        return fail(h, CHM_EINVAL, "chm_schur_solve: bad arguments");
    return guarded(h, [&]() {
        h->s.nrun = 1;
        chm::schur_solve(h->s, reinterpret_cast<const double2 *>(b), reinterpret_cast<double2 *>(x));
        CHM_HIP(hipGetLastError());
        CHM_HIP(hipStreamSynchronize(h->s.stream));
        return CHM_OK;
    });
}

int chm_apply_saddle(chm_solver_t *h, const double *x, double *y)
{
    if (!h || !x || !y)
        return fail(h, CHM_EINVAL, "chm_apply_saddle: bad arguments");
    return guarded(h, [&]() {
        h->s.nrun = 1;
        chm::apply_saddle(h->s, reinterpret_cast<const double2 *>(x), reinterpret_cast<double2 *>(y));
        CHM_HIP(hipGetLastError());
        CHM_HIP(hipStreamSynchronize(h->s.stream));
        return CHM_OK;
    });
}

int chm_apply_prec(chm_solver_t *h, const double *v, double *w)
{
    if (!h || !v || !w)
        return fail(h, CHM_EINVAL, "chm_apply_prec: bad arguments");
    return guarded(h, [&]() {
        h->s.nrun = 1;
        chm::apply_prec(h->s, reinterpret_cast<const double2 *>(v), reinterpret_cast<double2 *>(w));
        CHM_HIP(hipGetLastError());
        CHM_HIP(hipStreamSynchronize(h->s.stream));
        return CHM_OK;
    });
}

int chm_rhs(chm_solver_t *h, double *b)
{
    if (!h || !b)
        return fail(h, CHM_EINVAL, "chm_rhs: bad arguments");
    return guarded(h, [&]() {
        chm::Solver &S = h->s;
        S.nrun = 1;
        chm::compute_rhs(S);
        CHM_HIP(hipMemcpyAsync(b, S.b, sizeof(double2) * 2 * (size_t)S.nv, hipMemcpyDeviceToDevice,
                               S.stream));
        CHM_HIP(hipStreamSynchronize(S.stream));
        return CHM_OK;
    });
}

int chm_quadrature(int32_t dim, int32_t *npts, double *bary, double *w)
{
    if ((dim != 2 && dim != 3) || !npts || !bary || !w)
        return CHM_EINVAL;
    std::vector<double> b, ww;
    chm::build_quadrature(dim, b, ww);
    *npts = (int32_t)ww.size();
    std::memcpy(bary, b.data(), sizeof(double) * b.size());
    std::memcpy(w, ww.data(), sizeof(double) * ww.size());
    return CHM_OK;
}

int chm_timer_enable(chm_solver_t *h, int32_t kind, int32_t enable)
{
    if (!h || kind != 0)
        return fail(h, CHM_EINVAL, "chm_timer_enable: unknown kernel kind");
    chm::Timer &T = h->s.timer;
    T.on = enable != 0;
    T.kind = kind;
    T.used = 0;
    T.total_ms = 0.0;
    T.count = 0;
    T.bytes = 0;
    return CHM_OK;
}

int chm_timer_read(chm_solver_t *h, int64_t *launches, double *total_ms, int64_t *bytes)
{
    if (!h)
        return fail(nullptr, CHM_EINVAL, "chm_timer_read: NULL handle");
    return guarded(h, [&]() {
        chm::Timer &T = h->s.timer;
        CHM_HIP(hipStreamSynchronize(h->s.stream));
        for (size_t i = 0; i + 1 < T.used; i += 2) {
            float ms = 0.f;
            CHM_HIP(hipEventElapsedTime(&ms, T.ev[i], T.ev[i + 1]));
            T.total_ms += ms;
        }
        T.used = 0;
        if (launches)
            *launches = T.count;
        if (total_ms)
            *total_ms = T.total_ms;
        if (bytes)
            *bytes = T.bytes;
        return CHM_OK;
    });
}

int chm_setup_info(const chm_solver_t *h, double *setup_ms, int64_t *levels_m, int64_t *levels_as)
{
    if (!h)
        return CHM_EINVAL;
    if (setup_ms)
        *setup_ms = h->s.setup_ms;
    if (levels_m)
        *levels_m = h->s.hM.nlev;
    if (levels_as)
        *levels_as = h->s.hA.nlev;
    return CHM_OK;
}

int chm_set_guess(chm_solver_t *h, int32_t mode, chm_net_t *net, int32_t H, int32_t W)
{
    if (!h)
        return fail(nullptr, CHM_EINVAL, "chm_set_guess: NULL handle");
    chm::Solver &S = h->s;
    if (mode != CHM_GUESS_PREVIOUS && mode != CHM_GUESS_LINEAR && mode != CHM_GUESS_LEARNED)
        return fail(h, CHM_EINVAL, "chm_set_guess: unknown mode");
    if (mode == CHM_GUESS_LEARNED) {
        if (!net)
            return fail(h, CHM_EINVAL, "chm_set_guess: the learned guess needs a network");
        if (S.dim != 2 || H < 2 || W < 2 || (int64_t)H * W != S.nv)
            return fail(h, CHM_EINVAL, "chm_set_guess: the learned guess needs a 2D H x W vertex "
                                       "grid with H * W = n_vertices");
        if ((long long)H * W > chm::net_max_pixels(net))
            return fail(h, CHM_EINVAL, "chm_set_guess: the grid exceeds the network's max_pixels");
    }
    S.guess_mode = mode;
    S.net = mode == CHM_GUESS_LEARNED ? net : nullptr;
    S.gH = H;
    S.gW = W;
    return CHM_OK;
}

int chm_get_state(chm_solver_t *h, int32_t which, double *state)
{
    if (!h || !state || which < 0 || which > 1)
        return fail(h, CHM_EINVAL, "chm_get_state: bad arguments");
    return guarded(h, [&]() {
        chm::Solver &S = h->s;
        if (which == 1 && S.hist[0] < 1)
            throw chm::Failure(CHM_EINVAL, "chm_get_state: no solution yet");
        CHM_HIP(hipMemcpyAsync(state, which == 0 ? S.x : S.yh1, sizeof(double2) * 2 * (size_t)S.nv,
                               hipMemcpyDeviceToDevice, S.stream));
        CHM_HIP(hipStreamSynchronize(S.stream));
        return CHM_OK;
    });
}

int chm_batch_size(const chm_solver_t *h) { return h ? h->s.nb : CHM_EINVAL; }

int chm_schur_info(const chm_solver_t *h, int32_t *schur_pcg, double *contraction)
{
    if (!h)
        return CHM_EINVAL;
    if (schur_pcg)
        *schur_pcg = h->s.prm.schur_pcg;
    if (contraction)
        *contraction = h->s.vc_rho;
    return CHM_OK;
}

int chm_boundary(chm_solver_t *h, double *g)
{
    if (!h || !g)
        return fail(h, CHM_EINVAL, "chm_boundary: bad arguments");
    return guarded(h, [&]() {
        chm::Solver &S = h->s;
        S.nrun = 1;
        chm::boundary_rhs(S, reinterpret_cast<double2 *>(g));
        CHM_HIP(hipStreamSynchronize(S.stream));
        return CHM_OK;
    });
}

}  // extern "C"
