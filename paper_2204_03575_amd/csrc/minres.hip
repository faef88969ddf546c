// Preconditioned MINRES (Paige and Saunders 1975), the Krylov method of the
// paper's experiments, for both species of every run of a batch: the Lanczos
// process on P^-1 A in the P inner product with three-term recurrences, the
// QR factorisation of its tridiagonal matrix by Givens rotations (per
// species scalars on the device), and the iterate updated along the
// directions w.  P^-1 is Algorithm 1 with stationary V-cycles in both blocks
// (symmetric positive definite).  The method stops when phibar, the residual
// in the P^-1 norm given by the rotations, is at most rtol times the P^-1
// norm of b; the true 2-norm residual is reported.  Vectors are block
// vectors (2n pairs per run, runs back to back); reductions are fixed-grid
// partial sums added in a fixed order.
#include <cmath>

#include "device_util.h"

namespace chm {

namespace {

// per run: the recurrence scalars of both species
struct MrCtl {
    double beta[2], oldb[2], alfa[2], dbar[2], epsln[2], phibar[2], cs[2], sn[2];
    double phi[2], delta[2], oldeps[2], gamma[2], tol[2];
    int active[2];   // still iterating
    int upd[2];      // took part in the last iteration
    int nan;
    int pad;
};

constexpr int kSlotA = kSlotGuess;       // partial sums: alfa / b.P^-1 b / beta^2

__device__ inline double2 sum_parts(const double2 *__restrict__ part, int G, double2 *sh)
{
    reduce_parts(part, 1, G, sh);
    return sh[0];
}

// tol = rtol sqrt(b . P^-1 b) from partials; clears the non-finite flag
__global__ void __launch_bounds__(kBlock) k_mr_tol(MrCtl *c, const double2 *__restrict__ part, int G,
                                                   double rtol)
{
    __shared__ double2 sh[1];
    c += blockIdx.y;
    const double2 s = sum_parts(run_at(part, kSlotStride), G, sh);
    if (threadIdx.x == 0) {
        int bad = 0;
        for (int q = 0; q < 2; ++q) {
            const double v = q == 0 ? s.x : s.y;
            bad |= !(v >= 0.0);   // an indefinite preconditioner, or a non-finite b
            c->tol[q] = rtol * sqrt(v >= 0.0 ? v : 0.0);
        }
        c->nan = bad;
    }
}

// beta_1 = sqrt(r1 . P^-1 r1) from partials; the recurrence starts, and a
// species iterates while phibar = beta_1 exceeds its tolerance
__global__ void __launch_bounds__(kBlock) k_mr_start(MrCtl *c, const double2 *__restrict__ part, int G)
{
    __shared__ double2 sh[1];
    c += blockIdx.y;
    const double2 s = sum_parts(run_at(part, kSlotStride), G, sh);
    if (threadIdx.x == 0) {
        int bad = c->nan;
        for (int q = 0; q < 2; ++q) {
            const double v = q == 0 ? s.x : s.y;
            bad |= !(v >= 0.0);
            const double beta = sqrt(v >= 0.0 ? v : 0.0);
            c->beta[q] = beta;
            c->oldb[q] = 0.0;
            c->dbar[q] = 0.0;
            c->epsln[q] = 0.0;
            c->phibar[q] = beta;
            c->cs[q] = -1.0;
            c->sn[q] = 0.0;
            c->upd[q] = 0;
            c->active[q] = beta > c->tol[q];
        }
        c->nan = bad;
        if (bad)
            c->active[0] = c->active[1] = 0;
    }
}

// v = y / beta for active species (0 otherwise)
__global__ void __launch_bounds__(kBlock) k_mr_v(int len, const double2 *__restrict__ y, double2 *v,
                                                 const MrCtl *__restrict__ c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    c += blockIdx.y;
    const double2 a = run_at(y, len)[i];
    run_at(v, len)[i] = make_double2(c->active[0] ? a.x / c->beta[0] : 0.0,
                                     c->active[1] ? a.y / c->beta[1] : 0.0);
}

// y -= (beta / oldb) r1 (from the second step on), then partials of v . y
__global__ void __launch_bounds__(kBlock) k_mr_y1(int len, double2 *y, const double2 *__restrict__ r1,
                                                  const double2 *__restrict__ v,
                                                  const MrCtl *__restrict__ c, int second,
                                                  double2 *part)
{
    __shared__ double2 sh[kBlock / 64];
    c += blockIdx.y;
    y = run_at(y, len);
    r1 = run_at(r1, len);
    v = run_at(v, len);
    part = run_at(part, kSlotStride);
    const double f0 = (second && c->active[0]) ? c->beta[0] / c->oldb[0] : 0.0;
    const double f1 = (second && c->active[1]) ? c->beta[1] / c->oldb[1] : 0.0;
    double2 acc = d2(0.0, 0.0);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < len; i += gridDim.x * kBlock) {
        double2 a = y[i];
        if (second) {
            const double2 r = r1[i];
            a.x -= f0 * r.x;
            a.y -= f1 * r.y;
            y[i] = a;
        }
        const double2 vv = v[i];
        acc.x += vv.x * a.x;
        acc.y += vv.y * a.y;
    }
    const double2 s = block_sum(acc, sh);
    if (threadIdx.x == 0)
        part[blockIdx.x] = s;
}

// alfa = v . y from partials; y -= (alfa / beta) r2
__global__ void __launch_bounds__(kBlock) k_mr_y2(int len, double2 *y, const double2 *__restrict__ r2,
                                                  MrCtl *c, const double2 *__restrict__ part, int G)
{
    __shared__ double2 sh[1];
    c += blockIdx.y;
    const double2 al = sum_parts(run_at(part, kSlotStride), G, sh);
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->alfa[0] = al.x;
        c->alfa[1] = al.y;
    }
    if (i >= len)
        return;
    y = run_at(y, len);
    const double2 r = run_at(r2, len)[i];
    const double f0 = c->active[0] ? al.x / c->beta[0] : 0.0;
    const double f1 = c->active[1] ? al.y / c->beta[1] : 0.0;
    double2 a = y[i];
    a.x -= f0 * r.x;
    a.y -= f1 * r.y;
    y[i] = a;
}

// the rotation of this step from beta^2 = r2 . P^-1 r2 (partials), per species
__global__ void __launch_bounds__(kBlock) k_mr_rotate(MrCtl *c, const double2 *__restrict__ part, int G)
{
    __shared__ double2 sh[1];
    c += blockIdx.y;
    const double2 s = sum_parts(run_at(part, kSlotStride), G, sh);
    const int q = threadIdx.x;
    if (q >= 2)
        return;
    c->upd[q] = c->active[q];
    if (!c->active[q])
        return;
    const double b2 = q == 0 ? s.x : s.y;
    if (!(b2 >= 0.0)) {
        c->nan = 1;
        c->active[q] = 0;
        c->upd[q] = 0;
        return;
    }
    const double alfa = c->alfa[q];
    c->oldb[q] = c->beta[q];
    const double beta = sqrt(b2);
    c->beta[q] = beta;
    const double cs = c->cs[q], sn = c->sn[q], dbar = c->dbar[q];
    c->oldeps[q] = c->epsln[q];
    c->delta[q] = cs * dbar + sn * alfa;
    const double gbar = sn * dbar - cs * alfa;
    c->epsln[q] = sn * beta;
    c->dbar[q] = -cs * beta;
    double gamma = sqrt(gbar * gbar + beta * beta);
    if (gamma == 0.0)
        gamma = 1e-300;
    c->gamma[q] = gamma;
    const double ncs = gbar / gamma, nsn = beta / gamma;
    c->cs[q] = ncs;
    c->sn[q] = nsn;
    const double phibar = c->phibar[q];
    c->phi[q] = ncs * phibar;
    c->phibar[q] = nsn * phibar;
    if (!isfinite(c->phibar[q])) {
        c->nan = 1;
        c->active[q] = 0;
    } else if (!(c->phibar[q] > c->tol[q])) {
        c->active[q] = 0;
    }
}

// w_new = (v - oldeps w1 - delta w2) / gamma; w1 <- w2; w2 <- w_new; x += phi w_new
// (species that took part in the step)
__global__ void __launch_bounds__(kBlock) k_mr_w(int len, const double2 *__restrict__ v, double2 *w1,
                                                 double2 *w2, double2 *x, const MrCtl *__restrict__ c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    c += blockIdx.y;
    v = run_at(v, len);
    w1 = run_at(w1, len);
    w2 = run_at(w2, len);
    x = run_at(x, len);
    const double2 vv = v[i], a = w1[i], b = w2[i];
    double2 xv = x[i], na = a, nb = b;
    if (c->upd[0]) {
        const double wn = (vv.x - c->oldeps[0] * a.x - c->delta[0] * b.x) / c->gamma[0];
        na.x = b.x;
        nb.x = wn;
        xv.x += c->phi[0] * wn;
    }
    if (c->upd[1]) {
        const double wn = (vv.y - c->oldeps[1] * a.y - c->delta[1] * b.y) / c->gamma[1];
        na.y = b.y;
        nb.y = wn;
        xv.y += c->phi[1] * wn;
    }
    w1[i] = na;
    w2[i] = nb;
    x[i] = xv;
}

}  // namespace

// MINRES for every species of every run from S.xk with right-hand side
// S.b, given the residual S.r = b - A xk.  total: iterations per species (2
// per run, added to).  Returns CHM_OK, CHM_ENOCONV or CHM_ENAN (with
// S.nan_where); S.xk holds the iterate either way.
int minres_solve(Solver &S, std::vector<int> &total)
{
    const int n = S.nv, len = 2 * n, R = S.nrun;
    const size_t rl = (size_t)R * len;
    hipStream_t st = S.stream;
    const int Gv = red_blocks(len);
    double2 *r1 = S.mr, *r2 = S.mr + rl, *y = S.mr + 2 * rl, *v = S.mr + 3 * rl;
    double2 *w1 = S.mr + 4 * rl, *w2 = S.mr + 5 * rl;
    MrCtl *c = static_cast<MrCtl *>(S.mrctl);
    MrCtl *hc = static_cast<MrCtl *>(S.hmrctl);
    // tolerance from b . P^-1 b
    apply_prec(S, S.b, y);
    k_dot<double><<<grid(Gv, R), kBlock, 0, st>>>(len, S.b, y, slot(S, kSlotA));
    k_mr_tol<<<grid(1, R), kBlock, 0, st>>>(c, slot(S, kSlotA), Gv, S.prm.rtol);
    // r1 = r2 = b - A x, y = P^-1 r1, beta_1
    k_copy<double2><<<grid(nblk(len), R), kBlock, 0, st>>>(len, S.r, r1);
    k_copy<double2><<<grid(nblk(len), R), kBlock, 0, st>>>(len, S.r, r2);
    apply_prec(S, r1, y);
    k_dot<double><<<grid(Gv, R), kBlock, 0, st>>>(len, r1, y, slot(S, kSlotA));
    k_mr_start<<<grid(1, R), kBlock, 0, st>>>(c, slot(S, kSlotA), Gv);
    fill_double(reinterpret_cast<double *>(w1), 0.0, 2 * rl, st);
    fill_double(reinterpret_cast<double *>(w2), 0.0, 2 * rl, st);
    CHM_HIP(hipGetLastError());
    for (int k = 1;; ++k) {
        CHM_HIP(hipMemcpyAsync(hc, c, sizeof(MrCtl) * R, hipMemcpyDeviceToHost, st));
        CHM_HIP(hipStreamSynchronize(st));
        bool any = false, over = false;
        for (int r = 0; r < R; ++r) {
            if (hc[r].nan) {
                S.nan_where = "MINRES step " + std::to_string(k - 1) + ", run " + std::to_string(r) +
                              ": iterations " + std::to_string(total[2 * r]) + ", " +
                              std::to_string(total[2 * r + 1]);
                return CHM_ENAN;
            }
            for (int q = 0; q < 2; ++q) {
                if (k > 1 && hc[r].upd[q])
                    total[2 * r + q] += 1;
                any = any || hc[r].active[q];
                over = over || (hc[r].active[q] && total[2 * r + q] >= S.prm.max_iters);
            }
        }
        if (!any)
            return CHM_OK;
        if (over)
            return CHM_ENOCONV;
        k_mr_v<<<grid(nblk(len), R), kBlock, 0, st>>>(len, y, v, c);
        apply_saddle(S, v, y);
        k_mr_y1<<<grid(Gv, R), kBlock, 0, st>>>(len, y, r1, v, c, k >= 2, slot(S, kSlotA));
        k_mr_y2<<<grid(nblk(len), R), kBlock, 0, st>>>(len, y, r2, c, slot(S, kSlotA), Gv);
        // r1 <- r2, r2 <- y; y takes the old r1's storage for P^-1 r2
        std::swap(r1, r2);
        std::swap(r2, y);
        apply_prec(S, r2, y);
        k_dot<double><<<grid(Gv, R), kBlock, 0, st>>>(len, r2, y, slot(S, kSlotA));
        k_mr_rotate<<<grid(1, R), 64, 0, st>>>(c, slot(S, kSlotA), Gv);
        k_mr_w<<<grid(nblk(len), R), kBlock, 0, st>>>(len, v, w1, w2, S.xk, c);
        CHM_HIP(hipGetLastError());
    }
}

void minres_alloc(Solver &S)
{
    Pool &p = S.pool;
    const size_t len = 2 * (size_t)S.nv;
    S.mr = p.get<double2>(6 * (size_t)S.nb * len);
    S.mrctl = p.get<MrCtl>(S.nb);
    fill_int(reinterpret_cast<int *>(S.mrctl), 0, S.nb * sizeof(MrCtl) / sizeof(int), S.stream);
    CHM_HIP(hipHostMalloc(&S.hmrctl, S.nb * sizeof(MrCtl), hipHostMallocDefault));
}

}  // namespace chm
