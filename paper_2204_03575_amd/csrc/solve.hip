// Per-time-step solve on the GPU: right-hand side, Algorithm 1 of the paper
// (mass block by one AMG V-cycle; Schur block by the matching approximation
// As M^-1 As with As = tau' K + sqrt(tau'/eps) M, each As solve done with CG
// steps preconditioned by one V-cycle), the saddle-point operator of
// eq. saddle_point_system, and right-preconditioned flexible GMRES with
// classical Gram-Schmidt applied twice and Givens rotations kept on the
// device.  Both species run through every kernel together (pair vectors),
// each with its own scalars, convergence flag and iteration count.
//
// All reductions are deterministic: a fixed grid writes one partial per block,
// and the last block to finish (ticket counter) adds the partials in block
// order.
#include <chrono>
#include <cmath>

#include "chm_internal.h"

namespace chm {

namespace {

inline int nblk(long n, int bs = kBlock) { return (int)std::max<long>(1, (n + bs - 1) / bs); }
inline int red_blocks(long n) { return (int)std::min<long>(kRedBlocks, nblk(n)); }

__device__ inline double2 d2(double a, double b) { return make_double2(a, b); }

// ------------------------------------------------------------------ reductions
__device__ inline double2 wave_sum(double2 v)
{
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_down(v.x, off, 64);
        v.y += __shfl_down(v.y, off, 64);
    }
    return v;
}

// sum over a 256-thread block; the result is valid in thread 0
__device__ inline double2 block_sum(double2 v, double2 *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        sh[wid] = v;
    __syncthreads();
    double2 r = d2(0.0, 0.0);
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) {
            r.x += sh[w].x;
            r.y += sh[w].y;
        }
    __syncthreads();
    return r;
}

__device__ inline void store_partial(double2 *p, double2 v)
{
    __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double2 load_partial(const double2 *p)
{
    double2 v;
    v.x = __hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v.y = __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return v;
}

// true in every thread of the block that finishes last
__device__ inline bool last_block(unsigned *ticket)
{
    __shared__ int am_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = atomicAdd(ticket, 1u);
        am_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (am_last)
        __threadfence();
    return am_last != 0;
}

// the last block adds partials[v * G + g] over g in order into out[v]
__device__ inline void finish_partials(const double2 *partials, int nvec, double2 *out,
                                       unsigned *ticket)
{
    const int G = gridDim.x;
    for (int v = threadIdx.x; v < nvec; v += blockDim.x) {
        double2 s = d2(0.0, 0.0);
        for (int g = 0; g < G; ++g) {
            double2 p = load_partial(partials + (size_t)v * G + g);
            s.x += p.x;
            s.y += p.y;
        }
        out[v] = s;
    }
    if (threadIdx.x == 0)
        *ticket = 0u;
}

// ------------------------------------------------------------------ SELL SpMV family (pairs)
enum SpmvMode { SP_SET = 0, SP_ADD = 1, SP_RESID = 2 };

// SP_SET: y = A x; SP_ADD: y += A x; SP_RESID: y = b - A x
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_spmv(int n, const int *__restrict__ sptr,
                                                 const int *__restrict__ col,
                                                 const double *__restrict__ val,
                                                 const double2 *__restrict__ x,
                                                 const double2 *__restrict__ b, double2 *y)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= n)
        return;
    const int s = row / kSlice, lane = row % kSlice;
    const int base = sptr[s], width = (sptr[s + 1] - base) / kSlice;
    double ax = 0.0, ay = 0.0;
    for (int k = 0; k < width; ++k) {
        const int idx = base + k * kSlice + lane;
        const double a = val[idx];
        const double2 xv = x[col[idx]];
        ax += a * xv.x;
        ay += a * xv.y;
    }
    if (MODE == SP_SET) {
        y[row] = d2(ax, ay);
    } else if (MODE == SP_ADD) {
        double2 o = y[row];
        y[row] = d2(o.x + ax, o.y + ay);
    } else {
        double2 bb = b[row];
        y[row] = d2(bb.x - ax, bb.y - ay);
    }
}

// One smoothing step: r = b - A x_in; d = c1 d + c2 D^-1 r; x_out = x_in + d.
__global__ void __launch_bounds__(kBlock) k_cheb(int n, const int *__restrict__ sptr,
                                                 const int *__restrict__ col,
                                                 const double *__restrict__ val,
                                                 const double *__restrict__ dinv,
                                                 const double2 *__restrict__ b,
                                                 const double2 *__restrict__ xin,
                                                 double2 *__restrict__ xout, double2 *d, double c1,
                                                 double c2)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= n)
        return;
    const int s = row / kSlice, lane = row % kSlice;
    const int base = sptr[s], width = (sptr[s + 1] - base) / kSlice;
    double ax = 0.0, ay = 0.0;
    for (int k = 0; k < width; ++k) {
        const int idx = base + k * kSlice + lane;
        const double a = val[idx];
        const double2 xv = xin[col[idx]];
        ax += a * xv.x;
        ay += a * xv.y;
    }
    const double2 bb = b[row], xi = xin[row];
    const double di = dinv[row];
    double2 dd = d2(0.0, 0.0);
    if (c1 != 0.0)
        dd = d[row];
    dd.x = c1 * dd.x + c2 * (di * (bb.x - ax));
    dd.y = c1 * dd.y + c2 * (di * (bb.y - ay));
    d[row] = dd;
    xout[row] = d2(xi.x + dd.x, xi.y + dd.y);
}

// first smoothing step from x = 0: d = c2 D^-1 b; x = d
__global__ void __launch_bounds__(kBlock) k_cheb0(int n, const double *__restrict__ dinv,
                                                  const double2 *__restrict__ b, double2 *x,
                                                  double2 *d, double c2)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= n)
        return;
    const double2 bb = b[row];
    const double di = dinv[row];
    const double2 dd = d2(c2 * (di * bb.x), c2 * (di * bb.y));
    d[row] = dd;
    x[row] = dd;
}

// coarsest level: x = A^-1 b with the inverse stored column-major
__global__ void __launch_bounds__(kBlock) k_dense(int n, const double *__restrict__ inv,
                                                  const double2 *__restrict__ b, double2 *x)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= n)
        return;
    double ax = 0.0, ay = 0.0;
    for (int j = 0; j < n; ++j) {
        const double a = inv[(size_t)j * n + row];
        const double2 bv = b[j];
        ax += a * bv.x;
        ay += a * bv.y;
    }
    x[row] = d2(ax, ay);
}

__global__ void __launch_bounds__(kBlock) k_axpy_add(int n, const double2 *__restrict__ e, double2 *x)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= n)
        return;
    double2 a = x[row], b = e[row];
    x[row] = d2(a.x + b.x, a.y + b.y);
}

__global__ void __launch_bounds__(kBlock) k_copy(int n, const double2 *__restrict__ a, double2 *b)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row < n)
        b[row] = a[row];
}

// ------------------------------------------------------------------ dots (pairs, per species)
__global__ void __launch_bounds__(kBlock) k_dot(int n, const double2 *__restrict__ a,
                                                const double2 *__restrict__ b, double2 *partials,
                                                double2 *out, unsigned *ticket)
{
    __shared__ double2 sh[kBlock / 64];
    double2 acc = d2(0.0, 0.0);
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double2 x = a[i], y = b[i];
        acc.x += x.x * y.x;
        acc.y += x.y * y.y;
    }
    double2 s = block_sum(acc, sh);
    if (threadIdx.x == 0)
        store_partial(partials + blockIdx.x, s);
    if (last_block(ticket))
        finish_partials(partials, 1, out, ticket);
}

// ------------------------------------------------------------------ inner CG for As
// step length from slots: alpha = rz / dq per species (0 where dq == 0)
__device__ inline double2 ratio_or_zero(double2 num, double2 den)
{
    return d2(den.x != 0.0 ? num.x / den.x : 0.0, den.y != 0.0 ? num.y / den.y : 0.0);
}

// first == 1: x = alpha d, r = b - alpha q (x = 0 and r = b before the step)
__global__ void __launch_bounds__(kBlock) k_pcg_xr(int n, double2 *x, double2 *r,
                                                   const double2 *__restrict__ b,
                                                   const double2 *__restrict__ d,
                                                   const double2 *__restrict__ q,
                                                   const double2 *__restrict__ rz,
                                                   const double2 *__restrict__ dq, int first)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const double2 al = ratio_or_zero(*rz, *dq);
    const double2 dv = d[i], qv = q[i];
    double2 xv = first ? d2(0.0, 0.0) : x[i];
    double2 rv = first ? b[i] : r[i];
    xv.x += al.x * dv.x;
    xv.y += al.y * dv.y;
    rv.x -= al.x * qv.x;
    rv.y -= al.y * qv.y;
    x[i] = xv;
    r[i] = rv;
}

// d = z + beta d with beta = rz_new / rz_old (0 where rz_old == 0); first: d = z
__global__ void __launch_bounds__(kBlock) k_pcg_dir(int n, const double2 *__restrict__ z, double2 *d,
                                                    const double2 *__restrict__ rz_new,
                                                    const double2 *__restrict__ rz_old, int first)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const double2 zv = z[i];
    if (first) {
        d[i] = zv;
        return;
    }
    const double2 be = ratio_or_zero(*rz_new, *rz_old);
    const double2 dv = d[i];
    d[i] = d2(zv.x + be.x * dv.x, zv.y + be.y * dv.y);
}

// ------------------------------------------------------------------ saddle-point operator
// y0 = M x0 + t K x1; y1 = t K x0 - te M x1 (per species t, te);  RESID: y = b - A x,
// and the squared 2-norm of y per species goes to *out.
template <bool RESID>
__global__ void __launch_bounds__(kBlock) k_saddle(int n, const int *__restrict__ sptr,
                                                   const int *__restrict__ col,
                                                   const double *__restrict__ vm,
                                                   const double *__restrict__ vk,
                                                   const double2 *__restrict__ x,
                                                   const double2 *__restrict__ b, double2 *y,
                                                   double2 t, double2 te, double2 *partials,
                                                   double2 *out, unsigned *ticket)
{
    __shared__ double2 sh[kBlock / 64];
    const int row = blockIdx.x * kBlock + threadIdx.x;
    double2 nrm = d2(0.0, 0.0);
    if (row < n) {
        const int s = row / kSlice, lane = row % kSlice;
        const int base = sptr[s], width = (sptr[s + 1] - base) / kSlice;
        double m0x = 0, m0y = 0, k1x = 0, k1y = 0, k0x = 0, k0y = 0, m1x = 0, m1y = 0;
        for (int k = 0; k < width; ++k) {
            const int idx = base + k * kSlice + lane;
            const int c = col[idx];
            const double am = vm[idx], ak = vk[idx];
            const double2 x0 = x[c], x1 = x[n + c];
            m0x += am * x0.x;
            m0y += am * x0.y;
            k1x += ak * x1.x;
            k1y += ak * x1.y;
            k0x += ak * x0.x;
            k0y += ak * x0.y;
            m1x += am * x1.x;
            m1y += am * x1.y;
        }
        double2 y0 = d2(m0x + t.x * k1x, m0y + t.y * k1y);
        double2 y1 = d2(t.x * k0x - te.x * m1x, t.y * k0y - te.y * m1y);
        if (RESID) {
            const double2 b0 = b[row], b1 = b[n + row];
            y0 = d2(b0.x - y0.x, b0.y - y0.y);
            y1 = d2(b1.x - y1.x, b1.y - y1.y);
            nrm = d2(y0.x * y0.x + y1.x * y1.x, y0.y * y0.y + y1.y * y1.y);
        }
        y[row] = y0;
        y[n + row] = y1;
    }
    if (RESID) {
        double2 s = block_sum(nrm, sh);
        if (threadIdx.x == 0)
            store_partial(partials + blockIdx.x, s);
        if (last_block(ticket))
            finish_partials(partials, 1, out, ticket);
    }
}

// ------------------------------------------------------------------ Gram-Schmidt passes
// MODE 0: out[i] = V_i . w;  MODE 1: w -= sum_i V_i h[i], then out[i] = V_i . w;
// MODE 2: w -= sum_i V_i h[i], then out[0] = w . w.  All per species; len = 2n.
constexpr int kChunk = 8;

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_gs(int len, const double2 *__restrict__ V, int nvec,
                                               double2 *w, const double2 *__restrict__ h,
                                               double2 *partials, double2 *out, unsigned *ticket)
{
    __shared__ double2 sh[kBlock / 64];
    const int G = gridDim.x;
    const int start = blockIdx.x * kBlock + threadIdx.x, stride = G * kBlock;
    if (MODE > 0) {
        for (int i = start; i < len; i += stride) {
            double2 wv = w[i];
            for (int v = 0; v < nvec; ++v) {
                const double2 hv = h[v], vv = V[(size_t)v * len + i];
                wv.x -= hv.x * vv.x;
                wv.y -= hv.y * vv.y;
            }
            w[i] = wv;
        }
    }
    if (MODE == 2) {
        double2 acc = d2(0.0, 0.0);
        for (int i = start; i < len; i += stride) {
            const double2 wv = w[i];
            acc.x += wv.x * wv.x;
            acc.y += wv.y * wv.y;
        }
        double2 s = block_sum(acc, sh);
        if (threadIdx.x == 0)
            store_partial(partials + blockIdx.x, s);
        if (last_block(ticket))
            finish_partials(partials, 1, out, ticket);
        return;
    }
    for (int v0 = 0; v0 < nvec; v0 += kChunk) {
        double2 acc[kChunk];
        for (int c = 0; c < kChunk; ++c)
            acc[c] = d2(0.0, 0.0);
        for (int i = start; i < len; i += stride) {
            const double2 wv = w[i];
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                if (v0 + c < nvec) {
                    const double2 vv = V[(size_t)(v0 + c) * len + i];
                    acc[c].x += vv.x * wv.x;
                    acc[c].y += vv.y * wv.y;
                }
            }
        }
        for (int c = 0; c < kChunk && v0 + c < nvec; ++c) {
            double2 s = block_sum(acc[c], sh);
            if (threadIdx.x == 0)
                store_partial(partials + (size_t)(v0 + c) * G + blockIdx.x, s);
        }
    }
    if (last_block(ticket))
        finish_partials(partials, nvec, out, ticket);
}

// ------------------------------------------------------------------ FGMRES control (one block)
// start of a cycle: g = (||r||, 0, ...), active flags from the host, k = 0
__global__ void k_cycle_init(Ctl *c, int act0, int act1)
{
    const int s = threadIdx.x;
    if (s >= 2)
        return;
    c->active[s] = s == 0 ? act0 : act1;
    c->k[s] = 0;
    c->g[s][0] = sqrt(c->nrm[s]);
}

// keep only the species the host still lets iterate
__global__ void k_deactivate(Ctl *c, int act0, int act1)
{
    const int s = threadIdx.x;
    if (s < 2)
        c->active[s] = c->active[s] && (s == 0 ? act0 : act1);
}

// v0 = r / ||r|| for active species, 0 otherwise
__global__ void __launch_bounds__(kBlock) k_scale_first(int len, const double2 *__restrict__ r,
                                                        double2 *v, const Ctl *__restrict__ c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    const double s0 = (c->active[0] && c->nrm[0] > 0.0) ? 1.0 / sqrt(c->nrm[0]) : 0.0;
    const double s1 = (c->active[1] && c->nrm[1] > 0.0) ? 1.0 / sqrt(c->nrm[1]) : 0.0;
    const double2 rv = r[i];
    v[i] = d2(rv.x * s0, rv.y * s1);
}

// Column j of the Hessenberg matrix from the two Gram-Schmidt passes, the
// previous rotations applied, a new rotation that zeroes H[j+1][j], the
// residual estimate |g[j+1]|, and the convergence test against tol.
__global__ void k_givens(Ctl *c, int j, int m, const double2 *__restrict__ h1,
                         const double2 *__restrict__ h2, const double2 *__restrict__ nrm2)
{
    const int s = threadIdx.x;
    if (s >= 2 || !c->active[s])
        return;
    double *H = c->H[s];
    for (int i = 0; i <= j; ++i)
        H[i * m + j] = (s == 0 ? h1[i].x + h2[i].x : h1[i].y + h2[i].y);
    const double hn = sqrt(s == 0 ? nrm2->x : nrm2->y);
    c->hn[s] = hn;
    H[(j + 1) * m + j] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = H[i * m + j], b = H[(i + 1) * m + j];
        H[i * m + j] = c->cs[s][i] * a + c->sn[s][i] * b;
        H[(i + 1) * m + j] = -c->sn[s][i] * a + c->cs[s][i] * b;
    }
    const double a = H[j * m + j], b = H[(j + 1) * m + j];
    const double rr = sqrt(a * a + b * b);
    double cs = 1.0, sn = 0.0;
    if (rr != 0.0) {
        cs = a / rr;
        sn = b / rr;
    }
    c->cs[s][j] = cs;
    c->sn[s][j] = sn;
    H[j * m + j] = rr;
    H[(j + 1) * m + j] = 0.0;
    const double gj = c->g[s][j];
    c->g[s][j + 1] = -sn * gj;
    c->g[s][j] = cs * gj;
    c->k[s] = j + 1;
    const double est = fabs(c->g[s][j + 1]);
    c->resest[s] = est;
    if (!isfinite(est) || !isfinite(hn)) {
        c->nan = 1;
        c->active[s] = 0;
    } else if (est <= c->tol[s] || hn == 0.0) {
        c->active[s] = 0;
    }
}

// v_{j+1} = w / ||w|| for species still active, 0 otherwise
__global__ void __launch_bounds__(kBlock) k_scale_next(int len, double2 *v, const Ctl *__restrict__ c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    const double s0 = (c->active[0] && c->hn[0] > 0.0) ? 1.0 / c->hn[0] : 0.0;
    const double s1 = (c->active[1] && c->hn[1] > 0.0) ? 1.0 / c->hn[1] : 0.0;
    const double2 vv = v[i];
    v[i] = d2(vv.x * s0, vv.y * s1);
}

// back substitution of the rotated Hessenberg system, k[s] columns per species
__global__ void k_trisolve(Ctl *c, int m)
{
    const int s = threadIdx.x;
    if (s >= 2)
        return;
    const int k = c->k[s];
    const double *H = c->H[s];
    for (int i = k - 1; i >= 0; --i) {
        double v = c->g[s][i];
        for (int t = i + 1; t < k; ++t)
            v -= H[i * m + t] * c->y[s][t];
        c->y[s][i] = v / H[i * m + i];
    }
    for (int i = k; i < kMaxRestart; ++i)
        c->y[s][i] = 0.0;
}

// x += sum_{i < kmax} Z_i y_i, per species
__global__ void __launch_bounds__(kBlock) k_update_x(int len, double2 *x, const double2 *__restrict__ Z,
                                                     int kmax, const Ctl *__restrict__ c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    double2 xv = x[i];
    for (int t = 0; t < kmax; ++t) {
        const double2 z = Z[(size_t)t * len + i];
        xv.x += c->y[0][t] * z.x;
        xv.y += c->y[1][t] * z.y;
    }
    x[i] = xv;
}

__global__ void k_tol(Ctl *c, double rtol)
{
    const int s = threadIdx.x;
    if (s >= 2)
        return;
    const double bn = sqrt(c->nrm[s]);
    c->bnorm[s] = bn;
    c->tol[s] = rtol * bn;
}

__global__ void __launch_bounds__(kBlock) k_finite(int len, const double2 *__restrict__ x, Ctl *c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    const double2 v = x[i];
    if (!isfinite(v.x) || !isfinite(v.y))
        c->nan = 1;
}

// ------------------------------------------------------------------ right-hand side
struct Pot {
    int kind;
    double Np, Nn, Ns, chi_pn, chi_ps, chi_ns, floor_;
};

__device__ inline double clog(double v, double fl, int &clamps)
{
    if (v < fl) {
        ++clamps;
        v = fl;
    }
    return log(v);
}

// d f / d phi_p and d f / d phi_n with phi_s = 1 - phi_p - phi_n (paper Section 2,
// eq. logarithmicpotential; Section 4, eq. polynomial_potential)
__device__ inline void dpot(const Pot &P, double p, double q, double &fp, double &fq, int &clamps)
{
    const double s = 1.0 - p - q;
    if (P.kind == CHM_POT_FLORY_HUGGINS) {
        const double lp = clog(p, P.floor_, clamps), lq = clog(q, P.floor_, clamps);
        const double ls = clog(s, P.floor_, clamps);
        const double es = (ls + 1.0) / P.Ns;
        fp = (lp + 1.0) / P.Np - es + P.chi_pn * q + P.chi_ps * (s - p) - P.chi_ns * q;
        fq = (lq + 1.0) / P.Nn - es + P.chi_pn * p - P.chi_ps * p + P.chi_ns * (s - q);
    } else if (P.kind == CHM_POT_POLYNOMIAL) {
        fp = 7.0 * p * q * q - 0.2 * s;
        fq = 7.0 * p * p * q - 0.2 * s;
    } else {
        fp = 0.0;
        fq = 0.0;
    }
}

// f[v] += sum over the quadrature of f'(phi_h) lambda_v |T| for the cells of
// one colour (no two share a vertex, so the += are race free)
__global__ void __launch_bounds__(kBlock) k_rhs_color(const int *__restrict__ list, int count,
                                                      const int *__restrict__ cells, int nl,
                                                      const double *__restrict__ vol,
                                                      const double *__restrict__ qb,
                                                      const double *__restrict__ qw, int nq,
                                                      const double2 *__restrict__ phi, Pot P,
                                                      double2 *f, int *clamped)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= count)
        return;
    const int c = list[t];
    int vtx[4];
    double2 ph[4], acc[4];
    for (int a = 0; a < nl; ++a) {
        vtx[a] = cells[(size_t)c * nl + a];
        ph[a] = phi[vtx[a]];
        acc[a] = d2(0.0, 0.0);
    }
    int clamps = 0;
    for (int q = 0; q < nq; ++q) {
        double p = 0.0, r = 0.0;
        for (int a = 0; a < nl; ++a) {
            const double l = qb[q * nl + a];
            p += l * ph[a].x;
            r += l * ph[a].y;
        }
        double fp, fr;
        dpot(P, p, r, fp, fr, clamps);
        const double wq = qw[q];
        for (int a = 0; a < nl; ++a) {
            const double l = qb[q * nl + a];
            acc[a].x += wq * fp * l;
            acc[a].y += wq * fr * l;
        }
    }
    const double vc = vol[c];
    for (int a = 0; a < nl; ++a) {
        double2 o = f[vtx[a]];
        f[vtx[a]] = d2(o.x + vc * acc[a].x, o.y + vc * acc[a].y);
    }
    if (clamps)
        atomicAdd(clamped, clamps);
}

// b1 = -(tau'/eps) f
__global__ void __launch_bounds__(kBlock) k_rhs_second(int n, const double2 *__restrict__ f,
                                                       double2 *b1, double2 te)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const double2 v = f[i];
    b1[i] = d2(-te.x * v.x, -te.y * v.y);
}

__global__ void __launch_bounds__(kBlock) k_zero(int n, double2 *v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        v[i] = d2(0.0, 0.0);
}

// solvent removal after a step: phi_i += ds phi_i / (phi_p + phi_n), equal halves if the sum is <= 0
__global__ void __launch_bounds__(kBlock) k_evaporate(int n, double2 *phi, double ds)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    double2 v = phi[i];
    const double sum = v.x + v.y;
    if (sum > 0.0) {
        const double gp = ds * v.x / sum, gn = ds * v.y / sum;
        v.x += gp;
        v.y += gn;
    } else {
        v.x += 0.5 * ds;
        v.y += 0.5 * ds;
    }
    phi[i] = v;
}

// ------------------------------------------------------------------ host helpers
void timer_mark(Solver &S, bool begin)
{
    Timer &T = S.timer;
    if (T.used >= T.ev.size() && T.used >= 8192 && begin) {   // fold finished pairs
        CHM_HIP(hipStreamSynchronize(S.stream));
        for (size_t i = 0; i + 1 < T.used; i += 2) {
            float ms = 0.f;
            CHM_HIP(hipEventElapsedTime(&ms, T.ev[i], T.ev[i + 1]));
            T.total_ms += ms;
        }
        T.used = 0;
    }
    if (T.used >= T.ev.size()) {   // grow the event pool
        size_t old = T.ev.size();
        T.ev.resize(old + 2048);
        for (size_t i = old; i < T.ev.size(); ++i)
            CHM_HIP(hipEventCreate(&T.ev[i]));
    }
    (void)begin;
    CHM_HIP(hipEventRecord(T.ev[T.used++], S.stream));
}

void launch_cheb(Solver &S, Hierarchy &H, int l, const double2 *b, const double2 *xin, double2 *xout,
                 double2 *d, double c1, double c2)
{
    Level &L = H.lev[l];
    const bool timed = S.timer.on && S.timer.kind == 0 && &H == &S.hA && l == 0;
    if (timed)
        timer_mark(S, true);
    k_cheb<<<nblk(L.n), kBlock, 0, S.stream>>>(L.n, L.sA.sptr, L.sA.col, L.sA.val, L.dinv, b, xin,
                                                xout, d, c1, c2);
    if (timed) {
        timer_mark(S, false);
        S.timer.count += 1;
        S.timer.bytes += 12ll * L.A.nnz + 88ll * L.n;
    }
}

void vcycle_level(Solver &S, Hierarchy &H, int l, const double2 *b, double2 *x)
{
    Level &L = H.lev[l];
    hipStream_t st = S.stream;
    if (l == H.nlev - 1) {
        k_dense<<<nblk(L.n), kBlock, 0, st>>>(L.n, L.inv, b, x);
        return;
    }
    const int deg = H.degree;
    double2 *xt = H.xt[l], *d = H.d[l], *r = H.r[l];
    auto c1 = [&](int k) { return (H.jacobi || k == 1) ? 0.0 : L.cheb_c1[k]; };
    auto c2 = [&](int k) { return H.jacobi ? L.jac_omega : L.cheb_c2[k]; };
    // pre-smoothing from zero; 2 deg - 1 ping-pong steps follow, so starting in
    // xt leaves the result in x
    k_cheb0<<<nblk(L.n), kBlock, 0, st>>>(L.n, L.dinv, b, xt, d, c2(1));
    double2 *cur = xt, *oth = x;
    for (int k = 2; k <= deg; ++k) {
        launch_cheb(S, H, l, b, cur, oth, d, c1(k), c2(k));
        std::swap(cur, oth);
    }
    k_spmv<SP_RESID><<<nblk(L.n), kBlock, 0, st>>>(L.n, L.sA.sptr, L.sA.col, L.sA.val, cur, b, r);
    k_spmv<SP_SET><<<nblk(L.nc), kBlock, 0, st>>>(L.nc, L.sR.sptr, L.sR.col, L.sR.val, r, nullptr,
                                                  H.b[l + 1]);
    vcycle_level(S, H, l + 1, H.b[l + 1], H.x[l + 1]);
    k_spmv<SP_ADD><<<nblk(L.n), kBlock, 0, st>>>(L.n, L.sP.sptr, L.sP.col, L.sP.val, H.x[l + 1],
                                                 nullptr, cur);
    for (int k = 1; k <= deg; ++k) {
        launch_cheb(S, H, l, b, cur, oth, d, c1(k), c2(k));
        std::swap(cur, oth);
    }
}

inline double2 pair(const double *a) { return make_double2(a[0], a[1]); }

}  // namespace

void vcycle(Solver &S, Hierarchy &H, const double2 *b, double2 *x)
{
    vcycle_level(S, H, 0, b, x);
}

// stationary AMG solve of the mass matrix: x = V(b), then x += V(b - M x)
void mass_solve(Solver &S, const double2 *b, double2 *x)
{
    Hierarchy &H = S.hM;
    const int n = S.nv;
    vcycle(S, H, b, x);
    for (int c = 1; c < S.prm.amg_cycles; ++c) {
        k_spmv<SP_RESID><<<nblk(n), kBlock, 0, S.stream>>>(n, H.lev[0].sA.sptr, H.lev[0].sA.col,
                                                           H.lev[0].sA.val, x, b, S.mr);
        vcycle(S, H, S.mr, S.me);
        k_axpy_add<<<nblk(n), kBlock, 0, S.stream>>>(n, S.me, x);
    }
}

// As solve of Algorithm 1: schur_pcg CG steps preconditioned by one V-cycle
// (or amg_cycles stationary V-cycles when schur_pcg = 0)
void schur_solve(Solver &S, const double2 *b, double2 *x)
{
    Hierarchy &H = S.hA;
    const int n = S.nv, k = S.prm.schur_pcg;
    hipStream_t st = S.stream;
    const Sell &A = H.lev[0].sA;
    if (k <= 0) {
        vcycle(S, H, b, x);
        for (int c = 1; c < S.prm.amg_cycles; ++c) {
            k_spmv<SP_RESID><<<nblk(n), kBlock, 0, st>>>(n, A.sptr, A.col, A.val, x, b, S.mr);
            vcycle(S, H, S.mr, S.me);
            k_axpy_add<<<nblk(n), kBlock, 0, st>>>(n, S.me, x);
        }
        return;
    }
    double2 *r = S.pcg_r, *z = S.pcg_z, *d = S.pcg_d, *q = S.pcg_q;
    double2 *rz = S.pcg_s, *dq = S.pcg_s + 40;
    const int G = red_blocks(n);
    vcycle(S, H, b, z);                                            // z = V(b), r = b
    k_dot<<<G, kBlock, 0, st>>>(n, b, z, S.red, rz + 0, S.ticket);
    k_pcg_dir<<<nblk(n), kBlock, 0, st>>>(n, z, d, rz, rz, 1);      // d = z
    for (int it = 1; it <= k; ++it) {
        k_spmv<SP_SET><<<nblk(n), kBlock, 0, st>>>(n, A.sptr, A.col, A.val, d, nullptr, q);
        k_dot<<<G, kBlock, 0, st>>>(n, d, q, S.red, dq + it, S.ticket);
        k_pcg_xr<<<nblk(n), kBlock, 0, st>>>(n, x, r, b, d, q, rz + it - 1, dq + it, it == 1);
        if (it == k)
            break;
        vcycle(S, H, r, z);
        k_dot<<<G, kBlock, 0, st>>>(n, r, z, S.red, rz + it, S.ticket);
        k_pcg_dir<<<nblk(n), kBlock, 0, st>>>(n, z, d, rz + it, rz + it - 1, 0);
    }
}

// Algorithm 1 on a block vector: w1 = AMG(M) v1; w2 = As^-1 M As^-1 v2
void apply_prec(Solver &S, const double2 *v, double2 *w)
{
    const int n = S.nv;
    mass_solve(S, v, w);
    schur_solve(S, v + n, S.tmp);
    k_spmv<SP_SET><<<nblk(n), kBlock, 0, S.stream>>>(n, S.sM.sptr, S.sM.col, S.sM.val, S.tmp,
                                                      nullptr, S.tmp2);
    schur_solve(S, S.tmp2, w + n);
}

void apply_saddle(Solver &S, const double2 *x, double2 *y)
{
    const int n = S.nv;
    k_saddle<false><<<nblk(n), kBlock, 0, S.stream>>>(n, S.sM.sptr, S.sM.col, S.sM.val, S.sK, x,
                                                       nullptr, y, pair(S.tau_s), pair(S.te_s),
                                                       nullptr, nullptr, nullptr);
}

// b = (M phi, -(tau'/eps) f) for the current state
void compute_rhs(Solver &S)
{
    const int n = S.nv;
    hipStream_t st = S.stream;
    Pot P{S.prm.potential, S.prm.Np, S.prm.Nn, S.prm.Ns,
          S.prm.chi_pn,    S.prm.chi_ps, S.prm.chi_ns, S.prm.log_floor};
    k_zero<<<nblk(n), kBlock, 0, st>>>(n, S.f);
    fill_int(&S.ctl->clamped, 0, 1, st);
    for (int c = 0; c < S.ncolors; ++c) {
        const int cnt = S.color_ptr[c + 1] - S.color_ptr[c];
        if (!cnt)
            continue;
        k_rhs_color<<<nblk(cnt), kBlock, 0, st>>>(S.color_cells + S.color_ptr[c], cnt, S.cells,
                                                  S.nl, S.vol, S.qb, S.qw, S.nq, S.x, P, S.f,
                                                  &S.ctl->clamped);
    }
    k_spmv<SP_SET><<<nblk(n), kBlock, 0, st>>>(n, S.sM.sptr, S.sM.col, S.sM.val, S.x, nullptr, S.b);
    k_rhs_second<<<nblk(n), kBlock, 0, st>>>(n, S.f, S.b + n, pair(S.te_s));
    CHM_HIP(hipGetLastError());
}

void alloc_workspace(Solver &S)
{
    Pool &p = S.pool;
    const int n = S.nv;
    const size_t len = 2 * (size_t)n;
    S.m = S.prm.restart;
    S.x = p.get<double2>(len);
    S.xk = p.get<double2>(len);
    S.b = p.get<double2>(len);
    S.r = p.get<double2>(len);
    S.V = p.get<double2>(len * (S.m + 1));
    S.Z = p.get<double2>(len * S.m);
    S.f = p.get<double2>(n);
    S.pcg_r = p.get<double2>(n);
    S.pcg_z = p.get<double2>(n);
    S.pcg_d = p.get<double2>(n);
    S.pcg_q = p.get<double2>(n);
    S.pcg_s = p.get<double2>(80);
    S.tmp = p.get<double2>(n);
    S.tmp2 = p.get<double2>(n);
    S.mr = p.get<double2>(n);
    S.me = p.get<double2>(n);
    S.hbuf1 = p.get<double2>(kMaxRestart + 1);
    S.hbuf2 = p.get<double2>(kMaxRestart + 1);
    S.nrm2 = p.get<double2>(1);
    S.red = p.get<double2>(std::max<size_t>((size_t)kRedBlocks * (kMaxRestart + 1), nblk(n)));
    S.ticket = p.get<unsigned>(1);
    fill_int(reinterpret_cast<int *>(S.ticket), 0, 1, S.stream);
    S.ctl = p.get<Ctl>(1);
    fill_int(reinterpret_cast<int *>(S.ctl), 0, sizeof(Ctl) / sizeof(int), S.stream);
    CHM_HIP(hipHostMalloc(reinterpret_cast<void **>(&S.hctl), sizeof(Ctl), hipHostMallocDefault));
    k_zero<<<nblk(len), kBlock, 0, S.stream>>>((int)len, S.x);
    CHM_HIP(hipStreamSynchronize(S.stream));
}

namespace {

void read_ctl(Solver &S)
{
    CHM_HIP(hipMemcpyAsync(S.hctl, S.ctl, kCtlHead, hipMemcpyDeviceToHost, S.stream));
    CHM_HIP(hipStreamSynchronize(S.stream));
}

}  // namespace

// One time step: right-hand side, FGMRES for both species, commit and solvent removal.
int step_once(Solver &S, chm_stats_t *st_out)
{
    const int n = S.nv, len = 2 * n, m = S.m;
    hipStream_t st = S.stream;
    const int Gv = red_blocks(len);
    auto t0 = std::chrono::steady_clock::now();
    chm_stats_t stats{};

    compute_rhs(S);
    k_dot<<<Gv, kBlock, 0, st>>>(len, S.b, S.b, S.red, reinterpret_cast<double2 *>(S.ctl->nrm),
                                 S.ticket);
    k_tol<<<1, 64, 0, st>>>(S.ctl, S.prm.rtol);
    k_copy<<<nblk(len), kBlock, 0, st>>>(len, S.x, S.xk);
    fill_int(&S.ctl->nan, 0, 1, st);

    int total[2] = {0, 0};
    int rc = CHM_OK;
    double res[2] = {0.0, 0.0}, bn[2] = {0.0, 0.0};
    for (;;) {
        k_saddle<true><<<nblk(n), kBlock, 0, st>>>(
            n, S.sM.sptr, S.sM.col, S.sM.val, S.sK, S.xk, S.b, S.r, pair(S.tau_s), pair(S.te_s),
            S.red, reinterpret_cast<double2 *>(S.ctl->nrm), S.ticket);
        CHM_HIP(hipGetLastError());
        read_ctl(S);
        const Ctl &h = *S.hctl;
        int act[2];
        bool finite = true;
        for (int s = 0; s < 2; ++s) {
            res[s] = std::sqrt(h.nrm[s]);
            bn[s] = h.bnorm[s];
            finite = finite && std::isfinite(res[s]);
            act[s] = !(res[s] <= h.tol[s]);
        }
        if (!finite) {
            rc = CHM_ENAN;
            S.nan_where = "residual check: |r| = (" + std::to_string(res[0]) + ", " +
                          std::to_string(res[1]) + "), |b| = (" + std::to_string(bn[0]) + ", " +
                          std::to_string(bn[1]) + "), iterations (" + std::to_string(total[0]) +
                          ", " + std::to_string(total[1]) + ")";
            break;
        }
        if (!act[0] && !act[1])
            break;
        if ((act[0] && total[0] >= S.prm.max_iters) || (act[1] && total[1] >= S.prm.max_iters)) {
            rc = CHM_ENOCONV;
            break;
        }
        k_cycle_init<<<1, 64, 0, st>>>(S.ctl, act[0], act[1]);
        k_scale_first<<<nblk(len), kBlock, 0, st>>>(len, S.r, S.V, S.ctl);
        int kmax = 0;
        for (int j = 0; j < m; ++j) {
            double2 *vj = S.V + (size_t)j * len, *zj = S.Z + (size_t)j * len;
            double2 *w = S.V + (size_t)(j + 1) * len;
            apply_prec(S, vj, zj);
            apply_saddle(S, zj, w);
            k_gs<0><<<Gv, kBlock, 0, st>>>(len, S.V, j + 1, w, nullptr, S.red, S.hbuf1, S.ticket);
            k_gs<1><<<Gv, kBlock, 0, st>>>(len, S.V, j + 1, w, S.hbuf1, S.red, S.hbuf2, S.ticket);
            k_gs<2><<<Gv, kBlock, 0, st>>>(len, S.V, j + 1, w, S.hbuf2, S.red, S.nrm2, S.ticket);
            k_givens<<<1, 64, 0, st>>>(S.ctl, j, m, S.hbuf1, S.hbuf2, S.nrm2);
            k_scale_next<<<nblk(len), kBlock, 0, st>>>(len, w, S.ctl);
            CHM_HIP(hipGetLastError());
            for (int s = 0; s < 2; ++s)
                total[s] += act[s];
            read_ctl(S);
            kmax = std::max(S.hctl->k[0], S.hctl->k[1]);
            bool any = false, capped = false;
            for (int s = 0; s < 2; ++s) {
                act[s] = S.hctl->active[s];
                if (act[s] && total[s] >= S.prm.max_iters) {
                    act[s] = 0;   // iteration budget spent: the cycle ends for this species
                    capped = true;
                }
                any = any || act[s];
            }
            if (capped)
                k_deactivate<<<1, 64, 0, st>>>(S.ctl, act[0], act[1]);
            if (S.hctl->nan) {
                rc = CHM_ENAN;
                S.nan_where = "Arnoldi step " + std::to_string(j) + ": estimates (" +
                              std::to_string(S.hctl->resest[0]) + ", " +
                              std::to_string(S.hctl->resest[1]) + "), |w| (" +
                              std::to_string(S.hctl->hn[0]) + ", " + std::to_string(S.hctl->hn[1]) +
                              "), iterations (" + std::to_string(total[0]) + ", " +
                              std::to_string(total[1]) + ")";
                break;
            }
            if (!any)
                break;
        }
        if (rc)
            break;
        k_trisolve<<<1, 64, 0, st>>>(S.ctl, m);
        k_update_x<<<nblk(len), kBlock, 0, st>>>(len, S.xk, S.Z, kmax, S.ctl);
        CHM_HIP(hipGetLastError());
    }
    if (rc == CHM_OK) {
        k_finite<<<nblk(len), kBlock, 0, st>>>(len, S.xk, S.ctl);
        read_ctl(S);
        if (S.hctl->nan) {
            rc = CHM_ENAN;
            S.nan_where = "final iterate";
        }
    }
    stats.clamped = S.hctl->clamped;
    if (rc == CHM_OK) {
        k_copy<<<nblk(len), kBlock, 0, st>>>(len, S.xk, S.x);
        if (S.prm.evap_ds > 0.0 && S.step_count < S.prm.evap_steps)
            k_evaporate<<<nblk(n), kBlock, 0, st>>>(n, S.x, S.prm.evap_ds);
        CHM_HIP(hipGetLastError());
        CHM_HIP(hipStreamSynchronize(st));
        S.step_count++;
    }
    for (int s = 0; s < 2; ++s) {
        stats.iters[s] = total[s];
        stats.relres[s] = bn[s] > 0.0 ? res[s] / bn[s] : res[s];
    }
    stats.status = rc;
    stats.t_step_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st_out)
        *st_out = stats;
    return rc;
}

}  // namespace chm
