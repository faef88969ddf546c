// The block preconditioner of Algorithm 1 on the GPU: the mass block by AMG
// V-cycles, the Schur block by the matching approximation As M^-1 As with
// As = tau' K + sqrt(tau'/eps) M, each As solve done with CG steps
// preconditioned by one V-cycle.  Both species run through every kernel
// together (pair vectors), each with its own CG scalars.
//
// Batches: every launch covers S.nrun runs (gridDim.y), all vectors of a
// level holding the runs back to back (run r of an n-row vector at r n).
//
// All of it is templated on the value type T.  T = double is the FP64 path.
// T = float is the mixed-precision preconditioner: FP32 matrix values, work
// vectors, smoothing, restriction, prolongation and the product with M inside
// Algorithm 1; the dot products of the inner CG are still accumulated in FP64,
// the coarsest level still applies its FP64 inverse with FP64 sums, and the
// vectors at the interface (the Krylov basis vector in, the preconditioned
// vector out) stay FP64.  The flexible Krylov method outside accepts a
// preconditioner that varies with its input, so rounding at FP32 changes
// iteration counts, not the converged residual.
#include "device_util.h"

namespace chm {

namespace {

// ------------------------------------------------------------------ smoothing
// Chebyshev (or damped Jacobi) step in two-buffer form:
//   x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 D^-1 (b - A x_k),
// the same polynomial as the update d_k = c1 d_{k-1} + c2 D^-1 r_k with
// d_{k-1} = x_k - x_{k-1}.  x_{k+1} overwrites x_{k-1} row by row; with
// prev = 0 the previous iterate is taken as zero (start from x = 0) or is not
// needed (c1 = 0).
// the row's operands of the update, loaded apart from the product so that a
// kernel can issue them before the gathers of A x_k
template <class T> struct ChebRow {
    pair_t<T> bb, xi, xp;
    T di;
};

template <class T>
__device__ inline ChebRow<T> cheb_row(const pair_t<T> *__restrict__ b, const pair_t<T> *__restrict__ xk,
                                      const T *__restrict__ dinv, const pair_t<T> *xprev, int row,
                                      int prev)
{
    ChebRow<T> o;
    o.bb = b[row];
    o.xi = xk[row];
    o.di = dinv ? dinv[row] : T(0);
    o.xp = prev ? xprev[row] : mk<T>(0, 0);
    return o;
}

template <class T> __device__ inline pair_t<T> cheb_apply(pair_t<T> s, const ChebRow<T> &o, T c1, T c2)
{
    return mk<T>(fmad(c2, o.di * (o.bb.x - s.x), fmad(c1, o.xi.x - o.xp.x, o.xi.x)),
                 fmad(c2, o.di * (o.bb.y - s.y), fmad(c1, o.xi.y - o.xp.y, o.xi.y)));
}

template <class I, class T, int RB, class VA>
__global__ void __launch_bounds__(kBlock) k_cheb(int n, int R, const int *__restrict__ sptr,
                                                 const I *__restrict__ col, const VA val0,
                                                 const T *__restrict__ dinv,
                                                 const pair_t<T> *__restrict__ b,
                                                 const pair_t<T> *__restrict__ xk, pair_t<T> *xprev,
                                                 T c1, T c2, int prev)
{
    extern __shared__ __align__(8) unsigned char lds_tab[];
    using VS = typename Staged<VA>::type;
    const int row = xcd_block() * kBlock + threadIdx.x;
    // FP64: D^-1 of the row is 1 / a_ii of the entries just read, the value
    // the setup stored (the same IEEE division), so it is not loaded; the
    // FP32 path loads its rounded copy
    constexpr bool own = std::is_same<T, double>::value;
    // every run's operands of the update first (in flight while the block
    // stages its value table), then the row product
    const int r0 = run0<RB>();
    ChebRow<T> o[RB];
    if (row < n) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R) {
                const long off = (long)(r0 + q) * n;
                o[q] = cheb_row<T>(b + off, xk + off, own ? nullptr : dinv, xprev + off, row, prev);
            }
    }
    const SliceAt sl = slice_at(sptr, row, n);
    const VS val = Staged<VA>::stage(val0, lds_tab);
    if (row >= n)
        return;
    sell_row_runs<I, T, RB, VS>(sptr, sl, col, val, xk, n, row, R, [&](int q, int r, pair_t<T> s, T diag) {
        ChebRow<T> &w = o[q];
        if (own)
            w.di = T(1) / diag;
        xprev[(long)r * n + row] = cheb_apply<T>(s, w, c1, c2);
    });
}

// The first two smoothing steps from x = 0 in one launch (SELL levels):
// x_1 = c2' D^-1 b is formed on the fly for the row and for every column it
// gathers, by the expression of k_cheb0 (so with its bits), and the row's
// x_2 = x_1 + c1 x_1 + c2 D^-1 (b - A x_1) follows as in k_cheb.  Both are
// stored (step 3 reads x_1 as its previous iterate).  The launch reads b and
// D^-1 where k_cheb0 + k_cheb read b and D^-1 twice and x_1 once more.
template <class T> struct FirstIter {
    const pair_t<T> *__restrict__ b;
    const T *__restrict__ dinv;
    T c2;
    __device__ pair_t<T> operator()(int j) const
    {
        const pair_t<T> bb = b[j];
        const T di = dinv[j];
        return mk<T>(c2 * (di * bb.x), c2 * (di * bb.y));
    }
};

// the row's operands of step 2 with x_1 formed on the fly
template <class T> __device__ inline ChebRow<T> first_row(const FirstIter<T> &x1, int row)
{
    ChebRow<T> o;
    o.bb = x1.b[row];
    o.di = x1.dinv[row];
    o.xi = mk<T>(x1.c2 * (o.di * o.bb.x), x1.c2 * (o.di * o.bb.y));
    o.xp = mk<T>(0, 0);
    return o;
}

// the row products A x_1 of RB runs (x_1 formed from run r's b), entries
// loaded once on slices at most kSellUnroll wide; f(q, r, product) with
// q = r - r0
template <class I, class T, int RB, class VA, class F>
__device__ inline void sell_row_first_runs(SliceAt sl, const I *__restrict__ col,
                                           const VA &val, const pair_t<T> *__restrict__ b,
                                           const T *__restrict__ dinv, T c2f, int n, int row, int R,
                                           F &&f)
{
    const int r0 = run0<RB>();
    const int lane = row % kSlice, base = sl.base, width = sl.width;
    auto runs_w = [&](auto wtag) {
        constexpr int W = decltype(wtag)::value;
        int c[W];
        T a[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int idx = base + (k < width ? k : width - 1) * kSlice + lane;
            c[k] = sell_col(col, idx, row);
            const T v = val[idx];
            a[k] = k < width ? v : T(0);
        }
        T dv[W];
#pragma unroll
        for (int k = 0; k < W; ++k)
            dv[k] = dinv[c[k]];
        pair_t<T> bv[RB][W];
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R)
#pragma unroll
                for (int k = 0; k < W; ++k)
                    bv[q][k] = b[(long)(r0 + q) * n + c[k]];
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R) {
                T ax = 0, ay = 0;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    ax = fmad(a[k], c2f * (dv[k] * bv[q][k].x), ax);
                    ay = fmad(a[k], c2f * (dv[k] * bv[q][k].y), ay);
                }
                f(q, r0 + q, mk<T>(ax, ay));
            }
    };
    if (width == 0) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R)
                f(q, r0 + q, mk<T>(0, 0));
    } else if (width <= kSellUnroll) {
        runs_w(std::integral_constant<int, kSellUnroll>{});
    } else if (RB == 1 && width <= 2 * kSellUnroll) {
        runs_w(std::integral_constant<int, RB == 1 ? 2 * kSellUnroll : 1>{});
    } else {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R) {
                const FirstIter<T> x1{b + (long)(r0 + q) * n, dinv, c2f};
                T ax = 0, ay = 0;
                for (int k = 0; k < width; ++k) {
                    const int idx = base + k * kSlice + lane;
                    const T a = val[idx];
                    const pair_t<T> xv = x1(sell_col(col, idx, row));
                    ax = fmad(a, xv.x, ax);
                    ay = fmad(a, xv.y, ay);
                }
                f(q, r0 + q, mk<T>(ax, ay));
            }
    }
}

// (the register budget of at most 4 waves per SIMD lets the compiler issue
// every load of a 16-wide row before the first product; with the default
// budget it interleaved the FP64 gathers with waits)
template <class I, class T, int RB, class VA>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 4)))
k_cheb_first(int n, int R, const int *__restrict__ sptr,
                                                       const I *__restrict__ col, const VA val0,
                                                       const T *__restrict__ dinv,
                                                       const pair_t<T> *__restrict__ b,
                                                       pair_t<T> *x1out, pair_t<T> *x2, T c2first,
                                                       T c1, T c2)
{
    extern __shared__ __align__(8) unsigned char lds_tab[];
    using VS = typename Staged<VA>::type;
    const int row = xcd_block() * kBlock + threadIdx.x;
    const int r0 = run0<RB>();
    ChebRow<T> o[RB];   // loaded while the block stages its value table
    if (row < n) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R)
                o[q] = first_row(FirstIter<T>{b + (long)(r0 + q) * n, dinv, c2first}, row);
    }
    const SliceAt sl = slice_at(sptr, row, n);
    const VS val = Staged<VA>::stage(val0, lds_tab);
    if (row >= n)
        return;
    sell_row_first_runs<I, T, RB, VS>(sl, col, val, b, dinv, c2first, n, row, R,
                                  [&](int q, int r, pair_t<T> s) {
                                      const ChebRow<T> &w = o[q];
                                      x1out[(long)r * n + row] = w.xi;
                                      x2[(long)r * n + row] = cheb_apply<T>(s, w, c1, c2);
                                  });
}

// the same for a CSR level with a group of GS lanes per row
template <int GS, int U, class T>
__global__ void __launch_bounds__(kBlock) k_cheb_v_first(int n, const int *__restrict__ rp,
                                                         const int *__restrict__ ci,
                                                         const T *__restrict__ v,
                                                         const T *__restrict__ dinv,
                                                         const pair_t<T> *__restrict__ b,
                                                         pair_t<T> *x1out, pair_t<T> *x2,
                                                         T c2first, T c1, T c2)
{
    const int t = xcd_block() * kBlock + threadIdx.x;
    const int row = t / GS, lane = t % GS;
    if (row >= n)
        return;
    const FirstIter<T> x1{run_at(b, n), dinv, c2first};
    const ChebRow<T> o = first_row(x1, row);   // the group's lanes share these lines
    const pair_t<T> s = row_dot_g<GS, U, T>(rp, ci, v, x1, row, lane);
    if (lane != 0)
        return;
    run_at(x1out, n)[row] = o.xi;
    run_at(x2, n)[row] = cheb_apply<T>(s, o, c1, c2);
}

template <int GS, int U, class T>
__global__ void __launch_bounds__(kBlock) k_cheb_v(int n, const int *__restrict__ rp,
                                                   const int *__restrict__ ci,
                                                   const T *__restrict__ v,
                                                   const T *__restrict__ dinv,
                                                   const pair_t<T> *__restrict__ b,
                                                   const pair_t<T> *__restrict__ xk,
                                                   pair_t<T> *xprev, T c1, T c2, int prev)
{
    const int t = xcd_block() * kBlock + threadIdx.x;
    const int row = t / GS, lane = t % GS;
    if (row >= n)
        return;
    b = run_at(b, n);
    xk = run_at(xk, n);
    xprev = run_at(xprev, n);
    const ChebRow<T> o = cheb_row<T>(b, xk, dinv, xprev, row, prev);   // the group's lanes share these lines
    const pair_t<T> s = row_dot<GS, U, T>(rp, ci, v, xk, row, lane);
    if (lane != 0)
        return;
    xprev[row] = cheb_apply<T>(s, o, c1, c2);
}

// The prolongation and the first post-smoothing step in one launch (CSR
// levels): x0 = x + P e and x1 = x0 + c2 D^-1 (b - A x0), with A x0 from
// AM [x; e] = A x + (A P) e (no gather of x0, which the launch writes).  x0
// goes to x0out (the next step's previous iterate) and x1 to x1out; neither
// may be x.  Per run, b, x and the outputs advance by n, e by nc.
template <int GS, int U, class T>
__global__ void __launch_bounds__(kBlock) k_prolong_cheb_v(int n, int nc, const int *__restrict__ arp,
                                                           const int *__restrict__ aci,
                                                           const T *__restrict__ av,
                                                           const int *__restrict__ prp,
                                                           const int *__restrict__ pci,
                                                           const T *__restrict__ pv,
                                                           const T *__restrict__ dinv,
                                                           const pair_t<T> *__restrict__ b,
                                                           const pair_t<T> *__restrict__ x,
                                                           const pair_t<T> *__restrict__ e,
                                                           pair_t<T> *x0out, pair_t<T> *x1out, T c2)
{
    const int t = xcd_block() * kBlock + threadIdx.x;
    const int row = t / GS, lane = t % GS;
    if (row >= n)
        return;
    b = run_at(b, n);
    x = run_at(x, n);
    e = run_at(e, nc);
    const pair_t<T> s = row_dot_g<GS, U, T>(arp, aci, av, GatherBX<T>{x, e, n}, row, lane);
    const pair_t<T> pe = row_dot<GS, 1, T>(prp, pci, pv, e, row, lane);
    if (lane != 0)
        return;
    const pair_t<T> xi = x[row];
    ChebRow<T> o;
    o.bb = b[row];
    o.xi = mk<T>(xi.x + pe.x, xi.y + pe.y);
    o.di = dinv[row];
    o.xp = mk<T>(0, 0);
    run_at(x0out, n)[row] = o.xi;
    run_at(x1out, n)[row] = cheb_apply<T>(s, o, T(0), c2);
}

// first smoothing step from x = 0: x = c2 D^-1 b
template <class T>
__global__ void __launch_bounds__(kBlock) k_cheb0(int n, const T *__restrict__ dinv,
                                                  const pair_t<T> *__restrict__ b, pair_t<T> *x,
                                                  T c2)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= n)
        return;
    const pair_t<T> bb = run_at(b, n)[row];
    const T di = dinv[row];
    run_at(x, n)[row] = mk<T>(c2 * (di * bb.x), c2 * (di * bb.y));
}

// coarsest level: x = A^-1 b with the FP64 inverse stored row-major.  One
// wave per row (four rows per block): lane l takes columns l, l + 64, ...,
// four of them per pass into separate accumulators, so each lane keeps four
// loads of the row in flight (the inverse streams from the last-level cache;
// b stays in L2); the accumulators are added in a fixed order and the wave
// with a fixed shuffle tree.  FP64 sums in both precisions.
constexpr int kDenseRows = kBlock / 64;

template <class T, int RB>
__global__ void __launch_bounds__(kBlock) k_dense(int n, int R, const double *__restrict__ inv,
                                                  const pair_t<T> *__restrict__ b, pair_t<T> *x)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * kDenseRows + (threadIdx.x >> 6);
    if (row >= n)
        return;   // the whole wave: row depends on the wave only
    const double *a = inv + (size_t)row * n;
    const int r0 = run0<RB>();
    // every run's sums over the row, each with the single-run order; the
    // row's entries are loaded once for the RB runs
    double2 acc[RB][4];
#pragma unroll
    for (int q = 0; q < RB; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u)
            acc[q][u] = d2(0.0, 0.0);
    int j = lane;
    for (; j + 192 < n; j += 256) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            v[u] = a[j + 64 * u];
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R) {
                const pair_t<T> *bq = b + (long)(r0 + q) * n;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const pair_t<T> bv = bq[j + 64 * u];
                    acc[q][u].x = fmad(v[u], double(bv.x), acc[q][u].x);
                    acc[q][u].y = fmad(v[u], double(bv.y), acc[q][u].y);
                }
            }
    }
    for (; j < n; j += 64) {
        const double v = a[j];
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R) {
                const pair_t<T> bv = b[(long)(r0 + q) * n + j];
                acc[q][0].x = fmad(v, double(bv.x), acc[q][0].x);
                acc[q][0].y = fmad(v, double(bv.y), acc[q][0].y);
            }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        double2 s = d2((acc[q][0].x + acc[q][1].x) + (acc[q][2].x + acc[q][3].x),
                       (acc[q][0].y + acc[q][1].y) + (acc[q][2].y + acc[q][3].y));
        s = wave_sum(s);
        if (lane == 0 && (RB == 1 || r0 + q < R))
            x[(long)(r0 + q) * n + row] = mk<T>(T(s.x), T(s.y));
    }
}

// launches with rb runs per lane (1, 2 or 4) over R runs
template <class I, class T, class VA>
void cheb_rb(hipStream_t st, int rb, int n, int R, const int *sptr, const I *col, const VA &val,
             const T *dinv, const pair_t<T> *b, const pair_t<T> *xk, pair_t<T> *xprev, T c1, T c2,
             int prev)
{
    const dim3 g = grid_rb(nblk(n), R, rb);
    const size_t lb = lds_bytes(val);
    if (rb >= 4)
        k_cheb<I, T, 4, VA><<<g, kBlock, lb, st>>>(n, R, sptr, col, val, dinv, b, xk, xprev, c1, c2,
                                                  prev);
    else if (rb == 2)
        k_cheb<I, T, 2, VA><<<g, kBlock, lb, st>>>(n, R, sptr, col, val, dinv, b, xk, xprev, c1, c2,
                                                  prev);
    else
        k_cheb<I, T, 1, VA><<<g, kBlock, lb, st>>>(n, R, sptr, col, val, dinv, b, xk, xprev, c1, c2,
                                                  prev);
}

template <class I, class T, class VA>
void cheb_first_rb(hipStream_t st, int rb, int n, int R, const int *sptr, const I *col,
                   const VA &val, const T *dinv, const pair_t<T> *b, pair_t<T> *x1, pair_t<T> *x2,
                   T c2f, T c1, T c2)
{
    const dim3 g = grid_rb(nblk(n), R, rb);
    const size_t lb = lds_bytes(val);
    if (rb >= 4)
        k_cheb_first<I, T, 4, VA><<<g, kBlock, lb, st>>>(n, R, sptr, col, val, dinv, b, x1, x2, c2f,
                                                        c1, c2);
    else if (rb == 2)
        k_cheb_first<I, T, 2, VA><<<g, kBlock, lb, st>>>(n, R, sptr, col, val, dinv, b, x1, x2, c2f,
                                                        c1, c2);
    else
        k_cheb_first<I, T, 1, VA><<<g, kBlock, lb, st>>>(n, R, sptr, col, val, dinv, b, x1, x2, c2f,
                                                        c1, c2);
}

template <class T>
void dense_rb(hipStream_t st, int rb, int n, int R, const double *inv, const pair_t<T> *b,
              pair_t<T> *x)
{
    const dim3 g = grid_rb(nblk(n, kDenseRows), R, rb);
    if (rb >= 4)
        k_dense<T, 4><<<g, kBlock, 0, st>>>(n, R, inv, b, x);
    else if (rb == 2)
        k_dense<T, 2><<<g, kBlock, 0, st>>>(n, R, inv, b, x);
    else
        k_dense<T, 1><<<g, kBlock, 0, st>>>(n, R, inv, b, x);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_axpy_add(int n, const pair_t<T> *__restrict__ e,
                                                     pair_t<T> *x)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= n)
        return;
    e = run_at(e, n);
    x = run_at(x, n);
    const pair_t<T> a = x[row], b = e[row];
    x[row] = mk<T>(a.x + b.x, a.y + b.y);
}

// ------------------------------------------------------------------ inner tolerance
// Per run (blockIdx.y) and species: whether the stationary solve goes on,
// from the partials of b.b and r.r: it stops once ||r|| <= tol ||b|| (and
// stays stopped: the iterate no longer changes).
__global__ void __launch_bounds__(kBlock) k_amg_flags(const double2 *__restrict__ pb,
                                                      const double2 *__restrict__ pr, int G,
                                                      double tol, int2 *act, int first)
{
    __shared__ double2 sh[2];
    reduce_two(run_at(pb, kSlotStride), run_at(pr, kSlotStride), G, sh);
    if (threadIdx.x == 0) {
        const int2 a = first ? make_int2(1, 1) : act[blockIdx.y];
        const double bx = sqrt(sh[0].x), by = sqrt(sh[0].y);
        const double rx = sqrt(sh[1].x), ry = sqrt(sh[1].y);
        act[blockIdx.y] = make_int2(a.x && !(rx <= tol * bx), a.y && !(ry <= tol * by));
    }
}

// the residual of a stopped species is set to zero, so its V-cycle
// correction is exactly zero and its iterate stays as it is
template <class T>
__global__ void __launch_bounds__(kBlock) k_amg_mask(int n, pair_t<T> *r, const int2 *__restrict__ act)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row >= n)
        return;
    const int2 a = act[blockIdx.y];
    r = run_at(r, n);
    const pair_t<T> v = r[row];
    r[row] = mk<T>(a.x ? v.x : T(0), a.y ? v.y : T(0));
}

// ------------------------------------------------------------------ inner CG for As
__device__ inline double2 ratio_or_zero(double2 num, double2 den)
{
    return d2(den.x != 0.0 ? num.x / den.x : 0.0, den.y != 0.0 ? num.y / den.y : 0.0);
}

// alpha = rz / dq from partials; first == 1: x = alpha d, r = b - alpha q
// (x = 0 and r = b before the step), else x += alpha d, r -= alpha q; with
// want_r = 0 (the last step) r is left alone
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_xr(int n, pair_t<T> *x, pair_t<T> *r,
                                                   const pair_t<T> *__restrict__ b,
                                                   const pair_t<T> *__restrict__ d,
                                                   const pair_t<T> *__restrict__ q,
                                                   const double2 *__restrict__ rz_part,
                                                   const double2 *__restrict__ dq_part, int G,
                                                   int first, int want_r)
{
    __shared__ double2 sc[2];
    reduce_two(run_at(rz_part, kSlotStride), run_at(dq_part, kSlotStride), G, sc);
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    x = run_at(x, n);
    r = run_at(r, n);
    b = run_at(b, n);
    d = run_at(d, n);
    q = run_at(q, n);
    const double2 al = ratio_or_zero(sc[0], sc[1]);
    const T ax = T(al.x), ay = T(al.y);
    const pair_t<T> dv = d[i];
    pair_t<T> xv = first ? mk<T>(0, 0) : x[i];
    xv.x += ax * dv.x;
    xv.y += ay * dv.y;
    x[i] = xv;
    if (!want_r)
        return;
    const pair_t<T> qv = q[i];
    pair_t<T> rv = first ? b[i] : r[i];
    rv.x -= ax * qv.x;
    rv.y -= ay * qv.y;
    r[i] = rv;
}

// d = z + beta d with beta = rz_new / rz_old (0 where rz_old == 0)
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_dir(int n, const pair_t<T> *__restrict__ z,
                                                    pair_t<T> *d,
                                                    const double2 *__restrict__ new_part,
                                                    const double2 *__restrict__ old_part, int G)
{
    __shared__ double2 sc[2];
    reduce_two(run_at(new_part, kSlotStride), run_at(old_part, kSlotStride), G, sc);
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    z = run_at(z, n);
    d = run_at(d, n);
    const pair_t<T> zv = z[i];
    const double2 be = ratio_or_zero(sc[0], sc[1]);
    const T bx = T(be.x), by = T(be.y);
    const pair_t<T> dv = d[i];
    d[i] = mk<T>(zv.x + bx * dv.x, zv.y + by * dv.y);
}

// ------------------------------------------------------------------ batch layout
// per run: out[0..n) = in[run * stride + 0..n) (a half of a block vector into
// a contiguous work vector) and back
template <class T>
__global__ void __launch_bounds__(kBlock) k_gather_half(int n, const pair_t<T> *__restrict__ in,
                                                        long stride, pair_t<T> *out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        run_at(out, n)[i] = run_at(in, stride)[i];
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_scatter_half(int n, const pair_t<T> *__restrict__ in,
                                                         pair_t<T> *out, long stride)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        run_at(out, stride)[i] = run_at(in, n)[i];
}

// ------------------------------------------------------------------ precision boundary
__global__ void __launch_bounds__(kBlock) k_narrow_pairs(int n, const double2 *__restrict__ a,
                                                         float2 *b)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double2 v = run_at(a, n)[i];
        run_at(b, n)[i] = make_float2(float(v.x), float(v.y));
    }
}

__global__ void __launch_bounds__(kBlock) k_widen_pairs(int n, const float2 *__restrict__ a,
                                                        double2 *b)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const float2 v = run_at(a, n)[i];
        run_at(b, n)[i] = make_double2(double(v.x), double(v.y));
    }
}

__global__ void __launch_bounds__(kBlock) k_narrow(long n, const double *__restrict__ a, float *b)
{
    const long i = (long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        b[i] = float(a[i]);
}

// ------------------------------------------------------------------ per-precision buffers
template <class T> struct Vecs {
    pair_t<T> *x, *xt, *b, *r;
};
template <class T> Vecs<T> vecs(Hierarchy &H, int l);
template <> Vecs<double> vecs<double>(Hierarchy &H, int l) { return {H.x[l], H.xt[l], H.b[l], H.r[l]}; }
template <> Vecs<float> vecs<float>(Hierarchy &H, int l) { return {H.fx[l], H.fxt[l], H.fb[l], H.fr[l]}; }

template <class T> Work<T> &work(Solver &S);
template <> Work<double> &work<double>(Solver &S) { return S.w64; }
template <> Work<float> &work<float>(Solver &S) { return S.w32; }

template <class T> const T *mass_sell_values(const Solver &S);
template <> const double *mass_sell_values<double>(const Solver &S) { return S.sM.val; }
template <> const float *mass_sell_values<float>(const Solver &S) { return S.fsM; }
template <class T> const T *mass_sell_table(const Solver &S);
template <> const double *mass_sell_table<double>(const Solver &S) { return S.vtM.tab; }
template <> const float *mass_sell_table<float>(const Solver &S) { return S.vtM.ftab; }
template <class T> const uint16_t *mass_sell_index(const Solver &S);
template <> const uint16_t *mass_sell_index<double>(const Solver &S) { return S.vtM.ix; }
template <> const uint16_t *mass_sell_index<float>(const Solver &S)
{
    return fp32_table(S.sM) ? S.vtM.ix : nullptr;
}

// ------------------------------------------------------------------ V-cycle (host)
// The event timer brackets each run of back-to-back smoothing launches on the
// fine level of the As hierarchy (the pre- and post-smoothing sequences), so
// the event overhead is spread over the launches of a run.
bool timed_level(const Solver &S, const Hierarchy &H, int l)
{
    return S.timer.on && S.timer.kind == 0 && &H == &S.hA && l == 0;
}

// the CSR-vector smoothing launch for the matrix's entries per lane and pass
template <int GS, class T>
void cheb_v_u(hipStream_t st, int R, const MatView<T> &A, const T *dinv, const pair_t<T> *b,
              const pair_t<T> *xk, pair_t<T> *xprev, T c1, T c2, int prev)
{
    const dim3 g = grid(nblk((long)GS * A.n), R);
    if (A.u >= 4)
        k_cheb_v<GS, 4, T><<<g, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.cval, dinv, b, xk, xprev, c1, c2,
                                                 prev);
    else if (A.u == 2)
        k_cheb_v<GS, 2, T><<<g, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.cval, dinv, b, xk, xprev, c1, c2,
                                                 prev);
    else
        k_cheb_v<GS, 1, T><<<g, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.cval, dinv, b, xk, xprev, c1, c2,
                                                 prev);
}

template <int GS, class T>
void cheb_first_v_u(hipStream_t st, int R, const MatView<T> &A, const T *dinv, const pair_t<T> *b,
                    pair_t<T> *x1, pair_t<T> *x2, T c2f, T c1, T c2)
{
    const dim3 g = grid(nblk((long)GS * A.n), R);
    if (A.u >= 4)
        k_cheb_v_first<GS, 4, T><<<g, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.cval, dinv, b, x1, x2,
                                                       c2f, c1, c2);
    else if (A.u == 2)
        k_cheb_v_first<GS, 2, T><<<g, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.cval, dinv, b, x1, x2,
                                                       c2f, c1, c2);
    else
        k_cheb_v_first<GS, 1, T><<<g, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.cval, dinv, b, x1, x2,
                                                       c2f, c1, c2);
}

// smoothing steps 1 and 2 from x = 0 on level l in one launch: x1 <- x_1,
// x2 <- x_2 (step 1 with c2f, step 2 with c1, c2)
template <class T>
void launch_cheb_first(Solver &S, Hierarchy &H, int l, const pair_t<T> *b, pair_t<T> *x1,
                       pair_t<T> *x2, double c2fd, double c1d, double c2d)
{
    const Level &L = H.lev[l];
    const MatView<T> A = L.viewA<T>();
    const T *dinv = L.dinv_t<T>();
    const T c2f = T(c2fd), c1 = T(c1d), c2 = T(c2d);
    const int n = L.n, R = S.nrun;
    hipStream_t st = S.stream;
    switch (A.gs) {
    case 0:
        if (A.ocol && A.vix)
            cheb_first_rb<int16_t, T>(st, rb_of(S), n, R, A.sptr, A.ocol, VTab<T>{A.vix, A.vtab, A.vm},
                                      dinv, b, x1, x2, c2f, c1, c2);
        else if (A.ocol)
            cheb_first_rb<int16_t, T>(st, rb_of(S), n, R, A.sptr, A.ocol, VPlain<T>{A.sval}, dinv, b,
                                      x1, x2, c2f, c1, c2);
        else
            cheb_first_rb<int, T>(st, rb_of(S), n, R, A.sptr, A.col, VPlain<T>{A.sval}, dinv, b, x1,
                                  x2, c2f, c1, c2);
        break;
    case 4:
        cheb_first_v_u<4, T>(st, R, A, dinv, b, x1, x2, c2f, c1, c2);
        break;
    case 8:
        cheb_first_v_u<8, T>(st, R, A, dinv, b, x1, x2, c2f, c1, c2);
        break;
    case 16:
        cheb_first_v_u<16, T>(st, R, A, dinv, b, x1, x2, c2f, c1, c2);
        break;
    default:
        cheb_first_v_u<32, T>(st, R, A, dinv, b, x1, x2, c2f, c1, c2);
        break;
    }
}

// one smoothing step on level l: xprev <- x_{k+1} from xk (and xprev when prev = 1)
template <class T>
void launch_cheb(Solver &S, Hierarchy &H, int l, const pair_t<T> *b, const pair_t<T> *xk,
                 pair_t<T> *xprev, double c1d, double c2d, int prev)
{
    const Level &L = H.lev[l];
    const MatView<T> A = L.viewA<T>();
    const T *dinv = L.dinv_t<T>();
    const T c1 = T(c1d), c2 = T(c2d);
    const int n = L.n, R = S.nrun;
    hipStream_t st = S.stream;
    switch (A.gs) {
    case 0:
        if (A.ocol && A.vix)
            cheb_rb<int16_t, T>(st, rb_of(S), n, R, A.sptr, A.ocol, VTab<T>{A.vix, A.vtab, A.vm}, dinv, b,
                                xk, xprev, c1, c2, prev);
        else if (A.ocol)
            cheb_rb<int16_t, T>(st, rb_of(S), n, R, A.sptr, A.ocol, VPlain<T>{A.sval}, dinv, b, xk,
                                xprev, c1, c2, prev);
        else
            cheb_rb<int, T>(st, rb_of(S), n, R, A.sptr, A.col, VPlain<T>{A.sval}, dinv, b, xk, xprev,
                            c1, c2, prev);
        break;
    case 4:
        cheb_v_u<4, T>(st, R, A, dinv, b, xk, xprev, c1, c2, prev);
        break;
    case 8:
        cheb_v_u<8, T>(st, R, A, dinv, b, xk, xprev, c1, c2, prev);
        break;
    case 16:
        cheb_v_u<16, T>(st, R, A, dinv, b, xk, xprev, c1, c2, prev);
        break;
    default:
        cheb_v_u<32, T>(st, R, A, dinv, b, xk, xprev, c1, c2, prev);
        break;
    }
    if (timed_level(S, H, l)) {
        // algorithmic bytes: column index (2 B as a SELL offset, else 4) +
        // value per nonzero (its 2-byte index into the value table where the
        // matrix has one; the table itself stays in cache), once per launch;
        // per row D^-1 (except the FP64 SELL kernel, which takes it from the
        // diagonal entry) and per row and run x_k (gathered once), b, x_{k-1}
        // (when read) and the written x_{k+1}
        const long long ib = (A.gs == 0 && A.ocol) ? 2 : 4;
        const long long vb = (A.gs == 0 && A.ocol && A.vix) ? 2 : (long long)sizeof(T);
        const bool own = A.gs == 0 && std::is_same<T, double>::value;
        S.timer.count += 1;
        S.timer.bytes += (ib + vb) * L.A.nnz +
                         (own ? 0ll : (long long)sizeof(T) * L.n) +
                         (long long)R * (prev ? 8 : 6) * sizeof(T) * L.n;
    }
}

// The level's smoother from x = 0: deg steps (Chebyshev over the level's
// interval, or damped Jacobi) on b, the first into `first`, each further step
// into the other buffer.  Returns the buffer holding the result (first when
// deg is odd).
template <class T>
pair_t<T> *presmooth(Solver &S, Hierarchy &H, int l, const pair_t<T> *b, pair_t<T> *first,
                     pair_t<T> *other)
{
    const Level &L = H.lev[l];
    const int deg = L.degree, R = S.nrun;
    auto c1 = [&](int k) { return (H.jacobi || k == 1) ? 0.0 : L.cheb_c1[k]; };
    auto c2 = [&](int k) { return H.jacobi ? L.jac_omega : L.cheb_c2[k]; };
    pair_t<T> *cur = first, *oth = other;
    int k0 = 2;   // the first step k_cheb handles
    // FP64 SELL levels with a value table and slices wider than kSellUnroll
    // (3D patterns) take step 1 as its own light launch and step 2 as a k_cheb
    // step (x_1 gathered once, the same bits): the fused launch gathers b and
    // D^-1 per entry of its 16-wide rows (18.9 us on the 96x96x48 box against
    // 5.2 + 12.0 us).  FP32 and the 2D patterns gain nothing from the split.
    const MatView<T> A = L.viewA<T>();
    const bool fuse12 = !(std::is_same<T, double>::value && A.gs == 0 && A.ocol && A.vix &&
                          L.sA.wmax > kSellUnroll);
    if (deg >= 2 && fuse12) {
        // steps 1 and 2 in one launch; x_1 and x_2 land where the two
        // launches would put them
        launch_cheb_first<T>(S, H, l, b, cur, oth, c2(1), c1(2), c2(2));
        std::swap(cur, oth);
        k0 = 3;
    } else {
        k_cheb0<T><<<grid(nblk(L.n), R), kBlock, 0, S.stream>>>(L.n, L.dinv_t<T>(), b, first,
                                                                 T(c2(1)));
    }
    const bool timed = timed_level(S, H, l);
    if (timed && deg >= k0)
        timer_mark(S, true);
    for (int k = k0; k <= deg; ++k) {   // x_0 = 0: the previous iterate is zero at k = 2
        launch_cheb<T>(S, H, l, b, cur, oth, c1(k), c2(k), k > 2 && !H.jacobi);
        std::swap(cur, oth);
    }
    if (timed && deg >= k0)
        timer_mark(S, false);
    return cur;
}

template <int GS, class T>
void prolong_cheb_u(hipStream_t st, int R, const MatView<T> &AM, const MatView<T> &P,
                    const T *dinv, const pair_t<T> *b, const pair_t<T> *x, const pair_t<T> *e,
                    pair_t<T> *x0, pair_t<T> *x1, T c2)
{
    const dim3 g = grid(nblk((long)GS * AM.n), R);
    const int nc = AM.m - AM.n;
    if (AM.u >= 4)
        k_prolong_cheb_v<GS, 4, T><<<g, kBlock, 0, st>>>(AM.n, nc, AM.rp, AM.ci, AM.cval, P.rp,
                                                          P.ci, P.cval, dinv, b, x, e, x0, x1, c2);
    else if (AM.u == 2)
        k_prolong_cheb_v<GS, 2, T><<<g, kBlock, 0, st>>>(AM.n, nc, AM.rp, AM.ci, AM.cval, P.rp,
                                                          P.ci, P.cval, dinv, b, x, e, x0, x1, c2);
    else
        k_prolong_cheb_v<GS, 1, T><<<g, kBlock, 0, st>>>(AM.n, nc, AM.rp, AM.ci, AM.cval, P.rp,
                                                          P.ci, P.cval, dinv, b, x, e, x0, x1, c2);
}

template <class T>
void prolong_cheb(Solver &S, const Level &L, const pair_t<T> *b, const pair_t<T> *x,
                  const pair_t<T> *e, pair_t<T> *x0, pair_t<T> *x1, double c2d)
{
    const MatView<T> AM = L.viewAM<T>(), P = L.viewP<T>();
    if (!AM.cval || !P.cval || !P.rp)
        throw Failure(CHM_EINVAL, "fused prolongation without CSR values of [A | A P] and P");
    const T *dinv = L.dinv_t<T>();
    const T c2 = T(c2d);
    const int R = S.nrun;
    hipStream_t st = S.stream;
    switch (AM.gs) {
    case 4:
        prolong_cheb_u<4, T>(st, R, AM, P, dinv, b, x, e, x0, x1, c2);
        break;
    case 8:
        prolong_cheb_u<8, T>(st, R, AM, P, dinv, b, x, e, x0, x1, c2);
        break;
    case 16:
        prolong_cheb_u<16, T>(st, R, AM, P, dinv, b, x, e, x0, x1, c2);
        break;
    default:
        prolong_cheb_u<32, T>(st, R, AM, P, dinv, b, x, e, x0, x1, c2);
        break;
    }
}

template <class T>
void vcycle_level(Solver &S, Hierarchy &H, int l, const pair_t<T> *b, pair_t<T> *x)
{
    const Level &L = H.lev[l];
    hipStream_t st = S.stream;
    const int R = S.nrun;
    if (l == H.nlev - 1) {
        dense_rb<T>(st, rb_of(S), L.n, R, L.inv, b, x);
        return;
    }
    const Vecs<T> V = vecs<T>(H, l), Vc = vecs<T>(H, l + 1);
    const int deg = L.degree;
    auto c1 = [&](int k) { return (H.jacobi || k == 1) ? 0.0 : L.cheb_c1[k]; };
    auto c2 = [&](int k) { return H.jacobi ? L.jac_omega : L.cheb_c2[k]; };
    const bool timed = timed_level(S, H, l);
    // the prolongation fused with the first post-smoothing step (CSR levels
    // with AM): pre-smoothing then ends in xt, and the post-smoothing steps
    // alternate between x and r so that the last one lands in x
    // (it reads P's CSR values, which the FP32 copy holds only where P's
    // kernels use the CSR layout too)
    const bool fused_post = L.AM.nnz > 0 && L.gsP > 0 && !timed;
    // Pre-smoothing from zero.  Every step after the first writes the buffer
    // not holding the current iterate; 2 deg - 1 such steps follow the first,
    // so starting in xt leaves the result in x.
    pair_t<T> *cur = fused_post && deg % 2 == 0 ? presmooth<T>(S, H, l, b, x, V.xt)
                                                : presmooth<T>(S, H, l, b, V.xt, x);
    pair_t<T> *oth = cur == x ? V.xt : x;
    if (L.RR.nnz > 0) {   // b_c = R (b - A x) in one product
        resid_restrict<T>(st, R, L.viewRR<T>(), b, cur, Vc.b);
    } else {
        spmv_op<SP_RESID, T>(st, R, rb_of(S), L.viewA<T>(), cur, b, V.r);
        spmv_op<SP_SET, T>(st, R, rb_of(S), L.viewR<T>(), V.r, nullptr, Vc.b);
    }
    vcycle_level<T>(S, H, l + 1, Vc.b, Vc.x);
    if (fused_post) {
        // x_0 = cur + P e into a, x_1 into c; steps 2.. alternate, x_deg in x
        pair_t<T> *a0 = deg % 2 == 0 ? x : V.r, *a1 = deg % 2 == 0 ? V.r : x;
        prolong_cheb<T>(S, L, b, cur, Vc.x, a0, a1, c2(1));
        for (int k = 2; k <= deg; ++k) {
            launch_cheb<T>(S, H, l, b, a1, a0, c1(k), c2(k), !H.jacobi);
            std::swap(a0, a1);
        }
        return;
    }
    spmv_op<SP_ADD, T>(st, R, rb_of(S), L.viewP<T>(), Vc.x, nullptr, cur);
    if (timed)
        timer_mark(S, true);
    for (int k = 1; k <= deg; ++k) {
        launch_cheb<T>(S, H, l, b, cur, oth, c1(k), c2(k), k > 1 && !H.jacobi);
        std::swap(cur, oth);
    }
    if (timed)
        timer_mark(S, false);
}

// stationary AMG solve: x = V(b), then x += V(b - A x) for the further
// cycles: amg_cycles in all, or with amg_tol > 0 until each species' residual
// norm is at most amg_tol times that of its b (at most amg_cycles; the host
// reads the flags after each residual, so this mode runs eagerly).  The mass
// block with mass_solver = CHM_MASS_CHEBYSHEV is a Chebyshev semi-iteration
// instead (Section 3 names it as the alternative to AMG for M).
template <class T>
void stationary(Solver &S, Hierarchy &H, const pair_t<T> *b, pair_t<T> *x)
{
    Work<T> &W = work<T>(S);
    const Level &L0 = H.lev[0];
    const int n = L0.n, R = S.nrun, G = red_blocks(n);
    const double tol = S.prm.amg_tol;
    hipStream_t st = S.stream;
    if (&H == &S.hM && S.prm.mass_solver == CHM_MASS_CHEBYSHEV) {
        // the Chebyshev semi-iteration on M instead of V-cycles: the mass
        // hierarchy's fine-level smoother from zero, landing in x
        pair_t<T> *xt = vecs<T>(H, 0).xt;
        const bool odd = L0.degree % 2 == 1;
        presmooth<T>(S, H, 0, b, odd ? x : xt, odd ? xt : x);
        return;
    }
    vcycle_level<T>(S, H, 0, b, x);
    if (tol > 0.0 && S.prm.amg_cycles > 1)
        k_dot<T><<<grid(G, R), kBlock, 0, st>>>(n, b, b, slot(S, kSlotRz));
    for (int c = 1; c < S.prm.amg_cycles; ++c) {
        spmv_op<SP_RESID, T>(st, R, rb_of(S), L0.viewA<T>(), x, b, W.mr);
        if (tol > 0.0) {
            k_dot<T><<<grid(G, R), kBlock, 0, st>>>(n, W.mr, W.mr, slot(S, kSlotRz + 1));
            k_amg_flags<<<grid(1, R), kBlock, 0, st>>>(slot(S, kSlotRz), slot(S, kSlotRz + 1), G,
                                                       tol, S.amg_act, c == 1);
            CHM_HIP(hipMemcpyAsync(S.hamg_act, S.amg_act, sizeof(int2) * R, hipMemcpyDeviceToHost,
                                   st));
            CHM_HIP(hipStreamSynchronize(st));
            bool any = false;
            for (int r = 0; r < R; ++r)
                any = any || S.hamg_act[r].x || S.hamg_act[r].y;
            if (!any)
                break;
            k_amg_mask<T><<<grid(nblk(n), R), kBlock, 0, st>>>(n, W.mr, S.amg_act);
        }
        vcycle_level<T>(S, H, 0, W.mr, W.me);
        k_axpy_add<T><<<grid(nblk(n), R), kBlock, 0, st>>>(n, W.me, x);
    }
}

// As solve of Algorithm 1: schur_pcg CG steps preconditioned by one V-cycle
// (or amg_cycles stationary V-cycles when schur_pcg = 0)
template <class T>
void schur_solve_t(Solver &S, const pair_t<T> *b, pair_t<T> *x)
{
    Hierarchy &H = S.hA;
    const int n = S.nv, k = S.prm.schur_pcg;
    hipStream_t st = S.stream;
    if (k <= 0) {
        stationary<T>(S, H, b, x);
        return;
    }
    Work<T> &W = work<T>(S);
    const MatView<T> A = H.lev[0].viewA<T>();
    pair_t<T> *r = W.pcg_r, *q = W.pcg_q;
    const int G = red_blocks(n), R = S.nrun;
    // the first direction is z itself (no copy); each later z goes to the
    // buffer not holding the direction, which k_pcg_dir then updates in place
    pair_t<T> *d = W.pcg_z;
    vcycle_level<T>(S, H, 0, b, d);                                    // z = V(b), r = b
    for (int it = 1; it <= k; ++it) {
        spmv_op<SP_SET, T>(st, R, rb_of(S), A, d, nullptr, q);
        if (it == 1)   // r . z and d . q of the first step (d = z) in one launch
            k_dot2<T><<<grid(G, R), kBlock, 0, st>>>(n, b, d, slot(S, kSlotRz), d, q,
                                                     slot(S, kSlotDq + 1));
        else
            k_dot<T><<<grid(G, R), kBlock, 0, st>>>(n, d, q, slot(S, kSlotDq + it));
        k_pcg_xr<T><<<grid(nblk(n), R), kBlock, 0, st>>>(n, x, r, b, d, q, slot(S, kSlotRz + it - 1),
                                                         slot(S, kSlotDq + it), G, it == 1,
                                                         it < k);
        if (it == k)
            break;
        pair_t<T> *z = d == W.pcg_z ? W.pcg_d : W.pcg_z;
        vcycle_level<T>(S, H, 0, r, z);
        k_dot<T><<<grid(G, R), kBlock, 0, st>>>(n, r, z, slot(S, kSlotRz + it));
        k_pcg_dir<T><<<grid(nblk(n), R), kBlock, 0, st>>>(n, z, d, slot(S, kSlotRz + it),
                                                          slot(S, kSlotRz + it - 1), G);
    }
}

// Algorithm 1 on a block vector: w1 = AMG(M) v1; w2 = As^-1 M As^-1 v2.
// A batch holds its runs' block vectors back to back (2n apart); the two
// halves go through contiguous per-run work vectors (n apart), since the
// V-cycles take their runs n apart.
template <class T>
void apply_prec_t(Solver &S, const pair_t<T> *v, pair_t<T> *w)
{
    Work<T> &W = work<T>(S);
    const int n = S.nv, R = S.nrun;
    hipStream_t st = S.stream;
    const long len = 2l * n;
    if (R == 1) {
        stationary<T>(S, S.hM, v, w);
        schur_solve_t<T>(S, v + n, W.tmp);
        sell_spmv<SP_SET, T>(st, 1, 1, n, S.sM.sptr, S.sM.col, S.sM.ocol,
                             mass_sell_values<T>(S), mass_sell_index<T>(S), mass_sell_table<T>(S), S.vtM.m, W.tmp, n,
                             nullptr, W.tmp2, n);
        schur_solve_t<T>(S, W.tmp2, w + n);
        return;
    }
    k_gather_half<T><<<grid(nblk(n), R), kBlock, 0, st>>>(n, v, len, W.h1);
    stationary<T>(S, S.hM, W.h1, W.h2);
    k_scatter_half<T><<<grid(nblk(n), R), kBlock, 0, st>>>(n, W.h2, w, len);
    k_gather_half<T><<<grid(nblk(n), R), kBlock, 0, st>>>(n, v + n, len, W.h1);
    schur_solve_t<T>(S, W.h1, W.tmp);
    sell_spmv<SP_SET, T>(st, R, rb_of(S), n, S.sM.sptr, S.sM.col, S.sM.ocol,
                         mass_sell_values<T>(S), mass_sell_index<T>(S), mass_sell_table<T>(S), S.vtM.m, W.tmp, n,
                         nullptr, W.tmp2, n);
    schur_solve_t<T>(S, W.tmp2, W.h2);
    k_scatter_half<T><<<grid(nblk(n), R), kBlock, 0, st>>>(n, W.h2, w + n, len);
}

void narrow(Solver &S, int n, const double2 *a, float2 *b)
{
    k_narrow_pairs<<<grid(nblk(n), S.nrun), kBlock, 0, S.stream>>>(n, a, b);
}

void widen(Solver &S, int n, const float2 *a, double2 *b)
{
    k_widen_pairs<<<grid(nblk(n), S.nrun), kBlock, 0, S.stream>>>(n, a, b);
}

float *narrow_copy(Pool &pool, hipStream_t st, const double *a, long n)
{
    if (!a || n <= 0)
        return nullptr;
    float *b = pool.get<float>(n);
    k_narrow<<<nblk(n), kBlock, 0, st>>>(n, a, b);
    CHM_HIP(hipGetLastError());
    return b;
}

// FP32 values of one matrix: only the layout its kernels read
void narrow_matrix(Pool &pool, hipStream_t st, const Csr &C, const Sell &Sl, int gs, float *&fs,
                   float *&fc)
{
    if (gs == 0)
        fs = narrow_copy(pool, st, Sl.val, (long)Sl.stored);
    else
        fc = narrow_copy(pool, st, C.v, (long)C.nnz);
}

void narrow_hierarchy(Solver &S, Hierarchy &H)
{
    Pool &pool = S.pool;
    hipStream_t st = S.stream;
    for (int l = 0; l < H.nlev; ++l) {
        Level &L = H.lev[l];
        const size_t len = (size_t)S.nb * L.n;
        H.fx[l] = pool.get<float2>(len);
        H.fxt[l] = pool.get<float2>(len);
        H.fb[l] = pool.get<float2>(len);
        H.fr[l] = pool.get<float2>(len);
        // A on every level: the fine one also serves the inner CG and the
        // stationary cycles when it is the coarsest
        narrow_matrix(pool, st, L.A, L.sA, L.gsA, L.fA_s, L.fA_c);
        if (L.vtA.m > 0)
            L.vtA.ftab = narrow_copy(pool, st, L.vtA.tab, (long)L.vtA.m);
        if (l == H.nlev - 1)
            break;   // the coarsest level solves with its FP64 inverse
        narrow_matrix(pool, st, L.P, L.sP, L.gsP, L.fP_s, L.fP_c);
        narrow_matrix(pool, st, L.R, L.sR, L.gsR, L.fR_s, L.fR_c);
        if (L.RR.nnz > 0)
            L.fRR_c = narrow_copy(pool, st, L.RR.v, (long)L.RR.nnz);
        if (L.AM.nnz > 0)
            L.fAM_c = narrow_copy(pool, st, L.AM.v, (long)L.AM.nnz);
        L.fdinv = narrow_copy(pool, st, L.dinv, L.n);
    }
}

// ------------------------------------------------------------------ V-cycle contraction
// SplitMix64 (Steele, Lea and Flood 2014): output for counter i of stream 0
__device__ inline uint64_t mix64(uint64_t i)
{
    uint64_t z = (i + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// start vector of the power iteration: species s of row i takes counter
// 2^32 + 2 i + s, mapped to [-1, 1) through its top 53 bits
__global__ void __launch_bounds__(kBlock) k_seed_pairs(int n, double2 *e)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const uint64_t c = (1ull << 32) + 2ull * (uint64_t)i;
    const double u0 = (double)(mix64(c) >> 11) * 0x1.0p-53, u1 = (double)(mix64(c + 1) >> 11) * 0x1.0p-53;
    e[i] = d2(2.0 * u0 - 1.0, 2.0 * u1 - 1.0);
}

__global__ void __launch_bounds__(kBlock) k_sub_pairs(int n, const double2 *__restrict__ z, double2 *e)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double2 a = e[i], b = z[i];
        e[i] = d2(a.x - b.x, a.y - b.y);
    }
}

}  // namespace

// Contraction of one FP64 V-cycle V of the As hierarchy in the As-norm: the
// power iteration e <- (I - V As) e from a seeded start, `iters` times, for
// both species' start vectors; returns the larger of the two ratios
// ||e_new||_As / ||e_old||_As of the last step (the symmetric V-cycle makes
// I - V As self-adjoint in that norm, so the ratio tends to its spectral
// radius from below).  Run 0's work vectors; synchronises the stream.
double vcycle_contraction(Solver &S, int iters)
{
    Hierarchy &H = S.hA;
    const int n = H.lev[0].n, G = red_blocks(n);
    hipStream_t st = S.stream;
    S.nrun = 1;
    double2 *e = S.w64.tmp, *q = S.w64.tmp2, *z = S.w64.mr;
    k_seed_pairs<<<nblk(n), kBlock, 0, st>>>(n, e);
    std::vector<double2> part(G);
    double prev[2] = {0.0, 0.0}, rho[2] = {0.0, 0.0};
    for (int it = 0; it <= iters; ++it) {
        spmv_op<SP_SET, double>(st, 1, 1, H.lev[0].viewA<double>(), e, nullptr, q);
        k_dot<double><<<G, kBlock, 0, st>>>(n, e, q, slot(S, kSlotRz));
        CHM_HIP(hipMemcpyAsync(part.data(), slot(S, kSlotRz), sizeof(double2) * G,
                               hipMemcpyDeviceToHost, st));
        CHM_HIP(hipStreamSynchronize(st));
        double a[2] = {0.0, 0.0};
        for (int g = 0; g < G; ++g) {
            a[0] += part[g].x;
            a[1] += part[g].y;
        }
        for (int s = 0; s < 2; ++s) {
            if (it > 0)
                rho[s] = prev[s] > 0.0 ? std::sqrt(std::max(a[s], 0.0) / prev[s]) : 0.0;
            prev[s] = a[s];
        }
        if (it == iters)
            break;
        vcycle_level<double>(S, H, 0, q, z);
        k_sub_pairs<<<nblk(n), kBlock, 0, st>>>(n, z, e);
    }
    CHM_HIP(hipGetLastError());
    return std::max(rho[0], rho[1]);
}

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
    CHM_HIP(hipEventRecord(T.ev[T.used++], S.stream));
}

// work vectors of both precisions (FP32 ones and FP32 matrix copies only for
// the mixed-precision preconditioner); after amg_build of both hierarchies
void prec_setup(Solver &S)
{
    Pool &p = S.pool;
    const size_t n = S.nv, nb = S.nb;   // every work vector holds all runs
    Work<double> &D = S.w64;
    D.pcg_r = p.get<double2>(nb * n);
    D.pcg_z = p.get<double2>(nb * n);
    D.pcg_d = p.get<double2>(nb * n);
    D.pcg_q = p.get<double2>(nb * n);
    D.tmp = p.get<double2>(nb * n);
    D.tmp2 = p.get<double2>(nb * n);
    D.mr = p.get<double2>(nb * n);
    D.me = p.get<double2>(nb * n);
    D.h1 = p.get<double2>(nb * n);
    D.h2 = p.get<double2>(nb * n);
    S.amg_act = p.get<int2>(nb);
    CHM_HIP(hipHostMalloc(reinterpret_cast<void **>(&S.hamg_act), nb * sizeof(int2),
                          hipHostMallocDefault));
    if (!S.mixed)
        return;
    Work<float> &F = S.w32;
    F.pcg_r = p.get<float2>(nb * n);
    F.pcg_z = p.get<float2>(nb * n);
    F.pcg_d = p.get<float2>(nb * n);
    F.pcg_q = p.get<float2>(nb * n);
    F.tmp = p.get<float2>(nb * n);
    F.tmp2 = p.get<float2>(nb * n);
    F.mr = p.get<float2>(nb * n);
    F.me = p.get<float2>(nb * n);
    F.h1 = p.get<float2>(nb * n);
    F.h2 = p.get<float2>(nb * n);
    F.vin = p.get<float2>(2 * nb * n);
    F.wout = p.get<float2>(2 * nb * n);
    S.fsM = narrow_copy(p, S.stream, S.sM.val, (long)S.sM.stored);
    if (S.vtM.m > 0)
        S.vtM.ftab = narrow_copy(p, S.stream, S.vtM.tab, (long)S.vtM.m);
    narrow_hierarchy(S, S.hM);
    narrow_hierarchy(S, S.hA);
    CHM_HIP(hipStreamSynchronize(S.stream));
}

void vcycle(Solver &S, int hier, const double2 *b, double2 *x)
{
    Hierarchy &H = hier == 0 ? S.hM : S.hA;
    if (!S.mixed) {
        vcycle_level<double>(S, H, 0, b, x);
        return;
    }
    const int n = H.lev[0].n;
    narrow(S, n, b, S.w32.vin);
    vcycle_level<float>(S, H, 0, S.w32.vin, S.w32.wout);
    widen(S, n, S.w32.wout, x);
}

void schur_solve(Solver &S, const double2 *b, double2 *x)
{
    if (!S.mixed) {
        schur_solve_t<double>(S, b, x);
        return;
    }
    const int n = S.nv;
    narrow(S, n, b, S.w32.vin);
    schur_solve_t<float>(S, S.w32.vin, S.w32.wout);
    widen(S, n, S.w32.wout, x);
}

void apply_prec(Solver &S, const double2 *v, double2 *w)
{
    if (!S.mixed) {
        apply_prec_t<double>(S, v, w);
        return;
    }
    const int len = 2 * S.nv;
    narrow(S, len, v, S.w32.vin);
    apply_prec_t<float>(S, S.w32.vin, S.w32.wout);
    widen(S, len, S.w32.wout, w);
}

void apply_prec32(Solver &S, const double2 *v, float2 *w, bool narrowed)
{
    if (!narrowed)
        narrow(S, 2 * S.nv, v, S.w32.vin);
    apply_prec_t<float>(S, S.w32.vin, w);
}

}  // namespace chm
