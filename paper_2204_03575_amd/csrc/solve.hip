// Per-time-step solve on the GPU: right-hand side, the saddle-point operator
// of eq. saddle_point_system, and right-preconditioned flexible GMRES with
// classical Gram-Schmidt applied twice and Givens rotations kept on the
// device, preconditioned by Algorithm 1 (prec.hip).  Both species run through
// every kernel together (pair vectors), each with its own scalars,
// convergence flag and iteration count.  All of it is FP64.
#include <chrono>
#include <cmath>

#include "device_util.h"

namespace chm {

namespace {

// a pair vector entry as FP64 (an FP32 entry converts exactly)
__device__ inline double2 ld2(const double2 *p, long i) { return p[i]; }
__device__ inline double2 ld2(const float2 *p, long i)
{
    const float2 v = p[i];
    return d2((double)v.x, (double)v.y);
}

// ------------------------------------------------------------------ saddle-point operator
// y0 = M x0 + t K x1; y1 = t K x0 - te M x1 (per species t, te)
// A row is taken kSellUnroll entries at a time: every column and value load of
// the group, then every gather, then the products in column order (slots past
// the slice width repeat its last column with zero values).  U8: every slice
// of the pattern is at most kSellUnroll wide (2D meshes), so a row is one group.
struct SaddleEnt {
    int c[kSellUnroll];
    double am[kSellUnroll], ak[kSellUnroll];
};

// entries k0, ..., k0 + kSellUnroll - 1 of the row (k0 < width)
template <class I, class VA>
__device__ inline void saddle_load(int base, int width, int lane, int row, const I *__restrict__ col,
                                   const VA &vm, const VA &vk, SaddleEnt &e, int k0 = 0)
{
#pragma unroll
    for (int k = 0; k < kSellUnroll; ++k) {
        const int kk = k0 + k;
        const int idx = base + (kk < width ? kk : width - 1) * kSlice + lane;
        e.c[k] = sell_col(col, idx, row);
        const double vmk = vm[idx], vkk = vk[idx];
        e.am[k] = kk < width ? vmk : 0.0;
        e.ak[k] = kk < width ? vkk : 0.0;
    }
}

// y0 = M x0 + t K x1, y1 = t K x0 - te M x1 from the four row products
__device__ inline void saddle_combine(double m0x, double m0y, double k1x, double k1y, double k0x,
                                      double k0y, double m1x, double m1y, double2 t, double2 te,
                                      double2 &y0, double2 &y1)
{
    y0 = d2(fmad(t.x, k1x, m0x), fmad(t.y, k1y, m0y));
    y1 = d2(fmad(t.x, k0x, -(te.x * m1x)), fmad(t.y, k0y, -(te.y * m1y)));
}

// the four row products (M x0, K x1, K x0, M x1 per species), continued over
// one group of entries in column order
struct SaddleAcc {
    double m0x = 0, m0y = 0, k1x = 0, k1y = 0, k0x = 0, k0y = 0, m1x = 0, m1y = 0;
};

__device__ inline void saddle_acc(const SaddleEnt &e, const double2 *x0, const double2 *x1,
                                  SaddleAcc &a)
{
#pragma unroll
    for (int k = 0; k < kSellUnroll; ++k) {
        a.m0x = fmad(e.am[k], x0[k].x, a.m0x);
        a.m0y = fmad(e.am[k], x0[k].y, a.m0y);
        a.k1x = fmad(e.ak[k], x1[k].x, a.k1x);
        a.k1y = fmad(e.ak[k], x1[k].y, a.k1y);
        a.k0x = fmad(e.ak[k], x0[k].x, a.k0x);
        a.k0y = fmad(e.ak[k], x0[k].y, a.k0y);
        a.m1x = fmad(e.am[k], x1[k].x, a.m1x);
        a.m1y = fmad(e.am[k], x1[k].y, a.m1y);
    }
}

__device__ inline void saddle_dot(const SaddleEnt &e, const double2 *x0, const double2 *x1, double2 t,
                                  double2 te, double2 &y0, double2 &y1)
{
    SaddleAcc a;
    saddle_acc(e, x0, x1, a);
    saddle_combine(a.m0x, a.m0y, a.k1x, a.k1y, a.k0x, a.k0y, a.m1x, a.m1y, t, te, y0, y1);
}

template <class I, bool U8, class XT, class VA>
__device__ inline void saddle_row(int n, int row, SliceAt sl, const I *__restrict__ col,
                                  const VA &vm, const VA &vk, const XT *__restrict__ x, double2 t,
                                  double2 te, double2 &y0, double2 &y1)
{
    const int lane = row % kSlice, base = sl.base, width = sl.width;
    if (U8 && width > 0) {
        SaddleEnt e;
        saddle_load<I, VA>(base, width, lane, row, col, vm, vk, e);
        double2 x0[kSellUnroll], x1[kSellUnroll];
#pragma unroll
        for (int k = 0; k < kSellUnroll; ++k) {
            x0[k] = ld2(x, e.c[k]);
            x1[k] = ld2(x, n + e.c[k]);
        }
        saddle_dot(e, x0, x1, t, te, y0, y1);
        return;
    }
    SaddleAcc a;
    for (int k0 = 0; k0 < width; k0 += kSellUnroll) {
        SaddleEnt e;
        saddle_load<I, VA>(base, width, lane, row, col, vm, vk, e, k0);
        double2 x0[kSellUnroll], x1[kSellUnroll];
#pragma unroll
        for (int k = 0; k < kSellUnroll; ++k) {
            x0[k] = ld2(x, e.c[k]);
            x1[k] = ld2(x, n + e.c[k]);
        }
        saddle_acc(e, x0, x1, a);
    }
    saddle_combine(a.m0x, a.m0y, a.k1x, a.k1y, a.k0x, a.k0y, a.m1x, a.m1y, t, te, y0, y1);
}

// per run, x and y advance by 2n; RB runs per lane (block row blockIdx.y),
// R in all: on U8 patterns the row's entries are loaded once for the RB runs
template <class I, bool U8, int RB, class XT, class VA>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 4)))
k_saddle(int n, int R, const int *__restrict__ sptr, const I *__restrict__ col, const VA vm0,
         const VA vk0, const XT *__restrict__ x, double2 *y, double2 t, double2 te)
{
    extern __shared__ __align__(8) unsigned char lds_tab[];
    using VS = typename Staged<VA>::type;
    const int row = xcd_block() * kBlock + threadIdx.x;
    const SliceAt sl = slice_at(sptr, row, n);   // in flight while the tables are staged
    VS vm, vk;
    Staged<VA>::stage2(vm0, vk0, lds_tab, vm, vk);
    if (row >= n)
        return;
    const int r0 = run0<RB>();
    const long len = 2l * n;
    if (U8 && RB > 1) {
        const int lane = row % kSlice, base = sl.base, width = sl.width;
        if (width > 0) {
            SaddleEnt e;
            saddle_load<I, VS>(base, width, lane, row, col, vm, vk, e);
            double2 x0[RB][kSellUnroll], x1[RB][kSellUnroll];
#pragma unroll
            for (int q = 0; q < RB; ++q)
                if (r0 + q < R) {
                    const XT *xr = x + (r0 + q) * len;
#pragma unroll
                    for (int k = 0; k < kSellUnroll; ++k) {
                        x0[q][k] = ld2(xr, e.c[k]);
                        x1[q][k] = ld2(xr, n + e.c[k]);
                    }
                }
#pragma unroll
            for (int q = 0; q < RB; ++q)
                if (r0 + q < R) {
                    double2 y0, y1;
                    saddle_dot(e, x0[q], x1[q], t, te, y0, y1);
                    double2 *yr = y + (r0 + q) * len;
                    yr[row] = y0;
                    yr[n + row] = y1;
                }
            return;
        }
    }
    for (int q = 0; q < RB; ++q)
        if (RB == 1 || r0 + q < R) {
            double2 y0, y1;
            saddle_row<I, U8, XT, VS>(n, row, sl, col, vm, vk, x + (r0 + q) * len, t, te, y0, y1);
            double2 *yr = y + (r0 + q) * len;
            yr[row] = y0;
            yr[n + row] = y1;
        }
}

// y = b - A x over a grid-stride loop, and partial sums of |y1|^2 + w2 |y2|^2
// per species (y1, y2: the two block rows; w2 = 1 gives the 2-norm; per run:
// vectors advance by 2n, part by one run's slots)
template <class I, bool U8, class VA>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 4)))
k_saddle_resid(int n, const int *__restrict__ sptr, const I *__restrict__ col, const VA vm0,
               const VA vk0,
                                                         const double2 *__restrict__ x,
                                                         const double2 *__restrict__ b, double2 *y,
                                                         double2 t, double2 te, double2 *part,
                                                         double w2)
{
    __shared__ double2 sh[kBlock / 64];
    extern __shared__ __align__(8) unsigned char lds_tab[];
    using VS = typename Staged<VA>::type;
    VS vm, vk;
    Staged<VA>::stage2(vm0, vk0, lds_tab, vm, vk);
    x = run_at(x, 2l * n);
    b = run_at(b, 2l * n);
    y = run_at(y, 2l * n);
    part = run_at(part, kSlotStride);
    double2 nrm = d2(0.0, 0.0);
    for (int row = blockIdx.x * kBlock + threadIdx.x; row < n; row += gridDim.x * kBlock) {
        double2 y0, y1;
        saddle_row<I, U8, double2, VS>(n, row, slice_at(sptr, row, n), col, vm, vk, x, t, te, y0, y1);
        const double2 b0 = b[row], b1 = b[n + row];
        y0 = d2(b0.x - y0.x, b0.y - y0.y);
        y1 = d2(b1.x - y1.x, b1.y - y1.y);
        nrm.x += y0.x * y0.x + w2 * (y1.x * y1.x);
        nrm.y += y0.y * y0.y + w2 * (y1.y * y1.y);
        y[row] = y0;
        y[n + row] = y1;
    }
    const double2 s = block_sum(nrm, sh);
    if (threadIdx.x == 0)
        part[blockIdx.x] = s;
}

// ------------------------------------------------------------------ Gram-Schmidt passes
// MODE 0: partials of V_i . w;  MODE 1: w -= sum_i V_i h[i] with the
// finalised MODE-0 results h, then partials of V_i . w;  MODE 2: the same
// update with the MODE-1 results and, in the same loop, partials of w . w.  All per species;
// len = 2n.  The grid (up to kGsBlocks blocks per run) keeps several blocks
// per CU.  The Krylov vectors are [index][run][len] (index stride ks = runs
// len); per run, w advances by len, h by hs and the partials by ps.
constexpr int kChunk = 4;

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_gs(int len, long ks, const double2 *__restrict__ V,
                                               int nvec, double2 *w, const double2 *__restrict__ hin,
                                               long hs, double2 *part, long ps)
{
    __shared__ double2 sh[kBlock / 64];
    __shared__ double2 h[kMaxRestart + 1];
    const int G = gridDim.x;
    const int start = blockIdx.x * kBlock + threadIdx.x, stride = G * kBlock;
    V = run_at(V, len);
    w = run_at(w, len);
    hin = run_at(hin, hs);
    part = run_at(part, ps);
    double2 nrm = d2(0.0, 0.0);   // MODE 2: w . w of the updated elements, in element order
    if (MODE > 0) {
        for (int v = threadIdx.x; v < nvec; v += kBlock)
            h[v] = hin[v];
        __syncthreads();
        for (int i = start; i < len; i += stride) {
            double2 wv = w[i];
            for (int v = 0; v < nvec; ++v) {
                const double2 hv = h[v], vv = V[(size_t)v * ks + i];
                wv.x = fmad(-hv.x, vv.x, wv.x);
                wv.y = fmad(-hv.y, vv.y, wv.y);
            }
            w[i] = wv;
            if (MODE == 2) {
                nrm.x = fmad(wv.x, wv.x, nrm.x);
                nrm.y = fmad(wv.y, wv.y, nrm.y);
            }
        }
    }
    if (MODE == 2) {
        const double2 s = block_sum(nrm, sh);
        if (threadIdx.x == 0)
            part[blockIdx.x] = s;
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
                    const double2 vv = V[(size_t)(v0 + c) * ks + i];
                    acc[c].x = fmad(vv.x, wv.x, acc[c].x);
                    acc[c].y = fmad(vv.y, wv.y, acc[c].y);
                }
            }
        }
        for (int c = 0; c < kChunk && v0 + c < nvec; ++c) {
            const double2 s = block_sum(acc[c], sh);
            if (threadIdx.x == 0)
                part[(size_t)(v0 + c) * G + blockIdx.x] = s;
        }
    }
}

// MODE 1 for nvec <= NV basis vectors with the thread's V_i entries held in
// registers: each element's entries are loaded once, for the update and for
// the partials, which the MODE-1 kernel above loads twice.  The update runs
// over i = 0, 1, ... and each partial over the thread's elements in the same
// order as there, so the results are bitwise the same.
template <int NV>
__global__ void __launch_bounds__(kBlock) k_gs1_reg(int len, long ks, const double2 *__restrict__ V,
                                                    int nvec, double2 *w,
                                                    const double2 *__restrict__ hin, long hs,
                                                    double2 *part, long ps)
{
    __shared__ double2 sh[kBlock / 64];
    __shared__ double2 h[NV];
    const int G = gridDim.x;
    const int start = blockIdx.x * kBlock + threadIdx.x, stride = G * kBlock;
    V = run_at(V, len);
    w = run_at(w, len);
    hin = run_at(hin, hs);
    part = run_at(part, ps);
    for (int v = threadIdx.x; v < nvec; v += kBlock)
        h[v] = hin[v];
    __syncthreads();
    double2 acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        acc[v] = d2(0.0, 0.0);
#pragma unroll 1
    for (int i = start; i < len; i += stride) {
        double2 vv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v)   // slots past nvec repeat the last vector; unused
            vv[v] = V[(size_t)(v < nvec ? v : nvec - 1) * ks + i];
        double2 wv = w[i];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (v < nvec) {
                const double2 hv = h[v];
                wv.x = fmad(-hv.x, vv[v].x, wv.x);
                wv.y = fmad(-hv.y, vv[v].y, wv.y);
            }
        }
        w[i] = wv;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            acc[v].x = fmad(vv[v].x, wv.x, acc[v].x);
            acc[v].y = fmad(vv[v].y, wv.y, acc[v].y);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nvec) {
            const double2 t = block_sum(acc[v], sh);
            if (threadIdx.x == 0)
                part[(size_t)v * G + blockIdx.x] = t;
        }
    }
}

// MODE 1 for more than NV basis vectors: the update runs over every vector,
// the first NV held in registers for their dots as in k_gs1_reg; the dots of
// the others take a second sweep over the updated w (each thread reads back
// its own elements) in groups of kChunk.  The update and every partial follow
// the orders of k_gs<1>, so the results are bitwise the same, and the first
// NV vectors are read once instead of twice.
template <int NV>
__global__ void __launch_bounds__(kBlock) k_gs1_split(int len, long ks,
                                                      const double2 *__restrict__ V, int nvec,
                                                      double2 *w, const double2 *__restrict__ hin,
                                                      long hs, double2 *part, long ps)
{
    __shared__ double2 sh[kBlock / 64];
    __shared__ double2 h[kMaxRestart + 1];
    const int G = gridDim.x;
    const int start = blockIdx.x * kBlock + threadIdx.x, stride = G * kBlock;
    V = run_at(V, len);
    w = run_at(w, len);
    hin = run_at(hin, hs);
    part = run_at(part, ps);
    for (int v = threadIdx.x; v < nvec; v += kBlock)
        h[v] = hin[v];
    __syncthreads();
    double2 acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        acc[v] = d2(0.0, 0.0);
#pragma unroll 1
    for (int i = start; i < len; i += stride) {
        double2 vv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v)   // nvec > NV: every slot is a basis vector
            vv[v] = V[(size_t)v * ks + i];
        double2 wv = w[i];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double2 hv = h[v];
            wv.x = fmad(-hv.x, vv[v].x, wv.x);
            wv.y = fmad(-hv.y, vv[v].y, wv.y);
        }
        for (int v = NV; v < nvec; ++v) {
            const double2 hv = h[v], x = V[(size_t)v * ks + i];
            wv.x = fmad(-hv.x, x.x, wv.x);
            wv.y = fmad(-hv.y, x.y, wv.y);
        }
        w[i] = wv;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            acc[v].x = fmad(vv[v].x, wv.x, acc[v].x);
            acc[v].y = fmad(vv[v].y, wv.y, acc[v].y);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double2 t = block_sum(acc[v], sh);
        if (threadIdx.x == 0)
            part[(size_t)v * G + blockIdx.x] = t;
    }
    for (int v0 = NV; v0 < nvec; v0 += kChunk) {
        double2 a2[kChunk];
        for (int c = 0; c < kChunk; ++c)
            a2[c] = d2(0.0, 0.0);
        for (int i = start; i < len; i += stride) {
            const double2 wv = w[i];
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                if (v0 + c < nvec) {
                    const double2 vv = V[(size_t)(v0 + c) * ks + i];
                    a2[c].x = fmad(vv.x, wv.x, a2[c].x);
                    a2[c].y = fmad(vv.y, wv.y, a2[c].y);
                }
            }
        }
        for (int c = 0; c < kChunk && v0 + c < nvec; ++c) {
            const double2 t = block_sum(a2[c], sh);
            if (threadIdx.x == 0)
                part[(size_t)(v0 + c) * G + blockIdx.x] = t;
        }
    }
}

// ------------------------------------------------------------------ delayed reorthogonalisation
// With ortho = CHM_ORTHO_DCGS2, the second Gram-Schmidt pass of each basis
// vector runs in the iteration after it.  In iteration j, V_0..V_{j-1} are
// final, V_j holds u_j (the previous w after one projection, not
// normalised; the preconditioner took u_j) and V_{j+1} holds w = A z_j.  One
// sweep forms the dot products of V_0..V_j with u_j and with w.  The second
// makes v_j final, v_j = (u_j - sum_k s_k V_k) / nu with s_k = V_k . u_j and
// nu^2 = u_j . u_j - |s|^2 (the second pass and the normalisation at once),
// projects w on V_0..V_{j-1} and on the final v_j, and sums |w|^2 of the
// result.  At j = 0, V_0 is the normalised residual, already final: s is
// empty and nu = 1.  FGMRES takes any vector as the preconditioner's input,
// so the stored z_j = Prec(u_j) define the solution space as they are.

// dot products of V_0..V_j with u = V_j (partial rows 0..j) and with w
// (rows j+1..2j+1), C basis vectors per sweep; per run as k_gs
template <int C>
__global__ void __launch_bounds__(kBlock) k_dgs_dots(int len, long ks,
                                                     const double2 *__restrict__ V, int j,
                                                     const double2 *__restrict__ w,
                                                     double2 *part, long ps)
{
    __shared__ double2 sh[kBlock / 64];
    const int G = gridDim.x;
    const int start = blockIdx.x * kBlock + threadIdx.x, stride = G * kBlock;
    V = run_at(V, len);
    w = run_at(w, len);
    part = run_at(part, ps);
    const double2 *u = V + (size_t)j * ks;
    for (int v0 = 0; v0 <= j; v0 += C) {
        double2 au[C], aw[C];
        for (int c = 0; c < C; ++c) {
            au[c] = d2(0.0, 0.0);
            aw[c] = d2(0.0, 0.0);
        }
        for (int i = start; i < len; i += stride) {
            const double2 uv = u[i], wv = w[i];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (v0 + c <= j) {
                    const double2 vv = V[(size_t)(v0 + c) * ks + i];
                    au[c].x = fmad(vv.x, uv.x, au[c].x);
                    au[c].y = fmad(vv.y, uv.y, au[c].y);
                    aw[c].x = fmad(vv.x, wv.x, aw[c].x);
                    aw[c].y = fmad(vv.y, wv.y, aw[c].y);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {   // constant trip count: the sums stay in registers
            if (v0 + c <= j) {
                const double2 a = block_sum(au[c], sh);
                if (threadIdx.x == 0)
                    part[(size_t)(v0 + c) * G + blockIdx.x] = a;
                const double2 b = block_sum(aw[c], sh);
                if (threadIdx.x == 0)
                    part[(size_t)(j + 1 + v0 + c) * G + blockIdx.x] = b;
            }
        }
    }
}

// The delayed pass's scalars from the finished dot products h (rows as
// k_dgs_dots writes them), per species: nu, 1 / nu and the component of w
// along the final v_j, (w . u - s . t) / nu with t_k = V_k . w.  A zero u (a
// species no longer iterating) gives nu = 0 and zeros.  The update sweep and
// the Givens step both call this on the same values, so they agree bitwise.
struct DgsCoef {
    double2 nu, inv, hjj;
};

__device__ inline double dgs_one(double a, double b, double ss, double st, double &nu, double &inv)
{
    const double nu2 = a - ss;
    nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
    inv = nu > 0.0 ? 1.0 / nu : 0.0;
    return nu > 0.0 ? (b - st) / nu : 0.0;
}

__device__ inline DgsCoef dgs_coef(const double2 *h, int j)
{
    DgsCoef r;
    if (j == 0) {
        r.nu = d2(1.0, 1.0);
        r.inv = d2(1.0, 1.0);
        r.hjj = h[1];
        return r;
    }
    double2 ss = d2(0.0, 0.0), st = d2(0.0, 0.0);
    for (int k = 0; k < j; ++k) {
        const double2 sk = h[k], tk = h[j + 1 + k];
        ss.x = fmad(sk.x, sk.x, ss.x);
        ss.y = fmad(sk.y, sk.y, ss.y);
        st.x = fmad(sk.x, tk.x, st.x);
        st.y = fmad(sk.y, tk.y, st.y);
    }
    const double2 a = h[j], b = h[2 * j + 1];
    r.hjj.x = dgs_one(a.x, b.x, ss.x, st.x, r.nu.x, r.inv.x);
    r.hjj.y = dgs_one(a.y, b.y, ss.y, st.y, r.nu.y, r.inv.y);
    return r;
}

// v_j final (written over u_j, j > 0) and w -= sum_{k<j} t_k V_k + h_jj v_j,
// with partials of |w|^2 (per run: hin advances by hs, part by ps).  The
// projected w stays unnormalised: it is u_{j+1}, which the next iteration's
// sweep normalises together with its second pass.  A species no longer
// iterating gets w = 0.  With w32, the FP32 copy the FP32 preconditioner
// takes next: w times 1 / |u_j| (the previous |w|, 1 at j = 0), so its
// scale stays near one however far the basis norms drift.
__global__ void __launch_bounds__(kBlock) k_dgs_update(int len, long ks, double2 *V, int j,
                                                       double2 *w,
                                                       const double2 *__restrict__ hin, long hs,
                                                       double2 *part, long ps,
                                                       const Ctl *__restrict__ c, float2 *w32)
{
    __shared__ double2 sh[kBlock / 64];
    __shared__ double2 sc[kMaxRestart], tc[kMaxRestart];
    __shared__ DgsCoef cf;
    const int G = gridDim.x;
    const int start = blockIdx.x * kBlock + threadIdx.x, stride = G * kBlock;
    V = run_at(V, len);
    w = run_at(w, len);
    hin = run_at(hin, hs);
    part = run_at(part, ps);
    for (int k = threadIdx.x; k < j; k += kBlock) {
        sc[k] = hin[k];
        tc[k] = hin[j + 1 + k];
    }
    if (threadIdx.x == 0)
        cf = dgs_coef(hin, j);
    __syncthreads();
    const DgsCoef f = cf;
    c += blockIdx.y;
    const double on0 = c->active[0] ? 1.0 : 0.0, on1 = c->active[1] ? 1.0 : 0.0;
    const double sc0 = j == 0 ? 1.0 : (c->hn[0] > 0.0 ? 1.0 / c->hn[0] : 0.0);
    const double sc1 = j == 0 ? 1.0 : (c->hn[1] > 0.0 ? 1.0 / c->hn[1] : 0.0);
    w32 = run_at(w32, len);
    double2 *u = V + (size_t)j * ks;
    double2 nrm = d2(0.0, 0.0);
    for (int i = start; i < len; i += stride) {
        double2 uv = u[i], wv = w[i];
        for (int k = 0; k < j; ++k) {
            const double2 vv = V[(size_t)k * ks + i], sk = sc[k], tk = tc[k];
            uv.x = fmad(-sk.x, vv.x, uv.x);
            uv.y = fmad(-sk.y, vv.y, uv.y);
            wv.x = fmad(-tk.x, vv.x, wv.x);
            wv.y = fmad(-tk.y, vv.y, wv.y);
        }
        uv.x *= f.inv.x;
        uv.y *= f.inv.y;
        wv.x = on0 * fmad(-f.hjj.x, uv.x, wv.x);
        wv.y = on1 * fmad(-f.hjj.y, uv.y, wv.y);
        if (j > 0)
            u[i] = uv;
        w[i] = wv;
        if (w32)
            w32[i] = make_float2((float)(wv.x * sc0), (float)(wv.y * sc1));
        nrm.x = fmad(wv.x, wv.x, nrm.x);
        nrm.y = fmad(wv.y, wv.y, nrm.y);
    }
    const double2 t = block_sum(nrm, sh);
    if (threadIdx.x == 0)
        part[blockIdx.x] = t;
}

// out[v] = sum of the G partials of vector v; block v handles vector v
// (thread t adds g = t, t + 256, ... in order, then a fixed block tree);
// per run, part advances by ps and out by hs
__global__ void __launch_bounds__(kBlock) k_finish(const double2 *__restrict__ part, long ps, int G,
                                                  double2 *out, long hs)
{
    __shared__ double2 sh[kBlock / 64];
    part = run_at(part, ps);
    out = run_at(out, hs);
    const int v = blockIdx.x;
    double2 s = d2(0.0, 0.0);
    for (int g = threadIdx.x; g < G; g += kBlock) {
        const double2 p = part[(size_t)v * G + g];
        s.x += p.x;
        s.y += p.y;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0)
        out[v] = s;
}

// ------------------------------------------------------------------ FGMRES control (one block per run)
// The control kernels run one block per run (blockIdx.y); c points at run
// 0's control block.

// ||b||^2 from partials; tol = rtol ||b|| per species
__global__ void __launch_bounds__(kBlock) k_tol(Ctl *c, const double2 *__restrict__ part, int G,
                                                double rtol)
{
    __shared__ double2 r[1];
    c += blockIdx.y;
    reduce_parts(run_at(part, kSlotStride), 1, G, r);
    if (threadIdx.x < 2) {
        const int s = threadIdx.x;
        const double nb = s == 0 ? r[0].x : r[0].y;
        const double bn = sqrt(nb);
        c->nrm[s] = nb;
        c->bnorm[s] = bn;
        c->tol[s] = rtol * bn;
    }
}

// squared residual norms from partials
__global__ void __launch_bounds__(kBlock) k_nrm(Ctl *c, const double2 *__restrict__ part, int G)
{
    __shared__ double2 r[1];
    c += blockIdx.y;
    reduce_parts(run_at(part, kSlotStride), 1, G, r);
    if (threadIdx.x < 2)
        c->nrm[threadIdx.x] = threadIdx.x == 0 ? r[0].x : r[0].y;
}

// per-species flags of every run, from the host (2 per run)
struct Flags {
    int a[2 * kMaxRuns];
};

// start of a cycle: g = (||r||, 0, ...), active flags from the host, k = 0
__global__ void k_cycle_init(Ctl *c, Flags act)
{
    const int s = threadIdx.x;
    if (s >= 2)
        return;
    c += blockIdx.y;
    c->active[s] = act.a[2 * blockIdx.y + s];
    c->k[s] = 0;
    c->g[s][0] = sqrt(c->nrm[s]);
    c->beta[s] = c->g[s][0];
}

// keep only the species the host still lets iterate
__global__ void k_deactivate(Ctl *c, Flags act)
{
    const int s = threadIdx.x;
    if (s < 2) {
        c += blockIdx.y;
        c->active[s] = c->active[s] && act.a[2 * blockIdx.y + s];
    }
}

// the heads of the runs' control blocks, back to back, written straight into
// pinned (coherent) host memory through its device address; the host reads
// them after synchronising the stream
__global__ void k_pack_heads(const Ctl *__restrict__ c, int *out)
{
    constexpr int words = (int)(kCtlHead / sizeof(int));
    const int *src = reinterpret_cast<const int *>(c + blockIdx.y);
    for (int i = threadIdx.x; i < words; i += blockDim.x)
        out[blockIdx.y * words + i] = src[i];
    __threadfence_system();
}

// the counters of a step: clamps, non-finite flag, starts used, vertices outside [0, 1]
__global__ void k_ctl_reset(Ctl *c)
{
    c += blockIdx.y;
    if (threadIdx.x == 0) {
        c->clamped = 0;
        c->nan = 0;
        c->guess_used[0] = 0;
        c->guess_used[1] = 0;
        c->outside = 0;
    }
}

// vertices of the state (per run: phi is the first half of a block vector of
// 2n) whose phi_p, phi_n or phi_s = 1 - phi_p - phi_n lies outside [0, 1],
// added to the run's count (integer sums, so the order does not matter)
__global__ void __launch_bounds__(kBlock) k_outside(int n, const double2 *__restrict__ x, Ctl *c)
{
    __shared__ int cnt;
    if (threadIdx.x == 0)
        cnt = 0;
    __syncthreads();
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const double2 v = run_at(x, 2l * n)[i];
        const double s = 1.0 - v.x - v.y;
        if (v.x < 0.0 || v.x > 1.0 || v.y < 0.0 || v.y > 1.0 || s < 0.0 || s > 1.0)
            atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt)
        atomicAdd(&c[blockIdx.y].outside, cnt);
}

// v0 = r / ||r|| for active species, 0 otherwise (per run, r and v advance by len)
__global__ void __launch_bounds__(kBlock) k_scale_first(int len, const double2 *__restrict__ r,
                                                        double2 *v, const Ctl *__restrict__ c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    c += blockIdx.y;
    const double s0 = (c->active[0] && c->nrm[0] > 0.0) ? 1.0 / sqrt(c->nrm[0]) : 0.0;
    const double s1 = (c->active[1] && c->nrm[1] > 0.0) ? 1.0 / sqrt(c->nrm[1]) : 0.0;
    const double2 rv = run_at(r, len)[i];
    run_at(v, len)[i] = d2(rv.x * s0, rv.y * s1);
}

// Column j of the Hessenberg matrix from the two Gram-Schmidt passes, the
// previous rotations applied, a new rotation that zeroes H[j+1][j], the
// residual estimate |g[j+1]|, and the convergence test against tol.  Per
// run, h1 and h2 advance by hs and p3 by ps.
__global__ void __launch_bounds__(kBlock) k_givens(Ctl *c, int j, int m,
                                                   const double2 *__restrict__ h1,
                                                   const double2 *__restrict__ h2, long hs,
                                                   const double2 *__restrict__ p3, long ps, int G)
{
    // the column and the previous rotations are staged in LDS by the whole
    // block, so the sequential rotation loop below touches no global memory
    __shared__ double2 nn[1];
    __shared__ double col[2][kMaxRestart + 1], csl[2][kMaxRestart], snl[2][kMaxRestart];
    c += blockIdx.y;
    h1 = run_at(h1, hs);
    h2 = run_at(h2, hs);
    p3 = run_at(p3, ps);
    for (int t = threadIdx.x; t < 2 * (j + 1); t += kBlock) {
        const int s = t / (j + 1), i = t % (j + 1);
        col[s][i] = s == 0 ? h1[i].x + h2[i].x : h1[i].y + h2[i].y;
    }
    for (int t = threadIdx.x; t < 2 * j; t += kBlock) {
        const int s = t / j, i = t % j;
        csl[s][i] = c->cs[s][i];
        snl[s][i] = c->sn[s][i];
    }
    reduce_parts(p3, 1, G, nn);   // ends with a block barrier
    const int s = threadIdx.x;
    if (s >= 2 || !c->active[s])
        return;
    double *H = c->H[s];
    double *cl = col[s];
    const double hn = sqrt(s == 0 ? nn[0].x : nn[0].y);
    c->hn[s] = hn;
    cl[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = cl[i], b = cl[i + 1];
        cl[i] = csl[s][i] * a + snl[s][i] * b;
        cl[i + 1] = -snl[s][i] * a + csl[s][i] * b;
    }
    for (int i = 0; i < j; ++i)
        H[i * m + j] = cl[i];
    const double a = cl[j], b = cl[j + 1];
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

// The Givens step of the delayed pass (ortho = CHM_ORTHO_DCGS2).  Making
// v_j final changes the column of the previous iteration: its entry |u_j|
// (the norm of w_{j-1} after one projection) becomes s_k along V_k and nu
// along v_j.
// That column is rotated again by the rotations before it and gets a new
// rotation; then column j (t_k, h_jj, |w|) is rotated, g is formed again from
// the cycle's |r| through every rotation, and the convergence test runs on
// |g[j+1]| as in k_givens.
__device__ inline void rotate_col(double *cl, int upto, const double *cs, const double *sn)
{
    for (int i = 0; i < upto; ++i) {
        const double a = cl[i], b = cl[i + 1];
        cl[i] = cs[i] * a + sn[i] * b;
        cl[i + 1] = -sn[i] * a + cs[i] * b;
    }
}

__device__ inline void new_rotation(double a, double b, double &cs, double &sn, double &rr)
{
    rr = sqrt(a * a + b * b);
    cs = 1.0;
    sn = 0.0;
    if (rr != 0.0) {
        cs = a / rr;
        sn = b / rr;
    }
}

__global__ void __launch_bounds__(kBlock) k_givens_d(Ctl *c, int j, int m,
                                                     const double2 *__restrict__ hin, long hs,
                                                     const double2 *__restrict__ p3, long ps, int G)
{
    // the dots, the previous rotations and the last raw column are staged in
    // LDS by the whole block, so the sequential loops below touch no global
    // memory; the results are written back at the end
    __shared__ double2 nn[1];
    __shared__ double2 hl[2 * (kMaxRestart + 1)];
    __shared__ double col[2][kMaxRestart + 1], hrl[2][kMaxRestart + 1];
    __shared__ double csl[2][kMaxRestart], snl[2][kMaxRestart], gl[2][kMaxRestart + 1];
    c += blockIdx.y;
    hin = run_at(hin, hs);
    p3 = run_at(p3, ps);
    for (int t = threadIdx.x; t < 2 * (j + 1); t += kBlock)
        hl[t] = hin[t];
    for (int t = threadIdx.x; t < 2 * (j + 1); t += kBlock) {
        const int s = t / (j + 1), i = t % (j + 1);
        hrl[s][i] = c->hlast[s][i];
    }
    for (int t = threadIdx.x; t < 2 * j; t += kBlock) {
        const int s = t / j, i = t % j;
        csl[s][i] = c->cs[s][i];
        snl[s][i] = c->sn[s][i];
    }
    reduce_parts(p3, 1, G, nn);   // ends with a block barrier
    const int s = threadIdx.x;
    if (s >= 2 || !c->active[s])
        return;
    const DgsCoef f = dgs_coef(hl, j);
    auto pick = [s](double2 v) { return s == 0 ? v.x : v.y; };
    double *H = c->H[s], *hr = hrl[s], *cs = csl[s], *sn = snl[s], *g = gl[s];
    double *cl = col[s];
    const double hn = sqrt(s == 0 ? nn[0].x : nn[0].y);
    double rr;
    if (j > 0) {
        // u_j is w_{j-1} after its one projection, unnormalised: its parts
        // s_k along V_k and nu along v_j are column j-1's corrections
        for (int k = 0; k < j; ++k)
            hr[k] += pick(hl[k]);
        hr[j] = pick(f.nu);
        for (int k = 0; k <= j; ++k)
            cl[k] = hr[k];
        rotate_col(cl, j - 1, cs, sn);
        for (int i = 0; i < j - 1; ++i)
            H[i * m + (j - 1)] = cl[i];
        new_rotation(cl[j - 1], cl[j], cs[j - 1], sn[j - 1], rr);
        H[(j - 1) * m + (j - 1)] = rr;
    }
    for (int k = 0; k < j; ++k)
        hr[k] = pick(hl[j + 1 + k]);
    hr[j] = pick(f.hjj);
    hr[j + 1] = hn;
    for (int k = 0; k <= j + 1; ++k)
        cl[k] = hr[k];
    rotate_col(cl, j, cs, sn);
    for (int i = 0; i < j; ++i)
        H[i * m + j] = cl[i];
    new_rotation(cl[j], cl[j + 1], cs[j], sn[j], rr);
    H[j * m + j] = rr;
    H[(j + 1) * m + j] = 0.0;
    g[0] = c->beta[s];
    for (int i = 0; i <= j; ++i) {
        const double gi = g[i];
        g[i] = cs[i] * gi;
        g[i + 1] = -sn[i] * gi;
    }
    for (int i = 0; i <= j + 1; ++i) {
        c->hlast[s][i] = hr[i];
        c->g[s][i] = g[i];
    }
    if (j > 0) {
        c->cs[s][j - 1] = cs[j - 1];
        c->sn[s][j - 1] = sn[j - 1];
    }
    c->cs[s][j] = cs[j];
    c->sn[s][j] = sn[j];
    c->hn[s] = hn;
    c->k[s] = j + 1;
    const double est = fabs(g[j + 1]);
    c->resest[s] = est;
    if (!isfinite(est) || !isfinite(hn)) {
        c->nan = 1;
        c->active[s] = 0;
    } else if (est <= c->tol[s] || hn == 0.0) {
        c->active[s] = 0;
    }
}

// v_{j+1} = w / ||w|| for species still active, 0 otherwise (per run, v advances by len)
// (with v32: also its FP32 copy, the input the FP32 preconditioner takes
// next, so that it need not narrow v_{j+1} itself)
__global__ void __launch_bounds__(kBlock) k_scale_next(int len, double2 *v, const Ctl *__restrict__ c,
                                                       float2 *v32)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    c += blockIdx.y;
    v = run_at(v, len);
    const double s0 = (c->active[0] && c->hn[0] > 0.0) ? 1.0 / c->hn[0] : 0.0;
    const double s1 = (c->active[1] && c->hn[1] > 0.0) ? 1.0 / c->hn[1] : 0.0;
    const double2 vv = v[i];
    const double2 out = d2(vv.x * s0, vv.y * s1);
    v[i] = out;
    if (v32)
        run_at(v32, len)[i] = make_float2((float)out.x, (float)out.y);
}

// back substitution of the rotated Hessenberg system, k[s] columns per species
__global__ void k_trisolve(Ctl *c, int m)
{
    const int s = threadIdx.x;
    if (s >= 2)
        return;
    c += blockIdx.y;
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

// x += sum_{i < kmax} Z_i y_i, per species (Z is [index][run][len], index
// stride ks; per run x advances by len)
// (Z in FP64, or in FP32 where the preconditioner computes in FP32: its
// results are FP32 values, which convert exactly)
template <class ZT>
__global__ void __launch_bounds__(kBlock) k_update_x(int len, long ks, double2 *x,
                                                     const ZT *__restrict__ Z, int kmax,
                                                     const Ctl *__restrict__ c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    c += blockIdx.y;
    x = run_at(x, len);
    Z = run_at(Z, len);
    double2 xv = x[i];
    for (int t = 0; t < kmax; ++t) {
        const double2 z = ld2(Z, (size_t)t * ks + i);
        xv.x = fmad(c->y[0][t], z.x, xv.x);
        xv.y = fmad(c->y[1][t], z.y, xv.y);
    }
    x[i] = xv;
}

__global__ void __launch_bounds__(kBlock) k_finite(int len, const double2 *__restrict__ x, Ctl *c)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    const double2 v = run_at(x, len)[i];
    if (!isfinite(v.x) || !isfinite(v.y))
        c[blockIdx.y].nan = 1;
}

// ------------------------------------------------------------------ right-hand side
struct Pot {
    int kind;
    double iNp, iNn, iNs, chi_pn, chi_ps, chi_ns, floor_;   // iN*: 1 / N*
};

__device__ inline double clog(double v, double fl, int &clamps)
{
    if (v < fl) {
        ++clamps;
        v = fl;
    }
    return log_pos(v);
}

// d f / d phi_p and d f / d phi_n with phi_s = 1 - phi_p - phi_n (paper Section 2,
// eq. logarithmicpotential; Section 4, eq. polynomial_potential)
__device__ inline void dpot(const Pot &P, double p, double q, double &fp, double &fq, int &clamps)
{
    const double s = 1.0 - p - q;
    if (P.kind == CHM_POT_FLORY_HUGGINS) {
        const double lp = clog(p, P.floor_, clamps), lq = clog(q, P.floor_, clamps);
        const double ls = clog(s, P.floor_, clamps);
        const double es = (ls + 1.0) * P.iNs;
        fp = (lp + 1.0) * P.iNp - es + P.chi_pn * q + P.chi_ps * (s - p) - P.chi_ns * q;
        fq = (lq + 1.0) * P.iNn - es + P.chi_pn * p - P.chi_ps * p + P.chi_ns * (s - q);
    } else if (P.kind == CHM_POT_POLYNOMIAL) {
        fp = 7.0 * p * q * q - 0.2 * s;
        fq = 7.0 * p * p * q - 0.2 * s;
    } else {
        fp = 0.0;
        fq = 0.0;
    }
}

// Per cell and corner a: sum over the quadrature of f'(phi_h) lambda_a (times
// |T| in the gather below), for every cell in one launch, stored at the
// slot's place pos[cell * NL + a] in the vertices' slot lists.  Per run: the
// state x (phi is its first half) advances by 2n, the slot values by
// `stored`, and the run has its own potential parameters and clamp counter.
template <int NL>
__global__ void __launch_bounds__(kBlock) k_rhs_cells(int ncell, const int *__restrict__ cells,
                                                      const double *__restrict__ qb,
                                                      const double *__restrict__ qw, int nq, int n,
                                                      const double2 *__restrict__ phi,
                                                      const Pot *__restrict__ pots,
                                                      const int *__restrict__ pos, long stored,
                                                      double2 *slot, Ctl *ctl)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell)
        return;
    phi = run_at(phi, 2l * n);
    slot = run_at(slot, stored);
    const Pot P = pots[blockIdx.y];
    int *clamped = &ctl[blockIdx.y].clamped;
    int vtx[NL];
    double2 ph[NL], acc[NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) {
        vtx[a] = cells[(size_t)c * NL + a];
        ph[a] = phi[vtx[a]];
        acc[a] = d2(0.0, 0.0);
    }
    int clamps = 0;
    for (int q = 0; q < nq; ++q) {
        double p = 0.0, r = 0.0;
#pragma unroll
        for (int a = 0; a < NL; ++a) {
            const double l = qb[q * NL + a];
            p += l * ph[a].x;
            r += l * ph[a].y;
        }
        double fp, fr;
        dpot(P, p, r, fp, fr, clamps);
        const double wq = qw[q];
#pragma unroll
        for (int a = 0; a < NL; ++a) {
            const double l = qb[q * NL + a];
            acc[a].x += wq * fp * l;
            acc[a].y += wq * fr * l;
        }
    }
#pragma unroll
    for (int a = 0; a < NL; ++a)
        slot[pos[(size_t)c * NL + a]] = acc[a];
    if (clamps)
        atomicAdd(clamped, clamps);
}

// f[v] = sum of |T| times the value of slot (T, v) over the cells T at v, in
// colour order (the vertex's slot list is sorted that way): the sum a scatter
// of one colour after the other forms, without a launch per colour.  The
// lists are SELL-64 (lane = vertex of the slice, entry k at sptr + 64 k), so
// the loads of a wave are contiguous; padding has slot 0 and value 0.  Per
// run: the slot values advance by `stored`, f by n.
template <int NL>
__global__ void __launch_bounds__(kBlock) k_rhs_gather(int n, const int *__restrict__ sptr,
                                                       const int *__restrict__ vslot,
                                                       const double *__restrict__ vol, long stored,
                                                       const double2 *__restrict__ slot, double2 *f)
{
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n)
        return;
    slot = run_at(slot, stored);
    const int sl = __builtin_amdgcn_readfirstlane(v / kSlice), lane = v % kSlice;
    const int base = sptr[sl], width = (sptr[sl + 1] - base) / kSlice;
    double2 s = d2(0.0, 0.0);
    constexpr int U = 8;
    for (int k0 = 0; k0 < width; k0 += U) {
        int e[U];
        double2 a[U];
        double vc[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int p = base + (k0 + k < width ? k0 + k : width - 1) * kSlice + lane;
            e[k] = vslot[p];
            a[k] = slot[p];
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
            vc[k] = vol[e[k] / NL];
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (k0 + k < width)
                s = d2(fmad(vc[k], a[k].x, s.x), fmad(vc[k], a[k].y, s.y));
    }
    run_at(f, (long)n)[v] = s;
}

// b1 = -(tau'/eps) f (per run: f advances by n, b1, the second half of the
// right-hand side, by 2n)
__global__ void __launch_bounds__(kBlock) k_rhs_second(int n, const double2 *__restrict__ f,
                                                       double2 *b1, double2 te)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const double2 v = run_at(f, (long)n)[i];
    run_at(b1, 2l * n)[i] = d2(-te.x * v.x, -te.y * v.y);
}

__global__ void __launch_bounds__(kBlock) k_zero(int n, double2 *v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        run_at(v, (long)n)[i] = d2(0.0, 0.0);
}

// solvent removed per run in this step (0: none)
struct Evap {
    double ds[kMaxRuns];
};

// solvent removal after a step: phi_i += ds phi_i / (phi_p + phi_n), equal
// halves if the sum is <= 0 (per run: the state advances by 2n)
__global__ void __launch_bounds__(kBlock) k_evaporate(int n, double2 *phi, Evap e)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const double ds = e.ds[blockIdx.y];
    if (ds == 0.0)
        return;
    phi = run_at(phi, 2l * n);
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

// ------------------------------------------------------------------ initial guess
// xg = x + (x - xh): linear extrapolation of the last increment (x = y_{n-1}, xh = y_{n-2})
__global__ void __launch_bounds__(kBlock) k_extrapolate(int len, const double2 *__restrict__ xh,
                                                        const double2 *__restrict__ x, double2 *xg)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= len)
        return;
    const double2 a = run_at(x, len)[i], h = run_at(xh, len)[i];
    run_at(xg, len)[i] = d2(a.x + (a.x - h.x), a.y + (a.y - h.y));
}

// Per species, the start with the smallest norm (first block row) among the previous
// state x (code 0), the linear extrapolation xl (code 1; may be null) and the
// network's guess xg (code 2; may be null), from the partial sums in
// pg[code * kRedBlocks + g]; ties and non-finite norms keep the earlier code.
// A run without two solutions in its history (mask) keeps code 0.
// The chosen start goes to out (which may alias xl or xg), the codes to the
// control block.
// runs whose history holds two solutions (the others start from the previous state)
struct RunMask {
    int ok[kMaxRuns];
};

__global__ void __launch_bounds__(kBlock) k_pick_guess(int len, const double2 *__restrict__ x,
                                                       const double2 *xl, const double2 *xg,
                                                       const double2 *__restrict__ pg, int G,
                                                       double2 *out, Ctl *c, RunMask mask)
{
    __shared__ double2 nrm[3];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    pg = run_at(pg, kSlotStride);
    c += blockIdx.y;
    x = run_at(x, len);
    xl = run_at(xl, len);
    xg = run_at(xg, len);
    out = run_at(out, len);
    if (wid < 3) {
        double2 s = d2(0.0, 0.0);
        for (int g = lane; g < G; g += 64) {
            const double2 q = pg[(size_t)wid * kRedBlocks + g];
            s.x += q.x;
            s.y += q.y;
        }
        s = wave_sum(s);
        if (lane == 0)
            nrm[wid] = s;
    }
    __syncthreads();
    int cx = 0, cy = 0;
    double bx = nrm[0].x, by = nrm[0].y;
    if (!mask.ok[blockIdx.y]) {
        xl = nullptr;
        xg = nullptr;
    }
    if (xl) {
        if (nrm[1].x < bx) { cx = 1; bx = nrm[1].x; }
        if (nrm[1].y < by) { cy = 1; by = nrm[1].y; }
    }
    if (xg) {
        if (nrm[2].x < bx) { cx = 2; bx = nrm[2].x; }
        if (nrm[2].y < by) { cy = 2; by = nrm[2].y; }
    }
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) {
        c->guess_used[0] = cx;
        c->guess_used[1] = cy;
    }
    if (i >= len)
        return;
    const double2 a = x[i];
    const double2 l = xl ? xl[i] : a, g = xg ? xg[i] : a;
    out[i] = d2(cx == 0 ? a.x : (cx == 1 ? l.x : g.x), cy == 0 ? a.y : (cy == 1 ? l.y : g.y));
}

// ------------------------------------------------------------------ host helpers
inline double2 pair(const double *a) { return make_double2(a[0], a[1]); }

// the control-block head of run r in the pinned host mirror
inline const Ctl &head(const Solver &S, int r)
{
    return *reinterpret_cast<const Ctl *>(reinterpret_cast<const char *>(S.hctl) + r * kCtlHead);
}

}  // namespace

template <class I, bool U8, class XT, class VA>
static void saddle_rb(Solver &S, const I *col, const VA &vm, const VA &vk, const XT *x, double2 *y)
{
    const int n = S.nv, R = S.nrun, rb = rb_of(S);
    const dim3 g = grid_rb(nblk(n), R, rb);
    const double2 t = pair(S.tau_s), te = pair(S.te_s);
    const size_t lb = lds_bytes(vm) + lds_bytes(vk);
    if (rb >= 4)
        k_saddle<I, U8, 4, XT, VA><<<g, kBlock, lb, S.stream>>>(n, R, S.sM.sptr, col, vm, vk, x, y,
                                                               t, te);
    else if (rb == 2)
        k_saddle<I, U8, 2, XT, VA><<<g, kBlock, lb, S.stream>>>(n, R, S.sM.sptr, col, vm, vk, x, y,
                                                               t, te);
    else
        k_saddle<I, U8, 1, XT, VA><<<g, kBlock, lb, S.stream>>>(n, R, S.sM.sptr, col, vm, vk, x, y,
                                                               t, te);
}

template <class XT>
static void apply_saddle_t(Solver &S, const XT *x, double2 *y)
{
    const bool u8 = S.sM.wmax <= kSellUnroll;
    using VP = VPlain<double>;
    using VT = VTab<double>;
    const VP pm{S.sM.val}, pk{S.sK};
    const bool tab = S.sM.ocol && S.vtM.ix && S.vtK.ix;
    const VT tm{S.vtM.ix, S.vtM.tab, S.vtM.m}, tk{S.vtK.ix, S.vtK.tab, S.vtK.m};
    if (tab && u8)
        saddle_rb<int16_t, true, XT, VT>(S, S.sM.ocol, tm, tk, x, y);
    else if (tab)
        saddle_rb<int16_t, false, XT, VT>(S, S.sM.ocol, tm, tk, x, y);
    else if (S.sM.ocol && u8)
        saddle_rb<int16_t, true, XT, VP>(S, S.sM.ocol, pm, pk, x, y);
    else if (S.sM.ocol)
        saddle_rb<int16_t, false, XT, VP>(S, S.sM.ocol, pm, pk, x, y);
    else if (u8)
        saddle_rb<int, true, XT, VP>(S, S.sM.col, pm, pk, x, y);
    else
        saddle_rb<int, false, XT, VP>(S, S.sM.col, pm, pk, x, y);
}

void apply_saddle(Solver &S, const double2 *x, double2 *y) { apply_saddle_t<double2>(S, x, y); }

// y = b - A x and the partials of its norms (k_saddle_resid) on M's pattern
static void saddle_resid(Solver &S, dim3 g, const double2 *x, double2 *y, double2 *part, double w2)
{
    const int n = S.nv;
    const bool u8 = S.sM.wmax <= kSellUnroll;
    using VP = VPlain<double>;
    using VT = VTab<double>;
    const VP pm{S.sM.val}, pk{S.sK};
    const bool tab = S.sM.ocol && S.vtM.ix && S.vtK.ix;
    const VT tm{S.vtM.ix, S.vtM.tab, S.vtM.m}, tk{S.vtK.ix, S.vtK.tab, S.vtK.m};
    const double2 t = pair(S.tau_s), te = pair(S.te_s);
    const size_t lbt = lds_bytes(tm) + lds_bytes(tk);
    if (tab && u8)
        k_saddle_resid<int16_t, true, VT><<<g, kBlock, lbt, S.stream>>>(
            n, S.sM.sptr, S.sM.ocol, tm, tk, x, S.b, y, t, te, part, w2);
    else if (tab)
        k_saddle_resid<int16_t, false, VT><<<g, kBlock, lbt, S.stream>>>(
            n, S.sM.sptr, S.sM.ocol, tm, tk, x, S.b, y, t, te, part, w2);
    else if (S.sM.ocol && u8)
        k_saddle_resid<int16_t, true, VP><<<g, kBlock, 0, S.stream>>>(
            n, S.sM.sptr, S.sM.ocol, pm, pk, x, S.b, y, t, te, part, w2);
    else if (S.sM.ocol)
        k_saddle_resid<int16_t, false, VP><<<g, kBlock, 0, S.stream>>>(
            n, S.sM.sptr, S.sM.ocol, pm, pk, x, S.b, y, t, te, part, w2);
    else if (u8)
        k_saddle_resid<int, true, VP><<<g, kBlock, 0, S.stream>>>(
            n, S.sM.sptr, S.sM.col, pm, pk, x, S.b, y, t, te, part, w2);
    else
        k_saddle_resid<int, false, VP><<<g, kBlock, 0, S.stream>>>(
            n, S.sM.sptr, S.sM.col, pm, pk, x, S.b, y, t, te, part, w2);
}

// b = (M phi + tau G, -(tau'/eps) f) for the current state of every run
// (G: the boundary vector, zero without boundary terms)
void compute_rhs(Solver &S)
{
    const int n = S.nv, R = S.nrun;
    const long len = 2l * n;
    hipStream_t st = S.stream;
    const Pot *pots = static_cast<const Pot *>(S.pots);
    const int nc = S.ncell;
    const long ns = S.vslot_stored;
    if (S.nl == 3) {
        k_rhs_cells<3><<<grid(nblk(nc), R), kBlock, 0, st>>>(nc, S.cells, S.qb, S.qw, S.nq, n, S.x,
                                                             pots, S.vslot_pos, ns, S.fslot, S.ctl);
        k_rhs_gather<3><<<grid(nblk(n), R), kBlock, 0, st>>>(n, S.vslot_ptr, S.vslot, S.vol, ns,
                                                             S.fslot, S.f);
    } else {
        k_rhs_cells<4><<<grid(nblk(nc), R), kBlock, 0, st>>>(nc, S.cells, S.qb, S.qw, S.nq, n, S.x,
                                                             pots, S.vslot_pos, ns, S.fslot, S.ctl);
        k_rhs_gather<4><<<grid(nblk(n), R), kBlock, 0, st>>>(n, S.vslot_ptr, S.vslot, S.vol, ns,
                                                             S.fslot, S.f);
    }
    sell_spmv<SP_SET, double>(st, R, rb_of(S), n, S.sM.sptr, S.sM.col, S.sM.ocol, S.sM.val,
                              S.vtM.ix, S.vtM.tab, S.vtM.m, S.x, len, nullptr, S.b, len);
    boundary_rhs(S, nullptr);
    k_rhs_second<<<grid(nblk(n), R), kBlock, 0, st>>>(n, S.f, S.b + n, pair(S.te_s));
    CHM_HIP(hipGetLastError());
}

void alloc_workspace(Solver &S)
{
    Pool &p = S.pool;
    const int n = S.nv;
    const size_t len = 2 * (size_t)n, nb = S.nb;
    S.m = S.prm.restart;
    S.x = p.get<double2>(nb * len);
    S.xk = p.get<double2>(nb * len);
    S.xl = p.get<double2>(nb * len);
    S.yh1 = p.get<double2>(nb * len);
    S.yh2 = p.get<double2>(nb * len);
    S.b = p.get<double2>(nb * len);
    S.r = p.get<double2>(nb * len);
    S.V = p.get<double2>(nb * len * (S.m + 1));
    // the preconditioned vectors: FP32 where the preconditioner computes in FP32
    if (S.mixed)
        S.Z32 = p.get<float2>(nb * len * S.m);
    else
        S.Z = p.get<double2>(nb * len * S.m);
    S.f = p.get<double2>(nb * n);
    S.fslot = p.get<double2>(nb * (size_t)S.vslot_stored);
    // the padding of the slot lists adds zero
    fill_double(reinterpret_cast<double *>(S.fslot), 0.0, 2 * nb * (size_t)S.vslot_stored, S.stream);
    S.stage = p.get<double>(n);
    S.red = p.get<double2>(nb * kSlotStride);
    // (twice the rows for the delayed pass's dots with u_j and with w)
    S.gsp1 = p.get<double2>(nb * 2 * (kMaxRestart + 1) * kGsBlocks);
    S.gsp2 = p.get<double2>(nb * (kMaxRestart + 1) * kGsBlocks);
    S.gsp3 = p.get<double2>(nb * kGsBlocks);
    S.hfin = p.get<double2>(nb * 2 * (kMaxRestart + 1));
    S.ctl = p.get<Ctl>(nb);
    fill_int(reinterpret_cast<int *>(S.ctl), 0, nb * sizeof(Ctl) / sizeof(int), S.stream);
    std::vector<Pot> pots(nb);
    for (size_t r = 0; r < nb; ++r)
        pots[r] = Pot{S.prm.potential, 1.0 / S.prm.Np, 1.0 / S.prm.Nn, 1.0 / S.prm.Ns, S.runs[r].chi_pn,
                      S.runs[r].chi_ps, S.runs[r].chi_ns, S.prm.log_floor};
    Pot *dp = p.get<Pot>(nb);
    CHM_HIP(hipMemcpyAsync(dp, pots.data(), nb * sizeof(Pot), hipMemcpyHostToDevice, S.stream));
    S.pots = dp;
    CHM_HIP(hipHostMalloc(reinterpret_cast<void **>(&S.hctl), nb * kCtlHead,
                          hipHostMallocCoherent | hipHostMallocMapped));
    CHM_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&S.dheads), S.hctl, 0));
    k_zero<<<grid(nblk(len), (int)nb), kBlock, 0, S.stream>>>((int)len, S.x);
    CHM_HIP(hipStreamSynchronize(S.stream));
}

namespace {

constexpr long kGsStride = (long)(kMaxRestart + 1) * kGsBlocks;   // per run
constexpr long kHStride = 2 * (kMaxRestart + 1);                  // per run

// the heads of the runs' control blocks into the pinned mirror (one run:
// directly; a batch: packed on the device first, then one copy)
void copy_heads(Solver &S, hipStream_t st)
{
    k_pack_heads<<<grid(1, S.nrun), 64, 0, st>>>(S.ctl, S.dheads);
    CHM_HIP(hipGetLastError());
}

void read_ctl(Solver &S)
{
    copy_heads(S, S.stream);
    CHM_HIP(hipStreamSynchronize(S.stream));
}

// One Arnoldi step j of FGMRES for both species of every run: z_j =
// Prec(v_j) (Algorithm 1), w = A z_j, the Gram-Schmidt sweeps (the delayed
// pair of CHM_ORTHO_DCGS2, or both passes of CHM_ORTHO_CGS2), the Givens
// update and v_{j+1} = w/|w|, then the heads of the control blocks are copied
// to pinned host memory.  Everything is enqueued on S.stream without host
// synchronisation, so the sequence can be captured as a graph.
void iteration_body(Solver &S, int j)
{
    const int len = 2 * S.nv, m = S.m, R = S.nrun;
    const long ks = (long)R * len;   // Krylov index stride: [index][run][len]
    hipStream_t st = S.stream;
    const int Gg = (int)std::min<long>(kGsBlocks, nblk(len));
    double2 *vj = S.V + (size_t)j * ks;
    double2 *w = S.V + (size_t)(j + 1) * ks;
    if (S.mixed) {   // z_j stays FP32; v_j (j > 0) came with its FP32 copy
        float2 *zj = S.Z32 + (size_t)j * ks;
        apply_prec32(S, vj, zj, j > 0);
        apply_saddle_t<float2>(S, zj, w);
    } else {
        double2 *zj = S.Z + (size_t)j * ks;
        apply_prec(S, vj, zj);
        apply_saddle(S, zj, w);
    }
    if (S.prm.ortho == CHM_ORTHO_DCGS2) {
        k_dgs_dots<kChunk><<<grid(Gg, R), kBlock, 0, st>>>(len, ks, S.V, j, w, S.gsp1,
                                                           2 * kGsStride);
        k_finish<<<grid(2 * (j + 1), R), kBlock, 0, st>>>(S.gsp1, 2 * kGsStride, Gg, S.hfin,
                                                          kHStride);
        k_dgs_update<<<grid(Gg, R), kBlock, 0, st>>>(len, ks, S.V, j, w, S.hfin, kHStride,
                                                     S.gsp3, kGsBlocks, S.ctl,
                                                     S.mixed ? S.w32.vin : nullptr);
        k_givens_d<<<grid(1, R), kBlock, 0, st>>>(S.ctl, j, m, S.hfin, kHStride, S.gsp3,
                                                  kGsBlocks, Gg);
        CHM_HIP(hipGetLastError());
        copy_heads(S, st);
        return;
    }
    double2 *h1 = S.hfin, *h2 = S.hfin + kMaxRestart + 1;
    k_gs<0><<<grid(Gg, R), kBlock, 0, st>>>(len, ks, S.V, j + 1, w, nullptr, kHStride, S.gsp1,
                                            kGsStride);
    k_finish<<<grid(j + 1, R), kBlock, 0, st>>>(S.gsp1, kGsStride, Gg, h1, kHStride);
    if (j + 1 <= 8)
        k_gs1_reg<8><<<grid(Gg, R), kBlock, 0, st>>>(len, ks, S.V, j + 1, w, h1, kHStride, S.gsp2,
                                                     kGsStride);
    else if (j + 1 <= 16)
        k_gs1_reg<16><<<grid(Gg, R), kBlock, 0, st>>>(len, ks, S.V, j + 1, w, h1, kHStride,
                                                      S.gsp2, kGsStride);
    else
        k_gs1_split<16><<<grid(Gg, R), kBlock, 0, st>>>(len, ks, S.V, j + 1, w, h1, kHStride,
                                                        S.gsp2, kGsStride);
    k_finish<<<grid(j + 1, R), kBlock, 0, st>>>(S.gsp2, kGsStride, Gg, h2, kHStride);
    k_gs<2><<<grid(Gg, R), kBlock, 0, st>>>(len, ks, S.V, j + 1, w, h2, kHStride, S.gsp3,
                                            kGsBlocks);
    k_givens<<<grid(1, R), kBlock, 0, st>>>(S.ctl, j, m, h1, h2, kHStride, S.gsp3, kGsBlocks, Gg);
    k_scale_next<<<grid(nblk(len), R), kBlock, 0, st>>>(len, w, S.ctl,
                                                        S.mixed ? S.w32.vin : nullptr);
    CHM_HIP(hipGetLastError());
    copy_heads(S, st);
}

// Run iteration_body(j), as a HIP graph when enabled (captured once per j on
// the library's own stream, launched on the caller's stream), and wait for it.
// The event timer records around kernels, so timed runs stay eager.
void run_iteration(Solver &S, int j)
{
    if (!S.prm.use_graphs || S.timer.on || S.prm.amg_tol > 0.0) {
        iteration_body(S, j);
        CHM_HIP(hipStreamSynchronize(S.stream));
        return;
    }
    if ((int)S.iter_graphs.size() <= j)
        S.iter_graphs.resize(j + 1, nullptr);
    if (!S.iter_graphs[j]) {
        if (!S.cap_stream)
            CHM_HIP(hipStreamCreateWithFlags(&S.cap_stream, hipStreamNonBlocking));
        // the capture stream must not start before earlier work on the caller's stream
        CHM_HIP(hipStreamSynchronize(S.stream));
        hipStream_t user = S.stream;
        S.stream = S.cap_stream;
        hipGraph_t g = nullptr;
        CHM_HIP(hipStreamBeginCapture(S.cap_stream, hipStreamCaptureModeThreadLocal));
        try {
            iteration_body(S, j);
        } catch (...) {
            (void)hipStreamEndCapture(S.cap_stream, &g);
            if (g)
                (void)hipGraphDestroy(g);
            S.stream = user;
            throw;
        }
        S.stream = user;
        CHM_HIP(hipStreamEndCapture(S.cap_stream, &g));
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        CHM_HIP(e);
        S.iter_graphs[j] = ex;
    }
    CHM_HIP(hipGraphLaunch(S.iter_graphs[j], S.stream));
    CHM_HIP(hipStreamSynchronize(S.stream));
}

std::string pair_str(double a, double b)
{
    return "(" + std::to_string(a) + ", " + std::to_string(b) + ")";
}

}  // namespace

// One time step of every run of the batch: right-hand side, the Krylov
// method (FGMRES or MINRES) for both species, commit and solvent removal.  The runs' Arnoldi steps advance
// together; each species of each run has its own flags, iteration count and
// convergence test, so each run follows the same iterates as it would alone.
// A step that fails for any run commits no run.  st_out: nb entries.
int step_once(Solver &S, chm_stats_t *st_out)
{
    const int n = S.nv, len = 2 * n, m = S.m, R = S.nb;
    S.nrun = R;
    const long ks = (long)R * len;
    hipStream_t st = S.stream;
    const int Gv = red_blocks(len), Gn = red_blocks(n);
    auto t0 = std::chrono::steady_clock::now();
    std::vector<chm_stats_t> stats(R);

    k_ctl_reset<<<grid(1, R), 64, 0, st>>>(S.ctl);
    compute_rhs(S);
    k_dot<double><<<grid(Gv, R), kBlock, 0, st>>>(len, S.b, S.b, slot(S, kSlotB));
    k_tol<<<grid(1, R), kBlock, 0, st>>>(S.ctl, slot(S, kSlotB), Gv, S.prm.rtol);
    RunMask mask{};
    bool any_hist = false;
    for (int r = 0; r < R; ++r) {
        mask.ok[r] = S.hist[r] >= 2;
        any_hist = any_hist || mask.ok[r];
    }
    if (S.guess_mode != CHM_GUESS_PREVIOUS && any_hist) {
        // candidate starts from the last two solutions: linear extrapolation
        // and, in the learned mode, the network's guess; each species starts
        // from whichever of them and the previous state has the smallest
        // residual in the first block row (the mass balance).  The second
        // row's residual is dominated by a spatially constant error in mu,
        // which the preconditioned iteration removes almost at once, so its
        // 2-norm does not rank the starts by their cost.
        const bool learned = S.guess_mode == CHM_GUESS_LEARNED;
        double2 *xg = learned ? S.xk : nullptr;
        k_extrapolate<<<grid(nblk(len), R), kBlock, 0, st>>>(len, S.yh2, S.yh1, S.xl);
        if (learned)
            for (int r = 0; r < R; ++r)
                if (mask.ok[r])
                    net_guess_on(S.net, st, S.gH, S.gW,
                             reinterpret_cast<const double *>(S.yh2 + (size_t)r * len),
                             reinterpret_cast<const double *>(S.yh1 + (size_t)r * len),
                             reinterpret_cast<double *>(xg + (size_t)r * len));
        const double2 *cand[3] = {S.x, S.xl, xg};
        for (int k = 0; k < 3; ++k)
            if (cand[k])
                saddle_resid(S, grid(Gn, R), cand[k], S.r, slot(S, kSlotGuess + k), 0.0);
        k_pick_guess<<<grid(nblk(len), R), kBlock, 0, st>>>(len, S.x, S.xl, xg, slot(S, kSlotGuess),
                                                            Gn, S.xk, S.ctl, mask);
    } else {
        k_copy<double2><<<grid(nblk(len), R), kBlock, 0, st>>>(len, S.x, S.xk);
    }

    std::vector<int> total(2 * R, 0), act(2 * R, 0);
    std::vector<double> res(2 * R, 0.0), bn(2 * R, 0.0);
    int rc = CHM_OK;
    bool first = true;
    const bool minres = S.prm.krylov == CHM_KRYLOV_MINRES;
    bool mr_done = false;
    Flags flags{};
    for (;;) {
        saddle_resid(S, grid(Gn, R), S.xk, S.r, slot(S, kSlotR), 1.0);
        k_nrm<<<grid(1, R), kBlock, 0, st>>>(S.ctl, slot(S, kSlotR), Gn);
        CHM_HIP(hipGetLastError());
        read_ctl(S);
        bool finite = true, any = false, over = false;
        for (int r = 0; r < R; ++r) {
            const Ctl &h = head(S, r);
            for (int s = 0; s < 2; ++s) {
                const int q = 2 * r + s;
                res[q] = std::sqrt(h.nrm[s]);
                bn[q] = h.bnorm[s];
                finite = finite && std::isfinite(res[q]);
                act[q] = !(res[q] <= h.tol[s]);
                if (first)
                    stats[r].res0[s] = bn[q] > 0.0 ? res[q] / bn[q] : res[q];
                any = any || act[q];
                over = over || (act[q] && total[q] >= S.prm.max_iters);
            }
        }
        first = false;
        if (!finite) {
            rc = CHM_ENAN;
            for (int r = 0; r < R; ++r)
                if (!std::isfinite(res[2 * r]) || !std::isfinite(res[2 * r + 1])) {
                    S.nan_where = "residual check, run " + std::to_string(r) + ": |r| = " +
                                  pair_str(res[2 * r], res[2 * r + 1]) + ", |b| = " +
                                  pair_str(bn[2 * r], bn[2 * r + 1]) + ", iterations " +
                                  pair_str(total[2 * r], total[2 * r + 1]);
                    break;
                }
            break;
        }
        if (minres) {
            // one MINRES solve from the chosen start (its own stopping rule in
            // the P^-1 norm), then one more pass for the true residual
            if (mr_done)
                break;
            rc = minres_solve(S, total);
            if (rc)
                break;
            mr_done = true;
            continue;
        }
        if (!any)
            break;
        if (over) {
            rc = CHM_ENOCONV;
            break;
        }
        for (int q = 0; q < 2 * R; ++q)
            flags.a[q] = act[q];
        k_cycle_init<<<grid(1, R), 64, 0, st>>>(S.ctl, flags);
        k_scale_first<<<grid(nblk(len), R), kBlock, 0, st>>>(len, S.r, S.V, S.ctl);
        int kmax = 0;
        for (int j = 0; j < m; ++j) {
            run_iteration(S, j);
            for (int q = 0; q < 2 * R; ++q)
                total[q] += act[q];
            bool anyact = false, capped = false, nan = false;
            for (int r = 0; r < R; ++r) {
                const Ctl &h = head(S, r);
                kmax = std::max(kmax, std::max(h.k[0], h.k[1]));
                nan = nan || h.nan;
                for (int s = 0; s < 2; ++s) {
                    const int q = 2 * r + s;
                    act[q] = h.active[s];
                    if (act[q] && total[q] >= S.prm.max_iters) {
                        act[q] = 0;   // iteration budget spent: the cycle ends for this species
                        capped = true;
                    }
                    anyact = anyact || act[q];
                }
            }
            if (capped) {
                for (int q = 0; q < 2 * R; ++q)
                    flags.a[q] = act[q];
                k_deactivate<<<grid(1, R), 64, 0, st>>>(S.ctl, flags);
            }
            if (nan) {
                rc = CHM_ENAN;
                for (int r = 0; r < R; ++r) {
                    const Ctl &h = head(S, r);
                    if (h.nan) {
                        S.nan_where = "Arnoldi step " + std::to_string(j) + ", run " +
                                      std::to_string(r) + ": estimates " +
                                      pair_str(h.resest[0], h.resest[1]) + ", |w| " +
                                      pair_str(h.hn[0], h.hn[1]) + ", iterations " +
                                      pair_str(total[2 * r], total[2 * r + 1]);
                        break;
                    }
                }
                break;
            }
            if (!anyact)
                break;
        }
        if (rc)
            break;
        k_trisolve<<<grid(1, R), 64, 0, st>>>(S.ctl, m);
        if (S.mixed)
            k_update_x<<<grid(nblk(len), R), kBlock, 0, st>>>(len, ks, S.xk, S.Z32, kmax, S.ctl);
        else
            k_update_x<<<grid(nblk(len), R), kBlock, 0, st>>>(len, ks, S.xk, S.Z, kmax, S.ctl);
        CHM_HIP(hipGetLastError());
    }
    if (rc == CHM_OK) {
        // the new state: the solve's solution, then the solvent removal, in
        // the candidate buffer S.xl (the current state stays until commit)
        k_finite<<<grid(nblk(len), R), kBlock, 0, st>>>(len, S.xk, S.ctl);
        k_copy<double2><<<grid(nblk(len), R), kBlock, 0, st>>>(len, S.xk, S.xl);
        Evap e{};
        bool evap = false;
        for (int r = 0; r < R; ++r) {
            const RunPrm &P = S.runs[r];
            e.ds[r] = (P.evap_ds > 0.0 && S.steps[r] < P.evap_steps) ? P.evap_ds : 0.0;
            evap = evap || e.ds[r] > 0.0;
        }
        if (evap)
            k_evaporate<<<grid(nblk(n), R), kBlock, 0, st>>>(n, S.xl, e);
        k_outside<<<grid(nblk(n), R), kBlock, 0, st>>>(n, S.xl, S.ctl);
        CHM_HIP(hipGetLastError());
        read_ctl(S);
        for (int r = 0; r < R; ++r)
            if (head(S, r).nan) {
                rc = CHM_ENAN;
                S.nan_where = "final iterate, run " + std::to_string(r);
                break;
            }
        if (rc == CHM_OK && S.prm.range_check)
            for (int r = 0; r < R; ++r)
                if (head(S, r).outside) {
                    rc = CHM_EDOMAIN;
                    S.nan_where = "run " + std::to_string(r) + ": " +
                                  std::to_string(head(S, r).outside) +
                                  " vertices with a volume fraction outside [0, 1]";
                    break;
                }
    }
    for (int r = 0; r < R; ++r) {
        const Ctl &h = head(S, r);
        stats[r].clamped = h.clamped;
        stats[r].guess_used[0] = h.guess_used[0];
        stats[r].guess_used[1] = h.guess_used[1];
        stats[r].outside = h.outside;
    }
    if (rc == CHM_OK) {
        std::swap(S.yh1, S.yh2);   // y_{n-1} becomes y_{n-2}
        k_copy<double2><<<grid(nblk(len), R), kBlock, 0, st>>>(len, S.xk, S.yh1);
        for (int r = 0; r < R; ++r)
            S.hist[r] = std::min(S.hist[r] + 1, 2);
        std::swap(S.x, S.xl);   // commit the candidate state
        CHM_HIP(hipGetLastError());
        CHM_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < R; ++r)
            S.steps[r]++;
    }
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < R; ++r) {
        for (int s = 0; s < 2; ++s) {
            const int q = 2 * r + s;
            stats[r].iters[s] = total[q];
            stats[r].relres[s] = bn[q] > 0.0 ? res[q] / bn[q] : res[q];
        }
        stats[r].status = rc;
        stats[r].t_step_ms = ms;
        if (st_out)
            st_out[r] = stats[r];
    }
    return rc;
}

}  // namespace chm
