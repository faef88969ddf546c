// Device helpers and kernels shared by the preconditioner (prec.hip) and the
// Krylov solver (solve.hip): pair types, the XCD-aware block numbering, the
// deterministic reductions and the SpMV kernels, templated on the value type
// (double for the FP64 path, float for the FP32 preconditioner).  Everything
// sits in an unnamed namespace, so each source file has its own copies.
//
// Reductions need no inter-block synchronisation: a producer kernel with a
// fixed grid writes one partial sum per block; every consumer block adds the
// partials itself in a fixed order (so all blocks obtain the same bits) after
// the kernel boundary has made them visible.
#pragma once

#include "chm_internal.h"

#include <type_traits>

namespace chm {
namespace {

inline int nblk(long n, int bs = kBlock) { return (int)std::max<long>(1, (n + bs - 1) / bs); }
inline int red_blocks(long n) { return (int)std::min<long>(kRedBlocks, nblk(n)); }

__device__ inline double2 d2(double a, double b) { return make_double2(a, b); }

// pair type of a value type: double -> double2, float -> float2
template <class T> struct PairOf;
template <> struct PairOf<double> { using type = double2; };
template <> struct PairOf<float> { using type = float2; };
template <class T> using pair_t = typename PairOf<T>::type;

// a * b + c with one rounding.  The kernels that run in several variants
// (one run or several runs per lane) write every product they add as fmad,
// so no variant leaves the choice of which products to fuse to the compiler
// and all variants give the same bits.
__device__ inline double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Natural logarithm of a positive finite x, about a third of the FP64 work
// of the library's log.  With x = m 2^e, m in [sqrt(1/2), sqrt(2)), and
// f = m - 1 (exact), s = f / (2 + f):
//   log(m) = 2 atanh(s) = 2 s + s Q(s^2),  Q(z) = sum_{k >= 1} 2 z^k / (2k + 1),
// and 2 s = f - s f, so log(m) = f - s (f - Q).  |s| <= 0.1716, so z <= 0.0295
// and the terms past k = 10 are below 2^-60 relative.  ln 2 = ln2_hi +
// ln2_lo with ln2_hi holding 42 significant bits, so e ln2_hi is exact.
// Every product that is added is a written fused multiply-add, so host and
// device builds give the same bits.  Error: about one unit in the last place.
__host__ __device__ inline double log_pos(double x)
{
    constexpr double ln2_hi = 0x1.62e42fefa3800p-1, ln2_lo = 0x1.ef35793c76730p-45;
    int e;
    double m = frexp(x, &e);   // [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        --e;
    }
    const double f = m - 1.0, s = f / (2.0 + f), z = s * s;
    double q = 2.0 / 21.0;
    q = __builtin_fma(q, z, 2.0 / 19.0);
    q = __builtin_fma(q, z, 2.0 / 17.0);
    q = __builtin_fma(q, z, 2.0 / 15.0);
    q = __builtin_fma(q, z, 2.0 / 13.0);
    q = __builtin_fma(q, z, 2.0 / 11.0);
    q = __builtin_fma(q, z, 2.0 / 9.0);
    q = __builtin_fma(q, z, 2.0 / 7.0);
    q = __builtin_fma(q, z, 2.0 / 5.0);
    q = __builtin_fma(q, z, 2.0 / 3.0);
    q *= z;
    const double de = (double)e;
    const double r = __builtin_fma(-s, f - q, f);
    return __builtin_fma(de, ln2_hi, __builtin_fma(de, ln2_lo, r));
}

template <class T> __device__ inline pair_t<T> mk(T a, T b);
template <> __device__ inline double2 mk<double>(double a, double b) { return make_double2(a, b); }
template <> __device__ inline float2 mk<float>(float a, float b) { return make_float2(a, b); }

// XCD-aware block index.  The hardware hands workgroup (b, y) of a grid G
// blocks wide to XCD (y G + b) mod 8; this renumbering gives every XCD one
// contiguous range of the blocks of each grid row y, so the neighbouring rows
// that an SpMV row gathers from mostly sit in the same XCD's L2.  For each y
// it is a bijection of [0, G).
constexpr int kXcds = 8;

// the new index of block b of grid row y in a grid G blocks wide
__host__ __device__ inline int xcd_rank(int G, int b, unsigned y)
{
    const int off = (int)((y * (unsigned)G) % kXcds);             // rotation of row y
    const int x = (b + off) % kXcds;                              // this block's XCD
    const int j = (b - (x - off + kXcds) % kXcds) / kXcds;        // its rank on that XCD
    int start = 0;                                                // blocks of earlier XCDs
    for (int k = 0; k < x; ++k)
        start += (G - (k - off + kXcds) % kXcds + kXcds - 1) / kXcds;
    return start + j;
}

__device__ inline int xcd_block() { return xcd_rank(gridDim.x, blockIdx.x, blockIdx.y); }

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

// out[v] = sum over g < G of part[v * G + g] for v < nvec, into LDS, visible
// to the whole block on return.  Wave w takes vectors w, w + 4, ...; lane l
// adds g = l, l + 64, ... and the wave adds its lanes with a fixed shuffle
// tree.
__device__ inline void reduce_parts(const double2 *__restrict__ part, int nvec, int G, double2 *out)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int v = wid; v < nvec; v += kBlock / 64) {
        double2 s = d2(0.0, 0.0);
        for (int g = lane; g < G; g += 64) {
            const double2 p = part[(size_t)v * G + g];
            s.x += p.x;
            s.y += p.y;
        }
        s = wave_sum(s);
        if (lane == 0)
            out[v] = s;
    }
    __syncthreads();
}

// two independent scalars at once (waves 0 and 1)
__device__ inline void reduce_two(const double2 *__restrict__ pa, const double2 *__restrict__ pb,
                                  int G, double2 *out)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (wid < 2) {
        const double2 *p = wid == 0 ? pa : pb;
        double2 s = d2(0.0, 0.0);
        for (int g = lane; g < G; g += 64) {
            const double2 q = p[g];
            s.x += q.x;
            s.y += q.y;
        }
        s = wave_sum(s);
        if (lane == 0)
            out[wid] = s;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ partial-sum slots
// kRedBlocks pairs each, in Solver::red: the inner CG uses rz (0..39) and
// dq (40..79), the Krylov solver the right-hand-side norm (80) and the
// residual norm (81) and the residual norms of the initial-guess candidates
// (82 + CHM_GUESS_*: previous state, linear extrapolation, network); MINRES
// takes slot 82 for its inner products once the start is chosen.
constexpr int kSlotRz = 0, kSlotDq = 40, kSlotB = 80, kSlotR = 81, kSlotGuess = 82, kSlots = 85;
constexpr long kSlotStride = (long)kSlots * kRedBlocks;   // per run

// run 0's slot k; run r's is kSlotStride further
inline double2 *slot(Solver &S, int k) { return S.red + (size_t)k * kRedBlocks; }

// Batched launches: blockIdx.y is the run, and every per-run array of a kernel
// is offset by the run times its stride (elements).
template <class P> __device__ inline P *run_at(P *p, long stride) { return p ? p + blockIdx.y * stride : p; }
inline dim3 grid(int x, int runs) { return dim3(x, runs); }

// runs per lane of the SELL and coarsest-level kernels of this launch (one
// run: 1)
inline int rb_of(const Solver &S) { return S.nrun > 1 ? S.rb : 1; }

// ------------------------------------------------------------------ SpMV family (pairs)
// SP_SET: y = A x; SP_ADD: y += A x; SP_RESID: y = b - A x
enum SpmvMode { SP_SET = 0, SP_ADD = 1, SP_RESID = 2 };

// row of a SELL-64 matrix (one lane per row, columns of a slice stored
// column-major so that the 64 lanes read consecutive words).  A wave is one
// slice (64 consecutive rows, 64-aligned), so the slice bounds are scalar
// loads.  Slices up to kSellUnroll wide (the fine levels of P1 meshes), or
// twice that, take a fully unrolled path that issues every column and value
// load of the row, then every gather of x, before the first product: two
// dependent memory round trips instead of one per group of entries.  The
// products are added in column order either way.  (kSellUnroll = 8, in the
// internal header.)

// Column of SELL entry idx, which belongs to row `row`: stored as a 32-bit
// column (I = int), or as a 16-bit offset from the row (I = int16_t; square
// matrices whose entries all lie within 32767 of the diagonal, 2 B per entry
// instead of 4).
__device__ inline int sell_col(const int *__restrict__ col, int idx, int) { return col[idx]; }
__device__ inline int sell_col(const int16_t *__restrict__ col, int idx, int row)
{
    return row + (int)col[idx];
}

// The values of a SELL matrix as the kernels read them: stored per entry
// (VPlain), or as a 16-bit index per entry into the table of the matrix's
// distinct values (VTab, uniform meshes: a few to a few hundred values), which
// gives the same value.
template <class T> struct VPlain {
    const T *__restrict__ v;
    __device__ T operator[](int i) const { return v[i]; }
};
template <class T> struct VTab {
    const uint16_t *__restrict__ ix;
    const T *__restrict__ tab;
    int m;   // table entries
    __device__ T operator[](int i) const { return tab[ix[i]]; }
};

// A table staged in LDS by the block (the kernels read it through this):
// a short lookup instead of a dependent global load per entry.
template <class T> struct VLds {
    const uint16_t *__restrict__ ix;
    const T *tab;   // LDS
    __device__ T operator[](int i) const { return tab[ix[i]]; }
};

// The accessor a kernel reads with: plain values as they are; a table copied
// into the block's dynamic LDS at `lds` (every thread of the block must call
// this, before any early return, since it ends with a barrier).
template <class VA> struct Staged {
    using type = VA;
    static constexpr size_t bytes(const VA &) { return 0; }
    __device__ static VA stage(const VA &v, void *) { return v; }
    __device__ static void stage2(const VA &a, const VA &b, void *, VA &sa, VA &sb)
    {
        sa = a;
        sb = b;
    }
};
// N table entries per thread (entries i = thread + j kBlock; the kernels that
// stage tables run blocks of kBlock threads), every load issued before the
// first LDS write: a loop that stores after each load waits a whole memory
// round trip per pass.  Past the end (m >= 1) the last entry is loaded again
// and not stored.
template <int N, class T>
__device__ inline void stage_entries(const T *__restrict__ tab, int m, T *t)
{
    T v[N];
#pragma unroll
    for (int j = 0; j < N; ++j)
        v[j] = tab[min((int)threadIdx.x + j * kBlock, m - 1)];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int i = threadIdx.x + j * kBlock;
        if (i < m)
            t[i] = v[j];
    }
    // every load completes here, stored or not: a load left in flight past
    // the barrier would make each later write of its registers wait for it
#pragma unroll
    for (int j = 0; j < N; ++j)
        __asm__ volatile("" ::"v"(v[j]));
}

// the same for two tables (the second stored after the first), all loads
// of both issued before the first write
template <int N, class T>
__device__ inline void stage_entries2(const T *__restrict__ ta, int ma, const T *__restrict__ tb,
                                      int mb, T *t)
{
    T va[N], vb[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        va[j] = ta[min((int)threadIdx.x + j * kBlock, ma - 1)];
        vb[j] = tb[min((int)threadIdx.x + j * kBlock, mb - 1)];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int i = threadIdx.x + j * kBlock;
        if (i < ma)
            t[i] = va[j];
        if (i < mb)
            t[ma + i] = vb[j];
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
        __asm__ volatile("" ::"v"(va[j]), "v"(vb[j]));
}

template <class T> struct Staged<VTab<T>> {
    using type = VLds<T>;
    static size_t bytes(const VTab<T> &v) { return (size_t)v.m * sizeof(T); }
    __device__ static VLds<T> stage(const VTab<T> &v, void *lds)
    {
        static_assert(kVtMax <= 8 * kBlock, "a table takes at most 8 entries per thread");
        T *t = static_cast<T *>(lds);
        const int passes = (v.m + kBlock - 1) / kBlock;   // 0 (no table) to 8
        if (passes == 1) {
            if ((int)threadIdx.x < v.m)
                t[threadIdx.x] = v.tab[threadIdx.x];
        } else if (passes == 2)
            stage_entries<2, T>(v.tab, v.m, t);
        else if (passes > 2 && passes <= 4)
            stage_entries<4, T>(v.tab, v.m, t);
        else if (passes > 4)
            stage_entries<8, T>(v.tab, v.m, t);
        __syncthreads();
        return VLds<T>{v.ix, t};
    }
    // two tables (both with entries) behind one barrier: a's at lds, b's after it
    __device__ static void stage2(const VTab<T> &a, const VTab<T> &b, void *lds, VLds<T> &sa,
                                  VLds<T> &sb)
    {
        T *t = static_cast<T *>(lds);
        const int passes = (max(a.m, b.m) + kBlock - 1) / kBlock;   // 1 to 8
        if (passes == 1)
            stage_entries2<1, T>(a.tab, a.m, b.tab, b.m, t);
        else if (passes == 2)
            stage_entries2<2, T>(a.tab, a.m, b.tab, b.m, t);
        else if (passes > 2 && passes <= 4)
            stage_entries2<4, T>(a.tab, a.m, b.tab, b.m, t);
        else if (passes > 4)
            stage_entries2<8, T>(a.tab, a.m, b.tab, b.m, t);
        __syncthreads();
        sa = VLds<T>{a.ix, t};
        sb = VLds<T>{b.ix, t + a.m};
    }
};
template <class VA> inline size_t lds_bytes(const VA &v) { return Staged<VA>::bytes(v); }
// the same on the device (the offset of a second table in a kernel's LDS)
template <class T> __device__ inline size_t lds_bytes_dev(const VPlain<T> &) { return 0; }
template <class T> __device__ inline size_t lds_bytes_dev(const VTab<T> &v)
{
    return (size_t)v.m * sizeof(T);
}

// The entries of one SELL row for slices at most W wide (width >= 1):
// entries past the slice width repeat the last column with a zero
// coefficient, so every load is unconditional (no branch between the loads
// and the gathers) and hits the cache line just read.
template <int W, class T> struct SellEnt {
    int c[W];
    T a[W];
};

template <int W, class I, class T, class VA>
__device__ inline void sell_load(int base, int width, int lane, int row, const I *__restrict__ col,
                                 const VA &val, SellEnt<W, T> &e)
{
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int idx = base + (k < width ? k : width - 1) * kSlice + lane;
        e.c[k] = sell_col(col, idx, row);
        const T v = val[idx];
        e.a[k] = k < width ? v : T(0);
    }
}

// the row product from the gathered x[c[k]], added in column order; diag
// receives the row's nonzero diagonal entry (0 if it has none; the padding of
// a short row may repeat the diagonal column, with value 0)
template <int W, class T>
__device__ inline pair_t<T> sell_dot(const SellEnt<W, T> &e, const pair_t<T> *xv, int row, T &diag)
{
    T ax = 0, ay = 0, d = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        ax = fmad(e.a[k], xv[k].x, ax);
        ay = fmad(e.a[k], xv[k].y, ay);
        d = (e.c[k] == row && e.a[k] != T(0)) ? e.a[k] : d;   // not the zero padding
    }
    diag = d;
    return mk<T>(ax, ay);
}

// the unrolled row product for slices at most W wide (width >= 1): every
// column and value load, then every gather, then the products
template <int W, class I, class T, class VA>
__device__ inline pair_t<T> sell_row_w(int base, int width, int lane, int row,
                                       const I *__restrict__ col, const VA &val,
                                       const pair_t<T> *__restrict__ x, T &diag)
{
    SellEnt<W, T> e;
    sell_load<W, I, T>(base, width, lane, row, col, val, e);
    pair_t<T> xv[W];
#pragma unroll
    for (int k = 0; k < W; ++k)
        xv[k] = x[e.c[k]];
    return sell_dot<W, T>(e, xv, row, diag);
}

// the row product of a SELL-64 matrix; diag receives the row's diagonal
// entry (0 if it has none; callers that do not use it lose the selects)
template <class I, class T, class VA>
__device__ inline pair_t<T> sell_row(const int *__restrict__ sptr, const I *__restrict__ col,
                                     const VA &val, const pair_t<T> *__restrict__ x,
                                     int row, T &diag)
{
    const int s = __builtin_amdgcn_readfirstlane(row / kSlice), lane = row % kSlice;
    const int base = sptr[s], width = (sptr[s + 1] - base) / kSlice;
    diag = 0;
    if (width == 0)
        return mk<T>(0, 0);
    if (width <= kSellUnroll)
        return sell_row_w<kSellUnroll, I, T, VA>(base, width, lane, row, col, val, x, diag);
    if (width <= 2 * kSellUnroll)
        return sell_row_w<2 * kSellUnroll, I, T, VA>(base, width, lane, row, col, val, x, diag);
    T ax = 0, ay = 0, d = 0;
#pragma unroll 4
    for (int k = 0; k < width; ++k) {
        const int idx = base + k * kSlice + lane;
        const T a = val[idx];
        const int c = sell_col(col, idx, row);
        const pair_t<T> xv = x[c];
        ax = fmad(a, xv.x, ax);
        ay = fmad(a, xv.y, ay);
        d = (c == row && a != T(0)) ? a : d;
    }
    diag = d;
    return mk<T>(ax, ay);
}

// The bounds of the SELL-64 slice that holds `row` (wave-uniform: a wave's
// 64 rows form one slice).  Rows past n take the last slice, so a kernel
// can load the bounds before its early return (in flight with its other
// prologue loads) and stay in bounds.
struct SliceAt {
    int base, width;
};
__device__ inline SliceAt slice_at(const int *__restrict__ sptr, int row, int n)
{
    const int s = __builtin_amdgcn_readfirstlane(min(row, n - 1) / kSlice);
    const int base = sptr[s];
    return SliceAt{base, (sptr[s + 1] - base) / kSlice};
}

// ------------------------------------------------------------------ several runs per lane
// Batched launches of the SELL kernels: block row blockIdx.y covers the RB
// runs r0 = RB blockIdx.y, ..., r0 + RB - 1 (those below R), so every matrix
// entry a lane loads serves RB runs and a launch over R runs streams the
// matrix ceil(R / RB) times instead of R times.  Each run's product is the
// single-run product (same entries, same order), so results do not depend on
// RB.
template <int RB> __device__ inline int run0() { return RB * (int)blockIdx.y; }
inline dim3 grid_rb(int x, int runs, int rb) { return dim3(x, (runs + rb - 1) / rb); }

// For each run r of the block: the product of SELL row `row` with
// x + r sx, handed to f(q, r, product, diag) with q = r - r0 (a constant
// after unrolling, so per-run arrays indexed by q stay in registers).  Slices at most kSellUnroll wide
// (2D P1 patterns) load the row's entries once and issue every run's gathers
// before the first product; wider slices go run by run (with one run per
// lane, slices up to twice that width still take the unrolled path).
template <class I, class T, int RB, class VA, class F>
__device__ inline void sell_row_runs(const int *__restrict__ sptr, SliceAt sl,
                                     const I *__restrict__ col, const VA &val,
                                     const pair_t<T> *__restrict__ x, long sx, int row, int R,
                                     F &&f)
{
    const int r0 = run0<RB>();
    const int lane = row % kSlice, base = sl.base, width = sl.width;
    auto runs_w = [&](auto wtag) {
        constexpr int W = decltype(wtag)::value;
        SellEnt<W, T> e;
        sell_load<W, I, T>(base, width, lane, row, col, val, e);
        pair_t<T> xv[RB][W];
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R)
#pragma unroll
                for (int k = 0; k < W; ++k)
                    xv[q][k] = x[(r0 + q) * sx + e.c[k]];
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R) {
                T diag;
                const pair_t<T> p = sell_dot<W, T>(e, xv[q], row, diag);
                f(q, r0 + q, p, diag);
            }
    };
    if (width == 0) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R)
                f(q, r0 + q, mk<T>(0, 0), T(0));
    } else if (width <= kSellUnroll) {
        runs_w(std::integral_constant<int, kSellUnroll>{});
    } else if (RB == 1 && width <= 2 * kSellUnroll) {
        runs_w(std::integral_constant<int, RB == 1 ? 2 * kSellUnroll : 1>{});
    } else {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (RB == 1 || r0 + q < R) {
                T diag;
                const pair_t<T> p = sell_row<I, T, VA>(sptr, col, val, x + (r0 + q) * sx, row, diag);
                f(q, r0 + q, p, diag);
            }
    }
}

template <int MODE, class T>
__device__ inline void spmv_store(pair_t<T> s, const pair_t<T> *__restrict__ b, pair_t<T> *y, int row)
{
    if (MODE == SP_SET) {
        y[row] = s;
    } else if (MODE == SP_ADD) {
        const pair_t<T> o = y[row];
        y[row] = mk<T>(o.x + s.x, o.y + s.y);
    } else {
        const pair_t<T> bb = b[row];
        y[row] = mk<T>(bb.x - s.x, bb.y - s.y);
    }
}

// per run: x advances by sx, b and y by sy; RB runs per lane (block row
// blockIdx.y), R runs in all
template <int MODE, class I, class T, int RB, class VA>
__global__ void __launch_bounds__(kBlock) k_spmv(int n, int R, const int *__restrict__ sptr,
                                                 const I *__restrict__ col, const VA val0,
                                                 const pair_t<T> *__restrict__ x, long sx,
                                                 const pair_t<T> *__restrict__ b, pair_t<T> *y,
                                                 long sy)
{
    extern __shared__ __align__(8) unsigned char lds_tab[];
    using VS = typename Staged<VA>::type;
    const int row = xcd_block() * kBlock + threadIdx.x;
    // one run per lane: the row's y (SP_ADD) or b (SP_RESID) is loaded with the
    // slice bounds, in flight while the table is staged
    constexpr bool pre = RB == 1 && MODE != SP_SET;
    pair_t<T> o = mk<T>(0, 0);
    if (pre && row < n)
        o = (MODE == SP_ADD ? y : b)[(long)run0<RB>() * sy + row];
    const SliceAt sl = slice_at(sptr, row, n);
    const VS val = Staged<VA>::stage(val0, lds_tab);
    if (row >= n)
        return;
    sell_row_runs<I, T, RB, VS>(sptr, sl, col, val, x, sx, row, R, [&](int, int r, pair_t<T> s, T) {
        if (pre)
            y[r * sy + row] = MODE == SP_ADD ? mk<T>(o.x + s.x, o.y + s.y) : mk<T>(o.x - s.x, o.y - s.y);
        else
            spmv_store<MODE, T>(s, b ? b + r * sy : b, y + r * sy, row);
    });
}

template <int MODE, class I, class T, class VA>
void sell_spmv_i(hipStream_t st, int gx, int runs, int rb, int n, const int *sptr, const I *col,
                 const VA &val, const pair_t<T> *x, long sx, const pair_t<T> *b, pair_t<T> *y,
                 long sy)
{
    const dim3 g = grid_rb(gx, runs, rb);
    const size_t lb = lds_bytes(val);
    if (rb >= 4)
        k_spmv<MODE, I, T, 4, VA><<<g, kBlock, lb, st>>>(n, runs, sptr, col, val, x, sx, b, y, sy);
    else if (rb == 2)
        k_spmv<MODE, I, T, 2, VA><<<g, kBlock, lb, st>>>(n, runs, sptr, col, val, x, sx, b, y, sy);
    else
        k_spmv<MODE, I, T, 1, VA><<<g, kBlock, lb, st>>>(n, runs, sptr, col, val, x, sx, b, y, sy);
}

// k_spmv over a SELL matrix of n rows for `runs` runs, rb of them per lane,
// on its 16-bit column offsets when it has them (ocol), else on its columns
template <int MODE, class T>
void sell_spmv(hipStream_t st, int runs, int rb, int n, const int *sptr, const int *col,
               const int16_t *ocol, const T *val, const uint16_t *vix, const T *vtab, int vm,
               const pair_t<T> *x, long sx, const pair_t<T> *b, pair_t<T> *y, long sy)
{
    if (ocol && vix)
        sell_spmv_i<MODE, int16_t, T, VTab<T>>(st, nblk(n), runs, rb, n, sptr, ocol,
                                               VTab<T>{vix, vtab, vm}, x, sx, b, y, sy);
    else if (ocol)
        sell_spmv_i<MODE, int16_t, T, VPlain<T>>(st, nblk(n), runs, rb, n, sptr, ocol,
                                                 VPlain<T>{val}, x, sx, b, y, sy);
    else
        sell_spmv_i<MODE, int, T, VPlain<T>>(st, nblk(n), runs, rb, n, sptr, col, VPlain<T>{val},
                                             x, sx, b, y, sy);
}

// The same with a group of GS lanes per row (CSR), for matrices with long rows
// or few rows: lane l of the group takes entries l, l + GS, ... of the row and
// the group adds its lanes with a fixed shuffle tree.  Whole groups share a
// row, so they exit together.  A lane takes U of its entries per pass,
// loading all their indices and values, then all their gathers, before the
// products (entries past the row end repeat its last entry with a zero
// coefficient), so a pass costs two dependent memory round trips.
// The entries of x the row product gathers, x[j] by default; a kernel may
// form them on the fly instead (G: a callable taking the column).
template <class T> struct Gather {
    const pair_t<T> *__restrict__ x;
    __device__ pair_t<T> operator()(int j) const { return x[j]; }
};

template <int GS, int U, class T, class G>
__device__ inline pair_t<T> row_dot_g(const int *__restrict__ rp, const int *__restrict__ ci,
                                      const T *__restrict__ v, const G &x, int row, int lane)
{
    T ax = 0, ay = 0;
    const int s = rp[row], e = rp[row + 1];
    for (int k0 = s + lane; k0 < e; k0 += GS * U) {
        int c[U];
        T a[U];
        pair_t<T> xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * GS;
            const int kk = k < e ? k : e - 1;
            c[u] = ci[kk];
            const T val = v[kk];
            a[u] = k < e ? val : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            xv[u] = x(c[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ax += a[u] * xv[u].x;
            ay += a[u] * xv[u].y;
        }
    }
#pragma unroll
    for (int off = GS / 2; off > 0; off >>= 1) {
        ax += __shfl_down(ax, off, GS);
        ay += __shfl_down(ay, off, GS);
    }
    return mk<T>(ax, ay);
}

template <int GS, int U, class T>
__device__ inline pair_t<T> row_dot(const int *__restrict__ rp, const int *__restrict__ ci,
                                    const T *__restrict__ v, const pair_t<T> *__restrict__ x,
                                    int row, int lane)
{
    return row_dot_g<GS, U, T>(rp, ci, v, Gather<T>{x}, row, lane);
}

template <int GS, int U, int MODE, class T>
__global__ void __launch_bounds__(kBlock) k_spmv_v(int n, const int *__restrict__ rp,
                                                   const int *__restrict__ ci,
                                                   const T *__restrict__ v,
                                                   const pair_t<T> *__restrict__ x, long sx,
                                                   const pair_t<T> *__restrict__ b, pair_t<T> *y,
                                                   long sy)
{
    const int t = xcd_block() * kBlock + threadIdx.x;
    const int row = t / GS, lane = t % GS;
    if (row >= n)
        return;
    x = run_at(x, sx);
    b = run_at(b, sy);
    y = run_at(y, sy);
    const pair_t<T> s = row_dot<GS, U, T>(rp, ci, v, x, row, lane);
    if (lane == 0)
        spmv_store<MODE, T>(s, b, y, row);
}

// the CSR-vector launch for the matrix's entries per lane and pass
template <int GS, int MODE, class T>
void spmv_v_u(hipStream_t st, int runs, const MatView<T> &A, const pair_t<T> *x,
              const pair_t<T> *b, pair_t<T> *y, long sx, long sy)
{
    const dim3 g = grid(nblk((long)GS * A.n), runs);
    if (A.u >= 4)
        k_spmv_v<GS, 4, MODE, T><<<g, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.cval, x, sx, b, y, sy);
    else if (A.u == 2)
        k_spmv_v<GS, 2, MODE, T><<<g, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.cval, x, sx, b, y, sy);
    else
        k_spmv_v<GS, 1, MODE, T><<<g, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.cval, x, sx, b, y, sy);
}

// y = A x / y += A x / y = b - A x with the kernel shape chosen for the
// matrix, for `runs` runs whose x are A.m apart and whose b, y are A.n apart
// (or sx, sy when given); a SELL matrix serves rb runs per lane
template <int MODE, class T>
void spmv_op(hipStream_t st, int runs, int rb, const MatView<T> &A, const pair_t<T> *x,
             const pair_t<T> *b, pair_t<T> *y, long sx = -1, long sy = -1)
{
    const int n = A.n;
    if (sx < 0)
        sx = A.m;
    if (sy < 0)
        sy = A.n;
    if (A.gs == 0) {
        sell_spmv<MODE, T>(st, runs, rb, n, A.sptr, A.col, A.ocol, A.sval, A.vix, A.vtab, A.vm,
                           x, sx, b, y, sy);
        return;
    }
    switch (A.gs) {
    case 4:
        spmv_v_u<4, MODE, T>(st, runs, A, x, b, y, sx, sy);
        break;
    case 8:
        spmv_v_u<8, MODE, T>(st, runs, A, x, b, y, sx, sy);
        break;
    case 16:
        spmv_v_u<16, MODE, T>(st, runs, A, x, b, y, sx, sy);
        break;
    default:
        spmv_v_u<32, MODE, T>(st, runs, A, x, b, y, sx, sy);
        break;
    }
}

// The residual of a level and its restriction in one product:
// y = RR [b; x] = R (b - A x), with RR = [R | -R A] (n_c rows, columns j < n
// taken from b and n + j from x).  Same lane groups and passes as k_spmv_v;
// per run, b and x advance by n and y by n_c.
template <class T> struct GatherBX {
    const pair_t<T> *__restrict__ b;
    const pair_t<T> *__restrict__ x;
    int n;
    __device__ pair_t<T> operator()(int j) const { return *(j < n ? b + j : x + (j - n)); }
};

template <int GS, int U, class T>
__global__ void __launch_bounds__(kBlock) k_resid_restrict(int nc, int n, const int *__restrict__ rp,
                                                           const int *__restrict__ ci,
                                                           const T *__restrict__ v,
                                                           const pair_t<T> *__restrict__ b,
                                                           const pair_t<T> *__restrict__ x,
                                                           pair_t<T> *y)
{
    const int t = xcd_block() * kBlock + threadIdx.x;
    const int row = t / GS, lane = t % GS;
    if (row >= nc)
        return;
    b = run_at(b, (long)n);
    x = run_at(x, (long)n);
    y = run_at(y, (long)nc);
    const pair_t<T> s = row_dot_g<GS, U, T>(rp, ci, v, GatherBX<T>{b, x, n}, row, lane);
    if (lane == 0)
        y[row] = s;
}

template <int GS, class T>
void resid_restrict_u(hipStream_t st, int runs, const MatView<T> &RR, const pair_t<T> *b,
                      const pair_t<T> *x, pair_t<T> *y)
{
    const dim3 g = grid(nblk((long)GS * RR.n), runs);
    const int n = RR.m / 2;
    if (RR.u >= 4)
        k_resid_restrict<GS, 4, T><<<g, kBlock, 0, st>>>(RR.n, n, RR.rp, RR.ci, RR.cval, b, x, y);
    else if (RR.u == 2)
        k_resid_restrict<GS, 2, T><<<g, kBlock, 0, st>>>(RR.n, n, RR.rp, RR.ci, RR.cval, b, x, y);
    else
        k_resid_restrict<GS, 1, T><<<g, kBlock, 0, st>>>(RR.n, n, RR.rp, RR.ci, RR.cval, b, x, y);
}

template <class T>
void resid_restrict(hipStream_t st, int runs, const MatView<T> &RR, const pair_t<T> *b,
                    const pair_t<T> *x, pair_t<T> *y)
{
    switch (RR.gs) {
    case 4:
        resid_restrict_u<4, T>(st, runs, RR, b, x, y);
        break;
    case 8:
        resid_restrict_u<8, T>(st, runs, RR, b, x, y);
        break;
    case 16:
        resid_restrict_u<16, T>(st, runs, RR, b, x, y);
        break;
    default:
        resid_restrict_u<32, T>(st, runs, RR, b, x, y);
        break;
    }
}

// ------------------------------------------------------------------ vector kernels
// per-block partial sums of the two species' dot products, accumulated in
// FP64; per run, a and b advance by n and part by one run's slots.  A thread
// adds its elements i, i + stride, ... in that order; it loads four of them
// at a time, so a pass costs one memory round trip, not four.
// this thread's share of the two species' dot products a . b: elements i0,
// i0 + stride, ... in that order, four loads in flight per pass
template <class T>
__device__ inline double2 dot_share(int n, const pair_t<T> *__restrict__ a,
                                    const pair_t<T> *__restrict__ b, int i0, int stride)
{
    double2 acc = d2(0.0, 0.0);
    int i = i0;
    for (; i + 3 * stride < n; i += 4 * stride) {
        pair_t<T> x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[u] = a[i + u * stride];
            y[u] = b[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc.x = fmad(double(x[u].x), double(y[u].x), acc.x);
            acc.y = fmad(double(x[u].y), double(y[u].y), acc.y);
        }
    }
    for (; i < n; i += stride) {
        const pair_t<T> x = a[i], y = b[i];
        acc.x = fmad(double(x.x), double(y.x), acc.x);
        acc.y = fmad(double(x.y), double(y.y), acc.y);
    }
    return acc;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_dot(int n, const pair_t<T> *__restrict__ a,
                                                const pair_t<T> *__restrict__ b, double2 *part)
{
    __shared__ double2 sh[kBlock / 64];
    a = run_at(a, n);
    b = run_at(b, n);
    part = run_at(part, kSlotStride);
    const double2 acc = dot_share<T>(n, a, b, blockIdx.x * kBlock + threadIdx.x,
                                     gridDim.x * kBlock);
    const double2 s = block_sum(acc, sh);
    if (threadIdx.x == 0)
        part[blockIdx.x] = s;
}

// two dot products a1 . b1 and a2 . b2 in one launch, each with the partials
// k_dot writes for it (the same elements per thread, the same order)
template <class T>
__global__ void __launch_bounds__(kBlock) k_dot2(int n, const pair_t<T> *__restrict__ a1,
                                                 const pair_t<T> *__restrict__ b1, double2 *part1,
                                                 const pair_t<T> *__restrict__ a2,
                                                 const pair_t<T> *__restrict__ b2, double2 *part2)
{
    __shared__ double2 sh[kBlock / 64];
    a1 = run_at(a1, n);
    b1 = run_at(b1, n);
    a2 = run_at(a2, n);
    b2 = run_at(b2, n);
    part1 = run_at(part1, kSlotStride);
    part2 = run_at(part2, kSlotStride);
    const int i0 = blockIdx.x * kBlock + threadIdx.x, stride = gridDim.x * kBlock;
    const double2 acc1 = dot_share<T>(n, a1, b1, i0, stride);
    const double2 acc2 = dot_share<T>(n, a2, b2, i0, stride);
    const double2 s1 = block_sum(acc1, sh);
    const double2 s2 = block_sum(acc2, sh);
    if (threadIdx.x == 0) {
        part1[blockIdx.x] = s1;
        part2[blockIdx.x] = s2;
    }
}

// per run, a and b advance by n
template <class P>
__global__ void __launch_bounds__(kBlock) k_copy(int n, const P *__restrict__ a, P *b)
{
    const int row = blockIdx.x * kBlock + threadIdx.x;
    if (row < n)
        run_at(b, n)[row] = run_at(a, n)[row];
}

}  // namespace
}  // namespace chm
