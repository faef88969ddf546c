// Smoothed-aggregation AMG setup on the GPU (Vanek, Mandel and Brezina 1996),
// realising the AMG solves of Algorithm 1 of the paper.
//
// Per level, with A the level operator and B the near-null vector (constants
// on the finest level):
//   * D^-1 and the Gershgorin bound rho = max_i sum_j |a_ij| / a_ii of the
//     spectrum of D^-1 A;
//   * roots: a distance-2 maximal independent set of the matrix graph found in
//     synchronous rounds (Bell, Dalton and Olson 2012): each vertex carries
//     (state, hash, index) with state IN > UNDECIDED > OUT, two sweeps of
//     "max over self and neighbours" give every vertex the largest tuple
//     within distance 2, an undecided vertex that sees its own tuple joins
//     the set and one that sees an IN tuple leaves it.  The hash is the
//     SplitMix64 output of the vertex index.  Decisions use the sparsity
//     pattern only, so they are exact integer decisions;
//   * aggregates: each root with its neighbours; every other vertex joins the
//     neighbouring first-pass aggregate with the smallest number;
//   * tentative prolongator T[i, agg(i)] = B_i / ||B on agg(i)||, next B =
//     those norms;
//   * P = (I - 4/(3 rho) D^-1 A) T, R = P^T, A_c = R (A P).
// Sparse products are formed row by row: the products of a row are expanded
// in loop order, sorted by the key (column << 32 | position) and summed, so
// equal columns are added in loop order and the result does not depend on
// thread timing.
#include <cmath>

#include "chm_internal.h"

namespace chm {

namespace {

enum : int { OUT = 0, UND = 1, IN = 2 };

inline int nblk(long n, int bs = kBlock) { return (int)std::max<long>(1, (n + bs - 1) / bs); }

// The residual-and-restriction product RR = [R | -R A] is formed where its
// rows average at most this many entries (two passes of four entries on 32
// lanes); longer rows (3D patterns) run faster as the two products.
constexpr double kFuseRowMax = 256.0;
// R A is formed to try the fusion only on levels whose A averages at most this
// many entries per row: the 2D P1 levels (7 and 11.3 entries) give RR rows of
// 72 and 139, the 3D ones (15 and 40 entries) rows of 339 and 1,112, so on a
// 3D hierarchy the product was formed only to be thrown away.
constexpr double kFuseArow = 12.0;

__device__ inline uint64_t splitmix_at(uint64_t i)
{
    uint64_t z = (i + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Tup {
    uint64_t h;
    int state;
    int idx;
};

__device__ inline bool tup_gt(const Tup &a, const Tup &b)
{
    if (a.state != b.state)
        return a.state > b.state;
    if (a.h != b.h)
        return a.h > b.h;
    return a.idx > b.idx;
}

__global__ void k_diag(const int *rp, const int *ci, const double *v, int n, double *dinv,
                       double *ratio, int *bad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double d = 0.0, s = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        if (ci[k] == i)
            d = v[k];
        s += fabs(v[k]);
    }
    if (!(d > 0.0)) {
        atomicAdd(bad, 1);
        d = 1.0;
    }
    dinv[i] = 1.0 / d;
    ratio[i] = s / d;
}

__global__ void k_mis_init(const int *state, int n, Tup *t)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    Tup x;
    x.h = splitmix_at((uint64_t)i);
    x.state = state[i];
    x.idx = i;
    t[i] = x;
}

__global__ void k_mis_sweep(const int *rp, const int *ci, int n, const Tup *tin, Tup *tout)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    Tup best = tin[i];
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        Tup c = tin[ci[k]];
        if (tup_gt(c, best))
            best = c;
    }
    tout[i] = best;
}

__global__ void k_mis_update(int *state, const Tup *t, int n, int *undecided)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool still = false;
    if (i < n && state[i] == UND) {
        const Tup b = t[i];
        if (b.idx == i)
            state[i] = IN;
        else if (b.state == IN)
            state[i] = OUT;
        else
            still = true;
    }
    // one atomic per wave for the count of vertices still undecided
    const unsigned long long m = __ballot(still);
    if ((threadIdx.x & 63) == 0 && m)
        atomicAdd(undecided, __popcll(m));
}

__global__ void k_root_flags(const int *state, int n, int *flag)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        flag[i] = state[i] == IN ? 1 : 0;
}

__global__ void k_first_pass(const int *rp, const int *ci, const int *state, const int *rootid,
                             int n, int *first)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int f = -1;
    if (state[i] == IN) {
        f = rootid[i];
    } else {
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (state[ci[k]] == IN)
                f = rootid[ci[k]];
    }
    first[i] = f;
}

__global__ void k_second_pass(const int *rp, const int *ci, const int *first, int n, int *agg,
                              int *bad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int a = first[i];
    if (a < 0) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            int c = first[ci[k]];
            if (c >= 0 && (a < 0 || c < a))
                a = c;
        }
        if (a < 0) {
            atomicAdd(bad, 1);
            a = 0;
        }
    }
    agg[i] = a;
}

__global__ void k_count_keys(const int *key, int n, int *cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        atomicAdd(&cnt[key[i]], 1);
}

__global__ void k_bucket_fill(const int *key, int n, int *cursor, int *members)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        members[atomicAdd(&cursor[key[i]], 1)] = i;
}

__global__ void k_sort_int_segments(int *v, const int *ptr, int n)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    int b = ptr[s], e = ptr[s + 1];
    for (int k = b + 1; k < e; ++k) {
        int key = v[k], j = k - 1;
        while (j >= b && v[j] > key) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = key;
    }
}

// B_c[a] = sqrt(sum over members i of a, ascending, of B_i^2)
__global__ void k_agg_norm(const int *mptr, const int *members, const double *B, int nc, double *Bn)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nc)
        return;
    double s = 0.0;
    for (int k = mptr[a]; k < mptr[a + 1]; ++k) {
        double b = B[members[k]];
        s += b * b;
    }
    Bn[a] = sqrt(s);
}

__global__ void k_tentative(const double *B, const double *Bn, const int *agg, int n, double *t)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        t[i] = B[i] / Bn[agg[i]];
}

// heap sort of 64-bit keys in place
__device__ void heap_sort(uint64_t *a, int n)
{
    for (int start = n / 2 - 1; start >= 0; --start) {
        int root = start;
        for (;;) {
            int child = 2 * root + 1;
            if (child >= n)
                break;
            if (child + 1 < n && a[child + 1] > a[child])
                ++child;
            if (a[root] >= a[child])
                break;
            uint64_t tmp = a[root];
            a[root] = a[child];
            a[child] = tmp;
            root = child;
        }
    }
    for (int end = n - 1; end > 0; --end) {
        uint64_t tmp = a[0];
        a[0] = a[end];
        a[end] = tmp;
        int root = 0;
        for (;;) {
            int child = 2 * root + 1;
            if (child >= end)
                break;
            if (child + 1 < end && a[child + 1] > a[child])
                ++child;
            if (a[root] >= a[child])
                break;
            uint64_t t2 = a[root];
            a[root] = a[child];
            a[child] = t2;
            root = child;
        }
    }
}

// ---- P = (I - omega D^-1 A) T, T given by (agg, t) ----
__global__ void k_p_count(const int *rp, int n, int *cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        cnt[i] = rp[i + 1] - rp[i];
}

__global__ void k_p_expand(const int *rp, const int *ci, const double *v, const double *dinv,
                           const int *agg, const double *t, double omega, int n, const int *off,
                           uint64_t *keys, double *vals)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int o = off[i];
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        int j = ci[k];
        double s = (j == i ? 1.0 : 0.0) - omega * dinv[i] * v[k];
        int p = k - rp[i];
        keys[o + p] = ((uint64_t)(unsigned)agg[j] << 32) | (unsigned)p;
        vals[o + p] = s * t[j];
    }
}

// ---- generic row-wise product C = A B ----
__global__ void k_prod_count(const int *arp, const int *aci, const int *brp, int n, int *cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int c = 0;
    for (int k = arp[i]; k < arp[i + 1]; ++k)
        c += brp[aci[k] + 1] - brp[aci[k]];
    cnt[i] = c;
}

__global__ void k_prod_expand(const int *arp, const int *aci, const double *av, const int *brp,
                              const int *bci, const double *bv, int n, const int *off,
                              uint64_t *keys, double *vals)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int o = off[i], p = 0;
    for (int k = arp[i]; k < arp[i + 1]; ++k) {
        int j = aci[k];
        double a = av[k];
        for (int l = brp[j]; l < brp[j + 1]; ++l) {
            keys[o + p] = ((uint64_t)(unsigned)bci[l] << 32) | (unsigned)p;
            vals[o + p] = a * bv[l];
            ++p;
        }
    }
}

// sort each row's keys, count distinct columns
__global__ void k_rows_sort_count(const int *off, int n, uint64_t *keys, int *rowlen)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int b = off[i], e = off[i + 1];
    heap_sort(keys + b, e - b);
    int u = 0;
    unsigned prev = 0xffffffffu;
    for (int k = b; k < e; ++k) {
        unsigned c = (unsigned)(keys[k] >> 32);
        if (k == b || c != prev)
            ++u;
        prev = c;
    }
    rowlen[i] = u;
}

// Rows of a product with at most kDenseCols columns (the coarse levels, whose
// expanded rows can hold 10^5 entries): one block per row.  Every thread
// scans the row's entries in position order and accumulates those of its own
// columns (c mod kBlock) in LDS, so each column is summed in position order,
// exactly as the sorting path sums it.  phase 0 counts the row's distinct
// columns; phase 1 (after the scan of the counts) writes the row in column
// order.
constexpr int kDenseCols = 4096;

__global__ void __launch_bounds__(kBlock) k_rows_dense(const int *__restrict__ off,
                                                       const uint64_t *__restrict__ keys,
                                                       const double *__restrict__ vals, int ncols,
                                                       int phase, int *rowlen,
                                                       const int *__restrict__ crp, int *cci,
                                                       double *cv)
{
    __shared__ double acc[kDenseCols];
    __shared__ unsigned char present[kDenseCols];
    __shared__ int part[kBlock];
    const int i = blockIdx.x, t = threadIdx.x;
    for (int c = t; c < ncols; c += kBlock)
        present[c] = 0;
    __syncthreads();
    const int b = off[i], e = off[i + 1];
#pragma unroll 8
    for (int k = b; k < e; ++k) {
        const int c = (int)(keys[k] >> 32);
        if (c % kBlock == t) {
            if (present[c])
                acc[c] += vals[k];
            else
                acc[c] = vals[k];
            present[c] = 1;
        }
    }
    __syncthreads();
    // thread t takes the columns [t ch, (t + 1) ch) for the count and the output
    const int ch = (ncols + kBlock - 1) / kBlock, c0 = min(t * ch, ncols), c1 = min(c0 + ch, ncols);
    int cnt = 0;
    for (int c = c0; c < c1; ++c)
        cnt += present[c];
    part[t] = cnt;
    __syncthreads();
    if (phase == 0) {
        if (t == 0) {
            int tot = 0;
            for (int k = 0; k < kBlock; ++k)
                tot += part[k];
            rowlen[i] = tot;
        }
        return;
    }
    int o = crp[i];
    for (int k = 0; k < t; ++k)
        o += part[k];
    for (int c = c0; c < c1; ++c)
        if (present[c]) {
            cci[o] = c;
            cv[o] = acc[c];
            ++o;
        }
}

// sum equal columns in position order and write the row
__global__ void k_rows_compress(const int *off, int n, const uint64_t *keys, const double *vals,
                                const int *crp, int *cci, double *cv)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int b = off[i], e = off[i + 1], o = crp[i] - 1;
    unsigned prev = 0xffffffffu;
    for (int k = b; k < e; ++k) {
        unsigned c = (unsigned)(keys[k] >> 32);
        double x = vals[b + (int)(keys[k] & 0xffffffffu)];
        if (k == b || c != prev) {
            ++o;
            cci[o] = (int)c;
            cv[o] = x;
        } else {
            cv[o] += x;
        }
        prev = c;
    }
}

// ---- [A1 | s A2]: per row, A1's entries, then those of A2 with their
// columns shifted by n (A1's column count) and their values times s ----
__global__ void __launch_bounds__(kBlock) k_rr_count(const int *__restrict__ rp1,
                                                     const int *__restrict__ rp2, int m, int *rp)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < m)
        rp[i] = (rp1[i + 1] - rp1[i]) + (rp2[i + 1] - rp2[i]);
}

__global__ void __launch_bounds__(kBlock) k_rr_fill(const int *__restrict__ rp1,
                                                    const int *__restrict__ ci1,
                                                    const double *__restrict__ v1,
                                                    const int *__restrict__ rp2,
                                                    const int *__restrict__ ci2,
                                                    const double *__restrict__ v2, int m, int n,
                                                    double sign, const int *__restrict__ rp,
                                                    int *ci, double *v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= m)
        return;
    int o = rp[i];
    for (int k = rp1[i]; k < rp1[i + 1]; ++k, ++o) {
        ci[o] = ci1[k];
        v[o] = v1[k];
    }
    for (int k = rp2[i]; k < rp2[i + 1]; ++k, ++o) {
        ci[o] = n + ci2[k];
        v[o] = sign * v2[k];
    }
}

// ---- transpose: counting by column, rows filled then sorted by row index ----
__global__ void k_t_fill(const int *rp, const int *ci, const double *v, int n, int *cursor,
                         int *tci, double *tv)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        int pos = atomicAdd(&cursor[ci[k]], 1);
        tci[pos] = i;
        tv[pos] = v[k];
    }
}

// heap sort of (key, value) pairs by key (the keys of a segment are distinct,
// so the order is unique)
__device__ void heap_sort_pairs(int *key, double *val, int n)
{
    auto sift = [&](int root, int end) {
        for (;;) {
            int child = 2 * root + 1;
            if (child >= end)
                break;
            if (child + 1 < end && key[child + 1] > key[child])
                ++child;
            if (key[root] >= key[child])
                break;
            const int tk = key[root];
            key[root] = key[child];
            key[child] = tk;
            const double tv = val[root];
            val[root] = val[child];
            val[child] = tv;
            root = child;
        }
    };
    for (int start = n / 2 - 1; start >= 0; --start)
        sift(start, n);
    for (int end = n - 1; end > 0; --end) {
        const int tk = key[0];
        key[0] = key[end];
        key[end] = tk;
        const double tv = val[0];
        val[0] = val[end];
        val[end] = tv;
        sift(0, end);
    }
}

__global__ void k_sort_pairs_segments(int *key, double *val, const int *ptr, int n)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n)
        return;
    const int b = ptr[s];
    heap_sort_pairs(key + b, val + b, ptr[s + 1] - b);
}

// ---- coarsest level: Gauss-Jordan inverse of an SPD matrix (no pivoting) ----
__global__ void k_dense_from_csr(const int *rp, const int *ci, const double *v, int n, double *aug)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double *row = aug + (size_t)i * 2 * n;
    for (int j = 0; j < 2 * n; ++j)
        row[j] = (j == n + i) ? 1.0 : 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
        row[ci[k]] = v[k];
}

constexpr int kGJMax = 2048;

// ---- blocked Gauss-Jordan on [A | I] (n x 2n, row-major) in steps of kGB
// pivots: the pivot block's inverse Dinv (one workgroup, in LDS), the new
// pivot rows Rb = Dinv [A | I](pivot rows), and the rank-kGB update of every
// other row, [A | I](i, :) -= C(i, :) Rb with C the pivot columns before the
// step, on FP64 matrix cores (16x16x4 MFMA tiles).  No pivoting: every pivot
// block of an SPD matrix is SPD.
constexpr int kGB = 32;

__global__ void __launch_bounds__(kBlock) k_bgj_diag(int n, const double *__restrict__ aug, int k0,
                                                     int kb, double *dinv, int *bad)
{
    __shared__ double a[kGB][2 * kGB];
    constexpr int kPer = kGB * 2 * kGB / kBlock;   // elements per thread
    const int w = 2 * n, t = threadIdx.x;
    for (int idx = t; idx < kGB * 2 * kGB; idx += kBlock) {
        const int r = idx / (2 * kGB), c = idx % (2 * kGB);
        double v = 0.0;
        if (r < kb && c < kb)
            v = aug[(size_t)(k0 + r) * w + k0 + c];
        else if (r < kb && c >= kGB && c - kGB < kb)
            v = (c - kGB == r) ? 1.0 : 0.0;
        a[r][c] = v;
    }
    __syncthreads();
    int badp = 0;
    for (int p = 0; p < kb; ++p) {
        double piv = a[p][p];
        if (!(piv > 0.0)) {
            badp = 1;
            piv = 1.0;
        }
        double nv[kPer];
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int idx = t + e * kBlock, r = idx / (2 * kGB), c = idx % (2 * kGB);
            const double rowp = a[p][c] / piv;
            nv[e] = r == p ? rowp : a[r][c] - a[r][p] * rowp;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int idx = t + e * kBlock;
            a[idx / (2 * kGB)][idx % (2 * kGB)] = nv[e];
        }
        __syncthreads();
    }
    if (badp && t == 0)
        atomicAdd(bad, 1);
    for (int idx = t; idx < kGB * kGB; idx += kBlock) {
        const int r = idx / kGB, c = idx % kGB;
        dinv[idx] = (r < kb && c < kb) ? a[r][kGB + c] : 0.0;
    }
}

// Rb (kGB x w) = Dinv times the pivot rows (rows past kb are zero); C (n x kGB)
// = the pivot columns of every row before the step (columns past kb zero)
__global__ void __launch_bounds__(kBlock) k_bgj_rows(int n, const double *__restrict__ aug, int k0,
                                                     int kb, const double *__restrict__ dinv,
                                                     double *rb, double *cc)
{
    const int w = 2 * n;
    const long t = (long)blockIdx.x * kBlock + threadIdx.x;
    if (t < w) {
        const int j = (int)t;
        double col[kGB];
#pragma unroll
        for (int s = 0; s < kGB; ++s)
            col[s] = s < kb ? aug[(size_t)(k0 + s) * w + j] : 0.0;
        for (int r = 0; r < kGB; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < kGB; ++s)
                acc += dinv[r * kGB + s] * col[s];
            rb[(size_t)r * w + j] = acc;
        }
    }
    if (t < (long)n * kGB) {
        const int i = (int)(t / kGB), s = (int)(t % kGB);
        cc[t] = s < kb ? aug[(size_t)i * w + k0 + s] : 0.0;
    }
}

typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

// one wave per 16 x 16 tile of [A | I]: rows outside the pivot block take
// aug - C Rb (8 MFMA steps of K = 4), the pivot rows take Rb.  Lane l holds
// C(i0 + l % 16, 4 q + l / 16), Rb(4 q + l / 16, j0 + l % 16) and the results
// (i0 + 4 e + l / 16, j0 + l % 16), e = 0..3.
__global__ void __launch_bounds__(kBlock) k_bgj_update(int n, double *aug, int k0, int kb,
                                                       const double *__restrict__ rb,
                                                       const double *__restrict__ cc)
{
    const int w = 2 * n, lane = threadIdx.x & 63;
    const int ct = (w + 15) / 16, rt = (n + 15) / 16;
    const long tile = (long)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (tile >= (long)rt * ct)
        return;   // the whole wave
    const int i0 = (int)(tile / ct) * 16, j0 = (int)(tile % ct) * 16;
    const int lr = lane % 16, lq = lane / 16, col = j0 + lr;
    mfma_f64x4 acc;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = i0 + 4 * e + lq;
        acc[e] = (row < n && col < w) ? aug[(size_t)row * w + col] : 0.0;
    }
    const int arow = i0 + lr;
#pragma unroll
    for (int q = 0; q < kGB / 4; ++q) {
        const int s = 4 * q + lq;
        const double av = arow < n ? -cc[(size_t)arow * kGB + s] : 0.0;
        const double bv = col < w ? rb[(size_t)s * w + col] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = i0 + 4 * e + lq;
        if (row < n && col < w)
            aug[(size_t)row * w + col] =
                (row >= k0 && row < k0 + kb) ? rb[(size_t)(row - k0) * w + col] : acc[e];
    }
}

// inverse, row-major: inv[i * n + j] = (A^-1)[i][j]
__global__ void k_extract_inverse(const double *aug, int n, double *inv)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n)
        return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    inv[idx] = aug[(size_t)i * 2 * n + n + j];
}

struct Scratch {   // expansion buffers of one product
    uint64_t *keys = nullptr;
    double *vals = nullptr;
    int *off = nullptr;
};

// C = rows expanded in (keys, vals) with offsets off (n + 1 entries)
void finish_rows(int n, int ncols, Scratch &sc, Csr &C, Pool &pool, hipStream_t st)
{
    C.n = n;
    C.m = ncols;
    C.rp = pool.get<int>(n + 1);
    const bool dense = ncols <= kDenseCols && n > 0;
    if (dense)
        k_rows_dense<<<n, kBlock, 0, st>>>(sc.off, sc.keys, sc.vals, ncols, 0, C.rp, nullptr,
                                           nullptr, nullptr);
    else
        k_rows_sort_count<<<nblk(n), kBlock, 0, st>>>(sc.off, n, sc.keys, C.rp);
    CHM_HIP(hipGetLastError());
    scan_exclusive(C.rp, n, C.rp + n, pool, st);
    C.nnz = read_int(C.rp + n, st);
    C.ci = pool.get<int>(C.nnz);
    C.v = pool.get<double>(C.nnz);
    if (dense)
        k_rows_dense<<<n, kBlock, 0, st>>>(sc.off, sc.keys, sc.vals, ncols, 1, nullptr, C.rp,
                                           C.ci, C.v);
    else
        k_rows_compress<<<nblk(n), kBlock, 0, st>>>(sc.off, n, sc.keys, sc.vals, C.rp, C.ci, C.v);
    CHM_HIP(hipGetLastError());
}

void spgemm(const Csr &A, const Csr &B, Csr &C, Pool &pool, Pool &tmp, hipStream_t st)
{
    Scratch sc;
    sc.off = tmp.get<int>(A.n + 1);
    k_prod_count<<<nblk(A.n), kBlock, 0, st>>>(A.rp, A.ci, B.rp, A.n, sc.off);
    CHM_HIP(hipGetLastError());
    scan_exclusive(sc.off, A.n, sc.off + A.n, tmp, st);
    int total = read_int(sc.off + A.n, st);
    sc.keys = tmp.get<uint64_t>(total);
    sc.vals = tmp.get<double>(total);
    k_prod_expand<<<nblk(A.n), kBlock, 0, st>>>(A.rp, A.ci, A.v, B.rp, B.ci, B.v, A.n, sc.off,
                                                 sc.keys, sc.vals);
    CHM_HIP(hipGetLastError());
    finish_rows(A.n, B.m, sc, C, pool, st);
}

void transpose(const Csr &A, Csr &T, Pool &pool, Pool &tmp, hipStream_t st)
{
    T.n = A.m;
    T.m = A.n;
    T.nnz = A.nnz;
    T.rp = pool.get<int>(T.n + 1);
    fill_int(T.rp, 0, T.n + 1, st);
    k_count_keys<<<nblk(A.nnz), kBlock, 0, st>>>(A.ci, A.nnz, T.rp);
    CHM_HIP(hipGetLastError());
    scan_exclusive(T.rp, T.n, T.rp + T.n, tmp, st);
    int *cursor = tmp.get<int>(T.n);
    CHM_HIP(hipMemcpyAsync(cursor, T.rp, sizeof(int) * T.n, hipMemcpyDeviceToDevice, st));
    T.ci = pool.get<int>(T.nnz);
    T.v = pool.get<double>(T.nnz);
    k_t_fill<<<nblk(A.n), kBlock, 0, st>>>(A.rp, A.ci, A.v, A.n, cursor, T.ci, T.v);
    k_sort_pairs_segments<<<nblk(T.n), kBlock, 0, st>>>(T.ci, T.v, T.rp, T.n);
    CHM_HIP(hipGetLastError());
}

// Chebyshev recurrence coefficients (Saad, Iterative Methods, Algorithm 12.1)
// for the interval [rho/ratio, rho]: step 1 is d = D^-1 r / theta, step k >= 2
// is d = c1[k] d + c2[k] D^-1 r; every step then adds d to x.
void chebyshev_coefficients(Level &L, int degree, double ratio)
{
    double lmax = L.rho, lmin = L.rho / ratio;
    double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    double sigma = theta / delta, rho_old = 1.0 / sigma;
    L.cheb_c1[1] = 0.0;
    L.cheb_c2[1] = 1.0 / theta;
    for (int k = 2; k <= degree; ++k) {
        double rho = 1.0 / (2.0 * sigma - rho_old);
        L.cheb_c1[k] = rho * rho_old;
        L.cheb_c2[k] = 2.0 * rho / delta;
        rho_old = rho;
    }
    L.jac_omega = 4.0 / (3.0 * L.rho);
}

}  // namespace

// One lane per row (SELL-64) for rows the unrolled SELL path covers (up to
// 16 entries: the fine levels of P1 meshes in 2D and 3D) when there are
// enough rows to fill the chip; otherwise a power-of-two group of lanes per
// row, enough to reach about 128k threads and to cover an average row in two
// passes of four entries per lane, but no wider than the rows.
int lanes_per_row(const Csr &A)
{
    const double avg = A.n > 0 ? double(A.nnz) / A.n : 0.0;
    const long target = 131072;
    if (avg < 16.0 && A.n >= target)
        return 0;
    int want = 4;
    while (want < 32 && ((long)want * A.n < target || want * 8 < avg))
        want *= 2;
    int cap = 4;
    while (cap < 32 && cap < avg)
        cap *= 2;
    return std::min(want, cap);
}

// entries per CSR lane and pass: about the average row length over the
// lanes, so short rows do not load padding and long rows keep four loads in
// flight per lane
int unroll(const Csr &A, int gs)
{
    const double per_lane = (gs > 0 && A.n > 0) ? double(A.nnz) / A.n / gs : 1.0;
    return per_lane > 2.0 ? 4 : (per_lane > 1.0 ? 2 : 1);
}

// [A1 | s A2] row by row (A1, A2 with the same rows; A2's columns shifted by
// the column count of A1), into pool
void concat_rows(const Csr &A1, const Csr &A2, double sign, Csr &C, Pool &pool, Pool &tmp,
                 hipStream_t st)
{
    const int m = A1.n;
    C.n = m;
    C.m = A1.m + A2.m;
    C.rp = pool.get<int>(m + 1);
    k_rr_count<<<nblk(m), kBlock, 0, st>>>(A1.rp, A2.rp, m, C.rp);
    CHM_HIP(hipGetLastError());
    scan_exclusive(C.rp, m, C.rp + m, tmp, st);
    C.nnz = read_int(C.rp + m, st);
    C.ci = pool.get<int>(std::max(1, C.nnz));
    C.v = pool.get<double>(std::max(1, C.nnz));
    k_rr_fill<<<nblk(m), kBlock, 0, st>>>(A1.rp, A1.ci, A1.v, A2.rp, A2.ci, A2.v, m, A1.m, sign,
                                           C.rp, C.ci, C.v);
    CHM_HIP(hipGetLastError());
}

void amg_build(Solver &S, Hierarchy &H, const Csr &A0)
{
    hipStream_t st = S.stream;
    Pool &pool = S.pool;
    const int max_levels = std::min(S.prm.max_levels, kMaxLevels);
    int *flags = pool.get<int>(4);
    double *B = pool.get<double>(A0.n);
    fill_double(B, 1.0, A0.n, st);   // constants: near-null space of the stiffness part
    H.nlev = 1;
    H.lev[0] = Level();
    H.lev[0].n = A0.n;
    H.lev[0].A = A0;
    for (int l = 0;; ++l) {
        Pool tmp;   // per-level scratch, freed at the end of the iteration
        Level &L = H.lev[l];
        const Csr &A = L.A;
        const int n = L.n;
        fill_int(flags, 0, 4, st);
        L.dinv = pool.get<double>(n);
        double *ratio = tmp.get<double>(n);
        k_diag<<<nblk(n), kBlock, 0, st>>>(A.rp, A.ci, A.v, n, L.dinv, ratio, flags);
        CHM_HIP(hipGetLastError());
        L.rho = reduce_max_host(ratio, n, tmp, st);
        if (read_int(flags, st))
            throw Failure(CHM_EINVAL, "AMG level " + std::to_string(l) + " has a non-positive diagonal");
        L.degree = (l > 0 && H.degree_coarse > 0) ? H.degree_coarse : H.degree;
        chebyshev_coefficients(L, L.degree, H.ratio);
        if (n <= S.prm.coarse_max || l + 1 >= max_levels)
            break;

        // distance-2 maximal independent set in synchronous rounds
        int *state = tmp.get<int>(n);
        fill_int(state, UND, n, st);
        Tup *t0 = tmp.get<Tup>(n), *t1 = tmp.get<Tup>(n);
        for (int round = 0;; ++round) {
            k_mis_init<<<nblk(n), kBlock, 0, st>>>(state, n, t0);
            k_mis_sweep<<<nblk(n), kBlock, 0, st>>>(A.rp, A.ci, n, t0, t1);
            k_mis_sweep<<<nblk(n), kBlock, 0, st>>>(A.rp, A.ci, n, t1, t0);
            fill_int(flags + 1, 0, 1, st);
            k_mis_update<<<nblk(n), kBlock, 0, st>>>(state, t0, n, flags + 1);
            CHM_HIP(hipGetLastError());
            if (read_int(flags + 1, st) == 0)
                break;
            if (round > 10000)
                throw Failure(CHM_EINVAL, "aggregation did not terminate");
        }
        // aggregates
        int *rootid = tmp.get<int>(n + 1);
        k_root_flags<<<nblk(n), kBlock, 0, st>>>(state, n, rootid);
        scan_exclusive(rootid, n, rootid + n, tmp, st);
        const int nc = read_int(rootid + n, st);
        if (nc <= 0 || nc >= n)
            break;   // no coarsening possible: this level becomes the coarsest
        int *first = tmp.get<int>(n);
        L.agg = pool.get<int>(n);
        k_first_pass<<<nblk(n), kBlock, 0, st>>>(A.rp, A.ci, state, rootid, n, first);
        k_second_pass<<<nblk(n), kBlock, 0, st>>>(A.rp, A.ci, first, n, L.agg, flags + 2);
        CHM_HIP(hipGetLastError());
        if (read_int(flags + 2, st))
            throw Failure(CHM_EINVAL, "aggregation left a vertex unassigned");
        L.nc = nc;

        // aggregate norms of B (members summed in ascending index order)
        int *mptr = tmp.get<int>(nc + 1);
        fill_int(mptr, 0, nc + 1, st);
        k_count_keys<<<nblk(n), kBlock, 0, st>>>(L.agg, n, mptr);
        scan_exclusive(mptr, nc, mptr + nc, tmp, st);
        int *cursor = tmp.get<int>(nc);
        CHM_HIP(hipMemcpyAsync(cursor, mptr, sizeof(int) * nc, hipMemcpyDeviceToDevice, st));
        int *members = tmp.get<int>(n);
        k_bucket_fill<<<nblk(n), kBlock, 0, st>>>(L.agg, n, cursor, members);
        k_sort_int_segments<<<nblk(nc), kBlock, 0, st>>>(members, mptr, nc);
        double *Bn = pool.get<double>(nc);
        k_agg_norm<<<nblk(nc), kBlock, 0, st>>>(mptr, members, B, nc, Bn);
        double *tv = tmp.get<double>(n);
        k_tentative<<<nblk(n), kBlock, 0, st>>>(B, Bn, L.agg, n, tv);
        CHM_HIP(hipGetLastError());

        // smoothed prolongator
        Scratch sc;
        sc.off = tmp.get<int>(n + 1);
        k_p_count<<<nblk(n), kBlock, 0, st>>>(A.rp, n, sc.off);
        scan_exclusive(sc.off, n, sc.off + n, tmp, st);
        sc.keys = tmp.get<uint64_t>(A.nnz);
        sc.vals = tmp.get<double>(A.nnz);
        k_p_expand<<<nblk(n), kBlock, 0, st>>>(A.rp, A.ci, A.v, L.dinv, L.agg, tv, L.jac_omega, n,
                                               sc.off, sc.keys, sc.vals);
        CHM_HIP(hipGetLastError());
        finish_rows(n, nc, sc, L.P, pool, st);
        transpose(L.P, L.R, pool, tmp, st);

        // Galerkin coarse operator A_c = R (A P)
        Csr AP;
        Pool tmp2;
        spgemm(A, L.P, AP, tmp2, tmp, st);
        // RR = [R | -R A] for the residual and its restriction in one
        // product, where its rows are short enough (R A holds at least R's
        // entries, so R's rows bound it from below), and only tried on levels
        // whose A rows are short
        if (A.nnz <= kFuseArow * (double)n && 2.0 * L.R.nnz <= kFuseRowMax * (double)nc) {
            Csr RA;
            spgemm(L.R, A, RA, tmp2, tmp, st);
            if ((double)L.R.nnz + RA.nnz <= kFuseRowMax * (double)nc)
                concat_rows(L.R, RA, -1.0, L.RR, pool, tmp, st);
        }
        // AM = [A | A P] for the prolongation and the first post-smoothing
        // step in one product, on CSR levels with short enough rows
        if (lanes_per_row(A) > 0 && (double)A.nnz + AP.nnz <= kFuseRowMax * (double)n)
            concat_rows(A, AP, 1.0, L.AM, pool, tmp, st);
        Level &C = H.lev[l + 1];
        C = Level();
        C.n = nc;
        spgemm(L.R, AP, C.A, pool, tmp, st);
        CHM_HIP(hipStreamSynchronize(st));   // scratch pools are freed on return
        H.nlev = l + 2;
        B = Bn;
    }

    // coarsest level: explicit inverse
    Level &Lc = H.lev[H.nlev - 1];
    const int nc = Lc.n;
    if (nc > kGJMax)
        throw Failure(CHM_EINVAL, "coarsest AMG level has " + std::to_string(nc) +
                                      " rows (limit 2048): raise max_levels or coarse_max");
    {
        Pool tmp;
        double *aug = tmp.get<double>((size_t)nc * 2 * nc);
        k_dense_from_csr<<<nblk(nc), kBlock, 0, st>>>(Lc.A.rp, Lc.A.ci, Lc.A.v, nc, aug);
        fill_int(flags + 3, 0, 1, st);
        double *dinv = tmp.get<double>(kGB * kGB);
        double *rb = tmp.get<double>((size_t)kGB * 2 * nc), *cc = tmp.get<double>((size_t)nc * kGB);
        const long tiles = (long)((nc + 15) / 16) * ((2 * nc + 15) / 16);
        const long rows_threads = std::max<long>(2l * nc, (long)nc * kGB);
        for (int k0 = 0; k0 < nc; k0 += kGB) {
            const int kb = std::min(kGB, nc - k0);
            k_bgj_diag<<<1, kBlock, 0, st>>>(nc, aug, k0, kb, dinv, flags + 3);
            k_bgj_rows<<<nblk(rows_threads), kBlock, 0, st>>>(nc, aug, k0, kb, dinv, rb, cc);
            k_bgj_update<<<(int)((tiles + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, st>>>(
                nc, aug, k0, kb, rb, cc);
        }
        Lc.inv = pool.get<double>((size_t)nc * nc);
        k_extract_inverse<<<nblk((long)nc * nc), kBlock, 0, st>>>(aug, nc, Lc.inv);
        CHM_HIP(hipGetLastError());
        if (read_int(flags + 3, st))
            throw Failure(CHM_EINVAL, "coarsest AMG level is not positive definite");
        CHM_HIP(hipStreamSynchronize(st));
    }

    // SELL copies, kernel shapes and work vectors
    for (int l = 0; l < H.nlev; ++l) {
        Level &L = H.lev[l];
        const bool o16 = S.prm.wide_index == 0;
        csr_to_sell(L.A, L.sA, pool, st, o16);
        L.gsA = lanes_per_row(L.A);
        // the smoother's CSR levels take half the lanes where a lane still
        // holds at most 3 entries of an average row: the 2D level 1 (11.3
        // entries per row) runs its Chebyshev steps faster on 4 lanes than on
        // 8, the 3D one (40 entries) slower
        if (L.gsA > 4 && (double)L.A.nnz / L.n <= 3.0 * (L.gsA / 2))
            L.gsA /= 2;
        if (L.gsA == 0 && L.sA.ocol && !S.prm.values_direct)   // values through a table
            L.vtA = value_table(L.sA.val, L.sA.stored, pool, st);
        L.uA = unroll(L.A, L.gsA);
        if (l + 1 < H.nlev) {
            csr_to_sell(L.P, L.sP, pool, st, o16);
            csr_to_sell(L.R, L.sR, pool, st, o16);
            L.gsP = lanes_per_row(L.P);
            L.gsR = lanes_per_row(L.R);
            L.uP = unroll(L.P, L.gsP);
            L.uR = unroll(L.R, L.gsR);
            // RR is always a CSR-vector product (at least 4 lanes per row)
            L.gsRR = std::max(4, lanes_per_row(L.RR));
            L.uRR = unroll(L.RR, L.gsRR);
            L.gsAM = std::max(4, lanes_per_row(L.AM));
            L.uAM = unroll(L.AM, L.gsAM);
        }
        const size_t len = (size_t)S.nb * L.n;   // all runs of the batch
        H.x[l] = pool.get<double2>(len);
        H.xt[l] = pool.get<double2>(len);
        H.b[l] = pool.get<double2>(len);
        H.r[l] = pool.get<double2>(len);
    }
    CHM_HIP(hipStreamSynchronize(st));
}

}  // namespace chm
