// Small device utilities: exclusive scan, fills, max reduction, CSR -> SELL-64.
#include "chm_internal.h"

namespace chm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPerThread = 4;
constexpr int kScanTile = kScanThreads * kScanPerThread;

__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const int *in, int n, int *sums)
{
    __shared__ int sh[kScanThreads];
    const int t = threadIdx.x;
    const long base = (long)blockIdx.x * kScanTile + (long)t * kScanPerThread;
    int s = 0;
    for (int k = 0; k < kScanPerThread; ++k)
        if (base + k < n)
            s += in[base + k];
    sh[t] = s;
    __syncthreads();
    for (int off = kScanThreads / 2; off > 0; off >>= 1) {
        if (t < off)
            sh[t] += sh[t + off];
        __syncthreads();
    }
    if (t == 0)
        sums[blockIdx.x] = sh[0];
}

// exclusive scan of one tile, shifted by offsets[tile]; the last tile writes the total
__global__ void __launch_bounds__(kScanThreads) k_tile_scan(int *data, int n, const int *offsets,
                                                            int *total)
{
    __shared__ int sh[kScanThreads];
    const int t = threadIdx.x;
    const long base = (long)blockIdx.x * kScanTile + (long)t * kScanPerThread;
    int v[kScanPerThread];
    int s = 0;
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = (base + k < n) ? data[base + k] : 0;
        s += v[k];
    }
    sh[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int excl = sh[t] - s + (offsets ? offsets[blockIdx.x] : 0);
    for (int k = 0; k < kScanPerThread; ++k) {
        if (base + k < n)
            data[base + k] = excl;
        excl += v[k];
    }
    if (total && t == kScanThreads - 1 && blockIdx.x == gridDim.x - 1)
        *total = excl;
}

__global__ void k_fill_int(int *p, int v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void k_fill_double(double *p, double v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void __launch_bounds__(256) k_max_partial(const double *in, int n, double *out)
{
    __shared__ double sh[256];
    int t = threadIdx.x;
    double m = -1.0e300;
    for (int i = blockIdx.x * 256 + t; i < n; i += gridDim.x * 256)
        m = fmax(m, in[i]);
    sh[t] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off)
            sh[t] = fmax(sh[t], sh[t + off]);
        __syncthreads();
    }
    if (t == 0)
        out[blockIdx.x] = sh[0];
}

// width of each SELL slice, times the slice height
__global__ void k_slice_width(const int *rp, int n, int nslices, int *w)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslices)
        return;
    int r0 = s * kSlice, r1 = min(n, r0 + kSlice), mx = 0;
    for (int r = r0; r < r1; ++r)
        mx = max(mx, rp[r + 1] - rp[r]);
    w[s] = mx * kSlice;
}

__global__ void k_sell_fill(const int *rp, const int *ci, const double *v, int n, int nslices,
                            const int *sptr, int *col, double *val)
{
    int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nslices * kSlice)
        return;
    int s = row / kSlice, lane = row % kSlice;
    int base = sptr[s], width = (sptr[s + 1] - base) / kSlice;
    int b = 0, len = 0;
    if (row < n) {
        b = rp[row];
        len = rp[row + 1] - b;
    }
    // padding repeats the row's last column (a valid index of the input vector
    // for square and rectangular matrices alike) with value 0
    const int pad_col = len > 0 ? ci[b + len - 1] : 0;
    for (int k = 0; k < width; ++k) {
        int idx = base + k * kSlice + lane;
        if (k < len) {
            if (col)
                col[idx] = ci[b + k];
            val[idx] = v[b + k];
        } else {
            if (col)
                col[idx] = pad_col;
            val[idx] = 0.0;
        }
    }
}

__global__ void k_check_cols(const int *col, int64_t stored, int ncols, int *bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < stored && (col[i] < 0 || col[i] >= ncols))
        atomicAdd(bad, 1);
}

// col - row of every stored entry of the real rows as 16 bits (padding rows
// past n get 0 and are never read); bad is set when an offset does not fit
__global__ void k_sell_offsets(const int *sptr, const int *col, int n, int nslices,
                               int16_t *ocol, int *bad)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nslices * kSlice)
        return;
    const int s = row / kSlice, lane = row % kSlice;
    const int base = sptr[s], width = (sptr[s + 1] - base) / kSlice;
    for (int k = 0; k < width; ++k) {
        const int idx = base + k * kSlice + lane;
        int d = 0;
        if (row < n) {
            d = col[idx] - row;
            if (d < -32767 || d > 32767) {
                bad[0] = 1;
                d = 0;
            }
        }
        ocol[idx] = (int16_t)d;
    }
}

}  // namespace

void scan_exclusive(int *d, int n, int *d_total, Pool &pool, hipStream_t s)
{
    if (n <= 0) {
        if (d_total)
            fill_int(d_total, 0, 1, s);
        return;
    }
    int tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 1) {
        k_tile_scan<<<1, kScanThreads, 0, s>>>(d, n, nullptr, d_total);
        CHM_HIP(hipGetLastError());
        return;
    }
    int *sums = pool.get<int>(tiles);
    k_tile_sums<<<tiles, kScanThreads, 0, s>>>(d, n, sums);
    CHM_HIP(hipGetLastError());
    scan_exclusive(sums, tiles, nullptr, pool, s);
    k_tile_scan<<<tiles, kScanThreads, 0, s>>>(d, n, sums, d_total);
    CHM_HIP(hipGetLastError());
}

void fill_int(int *p, int v, size_t n, hipStream_t s)
{
    if (!n)
        return;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    k_fill_int<<<blocks, 256, 0, s>>>(p, v, n);
    CHM_HIP(hipGetLastError());
}

void fill_double(double *p, double v, size_t n, hipStream_t s)
{
    if (!n)
        return;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    k_fill_double<<<blocks, 256, 0, s>>>(p, v, n);
    CHM_HIP(hipGetLastError());
}

int read_int(const int *d, hipStream_t s)
{
    int v = 0;
    CHM_HIP(hipMemcpyAsync(&v, d, sizeof(int), hipMemcpyDeviceToHost, s));
    CHM_HIP(hipStreamSynchronize(s));
    return v;
}

double reduce_max_host(const double *d, int n, Pool &pool, hipStream_t s)
{
    int blocks = std::max(1, std::min((n + 255) / 256, 1024));
    double *part = pool.get<double>(blocks);
    k_max_partial<<<blocks, 256, 0, s>>>(d, n, part);
    CHM_HIP(hipGetLastError());
    std::vector<double> h(blocks);
    CHM_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * blocks, hipMemcpyDeviceToHost, s));
    CHM_HIP(hipStreamSynchronize(s));
    double m = -1.0e300;
    for (double v : h)
        m = std::max(m, v);
    return m;
}

void csr_to_sell(const Csr &A, Sell &S, Pool &pool, hipStream_t s, bool offsets16)
{
    S.n = A.n;
    S.nslices = (A.n + kSlice - 1) / kSlice;
    S.sptr = pool.get<int>(S.nslices + 1);
    if (S.nslices > 0) {
        k_slice_width<<<(S.nslices + 255) / 256, 256, 0, s>>>(A.rp, A.n, S.nslices, S.sptr);
        CHM_HIP(hipGetLastError());
    }
    scan_exclusive(S.sptr, S.nslices, S.sptr + S.nslices, pool, s);
    {
        std::vector<int> hp(S.nslices + 1);
        CHM_HIP(hipMemcpyAsync(hp.data(), S.sptr, sizeof(int) * hp.size(), hipMemcpyDeviceToHost,
                               s));
        CHM_HIP(hipStreamSynchronize(s));
        S.stored = hp[S.nslices];
        S.wmax = 0;
        for (int k = 0; k < S.nslices; ++k)
            S.wmax = std::max(S.wmax, (hp[k + 1] - hp[k]) / kSlice);
    }
    S.col = pool.get<int>(S.stored);
    S.val = pool.get<double>(S.stored);
    int rows = S.nslices * kSlice;
    if (rows > 0) {
        k_sell_fill<<<(rows + 255) / 256, 256, 0, s>>>(A.rp, A.ci, A.v, A.n, S.nslices, S.sptr,
                                                       S.col, S.val);
        CHM_HIP(hipGetLastError());
    }
    // every stored column (padding included) must index the input vector
    if (S.stored > 0) {
        int *bad = pool.get<int>(1);
        fill_int(bad, 0, 1, s);
        k_check_cols<<<(int)((S.stored + 255) / 256), 256, 0, s>>>(S.col, S.stored, A.m, bad);
        CHM_HIP(hipGetLastError());
        if (read_int(bad, s))
            throw Failure(CHM_EINVAL, "SELL conversion produced a column outside the matrix");
    }
    S.ocol = nullptr;
    if (offsets16 && A.n == A.m && S.stored > 0) {
        int16_t *oc = pool.get<int16_t>(S.stored);
        int *bad = pool.get<int>(1);
        fill_int(bad, 0, 1, s);
        k_sell_offsets<<<(rows + 255) / 256, 256, 0, s>>>(S.sptr, S.col, A.n, S.nslices, oc, bad);
        CHM_HIP(hipGetLastError());
        if (!read_int(bad, s))
            S.ocol = oc;
    }
}

// ---- value tables: the distinct values of an array (compared as bit
// patterns) in ascending bit order, and a 16-bit index per entry ----
constexpr unsigned long long kVtEmpty = 0x7FF8DEADBEEF0001ull;   // a NaN no kernel writes
constexpr int kVtSlots = 16384;                                  // hash slots (power of two)

__device__ inline unsigned vt_hash(unsigned long long k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    return (unsigned)k;
}

// every value's bit pattern into an open-addressing set; a pattern equal to
// the empty marker or a full probe sequence sets *bad
__global__ void __launch_bounds__(256) k_vt_insert(const double *__restrict__ v, int64_t n,
                                                   unsigned long long *slots, int *bad)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (__hip_atomic_load(bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;   // too many values for a table: stop early
        const unsigned long long key = (unsigned long long)__double_as_longlong(v[i]);
        if (key == kVtEmpty) {
            *bad = 1;
            return;
        }
        unsigned h = vt_hash(key) & (kVtSlots - 1);
        int probe = 0;
        for (; probe < 64; ++probe, h = (h + 1) & (kVtSlots - 1)) {
            // read past the L1 cache, which other CUs' inserts do not update
            const unsigned long long cur =
                __hip_atomic_load(slots + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur == key)
                break;
            if (cur == kVtEmpty) {
                const unsigned long long prev = atomicCAS(slots + h, kVtEmpty, key);
                if (prev == kVtEmpty || prev == key)
                    break;
            }
        }
        if (probe == 64)
            *bad = 1;
    }
}

// the occupied slots, packed (in no particular order) and counted
__global__ void __launch_bounds__(256) k_vt_pack(const unsigned long long *slots,
                                                 unsigned long long *keys, int *count)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kVtSlots || slots[i] == kVtEmpty)
        return;
    keys[atomicAdd(count, 1)] = slots[i];
}

// sorted table: key k goes to its rank among the (distinct) keys
__global__ void __launch_bounds__(256) k_vt_rank(const unsigned long long *__restrict__ keys,
                                                 int m, unsigned long long *tab)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m)
        return;
    const unsigned long long k = keys[i];
    int r = 0;
    for (int j = 0; j < m; ++j)
        r += keys[j] < k;
    tab[r] = k;
}

// each entry's position in the sorted table (binary search on bit patterns)
__global__ void __launch_bounds__(256) k_vt_index(const double *__restrict__ v, int64_t n,
                                                  const unsigned long long *__restrict__ tab,
                                                  int m, uint16_t *ix)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const unsigned long long key = (unsigned long long)__double_as_longlong(v[i]);
        int lo = 0, hi = m - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (tab[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        ix[i] = (uint16_t)lo;
    }
}

__global__ void __launch_bounds__(256) k_vt_fill(unsigned long long *p, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        p[i] = kVtEmpty;
}

ValueTable value_table(const double *v, int64_t n, Pool &pool, hipStream_t s)
{
    ValueTable t;
    if (n <= 0)
        return t;
    Pool tmp;
    unsigned long long *slots = tmp.get<unsigned long long>(kVtSlots);
    unsigned long long *keys = tmp.get<unsigned long long>(kVtSlots);
    int *flags = tmp.get<int>(2);
    k_vt_fill<<<kVtSlots / 256, 256, 0, s>>>(slots, kVtSlots);
    fill_int(flags, 0, 2, s);
    const int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
    k_vt_insert<<<grid, 256, 0, s>>>(v, n, slots, flags);
    k_vt_pack<<<kVtSlots / 256, 256, 0, s>>>(slots, keys, flags + 1);
    CHM_HIP(hipGetLastError());
    int hf[2];
    CHM_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    CHM_HIP(hipStreamSynchronize(s));
    const int m = hf[1];
    if (hf[0] || m <= 0 || m > kVtMax)
        return t;   // no table: the kernels read the values themselves
    unsigned long long *tab = pool.get<unsigned long long>(m);
    k_vt_rank<<<(m + 255) / 256, 256, 0, s>>>(keys, m, tab);
    t.ix = pool.get<uint16_t>(n);
    k_vt_index<<<grid, 256, 0, s>>>(v, n, tab, m, t.ix);
    CHM_HIP(hipGetLastError());
    t.tab = reinterpret_cast<double *>(tab);
    t.m = m;
    CHM_HIP(hipStreamSynchronize(s));   // the scratch pool is freed on return
    return t;
}

void sell_values(const Csr &A, const Sell &S, const double *csr_vals, double *sell_vals,
                 hipStream_t s)
{
    int rows = S.nslices * kSlice;
    if (rows > 0) {
        k_sell_fill<<<(rows + 255) / 256, 256, 0, s>>>(A.rp, A.ci, csr_vals, A.n, S.nslices,
                                                       S.sptr, nullptr, sell_vals);
        CHM_HIP(hipGetLastError());
    }
}

}  // namespace chm
