// Mesh setup on the GPU: vertex->cell incidence, the P1 sparsity pattern,
// a conflict-free colouring of the cells, and assembly of the P1 mass and
// stiffness matrices (paper Section 3, the matrices M and K of
// eq. chternary_space) by coloured scatter: cells of one colour share no
// vertex, so one thread per cell adds its element matrix into the global
// rows without atomics, and the summation order (colour by colour) is fixed.
#include <cmath>

#include "chm_internal.h"

namespace chm {

namespace {

constexpr int kMaxColors = 128;
constexpr int kMaxRowCand = 512;    // cap on (incident cells) x (vertices per cell)

__device__ inline uint64_t mix_hash(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_count_incidence(const int *cells, int ncell, int nl, int *deg)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell)
        return;
    for (int a = 0; a < nl; ++a)
        atomicAdd(&deg[cells[(size_t)c * nl + a]], 1);
}

__global__ void k_fill_incidence(const int *cells, int ncell, int nl, int *cursor, int *inc)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell)
        return;
    for (int a = 0; a < nl; ++a) {
        int pos = atomicAdd(&cursor[cells[(size_t)c * nl + a]], 1);
        inc[pos] = c;
    }
}

// sort each segment [ptr[i], ptr[i+1]) ascending (segments are short)
__global__ void k_sort_segments(int *v, const int *ptr, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int b = ptr[i], e = ptr[i + 1];
    for (int k = b + 1; k < e; ++k) {
        int key = v[k], j = k - 1;
        while (j >= b && v[j] > key) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = key;
    }
}

// pass 0: number of distinct vertices sharing a cell with vertex v (v included)
// pass 1: write them, ascending, at ci[rp[v]]
__global__ void k_pattern(const int *cells, int nl, const int *inc_ptr, const int *inc, int nv,
                          int pass, int *rowlen, const int *rp, int *ci, int *overflow)
{
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv)
        return;
    int buf[kMaxRowCand];
    int cnt = 0;
    for (int k = inc_ptr[v]; k < inc_ptr[v + 1]; ++k) {
        int c = inc[k];
        for (int a = 0; a < nl; ++a) {
            if (cnt >= kMaxRowCand) {
                atomicAdd(overflow, 1);
                return;
            }
            buf[cnt++] = cells[(size_t)c * nl + a];
        }
    }
    for (int k = 1; k < cnt; ++k) {
        int key = buf[k], j = k - 1;
        while (j >= 0 && buf[j] > key) {
            buf[j + 1] = buf[j];
            --j;
        }
        buf[j + 1] = key;
    }
    int u = 0;
    for (int k = 0; k < cnt; ++k) {
        if (u > 0 && buf[k] == buf[u - 1])
            continue;
        buf[u++] = buf[k];
    }
    if (pass == 0) {
        rowlen[v] = u;
    } else {
        int o = rp[v];
        for (int k = 0; k < u; ++k)
            ci[o + k] = buf[k];
    }
}

// one atomic per wave: lane 0 adds the number of lanes with pred set (every
// lane of the wave must reach the call)
__device__ inline void count_in_wave(int *counter, bool pred)
{
    const unsigned long long m = __ballot(pred);
    if ((threadIdx.x & 63) == 0 && m)
        atomicAdd(counter, __popcll(m));
}

// priority of a cell in the colouring (a fixed hash; ties broken by index)
__device__ inline uint64_t cell_prio(int c)
{
    return mix_hash(0x632BE59BD9B4E019ull + (uint64_t)c * 0x9E3779B97F4A7C15ull);
}
__device__ inline bool beats(int e, uint64_t he, int c, uint64_t hc)
{
    return he > hc || (he == hc && e > c);
}

// Speculative colouring of the cell conflict graph (cells conflict when they
// share a vertex), in synchronous rounds of two kernels.  Pick: every cell
// uncoloured at the start of the round tentatively takes the smallest colour
// absent among its coloured neighbours (col_in -> col_try).  Resolve: a
// tentative colour that a tentatively coloured neighbour of higher priority
// also took is dropped (col_in, col_try -> col_out); the others become final.
// The highest-priority uncoloured cell always keeps its colour, so every
// round colours at least one cell, and a final colour never repeats among
// neighbours.  Decisions depend on the previous round only.
__global__ void k_color_pick(const int *cells, int nl, int ncell, const int *inc_ptr,
                             const int *inc, const int *col_in, int *col_try, int *overflow)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell)
        return;
    const int mine = col_in[c];
    if (mine >= 0) {
        col_try[c] = mine;
        return;
    }
    uint64_t used0 = 0, used1 = 0;
    for (int a = 0; a < nl; ++a) {
        const int v = cells[(size_t)c * nl + a];
        for (int k = inc_ptr[v]; k < inc_ptr[v + 1]; ++k) {
            const int ce = col_in[inc[k]];
            if (ce >= 0 && ce < 64)
                used0 |= 1ull << ce;
            else if (ce >= 64)
                used1 |= 1ull << (ce - 64);
        }
    }
    int pick = -1;
    if (~used0)
        pick = __ffsll((unsigned long long)~used0) - 1;
    else if (~used1)
        pick = 64 + __ffsll((unsigned long long)~used1) - 1;
    if (pick < 0)
        atomicAdd(overflow, 1);
    col_try[c] = pick;
}

__global__ void k_color_resolve(const int *cells, int nl, int ncell, const int *inc_ptr,
                                const int *inc, const int *col_in, const int *col_try,
                                int *col_out, int *remaining, int *maxcolor)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    bool dropped = false;
    if (c < ncell) {
        const int t = col_try[c];
        if (col_in[c] >= 0 || t < 0) {
            col_out[c] = t;   // final before this round, or no colour left (overflow)
        } else {
            const uint64_t hc = cell_prio(c);
            for (int a = 0; a < nl && !dropped; ++a) {
                const int v = cells[(size_t)c * nl + a];
                for (int k = inc_ptr[v]; k < inc_ptr[v + 1]; ++k) {
                    const int e = inc[k];
                    if (e != c && col_in[e] < 0 && col_try[e] == t && beats(e, cell_prio(e), c, hc)) {
                        dropped = true;
                        break;
                    }
                }
            }
            col_out[c] = dropped ? -1 : t;
            if (!dropped)
                atomicMax(maxcolor, t);
        }
    }
    count_in_wave(remaining, dropped);
}

// cells that share a vertex with a cell of the same colour (must be none)
__global__ void k_color_check(const int *cells, int nl, int ncell, const int *inc_ptr,
                              const int *inc, const int *col, int *bad)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    bool clash = false;
    if (c < ncell) {
        const int mine = col[c];
        clash = mine < 0;
        for (int a = 0; a < nl && !clash; ++a) {
            const int v = cells[(size_t)c * nl + a];
            for (int k = inc_ptr[v]; k < inc_ptr[v + 1]; ++k) {
                const int e = inc[k];
                if (e != c && col[e] == mine) {
                    clash = true;
                    break;
                }
            }
        }
    }
    count_in_wave(bad, clash);
}

// cells per colour: a histogram per block in LDS, then one global atomic per
// block and colour (a global atomic per cell serialises on the few counters)
__global__ void k_color_count(const int *color, int ncell, int *cnt)
{
    __shared__ int h[kMaxColors];
    for (int t = threadIdx.x; t < kMaxColors; t += blockDim.x)
        h[t] = 0;
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell)
        atomicAdd(&h[color[c]], 1);
    __syncthreads();
    for (int t = threadIdx.x; t < kMaxColors; t += blockDim.x)
        if (h[t])
            atomicAdd(&cnt[t], h[t]);
}

// the cells of each colour listed from cursor[colour] on: each block takes
// one range per colour it holds (the order within a colour is free: its
// cells share no vertex, so the scatter's sums do not depend on it)
__global__ void k_color_fill(const int *color, int ncell, int *cursor, int *list)
{
    __shared__ int h[kMaxColors], base[kMaxColors];
    for (int t = threadIdx.x; t < kMaxColors; t += blockDim.x)
        h[t] = 0;
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    int col = -1, pos = 0;
    if (c < ncell) {
        col = color[c];
        pos = atomicAdd(&h[col], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kMaxColors; t += blockDim.x)
        if (h[t])
            base[t] = atomicAdd(&cursor[t], h[t]);
    __syncthreads();
    if (c < ncell)
        list[base[col] + pos] = c;
}

// 64 times the largest number of cells at a vertex of each 64-vertex slice
__global__ void k_slot_width(const int *__restrict__ inc_ptr, int nv, int *w)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (nv + kSlice - 1) / kSlice)
        return;
    int m = 0;
    for (int v = s * kSlice; v < nv && v < (s + 1) * kSlice; ++v)
        m = max(m, inc_ptr[v + 1] - inc_ptr[v]);
    w[s] = m * kSlice;
}

// slot cell * nl + a appended to the list of vertex v = cells[cell * nl + a]
// for the cells of one colour (no two share a vertex: one writer per
// cursor).  The lists are SELL-64: entry k of vertex v at sptr[v / 64] +
// 64 k + v % 64; pos records where each slot went.
__global__ void k_slot_fill(const int *__restrict__ list, int count, const int *__restrict__ cells,
                            int nl, const int *__restrict__ sptr, int *cursor, int *slot, int *pos)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count)
        return;
    const int c = list[t];
    for (int a = 0; a < nl; ++a) {
        const int v = cells[(size_t)c * nl + a];
        const int p = sptr[v / kSlice] + cursor[v]++ * kSlice + v % kSlice;
        slot[p] = c * nl + a;
        pos[(size_t)c * nl + a] = p;
    }
}

// element geometry: gradients of the barycentric coordinates and the volume
__device__ inline bool element_geometry(int dim, const double *coords, const int *vtx,
                                        double g[4][3], double *vol)
{
    double J[3][3];
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c)
            J[r][c] = coords[(size_t)vtx[c + 1] * dim + r] - coords[(size_t)vtx[0] * dim + r];
    double det, Ji[3][3];
    if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        if (det == 0.0)
            return false;
        double id = 1.0 / det;
        Ji[0][0] = J[1][1] * id;
        Ji[0][1] = -J[0][1] * id;
        Ji[1][0] = -J[1][0] * id;
        Ji[1][1] = J[0][0] * id;
        *vol = fabs(det) * 0.5;
    } else {
        // rows of J^-1 are the cross products of the columns of J, divided by det
        double c0[3] = {J[0][0], J[1][0], J[2][0]};
        double c1[3] = {J[0][1], J[1][1], J[2][1]};
        double c2[3] = {J[0][2], J[1][2], J[2][2]};
        double x12[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2],
                         c1[0] * c2[1] - c1[1] * c2[0]};
        double x20[3] = {c2[1] * c0[2] - c2[2] * c0[1], c2[2] * c0[0] - c2[0] * c0[2],
                         c2[0] * c0[1] - c2[1] * c0[0]};
        double x01[3] = {c0[1] * c1[2] - c0[2] * c1[1], c0[2] * c1[0] - c0[0] * c1[2],
                         c0[0] * c1[1] - c0[1] * c1[0]};
        det = c0[0] * x12[0] + c0[1] * x12[1] + c0[2] * x12[2];
        if (det == 0.0)
            return false;
        double id = 1.0 / det;
        for (int k = 0; k < 3; ++k) {
            Ji[0][k] = x12[k] * id;
            Ji[1][k] = x20[k] * id;
            Ji[2][k] = x01[k] * id;
        }
        *vol = fabs(det) / 6.0;
    }
    for (int k = 0; k < dim; ++k) {
        g[0][k] = 0.0;
        for (int a = 1; a <= dim; ++a) {
            g[a][k] = Ji[a - 1][k];
            g[0][k] -= Ji[a - 1][k];
        }
    }
    return true;
}

__device__ inline int find_in_row(const int *ci, int b, int e, int col)
{
    while (b < e) {
        int mid = (b + e) >> 1;
        int c = ci[mid];
        if (c == col)
            return mid;
        if (c < col)
            b = mid + 1;
        else
            e = mid;
    }
    return -1;
}

// coloured scatter of M_T = |T| (1 + delta_ab) / ((d+1)(d+2)) and
// K_T = |T| grad(lambda_a) . grad(lambda_b) for the cells of one colour
__global__ void k_assemble_color(const int *list, int count, const int *cells, int dim,
                                 const double *coords, const int *rp, const int *ci, double *Mv,
                                 double *Kv, double *vol_out, int *bad)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count)
        return;
    int c = list[t];
    int nl = dim + 1;
    int vtx[4];
    for (int a = 0; a < nl; ++a)
        vtx[a] = cells[(size_t)c * nl + a];
    double g[4][3], vol;
    if (!element_geometry(dim, coords, vtx, g, &vol)) {
        atomicAdd(bad, 1);
        return;
    }
    vol_out[c] = vol;
    double mdiag = vol * 2.0 / ((dim + 1) * (dim + 2));
    double moff = vol / ((dim + 1) * (dim + 2));
    for (int a = 0; a < nl; ++a) {
        int b0 = rp[vtx[a]], b1 = rp[vtx[a] + 1];
        for (int b = 0; b < nl; ++b) {
            double dotg = 0.0;
            for (int k = 0; k < dim; ++k)
                dotg += g[a][k] * g[b][k];
            int pos = find_in_row(ci, b0, b1, vtx[b]);
            if (pos < 0) {   // cannot happen for a pattern built from these cells
                atomicAdd(bad, 1);
                continue;
            }
            Mv[pos] += (a == b) ? mdiag : moff;
            Kv[pos] += vol * dotg;
        }
    }
}

__global__ void k_combine(const double *K, const double *M, double a, double b, double *out, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = a * K[i] + b * M[i];
}

inline int blocks_for(long n, int bs = kBlock) { return (int)std::max<long>(1, (n + bs - 1) / bs); }

// eigen-decomposition of a small symmetric matrix by cyclic Jacobi rotations
void sym_eig(int n, double *A, double *Q)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            Q[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j)
                off += A[i * n + j] * A[i * n + j];
        if (off < 1e-40)
            break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0)
                    continue;
                double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {   // A <- A R
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // A <- R^T A
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double qkp = Q[k * n + p], qkq = Q[k * n + q];
                    Q[k * n + p] = c * qkp - s * qkq;
                    Q[k * n + q] = s * qkp + c * qkq;
                }
            }
    }
}

// Gauss-Jacobi rule with 3 nodes for the weight (1-t)^alpha on [-1,1], by the
// Golub-Welsch method: nodes are the eigenvalues of the Jacobi matrix of the
// orthogonal polynomials, weights are mu0 times the squared first components
// of the normalised eigenvectors, mu0 = 2^(alpha+1)/(alpha+1).
void gauss_jacobi_gw(double alpha, double *t, double *w)
{
    const int n = 3;
    double J[9] = {0}, Q[9];
    for (int k = 0; k < n; ++k) {
        double s = 2.0 * k + alpha;
        J[k * n + k] = -alpha * alpha / (s * (s + 2.0));
        if (k == 0)
            J[0] = -alpha / (alpha + 2.0);
        if (k + 1 < n) {
            double m = k + 1.0, sm = 2.0 * m + alpha;
            double bm = 4.0 * m * (m + alpha) * m * (m + alpha) / (sm * sm * (sm + 1.0) * (sm - 1.0));
            J[k * n + k + 1] = J[(k + 1) * n + k] = std::sqrt(bm);
        }
    }
    sym_eig(n, J, Q);
    double mu0 = std::pow(2.0, alpha + 1.0) / (alpha + 1.0);
    for (int k = 0; k < n; ++k) {
        t[k] = J[k * n + k];
        w[k] = mu0 * Q[0 * n + k] * Q[0 * n + k];
    }
}

}  // namespace

// Collapsed-coordinate product rule on the d-simplex with three Gauss-Jacobi
// points per direction (exact to degree 5): direction k carries the weight
// (1-u)^(d-1-k) of the Duffy map x1 = u1, x2 = u2 (1-u1), x3 = u3 (1-u1)(1-u2).
void build_quadrature(int dim, std::vector<double> &bary, std::vector<double> &w)
{
    double u[3][3], wu[3][3];
    for (int k = 0; k < dim; ++k) {
        double t[3], wt[3], alpha = dim - 1 - k;
        gauss_jacobi_gw(alpha, t, wt);
        for (int q = 0; q < 3; ++q) {
            u[k][q] = 0.5 * (t[q] + 1.0);
            wu[k][q] = wt[q] * std::pow(0.5, alpha + 1.0);
        }
    }
    bary.clear();
    w.clear();
    if (dim == 1) {   // edges: Gauss-Legendre (weight (1-u)^0), weights summing to 1
        for (int a = 0; a < 3; ++a) {
            bary.insert(bary.end(), {1.0 - u[0][a], u[0][a]});
            w.push_back(wu[0][a]);
        }
        return;
    }
    double fact = (dim == 2) ? 2.0 : 6.0;   // 1 / volume of the reference simplex
    int n3 = (dim == 2) ? 1 : 3;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < n3; ++c) {
                double x1 = u[0][a];
                double x2 = u[1][b] * (1.0 - u[0][a]);
                double ww = wu[0][a] * wu[1][b] * fact;
                if (dim == 2) {
                    bary.insert(bary.end(), {1.0 - x1 - x2, x1, x2});
                } else {
                    double x3 = u[2][c] * (1.0 - u[1][b]) * (1.0 - u[0][a]);
                    ww *= wu[2][c];
                    bary.insert(bary.end(), {1.0 - x1 - x2 - x3, x1, x2, x3});
                }
                w.push_back(ww);
            }
}

void mesh_setup(Solver &S)
{
    hipStream_t st = S.stream;
    Pool &pool = S.pool;
    const int nv = S.nv, ncell = S.ncell, nl = S.nl;
    int *flags = pool.get<int>(4);   // overflow, remaining, maxcolor, bad
    fill_int(flags, 0, 4, st);

    // vertex -> cell incidence, each list ascending
    int *inc_ptr = pool.get<int>(nv + 1);
    fill_int(inc_ptr, 0, nv + 1, st);
    k_count_incidence<<<blocks_for(ncell), kBlock, 0, st>>>(S.cells, ncell, nl, inc_ptr);
    scan_exclusive(inc_ptr, nv, inc_ptr + nv, pool, st);
    int *cursor = pool.get<int>(nv);
    CHM_HIP(hipMemcpyAsync(cursor, inc_ptr, sizeof(int) * nv, hipMemcpyDeviceToDevice, st));
    int *inc = pool.get<int>((size_t)ncell * nl);
    k_fill_incidence<<<blocks_for(ncell), kBlock, 0, st>>>(S.cells, ncell, nl, cursor, inc);
    k_sort_segments<<<blocks_for(nv), kBlock, 0, st>>>(inc, inc_ptr, nv);
    CHM_HIP(hipGetLastError());

    // P1 pattern: vertices sharing a cell, columns ascending
    int *rp = pool.get<int>(nv + 1);
    k_pattern<<<blocks_for(nv), kBlock, 0, st>>>(S.cells, nl, inc_ptr, inc, nv, 0, rp, nullptr,
                                                 nullptr, flags);
    CHM_HIP(hipGetLastError());
    if (read_int(flags, st))
        throw Failure(CHM_EINVAL, "a vertex lies in too many cells for the pattern builder");
    scan_exclusive(rp, nv, rp + nv, pool, st);
    int nnz = read_int(rp + nv, st);
    int *ci = pool.get<int>(nnz);
    k_pattern<<<blocks_for(nv), kBlock, 0, st>>>(S.cells, nl, inc_ptr, inc, nv, 1, nullptr, rp, ci,
                                                 flags);
    CHM_HIP(hipGetLastError());

    // speculative colouring of the cells; a cell is uncoloured after a round
    // only if a neighbour of higher priority took its tentative colour
    int *colA = pool.get<int>(ncell), *colB = pool.get<int>(ncell), *colT = pool.get<int>(ncell);
    fill_int(colA, -1, ncell, st);
    for (int round = 0;; ++round) {
        fill_int(flags + 1, 0, 1, st);
        k_color_pick<<<blocks_for(ncell), kBlock, 0, st>>>(S.cells, nl, ncell, inc_ptr, inc, colA,
                                                           colT, flags);
        k_color_resolve<<<blocks_for(ncell), kBlock, 0, st>>>(S.cells, nl, ncell, inc_ptr, inc,
                                                              colA, colT, colB, flags + 1,
                                                              flags + 2);
        CHM_HIP(hipGetLastError());
        std::swap(colA, colB);
        if (read_int(flags, st))
            throw Failure(CHM_EINVAL, "cell colouring needs more than 128 colours");
        if (read_int(flags + 1, st) == 0)
            break;
        if (round > ncell)
            throw Failure(CHM_EINVAL, "cell colouring did not terminate");
    }
    fill_int(flags + 1, 0, 1, st);
    k_color_check<<<blocks_for(ncell), kBlock, 0, st>>>(S.cells, nl, ncell, inc_ptr, inc, colA,
                                                        flags + 1);
    CHM_HIP(hipGetLastError());
    if (read_int(flags + 1, st))
        throw Failure(CHM_EINVAL, "cell colouring left two cells that share a vertex in one colour");
    S.ncolors = read_int(flags + 2, st) + 1;
    int *ccount = pool.get<int>(kMaxColors + 1);
    fill_int(ccount, 0, kMaxColors + 1, st);
    k_color_count<<<blocks_for(ncell), kBlock, 0, st>>>(colA, ncell, ccount);
    CHM_HIP(hipGetLastError());
    std::vector<int> hc(kMaxColors);
    CHM_HIP(hipMemcpyAsync(hc.data(), ccount, sizeof(int) * kMaxColors, hipMemcpyDeviceToHost, st));
    CHM_HIP(hipStreamSynchronize(st));
    S.color_ptr.assign(S.ncolors + 1, 0);
    for (int c = 0; c < S.ncolors; ++c)
        S.color_ptr[c + 1] = S.color_ptr[c] + hc[c];
    CHM_HIP(hipMemcpyAsync(ccount, S.color_ptr.data(), sizeof(int) * S.ncolors,
                           hipMemcpyHostToDevice, st));
    S.color_cells = pool.get<int>(ncell);
    k_color_fill<<<blocks_for(ncell), kBlock, 0, st>>>(colA, ncell, ccount, S.color_cells);
    CHM_HIP(hipGetLastError());

    // slots cell * nl + corner of every vertex, listed colour by colour (a
    // colour holds at most one cell at a vertex, so each vertex's cursor has
    // one writer per launch), in a SELL-64 layout padded with slot 0
    const int nsl = (nv + kSlice - 1) / kSlice;
    S.vslot_ptr = pool.get<int>(nsl + 1);
    k_slot_width<<<blocks_for(nsl), kBlock, 0, st>>>(inc_ptr, nv, S.vslot_ptr);
    CHM_HIP(hipGetLastError());
    {
        std::vector<int> w(nsl);
        CHM_HIP(hipMemcpyAsync(w.data(), S.vslot_ptr, sizeof(int) * nsl, hipMemcpyDeviceToHost, st));
        CHM_HIP(hipStreamSynchronize(st));
        long total = 0;
        for (int x : w)
            total += x;
        if (total > 0x7fffffffl)
            throw Failure(CHM_EINVAL, "mesh too large for the right-hand side's slot lists");
    }
    scan_exclusive(S.vslot_ptr, nsl, S.vslot_ptr + nsl, pool, st);
    S.vslot_stored = read_int(S.vslot_ptr + nsl, st);
    S.vslot = pool.get<int>(S.vslot_stored);
    fill_int(S.vslot, 0, S.vslot_stored, st);
    S.vslot_pos = pool.get<int>((size_t)ncell * nl);
    fill_int(cursor, 0, nv, st);
    for (int c = 0; c < S.ncolors; ++c) {
        const int cnt = S.color_ptr[c + 1] - S.color_ptr[c];
        if (cnt == 0)
            continue;
        k_slot_fill<<<blocks_for(cnt), kBlock, 0, st>>>(S.color_cells + S.color_ptr[c], cnt, S.cells,
                                                        nl, S.vslot_ptr, cursor, S.vslot,
                                                        S.vslot_pos);
        CHM_HIP(hipGetLastError());
    }

    // assembly by coloured scatter
    Csr &M = S.M;
    M.n = M.m = nv;
    M.nnz = nnz;
    M.rp = rp;
    M.ci = ci;
    M.v = pool.get<double>(nnz);
    S.K = M;
    S.K.v = pool.get<double>(nnz);
    S.As = M;
    S.As.v = pool.get<double>(nnz);
    fill_double(M.v, 0.0, nnz, st);
    fill_double(S.K.v, 0.0, nnz, st);
    S.vol = pool.get<double>(ncell);
    for (int c = 0; c < S.ncolors; ++c) {
        int cnt = S.color_ptr[c + 1] - S.color_ptr[c];
        if (cnt == 0)
            continue;
        k_assemble_color<<<blocks_for(cnt), kBlock, 0, st>>>(
            S.color_cells + S.color_ptr[c], cnt, S.cells, S.dim, S.coords, rp, ci, M.v, S.K.v,
            S.vol, flags + 3);
        CHM_HIP(hipGetLastError());
    }
    if (read_int(flags + 3, st))
        throw Failure(CHM_EINVAL, "mesh has a cell of zero volume");

    // As = tau' K + sqrt(tau'/eps) M (the operator of Algorithm 1)
    double t = S.tau_s[0], sq = std::sqrt(S.tau_s[0] / S.prm.eps[0]);
    k_combine<<<blocks_for(nnz), kBlock, 0, st>>>(S.K.v, M.v, t, sq, S.As.v, nnz);
    CHM_HIP(hipGetLastError());

    // SELL-64 copies for the solve (one pattern, three value arrays)
    csr_to_sell(M, S.sM, pool, st, S.prm.wide_index == 0);
    S.sK = pool.get<double>(S.sM.stored);
    S.sAs = pool.get<double>(S.sM.stored);
    sell_values(M, S.sM, S.K.v, S.sK, st);
    sell_values(M, S.sM, S.As.v, S.sAs, st);
    if (S.sM.ocol && !S.prm.values_direct) {   // value tables go with the 16-bit column offsets
        S.vtM = value_table(S.sM.val, S.sM.stored, pool, st);
        S.vtK = value_table(S.sK, S.sM.stored, pool, st);
    }

    // quadrature
    std::vector<double> qb, qw;
    build_quadrature(S.dim, qb, qw);
    S.nq = (int)qw.size();
    S.qb = pool.get<double>(qb.size());
    S.qw = pool.get<double>(qw.size());
    CHM_HIP(hipMemcpyAsync(S.qb, qb.data(), sizeof(double) * qb.size(), hipMemcpyHostToDevice, st));
    CHM_HIP(hipMemcpyAsync(S.qw, qw.data(), sizeof(double) * qw.size(), hipMemcpyHostToDevice, st));
    CHM_HIP(hipStreamSynchronize(st));
}

}  // namespace chm
