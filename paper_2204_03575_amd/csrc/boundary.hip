// Boundary terms of eq. chternary:2 (Section 2; coefficients of Section 4),
// explicit in time.  The top facets (all vertices at the largest second
// coordinate) take the solvent evaporation as an inflow k phi_i phi_s of
// polymer and acceptor; the bottom facets (smallest second coordinate) the
// substrate flux p_i(x) (g_i + 2 h_i phi_i), with p_p = 1 on the first,
// third and fifth sixth of the bottom and p_n = 1 on the others (or both 1
// without patterning).  The first block row of the right-hand side gains
// tau G, G_j = integral over those facets of the flux times lambda_j.
//
// Setup finds the facets on the device, stores their vertices, measures and
// the patterning weights at the facet quadrature points, and builds the
// vertex -> facet-slot lists (ascending).  Per step, one thread per facet
// integrates its fluxes into per-slot partial values, and one thread per
// vertex adds its slots in list order: no floating-point atomics.
#include <cmath>

#include "device_util.h"

namespace chm {

namespace {

__global__ void k_coord(int n, int dim, int k, double sign, const double *__restrict__ xyz,
                        double *out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        out[i] = sign * xyz[(size_t)i * dim + k];
}

// flag[c * nl + omit]: 1 if the facet opposite local vertex `omit` lies on
// the top, 2 on the bottom, 0 otherwise
__global__ void k_facet_flags(int ncell, int nl, int dim, const int *__restrict__ cells,
                              const double *__restrict__ xyz, double ymin, double ymax,
                              double tol, int *flag)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= ncell * nl)
        return;
    const int c = t / nl, omit = t % nl;
    bool top = true, bot = true;
    for (int a = 0; a < nl; ++a) {
        if (a == omit)
            continue;
        const double y = xyz[(size_t)cells[(size_t)c * nl + a] * dim + 1];
        top = top && fabs(y - ymax) <= tol;
        bot = bot && fabs(y - ymin) <= tol;
    }
    flag[t] = top ? 1 : (bot ? 2 : 0);
}

__global__ void k_flag_count(int n, const int *__restrict__ flag, int *cnt)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < n)
        cnt[t] = flag[t] != 0;
}

// facet f = the facet with pos[t] = f: vertices (ascending local order),
// type, measure (edge length or triangle area) and the patterning weights
// at the quadrature points (x of the point from the facet's vertices)
__global__ void k_facet_fill(int ncell, int nl, int dim, const int *__restrict__ cells,
                             const double *__restrict__ xyz, const int *__restrict__ flag,
                             const int *__restrict__ pos, const double *__restrict__ qb, int nq,
                             int pattern, double xmin, double xmax, int *fv, int *ftype,
                             double *fmeas, double2 *fpat)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= ncell * nl || !flag[t])
        return;
    const int c = t / nl, omit = t % nl, D = nl - 1, f = pos[t];
    double p[3][3] = {};
    int k = 0;
    for (int a = 0; a < nl; ++a) {
        if (a == omit)
            continue;
        const int v = cells[(size_t)c * nl + a];
        fv[f * D + k] = v;
        for (int d = 0; d < dim; ++d)
            p[k][d] = xyz[(size_t)v * dim + d];
        ++k;
    }
    ftype[f] = flag[t];
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = p[1][d] - p[0][d];
        e2[d] = D == 3 ? p[2][d] - p[0][d] : 0.0;
    }
    if (D == 2) {
        fmeas[f] = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    } else {
        const double c0 = e1[1] * e2[2] - e1[2] * e2[1], c1 = e1[2] * e2[0] - e1[0] * e2[2],
                     c2 = e1[0] * e2[1] - e1[1] * e2[0];
        fmeas[f] = 0.5 * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    }
    for (int q = 0; q < nq; ++q) {
        double wp = 1.0, wn = 1.0;
        if (flag[t] == 2 && pattern) {
            double x = 0.0;
            for (int a = 0; a < D; ++a)
                x += qb[q * D + a] * p[a][0];
            int six = (int)floor(6.0 * (x - xmin) / (xmax - xmin));
            six = six < 0 ? 0 : (six > 5 ? 5 : six);
            wp = (six % 2 == 0) ? 1.0 : 0.0;
            wn = 1.0 - wp;
        }
        fpat[(size_t)f * nq + q] = make_double2(wp, wn);
    }
}

__global__ void k_slot_count(int nslots, const int *__restrict__ fv, int *cnt)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s < nslots)
        atomicAdd(&cnt[fv[s]], 1);
}

__global__ void k_slot_fill(int nslots, const int *__restrict__ fv, int *cursor, int *inc)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s < nslots)
        inc[atomicAdd(&cursor[fv[s]], 1)] = s;
}

__global__ void k_sort_lists(int n, const int *__restrict__ ptr, int *v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const int b = ptr[i], e = ptr[i + 1];
    for (int k = b + 1; k < e; ++k) {
        const int key = v[k];
        int j = k - 1;
        while (j >= b && v[j] > key) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = key;
    }
}

struct BcCoef {
    double k, g0, g1, h0, h1;
};

// per facet and run: the slot values meas * sum_q w_q g(x_q) lambda_a(x_q)
// for both species (the state's phi block: run r at x + r 2n)
template <int D>
__global__ void __launch_bounds__(kBlock) k_bc_facets(int nf, int n, const int *__restrict__ fv,
                                                      const int *__restrict__ ftype,
                                                      const double *__restrict__ fmeas,
                                                      const double2 *__restrict__ fpat,
                                                      const double *__restrict__ qb,
                                                      const double *__restrict__ qw, int nq,
                                                      const double2 *__restrict__ x, BcCoef C,
                                                      double2 *slot)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= nf)
        return;
    x = run_at(x, 2l * n);
    slot = run_at(slot, (long)nf * D);
    double2 ph[D], acc[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        ph[a] = x[fv[f * D + a]];
        acc[a] = make_double2(0.0, 0.0);
    }
    const bool top = ftype[f] == 1;
    for (int q = 0; q < nq; ++q) {
        double pp = 0.0, pn = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            pp += qb[q * D + a] * ph[a].x;
            pn += qb[q * D + a] * ph[a].y;
        }
        double gp, gn;
        if (top) {
            const double ps = 1.0 - pp - pn;
            gp = C.k * pp * ps;
            gn = C.k * pn * ps;
        } else {
            const double2 w = fpat[(size_t)f * nq + q];
            gp = w.x * (C.g0 + 2.0 * C.h0 * pp);
            gn = w.y * (C.g1 + 2.0 * C.h1 * pn);
        }
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double l = qb[q * D + a], wq = qw[q];
            acc[a].x += wq * gp * l;
            acc[a].y += wq * gn * l;
        }
    }
    const double m = fmeas[f];
#pragma unroll
    for (int a = 0; a < D; ++a)
        slot[f * D + a] = make_double2(m * acc[a].x, m * acc[a].y);
}

// G_v = sum of v's slots in list order; b[v] += tau G_v (or g[v] = G_v when
// g is given); per run: slots advance by nslots, b by 2n, g by n
__global__ void __launch_bounds__(kBlock) k_bc_gather(int n, int nslots, const int *__restrict__ ptr,
                                                      const int *__restrict__ inc,
                                                      const double2 *__restrict__ slot,
                                                      double tau, double2 *b, double2 *g)
{
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= n)
        return;
    slot = run_at(slot, (long)nslots);
    double2 s = make_double2(0.0, 0.0);
    for (int k = ptr[v]; k < ptr[v + 1]; ++k) {
        const double2 c = slot[inc[k]];
        s.x += c.x;
        s.y += c.y;
    }
    if (g) {
        run_at(g, (long)n)[v] = s;
        return;
    }
    if (ptr[v] == ptr[v + 1])
        return;
    b = run_at(b, 2l * n);
    const double2 o = b[v];
    b[v] = make_double2(o.x + tau * s.x, o.y + tau * s.y);
}

double extreme(Solver &S, int k, double sign, double *tmp)
{
    k_coord<<<nblk(S.nv), kBlock, 0, S.stream>>>(S.nv, S.dim, k, sign, S.coords, tmp);
    return sign * reduce_max_host(tmp, S.nv, S.pool, S.stream);
}

}  // namespace

void boundary_setup(Solver &S)
{
    Boundary &B = S.bc;
    if (!S.prm.boundary)
        return;
    hipStream_t st = S.stream;
    Pool &pool = S.pool;
    const int nl = S.nl, D = S.dim, ncell = S.ncell;
    double *tmp = pool.get<double>(S.nv);
    const double xmax = extreme(S, 0, 1.0, tmp), xmin = extreme(S, 0, -1.0, tmp);
    const double ymax = extreme(S, 1, 1.0, tmp), ymin = extreme(S, 1, -1.0, tmp);
    if (!(ymax > ymin) || !(xmax > xmin))
        throw Failure(CHM_EINVAL, "boundary terms need a mesh with extent in x and y");
    // facet rule: Gauss-Legendre on edges (2D), the degree-5 triangle rule (3D)
    std::vector<double> hb, hw;
    build_quadrature(D - 1, hb, hw);
    B.nq = (int)hw.size();
    B.D = D;
    B.qb = pool.get<double>(hb.size());
    B.qw = pool.get<double>(hw.size());
    CHM_HIP(hipMemcpyAsync(B.qb, hb.data(), sizeof(double) * hb.size(), hipMemcpyHostToDevice, st));
    CHM_HIP(hipMemcpyAsync(B.qw, hw.data(), sizeof(double) * hw.size(), hipMemcpyHostToDevice, st));
    const int nt = ncell * nl;
    int *flag = pool.get<int>(nt), *pos = pool.get<int>(nt + 1);
    k_facet_flags<<<nblk(nt), kBlock, 0, st>>>(ncell, nl, S.dim, S.cells, S.coords, ymin, ymax,
                                               1e-12 * (ymax - ymin), flag);
    k_flag_count<<<nblk(nt), kBlock, 0, st>>>(nt, flag, pos);
    scan_exclusive(pos, nt, pos + nt, pool, st);
    B.nf = read_int(pos + nt, st);
    if (B.nf == 0)
        return;
    B.fv = pool.get<int>((size_t)B.nf * D);
    B.ftype = pool.get<int>(B.nf);
    B.fmeas = pool.get<double>(B.nf);
    B.fpat = pool.get<double2>((size_t)B.nf * B.nq);
    k_facet_fill<<<nblk(nt), kBlock, 0, st>>>(ncell, nl, S.dim, S.cells, S.coords, flag, pos, B.qb,
                                              B.nq, S.prm.bc_pattern, xmin, xmax, B.fv, B.ftype,
                                              B.fmeas, B.fpat);
    const int ns = B.nf * D;
    B.inc_ptr = pool.get<int>(S.nv + 1);
    fill_int(B.inc_ptr, 0, S.nv + 1, st);
    k_slot_count<<<nblk(ns), kBlock, 0, st>>>(ns, B.fv, B.inc_ptr);
    scan_exclusive(B.inc_ptr, S.nv, B.inc_ptr + S.nv, pool, st);
    int *cursor = pool.get<int>(S.nv);
    CHM_HIP(hipMemcpyAsync(cursor, B.inc_ptr, sizeof(int) * S.nv, hipMemcpyDeviceToDevice, st));
    B.inc = pool.get<int>(ns);
    k_slot_fill<<<nblk(ns), kBlock, 0, st>>>(ns, B.fv, cursor, B.inc);
    k_sort_lists<<<nblk(S.nv), kBlock, 0, st>>>(S.nv, B.inc_ptr, B.inc);
    B.slot = pool.get<double2>((size_t)S.nb * ns);
    CHM_HIP(hipGetLastError());
    CHM_HIP(hipStreamSynchronize(st));
}

// b1 += tau G for the current state of every run (b1 = first half of S.b),
// or, with g, G of run 0 into the device pair vector g
void boundary_rhs(Solver &S, double2 *g)
{
    const Boundary &B = S.bc;
    if (!S.prm.boundary || B.nf == 0) {
        if (g)
            fill_double(reinterpret_cast<double *>(g), 0.0, 2 * (size_t)S.nv, S.stream);
        return;
    }
    hipStream_t st = S.stream;
    const int R = S.nrun, n = S.nv;
    const BcCoef C{S.prm.bc_k, S.prm.bc_g[0], S.prm.bc_g[1], S.prm.bc_h[0], S.prm.bc_h[1]};
    if (B.D == 2)
        k_bc_facets<2><<<grid(nblk(B.nf), R), kBlock, 0, st>>>(B.nf, n, B.fv, B.ftype, B.fmeas, B.fpat,
                                                               B.qb, B.qw, B.nq, S.x, C, B.slot);
    else
        k_bc_facets<3><<<grid(nblk(B.nf), R), kBlock, 0, st>>>(B.nf, n, B.fv, B.ftype, B.fmeas, B.fpat,
                                                               B.qb, B.qw, B.nq, S.x, C, B.slot);
    k_bc_gather<<<grid(nblk(n), R), kBlock, 0, st>>>(n, B.nf * B.D, B.inc_ptr, B.inc, B.slot,
                                                     S.prm.tau, S.b, g);
    CHM_HIP(hipGetLastError());
}

}  // namespace chm
