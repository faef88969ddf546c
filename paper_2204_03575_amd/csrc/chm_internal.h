// Internal declarations of the MI355X Cahn-Hilliard library.
//
// Vector layouts on the device:
//   * "pair" vectors: double2[n], .x = species 0 (polymer), .y = species 1
//     (acceptor).  Every multigrid kernel works on pairs, so each matrix entry
//     is read once for both species.
//   * block vectors (Krylov space of the saddle-point system): double2[2n],
//     entries [0, n) hold the volume-fraction block, [n, 2n) the
//     chemical-potential block.
//
// Sparse matrices are kept in CSR for setup and in SELL-64 for the solve:
// slice s holds rows [64 s, 64 s + 64); entry k of the row in lane l sits at
// sptr[s] + 64 k + l; rows shorter than the slice width are padded with
// (col = row, val = 0).  One wave64 handles one slice, so every col/val load
// of a wave is one contiguous 256-byte (col) or 512-byte (val) access.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/chm.h"
#include "../../include/chm_net.h"

namespace chm {

constexpr int kSlice = 64;      // SELL slice height = wavefront size
constexpr int kSellUnroll = 8;  // SELL rows up to this wide take the fully unrolled path
constexpr int kBlock = 256;     // threads per block for row kernels
constexpr int kMaxLevels = 24;
constexpr int kMaxRestart = 64;
constexpr int kMaxRuns = 64;      // runs of one batched solver
constexpr int kRedBlocks = 256;   // blocks of the two-stage reductions (one per CU)
constexpr int kGsBlocks = 1024;   // blocks of the Gram-Schmidt passes (four per CU)

struct Err {
    int code = CHM_OK;
    std::string msg;
};

#define CHM_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::chm::Failure(CHM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Failure {
    int code;
    std::string msg;
    Failure(int c, std::string m) : code(c), msg(std::move(m)) {}
};

// device memory owned by one solver
class Pool {
  public:
    ~Pool() { release(); }
    template <class T> T *get(size_t count) {
        if (count == 0)
            count = 1;
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess)
            throw Failure(CHM_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
        ptrs_.push_back(p);
        return static_cast<T *>(p);
    }
    void release() {
        for (void *p : ptrs_)
            (void)hipFree(p);
        ptrs_.clear();
    }
    size_t count() const { return ptrs_.size(); }

  private:
    std::vector<void *> ptrs_;
};

struct Csr {       // device CSR
    int n = 0, m = 0, nnz = 0;
    int *rp = nullptr, *ci = nullptr;
    double *v = nullptr;
};

// A value table of a matrix (see value_table): tab[ix[e]] is entry e's value.
constexpr int kVtMax = 2048;   // two FP64 tables fit 32 KB of LDS
struct ValueTable {
    uint16_t *ix = nullptr;
    double *tab = nullptr;
    float *ftab = nullptr;   // the table in FP32, for the FP32 preconditioner
    int m = 0;
};

struct Sell {      // device SELL-64
    int n = 0, nslices = 0;
    int64_t stored = 0;   // padded entry count
    int wmax = 0;         // entries in the widest slice
    int *sptr = nullptr;  // nslices + 1 offsets
    int *col = nullptr;
    double *val = nullptr;
    // col - row as 16 bits, for a square matrix whose offsets all fit (the
    // solve kernels then read these instead of col); else null
    int16_t *ocol = nullptr;
};

// One matrix of a level as the solve kernels see it, in value type T: the
// SELL-64 layout (sptr, col, sval) and the CSR layout (rp, ci, cval) share the
// pattern; gs = lanes per row (0: SELL-64 with one lane per row, 4..32: CSR
// with that many lanes per row, for long or few rows); u = entries a CSR lane
// loads per pass (1, 2 or 4: about the row length over gs).
template <class T> struct MatView {
    int n = 0, m = 0, nnz = 0, gs = 0, u = 1;   // rows, columns, nonzeros, lanes per row, unroll
    const int *sptr = nullptr, *col = nullptr, *rp = nullptr, *ci = nullptr;
    const int16_t *ocol = nullptr;              // SELL column offsets (see Sell), or null
    const T *sval = nullptr, *cval = nullptr;
    // the SELL values through a value table (vtab[vix[e]]), or null
    const uint16_t *vix = nullptr;
    const T *vtab = nullptr;
    int vm = 0;   // table entries
};

struct Level {
    int n = 0, nc = 0;
    int degree = 2;      // smoother degree (Chebyshev) or sweeps (Jacobi) on this level
    Csr A, P, R;
    Sell sA, sP, sR;
    ValueTable vtA;   // sA's values as a table, where it has few distinct values
    int gsA = 0, gsP = 0, gsR = 0;   // lanes per row (see MatView)
    int uA = 1, uP = 1, uR = 1;      // CSR entries per lane and pass (see MatView)
    // the residual and its restriction in one product: row i of RR is row i
    // of R (columns j < n, applied to b) followed by row i of -R A (columns
    // n + j, applied to x), so RR [b; x] = R (b - A x); CSR, rows of the next
    // level (empty on the coarsest level and where its rows would be long)
    Csr RR;
    int gsRR = 0, uRR = 1;
    // the prolongation and the first post-smoothing step in one launch: row
    // i of AM is row i of A (columns j < n, applied to x) followed by row i of
    // A P (columns n + k, applied to the coarse correction e), so AM [x; e] =
    // A (x + P e); CSR levels only, empty where its rows would be long
    Csr AM;
    int gsAM = 0, uAM = 1;
    double *dinv = nullptr;
    double rho = 0.0;
    int *agg = nullptr;
    // Chebyshev coefficients: step 1 uses c2[1] (c1 = 0); step k uses c1[k], c2[k]
    double cheb_c1[32], cheb_c2[32];
    double jac_omega = 0.0;
    // coarsest level: dense inverse (FP64 in both precisions), row-major n x n
    double *inv = nullptr;
    // FP32 copies of the values for the mixed-precision preconditioner
    float *fA_s = nullptr, *fA_c = nullptr, *fP_s = nullptr, *fP_c = nullptr;
    float *fR_s = nullptr, *fR_c = nullptr, *fdinv = nullptr, *fRR_c = nullptr;
    float *fAM_c = nullptr;

    template <class T> MatView<T> viewA() const;
    template <class T> MatView<T> viewP() const;
    template <class T> MatView<T> viewR() const;
    template <class T> MatView<T> viewRR() const;
    template <class T> MatView<T> viewAM() const;
    template <class T> const T *dinv_t() const;
};

// The FP32 kernels read a value table only on patterns with slices wider
// than kSellUnroll entries (3D): a 4-byte value against a 2-byte index saves
// too little to pay for the lookup on the 8-wide 2D rows (measured).
inline bool fp32_table(const Sell &S) { return S.wmax > kSellUnroll; }

template <class T>
inline MatView<T> make_view(const Csr &C, const Sell &S, int gs, int u, const T *sv, const T *cv)
{
    MatView<T> v;
    v.u = u;
    v.n = C.n;
    v.m = C.m;
    v.nnz = C.nnz;
    v.gs = gs;
    v.sptr = S.sptr;
    v.col = S.col;
    v.ocol = S.ocol;
    v.rp = C.rp;
    v.ci = C.ci;
    v.sval = sv;
    v.cval = cv;
    return v;
}
template <> inline MatView<double> Level::viewA<double>() const
{
    MatView<double> v = make_view<double>(A, sA, gsA, uA, sA.val, A.v);
    v.vix = vtA.ix;
    v.vtab = vtA.tab;
    v.vm = vtA.m;
    return v;
}
template <> inline MatView<double> Level::viewP<double>() const { return make_view<double>(P, sP, gsP, uP, sP.val, P.v); }
template <> inline MatView<double> Level::viewR<double>() const { return make_view<double>(R, sR, gsR, uR, sR.val, R.v); }
template <> inline MatView<float> Level::viewA<float>() const
{
    MatView<float> v = make_view<float>(A, sA, gsA, uA, fA_s, fA_c);
    if (fp32_table(sA)) {
        v.vix = vtA.ix;
        v.vtab = vtA.ftab;
        v.vm = vtA.m;
    }
    return v;
}
template <> inline MatView<float> Level::viewP<float>() const { return make_view<float>(P, sP, gsP, uP, fP_s, fP_c); }
template <> inline MatView<float> Level::viewR<float>() const { return make_view<float>(R, sR, gsR, uR, fR_s, fR_c); }
template <> inline MatView<double> Level::viewRR<double>() const { return make_view<double>(RR, Sell(), gsRR, uRR, nullptr, RR.v); }
template <> inline MatView<float> Level::viewRR<float>() const { return make_view<float>(RR, Sell(), gsRR, uRR, nullptr, fRR_c); }
template <> inline MatView<double> Level::viewAM<double>() const { return make_view<double>(AM, Sell(), gsAM, uAM, nullptr, AM.v); }
template <> inline MatView<float> Level::viewAM<float>() const { return make_view<float>(AM, Sell(), gsAM, uAM, nullptr, fAM_c); }
template <> inline const double *Level::dinv_t<double>() const { return dinv; }
template <> inline const float *Level::dinv_t<float>() const { return fdinv; }

struct Hierarchy {
    int nlev = 0;
    int degree = 2;          // smoother degree of the finest level
    int degree_coarse = 0;   // of the levels below it (0: degree)
    double ratio = 30.0;
    bool jacobi = false;
    Level lev[kMaxLevels];
    // per-level work vectors (pairs), FP64 and FP32
    double2 *x[kMaxLevels], *xt[kMaxLevels], *b[kMaxLevels], *r[kMaxLevels];
    float2 *fx[kMaxLevels], *fxt[kMaxLevels], *fb[kMaxLevels], *fr[kMaxLevels];
};

template <class T> struct Work;   // per-precision work vectors of the preconditioner
template <> struct Work<double> {
    double2 *pcg_r = nullptr, *pcg_z = nullptr, *pcg_d = nullptr, *pcg_q = nullptr;
    double2 *tmp = nullptr, *tmp2 = nullptr, *mr = nullptr, *me = nullptr;
    double2 *h1 = nullptr, *h2 = nullptr;     // block-vector halves of a batch
};
template <> struct Work<float> {
    float2 *pcg_r = nullptr, *pcg_z = nullptr, *pcg_d = nullptr, *pcg_q = nullptr;
    float2 *tmp = nullptr, *tmp2 = nullptr, *mr = nullptr, *me = nullptr;
    float2 *h1 = nullptr, *h2 = nullptr;
    float2 *vin = nullptr, *wout = nullptr;   // block vectors at the FP64 boundary
};

// device-side FGMRES control block (one per solver).  The small fields come
// first: the host reads only that prefix after each Arnoldi step.
struct Ctl {
    alignas(16) double nrm[2];   // last computed squared norms (||b||^2, true residual^2)
    alignas(16) double tol[2];
    alignas(16) double bnorm[2]; // ||b|| per species
    alignas(16) double resest[2];
    alignas(16) double hn[2];    // ||w|| of the last Arnoldi step before rotation
    int active[2];       // species still iterating in this cycle
    int k[2];            // Arnoldi steps of the species in this cycle
    int clamped;         // log-argument clamps in the last right-hand side
    int nan;             // a non-finite value was seen
    int guess_used[2];   // CHM_GUESS_* of the start the step used
    int outside;         // vertices of the new state with a fraction outside [0, 1]
    int pad_[3];
    // large part
    double H[2][(kMaxRestart + 1) * kMaxRestart];
    double cs[2][kMaxRestart], sn[2][kMaxRestart];
    double g[2][kMaxRestart + 1];
    double y[2][kMaxRestart];
    // delayed reorthogonalisation: the last Hessenberg column before the
    // rotations (its last two entries change when the next iteration makes
    // the newest basis vector final) and the cycle's initial residual norm
    double hlast[2][kMaxRestart + 1];
    double beta[2];
};
constexpr size_t kCtlHead = offsetof(Ctl, H);
static_assert(kCtlHead % 16 == 0, "control-block heads are packed back to back");

struct Timer {
    bool on = false;
    int kind = -1;                 // which kernel to time
    std::vector<hipEvent_t> ev;    // pairs
    size_t used = 0;
    double total_ms = 0.0;
    int64_t count = 0;
    int64_t bytes = 0;             // algorithmic bytes of the timed launches
};

// what differs between the runs of a batch: the interaction parameters of
// the free energy and the solvent removal
struct RunPrm {
    double chi_pn = 1.0, chi_ps = 0.3, chi_ns = 0.3;
    double evap_ds = 0.0;
    int evap_steps = 0;
};

// boundary facets of eq. chternary:2 (boundary.hip)
struct Boundary {
    int nf = 0, D = 0, nq = 0;       // facets, vertices per facet, quadrature points
    int *fv = nullptr;               // [nf][D] vertices
    int *ftype = nullptr;            // 1 top, 2 bottom
    double *fmeas = nullptr;         // length or area
    double2 *fpat = nullptr;         // [nf][nq] patterning weights (p_p, p_n)
    double *qb = nullptr, *qw = nullptr;   // facet rule: [nq][D] barycentric, [nq]
    int *inc_ptr = nullptr, *inc = nullptr;   // vertex -> facet slots f D + a, ascending
    double2 *slot = nullptr;         // [runs][nf D] per-slot values of a step
};

struct Solver {
    Err err;
    hipStream_t stream = nullptr;
    chm_params_t prm{};
    // Runs of the batch: nb runs share the mesh, the matrices and both AMG
    // hierarchies; every per-run vector holds the runs back to back.  nrun is
    // how many runs a launch covers (gridDim.y): nb for time steps, 1 for the
    // inspection calls, which work on run 0.
    int nb = 1, nrun = 1;
    int rb = 2;                // batches: runs per lane of the SELL and coarsest-level kernels
    std::vector<RunPrm> runs;
    void *pots = nullptr;      // device: per-run potential parameters
    int dim = 0, nv = 0, ncell = 0, nl = 0;
    Pool pool;

    // mesh
    double *coords = nullptr;
    int *cells = nullptr;
    double *vol = nullptr;
    int ncolors = 0;
    std::vector<int> color_ptr;   // host copy of colour offsets
    int *color_cells = nullptr;
    // per vertex, the slots cell * nl + corner of its cells in colour order,
    // SELL-64 (slice offsets vslot_ptr, vslot_stored entries with padding);
    // vslot_pos: the position of each slot in that layout
    int *vslot_ptr = nullptr, *vslot = nullptr, *vslot_pos = nullptr;
    int vslot_stored = 0;
    // quadrature (barycentric points, weights summing to 1)
    int nq = 0;
    double *qb = nullptr, *qw = nullptr;

    // matrices (shared pattern)
    Csr M, K, As;       // As values share M's pattern
    Sell sM;            // SELL of the pattern with M values
    double *sK = nullptr, *sAs = nullptr;  // SELL values of K and As on sM's layout
    ValueTable vtM, vtK;   // sM's and sK's values as tables, where they have few distinct values
    double tau_s[2], te_s[2];

    Hierarchy hM, hA;
    Boundary bc;

    // state and Krylov workspace
    int m = 30;
    double2 *x = nullptr;      // current state as a block vector: (phi, mu)
    double2 *xk = nullptr;     // FGMRES iterate (committed to x on success)
    double2 *b = nullptr, *r = nullptr;
    double2 *V = nullptr, *Z = nullptr;   // [Krylov index][run][2n]
    float2 *Z32 = nullptr;     // Z in FP32 (FP32 preconditioner: its results are FP32)
    double2 *xl = nullptr;     // linear-extrapolation candidate
    double2 *f = nullptr;      // potential term of the right-hand side (pairs)
    double2 *fslot = nullptr;  // its quadrature per cell and corner, before the gather
    Work<double> w64;
    Work<float> w32;
    float *fsM = nullptr;      // FP32 SELL values of M (Algorithm 1's product with M)
    bool mixed = false;        // FP32 preconditioner (precision = 1)
    double2 *red = nullptr;    // slots of per-block partial sums (kRedBlocks each)
    double2 *gsp1 = nullptr, *gsp2 = nullptr, *gsp3 = nullptr;  // Gram-Schmidt partials
    double2 *hfin = nullptr;   // finalised Gram-Schmidt coefficients of both passes
    Ctl *ctl = nullptr;        // device, one per run
    Ctl *hctl = nullptr;       // pinned host mirror (heads), one per run
    int *dheads = nullptr;     // device address of hctl (the heads are written there)
    std::vector<int64_t> steps;   // per run: completed time steps (the solvent removal counts them)
    double setup_ms = 0.0;
    double vc_rho = 0.0;       // measured V-cycle contraction of the As hierarchy (0: not measured)
    Timer timer;
    std::string nan_where;     // where the last CHM_ENAN was detected
    // HIP graphs of the FGMRES iteration body, one per Arnoldi index j,
    // captured on a library-owned stream and launched on `stream`
    hipStream_t cap_stream = nullptr;
    std::vector<hipGraphExec_t> iter_graphs;
    // initial guess of each Krylov solve (CHM_GUESS_*)
    int guess_mode = 0;
    chm_net *net = nullptr;
    int gH = 0, gW = 0;
    // the last two solutions of the Krylov solve (before solvent removal):
    // yh1 = y_{n-1}, yh2 = y_{n-2}; after chm_set_fields yh1 is the new state
    double2 *yh1 = nullptr, *yh2 = nullptr;
    std::vector<int> hist;     // per run: how many of yh1, yh2 are valid
    // MINRES (krylov = CHM_KRYLOV_MINRES): six block vectors per run (r1, r2,
    // y, v, w1, w2) and the per-run recurrence scalars, with a pinned mirror
    double2 *mr = nullptr;
    void *mrctl = nullptr, *hmrctl = nullptr;
    // stationary AMG solves to amg_tol: per run, which species go on (device
    // and pinned host mirror)
    int2 *amg_act = nullptr, *hamg_act = nullptr;
    double *stage = nullptr;   // one field, for host-side set/get of fields
};

// ---- util.hip
void scan_exclusive(int *d_in_out, int n, int *d_total, Pool &pool, hipStream_t s);
void fill_int(int *p, int v, size_t n, hipStream_t s);
void fill_double(double *p, double v, size_t n, hipStream_t s);
int read_int(const int *d, hipStream_t s);
double reduce_max_host(const double *d, int n, Pool &pool, hipStream_t s);
// offsets16: also store the 16-bit column offsets (Sell::ocol) when A is
// square and every offset fits
void csr_to_sell(const Csr &A, Sell &S, Pool &pool, hipStream_t s, bool offsets16);
void sell_values(const Csr &A, const Sell &S, const double *csr_vals, double *sell_vals, hipStream_t s);
// The distinct values of v[0..n) (as bit patterns, at most kVtMax of them) in
// ascending bit order, and each entry's 16-bit position among them; m = 0
// (no table) when there are more.
ValueTable value_table(const double *v, int64_t n, Pool &pool, hipStream_t s);

// ---- mesh_setup.hip
void build_quadrature(int dim, std::vector<double> &bary, std::vector<double> &w);
void mesh_setup(Solver &S);

// ---- amg_setup.hip
void amg_build(Solver &S, Hierarchy &H, const Csr &A0);

// ---- prec.hip (preconditioner; FP64 vectors at the interface, the
// configured precision inside)
void prec_setup(Solver &S);   // FP32 copies and work vectors (mixed precision)
void vcycle(Solver &S, int hier, const double2 *b, double2 *x);
void schur_solve(Solver &S, const double2 *b, double2 *x);
void apply_prec(Solver &S, const double2 *v, double2 *w);
// the FP32 preconditioner with an FP32 result; narrowed: S.w32.vin already
// holds v in FP32
void apply_prec32(Solver &S, const double2 *v, float2 *w, bool narrowed);
// As-norm contraction of one FP64 V-cycle of the As hierarchy (power iteration)
double vcycle_contraction(Solver &S, int iters);

// ---- boundary.hip
void boundary_setup(Solver &S);
// b1 += tau G for every run's state, or G of run 0 into g when g != nullptr
void boundary_rhs(Solver &S, double2 *g);

// ---- net.hip
long long net_max_pixels(const chm_net *net);
// the network's guess (device state vectors, solver layout) on stream st
void net_guess_on(chm_net *net, hipStream_t st, int H, int W, const double *x2, const double *x1,
                  double *out);

// ---- solve.hip
void alloc_workspace(Solver &S);
void apply_saddle(Solver &S, const double2 *x, double2 *y);
void compute_rhs(Solver &S);
int step_once(Solver &S, chm_stats_t *st);
void timer_mark(Solver &S, bool begin);

// ---- minres.hip
void minres_alloc(Solver &S);
// MINRES from S.xk for right-hand side S.b given S.r = b - A xk (every run);
// adds each species' iterations to total (2 per run)
int minres_solve(Solver &S, std::vector<int> &total);

}  // namespace chm
