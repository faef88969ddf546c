// Learned initial guess (include/chm_net.h): per-frame feature statistics,
// feature packing, the four-layer BF16 convolution network on MFMA (forward,
// backward to the input, backward to the weights), the masked loss, Adam, and
// the guess x1 + d + sigma * y.
//
// Tensors are NHWC: pixel p = (b * H + row) * W + col, channels innermost, so
// the 4 consecutive channels one MFMA lane supplies are one 8-byte load.  The
// MFMA is v_mfma_f32_16x16x16_bf16: a wave multiplies a 16 x 16 A tile (rows:
// pixels or channels, k: 16 reduction entries) by a 16 x 16 B tile; lane l
// supplies row l % 16 of A and column l % 16 of B for k = 4 (l / 16) .. + 3,
// and receives D[4 (l / 16) + j][l % 16], j = 0..3.
//
// Every reduction (weight and bias gradients, loss, frame statistics) has a
// fixed grid and a fixed summation order: results are bitwise reproducible.
#include <cmath>
#include <cstring>
#include <mutex>

#include "device_util.h"

using bf16_t = uint16_t;

namespace chm {
namespace {

constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {8, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 4};
constexpr int kRadius = kLayers;      // receptive radius of four 3x3 layers
constexpr int kChunk = 1024;          // pixels per block of the weight-gradient kernels
constexpr int kMaxBatch = 256;
constexpr int kPtrBatch = 64;         // samples per pointer-upload launch
constexpr double kBeta1 = 0.9, kBeta2 = 0.999, kAdamEps = 1e-8;
constexpr int kStat = 13;             // per-sample statistics: sigma[4], mean[4], tau[4], q
constexpr double kWeightFloor = 1e-4; // sample weight 1 / (q + floor)

constexpr int w_count(int k) { return 9 * kCin[k] * kCout[k]; }
constexpr int w_offset(int k) { return k == 0 ? 0 : w_offset(k - 1) + w_count(k - 1) + kCout[k - 1]; }
constexpr int b_offset(int k) { return w_offset(k) + w_count(k); }
static_assert(b_offset(kLayers - 1) + kCout[kLayers - 1] == CHM_NET_NPARAMS, "parameter count");

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// round to nearest even (finite values; overflow gives infinity)
__device__ inline bf16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ inline float from_bf16(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

// mirror index for i in [-1, n]: -1 -> 1, n -> n - 2 (n >= 2)
__device__ inline int refl(int i, int n) { return i < 0 ? -i : (i >= n ? 2 * (n - 1) - i : i); }

__device__ inline v4f mfma16(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// state vector index of field c at vertex v (n vertices): the solver's block
// layout, phi pairs then mu pairs
__device__ inline long sidx(int c, long v, long n) { return (c >> 1) * 2 * n + 2 * v + (c & 1); }

// ------------------------------------------------------------------ parameters
// BF16 copies of one layer's weights in the two layouts the kernels read:
// forward [9][co16][ci] (k = input channel contiguous), backward
// [9][ci][co16] (k = output channel contiguous); co16 pads the output
// channels to a multiple of 16 with zeros.
__global__ void k_wconv(int ci, int co, int co16, const float *__restrict__ w, bf16_t *wf,
                        bf16_t *wb)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= 9 * ci * co16)
        return;
    const int o = i % co16, c = (i / co16) % ci, tap = i / (co16 * ci);
    const bf16_t v = o < co ? to_bf16(w[(tap * ci + c) * co + o]) : (bf16_t)0;
    wf[((size_t)tap * co16 + o) * ci + c] = v;
    wb[((size_t)tap * ci + c) * co16 + o] = v;
}

__global__ void k_adam(int n, float *p, const float *__restrict__ g, float *m, float *v, float lr,
                       float b1, float b2, float eps, float c1, float c2)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float m1 = b1 * m[i] + (1.0f - b1) * gi;
    const float v1 = b2 * v[i] + (1.0f - b2) * (gi * gi);
    const float step = lr * (m1 / c1) / (sqrtf(v1 / c2) + eps);
    m[i] = m1;
    v[i] = v1;
    p[i] = p[i] - step;
}

// ------------------------------------------------------------------ convolutions
// out[p][o] = bias[o] + sum over taps and c of in[refl(p + tap)][c] * w[tap][c][o];
// hidden layers store BF16(ReLU(out)), the last layer FP32 out.  Each wave
// takes 64 consecutive pixels (four 16-row M tiles) and all output channels.
template <int CI, int CO, bool RELU>
__global__ void __launch_bounds__(kBlock) k_conv_fwd(int B, int H, int W,
                                                     const bf16_t *__restrict__ in,
                                                     const bf16_t *__restrict__ wf,
                                                     const float *__restrict__ bias,
                                                     bf16_t *__restrict__ act_out,
                                                     float *__restrict__ y_out)
{
    constexpr int NB = (CO + 15) / 16, KC = (CI + 15) / 16, CO16 = NB * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const long npx = (long)B * H * W;
    const long base = ((long)blockIdx.x * 4 + wave) * 64;
    if (base >= npx)
        return;   // the whole wave
    int pb[4], py[4], pxx[4];
    for (int mt = 0; mt < 4; ++mt) {
        long p = base + mt * 16 + r;
        if (p >= npx)
            p = npx - 1;   // a valid pixel; its result is not stored
        pxx[mt] = (int)(p % W);
        const long t = p / W;
        py[mt] = (int)(t % H);
        pb[mt] = (int)(t / H);
    }
    v4f acc[4][NB];
    for (int mt = 0; mt < 4; ++mt)
        for (int nb = 0; nb < NB; ++nb)
            acc[mt][nb] = v4f{0.f, 0.f, 0.f, 0.f};
    const v4s zero = {0, 0, 0, 0};
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        long q[4];
        for (int mt = 0; mt < 4; ++mt)
            q[mt] = ((long)pb[mt] * H + refl(py[mt] + dy, H)) * W + refl(pxx[mt] + dx, W);
        for (int kc = 0; kc < KC; ++kc) {
            const int k0 = kc * 16 + kq * 4;
            const bool kin = k0 < CI;   // lanes past the input channels supply zeros
            v4s bfr[NB];
            for (int nb = 0; nb < NB; ++nb)
                bfr[nb] = kin ? *reinterpret_cast<const v4s *>(wf + ((size_t)tap * CO16 + nb * 16 + r) * CI + k0)
                              : zero;
            for (int mt = 0; mt < 4; ++mt) {
                const v4s a = kin ? *reinterpret_cast<const v4s *>(in + q[mt] * CI + k0) : zero;
                for (int nb = 0; nb < NB; ++nb)
                    acc[mt][nb] = mfma16(a, bfr[nb], acc[mt][nb]);
            }
        }
    }
    for (int mt = 0; mt < 4; ++mt)
        for (int nb = 0; nb < NB; ++nb) {
            const int o = nb * 16 + r;
            if (o >= CO)
                continue;
            const float bo = bias[o];
            for (int j = 0; j < 4; ++j) {
                const long p = base + mt * 16 + kq * 4 + j;
                if (p >= npx)
                    continue;
                const float v = acc[mt][nb][j] + bo;
                if (RELU)
                    act_out[p * CO + o] = to_bf16(fmaxf(v, 0.0f));
                else
                    y_out[p * CO + o] = v;
            }
        }
}

// Output pixels p with refl(p + off) = q along one axis, for tap offset off
// in {-1, 0, 1}: the direct one q - off (when inside) and, on the mirrored
// lines, the border pixel whose reflected neighbour is q (-1 when absent).
__device__ inline void preimages(int q, int off, int n, int &c0, int &c1)
{
    c0 = q - off;
    if (c0 < 0 || c0 >= n)
        c0 = -1;
    c1 = (q == 1 && off == -1) ? 0 : ((q == n - 2 && off == 1) ? n - 1 : -1);
}

// g_in[q][c] = mask(a_in[q][c] > 0) * sum over taps, o and the output pixels
// p with refl(p + tap) = q of g_out[p][o] * w[tap][c][o], rounded to BF16.
// Each lane row is an input pixel q; the mirrored border lines have a second
// preimage per axis, handled by up to three extra MFMA passes that run only
// when some lane of the wave needs them.
template <int CI, int CO>
__global__ void __launch_bounds__(kBlock) k_conv_bwd_data(int B, int H, int W,
                                                          const bf16_t *__restrict__ gout,
                                                          const bf16_t *__restrict__ wb,
                                                          const bf16_t *__restrict__ ain,
                                                          bf16_t *__restrict__ gin)
{
    static_assert(CI % 16 == 0, "input channels");
    constexpr int NB = CI / 16, KC = (CO + 15) / 16, CO16 = KC * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const long npx = (long)B * H * W;
    const long base = ((long)blockIdx.x * 4 + wave) * 64;
    if (base >= npx)
        return;
    int pb[4], py[4], pxx[4];
    for (int mt = 0; mt < 4; ++mt) {
        long p = base + mt * 16 + r;
        if (p >= npx)
            p = npx - 1;
        pxx[mt] = (int)(p % W);
        const long t = p / W;
        py[mt] = (int)(t % H);
        pb[mt] = (int)(t / H);
    }
    v4f acc[4][NB];
    for (int mt = 0; mt < 4; ++mt)
        for (int nb = 0; nb < NB; ++nb)
            acc[mt][nb] = v4f{0.f, 0.f, 0.f, 0.f};
    const v4s zero = {0, 0, 0, 0};
    for (int tap = 0; tap < 9; ++tap) {
        const int oy = tap / 3 - 1, ox = tap % 3 - 1;
        int cy[4][2], cx[4][2];
        for (int mt = 0; mt < 4; ++mt) {
            preimages(py[mt], oy, H, cy[mt][0], cy[mt][1]);
            preimages(pxx[mt], ox, W, cx[mt][0], cx[mt][1]);
        }
        v4s bfr[KC][NB];
        for (int kc = 0; kc < KC; ++kc)
            for (int nb = 0; nb < NB; ++nb)
                bfr[kc][nb] = *reinterpret_cast<const v4s *>(
                    wb + ((size_t)tap * CI + nb * 16 + r) * CO16 + kc * 16 + kq * 4);
        for (int pass = 0; pass < 4; ++pass) {
            const int sy = pass & 1, sx = pass >> 1;
            bool any = pass == 0;
            if (pass > 0) {
                bool mine = false;
                for (int mt = 0; mt < 4; ++mt)
                    mine = mine || (cy[mt][sy] >= 0 && cx[mt][sx] >= 0);
                any = __ballot(mine) != 0;
            }
            if (!any)
                continue;   // wave-uniform
            for (int kc = 0; kc < KC; ++kc) {
                const int k0 = kc * 16 + kq * 4;
                for (int mt = 0; mt < 4; ++mt) {
                    const int yy = cy[mt][sy], xx = cx[mt][sx];
                    v4s a = zero;
                    if (yy >= 0 && xx >= 0 && k0 < CO)
                        a = *reinterpret_cast<const v4s *>(
                            gout + (((long)pb[mt] * H + yy) * W + xx) * CO + k0);
                    for (int nb = 0; nb < NB; ++nb)
                        acc[mt][nb] = mfma16(a, bfr[kc][nb], acc[mt][nb]);
                }
            }
        }
    }
    for (int mt = 0; mt < 4; ++mt)
        for (int nb = 0; nb < NB; ++nb) {
            const int c = nb * 16 + r;
            for (int j = 0; j < 4; ++j) {
                const long p = base + mt * 16 + kq * 4 + j;
                if (p >= npx)
                    continue;
                const bool on = from_bf16(ain[p * CI + c]) > 0.0f;
                gin[p * CI + c] = to_bf16(on ? acc[mt][nb][j] : 0.0f);
            }
        }
}

// Partial weight gradients of one tap over one chunk of kChunk pixels:
// part[chunk][tap][c][o] = sum over p in the chunk of a_in[refl(p + tap)][c] g_out[p][o].
// A rows are input channels, B columns output channels, k runs over pixels;
// the four waves take every fourth group of 16 pixels and their tiles are
// added in LDS in wave order.
template <int CI, int CO>
__global__ void __launch_bounds__(kBlock) k_conv_bwd_w(int B, int H, int W,
                                                       const bf16_t *__restrict__ ain,
                                                       const bf16_t *__restrict__ gout,
                                                       float *__restrict__ part)
{
    constexpr int MI = (CI + 15) / 16, NB = (CO + 15) / 16;
    __shared__ float red[4][MI * 16][NB * 16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int tap = blockIdx.y, oy = tap / 3 - 1, ox = tap % 3 - 1;
    const long npx = (long)B * H * W;
    const long c0 = (long)blockIdx.x * kChunk;
    v4f acc[MI][NB];
    for (int mi = 0; mi < MI; ++mi)
        for (int nb = 0; nb < NB; ++nb)
            acc[mi][nb] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int g = wave; g < kChunk / 16; g += 4) {
        const long p0 = c0 + g * 16 + kq * 4;
        if (c0 + g * 16 >= npx)
            break;   // wave-uniform: the rest of the chunk is past the end
        long qn[4];
        bool ok[4];
        for (int j = 0; j < 4; ++j) {
            const long p = p0 + j;
            ok[j] = p < npx;
            qn[j] = 0;
            if (ok[j]) {
                const int x = (int)(p % W);
                const long t = p / W;
                const int y = (int)(t % H), b = (int)(t / H);
                qn[j] = ((long)b * H + refl(y + oy, H)) * W + refl(x + ox, W);
            }
        }
        v4s bfr[NB];
        for (int nb = 0; nb < NB; ++nb) {
            const int o = nb * 16 + r;
            for (int j = 0; j < 4; ++j)
                bfr[nb][j] = (ok[j] && o < CO) ? (short)gout[(p0 + j) * CO + o] : (short)0;
        }
        for (int mi = 0; mi < MI; ++mi) {
            const int c = mi * 16 + r;
            v4s a;
            for (int j = 0; j < 4; ++j)
                a[j] = (ok[j] && c < CI) ? (short)ain[qn[j] * CI + c] : (short)0;
            for (int nb = 0; nb < NB; ++nb)
                acc[mi][nb] = mfma16(a, bfr[nb], acc[mi][nb]);
        }
    }
    for (int mi = 0; mi < MI; ++mi)
        for (int nb = 0; nb < NB; ++nb)
            for (int j = 0; j < 4; ++j)
                red[wave][mi * 16 + kq * 4 + j][nb * 16 + r] = acc[mi][nb][j];
    __syncthreads();
    float *out = part + ((size_t)blockIdx.x * 9 + tap) * CI * CO;
    for (int e = threadIdx.x; e < CI * CO; e += kBlock) {
        const int c = e / CO, o = e % CO;
        out[e] = ((red[0][c][o] + red[1][c][o]) + red[2][c][o]) + red[3][c][o];
    }
}

// per-chunk partial bias gradients: bpart[chunk][o] = sum over the chunk of g_out[p][o]
template <int CO>
__global__ void __launch_bounds__(kBlock) k_bias_part(long npx, const bf16_t *__restrict__ gout,
                                                      float *__restrict__ bpart)
{
    static_assert(kBlock % CO == 0, "output channels");
    __shared__ float sh[kBlock];
    const int o = threadIdx.x % CO, lane_p = threadIdx.x / CO;
    const long c0 = (long)blockIdx.x * kChunk;
    const long end = c0 + kChunk < npx ? c0 + kChunk : npx;
    float s = 0.f;
    for (long p = c0 + lane_p; p < end; p += kBlock / CO)
        s += from_bf16(gout[p * CO + o]);
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < CO) {
        float t = 0.f;
        for (int i = 0; i < kBlock / CO; ++i)
            t += sh[i * CO + threadIdx.x];
        bpart[(size_t)blockIdx.x * CO + threadIdx.x] = t;
    }
}

// gradients of one layer from the chunk partials, summed in chunk order
__global__ void k_grad_reduce(int nchunks, int nw, int co, const float *__restrict__ wpart,
                              const float *__restrict__ bpart, float *gw, float *gb)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e < nw) {
        float s = 0.f;
        for (int c = 0; c < nchunks; ++c)
            s += wpart[(size_t)c * nw + e];
        gw[e] = s;
    } else if (e < nw + co) {
        const int o = e - nw;
        float s = 0.f;
        for (int c = 0; c < nchunks; ++c)
            s += bpart[(size_t)c * co + o];
        gb[o] = s;
    }
}

// ------------------------------------------------------------------ loss
// L = (1/S) sum over samples of w_s / (4 m_s) times the sum over the 4
// channels of [sum over masked pixels of e^2 + smooth * sum over the
// horizontal and vertical neighbour pairs with both pixels masked of
// (e_p - e_q)^2], e = y - t (samples are ch x cw crops, m_s their masked
// pixels).  dL/dy_p = w_s (2 e_p + 2 smooth sum over masked neighbours q of
// (e_p - e_q)) / (4 m_s S), rounded to BF16; per-block partial sums of the
// loss terms (FP64, each pair counted at its left or upper pixel) in part.
__global__ void __launch_bounds__(kBlock) k_loss(long n4, int ch, int cw, int S,
                                                 const float *__restrict__ y,
                                                 const float *__restrict__ t,
                                                 const uint8_t *__restrict__ mask,
                                                 const double *__restrict__ wts,
                                                 const int *__restrict__ msum, double smooth,
                                                 bf16_t *__restrict__ gy, double *part)
{
    __shared__ double2 sh[kBlock / 64];
    const long chs = (long)ch * cw;
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n4; i += (long)gridDim.x * kBlock) {
        float g = 0.0f;
        const long p = i >> 2;
        if (mask[p]) {
            const int s = (int)(p / chs), c = (int)(i & 3);
            const long loc = p % chs;
            const int r = (int)(loc / cw), col = (int)(loc % cw);
            const double w = wts[s], denom = 4.0 * (double)msum[s] * (double)S;
            const double e = (double)y[i] - (double)t[i];
            double term = e * e, gsum = e;
            if (smooth != 0.0) {
                const long nb[4] = {col + 1 < cw ? p + 1 : -1, col > 0 ? p - 1 : -1,
                                    r + 1 < ch ? p + cw : -1, r > 0 ? p - cw : -1};
                for (int k = 0; k < 4; ++k) {
                    const long q = nb[k];
                    if (q < 0 || !mask[q])
                        continue;
                    const double eq = (double)y[q * 4 + c] - (double)t[q * 4 + c];
                    gsum += smooth * (e - eq);
                    if (k == 0 || k == 2)
                        term += smooth * (eq - e) * (eq - e);
                }
            }
            acc += w * term / denom;
            g = (float)(w * (2.0 * gsum) / denom);
        }
        gy[i] = to_bf16(g);
    }
    const double2 s = block_sum(d2(acc, 0.0), sh);
    if (threadIdx.x == 0)
        part[blockIdx.x] = s.x;
}

// sample weights 1 / (q_s + floor) from the statistics
__global__ void k_weights(int S, const double *__restrict__ stats, double *wts)
{
    const int s = threadIdx.x;
    if (s < S)
        wts[s] = 1.0 / (stats[s * kStat + 12] + kWeightFloor);
}

// ------------------------------------------------------------------ features and guess
struct BatchPtrs {
    const double *x2[kPtrBatch], *x1[kPtrBatch], *x0[kPtrBatch];
    int oy[kPtrBatch], ox[kPtrBatch], msum[kPtrBatch];
};

// copy count samples' pointers, crop origins and masked pixel counts into the
// device tables at base
__global__ void k_set_batch(BatchPtrs b, int base, int count, int cap, const double **ptrs,
                            int *crop, int *msum)
{
    const int i = threadIdx.x;
    if (i >= count)
        return;
    ptrs[base + i] = b.x2[i];
    ptrs[cap + base + i] = b.x1[i];
    ptrs[2 * cap + base + i] = b.x0[i];
    crop[base + i] = b.oy[i];
    crop[cap + base + i] = b.ox[i];
    msum[base + i] = b.msum[i];
}

// per sample: sigma_c = RMS of x1 - x2, mean_c of x1, tau_c = RMS of x1 - mean_c
// (stats[s][0..3], [4..7], [8..11]) and, with x0, q = mean over channels of
// the mean square of the target t_c = (x0 - x1 - (x1 - x2)) / sigma_c
// (stats[s][12]; 0 without x0); one block per sample
__global__ void __launch_bounds__(kBlock) k_stats(long n, const double *const *x2s,
                                                  const double *const *x1s,
                                                  const double *const *x0s, double *stats)
{
    __shared__ double2 sh[kBlock / 64];
    __shared__ double res[kStat];
    const double *x2 = x2s[blockIdx.x], *x1 = x1s[blockIdx.x];
    const double *x0 = x0s ? x0s[blockIdx.x] : nullptr;
    double sd[4] = {0.0, 0.0, 0.0, 0.0}, sm[4] = {0.0, 0.0, 0.0, 0.0};
    for (long v = threadIdx.x; v < n; v += kBlock)
        for (int c = 0; c < 4; ++c) {
            const double a = x1[sidx(c, v, n)], d = a - x2[sidx(c, v, n)];
            sd[c] += d * d;
            sm[c] += a;
        }
    for (int c = 0; c < 4; ++c) {
        const double2 s = block_sum(d2(sd[c], sm[c]), sh);
        if (threadIdx.x == 0) {
            res[c] = sqrt(s.x / (double)n);
            res[4 + c] = s.y / (double)n;
        }
    }
    __syncthreads();
    double st[4] = {0.0, 0.0, 0.0, 0.0}, sq[4] = {0.0, 0.0, 0.0, 0.0};
    double is[4];
    for (int c = 0; c < 4; ++c)
        is[c] = res[c] > 0.0 ? 1.0 / res[c] : 0.0;
    for (long v = threadIdx.x; v < n; v += kBlock)
        for (int c = 0; c < 4; ++c) {
            const long k = sidx(c, v, n);
            const double a = x1[k];
            const double e = a - res[4 + c];
            st[c] += e * e;
            if (x0) {
                const double t = (x0[k] - a - (a - x2[k])) * is[c];
                sq[c] += t * t;
            }
        }
    double qsum = 0.0;   // thread 0
    for (int c = 0; c < 4; c += 2) {
        const double2 s = block_sum(d2(st[c], st[c + 1]), sh);
        const double2 q = block_sum(d2(sq[c], sq[c + 1]), sh);
        if (threadIdx.x == 0) {
            res[8 + c] = sqrt(s.x / (double)n);
            res[9 + c] = sqrt(s.y / (double)n);
            qsum += q.x / (double)n + q.y / (double)n;
        }
    }
    if (threadIdx.x == 0)
        res[12] = 0.25 * qsum;
    __syncthreads();
    if (threadIdx.x < kStat)
        stats[blockIdx.x * kStat + threadIdx.x] = res[threadIdx.x];
}

__device__ inline double inv_or_zero(double s) { return s > 0.0 ? 1.0 / s : 0.0; }

// features (BF16) of the crop pixels of every sample, and optionally the
// training targets and the loss mask
__global__ void __launch_bounds__(kBlock) k_pack(int S, int H, int W, int ch, int cw, int cap,
                                                 const double *const *ptrs, const int *crop,
                                                 const double *__restrict__ stats, bf16_t *feat,
                                                 float *tgt, uint8_t *mask)
{
    const long i = (long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (long)S * ch * cw)
        return;
    const int cx = (int)(i % cw);
    const long t = i / cw;
    const int cy = (int)(t % ch), s = (int)(t / ch);
    const int oy = crop[s], ox = crop[cap + s];
    const long n = (long)H * W, v = (long)(oy + cy) * W + (ox + cx);
    const double *x2 = ptrs[s], *x1 = ptrs[cap + s], *x0 = ptrs[2 * cap + s];
    const double *st = stats + kStat * s;
    for (int c = 0; c < 4; ++c) {
        const double a = x1[sidx(c, v, n)];
        const double d = a - x2[sidx(c, v, n)];
        const double is = inv_or_zero(st[c]);
        feat[i * 8 + c] = to_bf16((float)(d * is));
        feat[i * 8 + 4 + c] = to_bf16((float)((a - st[4 + c]) * inv_or_zero(st[8 + c])));
        if (tgt)
            tgt[i * 4 + c] = (float)((x0[sidx(c, v, n)] - a - d) * is);
    }
    if (mask) {
        bool on = true;
        if (oy > 0 && cy < kRadius)
            on = false;
        if (oy + ch < H && cy >= ch - kRadius)
            on = false;
        if (ox > 0 && cx < kRadius)
            on = false;
        if (ox + cw < W && cx >= cw - kRadius)
            on = false;
        mask[i] = on ? 1 : 0;
    }
}

// guess = x1 + (x1 - x2) + sigma_c y_c over a state vector of 4 n doubles
__global__ void __launch_bounds__(kBlock) k_guess(long n, const double *__restrict__ x2,
                                                  const double *__restrict__ x1,
                                                  const float *__restrict__ y,
                                                  const double *__restrict__ stats, double *out)
{
    const long i = (long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= 4 * n)
        return;
    const long blk = i / (2 * n), v = (i % (2 * n)) / 2;
    const int c = (int)(2 * blk + (i & 1));
    const double a = x1[i];
    out[i] = a + (a - x2[i]) + stats[c] * (double)y[v * 4 + c];
}

__global__ void k_f32_to_bf16(long n, const float *__restrict__ a, bf16_t *b)
{
    const long i = (long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        b[i] = to_bf16(a[i]);
}

__global__ void k_bf16_to_f32(long n, const bf16_t *__restrict__ a, float *b)
{
    const long i = (long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        b[i] = from_bf16(a[i]);
}

inline int nblk_l(long n) { return (int)std::max<long>(1, (n + kBlock - 1) / kBlock); }

}  // namespace
}  // namespace chm

struct chm_net {
    chm::Err err;
    hipStream_t stream = nullptr;
    chm::Pool pool;
    long long max_px = 0;
    int max_chunks = 0;
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    int adam_t = 0;
    bf16_t *wf[chm::kLayers] = {}, *wb[chm::kLayers] = {};
    bf16_t *act[chm::kLayers] = {};   // act[0]: features [px][8]; act[k]: [px][32]
    float *y = nullptr, *tgt = nullptr;
    uint8_t *mask = nullptr;
    bf16_t *gy = nullptr, *gA = nullptr, *gB = nullptr;
    float *wpart = nullptr, *bpart = nullptr;
    double *lpart = nullptr;
    double *stats = nullptr;         // [kMaxBatch][kStat]
    double *wts = nullptr;           // sample weights [kMaxBatch]
    int *msum = nullptr;             // masked pixels per sample [kMaxBatch]
    const double **ptrs = nullptr;   // [3][kMaxBatch]
    int *crop = nullptr;             // [2][kMaxBatch]
};

namespace chm {
namespace {

void refresh_bf16(chm_net &N, hipStream_t st)
{
    for (int k = 0; k < kLayers; ++k) {
        const int co16 = (kCout[k] + 15) / 16 * 16;
        k_wconv<<<nblk_l(9l * kCin[k] * co16), kBlock, 0, st>>>(kCin[k], kCout[k], co16,
                                                                N.params + w_offset(k), N.wf[k],
                                                                N.wb[k]);
    }
    CHM_HIP(hipGetLastError());
}

void check_shape(const chm_net &N, long batch, long h, long w)
{
    if (batch < 1 || h < 2 || w < 2)
        throw Failure(CHM_EINVAL, "need batch >= 1 and h, w >= 2");
    if (batch * h * w > N.max_px)
        throw Failure(CHM_EINVAL, "batch * h * w exceeds the network's max_pixels");
}

// The four layers over npx = B H W pixels: features a0 -> a1 -> a2 -> a3 ->
// output y (a3 may alias a1)
void forward_on(chm_net &N, hipStream_t st, int B, int H, int W, const bf16_t *a0, bf16_t *a1,
                bf16_t *a2, bf16_t *a3, float *y)
{
    const long npx = (long)B * H * W;
    const int g = nblk_l(npx);
    k_conv_fwd<8, 32, true><<<g, kBlock, 0, st>>>(B, H, W, a0, N.wf[0], N.params + b_offset(0), a1,
                                                  nullptr);
    k_conv_fwd<32, 32, true><<<g, kBlock, 0, st>>>(B, H, W, a1, N.wf[1], N.params + b_offset(1), a2,
                                                   nullptr);
    k_conv_fwd<32, 32, true><<<g, kBlock, 0, st>>>(B, H, W, a2, N.wf[2], N.params + b_offset(2), a3,
                                                   nullptr);
    k_conv_fwd<32, 4, false><<<g, kBlock, 0, st>>>(B, H, W, a3, N.wf[3], N.params + b_offset(3),
                                                   nullptr, y);
    CHM_HIP(hipGetLastError());
}

// act[0] holds the BF16 features of npx = B H W pixels; y receives the output
// (the activations stay in act[1..3] for the backward pass)
void forward(chm_net &N, hipStream_t st, int B, int H, int W)
{
    forward_on(N, st, B, H, W, N.act[0], N.act[1], N.act[2], N.act[3], N.y);
}

template <int CI, int CO>
void layer_grads(chm_net &N, hipStream_t st, int k, int B, int H, int W, const bf16_t *gout)
{
    const long npx = (long)B * H * W;
    const int nch = (int)((npx + kChunk - 1) / kChunk);
    k_conv_bwd_w<CI, CO><<<dim3(nch, 9), kBlock, 0, st>>>(B, H, W, N.act[k], gout, N.wpart);
    k_bias_part<CO><<<nch, kBlock, 0, st>>>(npx, gout, N.bpart);
    const int nw = 9 * CI * CO;
    k_grad_reduce<<<nblk_l(nw + CO), kBlock, 0, st>>>(nch, nw, CO, N.wpart, N.bpart,
                                                      N.grads + w_offset(k), N.grads + b_offset(k));
}

// gradients into N.grads from N.gy (dL/dy, BF16) and the stored activations
void backward(chm_net &N, hipStream_t st, int B, int H, int W)
{
    const int g = nblk_l((long)B * H * W);
    layer_grads<32, 4>(N, st, 3, B, H, W, N.gy);
    k_conv_bwd_data<32, 4><<<g, kBlock, 0, st>>>(B, H, W, N.gy, N.wb[3], N.act[3], N.gA);
    layer_grads<32, 32>(N, st, 2, B, H, W, N.gA);
    k_conv_bwd_data<32, 32><<<g, kBlock, 0, st>>>(B, H, W, N.gA, N.wb[2], N.act[2], N.gB);
    layer_grads<32, 32>(N, st, 1, B, H, W, N.gB);
    k_conv_bwd_data<32, 32><<<g, kBlock, 0, st>>>(B, H, W, N.gB, N.wb[1], N.act[1], N.gA);
    layer_grads<8, 32>(N, st, 0, B, H, W, N.gA);
    CHM_HIP(hipGetLastError());
}

// loss gradient into N.gy for S samples of ch x cw pixels (weights and masked
// counts in N.wts, N.msum); returns the loss when want (synchronises)
double loss_grad(chm_net &N, hipStream_t st, int S, int ch, int cw, double smooth, bool want)
{
    k_loss<<<kRedBlocks, kBlock, 0, st>>>(4l * S * ch * cw, ch, cw, S, N.y, N.tgt, N.mask, N.wts,
                                          N.msum, smooth, N.gy, N.lpart);
    CHM_HIP(hipGetLastError());
    if (!want)
        return 0.0;
    double h[kRedBlocks];
    CHM_HIP(hipMemcpyAsync(h, N.lpart, sizeof(h), hipMemcpyDeviceToHost, st));
    CHM_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (int i = 0; i < kRedBlocks; ++i)
        s += h[i];
    return s;
}

void adam_step(chm_net &N, hipStream_t st, float lr)
{
    N.adam_t += 1;
    const float c1 = (float)(1.0 - std::pow(kBeta1, N.adam_t));
    const float c2 = (float)(1.0 - std::pow(kBeta2, N.adam_t));
    k_adam<<<nblk_l(CHM_NET_NPARAMS), kBlock, 0, st>>>(CHM_NET_NPARAMS, N.params, N.grads, N.adam_m,
                                                       N.adam_v, lr, (float)kBeta1, (float)kBeta2,
                                                       (float)kAdamEps, c1, c2);
    CHM_HIP(hipGetLastError());
    refresh_bf16(N, st);
}

void upload_batch(chm_net &N, hipStream_t st, int S, const double *const *x2,
                  const double *const *x1, const double *const *x0, const int32_t *oy,
                  const int32_t *ox, const int *msum)
{
    for (int base = 0; base < S; base += kPtrBatch) {
        BatchPtrs b{};
        const int cnt = std::min(kPtrBatch, S - base);
        for (int i = 0; i < cnt; ++i) {
            b.x2[i] = x2[base + i];
            b.x1[i] = x1[base + i];
            b.x0[i] = x0 ? x0[base + i] : nullptr;
            b.oy[i] = oy ? oy[base + i] : 0;
            b.ox[i] = ox ? ox[base + i] : 0;
            b.msum[i] = msum ? msum[base + i] : 0;
        }
        k_set_batch<<<1, kPtrBatch, 0, st>>>(b, base, cnt, kMaxBatch, N.ptrs, N.crop, N.msum);
    }
    CHM_HIP(hipGetLastError());
}

// Where the guess of one H x W frame keeps its work: the sample tables
// (pointers, crop origin, masked count; `cap` samples each), the frame
// statistics, the features, two hidden activations and the output.
struct GuessBufs {
    const double **ptrs;
    int *crop, *msum, cap;
    double *stats;
    bf16_t *feat, *h1, *h2;
    float *y;
};

// features of (x2, x1) over the whole H x W grid into B.feat; stats of sample 0
void features_into(hipStream_t st, int H, int W, const double *x2, const double *x1,
                   const GuessBufs &B)
{
    BatchPtrs b{};
    b.x2[0] = x2;
    b.x1[0] = x1;
    k_set_batch<<<1, kPtrBatch, 0, st>>>(b, 0, 1, B.cap, B.ptrs, B.crop, B.msum);
    k_stats<<<1, kBlock, 0, st>>>((long)H * W, B.ptrs, B.ptrs + B.cap, nullptr, B.stats);
    k_pack<<<nblk_l((long)H * W), kBlock, 0, st>>>(1, H, W, H, W, B.cap, B.ptrs, B.crop, B.stats,
                                                   B.feat, nullptr, nullptr);
    CHM_HIP(hipGetLastError());
}

GuessBufs own_bufs(chm_net &N)
{
    return GuessBufs{N.ptrs, N.crop, N.msum, kMaxBatch, N.stats, N.act[0], N.act[1], N.act[2], N.y};
}

// features of (x2, x1) over the whole H x W grid into act[0]; stats of sample 0
void full_features(chm_net &N, hipStream_t st, int H, int W, const double *x2, const double *x1)
{
    check_shape(N, 1, H, W);
    features_into(st, H, W, x2, x1, own_bufs(N));
}

// the guess of one frame: features, the network, x1 + d + sigma y
void guess_into(chm_net &N, hipStream_t st, int H, int W, const double *x2, const double *x1,
                double *out, const GuessBufs &B)
{
    features_into(st, H, W, x2, x1, B);
    forward_on(N, st, 1, H, W, B.feat, B.h1, B.h2, B.h1, B.y);
    const long n = (long)H * W;
    k_guess<<<nblk_l(4 * n), kBlock, 0, st>>>(n, x2, x1, B.y, B.stats, out);
    CHM_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ allocation-free guess
// The work buffers of chm_net_guess_noalloc live in one fixed device array,
// `scratch`, which every GPU the library runs on holds for the life of the
// process: a header (sample tables and frame statistics), then the features,
// two hidden activations and the output of at most kNoAllocPixels pixels.
// In host code `scratch` names a host-side stand-in, so its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and only that address is ever handed to kernels.  Nothing in it needs to
// start at zero: every kernel of the guess writes what the next one reads.
constexpr long kNoAllocPixels = CHM_NET_NOALLOC_MAX_PIXELS;
constexpr size_t kScratchHead = 1024;
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kFeatBytes = align256(kNoAllocPixels * 8 * sizeof(bf16_t));
constexpr size_t kHidBytes = align256(kNoAllocPixels * 32 * sizeof(bf16_t));
constexpr size_t kOutBytes = align256(kNoAllocPixels * 4 * sizeof(float));
constexpr size_t kScratchBytes = kScratchHead + kFeatBytes + 2 * kHidBytes + kOutBytes;
static_assert(3 * sizeof(double *) + 3 * sizeof(int) + kStat * sizeof(double) + 64 <= kScratchHead,
              "scratch header");

}  // namespace
}  // namespace chm

static __device__ __align__(256) unsigned char scratch[chm::kScratchBytes];

namespace chm {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on first use)
void *scratch_address()
{
    int dev = 0;
    CHM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        throw Failure(CHM_EINVAL, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        CHM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            throw Failure(CHM_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_dev[dev] = p;
    }
    return g_scratch_dev[dev];
}

// the guess buffers carved out of the scratch array at base
GuessBufs scratch_bufs(void *base)
{
    unsigned char *b = static_cast<unsigned char *>(base);
    GuessBufs g;
    g.ptrs = reinterpret_cast<const double **>(b);
    g.crop = reinterpret_cast<int *>(b + 3 * sizeof(double *));
    g.msum = g.crop + 2;
    g.cap = 1;
    g.stats = reinterpret_cast<double *>(b + 64);
    g.feat = reinterpret_cast<bf16_t *>(b + kScratchHead);
    g.h1 = reinterpret_cast<bf16_t *>(b + kScratchHead + kFeatBytes);
    g.h2 = reinterpret_cast<bf16_t *>(b + kScratchHead + kFeatBytes + kHidBytes);
    g.y = reinterpret_cast<float *>(b + kScratchHead + kFeatBytes + 2 * kHidBytes);
    return g;
}

thread_local std::string g_net_create_error;

int net_fail(chm_net *N, int code, const std::string &msg)
{
    if (N) {
        N->err.code = code;
        N->err.msg = msg;
    } else {
        g_net_create_error = msg;
    }
    return code;
}

template <class F> int net_guarded(chm_net *N, F &&f)
{
    try {
        return f();
    } catch (const Failure &e) {
        return net_fail(N, e.code, e.msg);
    } catch (const std::bad_alloc &) {
        return net_fail(N, CHM_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return net_fail(N, CHM_EINVAL, e.what());
    }
}

}  // namespace

long long net_max_pixels(const chm_net *net) { return net ? net->max_px : 0; }

void net_guess_on(chm_net *net, hipStream_t st, int H, int W, const double *x2, const double *x1,
                  double *out)
{
    check_shape(*net, 1, H, W);
    guess_into(*net, st, H, W, x2, x1, out, own_bufs(*net));
}

}  // namespace chm

using chm::net_fail;
using chm::net_guarded;

extern "C" {

int chm_net_create(int64_t max_pixels, void *stream, chm_net_t **out)
{
    if (!out)
        return CHM_EINVAL;
    *out = nullptr;
    if (max_pixels < 4 || max_pixels > (int64_t(1) << 26))
        return net_fail(nullptr, CHM_EINVAL, "max_pixels must be in [4, 2^26]");
    chm_net *N = new (std::nothrow) chm_net;
    if (!N)
        return CHM_ENOMEM;
    const int rc = net_guarded(N, [&]() {
        using namespace chm;
        N->stream = static_cast<hipStream_t>(stream);
        N->max_px = max_pixels;
        N->max_chunks = (int)((max_pixels + kChunk - 1) / kChunk);
        Pool &p = N->pool;
        const long px = max_pixels;
        N->params = p.get<float>(CHM_NET_NPARAMS);
        N->grads = p.get<float>(CHM_NET_NPARAMS);
        N->adam_m = p.get<float>(CHM_NET_NPARAMS);
        N->adam_v = p.get<float>(CHM_NET_NPARAMS);
        for (int k = 0; k < kLayers; ++k) {
            const size_t wn = 9 * (size_t)kCin[k] * ((kCout[k] + 15) / 16 * 16);
            N->wf[k] = p.get<bf16_t>(wn);
            N->wb[k] = p.get<bf16_t>(wn);
            N->act[k] = p.get<bf16_t>((size_t)px * kCin[k]);
        }
        N->y = p.get<float>((size_t)px * 4);
        N->tgt = p.get<float>((size_t)px * 4);
        N->mask = p.get<uint8_t>((size_t)px);
        N->gy = p.get<bf16_t>((size_t)px * 4);
        N->gA = p.get<bf16_t>((size_t)px * 32);
        N->gB = p.get<bf16_t>((size_t)px * 32);
        N->wpart = p.get<float>((size_t)N->max_chunks * 9 * 32 * 32);
        N->bpart = p.get<float>((size_t)N->max_chunks * 32);
        N->lpart = p.get<double>(kRedBlocks);
        N->stats = p.get<double>(kStat * kMaxBatch);
        N->wts = p.get<double>(kMaxBatch);
        N->msum = p.get<int>(kMaxBatch);
        N->ptrs = p.get<const double *>(3 * kMaxBatch);
        N->crop = p.get<int>(2 * kMaxBatch);
        hipStream_t st = N->stream;
        CHM_HIP(hipMemsetAsync(N->params, 0, sizeof(float) * CHM_NET_NPARAMS, st));
        CHM_HIP(hipMemsetAsync(N->adam_m, 0, sizeof(float) * CHM_NET_NPARAMS, st));
        CHM_HIP(hipMemsetAsync(N->adam_v, 0, sizeof(float) * CHM_NET_NPARAMS, st));
        refresh_bf16(*N, st);
        CHM_HIP(hipStreamSynchronize(st));
        (void)scratch_address();   // the allocation-free guess's array on this device
        return CHM_OK;
    });
    if (rc != CHM_OK) {
        chm::g_net_create_error = N->err.msg;
        delete N;
        return rc;
    }
    *out = N;
    return CHM_OK;
}

int chm_net_destroy(chm_net_t *net)
{
    if (!net)
        return CHM_EINVAL;
    (void)hipStreamSynchronize(net->stream);
    delete net;
    return CHM_OK;
}

const char *chm_net_last_error(const chm_net_t *net)
{
    return net ? net->err.msg.c_str() : chm::g_net_create_error.c_str();
}

int chm_net_set_params(chm_net_t *net, const float *params)
{
    if (!net || !params)
        return net_fail(net, CHM_EINVAL, "chm_net_set_params: bad arguments");
    return net_guarded(net, [&]() {
        hipStream_t st = net->stream;
        CHM_HIP(hipMemcpyAsync(net->params, params, sizeof(float) * CHM_NET_NPARAMS,
                               hipMemcpyHostToDevice, st));
        CHM_HIP(hipMemsetAsync(net->adam_m, 0, sizeof(float) * CHM_NET_NPARAMS, st));
        CHM_HIP(hipMemsetAsync(net->adam_v, 0, sizeof(float) * CHM_NET_NPARAMS, st));
        net->adam_t = 0;
        chm::refresh_bf16(*net, st);
        CHM_HIP(hipStreamSynchronize(st));
        return CHM_OK;
    });
}

int chm_net_get_params(chm_net_t *net, float *params)
{
    if (!net || !params)
        return net_fail(net, CHM_EINVAL, "chm_net_get_params: bad arguments");
    return net_guarded(net, [&]() {
        CHM_HIP(hipMemcpyAsync(params, net->params, sizeof(float) * CHM_NET_NPARAMS,
                               hipMemcpyDeviceToHost, net->stream));
        CHM_HIP(hipStreamSynchronize(net->stream));
        return CHM_OK;
    });
}

int chm_net_features(chm_net_t *net, int32_t H, int32_t W, const double *x2, const double *x1,
                     float *feats, double *sigma)
{
    if (!net || !x2 || !x1 || !feats)
        return net_fail(net, CHM_EINVAL, "chm_net_features: bad arguments");
    return net_guarded(net, [&]() {
        using namespace chm;
        hipStream_t st = net->stream;
        full_features(*net, st, H, W, x2, x1);
        const long n8 = 8l * H * W;
        k_bf16_to_f32<<<nblk_l(n8), kBlock, 0, st>>>(n8, net->act[0], feats);
        CHM_HIP(hipGetLastError());
        if (sigma)
            CHM_HIP(hipMemcpyAsync(sigma, net->stats, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
        CHM_HIP(hipStreamSynchronize(st));
        return CHM_OK;
    });
}

int chm_net_forward(chm_net_t *net, int32_t batch, int32_t h, int32_t w, const float *feats,
                    float *y)
{
    if (!net || !feats || !y)
        return net_fail(net, CHM_EINVAL, "chm_net_forward: bad arguments");
    return net_guarded(net, [&]() {
        using namespace chm;
        check_shape(*net, batch, h, w);
        hipStream_t st = net->stream;
        const long npx = (long)batch * h * w;
        k_f32_to_bf16<<<nblk_l(8 * npx), kBlock, 0, st>>>(8 * npx, feats, net->act[0]);
        forward(*net, st, batch, h, w);
        CHM_HIP(hipMemcpyAsync(y, net->y, sizeof(float) * 4 * npx, hipMemcpyDeviceToDevice, st));
        CHM_HIP(hipStreamSynchronize(st));
        return CHM_OK;
    });
}

int chm_net_gradients(chm_net_t *net, int32_t batch, int32_t h, int32_t w, const float *feats,
                      const float *target, const uint8_t *mask, const double *weights,
                      float smooth, float *grads, double *loss)
{
    if (!net || !feats || !target || !mask || !grads || !(smooth >= 0.0f))
        return net_fail(net, CHM_EINVAL, "chm_net_gradients: bad arguments");
    return net_guarded(net, [&]() {
        using namespace chm;
        check_shape(*net, batch, h, w);
        if (batch > kMaxBatch)
            throw Failure(CHM_EINVAL, "batch exceeds 256");
        hipStream_t st = net->stream;
        const long chs = (long)h * w, npx = batch * chs;
        std::vector<uint8_t> hm(npx);
        CHM_HIP(hipMemcpyAsync(hm.data(), mask, npx, hipMemcpyDeviceToHost, st));
        CHM_HIP(hipStreamSynchronize(st));
        std::vector<int> ms(batch, 0);
        std::vector<double> wt(batch, 1.0);
        for (long p = 0; p < npx; ++p)
            ms[p / chs] += hm[p] ? 1 : 0;
        if (weights)
            for (int s = 0; s < batch; ++s)
                wt[s] = weights[s];
        CHM_HIP(hipMemcpyAsync(net->msum, ms.data(), sizeof(int) * batch, hipMemcpyHostToDevice, st));
        CHM_HIP(hipMemcpyAsync(net->wts, wt.data(), sizeof(double) * batch, hipMemcpyHostToDevice, st));
        k_f32_to_bf16<<<nblk_l(8 * npx), kBlock, 0, st>>>(8 * npx, feats, net->act[0]);
        CHM_HIP(hipMemcpyAsync(net->tgt, target, sizeof(float) * 4 * npx, hipMemcpyDeviceToDevice, st));
        CHM_HIP(hipMemcpyAsync(net->mask, mask, npx, hipMemcpyDeviceToDevice, st));
        forward(*net, st, batch, h, w);
        const double l = loss_grad(*net, st, batch, h, w, smooth, true);
        backward(*net, st, batch, h, w);
        CHM_HIP(hipMemcpyAsync(grads, net->grads, sizeof(float) * CHM_NET_NPARAMS,
                               hipMemcpyDeviceToHost, st));
        CHM_HIP(hipStreamSynchronize(st));
        if (loss)
            *loss = l;
        return CHM_OK;
    });
}

int chm_net_adam(chm_net_t *net, const float *grads, float lr)
{
    if (!net || !grads || !(lr >= 0.0f))
        return net_fail(net, CHM_EINVAL, "chm_net_adam: bad arguments");
    return net_guarded(net, [&]() {
        hipStream_t st = net->stream;
        CHM_HIP(hipMemcpyAsync(net->grads, grads, sizeof(float) * CHM_NET_NPARAMS,
                               hipMemcpyHostToDevice, st));
        chm::adam_step(*net, st, lr);
        CHM_HIP(hipStreamSynchronize(st));
        return CHM_OK;
    });
}

int chm_net_guess(chm_net_t *net, int32_t H, int32_t W, const double *x2, const double *x1,
                  double *guess)
{
    if (!net || !x2 || !x1 || !guess)
        return net_fail(net, CHM_EINVAL, "chm_net_guess: bad arguments");
    return net_guarded(net, [&]() {
        chm::net_guess_on(net, net->stream, H, W, x2, x1, guess);
        CHM_HIP(hipStreamSynchronize(net->stream));
        return CHM_OK;
    });
}

int chm_net_guess_noalloc(chm_net_t *net, int32_t H, int32_t W, const double *x2,
                          const double *x1, double *guess)
{
    if (!net || !x2 || !x1 || !guess)
        return net_fail(net, CHM_EINVAL, "chm_net_guess_noalloc: bad arguments");
    if (H < 2 || W < 2 || (int64_t)H * W > CHM_NET_NOALLOC_MAX_PIXELS)
        return net_fail(net, CHM_EINVAL,
                        "chm_net_guess_noalloc: need H, W >= 2 and H * W <= "
                        "CHM_NET_NOALLOC_MAX_PIXELS (" +
                            std::to_string(CHM_NET_NOALLOC_MAX_PIXELS) + ")");
    return net_guarded(net, [&]() {
        using namespace chm;
        guess_into(*net, net->stream, H, W, x2, x1, guess, scratch_bufs(scratch_address()));
        return CHM_OK;
    });
}

int chm_net_train_step(chm_net_t *net, int32_t batch, int32_t H, int32_t W, int32_t crop_h,
                       int32_t crop_w, const double *const *x2, const double *const *x1,
                       const double *const *x0, const int32_t *oy, const int32_t *ox, float lr,
                       float smooth, double *loss)
{
    if (!net || !x2 || !x1 || !x0 || !oy || !ox || !(lr >= 0.0f) || !(smooth >= 0.0f))
        return net_fail(net, CHM_EINVAL, "chm_net_train_step: bad arguments");
    return net_guarded(net, [&]() {
        using namespace chm;
        if (batch > kMaxBatch)
            throw Failure(CHM_EINVAL, "batch exceeds 256");
        if (H < 2 || W < 2 || crop_h > H || crop_w > W)
            throw Failure(CHM_EINVAL, "crop larger than the grid");
        check_shape(*net, batch, crop_h, crop_w);
        std::vector<int> ms(batch);
        for (int i = 0; i < batch; ++i) {
            if (!x2[i] || !x1[i] || !x0[i])
                throw Failure(CHM_EINVAL, "null state pointer");
            if (oy[i] < 0 || ox[i] < 0 || oy[i] + crop_h > H || ox[i] + crop_w > W)
                throw Failure(CHM_EINVAL, "crop outside the grid");
            const int top = oy[i] > 0 ? kRadius : 0, bot = oy[i] + crop_h < H ? kRadius : 0;
            const int lft = ox[i] > 0 ? kRadius : 0, rgt = ox[i] + crop_w < W ? kRadius : 0;
            ms[i] = std::max(0, crop_h - top - bot) * std::max(0, crop_w - lft - rgt);
        }
        hipStream_t st = net->stream;
        upload_batch(*net, st, batch, x2, x1, x0, oy, ox, ms.data());
        k_stats<<<batch, kBlock, 0, st>>>((long)H * W, net->ptrs, net->ptrs + kMaxBatch,
                                          net->ptrs + 2 * kMaxBatch, net->stats);
        k_weights<<<1, kMaxBatch, 0, st>>>(batch, net->stats, net->wts);
        const long npx = (long)batch * crop_h * crop_w;
        k_pack<<<nblk_l(npx), kBlock, 0, st>>>(batch, H, W, crop_h, crop_w, kMaxBatch, net->ptrs,
                                               net->crop, net->stats, net->act[0], net->tgt,
                                               net->mask);
        CHM_HIP(hipGetLastError());
        forward(*net, st, batch, crop_h, crop_w);
        const double l = loss_grad(*net, st, batch, crop_h, crop_w, smooth, loss != nullptr);
        backward(*net, st, batch, crop_h, crop_w);
        adam_step(*net, st, lr);
        CHM_HIP(hipStreamSynchronize(st));
        if (loss)
            *loss = l;
        return CHM_OK;
    });
}

}  // extern "C"
