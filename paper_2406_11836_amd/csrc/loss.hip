// loss.hip -- L1 + w (1 - SSIM) on one view, forward and backward.
//
// SSIM uses an 11x11 Gaussian window (std 1.5, normalised), zero padding and
// C1 = 0.01^2, C2 = 0.03^2; the window is separable, so the local moments
// take a horizontal and a vertical 11-tap pass, both run from LDS on 32x16
// tiles with a 5-pixel halo.  E[x^2] and E[y^2] enter SSIM only through
// sigma_x^2 + sigma_y^2, so four moments are filtered: mu_x, mu_y,
// E[x^2 + y^2] and E[xy].  The backward needs d SSIM / d (mu_x, E[x^2], E[xy])
// per pixel, convolved again with the (symmetric) window.  Block partial sums
// are combined by one block in a fixed order, so the scalar is reproducible.
#include <mutex>

#include "common.hpp"

namespace rgs {

struct Win11 { float w[11]; };

static constexpr int LS_THREADS = 256;

__global__ __launch_bounds__(LS_THREADS) void k_l1_only(const float* __restrict__ x, const float* __restrict__ y, int64_t m,
                                                        float invN, float* __restrict__ dx, float* __restrict__ part) {
    __shared__ float s_w[4];
    const int64_t i = (int64_t)blockIdx.x * LS_THREADS + threadIdx.x;
    float a = 0.f;
    if (i < m) {
        const float d = x[i] - y[i];
        a = fabsf(d);
        dx[i] = (float)((d > 0.f) - (d < 0.f)) * invN;
    }
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
        part[2 * blockIdx.x + 1] = 0.f;
    }
}

// Tiled SSIM: one 256-thread block per 32x16 output tile of one channel,
// with the 5-pixel halo staged in LDS; both separable passes run from LDS.
// (32x16 rather than 32x32: 25 KB of LDS per block instead of 41 KB, so that
// five blocks share a CU instead of three and the passes of one block
// overlap the loads of another.)  Tiles are handed out in XCD bands: a tile's
// halo rows were loaded by the tile row above it into the same L2.
static constexpr int HALO = 5;
static constexpr int TS = 32, TW = TS + 2 * HALO;       // output / staged columns (42)
static constexpr int TSY = 16, TH = TSY + 2 * HALO;     // output / staged rows (26)
static constexpr int RPT = TSY / 8;                      // output rows per thread in the vertical pass
static constexpr int VWIN = RPT + 2 * HALO;              // its window of horizontal results
// Staging: thread (column c, row group g) of TW x SG loads rows g, g + SG, ...
// of the tile with its halo (index arithmetic once per thread, not per value).
static constexpr int SG = LS_THREADS / TW;               // 6 row groups
static_assert(SG >= 1 && TW * SG <= LS_THREADS, "staging layout");
static constexpr int SR = (TH + SG - 1) / SG;            // rows per thread (5)

// Forward: SSIM map terms and d SSIM / d (mu_x, E[x^2], E[xy]) per pixel,
// plus block sums of the SSIM map and of |x - y|.
__global__ __launch_bounds__(LS_THREADS) void k_ssim_fwd_tiled(const float* __restrict__ x, const float* __restrict__ y,
                                                               int H, int W, Win11 win, float* __restrict__ d3,
                                                               float* __restrict__ part) {
    __shared__ float sx[TH * TW], sy[TH * TW];
    __shared__ float hm[4][TH * TS];
    __shared__ float s_w[2][4];
    const int tiles_x = (W + TS - 1) / TS, tiles_y = (H + TSY - 1) / TSY;
    const int b = xcd_band((int)blockIdx.x, (int)gridDim.x);  // neighbouring tiles on one XCD
    const int ch = b / (tiles_x * tiles_y);
    const int tt = b % (tiles_x * tiles_y);
    const int x0 = (tt % tiles_x) * TS, y0 = (tt / tiles_x) * TSY;
    const int64_t HW = (int64_t)H * W;
    const float* xc = x + ch * HW;
    const float* yc = y + ch * HW;
    if (threadIdx.x < TW * SG) {
        const int c = threadIdx.x % TW, g = threadIdx.x / TW;
        const int gx = x0 + c - HALO;
        const bool xin = gx >= 0 && gx < W;
        // all loads of the thread are issued before the stores
        float vx[SR], vy[SR];
#pragma unroll
        for (int i = 0; i < SR; ++i) {
            const int r = g + SG * i, gy = y0 + r - HALO;
            const bool in = r < TH && xin && gy >= 0 && gy < H;
            const int64_t gi = (int64_t)gy * W + gx;
            vx[i] = in ? xc[gi] : 0.f;
            vy[i] = in ? yc[gi] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < SR; ++i) {
            const int r = g + SG * i;
            if (r < TH) {
                sx[r * TW + c] = vx[i];
                sy[r * TW + c] = vy[i];
            }
        }
    }
    __syncthreads();
    // horizontal pass: a thread takes 4 consecutive outputs of one row from a
    // 14-value window in registers (the taps of each output in the same order)
    for (int k = threadIdx.x; k < TH * (TS / 4); k += LS_THREADS) {
        const int r = k >> 3, c0 = (k & 7) * 4;
        float xv[14], yv[14], ss[14], xy[14];
#pragma unroll
        for (int j = 0; j < 14; ++j) {
            xv[j] = sx[r * TW + c0 + j];
            yv[j] = sy[r * TW + c0 + j];
            ss[j] = xv[j] * xv[j] + yv[j] * yv[j];  // products once per input, not once per tap
            xy[j] = xv[j] * yv[j];
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
            for (int t = 0; t < 11; ++t) {
                const float w = win.w[t];
                a0 = fmaf(w, xv[o + t], a0);
                a1 = fmaf(w, yv[o + t], a1);
                a2 = fmaf(w, ss[o + t], a2);
                a3 = fmaf(w, xy[o + t], a3);
            }
            const int q = r * TS + c0 + o;
            hm[0][q] = a0; hm[1][q] = a1; hm[2][q] = a2; hm[3][q] = a3;
        }
    }
    __syncthreads();
    float l1 = 0.f, ss = 0.f;
    // vertical pass: thread (column c, row group) takes RPT consecutive rows
    {
        const int c = threadIdx.x & 31, r0 = (threadIdx.x >> 5) * RPT;
        float mom[4][RPT];
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
            float hv[VWIN];
#pragma unroll
            for (int j = 0; j < VWIN; ++j) hv[j] = hm[mm][(r0 + j) * TS + c];
#pragma unroll
            for (int o = 0; o < RPT; ++o) {
                float a = 0.f;
#pragma unroll
                for (int t = 0; t < 11; ++t) a = fmaf(win.w[t], hv[o + t], a);
                mom[mm][o] = a;
            }
        }
#pragma unroll
        for (int o = 0; o < RPT; ++o) {
            const int r = r0 + o;
            const int gy = y0 + r, gx = x0 + c;
            if (gy >= H || gx >= W) continue;
            const float mu_x = mom[0][o], mu_y = mom[1][o], ess = mom[2][o], exy = mom[3][o];
            const float C1 = 1e-4f, C2 = 9e-4f;
            const float A1 = 2.f * mu_x * mu_y + C1;
            const float A2 = 2.f * (exy - mu_x * mu_y) + C2;
            const float m2 = mu_x * mu_x + mu_y * mu_y;
            const float B1 = m2 + C1;
            const float B2 = (ess - m2) + C2;
            const float Nn = A1 * A2, Dd = B1 * B2;
            const float iD = 1.f / Dd;
            ss += Nn * iD;
            const float dN = 2.f * mu_y * A2 - 2.f * mu_y * A1;
            const float dD = 2.f * mu_x * B2 - 2.f * mu_x * B1;
            const int64_t i = ch * HW + (int64_t)gy * W + gx;
            const int64_t m = 3 * HW;
            d3[i] = (dN * Dd - Nn * dD) * iD * iD;
            d3[m + i] = -Nn * B1 * iD * iD;
            d3[2 * m + i] = 2.f * A1 * iD;
            l1 += fabsf(sx[(r + HALO) * TW + c + HALO] - sy[(r + HALO) * TW + c + HALO]);
        }
    }
    l1 = wave_sum(l1);
    ss = wave_sum(ss);
    if ((threadIdx.x & 63) == 0) { s_w[0][threadIdx.x >> 6] = l1; s_w[1][threadIdx.x >> 6] = ss; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * b] = (s_w[0][0] + s_w[0][1]) + (s_w[0][2] + s_w[0][3]);
        part[2 * b + 1] = (s_w[1][0] + s_w[1][1]) + (s_w[1][2] + s_w[1][3]);
    }
}

// The final sums of the block partials in one block of NT threads: a fixed
// order of additions for a given NT (reproducible).  s_a, s_b: NT doubles of
// LDS each.
template <int NT>
__device__ __forceinline__ void loss_final_sums(const float* __restrict__ part, int nb, float invN, float w,
                                                float* __restrict__ loss, double* s_a, double* s_b) {
    double a = 0.0, b = 0.0;
    // the same order of additions per thread as one partial at a time; the
    // loads of eight steps are issued before their adds
    constexpr int U = 8;
    int k = threadIdx.x;
    for (; k + (U - 1) * NT < nb; k += U * NT) {
        float2 pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pv[u] = reinterpret_cast<const float2*>(part)[k + u * NT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a += pv[u].x;
            b += pv[u].y;
        }
    }
    for (; k < nb; k += NT) { a += part[2 * k]; b += part[2 * k + 1]; }
    s_a[threadIdx.x] = a;
    s_b[threadIdx.x] = b;
    __syncthreads();
    for (int st = NT / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) { s_a[threadIdx.x] += s_a[threadIdx.x + st]; s_b[threadIdx.x] += s_b[threadIdx.x + st]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double l = s_a[0] * (double)invN;
        if (w != 0.f) l += (double)w * (1.0 - s_b[0] * (double)invN);
        *loss = (float)l;
    }
}

// The final sums after the L1-only loss.
static constexpr int LF_THREADS = 1024;

__global__ __launch_bounds__(LF_THREADS) void k_loss_final(const float* __restrict__ part, int nb, float invN, float w,
                                                           float* __restrict__ loss) {
    __shared__ double s_a[LF_THREADS], s_b[LF_THREADS];
    loss_final_sums<LF_THREADS>(part, nb, invN, w, loss, s_a, s_b);
}

// Backward: convolve the three derivative maps with the (symmetric) window
// and combine: dL/dx = sign(x - y)/N + sc (w*g_mu + 2 x w*g_xx + y w*g_xy).
// Block 0 adds up the forward's block partials into the loss (dispatched
// first, it runs beside the tiles instead of as a launch of its own);
// blocks 1.. take the tiles.
__global__ __launch_bounds__(LS_THREADS) void k_ssim_bwd_tiled(const float* __restrict__ x, const float* __restrict__ y,
                                                               const float* __restrict__ d3, int H, int W, Win11 win,
                                                               float invN, float sc, float* __restrict__ dx,
                                                               const float* __restrict__ part, float ssim_w,
                                                               float* __restrict__ loss) {
    __shared__ __align__(16) float sd[3][TH * TW];
    __shared__ float hm[3][TH * TS];
    static_assert(sizeof(sd) >= 2 * LS_THREADS * sizeof(double), "final sums reuse the staging array");
    const int tiles_x = (W + TS - 1) / TS, tiles_y = (H + TSY - 1) / TSY;
    const int ntiles = (int)gridDim.x - 1;
    if (blockIdx.x == 0) {
        double* s2 = reinterpret_cast<double*>(&sd[0][0]);
        loss_final_sums<LS_THREADS>(part, ntiles, invN, ssim_w, loss, s2, s2 + LS_THREADS);
        return;
    }
    const int b = xcd_band((int)blockIdx.x - 1, ntiles);  // neighbouring tiles on one XCD
    const int ch = b / (tiles_x * tiles_y);
    const int tt = b % (tiles_x * tiles_y);
    const int x0 = (tt % tiles_x) * TS, y0 = (tt / tiles_x) * TSY;
    const int64_t HW = (int64_t)H * W;
    const int64_t m = 3 * HW;
    if (threadIdx.x < TW * SG) {
        const int c = threadIdx.x % TW, g = threadIdx.x / TW;
        const int gx = x0 + c - HALO;
        const bool xin = gx >= 0 && gx < W;
        float v0[SR], v1[SR], v2[SR];
#pragma unroll
        for (int k = 0; k < SR; ++k) {
            const int r = g + SG * k, gy = y0 + r - HALO;
            const bool in = r < TH && xin && gy >= 0 && gy < H;
            const int64_t i = ch * HW + (int64_t)gy * W + gx;
            v0[k] = in ? d3[i] : 0.f;
            v1[k] = in ? d3[m + i] : 0.f;
            v2[k] = in ? d3[2 * m + i] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < SR; ++k) {
            const int r = g + SG * k;
            if (r < TH) {
                sd[0][r * TW + c] = v0[k];
                sd[1][r * TW + c] = v1[k];
                sd[2][r * TW + c] = v2[k];
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < TH * (TS / 4); k += LS_THREADS) {
        const int r = k >> 3, c0 = (k & 7) * 4;
#pragma unroll
        for (int mm = 0; mm < 3; ++mm) {
            float v[14];
#pragma unroll
            for (int j = 0; j < 14; ++j) v[j] = sd[mm][r * TW + c0 + j];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                float a = 0.f;
#pragma unroll
                for (int t = 0; t < 11; ++t) a = fmaf(win.w[t], v[o + t], a);
                hm[mm][r * TS + c0 + o] = a;
            }
        }
    }
    __syncthreads();
    {
        const int c = threadIdx.x & 31, r0 = (threadIdx.x >> 5) * RPT;
        float gm[3][RPT];
#pragma unroll
        for (int mm = 0; mm < 3; ++mm) {
            float hv[VWIN];
#pragma unroll
            for (int j = 0; j < VWIN; ++j) hv[j] = hm[mm][(r0 + j) * TS + c];
#pragma unroll
            for (int o = 0; o < RPT; ++o) {
                float a = 0.f;
#pragma unroll
                for (int t = 0; t < 11; ++t) a = fmaf(win.w[t], hv[o + t], a);
                gm[mm][o] = a;
            }
        }
#pragma unroll
        for (int o = 0; o < RPT; ++o) {
            const int gy = y0 + r0 + o, gx = x0 + c;
            if (gy >= H || gx >= W) continue;
            const int64_t i = ch * HW + (int64_t)gy * W + gx;
            const float xv = x[i], yv = y[i];
            const float d = xv - yv;
            const float l1g = (float)((d > 0.f) - (d < 0.f)) * invN;
            dx[i] = l1g + sc * (gm[0][o] + 2.f * xv * gm[1][o] + yv * gm[2][o]);
        }
    }
}

size_t loss_ws_bytes(int H, int W) {
    const int64_t m = 3 * (int64_t)H * W;
    const int64_t nb = (m + LS_THREADS - 1) / LS_THREADS;
    const int64_t nt = 3 * (int64_t)((W + TS - 1) / TS) * ((H + TSY - 1) / TSY);
    const int64_t np = nb > nt ? nb : nt;
    return (size_t)3 * m * sizeof(float) + (size_t)2 * np * sizeof(float) + 1024;
}

rgs_status loss_launch(const float* image, const float* target, int H, int W, float ssim_w, float* loss, float* dimg,
                       void* ws, hipStream_t s) {
    const int64_t m = 3 * (int64_t)H * W;
    const int64_t nb = (m + LS_THREADS - 1) / LS_THREADS;
    const int64_t nt = 3 * (int64_t)((W + TS - 1) / TS) * ((H + TSY - 1) / TSY);
    WsCarver c{reinterpret_cast<char*>(ws), 0, (size_t)-1};
    float* d3 = c.take<float>(3 * m);
    float* part = c.take<float>(2 * (nb > nt ? nb : nt));
    const float invN = (float)(1.0 / (double)m);
    Win11 win;
    double g[11], gs = 0.0;
    for (int k = 0; k < 11; ++k) { g[k] = exp(-((k - 5) * (k - 5)) / (2.0 * 1.5 * 1.5)); gs += g[k]; }
    for (int k = 0; k < 11; ++k) win.w[k] = (float)(g[k] / gs);
    if (ssim_w == 0.f) {
        hipLaunchKernelGGL(k_l1_only, dim3((unsigned)nb), dim3(LS_THREADS), 0, s, image, target, m, invN, dimg, part);
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(LF_THREADS), 0, s, part, (int)nb, invN, ssim_w, loss);
    } else {
        hipLaunchKernelGGL(k_ssim_fwd_tiled, dim3((unsigned)nt), dim3(LS_THREADS), 0, s, image, target, H, W, win, d3, part);
        // the final sums in its block 0
        hipLaunchKernelGGL(k_ssim_bwd_tiled, dim3((unsigned)nt + 1u), dim3(LS_THREADS), 0, s, image, target, d3, H, W,
                           win, invN, -ssim_w * invN, dimg, part, ssim_w, loss);
    }
    return launch_check();
}

// Fixed workspace of the allocation-free loss entry point: one copy per
// device, held until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is a stand-in, not a device address); it
// uses the address hipGetSymbolAddress returns for the current device, taken
// once per device and kept.
static __device__ __align__(256) unsigned char scratch[RGS_LOSS_SCRATCH_BYTES];

static constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[SCRATCH_MAX_DEVICES];

rgs_status loss_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_hip_error(e);
        return RGS_E_HIP;
    }
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return RGS_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return RGS_E_HIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return RGS_OK;
}

}  // namespace rgs
