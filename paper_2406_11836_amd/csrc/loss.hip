// loss.hip -- L1 + w (1 - SSIM) on one view, forward and backward.
//
// SSIM uses an 11x11 Gaussian window (std 1.5, normalised), zero padding and
// C1 = 0.01^2, C2 = 0.03^2; the window is separable, so the five local
// moments (mu_x, mu_y, E[x^2], E[y^2], E[xy]) take a horizontal and a
// vertical 11-tap pass.  The backward needs d SSIM / d (mu_x, E[x^2], E[xy])
// per pixel, convolved again with the (symmetric) window.  Block partial sums
// are combined by one block in a fixed order, so the scalar is reproducible.
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

// Horizontal pass of the five moment images.
__global__ __launch_bounds__(LS_THREADS) void k_ssim_h(const float* __restrict__ x, const float* __restrict__ y, int H, int W,
                                                       int64_t m, Win11 win, float* __restrict__ h5) {
    const int64_t i = (int64_t)blockIdx.x * LS_THREADS + threadIdx.x;
    if (i >= m) return;
    const int c = (int)(i % W);
    const int64_t rowbase = i - c;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        const int cc = c + k - 5;
        if (cc < 0 || cc >= W) continue;
        const float xv = x[rowbase + cc], yv = y[rowbase + cc], w = win.w[k];
        a0 = fmaf(w, xv, a0);
        a1 = fmaf(w, yv, a1);
        a2 = fmaf(w, xv * xv, a2);
        a3 = fmaf(w, yv * yv, a3);
        a4 = fmaf(w, xv * yv, a4);
    }
    h5[i] = a0; h5[m + i] = a1; h5[2 * m + i] = a2; h5[3 * m + i] = a3; h5[4 * m + i] = a4;
}

// Vertical pass, SSIM map, its partial derivatives, and block sums.
__global__ __launch_bounds__(LS_THREADS) void k_ssim_v(const float* __restrict__ x, const float* __restrict__ y,
                                                       const float* __restrict__ h5, int H, int W, int64_t m, Win11 win,
                                                       float* __restrict__ d3, float* __restrict__ part) {
    __shared__ float s_w[2][4];
    const int64_t i = (int64_t)blockIdx.x * LS_THREADS + threadIdx.x;
    float l1 = 0.f, ss = 0.f;
    if (i < m) {
        const int64_t HW = (int64_t)H * W;
        const int64_t plane = i / HW;
        const int64_t within = i - plane * HW;
        const int r = (int)(within / W), c = (int)(within % W);
        float mu_x = 0.f, mu_y = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            const int rr = r + k - 5;
            if (rr < 0 || rr >= H) continue;
            const int64_t j = plane * HW + (int64_t)rr * W + c;
            const float w = win.w[k];
            mu_x = fmaf(w, h5[j], mu_x);
            mu_y = fmaf(w, h5[m + j], mu_y);
            exx = fmaf(w, h5[2 * m + j], exx);
            eyy = fmaf(w, h5[3 * m + j], eyy);
            exy = fmaf(w, h5[4 * m + j], exy);
        }
        const float C1 = 1e-4f, C2 = 9e-4f;
        const float A1 = 2.f * mu_x * mu_y + C1;
        const float A2 = 2.f * (exy - mu_x * mu_y) + C2;
        const float B1 = mu_x * mu_x + mu_y * mu_y + C1;
        const float B2 = (exx - mu_x * mu_x) + (eyy - mu_y * mu_y) + C2;
        const float Nn = A1 * A2, Dd = B1 * B2;
        const float iD = 1.f / Dd;
        ss = Nn * iD;
        const float dN = 2.f * mu_y * A2 - 2.f * mu_y * A1;
        const float dD = 2.f * mu_x * B2 - 2.f * mu_x * B1;
        d3[i] = (dN * Dd - Nn * dD) * iD * iD;
        d3[m + i] = -Nn * B1 * iD * iD;
        d3[2 * m + i] = 2.f * A1 * iD;
        l1 = fabsf(x[i] - y[i]);
    }
    l1 = wave_sum(l1);
    ss = wave_sum(ss);
    if ((threadIdx.x & 63) == 0) { s_w[0][threadIdx.x >> 6] = l1; s_w[1][threadIdx.x >> 6] = ss; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (s_w[0][0] + s_w[0][1]) + (s_w[0][2] + s_w[0][3]);
        part[2 * blockIdx.x + 1] = (s_w[1][0] + s_w[1][1]) + (s_w[1][2] + s_w[1][3]);
    }
}

__global__ __launch_bounds__(LS_THREADS) void k_conv_h3(const float* __restrict__ d3, int W, int64_t m, Win11 win,
                                                        float* __restrict__ e3) {
    const int64_t i = (int64_t)blockIdx.x * LS_THREADS + threadIdx.x;
    if (i >= m) return;
    const int c = (int)(i % W);
    const int64_t rowbase = i - c;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        const int cc = c + k - 5;
        if (cc < 0 || cc >= W) continue;
        const float w = win.w[k];
        a0 = fmaf(w, d3[rowbase + cc], a0);
        a1 = fmaf(w, d3[m + rowbase + cc], a1);
        a2 = fmaf(w, d3[2 * m + rowbase + cc], a2);
    }
    e3[i] = a0; e3[m + i] = a1; e3[2 * m + i] = a2;
}

__global__ __launch_bounds__(LS_THREADS) void k_ssim_grad(const float* __restrict__ x, const float* __restrict__ y,
                                                          const float* __restrict__ e3, int H, int W, int64_t m, Win11 win,
                                                          float invN, float sc, float* __restrict__ dx) {
    const int64_t i = (int64_t)blockIdx.x * LS_THREADS + threadIdx.x;
    if (i >= m) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t plane = i / HW;
    const int64_t within = i - plane * HW;
    const int r = (int)(within / W), c = (int)(within % W);
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        const int rr = r + k - 5;
        if (rr < 0 || rr >= H) continue;
        const int64_t j = plane * HW + (int64_t)rr * W + c;
        const float w = win.w[k];
        g0 = fmaf(w, e3[j], g0);
        g1 = fmaf(w, e3[m + j], g1);
        g2 = fmaf(w, e3[2 * m + j], g2);
    }
    const float xv = x[i], yv = y[i];
    const float d = xv - yv;
    const float l1g = (float)((d > 0.f) - (d < 0.f)) * invN;
    dx[i] = l1g + sc * (g0 + 2.f * xv * g1 + yv * g2);
}

__global__ __launch_bounds__(LS_THREADS) void k_loss_final(const float* __restrict__ part, int nb, float invN, float w,
                                                           float* __restrict__ loss) {
    __shared__ double s_a[LS_THREADS], s_b[LS_THREADS];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nb; k += LS_THREADS) { a += part[2 * k]; b += part[2 * k + 1]; }
    s_a[threadIdx.x] = a;
    s_b[threadIdx.x] = b;
    __syncthreads();
    for (int st = LS_THREADS / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) { s_a[threadIdx.x] += s_a[threadIdx.x + st]; s_b[threadIdx.x] += s_b[threadIdx.x + st]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double l = s_a[0] * (double)invN;
        if (w != 0.f) l += (double)w * (1.0 - s_b[0] * (double)invN);
        *loss = (float)l;
    }
}

size_t loss_ws_bytes(int H, int W) {
    const int64_t m = 3 * (int64_t)H * W;
    const int64_t nb = (m + LS_THREADS - 1) / LS_THREADS;
    return (size_t)(5 + 3 + 3) * m * sizeof(float) + (size_t)2 * nb * sizeof(float) + 1024;
}

rgs_status loss_launch(const float* image, const float* target, int H, int W, float ssim_w, float* loss, float* dimg,
                       void* ws, hipStream_t s) {
    const int64_t m = 3 * (int64_t)H * W;
    const int64_t nb = (m + LS_THREADS - 1) / LS_THREADS;
    WsCarver c{reinterpret_cast<char*>(ws), 0, (size_t)-1};
    float* h5 = c.take<float>(5 * m);
    float* d3 = c.take<float>(3 * m);
    float* e3 = c.take<float>(3 * m);
    float* part = c.take<float>(2 * nb);
    const float invN = (float)(1.0 / (double)m);
    Win11 win;
    double g[11], gs = 0.0;
    for (int k = 0; k < 11; ++k) { g[k] = exp(-((k - 5) * (k - 5)) / (2.0 * 1.5 * 1.5)); gs += g[k]; }
    for (int k = 0; k < 11; ++k) win.w[k] = (float)(g[k] / gs);
    const dim3 grid((unsigned)nb);
    if (ssim_w == 0.f) {
        hipLaunchKernelGGL(k_l1_only, grid, dim3(LS_THREADS), 0, s, image, target, m, invN, dimg, part);
    } else {
        hipLaunchKernelGGL(k_ssim_h, grid, dim3(LS_THREADS), 0, s, image, target, H, W, m, win, h5);
        hipLaunchKernelGGL(k_ssim_v, grid, dim3(LS_THREADS), 0, s, image, target, h5, H, W, m, win, d3, part);
        hipLaunchKernelGGL(k_conv_h3, grid, dim3(LS_THREADS), 0, s, d3, W, m, win, e3);
        hipLaunchKernelGGL(k_ssim_grad, grid, dim3(LS_THREADS), 0, s, image, target, e3, H, W, m, win, invN,
                           -ssim_w * invN, dimg);
    }
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(LS_THREADS), 0, s, part, (int)nb, invN, ssim_w, loss);
    return launch_check();
}

}  // namespace rgs
