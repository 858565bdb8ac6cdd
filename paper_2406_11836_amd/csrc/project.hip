// project.hip -- per-(view, Gaussian) projection, SH colour and cell sets
// (RetinaGS Sec. 3.1, with the cell sets that Eq. 6 needs), and its backward.
//
// One thread per Gaussian loops over the views, so the parameters (up to
// 59 floats) are read from HBM once per batch of views; loads and the
// structure-of-arrays stores are coalesced.  The decision path (activations,
// covariance, EWA, conic, screen mean, tau, rectangle, cell set) is a fixed
// sequence of IEEE operations with no contraction: the covariance chain in
// fp64 (+, -, *, /, sqrt), rounded once to fp32, then fp32 tests; its
// transcendentals are computed in fp64 and rounded once, so the integer
// outputs (rectangle, cell set, count) are reproducible on any IEEE machine.
#include "common.hpp"

namespace rgs {

static constexpr int PJ_THREADS = 256;

// Real SH basis (degree <= 3) in polynomial form on the unit sphere, with the
// Condon-Shortley phase; index j = l^2 + l + m.
__device__ __forceinline__ void sh_eval(int D, float x, float y, float z, float* Y) {
    Y[0] = 0.28209479177387814f;
    if (D < 1) return;
    Y[1] = -0.4886025119029199f * y;
    Y[2] = 0.4886025119029199f * z;
    Y[3] = -0.4886025119029199f * x;
    if (D < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, yz = y * z, xz = x * z;
    Y[4] = 1.0925484305920792f * xy;
    Y[5] = -1.0925484305920792f * yz;
    Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * xz;
    Y[8] = 0.5462742152960396f * (xx - yy);
    if (D < 3) return;
    Y[9] = -0.5900435899266435f * y * (3.0f * xx - yy);
    Y[10] = 2.890611442640554f * xy * z;
    Y[11] = -0.4570457994644658f * y * (4.0f * zz - xx - yy);
    Y[12] = 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -0.4570457994644658f * x * (4.0f * zz - xx - yy);
    Y[14] = 1.445305721320277f * z * (xx - yy);
    Y[15] = -0.5900435899266435f * x * (xx - 3.0f * yy);
}

// sum_j h_j grad Y_j (x, y, z) for the polynomial forms above, accumulated
// into g without materialising the 16 gradients.
__device__ __forceinline__ void sh_grad_dot(int D, float x, float y, float z, const float* h, float g[3]) {
    if (D < 1) return;
    const float c1 = 0.4886025119029199f;
    g[1] += -c1 * h[1];
    g[2] += c1 * h[2];
    g[0] += -c1 * h[3];
    if (D < 2) return;
    const float a = 1.0925484305920792f, b = 0.31539156525252005f, c = 0.5462742152960396f;
    g[0] += a * y * h[4]; g[1] += a * x * h[4];
    g[1] += -a * z * h[5]; g[2] += -a * y * h[5];
    g[0] += -2.f * b * x * h[6]; g[1] += -2.f * b * y * h[6]; g[2] += 4.f * b * z * h[6];
    g[0] += -a * z * h[7]; g[2] += -a * x * h[7];
    g[0] += 2.f * c * x * h[8]; g[1] += -2.f * c * y * h[8];
    if (D < 3) return;
    const float k0 = -0.5900435899266435f, k1 = 2.890611442640554f, k2 = -0.4570457994644658f,
                k3 = 0.3731763325901154f, k5 = 1.445305721320277f;
    const float xx = x * x, yy = y * y, zz = z * z;
    // y (3x^2 - y^2)
    g[0] += k0 * 6.f * x * y * h[9]; g[1] += k0 * (3.f * xx - 3.f * yy) * h[9];
    // x y z
    g[0] += k1 * y * z * h[10]; g[1] += k1 * x * z * h[10]; g[2] += k1 * x * y * h[10];
    // y (4z^2 - x^2 - y^2)
    g[0] += k2 * (-2.f * x * y) * h[11]; g[1] += k2 * (4.f * zz - xx - 3.f * yy) * h[11]; g[2] += k2 * 8.f * y * z * h[11];
    // z (2z^2 - 3x^2 - 3y^2)
    g[0] += k3 * (-6.f * x * z) * h[12]; g[1] += k3 * (-6.f * y * z) * h[12];
    g[2] += k3 * (6.f * zz - 3.f * xx - 3.f * yy) * h[12];
    // x (4z^2 - x^2 - y^2)
    g[0] += k2 * (4.f * zz - 3.f * xx - yy) * h[13]; g[1] += k2 * (-2.f * x * y) * h[13]; g[2] += k2 * 8.f * x * z * h[13];
    // z (x^2 - y^2)
    g[0] += k5 * 2.f * x * z * h[14]; g[1] += k5 * (-2.f * y * z) * h[14]; g[2] += k5 * (xx - yy) * h[14];
    // x (x^2 - 3y^2)
    g[0] += k0 * (3.f * xx - 3.f * yy) * h[15]; g[1] += k0 * (-6.f * x * y) * h[15];
}

struct Proj32 {
    float mx, my, ca, k, e, tau, z, alpha, s00, s11, rk;
    bool vis;
};

// The decision path in two parts: the view-independent activations and 3D
// covariance (once per Gaussian), then the per-view projection.  From the
// quaternion to the inverse of the screen covariance everything runs in
// fp64 (+, -, *, /, sqrt: correctly rounded, so the bits match any IEEE
// machine) and is rounded once to fp32, so that a nearly singular screen
// covariance (a needle-like footprint) keeps an accurate inverse.  The
// scale and opacity activations are fp64 transcendentals rounded to fp32.
struct Pre32 {
    float alpha, tau;
    double S[6];  // 3D covariance: 00, 01, 02, 11, 12, 22 (the product is exactly symmetric)
    bool ok;      // quaternion non-zero
};

__device__ __forceinline__ void pre32(float ls0, float ls1, float ls2, float qw32, float qx32, float qy32, float qz32,
                                      float logit, Pre32& q) {
    q.ok = false;
    const float s0 = (float)exp((double)ls0), s1 = (float)exp((double)ls1), s2 = (float)exp((double)ls2);
    q.alpha = (float)(1.0 / (1.0 + exp(-(double)logit)));
    q.tau = fminf(9.0f, (float)(2.0 * log(255.0 * (double)q.alpha)));
    const double qw = qw32, qx = qx32, qy = qy32, qz = qz32;
    const double qq = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (!(qq > 0.0)) return;
    const double qn = sqrt(qq);
    const double w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
    double r[3][3];
    r[0][0] = 1.0 - 2.0 * (y * y + z * z);
    r[0][1] = 2.0 * (x * y - w * z);
    r[0][2] = 2.0 * (x * z + w * y);
    r[1][0] = 2.0 * (x * y + w * z);
    r[1][1] = 1.0 - 2.0 * (x * x + z * z);
    r[1][2] = 2.0 * (y * z - w * x);
    r[2][0] = 2.0 * (x * z - w * y);
    r[2][1] = 2.0 * (y * z + w * x);
    r[2][2] = 1.0 - 2.0 * (x * x + y * y);
    const double sc[3] = {s0, s1, s2};
    double M[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) M[a][b] = r[a][b] * sc[b];
    auto cov = [&](int a, int b) { return (M[a][0] * M[b][0] + M[a][1] * M[b][1]) + M[a][2] * M[b][2]; };
    q.S[0] = cov(0, 0);
    q.S[1] = cov(0, 1);
    q.S[2] = cov(0, 2);
    q.S[3] = cov(1, 1);
    q.S[4] = cov(1, 2);
    q.S[5] = cov(2, 2);
    q.ok = true;
}

// Per view: camera transform, EWA (Jacobian clamped to 1.3x the half field of
// view), screen covariance + 0.3 I and its inverse in the factored form
// d^2 = ca (dx + k dy)^2 + e dy^2 with ca = s11/det, k = -s01/s11, e = 1/s11.
__device__ __forceinline__ void proj32(float mu0f, float mu1f, float mu2f, const Pre32& q, const ViewParams& V,
                                       Proj32& p) {
    p.vis = false;
    if (!q.ok) return;
    const double S[3][3] = {{q.S[0], q.S[1], q.S[2]}, {q.S[1], q.S[3], q.S[4]}, {q.S[2], q.S[4], q.S[5]}};
    const double mu0 = mu0f, mu1 = mu1f, mu2 = mu2f;
    double R[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = V.R[k];
    double tc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) tc[a] = ((R[3 * a] * mu0 + R[3 * a + 1] * mu1) + R[3 * a + 2] * mu2) + (double)V.t[a];
    const double zc = tc[2];
    if (!(zc > (double)V.znear)) return;
    const double fx = V.fx, fy = V.fy, gx = V.gx, gy = V.gy;
    const double xz = tc[0] / zc, yz = tc[1] / zc;
    const double xg = fmin(fmax(xz, -gx), gx) * zc;
    const double yg = fmin(fmax(yz, -gy), gy) * zc;
    const double zz = zc * zc;
    const double J00 = fx / zc, J02 = -(fx * xg) / zz, J11 = fy / zc, J12 = -(fy * yg) / zz;
    double T[2][3], U[2][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        T[0][b] = J00 * R[b] + J02 * R[6 + b];
        T[1][b] = J11 * R[3 + b] + J12 * R[6 + b];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) U[a][b] = (T[a][0] * S[0][b] + T[a][1] * S[1][b]) + T[a][2] * S[2][b];
    const double s00 = ((U[0][0] * T[0][0] + U[0][1] * T[0][1]) + U[0][2] * T[0][2]) + 0.3;
    const double s01 = (U[0][0] * T[1][0] + U[0][1] * T[1][1]) + U[0][2] * T[1][2];
    const double s11 = ((U[1][0] * T[1][0] + U[1][1] * T[1][1]) + U[1][2] * T[1][2]) + 0.3;
    const double det = s00 * s11 - s01 * s01;
    if (!(det > 0.0)) return;
    p.ca = (float)(s11 / det);
    p.k = (float)(-s01 / s11);
    p.e = (float)(1.0 / s11);
    p.rk = sqrtf(1.0f + (p.k * p.k) * (p.ca / p.e));
    p.mx = (float)(fx * xz + (double)V.cx);
    p.my = (float)(fy * yz + (double)V.cy);
    p.z = (float)zc;
    p.alpha = q.alpha;
    p.s00 = (float)s00;
    p.s11 = (float)s11;
    p.tau = q.tau;
    if (!(q.tau >= 0.0f)) return;
    if (!(isfinite(p.mx) && isfinite(p.my))) return;
    p.vis = true;
}

// Sample-pixel rectangle of the footprint d^2 <= tau.  Its half-widths
// sqrt(tau s00), sqrt(tau s11) are padded by 1e-3 px, a relative 1e-5 and a
// relative 2^-20 rk: the fp32 per-pixel test rounds u = dx + k dy with an
// absolute error up to about 2^-24 (|dx| + |k dy|), which near the long tip of
// an elongated footprint moves ca u^2 by up to about 2^-21 tau rk (ca s00 =
// rk^2); the ellipse of the rounded (ca, k, e) is within a few 2^-24 of s00.
__device__ __forceinline__ bool rect32(const Proj32& p, const ViewParams& V, int r[4]) {
    const float pad = 1.00001f + 0x1p-20f * p.rk;
    const float ex = sqrtf(p.tau * p.s00) * pad + 1e-3f;
    const float ey = sqrtf(p.tau * p.s11) * pad + 1e-3f;
    const float xlo = fmaxf(ceilf((p.mx - ex) - 0.5f), 0.0f);
    const float xhi = fminf(floorf((p.mx + ex) - 0.5f), (float)(V.W - 1));
    const float ylo = fmaxf(ceilf((p.my - ey) - 0.5f), 0.0f);
    const float yhi = fminf(floorf((p.my + ey) - 0.5f), (float)(V.H - 1));
    if (!(xlo <= xhi) || !(ylo <= yhi)) return false;
    r[0] = (int)xlo; r[1] = (int)xhi; r[2] = (int)ylo; r[3] = (int)yhi;
    return true;
}

// KD leaves met by the padded box of the crossing points x(p) = o + z D(p)
// over the rectangle's four corner samples (x(p) is affine in the pixel).
__device__ __forceinline__ uint64_t cellset32(const Proj32& p, const int r[4], const ViewParams& V, int L,
                                              const float* __restrict__ split) {
    if (L == 0) return 1ull;
    const float u0 = (float)r[0] + 0.5f, u1 = (float)r[1] + 0.5f;
    const float v0 = (float)r[2] + 0.5f, v1 = (float)r[3] + 0.5f;
    const float dx[2] = {(u0 - V.cx) / V.fx, (u1 - V.cx) / V.fx};
    const float dy[2] = {(v0 - V.cy) / V.fy, (v1 - V.cy) / V.fy};
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float oa = V.o[a];
        float mn = INFINITY, mxv = -INFINITY;
#pragma unroll
        for (int jy = 0; jy < 2; ++jy)
#pragma unroll
            for (int jx = 0; jx < 2; ++jx) {
                const float Da = (V.R[a] * dx[jx] + V.R[3 + a] * dy[jy]) + V.R[6 + a];
                const float xa = fmaf(p.z, Da, oa);
                mn = fminf(mn, xa);
                mxv = fmaxf(mxv, xa);
            }
        const float mdx = fmaxf(fabsf(dx[0]), fabsf(dx[1])), mdy = fmaxf(fabsf(dy[0]), fabsf(dy[1]));
        const float pad = 0x1p-16f * (fabsf(oa) + p.z * ((fabsf(V.R[a]) * mdx + fabsf(V.R[3 + a]) * mdy) + fabsf(V.R[6 + a])));
        lo[a] = mn - pad;
        hi[a] = mxv + pad;
    }
    // iterative traversal of the heap-ordered tree
    uint64_t mask = 0;
    int stack[RGS_MAX_L + 2];
    int sp = 0;
    stack[sp++] = 0;
    const int K = 1 << L;
    while (sp > 0) {
        const int nd = stack[--sp];
        if (nd >= K - 1) { mask |= 1ull << (nd - (K - 1)); continue; }
        int depth = 31 - __clz(nd + 1);
        const int a = depth % 3;
        const float s = split[nd];
        // push right first so that left is visited first (order is irrelevant for the mask)
        if (hi[a] >= s) stack[sp++] = 2 * nd + 2;
        if (lo[a] < s) stack[sp++] = 2 * nd + 1;
    }
    return mask;
}

// Conservative fp32 screen test ahead of the fp64 chain: false only where
// the chain would find z <= z_near or an empty rectangle, so skipping those
// pairs changes no output.  Bounds: tau <= 9; s00 <= (|J00| + |J02|)^2 smax^2
// + 0.3 (camera rotation rows are unit vectors, the 3D covariance's largest
// eigenvalue is smax^2), s11 alike; the rectangle pad's 2^-20 rk sqrt(tau s00)
// term is below 2^-17 (Bx + By) since det >= 0.3 max(s00, s11); then 1%, 2 px
// and 1e-5 |mx| for the fp32 evaluation.  The depth test allows the fp32
// camera transform's rounding (< 1e-6 of the sum of its terms).
__device__ __forceinline__ bool screen_may_hit(float mu0, float mu1, float mu2, float smax, const ViewParams& V) {
    const float t0 = ((V.R[0] * mu0 + V.R[1] * mu1) + V.R[2] * mu2) + V.t[0];
    const float t1 = ((V.R[3] * mu0 + V.R[4] * mu1) + V.R[5] * mu2) + V.t[1];
    const float t2 = ((V.R[6] * mu0 + V.R[7] * mu1) + V.R[8] * mu2) + V.t[2];
    const float az = ((fabsf(V.R[6] * mu0) + fabsf(V.R[7] * mu1)) + fabsf(V.R[8] * mu2)) + fabsf(V.t[2]);
    if (t2 + 1e-6f * az < V.znear) return false;
    const float iz = 1.0f / t2;
    const float xz = t0 * iz, yz = t1 * iz;
    const float jx = V.fx * iz * (1.0f + fabsf(fminf(fmaxf(xz, -V.gx), V.gx)));
    const float jy = V.fy * iz * (1.0f + fabsf(fminf(fmaxf(yz, -V.gy), V.gy)));
    const float s2 = smax * smax;
    const float Bx = jx * jx * s2 + 0.3f, By = jy * jy * s2 + 0.3f;
    const float mx = V.fx * xz + V.cx, my = V.fy * yz + V.cy;
    const float ex = 3.03f * sqrtf(Bx) + 0x1p-17f * (Bx + By) + 2.0f + 1e-5f * fabsf(mx);
    const float ey = 3.03f * sqrtf(By) + 0x1p-17f * (Bx + By) + 2.0f + 1e-5f * fabsf(my);
    // NaN compares false: such a pair is left to the exact chain
    return !(mx + ex < 0.0f || mx - ex > (float)V.W || my + ey < 0.0f || my - ey > (float)V.H);
}

// cells (which Gaussians each cell renders): RGS_CELLS_EXACT, the KD leaves
// the footprint's crossing points can reach; RGS_CELLS_PAPER_SUBSETS, those
// leaves whose subset N_k holds the Gaussian (own_mask); RGS_CELLS_EXCLUSIVE,
// the leaf of the centre only, with no indicator test in the render (flag
// bit 0 set: the render takes every pixel of the footprint for that cell).
template <int D>
__global__ __launch_bounds__(PJ_THREADS, 3) void k_project(rgs_gaussians g, const ViewTable* __restrict__ vt,
                                                        const float* __restrict__ split,
                                                        const int32_t* __restrict__ center_cell, int cells,
                                                        const uint32_t* __restrict__ own_mask, rgs_projected out) {
    const int64_t n = g.n;
    const int64_t i = (int64_t)blockIdx.x * PJ_THREADS + threadIdx.x;
    if (i >= n) return;
    constexpr int nc = (D + 1) * (D + 1);
    // cell culling: views that cannot see this Gaussian's cell get count 0,
    // and the parameters are not read unless some view needs them
    uint32_t view_ok = (1u << vt->n_views) - 1u;
    if (vt->culled) {
        const int cell = center_cell[i];
        view_ok = 0u;
        for (int v = 0; v < vt->n_views; ++v)
            if ((vt->v[v].cell_visible >> cell) & 1ull) view_ok |= 1u << v;
        for (int v = 0; v < vt->n_views; ++v)
            if (!((view_ok >> v) & 1u)) out.count[(int64_t)v * n + i] = 0u;
        if (view_ok == 0u) return;
    }
    const float mu0 = g.means[i], mu1 = g.means[n + i], mu2 = g.means[2 * n + i];
    const float ls0 = g.log_scales[i], ls1 = g.log_scales[n + i], ls2 = g.log_scales[2 * n + i];
    // pairs that cannot reach their image skip the fp64 chain (count 0, as the chain would give)
    const float smax = expf(fmaxf(fmaxf(ls0, ls1), ls2)) * 1.001f;
    uint32_t scr = 0u;  // views whose screen test passes
    for (int v = 0; v < vt->n_views; ++v)
        if (screen_may_hit(mu0, mu1, mu2, smax, vt->v[v])) scr |= 1u << v;
    if ((view_ok & scr) == 0u) {
        for (int v = 0; v < vt->n_views; ++v)
            if ((view_ok >> v) & 1u) out.count[(int64_t)v * n + i] = 0u;
        return;
    }
    const float qw = g.quats[i], qx = g.quats[n + i], qy = g.quats[2 * n + i], qz = g.quats[3 * n + i];
    const float logit = g.opacity[i];
    Pre32 pre;
    pre32(ls0, ls1, ls2, qw, qx, qy, qz, logit, pre);
    const int L = vt->L;
    for (int v = 0; v < vt->n_views; ++v) {
        if (!((view_ok >> v) & 1u)) continue;
        const ViewParams& V = vt->v[v];
        const int64_t src = (int64_t)v * n + i;
        Proj32 p;
        p.vis = false;
        if ((scr >> v) & 1u) proj32(mu0, mu1, mu2, pre, V, p);
        int r[4] = {0, 0, 0, 0};
        bool ok = p.vis && rect32(p, V, r);
        float4* rec = reinterpret_cast<float4*>(out.rec + src * RGS_REC_FLOATS);
        if (!ok) {
            // only the count is defined for a culled pair
            out.count[src] = 0u;
            continue;
        }
        const uint64_t reach = cellset32(p, r, V, L, split);
        uint64_t mask = reach;
        if (cells == RGS_CELLS_PAPER_SUBSETS) {
            const int Wm = ((1 << L) + 31) >> 5;
            uint64_t own = own_mask[i * Wm];
            if (Wm > 1) own |= (uint64_t)own_mask[i * Wm + 1] << 32;
            mask &= own;
        } else if (cells == RGS_CELLS_EXCLUSIVE) {
            mask = 1ull << center_cell[i];
        }
        if (mask == 0ull) {
            out.count[src] = 0u;
            continue;
        }
        // tiles per cell: the row spans of the footprint inside the rectangle
        SpanPre sp;
        span_pre(p.mx, p.my, p.ca, p.k, p.e, p.tau, sp);
        const int tx0 = r[0] >> 4, ty0 = r[2] >> 4, ty1 = r[3] >> 4;
        const bool small = ty1 - ty0 < 8 && (r[1] >> 4) - tx0 < 15;
        uint64_t desc = small ? 0ull : RGS_NO_SPANS;
        uint32_t nt = 0;
#pragma unroll 1
        for (int ty = ty0; ty <= ty1; ++ty) {
            const int2 cs = row_span(sp, r[0], r[1], r[2], r[3], ty);
            const uint32_t len = cs.x <= cs.y ? (uint32_t)(cs.y - cs.x + 1) : 0u;
            nt += len;
            if (small && len) desc |= (uint64_t)((len << 4) | (uint32_t)(cs.x - tx0)) << (8 * (ty - ty0));
        }
        const uint32_t cnt = (uint32_t)__popcll(mask) * nt;
        out.count[src] = cnt;
        out.depth[src] = p.z;
        const uint32_t rx = ((uint32_t)(uint16_t)r[0]) | ((uint32_t)(uint16_t)r[1] << 16);
        const uint32_t ry = ((uint32_t)(uint16_t)r[2]) | ((uint32_t)(uint16_t)r[3] << 16);
        {  // the binning record, one 32-byte line for the emission
            uint4* bp = reinterpret_cast<uint4*>(out.bin) + 2 * src;
            bp[0] = make_uint4(rx, ry, (uint32_t)desc, (uint32_t)(desc >> 32));
            bp[1] = make_uint4((uint32_t)mask, (uint32_t)(mask >> 32), cnt, nt);
        }
        // colour from the view direction (value path)
        float dx = mu0 - V.o[0], dy = mu1 - V.o[1], dz = mu2 - V.o[2];
        const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
        dx *= inv; dy *= inv; dz *= inv;
        float Y[16];
        sh_eval(D, dx, dy, dz, Y);
        // SH coefficients are streamed from memory (only views that keep the
        // Gaussian read them; a later view hits the cache), not held in
        // registers across the view loop, so that more waves fit per SIMD
        float col[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int l = 0; l <= D; ++l) {
            // one band at a time: the empty asm keeps the compiler from
            // hoisting every band's loads (and their registers) up front
            asm volatile("" ::: "memory");
#pragma unroll
            for (int j = l * l; j < (l + 1) * (l + 1); ++j)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) col[ch] = fmaf(g.sh[(int64_t)(3 * j + ch) * n + i], Y[j], col[ch]);
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) col[ch] = fmaxf(col[ch], 0.0f);
        // bit 0: no indicator test needed (every crossing point lies in the one cell, or exclusive cells)
        const uint32_t flags = (__popcll(reach) == 1 || cells == RGS_CELLS_EXCLUSIVE) ? 1u : 0u;
        rec[0] = make_float4(p.mx, p.my, p.ca, p.k);
        rec[1] = make_float4(p.e, p.alpha, p.tau, p.z);
        rec[2] = make_float4(col[0], col[1], col[2], __uint_as_float(flags));
        // the rectangle (render kernels) and the row-span descriptor (emission)
        rec[3] = make_float4(__uint_as_float(rx), __uint_as_float(ry), __uint_as_float((uint32_t)desc),
                             __uint_as_float((uint32_t)(desc >> 32)));
    }
}

rgs_status project_launch(const rgs_gaussians* g, const ViewTable* vt, const float* split, const int32_t* center_cell,
                          int cells, const uint32_t* own_mask, const rgs_projected* out, hipStream_t s) {
    if (g->n <= 0) return RGS_OK;
    const unsigned grid = (unsigned)((g->n + PJ_THREADS - 1) / PJ_THREADS);
    switch (g->sh_degree) {
        case 0: hipLaunchKernelGGL(k_project<0>, dim3(grid), dim3(PJ_THREADS), 0, s, *g, vt, split, center_cell, cells,
                                   own_mask, *out); break;
        case 1: hipLaunchKernelGGL(k_project<1>, dim3(grid), dim3(PJ_THREADS), 0, s, *g, vt, split, center_cell, cells,
                                   own_mask, *out); break;
        case 2: hipLaunchKernelGGL(k_project<2>, dim3(grid), dim3(PJ_THREADS), 0, s, *g, vt, split, center_cell, cells,
                                   own_mask, *out); break;
        default: hipLaunchKernelGGL(k_project<3>, dim3(grid), dim3(PJ_THREADS), 0, s, *g, vt, split, center_cell, cells,
                                    own_mask, *out); break;
    }
    return launch_check();
}

// ------------------------------------------------------------------ backward
// Two kernels, both a thread per Gaussian looping over the views that keep
// it, summing in registers and writing each gradient once: the geometric
// part (rotation, 3D covariance, EWA, screen covariance and its inverse, and
// their adjoints, plus opacity) runs in fp64 like the forward's decision
// chain, since for a needle-like footprint the inverse of the screen
// covariance and the conic-to-covariance adjoint -C G C lose accuracy in
// proportion to s00 s11 / det in fp32; the SH colour part (fp32) runs after
// it and adds its share of the mean gradient (the view direction).  Split,
// each kernel keeps fewer registers live than one kernel doing both.
__global__ __launch_bounds__(PJ_THREADS) void k_project_bwd_geo(const float* __restrict__ dproj, rgs_gaussians g,
                                                                const uint32_t* __restrict__ count,
                                                                const ViewTable* __restrict__ vt,
                                                                rgs_gaussians_grad out) {
    const int64_t n = g.n;
    const int64_t i = (int64_t)blockIdx.x * PJ_THREADS + threadIdx.x;
    if (i >= n) return;
    const int64_t VN = (int64_t)vt->n_views * n;
    const double mu[3] = {g.means[i], g.means[n + i], g.means[2 * n + i]};
    const float ls[3] = {g.log_scales[i], g.log_scales[n + i], g.log_scales[2 * n + i]};
    const double q4[4] = {g.quats[i], g.quats[n + i], g.quats[2 * n + i], g.quats[3 * n + i]};
    const float logit = g.opacity[i];
    double gmu[3] = {0.0, 0.0, 0.0};
    float gop = 0.f;

    // view-independent quantities (the forward's values)
    const double s[3] = {(float)exp((double)ls[0]), (float)exp((double)ls[1]), (float)exp((double)ls[2])};
    const float alpha = (float)(1.0 / (1.0 + exp(-(double)logit)));
    const double qn = sqrt(((q4[0] * q4[0] + q4[1] * q4[1]) + q4[2] * q4[2]) + q4[3] * q4[3]);
    const double w = q4[0] / qn, x = q4[1] / qn, y = q4[2] / qn, z = q4[3] / qn;
    const double Rq[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                             {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                             {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
    double S[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            S[a][b] = ((Rq[a][0] * s[0]) * (Rq[b][0] * s[0]) + (Rq[a][1] * s[1]) * (Rq[b][1] * s[1])) +
                      (Rq[a][2] * s[2]) * (Rq[b][2] * s[2]);
    double GS[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    bool any = false;

    for (int v = 0; v < vt->n_views; ++v) {
        const int64_t src = (int64_t)v * n + i;
        if (count[src] == 0u) continue;
        any = true;
        const ViewParams& V = vt->v[v];
        float gd[6];
        for (int c = 0; c < 6; ++c) gd[c] = dproj[c * VN + src];
        double R[9];
        for (int k = 0; k < 9; ++k) R[k] = V.R[k];
        const double fx = V.fx, fy = V.fy, gx = V.gx, gy = V.gy;
        double t[3];
        for (int a = 0; a < 3; ++a) t[a] = ((R[3 * a] * mu[0] + R[3 * a + 1] * mu[1]) + R[3 * a + 2] * mu[2]) + (double)V.t[a];
        const double zc = t[2];
        const double xz = t[0] / zc, yz = t[1] / zc;
        const int clx = (xz < -gx) ? -1 : (xz > gx ? 1 : 0);
        const int cly = (yz < -gy) ? -1 : (yz > gy ? 1 : 0);
        const double xg = clx ? (double)clx * gx * zc : t[0];
        const double yg = cly ? (double)cly * gy * zc : t[1];
        const double iz = 1.0 / zc, iz2 = iz * iz;
        const double J00 = fx * iz, J02 = -fx * xg * iz2, J11 = fy * iz, J12 = -fy * yg * iz2;
        double T[2][3];
        for (int b = 0; b < 3; ++b) {
            T[0][b] = J00 * R[b] + J02 * R[6 + b];
            T[1][b] = J11 * R[3 + b] + J12 * R[6 + b];
        }
        double TS[2][3];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) TS[a][b] = T[a][0] * S[0][b] + T[a][1] * S[1][b] + T[a][2] * S[2][b];
        const double a00 = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2] + 0.3;
        const double a01 = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
        const double a11 = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2] + 0.3;
        const double idet = 1.0 / (a00 * a11 - a01 * a01);
        const double Cn[2][2] = {{a11 * idet, -a01 * idet}, {-a01 * idet, a00 * idet}};
        // conic -> screen covariance: G_S2 = -Cn G_C Cn, G_C = [[ga, gb/2], [gb/2, gc]]
        const double GC[2][2] = {{gd[2], 0.5 * gd[3]}, {0.5 * gd[3], gd[4]}};
        double tmp[2][2], GS2[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) tmp[a][b] = Cn[a][0] * GC[0][b] + Cn[a][1] * GC[1][b];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) GS2[a][b] = -(tmp[a][0] * Cn[0][b] + tmp[a][1] * Cn[1][b]);
        // S2 = T S T^T: G_T = 2 G_S2 T S ; G_S += T^T G_S2 T
        double GT[2][3];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) GT[a][b] = 2.0 * (GS2[a][0] * TS[0][b] + GS2[a][1] * TS[1][b]);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                GS[a][b] += T[0][a] * (GS2[0][0] * T[0][b] + GS2[0][1] * T[1][b]) +
                            T[1][a] * (GS2[1][0] * T[0][b] + GS2[1][1] * T[1][b]);
        // T = J R: G_J = G_T R^T (only the four non-zero entries of J vary)
        double GJ00 = 0.0, GJ02 = 0.0, GJ11 = 0.0, GJ12 = 0.0;
        for (int b = 0; b < 3; ++b) {
            GJ00 += GT[0][b] * R[b];
            GJ02 += GT[0][b] * R[6 + b];
            GJ11 += GT[1][b] * R[3 + b];
            GJ12 += GT[1][b] * R[6 + b];
        }
        double gt[3] = {0.0, 0.0, 0.0};
        const double iz3 = iz2 * iz;
        gt[2] += -GJ00 * fx * iz2 - GJ11 * fy * iz2;
        gt[2] += GJ02 * 2.0 * fx * xg * iz3 + GJ12 * 2.0 * fy * yg * iz3;
        const double gxg = -GJ02 * fx * iz2, gyg = -GJ12 * fy * iz2;
        if (clx) gt[2] += gxg * (double)clx * gx; else gt[0] += gxg;
        if (cly) gt[2] += gyg * (double)cly * gy; else gt[1] += gyg;
        // screen mean mx = fx t.x / z + cx
        gt[0] += gd[0] * fx * iz;
        gt[2] += -gd[0] * fx * t[0] * iz2;
        gt[1] += gd[1] * fy * iz;
        gt[2] += -gd[1] * fy * t[1] * iz2;
        for (int a = 0; a < 3; ++a) gmu[a] += R[a] * gt[0] + R[3 + a] * gt[1] + R[6 + a] * gt[2];
        gop += gd[5] * alpha * (1.f - alpha);
    }
    double gls[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0};
    if (any) {
        // S = M M^T with M = Rq diag(s): G_M = 2 G_S M
        double GR[3][3];
        for (int b = 0; b < 3; ++b) {
            double gs = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double GMab = 2.0 * ((GS[a][0] * (Rq[0][b] * s[b]) + GS[a][1] * (Rq[1][b] * s[b])) +
                                           GS[a][2] * (Rq[2][b] * s[b]));
                gs += GMab * Rq[a][b];
                GR[a][b] = GMab * s[b];
            }
            gls[b] = gs * s[b];
        }
        double gw = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        gy += GR[0][0] * (-4.0 * y); gz += GR[0][0] * (-4.0 * z);
        gw += GR[0][1] * (-2.0 * z); gx += GR[0][1] * (2.0 * y); gy += GR[0][1] * (2.0 * x); gz += GR[0][1] * (-2.0 * w);
        gw += GR[0][2] * (2.0 * y); gx += GR[0][2] * (2.0 * z); gy += GR[0][2] * (2.0 * w); gz += GR[0][2] * (2.0 * x);
        gw += GR[1][0] * (2.0 * z); gx += GR[1][0] * (2.0 * y); gy += GR[1][0] * (2.0 * x); gz += GR[1][0] * (2.0 * w);
        gx += GR[1][1] * (-4.0 * x); gz += GR[1][1] * (-4.0 * z);
        gw += GR[1][2] * (-2.0 * x); gx += GR[1][2] * (-2.0 * w); gy += GR[1][2] * (2.0 * z); gz += GR[1][2] * (2.0 * y);
        gw += GR[2][0] * (-2.0 * y); gx += GR[2][0] * (2.0 * z); gy += GR[2][0] * (-2.0 * w); gz += GR[2][0] * (2.0 * x);
        gw += GR[2][1] * (2.0 * x); gx += GR[2][1] * (2.0 * w); gy += GR[2][1] * (2.0 * z); gz += GR[2][1] * (2.0 * y);
        gx += GR[2][2] * (-4.0 * x); gy += GR[2][2] * (-4.0 * y);
        const double qh[4] = {w, x, y, z}, gqh[4] = {gw, gx, gy, gz};
        const double dot = qh[0] * gqh[0] + qh[1] * gqh[1] + qh[2] * gqh[2] + qh[3] * gqh[3];
        for (int a = 0; a < 4; ++a) gq[a] = (gqh[a] - qh[a] * dot) / qn;
    }
    for (int a = 0; a < 3; ++a) { out.means[a * n + i] = (float)gmu[a]; out.log_scales[a * n + i] = (float)gls[a]; }
    for (int a = 0; a < 4; ++a) out.quats[a * n + i] = (float)gq[a];
    out.opacity[i] = gop;
}

// SH colour part: gradients of the SH coefficients, and the view-direction
// share of the mean gradient added to what the geometric kernel wrote.
template <int D>
__global__ __launch_bounds__(PJ_THREADS) void k_project_bwd_sh(const float* __restrict__ dproj, rgs_gaussians g,
                                                               const uint32_t* __restrict__ count,
                                                               const ViewTable* __restrict__ vt,
                                                               rgs_gaussians_grad out) {
    const int64_t n = g.n;
    const int64_t i = (int64_t)blockIdx.x * PJ_THREADS + threadIdx.x;
    if (i >= n) return;
    constexpr int nc = (D + 1) * (D + 1);
    const int64_t VN = (int64_t)vt->n_views * n;
    const float mu[3] = {g.means[i], g.means[n + i], g.means[2 * n + i]};
    float gmu[3] = {0.f, 0.f, 0.f};
    float gsh[3 * nc], fsh[3 * nc];
#pragma unroll
    for (int k = 0; k < 3 * nc; ++k) {
        gsh[k] = 0.f;
        fsh[k] = g.sh[(int64_t)k * n + i];
    }
    bool any = false;
    for (int v = 0; v < vt->n_views; ++v) {
        const int64_t src = (int64_t)v * n + i;
        if (count[src] == 0u) continue;
        any = true;
        const ViewParams& V = vt->v[v];
        const float gd6 = dproj[6 * VN + src], gd7 = dproj[7 * VN + src], gd8 = dproj[8 * VN + src];
        float d[3] = {mu[0] - V.o[0], mu[1] - V.o[1], mu[2] - V.o[2]};
        const float dn = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const float idn = 1.0f / dn;
        const float dir[3] = {d[0] * idn, d[1] * idn, d[2] * idn};
        float Y[16];
        sh_eval(D, dir[0], dir[1], dir[2], Y);
        const float gdc[3] = {gd6, gd7, gd8};
        float gc[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float acc = 0.5f;
#pragma unroll
            for (int j = 0; j < nc; ++j) acc = fmaf(fsh[3 * j + ch], Y[j], acc);
            gc[ch] = (acc > 0.f) ? gdc[ch] : 0.f;  // the colour's clamp at 0
        }
        // d colour / d dir = sum_j (sum_ch gc_ch f_j,ch) grad Y_j
        float h[16];
#pragma unroll
        for (int j = 0; j < nc; ++j) {
            h[j] = (fsh[3 * j] * gc[0] + fsh[3 * j + 1] * gc[1]) + fsh[3 * j + 2] * gc[2];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gsh[3 * j + ch] += Y[j] * gc[ch];
        }
        float gdir[3] = {0.f, 0.f, 0.f};
        sh_grad_dot(D, dir[0], dir[1], dir[2], h, gdir);
        const float dg = dir[0] * gdir[0] + dir[1] * gdir[1] + dir[2] * gdir[2];
        for (int a = 0; a < 3; ++a) gmu[a] += (gdir[a] - dir[a] * dg) * idn;
    }
    if (any)
        for (int a = 0; a < 3; ++a) out.means[a * n + i] += gmu[a];
#pragma unroll
    for (int k = 0; k < 3 * nc; ++k) out.sh[(int64_t)k * n + i] = gsh[k];
}

rgs_status project_bwd_launch(const float* dproj, const rgs_gaussians* g, const uint32_t* count, const ViewTable* vt,
                              const rgs_gaussians_grad* out, hipStream_t s) {
    if (g->n <= 0) return RGS_OK;
    const unsigned grid = (unsigned)((g->n + PJ_THREADS - 1) / PJ_THREADS);
    hipLaunchKernelGGL(k_project_bwd_geo, dim3(grid), dim3(PJ_THREADS), 0, s, dproj, *g, count, vt, *out);
    switch (g->sh_degree) {
        case 0: hipLaunchKernelGGL(k_project_bwd_sh<0>, dim3(grid), dim3(PJ_THREADS), 0, s, dproj, *g, count, vt, *out); break;
        case 1: hipLaunchKernelGGL(k_project_bwd_sh<1>, dim3(grid), dim3(PJ_THREADS), 0, s, dproj, *g, count, vt, *out); break;
        case 2: hipLaunchKernelGGL(k_project_bwd_sh<2>, dim3(grid), dim3(PJ_THREADS), 0, s, dproj, *g, count, vt, *out); break;
        default: hipLaunchKernelGGL(k_project_bwd_sh<3>, dim3(grid), dim3(PJ_THREADS), 0, s, dproj, *g, count, vt, *out); break;
    }
    return launch_check();
}

}  // namespace rgs
