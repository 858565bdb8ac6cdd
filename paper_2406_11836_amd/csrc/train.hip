// train.hip -- the parameter update of the training loop (the paper trains
// with 3DGS's optimiser: Adam, per-group learning rates, the position rate
// decaying exponentially, Sec. 4 implementation details) and the reorder of
// parameters and optimiser states after a re-partition (Sec. 3.4: the KD
// partition is redone after a set number of epochs).
//
// Adam is one pass over the five parameter arrays, fp32 states: per element
// read p, g, m, v and write p, m, v (28 bytes), HBM-bound.  Every array is a
// structure of rows of length n, so a flat index walks it coalesced; four
// consecutive elements per thread (16-byte loads) where the buffers allow.
#include "common.hpp"

namespace rgs {

static constexpr int TR_THREADS = 256;

struct AdamGroup {
    float* p;
    const float* g;
    float* m;
    float* v;
    int64_t len;       // rows * n
    int64_t dc_len;    // elements using lr_a (the rest use lr_b): SH degree 0 rows; == len elsewhere
    float lr_a, lr_b;
};

// The hyperparameters arrive in fp64; each constant the update uses is
// formed there and rounded to fp32 once (1 - b2 for b2 = 0.999 would lose
// 13 bits if formed from the rounded b2).
struct AdamArgs {
    AdamGroup grp[5];
    float beta1, beta2, omb1, omb2, eps, c1, c2;  // omb = 1 - beta; c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
};

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, const AdamArgs& a) {
    m = fmaf(a.beta1, m, a.omb1 * g);
    v = fmaf(a.beta2, v, (a.omb2 * g) * g);
    const float mh = m * a.c1, vh = v * a.c2;
    p = p - lr * (mh / (sqrtf(vh) + a.eps));
}

// blockIdx.y selects the parameter array; each thread takes four consecutive
// elements (grid-stride), with 16-byte accesses when all four buffers are
// 16-byte aligned, else one element at a time.
__global__ __launch_bounds__(TR_THREADS) void k_adam(AdamArgs a) {
    const AdamGroup G = a.grp[blockIdx.y];
    const int64_t len = G.len;
    if (len <= 0) return;
    const bool vec = ((reinterpret_cast<uintptr_t>(G.p) | reinterpret_cast<uintptr_t>(G.g) |
                       reinterpret_cast<uintptr_t>(G.m) | reinterpret_cast<uintptr_t>(G.v)) & 15u) == 0;
    const int64_t stride = (int64_t)gridDim.x * TR_THREADS * 4;
    for (int64_t e0 = ((int64_t)blockIdx.x * TR_THREADS + threadIdx.x) * 4; e0 < len; e0 += stride) {
        if (vec && e0 + 4 <= len) {
            float4 p = *reinterpret_cast<const float4*>(G.p + e0);
            const float4 g = *reinterpret_cast<const float4*>(G.g + e0);
            float4 m = *reinterpret_cast<const float4*>(G.m + e0);
            float4 v = *reinterpret_cast<const float4*>(G.v + e0);
            adam_one(p.x, g.x, m.x, v.x, e0 + 0 < G.dc_len ? G.lr_a : G.lr_b, a);
            adam_one(p.y, g.y, m.y, v.y, e0 + 1 < G.dc_len ? G.lr_a : G.lr_b, a);
            adam_one(p.z, g.z, m.z, v.z, e0 + 2 < G.dc_len ? G.lr_a : G.lr_b, a);
            adam_one(p.w, g.w, m.w, v.w, e0 + 3 < G.dc_len ? G.lr_a : G.lr_b, a);
            *reinterpret_cast<float4*>(G.p + e0) = p;
            *reinterpret_cast<float4*>(G.m + e0) = m;
            *reinterpret_cast<float4*>(G.v + e0) = v;
        } else {
            for (int64_t e = e0; e < e0 + 4 && e < len; ++e) {
                float p = G.p[e], m = G.m[e], v = G.v[e];
                adam_one(p, G.g[e], m, v, e < G.dc_len ? G.lr_a : G.lr_b, a);
                G.p[e] = p;
                G.m[e] = m;
                G.v[e] = v;
            }
        }
    }
}

rgs_status adam_launch(const rgs_gaussians_grad* params, const rgs_gaussians_grad* grads, const rgs_gaussians_grad* m,
                       const rgs_gaussians_grad* v, int64_t n, int sh_degree, const rgs_adam_params* hp, hipStream_t s) {
    if (n <= 0) return RGS_OK;
    const int64_t nc = (int64_t)(sh_degree + 1) * (sh_degree + 1);
    AdamArgs a;
    const int64_t rows[5] = {3, 3, 4, 1, 3 * nc};
    float* const P[5] = {params->means, params->log_scales, params->quats, params->opacity, params->sh};
    const float* const Gr[5] = {grads->means, grads->log_scales, grads->quats, grads->opacity, grads->sh};
    float* const M[5] = {m->means, m->log_scales, m->quats, m->opacity, m->sh};
    float* const V[5] = {v->means, v->log_scales, v->quats, v->opacity, v->sh};
    const float lr[5] = {hp->lr_means, hp->lr_log_scales, hp->lr_quats, hp->lr_opacity, hp->lr_sh_dc};
    for (int k = 0; k < 5; ++k) {
        a.grp[k] = AdamGroup{P[k], Gr[k], M[k], V[k], rows[k] * n, rows[k] * n, lr[k], lr[k]};
    }
    a.grp[4].dc_len = 3 * n;  // SH rows 0..2: degree 0 (one per channel)
    a.grp[4].lr_b = hp->lr_sh_rest;
    // bias corrections from the 1-based step count, in fp64 on the host
    const double b1t = pow(hp->beta1, (double)hp->step), b2t = pow(hp->beta2, (double)hp->step);
    a.beta1 = (float)hp->beta1;
    a.beta2 = (float)hp->beta2;
    a.omb1 = (float)(1.0 - hp->beta1);
    a.omb2 = (float)(1.0 - hp->beta2);
    a.eps = (float)hp->eps;
    a.c1 = (float)(1.0 / (1.0 - b1t));
    a.c2 = (float)(1.0 / (1.0 - b2t));
    const int64_t most = 3 * nc * n;
    int64_t blocks = (most + TR_THREADS * 4 - 1) / (TR_THREADS * 4);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks, 5), dim3(TR_THREADS), 0, s, a);
    return launch_check();
}

// out row j = in row perm[j] in every array (perm entries outside [0, n) leave
// row j untouched).
struct PermOut {
    float *means, *log_scales, *quats, *opacity, *sh;
};

__global__ __launch_bounds__(TR_THREADS) void k_permute(rgs_gaussians in, PermOut out, int nc,
                                                        const int32_t* __restrict__ perm) {
    const int64_t n = in.n;
    const int64_t j = (int64_t)blockIdx.x * TR_THREADS + threadIdx.x;
    if (j >= n) return;
    const int64_t s = perm[j];
    if (s < 0 || s >= n) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        out.means[a * n + j] = in.means[a * n + s];
        out.log_scales[a * n + j] = in.log_scales[a * n + s];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) out.quats[a * n + j] = in.quats[a * n + s];
    out.opacity[j] = in.opacity[s];
    for (int k = 0; k < 3 * nc; ++k) out.sh[(int64_t)k * n + j] = in.sh[(int64_t)k * n + s];
}

rgs_status permute_launch(const rgs_gaussians* in, const int32_t* perm, const rgs_gaussians_grad* out, hipStream_t s) {
    if (in->n <= 0) return RGS_OK;
    const int nc = (in->sh_degree + 1) * (in->sh_degree + 1);
    const PermOut o{out->means, out->log_scales, out->quats, out->opacity, out->sh};
    hipLaunchKernelGGL(k_permute, dim3((unsigned)((in->n + TR_THREADS - 1) / TR_THREADS)), dim3(TR_THREADS), 0, s, *in, o,
                       nc, perm);
    return launch_check();
}

}  // namespace rgs
