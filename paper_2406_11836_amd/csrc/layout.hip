// layout.hip -- a copy of the Gaussians grouped by the KD leaf of their
// centre (each sub-model's subset of Sec. 3.3 contiguous in memory), ordered
// inside a leaf along a Morton curve over the leaf's bounds.  Views that
// cannot see a cell then skip a contiguous index range whose parameters are
// never fetched, and Gaussians visible together share cache lines.
//
// Key = leaf << 24 | interleaved 8-bit coordinates of the centre quantised
// to the leaf's centre-bounds box; a stable radix sort on the key keeps gid
// order among equal keys, so the permutation is deterministic.
#include "common.hpp"

namespace rgs {

static constexpr int LY_THREADS = 256;

__device__ __forceinline__ uint32_t spread3_8(uint32_t v) {  // bit b of v -> bit 3b
    v &= 0xffu;
    v = (v | (v << 8)) & 0x0000f00fu;
    v = (v | (v << 4)) & 0x000c30c3u;
    v = (v | (v << 2)) & 0x00249249u;
    return v;
}

__global__ __launch_bounds__(LY_THREADS) void k_group_keys(const float* __restrict__ means,
                                                           const int32_t* __restrict__ center_cell,
                                                           const float* __restrict__ cell_bounds, int K, int64_t n,
                                                           uint32_t* __restrict__ keys, uint32_t* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * LY_THREADS + threadIdx.x;
    if (i >= n) return;
    const int cell = center_cell[i];
    uint32_t code = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = cell_bounds[a * K + cell], hi = cell_bounds[(3 + a) * K + cell];
        const float x = means[a * n + i];
        const float u = hi > lo ? (x - lo) / (hi - lo) : 0.0f;
        const int q = (int)fminf(fmaxf(u * 256.0f, 0.0f), 255.0f);
        code |= spread3_8((uint32_t)q) << a;
    }
    keys[i] = ((uint32_t)cell << 24) | code;
    idx[i] = (uint32_t)i;
}

struct GaussOut {  // writable view of the output parameter buffers
    float *means, *log_scales, *quats, *opacity, *sh;
};

__global__ __launch_bounds__(LY_THREADS) void k_group_gather(rgs_gaussians in, GaussOut out, int nc,
                                                             const uint32_t* __restrict__ perm,
                                                             int32_t* __restrict__ perm_out) {
    const int64_t n = in.n;
    const int64_t j = (int64_t)blockIdx.x * LY_THREADS + threadIdx.x;
    if (j >= n) return;
    const int64_t s = perm[j];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        out.means[a * n + j] = in.means[a * n + s];
        out.log_scales[a * n + j] = in.log_scales[a * n + s];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) out.quats[a * n + j] = in.quats[a * n + s];
    out.opacity[j] = in.opacity[s];
    for (int k = 0; k < 3 * nc; ++k) out.sh[(int64_t)k * n + j] = in.sh[(int64_t)k * n + s];
    if (perm_out) perm_out[j] = (int32_t)s;
}

size_t group_ws_bytes(int64_t n) {
    WsCarver c{nullptr, 0, 0};
    for (int k = 0; k < 4; ++k) c.take<uint32_t>(n + 1);
    c.take<char>(radix_ws_bytes(n + 1));
    return c.used + 256;
}

rgs_status group_by_cell(const rgs_gaussians* in, const rgs_kdtree* kd, int L, const rgs_gaussians* out,
                         int32_t* perm, void* ws, size_t ws_bytes, hipStream_t s) {
    const int64_t n = in->n;
    if (n <= 0) return RGS_OK;
    WsCarver c{reinterpret_cast<char*>(ws), 0, ws_bytes};
    uint32_t* keys = c.take<uint32_t>(n + 1);
    uint32_t* idx = c.take<uint32_t>(n + 1);
    uint32_t* keys_alt = c.take<uint32_t>(n + 1);
    uint32_t* idx_alt = c.take<uint32_t>(n + 1);
    void* rws = c.take<char>(radix_ws_bytes(n + 1));
    if (!c.ok()) return RGS_E_ARG;
    const unsigned grid = (unsigned)((n + LY_THREADS - 1) / LY_THREADS);
    hipLaunchKernelGGL(k_group_keys, dim3(grid), dim3(LY_THREADS), 0, s, in->means, kd->center_cell, kd->cell_bounds,
                       1 << L, n, keys, idx);
    RGS_LAUNCH_CHECK();
    rgs_status st = radix_sort_u32_u32(keys, idx, keys_alt, idx_alt, n, 24 + L, rws, s);
    if (st != RGS_OK) return st;
    const int nc = (in->sh_degree + 1) * (in->sh_degree + 1);
    // `out` describes the caller's destination buffers, which this call fills
    const GaussOut o{const_cast<float*>(out->means), const_cast<float*>(out->log_scales), const_cast<float*>(out->quats),
                     const_cast<float*>(out->opacity), const_cast<float*>(out->sh)};
    hipLaunchKernelGGL(k_group_gather, dim3(grid), dim3(LY_THREADS), 0, s, *in, o, nc, idx, perm);
    return launch_check();
}

}  // namespace rgs
