// merge.hip -- ray-order merge of the partial maps (RetinaGS Eq. 5) and its
// backward (the gradient the manager returns to each sub-model, Sec. 3.4).
//
// One 256-thread block per global tile, one thread per pixel; the slots of a
// tile are contiguous and already in the view's cell order, so each thread
// folds (C, T) <- (C + T C_k, T T_k) over them.  Partial maps are read as
// 256-float rows, so every load is a coalesced 1 KB line per slot.
#include "common.hpp"

namespace rgs {

static constexpr int MB_REG = 8;  // slots per tile whose T_k, P_k the merge backward keeps in registers

__global__ __launch_bounds__(256) void k_merge_fwd(const float* __restrict__ pC, const float* __restrict__ pT,
                                                   const uint32_t* __restrict__ tile_slot,
                                                   const ViewTable* __restrict__ vt, float* __restrict__ image,
                                                   float* __restrict__ T_final) {
    const uint32_t gt = blockIdx.x;
    const int v = view_of_tile(vt, gt);
    const ViewParams& V = vt->v[v];
    const uint32_t lt = gt - V.tile_offset;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int p = threadIdx.x;
    const int x = tx * 16 + (p & 15), y = ty * 16 + (p >> 4);
    if (x >= V.W || y >= V.H) return;
    const uint32_t s0 = tile_slot[gt], s1 = tile_slot[gt + 1];
    float c0 = 0.f, c1 = 0.f, c2 = 0.f, T = 1.f;
    uint32_t s = s0;
    // two slots per step, both slots' loads issued before the folds
    for (; s + 1 < s1; s += 2) {
        const float* ca = pC + (size_t)s * 768;
        const float* cb = ca + 768;
        const float a0 = ca[p], a1 = ca[256 + p], a2 = ca[512 + p], ta = pT[(size_t)s * 256 + p];
        const float b0 = cb[p], b1 = cb[256 + p], b2 = cb[512 + p], tb = pT[(size_t)s * 256 + 256 + p];
        c0 = fmaf(T, a0, c0);
        c1 = fmaf(T, a1, c1);
        c2 = fmaf(T, a2, c2);
        T *= ta;
        c0 = fmaf(T, b0, c0);
        c1 = fmaf(T, b1, c1);
        c2 = fmaf(T, b2, c2);
        T *= tb;
    }
    if (s < s1) {
        const float* cc = pC + (size_t)s * 768;
        c0 = fmaf(T, cc[p], c0);
        c1 = fmaf(T, cc[256 + p], c1);
        c2 = fmaf(T, cc[512 + p], c2);
        T *= pT[(size_t)s * 256 + p];
    }
    const size_t HW = (size_t)V.W * V.H;
    const size_t pix = (size_t)y * V.W + x;
    float* img = image + 3 * (size_t)V.pix_offset;
    img[pix] = fmaf(T, V.bg[0], c0);
    img[HW + pix] = fmaf(T, V.bg[1], c1);
    img[2 * HW + pix] = fmaf(T, V.bg[2], c2);
    T_final[V.pix_offset + pix] = T;
}

// dC_k = P_k g;  dT_k = P_k (<g, R_k> + gT Q_k), with P_k the transmittance in
// front of slot k, R_k the merged colour behind it (background included) and
// Q_k the transmittance behind it.  For up to MB_REG slots per tile the T_k
// and P_k stay in registers (the slot count is uniform over the block);
// beyond, P_k is parked in dT on the way forward.
__global__ __launch_bounds__(256) void k_merge_bwd(const float* __restrict__ dimage, const float* __restrict__ dTfinal,
                                                   const float* __restrict__ pC, const float* __restrict__ pT,
                                                   const uint32_t* __restrict__ tile_slot,
                                                   const ViewTable* __restrict__ vt, float* __restrict__ dC,
                                                   float* __restrict__ dT) {
    const uint32_t gt = blockIdx.x;
    const int v = view_of_tile(vt, gt);
    const ViewParams& V = vt->v[v];
    const uint32_t lt = gt - V.tile_offset;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int p = threadIdx.x;
    const int x = tx * 16 + (p & 15), y = ty * 16 + (p >> 4);
    const uint32_t s0 = tile_slot[gt], s1 = tile_slot[gt + 1];
    const bool valid = x < V.W && y < V.H;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, gT = 0.f;
    if (valid) {
        const size_t HW = (size_t)V.W * V.H;
        const size_t pix = (size_t)y * V.W + x;
        const float* di = dimage + 3 * (size_t)V.pix_offset;
        g0 = di[pix];
        g1 = di[HW + pix];
        g2 = di[2 * HW + pix];
        gT = dTfinal ? dTfinal[V.pix_offset + pix] : 0.f;
    }
    float R0 = V.bg[0], R1 = V.bg[1], R2 = V.bg[2], Q = 1.f;
    const uint32_t ns = s1 - s0;
    if (ns <= (uint32_t)MB_REG) {
        float Tr[MB_REG], Pr[MB_REG];
        float P = 1.f;
#pragma unroll
        for (int k = 0; k < MB_REG; ++k)
            if ((uint32_t)k < ns) Tr[k] = pT[(size_t)(s0 + k) * 256 + p];
#pragma unroll
        for (int k = 0; k < MB_REG; ++k)
            if ((uint32_t)k < ns) {
                Pr[k] = P;
                P *= Tr[k];
            }
#pragma unroll
        for (int k = MB_REG - 1; k >= 0; --k) {
            if ((uint32_t)k >= ns) continue;
            const size_t s = s0 + (uint32_t)k;
            const float* cc = pC + s * 768;
            const float a0 = cc[p], a1 = cc[256 + p], a2 = cc[512 + p];
            dC[s * 768 + p] = Pr[k] * g0;
            dC[s * 768 + 256 + p] = Pr[k] * g1;
            dC[s * 768 + 512 + p] = Pr[k] * g2;
            dT[s * 256 + p] = Pr[k] * (g0 * R0 + g1 * R1 + g2 * R2 + gT * Q);
            R0 = fmaf(Tr[k], R0, a0);
            R1 = fmaf(Tr[k], R1, a1);
            R2 = fmaf(Tr[k], R2, a2);
            Q *= Tr[k];
        }
        return;
    }
    float P = 1.f;
    for (uint32_t s = s0; s < s1; ++s) {
        dT[(size_t)s * 256 + p] = P;
        P *= pT[(size_t)s * 256 + p];
    }
    for (uint32_t s = s1; s > s0; --s) {
        const size_t k = s - 1;
        const float Pk = dT[k * 256 + p];
        dC[k * 768 + p] = Pk * g0;
        dC[k * 768 + 256 + p] = Pk * g1;
        dC[k * 768 + 512 + p] = Pk * g2;
        dT[k * 256 + p] = Pk * (g0 * R0 + g1 * R1 + g2 * R2 + gT * Q);
        const float Tk = pT[k * 256 + p];
        R0 = fmaf(Tk, R0, pC[k * 768 + p]);
        R1 = fmaf(Tk, R1, pC[k * 768 + 256 + p]);
        R2 = fmaf(Tk, R2, pC[k * 768 + 512 + p]);
        Q *= Tk;
    }
}

rgs_status merge_fwd_launch(const rgs_partials* parts, const rgs_bins* bins, const ViewTable* vt, int64_t total_tiles,
                            float* image, float* T_final, hipStream_t s) {
    if (total_tiles <= 0) return RGS_OK;
    hipLaunchKernelGGL(k_merge_fwd, dim3((unsigned)total_tiles), dim3(256), 0, s, parts->C, parts->T, bins->tile_slot, vt,
                       image, T_final);
    return launch_check();
}

rgs_status merge_bwd_launch(const float* dimage, const float* dTfinal, const rgs_partials* parts, const rgs_bins* bins,
                            const ViewTable* vt, int64_t total_tiles, const rgs_partials_grad* out, hipStream_t s) {
    if (total_tiles <= 0) return RGS_OK;
    hipLaunchKernelGGL(k_merge_bwd, dim3((unsigned)total_tiles), dim3(256), 0, s, dimage, dTfinal, parts->C, parts->T,
                       bins->tile_slot, vt, out->dC, out->dT);
    return launch_check();
}

}  // namespace rgs
