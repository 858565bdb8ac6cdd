// render.hip -- per-cell partial blending (RetinaGS Eq. 3, Eq. 4 with the
// indicator of Eq. 6), its backward, and the per-pair gradient reduction.
//
// One wave64 per slot (tile t, cell k).  Lane l owns the four pixels of
// column l mod 16 in rows l/16, l/16 + 4, l/16 + 8, l/16 + 12, so the
// x-only terms of d^2 are computed once per Gaussian and lane:
//   dx = (x + 0.5) - mx, A = (ca dx) dx, B = (2 cb) dx,
//   d^2 = fma(dy, fma(cc, dy, B), A),          dy = (y + 0.5) - my,
// the exact fp32 operation sequence the CPU oracle mirrors for the contribute
// decision d^2 <= tau.  Gaussians are staged 64 at a time through LDS (one
// coalesced 48-byte record per lane) and read back as wave-uniform
// broadcasts.  A pixel stops after the contribution that takes its T_k below
// eps_T; the wave leaves as soon as all 256 pixels have stopped.
//
// Backward walks each slot back to front from the largest per-pixel `last`,
// recovers the transmittance before every contribution by division, sums
// each instance's gradient over the lane's four pixels, then over the wave
// with DPP row operations (no atomics), and stores one 9-float record at
// the instance's emission position; a second kernel sums each pair's
// records (contiguous by construction) in a fixed order.
#include "common.hpp"

namespace rgs {

static constexpr int RD_BATCH = 64;

struct SlotGeom {
    int v, px, py0, cell;
    bool ok;
};

__device__ __forceinline__ SlotGeom slot_geom(const ViewTable* __restrict__ vt, uint32_t key, int L) {
    SlotGeom g;
    const uint32_t gt = key >> L;
    const uint32_t rank = key & ((1u << L) - 1u);
    g.v = view_of_tile(vt, gt);
    const ViewParams& V = vt->v[g.v];
    const uint32_t lt = gt - V.tile_offset;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int lane = lane_id();
    g.px = tx * 16 + (lane & 15);
    g.py0 = ty * 16 + (lane >> 4);
    g.cell = V.cell_of_rank[rank];
    g.ok = true;
    return g;
}

__global__ __launch_bounds__(64) void k_render_fwd(const float* __restrict__ rec, const uint64_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ slot_key,
                                                   const uint32_t* __restrict__ slot_range,
                                                   const uint32_t* __restrict__ counters,
                                                   const ViewTable* __restrict__ vt, const float* __restrict__ box_lo,
                                                   const float* __restrict__ box_hi, float eps_T,
                                                   float* __restrict__ outC, float* __restrict__ outT,
                                                   uint32_t* __restrict__ outLast,
                                                   unsigned long long* __restrict__ stats) {
    __shared__ float4 sA[RD_BATCH], sB[RD_BATCH], sCl[RD_BATCH];
    const uint32_t slot = blockIdx.x;
    if (slot >= counters[2]) return;
    const int L = vt->L, K = 1 << L;
    const int lane = lane_id();
    const uint32_t key = slot_key[slot];
    const SlotGeom sg = slot_geom(vt, key, L);
    const ViewParams& V = vt->v[sg.v];
    const uint32_t begin = slot_range[2 * slot], end = slot_range[2 * slot + 1];
    float blo[3], bhi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        blo[a] = box_lo[a * K + sg.cell];
        bhi[a] = box_hi[a * K + sg.cell];
    }
    // per-pixel ray direction D(p) (fixed fp32 order, mirrored by the oracle)
    const float fxp = (float)sg.px + 0.5f;
    const float dxp = (fxp - V.cx) / V.fx;
    float Dp[4][3];
    float fyp[4];
    float T[4], C[4][3];
    uint32_t last[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int py = sg.py0 + 4 * r;
        fyp[r] = (float)py + 0.5f;
        const float dyp = (fyp[r] - V.cy) / V.fy;
#pragma unroll
        for (int a = 0; a < 3; ++a) Dp[r][a] = (V.R[a] * dxp + V.R[3 + a] * dyp) + V.R[6 + a];
        // a stopped (or off-image) pixel samples row +inf: d^2 = inf fails every test
        if (!(sg.px < V.W && py < V.H)) fyp[r] = INFINITY;
        T[r] = 1.0f;
        C[r][0] = C[r][1] = C[r][2] = 0.0f;
        last[r] = 0u;
    }
    const float o0 = V.o[0], o1 = V.o[1], o2 = V.o[2];
    uint32_t n_eval = 0, n_con = 0;

    for (uint32_t base = begin; base < end; base += RD_BATCH) {
        const bool alive = (fyp[0] != INFINITY) | (fyp[1] != INFINITY) | (fyp[2] != INFINITY) | (fyp[3] != INFINITY);
        if (__ballot(alive) == 0ull) break;
        const uint32_t idx = base + lane;
        if (idx < end) {
            const uint32_t src = (uint32_t)(vals[idx] >> 32);
            const float4* rp = reinterpret_cast<const float4*>(rec + (size_t)src * RGS_REC_FLOATS);
            float4 a = rp[0], b = rp[1], cl = rp[2];
            a.w = 2.0f * a.w;  // 2 cb (exact)
            sA[lane] = a;
            sB[lane] = b;
            sCl[lane] = cl;
        }
        __syncthreads();
        const int nb = (int)((end - base) < (uint32_t)RD_BATCH ? (end - base) : (uint32_t)RD_BATCH);
        for (int t = 0; t < nb; ++t) {
            const float4 a = sA[t];
            const float4 b = sB[t];
            const float dx = fxp - a.x;
            const float A = (a.z * dx) * dx;
            const float B = a.w * dx;
            float d2[4];
            bool hit[4];
            bool any = false;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float dy = fyp[r] - a.y;
                d2[r] = fmaf(dy, fmaf(b.x, dy, B), A);
                hit[r] = d2[r] <= b.z;
                any |= hit[r];
                if (stats) n_eval += (fyp[r] != INFINITY) ? 1u : 0u;
            }
            if (!any) continue;
            const float4 cl = sCl[t];
            const bool interior = (__float_as_uint(cl.w) & 1u) != 0u;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!hit[r]) continue;
                if (!interior) {
                    const float x0 = fmaf(b.w, Dp[r][0], o0);
                    const float x1 = fmaf(b.w, Dp[r][1], o1);
                    const float x2 = fmaf(b.w, Dp[r][2], o2);
                    const bool in = (blo[0] <= x0) && (x0 < bhi[0]) && (blo[1] <= x1) && (x1 < bhi[1]) &&
                                    (blo[2] <= x2) && (x2 < bhi[2]);
                    if (!in) continue;
                }
                if (stats) ++n_con;
                const float G = __builtin_amdgcn_exp2f(d2[r] * -0.72134752044448170368f);  // exp(-d^2/2)
                const float sg_ = fminf(0.99f, b.y * G);
                const float wgt = sg_ * T[r];
                C[r][0] = fmaf(wgt, cl.x, C[r][0]);
                C[r][1] = fmaf(wgt, cl.y, C[r][1]);
                C[r][2] = fmaf(wgt, cl.z, C[r][2]);
                T[r] = T[r] * (1.0f - sg_);
                last[r] = base - begin + (uint32_t)t + 1u;
                if (T[r] < eps_T) fyp[r] = INFINITY;
            }
        }
        __syncthreads();
    }
    if (stats) {
        unsigned long long e = n_eval, c = n_con;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            e += __shfl_xor(e, d, 64);
            c += __shfl_xor(c, d, 64);
        }
        if (lane == 0) {
            atomicAdd(&stats[0], e);
            atomicAdd(&stats[1], c);
        }
    }
    float* oc = outC + (size_t)slot * 768;
    float* ot = outT + (size_t)slot * 256;
    uint32_t* ol = outLast + (size_t)slot * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = ((lane >> 4) + 4 * r) * 16 + (lane & 15);
        oc[p] = C[r][0];
        oc[256 + p] = C[r][1];
        oc[512 + p] = C[r][2];
        ot[p] = T[r];
        ol[p] = last[r];
    }
}

rgs_status render_fwd_launch(const rgs_projected* proj, const rgs_bins* bins, const ViewTable* vt, const rgs_kdtree* kd,
                             float eps_T, const rgs_partials* out, uint64_t* stats, int64_t slot_bound, hipStream_t s) {
    if (slot_bound <= 0) return RGS_OK;
    hipLaunchKernelGGL(k_render_fwd, dim3((unsigned)slot_bound), dim3(64), 0, s, proj->rec, bins->vals, bins->slot_key,
                       bins->slot_range, bins->counters, vt, kd->box_lo, kd->box_hi, eps_T, out->C, out->T, out->last,
                       reinterpret_cast<unsigned long long*>(stats));
    return launch_check();
}

// ------------------------------------------------------------------ backward
__global__ __launch_bounds__(64) void k_render_bwd(const float* __restrict__ rec, const uint64_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ slot_key,
                                                   const uint32_t* __restrict__ slot_range,
                                                   const uint32_t* __restrict__ counters,
                                                   const ViewTable* __restrict__ vt, const float* __restrict__ box_lo,
                                                   const float* __restrict__ box_hi, const float* __restrict__ partT,
                                                   const uint32_t* __restrict__ partLast, const float* __restrict__ dC,
                                                   const float* __restrict__ dT, float* __restrict__ records) {
    __shared__ float4 sA[RD_BATCH], sB[RD_BATCH], sCl[RD_BATCH];
    __shared__ uint32_t sJ[RD_BATCH];
    const uint32_t slot = blockIdx.x;
    if (slot >= counters[2]) return;
    const int L = vt->L, K = 1 << L;
    const int lane = lane_id();
    const uint32_t key = slot_key[slot];
    const SlotGeom sg = slot_geom(vt, key, L);
    const ViewParams& V = vt->v[sg.v];
    const uint32_t begin = slot_range[2 * slot], end = slot_range[2 * slot + 1];
    float blo[3], bhi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        blo[a] = box_lo[a * K + sg.cell];
        bhi[a] = box_hi[a * K + sg.cell];
    }
    const float fxp = (float)sg.px + 0.5f;
    const float dxp = (fxp - V.cx) / V.fx;
    float Dp[4][3], fyp[4];
    float Tcur[4], gTf[4], gC[4][3], Bc[4][3];
    uint32_t last[4];
    uint32_t maxlast = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int py = sg.py0 + 4 * r;
        fyp[r] = (float)py + 0.5f;
        const float dyp = (fyp[r] - V.cy) / V.fy;
#pragma unroll
        for (int a = 0; a < 3; ++a) Dp[r][a] = (V.R[a] * dxp + V.R[3 + a] * dyp) + V.R[6 + a];
        const int p = ((lane >> 4) + 4 * r) * 16 + (lane & 15);
        const bool valid = sg.px < V.W && py < V.H;
        const float Tf = partT[(size_t)slot * 256 + p];
        last[r] = valid ? partLast[(size_t)slot * 256 + p] : 0u;
        Tcur[r] = Tf;
        gTf[r] = valid ? dT[(size_t)slot * 256 + p] * Tf : 0.f;
        for (int ch = 0; ch < 3; ++ch) {
            gC[r][ch] = valid ? dC[(size_t)slot * 768 + ch * 256 + p] : 0.f;
            Bc[r][ch] = 0.f;
        }
        maxlast = last[r] > maxlast ? last[r] : maxlast;
    }
    maxlast = wave_max_u32(maxlast);
    const float o0 = V.o[0], o1 = V.o[1], o2 = V.o[2];
    const uint32_t len = end - begin;

    // instances never reached by any pixel get zero records
    for (uint32_t k = maxlast + lane; k < len; k += 64) {
        const uint32_t j = (uint32_t)vals[begin + k];
        float* rp = records + (size_t)j * 9;
        for (int c = 0; c < 9; ++c) rp[c] = 0.f;
    }
    if (maxlast == 0) return;

    int bstart = (int)(((maxlast - 1) / RD_BATCH) * RD_BATCH);
    for (; bstart >= 0; bstart -= RD_BATCH) {
        const uint32_t idx = begin + (uint32_t)bstart + lane;
        if ((uint32_t)bstart + lane < maxlast) {
            const uint64_t vv = vals[idx];
            const uint32_t src = (uint32_t)(vv >> 32);
            const float4* rp = reinterpret_cast<const float4*>(rec + (size_t)src * RGS_REC_FLOATS);
            float4 a = rp[0], b = rp[1], cl = rp[2];
            sA[lane] = a;
            sB[lane] = b;
            sCl[lane] = cl;
            sJ[lane] = (uint32_t)vv;
        }
        __syncthreads();
        int tmax = (int)maxlast - 1 - bstart;
        if (tmax > RD_BATCH - 1) tmax = RD_BATCH - 1;
        for (int t = tmax; t >= 0; --t) {
            const uint32_t pos1 = (uint32_t)(bstart + t) + 1u;  // this instance's index + 1
            const float4 a = sA[t];
            const float4 b = sB[t];
            const float4 cl = sCl[t];
            const bool interior = (__float_as_uint(cl.w) & 1u) != 0u;
            const float cb2 = 2.0f * a.w;
            const float dx = fxp - a.x;
            const float A = (a.z * dx) * dx;
            const float Bx = cb2 * dx;
            float g[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) g[c] = 0.f;
            bool contrib = false;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (pos1 > last[r]) continue;
                const float dy = fyp[r] - a.y;
                const float d2 = fmaf(dy, fmaf(b.x, dy, Bx), A);
                if (!(d2 <= b.z)) continue;
                if (!interior) {
                    const float x0 = fmaf(b.w, Dp[r][0], o0);
                    const float x1 = fmaf(b.w, Dp[r][1], o1);
                    const float x2 = fmaf(b.w, Dp[r][2], o2);
                    const bool in = (blo[0] <= x0) && (x0 < bhi[0]) && (blo[1] <= x1) && (x1 < bhi[1]) &&
                                    (blo[2] <= x2) && (x2 < bhi[2]);
                    if (!in) continue;
                }
                contrib = true;
                const float G = __builtin_amdgcn_exp2f(d2 * -0.72134752044448170368f);  // exp(-d^2/2)
                const float aG = b.y * G;
                const float sgm = fminf(0.99f, aG);
                const float om = 1.0f - sgm;
                const float rom = __builtin_amdgcn_rcpf(om);
                const float Tb = Tcur[r] * rom;  // transmittance before this contribution
                const float dot = gC[r][0] * (cl.x - Bc[r][0]) + gC[r][1] * (cl.y - Bc[r][1]) + gC[r][2] * (cl.z - Bc[r][2]);
                const float dsg = Tb * dot - gTf[r] * rom;
                const float wc = Tb * sgm;
                g[6] = fmaf(wc, gC[r][0], g[6]);
                g[7] = fmaf(wc, gC[r][1], g[7]);
                g[8] = fmaf(wc, gC[r][2], g[8]);
                Bc[r][0] = fmaf(sgm, cl.x - Bc[r][0], Bc[r][0]);
                Bc[r][1] = fmaf(sgm, cl.y - Bc[r][1], Bc[r][1]);
                Bc[r][2] = fmaf(sgm, cl.z - Bc[r][2], Bc[r][2]);
                Tcur[r] = Tb;
                if (aG < 0.99f) {
                    const float dd2 = -0.5f * aG * dsg;
                    g[5] = fmaf(dsg, G, g[5]);
                    g[0] -= dd2 * 2.0f * (a.z * dx + a.w * dy);
                    g[1] -= dd2 * 2.0f * (a.w * dx + b.x * dy);
                    g[2] = fmaf(dd2, dx * dx, g[2]);
                    g[3] = fmaf(dd2, 2.0f * dx * dy, g[3]);
                    g[4] = fmaf(dd2, dy * dy, g[4]);
                }
            }
            float* rp = records + (size_t)sJ[t] * 9;
            if (__ballot(contrib) == 0ull) {
                if (lane < 9) rp[lane] = 0.f;
                continue;
            }
            // values 0..7: reduce-scatter over lane bits 5, 4, 3 (exchanging the
            // half a lane does not keep), then a full sum over bits 2, 1, 0;
            // lane 8v ends with the total of value v.  Value 8: full sum.
            const float s8 = wave_sum_to_lane63(g[8]);
            const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0, h3 = (lane & 8) != 0;
            float q4[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float keep = h5 ? g[4 + k] : g[k];
                const float give = h5 ? g[k] : g[4 + k];
                q4[k] = keep + __shfl_xor(give, 32, 64);
            }
            float q2[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const float keep = h4 ? q4[2 + k] : q4[k];
                const float give = h4 ? q4[k] : q4[2 + k];
                q2[k] = keep + __shfl_xor(give, 16, 64);
            }
            float q1 = (h3 ? q2[1] : q2[0]) + __shfl_xor(h3 ? q2[0] : q2[1], 8, 64);
            q1 += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, q1), 0xb1, 0xf, 0xf, false));  // xor 1
            q1 += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, q1), 0x4e, 0xf, 0xf, false));  // xor 2
            q1 += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, q1), 0x141, 0xf, 0xf, false)); // half-row mirror
            if ((lane & 7) == 0) rp[lane >> 3] = q1;
            if (lane == 63) rp[8] = s8;
        }
        __syncthreads();
    }
}

// Per (view, Gaussian) pair: sum its instance records in emission order.
__global__ __launch_bounds__(256) void k_pair_reduce(const float* __restrict__ records, const uint32_t* __restrict__ count,
                                                     const int32_t* __restrict__ pair_rank,
                                                     const uint32_t* __restrict__ pair_off, int64_t m,
                                                     float* __restrict__ dproj) {
    const int64_t sidx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (sidx >= m) return;
    float acc[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] = 0.f;
    if (count[sidx] > 0u) {
        const int32_t r = pair_rank[sidx];
        const uint32_t b = pair_off[r], e = pair_off[r + 1];
        for (uint32_t j = b; j < e; ++j) {
            const float* rp = records + (size_t)j * 9;
#pragma unroll
            for (int c = 0; c < 9; ++c) acc[c] += rp[c];
        }
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) dproj[c * m + sidx] = acc[c];
}

size_t render_bwd_ws_bytes(int64_t capacity) { return (size_t)(capacity > 0 ? capacity : 1) * 9 * sizeof(float) + 256; }

rgs_status render_bwd_launch(const rgs_partials_grad* dparts, const rgs_partials* parts, const rgs_bins* bins,
                             const rgs_projected* proj, int64_t n, int n_views, const ViewTable* vt,
                             const rgs_kdtree* kd, float* dproj, void* ws, int64_t slot_bound, hipStream_t s) {
    float* records = reinterpret_cast<float*>(ws);
    if (slot_bound > 0)
        hipLaunchKernelGGL(k_render_bwd, dim3((unsigned)slot_bound), dim3(64), 0, s, proj->rec, bins->vals, bins->slot_key,
                           bins->slot_range, bins->counters, vt, kd->box_lo, kd->box_hi, parts->T, parts->last, dparts->dC,
                           dparts->dT, records);
    RGS_LAUNCH_CHECK();
    const int64_t m = (int64_t)n_views * n;
    if (m > 0)
        hipLaunchKernelGGL(k_pair_reduce, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, records, proj->count,
                           bins->pair_rank, bins->pair_off, m, dproj);
    return launch_check();
}

}  // namespace rgs
