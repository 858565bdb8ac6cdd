// render.hip -- per-cell partial blending (RetinaGS Eq. 3, Eq. 4 with the
// indicator of Eq. 6), its backward, and the per-pair gradient reduction.
//
// One 256-thread block per slot (tile t, cell k); wave w owns the 8x8
// quadrant (w & 1, w >> 1) of the 16x16 tile, one pixel per lane.  The
// contribute decision d^2 <= tau uses the exact fp32 operation sequence the
// CPU oracle mirrors, on the factored form of the quadratic (no cancellation
// for elongated footprints):
//   dx = (x + 0.5) - mx, dy = (y + 0.5) - my, u = fma(k, dy, dx),
//   d^2 = fma(e dy, dy, (ca u) u).
// The conic (ca, cb, cc) = (ca, k ca, e + k cb) is rebuilt per instance where
// the quadrant test and the gradients need it.  Gaussian records are staged
// through LDS (one coalesced 64-byte record per thread) with a 4-bit mask of
// the quadrants their rectangle meets, and read
// back as wave-uniform broadcasts; a wave skips Gaussians outside its
// quadrant with a scalar branch.  A pixel stops after the contribution that
// takes its T_k below eps_T; the block leaves once all 256 pixels stopped.
//
// Backward (a 128-thread block per slot, two pixels of one row per lane)
// walks each slot back to front from the largest per-pixel `last`, recovers
// the transmittance before every contribution from a reciprocal, adds each
// lane's two pixels and sums each instance's gradient over the wave's 128
// pixels with a reduce-scatter butterfly (no atomics), adds the two half-tile
// sums in a fixed order and stores one record (9 floats, 36 bytes) at the
// instance's emission position; a segmented reduction then sums each pair's
// records (contiguous by construction) in a fixed order.
#include "common.hpp"

namespace rgs {

static constexpr int RD_BATCH = 64;
static constexpr int RD_REC = 9;   // floats per backward record (36 bytes, read back contiguously)
static constexpr int PS_REC = 12;  // floats per per-pair / per-wave sum (48 bytes, float4-aligned)
// The backward's launch order: slots per block of its two passes, and the
// size classes (half octaves of the instances a slot is walked over)
static constexpr int SW_SLOTS = 64;
static constexpr int SW_CLS = 64;

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

// Quadrant mask of a Gaussian's rectangle within tile (tx, ty): bit q set iff
// the rectangle meets 8x8 quadrant q = 2 qy + qx of the 16x16 tile.
__device__ __forceinline__ uint32_t quad_mask(uint2 rr, int tx, int ty) {
    const int x0 = (int)(int16_t)(rr.x & 0xffffu) - tx * 16, x1 = (int)(int16_t)(rr.x >> 16) - tx * 16;
    const int y0 = (int)(int16_t)(rr.y & 0xffffu) - ty * 16, y1 = (int)(int16_t)(rr.y >> 16) - ty * 16;
    const uint32_t mx = ((x0 <= 7 && x1 >= 0) ? 1u : 0u) | ((x0 <= 15 && x1 >= 8) ? 2u : 0u);
    const uint32_t my = ((y0 <= 7 && y1 >= 0) ? 1u : 0u) | ((y0 <= 15 && y1 >= 8) ? 2u : 0u);
    uint32_t m = 0;
    if (my & 1u) m |= mx;
    if (my & 2u) m |= mx << 2;
    return m;
}

// Can a pixel centre of the wx-by-wy block of pixels whose first pixel is
// (x0, y0) pass the fp32 decision d^2 <= tau?  The minimum of the quadratic
// form over the box of the block's pixel centres is 0 if the mean is inside,
// else the least of its four edge minima (a convex function of one variable
// each, minimised at the clamped stationary point).  Against the fp32
// sequence used per pixel the test adds a margin of 2^-18 (ca dx^2 + cc dy^2)
// at the box's far corner, above the rounding error of both evaluations (a
// few ulp of |ca dx^2| + 2|cb dx dy| + |cc dy^2| <= 2 (ca dx^2 + cc dy^2)),
// plus 2^-20 tau: a block is only dropped when no pixel can contribute.
__device__ __forceinline__ bool box_hits(float mx, float my, float ca, float cb, float cc, float tau, float x0,
                                         float y0, float wx, float wy) {
    const float lx = (x0 + 0.5f) - mx, hx = (x0 + (wx - 0.5f)) - mx;
    const float ly = (y0 + 0.5f) - my, hy = (y0 + (wy - 0.5f)) - my;
    if (lx <= 0.0f && hx >= 0.0f && ly <= 0.0f && hy >= 0.0f) return true;
    const float ica = __builtin_amdgcn_rcpf(ca), icc = __builtin_amdgcn_rcpf(cc);
    float qmin = INFINITY;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float ex = e ? hx : lx;  // vertical edge dx = ex
        const float dy = fminf(fmaxf(-(cb * ex) * icc, ly), hy);
        qmin = fminf(qmin, (ca * ex) * ex + dy * (2.0f * cb * ex + cc * dy));
        const float ey = e ? hy : ly;  // horizontal edge dy = ey
        const float dx = fminf(fmaxf(-(cb * ey) * ica, lx), hx);
        qmin = fminf(qmin, (cc * ey) * ey + dx * (2.0f * cb * ey + ca * dx));
    }
    const float far = ca * fmaxf(lx * lx, hx * hx) + cc * fmaxf(ly * ly, hy * hy);
    return qmin <= tau + 0x1p-18f * far + 0x1p-20f * tau;
}

// Forward: one 256-thread block per tile, walking the tile's slots (one per
// cell that has instances there) in the view's merge order; wave w owns the
// 8x8 quadrant (w & 1, w >> 1) of the tile, one pixel per lane.  Each pixel
// carries P, the product of the T_k of the slots already done: the merged
// transmittance in front of the current cell.  Within a slot, T_k starts at
// 1 and P T_k is the merged transmittance, so a pixel stops (in this cell
// and all later ones) after the contribution that takes P T_k below eps_T:
// the plain render's early termination, which a pixel reaches in the cell
// where it happens, so cells behind an opaque front are not rendered there
// (their partial stays C = 0, T = 1, last = 0).  Records are staged 256 at a
// time in LDS, each with the quadrant mask of its rectangle so that a wave
// skips Gaussians that cannot touch its quadrant with a scalar branch.
template <bool STATS>
__global__ __launch_bounds__(256) void k_render_fwd(const float* __restrict__ rec,
                                                    const uint64_t* __restrict__ vals,
                                                    const uint32_t* __restrict__ slot_key,
                                                    const uint32_t* __restrict__ slot_range,
                                                    const uint32_t* __restrict__ tile_slot,
                                                    const uint32_t* __restrict__ tile_order,
                                                    const ViewTable* __restrict__ vt, const float* __restrict__ box_lo,
                                                    const float* __restrict__ box_hi, float eps_T,
                                                    float* __restrict__ outC, float* __restrict__ outT,
                                                    uint32_t* __restrict__ outLast,
                                                    unsigned long long* __restrict__ stats,
                                                    float* __restrict__ image, float* __restrict__ T_final) {
    constexpr int NB = 256;
    __shared__ float4 sA[NB], sB[NB], sCl[NB];
    __shared__ uint32_t sM[NB];
    __shared__ uint2 sR[NB];
    __shared__ uint32_t s_alive[4];
    __shared__ uint32_t s_live[4];
    const uint32_t gt = tile_order[blockIdx.x];
    const uint32_t s0 = tile_slot[gt], s1 = tile_slot[gt + 1];
    if (s0 >= s1 && !image) return;
    const int L = vt->L, K = 1 << L;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int v = view_of_tile(vt, gt);
    const ViewParams& V = vt->v[v];
    const uint32_t lt = gt - V.tile_offset;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int lx = (w & 1) * 8 + (lane & 7), ly = (w >> 1) * 8 + (lane >> 3);
    const int px = tx * 16 + lx, py = ty * 16 + ly;
    // merged image (image != null): the fold of Eq. 5 over the tile's slots in
    // their order, as the merge does it from the stored partials
    float M0 = 0.f, M1 = 0.f, M2 = 0.f;
    const float fxp = (float)px + 0.5f;
    const float dxp = (fxp - V.cx) / V.fx, dyp = ((float)py + 0.5f - V.cy) / V.fy;
    const float D0 = (V.R[0] * dxp + V.R[3] * dyp) + V.R[6];
    const float D1 = (V.R[1] * dxp + V.R[4] * dyp) + V.R[7];
    const float D2 = (V.R[2] * dxp + V.R[5] * dyp) + V.R[8];
    const float o0 = V.o[0], o1 = V.o[1], o2 = V.o[2];
    // a stopped (or off-image) pixel samples row +inf: d^2 = inf fails every test
    bool live = px < V.W && py < V.H;
    float P = 1.0f;
    uint32_t n_eval = 0u, n_con = 0u;
    const uint32_t qbit = 1u << (w + 1);
    const int p = ly * 16 + lx;

    for (uint32_t slot = s0; slot < s1; ++slot) {
        if (slot > s0) {
            // once every pixel of the tile has stopped, the remaining slots are
            // neutral: written without staging a record (P only decreases, so
            // the tile stays stopped)
            const uint64_t lv = __ballot(live);
            if (lane == 0) s_live[w] = lv != 0ull ? 1u : 0u;
            __syncthreads();
            if ((s_live[0] | s_live[1] | s_live[2] | s_live[3]) == 0u) {
                for (uint32_t sn = slot; sn < s1; ++sn) {
                    float* on = outC + (size_t)sn * 768;
                    on[p] = 0.f;
                    on[256 + p] = 0.f;
                    on[512 + p] = 0.f;
                    outT[(size_t)sn * 256 + p] = 1.f;
                    outLast[(size_t)sn * 256 + p] = 0u;
                }
                break;
            }
        }
        const uint32_t key = slot_key[slot];
        const int cell = V.cell_of_rank[key & ((1u << L) - 1u)];
        const uint32_t begin = slot_range[2 * slot], end = slot_range[2 * slot + 1];
        const float blo0 = box_lo[cell], blo1 = box_lo[K + cell], blo2 = box_lo[2 * K + cell];
        const float bhi0 = box_hi[cell], bhi1 = box_hi[K + cell], bhi2 = box_hi[2 * K + cell];
        // stop once P T < eps_T, i.e. T < eps_T / P (>= eps_T: T stays normal)
        const float thr = live ? eps_T / P : 0.0f;
        float fyp = live ? (float)py + 0.5f : INFINITY;
        float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
        uint32_t last = 0u;
        for (uint32_t base = begin; base < end; base += NB) {
            const uint64_t alive = __ballot(fyp != INFINITY);
            if (lane == 0) s_alive[w] = alive != 0ull ? 1u : 0u;
            const uint32_t idx = base + tid;
            if (idx < end) {
                const uint32_t src = (uint32_t)(vals[idx] >> 32);
                const float4* rp = reinterpret_cast<const float4*>(rec + (size_t)src * RGS_REC_FLOATS);
                const float4 a = rp[0];
                const float4 b = rp[1], cl = rp[2], r4 = rp[3];
                const uint2 rr = make_uint2(__float_as_uint(r4.x), __float_as_uint(r4.y));
                sM[tid] = (quad_mask(rr, tx, ty) << 1) | (__float_as_uint(cl.w) & 1u);
                sA[tid] = a;
                sB[tid] = b;
                sCl[tid] = cl;
                if (STATS) sR[tid] = rr;
            }
            __syncthreads();
            if ((s_alive[0] | s_alive[1] | s_alive[2] | s_alive[3]) == 0u) break;
            const int nb = (int)((end - base) < (uint32_t)NB ? (end - base) : (uint32_t)NB);
            if (alive != 0ull) {
                // Gaussians of this batch whose footprint can reach the wave's
                // quadrant, walked in order (other waves hide the LDS latency);
                // the wave leaves the batch once all its pixels have stopped
#pragma unroll
                for (int k = 0; k < NB / 64; ++k) {
                    if (k > 0 && __ballot(fyp != INFINITY) == 0ull) break;
                    const int tl = k * 64 + lane;
                    const uint32_t mk = tl < nb ? sM[tl] : 0u;
                    uint64_t rel = __ballot((mk & qbit) != 0u);
                    const uint64_t inside = __ballot((mk & 1u) != 0u);  // footprint in one cell: no indicator test
                    while (rel) {
                        const int bit = (int)__builtin_ctzll(rel);
                        const int tc = k * 64 + bit;
                        rel &= rel - 1ull;
                        const float4 ac = sA[tc], bc = sB[tc];
                        const float dx = fxp - ac.x, dy = fyp - ac.y;
                        const float u = fmaf(ac.w, dy, dx);  // d^2 = ca u^2 + e dy^2
                        const float d2 = fmaf(bc.x * dy, dy, (ac.z * u) * u);
                        if (STATS && fyp != INFINITY) {
                            // pairs the method must test: pixel inside the Gaussian's rectangle
                            const uint2 rr = sR[tc];
                            const bool inr = px >= (int)(int16_t)(rr.x & 0xffffu) && px <= (int)(int16_t)(rr.x >> 16) &&
                                             py >= (int)(int16_t)(rr.y & 0xffffu) && py <= (int)(int16_t)(rr.y >> 16);
                            n_eval += inr ? 1u : 0u;
                        }
                        if (!(d2 <= bc.z)) continue;
                        const float4 cl = sCl[tc];
                        if (!((inside >> bit) & 1ull)) {
                            const float x0 = fmaf(bc.w, D0, o0), x1 = fmaf(bc.w, D1, o1), x2 = fmaf(bc.w, D2, o2);
                            const bool in = (blo0 <= x0) && (x0 < bhi0) && (blo1 <= x1) && (x1 < bhi1) && (blo2 <= x2) &&
                                            (x2 < bhi2);
                            if (!in) continue;
                        }
                        if (STATS) ++n_con;
                        const float G = __builtin_amdgcn_exp2f(d2 * -0.72134752044448170368f);  // exp(-d^2/2)
                        const float sg = fminf(0.99f, bc.y * G);
                        const float wgt = sg * T;
                        C0 = fmaf(wgt, cl.x, C0);
                        C1 = fmaf(wgt, cl.y, C1);
                        C2 = fmaf(wgt, cl.z, C2);
                        T = T * (1.0f - sg);
                        last = base - begin + (uint32_t)tc + 1u;
                        if (T < thr) fyp = INFINITY;
                    }
                }
            }
            __syncthreads();
        }
        float* oc = outC + (size_t)slot * 768;
        oc[p] = C0;
        oc[256 + p] = C1;
        oc[512 + p] = C2;
        outT[(size_t)slot * 256 + p] = T;
        outLast[(size_t)slot * 256 + p] = last;
        // the walk stopped in this cell: every later cell is neutral here
        if (live && T < thr) live = false;
        M0 = fmaf(P, C0, M0);
        M1 = fmaf(P, C1, M1);
        M2 = fmaf(P, C2, M2);
        P *= T;
    }
    if (image && px < V.W && py < V.H) {
        const size_t HW = (size_t)V.W * V.H, pix = (size_t)py * V.W + px;
        float* img = image + 3 * (size_t)V.pix_offset;
        img[pix] = fmaf(P, V.bg[0], M0);
        img[HW + pix] = fmaf(P, V.bg[1], M1);
        img[2 * HW + pix] = fmaf(P, V.bg[2], M2);
        T_final[V.pix_offset + pix] = P;
    }
    if (STATS) {
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
}

rgs_status render_fwd_launch(const rgs_projected* proj, const rgs_bins* bins, const ViewTable* vt, const rgs_kdtree* kd,
                             float eps_T, const rgs_partials* out, uint64_t* stats, int64_t total_tiles, hipStream_t s,
                             float* image, float* T_final) {
    if (total_tiles <= 0) return RGS_OK;
    // a pixel stops once its merged transmittance falls below max(eps_T,
    // 2^-100): the backward recovers the transmittance before each
    // contribution from the stored T_k by division, which needs T_k to stay
    // a normal fp32 number (T_k >= 0.01 eps_T / P >= 2^-107)
    eps_T = fmaxf(eps_T, RGS_T_FLOOR);
    if (stats)
        hipLaunchKernelGGL(k_render_fwd<true>, dim3((unsigned)total_tiles), dim3(256), 0, s, proj->rec, bins->vals,
                           bins->slot_key, bins->slot_range, bins->tile_slot, bins->tile_order, vt, kd->box_lo, kd->box_hi,
                           eps_T, out->C, out->T, out->last, reinterpret_cast<unsigned long long*>(stats), image,
                           T_final);
    else
        hipLaunchKernelGGL(k_render_fwd<false>, dim3((unsigned)total_tiles), dim3(256), 0, s, proj->rec, bins->vals,
                           bins->slot_key, bins->slot_range, bins->tile_slot, bins->tile_order, vt, kd->box_lo, kd->box_hi,
                           eps_T, out->C, out->T, out->last, nullptr, image, T_final);
    return launch_check();
}

// ------------------------------------------------------------------ backward
// Sum of g[0..8] over the wave: values 0..7 by reduce-scatter over lane bits
// 5, 4, 3 and a full sum over bits 2, 1, 0, so lane 8v ends with value v;
// value 8 ends in lane 63.  Bits 5 and 4 use the gfx950 lane-swap
// instructions: swapping the upper 32 lanes of x with the lower 32 lanes of y
// leaves, in both outputs, x's half where lane bit 5 is clear and y's half
// where it is set, with the partner lane's copy in the other output, so one
// add reduces over bit 5 without a select; the 16-lane swap does the same for
// bit 4.  Bit 3 is a row rotation by 8 (DPP), bits 2..0 quad permutes and a
// half-row mirror; no exchange goes through LDS.
__device__ __forceinline__ float swap32_sum(float x, float y) {
    const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                                   false, false);
    unsigned a = r[0], b = r[1];
    asm volatile("" : "+v"(a), "+v"(b));  // keeps the two results apart (r[0] + r[1] otherwise folds to 2 r[0])
    return __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
}

__device__ __forceinline__ float swap16_sum(float x, float y) {
    const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                                   false, false);
    unsigned a = r[0], b = r[1];
    asm volatile("" : "+v"(a), "+v"(b));  // keeps the two results apart (r[0] + r[1] otherwise folds to 2 r[0])
    return __builtin_bit_cast(float, a) + __builtin_bit_cast(float, b);
}

// Lane mask of a comparison (the compare writes it to scalar registers).
__device__ __forceinline__ uint64_t wmask(bool p) { return __builtin_amdgcn_ballot_w64(p); }

#define RGS_DPP(v, ctrl) __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, (v)), (ctrl), 0xf, 0xf, false))

__device__ __forceinline__ void wave_sum9(const float* g, int lane, float* out_v, float* out_8) {
    *out_8 = wave_sum_to_lane63(g[8]);
    float q4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q4[k] = swap32_sum(g[k], g[4 + k]);  // bit 5 clear keeps k, set keeps 4 + k
    const float q20 = swap16_sum(q4[0], q4[2]);                      // bit 4 clear keeps 4 h5 + 0, set + 2
    const float q21 = swap16_sum(q4[1], q4[3]);
    const bool h3 = (lane & 8) != 0;
    float q1 = (h3 ? q21 : q20) + RGS_DPP(h3 ? q20 : q21, 0x128);     // row_ror:8 = lane xor 8 within a row
    q1 += RGS_DPP(q1, 0xb1);                                          // quad_perm [1,0,3,2]
    q1 += RGS_DPP(q1, 0x4e);                                          // quad_perm [2,3,0,1]
    q1 += RGS_DPP(q1, 0x141);                                         // row_half_mirror
    *out_v = q1;
}
#undef RGS_DPP

// Backward: 128-thread block per slot.  Wave w owns the 16x8 half (rows
// 8w .. 8w + 7) of the tile and every lane two pixels of one row, eight
// columns apart (quadrants (0, w) and (1, w)): the lane adds its two pixels'
// gradient terms before the cross-lane sum, so one wave sum covers 128
// pixels.  Batches of 64 instances are walked back to front from the block's
// largest `last`; every wave sums each instance's gradient over its 128
// pixels (zero when culled or not contributing) into LDS, and the two half
// sums are added in a fixed order into the instance's record.
struct BwdPix {
    float fx, D0, D1, D2;  // sample x, ray direction
    float T, gB, gC0, gC1, gC2, gTf;
    uint32_t last;
};

// One pixel's share of an instance's gradient.  A pixel that does not
// contribute comes with d^2 = +inf: G = 0 and sigma = 0, so 1 / (1 - sigma) = 1
// exactly, T and <dC, B> stay as they are, and every term returned is zero.
struct PixTerms {
    float q, dsg_g, G, wc;
};

__device__ __forceinline__ PixTerms pix_step(BwdPix& P, float d2, float alpha, float4 cl) {
    PixTerms r;
    r.G = __builtin_amdgcn_exp2f(d2 * -0.72134752044448170368f);  // exp(-d^2/2)
    const float aG = alpha * r.G;
    const float sgm = fminf(0.99f, aG);
    const float rom = __builtin_amdgcn_rcpf(1.0f - sgm);
    const float Tb = P.T * rom;  // transmittance before this contribution
    const float dot = fmaf(P.gC2, cl.z, fmaf(P.gC1, cl.y, P.gC0 * cl.x)) - P.gB;  // <dC, c - B>
    const float dsg = rom * fmaf(P.T, dot, -P.gTf);                               // dL/dsigma
    r.wc = Tb * sgm;
    P.gB = fmaf(sgm, dot, P.gB);  // B <- B + sigma (c - B)
    P.T = Tb;
    // clamped at 0.99: no gradient to alpha or the footprint
    r.dsg_g = aG < 0.99f ? dsg : 0.0f;
    r.q = aG * r.dsg_g;
    return r;
}

template <bool STATS>
__global__ __launch_bounds__(128) void k_render_bwd(const float* __restrict__ rec,
                                                    const uint64_t* __restrict__ vals,
                                                    const uint32_t* __restrict__ slot_key,
                                                    const uint32_t* __restrict__ slot_range,
                                                    const uint32_t* __restrict__ slot_order,
                                                    const uint32_t* __restrict__ n_launch,
                                                    const ViewTable* __restrict__ vt, const float* __restrict__ box_lo,
                                                    const float* __restrict__ box_hi, const float* __restrict__ partT,
                                                    const uint32_t* __restrict__ partLast, const float* __restrict__ dC,
                                                    const float* __restrict__ dT, float* __restrict__ records,
                                                    uint32_t* __restrict__ touched,
                                                    unsigned long long* __restrict__ stats) {
    constexpr int NB = 64;
    __shared__ float4 sA[NB], sB[NB], sCl[NB];
    __shared__ uint2 sR[NB];
    __shared__ uint32_t sJ[NB];
    __shared__ float sG[2][NB][9];
    __shared__ uint32_t s_max[2];
    __shared__ uint64_t s_wrote[2];  // per wave: the batch's instances it wrote half sums for
    if (blockIdx.x >= *n_launch) return;
    const uint32_t slot = slot_order[blockIdx.x];
    const int L = vt->L, K = 1 << L;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t key = slot_key[slot];
    const uint32_t gt = key >> L;
    const int v = view_of_tile(vt, gt);
    const ViewParams& V = vt->v[v];
    const uint32_t lt = gt - V.tile_offset;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int cell = V.cell_of_rank[key & ((1u << L) - 1u)];
    const uint32_t begin = slot_range[2 * slot], end = slot_range[2 * slot + 1];
    const float blo0 = box_lo[cell], blo1 = box_lo[K + cell], blo2 = box_lo[2 * K + cell];
    const float bhi0 = box_hi[cell], bhi1 = box_hi[K + cell], bhi2 = box_hi[2 * K + cell];
    const int lx = lane & 7, ly = w * 8 + (lane >> 3);
    const int py = ty * 16 + ly;
    const float fyp = (float)py + 0.5f;
    const float dyp = (fyp - V.cy) / V.fy;
    const float o0 = V.o[0], o1 = V.o[1], o2 = V.o[2];
    BwdPix P[2];
    int pxs[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int px = tx * 16 + lx + 8 * h;
        pxs[h] = px;
        P[h].fx = (float)px + 0.5f;
        const float dxp = (P[h].fx - V.cx) / V.fx;
        P[h].D0 = (V.R[0] * dxp + V.R[3] * dyp) + V.R[6];
        P[h].D1 = (V.R[1] * dxp + V.R[4] * dyp) + V.R[7];
        P[h].D2 = (V.R[2] * dxp + V.R[5] * dyp) + V.R[8];
        const int p = ly * 16 + lx + 8 * h;
        const bool valid = px < V.W && py < V.H;
        const float Tf = partT[(size_t)slot * 256 + p];
        P[h].T = Tf;
        P[h].last = valid ? partLast[(size_t)slot * 256 + p] : 0u;
        P[h].gTf = valid ? dT[(size_t)slot * 256 + p] * Tf : 0.f;
        P[h].gC0 = valid ? dC[(size_t)slot * 768 + p] : 0.f;
        P[h].gC1 = valid ? dC[(size_t)slot * 768 + 256 + p] : 0.f;
        P[h].gC2 = valid ? dC[(size_t)slot * 768 + 512 + p] : 0.f;
        // gB = <dC_k, B>, where B is the colour blended behind the current
        // instance (the suffix of Eq. 3): the only way B enters the gradient
        P[h].gB = 0.f;
    }
    uint32_t n_eval = 0u, n_con = 0u;
    const uint32_t wmax = wave_max_u32(max(P[0].last, P[1].last));
    if (lane == 0) s_max[w] = wmax;
    __syncthreads();
    const uint32_t bmax = max(s_max[0], s_max[1]);
    // instances behind every pixel's last contributor (k >= bmax) get no
    // record: their bit in `touched` stays clear and the pair reduction
    // counts them as zero
    const float hx0 = (float)(tx * 16), hy0 = (float)(ty * 16 + w * 8);
    for (int bstart = bmax == 0 ? -1 : (int)(((bmax - 1) / NB) * NB); bstart >= 0; bstart -= NB) {
        if (tid < NB && (uint32_t)bstart + tid < bmax) {
            const uint64_t vv = vals[begin + bstart + tid];
            const uint32_t src = (uint32_t)(vv >> 32);
            const float4* rp = reinterpret_cast<const float4*>(rec + (size_t)src * RGS_REC_FLOATS);
            const float4 cl = rp[2];
            const float4 a = rp[0], b = rp[1], r4 = rp[3];
            sA[tid] = a;
            sB[tid] = b;
            sCl[tid] = cl;
            sR[tid] = make_uint2(__float_as_uint(r4.x), __float_as_uint(r4.y));
            sJ[tid] = (uint32_t)vv;
        }
        __syncthreads();
        // Gaussians of this batch below the wave's largest `last` whose
        // footprint can reach the wave's half tile (each wave tests its own
        // half, one record per lane), walked back to front
        const int tl = lane;
        bool hit = (uint32_t)(bstart + tl) + 1u <= wmax && (uint32_t)(bstart + tl) < bmax;
        if (hit) {
            const float4 a = sA[tl], b = sB[tl];
            const float cb = a.w * a.z, cc = b.x + a.w * cb;  // conic from (ca, k, e)
            hit = ((quad_mask(sR[tl], tx, ty) >> (2 * w)) & 3u) &&
                  box_hits(a.x, a.y, a.z, cb, cc, b.z, hx0, hy0, 16.0f, 8.0f);
        }
        uint64_t rel = __ballot(hit);
        uint64_t wrote = 0ull;
        const uint64_t inside = __ballot(hit && (__float_as_uint(sCl[tl].w) & 1u));  // in one cell: no indicator test
        while (rel) {
            const int t = 63 - (int)__builtin_clzll(rel);
            rel &= ~(1ull << t);
            const uint32_t pos1 = (uint32_t)(bstart + t) + 1u;  // this instance's index + 1
            const float4 a = sA[t];
            const float4 b = sB[t];
            const float dy = fyp - a.y;
            const float edy = b.x * dy;
            const float dx0 = P[0].fx - a.x, dx1 = P[1].fx - a.x;
            const float u0 = fmaf(a.w, dy, dx0), u1 = fmaf(a.w, dy, dx1);  // d^2 = ca u^2 + e dy^2
            const float d20 = fmaf(edy, dy, (a.z * u0) * u0), d21 = fmaf(edy, dy, (a.z * u1) * u1);
            // contributing lanes as wave masks: one ballot per comparison (the
            // compare's own lane mask), combined in scalar registers; a lane's
            // flag is read back with an inverse ballot
            uint64_t m0 = wmask(pos1 <= P[0].last) & wmask(d20 <= b.z);
            uint64_t m1 = wmask(pos1 <= P[1].last) & wmask(d21 <= b.z);
            if (STATS) {
                // pairs the backward must re-test: pixel inside the rectangle, at or before its last contributor
                const uint2 rr = sR[t];
                const bool rowin = py >= (int)(int16_t)(rr.y & 0xffffu) && py <= (int)(int16_t)(rr.y >> 16);
                const int xl = (int)(int16_t)(rr.x & 0xffffu), xh = (int)(int16_t)(rr.x >> 16);
                n_eval += (pos1 <= P[0].last && rowin && pxs[0] >= xl && pxs[0] <= xh) ? 1u : 0u;
                n_eval += (pos1 <= P[1].last && rowin && pxs[1] >= xl && pxs[1] <= xh) ? 1u : 0u;
            }
            if ((m0 | m1) == 0ull) continue;
            const float4 cl = sCl[t];
            if (!((inside >> t) & 1ull)) {  // not interior to the cell: the indicator of Eq. 6
                const float x0 = fmaf(b.w, P[0].D0, o0), y0 = fmaf(b.w, P[0].D1, o1), z0 = fmaf(b.w, P[0].D2, o2);
                const float x1 = fmaf(b.w, P[1].D0, o0), y1 = fmaf(b.w, P[1].D1, o1), z1 = fmaf(b.w, P[1].D2, o2);
                m0 &= wmask(blo0 <= x0) & wmask(x0 < bhi0) & wmask(blo1 <= y0) & wmask(y0 < bhi1) & wmask(blo2 <= z0) &
                      wmask(z0 < bhi2);
                m1 &= wmask(blo0 <= x1) & wmask(x1 < bhi0) & wmask(blo1 <= y1) & wmask(y1 < bhi1) & wmask(blo2 <= z1) &
                      wmask(z1 < bhi2);
                if ((m0 | m1) == 0ull) continue;
            }
            const bool c0 = __builtin_amdgcn_inverse_ballot_w64(m0), c1 = __builtin_amdgcn_inverse_ballot_w64(m1);
            if (STATS) n_con += (c0 ? 1u : 0u) + (c1 ? 1u : 0u);
            // a pixel column of the wave where no lane contributes (the
            // instance reaches one quadrant of the half only) is skipped: its
            // step would leave T and <dC, B> as they are and add zeros
            const float d2c0 = c0 ? d20 : INFINITY, d2c1 = c1 ? d21 : INFINITY;
            const bool any0 = m0 != 0ull, any1 = m1 != 0ull;
            PixTerms r0 = {0.f, 0.f, 0.f, 0.f}, r1 = {0.f, 0.f, 0.f, 0.f};
            if (any0) r0 = pix_step(P[0], d2c0, b.y, cl);
            if (any1) r1 = pix_step(P[1], d2c1, b.y, cl);
            // Raw sums over the lane's two pixels; the conic and constant
            // factors are applied per instance after the reduction
            // (dL/d(d^2) = -q / 2)
            float g[9];
            const float qx0 = r0.q * dx0, qx1 = r1.q * dx1;
            g[0] = qx0 + qx1;                      // q dx
            g[1] = (r0.q + r1.q) * dy;             // q dy
            g[2] = fmaf(qx1, dx1, qx0 * dx0);      // q dx^2
            g[3] = g[0] * dy;                      // q dx dy
            g[4] = g[1] * dy;                      // q dy^2
            g[5] = fmaf(r1.dsg_g, r1.G, r0.dsg_g * r0.G);
            g[6] = fmaf(r1.wc, P[1].gC0, r0.wc * P[0].gC0);
            g[7] = fmaf(r1.wc, P[1].gC1, r0.wc * P[0].gC1);
            g[8] = fmaf(r1.wc, P[1].gC2, r0.wc * P[0].gC2);
            float sv, s8;
            wave_sum9(g, lane, &sv, &s8);
            // 32-bit LDS offsets (t * 9 in scalar registers)
            float* const gw = &sG[w][0][0];
            const uint32_t gt = (uint32_t)t * 9u;
            if ((lane & 7) == 0) gw[gt + (uint32_t)(lane >> 3)] = sv;
            if (lane == 63) gw[gt + 8u] = s8;
            wrote |= 1ull << t;
        }
        if (lane == 0) s_wrote[w] = wrote;
        __syncthreads();
        const uint64_t h0 = s_wrote[0], h1 = s_wrote[1];
        // a record for every instance that either half wrote (the others add nothing)
        if (tid < NB && (uint32_t)bstart + tid < bmax && (((h0 | h1) >> tid) & 1ull)) {
            // S_c = sum over the two halves, in a fixed order (a half that
            // wrote nothing adds zero)
            const int t = tid;
            const bool w0 = (h0 >> t) & 1ull, w1 = (h1 >> t) & 1ull;
            float S[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) S[c] = (w0 ? sG[0][t][c] : 0.f) + (w1 ? sG[1][t][c] : 0.f);
            const float4 a = sA[t];
            const float cb = a.w * a.z, cc = sB[t].x + a.w * cb;  // conic from (ca, k, e)
            const uint32_t jr = sJ[t];
            float* rp = records + (size_t)jr * RD_REC;
            atomicOr(&touched[jr >> 5], 1u << (jr & 31u));
            // d mx = sum q (ca dx + cb dy), d my = sum q (cb dx + cc dy); d ca, d cb, d cc
            // carry dL/d(d^2) = -q / 2 (d cb counts the cross term twice); then d alpha, colour
            rp[0] = a.z * S[0] + cb * S[1];
            rp[1] = cb * S[0] + cc * S[1];
            rp[2] = -0.5f * S[2];
            rp[3] = -S[3];
            rp[4] = -0.5f * S[4];
            rp[5] = S[5];
            rp[6] = S[6];
            rp[7] = S[7];
            rp[8] = S[8];
        }
        __syncthreads();
    }
    if (STATS) {
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
}

// Per (view, Gaussian) pair: sum of its instance records.  The records of a
// pair are contiguous (emission order), so the sum is a segmented reduction
// over the instance array, balanced over instances:
//  1. k_pair_seg: a wave takes 64 consecutive records; the pairs covering
//     them come from the wave's first pair (first_pair, written by the
//     backward's records call along with its launch order) and one coalesced
//     load of the next 64 pair offsets; a segmented inclusive scan (fixed tree of
//     shuffles) sums each pair's records within the wave.  The wave's first
//     segment (pair begun before it) and last segment (pair going on after
//     it) are kept as wave partials; every pair gets its psum[rank] entry in
//     the wave where it ends: its sum if it lies in that wave, else the
//     first and last wave it spans (a flag in the entry's last word).
//  2. k_pair_gather: thread per (view, Gaussian): zero if culled, else the
//     pair's psum entry, or, for a pair spanning several waves, its tail
//     partial + whole-wave partials + head partial, in instance order.
// first_pair[w] = the pair holding instance 64 w: each pair writes the waves
// that start inside it (one thread per pair, grid-stride over the device count).
__device__ __forceinline__ void wave_first_pairs(const uint32_t* __restrict__ pair_off,
                                                 const uint32_t* __restrict__ counters,
                                                 uint32_t* __restrict__ first_pair) {
    const int64_t np = counters[0];
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < np; r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t b = pair_off[r], e = pair_off[r + 1];
        for (uint32_t w = (b + 63u) >> 6; (w << 6) < e; ++w) first_pair[w] = (uint32_t)r;
    }
}

__global__ __launch_bounds__(256) void k_wave_first(const uint32_t* __restrict__ pair_off,
                                                    const uint32_t* __restrict__ counters,
                                                    uint32_t* __restrict__ first_pair) {
    wave_first_pairs(pair_off, counters, first_pair);
}

__global__ __launch_bounds__(256) void k_pair_seg(const float* __restrict__ records,
                                                  const uint32_t* __restrict__ touched,
                                                  const uint32_t* __restrict__ pair_off,
                                                  const uint32_t* __restrict__ counters,
                                                  const uint32_t* __restrict__ first_pair, float* __restrict__ psum,
                                                  float* __restrict__ wpart) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t n_pairs = counters[0], n_inst = counters[1];
    const int64_t j0 = w * 64;
    if (j0 >= (int64_t)n_inst) return;  // uniform per wave
    const int64_t j = j0 + lane;
    const bool valid = j < (int64_t)n_inst;
    // the records first (they do not depend on the pair lookup); an instance
    // without a record (behind its tile's last contributors) counts as zero
    float v[9];
    bool has;
    {
        const uint32_t jc = (uint32_t)(valid ? j : (int64_t)n_inst - 1);
        has = valid && ((touched[jc >> 5] >> (jc & 31u)) & 1u);
#pragma unroll
        for (int c = 0; c < 9; ++c) v[c] = 0.f;
        if (has) {
            const float* rp = records + (size_t)jc * RD_REC;
#pragma unroll
            for (int c = 0; c < 9; ++c) v[c] = rp[c];
        }
    }
    const uint32_t r0 = first_pair[w];  // the pair holding instance j0
    // starts of the next 64 pairs (increasing, the tail entry included); pos =
    // how many start at or before j (at most 63: they start after j0)
    const uint32_t rk = r0 + 1u + (uint32_t)lane;
    const int64_t bk = rk <= n_pairs ? (int64_t)pair_off[rk] : INT64_MAX;
    const int64_t b_r0 = (int64_t)pair_off[r0];
    // the lanes where those pairs start, as a lane mask: a start inside the
    // wave (never at its lane 0) sets its lane's byte in the wave's 64 bytes of
    // LDS (starts are distinct; one wave's LDS operations run in order)
    __shared__ uint8_t s_flag[4][64];
    uint8_t* fl = s_flag[threadIdx.x >> 6];
    fl[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    const int64_t dl = bk - j0;
    if (dl > 0 && dl < 64) fl[dl] = 1;
    __builtin_amdgcn_wave_barrier();
    const uint64_t starts = __ballot(fl[lane] != 0);
    const uint64_t le_mask = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const int pos = __popcll(starts & le_mask);  // pairs after r0 starting at or before j
    const uint64_t heads = starts | 1ull;
    const int seg0 = 63 - __builtin_clzll(heads & le_mask);  // first lane of this lane's segment
    // the start and end of this lane's pair, from the starts already loaded
    const int64_t b_at = __shfl(bk, pos > 0 ? pos - 1 : 0, 64);
    const int64_t e_at = __shfl(bk, pos, 64);
    // Segmented inclusive scan: in-row steps by DPP row shifts (1, 2, 4, 8;
    // lanes shifted in from outside the row read 0), then the row broadcasts
    // of lanes 15 and 47 (into rows 1 and 3) and of lane 31 (into rows 2 and
    // 3); a lane only adds values from its own segment.
    const int row = lane >> 4;
#define RGS_SEG_STEP(ctrl, rmask, take)                                                                            \
    {                                                                                                              \
        const bool tk = (take);                                                                                    \
        _Pragma("unroll") for (int c = 0; c < 9; ++c) {                                                            \
            const float u = __builtin_bit_cast(                                                                    \
                float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v[c]), (ctrl), (rmask), 0xf, false)); \
            if (tk) v[c] += u;                                                                                     \
        }                                                                                                          \
    }
    if (__ballot(has) != 0ull) {  // a wave without records sums zeros: no scan
        RGS_SEG_STEP(0x111, 0xf, lane - 1 >= seg0)             // row_shr:1
        RGS_SEG_STEP(0x112, 0xf, lane - 2 >= seg0)             // row_shr:2
        RGS_SEG_STEP(0x114, 0xf, lane - 4 >= seg0)             // row_shr:4
        RGS_SEG_STEP(0x118, 0xf, lane - 8 >= seg0)             // row_shr:8
        RGS_SEG_STEP(0x142, 0xa, (row & 1) && seg0 < 16 * row)  // row_bcast:15
        RGS_SEG_STEP(0x143, 0xc, row >= 2 && seg0 < 32)         // row_bcast:31
    }
#undef RGS_SEG_STEP
    const int pos_next = __shfl_down(pos, 1, 64);
    const bool next_valid = lane < 63 && j + 1 < (int64_t)n_inst;
    const bool seg_end = valid && (!next_valid || pos_next != pos);
    if (!seg_end) return;
    const uint32_t r = r0 + (uint32_t)pos;
    const int64_t pb = pos > 0 ? b_at : b_r0;  // the pair's instances: [pb, e_at)
    const bool began_before = pb < j0;
    const bool goes_on = e_at > j0 + 64;
    const float4 o0 = make_float4(v[0], v[1], v[2], v[3]), o1 = make_float4(v[4], v[5], v[6], v[7]),
                 o2 = make_float4(v[8], 0.f, 0.f, 0.f);
    if (!goes_on) {
        float4* q = reinterpret_cast<float4*>(psum + (size_t)r * PS_REC);
        if (!began_before) {
            q[0] = o0; q[1] = o1; q[2] = o2;
        } else {  // spans waves pb / 64 .. (e_at - 1) / 64: its sum is in the wave partials
            q[2] = make_float4(0.f, __uint_as_float((uint32_t)(pb >> 6)), __uint_as_float((uint32_t)((e_at - 1) >> 6)),
                               __uint_as_float(1u));
        }
    }
    if (began_before) {
        float4* q = reinterpret_cast<float4*>(wpart + ((size_t)w * 2 + 0) * PS_REC);
        q[0] = o0; q[1] = o1; q[2] = o2;
    }
    if (goes_on) {
        float4* q = reinterpret_cast<float4*>(wpart + ((size_t)w * 2 + 1) * PS_REC);
        q[0] = o0; q[1] = o1; q[2] = o2;
    }
}

__device__ __forceinline__ void acc_rec(const float* __restrict__ p, float4& a0, float4& a1, float& a8) {
    const float4* q = reinterpret_cast<const float4*>(p);
    const float4 x = q[0], y = q[1];
    a0.x += x.x; a0.y += x.y; a0.z += x.z; a0.w += x.w;
    a1.x += y.x; a1.y += y.y; a1.z += y.z; a1.w += y.w;
    a8 += q[2].x;
}

__global__ __launch_bounds__(256) void k_pair_gather(const float* __restrict__ psum, const float* __restrict__ wpart,
                                                     const uint32_t* __restrict__ count,
                                                     const int32_t* __restrict__ pair_rank,
                                                     const uint32_t* __restrict__ counters, int64_t m,
                                                     float* __restrict__ dproj) {
    const int64_t sidx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (sidx >= m) return;
    float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0;
    float a8 = 0.f;
    const int32_t r = count[sidx] > 0u ? pair_rank[sidx] : -1;
    if (r >= 0 && (uint32_t)r < counters[0]) {  // a pass that ran out of capacity has no pairs
        const float4* q = reinterpret_cast<const float4*>(psum + (size_t)r * PS_REC);
        const float4 x = q[0], y = q[1], z = q[2];
        if (__float_as_uint(z.w) == 0u) {  // the pair lies in one wave: its sum
            a0 = x;
            a1 = y;
            a8 = z.x;
        } else {
            const uint32_t wb = __float_as_uint(z.y), we = __float_as_uint(z.z);
            // the range the pair reduction wrote lies in the instance array (checked all the same)
            const uint32_t nw = (uint32_t)(((uint64_t)counters[1] + 63u) >> 6);
            if (wb < we && we < nw) {
                acc_rec(wpart + ((size_t)wb * 2 + 1) * PS_REC, a0, a1, a8);  // tail of the first wave
                for (uint32_t w = wb + 1; w < we; ++w) acc_rec(wpart + (size_t)w * 2 * PS_REC, a0, a1, a8);  // whole waves
                acc_rec(wpart + (size_t)we * 2 * PS_REC, a0, a1, a8);       // head of the last wave
            }
        }
    }
    dproj[0 * m + sidx] = a0.x;
    dproj[1 * m + sidx] = a0.y;
    dproj[2 * m + sidx] = a0.z;
    dproj[3 * m + sidx] = a0.w;
    dproj[4 * m + sidx] = a1.x;
    dproj[5 * m + sidx] = a1.y;
    dproj[6 * m + sidx] = a1.z;
    dproj[7 * m + sidx] = a1.w;
    dproj[8 * m + sidx] = a8;
}

// Backward workspace: 36-byte records and 48-byte per-pair sums (pairs <=
// instances <= capacity), two 48-byte partials and the first pair per 64
// instances.
size_t render_bwd_ws_bytes(int64_t capacity) {
    const size_t c = (size_t)(capacity > 0 ? capacity : 1);
    const size_t rec = c * RD_REC * sizeof(float), ps = c * PS_REC * sizeof(float);
    const size_t nw = (c + 63) / 64;
    const size_t wp = nw * 2 * PS_REC * sizeof(float);
    const size_t tw = ((c + 31) / 32 + 64) * sizeof(uint32_t);  // bitmask + launch count
    const size_t tab = (c + SW_SLOTS - 1) / SW_SLOTS * SW_CLS * sizeof(uint32_t);  // launch-order class counts
    return ((rec + 255) & ~size_t(255)) + ((ps + 255) & ~size_t(255)) + ((wp + 255) & ~size_t(255)) +
           ((nw * sizeof(uint32_t) + 255) & ~size_t(255)) + ((tw + 255) & ~size_t(255)) +
           2 * ((c * sizeof(uint32_t) + 255) & ~size_t(255)) + ((tab + 255) & ~size_t(255)) + 256;
}

struct BwdWs {
    float *records, *psum, *wpart;
    uint32_t* first_pair;
    uint32_t* touched;  // bit j: instance j (emission position) has a record
    size_t touched_words;
    uint32_t* wcls;     // the number of slots launched (after the bitmask)
    uint32_t* work;     // per slot: instances the backward visits (its largest `last`)
    uint32_t* order;    // the backward's launch order
    uint32_t* wtab;     // [blocks of SW_SLOTS slots][32] class counts
};

__global__ __launch_bounds__(256) void k_clear_words(uint32_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

static BwdWs carve_bwd(const rgs_bins* bins, void* ws) {
    const size_t c = (size_t)(bins->capacity > 0 ? bins->capacity : 1);
    const size_t rec_bytes = (c * RD_REC * sizeof(float) + 255) & ~size_t(255);
    const size_t ps_bytes = (c * PS_REC * sizeof(float) + 255) & ~size_t(255);
    BwdWs w;
    w.records = reinterpret_cast<float*>(ws);
    w.psum = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + rec_bytes);
    w.wpart = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + rec_bytes + ps_bytes);
    const size_t nw = (c + 63) / 64;
    w.first_pair = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(w.wpart) +
                                               ((nw * 2 * PS_REC * sizeof(float) + 255) & ~size_t(255)));
    w.touched = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(w.first_pair) +
                                            ((nw * sizeof(uint32_t) + 255) & ~size_t(255)));
    w.touched_words = (c + 31) / 32;
    w.wcls = w.touched + w.touched_words;
    const size_t tw = ((c + 31) / 32 + 64) * sizeof(uint32_t);
    w.work = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(w.touched) + ((tw + 255) & ~size_t(255)));
    w.order = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(w.work) + ((c * sizeof(uint32_t) + 255) & ~size_t(255)));
    w.wtab = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(w.order) + ((c * sizeof(uint32_t) + 255) & ~size_t(255)));
    return w;
}

// The backward's launch order: the slots by decreasing size class (half
// octaves, slot_class) of the instances the backward visits (w = the largest `last`
// over the slot's pixels: it walks instances 0 .. w - 1), so that the
// heaviest blocks start first; a slot with w = 0 (no contribution) is not
// launched.  Two passes without global atomics (which serialise on a handful
// of class counters): k_slot_work, SW_SLOTS slots per block, a wave per slot
// at a time (256 `last` values, four per lane), stores w and the block's
// class counts as one row of a table; k_slot_place, the same SW_SLOTS slots
// per block, derives every class's start and the block's offset in it from
// the table and places its slots (the order inside a class is the launch
// order only and affects no result).
static constexpr int SW_CHUNK = 16;  // slots per wave whose loads are issued together
static_assert(SW_SLOTS % (4 * SW_CHUNK) == 0, "a block's four waves take whole chunks");
static_assert(SW_CLS == 32 || SW_CLS == 64 || SW_CLS == 128, "the placement's column sums split 256 threads by class");

// Class of w > 0: 2 floor(log2 w) plus the bit below the leading one (half
// octaves; whole or quarter octaves for 32 or 128 classes).
__device__ __forceinline__ int slot_class(uint32_t w) {
    const int hb = 31 - __clz(w);
    if (SW_CLS == 32) return hb;
    if (SW_CLS == 64) return 2 * hb + (hb > 0 ? (int)((w >> (hb - 1)) & 1u) : 0);
    return 4 * hb + (hb >= 2 ? (int)((w >> (hb - 2)) & 3u) : (hb == 1 ? (int)((w & 1u) << 1) : 0));
}

// Largest u32 of the wave, into lane 63 (DPP row operations, as the sums
// above; a lane a broadcast does not reach keeps its value: max with 0).
__device__ __forceinline__ uint32_t wave_max_to_lane63(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false));  // row_ror:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false));  // row_ror:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// (The same launch clears the record bitmask and writes the pair reduction's
// first pair of every 64 instances, both grid-stride.)
__global__ __launch_bounds__(256) void k_slot_work(const uint32_t* __restrict__ partLast,
                                                   const uint32_t* __restrict__ counters, uint32_t* __restrict__ work,
                                                   uint32_t* __restrict__ wtab, uint32_t* __restrict__ touched,
                                                   int64_t touched_words, const uint32_t* __restrict__ pair_off,
                                                   uint32_t* __restrict__ first_pair) {
    __shared__ uint32_t s_c[SW_CLS];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < touched_words; i += (int64_t)gridDim.x * 256)
        touched[i] = 0u;
    wave_first_pairs(pair_off, counters, first_pair);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x < SW_CLS) s_c[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t ns = (int64_t)counters[2];
    const int64_t base = (int64_t)blockIdx.x * SW_SLOTS + wv * (SW_SLOTS / 4);
    for (int k0 = 0; k0 < SW_SLOTS / 4; k0 += SW_CHUNK) {
        // all loads first (a slot past the count reads slot 0 and is not stored;
        // this launch has at least one slot of capacity)
        uint4 v[SW_CHUNK];
#pragma unroll
        for (int k = 0; k < SW_CHUNK; ++k) {
            const int64_t slot = base + k0 + k;
            v[k] = reinterpret_cast<const uint4*>(partLast + (slot < ns ? slot : 0) * 256)[lane];
        }
#pragma unroll
        for (int k = 0; k < SW_CHUNK; ++k) {
            const int64_t slot = base + k0 + k;
            const uint32_t m = wave_max_to_lane63(max(max(v[k].x, v[k].y), max(v[k].z, v[k].w)));
            if (lane == 63 && slot < ns) {
                work[slot] = m;
                if (m) atomicAdd(&s_c[slot_class(m)], 1u);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < SW_CLS) wtab[(size_t)blockIdx.x * SW_CLS + threadIdx.x] = s_c[threadIdx.x];
}

// n_launch: the number of launched slots (written by block 0).
__global__ __launch_bounds__(256) void k_slot_place(const uint32_t* __restrict__ work,
                                                    const uint32_t* __restrict__ counters,
                                                    const uint32_t* __restrict__ wtab, uint32_t* __restrict__ n_launch,
                                                    uint32_t* __restrict__ order) {
    constexpr int NG = 256 / SW_CLS;  // row groups per class column
    __shared__ uint32_t s_tot[NG][SW_CLS], s_bef[NG][SW_CLS], s_base[SW_CLS], s_c[SW_CLS];
    const int t = threadIdx.x, c = t % SW_CLS, g = t / SW_CLS;
    const int64_t ns = (int64_t)counters[2];
    const int nblk = (int)((ns + SW_SLOTS - 1) / SW_SLOTS);
    {  // the table's column c, rows g, g + NG, ...: all blocks, and the blocks before this one
        uint32_t tot = 0, bef = 0;
        for (int r0 = g; r0 < nblk; r0 += 8 * NG) {
            uint32_t x[8];  // eight loads issued before their adds
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int r = r0 + NG * k;
                x[k] = r < nblk ? wtab[(size_t)r * SW_CLS + c] : 0u;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                tot += x[k];
                bef += r0 + NG * k < (int)blockIdx.x ? x[k] : 0u;
            }
        }
        s_tot[g][c] = tot;
        s_bef[g][c] = bef;
    }
    if (t < SW_CLS) s_c[t] = 0u;
    __syncthreads();
    if (t < SW_CLS) {
        uint32_t tot = 0, bef = 0;
        for (int k = 0; k < NG; ++k) {
            tot += s_tot[k][t];
            bef += s_bef[k][t];
        }
        s_tot[0][t] = tot;
        s_bef[0][t] = bef;
    }
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (int k = SW_CLS - 1; k >= 0; --k) {
            s_base[k] = run + s_bef[0][k];
            run += s_tot[0][k];
        }
        if (blockIdx.x == 0) *n_launch = run;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * SW_SLOTS + t;
    const uint32_t wk = (t < SW_SLOTS && i < ns) ? work[i] : 0u;
    if (wk) {
        const int k = slot_class(wk);
        order[s_base[k] + atomicAdd(&s_c[k], 1u)] = (uint32_t)i;
    }
}

// The partial-render backward alone: per-instance records into the workspace.
rgs_status render_bwd_records_launch(const rgs_partials_grad* dparts, const rgs_partials* parts, const rgs_bins* bins,
                                     const rgs_projected* proj, const ViewTable* vt, const rgs_kdtree* kd, void* ws,
                                     uint64_t* stats, int64_t slot_bound, hipStream_t s) {
    const BwdWs w = carve_bwd(bins, ws);
    // no record yet: the bitmask is cleared by a fill kernel (not a memset:
    // the call may be captured), with the launch order's first pass
    // (and the pair reduction's first pair of every 64 instances, which it
    // reads from this workspace)
    if (slot_bound <= 0) {
        const int64_t nb = ((int64_t)w.touched_words + 255) / 256;
        hipLaunchKernelGGL(k_clear_words, dim3((unsigned)(nb < 1024 ? (nb > 0 ? nb : 1) : 1024)), dim3(256), 0, s,
                           w.touched, (int64_t)w.touched_words);
        const int64_t pb = (bins->capacity + 255) / 256;
        hipLaunchKernelGGL(k_wave_first, dim3((unsigned)(pb < 2048 ? (pb > 0 ? pb : 1) : 2048)), dim3(256), 0, s,
                           bins->pair_off, bins->counters, w.first_pair);
        return launch_check();
    }
    const unsigned nblk = (unsigned)((slot_bound + SW_SLOTS - 1) / SW_SLOTS);
    hipLaunchKernelGGL(k_slot_work, dim3(nblk), dim3(256), 0, s, parts->last, bins->counters, w.work, w.wtab, w.touched,
                       (int64_t)w.touched_words, bins->pair_off, w.first_pair);
    hipLaunchKernelGGL(k_slot_place, dim3(nblk), dim3(256), 0, s, w.work, bins->counters, w.wtab, w.wcls, w.order);
    if (stats)
        hipLaunchKernelGGL(k_render_bwd<true>, dim3((unsigned)slot_bound), dim3(128), 0, s, proj->rec, bins->vals,
                           bins->slot_key, bins->slot_range, w.order, w.wcls, vt, kd->box_lo, kd->box_hi,
                           parts->T, parts->last, dparts->dC, dparts->dT, w.records, w.touched,
                           reinterpret_cast<unsigned long long*>(stats));
    else
        hipLaunchKernelGGL(k_render_bwd<false>, dim3((unsigned)slot_bound), dim3(128), 0, s, proj->rec, bins->vals,
                           bins->slot_key, bins->slot_range, w.order, w.wcls, vt, kd->box_lo, kd->box_hi,
                           parts->T, parts->last, dparts->dC, dparts->dT, w.records, w.touched, nullptr);
    return launch_check();
}

// The per-pair sums of the records in the workspace.
rgs_status pair_reduce_launch(const rgs_bins* bins, const rgs_projected* proj, int64_t n, int n_views, float* dproj,
                              void* ws, hipStream_t s) {
    const BwdWs w = carve_bwd(bins, ws);
    const int64_t m = (int64_t)n_views * n;
    // one wave per 64 instances up to the capacity; waves past the device-side
    // instance count return at once
    // (the records call wrote first_pair)
    if (bins->capacity > 0) {
        hipLaunchKernelGGL(k_pair_seg, dim3((unsigned)((bins->capacity + 255) / 256)), dim3(256), 0, s, w.records,
                           w.touched, bins->pair_off, bins->counters, w.first_pair, w.psum, w.wpart);
    }
    RGS_LAUNCH_CHECK();
    if (m > 0)
        hipLaunchKernelGGL(k_pair_gather, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, w.psum, w.wpart,
                           proj->count, bins->pair_rank, bins->counters, m, dproj);
    return launch_check();
}

}  // namespace rgs
