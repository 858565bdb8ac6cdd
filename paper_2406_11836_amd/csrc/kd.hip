// kd.hip -- KD-tree partition of the Gaussian centres (RetinaGS Sec. 3.3).
//
// Level by level, every node's split is the floor(n/2)-th smallest centre
// coordinate (IEEE total order) on axis depth mod 3, found exactly by a radix
// select over the 32 key bits, 8 bits per pass: each pass histograms the
// digit of the members still matching the selected prefix, per node, and one
// thread per node picks the digit holding the target rank.  Members are then
// moved to the child (coordinate < split: left).  Leaf boxes are the
// intersections of the half-spaces along each root-to-leaf path.
//
// The fixed-size partition the paper compares against (Sec. 4.2, Table 2)
// uses the same tree with every node cut at the midpoint of its extent,
// starting from the bounding box of the centres: the leaves form a uniform
// grid.
#include "common.hpp"

namespace rgs {

static constexpr int KD_THREADS = 256;

struct KdState {        // per node of the current level
    uint32_t prefix;    // selected high bits of the split key
    uint32_t mask;      // which bits are selected
    uint32_t k;         // rank still to find among members matching prefix
    uint32_t n;         // members of the node
};

__global__ __launch_bounds__(KD_THREADS) void k_kd_init(int32_t* __restrict__ node, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * KD_THREADS + threadIdx.x;
    if (i < n) node[i] = 0;
}

// hist[(node - first) * 256 + digit] over members whose key matches the node's prefix.
__global__ __launch_bounds__(KD_THREADS) void k_kd_hist(const float* __restrict__ coord, const int32_t* __restrict__ node,
                                                        int64_t n, int first, int cnt, const KdState* __restrict__ st,
                                                        int shift, uint32_t* __restrict__ hist) {
    extern __shared__ uint32_t s_h[];  // [cnt][256]
    for (int k = threadIdx.x; k < cnt * 256; k += KD_THREADS) s_h[k] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * KD_THREADS;
    for (int64_t i = (int64_t)blockIdx.x * KD_THREADS + threadIdx.x; i < n; i += stride) {
        const int nd = node[i] - first;
        const uint32_t key = f2key(coord[i]);
        const KdState s = st[nd];
        if ((key & s.mask) == s.prefix) atomicAdd(&s_h[nd * 256 + ((key >> shift) & 0xffu)], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < cnt * 256; k += KD_THREADS)
        if (s_h[k]) atomicAdd(&hist[k], s_h[k]);
}

__global__ void k_kd_state_init(KdState* __restrict__ st, int cnt) {
    int t = threadIdx.x;
    if (t < cnt) st[t] = KdState{0u, 0u, 0u, 0u};
}

__global__ void k_kd_zero(uint32_t* __restrict__ p, int m) {
    for (int k = threadIdx.x + blockIdx.x * blockDim.x; k < m; k += blockDim.x * gridDim.x) p[k] = 0;
}

__global__ void k_kd_fill_ones(uint32_t* __restrict__ p, int m) {
    for (int k = threadIdx.x + blockIdx.x * blockDim.x; k < m; k += blockDim.x * gridDim.x) p[k] = 0xffffffffu;
}

// One thread per node: pick the digit containing rank k.
__global__ void k_kd_select(KdState* __restrict__ st, const uint32_t* __restrict__ hist, int cnt, int shift, int pass) {
    int t = threadIdx.x;
    if (t >= cnt) return;
    KdState s = st[t];
    const uint32_t* h = hist + t * 256;
    if (pass == 0) {
        uint32_t tot = 0;
        for (int d = 0; d < 256; ++d) tot += h[d];
        s.n = tot;
        s.k = tot / 2;
    }
    if (s.n == 0) { st[t] = s; return; }
    uint32_t cum = 0;
    int dsel = 255;
    for (int d = 0; d < 256; ++d) {
        if (cum + h[d] > s.k) { dsel = d; break; }
        cum += h[d];
    }
    s.k -= cum;
    s.prefix |= (uint32_t)dsel << shift;
    s.mask |= 0xffu << shift;
    st[t] = s;
}

// Node bounds along the path (for empty nodes, or for every node under the
// grid rule, starting from the centres' bounding box) and the split value.
__global__ void k_kd_finish_level(const KdState* __restrict__ st, float* __restrict__ split, int first, int cnt,
                                  int level, const uint32_t* __restrict__ root_key) {
    int t = threadIdx.x;
    if (t >= cnt) return;
    const int nd = first + t;
    const int a = level % 3;
    float s;
    if (root_key) {
        // grid rule: midpoint of the node's extent inside the bounding box
        const uint32_t klo = root_key[a], khi = root_key[3 + a];
        float lo = klo == 0xffffffffu ? INFINITY : key2f(klo), hi = khi == 0u ? -INFINITY : key2f(khi);
        int c = nd;
        while (c > 0) {
            const int p = (c - 1) >> 1;
            const int dp = 31 - __builtin_clz((unsigned)(p + 1));  // depth of p
            if (dp % 3 == a) {
                if (c == 2 * p + 1) { if (split[p] < hi) hi = split[p]; }
                else { if (split[p] > lo) lo = split[p]; }
            }
            c = p;
        }
        s = (isfinite(lo) && isfinite(hi)) ? 0.5f * (lo + hi) : 0.0f;
    } else if (st[t].n > 0) {
        s = key2f(st[t].prefix);
    } else {
        float lo = -INFINITY, hi = INFINITY;
        int c = nd, d = level;
        while (c > 0) {
            int p = (c - 1) >> 1;
            --d;
            if (d % 3 == a) {
                if (c == 2 * p + 1) { if (split[p] < hi) hi = split[p]; }
                else { if (split[p] > lo) lo = split[p]; }
            }
            c = p;
        }
        if (isfinite(lo) && isfinite(hi)) s = 0.5f * (lo + hi);
        else if (isfinite(lo)) s = lo;
        else if (isfinite(hi)) s = hi;
        else s = 0.0f;
    }
    split[nd] = s;
}

// Bounding box of the centres as IEEE total-order keys: min of x, y, z then max.
__global__ __launch_bounds__(KD_THREADS) void k_kd_root_box(const float* __restrict__ means, int64_t n,
                                                            uint32_t* __restrict__ key) {
    __shared__ uint32_t s_k[6];
    if (threadIdx.x < 6) s_k[threadIdx.x] = threadIdx.x < 3 ? 0xffffffffu : 0u;
    __syncthreads();
    uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * KD_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * KD_THREADS)
        for (int a = 0; a < 3; ++a) {
            const uint32_t k = f2key(means[a * n + i]);
            mn[a] = min(mn[a], k);
            mx[a] = max(mx[a], k);
        }
    for (int a = 0; a < 3; ++a) {
        mn[a] = ~wave_max_u32(~mn[a]);
        mx[a] = wave_max_u32(mx[a]);
    }
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            atomicMin(&s_k[a], mn[a]);
            atomicMax(&s_k[3 + a], mx[a]);
        }
    __syncthreads();
    if (threadIdx.x < 3) atomicMin(&key[threadIdx.x], s_k[threadIdx.x]);
    else if (threadIdx.x < 6) atomicMax(&key[threadIdx.x], s_k[threadIdx.x]);
}

__global__ __launch_bounds__(KD_THREADS) void k_kd_assign(const float* __restrict__ coord, int32_t* __restrict__ node,
                                                          int64_t n, const float* __restrict__ split) {
    int64_t i = (int64_t)blockIdx.x * KD_THREADS + threadIdx.x;
    if (i >= n) return;
    const int nd = node[i];
    node[i] = (coord[i] < split[nd]) ? 2 * nd + 1 : 2 * nd + 2;
}

__global__ void k_kd_boxes(const float* __restrict__ split, int L, float* __restrict__ lo, float* __restrict__ hi,
                           int32_t* __restrict__ counts) {
    const int K = 1 << L;
    int k = threadIdx.x;
    if (k >= K) return;
    float l[3] = {-INFINITY, -INFINITY, -INFINITY}, h[3] = {INFINITY, INFINITY, INFINITY};
    int nd = 0;
    for (int d = 0; d < L; ++d) {
        const int a = d % 3;
        const int right = (k >> (L - 1 - d)) & 1;
        if (right) { l[a] = split[nd]; nd = 2 * nd + 2; }
        else { h[a] = split[nd]; nd = 2 * nd + 1; }
    }
    for (int a = 0; a < 3; ++a) {
        lo[a * K + k] = l[a];
        hi[a * K + k] = h[a];
    }
    counts[k] = 0;
}

// Leaf of every centre, per-leaf counts, ownership masks and per-leaf
// bounds (the box of the centres and the largest scale).  Grid-stride
// blocks: counts and bounds are reduced in LDS (integer keys, so min/max are
// exact and order-independent) and each block issues one global atomic per
// (leaf, bound) it touched.
static constexpr int KD_LEAF_BLOCKS = 1024;

__global__ __launch_bounds__(KD_THREADS) void k_kd_leaves(const int32_t* __restrict__ node, int64_t n, int L,
                                                          const float* __restrict__ means,
                                                          const float* __restrict__ log_scales, float d_factor,
                                                          const float* __restrict__ lo, const float* __restrict__ hi,
                                                          int32_t* __restrict__ center_cell, int32_t* __restrict__ counts,
                                                          uint32_t* __restrict__ own_mask, uint32_t* __restrict__ bounds_key) {
    __shared__ int32_t s_cnt[RGS_MAXK];
    __shared__ uint32_t s_bk[7 * RGS_MAXK];
    const int K = 1 << L;
    for (int t = threadIdx.x; t < K; t += KD_THREADS) s_cnt[t] = 0;
    for (int t = threadIdx.x; t < 7 * K; t += KD_THREADS) s_bk[t] = (t < 3 * K) ? 0xffffffffu : 0u;
    __syncthreads();
    const int Wm = (K + 31) / 32;
    for (int64_t i = (int64_t)blockIdx.x * KD_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * KD_THREADS) {
        const int leaf = node[i] - (K - 1);
        atomicAdd(&s_cnt[leaf], 1);
        center_cell[i] = leaf;
        if (!own_mask && !bounds_key) continue;
        // D_i = d_factor * max scale; transcendental in fp64, rounded once
        const float s0 = (float)exp((double)log_scales[i]);
        const float s1 = (float)exp((double)log_scales[n + i]);
        const float s2 = (float)exp((double)log_scales[2 * n + i]);
        const float smax = fmaxf(fmaxf(s0, s1), s2);
        const float Di = d_factor * smax;
        const float u[3] = {means[i], means[n + i], means[2 * n + i]};
        if (bounds_key) {
            for (int a = 0; a < 3; ++a) {
                atomicMin(&s_bk[a * K + leaf], f2key(u[a]));
                atomicMax(&s_bk[(3 + a) * K + leaf], f2key(u[a]));
            }
            atomicMax(&s_bk[6 * K + leaf], f2key(smax));
        }
        if (!own_mask) continue;
        uint32_t m[2] = {0u, 0u};
        for (int k = 0; k < K; ++k) {
            bool in = true;
            for (int a = 0; a < 3; ++a) {
                if (!((lo[a * K + k] - u[a]) <= Di)) in = false;
                if (!((u[a] - hi[a * K + k]) <= Di)) in = false;
            }
            if (in) m[k >> 5] |= 1u << (k & 31);
        }
        for (int w = 0; w < Wm; ++w) own_mask[i * Wm + w] = m[w];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < K; t += KD_THREADS)
        if (s_cnt[t]) atomicAdd(&counts[t], s_cnt[t]);
    if (bounds_key)
        for (int t = threadIdx.x; t < 7 * K; t += KD_THREADS) {
            const uint32_t v = s_bk[t];
            if (t < 3 * K) {
                if (v != 0xffffffffu) atomicMin(&bounds_key[t], v);
            } else if (v != 0u) {
                atomicMax(&bounds_key[t], v);
            }
        }
}

__global__ void k_kd_bounds_init(uint32_t* __restrict__ bk, int K) {
    int t = threadIdx.x;
    if (t < 7 * K) bk[t] = (t < 3 * K) ? 0xffffffffu : 0u;
}

// cell_bounds rows: min x, y, z; max x, y, z of the centres (+inf / -inf for an
// empty cell); the largest scale exp(log_scale) of the cell (0 if empty); 0.
__global__ void k_kd_bounds_final(const uint32_t* __restrict__ bk, int K, float* __restrict__ bounds) {
    int t = threadIdx.x;
    if (t >= 8 * K) return;
    if (t >= 7 * K) { bounds[t] = 0.0f; return; }
    const uint32_t k = bk[t];
    if (t < 3 * K) bounds[t] = (k == 0xffffffffu) ? INFINITY : key2f(k);
    else if (t < 6 * K) bounds[t] = (k == 0u) ? -INFINITY : key2f(k);
    else bounds[t] = (k == 0u) ? 0.0f : key2f(k);
}

size_t kd_ws_bytes(int64_t n, int L) {
    const int K = 1 << L;
    return (size_t)n * sizeof(int32_t) + 256 + (size_t)K * 256 * sizeof(uint32_t) + 256 + (size_t)K * sizeof(KdState) + 256 +
           (size_t)7 * K * sizeof(uint32_t) + 256 + 6 * sizeof(uint32_t) + 256;
}

rgs_status kd_partition(const rgs_gaussians* g, int L, float d_factor, int rule, const rgs_kdtree* kd, void* ws,
                        hipStream_t s) {
    const int64_t n = g->n;
    const int K = 1 << L;
    WsCarver c{reinterpret_cast<char*>(ws), 0, (size_t)-1};
    int32_t* node = c.take<int32_t>(n > 0 ? n : 1);
    uint32_t* hist = c.take<uint32_t>((size_t)K * 256);
    KdState* st = c.take<KdState>(K);
    uint32_t* bk = c.take<uint32_t>((size_t)7 * K);
    uint32_t* root = c.take<uint32_t>(6);
    const unsigned gridN = (unsigned)((n + KD_THREADS - 1) / KD_THREADS);
    if (n > 0) hipLaunchKernelGGL(k_kd_init, dim3(gridN), dim3(KD_THREADS), 0, s, node, n);
    int hist_blocks = (int)((n + KD_THREADS * 16 - 1) / (KD_THREADS * 16));
    if (hist_blocks < 1) hist_blocks = 1;
    if (hist_blocks > 4096) hist_blocks = 4096;
    const bool grid = rule == RGS_SPLIT_MIDPOINT;
    if (grid) {
        // min keys start at all ones, max keys at zero
        hipLaunchKernelGGL(k_kd_fill_ones, dim3(1), dim3(64), 0, s, root, 3);
        hipLaunchKernelGGL(k_kd_zero, dim3(1), dim3(64), 0, s, root + 3, 3);
        if (n > 0) hipLaunchKernelGGL(k_kd_root_box, dim3(hist_blocks), dim3(KD_THREADS), 0, s, g->means, n, root);
    }
    for (int l = 0; l < L; ++l) {
        const int first = (1 << l) - 1, cnt = 1 << l;
        const float* coord = g->means + (int64_t)(l % 3) * n;
        if (!grid) {
            hipLaunchKernelGGL(k_kd_state_init, dim3(1), dim3(64), 0, s, st, cnt);
            for (int p = 0; p < 4; ++p) {
                const int shift = 24 - 8 * p;
                hipLaunchKernelGGL(k_kd_zero, dim3(16), dim3(256), 0, s, hist, cnt * 256);
                if (n > 0)
                    hipLaunchKernelGGL(k_kd_hist, dim3(hist_blocks), dim3(KD_THREADS), cnt * 256 * sizeof(uint32_t), s,
                                       coord, node, n, first, cnt, st, shift, hist);
                hipLaunchKernelGGL(k_kd_select, dim3(1), dim3(64), 0, s, st, hist, cnt, shift, p);
            }
        }
        hipLaunchKernelGGL(k_kd_finish_level, dim3(1), dim3(64), 0, s, st, kd->split, first, cnt, l,
                           grid ? root : nullptr);
        if (n > 0) hipLaunchKernelGGL(k_kd_assign, dim3(gridN), dim3(KD_THREADS), 0, s, coord, node, n, kd->split);
        RGS_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_kd_boxes, dim3(1), dim3(64), 0, s, kd->split, L, kd->box_lo, kd->box_hi, kd->counts);
    if (kd->cell_bounds) hipLaunchKernelGGL(k_kd_bounds_init, dim3(1), dim3(448), 0, s, bk, K);
    const unsigned gridL = gridN < (unsigned)KD_LEAF_BLOCKS ? gridN : (unsigned)KD_LEAF_BLOCKS;
    if (n > 0)
        hipLaunchKernelGGL(k_kd_leaves, dim3(gridL), dim3(KD_THREADS), 0, s, node, n, L, g->means, g->log_scales, d_factor,
                           kd->box_lo, kd->box_hi, kd->center_cell, kd->counts, kd->own_mask,
                           kd->cell_bounds ? bk : nullptr);
    if (kd->cell_bounds) hipLaunchKernelGGL(k_kd_bounds_final, dim3(1), dim3(512), 0, s, bk, K, kd->cell_bounds);
    return launch_check();
}

}  // namespace rgs
