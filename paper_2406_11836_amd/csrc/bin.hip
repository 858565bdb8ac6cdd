// bin.hip -- tile/cell instance lists, depth order and slot table.
//
// 1. The visible (view, Gaussian) pairs are compacted in (view, gid) order
//    and sorted stably by the fp32 bits of their camera depth (positive
//    floats order like their bits), then by view: (view, z, gid) order.
// 2. Each pair emits, contiguously and in that order, one instance per
//    (cell of its cell set, tile of its rectangle that the footprint can
//    reach: the row spans of the projection), keyed
//    (global tile << L) | rank of the cell in the view's merge order.
// 3. A stable LSD radix sort on the key alone keeps every (tile, cell)
//    group in depth order, so the sort never looks at the depth bits.
// 4. Slot boundaries are found on a dense (tile, rank) table, compacted by a
//    scan; the slots of a tile come out contiguous and in merge order.
#include "common.hpp"

namespace rgs {

static constexpr int BN_THREADS = 256;

// Visible-pair compaction in (view, gid) order: VC_TILE consecutive entries
// per block; the counts are read twice (tile sums, then the ordered write),
// 8 bytes per (view, Gaussian) entry in all.
static constexpr int VC_ITEMS = 16;
static constexpr int VC_TILE = BN_THREADS * VC_ITEMS;

__global__ __launch_bounds__(BN_THREADS) void k_vis_count(const uint32_t* __restrict__ count, int64_t m,
                                                          uint32_t* __restrict__ tile_sum) {
    __shared__ uint32_t s_w[4];
    const int64_t base = (int64_t)blockIdx.x * VC_TILE;
    // all loads first (a lane past the end reads the last entry and counts nothing)
    uint32_t cv[VC_ITEMS];
#pragma unroll
    for (int k = 0; k < VC_ITEMS; ++k) {
        const int64_t i = base + k * BN_THREADS + threadIdx.x;
        cv[k] = count[i < m ? i : m - 1];
    }
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < VC_ITEMS; ++k) c += (base + k * BN_THREADS + threadIdx.x < m && cv[k] != 0u) ? 1u : 0u;
    c = wave_sum_u32(c);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

// Entry i = base + k * 256 + t is the k-th item of thread t, so index order is
// (k, wave, lane) order: one exclusive scan over the 64 (k, wave) ballot
// counts gives every wave's offset for every k.
// fold = 1: tile_off holds the tile counts unscanned; the block sums those
// before its tile (few tiles) and the last block writes the pair count.
__global__ __launch_bounds__(BN_THREADS) void k_vis_compact(const uint32_t* __restrict__ count,
                                                            const float* __restrict__ depth, int64_t m,
                                                            const uint32_t* __restrict__ tile_off, int fold,
                                                            uint32_t* __restrict__ n_pairs,
                                                            uint32_t* __restrict__ zkey, uint32_t* __restrict__ src_out) {
    __shared__ uint32_t s_c[VC_ITEMS * 4];
    __shared__ uint32_t s_r[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * VC_TILE;
    uint32_t fl = 0;
    uint32_t cv[VC_ITEMS];
#pragma unroll
    for (int k = 0; k < VC_ITEMS; ++k) {
        const int64_t i = base + k * BN_THREADS + threadIdx.x;
        cv[k] = count[i < m ? i : m - 1];
    }
#pragma unroll
    for (int k = 0; k < VC_ITEMS; ++k) {
        const int64_t i = base + k * BN_THREADS + threadIdx.x;
        const bool f = i < m && cv[k] != 0u;
        fl |= (f ? 1u : 0u) << k;
        const uint64_t b = __ballot(f);
        if (lane == 0) s_c[k * 4 + w] = (uint32_t)__popcll(b);
    }
    __syncthreads();
    if (w == 0) {
        const uint32_t v = s_c[lane];
        const uint32_t inc = wave_incl_scan(v);
        s_c[lane] = inc - v;  // lane = k * 4 + wave: every lane read its value before any write
    }
    __syncthreads();
    uint32_t t0;
    if (fold) {
        uint32_t a = 0;
        for (uint32_t t = threadIdx.x; t < blockIdx.x; t += BN_THREADS) a += tile_off[t];
        a = wave_sum_u32(a);
        if (lane == 0) s_r[w] = a;
        __syncthreads();
        t0 = (s_r[0] + s_r[1]) + (s_r[2] + s_r[3]);
        if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *n_pairs = t0 + tile_off[blockIdx.x];
    } else {
        t0 = tile_off[blockIdx.x];
    }
    // the depths of the kept entries, all loads before the stores
    float dv[VC_ITEMS];
#pragma unroll
    for (int k = 0; k < VC_ITEMS; ++k) {
        const int64_t i = base + k * BN_THREADS + threadIdx.x;
        dv[k] = ((fl >> k) & 1u) ? depth[i] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < VC_ITEMS; ++k) {
        const bool f = (fl >> k) & 1u;
        const uint64_t b = __ballot(f);
        if (f) {
            const int64_t i = base + k * BN_THREADS + threadIdx.x;
            const uint32_t p = t0 + s_c[k * 4 + w] + (uint32_t)__popcll(b & lt_mask);
            zkey[p] = __float_as_uint(dv[k]);
            src_out[p] = (uint32_t)i;
        }
    }
}

__global__ __launch_bounds__(BN_THREADS) void k_view_keys(const uint32_t* __restrict__ src, const uint32_t* __restrict__ n_dev,
                                                          int64_t n_gauss, uint32_t* __restrict__ vkey) {
    const int64_t np = (int64_t)*n_dev;
    for (int64_t i = (int64_t)blockIdx.x * BN_THREADS + threadIdx.x; i < np; i += (int64_t)gridDim.x * BN_THREADS)
        vkey[i] = (uint32_t)(src[i] / (uint64_t)n_gauss);
}

// Per ordered pair: its rank, and its instance count (for the offsets scan).
// A block takes RGS_SCAN_TILE consecutive pairs, a tile of that scan, and
// writes the tile's count sum to tsum[tile], so the scan skips its reduce
// pass.  All blocks also fill the slot table's empty marks.
static constexpr int PC_ITEMS = (int)(RGS_SCAN_TILE / BN_THREADS);
static_assert(PC_ITEMS * BN_THREADS == RGS_SCAN_TILE, "a block covers one scan tile");

__global__ __launch_bounds__(BN_THREADS) void k_pair_counts(const uint32_t* __restrict__ pair_src,
                                                            const uint32_t* __restrict__ n_dev,
                                                            const uint32_t* __restrict__ count,
                                                            int32_t* __restrict__ pair_rank, uint32_t* __restrict__ cnt,
                                                            uint32_t* __restrict__ tsum, uint32_t* __restrict__ fill,
                                                            int64_t n_fill) {
    __shared__ uint32_t s_w[BN_THREADS / 64];
    const int64_t np = (int64_t)*n_dev;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t tile = blockIdx.x; tile * RGS_SCAN_TILE < np; tile += gridDim.x) {
        const int64_t base = tile * RGS_SCAN_TILE;
        // all loads first (a lane past the end reads the last pair and adds nothing)
        uint32_t sv[PC_ITEMS], cv[PC_ITEMS];
#pragma unroll
        for (int k = 0; k < PC_ITEMS; ++k) {
            const int64_t i = base + k * BN_THREADS + threadIdx.x;
            sv[k] = pair_src[i < np ? i : np - 1];
        }
#pragma unroll
        for (int k = 0; k < PC_ITEMS; ++k) cv[k] = count[sv[k]];
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < PC_ITEMS; ++k) {
            const int64_t i = base + k * BN_THREADS + threadIdx.x;
            if (i < np) {
                pair_rank[sv[k]] = (int32_t)i;
                cnt[i] = cv[k];
                acc += cv[k];
            }
        }
        acc = wave_sum_u32(acc);
        if (lane == 0) s_w[w] = acc;
        __syncthreads();
        if (threadIdx.x == 0) tsum[tile] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
        __syncthreads();  // s_w is reused by the next tile
    }
    // the slot table's empty marks, needed after the instance sort
    for (int64_t i = (int64_t)blockIdx.x * BN_THREADS + threadIdx.x; i < n_fill; i += (int64_t)gridDim.x * BN_THREADS)
        fill[i] = 0xffffffffu;
}

// Position of the c-th set bit (0-based) of a 64-bit mask.
__device__ __forceinline__ int nth_set_bit(uint64_t m, int c) {
    const int lo = __popc((uint32_t)m);
    int base = 0;
    uint32_t w = (uint32_t)m;
    if (c >= lo) { c -= lo; w = (uint32_t)(m >> 32); base = 32; }
    for (int k = 0; k < c; ++k) w &= w - 1u;
    return base + __ffs(w) - 1;
}

// a / b for a, b < 2^24: float estimate, then exact integer correction.
__device__ __forceinline__ uint32_t udiv_small(uint32_t a, uint32_t b) {
    uint32_t q = (uint32_t)((float)a * __builtin_amdgcn_rcpf((float)b));
    while (q * b > a) --q;
    while ((q + 1u) * b <= a) ++q;
    return q;
}

// Instance emission, balanced over instances: a block takes 256 consecutive
// ordered pairs, stages their offsets in LDS and walks the block's instances
// in chunks of 256; each thread finds its pair by binary search and decodes
// (cell, tile) from the index inside the pair (cells ascending, then the row
// spans' tiles top to bottom, left to right), so writes are coalesced
// whatever the per-pair counts.  Small rectangles carry their spans in the
// record's descriptor.  For larger ones the block computes each row's span
// once, rows spread over the threads, into an LDS pool with per-pair running
// sums, and an instance finds its row by binary search; when a chunk's large
// rectangles hold more rows than the pool, the chunk is taken in runs of
// consecutive pairs whose rows fit.
__global__ __launch_bounds__(BN_THREADS) void k_emit(const uint32_t* __restrict__ pair_src, const uint32_t* __restrict__ n_dev,
                                                     const uint32_t* __restrict__ pair_off, const float* __restrict__ rec,
                                                     const uint32_t* __restrict__ bin, int64_t n_gauss,
                                                     const ViewTable* __restrict__ vt, uint32_t* __restrict__ keys,
                                                     uint64_t* __restrict__ vals) {
    constexpr int ROWPOOL = 2048;  // rows of one run; a rectangle has at most 256 tile rows
    __shared__ uint32_t s_off[BN_THREADS + 1];
    __shared__ uint32_t s_src[BN_THREADS];
    __shared__ uint64_t s_mask[BN_THREADS];
    __shared__ uint64_t s_desc[BN_THREADS];  // row-span descriptor, or RGS_NO_SPANS
    __shared__ uint2 s_rect[BN_THREADS];     // packed rectangle of the record
    // per pair: tiles per cell, the view's first global tile and tiles per row
    __shared__ uint32_t s_nt[BN_THREADS], s_vto[BN_THREADS], s_vtx[BN_THREADS];
    __shared__ uint8_t s_view[BN_THREADS];
    __shared__ uint32_t s_rows[BN_THREADS], s_rend[BN_THREADS];  // pooled rows per pair, inclusive scan
    __shared__ uint32_t s_rcum[ROWPOOL];  // a row's tile count, then the pair's running sum
    __shared__ int16_t s_rc0[ROWPOOL];    // the row's first tile column
    __shared__ uint32_t s_wsum[BN_THREADS / 64];
    const int64_t npairs = (int64_t)*n_dev;
    const int L = vt->L;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int64_t r0 = (int64_t)blockIdx.x * BN_THREADS; r0 < npairs; r0 += (int64_t)gridDim.x * BN_THREADS) {
        const int nb = (int)((npairs - r0) < BN_THREADS ? (npairs - r0) : BN_THREADS);
        uint32_t rows = 0;
        if (t < nb) {
            const uint32_t src = pair_src[r0 + t];
            // the pair's binning record: one 32-byte line
            const uint4* bp = reinterpret_cast<const uint4*>(bin) + 2 * (size_t)src;
            const uint4 b0 = bp[0], b1 = bp[1];
            const int v = (int)(src / (uint64_t)n_gauss);  // once per pair
            const ViewParams& V = vt->v[v];
            const uint64_t desc = (uint64_t)b0.z | ((uint64_t)b0.w << 32);
            const uint32_t ry = b0.y;
            s_src[t] = src;
            s_mask[t] = (uint64_t)b1.x | ((uint64_t)b1.y << 32);
            s_nt[t] = b1.w;
            s_rect[t] = make_uint2(b0.x, ry);
            s_desc[t] = desc;
            s_off[t] = pair_off[r0 + t];
            s_vto[t] = V.tile_offset;
            s_vtx[t] = (uint32_t)V.tiles_x;
            s_view[t] = (uint8_t)v;
            if (desc == RGS_NO_SPANS)
                rows = (uint32_t)(((int)(int16_t)(ry >> 16) >> 4) - ((int)(int16_t)(ry & 0xffffu) >> 4) + 1);
        }
        s_rows[t] = rows;
        if (t == 0) s_off[nb] = pair_off[r0 + nb];
        if (t > nb) s_off[t] = 0xffffffffu;  // past the chunk: above every instance index
        {  // inclusive scan of the pooled rows over the chunk's pairs
            const uint32_t inc = wave_incl_scan(rows);
            if (lane == 63) s_wsum[w] = inc;
            __syncthreads();
            uint32_t before = 0;
            for (int k = 0; k < w; ++k) before += s_wsum[k];
            s_rend[t] = before + inc;
        }
        __syncthreads();
        for (int p0 = 0; p0 < nb;) {
            // the longest run of pairs from p0 whose pooled rows fit (at least p0 itself)
            const uint32_t rbase = p0 > 0 ? s_rend[p0 - 1] : 0u;
            int lo = p0 + 1, hi = nb;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_rend[mid - 1] - rbase <= (uint32_t)ROWPOOL) lo = mid; else hi = mid - 1;
            }
            const int p1 = lo;
            const uint32_t nrows = s_rend[p1 - 1] - rbase;
            // spans of the run's pooled rows, one row per thread
            for (uint32_t r = t; r < nrows; r += BN_THREADS) {
                const uint32_t g = rbase + r;
                int a = p0, b = p1 - 1;  // owner: the first pair whose scan end exceeds g
                while (a < b) {
                    const int mid = (a + b) >> 1;
                    if (s_rend[mid] > g) b = mid; else a = mid + 1;
                }
                const float4* rp = reinterpret_cast<const float4*>(rec + (size_t)s_src[a] * RGS_REC_FLOATS);
                const float4 ra = rp[0], rb = rp[1];
                SpanPre sp;
                span_pre(ra.x, ra.y, ra.z, ra.w, rb.x, rb.z, sp);
                const uint2 rr = s_rect[a];
                const int x_lo = (int)(int16_t)(rr.x & 0xffffu), x_hi = (int)(int16_t)(rr.x >> 16);
                const int y_lo = (int)(int16_t)(rr.y & 0xffffu), y_hi = (int)(int16_t)(rr.y >> 16);
                const int row = (int)(g - (s_rend[a] - s_rows[a]));
                const int2 cs = row_span(sp, x_lo, x_hi, y_lo, y_hi, (y_lo >> 4) + row);
                s_rcum[r] = cs.x <= cs.y ? (uint32_t)(cs.y - cs.x + 1) : 0u;
                s_rc0[r] = (int16_t)cs.x;
            }
            __syncthreads();
            if (t >= p0 && t < p1 && s_rows[t] > 0u) {  // running sums per pooled pair
                const uint32_t b0 = s_rend[t] - s_rows[t] - rbase;
                uint32_t run = 0;
                for (uint32_t r = 0; r < s_rows[t]; ++r) {
                    run += s_rcum[b0 + r];
                    s_rcum[b0 + r] = run;
                }
            }
            __syncthreads();
            const uint32_t j0 = s_off[p0], j1 = s_off[p1];
            for (uint32_t j = j0 + t; j < j1; j += BN_THREADS) {
                // last pair with s_off[p] <= j (offsets increase; entries past nb are ~0)
                int pl = 0;
#pragma unroll
                for (int step = BN_THREADS / 2; step > 0; step >>= 1)
                    if (s_off[pl + step] <= j) pl += step;
                const uint32_t nt = s_nt[pl];
                const uint32_t q = j - s_off[pl];
                const uint32_t c = udiv_small(q, nt);
                const uint32_t tt = q - c * nt;  // index among the pair's tiles, rows top to bottom
                const uint2 rr = s_rect[pl];
                const int tx0 = (int)(int16_t)(rr.x & 0xffffu) >> 4;
                const int ty0 = (int)(int16_t)(rr.y & 0xffffu) >> 4;
                int tx, ty;
                const uint64_t desc = s_desc[pl];
                if (desc != RGS_NO_SPANS) {
                    // row of tile tt by byte-wise prefix sums of the 8 row lengths
                    // (each < 16, total < 128): byte k of `pre` = tiles in rows 0..k,
                    // and the high bit of byte k of `ge` is set iff pre_k > tt
                    constexpr uint64_t ONES = 0x0101010101010101ull, HIGH = 0x8080808080808080ull;
                    const uint64_t lens = (desc >> 4) & 0x0f0f0f0f0f0f0f0full;
                    const uint64_t pre = lens * ONES;
                    const uint64_t ge = ((pre | HIGH) - (uint64_t)(tt + 1u) * ONES) & HIGH;
                    const int k = ge ? (__builtin_ctzll(ge) >> 3) : 7;
                    const uint32_t before = ((uint32_t)(pre >> (8 * k)) & 0xffu) - ((uint32_t)(lens >> (8 * k)) & 0xffu);
                    tx = tx0 + (int)((uint32_t)(desc >> (8 * k)) & 15u) + (int)(tt - before);
                    ty = ty0 + k;
                } else {
                    // pooled rows: the first row whose running sum exceeds tt
                    const uint32_t b0 = s_rend[pl] - s_rows[pl] - rbase;
                    int a = 0, b = (int)s_rows[pl] - 1;
                    while (a < b) {
                        const int mid = (a + b) >> 1;
                        if (s_rcum[b0 + mid] > tt) b = mid; else a = mid + 1;
                    }
                    const uint32_t before = a > 0 ? s_rcum[b0 + a - 1] : 0u;
                    tx = (int)s_rc0[b0 + a] + (int)(tt - before);
                    ty = ty0 + a;
                }
                const int cell = nth_set_bit(s_mask[pl], (int)c);
                keys[j] = ((s_vto[pl] + (uint32_t)ty * s_vtx[pl] + (uint32_t)tx) << L) |
                          (uint32_t)vt->v[s_view[pl]].rank_of_cell[cell];
                vals[j] = ((uint64_t)s_src[pl] << 32) | j;
            }
            __syncthreads();  // the pool is reused by the next run
            p0 = p1;
        }
    }
}

__global__ __launch_bounds__(BN_THREADS) void k_fill_u32(uint32_t* __restrict__ p, int64_t m, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * BN_THREADS + threadIdx.x;
    if (i < m) p[i] = v;
}

// Size classes of the launch orders: the slots by whole octaves of their
// length (32 classes), the tiles (the forward's order) by half octaves of
// their instance count (TCLS classes).  cls holds the slot counts [0, 32),
// the slot reservations [32, 64), the tile counts [64, 64 + TCLS) and the tile
// reservations [64 + TCLS, 64 + 2 TCLS).
static constexpr int TCLS = 64;
static constexpr int NCLS_WORDS = 64 + 2 * TCLS;
static_assert(TCLS == 32 || TCLS == 64 || TCLS == 128, "octaves, half or quarter octaves");
static_assert(32 + TCLS <= BN_THREADS, "a thread per class in the count and placement passes");

__device__ __forceinline__ int tile_class(uint32_t len) {
    const uint32_t v = len | 1u;
    const int hb = 31 - __clz(v);
    if (TCLS == 32) return hb;
    if (TCLS == 64) return 2 * hb + (hb > 0 ? (int)((v >> (hb - 1)) & 1u) : 0);
    return 4 * hb + (hb >= 2 ? (int)((v >> (hb - 2)) & 3u) : (hb == 1 ? (int)((v & 1u) << 1) : 0));
}

// Slot boundaries on the dense (tile, rank) table; block 0 also clears the
// size-class counters of the launch orders (launched even without instances).
// (A key at or past the table's end would mean an emission bug; it is skipped
// rather than written out of bounds.)
__global__ __launch_bounds__(BN_THREADS) void k_slot_bounds(const uint32_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ n_dev, int64_t dense,
                                                            uint32_t* __restrict__ dstart, uint32_t* __restrict__ dend,
                                                            uint32_t* __restrict__ cls) {
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < NCLS_WORDS; k += BN_THREADS) cls[k] = 0u;
    const int64_t n_inst = (int64_t)*n_dev;
    // a thread takes SB_ITEMS keys BN_THREADS apart per step; every key and
    // its two neighbours are loaded (coalesced, overlapping in cache) before
    // any is used
    constexpr int SB_ITEMS = 4;
    for (int64_t i0 = (int64_t)blockIdx.x * (BN_THREADS * SB_ITEMS) + threadIdx.x; i0 < n_inst;
         i0 += (int64_t)gridDim.x * (BN_THREADS * SB_ITEMS)) {
        uint32_t k[SB_ITEMS], pv[SB_ITEMS], nx[SB_ITEMS];
#pragma unroll
        for (int u = 0; u < SB_ITEMS; ++u) {
            const int64_t i = i0 + u * BN_THREADS;
            const int64_t ic = i < n_inst ? i : n_inst - 1;
            k[u] = keys[ic];
            pv[u] = keys[ic > 0 ? ic - 1 : 0];
            nx[u] = keys[ic + 1 < n_inst ? ic + 1 : ic];
        }
#pragma unroll
        for (int u = 0; u < SB_ITEMS; ++u) {
            const int64_t i = i0 + u * BN_THREADS;
            if (i >= n_inst || (int64_t)k[u] >= dense) continue;
            if (i == 0 || pv[u] != k[u]) dstart[k[u]] = (uint32_t)i;
            if (i == n_inst - 1 || nx[u] != k[u]) dend[k[u]] = (uint32_t)(i + 1);
        }
    }
}

// Launch orders, largest first by size class (tile_class; octaves for the slots): the slots
// (len = instances; the backward's order) and the tiles (len = instances of
// all the tile's slots, which are contiguous in the sorted list; the
// forward's order), so that long blocks do not start last and stretch the
// tail of the render.  One count and one placement kernel serve both, a
// thread taking slot i and tile i (class layout of cls above).
__device__ __forceinline__ uint32_t tile_len(const uint32_t* __restrict__ tile_slot,
                                             const uint32_t* __restrict__ slot_range, int64_t t) {
    const uint32_t s0 = tile_slot[t], s1 = tile_slot[t + 1];
    return s0 < s1 ? slot_range[2 * (s1 - 1) + 1] - slot_range[2 * s0] : 0u;
}

// The slot table from the dense (tile, rank) table, RGS_SCAN_TILE entries
// per block, in one pass: an entry is a slot iff its start is not ~0, and its
// slot index is the number of slots before it (the tile sums of the marks,
// summed over the earlier tiles of the dense table when fold = 1, else
// already scanned, plus the block's own exclusive scan).  Writes slot_key,
// slot_range, tile_slot (a tile's first slot; entry T = the slot count) and,
// with fold = 1, the slot count; counts the size classes of the slots and of
// all T tiles (a tile's length: its instances, from its first slot's start to
// its last slot's end) into cls (layout above).
static constexpr int SL_ITEMS = (int)(RGS_SCAN_TILE / BN_THREADS);
// Up to this many tiles a block sums the earlier tiles' marks itself.
static constexpr int64_t SLOT_FOLD_TILES = 1024;

__global__ __launch_bounds__(BN_THREADS) void k_slot_build(const uint32_t* __restrict__ dstart,
                                                           const uint32_t* __restrict__ dend,
                                                           const uint32_t* __restrict__ partial, int fold, int64_t dense,
                                                           int L, uint32_t* __restrict__ n_slots,
                                                           uint32_t* __restrict__ slot_key,
                                                           uint32_t* __restrict__ slot_range,
                                                           uint32_t* __restrict__ tile_slot, uint32_t* __restrict__ cls) {
    __shared__ uint32_t s_st[RGS_SCAN_TILE], s_en[RGS_SCAN_TILE];
    __shared__ uint32_t s_c[32 + TCLS];
    __shared__ uint32_t s_w[BN_THREADS / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * RGS_SCAN_TILE;
    const int nloc = (int)((dense - base) < RGS_SCAN_TILE ? (dense - base) : RGS_SCAN_TILE);
    const int K = 1 << L;
    if (t < 32 + TCLS) s_c[t] = 0u;
    // the first earlier tile sum of the thread is loaded with the entries
    const uint32_t p0 = (fold && (uint32_t)t < blockIdx.x) ? partial[t] : 0u;
    {  // coalesced loads (all first), into LDS
        uint32_t a[SL_ITEMS], b[SL_ITEMS];
#pragma unroll
        for (int k = 0; k < SL_ITEMS; ++k) {
            const int e = k * BN_THREADS + t;
            const int64_t i = base + (e < nloc ? e : nloc - 1);
            a[k] = dstart[i];
            b[k] = dend[i];
        }
#pragma unroll
        for (int k = 0; k < SL_ITEMS; ++k) {
            const int e = k * BN_THREADS + t;
            s_st[e] = e < nloc ? a[k] : 0xffffffffu;
            s_en[e] = b[k];
        }
    }
    uint32_t toff;
    if (fold) {
        uint32_t a = p0;
        for (uint32_t u = t + BN_THREADS; u < blockIdx.x; u += BN_THREADS) a += partial[u];
        a = wave_sum_u32(a);
        if (lane == 0) s_w[w] = a;
        __syncthreads();
        toff = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
        __syncthreads();  // s_w is reused by the scan
    } else {
        toff = partial[blockIdx.x];
        __syncthreads();
    }
    // thread t takes entries t * SL_ITEMS .. + SL_ITEMS - 1
    const int e0 = t * SL_ITEMS;
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < SL_ITEMS; ++j) c += s_st[e0 + j] != 0xffffffffu ? 1u : 0u;
    const uint32_t inc = wave_incl_scan(c);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < BN_THREADS / 64; ++k) {
        before += k < w ? s_w[k] : 0u;
        tot += s_w[k];
    }
    uint32_t run = toff + before + inc - c;
#pragma unroll
    for (int j = 0; j < SL_ITEMS; ++j) {
        const int e = e0 + j;
        if (e >= nloc) break;
        const int64_t ge = base + e;
        if ((ge & (K - 1)) == 0) {
            // the tile's first slot, and its length over its K entries (in LDS: a
            // tile never crosses a block, K dividing RGS_SCAN_TILE)
            tile_slot[ge >> L] = run;
            uint32_t lo = 0xffffffffu, hi = 0u;
            for (int q = 0; q < K && e + q < nloc; ++q) {
                const uint32_t a = s_st[e + q];
                if (a != 0xffffffffu) {
                    lo = lo < a ? lo : a;
                    hi = s_en[e + q];
                }
            }
            const uint32_t tl = lo != 0xffffffffu ? hi - lo : 0u;
            atomicAdd(&s_c[32 + tile_class(tl)], 1u);
        }
        const uint32_t a = s_st[e];
        if (a != 0xffffffffu) {
            const uint32_t b = s_en[e];
            slot_key[run] = (uint32_t)ge;
            slot_range[2 * run] = a;
            slot_range[2 * run + 1] = b;
            atomicAdd(&s_c[31 - __clz((b - a) | 1u)], 1u);
            ++run;
        }
    }
    if (base + nloc == dense && t == 0) {
        tile_slot[dense >> L] = toff + tot;
        if (fold) *n_slots = toff + tot;
    }
    __syncthreads();
    if (t < 32 + TCLS && s_c[t]) atomicAdd(&cls[t < 32 ? t : t + 32], s_c[t]);
}

// Items are placed class by class, classes in decreasing order: every block
// derives the class starts from the 32 counts, positions inside a block come
// from LDS counters and one global reservation per (block, class), so the
// global atomics do not serialise on a handful of counters.  The order inside
// a class is the launch order only and affects no result.
__global__ __launch_bounds__(BN_THREADS) void k_class_place(const uint32_t* __restrict__ slot_range,
                                                            const uint32_t* __restrict__ n_slots,
                                                            const uint32_t* __restrict__ tile_slot, int64_t T,
                                                            uint32_t* __restrict__ cls, uint32_t* __restrict__ slot_order,
                                                            uint32_t* __restrict__ tile_order) {
    __shared__ uint32_t s_c[32 + TCLS], s_base[32 + TCLS];
    if (threadIdx.x < 32 + TCLS) s_c[threadIdx.x] = 0u;
    if (threadIdx.x < 2) {
        // slots: counts cls[0..31] into s_base[0..31]; tiles: cls[64..] into s_base[32..]
        const int nc = threadIdx.x == 0 ? 32 : TCLS;
        const uint32_t* cnt = cls + 64 * threadIdx.x;
        uint32_t run = 0;
        for (int c = nc - 1; c >= 0; --c) {
            s_base[32 * threadIdx.x + c] = run;
            run += cnt[c];
        }
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * BN_THREADS + threadIdx.x;
    const bool oks = i < (int64_t)*n_slots, okt = i < T;
    int cs = 0, ct = 0;
    uint32_t ls = 0, lt = 0;
    if (oks) {
        cs = 31 - __clz((slot_range[2 * i + 1] - slot_range[2 * i]) | 1u);
        ls = atomicAdd(&s_c[cs], 1u);
    }
    if (okt) {
        ct = 32 + tile_class(tile_len(tile_slot, slot_range, i));
        lt = atomicAdd(&s_c[ct], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 32 + TCLS && s_c[threadIdx.x]) {
        const int r = threadIdx.x < 32 ? 32 + threadIdx.x : 64 + TCLS + (threadIdx.x - 32);  // reservation counters
        s_base[threadIdx.x] += atomicAdd(&cls[r], s_c[threadIdx.x]);
    }
    __syncthreads();
    if (oks) slot_order[s_base[cs] + ls] = (uint32_t)i;
    if (okt) tile_order[s_base[ct] + lt] = (uint32_t)i;
}

size_t bin_ws_bytes(int64_t n, int n_views, int64_t total_tiles, int L, int64_t capacity) {
    const int64_t m = (int64_t)n_views * n;
    const int64_t dense = total_tiles << L;
    WsCarver c{nullptr, 0, 0};
    c.take<uint32_t>(m + 1);          // flags / counts
    c.take<uint32_t>(m + 1);          // positions
    c.take<uint32_t>(m + 1);          // z keys
    c.take<uint32_t>(m + 1);          // z keys alt
    c.take<uint32_t>(m + 1);          // src alt
    c.take<uint32_t>(capacity + 1);   // instance keys alt
    c.take<uint64_t>(capacity + 1);   // instance vals alt
    c.take<uint32_t>(dense + 1);      // dense start
    c.take<uint32_t>(dense + 1);      // dense end
    c.take<uint32_t>(NCLS_WORDS);     // slot and tile size classes
    const int64_t big = m > capacity ? m : capacity;
    const int64_t big2 = big > dense ? big : dense;
    c.take<char>(radix_ws_bytes(big2 + 1));
    c.take<char>(scan_ws_bytes(big2 + 1));
    return c.used + 256;
}

static inline int bits_for(uint64_t v) {  // bits needed to represent values < v
    int b = 0;
    while (b < 63 && (1ull << b) < v) ++b;
    return b;
}

rgs_status bin_sort(const rgs_projected* proj, int64_t n, int n_views, const ViewTable* vt_dev, int L,
                    int64_t total_tiles, rgs_bins* bins, int64_t* n_required, bool sync, void* ws, size_t ws_bytes,
                    hipStream_t s) {
    const int64_t m = (int64_t)n_views * n;
    const int64_t dense = total_tiles << L;
    WsCarver c{reinterpret_cast<char*>(ws), 0, ws_bytes};
    uint32_t* flag = c.take<uint32_t>(m + 1);
    uint32_t* pos = c.take<uint32_t>(m + 1);
    uint32_t* zkey = c.take<uint32_t>(m + 1);
    uint32_t* zkey_alt = c.take<uint32_t>(m + 1);
    uint32_t* src_alt = c.take<uint32_t>(m + 1);
    uint32_t* keys_alt = c.take<uint32_t>(bins->capacity + 1);
    uint64_t* vals_alt = c.take<uint64_t>(bins->capacity + 1);
    uint32_t* dstart = c.take<uint32_t>(dense + 1);
    uint32_t* dend = c.take<uint32_t>(dense + 1);
    uint32_t* cls = c.take<uint32_t>(NCLS_WORDS);
    const int64_t big = m > bins->capacity ? m : bins->capacity;
    const int64_t big2 = big > dense ? big : dense;
    void* rws = c.take<char>(radix_ws_bytes(big2 + 1));
    void* sws = c.take<char>(scan_ws_bytes(big2 + 1));
    if (!c.ok()) return RGS_E_ARG;
    uint32_t* cnt = bins->counters;  // [0] pairs [1] instances [2] slots
    rgs_status st;
    auto grid = [](int64_t k) { return dim3((unsigned)((k + BN_THREADS - 1) / BN_THREADS > 0 ? (k + BN_THREADS - 1) / BN_THREADS : 1)); };
    // kernels over the visible pairs read their count on the device: capped grid, loops inside
    auto dgrid = [](int64_t k) {
        const int64_t b = (k + BN_THREADS - 1) / BN_THREADS;
        return dim3((unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b)));
    };

    // 1. visible pairs in (view, gid) order, then stable sorts by depth and by view
    const int64_t vtiles = (m + VC_TILE - 1) / VC_TILE;
    // up to 1024 tiles the compaction sums the tile counts itself
    const bool vfold = vtiles <= 1024;
    if (m > 0)
        hipLaunchKernelGGL(k_vis_count, dim3((unsigned)vtiles), dim3(BN_THREADS), 0, s, proj->count, m, pos);
    if (m <= 0 || !vfold)
        if ((st = scan_tile_sums(pos, DevN{nullptr, m, 1, 1}, VC_TILE, &cnt[0], s)) != RGS_OK) return st;
    if (m > 0)
        hipLaunchKernelGGL(k_vis_compact, dim3((unsigned)vtiles), dim3(BN_THREADS), 0, s, proj->count, proj->depth, m, pos,
                           vfold ? 1 : 0, &cnt[0], zkey, bins->pair_src);
    RGS_LAUNCH_CHECK();
    if ((st = radix_sort_u32_u32_dev(zkey, bins->pair_src, zkey_alt, src_alt, &cnt[0], m, 32, rws, s)) != RGS_OK)
        return st;
    if (n_views > 1) {
        hipLaunchKernelGGL(k_view_keys, dgrid(m), dim3(BN_THREADS), 0, s, bins->pair_src, &cnt[0], n, zkey);
        if ((st = radix_sort_u32_u32_dev(zkey, bins->pair_src, zkey_alt, src_alt, &cnt[0], m, bits_for(n_views), rws, s)) !=
            RGS_OK)
            return st;
    }
    // 2. instance offsets per ordered pair; the instance count goes to the host
    // (with the empty marks of the dense slot table: dstart = ~0)
    if (m > 0)
        hipLaunchKernelGGL(k_pair_counts, dgrid(m), dim3(BN_THREADS), 0, s, bins->pair_src, &cnt[0], proj->count,
                           bins->pair_rank, flag, reinterpret_cast<uint32_t*>(sws), dstart, dense);
    else
        hipLaunchKernelGGL(k_fill_u32, grid(dense), dim3(BN_THREADS), 0, s, dstart, dense, 0xffffffffu);
    // with the tail of pair_off and, without a host copy, the capacity guard
    const ScanTail tail{cnt, sync ? 0 : 1, bins->capacity};
    // (k_pair_counts wrote the tile sums; without pairs the scan reads none)
    if ((st = exclusive_scan_u32_dev(flag, bins->pair_off, DevN{&cnt[0], m, 1, 1}, m, &cnt[1], sws, s, 0, &tail, 1)) !=
        RGS_OK)
        return st;
    int64_t n_inst, slot_bound;
    if (sync) {
        uint32_t h_cnt[2] = {0u, 0u};
        RGS_HIP_CHECK(hipMemcpyAsync(h_cnt, cnt, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        RGS_HIP_CHECK(hipStreamSynchronize(s));
        n_inst = h_cnt[1];
        bins->n_instances = n_inst;
        if (n_required) *n_required = n_inst;
        slot_bound = n_inst < dense ? n_inst : dense;
        if (n_inst > bins->capacity || slot_bound > bins->slot_capacity) return RGS_E_CAPACITY;
    } else {
        // the count stays on the device; grids are sized by the capacity
        bins->n_instances = -1;
        n_inst = bins->capacity;
        slot_bound = n_inst < dense ? n_inst : dense;
    }

    // 3. emit and sort instances by (tile, rank)
    if (m > 0)
        hipLaunchKernelGGL(k_emit, dgrid(m), dim3(BN_THREADS), 0, s, bins->pair_src, &cnt[0], bins->pair_off, proj->rec,
                           proj->bin, n, vt_dev, bins->keys, bins->vals);
    RGS_LAUNCH_CHECK();
    const int key_bits = L + bits_for((uint64_t)total_tiles);
    if (key_bits > 32) return RGS_E_UNSUPPORTED;
    if (sync) st = radix_sort_u32_u64(bins->keys, bins->vals, keys_alt, vals_alt, n_inst, key_bits, rws, s);
    else st = radix_sort_u32_u64_dev(bins->keys, bins->vals, keys_alt, vals_alt, &cnt[1], n_inst, key_bits, rws, s);
    if (st != RGS_OK) return st;

    // 4. slots (k_slot_bounds also clears the size-class counters): the tile
    // sums of the slot marks, then the slot table and the class counts
    hipLaunchKernelGGL(k_slot_bounds, dgrid(n_inst), dim3(BN_THREADS), 0, s, bins->keys, &cnt[1], dense, dstart, dend,
                       cls);
    if (dense > 0) {
        uint32_t* dpart = reinterpret_cast<uint32_t*>(sws);
        const int64_t dtiles = (dense + RGS_SCAN_TILE - 1) / RGS_SCAN_TILE;
        const bool fold = dtiles <= SLOT_FOLD_TILES;
        if ((st = scan_tile_reduce(dstart, dense, 1, dpart, s)) != RGS_OK) return st;
        if (!fold && (st = scan_tile_sums(dpart, DevN{nullptr, dense, 1, 1}, RGS_SCAN_TILE, &cnt[2], s)) != RGS_OK)
            return st;
        hipLaunchKernelGGL(k_slot_build, dim3((unsigned)dtiles), dim3(BN_THREADS), 0, s, dstart, dend, dpart,
                           fold ? 1 : 0, dense, L, &cnt[2], bins->slot_key, bins->slot_range, bins->tile_slot, cls);
    } else {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(BN_THREADS), 0, s, bins->tile_slot, (int64_t)1, 0u);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(BN_THREADS), 0, s, &cnt[2], (int64_t)1, 0u);
    }
    // 5. launch orders of the slots and the tiles (largest size class first)
    const int64_t nord = slot_bound > total_tiles ? slot_bound : total_tiles;
    if (nord > 0)
        hipLaunchKernelGGL(k_class_place, grid(nord), dim3(BN_THREADS), 0, s, bins->slot_range, &cnt[2], bins->tile_slot,
                           total_tiles, cls, bins->slot_order, bins->tile_order);
    return launch_check();
}

}  // namespace rgs
