// sort.hip -- device-wide exclusive scan and stable LSD radix sort (gfx950).
//
// Scan: reduce per 4096-element tile, scan the tile sums in one block, then
// scan each tile with its offset.  Tiles are staged through LDS so that
// global loads and stores stay coalesced.
//
// Radix sort: 8-bit digits, least significant first.  Per pass a histogram
// kernel counts digits per 2048-key tile (LDS atomics on integers), one
// block per digit scans that digit's row of the [256][tiles] table (the
// digit bases come from the 256 row totals), and a scatter kernel ranks each
// key stably inside its tile: every wave walks its strip in order, finds the
// lanes sharing its digit with eight ballots, and keeps a running count per
// digit in LDS; keys are then reordered in LDS by digit so that the global
// writes come out as contiguous runs.
#include "common.hpp"

namespace rgs {

// ------------------------------------------------------------------ scan
static constexpr int SCAN_THREADS = 256;
// Grid cap for kernels whose element count is read on the device.
static constexpr unsigned DEV_GRID = 2048;
static constexpr int SCAN_ITEMS = 16;
static constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
static_assert(SCAN_TILE == RGS_SCAN_TILE, "callers producing tile sums use RGS_SCAN_TILE");

__device__ __forceinline__ int skew(int i) { return i + (i >> 5); }

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ uint32_t block_excl_scan_256(uint32_t v, uint32_t* s_wave /*[4]*/, uint32_t* excl) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int k = 0; k < 4; ++k) {
        uint32_t t = s_wave[k];
        if (k < w) base += t;
        tot += t;
    }
    *excl = base + inc - v;
    __syncthreads();
    return tot;
}

// marks = 1: the scanned value of entry i is 1 if in[i] != ~0 (an occupied
// entry of a table whose empty entries hold all ones), else 0.
__device__ __forceinline__ uint32_t scan_val(const uint32_t* __restrict__ in, int64_t i, int marks) {
    const uint32_t v = in[i];
    return marks ? (v != 0xffffffffu ? 1u : 0u) : v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint32_t* __restrict__ in, DevN dn, int marks,
                                                              uint32_t* __restrict__ partial) {
    __shared__ uint32_t s_wave[4];
    const int64_t n = dn.get();
    for (int64_t tile = blockIdx.x; tile * SCAN_TILE < n; tile += gridDim.x) {
        const int64_t base = tile * SCAN_TILE;
        // all loads first (a lane past the end reads the last entry and adds nothing)
        uint32_t v[SCAN_ITEMS];
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            const int64_t i = base + k * SCAN_THREADS + threadIdx.x;
            v[k] = scan_val(in, i < n ? i : n - 1, marks);
        }
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) acc += base + k * SCAN_THREADS + threadIdx.x < n ? v[k] : 0u;
        uint32_t ex;
        uint32_t tot = block_excl_scan_256(acc, s_wave, &ex);
        if (threadIdx.x == 0) partial[tile] = tot;
    }
}

// Exclusive scan, in place, of the sums of the first ceil(dn / tile) tiles;
// the total to *total if non-null.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_partials(uint32_t* __restrict__ partial, DevN dn, int64_t tile,
                                                                uint32_t* __restrict__ total) {
    __shared__ uint32_t s_wave[4];
    const int64_t m = (dn.get() + tile - 1) / tile;
    uint32_t carry = 0;
    for (int64_t b = 0; b < m; b += SCAN_THREADS) {
        int64_t i = b + threadIdx.x;
        uint32_t v = i < m ? partial[i] : 0u;
        uint32_t ex;
        uint32_t tot = block_excl_scan_256(v, s_wave, &ex);
        if (i < m) partial[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// The optional tail of a scan of per-pair instance counts: out[n] = total,
// and, with guard set (no host copy of the instance count), if the total
// exceeds the capacity, counters[3] = total and the pair, instance and slot
// counts are zeroed so that every later kernel of the pass finds no work;
// else (and always without guard) counters[3] = 0.
__device__ __forceinline__ void scan_tail(const ScanTail& t, uint32_t* __restrict__ out, int64_t n, uint32_t total) {
    if (!t.cnt) return;
    out[n] = total;
    if (t.guard && (int64_t)total > t.capacity) {
        t.cnt[3] = total;
        t.cnt[0] = 0u;
        t.cnt[1] = 0u;
        t.cnt[2] = 0u;
    } else {
        t.cnt[3] = 0u;
    }
}

// fold = 1: the tile sums are not scanned beforehand; every block adds up the
// sums of the tiles before its own (for at most SCAN_FOLD_TILES tiles), and
// the block of the last tile writes the total and the tail.  fold = 0: the
// partials hold the scanned tile offsets (k_scan_partials wrote the total).
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const uint32_t* __restrict__ in, DevN dn, int marks,
                                                             const uint32_t* __restrict__ partial, int fold,
                                                             uint32_t* __restrict__ total, ScanTail tail,
                                                             uint32_t* __restrict__ out) {
    __shared__ uint32_t s[SCAN_TILE + SCAN_TILE / 32];
    __shared__ uint32_t s_wave[4];
    const int64_t n = dn.get();
    if (fold && n <= 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (total) *total = 0u;
            scan_tail(tail, out, 0, 0u);
        }
        return;
    }
    const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t base = tile * SCAN_TILE;
        uint32_t toff;
        if (fold) {
            uint32_t a = 0;
            for (int64_t t = threadIdx.x; t < tile; t += SCAN_THREADS) a += partial[t];
            uint32_t ex;
            toff = block_excl_scan_256(a, s_wave, &ex);  // the block total of the per-thread sums
        } else {
            toff = partial[tile];
        }
        {
            uint32_t lv[SCAN_ITEMS];
#pragma unroll
            for (int k = 0; k < SCAN_ITEMS; ++k) {
                const int64_t i = base + k * SCAN_THREADS + threadIdx.x;
                lv[k] = scan_val(in, i < n ? i : n - 1, marks);
            }
#pragma unroll
            for (int k = 0; k < SCAN_ITEMS; ++k) {
                const int li = k * SCAN_THREADS + threadIdx.x;
                s[skew(li)] = base + li < n ? lv[k] : 0u;
            }
        }
        __syncthreads();
        uint32_t v[SCAN_ITEMS], acc = 0;
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            v[k] = s[skew(threadIdx.x * SCAN_ITEMS + k)];
            acc += v[k];
        }
        uint32_t ex;
        const uint32_t tsum = block_excl_scan_256(acc, s_wave, &ex);
        if (fold && tile == ntiles - 1 && threadIdx.x == 0) {
            if (total) *total = toff + tsum;
            scan_tail(tail, out, n, toff + tsum);
        }
        uint32_t run = toff + ex;
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            s[skew(threadIdx.x * SCAN_ITEMS + k)] = run;
            run += v[k];
        }
        __syncthreads();
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            int li = k * SCAN_THREADS + threadIdx.x;
            int64_t i = base + li;
            if (i < n) out[i] = s[skew(li)];
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// The tail for the path with a separate scan of the tile sums (total known).
__global__ void k_scan_tail(uint32_t* __restrict__ out, ScanTail tail) {
    if (threadIdx.x != 0) return;
    scan_tail(tail, out, tail.cnt[0], tail.cnt[1]);
}

size_t scan_ws_bytes(int64_t n) {
    int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    return (size_t)(tiles + 1) * sizeof(uint32_t) + 256;
}

rgs_status scan_tile_reduce(const uint32_t* in, int64_t n, int marks, uint32_t* partial, hipStream_t s) {
    if (n <= 0) return RGS_OK;
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(SCAN_THREADS), 0, s, in, DevN{nullptr, n, 1, 1}, marks,
                       partial);
    return launch_check();
}

rgs_status scan_tile_sums(uint32_t* partial, DevN dn, int64_t tile, uint32_t* total, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_THREADS), 0, s, partial, dn, tile, total);
    return launch_check();
}

// Up to this many tiles, the apply kernel sums the tile sums itself (one
// launch fewer); beyond it a single block scans them first.
static constexpr int64_t SCAN_FOLD_TILES = 1024;

rgs_status exclusive_scan_u32_dev(const uint32_t* in, uint32_t* out, DevN dn, int64_t n_max, uint32_t* total, void* ws,
                                  hipStream_t s, int marks, const ScanTail* tail, int sums_ready) {
    uint32_t* partial = reinterpret_cast<uint32_t*>(ws);
    const ScanTail tl = tail ? *tail : ScanTail{nullptr, 0, 0};
    const int64_t tiles = (n_max + SCAN_TILE - 1) / SCAN_TILE;
    const bool fold = tiles <= SCAN_FOLD_TILES;
    const unsigned grid = (unsigned)(tiles < 1 ? 1 : (dn.p && tiles > DEV_GRID ? DEV_GRID : tiles));
    if (n_max > 0 && !sums_ready)
        hipLaunchKernelGGL(k_scan_reduce, dim3(grid), dim3(SCAN_THREADS), 0, s, in, dn, marks, partial);
    if (!fold) hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_THREADS), 0, s, partial, dn, (int64_t)SCAN_TILE, total);
    hipLaunchKernelGGL(k_scan_apply, dim3(grid), dim3(SCAN_THREADS), 0, s, in, dn, marks, partial, fold ? 1 : 0,
                       total, tl, out);
    if (!fold && tl.cnt) {
        // the tail after the single-block scan of the tile sums
        hipLaunchKernelGGL(k_scan_tail, dim3(1), dim3(64), 0, s, out, tl);
    }
    return launch_check();
}

rgs_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, void* ws,
                              hipStream_t s, int marks) {
    return exclusive_scan_u32_dev(in, out, DevN{nullptr, n, 1, 1}, n, total, ws, s, marks, nullptr);
}

// ------------------------------------------------------------------ radix sort
static constexpr int RS_THREADS = 256;
static constexpr int RS_ITEMS = 8;
static constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // 2048 keys per block
static constexpr int RS_WAVE_ITEMS = 64 * RS_ITEMS;    // a wave's strip

__device__ __forceinline__ int64_t rs_n(int64_t n, const uint32_t* n_dev) {
    return n_dev ? (int64_t)*n_dev : n;
}

// Blocks loop over tiles (with a device-side count the grid is capped and
// sized for the largest possible count, so no block is launched only to exit);
// the n-th tile a block takes (n = block + round * grid) is tile
// xcd_band(n, tiles): with a grid that is a multiple of 8 (or a single
// round) every XCD takes one contiguous band of tiles, the same number each,
// so that the tiles that write neighbouring parts of a digit's output run on
// one XCD and the cache lines their runs share are completed in one L2.
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n_host,
                                                        const uint32_t* __restrict__ n_dev, int shift,
                                                        uint32_t* __restrict__ hist, int ntiles) {
    __shared__ uint32_t s_h[256];
    const int64_t n = rs_n(n_host, n_dev);
    // with a device count the table is [256][tiles in use]
    if (n_dev) ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
    for (int nth = blockIdx.x; nth < ntiles; nth += gridDim.x) {
        const int tile = xcd_band(nth, ntiles);
        s_h[threadIdx.x] = 0;
        __syncthreads();
        const int64_t base = (int64_t)tile * RS_TILE;
        // all loads first (a lane past the end reads the last key and adds nothing)
        uint32_t kv[RS_ITEMS];
#pragma unroll
        for (int k = 0; k < RS_ITEMS; ++k) {
            const int64_t i = base + k * RS_THREADS + threadIdx.x;
            kv[k] = keys[i < n ? i : n - 1];
        }
#pragma unroll
        for (int k = 0; k < RS_ITEMS; ++k)
            if (base + k * RS_THREADS + threadIdx.x < n) atomicAdd(&s_h[(kv[k] >> shift) & 0xffu], 1u);
        __syncthreads();
        hist[(int64_t)threadIdx.x * ntiles + tile] = s_h[threadIdx.x];
        __syncthreads();
    }
}

// Per digit d (one block each): exclusive scan over tiles of the digit's row
// hist[d][*] into offs[d][*], and the row total into dtot[d].  The scatter
// adds the digit's base (an exclusive scan of the 256 totals, done in LDS).
__global__ __launch_bounds__(RS_THREADS) void k_rs_colscan(const uint32_t* __restrict__ hist, int64_t n_host,
                                                           const uint32_t* __restrict__ n_dev, int ntiles,
                                                           uint32_t* __restrict__ offs, uint32_t* __restrict__ dtot) {
    __shared__ uint32_t s_wave[4];
    const int64_t n = rs_n(n_host, n_dev);
    if (n_dev) ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
    const int64_t row = (int64_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (int t0 = 0; t0 < ntiles; t0 += RS_THREADS * 4) {
        uint32_t v[4], acc = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int t = t0 + threadIdx.x * 4 + k;
            v[k] = t < ntiles ? hist[row + t] : 0u;
            acc += v[k];
        }
        uint32_t ex;
        const uint32_t tot = block_excl_scan_256(acc, s_wave, &ex);
        uint32_t run = carry + ex;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int t = t0 + threadIdx.x * 4 + k;
            if (t < ntiles) offs[row + t] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

template <typename V>
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint32_t* __restrict__ keys_in,
                                                           const V* __restrict__ vals_in, int64_t n_host,
                                                           const uint32_t* __restrict__ n_dev, int shift,
                                                           const uint32_t* __restrict__ offsets,
                                                           const uint32_t* __restrict__ dtot, int ntiles,
                                                           uint32_t* __restrict__ keys_out,
                                                           V* __restrict__ vals_out) {
    __shared__ uint32_t s_cnt[4][256];  // per-wave running digit counts, then wave prefixes
    __shared__ uint32_t s_dstart[256];  // tile-local start of each digit
    __shared__ uint32_t s_goff[256];    // global start of each digit for this tile
    __shared__ uint32_t s_dbase[256];   // global start of each digit
    __shared__ uint32_t s_wave[4];
    __shared__ uint32_t s_keys[RS_TILE];
    __shared__ V s_vals[RS_TILE];

    const int64_t n = rs_n(n_host, n_dev);
    if (n_dev) ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if ((int)blockIdx.x < ntiles) {  // the block has a tile (uniform per block)
        uint32_t ex;
        block_excl_scan_256(dtot[threadIdx.x], s_wave, &ex);
        s_dbase[threadIdx.x] = ex;
    }
    for (int nth = blockIdx.x; nth < ntiles; nth += gridDim.x) {
        const int tile = xcd_band(nth, ntiles);
        for (int k = threadIdx.x; k < 4 * 256; k += RS_THREADS) (&s_cnt[0][0])[k] = 0;
        __syncthreads();

        const int64_t base = (int64_t)tile * RS_TILE;
        const int64_t tile_n = (n - base) < RS_TILE ? (n - base) : RS_TILE;
        uint32_t key[RS_ITEMS];
        V val[RS_ITEMS];
        uint32_t rank[RS_ITEMS];
        // all loads first, without branches (a lane past the end reads the last element)
#pragma unroll
        for (int k = 0; k < RS_ITEMS; ++k) {
            const int64_t i = base + (int64_t)w * RS_WAVE_ITEMS + k * 64 + lane;
            const int64_t ic = i < n ? i : n - 1;
            key[k] = keys_in[ic];
            val[k] = vals_in[ic];
        }
        for (int k = 0; k < RS_ITEMS; ++k) {
            const int64_t i = base + (int64_t)w * RS_WAVE_ITEMS + k * 64 + lane;
            const bool valid = i < n;
            const uint32_t d = (key[k] >> shift) & 0xffu;
            uint64_t m = __ballot(valid);
    #pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                m &= bit ? bb : ~bb;
            }
            uint32_t prior = 0;
            if (valid) prior = s_cnt[w][d];
            rank[k] = prior + (uint32_t)__popcll(m & lt_mask);
            // the highest lane of each digit group publishes the new count
            if (valid && (m >> lane) == 1ull) s_cnt[w][d] = prior + (uint32_t)__popcll(m);
            if (!valid) rank[k] = 0xffffffffu;
        }
        __syncthreads();
        {
            const int d = threadIdx.x;
            const uint32_t c0 = s_cnt[0][d], c1 = s_cnt[1][d], c2 = s_cnt[2][d], c3 = s_cnt[3][d];
            s_cnt[0][d] = 0;
            s_cnt[1][d] = c0;
            s_cnt[2][d] = c0 + c1;
            s_cnt[3][d] = c0 + c1 + c2;
            const uint32_t tot = c0 + c1 + c2 + c3;
            s_goff[d] = s_dbase[d] + offsets[(int64_t)d * ntiles + tile];
            uint32_t ex;
            block_excl_scan_256(tot, s_wave, &ex);
            s_dstart[d] = ex;
        }
        __syncthreads();
        for (int k = 0; k < RS_ITEMS; ++k) {
            if (rank[k] == 0xffffffffu) continue;
            const uint32_t d = (key[k] >> shift) & 0xffu;
            const uint32_t p = s_dstart[d] + s_cnt[w][d] + rank[k];
            s_keys[p] = key[k];
            s_vals[p] = val[k];
        }
        __syncthreads();
        for (int k = 0; k < RS_ITEMS; ++k) {
            const int p = k * RS_THREADS + threadIdx.x;
            if (p < tile_n) {
                const uint32_t kk = s_keys[p];
                const uint32_t d = (kk >> shift) & 0xffu;
                const uint32_t o = s_goff[d] + ((uint32_t)p - s_dstart[d]);
                keys_out[o] = kk;
                vals_out[o] = s_vals[p];
            }
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

template <typename V>
__global__ __launch_bounds__(256) void k_rs_copy(const uint32_t* __restrict__ ki, const V* __restrict__ vi,
                                                 int64_t n_host, const uint32_t* __restrict__ n_dev,
                                                 uint32_t* __restrict__ ko, V* __restrict__ vo) {
    const int64_t n = rs_n(n_host, n_dev);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        ko[i] = ki[i];
        vo[i] = vi[i];
    }
}

size_t radix_ws_bytes(int64_t n) {
    int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    if (tiles < 1) tiles = 1;
    size_t h = (size_t)256 * tiles * sizeof(uint32_t);
    return 2 * ((h + 255) & ~size_t(255)) + 256 * sizeof(uint32_t) + 512;
}

template <typename V>
static rgs_status radix_sort_impl(uint32_t* keys, V* vals, uint32_t* keys_alt, V* vals_alt, int64_t n,
                                  const uint32_t* n_dev, int bits, void* ws, hipStream_t s) {
    if (n <= 0 || bits <= 0) return RGS_OK;
    int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    size_t h = (size_t)256 * tiles * sizeof(uint32_t);
    size_t hpad = (h + 255) & ~size_t(255);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws);
    uint32_t* offs = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ws) + hpad);
    uint32_t* dtot = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ws) + 2 * hpad);  // [256]
    int passes = (bits + 7) / 8;
    const unsigned grid = (unsigned)(n_dev && tiles > DEV_GRID ? DEV_GRID : tiles);
    uint32_t *ki = keys, *ko = keys_alt;
    V *vi = vals, *vo = vals_alt;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3(grid), dim3(RS_THREADS), 0, s, ki, n, n_dev, shift, hist,
                           (int)tiles);
        hipLaunchKernelGGL(k_rs_colscan, dim3(256), dim3(RS_THREADS), 0, s, hist, n, n_dev, (int)tiles, offs, dtot);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rs_scatter<V>), dim3(grid), dim3(RS_THREADS), 0, s, ki, vi,
                           n, n_dev, shift, offs, dtot, (int)tiles, ko, vo);
        RGS_LAUNCH_CHECK();
        uint32_t* tk = ki; ki = ko; ko = tk;
        V* tv = vi; vi = vo; vo = tv;
    }
    if (ki != keys) {
        // odd number of passes: copy back (the elements in use only)
        const int64_t g0 = (n + 255) / 256;
        const unsigned g = (unsigned)(g0 > DEV_GRID * 8 ? DEV_GRID * 8 : g0);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rs_copy<V>), dim3(g), dim3(256), 0, s, ki, vi, n, n_dev, keys, vals);
        RGS_LAUNCH_CHECK();
    }
    return RGS_OK;
}

rgs_status radix_sort_u32_u64(uint32_t* keys, uint64_t* vals, uint32_t* keys_alt, uint64_t* vals_alt, int64_t n,
                              int bits, void* ws, hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n, nullptr, bits, ws, s);
}
rgs_status radix_sort_u32_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t n,
                              int bits, void* ws, hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, nullptr, bits, ws, s);
}
rgs_status radix_sort_u32_u64_dev(uint32_t* keys, uint64_t* vals, uint32_t* keys_alt, uint64_t* vals_alt,
                                  const uint32_t* n_dev, int64_t n_max, int bits, void* ws, hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n_max, n_dev, bits, ws, s);
}
rgs_status radix_sort_u32_u32_dev(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                                  const uint32_t* n_dev, int64_t n_max, int bits, void* ws, hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n_max, n_dev, bits, ws, s);
}

}  // namespace rgs
