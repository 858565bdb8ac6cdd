// common.hpp -- shared device definitions of librgs (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rgs.h"

#define RGS_MAXK 64

// Per-view constants used by every kernel, uploaded once per call batch.
struct ViewParams {
    float R[9];          // world -> camera rotation, row-major
    float t[3];
    float o[3];          // camera centre
    float fx, fy, cx, cy;
    float gx, gy;        // guard of the EWA Jacobian: |x/z| <= gx, |y/z| <= gy
    float znear;
    float bg[3];
    int32_t W, H, tiles_x, tiles_y;
    uint32_t tile_offset;   // first global tile of this view
    uint32_t pix_offset;    // first pixel of this view in concatenated [H][W] maps
    uint8_t cell_of_rank[RGS_MAXK];
    uint8_t rank_of_cell[RGS_MAXK];
    uint64_t cell_visible;  // bit k: cell k may reach this view
};

struct ViewTable {
    int32_t n_views;
    int32_t L;
    uint32_t total_tiles;
    uint32_t culled;     // 1 if some view's cell_visible mask is not full
    ViewParams v[RGS_MAX_VIEWS];
};

// Which view owns global tile gt (views are few; linear scan, uniform per wave).
__device__ __forceinline__ int view_of_tile(const ViewTable* __restrict__ vt, uint32_t gt) {
    int v = 0;
    for (int k = 1; k < vt->n_views; ++k)
        if (gt >= vt->v[k].tile_offset) v = k;
    return v;
}

// IEEE total-order key of a non-NaN float (larger key <=> larger value, -0 < +0).
__device__ __forceinline__ uint32_t f2key(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

// Row spans of a footprint's tiles (decision path: fp32, fixed order, no
// contraction, IEEE division and square root, so that the projection's
// instance count and the emission's tile list agree bit for bit).
//
// With the factored quadratic form d^2 = ca u^2 + e dy^2, u = dx + k dy, the
// chord of {d^2 <= tau} at height dy runs from -k dy - w to -k dy + w, w =
// sqrt((tau - e dy^2) / ca).  Its right end is concave in dy, largest at the
// height of the rightmost point dy_r = -k sqrt(ca tau / (e (e + k^2 ca))); its
// left end is convex, smallest at -dy_r.  A tile row's band of pixel-centre
// heights [ly, hy] thus meets the ellipse between the chord ends at
// clamp(-dy_r) and clamp(dy_r).  tau is enlarged to tau (1 + 2^-18 (1 + rk)),
// rk = sqrt(1 + k^2 ca / e), above what the fp32 per-pixel test can accept
// (its rounding of u moves ca u^2 by at most about 2^-21 tau (1 + rk)), and
// the ends are padded by 1/64 px plus 2^-16 of their magnitude.  All terms
// are sums of non-negative parts, so no elongation loses accuracy; a
// non-finite end keeps the rectangle's bound.
struct SpanPre {
    float mx, my, ca, k, e, taup, dyr;
};

__device__ __forceinline__ void span_pre(float mx, float my, float ca, float k, float e, float tau, SpanPre& s) {
    s.mx = mx;
    s.my = my;
    s.ca = ca;
    s.k = k;
    s.e = e;
    const float rk = sqrtf(1.0f + (k * k) * (ca / e));
    s.taup = tau + tau * (0x1p-18f * (1.0f + rk));
    s.dyr = -(k * sqrtf((ca * s.taup) / (e * (e + (k * k) * ca))));
}

// Tile columns (c0, c1) of tile row ty inside the rectangle [x_lo, x_hi] x
// [y_lo, y_hi] whose pixel centres the footprint can reach; c0 > c1 if none.
__device__ __forceinline__ int2 row_span(const SpanPre& s, int x_lo, int x_hi, int y_lo, int y_hi, int ty) {
    const int y0 = max(ty * 16, y_lo), y1 = min(ty * 16 + 15, y_hi);
    const float ly = ((float)y0 + 0.5f) - s.my, hy = ((float)y1 + 0.5f) - s.my;
    const float dR = fminf(fmaxf(s.dyr, ly), hy), dL = fminf(fmaxf(-s.dyr, ly), hy);
    const float wR = fmaxf(s.taup - s.e * (dR * dR), 0.0f);
    const float wL = fmaxf(s.taup - s.e * (dL * dL), 0.0f);
    const float xr = s.mx + (sqrtf(wR / s.ca) - s.k * dR);
    const float xl = s.mx - (sqrtf(wL / s.ca) + s.k * dL);
    const float pr = 0x1p-6f + 0x1p-16f * (fabsf(s.mx) + fabsf(xr - s.mx));
    const float pl = 0x1p-6f + 0x1p-16f * (fabsf(s.mx) + fabsf(xl - s.mx));
    // a NaN end leaves the rectangle's bound (fmaxf/fminf drop NaN)
    const float lo = fmaxf(ceilf((xl - pl) - 0.5f), (float)x_lo);
    const float hi = fminf(floorf((xr + pr) - 0.5f), (float)x_hi);
    if (!(lo <= hi)) return make_int2(1, 0);
    return make_int2((int)lo >> 4, (int)hi >> 4);
}

// Row-span descriptor of a rectangle of at most 8 tile rows and 15 tile
// columns: byte k = (tiles in row ty0 + k) << 4 | (first column - tx0).  A
// byte of 0xff cannot occur, so ~0 marks a rectangle without descriptor.
static constexpr uint64_t RGS_NO_SPANS = ~0ull;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Work item of block b out of n: workgroups are handed to the eight XCDs in
// turn (block b to XCD b mod 8), and each XCD has its own L2, so block b
// takes item (b mod 8) q + min(b mod 8, n mod 8) + b / 8 (q = n / 8): every
// XCD walks one contiguous band of items, and lines that neighbouring items
// share (a halo, the ends of a run of writes) stay in one L2.  A bijection of
// [0, n) for every n.
__device__ __forceinline__ int xcd_band(int b, int n) {
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Wave64 sum reduction with DPP row operations; the total lands in lane 63.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xb1, 0xf, 0xf, false)); // quad_perm [1,0,3,2]
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4e, 0xf, 0xf, false)); // quad_perm [2,3,0,1]
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x124, 0xf, 0xf, false)); // row_ror:4
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128, 0xf, 0xf, false)); // row_ror:8
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xa, 0xf, false)); // row_bcast:15
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xc, 0xf, false)); // row_bcast:31
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
    v = wave_sum_to_lane63(v);
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Inclusive wave64 scan of u32 (shuffle based).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t u = __shfl_xor(v, d, 64);
        v = v > u ? v : u;
    }
    return v;
}

// ------------------------------------------------------------------ host side
namespace rgs {
void set_hip_error(hipError_t e);
rgs_status launch_check();
}  // namespace rgs

#define RGS_LAUNCH_CHECK()                        \
    do {                                          \
        rgs_status _s = rgs::launch_check();      \
        if (_s != RGS_OK) return _s;              \
    } while (0)

#define RGS_HIP_CHECK(expr)                       \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) {                   \
            rgs::set_hip_error(_e);               \
            return RGS_E_HIP;                     \
        }                                         \
    } while (0)

// Workspace carving: 256-byte aligned sub-buffers.
struct WsCarver {
    char* base;
    size_t used;
    size_t cap;
    template <typename T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
    bool ok() const { return used <= cap; }
};

// Device-wide primitives (sort.hip).
namespace rgs {
// An element count known on the host, or read on the device: ceil(*p / div) * mul.
struct DevN {
    const uint32_t* p;
    int64_t host;
    uint32_t div, mul;
    __device__ __forceinline__ int64_t get() const {
        if (!p) return host;
        const int64_t v = (int64_t)*p;
        return ((v + (int64_t)div - 1) / (int64_t)div) * (int64_t)mul;
    }
};
size_t scan_ws_bytes(int64_t n);
// Optional tail of the scan of per-pair instance counts (counters cnt =
// [pairs, instances, slots, required]; the scan's total must be &cnt[1]):
// out[pairs] = total and the capacity guard (see k_scan_apply).
struct ScanTail {
    uint32_t* cnt;
    int guard;
    int64_t capacity;
};
// Elements per tile of the scans below.
static constexpr int64_t RGS_SCAN_TILE = 4096;
// out[i] = sum_{j<i} in[j]; if total != nullptr, *total (device) = sum of all.
// marks = 1 scans (in[j] != ~0) instead of in[j].
rgs_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, void* ws,
                              hipStream_t s, int marks = 0);
// The same over the first dn.get() elements (n_max bounds the grid).
// sums_ready = 1: the caller has written the sums of the RGS_SCAN_TILE-element
// tiles to the first words of ws (the reduce pass is skipped).
rgs_status exclusive_scan_u32_dev(const uint32_t* in, uint32_t* out, DevN dn, int64_t n_max, uint32_t* total, void* ws,
                                  hipStream_t s, int marks = 0, const ScanTail* tail = nullptr, int sums_ready = 0);
// Block-level tile scan pieces, for callers that produce the tile sums themselves:
// exclusive scan (in place) of the sums of the first ceil(dn.get() / tile) tiles.
rgs_status scan_tile_sums(uint32_t* partial, DevN dn, int64_t tile, uint32_t* total, hipStream_t s);
// ... and the sums of the RGS_SCAN_TILE-element tiles of in[0, n) (marks as above).
rgs_status scan_tile_reduce(const uint32_t* in, int64_t n, int marks, uint32_t* partial, hipStream_t s);
size_t radix_ws_bytes(int64_t n);
// Stable LSD sort of (key, value) by key bits [0, bits); the result ends in
// keys/vals (the alt buffers are scratch of the same size).
rgs_status radix_sort_u32_u64(uint32_t* keys, uint64_t* vals, uint32_t* keys_alt, uint64_t* vals_alt,
                              int64_t n, int bits, void* ws, hipStream_t s);
rgs_status radix_sort_u32_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                              int64_t n, int bits, void* ws, hipStream_t s);
// The same, with n read on the device (upper bound n_max for the grid).
rgs_status radix_sort_u32_u64_dev(uint32_t* keys, uint64_t* vals, uint32_t* keys_alt, uint64_t* vals_alt,
                                  const uint32_t* n_dev, int64_t n_max, int bits, void* ws, hipStream_t s);
rgs_status radix_sort_u32_u32_dev(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                                  const uint32_t* n_dev, int64_t n_max, int bits, void* ws, hipStream_t s);
}  // namespace rgs
