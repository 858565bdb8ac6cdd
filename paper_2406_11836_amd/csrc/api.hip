// api.hip -- the extern "C" entry points of librgs (declared in include/rgs.h):
// argument validation, the device view table, and kernel dispatch.
#include <math.h>
#include <string.h>

#include <vector>

#include "common.hpp"

namespace rgs {
static thread_local int32_t g_last_hip = 0;
void set_hip_error(hipError_t e) { g_last_hip = (int32_t)e; }
rgs_status launch_check() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_last_hip = (int32_t)e;
        return RGS_E_HIP;
    }
    return RGS_OK;
}

size_t kd_ws_bytes(int64_t n, int L);
rgs_status kd_partition(const rgs_gaussians* g, int L, float d_factor, int rule, const rgs_kdtree* kd, void* ws,
                        hipStream_t s);
rgs_status project_launch(const rgs_gaussians* g, const ViewTable* vt, const float* split, const int32_t* center_cell,
                          int cells, const uint32_t* own_mask, const rgs_projected* out, hipStream_t s);
rgs_status project_bwd_launch(const float* dproj, const rgs_gaussians* g, const uint32_t* count, const ViewTable* vt,
                              const rgs_gaussians_grad* out, hipStream_t s);
size_t bin_ws_bytes(int64_t n, int n_views, int64_t total_tiles, int L, int64_t capacity);
size_t group_ws_bytes(int64_t n);
rgs_status group_by_cell(const rgs_gaussians* in, const rgs_kdtree* kd, int L, const rgs_gaussians* out, int32_t* perm,
                         void* ws, size_t ws_bytes, hipStream_t s);
rgs_status bin_sort(const rgs_projected* proj, int64_t n, int n_views, const ViewTable* vt_dev, int L, int64_t total_tiles,
                    rgs_bins* bins, int64_t* n_required, bool sync, void* ws, size_t ws_bytes, hipStream_t s);
// image / T_final non-null: the merged image of the partials as well (the
// merge's fold, run in the render block)
rgs_status render_fwd_launch(const rgs_projected* proj, const rgs_bins* bins, const ViewTable* vt, const rgs_kdtree* kd,
                             float eps_T, const rgs_partials* out, uint64_t* stats, int64_t total_tiles, hipStream_t s,
                             float* image = nullptr, float* T_final = nullptr);
size_t render_bwd_ws_bytes(int64_t capacity);
rgs_status render_bwd_records_launch(const rgs_partials_grad* dparts, const rgs_partials* parts, const rgs_bins* bins,
                                     const rgs_projected* proj, const ViewTable* vt, const rgs_kdtree* kd, void* ws,
                                     uint64_t* stats, int64_t slot_bound, hipStream_t s);
rgs_status pair_reduce_launch(const rgs_bins* bins, const rgs_projected* proj, int64_t n, int n_views, float* dproj,
                              void* ws, hipStream_t s);
rgs_status merge_fwd_launch(const rgs_partials* parts, const rgs_bins* bins, const ViewTable* vt, int64_t total_tiles,
                            float* image, float* T_final, hipStream_t s);
rgs_status merge_bwd_launch(const float* dimage, const float* dTfinal, const rgs_partials* parts, const rgs_bins* bins,
                            const ViewTable* vt, int64_t total_tiles, const rgs_partials_grad* out, hipStream_t s);
rgs_status adam_launch(const rgs_gaussians_grad* params, const rgs_gaussians_grad* grads, const rgs_gaussians_grad* m,
                       const rgs_gaussians_grad* v, int64_t n, int sh_degree, const rgs_adam_params* hp, hipStream_t s);
rgs_status permute_launch(const rgs_gaussians* in, const int32_t* perm, const rgs_gaussians_grad* out, hipStream_t s);
size_t loss_ws_bytes(int H, int W);
rgs_status loss_launch(const float* image, const float* target, int H, int W, float ssim_w, float* loss, float* dimg,
                       void* ws, hipStream_t s);
rgs_status loss_scratch(void** out);
}  // namespace rgs

using namespace rgs;

static inline hipStream_t S(rgs_stream s) { return reinterpret_cast<hipStream_t>(s); }

static bool cams_ok(const rgs_camera* cams, int32_t n_views) {
    if (!cams || n_views < 1 || n_views > RGS_MAX_VIEWS) return false;
    for (int v = 0; v < n_views; ++v) {
        const rgs_camera& c = cams[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 32767 || c.height > 32767) return false;
        if (!(c.z_near > 0.f) || !(c.fx > 0.f) || !(c.fy > 0.f)) return false;
        for (int k = 0; k < 9; ++k) if (!isfinite(c.R[k])) return false;
        for (int k = 0; k < 3; ++k) if (!isfinite(c.t[k]) || !isfinite(c.campos[k])) return false;
    }
    return true;
}

// A workspace: non-null, 256-byte aligned, at least `need` bytes.
static bool ws_ok(const void* ws, size_t have, size_t need) {
    return ws && (reinterpret_cast<uintptr_t>(ws) & 255u) == 0 && have >= need;
}

static bool gauss_ok(const rgs_gaussians* g) {
    if (!g || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3) return false;
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity || !g->sh)) return false;
    return true;
}

// Byte ranges of buffers, for the aliasing checks: no output may overlap an
// input or another output (a null pointer or an empty range is skipped).
struct Span {
    const void* p;
    size_t n;
};
using Spans = std::vector<Span>;

static bool overlap(const Span& a, const Span& b) {
    if (!a.p || !b.p || a.n == 0 || b.n == 0) return false;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a.p), b0 = reinterpret_cast<uintptr_t>(b.p);
    return a0 < b0 + b.n && b0 < a0 + a.n;
}

// outputs pairwise disjoint, and disjoint from every input
static bool disjoint(const Spans& outs, const Spans& ins) {
    for (size_t i = 0; i < outs.size(); ++i) {
        for (size_t j = i + 1; j < outs.size(); ++j)
            if (overlap(outs[i], outs[j])) return false;
        for (const Span& b : ins)
            if (overlap(outs[i], b)) return false;
    }
    return true;
}

static Spans gauss_spans(const rgs_gaussians* g) {
    const size_t n = (size_t)(g->n > 0 ? g->n : 0);
    const size_t nc = (size_t)(g->sh_degree + 1) * (g->sh_degree + 1);
    return {{g->means, 12 * n}, {g->log_scales, 12 * n}, {g->quats, 16 * n}, {g->opacity, 4 * n}, {g->sh, 12 * nc * n}};
}

static Spans grad_spans(const rgs_gaussians_grad* o, const rgs_gaussians* g) {
    const size_t n = (size_t)(g->n > 0 ? g->n : 0);
    const size_t nc = (size_t)(g->sh_degree + 1) * (g->sh_degree + 1);
    return {{o->means, 12 * n}, {o->log_scales, 12 * n}, {o->quats, 16 * n}, {o->opacity, 4 * n}, {o->sh, 12 * nc * n}};
}

// m = views * Gaussians
static Spans proj_spans(const rgs_projected* p, size_t m) {
    return {{p->rec, (size_t)RGS_REC_FLOATS * 4 * m}, {p->bin, 32 * m}, {p->count, 4 * m},
            {p->depth, 4 * m}};
}

static Spans bins_spans(const rgs_bins* b, size_t m, size_t total_tiles) {
    const size_t c = (size_t)(b->capacity > 0 ? b->capacity : 0), sc = (size_t)(b->slot_capacity > 0 ? b->slot_capacity : 0);
    return {{b->keys, 4 * c}, {b->vals, 8 * c}, {b->pair_src, 4 * m}, {b->pair_off, 4 * (m + 1)}, {b->pair_rank, 4 * m},
            {b->slot_key, 4 * sc}, {b->slot_range, 8 * sc}, {b->tile_slot, 4 * (total_tiles + 1)},
            {b->slot_order, 4 * sc}, {b->tile_order, 4 * total_tiles}, {b->counters, 16}};
}

static Spans parts_spans(const rgs_partials* p, const rgs_bins* b) {
    const size_t sc = (size_t)(b->slot_capacity > 0 ? b->slot_capacity : 0);
    return {{p->C, 3072 * sc}, {p->T, 1024 * sc}, {p->last, 1024 * sc}};
}

static Spans concat(Spans a, const Spans& b) {
    a.insert(a.end(), b.begin(), b.end());
    return a;
}

static int64_t tiles_of(const rgs_camera& c) {
    return (int64_t)((c.width + 15) / 16) * (int64_t)((c.height + 15) / 16);
}

static size_t pixels_of(const rgs_camera* cams, int32_t n_views) {
    size_t px = 0;
    for (int v = 0; v < n_views; ++v) px += (size_t)cams[v].width * (size_t)cams[v].height;
    return px;
}

static size_t total_tiles_of(const rgs_camera* cams, int32_t n_views) {
    size_t t = 0;
    for (int v = 0; v < n_views; ++v) t += (size_t)tiles_of(cams[v]);
    return t;
}

extern "C" {

int32_t rgs_abi_version(void) { return RGS_ABI_VERSION; }

const char* rgs_status_string(rgs_status s) {
    switch (s) {
        case RGS_OK: return "ok";
        case RGS_E_ARG: return "invalid argument";
        case RGS_E_CAPACITY: return "buffer capacity too small";
        case RGS_E_HIP: return "HIP error";
        case RGS_E_UNSUPPORTED: return "unsupported size";
        default: return "unknown status";
    }
}

int32_t rgs_last_hip_error(void) { return g_last_hip; }

size_t rgs_views_bytes(void) { return sizeof(ViewTable); }

int64_t rgs_total_tiles(const rgs_camera* cams, int32_t n_views) {
    if (!cams || n_views < 1) return 0;
    int64_t t = 0;
    for (int v = 0; v < n_views; ++v) t += tiles_of(cams[v]);
    return t;
}

rgs_status rgs_views_pack(const rgs_camera* cams, int32_t n_views, int32_t L, const int32_t* rank_of,
                          const uint64_t* cell_visible, void* views_host) {
    if (!cams_ok(cams, n_views) || L < 0 || L > RGS_MAX_L || !rank_of || !views_host) return RGS_E_ARG;
    const int K = 1 << L;
    ViewTable vt;
    memset(&vt, 0, sizeof(vt));
    vt.n_views = n_views;
    vt.L = L;
    uint32_t tile_off = 0, pix_off = 0;
    for (int v = 0; v < n_views; ++v) {
        const rgs_camera& c = cams[v];
        ViewParams& p = vt.v[v];
        memcpy(p.R, c.R, sizeof(p.R));
        memcpy(p.t, c.t, sizeof(p.t));
        memcpy(p.o, c.campos, sizeof(p.o));
        p.fx = c.fx; p.fy = c.fy; p.cx = c.cx; p.cy = c.cy;
        // guard of the EWA Jacobian, fixed fp32 order: 1.3 * (max(cx, W - cx) / fx)
        const float Wf = (float)c.width, Hf = (float)c.height;
        p.gx = 1.3f * (fmaxf(c.cx, Wf - c.cx) / c.fx);
        p.gy = 1.3f * (fmaxf(c.cy, Hf - c.cy) / c.fy);
        p.znear = c.z_near;
        memcpy(p.bg, c.bg, sizeof(p.bg));
        p.W = c.width; p.H = c.height;
        p.tiles_x = (c.width + 15) / 16; p.tiles_y = (c.height + 15) / 16;
        p.tile_offset = tile_off;
        p.pix_offset = pix_off;
        tile_off += (uint32_t)(p.tiles_x * p.tiles_y);
        pix_off += (uint32_t)(c.width * c.height);
        for (int k = 0; k < K; ++k) {
            const int r = rank_of[v * K + k];
            if (r < 0 || r >= K) return RGS_E_ARG;
            p.rank_of_cell[k] = (uint8_t)r;
            p.cell_of_rank[r] = (uint8_t)k;
        }
        const uint64_t full = (K == 64) ? ~0ull : ((1ull << K) - 1ull);
        p.cell_visible = cell_visible ? (cell_visible[v] & full) : full;
        if (p.cell_visible != full) vt.culled = 1u;
    }
    vt.total_tiles = tile_off;
    // pixel offsets and global tile ids are 32-bit on the device; a cell rank is
    // packed below the tile id in 31 bits
    int64_t tot_px = 0, tot_tiles = 0;
    for (int v = 0; v < n_views; ++v) {
        tot_px += (int64_t)cams[v].width * cams[v].height;
        tot_tiles += tiles_of(cams[v]);
    }
    if (tot_px >= (1LL << 32) || (tot_tiles << L) >= (1LL << 31)) return RGS_E_UNSUPPORTED;
    memcpy(views_host, &vt, sizeof(vt));
    return RGS_OK;
}

rgs_status rgs_views_upload(const rgs_camera* cams, int32_t n_views, int32_t L, const int32_t* rank_of,
                            const uint64_t* cell_visible, void* views_dev, rgs_stream stream) {
    if (!views_dev) return RGS_E_ARG;
    ViewTable vt;
    const rgs_status st = rgs_views_pack(cams, n_views, L, rank_of, cell_visible, &vt);
    if (st != RGS_OK) return st;
    RGS_HIP_CHECK(hipMemcpyAsync(views_dev, &vt, sizeof(vt), hipMemcpyHostToDevice, S(stream)));
    // the host copy lives on this stack frame: make sure it has been consumed
    RGS_HIP_CHECK(hipStreamSynchronize(S(stream)));
    return RGS_OK;
}

size_t rgs_kd_partition_workspace(int64_t n, int32_t L) {
    if (n < 0 || L < 0 || L > RGS_MAX_L) return 0;
    return kd_ws_bytes(n, L);
}

rgs_status rgs_kd_partition(const rgs_gaussians* g, int32_t L, float d_factor, int32_t rule, const rgs_kdtree* kd,
                            void* ws, size_t ws_bytes, rgs_stream stream) {
    if (!gauss_ok(g) || !kd || L < 0 || L > RGS_MAX_L || !kd->split || !kd->box_lo || !kd->box_hi || !kd->counts)
        return RGS_E_ARG;
    if (rule != RGS_SPLIT_MEDIAN && rule != RGS_SPLIT_MIDPOINT) return RGS_E_ARG;
    if (g->n > 0 && !kd->center_cell) return RGS_E_ARG;
    if (!ws_ok(ws, ws_bytes, kd_ws_bytes(g->n, L))) return RGS_E_ARG;
    if (g->n > 0x7fffffff) return RGS_E_UNSUPPORTED;
    const int K = 1 << L;
    const int64_t n = g->n;
    const size_t mb = (size_t)(n > 0 ? n : 0) * ((K + 31) / 32) * 4;
    if (!disjoint({{kd->split, (size_t)(K > 1 ? K - 1 : 1) * 4}, {kd->box_lo, (size_t)12 * K}, {kd->box_hi, (size_t)12 * K},
                   {kd->center_cell, (size_t)n * 4}, {kd->counts, (size_t)4 * K}, {kd->own_mask, mb},
                   {kd->cell_bounds, (size_t)32 * K}, {ws, ws_bytes}},
                  {{g->means, (size_t)12 * n}, {g->log_scales, (size_t)12 * n}}))
        return RGS_E_ARG;
    return kd_partition(g, L, d_factor, rule, kd, ws, S(stream));
}

size_t rgs_group_by_cell_workspace(int64_t n) { return n < 0 ? 0 : group_ws_bytes(n); }

rgs_status rgs_group_by_cell(const rgs_gaussians* in, const rgs_kdtree* kd, int32_t L, const rgs_gaussians* out,
                             int32_t* perm, void* ws, size_t ws_bytes, rgs_stream stream) {
    if (!gauss_ok(in) || !gauss_ok(out) || !kd || L < 0 || L > RGS_MAX_L) return RGS_E_ARG;
    if (out->n != in->n || out->sh_degree != in->sh_degree) return RGS_E_ARG;
    if (in->n > 0 && (!kd->center_cell || !kd->cell_bounds)) return RGS_E_ARG;
    const int K = 1 << L;
    if (!disjoint(concat(gauss_spans(out), {{perm, (size_t)4 * (size_t)in->n}, {ws, ws_bytes}}),
                  concat(gauss_spans(in), {{kd->center_cell, (size_t)4 * (size_t)in->n}, {kd->cell_bounds, (size_t)32 * K}})))
        return RGS_E_ARG;
    if (!ws_ok(ws, ws_bytes, group_ws_bytes(in->n))) return RGS_E_ARG;
    if (in->n > 0x7fffffff) return RGS_E_UNSUPPORTED;
    return group_by_cell(in, kd, L, out, perm, ws, ws_bytes, S(stream));
}

static void order_rec(int nd, int depth, int L, const float* split, const float* o, int32_t* order, int* pos) {
    const int K = 1 << L;
    if (depth == L) { order[(*pos)++] = nd - (K - 1); return; }
    const int a = depth % 3;
    if (o[a] < split[nd]) {
        order_rec(2 * nd + 1, depth + 1, L, split, o, order, pos);
        order_rec(2 * nd + 2, depth + 1, L, split, o, order, pos);
    } else {
        order_rec(2 * nd + 2, depth + 1, L, split, o, order, pos);
        order_rec(2 * nd + 1, depth + 1, L, split, o, order, pos);
    }
}

rgs_status rgs_cell_order(int32_t L, const float* split_host, const float campos[3], int32_t* order, int32_t* rank_of) {
    if (L < 0 || L > RGS_MAX_L || !campos || !order || !rank_of || (L > 0 && !split_host)) return RGS_E_ARG;
    int pos = 0;
    order_rec(0, 0, L, split_host, campos, order, &pos);
    for (int r = 0; r < (1 << L); ++r) rank_of[order[r]] = r;
    return RGS_OK;
}

// Per view, the cells that may hold a Gaussian whose footprint reaches the
// image.  A Gaussian reaches pixel columns only within its rectangle
// m_x +- e_x, and the projection's own screen test shows e_x <= 3.03 sqrt(B)
// + 2^-17 (B_x + B_y) + 2 + 1e-5 |m_x| with B = (f/z)^2 (1 + g)^2 s^2 + 0.3:
// the camera rotation keeps lengths, the 3D covariance's largest eigenvalue
// is s^2 (s the largest scale), the Jacobian row at the guarded centre has
// norm <= (f/z)(1 + g) (g the guard: the linearisation reaches beyond the
// perspective image of the 3-sigma sphere by up to that factor), tau <= 9
// covers the 3-sigma cut and the 0.3 px^2 low-pass, and the rectangle's
// fp32 rounding pads are inside the 2^-17 and constant terms.  Multiplying
// m_x + e_x >= 0 by z / f (z > z_near > 0) gives a test affine in the
// camera-space centre: x + a z + r >= 0, with a = (cx + 3.03 sqrt(0.3) + 3)
// / f and r = 3.03 (1 + g) s + 2^-17 (fx + fy^2 / fx) (1 + g)^2 s^2 / z_lo +
// 1e-5 (|x| + z cx / f); likewise for the other three sides.  Over a cell's
// box of centres (the largest scale of its Gaussians) an affine function
// peaks at a corner, so a cell is dropped only if some side fails at all
// eight corners, or every corner lies at z <= z_near: every Gaussian of the
// cell then has an empty rectangle or is behind the near plane, exactly the
// pairs the projection would cull.  All in fp64 with a relative pad of 1e-5.
static uint64_t cell_visible_mask(const rgs_camera& c, int L, const float* cb) {
    const int K = 1 << L;
    const double R[9] = {c.R[0], c.R[1], c.R[2], c.R[3], c.R[4], c.R[5], c.R[6], c.R[7], c.R[8]};
    const double tc[3] = {c.t[0], c.t[1], c.t[2]};
    const double fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy, W = c.width, H = c.height, zn = c.z_near;
    const double gx = 1.3 * (fmax(cx, W - cx) / fx), gy = 1.3 * (fmax(cy, H - cy) / fy);
    const double pad_px = 3.03 * sqrt(0.3) + 3.0;
    const double aL = (cx + pad_px) / fx, aR = (W - cx + pad_px) / fx;
    const double aT = (cy + pad_px) / fy, aB = (H - cy + pad_px) / fy;
    const double g2 = fmax(gx, gy);
    uint64_t vis = 0;
    for (int k = 0; k < K; ++k) {
        const double lo[3] = {cb[0 * K + k], cb[1 * K + k], cb[2 * K + k]};
        const double hi[3] = {cb[3 * K + k], cb[4 * K + k], cb[5 * K + k]};
        const double smax = cb[6 * K + k];
        bool empty = false, finite = isfinite(smax) && smax >= 0.0;
        for (int a = 0; a < 3; ++a) {
            if (lo[a] > hi[a]) empty = true;               // no centres (+inf / -inf bounds)
            if (!isfinite(lo[a]) || !isfinite(hi[a])) finite = false;
        }
        if (empty) continue;
        if (!finite) { vis |= 1ull << k; continue; }
        double t[8][3], zmin = INFINITY, zmax = -INFINITY, amax = 0.0;
        for (int j = 0; j < 8; ++j) {
            const double p[3] = {(j & 1) ? hi[0] : lo[0], (j & 2) ? hi[1] : lo[1], (j & 4) ? hi[2] : lo[2]};
            for (int r = 0; r < 3; ++r) {
                t[j][r] = R[3 * r] * p[0] + R[3 * r + 1] * p[1] + R[3 * r + 2] * p[2] + tc[r];
                amax = fmax(amax, fabs(R[3 * r] * p[0]) + fabs(R[3 * r + 1] * p[1]) + fabs(R[3 * r + 2] * p[2]) +
                                      fabs(tc[r]));
            }
            zmin = fmin(zmin, t[j][2]);
            zmax = fmax(zmax, t[j][2]);
        }
        const double eps = 1e-5 * amax + 1e-30;   // fp32 camera transform and rounding of the corners
        if (zmax + eps <= zn) continue;            // every centre behind the near plane
        const double zlo = fmax(zn, zmin) * (1.0 - 1e-5);
        const double s = smax * 1.001;
        const double quad = 0x1p-17 * (fx + fy * fy / fx + fy + fx * fx / fy) * (1.0 + g2) * (1.0 + g2) * s * s / zlo;
        double xmax = 0.0, ymax = 0.0;
        for (int j = 0; j < 8; ++j) {
            xmax = fmax(xmax, fabs(t[j][0]) + t[j][2] * cx / fx);
            ymax = fmax(ymax, fabs(t[j][1]) + t[j][2] * cy / fy);
        }
        const double rx = 3.03 * (1.0 + gx) * s + quad + 1e-5 * xmax + eps * (1.0 + aL + aR);
        const double ry = 3.03 * (1.0 + gy) * s + quad + 1e-5 * ymax + eps * (1.0 + aT + aB);
        double mL = -INFINITY, mR = -INFINITY, mT = -INFINITY, mB = -INFINITY;
        for (int j = 0; j < 8; ++j) {
            mL = fmax(mL, t[j][0] + aL * t[j][2]);
            mR = fmax(mR, -t[j][0] + aR * t[j][2]);
            mT = fmax(mT, t[j][1] + aT * t[j][2]);
            mB = fmax(mB, -t[j][1] + aB * t[j][2]);
        }
        if (mL + rx < 0.0 || mR + rx < 0.0 || mT + ry < 0.0 || mB + ry < 0.0) continue;
        vis |= 1ull << k;
    }
    return vis;
}

rgs_status rgs_cell_visibility(const rgs_camera* cams, int32_t n_views, int32_t L, const float* cell_bounds_host,
                               uint64_t* visible) {
    if (!cams || n_views < 1 || L < 0 || L > RGS_MAX_L || !cell_bounds_host || !visible) return RGS_E_ARG;
    for (int v = 0; v < n_views; ++v)
        if (!cams_ok(cams + v, 1)) return RGS_E_ARG;
    for (int v = 0; v < n_views; ++v) visible[v] = cell_visible_mask(cams[v], L, cell_bounds_host);
    return RGS_OK;
}

static bool proj_ok(const rgs_projected* p) { return p && p->rec && p->bin && p->count && p->depth; }

rgs_status rgs_project_sh(const rgs_gaussians* g, const rgs_camera* cams, int32_t n_views, const void* views_dev,
                          const rgs_kdtree* kd, int32_t cells, const rgs_projected* out, rgs_stream stream) {
    if (!gauss_ok(g) || !cams_ok(cams, n_views) || !views_dev || !kd || !proj_ok(out)) return RGS_E_ARG;
    if (kd->L < 0 || kd->L > RGS_MAX_L || (kd->L > 0 && !kd->split)) return RGS_E_ARG;
    if (cells != RGS_CELLS_EXACT && cells != RGS_CELLS_PAPER_SUBSETS && cells != RGS_CELLS_EXCLUSIVE) return RGS_E_ARG;
    if (g->n > 0 && cells == RGS_CELLS_PAPER_SUBSETS && !kd->own_mask) return RGS_E_ARG;
    if (g->n > 0 && cells == RGS_CELLS_EXCLUSIVE && !kd->center_cell) return RGS_E_ARG;
    if ((int64_t)n_views * g->n >= 0x7fffffffLL) return RGS_E_UNSUPPORTED;
    const size_t m = (size_t)n_views * (size_t)g->n;
    if (!disjoint(proj_spans(out, m), gauss_spans(g)) || !disjoint(proj_spans(out, m), {{views_dev, sizeof(ViewTable)}}))
        return RGS_E_ARG;
    return project_launch(g, reinterpret_cast<const ViewTable*>(views_dev), kd->split, kd->center_cell, cells,
                          kd->own_mask, out, S(stream));
}

size_t rgs_bin_sort_workspace(int64_t n, int32_t n_views, int64_t total_tiles, int32_t L, int64_t capacity) {
    if (n < 0 || n_views < 1 || total_tiles < 0 || L < 0 || L > RGS_MAX_L || capacity < 0) return 0;
    return bin_ws_bytes(n, n_views, total_tiles, L, capacity);
}

static bool bins_ok(const rgs_bins* b) {
    return b && b->keys && b->vals && b->pair_src && b->pair_off && b->pair_rank && b->slot_key && b->slot_range &&
           b->tile_slot && b->slot_order && b->tile_order && b->counters && b->capacity >= 0 && b->slot_capacity >= 0;
}

rgs_status rgs_bin_sort(const rgs_projected* proj, int64_t n, const rgs_camera* cams, int32_t n_views,
                        const void* views_dev, int32_t L, rgs_bins* bins, int64_t* n_required, void* ws,
                        size_t ws_bytes, rgs_stream stream) {
    if (!proj_ok(proj) || n < 0 || !cams_ok(cams, n_views) || !views_dev || L < 0 || L > RGS_MAX_L || !bins_ok(bins) ||
        !ws)
        return RGS_E_ARG;
    const int64_t T = rgs_total_tiles(cams, n_views);
    if (!ws_ok(ws, ws_bytes, bin_ws_bytes(n, n_views, T, L, bins->capacity))) return RGS_E_ARG;
    if ((int64_t)n_views * n >= 0x7fffffffLL || bins->capacity >= 0xffffffffLL || (T << L) >= 0x7fffffffLL)
        return RGS_E_UNSUPPORTED;
    const size_t m = (size_t)n_views * (size_t)n;
    if (!disjoint(concat(bins_spans(bins, m, (size_t)T), {{ws, ws_bytes}}),
                  concat(proj_spans(proj, m), {{views_dev, sizeof(ViewTable)}})))
        return RGS_E_ARG;
    return bin_sort(proj, n, n_views, reinterpret_cast<const ViewTable*>(views_dev), L, T, bins, n_required, true, ws,
                    ws_bytes, S(stream));
}

rgs_status rgs_bin_sort_async(const rgs_projected* proj, int64_t n, const rgs_camera* cams, int32_t n_views,
                              const void* views_dev, int32_t L, rgs_bins* bins, void* ws, size_t ws_bytes,
                              rgs_stream stream) {
    if (!proj_ok(proj) || n < 0 || !cams_ok(cams, n_views) || !views_dev || L < 0 || L > RGS_MAX_L || !bins_ok(bins))
        return RGS_E_ARG;
    const int64_t T = rgs_total_tiles(cams, n_views);
    if (!ws_ok(ws, ws_bytes, bin_ws_bytes(n, n_views, T, L, bins->capacity))) return RGS_E_ARG;
    if ((int64_t)n_views * n >= 0x7fffffffLL || bins->capacity >= 0xffffffffLL || (T << L) >= 0x7fffffffLL)
        return RGS_E_UNSUPPORTED;
    const int64_t dense = T << L;
    if (bins->slot_capacity < (bins->capacity < dense ? bins->capacity : dense)) return RGS_E_ARG;
    const size_t m = (size_t)n_views * (size_t)n;
    if (!disjoint(concat(bins_spans(bins, m, (size_t)T), {{ws, ws_bytes}}),
                  concat(proj_spans(proj, m), {{views_dev, sizeof(ViewTable)}})))
        return RGS_E_ARG;
    return bin_sort(proj, n, n_views, reinterpret_cast<const ViewTable*>(views_dev), L, T, bins, nullptr, false, ws,
                    ws_bytes, S(stream));
}

// Grid bound for the per-slot kernels: slots <= min(instances, tiles x cells);
// with the instance count left on the device (n_instances < 0), the capacity.
static int64_t slot_bound_of(const rgs_bins* bins, const rgs_camera* cams, int32_t n_views, int L) {
    const int64_t dense = rgs_total_tiles(cams, n_views) << L;
    const int64_t ni = bins->n_instances >= 0 ? bins->n_instances : bins->capacity;
    int64_t b = ni < dense ? ni : dense;
    return b < bins->slot_capacity ? b : bins->slot_capacity;
}

rgs_status rgs_render_partial(const rgs_projected* proj, int64_t n, const rgs_bins* bins, const rgs_camera* cams,
                              int32_t n_views, const void* views_dev, const rgs_kdtree* kd, float eps_T,
                              const rgs_partials* out, uint64_t* stats, rgs_stream stream) {
    if (!proj_ok(proj) || n < 0 || !bins_ok(bins) || !cams_ok(cams, n_views) || !views_dev || !kd || !kd->box_lo ||
        !kd->box_hi || !out || !out->C || !out->T || !out->last || !(eps_T >= 0.f) || eps_T >= 1.f)
        return RGS_E_ARG;
    const size_t m = (size_t)n_views * (size_t)(n > 0 ? n : 0);
    const int K = 1 << kd->L;
    const Spans ins = concat(concat(proj_spans(proj, m), bins_spans(bins, m, total_tiles_of(cams, n_views))),
                             {{views_dev, sizeof(ViewTable)}, {kd->box_lo, (size_t)12 * K}, {kd->box_hi, (size_t)12 * K}});
    if (!disjoint(concat(parts_spans(out, bins), {{stats, 16}}), ins)) return RGS_E_ARG;
    return render_fwd_launch(proj, bins, reinterpret_cast<const ViewTable*>(views_dev), kd, eps_T, out, stats,
                             rgs_total_tiles(cams, n_views), S(stream));
}

rgs_status rgs_render_partial_merged(const rgs_projected* proj, int64_t n, const rgs_bins* bins,
                                     const rgs_camera* cams, int32_t n_views, const void* views_dev,
                                     const rgs_kdtree* kd, float eps_T, const rgs_partials* out, float* image,
                                     float* T_final, uint64_t* stats, rgs_stream stream) {
    if (!proj_ok(proj) || n < 0 || !bins_ok(bins) || !cams_ok(cams, n_views) || !views_dev || !kd || !kd->box_lo ||
        !kd->box_hi || !out || !out->C || !out->T || !out->last || !(eps_T >= 0.f) || eps_T >= 1.f || !image ||
        !T_final)
        return RGS_E_ARG;
    const size_t m = (size_t)n_views * (size_t)(n > 0 ? n : 0);
    const int K = 1 << kd->L;
    const size_t px = pixels_of(cams, n_views);
    const Spans ins = concat(concat(proj_spans(proj, m), bins_spans(bins, m, total_tiles_of(cams, n_views))),
                             {{views_dev, sizeof(ViewTable)}, {kd->box_lo, (size_t)12 * K}, {kd->box_hi, (size_t)12 * K}});
    // outputs pairwise disjoint and disjoint from the inputs
    if (!disjoint(concat(parts_spans(out, bins), {{stats, 16}, {image, 12 * px}, {T_final, 4 * px}}), ins))
        return RGS_E_ARG;
    return render_fwd_launch(proj, bins, reinterpret_cast<const ViewTable*>(views_dev), kd, eps_T, out, stats,
                             rgs_total_tiles(cams, n_views), S(stream), image, T_final);
}

rgs_status rgs_merge_partials(const rgs_partials* parts, const rgs_bins* bins, const rgs_camera* cams, int32_t n_views,
                              const void* views_dev, float* image, float* T_final, rgs_stream stream) {
    if (!parts || !parts->C || !parts->T || !bins_ok(bins) || !cams_ok(cams, n_views) || !views_dev || !image || !T_final)
        return RGS_E_ARG;
    const size_t px = pixels_of(cams, n_views);
    if (!disjoint({{image, 12 * px}, {T_final, 4 * px}},
                  concat(concat(parts_spans(parts, bins), bins_spans(bins, 0, total_tiles_of(cams, n_views))),
                         {{views_dev, sizeof(ViewTable)}})))
        return RGS_E_ARG;
    return merge_fwd_launch(parts, bins, reinterpret_cast<const ViewTable*>(views_dev), rgs_total_tiles(cams, n_views),
                            image, T_final, S(stream));
}

size_t rgs_loss_workspace(int32_t H, int32_t W) {
    if (H <= 0 || W <= 0) return 0;
    return loss_ws_bytes(H, W);
}

rgs_status rgs_loss_l1_ssim(const float* image, const float* target, int32_t H, int32_t W, float ssim_weight, float* loss,
                            float* d_image, void* ws, size_t ws_bytes, rgs_stream stream) {
    if (!image || !target || !loss || !d_image || !ws || H <= 0 || W <= 0 || !isfinite(ssim_weight)) return RGS_E_ARG;
    if (!ws_ok(ws, ws_bytes, loss_ws_bytes(H, W))) return RGS_E_ARG;
    const size_t hw = (size_t)H * (size_t)W;
    if (!disjoint({{loss, 4}, {d_image, 12 * hw}, {ws, ws_bytes}}, {{image, 12 * hw}, {target, 12 * hw}}))
        return RGS_E_ARG;
    return loss_launch(image, target, H, W, ssim_weight, loss, d_image, ws, S(stream));
}

rgs_status rgs_loss_l1_ssim_noalloc(const float* image, const float* target, int32_t H, int32_t W, float ssim_weight,
                                    float* loss, float* d_image, rgs_stream stream) {
    if (!image || !target || !loss || !d_image || H <= 0 || W <= 0 || !isfinite(ssim_weight)) return RGS_E_ARG;
    if (loss_ws_bytes(H, W) > RGS_LOSS_SCRATCH_BYTES) return RGS_E_CAPACITY;
    const size_t hw = (size_t)H * (size_t)W;
    if (!disjoint({{loss, 4}, {d_image, 12 * hw}}, {{image, 12 * hw}, {target, 12 * hw}})) return RGS_E_ARG;
    void* ws = nullptr;
    const rgs_status st = loss_scratch(&ws);
    if (st != RGS_OK) return st;
    return loss_launch(image, target, H, W, ssim_weight, loss, d_image, ws, S(stream));
}

rgs_status rgs_merge_partials_bwd(const float* d_image, const float* d_T_final, const rgs_partials* parts,
                                  const rgs_bins* bins, const rgs_camera* cams, int32_t n_views, const void* views_dev,
                                  const rgs_partials_grad* out, rgs_stream stream) {
    if (!d_image || !parts || !parts->C || !parts->T || !bins_ok(bins) || !cams_ok(cams, n_views) || !views_dev || !out ||
        !out->dC || !out->dT)
        return RGS_E_ARG;
    const size_t px = pixels_of(cams, n_views);
    const size_t sc = (size_t)(bins->slot_capacity > 0 ? bins->slot_capacity : 0);
    if (!disjoint({{out->dC, 3072 * sc}, {out->dT, 1024 * sc}},
                  concat(concat(parts_spans(parts, bins), bins_spans(bins, 0, total_tiles_of(cams, n_views))),
                         {{views_dev, sizeof(ViewTable)}, {d_image, 12 * px}, {d_T_final, 4 * px}})))
        return RGS_E_ARG;
    return merge_bwd_launch(d_image, d_T_final, parts, bins, reinterpret_cast<const ViewTable*>(views_dev),
                            rgs_total_tiles(cams, n_views), out, S(stream));
}

size_t rgs_render_bwd_workspace(int64_t capacity) {
    if (capacity < 0) return 0;
    return render_bwd_ws_bytes(capacity);
}

static bool bwd_args_ok(const rgs_partials_grad* dparts, const rgs_partials* parts, const rgs_bins* bins,
                        const rgs_projected* proj, int64_t n, const rgs_camera* cams, int32_t n_views,
                        const void* views_dev, const rgs_kdtree* kd, const void* ws, size_t ws_bytes,
                        const Spans& extra_out) {
    if (!dparts || !dparts->dC || !dparts->dT || !parts || !parts->T || !parts->last || !bins_ok(bins) || !proj_ok(proj) ||
        n < 0 || !cams_ok(cams, n_views) || !views_dev || !kd || !kd->box_lo || !kd->box_hi)
        return false;
    if (!ws_ok(ws, ws_bytes, render_bwd_ws_bytes(bins->capacity))) return false;
    const size_t m = (size_t)n_views * (size_t)n;
    const size_t sc = (size_t)(bins->slot_capacity > 0 ? bins->slot_capacity : 0);
    const int K = 1 << kd->L;
    const Spans ins =
        concat(concat(concat(proj_spans(proj, m), bins_spans(bins, m, total_tiles_of(cams, n_views))), parts_spans(parts, bins)),
               {{dparts->dC, 3072 * sc}, {dparts->dT, 1024 * sc}, {views_dev, sizeof(ViewTable)},
                {kd->box_lo, (size_t)12 * K}, {kd->box_hi, (size_t)12 * K}});
    return disjoint(concat({{ws, ws_bytes}}, extra_out), ins);
}

rgs_status rgs_render_partial_bwd_records(const rgs_partials_grad* dparts, const rgs_partials* parts,
                                          const rgs_bins* bins, const rgs_projected* proj, int64_t n,
                                          const rgs_camera* cams, int32_t n_views, const void* views_dev,
                                          const rgs_kdtree* kd, void* ws, size_t ws_bytes, uint64_t* stats,
                                          rgs_stream stream) {
    if (!bwd_args_ok(dparts, parts, bins, proj, n, cams, n_views, views_dev, kd, ws, ws_bytes, {{stats, 16}}))
        return RGS_E_ARG;
    return render_bwd_records_launch(dparts, parts, bins, proj, reinterpret_cast<const ViewTable*>(views_dev), kd, ws,
                                     stats, slot_bound_of(bins, cams, n_views, kd->L), S(stream));
}

rgs_status rgs_pair_reduce(const rgs_bins* bins, const rgs_projected* proj, int64_t n, int32_t n_views, float* d_proj,
                           void* ws, size_t ws_bytes, rgs_stream stream) {
    if (!bins_ok(bins) || !proj_ok(proj) || n < 0 || n_views < 1 || n_views > RGS_MAX_VIEWS || !d_proj) return RGS_E_ARG;
    if (!ws_ok(ws, ws_bytes, render_bwd_ws_bytes(bins->capacity))) return RGS_E_ARG;
    const size_t m = (size_t)n_views * (size_t)n;
    if (!disjoint({{d_proj, 36 * m}}, concat(concat(proj_spans(proj, m), bins_spans(bins, m, 0)), {{ws, ws_bytes}})))
        return RGS_E_ARG;
    return pair_reduce_launch(bins, proj, n, n_views, d_proj, ws, S(stream));
}

rgs_status rgs_render_partial_bwd(const rgs_partials_grad* dparts, const rgs_partials* parts, const rgs_bins* bins,
                                  const rgs_projected* proj, int64_t n, const rgs_camera* cams, int32_t n_views,
                                  const void* views_dev, const rgs_kdtree* kd, float* d_proj, void* ws, size_t ws_bytes,
                                  rgs_stream stream) {
    if (!d_proj || n < 0 ||
        !bwd_args_ok(dparts, parts, bins, proj, n, cams, n_views, views_dev, kd, ws, ws_bytes,
                     {{d_proj, (size_t)36 * (size_t)n_views * (size_t)n}}))
        return RGS_E_ARG;
    rgs_status st = render_bwd_records_launch(dparts, parts, bins, proj, reinterpret_cast<const ViewTable*>(views_dev),
                                              kd, ws, nullptr, slot_bound_of(bins, cams, n_views, kd->L), S(stream));
    if (st != RGS_OK) return st;
    return pair_reduce_launch(bins, proj, n, n_views, d_proj, ws, S(stream));
}

rgs_status rgs_project_sh_bwd(const float* d_proj, const rgs_gaussians* g, const rgs_projected* proj,
                              const rgs_camera* cams, int32_t n_views, const void* views_dev,
                              const rgs_gaussians_grad* out, rgs_stream stream) {
    if (!d_proj || !gauss_ok(g) || !proj_ok(proj) || !cams_ok(cams, n_views) || !views_dev || !out) return RGS_E_ARG;
    if (g->n > 0 && (!out->means || !out->log_scales || !out->quats || !out->opacity || !out->sh)) return RGS_E_ARG;
    const size_t m = (size_t)n_views * (size_t)g->n;
    if (!disjoint(grad_spans(out, g), concat(concat(gauss_spans(g), proj_spans(proj, m)),
                                             {{d_proj, 36 * m}, {views_dev, sizeof(ViewTable)}})))
        return RGS_E_ARG;
    return project_bwd_launch(d_proj, g, proj->count, reinterpret_cast<const ViewTable*>(views_dev), out, S(stream));
}

static bool grad_ptrs_ok(const rgs_gaussians_grad* g) {
    return g && g->means && g->log_scales && g->quats && g->opacity && g->sh;
}

rgs_status rgs_adam_step(const rgs_gaussians_grad* params, const rgs_gaussians_grad* grads, const rgs_gaussians_grad* m,
                         const rgs_gaussians_grad* v, int64_t n, int32_t sh_degree, const rgs_adam_params* hp,
                         rgs_stream stream) {
    if (n < 0 || sh_degree < 0 || sh_degree > 3 || !hp || !params || !grads || !m || !v) return RGS_E_ARG;
    if (n > 0 && (!grad_ptrs_ok(params) || !grad_ptrs_ok(grads) || !grad_ptrs_ok(m) || !grad_ptrs_ok(v))) return RGS_E_ARG;
    if (hp->step < 1 || !(hp->beta1 >= 0.0 && hp->beta1 < 1.0) || !(hp->beta2 >= 0.0 && hp->beta2 < 1.0) ||
        !(hp->eps >= 0.0) || !isfinite(hp->eps))
        return RGS_E_ARG;
    const float lrs[6] = {hp->lr_means, hp->lr_log_scales, hp->lr_quats, hp->lr_opacity, hp->lr_sh_dc, hp->lr_sh_rest};
    for (float lr : lrs)
        if (!isfinite(lr)) return RGS_E_ARG;
    rgs_gaussians shape;
    shape.n = n;
    shape.sh_degree = sh_degree;
    shape.means = shape.log_scales = shape.quats = shape.opacity = shape.sh = nullptr;
    const Spans sp = grad_spans(params, &shape), sm = grad_spans(m, &shape), sv = grad_spans(v, &shape),
                sg = grad_spans(grads, &shape);
    if (!disjoint(concat(concat(sp, sm), sv), sg)) return RGS_E_ARG;
    return adam_launch(params, grads, m, v, n, sh_degree, hp, S(stream));
}

rgs_status rgs_permute_gaussians(const rgs_gaussians* in, const int32_t* perm, const rgs_gaussians_grad* out,
                                 rgs_stream stream) {
    if (!gauss_ok(in) || !out) return RGS_E_ARG;
    if (in->n > 0 && (!perm || !grad_ptrs_ok(out))) return RGS_E_ARG;
    if (in->n > 0x7fffffff) return RGS_E_UNSUPPORTED;
    if (!disjoint(grad_spans(out, in), concat(gauss_spans(in), {{perm, (size_t)4 * (size_t)in->n}}))) return RGS_E_ARG;
    return permute_launch(in, perm, out, S(stream));
}

}  // extern "C"
