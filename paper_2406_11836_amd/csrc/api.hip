// api.hip -- the extern "C" entry points of librgs (declared in include/rgs.h):
// argument validation, the device view table, and kernel dispatch.
#include <math.h>
#include <string.h>

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
rgs_status kd_partition(const rgs_gaussians* g, int L, float d_factor, const rgs_kdtree* kd, void* ws, hipStream_t s);
rgs_status project_launch(const rgs_gaussians* g, const ViewTable* vt, const float* split, const int32_t* center_cell,
                          const rgs_projected* out, hipStream_t s);
rgs_status project_bwd_launch(const float* dproj, const rgs_gaussians* g, const uint32_t* count, const ViewTable* vt,
                              const rgs_gaussians_grad* out, hipStream_t s);
size_t bin_ws_bytes(int64_t n, int n_views, int64_t total_tiles, int L, int64_t capacity);
size_t group_ws_bytes(int64_t n);
rgs_status group_by_cell(const rgs_gaussians* in, const rgs_kdtree* kd, int L, const rgs_gaussians* out, int32_t* perm,
                         void* ws, size_t ws_bytes, hipStream_t s);
rgs_status bin_sort(const rgs_projected* proj, int64_t n, int n_views, const ViewTable* vt_dev, int L, int64_t total_tiles,
                    rgs_bins* bins, int64_t* n_required, bool sync, void* ws, size_t ws_bytes, hipStream_t s);
rgs_status render_fwd_launch(const rgs_projected* proj, const rgs_bins* bins, const ViewTable* vt, const rgs_kdtree* kd,
                             float eps_T, const rgs_partials* out, uint64_t* stats, int64_t slot_bound, hipStream_t s);
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
size_t loss_ws_bytes(int H, int W);
rgs_status loss_launch(const float* image, const float* target, int H, int W, float ssim_w, float* loss, float* dimg,
                       void* ws, hipStream_t s);
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

static int64_t tiles_of(const rgs_camera& c) {
    return (int64_t)((c.width + 15) / 16) * (int64_t)((c.height + 15) / 16);
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

rgs_status rgs_kd_partition(const rgs_gaussians* g, int32_t L, float d_factor, const rgs_kdtree* kd, void* ws,
                            size_t ws_bytes, rgs_stream stream) {
    if (!gauss_ok(g) || !kd || L < 0 || L > RGS_MAX_L || !kd->split || !kd->box_lo || !kd->box_hi || !kd->counts)
        return RGS_E_ARG;
    if (g->n > 0 && !kd->center_cell) return RGS_E_ARG;
    if (!ws_ok(ws, ws_bytes, kd_ws_bytes(g->n, L))) return RGS_E_ARG;
    if (g->n > 0x7fffffff) return RGS_E_UNSUPPORTED;
    return kd_partition(g, L, d_factor, kd, ws, S(stream));
}

size_t rgs_group_by_cell_workspace(int64_t n) { return n < 0 ? 0 : group_ws_bytes(n); }

rgs_status rgs_group_by_cell(const rgs_gaussians* in, const rgs_kdtree* kd, int32_t L, const rgs_gaussians* out,
                             int32_t* perm, void* ws, size_t ws_bytes, rgs_stream stream) {
    if (!gauss_ok(in) || !gauss_ok(out) || !kd || L < 0 || L > RGS_MAX_L) return RGS_E_ARG;
    if (out->n != in->n || out->sh_degree != in->sh_degree) return RGS_E_ARG;
    if (in->n > 0 && (!kd->center_cell || !kd->cell_bounds)) return RGS_E_ARG;
    if (in->n > 0 && (out->means == in->means || out->sh == in->sh || out->quats == in->quats ||
                      out->log_scales == in->log_scales || out->opacity == in->opacity))
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

static bool proj_ok(const rgs_projected* p) { return p && p->rec && p->rect && p->cellmask && p->count && p->depth; }

rgs_status rgs_project_sh(const rgs_gaussians* g, const rgs_camera* cams, int32_t n_views, const void* views_dev,
                          const rgs_kdtree* kd, const rgs_projected* out, rgs_stream stream) {
    if (!gauss_ok(g) || !cams_ok(cams, n_views) || !views_dev || !kd || !proj_ok(out)) return RGS_E_ARG;
    if (kd->L < 0 || kd->L > RGS_MAX_L || (kd->L > 0 && !kd->split)) return RGS_E_ARG;
    if ((int64_t)n_views * g->n >= 0x7fffffffLL) return RGS_E_UNSUPPORTED;
    return project_launch(g, reinterpret_cast<const ViewTable*>(views_dev), kd->split, kd->center_cell, out, S(stream));
}

size_t rgs_bin_sort_workspace(int64_t n, int32_t n_views, int64_t total_tiles, int32_t L, int64_t capacity) {
    if (n < 0 || n_views < 1 || total_tiles < 0 || L < 0 || L > RGS_MAX_L || capacity < 0) return 0;
    return bin_ws_bytes(n, n_views, total_tiles, L, capacity);
}

static bool bins_ok(const rgs_bins* b) {
    return b && b->keys && b->vals && b->pair_src && b->pair_off && b->pair_rank && b->slot_key && b->slot_range &&
           b->tile_slot && b->slot_order && b->counters && b->capacity >= 0 && b->slot_capacity >= 0;
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
    return render_fwd_launch(proj, bins, reinterpret_cast<const ViewTable*>(views_dev), kd, eps_T, out, stats,
                             slot_bound_of(bins, cams, n_views, kd->L), S(stream));
}

rgs_status rgs_merge_partials(const rgs_partials* parts, const rgs_bins* bins, const rgs_camera* cams, int32_t n_views,
                              const void* views_dev, float* image, float* T_final, rgs_stream stream) {
    if (!parts || !parts->C || !parts->T || !bins_ok(bins) || !cams_ok(cams, n_views) || !views_dev || !image || !T_final)
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
    if (d_image == image || d_image == target) return RGS_E_ARG;
    return loss_launch(image, target, H, W, ssim_weight, loss, d_image, ws, S(stream));
}

rgs_status rgs_merge_partials_bwd(const float* d_image, const float* d_T_final, const rgs_partials* parts,
                                  const rgs_bins* bins, const rgs_camera* cams, int32_t n_views, const void* views_dev,
                                  const rgs_partials_grad* out, rgs_stream stream) {
    if (!d_image || !parts || !parts->C || !parts->T || !bins_ok(bins) || !cams_ok(cams, n_views) || !views_dev || !out ||
        !out->dC || !out->dT)
        return RGS_E_ARG;
    if (out->dC == parts->C || out->dT == parts->T) return RGS_E_ARG;
    return merge_bwd_launch(d_image, d_T_final, parts, bins, reinterpret_cast<const ViewTable*>(views_dev),
                            rgs_total_tiles(cams, n_views), out, S(stream));
}

size_t rgs_render_bwd_workspace(int64_t capacity) {
    if (capacity < 0) return 0;
    return render_bwd_ws_bytes(capacity);
}

static bool bwd_args_ok(const rgs_partials_grad* dparts, const rgs_partials* parts, const rgs_bins* bins,
                        const rgs_projected* proj, int64_t n, const rgs_camera* cams, int32_t n_views,
                        const void* views_dev, const rgs_kdtree* kd, const void* ws, size_t ws_bytes) {
    if (!dparts || !dparts->dC || !dparts->dT || !parts || !parts->T || !parts->last || !bins_ok(bins) || !proj_ok(proj) ||
        n < 0 || !cams_ok(cams, n_views) || !views_dev || !kd || !kd->box_lo || !kd->box_hi)
        return false;
    return ws_ok(ws, ws_bytes, render_bwd_ws_bytes(bins->capacity));
}

rgs_status rgs_render_partial_bwd_records(const rgs_partials_grad* dparts, const rgs_partials* parts,
                                          const rgs_bins* bins, const rgs_projected* proj, int64_t n,
                                          const rgs_camera* cams, int32_t n_views, const void* views_dev,
                                          const rgs_kdtree* kd, void* ws, size_t ws_bytes, uint64_t* stats,
                                          rgs_stream stream) {
    if (!bwd_args_ok(dparts, parts, bins, proj, n, cams, n_views, views_dev, kd, ws, ws_bytes)) return RGS_E_ARG;
    return render_bwd_records_launch(dparts, parts, bins, proj, reinterpret_cast<const ViewTable*>(views_dev), kd, ws,
                                     stats, slot_bound_of(bins, cams, n_views, kd->L), S(stream));
}

rgs_status rgs_pair_reduce(const rgs_bins* bins, const rgs_projected* proj, int64_t n, int32_t n_views, float* d_proj,
                           void* ws, size_t ws_bytes, rgs_stream stream) {
    if (!bins_ok(bins) || !proj_ok(proj) || n < 0 || n_views < 1 || n_views > RGS_MAX_VIEWS || !d_proj) return RGS_E_ARG;
    if (!ws_ok(ws, ws_bytes, render_bwd_ws_bytes(bins->capacity))) return RGS_E_ARG;
    return pair_reduce_launch(bins, proj, n, n_views, d_proj, ws, S(stream));
}

rgs_status rgs_render_partial_bwd(const rgs_partials_grad* dparts, const rgs_partials* parts, const rgs_bins* bins,
                                  const rgs_projected* proj, int64_t n, const rgs_camera* cams, int32_t n_views,
                                  const void* views_dev, const rgs_kdtree* kd, float* d_proj, void* ws, size_t ws_bytes,
                                  rgs_stream stream) {
    if (!bwd_args_ok(dparts, parts, bins, proj, n, cams, n_views, views_dev, kd, ws, ws_bytes) || !d_proj)
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
    return project_bwd_launch(d_proj, g, proj->count, reinterpret_cast<const ViewTable*>(views_dev), out, S(stream));
}

}  // extern "C"
