// Host runtime and C ABI of libflood (declared in include/flood.h).
//
// The runtime owns all device memory of a handle, validates every argument
// before touching the device, and drives the per-step kernel pair
// (planner + fused step) in batches.  A batch of G steps is captured once into
// a HIP graph and replayed; after each batch a one-lane kernel counts the
// members still short of t_end and the count is copied to pinned host memory.
// Two batches are kept in flight, so the host never stalls the device and at
// most one batch of no-op steps runs after the last member arrives.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/flood.h"
#include "flood_internal.h"
#include "flood_runtime.h"

namespace flood {

thread_local std::string g_create_error;

const char* status_name(flood_status s) {
    switch (s) {
        case FLOOD_OK: return "ok";
        case FLOOD_EINVAL: return "invalid argument";
        case FLOOD_ENOMEM: return "out of memory";
        case FLOOD_EHIP: return "HIP runtime error";
        case FLOOD_ESTATE: return "invalid state for this call";
        case FLOOD_ENUMERIC: return "non-finite or runaway depth";
        default: return "unknown status";
    }
}

bool finite_d(double v) { return std::isfinite(v); }

flood_status validate_grid(const flood_grid* g, std::string& err) {
    if (!g) { err = "grid is NULL"; return FLOOD_EINVAL; }
    if (g->ny < 1 || g->nx < 1) { err = "ny and nx must be >= 1"; return FLOOD_EINVAL; }
    if ((int64_t)g->ny * g->nx > (int64_t(1) << 28)) { err = "grid larger than 2^28 cells"; return FLOOD_EINVAL; }
    if (!(g->dx > 0.0) || !finite_d(g->dx)) { err = "dx must be finite and > 0"; return FLOOD_EINVAL; }
    if (!g->dem || !g->manning_n) { err = "dem and manning_n are required"; return FLOOD_EINVAL; }
    const int64_t nc = (int64_t)g->ny * g->nx;
    for (int64_t i = 0; i < nc; ++i) {
        if (!std::isfinite(g->dem[i])) { err = "dem has a non-finite value"; return FLOOD_EINVAL; }
        if (!(g->manning_n[i] > 0.0f) || !std::isfinite(g->manning_n[i])) {
            err = "manning_n must be finite and > 0";
            return FLOOD_EINVAL;
        }
        if (g->h0 && (!(g->h0[i] >= 0.0f) || !std::isfinite(g->h0[i]))) {
            err = "h0 must be finite and >= 0";
            return FLOOD_EINVAL;
        }
    }
    for (int e = 0; e < 4; ++e) {
        if (g->edge_kind[e] != FLOOD_EDGE_WALL && g->edge_kind[e] != FLOOD_EDGE_OPEN) {
            err = "edge_kind must be FLOOD_EDGE_WALL or FLOOD_EDGE_OPEN";
            return FLOOD_EINVAL;
        }
        if (g->edge_kind[e] == FLOOD_EDGE_OPEN && (!(g->edge_slope[e] > 0.0) || !finite_d(g->edge_slope[e]))) {
            err = "an open edge needs a finite edge_slope > 0";
            return FLOOD_EINVAL;
        }
    }
    return FLOOD_OK;
}

static bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

flood_status validate_params(const flood_params* p, std::string& err) {
    if (!p) { err = "params is NULL"; return FLOOD_EINVAL; }
    if (p->n_rain < 0 || (p->n_rain > 0 && !p->rain_rate)) { err = "rain_rate/n_rain inconsistent"; return FLOOD_EINVAL; }
    for (int i = 0; i < p->n_rain; ++i)
        if (!(p->rain_rate[i] >= 0.0) || !finite_d(p->rain_rate[i])) {
            err = "rain rates must be finite and >= 0";
            return FLOOD_EINVAL;
        }
    if (!(p->rain_interval > 0.0) || !finite_d(p->rain_interval)) { err = "rain_interval must be > 0"; return FLOOD_EINVAL; }
    if (!(p->g > 0.0) || !finite_d(p->g)) { err = "g must be > 0"; return FLOOD_EINVAL; }
    if (!(p->h_dry >= 0.0) || !finite_d(p->h_dry)) { err = "h_dry must be >= 0"; return FLOOD_EINVAL; }
    if (!(p->dt_fixed >= 0.0) || !finite_d(p->dt_fixed)) { err = "dt_fixed must be >= 0"; return FLOOD_EINVAL; }
    if (p->dt_fixed == 0.0) {
        if (!(p->cfl_alpha > 0.0 && p->cfl_alpha <= 1.0)) { err = "cfl_alpha must be in (0, 1]"; return FLOOD_EINVAL; }
        if (!(p->dt_cap > 0.0) || !finite_d(p->dt_cap)) { err = "dt_cap must be > 0"; return FLOOD_EINVAL; }
    }
    if (p->real_bytes != 4 && p->real_bytes != 8) { err = "real_bytes must be 4 or 8"; return FLOOD_EINVAL; }
    if (p->member_interleave != 0 && !pow2_in(p->member_interleave, 1, 8)) {
        err = "member_interleave must be 0, 1, 2, 4 or 8";
        return FLOOD_EINVAL;
    }
    if (p->tile_rows != 0 && !pow2_in(p->tile_rows, 1, 8)) { err = "tile_rows must be 0, 1, 2, 4 or 8"; return FLOOD_EINVAL; }
    if (p->chunks_per_block < 0) { err = "chunks_per_block must be >= 0"; return FLOOD_EINVAL; }
    if (p->step_kernel < 0 || p->step_kernel > 3) { err = "step_kernel must be 0, 1, 2 or 3"; return FLOOD_EINVAL; }
    if (p->step_kernel >= 2 && p->member_interleave > 1) {
        err = "the row-marching kernels need member_interleave 1";
        return FLOOD_EINVAL;
    }
    if (p->march_rows < 0 || p->march_rows > 4096) { err = "march_rows must be in [0, 4096]"; return FLOOD_EINVAL; }
    if (p->march_members != 0 && !pow2_in(p->march_members, 1, 8)) {
        err = "march_members must be 0, 1, 2, 4 or 8";
        return FLOOD_EINVAL;
    }
    if (p->track_peak != 0 && p->track_peak != 1) { err = "track_peak must be 0 or 1"; return FLOOD_EINVAL; }
    if (p->n_classes < 0 || p->n_classes > 4) { err = "n_classes must be in [0, 4]"; return FLOOD_EINVAL; }
    if (p->n_classes > 0) {
        if (!p->class_runoff || !p->class_drain) { err = "class_runoff and class_drain are required"; return FLOOD_EINVAL; }
        for (int k = 0; k < p->n_classes; ++k) {
            if (!(p->class_runoff[k] >= 0.0 && p->class_runoff[k] <= 1.0)) { err = "class_runoff must be in [0, 1]"; return FLOOD_EINVAL; }
            if (p->class_drain[k] != 0 && p->class_drain[k] != 1) { err = "class_drain must be 0 or 1"; return FLOOD_EINVAL; }
        }
        if (p->step_kernel == 1 || p->step_kernel == 2) { err = "land cover needs step_kernel 0 or 3"; return FLOOD_EINVAL; }
        if (p->member_interleave > 1) { err = "land cover needs member_interleave 0 or 1"; return FLOOD_EINVAL; }
    }
    if (p->n_inflow < 0) { err = "n_inflow must be >= 0"; return FLOOD_EINVAL; }
    if (p->n_inflow > 0) {
        if (!p->inflow) { err = "inflow is required"; return FLOOD_EINVAL; }
        if (p->n_series < 1 || p->n_series > 4) { err = "n_series must be in [1, 4]"; return FLOOD_EINVAL; }
        if (p->n_rain > 0 && !p->inflow_q) { err = "inflow_q is required"; return FLOOD_EINVAL; }
        for (int j = 0; j < p->n_series * p->n_rain; ++j)
            if (!(p->inflow_q[j] >= 0.0) || !finite_d(p->inflow_q[j])) {
                err = "inflow_q must be finite and >= 0";
                return FLOOD_EINVAL;
            }
        if (p->step_kernel == 1 || p->step_kernel == 2) { err = "inflow links need step_kernel 0 or 3"; return FLOOD_EINVAL; }
        if (p->member_interleave > 1) { err = "inflow links need member_interleave 0 or 1"; return FLOOD_EINVAL; }
    }
    return FLOOD_OK;
}

}  // namespace flood

using namespace flood;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* flood_strerror(flood_status s) { return status_name(s); }

const char* flood_last_error(const flood_handle* h) {
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

flood_status flood_create_batch(int32_t n_catch, const flood_grid* grids, const flood_params* params,
                                const int32_t* members_per_catch, const double* const* n_scale,
                                const double* const* rain_mult, void* hip_stream, flood_handle** out) {
    g_create_error.clear();
    if (!out) { g_create_error = "out is NULL"; return FLOOD_EINVAL; }
    *out = nullptr;
    if (n_catch < 1 || n_catch > FLOOD_MAX_CATCHMENTS) {
        g_create_error = "n_catch must be in [1, 8]";
        return FLOOD_EINVAL;
    }
    if (!grids || !params || !members_per_catch) { g_create_error = "grids/params/members are required"; return FLOOD_EINVAL; }
    for (int i = 0; i < n_catch; ++i) {
        flood_status st = validate_grid(&grids[i], g_create_error);
        if (st) return st;
        st = validate_params(&params[i], g_create_error);
        if (st) return st;
        if (params[i].real_bytes != params[0].real_bytes) {
            g_create_error = "real_bytes must agree across catchments";
            return FLOOD_EINVAL;
        }
        if (params[i].member_interleave != params[0].member_interleave) {
            g_create_error = "member_interleave must agree across catchments";
            return FLOOD_EINVAL;
        }
        if (params[i].step_kernel != params[0].step_kernel) {
            g_create_error = "step_kernel must agree across catchments";
            return FLOOD_EINVAL;
        }
        const int N = members_per_catch[i];
        if (N < 1 || N > FLOOD_MAX_MEMBERS) { g_create_error = "members per catchment must be in [1, 1024]"; return FLOOD_EINVAL; }
        // inflow links against the grid: edge, position, series, each link once
        if (params[i].n_inflow > 2 * (grids[i].nx + grids[i].ny)) {
            g_create_error = "n_inflow must be <= 2*(nx+ny)";
            return FLOOD_EINVAL;
        }
        {
            std::vector<uint8_t> seen(2 * ((size_t)grids[i].nx + grids[i].ny), 0);
            for (int k = 0; k < params[i].n_inflow; ++k) {
                const int32_t* f = params[i].inflow + 3 * k;
                const int e = f[0], pos = f[1];
                if (e < 0 || e > 3) { g_create_error = "inflow edge must be 0..3"; return FLOOD_EINVAL; }
                const int len = (e == 0 || e == 2) ? grids[i].nx : grids[i].ny;
                if (pos < 0 || pos >= len) { g_create_error = "inflow position outside the edge"; return FLOOD_EINVAL; }
                if (f[2] < 0 || f[2] >= params[i].n_series) {
                    g_create_error = "inflow series index must be < n_series";
                    return FLOOD_EINVAL;
                }
                const size_t at = e == 0 ? pos : e == 2 ? grids[i].nx + pos
                                                : e == 3 ? 2 * (size_t)grids[i].nx + pos
                                                         : 2 * (size_t)grids[i].nx + grids[i].ny + pos;
                if (seen[at]) { g_create_error = "an inflow link appears twice"; return FLOOD_EINVAL; }
                seen[at] = 1;
            }
        }
        const int K = params[i].n_classes;
        if ((K > 0) != (grids[i].land_class != nullptr)) {
            g_create_error = "a class map and n_classes > 0 go together";
            return FLOOD_EINVAL;
        }
        if (K > 0) {
            const size_t ncell = (size_t)grids[i].ny * grids[i].nx;
            for (size_t j = 0; j < ncell; ++j)
                if (grids[i].land_class[j] >= K) { g_create_error = "land_class values must be < n_classes"; return FLOOD_EINVAL; }
            if (!params[i].member_class_n) { g_create_error = "member_class_n is required"; return FLOOD_EINVAL; }
            for (size_t j = 0; j < (size_t)N * K; ++j)
                if (!(params[i].member_class_n[j] > 0.0) || !finite_d(params[i].member_class_n[j])) {
                    g_create_error = "member_class_n must be finite and > 0";
                    return FLOOD_EINVAL;
                }
            if (params[i].member_drain)
                for (int m = 0; m < N; ++m)
                    if (!(params[i].member_drain[m] >= 0.0) || !finite_d(params[i].member_drain[m])) {
                        g_create_error = "member_drain must be finite and >= 0";
                        return FLOOD_EINVAL;
                    }
        }
        for (int m = 0; m < N; ++m) {
            if (n_scale && n_scale[i] && (!(n_scale[i][m] > 0.0) || !finite_d(n_scale[i][m]))) {
                g_create_error = "n_scale must be finite and > 0";
                return FLOOD_EINVAL;
            }
            if (rain_mult && rain_mult[i] && (!(rain_mult[i][m] >= 0.0) || !finite_d(rain_mult[i][m]))) {
                g_create_error = "rain_mult must be finite and >= 0";
                return FLOOD_EINVAL;
            }
        }
    }
    std::unique_ptr<flood_handle> h(new flood_handle());
    flood_status st = create_impl(h.get(), n_catch, grids, params, members_per_catch, n_scale, rain_mult,
                                  (hipStream_t)hip_stream, g_create_error);
    if (st) return st;
    *out = h.release();
    return FLOOD_OK;
}

flood_status flood_create(const flood_grid* grid, const flood_params* params, int32_t n_members,
                          const double* n_scale, const double* rain_mult, void* hip_stream, flood_handle** out) {
    const double* ns[1] = {n_scale};
    const double* rm[1] = {rain_mult};
    return flood_create_batch(1, grid, params, &n_members, ns, rm, hip_stream, out);
}

#define FLOOD_NEED_HANDLE(h)                                  \
    do {                                                      \
        if (!(h) || !(h)->impl) return FLOOD_EINVAL;          \
        (h)->err.clear();                                     \
    } while (0)

flood_status flood_step(flood_handle* h, double t_end) {
    FLOOD_NEED_HANDLE(h);
    if (!std::isfinite(t_end)) { h->err = "t_end must be finite"; return FLOOD_EINVAL; }
    return h->impl->step(t_end, -1, h->err);
}

flood_status flood_step_n(flood_handle* h, double t_end, int64_t max_steps) {
    FLOOD_NEED_HANDLE(h);
    if (!std::isfinite(t_end)) { h->err = "t_end must be finite"; return FLOOD_EINVAL; }
    if (max_steps < 1) { h->err = "max_steps must be >= 1"; return FLOOD_EINVAL; }
    return h->impl->step(t_end, max_steps, h->err);
}

flood_status flood_get_wet_mask(flood_handle* h, int32_t catchment, int32_t member, uint8_t* wet_x, uint8_t* wet_y) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->get_wet_mask(catchment, member, wet_x, wet_y, h->err);
}

flood_status flood_log_steps(flood_handle* h, int32_t capacity) {
    FLOOD_NEED_HANDLE(h);
    if (capacity < 0 || capacity > (1 << 24)) { h->err = "capacity must be in [0, 2^24]"; return FLOOD_EINVAL; }
    return h->impl->log_steps(capacity, h->err);
}

flood_status flood_get_step_log(flood_handle* h, int32_t catchment, double* dt_out, double* t_end_out,
                                int64_t* count_out) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->get_step_log(catchment, dt_out, t_end_out, count_out, h->err);
}

flood_status flood_assimilate(flood_handle* h, int32_t catchment, int32_t n_gauges, const int32_t* gauge_rc,
                              const double* obs, const double* sigma, double neff_frac, double u0,
                              const double* beta, double* neff_out, int32_t* ancestors_out,
                              int32_t* resampled_out) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->assimilate(catchment, n_gauges, gauge_rc, obs, sigma, 0, 0.0, neff_frac, u0, beta, neff_out,
                               ancestors_out, resampled_out, h->err);
}

flood_status flood_assimilate_obs(flood_handle* h, int32_t catchment, int32_t n_gauges, const int32_t* gauge_rc,
                                  const double* obs, const double* sigma, double alpha, double neff_frac, double u0,
                                  const double* beta, double* neff_out, int32_t* ancestors_out,
                                  int32_t* resampled_out) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->assimilate(catchment, n_gauges, gauge_rc, obs, sigma, 1, alpha, neff_frac, u0, beta, neff_out,
                               ancestors_out, resampled_out, h->err);
}

flood_status flood_set_sections(flood_handle* h, int32_t catchment, int32_t n_sections, const int32_t* link_count,
                                const int32_t* links) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->set_sections(catchment, n_sections, link_count, links, h->err);
}

flood_status flood_get_sections(flood_handle* h, int32_t catchment, double* q_out) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->get_sections(catchment, q_out, h->err);
}

flood_status flood_adjoint(flood_handle* h, int32_t catchment, double t_end, double sample_dt, int32_t n_gauges,
                           const int32_t* gauge_rc, const double* obs, int32_t ckpt_every, double* loss_out,
                           double* grad_n_out, double* grad_mult_out) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->adjoint(catchment, t_end, sample_dt, n_gauges, gauge_rc, obs, ckpt_every, loss_out, grad_n_out,
                            grad_mult_out, h->err);
}

flood_status flood_get_field(flood_handle* h, int32_t catchment, int32_t member, int32_t which, double* host_out) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->get_field(catchment, member, which, host_out, h->err);
}

flood_status flood_set_state(flood_handle* h, int32_t catchment, int32_t member, const double* hh, const double* qx,
                             const double* qy, double t) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->set_state(catchment, member, hh, qx, qy, t, h->err);
}

flood_status flood_set_params(flood_handle* h, int32_t catchment, const float* manning_n, const double* n_scale,
                              const double* rain_mult) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->set_params(catchment, manning_n, n_scale, rain_mult, h->err);
}

flood_status flood_get_ledger(flood_handle* h, int32_t catchment, double* storage, double* rain_in, double* outflow,
                              double* clamp, double* drained, double* inflow, double* t, int64_t* steps) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->get_ledger(catchment, storage, rain_in, outflow, clamp, drained, inflow, t, steps, h->err);
}

flood_status flood_get_land_params(flood_handle* h, int32_t catchment, double* class_n_out, double* drain_out) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->get_land_params(catchment, class_n_out, drain_out, h->err);
}

flood_status flood_get_weights(flood_handle* h, int32_t catchment, double* logw, double* rain_mult, double* n_scale) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->get_weights(catchment, logw, rain_mult, n_scale, h->err);
}

flood_status flood_systematic_resample(const double* w, int32_t n, double u0, int32_t* anc_out, void* hip_stream) {
    if (!w || !anc_out || n < 1 || n > FLOOD_MAX_MEMBERS || !(u0 >= 0.0 && u0 < 1.0)) return FLOOD_EINVAL;
    double tot = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(w[i] >= 0.0) || !finite_d(w[i])) return FLOOD_EINVAL;
        tot += w[i];
    }
    if (!(tot > 0.0) || !finite_d(tot)) return FLOOD_EINVAL;
    return systematic_resample_impl(w, n, u0, anc_out, (hipStream_t)hip_stream);
}

flood_status flood_systematic_resample_noalloc(const double* w, int32_t n, double u0, int32_t* anc_out,
                                               void* hip_stream) {
    if (!w || !anc_out || n < 1 || n > FLOOD_MAX_MEMBERS || !(u0 >= 0.0 && u0 < 1.0)) return FLOOD_EINVAL;
    double tot = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(w[i] >= 0.0) || !finite_d(w[i])) return FLOOD_EINVAL;
        tot += w[i];
    }
    if (!(tot > 0.0) || !finite_d(tot)) return FLOOD_EINVAL;
    return systematic_resample_noalloc_impl(w, n, u0, anc_out, (hipStream_t)hip_stream);
}

flood_status flood_ensemble_products(flood_handle* h, int32_t catchment, double threshold, int32_t n_pct,
                                     const double* pct, const double* weights, double* prob_out, double* pct_out) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->products(catchment, threshold, n_pct, pct, weights, prob_out, pct_out, h->err);
}

flood_status flood_save(flood_handle* h, const char* path) {
    FLOOD_NEED_HANDLE(h);
    if (!path) { h->err = "path is NULL"; return FLOOD_EINVAL; }
    return h->impl->save(path, h->err);
}

flood_status flood_load(flood_handle* h, const char* path) {
    FLOOD_NEED_HANDLE(h);
    if (!path) { h->err = "path is NULL"; return FLOOD_EINVAL; }
    return h->impl->load(path, h->err);
}

flood_status flood_device_snapshot(flood_handle* h, int32_t op) {
    FLOOD_NEED_HANDLE(h);
    if (op != FLOOD_SNAPSHOT_TAKE && op != FLOOD_SNAPSHOT_RESTORE && op != FLOOD_SNAPSHOT_RELEASE) {
        h->err = "op must be FLOOD_SNAPSHOT_TAKE, FLOOD_SNAPSHOT_RESTORE or FLOOD_SNAPSHOT_RELEASE";
        return FLOOD_EINVAL;
    }
    return h->impl->device_snapshot(op, h->err);
}

flood_status flood_get_config(const flood_handle* h, int32_t* mi, int32_t* tile_rows, int32_t* cpb, int32_t* gsteps,
                              int32_t* step_kernel, int32_t* march_rows, int32_t* march_members,
                              int32_t* march_order) {
    if (!h || !h->impl) return FLOOD_EINVAL;
    h->impl->get_config(mi, tile_rows, cpb, gsteps, step_kernel, march_rows, march_members, march_order);
    return FLOOD_OK;
}

flood_status flood_adjoint_release(flood_handle* h) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->adjoint_release(h->err);
}

flood_status flood_get_adjoint_info(const flood_handle* h, int32_t* groups, int32_t* group_size, int32_t* segments) {
    if (!h || !h->impl) return FLOOD_EINVAL;
    h->impl->get_adjoint_info(groups, group_size, segments);
    return FLOOD_OK;
}

flood_status flood_get_march_rows(flood_handle* h, int32_t catchment, int32_t* march_rows) {
    FLOOD_NEED_HANDLE(h);
    return h->impl->get_march_rows(catchment, march_rows, h->err);
}

flood_status flood_timing(flood_handle* h, int32_t mode) {
    FLOOD_NEED_HANDLE(h);
    if (mode != 0 && mode != FLOOD_TIMING_LAUNCH && mode != FLOOD_TIMING_BATCH) {
        h->err = "mode must be 0, FLOOD_TIMING_LAUNCH or FLOOD_TIMING_BATCH";
        return FLOOD_EINVAL;
    }
    return h->impl->timing(mode, h->err);
}

flood_status flood_get_timing(const flood_handle* h, double* avg_ms, int64_t* launches) {
    if (!h || !h->impl) return FLOOD_EINVAL;
    h->impl->get_timing(avg_ms, launches);
    return FLOOD_OK;
}

void flood_destroy(flood_handle* h) { delete h; }

}  // extern "C"
