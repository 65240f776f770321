// Argument checks of the handle's calls, in host code that touches no device
// state: the runtime calls them before any HIP call of a method, and a CPU
// build with sanitizers drives them directly.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "flood_validate.h"

namespace flood {

static bool fin(double v) { return std::isfinite(v); }

flood_status check_state_args(int ny, int nx, const int32_t edge_kind[4], const int8_t* inflow_id, const double* h,
                              const double* qx, const double* qy, double t, std::string& err) {
    if (!h || !qx || !qy) { err = "h, qx and qy are required"; return FLOOD_EINVAL; }
    if (!(t >= 0.0) || !fin(t)) { err = "t must be finite and >= 0"; return FLOOD_EINVAL; }
    for (size_t i = 0; i < (size_t)ny * nx; ++i)
        if (!(h[i] >= 0.0) || !fin(h[i])) { err = "depths must be finite and >= 0"; return FLOOD_EINVAL; }
    for (size_t i = 0; i < (size_t)ny * (nx + 1); ++i)
        if (!fin(qx[i])) { err = "qx must be finite"; return FLOOD_EINVAL; }
    for (size_t i = 0; i < (size_t)(ny + 1) * nx; ++i)
        if (!fin(qy[i])) { err = "qy must be finite"; return FLOOD_EINVAL; }
    // wall links carry no flow, except inflow links (edge-link order N, S, W, E)
    auto wall = [&](int e, size_t at) { return edge_kind[e] == FLOOD_EDGE_WALL && (!inflow_id || inflow_id[at] < 0); };
    for (int r = 0; r < ny; ++r) {
        if (wall(3, 2 * (size_t)nx + r) && qx[(size_t)r * (nx + 1)] != 0.0) { err = "west wall link must be 0"; return FLOOD_EINVAL; }
        if (wall(1, 2 * (size_t)nx + ny + r) && qx[(size_t)r * (nx + 1) + nx] != 0.0) { err = "east wall link must be 0"; return FLOOD_EINVAL; }
    }
    for (int c = 0; c < nx; ++c) {
        if (wall(0, c) && qy[c] != 0.0) { err = "north wall link must be 0"; return FLOOD_EINVAL; }
        if (wall(2, (size_t)nx + c) && qy[(size_t)ny * nx + c] != 0.0) { err = "south wall link must be 0"; return FLOOD_EINVAL; }
    }
    return FLOOD_OK;
}

flood_status check_param_update(size_t ncell, int N, int n_classes, const float* manning, const double* n_scale,
                                const double* rain_mult, std::string& err) {
    if (n_classes && (manning || n_scale)) {
        err = "with land cover the roughness is per class and member; manning_n and n_scale do not apply";
        return FLOOD_EINVAL;
    }
    if (manning)
        for (size_t i = 0; i < ncell; ++i)
            if (!(manning[i] > 0.0f) || !std::isfinite(manning[i])) { err = "manning_n must be finite and > 0"; return FLOOD_EINVAL; }
    for (int m = 0; m < N; ++m) {
        if (n_scale && (!(n_scale[m] > 0.0) || !fin(n_scale[m]))) { err = "n_scale must be finite and > 0"; return FLOOD_EINVAL; }
        if (rain_mult && (!(rain_mult[m] >= 0.0) || !fin(rain_mult[m]))) { err = "rain_mult must be finite and >= 0"; return FLOOD_EINVAL; }
    }
    return FLOOD_OK;
}

static flood_status check_gauges(int ny, int nx, int K, const int32_t* grc, std::string& err) {
    for (int k = 0; k < K; ++k)
        if (grc[2 * k] < 0 || grc[2 * k] >= ny || grc[2 * k + 1] < 0 || grc[2 * k + 1] >= nx) {
            err = "gauge outside the grid";
            return FLOOD_EINVAL;
        }
    return FLOOD_OK;
}

flood_status check_observations(int ny, int nx, int N, int K, int S, const int32_t* grc, const double* obs,
                                const double* sigma, double alpha, double neff_frac, double u0, const double* beta,
                                std::string& err) {
    const int KT = K + S;
    if (K < 0 || KT > 4096) { err = "n_gauges (plus sections) must be in [0, 4096]"; return FLOOD_EINVAL; }
    if (K > 0 && !grc) { err = "gauge_rc is required"; return FLOOD_EINVAL; }
    if (KT > 0 && (!obs || !sigma)) { err = "obs and sigma are required"; return FLOOD_EINVAL; }
    if (!(alpha >= 0.0) || !fin(alpha)) { err = "alpha must be finite and >= 0"; return FLOOD_EINVAL; }
    if (check_gauges(ny, nx, K, grc, err)) return FLOOD_EINVAL;
    for (int k = 0; k < KT; ++k) {
        if (!fin(obs[k])) { err = "obs must be finite"; return FLOOD_EINVAL; }
        if (!(sigma[k] > 0.0) || !fin(sigma[k])) { err = "sigma must be finite and > 0"; return FLOOD_EINVAL; }
    }
    if (!(neff_frac > 0.0 && neff_frac <= 1.0)) { err = "neff_frac must be in (0, 1]"; return FLOOD_EINVAL; }
    if (!(u0 >= 0.0 && u0 < 1.0)) { err = "u0 must be in [0, 1)"; return FLOOD_EINVAL; }
    if (beta)
        for (int m = 0; m < N; ++m)
            if (!(beta[m] >= 0.0) || !fin(beta[m])) { err = "beta must be finite and >= 0"; return FLOOD_EINVAL; }
    return FLOOD_OK;
}

flood_status parse_sections(int ny, int nx, int n, const int32_t* count, const int32_t* links,
                            std::vector<int32_t>& offs, std::vector<int32_t>& code, std::vector<int32_t>& index,
                            std::string& err) {
    if (n < 0 || n > kMaxSectionsAbi) { err = "n_sections must be in [0, 64]"; return FLOOD_EINVAL; }
    if (n > 0 && (!count || !links)) { err = "link_count and links are required"; return FLOOD_EINVAL; }
    offs.assign(1, 0);
    code.clear();
    index.clear();
    for (int s = 0; s < n; ++s) {
        if (count[s] < 1) { err = "every section needs at least one link"; return FLOOD_EINVAL; }
        if ((int64_t)offs.back() + count[s] > 65536) { err = "at most 65536 section links"; return FLOOD_EINVAL; }
        for (int l = offs.back(); l < offs.back() + count[s]; ++l) {
            const int32_t* f = links + 4 * (size_t)l;
            const int kind = f[0], r = f[1], c = f[2], sg = f[3];
            if (sg != 1 && sg != -1) { err = "link sign must be +1 or -1"; return FLOOD_EINVAL; }
            int cd, ix;
            if (kind == 0 && r >= 0 && r < ny && c >= 0 && c <= nx) {
                cd = c == 0 ? 2 : 0;
                ix = c == 0 ? r : r * nx + c - 1;
            } else if (kind == 1 && r >= 0 && r <= ny && c >= 0 && c < nx) {
                cd = r == 0 ? 3 : 1;
                ix = r == 0 ? c : (r - 1) * nx + c;
            } else {
                err = "section link outside the grid (kind 0: r < ny, c <= nx; kind 1: r <= ny, c < nx)";
                return FLOOD_EINVAL;
            }
            code.push_back(cd | (sg < 0 ? 4 : 0));
            index.push_back(ix);
        }
        offs.push_back(offs.back() + count[s]);
    }
    return FLOOD_OK;
}

flood_status check_products(int N, double threshold, int n_pct, const double* pct, const double* weights,
                            std::vector<double>& w, std::string& err) {
    if (!fin(threshold)) { err = "threshold must be finite"; return FLOOD_EINVAL; }
    if (n_pct < 0 || n_pct > 16) { err = "n_pct must be in [0, 16]"; return FLOOD_EINVAL; }
    if (n_pct > 0 && !pct) { err = "pct is NULL"; return FLOOD_EINVAL; }
    for (int i = 0; i < n_pct; ++i)
        if (!(pct[i] > 0.0 && pct[i] <= 1.0)) { err = "percentiles must be in (0, 1]"; return FLOOD_EINVAL; }
    w.assign(N, 1.0);
    if (weights)
        for (int m = 0; m < N; ++m) {
            if (!(weights[m] >= 0.0) || !fin(weights[m])) { err = "weights must be finite and >= 0"; return FLOOD_EINVAL; }
            w[m] = weights[m];
        }
    double W = 0.0;
    for (int m = 0; m < N; ++m) W += w[m];   // member order, as the kernel's sums
    if (!(W > 0.0) || !fin(W)) { err = "weights must have a positive finite sum"; return FLOOD_EINVAL; }
    return FLOOD_OK;
}

flood_status check_adjoint_args(int ny, int nx, int n_classes, int n_series, double t_end, double sample_dt, int K,
                                const int32_t* grc, const double* obs, int ckpt_every, std::string& err) {
    if (n_classes) { err = "the adjoint does not support land cover"; return FLOOD_EINVAL; }
    if (n_series) { err = "the adjoint does not support inflow links"; return FLOOD_EINVAL; }
    if (!(sample_dt > 0.0) || !fin(sample_dt)) { err = "sample_dt must be finite and > 0"; return FLOOD_EINVAL; }
    if (!fin(t_end)) { err = "t_end must be finite"; return FLOOD_EINVAL; }
    if (K < 0 || K > 4096) { err = "n_gauges must be in [0, 4096]"; return FLOOD_EINVAL; }
    if (K > 0 && (!grc || !obs)) { err = "gauge_rc and obs are required"; return FLOOD_EINVAL; }
    if (ckpt_every < 1) { err = "ckpt_every must be >= 1"; return FLOOD_EINVAL; }
    return check_gauges(ny, nx, K, grc, err);
}

flood_status adjoint_samples(int nx, double t0, double t_end, double sample_dt, int K, const int32_t* grc,
                             const double* obs, int* S_out, int* distinct_out, std::string& err) {
    int distinct = 1;
    std::vector<int64_t> cells(K);
    for (int k = 0; k < K; ++k) cells[k] = (int64_t)grc[2 * k] * nx + grc[2 * k + 1];
    std::sort(cells.begin(), cells.end());
    for (int k = 1; k < K; ++k) distinct &= cells[k] != cells[k - 1];
    const double span = std::floor((t_end - t0) / sample_dt + 1e-9);
    if (!(span >= 1.0)) { err = "no sample time in (t0, t_end]"; return FLOOD_EINVAL; }
    if (span * std::max(K, 1) > 2e9) { err = "too many samples (t_end - t0) / sample_dt"; return FLOOD_EINVAL; }
    const int S = (int)span;
    for (size_t i = 0; i < (size_t)S * K; ++i)
        if (!fin(obs[i])) { err = "obs must be finite"; return FLOOD_EINVAL; }
    *S_out = S;
    *distinct_out = distinct;
    return FLOOD_OK;
}

}  // namespace flood
