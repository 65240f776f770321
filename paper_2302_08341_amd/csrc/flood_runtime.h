// Host-side handle of libflood: the precision-independent interface the C ABI
// calls into, implemented per state precision in flood_runtime.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>

#include "../../include/flood.h"

namespace flood {

struct ImplBase {
    virtual ~ImplBase() {}
    virtual flood_status step(double t_end, int64_t max_steps, std::string& err) = 0;
    virtual flood_status get_wet_mask(int c, int m, uint8_t* wx, uint8_t* wy, std::string& err) = 0;
    virtual flood_status log_steps(int32_t cap, std::string& err) = 0;
    virtual flood_status get_step_log(int c, double* dt, double* te, int64_t* count, std::string& err) = 0;
    virtual flood_status assimilate(int c, int K, const int32_t* grc, const double* obs, const double* sigma,
                                    int with_sections, double alpha, double neff_frac, double u0,
                                    const double* beta, double* neff_out, int32_t* anc_out, int32_t* res_out,
                                    std::string& err) = 0;
    virtual flood_status set_sections(int c, int n, const int32_t* count, const int32_t* links,
                                      std::string& err) = 0;
    virtual flood_status get_sections(int c, double* q_out, std::string& err) = 0;
    virtual flood_status adjoint(int c, double t_end, double sample_dt, int K, const int32_t* grc,
                                 const double* obs, int ckpt_every, double* loss_out, double* grad_n_out,
                                 double* grad_mult_out, std::string& err) = 0;
    virtual flood_status adjoint_release(std::string& err) = 0;
    virtual flood_status get_field(int c, int m, int which, double* out, std::string& err) = 0;
    virtual flood_status set_state(int c, int m, const double* h, const double* qx, const double* qy, double t,
                                   std::string& err) = 0;
    virtual flood_status set_params(int c, const float* manning, const double* n_scale, const double* rain_mult,
                                    std::string& err) = 0;
    virtual flood_status get_ledger(int c, double* storage, double* rain_in, double* outflow, double* clamp,
                                    double* drained, double* inflow, double* t, int64_t* steps,
                                    std::string& err) = 0;
    virtual flood_status get_land_params(int c, double* class_n, double* drain, std::string& err) = 0;
    virtual flood_status get_weights(int c, double* logw, double* rain_mult, double* n_scale,
                                     std::string& err) = 0;
    virtual flood_status products(int c, double threshold, int n_pct, const double* pct, const double* weights,
                                  double* prob_out, double* pct_out, std::string& err) = 0;
    virtual flood_status save(const char* path, std::string& err) = 0;
    virtual flood_status load(const char* path, std::string& err) = 0;
    virtual flood_status device_snapshot(int op, std::string& err) = 0;
    virtual void get_config(int32_t* mi, int32_t* tile_rows, int32_t* cpb, int32_t* gsteps, int32_t* step_kernel,
                            int32_t* march_rows, int32_t* march_members, int32_t* march_order) const = 0;
    virtual flood_status timing(int mode, std::string& err) = 0;
    virtual void get_timing(double* avg_ms, int64_t* launches) const = 0;
    virtual void get_adjoint_info(int32_t* groups, int32_t* group_size, int32_t* segments) const = 0;
    virtual flood_status get_march_rows(int c, int32_t* rows, std::string& err) const = 0;
};

const char* status_name(flood_status s);
bool finite_d(double v);
flood_status validate_grid(const flood_grid* g, std::string& err);
flood_status validate_params(const flood_params* p, std::string& err);

}  // namespace flood

struct flood_handle {
    std::unique_ptr<flood::ImplBase> impl;
    std::string err;
};

namespace flood {
flood_status create_impl(flood_handle* h, int n_catch, const flood_grid* grids, const flood_params* params,
                         const int32_t* members, const double* const* n_scale, const double* const* rain_mult,
                         hipStream_t stream, std::string& err);
flood_status systematic_resample_impl(const double* w, int n, double u0, int32_t* anc, hipStream_t s);
flood_status systematic_resample_noalloc_impl(const double* w, int n, double u0, int32_t* anc, hipStream_t s);
}  // namespace flood
