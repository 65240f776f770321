// Host-only argument checks of the handle's calls (no HIP state); each returns
// FLOOD_OK or FLOOD_EINVAL with err set.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/flood.h"

namespace flood {

constexpr int kMaxSectionsAbi = 64;   // sections per catchment

// flood_set_state: shapes [ny, nx], [ny, nx+1], [ny+1, nx]; wall links must
// carry no flow unless they are inflow links (inflow_id: edge-link series
// index in N, S, W, E order, < 0 for none; NULL when there are no inflow links)
flood_status check_state_args(int ny, int nx, const int32_t edge_kind[4], const int8_t* inflow_id, const double* h,
                              const double* qx, const double* qy, double t, std::string& err);

// flood_set_params
flood_status check_param_update(size_t ncell, int N, int n_classes, const float* manning, const double* n_scale,
                                const double* rain_mult, std::string& err);

// flood_assimilate / flood_assimilate_obs: K gauges then S section discharges
flood_status check_observations(int ny, int nx, int N, int K, int S, const int32_t* grc, const double* obs,
                                const double* sigma, double alpha, double neff_frac, double u0, const double* beta,
                                std::string& err);

// flood_set_sections: flattens the links into CSR offsets, direction codes and
// link indices
flood_status parse_sections(int ny, int nx, int n, const int32_t* count, const int32_t* links,
                            std::vector<int32_t>& offs, std::vector<int32_t>& code, std::vector<int32_t>& index,
                            std::string& err);

// flood_ensemble_products: w receives the member weights (all ones for NULL)
flood_status check_products(int N, double threshold, int n_pct, const double* pct, const double* weights,
                            std::vector<double>& w, std::string& err);

// flood_adjoint, before the members' common time is known
flood_status check_adjoint_args(int ny, int nx, int n_classes, int n_series, double t_end, double sample_dt, int K,
                                const int32_t* grc, const double* obs, int ckpt_every, std::string& err);

// flood_adjoint, from the common time t0: number of samples S in (t0, t_end],
// whether the gauges are distinct cells, and the S*K observations finite
flood_status adjoint_samples(int nx, double t0, double t_end, double sample_dt, int K, const int32_t* grc,
                             const double* obs, int* S_out, int* distinct_out, std::string& err);

}  // namespace flood
