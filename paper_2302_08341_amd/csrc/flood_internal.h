// Internal declarations shared by the HIP kernels and the host runtime of
// libflood.  Device memory layout (one catchment, MI = member interleave):
//
//   state  X[chunk][r][c][mi]   X in {h, qx, qy}, chunk = member / MI,
//          qx[..][r][c] is the east link of cell (r,c) (c = nx-1: east edge),
//          qy[..][r][c] is the south link of cell (r,c) (r = ny-1: south edge)
//   strips qw[chunk][r][mi] (west edge links), qn[chunk][c][mi] (north edge)
//   two copies of every state array; member m's current copy is par[m]
//   shared z[r][c], n[r][c] (one copy for all members, Sec. 3.2)
//
// Members in the same chunk occupy adjacent addresses, so a wavefront reads
// 64/MI cells x MI members contiguously, and the shared per-cell arrays are
// read once per MI members.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace flood {

constexpr int kMaxCatch = 8;
constexpr int kBins = 64;      // partial-max bins per member for the depth maximum
constexpr int kBlock = 256;    // lanes per workgroup of the step kernels
constexpr int kMaxMembers = 1024;
constexpr int kMaxClasses = 4;  // land-cover classes
constexpr int kMaxSeries = 4;     // inflow hydrograph series per catchment
constexpr int kMaxSections = 64;  // streamflow sections per catchment

template <typename T> struct HBits;
template <> struct HBits<float> { using type = uint32_t; };
template <> struct HBits<double> { using type = unsigned long long; };

// Per-member coefficients of one step, written by the step planner.
template <typename T> struct MemberStep {
    T dtdx;    // dt / dx
    T gdtdx;   // g dt / dx
    T gdt;     // g dt
    T s2dt;    // (Manning scale)^2 dt
    T capf;    // dx / (4 dt): donor-limiter factor
    T rinc;    // rain depth of this step, mu R dt
    double dxdt;  // dx dt (outflow volume per unit discharge)
    int32_t active;
    int32_t parity;  // state copy holding the state before this step
    int32_t slot;    // adjoint record: the member's step index within the tape segment
    int32_t blk;     // adjoint record: tape block holding the member's state before the step
    int32_t blk_next;  // and the block the step writes
    uint32_t seed;   // random seed of the step's depth rounding, from the member's time
    T cn[kMaxClasses];  // land cover: the member's Manning n of each class
    T drain;            // land cover: drainage depth of the step (rate x dt)
    T qin[kMaxSeries];  // inward discharge of each inflow series during the step
};

template <typename T> struct CatchDev {
    int32_t ny, nx, n_members, n_chunks;
    int32_t tx_log2;          // log2(tile width in cells)
    int32_t tiles_x, tiles_y;
    int32_t groups;           // member-chunk groups per tile
    int32_t chunks_per_group;
    int32_t member_off;       // first global member index of this catchment
    int32_t block_begin;      // first linear workgroup of this catchment in a launch
    int32_t n_blocks;
    int32_t edge_open[4];
    // row-march variants (members in planes): strips of march_rows rows, one
    // wavefront per (strip, group of march_seg members); strips_x counts the
    // strips of the kernel the view is launched with (62 cells for k_march, 64 V
    // for k_marchv), strips_xa those of the adjoint's reverse step (62 x 2 cells)
    int32_t march_rows, strips_x, strips_y, strips_xa;
    int32_t wave_begin, n_waves;
    int32_t march_order;      // wavefront order, see march_wave
    int32_t march_bands;      // order 4: bands of rows of strips, a multiple of 8
    T edge_slope[4];
    T hdry, g;
    double dx;
    T* h[2];
    T* qx[2];
    T* qy[2];
    T* qw[2];
    T* qn[2];
    const T* z;
    const T* n;
    double* out_acc;          // [n_members][2*(nx+ny)] outflow volume per edge link (N, S, W, E)
    T* peak;                  // running maximum depth, state layout, one copy; null when not tracked
    // land cover (row-march kernel only): class map, runoff coefficient per class,
    // bit k of drain_mask set when class k drains; cls null: shared Manning field
    const uint8_t* cls;
    double* drain_acc;        // [n_members][kBins] drained volume, one bin per workgroup id mod kBins
    T class_rc[kMaxClasses];
    int32_t drain_mask;
    // inflow links: series index of each edge link in the order of out_acc
    // (N, S, W, E), -1 for none; null when the catchment has no inflow link
    const int8_t* inflow_id;
};

template <typename T> struct StepLaunch {
    int32_t n_catch;
    int32_t total_blocks;
    int32_t n_total;          // members over all catchments
    int32_t recompute;        // 1: adjoint tape recomputation (see k_step)
    CatchDev<T> c[kMaxCatch];
    const MemberStep<T>* ms;  // indexed by global member
    typename HBits<T>::type* hbins;  // [kBins][n_total]
    double* vclamp;           // [n_total]
    uint8_t* clamp_out;       // tiled recompute only: 1 where the new depth was clamped at zero
    // tape recording and recomputation by the row-march kernel: c[0]'s copy-0
    // arrays are the tape's block pools (block b of a field at b times the member
    // stride); a member reads block ms.blk and writes block ms.blk_next, a
    // clamped depth as -0
};

struct PlanCatch {
    int32_t member_off, n_members;
    int32_t n_rain;
    const double* rain;
    double rain_interval, alpha, hdry, dt_cap, dt_fixed, g, dx;
    double ncells;
    // inflow hydrographs: [n_series][n_rain] discharge per unit width; wq[j] =
    // links of series j x dx, so the inflow rate is sum_j wq[j] q_j
    const double* inflow_q;
    int32_t n_series;
    double wq[kMaxSeries];
};

template <typename T> struct PlanLaunch {
    int32_t n_catch, n_total;
    PlanCatch c[kMaxCatch];
    const double* t_end;      // device scalar
    double* t;
    const double* s;
    const double* mu;
    int32_t* par;
    int64_t* steps;
    int32_t* fault;
    int32_t* status;          // bit 0: non-finite depth seen
    double* vrain;
    double* vin;              // [n_total] inflow volume
    typename HBits<T>::type* hbins;
    MemberStep<T>* ms;
    double* dtlog;            // optional [n_total][dtlog_cap] step lengths
    double* telog;            // optional [n_total][dtlog_cap] step end times
    int64_t* log_n;           // [n_total] steps logged since the log was opened (may exceed dtlog_cap)
    int32_t dtlog_cap;
    const int64_t* step_lim;  // optional [n_total]: a member whose step count has reached it does not step
    int32_t m_begin, m_end;   // members planned by this launch (global indices)
    // adjoint record of this launch (null when not recording), indexed by m - m_begin
    MemberStep<T>* ms_log;
    double* rdt_log;          // R dt of the step (rain depth per unit multiplier)
    int32_t* tag_log;         // sample index completed by the step, or -1
    int32_t* any_log;         // set to 1 when any member steps
    int32_t tag_value;
    int32_t* seg_cnt;         // optional, by m - m_begin: steps taken since the last checkpoint
    const double* clsn;       // optional [n_total][kMaxClasses] land-cover Manning n per member
    const double* drain;      // optional [n_total] drainage rate per member, m/s
    // member-local records (rec_stride > 0): the record of a member's step goes to
    // [slot][rec_stride] + (m - m_begin), slot = its step index in the tape segment,
    // and members that do not step write nothing
    int32_t rec_stride;
    // sample schedule of the adjoint's recording forward (s_dt > 0): a member's step
    // is also clipped to its next sample time s_t0 + (smp + 1) s_dt; a step ending
    // there carries the sample index as its tag and moves the member to the next
    // sample.  The gauge misfit of the state after a tagged step is added to the
    // member's loss by the member's next planner call, from its current tape block.
    double s_t0, s_dt;
    int32_t* smp;             // [group] next sample index
    int32_t* pend;            // [group] sample whose misfit is still to be taken, or -1
    // tape blocks (with seg_cnt): a stepping member takes the next free block of
    // the pool for its new state (pool_next counts the blocks in use) and cur_blk
    // follows the block of its latest state
    int32_t* cur_blk;         // [group]
    int32_t* pool_next;       // device scalar
    const T* tape_h;          // depth pool of the tape: block b's plane at b * plane
    size_t plane;
    int32_t nx;
    int32_t n_gauges;
    const int32_t* grc;       // [n_gauges][2]
    const double* obs;        // [samples][n_gauges]
    double* loss_m;           // [group] misfit per member (FP64, sample order)
};

// ---------------------------------------------------------------------------
// launchers (flood_kernels.hip)
// ---------------------------------------------------------------------------
template <typename T> void launch_plan(const PlanLaunch<T>& P, hipStream_t s);
template <typename T, int MI> void launch_step(const StepLaunch<T>& L, hipStream_t s);
template <typename T> void launch_step_mi(int mi, const StepLaunch<T>& L, hipStream_t s);
template <typename T> void launch_march(const StepLaunch<T>& L, int seg, int total_waves, hipStream_t s);
// cells per lane of the vectorised row-marching kernel (nx must be a multiple of it)
template <typename T> constexpr int march_vec() { return sizeof(T) == 4 ? 4 : 2; }
// Cells per lane of the adjoint's reverse row march, in both precisions: with
// four FP32 cells per lane the reverse step needs 138 VGPRs (3 waves per SIMD),
// with two 85 (5 waves per SIMD), and runs faster.
template <typename T> constexpr int adj_vec() { return 2; }
template <typename T>
void launch_marchv(const StepLaunch<T>& L, int nt, int pf, int ext, int total_waves, hipStream_t s);
// wavefronts of a row-march launch over one catchment: strips x member units,
// units padded to a multiple of four in wavefront order 2
// wavefronts of one row-march launch over a catchment (see march_wave)
inline int march_waves(int strips_x, int strips_y, int units, int order, int bands = 8) {
    if (order == 2) return strips_x * strips_y * ((units + 3) / 4 * 4);
    if (order == 4) return strips_x * ((strips_y + bands - 1) / bands * bands) * units;
    return strips_x * strips_y * units;
}
// members still short of t_end (and, when lim is given, of their step limit)
void launch_count_active(int n_total, const double* t, const int32_t* fault, const double* t_end,
                         const int32_t* status, const int64_t* steps, const int64_t* lim, int32_t* out,
                         hipStream_t s);
// lim[m] = steps[m] + n for the n_total members (n < 0: no limit)
void launch_step_limit(int n_total, const int64_t* steps, int64_t n, int64_t* lim, hipStream_t s);
// wet/dry decision every link of one member takes in the next step, from the
// member's current state (copy p), in the host link layouts: wx [ny][nx+1],
// wy [ny+1][nx]; 1 wet, 0 dry, wall or inflow link
template <typename T>
void launch_wetmask(int mi, const CatchDev<T>& C, int member, int p, uint8_t* wx, uint8_t* wy, hipStream_t s);
template <typename HB> void launch_zero_bins(int off, int n, int n_total, HB* bins, hipStream_t s);
template <typename HB>
void launch_permute_bins(int off, int n, int n_total, HB* bins, const int32_t* anc, const int32_t* flag,
                         hipStream_t s);
template <typename T>
void launch_hmax_init(int mi, const CatchDev<T>& C, const int32_t* par, typename HBits<T>::type* hbins,
                      int n_total, hipStream_t s);
template <typename T>
void launch_storage(int mi, const CatchDev<T>& C, const int32_t* par, double* out, hipStream_t s);
template <typename T>
void launch_get_field(int mi, const CatchDev<T>& C, int member, int par, int which, double* out,
                      hipStream_t s);
template <typename T>
void launch_set_field(int mi, const CatchDev<T>& C, int member, int par, int which, const double* in,
                      hipStream_t s);
template <typename T>
void launch_gauges(int mi, const CatchDev<T>& C, const int32_t* par, int n_gauges, const int32_t* grc,
                   double* y, int y_stride, hipStream_t s);
// streamflow sections: each link is (code, index): code bits 0-1 the array
// (0 qx cell, 1 qy cell, 2 west strip row, 3 north strip column), bit 2 set
// for a negative sign; index the cell (r*nx + c) or strip position.
// out[m*out_stride + out_off + s] = dx * sum of sign * q over section s.
template <typename T>
void launch_sections(int mi, const CatchDev<T>& C, const int32_t* par, int n_sections, const int32_t* offs,
                     const int32_t* code, const int32_t* index, double* out, int out_stride, int out_off,
                     hipStream_t s);
void launch_flush_outflow(int n_members, int nb, double* out_acc, double* vout, hipStream_t s);
// ensemble products of the running maximum depth: prob [ny*nx], pct [n_pct][ny*nx]
template <typename T>
void launch_products(int mi, const CatchDev<T>& C, double threshold, int n_pct, const double* pct, const double* w,
                     double W, double* prob, double* pct_out, hipStream_t s);

// adjoint (flood_adjoint.hip)
template <typename T> struct AdjLaunch {
    CatchDev<T> c;            // view of the member group; h[0].. = state before the step (tape slot)
    T* lh[2];                 // adjoint of h: [0] after the step (in), [1] before (out)
    T* lqx[2];
    T* lqy[2];
    T* lqw[2];
    T* lqn[2];
    const uint8_t* clamp;     // clamp flags of this step (state layout)
    const MemberStep<T>* ms;  // [group members] coefficients of this step
    const double* rdt;        // [group members]
    double* nbar;             // [ny*nx] Manning-field adjoint (accumulated)
    double* mubar_part;       // [blocks][group members] rain-multiplier adjoint partials (accumulated)
};
template <typename T> void launch_adjoint_step(int mi, const AdjLaunch<T>& A, hipStream_t s);

// Reverse step in row-march form (members in planes, nx a multiple of the
// vector width).  The tape is a pool of blocks, one member state each: a member
// active in this launch reads its state before the step from block ms.blk;
// members that did not step are skipped and keep their adjoint in place.
template <typename T> struct AdjvLaunch {
    CatchDev<T> c;            // group view: copy-0 arrays are the tape's block pools; strip / wave geometry
    T* lh[2];                 // two copies of the adjoint state, [member][...]
    T* lqx[2];
    T* lqy[2];
    T* lqw[2];
    T* lqn[2];
    // launch i of a tape segment whose member k took n[k] steps: member k reverses
    // its step j = n[k] - 1 - i (none when j < 0), from the member-local records
    // of the segment ([slot][stride], member k at k); its adjoint after the step is
    // in copy lbase[k] ^ (i & 1)
    int32_t i;
    int32_t stride;
    const int32_t* n;
    const int32_t* lbase;
    const MemberStep<T>* rec;
    const double* rec_rdt;
    const int32_t* rec_tag;
    // gauge misfit: the seed of a sample completed by step j - 1 is added to the
    // depth adjoint this launch writes (gauge cells [n_gauges][2], obs [samples][n_gauges])
    int32_t n_gauges;
    const int32_t* grc;
    const double* obs;
    T* nacc;                  // [member quads][cell] Manning-field adjoint per quad of members (accumulated)
    double* mubar_part;       // [strips][group members] rain-multiplier adjoint partials (accumulated)
    int32_t pf;               // 1: one row of load lookahead in the reverse march
};
template <typename T> void launch_adjoint_march(const AdjvLaunch<T>& A, hipStream_t s);
template <typename T>
void launch_nacc_reduce(int G, size_t ncell, const T* nacc, double* nbar, hipStream_t s);
// Start of the reverse of a tape segment whose member m took n[m] steps
// (records [slot][stride], member m at m): first the adjoint copy index lbase[m]
// moves past the n_prev[m] steps of the segment reversed before (n_prev null:
// the group's last segment, lbase starts at 0), then the gauge misfit of a
// sample completed by the segment's last step of the member, 2 (h - d), is
// seeded into the adjoint of the depths after it (h read from the tape block
// the step wrote; a gauge cell the step clamped gets none).  Seeds of the
// samples completed by earlier steps are added by the reverse step itself.
// tape_h: the tape's depth pool.
template <typename T>
void launch_adj_segment(int G, int stride, const int32_t* n_prev, const int32_t* n, const MemberStep<T>* rec,
                        const int32_t* rec_tag, int K, const int32_t* grc, const double* obs, const T* tape_h,
                        size_t plane, int nx, int32_t* lbase, T* lh0, T* lh1, hipStream_t s);
// Copy each member's state from tape block blk[m] (tape: copy-0 arrays are the
// block pools) to dst, into copy dpar[dst.member_off + m] (dpar null: copy 0).
template <typename T>
void launch_tape_gather(const CatchDev<T>& tape, const int32_t* blk, const CatchDev<T>& dst, const int32_t* dpar,
                        hipStream_t s);
// [0] members of the group still short of t_end, [1] status word, [2] largest
// seg_cnt, [3] tape blocks in use
void launch_count_group(int G, const double* t, const int32_t* fault, const double* t_end, const int32_t* status,
                        const int32_t* seg_cnt, const int32_t* pool_next, int32_t* out, hipStream_t s);
template <typename T>
void launch_marchv_rec(const StepLaunch<T>& L, int pf, int record, int total_waves, hipStream_t s);
template <typename T>
void launch_inject(int mi, const CatchDev<T>& after, const int32_t* tags, int K, const int32_t* grc,
                   const double* obs, T* lh, hipStream_t s);
template <typename T>
void launch_snapshot(int mi, const CatchDev<T>& C, const int32_t* par, const CatchDev<T>& dst, hipStream_t s);
template <typename T>
void launch_misfit(int mi, const CatchDev<T>& C, const int32_t* par, int K, const int32_t* grc,
                   const double* obs, double* loss, hipStream_t s);
void launch_sum_parts(int n_blocks, int n_members, const double* parts, double* out, hipStream_t s);

// particle filter (flood_pf.hip)
struct PfArgs {
    int32_t N, K;
    const double* y;          // [N*K]
    const double* d;          // [K]
    const double* sigma;      // [K]
    double neff_frac, u0;
    const double* beta;       // [N] or null
    double* logw;             // [N] in/out
    double* t;                // member scalars permuted on resampling
    double* s;
    double* mu;
    double* vrain;
    double* vout;
    double* vclamp;
    int64_t* steps;
    int32_t* par;
    int32_t* src_par;         // [N] out: copy-from parity of each slot's ancestor
    int32_t* dst_par;         // [N] out: copy-to parity of each slot
    int32_t* anc;             // [N] out
    double* neff;             // [1] out
    int32_t* flag;            // [1] out: 1 if resampled
    double* clsn;             // land cover, permuted with the members: [N][kMaxClasses] or null
    double* drain;            // [N] or null
    double* vdrain;           // [N]
    double* vin;              // [N]
    double alpha;             // > 0: sigma_k = max(alpha |d_k|, sigma[k])
};
void launch_pf(const PfArgs& a, hipStream_t s);
// running maxima follow their members on resampling: gather into tmp, then commit
template <typename T>
void launch_permute_peak(int mi, const CatchDev<T>& C, const int32_t* anc, const int32_t* flag, T* tmp,
                         hipStream_t s);
void launch_systematic(int n, const double* w, double u0, int32_t* anc, hipStream_t s);
template <typename T>
void launch_permute(int mi, const CatchDev<T>& C, const int32_t* anc, const int32_t* src_par,
                    const int32_t* dst_par, const int32_t* flag, hipStream_t s);

}  // namespace flood
