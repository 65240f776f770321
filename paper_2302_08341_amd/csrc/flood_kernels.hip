// Forward kernels of libflood for gfx950: step planner, fused link + continuity
// step with the per-member depth maximum, and state utilities.
//
// The step is memory-bound (about 60 flops per 24 bytes per member-cell), so it
// uses plain vector ALU work with coalesced structure-of-arrays streams and no
// matrix cores.  All kernels are compiled with FP contraction off, so every
// link is evaluated with the same rounding wherever it is computed (a link
// shared by two cells is computed by both, identically).
#include <cfloat>
#include <cmath>

#include "flood_device.h"

namespace flood {

// ---------------------------------------------------------------------------
// step planner: per-member Eq. 4 step, clipped to rain-block edges and t_end
// ---------------------------------------------------------------------------
// One wavefront per member: lane k folds depth-maximum bin k (kBins = 64) and
// the lanes share the gauge misfit; the plan itself is the same scalar work on
// every lane, written out by lane 0.
template <typename T>
__global__ __launch_bounds__(256) void k_plan(const PlanLaunch<T> P) {
    using HB = typename HBits<T>::type;
    static_assert(kBins == 64, "one depth-maximum bin per lane");
    const int lane = threadIdx.x & 63;
    const int m = P.m_begin + blockIdx.x * (blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    if (m >= P.m_end) return;
    const bool w0 = lane == 0;
    int ci = 0;
    for (int i = 1; i < P.n_catch; ++i)
        if (m >= P.c[i].member_off) ci = i;
    const PlanCatch& C = P.c[ci];
    const int lm = m - P.m_begin;
    // The loads of the plan that depend on nothing else go out together, before
    // any store (a planner is a chain of memory round trips, not of arithmetic).
    const int par = P.par[m];
    const double t = P.t[m];
    const double t_end = *P.t_end;
    const int fault = P.fault[m];
    const int64_t st = P.steps[m];
    const bool at_lim = P.step_lim && st >= P.step_lim[m];
    HB hb = P.hbins[(size_t)lane * P.n_total + m];
    const int pend = P.pend ? P.pend[lm] : -1;
    const int cb = P.cur_blk ? P.cur_blk[lm] : 0;
    const int nsmp = P.s_dt > 0.0 ? P.smp[lm] : 0;
    const int nseg = P.seg_cnt ? P.seg_cnt[lm] : 0;
    const double sc = P.s[m];
    const double mu = P.mu[m];
    const double jf = floor(t / C.rain_interval);
    const double R = (jf >= 0.0 && jf < (double)C.n_rain) ? C.rain[(int64_t)jf] : 0.0;
    MemberStep<T> ms;
    ms.dtdx = ms.gdtdx = ms.gdt = ms.s2dt = ms.capf = ms.rinc = T(0);
    ms.dxdt = 0.0;
    ms.active = 0;
    ms.parity = par;
    ms.slot = ms.blk = ms.blk_next = -1;
    ms.seed = 0;
    for (int k = 0; k < kMaxClasses; ++k) ms.cn[k] = T(0);
    ms.drain = T(0);
    for (int k = 0; k < kMaxSeries; ++k) ms.qin[k] = T(0);
    if (pend >= 0) {
        // misfit of the state after the member's last step, which completed sample pend
        const T* h = P.tape_h + (size_t)cb * P.plane;
        double acc = 0.0;
        for (int q = lane; q < P.n_gauges; q += 64) {
            const double d = (double)h[(size_t)P.grc[2 * q] * P.nx + P.grc[2 * q + 1]] -
                             P.obs[(size_t)pend * P.n_gauges + q];
            acc += d * d;
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (w0) {
            P.loss_m[lm] += acc;
            P.pend[lm] = -1;
        }
    }
    if (fault || !(t < t_end) || at_lim) {
        if (w0) {
            P.ms[m] = ms;
            if (P.ms_log && !P.rec_stride) {
                P.ms_log[lm] = ms;
                P.rdt_log[lm] = 0.0;
                P.tag_log[lm] = -1;
            }
        }
        return;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const HB o = __shfl_xor(hb, off, 64);
        hb = o > hb ? o : hb;
    }
    const T H = from_bits<T>(hb);
    const auto freeze = [&]() {
        if (w0) {
            P.fault[m] = 1;
            atomicOr(P.status, 1);
            P.ms[m] = ms;
            if (P.ms_log && !P.rec_stride) {
                P.ms_log[lm] = ms;
                P.rdt_log[lm] = 0.0;
                P.tag_log[lm] = -1;
            }
        }
    };
    if (!(H <= (sizeof(T) == 4 ? T(FLT_MAX) : T(DBL_MAX)))) {
        freeze();
        return;
    }
    double dt;
    if (C.dt_fixed > 0.0) {
        dt = C.dt_fixed;
    } else {
        double Hd = (double)H;
        if (Hd < C.hdry) Hd = C.hdry;
        dt = C.alpha * C.dx / sqrt(C.g * Hd);
        if (dt > C.dt_cap) dt = C.dt_cap;
    }
    const double edge = (jf + 1.0 > (double)C.n_rain) ? INFINITY : (jf + 1.0) * C.rain_interval;
    double tev = t_end < edge ? t_end : edge;
    const double ts = P.s_dt > 0.0 ? P.s_t0 + (double)(nsmp + 1) * P.s_dt : INFINITY;
    if (ts < tev) tev = ts;
    double tn;
    if (dt >= tev - t) {
        dt = tev - t;
        tn = tev;
    } else {
        tn = t + dt;
    }
    if (!(tn > t)) {
        // an Eq. 4 step below the resolution of the member's clock (a depth so
        // large that the member can no longer advance): a numeric fault too
        freeze();
        return;
    }
    // every lane has read its bin: clear it for the step's new maximum
    P.hbins[(size_t)lane * P.n_total + m] = 0;
    if (!w0) return;
    ms.dtdx = (T)(dt / C.dx);
    ms.gdtdx = (T)(C.g * dt / C.dx);
    ms.gdt = (T)(C.g * dt);
    ms.s2dt = (T)(sc * sc * dt);
    ms.capf = (T)(C.dx / (4.0 * dt));
    ms.rinc = (T)(mu * R * dt);
    ms.dxdt = C.dx * dt;
    ms.active = 1;
    {
        // the step's random bits follow from the member's time: a state set back
        // to an earlier time replays the same rounding
        const uint64_t tb = (uint64_t)__double_as_longlong(t);
        ms.seed = mix32((uint32_t)tb ^ mix32((uint32_t)(tb >> 32) + 0x632be5abu));
    }
    if (P.seg_cnt) {
        // the member's new state goes to the next free block of the tape
        ms.slot = nseg;
        P.seg_cnt[lm] = nseg + 1;
        ms.blk = cb;
        ms.blk_next = atomicAdd(P.pool_next, 1);
        P.cur_blk[lm] = ms.blk_next;
    }
    if (P.clsn)
        for (int k = 0; k < kMaxClasses; ++k) ms.cn[k] = (T)P.clsn[(size_t)m * kMaxClasses + k];
    if (P.drain) ms.drain = (T)(P.drain[m] * dt);
    if (C.n_series > 0) {
        // inflow hydrographs: the series value of the current rain block
        double vq = 0.0;
        for (int j = 0; j < C.n_series; ++j) {
            const double q = (jf >= 0.0 && jf < (double)C.n_rain) ? C.inflow_q[(size_t)j * C.n_rain + (int64_t)jf]
                                                                     : 0.0;
            ms.qin[j] = (T)q;
            vq += C.wq[j] * q;
        }
        P.vin[m] += vq * dt;
    }
    P.ms[m] = ms;
    int tag = (tn == t_end) ? P.tag_value : -1;
    if (P.s_dt > 0.0) {
        tag = (tn == ts) ? nsmp : -1;
        if (tag >= 0) {
            P.smp[lm] = tag + 1;
            P.pend[lm] = tag;
        }
    }
    if (P.ms_log) {
        const size_t li = P.rec_stride ? (size_t)ms.slot * P.rec_stride + lm : (size_t)lm;
        P.ms_log[li] = ms;
        P.rdt_log[li] = R * dt;
        P.tag_log[li] = tag;
        if (P.any_log) P.any_log[0] = 1;
    }
    if (P.dtlog) {
        const int64_t li = P.log_n[m];
        if (li < P.dtlog_cap) {
            P.dtlog[(size_t)m * P.dtlog_cap + li] = dt;
            P.telog[(size_t)m * P.dtlog_cap + li] = tn;
        }
        P.log_n[m] = li + 1;
    }
    P.t[m] = tn;
    P.par[m] = ms.parity ^ 1;
    P.steps[m] = st + 1;
    P.vrain[m] += (double)ms.rinc * C.ncells * (C.dx * C.dx);
}

template <typename T> void launch_plan(const PlanLaunch<T>& P, hipStream_t s) {
    const int n = P.m_end - P.m_begin;
    if (n > 0) hipLaunchKernelGGL(k_plan<T>, dim3((n + 3) / 4), dim3(256), 0, s, P);
}

// ---------------------------------------------------------------------------
// fused step: every link around a cell from (h^n, q^n), continuity with the
// new discharges and the rain depth, per-member maximum of the new depth.
// One lane per (cell, member-in-chunk); a workgroup covers a tile of cells for
// `chunks_per_group` consecutive member chunks, reusing the shared bed and
// roughness of its cells from registers.
// ---------------------------------------------------------------------------
template <typename T, int MI>
__global__ __launch_bounds__(kBlock) void k_step(const StepLaunch<T> L) {
    using HB = typename HBits<T>::type;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int ci = 0;
    for (int i = 1; i < L.n_catch; ++i)
        if (b >= L.c[i].block_begin) ci = i;
    const CatchDev<T>& C = L.c[ci];
    const int lb = b - C.block_begin;
    const int grp = lb % C.groups;
    const int tile = lb / C.groups;
    const int tyi = tile / C.tiles_x;
    const int txi = tile - tyi * C.tiles_x;
    const int txl = C.tx_log2;
    const int lane = threadIdx.x % MI;
    const int p = threadIdx.x / MI;
    const int TY = (kBlock / MI) >> txl;
    const int nx = C.nx, ny = C.ny;
    const int cx = (txi << txl) + (p & ((1 << txl) - 1));
    const int cy = tyi * TY + (p >> txl);
    const bool in = cx < nx && cy < ny;
    const int k0 = grp * C.chunks_per_group;
    const int k1 = min(k0 + C.chunks_per_group, C.n_chunks);
    const int mend = min(k1 * MI, C.n_members);
    // Recompute mode (adjoint tape): every member reads copy 0 and writes copy 1, members that
    // do not step copy their state across, clamp flags are recorded, ledgers and the depth
    // maximum are left alone.
    const bool rec = L.recompute != 0;
    int any = rec ? 1 : 0;
    for (int m = k0 * MI + (int)threadIdx.x; m < mend && !rec; m += kBlock) any |= L.ms[C.member_off + m].active;
    if (!__syncthreads_or(any)) return;

    // shared bed and roughness of this cell and its four neighbours
    const bool hasE = cx + 1 < nx, hasW = cx > 0, hasS = cy + 1 < ny, hasN = cy > 0;
    const T g = C.g;
    T dzE = 0, dzW = 0, dzS = 0, dzN = 0, GE = 0, GW = 0, GS = 0, GN = 0;
    if (in) {
        const size_t c0 = (size_t)cy * nx + cx;
        const T z0 = C.z[c0], n0 = C.n[c0];
        const T gb = g * (n0 * n0);
        if (hasE) {
            const T z1 = C.z[c0 + 1], n1 = C.n[c0 + 1];
            const T nf = T(0.5) * (n0 + n1);
            dzE = z1 - z0;
            GE = g * (nf * nf);
        } else {
            GE = gb;
        }
        if (hasW) {
            const T z1 = C.z[c0 - 1], n1 = C.n[c0 - 1];
            const T nf = T(0.5) * (n1 + n0);
            dzW = z0 - z1;
            GW = g * (nf * nf);
        } else {
            GW = gb;
        }
        if (hasS) {
            const T z1 = C.z[c0 + nx], n1 = C.n[c0 + nx];
            const T nf = T(0.5) * (n0 + n1);
            dzS = z1 - z0;
            GS = g * (nf * nf);
        } else {
            GS = gb;
        }
        if (hasN) {
            const T z1 = C.z[c0 - nx], n1 = C.n[c0 - nx];
            const T nf = T(0.5) * (n1 + n0);
            dzN = z0 - z1;
            GN = g * (nf * nf);
        } else {
            GN = gb;
        }
    }
    const T hdry = C.hdry;
    const int nb = 2 * (nx + ny);
    const int bin = blockIdx.x & (kBins - 1);
    const size_t plane = (size_t)ny * nx * MI;
    const size_t rowMI = (size_t)nx * MI;

    for (int k = k0; k < k1; ++k) {
        const int ml = k * MI + lane;
        MemberStep<T> ms;
        bool act = false;
        if (ml < C.n_members) {
            ms = L.ms[C.member_off + ml];
            act = in && ms.active;
        }
        T hn = T(0);
        if (rec && in && ml < C.n_members && !act) {
            const size_t idx = (size_t)k * plane + ((size_t)cy * nx + cx) * MI + lane;
            C.h[1][idx] = C.h[0][idx];
            C.qx[1][idx] = C.qx[0][idx];
            C.qy[1][idx] = C.qy[0][idx];
            if (!hasW) C.qw[1][((size_t)k * ny + cy) * MI + lane] = C.qw[0][((size_t)k * ny + cy) * MI + lane];
            if (!hasN) C.qn[1][((size_t)k * nx + cx) * MI + lane] = C.qn[0][((size_t)k * nx + cx) * MI + lane];
            L.clamp_out[idx] = 0;
        }
        if (act) {
            const int sp = rec ? 0 : ms.parity, dp = sp ^ 1;
            const T* __restrict__ hs = C.h[sp];
            const T* __restrict__ qxs = C.qx[sp];
            const T* __restrict__ qys = C.qy[sp];
            const size_t idx = (size_t)k * plane + ((size_t)cy * nx + cx) * MI + lane;
            const T h0 = hs[idx];
            const T hE = hasE ? hs[idx + MI] : T(0);
            const T hW = hasW ? hs[idx - MI] : T(0);
            const T hS = hasS ? hs[idx + rowMI] : T(0);
            const T hN = hasN ? hs[idx - rowMI] : T(0);
            const T qE = qxs[idx];
            const T qS = qys[idx];
            const T qW = hasW ? qxs[idx - MI] : C.qw[sp][((size_t)k * ny + cy) * MI + lane];
            const T qN = hasN ? qys[idx - rowMI] : C.qn[sp][((size_t)k * nx + cx) * MI + lane];
            T fE, fS, fW, fN;
            if (hasE)
                fE = link_in(qE, h0, hE, dzE, GE, ms, hdry);
            else
                fE = C.edge_open[1] ? link_open(qE, h0, GE, C.edge_slope[1], ms, hdry) : T(0);
            if (hasS)
                fS = link_in(qS, h0, hS, dzS, GS, ms, hdry);
            else
                fS = C.edge_open[2] ? link_open(qS, h0, GS, C.edge_slope[2], ms, hdry) : T(0);
            if (hasW)
                fW = link_in(qW, hW, h0, dzW, GW, ms, hdry);
            else
                fW = C.edge_open[3] ? -link_open(-qW, h0, GW, C.edge_slope[3], ms, hdry) : T(0);
            if (hasN)
                fN = link_in(qN, hN, h0, dzN, GN, ms, hdry);
            else
                fN = C.edge_open[0] ? -link_open(-qN, h0, GN, C.edge_slope[0], ms, hdry) : T(0);
            // Eq. 1 with the four links of Sec. 3.1 (west/east x-links, north/south y-links)
            const T dv = ((fW - fE) + fN) - fS;
            hn = depth_add(h0, ms.dtdx * dv + ms.rinc, ms.seed, (uint32_t)(cy * nx + cx));
            const bool clamped = hn < T(0);
            if (clamped) {
                if (!rec) atomicAdd(&L.vclamp[C.member_off + ml], -(double)hn * (C.dx * C.dx));
                hn = T(0);
            }
            if (rec) L.clamp_out[idx] = clamped ? 1 : 0;
            if (hn == T(0)) hn = T(0);  // canonical +0 for the bit-pattern maximum
            C.h[dp][idx] = hn;
            if (!rec && C.peak) C.peak[idx] = fmax(C.peak[idx], hn);
            C.qx[dp][idx] = fE;
            C.qy[dp][idx] = fS;
            if (!hasW) C.qw[dp][((size_t)k * ny + cy) * MI + lane] = fW;
            if (!hasN) C.qn[dp][((size_t)k * nx + cx) * MI + lane] = fN;
            if (!rec && !(hasE && hasW && hasS && hasN)) {
                double* acc = C.out_acc + (size_t)ml * nb;
                if (!hasN && C.edge_open[0]) acc[cx] += -(double)fN * ms.dxdt;
                if (!hasS && C.edge_open[2]) acc[nx + cx] += (double)fS * ms.dxdt;
                if (!hasW && C.edge_open[3]) acc[2 * nx + cy] += -(double)fW * ms.dxdt;
                if (!hasE && C.edge_open[1]) acc[2 * nx + ny + cy] += (double)fE * ms.dxdt;
            }
        }
        // depth maximum per member over the wavefront, on the IEEE bit pattern
        // (depths are >= 0, and a NaN or Inf compares above every finite depth)
        HB v = to_bits(hn);
#pragma unroll
        for (int off = MI; off < 64; off <<= 1) {
            const HB o = __shfl_xor(v, off, 64);
            v = o > v ? o : v;
        }
        if (!rec && (threadIdx.x & 63) < MI && ml < C.n_members && v != 0) {
            HB* a = L.hbins + (size_t)bin * L.n_total + C.member_off + ml;
            const HB cur = __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v > cur) atomicMax(a, v);
        }
    }
}

template <typename T, int MI> void launch_step(const StepLaunch<T>& L, hipStream_t s) {
    hipLaunchKernelGGL((k_step<T, MI>), dim3(L.total_blocks), dim3(kBlock), 0, s, L);
}

template <typename T> void launch_step_mi(int mi, const StepLaunch<T>& L, hipStream_t s) {
    switch (mi) {
        case 1: launch_step<T, 1>(L, s); break;
        case 2: launch_step<T, 2>(L, s); break;
        case 4: launch_step<T, 4>(L, s); break;
        default: launch_step<T, 8>(L, s); break;
    }
}

// ---------------------------------------------------------------------------
// members still short of t_end
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_count_active(int n, const double* t, const int32_t* fault,
                                                      const double* t_end, const int32_t* status,
                                                      const int64_t* steps, const int64_t* lim, int32_t* out) {
    __shared__ int part[4];
    int c = 0;
    const double te = *t_end;
    for (int m = threadIdx.x; m < n; m += 256)
        c += (!fault[m] && t[m] < te && (!lim || steps[m] < lim[m])) ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = part[0] + part[1] + part[2] + part[3];
        out[1] = status[0];
    }
}

void launch_count_active(int n_total, const double* t, const int32_t* fault, const double* t_end,
                         const int32_t* status, const int64_t* steps, const int64_t* lim, int32_t* out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, n_total, t, fault, t_end, status, steps, lim, out);
}

__global__ __launch_bounds__(256) void k_count_group(int n, const double* t, const int32_t* fault,
                                                     const double* t_end, const int32_t* status,
                                                     const int32_t* seg_cnt, const int32_t* pool_next,
                                                     int32_t* out) {
    __shared__ int part[4], mpart[4];
    int c = 0, mx = 0;
    const double te = *t_end;
    for (int m = threadIdx.x; m < n; m += 256) {
        c += (!fault[m] && t[m] < te) ? 1 : 0;
        mx = max(mx, seg_cnt[m]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_xor(c, off, 64);
        mx = max(mx, __shfl_xor(mx, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6] = c;
        mpart[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = part[0] + part[1] + part[2] + part[3];
        out[1] = status[0];
        out[2] = max(max(mpart[0], mpart[1]), max(mpart[2], mpart[3]));
        out[3] = *pool_next;
    }
}

void launch_count_group(int G, const double* t, const int32_t* fault, const double* t_end, const int32_t* status,
                        const int32_t* seg_cnt, const int32_t* pool_next, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_count_group, dim3(1), dim3(256), 0, s, G, t, fault, t_end, status, seg_cnt, pool_next,
                       out);
}

__global__ __launch_bounds__(256) void k_step_limit(int n, const int64_t* steps, int64_t add, int64_t* lim) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < n) lim[m] = add < 0 ? INT64_MAX : steps[m] + add;
}

void launch_step_limit(int n_total, const int64_t* steps, int64_t n, int64_t* lim, hipStream_t s) {
    hipLaunchKernelGGL(k_step_limit, dim3((n_total + 255) / 256), dim3(256), 0, s, n_total, steps, n, lim);
}

template <typename HB> __global__ __launch_bounds__(256) void k_zero_bins(int off, int n, int n_total, HB* bins) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * kBins) return;
    bins[(size_t)(e / n) * n_total + off + e % n] = 0;
}

template <typename HB> void launch_zero_bins(int off, int n, int n_total, HB* bins, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_bins<HB>, dim3((n * kBins + 255) / 256), dim3(256), 0, s, off, n, n_total, bins);
}

// After resampling slot j holds a copy of member anc[j]: its depth maximum follows.
template <typename HB>
__global__ __launch_bounds__(1024) void k_permute_bins(int off, int n, int n_total, HB* bins, const int32_t* anc,
                                                       const int32_t* flag) {
    if (flag[0] == 0) return;
    const int j = threadIdx.x;
    HB v = 0;
    if (j < n) {
        const int a = anc[j];
        for (int b = 0; b < kBins; ++b) {
            const HB x = bins[(size_t)b * n_total + off + a];
            v = x > v ? x : v;
        }
    }
    __syncthreads();
    if (j < n)
        for (int b = 0; b < kBins; ++b) bins[(size_t)b * n_total + off + j] = b == 0 ? v : HB(0);
}

template <typename HB>
void launch_permute_bins(int off, int n, int n_total, HB* bins, const int32_t* anc, const int32_t* flag,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_permute_bins<HB>, dim3(1), dim3(((n + 63) / 64) * 64), 0, s, off, n, n_total, bins, anc,
                       flag);
}

template void launch_zero_bins<uint32_t>(int, int, int, uint32_t*, hipStream_t);
template void launch_zero_bins<unsigned long long>(int, int, int, unsigned long long*, hipStream_t);
template void launch_permute_bins<uint32_t>(int, int, int, uint32_t*, const int32_t*, const int32_t*, hipStream_t);
template void launch_permute_bins<unsigned long long>(int, int, int, unsigned long long*, const int32_t*,
                                                      const int32_t*, hipStream_t);

// ---------------------------------------------------------------------------
// element-wise helpers over one catchment: lane = (cell, member)
// ---------------------------------------------------------------------------
// Depth maximum of the current state into bin 0 (bins must be zero);
// blockIdx.y = member.
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_hmax_init(const CatchDev<T> C, const int32_t* par,
                                                   typename HBits<T>::type* hbins, int n_total) {
    using HB = typename HBits<T>::type;
    const int m = blockIdx.y;
    const size_t ncell = (size_t)C.ny * C.nx;
    const T* h = C.h[par[C.member_off + m]];
    HB best = 0;
    for (size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x; cell < ncell;
         cell += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(cell / C.nx), c = (int)(cell % C.nx);
        const HB bv = to_bits(h[state_index<T, MI>(C, m, r, c)] + T(0));
        best = bv > best ? bv : best;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const HB o = __shfl_xor(best, off, 64);
        best = o > best ? o : best;
    }
    if ((threadIdx.x & 63) == 0 && best != 0) atomicMax(hbins + C.member_off + m, best);
}

template <typename T>
void launch_hmax_init(int mi, const CatchDev<T>& C, const int32_t* par, typename HBits<T>::type* hbins,
                      int n_total, hipStream_t s) {
    const size_t ncell = (size_t)C.ny * C.nx;
    dim3 grid((unsigned)std::min<size_t>((ncell + 255) / 256, 512), C.n_members);
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_hmax_init<T, 1>), grid, dim3(256), 0, s, C, par, hbins, n_total); break;
        case 2: hipLaunchKernelGGL((k_hmax_init<T, 2>), grid, dim3(256), 0, s, C, par, hbins, n_total); break;
        case 4: hipLaunchKernelGGL((k_hmax_init<T, 4>), grid, dim3(256), 0, s, C, par, hbins, n_total); break;
        default: hipLaunchKernelGGL((k_hmax_init<T, 8>), grid, dim3(256), 0, s, C, par, hbins, n_total); break;
    }
}

// Storage sum(h) dx^2 per member, added into out[member] (out must be zero).
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_storage(const CatchDev<T> C, const int32_t* par, double* out) {
    const int m = blockIdx.y;
    const size_t ncell = (size_t)C.ny * C.nx;
    const T* h = C.h[par[C.member_off + m]];
    double acc = 0.0;
    for (size_t cell = (size_t)blockIdx.x * blockDim.x + threadIdx.x; cell < ncell;
         cell += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(cell / C.nx), c = (int)(cell % C.nx);
        acc += (double)h[state_index<T, MI>(C, m, r, c)];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out + m, ((part[0] + part[1]) + (part[2] + part[3])) * (C.dx * C.dx));
}

template <typename T>
void launch_storage(int mi, const CatchDev<T>& C, const int32_t* par, double* out, hipStream_t s) {
    const size_t ncell = (size_t)C.ny * C.nx;
    dim3 grid((unsigned)std::min<size_t>((ncell + 255) / 256, 1024), C.n_members);
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_storage<T, 1>), grid, dim3(256), 0, s, C, par, out); break;
        case 2: hipLaunchKernelGGL((k_storage<T, 2>), grid, dim3(256), 0, s, C, par, out); break;
        case 4: hipLaunchKernelGGL((k_storage<T, 4>), grid, dim3(256), 0, s, C, par, out); break;
        default: hipLaunchKernelGGL((k_storage<T, 8>), grid, dim3(256), 0, s, C, par, out); break;
    }
}

// One member's field in the host layout (H: ny*nx, QX: ny*(nx+1), QY: (ny+1)*nx).
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_field(const CatchDev<T> C, int m, int p, int which, double* buf,
                                               int to_state) {
    const int ny = C.ny, nx = C.nx;
    const size_t n = (which == 0 || which == 3) ? (size_t)ny * nx
                     : which == 1               ? (size_t)ny * (nx + 1)
                                                : (size_t)(ny + 1) * nx;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int k = m / MI, lane = m % MI;
    T* ptr;
    if (which == 3) {
        ptr = C.peak + state_index<T, MI>(C, m, (int)(e / nx), (int)(e % nx));
    } else if (which == 0) {
        ptr = C.h[p] + state_index<T, MI>(C, m, (int)(e / nx), (int)(e % nx));
    } else if (which == 1) {
        const int r = (int)(e / (nx + 1)), c = (int)(e % (nx + 1));
        ptr = (c == 0) ? C.qw[p] + ((size_t)k * ny + r) * MI + lane : C.qx[p] + state_index<T, MI>(C, m, r, c - 1);
    } else {
        const int r = (int)(e / nx), c = (int)(e % nx);
        ptr = (r == 0) ? C.qn[p] + ((size_t)k * nx + c) * MI + lane : C.qy[p] + state_index<T, MI>(C, m, r - 1, c);
    }
    if (to_state)
        *ptr = (T)buf[e] + T(0);
    else
        buf[e] = (double)*ptr;
}

template <typename T>
static void launch_field(int mi, const CatchDev<T>& C, int member, int par, int which, double* buf, int to_state,
                         hipStream_t s) {
    const int ny = C.ny, nx = C.nx;
    const size_t n = (which == 0 || which == 3) ? (size_t)ny * nx
                     : which == 1               ? (size_t)ny * (nx + 1)
                                                : (size_t)(ny + 1) * nx;
    dim3 grid((unsigned)((n + 255) / 256));
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_field<T, 1>), grid, dim3(256), 0, s, C, member, par, which, buf, to_state); break;
        case 2: hipLaunchKernelGGL((k_field<T, 2>), grid, dim3(256), 0, s, C, member, par, which, buf, to_state); break;
        case 4: hipLaunchKernelGGL((k_field<T, 4>), grid, dim3(256), 0, s, C, member, par, which, buf, to_state); break;
        default: hipLaunchKernelGGL((k_field<T, 8>), grid, dim3(256), 0, s, C, member, par, which, buf, to_state); break;
    }
}

template <typename T>
void launch_get_field(int mi, const CatchDev<T>& C, int member, int par, int which, double* out, hipStream_t s) {
    launch_field<T>(mi, C, member, par, which, out, 0, s);
}
template <typename T>
void launch_set_field(int mi, const CatchDev<T>& C, int member, int par, int which, const double* in,
                      hipStream_t s) {
    launch_field<T>(mi, C, member, par, which, const_cast<double*>(in), 1, s);
}

// Wet/dry decision of every link of member m from its state in copy p, in the
// host link layouts (x-links [ny][nx+1], y-links [ny+1][nx]).  Interior links
// use link_depth, as the step does; an open edge link is wet when its inner
// cell's depth exceeds h_dry; walls and inflow links (prescribed discharge,
// no decision) are 0.  One lane per link.
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_wetmask(const CatchDev<T> C, int m, int p, uint8_t* wx, uint8_t* wy) {
    const int ny = C.ny, nx = C.nx;
    const size_t nxl = (size_t)ny * (nx + 1), nyl = (size_t)(ny + 1) * nx;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nxl + nyl) return;
    const T* H = C.h[p];
    const T hdry = C.hdry;
    auto hat = [&](int r, int c) -> T { return H[state_index<T, MI>(C, m, r, c)]; };
    auto zat = [&](int r, int c) -> T { return C.z[(size_t)r * nx + c]; };
    // inflow link ids in the order N (c), S (nx + c), W (2 nx + r), E (2 nx + ny + r)
    auto inflow = [&](int i) -> bool { return C.inflow_id && C.inflow_id[i] >= 0; };
    uint8_t w = 0;
    if (e < nxl) {
        const int r = (int)(e / (nx + 1)), c = (int)(e % (nx + 1));
        if (c == 0)
            w = C.edge_open[3] && !inflow(2 * nx + r) && hat(r, 0) > hdry;
        else if (c == nx)
            w = C.edge_open[1] && !inflow(2 * nx + ny + r) && hat(r, nx - 1) > hdry;
        else
            w = link_depth(hat(r, c - 1), hat(r, c), zat(r, c) - zat(r, c - 1)) > hdry;
        wx[e] = w;
    } else {
        const size_t f = e - nxl;
        const int r = (int)(f / nx), c = (int)(f % nx);
        if (r == 0)
            w = C.edge_open[0] && !inflow(c) && hat(0, c) > hdry;
        else if (r == ny)
            w = C.edge_open[2] && !inflow(nx + c) && hat(ny - 1, c) > hdry;
        else
            w = link_depth(hat(r - 1, c), hat(r, c), zat(r, c) - zat(r - 1, c)) > hdry;
        wy[f] = w;
    }
}

template <typename T>
void launch_wetmask(int mi, const CatchDev<T>& C, int member, int p, uint8_t* wx, uint8_t* wy, hipStream_t s) {
    const size_t n = (size_t)C.ny * (C.nx + 1) + (size_t)(C.ny + 1) * C.nx;
    dim3 grid((unsigned)((n + 255) / 256));
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_wetmask<T, 1>), grid, dim3(256), 0, s, C, member, p, wx, wy); break;
        case 2: hipLaunchKernelGGL((k_wetmask<T, 2>), grid, dim3(256), 0, s, C, member, p, wx, wy); break;
        case 4: hipLaunchKernelGGL((k_wetmask<T, 4>), grid, dim3(256), 0, s, C, member, p, wx, wy); break;
        default: hipLaunchKernelGGL((k_wetmask<T, 8>), grid, dim3(256), 0, s, C, member, p, wx, wy); break;
    }
}

// Observation operator: depth of every member at every gauge cell, [N*K].
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_gauges(const CatchDev<T> C, const int32_t* par, int K, const int32_t* grc,
                                                double* y, int ys) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= C.n_members * K) return;
    const int m = e / K, k = e % K;
    const T* h = C.h[par[C.member_off + m]];
    y[(size_t)m * ys + k] = (double)h[state_index<T, MI>(C, m, grc[2 * k], grc[2 * k + 1])];
}

template <typename T>
void launch_gauges(int mi, const CatchDev<T>& C, const int32_t* par, int n_gauges, const int32_t* grc, double* y,
                   int ys, hipStream_t s) {
    dim3 grid((C.n_members * n_gauges + 255) / 256);
    if (grid.x == 0) return;
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_gauges<T, 1>), grid, dim3(256), 0, s, C, par, n_gauges, grc, y, ys); break;
        case 2: hipLaunchKernelGGL((k_gauges<T, 2>), grid, dim3(256), 0, s, C, par, n_gauges, grc, y, ys); break;
        case 4: hipLaunchKernelGGL((k_gauges<T, 4>), grid, dim3(256), 0, s, C, par, n_gauges, grc, y, ys); break;
        default: hipLaunchKernelGGL((k_gauges<T, 8>), grid, dim3(256), 0, s, C, par, n_gauges, grc, y, ys); break;
    }
}

// Streamflow through sections (Sec. 4.4): one workgroup per (section, member)
// sums sign * q over the section's links in FP64 (lanes stride the links, then
// a fixed reduction tree), times dx.
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_sections(const CatchDev<T> C, const int32_t* par, const int32_t* offs,
                                                  const int32_t* code, const int32_t* index, double* out,
                                                  int ostride, int ooff) {
    const int sec = blockIdx.x, m = blockIdx.y;
    const int p = par[C.member_off + m];
    const int chunk = m / MI, lane = m % MI;
    const size_t plane = (size_t)C.ny * C.nx * MI;
    double acc = 0.0;
    for (int l = offs[sec] + (int)threadIdx.x; l < offs[sec + 1]; l += 256) {
        const int cd = code[l], ix = index[l];
        double q;
        switch (cd & 3) {
            case 0: q = (double)C.qx[p][(size_t)chunk * plane + (size_t)ix * MI + lane]; break;
            case 1: q = (double)C.qy[p][(size_t)chunk * plane + (size_t)ix * MI + lane]; break;
            case 2: q = (double)C.qw[p][((size_t)chunk * C.ny + ix) * MI + lane]; break;
            default: q = (double)C.qn[p][((size_t)chunk * C.nx + ix) * MI + lane]; break;
        }
        acc += (cd & 4) ? -q : q;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[(size_t)m * ostride + ooff + sec] = ((part[0] + part[1]) + (part[2] + part[3])) * C.dx;
}

template <typename T>
void launch_sections(int mi, const CatchDev<T>& C, const int32_t* par, int n_sections, const int32_t* offs,
                     const int32_t* code, const int32_t* index, double* out, int ostride, int ooff, hipStream_t s) {
    if (n_sections <= 0 || C.n_members <= 0) return;
    const dim3 grid(n_sections, C.n_members);
    switch (mi) {
        case 1:
            hipLaunchKernelGGL((k_sections<T, 1>), grid, dim3(256), 0, s, C, par, offs, code, index, out, ostride, ooff);
            break;
        case 2:
            hipLaunchKernelGGL((k_sections<T, 2>), grid, dim3(256), 0, s, C, par, offs, code, index, out, ostride, ooff);
            break;
        case 4:
            hipLaunchKernelGGL((k_sections<T, 4>), grid, dim3(256), 0, s, C, par, offs, code, index, out, ostride, ooff);
            break;
        default:
            hipLaunchKernelGGL((k_sections<T, 8>), grid, dim3(256), 0, s, C, par, offs, code, index, out, ostride, ooff);
            break;
    }
}

// Fold the per-edge-link outflow accumulators into the per-member total.
__global__ __launch_bounds__(256) void k_flush_outflow(int nb, double* acc, double* vout) {
    const int m = blockIdx.x;
    double* a = acc + (size_t)m * nb;
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        s += a[i];
        a[i] = 0.0;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) vout[m] += (part[0] + part[1]) + (part[2] + part[3]);
}

void launch_flush_outflow(int n_members, int nb, double* out_acc, double* vout, hipStream_t s) {
    if (n_members > 0) hipLaunchKernelGGL(k_flush_outflow, dim3(n_members), dim3(256), 0, s, nb, out_acc, vout);
}

// explicit instantiations
template void launch_plan<float>(const PlanLaunch<float>&, hipStream_t);
template void launch_plan<double>(const PlanLaunch<double>&, hipStream_t);
template void launch_step_mi<float>(int, const StepLaunch<float>&, hipStream_t);
template void launch_step_mi<double>(int, const StepLaunch<double>&, hipStream_t);
template void launch_hmax_init<float>(int, const CatchDev<float>&, const int32_t*, uint32_t*, int, hipStream_t);
template void launch_hmax_init<double>(int, const CatchDev<double>&, const int32_t*, unsigned long long*, int,
                                       hipStream_t);
template void launch_storage<float>(int, const CatchDev<float>&, const int32_t*, double*, hipStream_t);
template void launch_storage<double>(int, const CatchDev<double>&, const int32_t*, double*, hipStream_t);
template void launch_get_field<float>(int, const CatchDev<float>&, int, int, int, double*, hipStream_t);
template void launch_get_field<double>(int, const CatchDev<double>&, int, int, int, double*, hipStream_t);
template void launch_set_field<float>(int, const CatchDev<float>&, int, int, int, const double*, hipStream_t);
template void launch_set_field<double>(int, const CatchDev<double>&, int, int, int, const double*, hipStream_t);
template void launch_wetmask<float>(int, const CatchDev<float>&, int, int, uint8_t*, uint8_t*, hipStream_t);
template void launch_wetmask<double>(int, const CatchDev<double>&, int, int, uint8_t*, uint8_t*, hipStream_t);
template void launch_gauges<float>(int, const CatchDev<float>&, const int32_t*, int, const int32_t*, double*, int,
                                   hipStream_t);
template void launch_gauges<double>(int, const CatchDev<double>&, const int32_t*, int, const int32_t*, double*, int,
                                    hipStream_t);
template void launch_sections<float>(int, const CatchDev<float>&, const int32_t*, int, const int32_t*,
                                     const int32_t*, const int32_t*, double*, int, int, hipStream_t);
template void launch_sections<double>(int, const CatchDev<double>&, const int32_t*, int, const int32_t*,
                                      const int32_t*, const int32_t*, double*, int, int, hipStream_t);

}  // namespace flood

namespace flood {

// ---------------------------------------------------------------------------
// Row-marching step for members stored in planes (MI = 1).
//
// One wavefront handles SEG members on a strip 62 cells wide and `march_rows`
// rows tall.  Lane l holds cell x0 - 1 + l: lanes 0 and 63 are halo cells that
// only supply their values to the neighbouring lanes, so horizontal neighbours
// (depth, bed, roughness, the east link of the lane to the left) come from
// lane shuffles.  Walking down the strip, the next row's depth, bed and
// roughness are loaded once and carried into the following iteration, and the
// new south link of a row is the north link of the next, so every state
// element is read once and written once; the bed and roughness rows are shared
// by the SEG members, whose independent streams keep more loads in flight per
// wavefront.  Whether a member steps is uniform across the wavefront, so idle
// members cost no divergence.  Each cell evaluates the same link functions on
// the same operands as k_step, so both kernels produce identical bits.
// ---------------------------------------------------------------------------
template <typename T, int SEG>
__global__ __launch_bounds__(kBlock) void k_march(const StepLaunch<T> L) {
    using HB = typename HBits<T>::type;
    const int lane = threadIdx.x & 63;
    // the wavefront index is uniform across the wavefront; saying so lets every
    // per-member quantity live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wg = xcd_remap(blockIdx.x, gridDim.x) * (kBlock / 64) + wave;
    int ci = 0;
    for (int i = 1; i < L.n_catch; ++i)
        if (wg >= L.c[i].wave_begin) ci = i;
    const CatchDev<T>& C = L.c[ci];
    const int local = wg - C.wave_begin;
    if (local >= C.n_waves) return;
    const int n_groups = (C.n_members + SEG - 1) / SEG;
    int kg, sx, sy;
    if (!march_wave(C, local, n_groups, kg, sx, sy)) return;
    MemberStep<T> ms[SEG];
    bool act[SEG];
    bool any = false;
#pragma unroll
    for (int s = 0; s < SEG; ++s) {
        const int k = kg * SEG + s;
        act[s] = false;
        if (k < C.n_members) {
            ms[s] = L.ms[C.member_off + k];
            act[s] = ms[s].active != 0;
        }
        any |= act[s];
    }
    if (!any) return;
    const int nx = C.nx, ny = C.ny;
    const int x = sx * 62 - 1 + lane;
    const bool inx = x >= 0 && x < nx;
    const bool own = lane >= 1 && lane <= 62 && inx;
    const bool hasE = x + 1 < nx, hasW = x > 0;
    const int r0 = sy * C.march_rows;
    const int r1 = min(r0 + C.march_rows, ny);
    const size_t plane = (size_t)ny * nx;
    const T* __restrict__ Z = C.z;
    const T* __restrict__ Nn = C.n;
    const T g = C.g, hdry = C.hdry;
    const int nb = 2 * (nx + ny);

    size_t c0 = (size_t)r0 * nx + x;
    T zc = inx ? Z[c0] : T(0);
    T nc = inx ? Nn[c0] : T(0);
    T zN = T(0), nN = T(0);
    if (inx && r0 > 0) {
        zN = Z[c0 - nx];
        nN = Nn[c0 - nx];
    }
    T hc[SEG], fN[SEG];
    HB vmax[SEG];
#pragma unroll
    for (int s = 0; s < SEG; ++s) {
        hc[s] = T(0);
        fN[s] = T(0);
        vmax[s] = 0;
        if (!act[s]) continue;
        const int k = kg * SEG + s;
        const int sp = ms[s].parity;
        const T* __restrict__ H = C.h[sp] + (size_t)k * plane;
        if (inx) {
            hc[s] = H[c0];
            if (r0 > 0) {
                const T nf = T(0.5) * (nN + nc);
                fN[s] = link_in(C.qy[sp][(size_t)k * plane + c0 - nx], H[c0 - nx], hc[s], zc - zN, g * (nf * nf),
                                ms[s], hdry);
            } else if (C.edge_open[0]) {
                fN[s] = -link_open(-C.qn[sp][(size_t)k * nx + x], hc[s], g * (nc * nc), C.edge_slope[0], ms[s], hdry);
            }
        }
    }
    for (int r = r0; r < r1; ++r) {
        const bool hasS = r + 1 < ny;
        T zs = T(0), ns = T(0);
        if (inx && hasS) {
            zs = Z[c0 + nx];
            ns = Nn[c0 + nx];
        }
        const T zE = __shfl_down(zc, 1, 64);
        const T nE = __shfl_down(nc, 1, 64);
        const T gb = g * (nc * nc);
        T nfE = T(0.5) * (nc + nE);
        const T GE = g * (nfE * nfE);
        const T nfS = T(0.5) * (nc + ns);
        const T GS = g * (nfS * nfS);
#pragma unroll
        for (int s = 0; s < SEG; ++s) {
            if (!act[s]) continue;
            const int k = kg * SEG + s;
            const MemberStep<T>& m = ms[s];
            const int sp = m.parity, dp = sp ^ 1;
            const size_t base = (size_t)k * plane;
            const T* __restrict__ H = C.h[sp] + base;
            T hs = T(0), qE = T(0), qS = T(0);
            if (inx) {
                qE = C.qx[sp][base + c0];
                qS = C.qy[sp][base + c0];
                if (hasS) hs = H[c0 + nx];
            }
            const T h0 = hc[s];
            const T hE = __shfl_down(h0, 1, 64);
            T fE;
            if (hasE)
                fE = link_in(qE, h0, hE, zE - zc, GE, m, hdry);
            else
                fE = C.edge_open[1] ? link_open(qE, h0, gb, C.edge_slope[1], m, hdry) : T(0);
            const T fWn = __shfl_up(fE, 1, 64);
            if (own) {
                T fW, fS;
                if (hasW)
                    fW = fWn;
                else
                    fW = C.edge_open[3] ? -link_open(-C.qw[sp][(size_t)k * ny + r], h0, gb, C.edge_slope[3], m, hdry)
                                        : T(0);
                if (hasS)
                    fS = link_in(qS, h0, hs, zs - zc, GS, m, hdry);
                else
                    fS = C.edge_open[2] ? link_open(qS, h0, gb, C.edge_slope[2], m, hdry) : T(0);
                const T dv = ((fW - fE) + fN[s]) - fS;
                T hn = depth_add(h0, m.dtdx * dv + m.rinc, m.seed, (uint32_t)(r * nx + x));
                if (hn < T(0)) {
                    atomicAdd(&L.vclamp[C.member_off + k], -(double)hn * (C.dx * C.dx));
                    hn = T(0);
                }
                if (hn == T(0)) hn = T(0);
                C.h[dp][base + c0] = hn;
                if (C.peak) C.peak[base + c0] = fmax(C.peak[base + c0], hn);
                C.qx[dp][base + c0] = fE;
                C.qy[dp][base + c0] = fS;
                if (!hasW) C.qw[dp][(size_t)k * ny + r] = fW;
                if (r == 0) C.qn[dp][(size_t)k * nx + x] = fN[s];
                if (!(hasE && hasW && hasS && r > 0)) {
                    double* acc = C.out_acc + (size_t)k * nb;
                    if (r == 0 && C.edge_open[0]) acc[x] += -(double)fN[s] * m.dxdt;
                    if (!hasS && C.edge_open[2]) acc[nx + x] += (double)fS * m.dxdt;
                    if (!hasW && C.edge_open[3]) acc[2 * nx + r] += -(double)fW * m.dxdt;
                    if (!hasE && C.edge_open[1]) acc[2 * nx + ny + r] += (double)fE * m.dxdt;
                }
                const HB hb = to_bits(hn);
                vmax[s] = hb > vmax[s] ? hb : vmax[s];
                fN[s] = fS;
            }
            hc[s] = hs;
        }
        zc = zs;
        nc = ns;
        c0 += nx;
    }
#pragma unroll
    for (int s = 0; s < SEG; ++s) {
        if (!act[s]) continue;
        HB v = vmax[s];
        for (int off = 32; off > 0; off >>= 1) {
            const HB o = __shfl_xor(v, off, 64);
            v = o > v ? o : v;
        }
        if (lane == 0 && v != 0) {
            HB* a = L.hbins + (size_t)(blockIdx.x & (kBins - 1)) * L.n_total + C.member_off + kg * SEG + s;
            const HB cur = __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v > cur) atomicMax(a, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Vectorised row-marching step (members in planes, nx a multiple of V): each
// lane owns V adjacent cells and moves them with one V-wide load or store, so a
// wavefront streams a strip of 64 V cells per row with five loads and three
// stores.  Every lane owns cells: the strip starts at a multiple of 64 V cells,
// so with a row pitch that is a multiple of 16 cells its stores cover whole
// 64-byte blocks and no block is shared with a neighbouring strip.  The two
// cells beside the strip come from four single-lane loads per row: lane 0 reads
// the west neighbour (depth, bed, roughness and its east link) and computes the
// strip's west link from it exactly as the neighbouring strip computes its
// east link, lane 63 reads the east neighbour (depth, bed, roughness).  Same
// link functions and operands as k_step: identical bits.
// ---------------------------------------------------------------------------
// PF = 1 issues the next row's loads before computing the current row (one row
// of lookahead), so each wavefront keeps its own loads in flight while it
// computes.  Loads use a column clamped into the grid and a row clamped to the
// last row, so no lane needs a branch or a zero fill around them: values of
// lanes outside the grid and of the row below the last are read but never used.
// REC = 0: the plain step between the member's two state copies.  REC = 1: tape
// recomputation for the adjoint (tape block ms.blk to block ms.blk_next, a
// clamped depth stored as -0, no ledger).  REC = 2: the adjoint's recording
// forward, the same blocks and marks with the plain step's ledger, depth-maximum
// bins and outflow.
template <typename T, int V, int NT, int REC, int PF, int EXT>
__global__ __launch_bounds__(kBlock) void k_marchv(const StepLaunch<T> L) {
    using HB = typename HBits<T>::type;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wg = xcd_remap(blockIdx.x, gridDim.x) * (kBlock / 64) + wave;
    int ci = 0;
    for (int i = 1; i < L.n_catch; ++i)
        if (wg >= L.c[i].wave_begin) ci = i;
    const CatchDev<T>& C = L.c[ci];
    const int local = wg - C.wave_begin;
    if (local >= C.n_waves) return;
    int k, sx, sy;
    if (!march_wave(C, local, C.n_members, k, sx, sy)) return;
    const MemberStep<T> ms = L.ms[C.member_off + k];
    if (!ms.active) return;
    const int nx = C.nx, ny = C.ny;
    const int x0 = sx * (64 * V);                          // first cell of the strip
    const int xl = x0 + V * lane;                          // first cell of this lane
    const bool own = xl < nx;                              // nx % V == 0: all V cells or none
    const bool westw = sx == 0;                            // wavefront-uniform edge tests
    const bool eastw = sx == C.strips_x - 1;
    const int xa = min(xl, nx - V);                        // load column
    // halo: lane 0 the cell west of the strip, lane 63 the one east of it
    // (clamped into the grid where there is none; then never used)
    const bool halo_lane = lane == 0 || lane == 63;
    const int xh = lane == 0 ? (westw ? 0 : x0 - 1) : (eastw ? nx - 1 : x0 + 64 * V);
    const int r0 = sy * C.march_rows;
    const int r1 = min(r0 + C.march_rows, ny);
    const size_t plane = (size_t)ny * nx;
    // source and destination of this member's state: the two copies, or (tape
    // recording and recomputation) the member's tape block and the block of its new state
    const T* __restrict__ H;
    const T* __restrict__ QX;
    const T* __restrict__ QY;
    T* __restrict__ Ho;
    T* __restrict__ QXo;
    T* __restrict__ QYo;
    const T* QWs;
    const T* QNs;
    T* QWo;
    T* QNo;
    if constexpr (REC) {
        const size_t bs = (size_t)ms.blk, bd = (size_t)ms.blk_next;
        H = C.h[0] + bs * plane;
        QX = C.qx[0] + bs * plane;
        QY = C.qy[0] + bs * plane;
        Ho = C.h[0] + bd * plane;
        QXo = C.qx[0] + bd * plane;
        QYo = C.qy[0] + bd * plane;
        QWs = C.qw[0] + bs * ny;
        QWo = C.qw[0] + bd * ny;
        QNs = C.qn[0] + bs * nx;
        QNo = C.qn[0] + bd * nx;
    } else {
        const int sp = ms.parity, dp = sp ^ 1;
        H = C.h[sp] + (size_t)k * plane;
        QX = C.qx[sp] + (size_t)k * plane;
        QY = C.qy[sp] + (size_t)k * plane;
        Ho = C.h[dp] + (size_t)k * plane;
        QXo = C.qx[dp] + (size_t)k * plane;
        QYo = C.qy[dp] + (size_t)k * plane;
        QWs = C.qw[sp] + (size_t)k * ny;
        QWo = C.qw[dp] + (size_t)k * ny;
        QNs = C.qn[sp] + (size_t)k * nx;
        QNo = C.qn[dp] + (size_t)k * nx;
    }
    const T* __restrict__ Z = C.z;
    const T* __restrict__ Nn = C.n;
    const T g = C.g, hdry = C.hdry;
    const int nb = 2 * (nx + ny);
    // inflow links (edge links with a prescribed inward discharge): the series
    // index of an edge link in the out_acc order, or -1; the series value is
    // picked by a select chain (a per-lane index into the step record would
    // go through private memory)
    const int8_t* __restrict__ INF = (EXT & 2) ? C.inflow_id : nullptr;
    auto inflow_q = [&](int id) -> T {
        T v = ms.qin[0];
        v = (id == 1) ? ms.qin[1] : v;
        v = (id == 2) ? ms.qin[2] : v;
        return (id == 3) ? ms.qin[3] : v;
    };
    // land cover: the cell's roughness is the member's value for its class, and
    // its rain is scaled by the class's runoff coefficient
    const uint8_t* __restrict__ CLS = (EXT & 1) ? C.cls : nullptr;
    const bool lc = (EXT & 1) && CLS != nullptr;
    // the member's class table lives in lanes: 0-3 its Manning n of each class,
    // 4-7 the runoff coefficients, 8-11 the drainage depth of the step for
    // draining classes (0 for the others); a cell's entries are read from those
    // lanes with ds_bpermute, a cross-lane read served by the LDS unit, instead
    // of compare-and-select chains on the VALU.  Every lookup is made where the
    // whole wavefront is active (the early returns above are wavefront-uniform).
    T tab = T(0);
    if (lc) {
        const int k = lane & 3;
        T cn = ms.cn[0], rc = C.class_rc[0];
        cn = (k == 1) ? ms.cn[1] : cn;
        cn = (k == 2) ? ms.cn[2] : cn;
        cn = (k == 3) ? ms.cn[3] : cn;
        rc = (k == 1) ? C.class_rc[1] : rc;
        rc = (k == 2) ? C.class_rc[2] : rc;
        rc = (k == 3) ? C.class_rc[3] : rc;
        const T dk = ((C.drain_mask >> k) & 1) ? ms.drain : T(0);
        tab = lane < 4 ? cn : lane < 8 ? rc : lane < 12 ? dk : T(0);
    }
    auto lut = [&](uint32_t k, int base) -> T { return lane_read(tab, (int)k + base); };
    auto rough = [&](uint32_t k) -> T { return lut(k, 0); };
    auto runoff = [&](uint32_t k) -> T { return lut(k, 4); };
    // roughness of V cells from the shared field, or from their classes (whose
    // packed bytes are returned in cw)
    auto load_n = [&](size_t c, T (&nv)[V], uint32_t& cw) {
        if (lc) {
            if constexpr (V == 4)
                cw = *reinterpret_cast<const uint32_t*>(CLS + c);
            else
                cw = *reinterpret_cast<const uint16_t*>(CLS + c);
#pragma unroll
            for (int j = 0; j < V; ++j) nv[j] = rough((cw >> (8 * j)) & 0xffu);
        } else {
            cw = 0;
            vload<T, V>(Nn + c, nv);
        }
    };

    size_t ca = (size_t)r0 * nx + xa;
    T hc[V], zc[V], nc[V], fN[V];
    uint32_t ccw;
    vload<T, V>(H + ca, hc);
    vload<T, V>(Z + ca, zc);
    load_n(ca, nc, ccw);
    if (r0 > 0) {
        T hN[V], zN[V], nN[V], qN[V];
        uint32_t cwN;
        vload<T, V>(H + ca - nx, hN);
        vload<T, V>(Z + ca - nx, zN);
        load_n(ca - nx, nN, cwN);
        vload<T, V>(QY + ca - nx, qN);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const T nf = T(0.5) * (nN[j] + nc[j]);
            fN[j] = link_in(qN[j], hN[j], hc[j], zc[j] - zN[j], g * (nf * nf), ms, hdry);
        }
    } else if (C.edge_open[0]) {
#pragma unroll
        for (int j = 0; j < V; ++j)
            fN[j] = -link_open(-QNs[xa + j], hc[j], g * (nc[j] * nc[j]), C.edge_slope[0], ms, hdry);
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j) fN[j] = T(0);
    }
    // inflow ids of the strip's north and south edge links, one byte per cell of
    // the lane (0xff: none), read before the row loop so that the loop keeps no
    // table addresses; the west and east ids are read per row, wavefront-uniform
    uint32_t nid4 = 0xffffffffu, sid4 = 0xffffffffu;
    if (INF) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            if (r0 == 0) nid4 = (nid4 & ~(0xffu << (8 * j))) | ((uint32_t)(uint8_t)INF[xa + j] << (8 * j));
            if (r1 == ny) sid4 = (sid4 & ~(0xffu << (8 * j))) | ((uint32_t)(uint8_t)INF[nx + xa + j] << (8 * j));
        }
    }
    auto id_of = [](uint32_t w, int j) -> int { return (int)(int8_t)(uint8_t)((w >> (8 * j)) & 0xffu); };
    if (INF && r0 == 0) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int id = id_of(nid4, j);
            if (id >= 0) fN[j] = inflow_q(id);
        }
    }
    // current row's links (qE, qS), the row below (hs, zs, ns, classes csw) and
    // the current row's halo cell (depth, bed, roughness or class, east link)
    T hs[V], zs[V], ns[V], qE[V], qS[V];
    uint32_t csw = 0;
    Halo<T> hx;
    auto load_row = [&](size_t c, bool below, T (&qe)[V], T (&qs)[V], T (&h2)[V], T (&z2)[V], T (&n2)[V],
                        uint32_t& cw2, Halo<T>& ho) {
        const size_t cb = below ? c + nx : c;
        if (NT) {
            vload_nt<T, V>(QX + c, qe);
            vload_nt<T, V>(QY + c, qs);
        } else {
            vload<T, V>(QX + c, qe);
            vload<T, V>(QY + c, qs);
        }
        vload<T, V>(H + cb, h2);
        vload<T, V>(Z + cb, z2);
        load_n(cb, n2, cw2);
        if (halo_lane) {
            const size_t c1 = c - xa + xh;
            ho.h = H[c1];
            ho.z = Z[c1];
            ho.q = QX[c1];
            if (lc)
                ho.cls = CLS[c1];
            else
                ho.n = Nn[c1];
        }
    };
    // roughness of the halo cell from its class: a cross-lane read, made with the
    // whole wavefront active
    auto halo_n = [&](const Halo<T>& ho) -> T { return lc ? rough(halo_lane ? ho.cls : 0u) : ho.n; };
    if (PF) load_row(ca, r0 + 1 < ny, qE, qS, hs, zs, ns, csw, hx);
    // PF == 2: a second row in flight (the links of the next row and the state
    // of the row after it), so each row's loads have two rows of work to arrive
    T hsB[V], zsB[V], nsB[V], qEB[V], qSB[V];
    uint32_t cswB = 0;
    Halo<T> hxB;
#pragma unroll
    for (int j = 0; j < V; ++j) hsB[j] = zsB[j] = nsB[j] = qEB[j] = qSB[j] = T(0);
    if (PF == 2 && r0 + 1 < r1) load_row(ca + nx, r0 + 2 < ny, qEB, qSB, hsB, zsB, nsB, cswB, hxB);
    HB vmax = 0;
    T vcl = T(0);
    T vdr = T(0);
    for (int r = r0; r < r1; ++r) {
        const bool hasS = r + 1 < ny;
        const int idW = (INF && westw) ? (int)INF[2 * nx + r] : -1;
        const int idE = (INF && eastw) ? (int)INF[2 * nx + ny + r] : -1;
        T hs2[V], zs2[V], ns2[V], qE2[V], qS2[V];
        uint32_t csw2 = 0;
        Halo<T> hx2;
        if (PF == 2) {
            if (r + 2 < r1) load_row(ca + 2 * (size_t)nx, r + 3 < ny, qE2, qS2, hs2, zs2, ns2, csw2, hx2);
        } else if (PF) {
            if (r + 1 < r1) load_row(ca + nx, r + 2 < ny, qE2, qS2, hs2, zs2, ns2, csw2, hx2);
        } else {
            load_row(ca, hasS, qE, qS, hs, zs, ns, csw, hx);
        }
        const T nH = halo_n(hx);
        // east neighbour of the lane's last cell = first cell of the next lane; for
        // lane 63 the halo cell east of the strip
        T hE = __shfl_down(hc[0], 1, 64);
        T zE = __shfl_down(zc[0], 1, 64);
        T nE = __shfl_down(nc[0], 1, 64);
        if (lane == 63) {
            hE = hx.h;
            zE = hx.z;
            nE = nH;
        }
        T fE[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const T h2 = (j + 1 < V) ? hc[j + 1] : hE;
            const T z2 = (j + 1 < V) ? zc[j + 1] : zE;
            const T n2 = (j + 1 < V) ? nc[j + 1] : nE;
            const T nf = T(0.5) * (nc[j] + n2);
            fE[j] = link_in(qE[j], hc[j], h2, z2 - zc[j], g * (nf * nf), ms, hdry);
        }
        if (eastw) {
#pragma unroll
            for (int j = 0; j < V; ++j)
                if (xl + j + 1 == nx) {
                    fE[j] = C.edge_open[1] ? link_open(qE[j], hc[j], g * (nc[j] * nc[j]), C.edge_slope[1], ms, hdry)
                                           : T(0);
                    if (idE >= 0) fE[j] = -inflow_q(idE);
                }
        }
        T fW[V];
        fW[0] = __shfl_up(fE[V - 1], 1, 64);
        if (lane == 0 && !westw) {
            // the strip's west link, as the strip to the west computes it (its last
            // cell's east link: same operands in the same order)
            const T nf = T(0.5) * (nH + nc[0]);
            fW[0] = link_in(hx.q, hx.h, hc[0], zc[0] - hx.z, g * (nf * nf), ms, hdry);
        }
#pragma unroll
        for (int j = 1; j < V; ++j) fW[j] = fE[j - 1];
        if (westw && xl == 0) {
            fW[0] = C.edge_open[3] ? -link_open(-QWs[r], hc[0], g * (nc[0] * nc[0]), C.edge_slope[3], ms, hdry)
                                   : T(0);
            if (idW >= 0) fW[0] = inflow_q(idW);
        }
        T fS[V];
        if (hasS) {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const T nf = T(0.5) * (nc[j] + ns[j]);
                fS[j] = link_in(qS[j], hc[j], hs[j], zs[j] - zc[j], g * (nf * nf), ms, hdry);
            }
        } else {
            if (C.edge_open[2]) {
#pragma unroll
                for (int j = 0; j < V; ++j)
                    fS[j] = link_open(qS[j], hc[j], g * (nc[j] * nc[j]), C.edge_slope[2], ms, hdry);
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j) fS[j] = T(0);
            }
            if (INF) {
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const int id = id_of(sid4, j);
                    if (id >= 0) fS[j] = -inflow_q(id);
                }
            }
        }
        T hn4[V];
        bool cf[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const T dv = ((fW[j] - fE[j]) + fN[j]) - fS[j];
            const uint32_t kc = (ccw >> (8 * j)) & 0xffu;
            const T rn = lc ? ms.rinc * runoff(kc) : ms.rinc;
            T hn = depth_add(hc[j], ms.dtdx * dv + rn, ms.seed, (uint32_t)(r * nx + xl + j));
            cf[j] = hn < T(0);
            vcl += (own && hn < T(0)) ? -hn : T(0);
            hn = (hn < T(0)) ? T(0) : hn;
            // drainage of draining classes, up to the water the cell holds
            const T loss = lc ? fmin(lut(kc, 8), hn) : T(0);
            hn = hn - loss;
            vdr += own ? loss : T(0);
            hn = (hn == T(0)) ? T(0) : hn;
            hn4[j] = hn;
            const HB hb = to_bits(hn);
            vmax = (own && hb > vmax) ? hb : vmax;
        }
        if (own) {
            // the tape keeps a clamped depth as -0 (the clamp branch for the adjoint)
            T ho4[V];
#pragma unroll
            for (int j = 0; j < V; ++j) ho4[j] = (REC && cf[j]) ? -T(0) : hn4[j];
            if (NT) {
                vstore_nt<T, V>(Ho + ca, ho4);
                vstore_nt<T, V>(QXo + ca, fE);
                vstore_nt<T, V>(QYo + ca, fS);
            } else {
                vstore<T, V>(Ho + ca, ho4);
                vstore<T, V>(QXo + ca, fE);
                vstore<T, V>(QYo + ca, fS);
            }
            if constexpr (REC != 1) {
                if (C.peak) {
                    T* PK = C.peak + (size_t)k * plane + ca;
                    T pk4[V];
                    vload<T, V>(PK, pk4);
#pragma unroll
                    for (int j = 0; j < V; ++j) pk4[j] = fmax(pk4[j], hn4[j]);
                    vstore<T, V>(PK, pk4);
                }
            }
            if (westw && xl == 0) QWo[r] = fW[0];
            if (r == 0) {
#pragma unroll
                for (int j = 0; j < V; ++j) QNo[xl + j] = fN[j];
            }
            // outflow through open edges (FP64 per member and edge link)
            if (REC != 1 && (westw || eastw || r == 0 || !hasS)) {
                double* acc = C.out_acc + (size_t)k * nb;
                // inflow links are not outflow: their volume is logged by the step planner
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const int x = xl + j;
                    if (r == 0 && C.edge_open[0] && id_of(nid4, j) < 0) acc[x] += -(double)fN[j] * ms.dxdt;
                    if (!hasS && C.edge_open[2] && id_of(sid4, j) < 0) acc[nx + x] += (double)fS[j] * ms.dxdt;
                    if (x == 0 && C.edge_open[3] && idW < 0) acc[2 * nx + r] += -(double)fW[j] * ms.dxdt;
                    if (x + 1 == nx && C.edge_open[1] && idE < 0) acc[2 * nx + ny + r] += (double)fE[j] * ms.dxdt;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
            fN[j] = fS[j];
            hc[j] = hs[j];
            zc[j] = zs[j];
            nc[j] = ns[j];
        }
        ccw = csw;
        if (PF == 2) {
            csw = cswB;
            cswB = csw2;
            hx = hxB;
            hxB = hx2;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                qE[j] = qEB[j];
                qS[j] = qSB[j];
                hs[j] = hsB[j];
                zs[j] = zsB[j];
                ns[j] = nsB[j];
                qEB[j] = qE2[j];
                qSB[j] = qS2[j];
                hsB[j] = hs2[j];
                zsB[j] = zs2[j];
                nsB[j] = ns2[j];
            }
        } else if (PF) {
            csw = csw2;
            hx = hx2;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                qE[j] = qE2[j];
                qS[j] = qS2[j];
                hs[j] = hs2[j];
                zs[j] = zs2[j];
                ns[j] = ns2[j];
            }
        }
        ca += nx;
    }
    if constexpr (REC != 1) {
        for (int off = 32; off > 0; off >>= 1) {
            const HB o = __shfl_xor(vmax, off, 64);
            vmax = o > vmax ? o : vmax;
        }
        double cl = (double)vcl;
        for (int off = 32; off > 0; off >>= 1) cl += __shfl_xor(cl, off, 64);
        if (lc) {
            double dr = (double)vdr;
            for (int off = 32; off > 0; off >>= 1) dr += __shfl_xor(dr, off, 64);
            // spread over kBins accumulators per member: the wavefronts in flight
            // mostly belong to one member, so a single address would serialise them
            if (lane == 0 && dr != 0.0)
                atomicAdd(C.drain_acc + (size_t)k * kBins + (blockIdx.x & (kBins - 1)), dr * (C.dx * C.dx));
        }
        if (lane == 0) {
            if (vmax != 0) {
                HB* a = L.hbins + (size_t)(blockIdx.x & (kBins - 1)) * L.n_total + C.member_off + k;
                const HB cur = __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (vmax > cur) atomicMax(a, vmax);
            }
            if (cl != 0.0) atomicAdd(&L.vclamp[C.member_off + k], cl * (C.dx * C.dx));
        }
    }
}

template <typename T, int EXT>
static void launch_marchv_ext(const StepLaunch<T>& L, int nt, int pf, const dim3 grid, hipStream_t s) {
    constexpr int V = march_vec<T>();
    if (nt && pf == 2)
        hipLaunchKernelGGL((k_marchv<T, V, 1, 0, 2, EXT>), grid, dim3(kBlock), 0, s, L);
    else if (nt && pf)
        hipLaunchKernelGGL((k_marchv<T, V, 1, 0, 1, EXT>), grid, dim3(kBlock), 0, s, L);
    else if (nt)
        hipLaunchKernelGGL((k_marchv<T, V, 1, 0, 0, EXT>), grid, dim3(kBlock), 0, s, L);
    else if (pf)
        hipLaunchKernelGGL((k_marchv<T, V, 0, 0, 1, EXT>), grid, dim3(kBlock), 0, s, L);
    else
        hipLaunchKernelGGL((k_marchv<T, V, 0, 0, 0, EXT>), grid, dim3(kBlock), 0, s, L);
}

// ext: bit 0 land cover, bit 1 inflow links; an instantiation carries only the
// code of the extensions it names, so the plain step keeps its register budget
template <typename T>
void launch_marchv(const StepLaunch<T>& L, int nt, int pf, int ext, int total_waves, hipStream_t s) {
    const int per = kBlock / 64;
    const dim3 grid((total_waves + per - 1) / per);
    switch (ext & 3) {
        case 0: launch_marchv_ext<T, 0>(L, nt, pf, grid, s); break;
        case 1: launch_marchv_ext<T, 1>(L, nt, pf, grid, s); break;
        case 2: launch_marchv_ext<T, 2>(L, nt, pf, grid, s); break;
        default: launch_marchv_ext<T, 3>(L, nt, pf, grid, s); break;
    }
}

// Tape recomputation of the adjoint (record = 0): the same step, reading and
// writing tape blocks, marking clamped depths as -0, leaving the ledger, the
// outflow accumulators and the depth maximum alone; members that do not step in
// the launch are skipped.  Recording forward (record = 1): the same blocks and
// marks, plus everything the plain step
// updates (depth maximum bins, clamp and outflow ledgers, running maximum).
template <typename T>
void launch_marchv_rec(const StepLaunch<T>& L, int pf, int record, int total_waves, hipStream_t s) {
    const int per = kBlock / 64;
    const dim3 grid((total_waves + per - 1) / per);
    constexpr int V = march_vec<T>();
    if (record) {
        if (pf)
            hipLaunchKernelGGL((k_marchv<T, V, 1, 2, 1, 0>), grid, dim3(kBlock), 0, s, L);
        else
            hipLaunchKernelGGL((k_marchv<T, V, 1, 2, 0, 0>), grid, dim3(kBlock), 0, s, L);
    } else if (pf) {
        hipLaunchKernelGGL((k_marchv<T, V, 0, 1, 1, 0>), grid, dim3(kBlock), 0, s, L);
    } else {
        hipLaunchKernelGGL((k_marchv<T, V, 0, 1, 0, 0>), grid, dim3(kBlock), 0, s, L);
    }
}

template void launch_marchv<float>(const StepLaunch<float>&, int, int, int, int, hipStream_t);
template void launch_marchv<double>(const StepLaunch<double>&, int, int, int, int, hipStream_t);
template void launch_marchv_rec<float>(const StepLaunch<float>&, int, int, int, hipStream_t);
template void launch_marchv_rec<double>(const StepLaunch<double>&, int, int, int, hipStream_t);

template <typename T> void launch_march(const StepLaunch<T>& L, int seg, int total_waves, hipStream_t s) {
    const int per = kBlock / 64;
    const dim3 grid((total_waves + per - 1) / per);
    switch (seg) {
        case 1: hipLaunchKernelGGL((k_march<T, 1>), grid, dim3(kBlock), 0, s, L); break;
        case 2: hipLaunchKernelGGL((k_march<T, 2>), grid, dim3(kBlock), 0, s, L); break;
        case 4: hipLaunchKernelGGL((k_march<T, 4>), grid, dim3(kBlock), 0, s, L); break;
        default: hipLaunchKernelGGL((k_march<T, 8>), grid, dim3(kBlock), 0, s, L); break;
    }
}

template void launch_march<float>(const StepLaunch<float>&, int, int, hipStream_t);
template void launch_march<double>(const StepLaunch<double>&, int, int, hipStream_t);


// ---------------------------------------------------------------------------
// Ensemble products of the running maximum depth (Sec. 4.4, Figs. 15-16).  A
// workgroup covers 64 cells with four wavefronts, one lane per cell in each:
// it stages its cells' member values in LDS (member-major, so the staging
// loads are contiguous in every member's plane), the first wavefront forms, in
// member order and FP64, the weight of the members at or above the threshold,
// and the four wavefronts share the candidates k: for each, the weight of the
// members at or below member k's value, again in member order; the smallest
// value whose weight reaches p W is the p-quantile (inverted distribution
// function), a minimum over the candidates that is the same in any order.
// ---------------------------------------------------------------------------
constexpr int kProdCells = 64;
constexpr int kProdWaves = 4;      // wavefronts per workgroup, splitting the candidates
constexpr int kProdMaxPct = 16;

constexpr int kProdUnroll = 8;   // percentile candidates evaluated per pass over the members

template <typename T, int MI, bool LDS>
__global__ __launch_bounds__(kProdCells * kProdWaves) void k_products(const CatchDev<T> C, double thr, int n_pct,
                                                                       const double* __restrict__ pct,
                                                                       const double* __restrict__ w, double W,
                                                                       double* __restrict__ prob,
                                                                       double* __restrict__ pout) {
    extern __shared__ unsigned char smem[];
    T* vals = reinterpret_cast<T*>(smem);
    const int N = C.n_members;
    const size_t ncell = (size_t)C.ny * C.nx;
    const int lane = (int)threadIdx.x % kProdCells;
    const int wave = (int)threadIdx.x / kProdCells;
    const size_t cell = (size_t)blockIdx.x * kProdCells + lane;
    const bool in = cell < ncell;
    const int r = in ? (int)(cell / C.nx) : 0, c = in ? (int)(cell % C.nx) : 0;
    auto value = [&](int m) -> T {
        if constexpr (LDS) return vals[(size_t)m * kProdCells + lane];
        else return C.peak[state_index<T, MI>(C, m, r, c)];
    };
    if constexpr (LDS) {
        for (int m = wave; m < N; m += kProdWaves)
            vals[(size_t)m * kProdCells + lane] = in ? C.peak[state_index<T, MI>(C, m, r, c)] : T(0);
    }
    __syncthreads();
    const bool want_pct = n_pct > 0 && pout != nullptr;   // the same for the whole grid
    double best[kProdMaxPct];
    double lim[kProdMaxPct];
    for (int i = 0; i < n_pct; ++i) {
        best[i] = INFINITY;
        lim[i] = pct[i] * W;
    }
    if (in) {
        if (wave == 0) {
            // w_m x 1 or x 0 in one FMA: the sum of the selected weights, rounded as
            // the plain additions are (weights are finite and >= 0)
            double hit = 0.0;
            for (int m = 0; m < N; ++m) hit = __builtin_fma(w[m], ((double)value(m) >= thr) ? 1.0 : 0.0, hit);
            if (prob) prob[cell] = hit / W;
        }
        // kProdUnroll candidates k per pass over the members: independent sums
        // (each still in member order), one read of each member value per pass;
        // the wavefronts take interleaved groups of candidates
        if (want_pct) {
            for (int k0 = wave * kProdUnroll; k0 < N; k0 += kProdWaves * kProdUnroll) {
                T vk[kProdUnroll];
                double cum[kProdUnroll];
#pragma unroll
                for (int q = 0; q < kProdUnroll; ++q) {
                    vk[q] = value(k0 + q < N ? k0 + q : N - 1);
                    cum[q] = 0.0;
                }
                for (int m = 0; m < N; ++m) {
                    const T vm = value(m);
                    const double wm = w[m];
#pragma unroll
                    for (int q = 0; q < kProdUnroll; ++q) cum[q] = __builtin_fma(wm, (vm <= vk[q]) ? 1.0 : 0.0, cum[q]);
                }
#pragma unroll
                for (int q = 0; q < kProdUnroll; ++q) {
                    if (k0 + q >= N) break;
                    for (int i = 0; i < n_pct; ++i)
                        if (cum[q] >= lim[i] && (double)vk[q] < best[i]) best[i] = (double)vk[q];
                }
            }
        }
    }
    if (!want_pct) return;   // uniform: no wavefront is left waiting at the barriers below
    // minimum over the wavefronts' candidates, through LDS (the staged values are done with)
    __syncthreads();
    double* red = reinterpret_cast<double*>(smem);   // [wave][percentile][lane]
    for (int i = 0; i < n_pct; ++i) red[((size_t)wave * n_pct + i) * kProdCells + lane] = best[i];
    __syncthreads();
    if (wave == 0 && in)
        for (int i = 0; i < n_pct; ++i) {
            double b = red[(size_t)i * kProdCells + lane];
            for (int v = 1; v < kProdWaves; ++v) {
                const double o = red[((size_t)v * n_pct + i) * kProdCells + lane];
                b = o < b ? o : b;
            }
            pout[(size_t)i * ncell + cell] = b;
        }
}

template <typename T, int MI>
static void launch_products_mi(const CatchDev<T>& C, double thr, int n_pct, const double* pct, const double* w,
                               double W, double* prob, double* pout, hipStream_t s) {
    const size_t ncell = (size_t)C.ny * C.nx;
    const dim3 grid((unsigned)((ncell + kProdCells - 1) / kProdCells));
    const dim3 block(kProdCells * kProdWaves);
    const size_t stage = (size_t)C.n_members * kProdCells * sizeof(T);
    const size_t red = (size_t)kProdWaves * std::max(n_pct, 1) * kProdCells * sizeof(double);
    if (stage <= 48 * 1024)
        hipLaunchKernelGGL((k_products<T, MI, true>), grid, block, std::max(stage, red), s, C, thr, n_pct, pct, w, W,
                           prob, pout);
    else
        hipLaunchKernelGGL((k_products<T, MI, false>), grid, block, red, s, C, thr, n_pct, pct, w, W, prob, pout);
}

template <typename T>
void launch_products(int mi, const CatchDev<T>& C, double thr, int n_pct, const double* pct, const double* w,
                     double W, double* prob, double* pout, hipStream_t s) {
    switch (mi) {
        case 1: launch_products_mi<T, 1>(C, thr, n_pct, pct, w, W, prob, pout, s); break;
        case 2: launch_products_mi<T, 2>(C, thr, n_pct, pct, w, W, prob, pout, s); break;
        case 4: launch_products_mi<T, 4>(C, thr, n_pct, pct, w, W, prob, pout, s); break;
        default: launch_products_mi<T, 8>(C, thr, n_pct, pct, w, W, prob, pout, s); break;
    }
}

template void launch_products<float>(int, const CatchDev<float>&, double, int, const double*, const double*, double,
                                     double*, double*, hipStream_t);
template void launch_products<double>(int, const CatchDev<double>&, double, int, const double*, const double*, double,
                                      double*, double*, hipStream_t);

}  // namespace flood
