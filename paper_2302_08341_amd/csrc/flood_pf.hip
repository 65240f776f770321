// Particle filter kernels of libflood (Sec. 2.2 Eqs. 9-12, Sec. 3.3 steps II-V).
//
// One workgroup holds the whole ensemble of a catchment (N <= 1024 members, one
// lane each).  Weights are computed in FP64 in log space: the maximum is
// subtracted before exponentiation (log-sum-exp), so likelihoods far in the
// tail stay finite.  The cumulative weight used by systematic resampling is
// summed by one lane in member order, so the ancestors depend only on the
// weights and the offset, not on the reduction tree.
#include <cmath>
#include <mutex>

#include "../../include/flood.h"
#include "flood_internal.h"

namespace flood {

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Workgroup-wide reductions through one LDS slot per wavefront (fixed tree).
__device__ double block_max(double v, double* red) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int i = 1; i < nw; ++i) r = fmax(r, red[i]);
    return r;
}
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int i = 1; i < nw; ++i) r += red[i];
    return r;
}

// Systematic resampling over weights sw[0..N): lane j takes the first particle
// whose running weight exceeds its position ((u0 + j)/N) * total.
__device__ int systematic_lane(int N, const double* sw, double* C, double u0) {
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int i = 0; i < N; ++i) {
            run += sw[i];
            C[i] = run;
        }
    }
    __syncthreads();
    const int j = threadIdx.x;
    if (j >= N) return -1;
    const double tj = ((u0 + (double)j) / (double)N) * C[N - 1];
    int lo = 0, hi = N;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tj < C[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo < N ? lo : N - 1;
}

__global__ __launch_bounds__(1024) void k_pf(const PfArgs a) {
    __shared__ double red[16];
    __shared__ double sw[kMaxMembers];
    __shared__ double C[kMaxMembers];
    const int N = a.N, K = a.K;
    const int m = threadIdx.x;
    // Eq. 9 (diagonal covariance, constant dropped) plus the prior log-weight (Eq. 10)
    double av = -INFINITY;
    if (m < N) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
            // relative observation error with a floor (Sec. 4.4), or absolute
            double sg = a.sigma[k];
            if (a.alpha > 0.0) {
                const double rel = a.alpha * fabs(a.d[k]);
                sg = rel > sg ? rel : sg;
            }
            const double e = (a.y[(size_t)m * K + k] - a.d[k]) / sg;
            acc += e * e;
        }
        av = a.logw[m] + -0.5 * acc;
    }
    const double M = block_max(av, red);
    const double e = (m < N) ? exp(av - M) : 0.0;
    const double Z = block_sum(e, red);
    const double w = e / Z;                     // Eq. 11
    const double s2 = block_sum(w * w, red);
    const double neff = 1.0 / s2;               // Eq. 12
    const bool res = neff < a.neff_frac * (double)N;
    if (m == 0) {
        a.neff[0] = neff;
        a.flag[0] = res ? 1 : 0;
    }
    if (!res) {
        if (m < N) {
            a.logw[m] = av - M - log(Z);
            a.anc[m] = m;
            a.src_par[m] = a.par[m];
            a.dst_par[m] = a.par[m];
        }
        return;
    }
    if (m < N) sw[m] = w;
    const int anc = systematic_lane(N, sw, C, a.u0);
    // replacement (step V): slot m takes its ancestor's scalars; the state arrays
    // are copied by k_permute into the slot's other state copy
    double t = 0, s = 0, mu = 0, vr = 0, vo = 0, vc = 0, vd = 0, dr = 0, vi = 0;
    double cn[kMaxClasses] = {0.0, 0.0, 0.0, 0.0};
    int64_t st = 0;
    int sp = 0, mypar = 0;
    if (m < N) {
        if (a.clsn)
            for (int k = 0; k < kMaxClasses; ++k) cn[k] = a.clsn[(size_t)anc * kMaxClasses + k];
        if (a.drain) dr = a.drain[anc];
        vd = a.vdrain[anc];
        vi = a.vin[anc];
        t = a.t[anc];
        s = a.s[anc];
        mu = a.mu[anc];
        vr = a.vrain[anc];
        vo = a.vout[anc];
        vc = a.vclamp[anc];
        st = a.steps[anc];
        sp = a.par[anc];
        mypar = a.par[m];
    }
    __syncthreads();
    if (m < N) {
        a.anc[m] = anc;
        a.t[m] = t;
        a.s[m] = s;
        a.mu[m] = a.beta ? mu * a.beta[m] : mu;
        a.vrain[m] = vr;
        a.vout[m] = vo;
        a.vclamp[m] = vc;
        if (a.clsn)
            for (int k = 0; k < kMaxClasses; ++k) a.clsn[(size_t)m * kMaxClasses + k] = cn[k];
        if (a.drain) a.drain[m] = dr;
        a.vdrain[m] = vd;
        a.vin[m] = vi;
        a.steps[m] = st;
        a.logw[m] = -log((double)N);
        a.src_par[m] = sp;
        const int dp = (anc == m) ? mypar : (mypar ^ 1);
        a.dst_par[m] = dp;
        a.par[m] = dp;
    }
}

void launch_pf(const PfArgs& a, hipStream_t s) {
    const int threads = ((a.N + 63) / 64) * 64;
    hipLaunchKernelGGL(k_pf, dim3(1), dim3(threads), 0, s, a);
}

__global__ __launch_bounds__(1024) void k_systematic(int n, const double* w, double u0, int32_t* anc) {
    __shared__ double sw[kMaxMembers];
    __shared__ double C[kMaxMembers];
    if ((int)threadIdx.x < n) sw[threadIdx.x] = w[threadIdx.x];
    const int a = systematic_lane(n, sw, C, u0);
    if ((int)threadIdx.x < n) anc[threadIdx.x] = a;
}

void launch_systematic(int n, const double* w, double u0, int32_t* anc, hipStream_t s) {
    const int threads = ((n + 63) / 64) * 64;
    hipLaunchKernelGGL(k_systematic, dim3(1), dim3(threads), 0, s, n, w, u0, anc);
}

// Device staging of flood_systematic_resample_noalloc: the weights (kMaxMembers
// doubles) followed by the ancestors (kMaxMembers int32) of one call, 12 KiB,
// one copy on each GPU the library runs on, held until the process ends.  Every
// call on a GPU reuses it, so calls that overlap on one GPU race.  Host code
// never passes this name to a kernel or a copy: it takes the array's device
// address once per device (hipGetSymbolAddress) and uses that.
static __device__ __align__(256) unsigned char scratch[kMaxMembers * (sizeof(double) + sizeof(int32_t))];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

flood_status systematic_resample_noalloc_impl(const double* w, int n, double u0, int32_t* anc, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return FLOOD_EHIP;
    }
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
                (void)hipGetLastError();
                return FLOOD_EHIP;
            }
            g_scratch_ptr[dev] = p;
        }
        base = g_scratch_ptr[dev];
    }
    double* dw = static_cast<double*>(base);
    int32_t* da = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(base) + kMaxMembers * sizeof(double));
    if (hipMemcpyAsync(dw, w, n * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess) {
        (void)hipGetLastError();
        return FLOOD_EHIP;
    }
    launch_systematic(n, dw, u0, da, s);
    if (hipGetLastError() != hipSuccess) return FLOOD_EHIP;
    if (hipMemcpyAsync(anc, da, n * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        return FLOOD_EHIP;
    }
    return FLOOD_OK;
}

// Copy every resampled slot's state from its ancestor (copy src_par) into the
// slot's other state copy (dst_par).  Slots that keep their own particle are
// not touched.  Lane = (cell, member-in-chunk), blockIdx.y = chunk.
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_permute(const CatchDev<T> C, const int32_t* anc, const int32_t* src_par,
                                                 const int32_t* dst_par, const int32_t* flag) {
    if (flag[0] == 0) return;
    const int k = blockIdx.y;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t ncell = (size_t)C.ny * C.nx;
    if (e >= ncell * MI) return;
    const int lane = (int)(e % MI);
    const size_t cell = e / MI;
    const int j = k * MI + lane;
    if (j >= C.n_members) return;
    const int a = anc[j];
    if (a == j) return;
    const int sp = src_par[j], dp = dst_par[j];
    const size_t plane = ncell * MI;
    const size_t di = (size_t)k * plane + cell * MI + lane;
    const size_t si = (size_t)(a / MI) * plane + cell * MI + (a % MI);
    C.h[dp][di] = C.h[sp][si];
    C.qx[dp][di] = C.qx[sp][si];
    C.qy[dp][di] = C.qy[sp][si];
    const int r = (int)(cell / C.nx), c = (int)(cell % C.nx);
    if (c == 0) C.qw[dp][((size_t)k * C.ny + r) * MI + lane] = C.qw[sp][((size_t)(a / MI) * C.ny + r) * MI + a % MI];
    if (r == 0) C.qn[dp][((size_t)k * C.nx + c) * MI + lane] = C.qn[sp][((size_t)(a / MI) * C.nx + c) * MI + a % MI];
}

template <typename T>
void launch_permute(int mi, const CatchDev<T>& C, const int32_t* anc, const int32_t* src_par,
                    const int32_t* dst_par, const int32_t* flag, hipStream_t s) {
    const size_t ncell = (size_t)C.ny * C.nx;
    dim3 grid((unsigned)((ncell * mi + 255) / 256), C.n_chunks);
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_permute<T, 1>), grid, dim3(256), 0, s, C, anc, src_par, dst_par, flag); break;
        case 2: hipLaunchKernelGGL((k_permute<T, 2>), grid, dim3(256), 0, s, C, anc, src_par, dst_par, flag); break;
        case 4: hipLaunchKernelGGL((k_permute<T, 4>), grid, dim3(256), 0, s, C, anc, src_par, dst_par, flag); break;
        default: hipLaunchKernelGGL((k_permute<T, 8>), grid, dim3(256), 0, s, C, anc, src_par, dst_par, flag); break;
    }
}

template void launch_permute<float>(int, const CatchDev<float>&, const int32_t*, const int32_t*, const int32_t*,
                                    const int32_t*, hipStream_t);
template void launch_permute<double>(int, const CatchDev<double>&, const int32_t*, const int32_t*, const int32_t*,
                                     const int32_t*, hipStream_t);


// Running maxima follow their members on resampling.  There is one copy of
// the array, so the slots that change are gathered into tmp first (reading only
// the old maxima) and committed in a second pass.
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_peak_gather(const CatchDev<T> C, const int32_t* anc, const int32_t* flag,
                                                     T* tmp) {
    if (flag[0] == 0) return;
    const int k = blockIdx.y;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t ncell = (size_t)C.ny * C.nx;
    if (e >= ncell * MI) return;
    const int lane = (int)(e % MI);
    const size_t cell = e / MI;
    const int j = k * MI + lane;
    if (j >= C.n_members) return;
    const int a = anc[j];
    if (a == j) return;
    const size_t plane = ncell * MI;
    tmp[(size_t)k * plane + cell * MI + lane] = C.peak[(size_t)(a / MI) * plane + cell * MI + (a % MI)];
}

template <typename T, int MI>
__global__ __launch_bounds__(256) void k_peak_commit(const CatchDev<T> C, const int32_t* anc, const int32_t* flag,
                                                     const T* tmp) {
    if (flag[0] == 0) return;
    const int k = blockIdx.y;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t ncell = (size_t)C.ny * C.nx;
    if (e >= ncell * MI) return;
    const int lane = (int)(e % MI);
    const int j = k * MI + lane;
    if (j >= C.n_members || anc[j] == j) return;
    const size_t i = (size_t)k * ncell * MI + (e / MI) * MI + lane;
    C.peak[i] = tmp[i];
}

template <typename T>
void launch_permute_peak(int mi, const CatchDev<T>& C, const int32_t* anc, const int32_t* flag, T* tmp,
                         hipStream_t s) {
    const size_t ncell = (size_t)C.ny * C.nx;
    dim3 grid((unsigned)((ncell * mi + 255) / 256), C.n_chunks);
    switch (mi) {
        case 1:
            hipLaunchKernelGGL((k_peak_gather<T, 1>), grid, dim3(256), 0, s, C, anc, flag, tmp);
            hipLaunchKernelGGL((k_peak_commit<T, 1>), grid, dim3(256), 0, s, C, anc, flag, tmp);
            break;
        case 2:
            hipLaunchKernelGGL((k_peak_gather<T, 2>), grid, dim3(256), 0, s, C, anc, flag, tmp);
            hipLaunchKernelGGL((k_peak_commit<T, 2>), grid, dim3(256), 0, s, C, anc, flag, tmp);
            break;
        case 4:
            hipLaunchKernelGGL((k_peak_gather<T, 4>), grid, dim3(256), 0, s, C, anc, flag, tmp);
            hipLaunchKernelGGL((k_peak_commit<T, 4>), grid, dim3(256), 0, s, C, anc, flag, tmp);
            break;
        default:
            hipLaunchKernelGGL((k_peak_gather<T, 8>), grid, dim3(256), 0, s, C, anc, flag, tmp);
            hipLaunchKernelGGL((k_peak_commit<T, 8>), grid, dim3(256), 0, s, C, anc, flag, tmp);
            break;
    }
}

template void launch_permute_peak<float>(int, const CatchDev<float>&, const int32_t*, const int32_t*, float*,
                                         hipStream_t);
template void launch_permute_peak<double>(int, const CatchDev<double>&, const int32_t*, const int32_t*, double*,
                                          hipStream_t);

}  // namespace flood
