// Attainable bandwidth of the row-marching step's access pattern on this device
// (flood_probe_stream): the step kernel's streams with its arithmetic taken out.
//
// One wavefront per (strip of 64 x 4 cells, member) marches down `rows` rows of
// a members-in-planes ensemble exactly as the vectorised step does: per row it
// reads the member's three state arrays and the shared bed and roughness with
// 16-byte loads (state non-temporal), and writes three state arrays with 16-byte
// non-temporal stores; wavefronts are numbered strips along x fastest, then
// members, then rows of strips (so the members of a row of strips share its bed
// and roughness in L2), and spread over the XCDs in contiguous ranges.  There
// are no halo cells, no prologue row and no link arithmetic: the written values
// depend on every loaded value, so no load can be dropped.  What it reaches is
// the ceiling for the step's 24 bytes per member-cell update with this pattern.
// Its 32 registers let 8 wavefronts share a SIMD; waves_per_simd > 0 caps that
// with LDS that every workgroup reserves (160 KiB per CU), so the pattern can
// also be measured at the step kernel's own occupancy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/flood.h"
#include "flood_device.h"
#include "flood_internal.h"

namespace flood {

__global__ __launch_bounds__(256) void k_stream_probe(int ny, int nx, int n_members, int rows, int strips_x,
                                                      int strips_y, const float* __restrict__ h,
                                                      const float* __restrict__ qx, const float* __restrict__ qy,
                                                      const float* __restrict__ z, const float* __restrict__ n,
                                                      float* __restrict__ ho, float* __restrict__ qxo,
                                                      float* __restrict__ qyo) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int w = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    const int sx = w % strips_x;
    const int rest = w / strips_x;
    const int k = rest % n_members;
    const int sy = rest / n_members;
    if (sy >= strips_y) return;
    const int xl = sx * 256 + 4 * lane;
    if (xl >= nx) return;
    const int r0 = sy * rows, r1 = min(r0 + rows, ny);
    const size_t plane = (size_t)ny * nx;
    const size_t base = (size_t)k * plane;
    for (int r = r0; r < r1; ++r) {
        const size_t c = (size_t)r * nx + xl;
        float a[4], b[4], d[4], e[4], f[4];
        vload_nt<float, 4>(h + base + c, a);
        vload_nt<float, 4>(qx + base + c, b);
        vload_nt<float, 4>(qy + base + c, d);
        vload<float, 4>(z + c, e);
        vload<float, 4>(n + c, f);
        float o1[4], o2[4], o3[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float s = e[j] * f[j] * 1e-30f;
            o1[j] = a[j] + s;
            o2[j] = b[j] - s;
            o3[j] = d[j] + s;
        }
        vstore_nt<float, 4>(ho + base + c, o1);
        vstore_nt<float, 4>(qxo + base + c, o2);
        vstore_nt<float, 4>(qyo + base + c, o3);
    }
}

flood_status probe_stream_impl(int ny, int nx, int n_members, int rows, int reps, int waves_per_simd, hipStream_t st,
                               double* gbps, double* ms_per_launch, std::string& err) {
    const size_t plane = (size_t)ny * nx;
    const size_t state = plane * n_members;
    std::vector<void*> bufs;
    auto release = [&]() {
        (void)hipStreamSynchronize(st);
        for (void* p : bufs) (void)hipFree(p);
    };
    auto alloc = [&](size_t elems) -> float* {
        void* p = nullptr;
        if (hipMalloc(&p, elems * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        bufs.push_back(p);
        return static_cast<float*>(p);
    };
    float* a[8];
    for (int i = 0; i < 6; ++i) a[i] = alloc(state);
    a[6] = alloc(plane);
    a[7] = alloc(plane);
    for (int i = 0; i < 8; ++i)
        if (!a[i]) {
            release();
            err = "hipMalloc failed for the probe's buffers";
            return FLOOD_ENOMEM;
        }
    for (int i = 0; i < 8; ++i)
        if (hipMemsetAsync(a[i], 0, (i < 6 ? state : plane) * sizeof(float), st) != hipSuccess) {
            release();
            err = "hipMemsetAsync failed";
            return FLOOD_EHIP;
        }
    const int strips_x = (nx + 255) / 256, strips_y = (ny + rows - 1) / rows;
    const long long waves = (long long)strips_x * strips_y * n_members;
    const dim3 grid((unsigned)((waves + 3) / 4));
    // a workgroup is four wavefronts, one per SIMD: k workgroups per CU are k waves per SIMD
    const size_t lds = waves_per_simd > 0 ? (size_t)(160 * 1024 / waves_per_simd - 256) / 256 * 256 : 0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        release();
        err = "hipEventCreate failed";
        return FLOOD_EHIP;
    }
    flood_status rc = FLOOD_OK;
    float best = 1e30f;
    for (int rep = 0; rep <= reps && rc == FLOOD_OK; ++rep) {   // rep 0 warms up
        const int s = rep & 1;                                   // ping-pong like the step's two copies
        (void)hipEventRecord(e0, st);
        hipLaunchKernelGGL(k_stream_probe, grid, dim3(256), lds, st, ny, nx, n_members, rows, strips_x, strips_y,
                           a[3 * s], a[3 * s + 1], a[3 * s + 2], a[6], a[7], a[3 * (1 - s)], a[3 * (1 - s) + 1],
                           a[3 * (1 - s) + 2]);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = FLOOD_EHIP;
            err = "probe launch failed";
            break;
        }
        float el = 0.0f;
        (void)hipEventElapsedTime(&el, e0, e1);
        if (rep) best = std::min(best, el);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release();
    if (rc) return rc;
    *ms_per_launch = best;
    *gbps = 24.0 * (double)state / (best * 1e-3) / 1e9;
    return FLOOD_OK;
}

}  // namespace flood

extern "C" flood_status flood_probe_stream(int32_t ny, int32_t nx, int32_t n_members, int32_t rows, int32_t reps,
                                           int32_t waves_per_simd, void* hip_stream, double* gbps_out,
                                           double* ms_per_launch_out) {
    if (ny < 1 || nx < 4 || nx % 4 || n_members < 1 || rows < 1 || rows > 4096 || reps < 1 || reps > 1000 ||
        (waves_per_simd != 0 && (waves_per_simd < 3 || waves_per_simd > 8)) || !gbps_out || !ms_per_launch_out)
        return FLOOD_EINVAL;
    if ((long long)ny * nx * n_members > (1LL << 31)) return FLOOD_EINVAL;   // 8 GiB per state array
    std::string err;
    return flood::probe_stream_impl(ny, nx, n_members, rows, reps, waves_per_simd, (hipStream_t)hip_stream,
                                    gbps_out, ms_per_launch_out, err);
}
