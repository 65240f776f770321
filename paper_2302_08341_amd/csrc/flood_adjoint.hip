// Discrete adjoint kernels of libflood.
//
// The forward step maps (h, q) at step n to (h, q) at step n+1 with the step
// length and every branch (wet/dry threshold, which surface is higher, donor
// limiter, clamp at zero) fixed by the recorded forward.  k_adj applies the
// transpose of that map for one recorded launch: given the adjoint of the state
// after the step it produces the adjoint of the state before it, and
// accumulates the adjoints of the shared Manning field (per cell) and of each
// member's rain multiplier.  It is written in gather form: every lane owns one
// (cell, member), recomputes the four links around its cell from the tape and
// collects their contributions, so nothing is scattered with atomics.
#include "flood_device.h"

namespace flood {

// Interior link with the partial derivatives of the new discharge with respect
// to the old discharge q, the two depths, and (cn) the Manning value of either
// adjacent cell: A = G s^2 dt hf^(-7/3) with G = g nf^2 and nf = (n1 + n2)/2,
// so dF/dn_i = -F|q|/D * g nf s^2 dt hf^(-7/3).  Gn = g nf.
template <typename T>
__device__ __forceinline__ void link_in_d(T q, T h1, T h2, T dz, T G, T Gn, const MemberStep<T>& ms, T hdry,
                                          T& dq, T& dh1, T& dh2, T& cn) {
    dq = dh1 = dh2 = cn = T(0);
    const T d = h1 - h2;
    const bool up1 = d >= dz;
    const T hf = up1 ? h1 - fmax(dz, T(0)) : h2 - fmax(-dz, T(0));
    if (!(hf > hdry)) return;
    const T p = pow_m73(hf);
    const T A = G * ms.s2dt * p;
    const T aq = fabs(q);
    const T D = T(1) + A * aq;
    const T num = q - ms.gdtdx * hf * (dz - d);
    const T invD = qdiv(T(1), D);
    const T F = qdiv(num, D);
    const T sg = q > T(0) ? T(1) : (q < T(0) ? T(-1) : T(0));
    if (F > T(0)) {
        const T cap = h1 * ms.capf;
        if (cap < F) {
            dh1 = ms.capf;
            return;
        }
    } else {
        const T cap = -h2 * ms.capf;
        if (F < cap) {
            dh2 = -ms.capf;
            return;
        }
    }
    const T slope = dz - d;                          // dx times the surface slope
    const T dDdhf = T(-7.0 / 3.0) * A * aq / hf;
    const T t_hf = -ms.gdtdx * slope - F * dDdhf;    // d(num - F D)/d(hf)
    dq = (T(1) - F * A * sg) * invD;
    dh1 = ((up1 ? t_hf : T(0)) + ms.gdtdx * hf) * invD;
    dh2 = ((up1 ? T(0) : t_hf) - ms.gdtdx * hf) * invD;
    cn = -F * aq * invD * Gn * ms.s2dt * p;
}

// Open edge link (outward discharge qo, inner depth h), partials with respect
// to qo, h and the inner cell's Manning value (A = g n^2 s^2 dt h^(-7/3),
// Gn = 2 g n).
template <typename T>
__device__ __forceinline__ void link_open_d(T qo, T h, T G, T Gn, T Se, const MemberStep<T>& ms, T hdry, T& dq,
                                            T& dh, T& cn) {
    dq = dh = cn = T(0);
    if (!(h > hdry)) return;
    const T p = pow_m73(h);
    const T A = G * ms.s2dt * p;
    const T aq = fabs(qo);
    const T D = T(1) + A * aq;
    const T invD = qdiv(T(1), D);
    const T F = qdiv(qo + ms.gdt * h * Se, D);
    const T cap = h * ms.capf;
    if (cap < F) {
        dh = ms.capf;
        if (cap < T(0)) dh = T(0);
        return;
    }
    if (F < T(0)) return;
    const T sg = qo > T(0) ? T(1) : (qo < T(0) ? T(-1) : T(0));
    const T dDdh = T(-7.0 / 3.0) * A * aq / h;
    dq = (T(1) - F * A * sg) * invD;
    dh = (ms.gdt * Se - F * dDdh) * invD;
    cn = -F * aq * invD * Gn * ms.s2dt * p;
}

template <typename T, int MI>
__global__ __launch_bounds__(kBlock) void k_adj(const AdjLaunch<T> A) {
    const CatchDev<T>& C = A.c;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tyi = b / C.tiles_x;
    const int txi = b - tyi * C.tiles_x;
    const int txl = C.tx_log2;
    const int lane = threadIdx.x % MI;
    const int p = threadIdx.x / MI;
    const int TY = (kBlock / MI) >> txl;
    const int nx = C.nx, ny = C.ny;
    const int cx = (txi << txl) + (p & ((1 << txl) - 1));
    const int cy = tyi * TY + (p >> txl);
    const bool in = cx < nx && cy < ny;
    const bool hasE = cx + 1 < nx, hasW = cx > 0, hasS = cy + 1 < ny, hasN = cy > 0;
    const T g = C.g;
    T dzE = 0, dzW = 0, dzS = 0, dzN = 0, GE = 0, GW = 0, GS = 0, GN = 0;
    T NE = 0, NW = 0, NS = 0, NN = 0;   // g nf for interior links, 2 g n for edge links
    size_t c0 = 0;
    if (in) {
        c0 = (size_t)cy * nx + cx;
        const T z0 = C.z[c0], n0 = C.n[c0];
        const T gb = g * (n0 * n0), nb = T(2) * g * n0;
        if (hasE) {
            const T z1 = C.z[c0 + 1], n1 = C.n[c0 + 1];
            const T nf = T(0.5) * (n0 + n1);
            dzE = z1 - z0;
            GE = g * (nf * nf);
            NE = g * nf;
        } else {
            GE = gb;
            NE = nb;
        }
        if (hasW) {
            const T z1 = C.z[c0 - 1], n1 = C.n[c0 - 1];
            const T nf = T(0.5) * (n1 + n0);
            dzW = z0 - z1;
            GW = g * (nf * nf);
            NW = g * nf;
        } else {
            GW = gb;
            NW = nb;
        }
        if (hasS) {
            const T z1 = C.z[c0 + nx], n1 = C.n[c0 + nx];
            const T nf = T(0.5) * (n0 + n1);
            dzS = z1 - z0;
            GS = g * (nf * nf);
            NS = g * nf;
        } else {
            GS = gb;
            NS = nb;
        }
        if (hasN) {
            const T z1 = C.z[c0 - nx], n1 = C.n[c0 - nx];
            const T nf = T(0.5) * (n1 + n0);
            dzN = z0 - z1;
            GN = g * (nf * nf);
            NN = g * nf;
        } else {
            GN = gb;
            NN = nb;
        }
    }
    const T hdry = C.hdry;
    const size_t plane = (size_t)ny * nx * MI;
    const size_t rowMI = (size_t)nx * MI;
    __shared__ T red[kBlock / 64][MI];
    T nacc = T(0);

    for (int k = 0; k < C.n_chunks; ++k) {
        const int ml = k * MI + lane;
        T lsum = T(0);
        bool act = false;
        if (in && ml < C.n_members) {
            const MemberStep<T> ms = A.ms[ml];
            act = ms.active != 0;
            const size_t idx = (size_t)k * plane + c0 * MI + lane;
            const size_t iw = ((size_t)k * ny + cy) * MI + lane;
            const size_t in_ = ((size_t)k * nx + cx) * MI + lane;
            if (!act) {
                A.lh[1][idx] = A.lh[0][idx];
                A.lqx[1][idx] = A.lqx[0][idx];
                A.lqy[1][idx] = A.lqy[0][idx];
                if (!hasW) A.lqw[1][iw] = A.lqw[0][iw];
                if (!hasN) A.lqn[1][in_] = A.lqn[0][in_];
            } else {
                const T* __restrict__ hs = C.h[0];
                const T h0 = hs[idx];
                const T hE = hasE ? hs[idx + MI] : T(0);
                const T hW = hasW ? hs[idx - MI] : T(0);
                const T hS = hasS ? hs[idx + rowMI] : T(0);
                const T hN = hasN ? hs[idx - rowMI] : T(0);
                const T qE = C.qx[0][idx];
                const T qS = C.qy[0][idx];
                const T qW = hasW ? C.qx[0][idx - MI] : C.qw[0][iw];
                const T qN = hasN ? C.qy[0][idx - rowMI] : C.qn[0][in_];
                // adjoint of the new depths after the clamp branch
                const T* __restrict__ lh = A.lh[0];
                const uint8_t* __restrict__ cl = A.clamp;
                const T le_c = cl[idx] ? T(0) : lh[idx];
                const T le_E = hasE ? (cl[idx + MI] ? T(0) : lh[idx + MI]) : T(0);
                const T le_W = hasW ? (cl[idx - MI] ? T(0) : lh[idx - MI]) : T(0);
                const T le_S = hasS ? (cl[idx + rowMI] ? T(0) : lh[idx + rowMI]) : T(0);
                const T le_N = hasN ? (cl[idx - rowMI] ? T(0) : lh[idx - rowMI]) : T(0);
                const T lqE = A.lqx[0][idx];
                const T lqS = A.lqy[0][idx];
                const T lqW = hasW ? A.lqx[0][idx - MI] : A.lqw[0][iw];
                const T lqN = hasN ? A.lqy[0][idx - rowMI] : A.lqn[0][in_];
                const T k_ = ms.dtdx;
                T nh = le_c, oqx = T(0), oqy = T(0), oqw = T(0), oqn = T(0);
                T dq, d1, d2, cn;
                // east link (this cell is cell 1)
                if (hasE) {
                    link_in_d(qE, h0, hE, dzE, GE, NE, ms, hdry, dq, d1, d2, cn);
                    const T lt = lqE + k_ * (le_E - le_c);
                    oqx = lt * dq;
                    nh += lt * d1;
                    nacc += lt * cn;
                } else if (C.edge_open[1]) {
                    link_open_d(qE, h0, GE, NE, C.edge_slope[1], ms, hdry, dq, d1, cn);
                    const T lt = lqE - k_ * le_c;
                    oqx = lt * dq;
                    nh += lt * d1;
                    nacc += lt * cn;
                }
                // south link (this cell is cell 1)
                if (hasS) {
                    link_in_d(qS, h0, hS, dzS, GS, NS, ms, hdry, dq, d1, d2, cn);
                    const T lt = lqS + k_ * (le_S - le_c);
                    oqy = lt * dq;
                    nh += lt * d1;
                    nacc += lt * cn;
                } else if (C.edge_open[2]) {
                    link_open_d(qS, h0, GS, NS, C.edge_slope[2], ms, hdry, dq, d1, cn);
                    const T lt = lqS - k_ * le_c;
                    oqy = lt * dq;
                    nh += lt * d1;
                    nacc += lt * cn;
                }
                // west link (this cell is cell 2); stored edge value is -qo(-q)
                if (hasW) {
                    link_in_d(qW, hW, h0, dzW, GW, NW, ms, hdry, dq, d1, d2, cn);
                    const T lt = lqW + k_ * (le_c - le_W);
                    nh += lt * d2;
                    nacc += lt * cn;
                } else if (C.edge_open[3]) {
                    link_open_d(-qW, h0, GW, NW, C.edge_slope[3], ms, hdry, dq, d1, cn);
                    const T lt = lqW + k_ * le_c;
                    oqw = lt * dq;
                    nh -= lt * d1;
                    nacc -= lt * cn;
                }
                // north link (this cell is cell 2)
                if (hasN) {
                    link_in_d(qN, hN, h0, dzN, GN, NN, ms, hdry, dq, d1, d2, cn);
                    const T lt = lqN + k_ * (le_c - le_N);
                    nh += lt * d2;
                    nacc += lt * cn;
                } else if (C.edge_open[0]) {
                    link_open_d(-qN, h0, GN, NN, C.edge_slope[0], ms, hdry, dq, d1, cn);
                    const T lt = lqN + k_ * le_c;
                    oqn = lt * dq;
                    nh -= lt * d1;
                    nacc -= lt * cn;
                }
                A.lh[1][idx] = nh;
                A.lqx[1][idx] = oqx;
                A.lqy[1][idx] = oqy;
                if (!hasW) A.lqw[1][iw] = oqw;
                if (!hasN) A.lqn[1][in_] = oqn;
                lsum = le_c;
            }
        }
        // rain-multiplier adjoint: sum over the workgroup's cells of the depth adjoint,
        // times R dt of the member's step
        T v = lsum;
#pragma unroll
        for (int off = MI; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) < MI) red[threadIdx.x >> 6][lane] = v;
        __syncthreads();
        if ((int)threadIdx.x < MI) {
            const int m2 = k * MI + (int)threadIdx.x;
            if (m2 < C.n_members) {
                T sum = T(0);
                for (int w = 0; w < kBlock / 64; ++w) sum += red[w][threadIdx.x];
                if (sum != T(0)) A.mubar_part[(size_t)b * C.n_members + m2] += (double)sum * A.rdt[m2];
            }
        }
        __syncthreads();
    }
    // the MI lanes of a cell hold different members' contributions to the same
    // Manning-field entry: combine them before the single read-modify-write
    double nsum = (double)nacc;
#pragma unroll
    for (int off = 1; off < MI; off <<= 1) nsum += __shfl_xor(nsum, off, 64);
    if (in && lane == 0 && nsum != 0.0) A.nbar[c0] += nsum;
}

template <typename T> void launch_adjoint_step(int mi, const AdjLaunch<T>& A, hipStream_t s) {
    const int blocks = A.c.tiles_x * A.c.tiles_y;
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_adj<T, 1>), dim3(blocks), dim3(kBlock), 0, s, A); break;
        case 2: hipLaunchKernelGGL((k_adj<T, 2>), dim3(blocks), dim3(kBlock), 0, s, A); break;
        case 4: hipLaunchKernelGGL((k_adj<T, 4>), dim3(blocks), dim3(kBlock), 0, s, A); break;
        default: hipLaunchKernelGGL((k_adj<T, 8>), dim3(blocks), dim3(kBlock), 0, s, A); break;
    }
}

// Gauge misfit seeds the adjoint: d/dh of (h - d)^2 at every gauge of every
// member whose step just completed a sample.  One lane per member.
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_inject(const CatchDev<T> after, const int32_t* tags, int K,
                                                const int32_t* grc, const double* obs, T* lh) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= after.n_members) return;
    const int s = tags[m];
    if (s < 0) return;
    for (int k = 0; k < K; ++k) {
        const size_t i = state_index<T, MI>(after, m, grc[2 * k], grc[2 * k + 1]);
        lh[i] += (T)(2.0 * ((double)after.h[0][i] - obs[(size_t)s * K + k]));
    }
}

template <typename T>
void launch_inject(int mi, const CatchDev<T>& after, const int32_t* tags, int K, const int32_t* grc, const double* obs,
                   T* lh, hipStream_t s) {
    if (K == 0) return;
    dim3 grid((after.n_members + 255) / 256);
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_inject<T, 1>), grid, dim3(256), 0, s, after, tags, K, grc, obs, lh); break;
        case 2: hipLaunchKernelGGL((k_inject<T, 2>), grid, dim3(256), 0, s, after, tags, K, grc, obs, lh); break;
        case 4: hipLaunchKernelGGL((k_inject<T, 4>), grid, dim3(256), 0, s, after, tags, K, grc, obs, lh); break;
        default: hipLaunchKernelGGL((k_inject<T, 8>), grid, dim3(256), 0, s, after, tags, K, grc, obs, lh); break;
    }
}

// Checkpoint: copy every member's current state (copy par[m]) into copy 0 of dst.
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_snapshot(const CatchDev<T> C, const int32_t* par, const CatchDev<T> D) {
    const int k = blockIdx.y;
    const size_t ncell = (size_t)C.ny * C.nx;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ncell * MI) return;
    const int lane = (int)(e % MI);
    const int m = k * MI + lane;
    if (m >= C.n_members) return;
    const int p = par[C.member_off + m];
    const size_t cell = e / MI;
    const size_t i = (size_t)k * ncell * MI + cell * MI + lane;
    D.h[0][i] = C.h[p][i];
    D.qx[0][i] = C.qx[p][i];
    D.qy[0][i] = C.qy[p][i];
    const int r = (int)(cell / C.nx), c = (int)(cell % C.nx);
    if (c == 0) D.qw[0][((size_t)k * C.ny + r) * MI + lane] = C.qw[p][((size_t)k * C.ny + r) * MI + lane];
    if (r == 0) D.qn[0][((size_t)k * C.nx + c) * MI + lane] = C.qn[p][((size_t)k * C.nx + c) * MI + lane];
}

template <typename T>
void launch_snapshot(int mi, const CatchDev<T>& C, const int32_t* par, const CatchDev<T>& dst, hipStream_t s) {
    const size_t ncell = (size_t)C.ny * C.nx;
    dim3 grid((unsigned)((ncell * mi + 255) / 256), C.n_chunks);
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_snapshot<T, 1>), grid, dim3(256), 0, s, C, par, dst); break;
        case 2: hipLaunchKernelGGL((k_snapshot<T, 2>), grid, dim3(256), 0, s, C, par, dst); break;
        case 4: hipLaunchKernelGGL((k_snapshot<T, 4>), grid, dim3(256), 0, s, C, par, dst); break;
        default: hipLaunchKernelGGL((k_snapshot<T, 8>), grid, dim3(256), 0, s, C, par, dst); break;
    }
}

// Gauge misfit of the current state, summed over members and gauges into *loss.
template <typename T, int MI>
__global__ __launch_bounds__(256) void k_misfit(const CatchDev<T> C, const int32_t* par, int K, const int32_t* grc,
                                                const double* obs, double* loss) {
    double acc = 0.0;
    for (int e = threadIdx.x; e < C.n_members * K; e += 256) {
        const int m = e / K, k = e % K;
        const T* h = C.h[par[C.member_off + m]];
        const double d = (double)h[state_index<T, MI>(C, m, grc[2 * k], grc[2 * k + 1])] - obs[k];
        acc += d * d;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *loss += (part[0] + part[1]) + (part[2] + part[3]);
}

template <typename T>
void launch_misfit(int mi, const CatchDev<T>& C, const int32_t* par, int K, const int32_t* grc, const double* obs,
                   double* loss, hipStream_t s) {
    if (K == 0) return;
    switch (mi) {
        case 1: hipLaunchKernelGGL((k_misfit<T, 1>), dim3(1), dim3(256), 0, s, C, par, K, grc, obs, loss); break;
        case 2: hipLaunchKernelGGL((k_misfit<T, 2>), dim3(1), dim3(256), 0, s, C, par, K, grc, obs, loss); break;
        case 4: hipLaunchKernelGGL((k_misfit<T, 4>), dim3(1), dim3(256), 0, s, C, par, K, grc, obs, loss); break;
        default: hipLaunchKernelGGL((k_misfit<T, 8>), dim3(1), dim3(256), 0, s, C, par, K, grc, obs, loss); break;
    }
}

// out[m] = sum over workgroups of parts[b][m]
__global__ __launch_bounds__(256) void k_sum_parts(int n_blocks, int n_members, const double* parts, double* out) {
    const int m = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += 256) acc += parts[(size_t)b * n_members + m];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[m] = (part[0] + part[1]) + (part[2] + part[3]);
}

void launch_sum_parts(int n_blocks, int n_members, const double* parts, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_parts, dim3(n_members), dim3(256), 0, s, n_blocks, n_members, parts, out);
}

template void launch_adjoint_step<float>(int, const AdjLaunch<float>&, hipStream_t);
template void launch_adjoint_step<double>(int, const AdjLaunch<double>&, hipStream_t);
template void launch_inject<float>(int, const CatchDev<float>&, const int32_t*, int, const int32_t*, const double*,
                                   float*, hipStream_t);
template void launch_inject<double>(int, const CatchDev<double>&, const int32_t*, int, const int32_t*, const double*,
                                    double*, hipStream_t);
template void launch_snapshot<float>(int, const CatchDev<float>&, const int32_t*, const CatchDev<float>&, hipStream_t);
template void launch_snapshot<double>(int, const CatchDev<double>&, const int32_t*, const CatchDev<double>&,
                                      hipStream_t);
template void launch_misfit<float>(int, const CatchDev<float>&, const int32_t*, int, const int32_t*, const double*,
                                   double*, hipStream_t);
template void launch_misfit<double>(int, const CatchDev<double>&, const int32_t*, int, const int32_t*, const double*,
                                    double*, hipStream_t);

}  // namespace flood
