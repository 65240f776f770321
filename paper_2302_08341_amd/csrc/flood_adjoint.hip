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
#include <algorithm>

#include "flood_device.h"

namespace flood {

// Interior link with the partial derivatives of the new discharge with respect
// to the old discharge q, the two depths, and (cn) the Manning value of either
// adjacent cell: A = G s^2 dt hf^(-7/3) with G = g nf^2 and nf = (n1 + n2)/2,
// so dF/dn_i = -F|q|/D * g nf s^2 dt hf^(-7/3).  Gn = g nf.
template <typename T>
__device__ __forceinline__ void link_in_d(T q, T h1, T h2, T dz, T G, T Gn, const MemberStep<T>& ms, T hdry,
                                          T& dq, T& dh1, T& dh2, T& cn) {
    // evaluated without branches and selected at the end, as in the forward:
    // dry, limited and free links in one wavefront do not split it, and a dry
    // link's intermediate values (possibly inf or NaN) are discarded
    const T d = h1 - h2;
    const bool up1 = d >= dz;
    const T hf = link_depth(h1, h2, dz);
    const bool wet = hf > hdry;
    const T p = pow_m73(hf);
    const T A = G * ms.s2dt * p;
    const T aq = fabs(q);
    const T D = T(1) + A * aq;
    const T num = q - ms.gdtdx * hf * (dz - d);
    const T invD = qdiv(T(1), D);
    const T F = qdiv(num, D);
    const T sg = q > T(0) ? T(1) : (q < T(0) ? T(-1) : T(0));
    // donor limiter: a limited link depends on its upwind depth only
    const bool pos = F > T(0);
    const bool cap1 = pos && (h1 * ms.capf < F);
    const bool cap2 = !pos && (F < -h2 * ms.capf);
    const bool free_ = wet && !cap1 && !cap2;
    const T slope = dz - d;                          // dx times the surface slope
    const T dDdhf = T(-7.0 / 3.0) * A * aq * qdiv(T(1), hf);
    const T t_hf = -ms.gdtdx * slope - F * dDdhf;    // d(num - F D)/d(hf)
    const T dq_ = (T(1) - F * A * sg) * invD;
    const T dh1_ = ((up1 ? t_hf : T(0)) + ms.gdtdx * hf) * invD;
    const T dh2_ = ((up1 ? T(0) : t_hf) - ms.gdtdx * hf) * invD;
    const T cn_ = -F * aq * invD * Gn * ms.s2dt * p;
    dq = free_ ? dq_ : T(0);
    cn = free_ ? cn_ : T(0);
    dh1 = !wet ? T(0) : (cap1 ? ms.capf : (cap2 ? T(0) : dh1_));
    dh2 = !wet ? T(0) : (cap2 ? -ms.capf : (cap1 ? T(0) : dh2_));
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

// Reverse step in row-march form.  Geometry as the forward row march: a
// wavefront marches a strip of 62 V cells down its rows for one member; lanes
// 0 and 63 are halo lanes.  A workgroup holds the four members of a member
// quad on the same strip (wavefront w: member 4u + w), so their contributions
// to the shared Manning-field adjoint are added in LDS, member by member in
// that order, and the quad's accumulator in HBM is read and written once per
// cell and step: 2 B per member-cell update instead of 8 with one accumulator
// per member.  Per row each lane evaluates the derivatives of the east and
// south links of its V cells once; the west link of its first cell comes from
// the neighbouring lane and the north link from the previous row, so every
// link is differentiated once per step.  Contributions to a cell's depth
// adjoint are added in the order east, south, west, north (as in k_adj).  The
// clamp branch comes from the tape: where the step before this one clamped the
// depth (-0 in the tape), the depth adjoint written here is zero, so the reverse
// of that step reads the adjoint of its new depths already masked.  The
// rain-multiplier adjoint is accumulated per (strip, member).  Members that do
// not step in this launch (or pad the last quad) skip the march and keep their
// adjoint in place, but still meet the workgroup barrier.  PF = 1 issues the
// next row's loads before the current row's derivatives (one row of lookahead).
template <typename T, int V, int PF>
__global__ __launch_bounds__(kBlock) void k_adjv(const AdjvLaunch<T> A) {
    extern __shared__ unsigned char adj_lds[];
    const CatchDev<T>& C = A.c;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int nq = (C.n_members + 3) / 4;
    int u, sx, sy;
    if (!march_wave(C, b, nq, u, sx, sy, C.strips_xa)) return;   // uniform over the workgroup
    const int k = 4 * u + wave;
    bool actq[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) actq[w] = 4 * u + w < C.n_members && A.i < A.n[4 * u + w];
    const bool act = actq[wave];
    const int nx = C.nx, ny = C.ny;
    const int rows = C.march_rows;
    // this wavefront's Manning contributions, [row][lane][V]
    T* NL = reinterpret_cast<T*>(adj_lds) + (size_t)wave * rows * 64 * V;
    const int xl = sx * (62 * V) - V + V * lane;
    const bool inx = xl >= 0 && xl < nx;
    const bool own = lane >= 1 && lane <= 62 && inx;
    const bool westw = sx == 0;                        // wavefront-uniform edge tests
    const bool eastw = sx == C.strips_xa - 1;
    const int xa = min(max(xl, 0), nx - V);            // load column (lanes outside the grid read, never use)
    const int r0 = sy * C.march_rows;
    const int r1 = min(r0 + C.march_rows, ny);
    const size_t plane = (size_t)ny * nx;
    if (act) {
        // the member's step j = n[k] - 1 - i, its record, and the sample (if any)
        // completed by its step before (whose seed goes into the depth adjoint written here)
        const int jst = A.n[k] - 1 - A.i;
        const size_t rr = (size_t)jst * A.stride + k;
        const MemberStep<T> ms = A.rec[rr];
        const double rdt = A.rec_rdt[rr];
        const int tag_prev = (jst >= 1 && A.n_gauges > 0) ? A.rec_tag[rr - A.stride] : -1;
        const size_t bs = (size_t)ms.blk;
        const T* __restrict__ H = C.h[0] + bs * plane;
        const T* __restrict__ QX = C.qx[0] + bs * plane;
        const T* __restrict__ QY = C.qy[0] + bs * plane;
        const T* __restrict__ QWs = C.qw[0] + bs * ny;
        const T* __restrict__ QNs = C.qn[0] + bs * nx;
        const int lp = A.lbase[k] ^ (A.i & 1);
        const T* __restrict__ LH = A.lh[lp] + (size_t)k * plane;
        const T* __restrict__ LQX = A.lqx[lp] + (size_t)k * plane;
        const T* __restrict__ LQY = A.lqy[lp] + (size_t)k * plane;
        const T* __restrict__ LQWs = A.lqw[lp] + (size_t)k * ny;
        const T* __restrict__ LQNs = A.lqn[lp] + (size_t)k * nx;
        T* __restrict__ LHo = A.lh[lp ^ 1] + (size_t)k * plane;
        T* __restrict__ LQXo = A.lqx[lp ^ 1] + (size_t)k * plane;
        T* __restrict__ LQYo = A.lqy[lp ^ 1] + (size_t)k * plane;
        T* __restrict__ LQWo = A.lqw[lp ^ 1] + (size_t)k * ny;
        T* __restrict__ LQNo = A.lqn[lp ^ 1] + (size_t)k * nx;
        const T* __restrict__ Z = C.z;
        const T* __restrict__ Nn = C.n;
        const T g = C.g, hdry = C.hdry, kk = ms.dtdx;

        size_t ca = (size_t)r0 * nx + xa;
        T hc[V], zc[V], nc[V], lec[V], pNh[V], pNn[V];
        vload<T, V>(H + ca, hc);
        vload<T, V>(Z + ca, zc);
        vload<T, V>(Nn + ca, nc);
        vload<T, V>(LH + ca, lec);
        if (r0 > 0) {
            // the south links of the row above the strip feed its first row's north links
            T hN[V], zN[V], nN[V], qN[V], lqN[V], leN[V];
            vload<T, V>(H + ca - nx, hN);
            vload<T, V>(Z + ca - nx, zN);
            vload<T, V>(Nn + ca - nx, nN);
            vload<T, V>(QY + ca - nx, qN);
            vload<T, V>(LQY + ca - nx, lqN);
            vload<T, V>(LH + ca - nx, leN);
    #pragma unroll
            for (int j = 0; j < V; ++j) {
                const T nf = T(0.5) * (nN[j] + nc[j]);
                T dq, d1, d2, cn;
                link_in_d(qN[j], hN[j], hc[j], zc[j] - zN[j], g * (nf * nf), g * nf, ms, hdry, dq, d1, d2, cn);
                const T lt = lqN[j] + kk * (lec[j] - leN[j]);
                pNh[j] = lt * d2;
                pNn[j] = lt * cn;
            }
        } else {
    #pragma unroll
            for (int j = 0; j < V; ++j) pNh[j] = pNn[j] = T(0);
        }
        double lsum = 0.0;
        // a row's links (qE, qS and their adjoints) and the row below it (hs, zs, ns, les)
        auto load_row = [&](size_t c, bool below, T (&qe)[V], T (&qs)[V], T (&lqe)[V], T (&lqs)[V], T (&h2)[V],
                            T (&z2)[V], T (&n2)[V], T (&le2)[V]) {
            const size_t cb = below ? c + nx : c;
            vload<T, V>(QX + c, qe);
            vload<T, V>(QY + c, qs);
            vload<T, V>(H + cb, h2);
            vload<T, V>(LQX + c, lqe);
            vload<T, V>(LQY + c, lqs);
            vload<T, V>(Z + cb, z2);
            vload<T, V>(Nn + cb, n2);
            vload<T, V>(LH + cb, le2);
        };
        T qE[V], qS[V], lqE[V], lqS[V], hs[V], zs[V], ns[V], les[V];
        if (PF) load_row(ca, r0 + 1 < ny, qE, qS, lqE, lqS, hs, zs, ns, les);
        for (int r = r0; r < r1; ++r) {
            const bool hasS = r + 1 < ny;
            T qE2[V], qS2[V], lqE2[V], lqS2[V], hs2[V], zs2[V], ns2[V], les2[V];
            if (PF) {
                if (r + 1 < r1) load_row(ca + nx, r + 2 < ny, qE2, qS2, lqE2, lqS2, hs2, zs2, ns2, les2);
            } else {
                load_row(ca, hasS, qE, qS, lqE, lqS, hs, zs, ns, les);
            }
            // east neighbour of the lane's last cell = first cell of the next lane
            const T hE = __shfl_down(hc[0], 1, 64);
            const T zE = __shfl_down(zc[0], 1, 64);
            const T nE = __shfl_down(nc[0], 1, 64);
            const T leE = __shfl_down(lec[0], 1, 64);
            T ltE[V], dqE[V], d1E[V], d2E[V], cnE[V];
    #pragma unroll
            for (int j = 0; j < V; ++j) {
                const T h2 = (j + 1 < V) ? hc[j + 1] : hE;
                const T z2 = (j + 1 < V) ? zc[j + 1] : zE;
                const T n2 = (j + 1 < V) ? nc[j + 1] : nE;
                const T le2 = (j + 1 < V) ? lec[j + 1] : leE;
                const T nf = T(0.5) * (nc[j] + n2);
                link_in_d(qE[j], hc[j], h2, z2 - zc[j], g * (nf * nf), g * nf, ms, hdry, dqE[j], d1E[j], d2E[j], cnE[j]);
                ltE[j] = lqE[j] + kk * (le2 - lec[j]);
            }
            if (eastw) {
    #pragma unroll
                for (int j = 0; j < V; ++j) {
                    if (xl + j + 1 != nx) continue;
                    d2E[j] = T(0);
                    if (C.edge_open[1]) {
                        link_open_d(qE[j], hc[j], g * (nc[j] * nc[j]), T(2) * g * nc[j], C.edge_slope[1], ms, hdry,
                                    dqE[j], d1E[j], cnE[j]);
                        ltE[j] = lqE[j] - kk * lec[j];
                    } else {
                        dqE[j] = d1E[j] = cnE[j] = ltE[j] = T(0);
                    }
                }
            }
            // west link of the first cell: the previous lane's last east link
            const T wH = __shfl_up(ltE[V - 1] * d2E[V - 1], 1, 64);
            const T wN = __shfl_up(ltE[V - 1] * cnE[V - 1], 1, 64);
            // south links
            T ltS[V], dqS[V], d1S[V], d2S[V], cnS[V];
            if (hasS) {
    #pragma unroll
                for (int j = 0; j < V; ++j) {
                    const T nf = T(0.5) * (nc[j] + ns[j]);
                    link_in_d(qS[j], hc[j], hs[j], zs[j] - zc[j], g * (nf * nf), g * nf, ms, hdry, dqS[j], d1S[j],
                              d2S[j], cnS[j]);
                    ltS[j] = lqS[j] + kk * (les[j] - lec[j]);
                }
            } else {
    #pragma unroll
                for (int j = 0; j < V; ++j) {
                    d2S[j] = T(0);
                    if (C.edge_open[2]) {
                        link_open_d(qS[j], hc[j], g * (nc[j] * nc[j]), T(2) * g * nc[j], C.edge_slope[2], ms, hdry,
                                    dqS[j], d1S[j], cnS[j]);
                        ltS[j] = lqS[j] - kk * lec[j];
                    } else {
                        dqS[j] = d1S[j] = cnS[j] = ltS[j] = T(0);
                    }
                }
            }
            if (own) {
                T nh4[V], oqx4[V], oqy4[V], na4[V];
    #pragma unroll
                for (int j = 0; j < V; ++j) {
                    const int x = xl + j;
                    const T le_c = lec[j];
                    // east, south (this cell is cell 1), west, north (cell 2), as in k_adj
                    T nh = le_c;
                    T nac = T(0);
                    nh += ltE[j] * d1E[j];
                    nac += ltE[j] * cnE[j];
                    nh += ltS[j] * d1S[j];
                    nac += ltS[j] * cnS[j];
                    if (j == 0 && westw && x == 0) {
                        // west edge link; its strip holds -qo
                        T oqw = T(0);
                        if (C.edge_open[3]) {
                            T dq, d1, cn;
                            link_open_d(-QWs[r], hc[0], g * (nc[0] * nc[0]), T(2) * g * nc[0], C.edge_slope[3], ms,
                                        hdry, dq, d1, cn);
                            const T lt = LQWs[r] + kk * le_c;
                            oqw = lt * dq;
                            nh -= lt * d1;
                            nac -= lt * cn;
                        }
                        LQWo[r] = oqw;
                    } else {
                        nh += (j > 0) ? ltE[j - 1] * d2E[j - 1] : wH;
                        nac += (j > 0) ? ltE[j - 1] * cnE[j - 1] : wN;
                    }
                    if (r > 0) {
                        nh += pNh[j];
                        nac += pNn[j];
                    } else {
                        // north edge link; its strip holds -qo
                        T oqn = T(0);
                        if (C.edge_open[0]) {
                            T dq, d1, cn;
                            link_open_d(-QNs[x], hc[j], g * (nc[j] * nc[j]), T(2) * g * nc[j], C.edge_slope[0], ms,
                                        hdry, dq, d1, cn);
                            const T lt = LQNs[x] + kk * le_c;
                            oqn = lt * dq;
                            nh -= lt * d1;
                            nac -= lt * cn;
                        }
                        LQNo[x] = oqn;
                    }
                    // zero where the step before this one clamped the depth (the tape's
                    // -0): that step's reverse then sees no adjoint of the clamped depth
                    nh4[j] = clamp_mark(hc[j]) ? T(0) : nh;
                    oqx4[j] = ltE[j] * dqE[j];
                    oqy4[j] = ltS[j] * dqS[j];
                    na4[j] = nac;
                    lsum += (double)le_c;
                }
                vstore<T, V>(LHo + ca, nh4);
                vstore<T, V>(LQXo + ca, oqx4);
                vstore<T, V>(LQYo + ca, oqy4);
    #pragma unroll
                for (int j = 0; j < V; ++j) NL[((size_t)(r - r0) * 64 + lane) * V + j] = na4[j];
            }
    #pragma unroll
            for (int j = 0; j < V; ++j) {
                hc[j] = hs[j];
                zc[j] = zs[j];
                nc[j] = ns[j];
                lec[j] = les[j];
                pNh[j] = ltS[j] * d2S[j];
                pNn[j] = ltS[j] * cnS[j];
            }
            if (PF) {
    #pragma unroll
                for (int j = 0; j < V; ++j) {
                    qE[j] = qE2[j];
                    qS[j] = qS2[j];
                    lqE[j] = lqE2[j];
                    lqS[j] = lqS2[j];
                    hs[j] = hs2[j];
                    zs[j] = zs2[j];
                    ns[j] = ns2[j];
                    les[j] = les2[j];
                }
            }
            ca += nx;
        }
        if (tag_prev >= 0 && own) {
            // the seeds 2 (h - d) of the sample the step before completed, in gauge
            // order, added to the depth adjoint just written at the gauge cells among
            // this lane's (none where that step clamped the depth); outside the row
            // loop, so that the march itself carries no gauge work
            for (int q = 0; q < A.n_gauges; ++q) {
                const int gr = A.grc[2 * q], gc = A.grc[2 * q + 1];
                if (gr < r0 || gr >= r1 || gc < xl || gc >= xl + V) continue;
                const size_t cell = (size_t)gr * nx + gc;
                const T hg = H[cell];
                if (!clamp_mark(hg)) LHo[cell] += (T)(2.0 * ((double)hg - A.obs[(size_t)tag_prev * A.n_gauges + q]));
            }
        }
        // rain-multiplier adjoint: the depth adjoint after the step summed over the
        // strip's cells, times R dt of the member's step
        for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
        if (lane == 0) A.mubar_part[(size_t)(sy * C.strips_xa + sx) * C.n_members + k] += lsum * rdt;
    }
    __syncthreads();
    // the quad's Manning-field adjoint: wavefront w adds rows w, w + 4, ... of the
    // strip, the contributions of the stepping members in member order
    if (!(actq[0] || actq[1] || actq[2] || actq[3]) || !own) return;
    T* __restrict__ NA = A.nacc + (size_t)u * plane;
    const T* L0 = reinterpret_cast<const T*>(adj_lds);
    for (int i = wave; i < r1 - r0; i += 4) {
        const size_t ca = (size_t)(r0 + i) * nx + xa;
        T na4[V];
        vload<T, V>(NA + ca, na4);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            T add = T(0);
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (actq[w]) add += L0[(((size_t)w * rows + i) * 64 + lane) * V + j];
            na4[j] += add;
        }
        vstore<T, V>(NA + ca, na4);
    }
}

template <typename T> void launch_adjoint_march(const AdjvLaunch<T>& A, hipStream_t s) {
    constexpr int V = adj_vec<T>();
    const CatchDev<T>& C = A.c;
    const int nq = (C.n_members + 3) / 4;
    const dim3 grid(march_waves(C.strips_xa, C.strips_y, nq, C.march_order, C.march_bands));
    const size_t lds = (size_t)4 * C.march_rows * 64 * V * sizeof(T);
    if (A.pf)
        hipLaunchKernelGGL((k_adjv<T, V, 1>), grid, dim3(kBlock), lds, s, A);
    else
        hipLaunchKernelGGL((k_adjv<T, V, 0>), grid, dim3(kBlock), lds, s, A);
}

// One thread per member of the group (see launch_adj_segment); a cell seen by
// two gauges takes both seeds, in gauge order.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_segment(int G, int stride, const int32_t* n_prev, const int32_t* n,
                                                     const MemberStep<T>* rec, const int32_t* rec_tag, int K,
                                                     const int32_t* grc, const double* obs, const T* tape_h,
                                                     size_t plane, int nx, int32_t* lbase, T* lh0, T* lh1) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= G) return;
    int p = lbase[m];
    if (n_prev) {
        p ^= n_prev[m] & 1;
        lbase[m] = p;
    }
    if (K == 0 || n[m] < 1) return;
    const size_t r = (size_t)(n[m] - 1) * stride + m;
    const int smp = rec_tag[r];
    if (smp < 0) return;
    const T* h = tape_h + (size_t)rec[r].blk_next * plane;
    T* lh = (p ? lh1 : lh0) + (size_t)m * plane;
    for (int q = 0; q < K; ++q) {
        const size_t cell = (size_t)grc[2 * q] * nx + grc[2 * q + 1];
        if (!clamp_mark(h[cell])) lh[cell] += (T)(2.0 * ((double)h[cell] - obs[(size_t)smp * K + q]));
    }
}

template <typename T>
void launch_adj_segment(int G, int stride, const int32_t* n_prev, const int32_t* n, const MemberStep<T>* rec,
                        const int32_t* rec_tag, int K, const int32_t* grc, const double* obs, const T* tape_h,
                        size_t plane, int nx, int32_t* lbase, T* lh0, T* lh1, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_segment<T>), dim3((G + 255) / 256), dim3(256), 0, s, G, stride, n_prev, n, rec, rec_tag,
                       K, grc, obs, tape_h, plane, nx, lbase, lh0, lh1);
}

// Member m of the group, element e of its plane and edge strips: tape block
// blk[m] -> destination copy (dpar[dst.member_off + m], or 0).  Members in
// planes.  The destination may be the tape's first blocks (block m for member m)
// as long as no member's source is one of them but its own; there (dpar null)
// the depths keep their bits, into the ensemble's state (dpar given) a clamped
// depth's -0 becomes +0.
template <typename T>
__global__ __launch_bounds__(256) void k_tape_gather(const CatchDev<T> tape, const int32_t* blk, const CatchDev<T> dst,
                                                     const int32_t* dpar) {
    const int m = blockIdx.y;
    const size_t plane = (size_t)tape.ny * tape.nx;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t b = (size_t)blk[m];
    const int p = dpar ? dpar[dst.member_off + m] : 0;
    if (e < plane) {
        const size_t i = (size_t)m * plane + e;
        const T hv = tape.h[0][b * plane + e];
        dst.h[p][i] = (dpar && hv == T(0)) ? T(0) : hv;
        dst.qx[p][i] = tape.qx[0][b * plane + e];
        dst.qy[p][i] = tape.qy[0][b * plane + e];
    }
    if (e < (size_t)tape.ny) dst.qw[p][(size_t)m * tape.ny + e] = tape.qw[0][b * tape.ny + e];
    if (e < (size_t)tape.nx) dst.qn[p][(size_t)m * tape.nx + e] = tape.qn[0][b * tape.nx + e];
}

template <typename T>
void launch_tape_gather(const CatchDev<T>& tape, const int32_t* blk, const CatchDev<T>& dst, const int32_t* dpar,
                        hipStream_t s) {
    const size_t plane = (size_t)tape.ny * tape.nx;
    const size_t n = std::max(plane, (size_t)std::max(tape.ny, tape.nx));
    hipLaunchKernelGGL((k_tape_gather<T>), dim3((unsigned)((n + 255) / 256), tape.n_members), dim3(256), 0, s, tape,
                       blk, dst, dpar);
}

// nbar[c] += sum over the group's members of their Manning-field adjoint
template <typename T>
__global__ __launch_bounds__(256) void k_nacc_reduce(int G, size_t ncell, const T* nacc, double* nbar) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    double acc = 0.0;
    for (int m = 0; m < G; ++m) acc += (double)nacc[(size_t)m * ncell + c];
    nbar[c] += acc;
}

template <typename T> void launch_nacc_reduce(int G, size_t ncell, const T* nacc, double* nbar, hipStream_t s) {
    hipLaunchKernelGGL((k_nacc_reduce<T>), dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, G, ncell, nacc,
                       nbar);
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

template void launch_adjoint_march<float>(const AdjvLaunch<float>&, hipStream_t);
template void launch_adjoint_march<double>(const AdjvLaunch<double>&, hipStream_t);
template void launch_adj_segment<float>(int, int, const int32_t*, const int32_t*, const MemberStep<float>*,
                                        const int32_t*, int, const int32_t*, const double*, const float*, size_t, int,
                                        int32_t*, float*, float*, hipStream_t);
template void launch_adj_segment<double>(int, int, const int32_t*, const int32_t*, const MemberStep<double>*,
                                         const int32_t*, int, const int32_t*, const double*, const double*, size_t,
                                         int, int32_t*, double*, double*, hipStream_t);
template void launch_tape_gather<float>(const CatchDev<float>&, const int32_t*, const CatchDev<float>&,
                                        const int32_t*, hipStream_t);
template void launch_tape_gather<double>(const CatchDev<double>&, const int32_t*, const CatchDev<double>&,
                                         const int32_t*, hipStream_t);
template void launch_nacc_reduce<float>(int, size_t, const float*, double*, hipStream_t);
template void launch_nacc_reduce<double>(int, size_t, const double*, double*, hipStream_t);
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
