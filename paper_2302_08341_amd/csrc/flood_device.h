// Device-side helpers shared by the forward and adjoint kernels of libflood:
// workgroup order, IEEE bit patterns, the Eq. 2 friction power, and the link
// discharge functions (Eqs. 2-3 with the donor limiter and open edges).
#pragma once

#include "flood_internal.h"

namespace flood {

// Workgroups are dispatched round-robin over the 8 XCDs (id % 8).  Remap the
// id so that each XCD walks a contiguous range of logical tiles; vertically
// adjacent tiles then meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ uint32_t to_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ unsigned long long to_bits(double v) {
    return (unsigned long long)__double_as_longlong(v);
}
template <typename T> __device__ __forceinline__ T from_bits(typename HBits<T>::type b);
template <> __device__ __forceinline__ float from_bits<float>(uint32_t b) { return __uint_as_float(b); }
template <> __device__ __forceinline__ double from_bits<double>(unsigned long long b) {
    return __longlong_as_double((long long)b);
}

// h^(-7/3) of the friction denominator of Eq. 2, as h^(-1/3) / h^2: a few ulp.
// h^(-1/3) starts from the hardware exp2(-log2(h) / 3), whose error (the
// logarithm's, a third of it carried by the exponent, a few 1e-7 relative) one
// Newton step on y^3 h = 1 squares away.  The hardware exp2(-7/3 log2 h) alone
// carries seven times that error, about 2e-6 relative and of one sign step
// after step, which moved single-precision discharges on shallow
// friction-dominated links by 3e-4 of the largest discharge within 80 steps.
// For h > 0 only (dry links discard the result).
__device__ __forceinline__ float pow_m73(float h) {
    const float y0 = __builtin_amdgcn_exp2f(-0.333333343f * __builtin_amdgcn_logf(h));
    const float t = (y0 * y0) * (y0 * h);
    const float y = y0 + y0 * ((1.0f - t) * 0.333333343f);
    return y * __builtin_amdgcn_rcpf(h * h);
}
__device__ __forceinline__ double pow_m73(double h) { return 1.0 / pow(h, 7.0 / 3.0); }

__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }

// Interior link between cell 1 (west/north) and cell 2 (east/south).
// Eq. 3 in difference form: with dz = z2 - z1, the higher surface is cell 1
// iff h1 - h2 >= dz, and max(eta) - max(z) = h_up - max(+-dz, 0); the surface
// slope is (h2 - h1 + dz)/dx.  Eq. 2 semi-implicit friction, then the donor
// limiter |q| <= h_up dx / (4 dt).  Evaluated without branches and selected at
// the end, so dry and wet links in one wavefront do not split it; a dry link's
// intermediate values (possibly inf or NaN from the friction power) are
// discarded by the final select.
// 32-bit integer hash (an xorshift-multiply finaliser) used as a counter-based
// random number generator: the random bits of a cell in a step are a function
// of the member's step count and the cell index only, so they are the same
// whichever kernel, tiling or batch computes the cell.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Depth update of Eq. 1, h + inc.  In single precision it is rounded
// stochastically: the exact sum is split into its rounded value s and the
// exact error e (h + inc = s + e, Knuth's TwoSum, exact with contraction off),
// and s moves one ulp toward e with probability |e| / ulp, resolved to 2^-16.
// The expected result is the exact sum (to 2^-17 ulp), so rounding errors no
// longer pile up in one direction where nearly equal small increments (rain on
// a pond) meet the same large depth step after step: the stored depth and the
// mass ledger drift like a random walk instead of linearly.  The 16 random bits
// of a cell are half of the hash of (seed, cell pair), so a lane moving
// adjacent cells hashes once per pair.  In double precision the sum is
// rounded to nearest.
template <typename T> __device__ __forceinline__ T depth_add(T h, T inc, uint32_t seed, uint32_t cell);
template <> __device__ __forceinline__ float depth_add<float>(float h, float inc, uint32_t seed, uint32_t cell) {
    const float s = h + inc;
    const float bb = s - h;
    const float e = (h - (s - bb)) + (inc - bb);
    const uint32_t sb = __float_as_uint(s);
    const bool away = (e > 0.0f) == (s > 0.0f);          // toward e: away from zero when e has s's sign
    const float nb = __uint_as_float(away ? sb + 1u : sb - 1u);
    const float gap = fabsf(nb - s);
    const uint32_t r = mix32(seed ^ (cell >> 1)) >> ((cell & 1u) << 4);
    const float u = (float)(r & 0xffffu) * 0x1p-16f;
    return (e != 0.0f && s != 0.0f && u * gap < fabsf(e)) ? nb : s;
}
template <> __device__ __forceinline__ double depth_add<double>(double h, double inc, uint32_t, uint32_t) {
    return h + inc;
}

// The adjoint's row-march tape keeps a depth that the step clamped at zero as
// -0 (every other zero depth is +0), so the tape itself records the clamp
// branch of each cell and step.  Only the tape carries -0: the step's values do
// not depend on which zero it reads (a zero discharge may come out as -0), and
// depths handed back to the ensemble are +0 again.
template <typename T> __device__ __forceinline__ bool clamp_mark(T h) {
    if constexpr (sizeof(T) == 4)
        return __float_as_uint(h) == 0x80000000u;
    else
        return (unsigned long long)__double_as_longlong(h) == 0x8000000000000000ull;
}

// Eq. 3 flow depth of an interior link in difference form: the depth of the
// cell with the higher water surface minus the positive part of the bed step
// towards the other cell.  Every kernel that decides whether a link is wet
// (step, adjoint, exported wet/dry mask) forms the flow depth here, so their
// decisions agree bit for bit.
template <typename T> __device__ __forceinline__ T link_depth(T h1, T h2, T dz) {
    const T d = h1 - h2;
    return (d >= dz) ? h1 - fmax(dz, T(0)) : h2 - fmax(-dz, T(0));
}

template <typename T>
__device__ __forceinline__ T link_in(T q, T h1, T h2, T dz, T G, const MemberStep<T>& ms, T hdry) {
    const T d = h1 - h2;
    const T hf = link_depth(h1, h2, dz);
    const T num = q - ms.gdtdx * hf * (dz - d);
    const T A = G * ms.s2dt * pow_m73(hf);
    const T qn = qdiv(num, T(1) + A * fabs(q));
    // donor limiter, branch-free: the lower bound only binds when qn < 0 and the
    // upper bound only when qn > 0 (both bounds straddle zero)
    const T lim = fmin(fmax(qn, -h2 * ms.capf), h1 * ms.capf);
    return (hf > hdry) ? lim : T(0);
}

// Open edge link: outward discharge qo driven by the fixed outward slope Se,
// flow depth = inner cell depth; outflow only.
template <typename T>
__device__ __forceinline__ T link_open(T qo, T h, T G, T Se, const MemberStep<T>& ms, T hdry) {
    const T A = G * ms.s2dt * pow_m73(h);
    const T qn = qdiv(qo + ms.gdt * h * Se, T(1) + A * fabs(qo));
    const T lim = fmax(fmin(qn, h * ms.capf), T(0));
    return (h > hdry) ? lim : T(0);
}

template <typename T, int MI>
__device__ __forceinline__ size_t state_index(const CatchDev<T>& C, int member, int r, int c) {
    return ((size_t)(member / MI) * C.ny + r) * ((size_t)C.nx * MI) + (size_t)c * MI + member % MI;
}

// Wavefront -> (member unit, strip) of the row-march kernels.  A member unit is
// one member, or a group of members marched together.  Orders:
//   0  units fastest (neighbouring wavefronts share the strip's bed and roughness)
//   1  strips along x fastest, then rows of strips, then units (neighbouring
//      wavefronts stream neighbouring segments of the same rows of one member)
//   2  quads of units fastest, then strips as in 1, then quads: the four
//      wavefronts of a workgroup march the same strip for four units, so the
//      shared arrays are fetched once per workgroup and each member's rows are
//      still streamed strip after strip
//   3  strips along x fastest, then units, then rows of strips: the 8 XCDs,
//      each walking a contiguous range of workgroups, take bands of rows of
//      every member instead of whole members, so members that are already done
//      leave every XCD the same share of work, and all units of a row of
//      strips run on one XCD close in time (the shared bed and roughness of
//      those rows stay in its L2)
//   4  the rows of strips cut into march_bands bands (a multiple of 8, so each
//      XCD range of workgroups holds whole bands), then units, then rows of
//      strips within the band, then strips along x: order 1 inside each band,
//      with every XCD holding bands of every unit, and a band's bed and
//      roughness shared by the units that follow one another on that XCD
// Order 2 pads the unit count to a multiple of four and order 4 the rows of
// strips to a multiple of the band count; padding wavefronts get false.
template <typename T>
__device__ __forceinline__ bool march_wave(const CatchDev<T>& C, int local, int units, int& k, int& sx, int& sy,
                                           int strips_x) {
    if (C.march_order == 0) {
        k = local % units;
        const int strip = local / units;
        sy = strip / strips_x;
        sx = strip - sy * strips_x;
    } else if (C.march_order == 1) {
        sx = local % strips_x;
        const int rest = local / strips_x;
        sy = rest % C.strips_y;
        k = rest / C.strips_y;
    } else if (C.march_order == 4) {
        const int bh = (C.strips_y + C.march_bands - 1) / C.march_bands;   // rows of strips per band
        const int per_unit = bh * strips_x;
        const int band = local / (per_unit * units);
        const int rem = local - band * per_unit * units;
        k = rem / per_unit;
        const int rem2 = rem - k * per_unit;
        sy = band * bh + rem2 / strips_x;
        sx = rem2 % strips_x;
        return sy < C.strips_y && k < units;
    } else if (C.march_order == 3) {
        sx = local % strips_x;
        const int rest = local / strips_x;
        k = rest % units;
        sy = rest / units;
        return sy < C.strips_y;
    } else {
        const int q = local & 3;
        const int rest = local >> 2;
        sx = rest % strips_x;
        const int rest2 = rest / strips_x;
        sy = rest2 % C.strips_y;
        k = (rest2 / C.strips_y) * 4 + q;
    }
    return k < units;
}

template <typename T>
__device__ __forceinline__ bool march_wave(const CatchDev<T>& C, int local, int units, int& k, int& sx, int& sy) {
    return march_wave(C, local, units, k, sx, sy, C.strips_x);
}

// the cell beside a row-march strip, as loaded by the halo lanes of k_marchv
template <typename T>
struct Halo {
    T h = T(0), z = T(0), n = T(0), q = T(0);   // depth, bed, roughness, east link
    uint32_t cls = 0;                           // land-cover class (roughness from the member's table)
};

// v as held by lane src of the wavefront (ds_bpermute: byte address = 4 x lane)
__device__ __forceinline__ float lane_read(float v, int src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ double lane_read(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// V adjacent cells moved with one V-wide access (p must be V-element aligned)
template <typename T, int V> struct VecOf;
template <> struct VecOf<float, 4> { typedef float __attribute__((ext_vector_type(4))) type; };
template <> struct VecOf<float, 2> { typedef float __attribute__((ext_vector_type(2))) type; };
template <> struct VecOf<double, 2> { typedef double __attribute__((ext_vector_type(2))) type; };

template <typename T, int V>
__device__ __forceinline__ void vload(const T* p, T (&d)[V]) {
    typedef typename VecOf<T, V>::type vt;
    const vt v = *reinterpret_cast<const vt*>(p);
#pragma unroll
    for (int j = 0; j < V; ++j) d[j] = v[j];
}
template <typename T, int V>
__device__ __forceinline__ void vstore(T* p, const T (&d)[V]) {
    typedef typename VecOf<T, V>::type vt;
    vt v;
#pragma unroll
    for (int j = 0; j < V; ++j) v[j] = d[j];
    *reinterpret_cast<vt*>(p) = v;
}
// streaming variants: the state is touched once per step, so these accesses are
// marked non-temporal and leave cache capacity to the shared bed and roughness
template <typename T, int V>
__device__ __forceinline__ void vload_nt(const T* p, T (&d)[V]) {
    typedef typename VecOf<T, V>::type vt;
    const vt v = __builtin_nontemporal_load(reinterpret_cast<const vt*>(p));
#pragma unroll
    for (int j = 0; j < V; ++j) d[j] = v[j];
}
template <typename T, int V>
__device__ __forceinline__ void vstore_nt(T* p, const T (&d)[V]) {
    typedef typename VecOf<T, V>::type vt;
    vt v;
#pragma unroll
    for (int j = 0; j < V; ++j) v[j] = d[j];
    __builtin_nontemporal_store(v, reinterpret_cast<vt*>(p));
}

}  // namespace flood
