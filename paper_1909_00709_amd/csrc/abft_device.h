// Device-side building blocks for the gfx950 kernels: wavefront reductions (DPP), compensated
// fp32 pairs, 16-byte vector access, boundary mapping and the event log.
#pragma once

#include "abft_internal.h"

namespace abft {

// ------------------------------------------------------------------------------------------
// 16-byte vector access.
// ------------------------------------------------------------------------------------------
template <typename T, int V>
struct VecOps;

template <typename T>
struct VecOps<T, 1> {
    static __device__ __forceinline__ void load(const T* p, T (&d)[1]) { d[0] = *p; }
    static __device__ __forceinline__ void load_nt(const T* p, T (&d)[1])
    {
        d[0] = __builtin_nontemporal_load(p);
    }
    static __device__ __forceinline__ void store(T* p, const T (&s)[1]) { *p = s[0]; }
    static __device__ __forceinline__ void store_nt(T* p, const T (&s)[1])
    {
        __builtin_nontemporal_store(s[0], p);
    }
};

template <>
struct VecOps<float, 4> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ void load(const float* p, float (&d)[4])
    {
        const v4 t = *reinterpret_cast<const v4*>(p);
        d[0] = t.x; d[1] = t.y; d[2] = t.z; d[3] = t.w;
    }
    static __device__ __forceinline__ void load_nt(const float* p, float (&d)[4])
    {
        const v4 t = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
        d[0] = t.x; d[1] = t.y; d[2] = t.z; d[3] = t.w;
    }
    static __device__ __forceinline__ void store(float* p, const float (&s)[4])
    {
        v4 t;
        t.x = s[0]; t.y = s[1]; t.z = s[2]; t.w = s[3];
        *reinterpret_cast<v4*>(p) = t;
    }
    static __device__ __forceinline__ void store_nt(float* p, const float (&s)[4])
    {
        v4 t;
        t.x = s[0]; t.y = s[1]; t.z = s[2]; t.w = s[3];
        __builtin_nontemporal_store(t, reinterpret_cast<v4*>(p));
    }
};

template <>
struct VecOps<double, 2> {
    typedef double v2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ void load(const double* p, double (&d)[2])
    {
        const v2 t = *reinterpret_cast<const v2*>(p);
        d[0] = t.x; d[1] = t.y;
    }
    static __device__ __forceinline__ void load_nt(const double* p, double (&d)[2])
    {
        const v2 t = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
        d[0] = t.x; d[1] = t.y;
    }
    static __device__ __forceinline__ void store(double* p, const double (&s)[2])
    {
        v2 t;
        t.x = s[0]; t.y = s[1];
        *reinterpret_cast<v2*>(p) = t;
    }
    static __device__ __forceinline__ void store_nt(double* p, const double (&s)[2])
    {
        v2 t;
        t.x = s[0]; t.y = s[1];
        __builtin_nontemporal_store(t, reinterpret_cast<v2*>(p));
    }
};

// ------------------------------------------------------------------------------------------
// Wavefront data movement.  DPP row operations act within 16-lane rows; readlane moves a
// value from one lane to all.  Every reduction below gives the same bits in every lane of a
// row (the combining operations are commutative), so the results are deterministic.
// ------------------------------------------------------------------------------------------
enum : int {
    DPP_QUAD_1032 = 0xB1,      // quad_perm [1,0,3,2]
    DPP_QUAD_2301 = 0x4E,      // quad_perm [2,3,0,1]
    DPP_ROW_MIRROR = 0x140,
    DPP_ROW_HALF_MIRROR = 0x141
};

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi =
        __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double,
                              ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}

__device__ __forceinline__ float readlane_f(float v, int lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __builtin_bit_cast(double,
                              ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}

// Sum over each 16-lane row; every lane of the row receives the row total.
__device__ __forceinline__ double row16_sum(double v)
{
    v += dpp_d<DPP_QUAD_1032>(v);
    v += dpp_d<DPP_QUAD_2301>(v);
    v += dpp_d<DPP_ROW_HALF_MIRROR>(v);
    v += dpp_d<DPP_ROW_MIRROR>(v);
    return v;
}

__device__ __forceinline__ double row16_max(double v)
{
    v = fmax(v, dpp_d<DPP_QUAD_1032>(v));
    v = fmax(v, dpp_d<DPP_QUAD_2301>(v));
    v = fmax(v, dpp_d<DPP_ROW_HALF_MIRROR>(v));
    v = fmax(v, dpp_d<DPP_ROW_MIRROR>(v));
    return v;
}

// Knuth's two-sum: s + e == a + b exactly, |e| <= ulp(s)/2.  A compensated fp32 value is the
// unevaluated pair (s, e); adding two pairs keeps the rounding error of the leading parts.
struct CPair {
    float s, e;
};

__device__ __forceinline__ CPair cpair_add(CPair a, CPair b)
{
    const float t = a.s + b.s;
    const float bp = t - a.s;
    const float err = (a.s - (t - bp)) + (b.s - bp);
    return CPair{t, (a.e + b.e) + err};
}

__device__ __forceinline__ CPair cpair_add1(CPair a, float v)
{
    const float t = a.s + v;
    const float bp = t - a.s;
    const float err = (a.s - (t - bp)) + (v - bp);
    return CPair{t, a.e + err};
}

template <int CTRL>
__device__ __forceinline__ CPair dpp_pair(CPair p)
{
    return CPair{dpp_f<CTRL>(p.s), dpp_f<CTRL>(p.e)};
}

__device__ __forceinline__ CPair row16_pair(CPair p)
{
    p = cpair_add(p, dpp_pair<DPP_QUAD_1032>(p));
    p = cpair_add(p, dpp_pair<DPP_QUAD_2301>(p));
    p = cpair_add(p, dpp_pair<DPP_ROW_HALF_MIRROR>(p));
    p = cpair_add(p, dpp_pair<DPP_ROW_MIRROR>(p));
    return p;
}

// Totals of segments of LPR lanes (16, 32 or 64) from per-row totals.
template <int LPR>
__device__ __forceinline__ double segment_total(double rowsum)
{
    if constexpr (LPR == 16) {
        return rowsum;
    } else {
        const double r0 = readlane_d(rowsum, 0), r1 = readlane_d(rowsum, 16);
        const double r2 = readlane_d(rowsum, 32), r3 = readlane_d(rowsum, 48);
        if constexpr (LPR == 64) return (r0 + r1) + (r2 + r3);
        return (threadIdx.x & 32) ? (r2 + r3) : (r0 + r1);
    }
}

template <int LPR>
__device__ __forceinline__ double segment_total(CPair rowsum)
{
    if constexpr (LPR == 16) {
        return (double)rowsum.s + (double)rowsum.e;
    } else {
        const CPair r0{readlane_f(rowsum.s, 0), readlane_f(rowsum.e, 0)};
        const CPair r1{readlane_f(rowsum.s, 16), readlane_f(rowsum.e, 16)};
        const CPair r2{readlane_f(rowsum.s, 32), readlane_f(rowsum.e, 32)};
        const CPair r3{readlane_f(rowsum.s, 48), readlane_f(rowsum.e, 48)};
        CPair t;
        if constexpr (LPR == 64)
            t = cpair_add(cpair_add(r0, r1), cpair_add(r2, r3));
        else
            t = (threadIdx.x & 32) ? cpair_add(r2, r3) : cpair_add(r0, r1);
        return (double)t.s + (double)t.e;
    }
}

__device__ __forceinline__ double wave_max(double v)
{
    v = row16_max(v);
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

__device__ __forceinline__ double wave_sum(double v)
{
    v = row16_sum(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// ------------------------------------------------------------------------------------------
// Boundary rule on one coordinate: index inside [0, n), or -1 for a constant ghost.
// Stencils of radius at most 2 only step up to two points outside the grid, so c lies in
// [-2n, 3n) for every n >= 1 (an axis of length 1 included) and the periodic wrap takes at
// most two steps of n, with no division.
// ------------------------------------------------------------------------------------------
__host__ __device__ __forceinline__ int map_coord(int c, int n, int bc)
{
    if (c >= 0 && c < n) return c;
    if (bc == ABFT_BC_CLAMP) return c < 0 ? 0 : n - 1;
    if (bc == ABFT_BC_PERIODIC) {
        if (c < 0) {
            c += n;
            if (c < 0) c += n;
        } else {
            c -= n;
            if (c >= n) c -= n;
        }
        return c;
    }
    return -1;
}

__device__ __forceinline__ void emit_event(Counters* cnt, abft_event* ev, int cap, int64_t sweep,
                                           int kind, int z, int y, int x, double va, double vb,
                                           int grid)
{
    const unsigned long long i = atomicAdd(&cnt->events_total, 1ull);
    if (ev != nullptr && i < (unsigned long long)cap) {
        abft_event e;
        e.sweep = sweep;
        e.kind = kind;
        e.z = z;
        e.y = y;
        e.x = x;
        e.a = va;
        e.b = vb;
        e.grid = grid;
        e.pad = 0;
        ev[i] = e;
    }
}

// The stored maximum, read early by a caller that wants the read's latency out of its tail.
__device__ __forceinline__ unsigned long long noise_known(const Counters* cnt)
{
    return __hip_atomic_load(&cnt->noise_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every wavefront of a sweep reaches this at about the same time, and atomics on one address
// serialise at the coherence point (measured: ~12 us per 2048-wavefront sweep).  The maximum
// only grows, so a wavefront whose value does not exceed a value already stored (known, read
// at any earlier time) can skip the atomic without changing the result.
__device__ __forceinline__ void record_noise(Counters* cnt, double noise,
                                             unsigned long long known)
{
    const double m = wave_max(noise);
    if ((threadIdx.x & 63) == 0 && m > 0.0) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(m);
        if (b > known) atomicMax(&cnt->noise_bits, b);
    }
}

__device__ __forceinline__ void record_noise(Counters* cnt, double noise)
{
    record_noise(cnt, noise, noise_known(cnt));
}

}  // namespace abft
