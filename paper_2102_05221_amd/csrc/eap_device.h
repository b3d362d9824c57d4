// Device-side helpers shared by the sweep kernels of libeap (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eap {

enum Kind : int { DTW = 0, CDTW = 1, WDTW = 2, ERP = 3, MSM = 4, TWE = 5 };

template <typename T> __device__ __forceinline__ T inf_v();
template <> __device__ __forceinline__ double inf_v<double>() { return __builtin_huge_val(); }
template <> __device__ __forceinline__ float inf_v<float>() { return __builtin_huge_valf(); }

template <typename T> __device__ __forceinline__ T vmin(T a, T b) { return a < b ? a : b; }
template <typename T> __device__ __forceinline__ T vmax(T a, T b) { return a > b ? a : b; }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double vabs(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float vabs(float a) { return __builtin_fabsf(a); }

// Lane k receives lane k-1's value (DPP wave_shr:1; lane 0 receives 0 through
// bound_ctrl, so no old value has to be set up).  Must be executed with every
// lane of the wave active, so that the source lanes hold defined values.
__device__ __forceinline__ int shr1_i32(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ float shr1(float v) {
    return __builtin_bit_cast(float, shr1_i32(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double shr1(double v) {
    long long b = __builtin_bit_cast(long long, v);
    int lo = shr1_i32((int)(unsigned long long)b);
    int hi = shr1_i32((int)((unsigned long long)b >> 32));
    unsigned long long r = (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32);
    return __builtin_bit_cast(double, r);
}

// Within each row of 16 lanes: lane k > 0 receives lane k-1's v, lane 0 of
// the row keeps `first` (DPP row_shr:1 without bound_ctrl leaves lanes whose
// source lies outside the row unwritten).  For groups of exactly 16 lanes
// this shifts within the group and feeds its first lane in one instruction.
__device__ __forceinline__ float row_shr1_or(float v, float first) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, first),
                                                                 __builtin_bit_cast(int, v), 0x111, 0xf, 0xf, false));
}
__device__ __forceinline__ double row_shr1_or(double v, double first) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long f = __builtin_bit_cast(unsigned long long, first);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)f, (int)(unsigned)b, 0x111, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(f >> 32), (int)(unsigned)(b >> 32), 0x111, 0xf, 0xf,
                                               false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Value of the lane whose byte address (lane * 4) is `addr`, from every lane
// (ds_bpermute).  With a loop-invariant base and a constant added to it, the
// constant lands in the instruction's offset field.
__device__ __forceinline__ float bperm(int addr, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double bperm(int addr, double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)b);
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// One series point of ND channels (multivariate series: ND > 1), moved between
// lanes channel by channel.
template <typename V, int ND> struct Pt {
    V c[ND];
};
template <typename V, int ND> __device__ __forceinline__ Pt<V, ND> shr1(const Pt<V, ND>& p) {
    Pt<V, ND> r;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.c[i] = shr1(p.c[i]);
    return r;
}
template <typename V, int ND> __device__ __forceinline__ Pt<V, ND> row_shr1_or(const Pt<V, ND>& p,
                                                                              const Pt<V, ND>& first) {
    Pt<V, ND> r;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.c[i] = row_shr1_or(p.c[i], first.c[i]);
    return r;
}
template <typename V, int ND> __device__ __forceinline__ Pt<V, ND> bperm(int addr, const Pt<V, ND>& p) {
    Pt<V, ND> r;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.c[i] = bperm(addr, p.c[i]);
    return r;
}
template <typename V, int ND> __device__ __forceinline__ Pt<V, ND> pt_fill(V v) {
    Pt<V, ND> r;
#pragma unroll
    for (int i = 0; i < ND; ++i) r.c[i] = v;
    return r;
}

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// Non-negative doubles order like their bit patterns, +inf above every finite.
__device__ __forceinline__ unsigned long long dbits(double v) {
    return (unsigned long long)__builtin_bit_cast(long long, v);
}
__device__ __forceinline__ double bitsd(unsigned long long b) { return __builtin_bit_cast(double, (long long)b); }

// The next representable value above a non-negative finite t.
__device__ __forceinline__ float round_up_next(float t) {
    return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, t) + 1u);
}
__device__ __forceinline__ double round_up_next(double t) {
    return __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, t) + 1ull);
}

// A load that does not hit the CU's L1 (relaxed atomic at agent scope), for
// values this wave wrote earlier to a location it had read before.
__device__ __forceinline__ double load_nc(const double* p) {
    unsigned long long b = __hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<double*>(p)),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(double, b);
}
__device__ __forceinline__ float load_nc(const float* p) {
    unsigned b = __hip_atomic_load(reinterpret_cast<unsigned*>(const_cast<float*>(p)), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(float, b);
}

// One set of series: concatenated values, int64 offsets (n+1), and for ERP the
// running border sums B[off+i-1] = sum_{m<=i} |x_m - gap| (same layout).
template <typename T> struct Series {
    const T* v;
    const int64_t* off;
    const T* border;
};

}  // namespace eap
