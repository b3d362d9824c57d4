// Auxiliary kernels of libeap: ERP border sums, path upper bounds, NN seeding,
// the final lexicographic argmin, type conversion and buffer fills.
#include <algorithm>

#include "eap_pairs.h"

namespace eap {

// ERP borders (eq. ERP vborder/hborder): B[i] = B[i-1] + |x_i - gap|, one
// series per thread, summed left to right like the recurrence.
__global__ void erp_border_kernel(const double* v, const int64_t* off, int64_t n, double gap, double* out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double acc = 0.0;
    for (int64_t x = off[s]; x < off[s + 1]; ++x) {
        acc = acc + __builtin_fabs(v[x] - gap);
        out[x] = acc;
    }
}

__global__ void to_f32_kernel(const double* v, int64_t n, float* out) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        out[x] = (float)v[x];
}

__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long v, int64_t n) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        p[x] = v;
}

// Cost of the warping path (1,1), (2,2), .., (m,m) followed by straight moves
// along the longer series (Section 4: any path bounds the optimum).  Every step
// adds its term exactly as the recurrence would, so the value is >= the
// distance in floating point as well.  Rows are the longer series.
__device__ double path_ub(int kind, const SweepArgs& A, const double* li, int Lli, const double* co, int Lco) {
    const double INF = __builtin_huge_val();
    const int L = Lli > Lco ? Lli : Lco;
    if (kind == CDTW || kind == ERP) {
        const double r = A.window_ratio;
        if (r < 1.0) {
            int w = (int)floor(r * (double)L);
            if (w < Lli - Lco) return INF;
        }
    }
    double wd = 1.0;   // WDTW weight of the diagonal, w(0)
    if (kind == WDTW) {
        int gi = -L + A.gtab_off;
        gi = gi < 0 ? 0 : (gi >= A.gtab_len ? A.gtab_len - 1 : gi);
        wd = A.gtab[gi];
    }
    double acc = 0.0;
    double sp = 0.0, tp = 0.0;
    for (int k = 1; k <= Lco; ++k) {
        const double s = li[k - 1], t = co[k - 1], d = s - t;
        switch (kind) {
        case DTW: case CDTW: acc = (d * d) + acc; break;
        case WDTW: acc = (wd * (d * d)) + acc; break;
        case ERP: case MSM: acc = acc + __builtin_fabs(d); break;
        case TWE: acc = acc + ((__builtin_fabs(d) + __builtin_fabs(sp - tp)) + A.nu * 0.0); break;
        }
        sp = s;
        tp = t;
    }
    // straight down column L_co: moves (i-1, L_co) -> (i, L_co), |i - L_co| grows
    const double t = co[Lco - 1];
    for (int i = Lco + 1; i <= Lli; ++i) {
        const double s = li[i - 1], d = s - t;
        switch (kind) {
        case DTW: case CDTW: acc = (d * d) + acc; break;
        case WDTW: {
            int gi = 2 * (i - Lco) - L + A.gtab_off;
            gi = gi < 0 ? 0 : (gi >= A.gtab_len ? A.gtab_len - 1 : gi);
            acc = (A.gtab[gi] * (d * d)) + acc;
            break;
        }
        case ERP: acc = acc + __builtin_fabs(s - A.gap); break;
        case MSM: {
            // C(s_i, s_{i-1}, t) of eq. MSMCost
            const double x = li[i - 2];
            double c;
            if ((x <= s && s <= t) || (x >= s && s >= t)) c = A.c;
            else {
                const double p1 = __builtin_fabs(s - x), p2 = __builtin_fabs(s - t);
                c = A.c + (p1 < p2 ? p1 : p2);
            }
            acc = acc + c;
            break;
        }
        case TWE: acc = acc + ((__builtin_fabs(s - li[i - 2]) + A.nu) + A.lam); break;
        }
    }
    return acc;
}

// UB for every (query, candidate) pair, written to ub[a*nB + b].
__global__ void ub_nn_kernel(int kind, SweepArgs A, const double* qv, const int64_t* qoff, const double* rv,
                             const int64_t* roff, double* ub) {
    const int64_t total = A.nA * A.nB;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = p / A.nB, b = p - a * A.nB;
        const double* x = qv + qoff[a];
        const double* y = rv + roff[b];
        const int lx = (int)(qoff[a + 1] - qoff[a]), ly = (int)(roff[b + 1] - roff[b]);
        ub[p] = (lx >= ly) ? path_ub(kind, A, x, lx, y, ly) : path_ub(kind, A, y, ly, x, lx);
    }
}

// The next double above a non-negative value (+inf stays +inf): its bit
// pattern plus one, since non-negative doubles order like their bits.
__device__ __forceinline__ double next_up(double u) {
    if (!(u < __builtin_huge_val())) return u;
    return bitsd(dbits(u) + 1ull);
}

// Prune-only cut-off for every condensed pair: one ulp above its path bound.
__global__ void ub_condensed_kernel(int kind, SweepArgs A, const double* v, const int64_t* off, int64_t n,
                                    double* cut) {
    const int64_t total = n * (n - 1) / 2;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        int64_t i, j;
        condensed_ij(p, n, i, j);
        const double* x = v + off[i];
        const double* y = v + off[j];
        const int lx = (int)(off[i + 1] - off[i]), ly = (int)(off[j + 1] - off[j]);
        const double u = (lx >= ly) ? path_ub(kind, A, x, lx, y, ly) : path_ub(kind, A, y, ly, x, lx);
        cut[p] = next_up(u);
    }
}

// Per query: the candidate with the smallest upper bound (lowest index on
// ties) is swept first, with that bound as its cut-off.  One wave per query.
__global__ void seed_kernel(const double* ub, int64_t nq, int64_t nr, int32_t* seed_b, int32_t* items,
                            unsigned long long* best) {
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= nq) return;
    double bv = __builtin_huge_val();
    int64_t bi = nr;
    for (int64_t r = lane; r < nr; r += 64) {
        const double u = ub[q * nr + r];
        if (u < bv || (u == bv && r < bi)) {
            bv = u;
            bi = r;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o);
        const int64_t oi = __shfl_xor(bi, o);
        if (ov < bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane == 0) {
        if (bi >= nr) bi = 0;
        seed_b[q] = (int32_t)bi;
        items[q] = (int32_t)(q * nr + bi);
        best[q] = dbits(bv);
    }
}

// Alg. 1's result: the lexicographically smallest (distance, index) per query;
// index -1 and +inf when no candidate is finite.  One wave per query.
__global__ void argmin_kernel(const double* res, int64_t nq, int64_t nr, const int32_t* labels, int64_t* out_idx,
                              double* out_dist, int32_t* out_label) {
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= nq) return;
    double bv = __builtin_huge_val();
    int64_t bi = -1;
    for (int64_t r = lane; r < nr; r += 64) {
        const double d = res[q * nr + r];
        if (d < bv) {   // per lane r increases, so strict '<' keeps the lowest index
            bv = d;
            bi = r;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o);
        const int64_t oi = __shfl_xor(bi, o);
        if (ov < bv || (ov == bv && oi >= 0 && (bi < 0 || oi < bi))) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane == 0) {
        out_idx[q] = bi;
        out_dist[q] = bv;
        if (out_label) out_label[q] = (bi >= 0 && labels) ? labels[bi] : -1;
    }
}

// Largest |x| over a set, as the bit pattern of a non-negative double.
__global__ void absmax_kernel(const double* v, int64_t n, unsigned long long* out) {
    double m = 0.0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, __builtin_fabs(v[x]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) atomicMax(out, dbits(m));
}

// Certified bound on |D32 - D64| for any warping path whose exact cost is at
// most B, with at most N steps, over values of magnitude <= A, in FP32 (unit
// roundoff u = 2^-24): each term carries the rounding of its inputs
// (u|a| + u|b|), of its own operations, and the running sum adds gamma_N on the
// total.  Squared costs: |fl(d)^2 - d^2| <= 4uA|d| + 3u d^2 per term and
// sum|d| <= sqrt(N sum d^2) (Cauchy-Schwarz; WDTW's weights are <= 1 and add
// one more rounding).  L1 costs (ERP, MSM, TWE): <= u(4A + 3|term|) per term.
// The FP64 reference carries the same error with 2^-53, covered by the factor
// 1.01; the last term covers FP32 underflow of tiny squares.
__device__ double screen_eps(int kind, double B, double N, double A) {
    const double u = 0x1p-24;
    double e;
    if (kind == DTW || kind == CDTW || kind == WDTW) e = u * ((N + 5.0) * B + 4.0 * A * sqrt(N * B));
    else e = u * ((N + 3.0) * B + 4.0 * N * A);
    return 1.01 * e + N * 4e-38;
}

// Largest exact cost C that can still satisfy C <= b + eps(C), i.e. a bound on
// the exact cost of any path whose FP32 evaluation is <= b.  eps grows like
// sqrt(C) for the squared costs, so for b near 0 this is about (4uA)^2 N, not 0.
__device__ double screen_bound(int kind, double b, double N, double A) {
    const double u = 1.01 * 0x1p-24;
    const double e0 = b + N * 4e-38;
    double B;
    if (kind == DTW || kind == CDTW || kind == WDTW) {
        const double a = u * (N + 5.0), c = u * 4.0 * A * sqrt(N);
        const double r = (c + sqrt(c * c + 4.0 * (1.0 - a) * e0)) / (2.0 * (1.0 - a));
        B = r * r;
    } else {
        B = (e0 + u * 4.0 * N * A) / (1.0 - u * (N + 3.0));
    }
    return B * (1.0 + 1e-9);
}

// Widening of each query's FP32 cut-off during the screening sweep.  The
// best-so-far b is an FP32 distance (or the FP64 path bound UB >= b), so the
// exact NN distance is <= screen_bound(b) and any prefix of its path evaluates
// in FP32 to <= b + 2 eps(screen_bound(UB)).
__global__ void screen_widen_kernel(int kind, SweepArgs A, const int64_t* qoff, int64_t lr_max, double gap,
                                    const unsigned long long* absmax, double* widen_abs) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A.nA) return;
    const double N = (double)(qoff[q + 1] - qoff[q] + lr_max);
    double Amax = bitsd(*absmax);
    if (kind == ERP) Amax = fmax(Amax, __builtin_fabs(gap));
    const double ub = bitsd(A.best[q]);
    widen_abs[q] = (ub < __builtin_huge_val()) ? 2.0 * screen_eps(kind, screen_bound(kind, ub, N, Amax), N, Amax)
                                               : 0.0;
}

// After the FP32 sweep: every candidate of query q whose FP32 distance is
// <= b32 + 2 eps(screen_bound(b32)) is listed for the FP64 recheck.  The FP64
// NN cannot be elsewhere: its exact cost is <= that of the FP32 winner, which
// is <= screen_bound(b32), and its FP32 value exceeds that by at most eps.
// The margin m widens b32 by a relative (1 + m) on top.  The result slots are
// reset to +inf, and best[q] becomes screen_bound(b32), an upper bound on the
// FP64 NN distance that serves as the recheck's first cut-off.  One wave per query.
__global__ void screen_filter_kernel(int kind, SweepArgs A, const int64_t* qoff, int64_t lr_max, double gap,
                                     const unsigned long long* absmax, double margin_rel, double* res,
                                     unsigned long long* best, int32_t* items, unsigned int* count,
                                     unsigned long long* rechecks) {
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= A.nA) return;
    const double N = (double)(qoff[q + 1] - qoff[q] + lr_max);
    double Amax = bitsd(*absmax);
    if (kind == ERP) Amax = fmax(Amax, __builtin_fabs(gap));
    const double b32 = bitsd(best[q]);
    double thr = __builtin_huge_val(), cut64 = __builtin_huge_val();
    if (b32 < __builtin_huge_val()) {
        const double b = b32 * (1.0 + margin_rel);
        cut64 = screen_bound(kind, b, N, Amax);
        thr = b + 2.0 * screen_eps(kind, cut64, N, Amax);
    }
    unsigned long long n = 0;
    for (int64_t r = lane; r < A.nB; r += 64) {
        const int64_t p = q * A.nB + r;
        if (res[p] <= thr) {
            const unsigned int k = atomicAdd(count, 1u);
            items[k] = (int32_t)p;
            ++n;
        }
        res[p] = __builtin_huge_val();
    }
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
    if (lane == 0) {
        best[q] = dbits(cut64);
        if (n) atomicAdd(rechecks, n);
    }
}

static int blocks_for(int64_t n, int per) {
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return (int)b;
}

hipError_t launch_erp_border(const double* v, const int64_t* off, int64_t n, double gap, double* out, hipStream_t s) {
    hipLaunchKernelGGL(erp_border_kernel, dim3(blocks_for(n, 64)), dim3(64), 0, s, v, off, n, gap, out);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double* v, int64_t n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(to_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, v, n, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_absmax(const double* v, int64_t n, unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(absmax_kernel, dim3(std::min(blocks_for(n, 256), 1024)), dim3(256), 0, s, v, n, out);
    return hipGetLastError();
}

hipError_t launch_screen_widen(int kind, const SweepArgs& a, const int64_t* qoff, int64_t lr_max, double gap,
                               const unsigned long long* absmax, double* widen_abs, hipStream_t s) {
    hipLaunchKernelGGL(screen_widen_kernel, dim3(blocks_for(a.nA, 256)), dim3(256), 0, s, kind, a, qoff, lr_max, gap,
                       absmax, widen_abs);
    return hipGetLastError();
}

hipError_t launch_screen_filter(int kind, const SweepArgs& a, const int64_t* qoff, int64_t lr_max, double gap,
                                const unsigned long long* absmax, double margin_rel, double* res,
                                unsigned long long* best, double* widen_abs, int32_t* items, unsigned int* count,
                                unsigned long long* rechecks, hipStream_t s) {
    (void)widen_abs;
    hipLaunchKernelGGL(screen_filter_kernel, dim3(blocks_for(a.nA, 4)), dim3(256), 0, s, kind, a, qoff, lr_max, gap,
                       absmax, margin_rel, res, best, items, count, rechecks);
    return hipGetLastError();
}

hipError_t launch_ub_nn(int kind, const SweepArgs& a, const double* qv, const int64_t* qoff, const double* rv,
                        const int64_t* roff, double* ub, hipStream_t s) {
    hipLaunchKernelGGL(ub_nn_kernel, dim3(blocks_for(a.nA * a.nB, 256)), dim3(256), 0, s, kind, a, qv, qoff, rv, roff,
                       ub);
    return hipGetLastError();
}

hipError_t launch_ub_condensed(int kind, const SweepArgs& a, const double* v, const int64_t* off, int64_t n,
                               double* cut, hipStream_t s) {
    hipLaunchKernelGGL(ub_condensed_kernel, dim3(blocks_for(n * (n - 1) / 2, 256)), dim3(256), 0, s, kind, a, v, off,
                       n, cut);
    return hipGetLastError();
}

hipError_t launch_seed(const double* ub, int64_t nq, int64_t nr, int32_t* seed_b, int32_t* items,
                       unsigned long long* best, hipStream_t s) {
    hipLaunchKernelGGL(seed_kernel, dim3(blocks_for(nq, 4)), dim3(256), 0, s, ub, nq, nr, seed_b, items, best);
    return hipGetLastError();
}

hipError_t launch_argmin(const double* res, int64_t nq, int64_t nr, const int32_t* labels, int64_t* out_idx,
                         double* out_dist, int32_t* out_label, hipStream_t s) {
    hipLaunchKernelGGL(argmin_kernel, dim3(blocks_for(nq, 4)), dim3(256), 0, s, res, nq, nr, labels, out_idx,
                       out_dist, out_label);
    return hipGetLastError();
}

}  // namespace eap
