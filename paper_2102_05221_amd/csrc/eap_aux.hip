// Auxiliary kernels of libeap: ERP border sums, path upper bounds, NN seeding,
// the final lexicographic argmin, type conversion and buffer fills.
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
