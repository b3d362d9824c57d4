// Auxiliary kernels of libeap: ERP border sums, path upper bounds, NN seeding,
// the final lexicographic argmin, type conversion and buffer fills.
#include <algorithm>

#include "eap_pairs.h"
#include "eap_screen.h"

namespace eap {

// ERP borders (eq. ERP vborder/hborder): B[i] = B[i-1] + |x_i - gap|, one
// series per thread, summed left to right like the recurrence.
__global__ void erp_border_kernel(const double* v, const int64_t* off, int64_t n, double gap, double* out) {
    constexpr int CH = 16;   // values loaded ahead of the (sequential) sum
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = off[s], e = off[s + 1];
        double acc = 0.0;
        for (int64_t x0 = b; x0 < e; x0 += CH) {
            double xv[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) xv[u] = v[x0 + u < e ? x0 + u : e - 1];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                if (x0 + u < e) {
                    acc = acc + __builtin_fabs(xv[u] - gap);
                    out[x0 + u] = acc;
                }
            }
        }
    }
}

// Derivative series (Keogh-Pazzani estimate): one block per series, series by
// grid stride.  The two ends repeat the estimate at their neighbour.
__global__ void derivative_kernel(const double* v, const int64_t* off, int64_t n, double* out) {
    for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
        const int64_t a = off[s];
        const int m = (int)(off[s + 1] - a);
        const double* q = v + a;
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            double d;
            if (m == 1) {
                d = 0.0;
            } else if (m == 2) {
                d = q[1] - q[0];
            } else {
                const int c = i < 1 ? 1 : (i > m - 2 ? m - 2 : i);
                d = ((q[c] - q[c - 1]) + (q[c + 1] - q[c - 1]) / 2.0) / 2.0;
            }
            out[a + i] = d;
        }
    }
}

// Z-normalised windows of length m (sub-sequence search candidates): one
// thread per window by grid stride, sums left to right as written.
// z-normalised windows of a series, 256 windows per block: the block's
// 256 + m - 1 values go to LDS, thread t takes the mean and standard deviation
// of window t (sums in index order), then the block writes its windows, which
// are contiguous in the output, with consecutive threads on consecutive
// doubles.  sd == 0 gives a window of zeros.
constexpr int kWinPerBlock = 256;
__global__ __launch_bounds__(256) void subseq_windows_kernel(const double* s, int64_t nw, int m, double* out) {
    extern __shared__ double xs[];   // kWinPerBlock + m - 1 values, then the means and deviations
    double* mu = xs + kWinPerBlock + m - 1;
    double* sdv = mu + kWinPerBlock;
    for (int64_t w0 = (int64_t)blockIdx.x * kWinPerBlock; w0 < nw; w0 += (int64_t)gridDim.x * kWinPerBlock) {
        const int nb = (int)(nw - w0 < kWinPerBlock ? nw - w0 : kWinPerBlock);
        __syncthreads();   // the previous tile has been written out
        for (int k = threadIdx.x; k < nb + m - 1; k += blockDim.x) xs[k] = s[w0 + k];
        __syncthreads();
        if ((int)threadIdx.x < nb) {
            const double* x = xs + threadIdx.x;
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc = acc + x[k];
            const double mean = acc / (double)m;
            double v = 0.0;
            for (int k = 0; k < m; ++k) {
                const double d = x[k] - mean;
                v = v + d * d;
            }
            mu[threadIdx.x] = mean;
            sdv[threadIdx.x] = sqrt(v / (double)m);
        }
        __syncthreads();
        double* o = out + w0 * m;
        const int tot = nb * m;
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int w = e / m, k = e - w * m;
            const double sd = sdv[w];
            o[e] = sd > 0.0 ? (xs[w + k] - mu[w]) / sd : 0.0;
        }
    }
}

// z-normalisation of each series of a ragged set, one block per series (grid
// stride): thread 0 takes the sums in index order (the order is part of the
// result: it matches subseq_windows_kernel for a window covering the whole
// series), then the block writes the series.
__global__ __launch_bounds__(256) void znorm_kernel(const double* v, const int64_t* off, int64_t n, double* out) {
    __shared__ double stat[2];
    for (int64_t a = blockIdx.x; a < n; a += gridDim.x) {
        const int64_t o = off[a];
        const int64_t L = off[a + 1] - o;
        const double* x = v + o;
        __syncthreads();   // the previous series' statistics have been used
        if (threadIdx.x == 0) {
            double acc = 0.0;
            for (int64_t k = 0; k < L; ++k) acc = acc + x[k];
            const double mean = acc / (double)L;
            double s2 = 0.0;
            for (int64_t k = 0; k < L; ++k) {
                const double d = x[k] - mean;
                s2 = s2 + d * d;
            }
            stat[0] = mean;
            stat[1] = sqrt(s2 / (double)L);
        }
        __syncthreads();
        const double mean = stat[0], sd = stat[1];
        for (int64_t k = threadIdx.x; k < L; k += blockDim.x) out[o + k] = sd > 0.0 ? (x[k] - mean) / sd : 0.0;
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

// x[i] = the next double above x[i] (+inf stays +inf): prune-only cut-offs
// from path bounds, in place.
__global__ void next_up_kernel(double* x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double u = x[i];
        if (u < __builtin_huge_val()) x[i] = bitsd(dbits(u) + 1ull);
    }
}

// Host words delivered through the kernel's argument block (no staging
// buffer, no copy call): dst[x] = w.w[x] for x < n <= kPutWords.
__global__ void put_u64_kernel(unsigned long long* dst, int n, PutWords w) {
    const int x = threadIdx.x;
    if (x < n) dst[x] = w.w[x];
}

// Cost of the warping path (1,1), (2,2), .., (m,m) followed by straight moves
// along the longer series (Section 4: any path bounds the optimum).  Every step
// adds its term exactly as the recurrence would, so the value is >= the
// distance in floating point as well.  Rows are the longer series.  The
// series are read in chunks of 16 values per lane (one or two cache lines
// each), so that a wave's lanes, each on its own series, reuse what they load.
template <int KIND>
__device__ double path_ub(const SweepArgs& A, const double* li, int Lli, const double* co, int Lco) {
    constexpr int CH = 16;
    const double INF = __builtin_huge_val();
    const int L = Lli > Lco ? Lli : Lco;
    if (KIND == CDTW || KIND == ERP) {
        const double r = A.window_ratio;
        if (r < 1.0) {
            int w = (int)floor(r * (double)L);
            if (w < Lli - Lco) return INF;
        }
    }
    double wd = 1.0;   // WDTW weight of the diagonal, w(0)
    if (KIND == WDTW) {
        int gi = -L + A.gtab_off;
        gi = gi < 0 ? 0 : (gi >= A.gtab_len ? A.gtab_len - 1 : gi);
        wd = A.gtab[gi];
    }
    double acc = 0.0;
    double sp = 0.0, tp = 0.0;
    for (int k0 = 0; k0 < Lco; k0 += CH) {
        double sv[CH], tv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int k = (k0 + u < Lco) ? k0 + u : Lco - 1;
            sv[u] = li[k];
            tv[u] = co[k];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (k0 + u < Lco) {
                const double s = sv[u], t = tv[u], d = s - t;
                if constexpr (KIND == DTW || KIND == CDTW) acc = (d * d) + acc;
                if constexpr (KIND == WDTW) acc = (wd * (d * d)) + acc;
                if constexpr (KIND == ERP || KIND == MSM) acc = acc + __builtin_fabs(d);
                if constexpr (KIND == TWE) acc = acc + ((__builtin_fabs(d) + __builtin_fabs(sp - tp)) + A.nu * 0.0);
                sp = s;
                tp = t;
            }
        }
    }
    // straight down column L_co: moves (i-1, L_co) -> (i, L_co), |i - L_co| grows
    const double t = co[Lco - 1];
    double xprev = li[Lco - 1];   // s_{i-1}
    for (int i0 = Lco + 1; i0 <= Lli; i0 += CH) {
        double sv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) sv[u] = li[(i0 + u <= Lli ? i0 + u : Lli) - 1];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int i = i0 + u;
            if (i <= Lli) {
                const double s = sv[u], d = s - t;
                if constexpr (KIND == DTW || KIND == CDTW) acc = (d * d) + acc;
                if constexpr (KIND == WDTW) {
                    int gi = 2 * (i - Lco) - L + A.gtab_off;
                    gi = gi < 0 ? 0 : (gi >= A.gtab_len ? A.gtab_len - 1 : gi);
                    acc = (A.gtab[gi] * (d * d)) + acc;
                }
                if constexpr (KIND == ERP) acc = acc + __builtin_fabs(s - A.gap);
                if constexpr (KIND == MSM) {
                    // C(s_i, s_{i-1}, t) of eq. MSMCost
                    const double x = xprev;
                    double c;
                    if ((x <= s && s <= t) || (x >= s && s >= t)) c = A.c;
                    else {
                        const double p1 = __builtin_fabs(s - x), p2 = __builtin_fabs(s - t);
                        c = A.c + (p1 < p2 ? p1 : p2);
                    }
                    acc = acc + c;
                }
                if constexpr (KIND == TWE) acc = acc + ((__builtin_fabs(s - xprev) + A.nu) + A.lam);
                xprev = s;
            }
        }
    }
    return acc;
}

// The same path cost with the series behind accessors: rowv(k) = s_{k+1} of
// the longer series, colv(k) = t_{k+1} (same terms, same order).
template <int KIND, typename FR, typename FC>
__device__ double path_ub_acc(const SweepArgs& A, FR rowv, int Lli, FC colv, int Lco) {
    const double INF = __builtin_huge_val();
    const int L = Lli > Lco ? Lli : Lco;
    if (KIND == CDTW || KIND == ERP) {
        const double r = A.window_ratio;
        if (r < 1.0) {
            int w = (int)floor(r * (double)L);
            if (w < Lli - Lco) return INF;
        }
    }
    double wd = 1.0;
    if (KIND == WDTW) {
        int gi = -L + A.gtab_off;
        gi = gi < 0 ? 0 : (gi >= A.gtab_len ? A.gtab_len - 1 : gi);
        wd = A.gtab[gi];
    }
    double acc = 0.0, sp = 0.0, tp = 0.0;
    for (int k = 0; k < Lco; ++k) {
        const double s = rowv(k), t = colv(k), d = s - t;
        if constexpr (KIND == DTW || KIND == CDTW) acc = (d * d) + acc;
        if constexpr (KIND == WDTW) acc = (wd * (d * d)) + acc;
        if constexpr (KIND == ERP || KIND == MSM) acc = acc + __builtin_fabs(d);
        if constexpr (KIND == TWE) acc = acc + ((__builtin_fabs(d) + __builtin_fabs(sp - tp)) + A.nu * 0.0);
        sp = s;
        tp = t;
    }
    const double t = colv(Lco - 1);
    double xprev = rowv(Lco - 1);
    for (int i = Lco + 1; i <= Lli; ++i) {
        const double s = rowv(i - 1), d = s - t;
        if constexpr (KIND == DTW || KIND == CDTW) acc = (d * d) + acc;
        if constexpr (KIND == WDTW) {
            int gi = 2 * (i - Lco) - L + A.gtab_off;
            gi = gi < 0 ? 0 : (gi >= A.gtab_len ? A.gtab_len - 1 : gi);
            acc = (A.gtab[gi] * (d * d)) + acc;
        }
        if constexpr (KIND == ERP) acc = acc + __builtin_fabs(s - A.gap);
        if constexpr (KIND == MSM) {
            const double x = xprev;
            double c;
            if ((x <= s && s <= t) || (x >= s && s >= t)) c = A.c;
            else {
                const double p1 = __builtin_fabs(s - x), p2 = __builtin_fabs(s - t);
                c = A.c + (p1 < p2 ? p1 : p2);
            }
            acc = acc + c;
        }
        if constexpr (KIND == TWE) acc = acc + ((__builtin_fabs(s - xprev) + A.nu) + A.lam);
        xprev = s;
    }
    return acc;
}

// Candidates interleaved for coalesced reads: rT[k * nr + b] = value k of
// candidate b (0 past its end).
// A tile of 64 series x 64 positions per block, through LDS: each wave reads
// 64 consecutive values of one series and writes 64 consecutive series of one
// position.  Grid: (ceil(nr / 64), ceil(lmax / 64)), 256 threads.
__global__ __launch_bounds__(256) void interleave_kernel(const double* rv, const int64_t* roff, int64_t nr, int lmax,
                                                         double* rT, float* r32, unsigned long long* absmax) {
    __shared__ double tile[64][65];
    __shared__ double part[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * 64;
    const int k0 = blockIdx.y * 64;
    // wave w reads candidates b0 + w + 4 ii: offsets first, then all 16 loads
    // in flight, then the tile (and, when asked, the FP32 copy in the input's
    // own layout and the largest |x|)
    int64_t o[16];
    int len[16];
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) {
        const int64_t b = b0 + w + 4 * ii;
        o[ii] = b < nr ? roff[b] : 0;
        len[ii] = b < nr ? (int)(roff[b + 1] - o[ii]) : 0;
    }
    double v[16];
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) v[ii] = (k0 + lane < len[ii]) ? rv[o[ii] + k0 + lane] : 0.0;
    double m = 0.0;
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) {
        tile[w + 4 * ii][lane] = v[ii];
        if (r32 && k0 + lane < len[ii]) r32[o[ii] + k0 + lane] = (float)v[ii];
        m = fmax(m, __builtin_fabs(v[ii]));
    }
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) {
        const int k = k0 + w + 4 * ii;
        const int64_t b = b0 + lane;
        if (rT && k < lmax && b < nr) rT[(int64_t)k * nr + b] = tile[lane][w + 4 * ii];
    }
    if (absmax) {
        for (int s = 32; s > 0; s >>= 1) m = fmax(m, __shfl_xor(m, s));
        if (lane == 0) part[w] = m;
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(absmax, dbits(fmax(fmax(part[0], part[1]), fmax(part[2], part[3]))));
    }
}

// Envelopes for LB_Keogh (Section 2.1; Section 5.2 computes them in O(L) with
// Lemire's streaming algorithm).  For series s of a ragged set and positions
// j = 1..npos: up_j / lo_j = max / min of s_i over i in [j-w, j+w] and
// [1, L_s], with w = floor(ratio * max(L_s, other_max)), the widest window of
// any pair of s (a wider window only loosens the bound); a position whose
// range is empty (j > L_s + w) gets (+inf, -inf), which adds nothing.
//
// O(L) on the GPU without a sequential deque: the van Herk / Gil-Werman
// decomposition.  Padded with the operation's identity to P[0 .. M), M =
// npos + 2w, every window is the k = 2w + 1 entries P[j-1 .. j-1+2w]; with
// P cut into blocks of k, g[p] = max of P from p's block start to p and
// h[p] = max from p to its block end, the window's max is max(h[j-1],
// g[j-1+2w]) (one block boundary inside).  Both are segmented scans: 256
// threads take consecutive chunks, scan them, pass the carries across
// chunks with a segmented Hillis-Steele scan in LDS, and rescan.  Three
// comparisons per entry for each of max and min.  One block per series; w
// at or above max(L_s, npos) is clamped there (the window then covers the
// whole series).  Results are copies of input values, so the layout of the
// arithmetic cannot change them.
//
// Layout: out[s * s_stride + (j-1) * p_stride]; with qx != NULL also the
// series extended by its last value, qx[..] = s_{min(j, L_s)}.
template <bool MAX>
__device__ __forceinline__ double env_op(double a, double b) { return MAX ? fmax(a, b) : fmin(a, b); }

template <bool MAX>
__device__ void env_pass(const double* v, int L, int w, int npos, int M, double* g, double* h, double* out,
                         int64_t p_stride, double* carry, unsigned char* head) {
    const double ID = MAX ? -__builtin_huge_val() : __builtin_huge_val();
    const int k = 2 * w + 1;
    const int T = blockDim.x, t = threadIdx.x;
    const int E = (M + T - 1) / T, p0 = t * E, p1 = p0 + E < M ? p0 + E : M;
    auto P = [&](int p) { return (p >= w && p - w < L) ? v[p - w] : ID; };
    // forward: prefix within blocks of k (heads at p % k == 0)
    double run = ID;
    bool hd = false;
    for (int p = p0; p < p1; ++p) {
        const double x = P(p);
        if (p % k == 0) {
            run = x;
            hd = true;
        } else {
            run = env_op<MAX>(run, x);
        }
        g[p] = run;
    }
    carry[t] = run;
    head[t] = hd ? 1 : 0;
    __syncthreads();
    for (int o = 1; o < T; o <<= 1) {   // inclusive segmented scan of (head, value) over the chunks
        const double cv = t >= o ? carry[t - o] : ID;
        const unsigned char ch = t >= o ? head[t - o] : 1;
        __syncthreads();
        if (t >= o && !head[t]) {
            carry[t] = env_op<MAX>(cv, carry[t]);
            head[t] = ch;
        }
        __syncthreads();
    }
    const double cin = t > 0 ? carry[t - 1] : ID;   // the block's part before this chunk
    for (int p = p0; p < p1 && p % k != 0; ++p) g[p] = env_op<MAX>(cin, g[p]);
    __syncthreads();
    // backward: suffix within blocks (heads at block ends: p % k == k - 1 or p == M - 1)
    run = ID;
    hd = false;
    for (int p = p1 - 1; p >= p0; --p) {
        const double x = P(p);
        if (p % k == k - 1 || p == M - 1) {
            run = x;
            hd = true;
        } else {
            run = env_op<MAX>(run, x);
        }
        h[p] = run;
    }
    carry[t] = run;
    head[t] = hd ? 1 : 0;
    __syncthreads();
    for (int o = 1; o < T; o <<= 1) {   // the same scan from the right
        const double cv = t + o < T ? carry[t + o] : ID;
        const unsigned char ch = t + o < T ? head[t + o] : 1;
        __syncthreads();
        if (t + o < T && !head[t]) {
            carry[t] = env_op<MAX>(cv, carry[t]);
            head[t] = ch;
        }
        __syncthreads();
    }
    const double cout = t + 1 < T ? carry[t + 1] : ID;
    for (int p = p1 - 1; p >= p0 && !(p % k == k - 1 || p == M - 1); --p) h[p] = env_op<MAX>(cout, h[p]);
    __syncthreads();
    for (int j = t; j < npos; j += T) {
        const int e = j + k - 1 < M ? j + k - 1 : M - 1;
        double r = env_op<MAX>(h[j], g[e]);
        if (j + 1 - w > L) r = -ID;   // empty range: up = +inf, lo = -inf
        out[(int64_t)j * p_stride] = r;
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void envelope_kernel(const double* v, const int64_t* off, int64_t n, int npos,
                                                       int other_max, double ratio, double* up, double* lo,
                                                       double* qx, int64_t s_stride, int64_t p_stride) {
    extern __shared__ double env_lds[];
    __shared__ double carry[256];
    __shared__ unsigned char head[256];
    for (int64_t a = blockIdx.x; a < n; a += gridDim.x) {
        const double* x = v + off[a];
        const int L = (int)(off[a + 1] - off[a]);
        const int Lw = L > other_max ? L : other_max;
        const int cap = L > npos ? L : npos;
        int w = ratio >= 1.0 ? cap : (int)floor(ratio * (double)Lw);
        w = w > cap ? cap : w;
        const int M = npos + 2 * w;
        double* g = env_lds;
        double* h = env_lds + M;
        env_pass<true>(x, L, w, npos, M, g, h, up + a * s_stride, p_stride, carry, head);
        env_pass<false>(x, L, w, npos, M, g, h, lo + a * s_stride, p_stride, carry, head);
        if (qx)
            for (int j = threadIdx.x; j < npos; j += blockDim.x)
                qx[a * s_stride + (int64_t)j * p_stride] = x[(j + 1 < L ? j + 1 : L) - 1];
    }
}

// Reversed LB_Keogh ("lb-keogh2", Section 5.2): for the pairs listed by the
// first bound, the candidate's envelope against the query's values.  Every
// path visits each row i of the query at a column within the candidate's
// window of i, so D >= sum_i dist(q_i, [clo_i, cup_i])^2; as in the first
// bound, the first and last rows take the exact costs of the corner cells
// (1,1) and (L_q, L_r), which every path contains (LB_Kim).  The pair keeps
// the larger of its two bounds.  Candidate envelopes are interleaved
// (cup[i * nr + b]), so lanes on consecutive candidates read consecutive
// addresses.  One lane per listed pair, grid-stride up to the device count.
__global__ __launch_bounds__(256) void lb_reverse_kernel(const double* qv, const int64_t* qoff, const double* rv,
                                                         const int64_t* roff, int64_t nr, const double* cup,
                                                         const double* clo, const int32_t* items,
                                                         const unsigned int* count, double* lb) {
    const int64_t n = (int64_t)*count;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = items[x];
        const int64_t a = p / nr, b = p - a * nr;
        const double* q = qv + qoff[a];
        const int lq = (int)(qoff[a + 1] - qoff[a]);
        const double* r = rv + roff[b];
        const int lr = (int)(roff[b + 1] - roff[b]);
        double s = 0.0;
        for (int i = 0; i < lq; ++i) {
            const double y = q[i];
            const double e = fmax(fmax(y - cup[(int64_t)i * nr + b], clo[(int64_t)i * nr + b] - y), 0.0);
            s = s + e * e;
        }
        // corners: row 1 holds (1,1), row L_q holds (L_q, L_r)
        const double d1 = q[0] - r[0], dL = q[lq - 1] - r[lr - 1];
        const double e1 = fmax(fmax(q[0] - cup[b], clo[b] - q[0]), 0.0);
        s = s + (d1 * d1 - e1 * e1);
        if (lq >= 2) {
            const double eL = fmax(fmax(q[lq - 1] - cup[(int64_t)(lq - 1) * nr + b], clo[(int64_t)(lq - 1) * nr + b] -
                                                                                          q[lq - 1]),
                                   0.0);
            s = s + (dL * dL - eL * eL);
        } else if (lr >= 2) {
            s = s + dL * dL;   // row 1 also holds (1, L_r)
        }
        lb[p] = fmax(lb[p], s);
    }
}

// UB of every (query, candidate) pair from the interleaved candidates: the
// terms of path_ub_acc in its order, for QT queries per pass over 256
// candidates per block (a lane per candidate, its values read once, coalesced,
// for all QT queries; query values by scalar loads).  The position loop is
// uniform over the wave: the diagonal terms depend on the two values only
// through |d| or d^2 (d and -d round alike), so they are formed from the pair
// (q_k, r_k) whatever the orientation, and past the shorter series' end the
// clamped index repeats its last value, which is the tail's fixed column
// value.  Only the tail terms of ERP, MSM and TWE, which also depend on the
// longer series' own previous value, pick the longer series by a select.
template <int KIND, int QT>
__global__ __launch_bounds__(256) void ub_nn_t_kernel(SweepArgs A, const double* qv, const int64_t* qoff,
                                                      const double* rT, const int64_t* roff, int lr_max, int ltab,
                                                      double* ub) {
    typedef const __attribute__((address_space(4))) double* cdp;
    typedef const __attribute__((address_space(4))) int64_t* cip;
    // WDTW: the weights of m = -ltab .. ltab (every m = 2|d| - L a pair of
    // these lengths forms) copied to LDS, gsh[m + ltab]: the tail's weight is a
    // different entry for every lane, an LDS read instead of a global gather
    extern __shared__ double gsh[];
    if constexpr (KIND == WDTW) {
        for (int i = threadIdx.x; i <= 2 * ltab; i += blockDim.x) gsh[i] = A.gtab[A.gtab_off - ltab + i];
        __syncthreads();
    }
    const int64_t nB = A.nB;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = b < nB;
    const int64_t bb = live ? b : nB - 1;   // lanes past the end read the last candidate, store nothing
    const int lr = (int)(roff[bb + 1] - roff[bb]);
    int lw = lr;   // the wave's longest candidate
    for (int o = 32; o > 0; o >>= 1) lw = max(lw, __shfl_xor(lw, o));
    lw = __builtin_amdgcn_readfirstlane(lw);
    const double rlast = rT[(int64_t)(lr - 1) * nB + bb];
    const double ratio = A.window_ratio;
    const cip qo = (cip)qoff;
    const cdp qc = (cdp)qv;
    for (int64_t a0 = (int64_t)blockIdx.y * QT; a0 < A.nA; a0 += (int64_t)gridDim.y * QT) {
        const int nqt = (int)((A.nA - a0) < QT ? (A.nA - a0) : QT);
        int64_t qb[QT];
        int lq[QT], Lco[QT], Lli[QT];
        double acc[QT], sp[QT], wd[QT];
        bool feasible[QT];
        int kmax = lw;
#pragma unroll
        for (int t = 0; t < QT; ++t) {
            qb[t] = t < nqt ? qo[a0 + t] : 0;
            lq[t] = t < nqt ? (int)(qo[a0 + t + 1] - qb[t]) : 1;
            kmax = kmax > lq[t] ? kmax : lq[t];
            Lco[t] = lq[t] < lr ? lq[t] : lr;
            Lli[t] = lq[t] < lr ? lr : lq[t];
            feasible[t] = true;
            if constexpr (KIND == CDTW || KIND == ERP)
                if (ratio < 1.0 && (int)floor(ratio * (double)Lli[t]) < Lli[t] - Lco[t]) feasible[t] = false;
            wd[t] = 1.0;
            if constexpr (KIND == WDTW) {
                int gi = -Lli[t] + A.gtab_off;
                gi = gi < 0 ? 0 : (gi >= A.gtab_len ? A.gtab_len - 1 : gi);
                wd[t] = A.gtab[gi];
            }
            acc[t] = 0.0;
            sp[t] = 0.0;
        }
        if constexpr (KIND == DTW || KIND == CDTW || KIND == WDTW) {
            constexpr int CH = 2;
            // The squared costs, a chunk of CH positions at a time: the candidate
            // values (coalesced loads) and the queries' values (scalar loads) are
            // all issued before any is used, and each term enters its sum through
            // a select, so no branch sits between a load and its use (a branch
            // around each term would hold each query value's load until its use).
            // A full tile of QT queries runs without a per-query guard.
            auto chunk = [&](int k0, auto full_tag) {
                constexpr bool FULL = decltype(full_tag)::value;
                double rv[CH], qv[QT][CH];
                // past its end a lane reads its own last value (the tail's fixed
                // column value): the index is clamped, the load unconditional
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int k = k0 + u;
                    rv[u] = rT[(int64_t)(k < lr ? k : lr - 1) * nB + bb];
                }
#pragma unroll
                for (int t = 0; t < QT; ++t) {
                    if (!FULL && t >= nqt) continue;
#pragma unroll
                    for (int u = 0; u < CH; ++u) {
                        const int k = k0 + u;
                        qv[t][u] = qc[qb[t] + (k < lq[t] ? k : lq[t] - 1)];
                    }
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int k = k0 + u;
                    const double r = rv[u];
#pragma unroll
                    for (int t = 0; t < QT; ++t) {
                        if (!FULL && t >= nqt) continue;
                        const double q = qv[t][u];
                        const bool dg = k < Lco[t], tl = !dg && k < Lli[t];
                        const double d = q - r;
                        double term = 0.0;
                        if constexpr (KIND == DTW || KIND == CDTW) term = d * d;
                        if constexpr (KIND == WDTW) {
                            // a tail cell's m lies in 2 - L .. L; others read a clamped entry
                            int gi = 2 * (k + 1 - Lco[t]) - Lli[t] + ltab;
                            gi = gi < 0 ? 0 : (gi > 2 * ltab ? 2 * ltab : gi);
                            const double wt = gsh[gi];
                            term = (tl ? wt : wd[t]) * (d * d);
                        }
                        const double na = term + acc[t];
                        acc[t] = (dg || tl) ? na : acc[t];
                    }
                }
            };
            if (nqt == QT) {
                for (int k0 = 0; k0 < kmax; k0 += CH) chunk(k0, std::true_type{});
            } else {
                for (int k0 = 0; k0 < kmax; k0 += CH) chunk(k0, std::false_type{});
            }
        } else {
            // ERP, MSM and TWE: one query load per term (their tail terms also
            // take the longer series' previous value, and batching their loads
            // costs more registers than it saves)
            // TWE: |q_{k-1} - r_{k-1}|, the previous position's |d| (0 before the first)
            double adp[KIND == TWE ? QT : 1];
#pragma unroll
            for (int t = 0; t < (KIND == TWE ? QT : 1); ++t) adp[t] = 0.0;
            constexpr int CH = 4;
            for (int k0 = 0; k0 < kmax; k0 += CH) {
                double rv[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int k = k0 + u;
                    rv[u] = (k < lr) ? rT[(int64_t)(k < lr_max ? k : lr_max - 1) * nB + bb] : rlast;
                }
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    const int k = k0 + u;
                    const double r = rv[u];
#pragma unroll
                    for (int t = 0; t < QT; ++t) {
                        if (t >= nqt) continue;
                        const int kq = k < lq[t] ? k : lq[t] - 1;
                        const double q = qc[qb[t] + kq];
                        const bool dg = k < Lco[t], tl = !dg && k < Lli[t];
                        const double d = q - r;
                        double term = 0.0;
                        // the longer series' value (rows of the path) and the previous one
                        const double s = (lq[t] >= lr) ? q : r;
                        if constexpr (KIND == ERP) term = dg ? __builtin_fabs(d) : __builtin_fabs(s - A.gap);
                        if constexpr (KIND == MSM) {
                            // C(s_i, s_{i-1}, t) of eq. MSMCost, t the shorter series'
                            // last value: c, plus the distance from s to the nearer end
                            // of [min(x, t), max(x, t)] when s lies outside it (that
                            // end's rounded difference is the smaller of the two, so
                            // the value equals the case-by-case form), without branches
                            const double x = sp[t], tt = (lq[t] >= lr) ? r : q;
                            const double lo = fmin(x, tt), hi = fmax(x, tt);
                            const double tail = A.c + fmax(fmax(lo - s, s - hi), 0.0);
                            term = dg ? __builtin_fabs(d) : tail;
                        }
                        if constexpr (KIND == TWE) {
                            // the match's second difference is the previous position's
                            // (the same operands, so the same rounded value)
                            term = dg ? ((__builtin_fabs(d) + adp[t < (KIND == TWE ? QT : 1) ? t : 0]) + A.nu * 0.0)
                                      : ((__builtin_fabs(s - sp[t]) + A.nu) + A.lam);
                            adp[t < (KIND == TWE ? QT : 1) ? t : 0] = __builtin_fabs(d);
                        }
                        if (dg || tl) acc[t] = acc[t] + term;
                        sp[t] = s;
                    }
                }
            }
        }
        if (live) {
#pragma unroll
            for (int t = 0; t < QT; ++t)
                if (t < nqt) ub[(a0 + t) * nB + b] = feasible[t] ? acc[t] : __builtin_huge_val();
        }
    }
}

// DTW and CDTW: the path bound and LB_Keogh (with LB_Kim's exact corner
// cells) of QT queries against 256 candidates per block, in one pass over each
// candidate's values (read once for all QT queries; query values and
// envelopes by scalar loads).  For DTW the envelope is the query's range.  The candidates come
// from the interleaved copy rT (coalesced), or with rv != NULL from their own
// layout: a lane takes 8 consecutive values of its candidate per chunk, which
// for very large candidate sets costs less than building the copy.  Each bound adds its
// terms in path order (the diagonal, then the longer series' tail), like
// path_ub_acc; (a - b)^2 and (b - a)^2 are the same double.
template <int QT>
__global__ __launch_bounds__(256) void ub_lb_kernel(SweepArgs A, const double* qv, const int64_t* qoff,
                                                         const double* rv, const double* rT, const int64_t* roff,
                                                         int64_t ld,
                                                         const double* env_up, const double* env_lo,
                                                         const double* env_q, double* lb, double* ub) {
    // Every lane of a wave reads the same query value and envelope entries:
    // through the constant address space they arrive by scalar loads, one per
    // wave, and enter the arithmetic as scalar operands.  Nothing this kernel
    // writes is read through these pointers.
    typedef double d8 __attribute__((ext_vector_type(8)));
    typedef const __attribute__((address_space(4))) d8* cd8p;
    typedef const __attribute__((address_space(4))) int64_t* cip;
    const int64_t nB = A.nB;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = b < nB;
    const int64_t bb = live ? b : nB - 1;   // lanes past the end read the last candidate, store nothing
    const int64_t ro = roff[bb];
    const int lr = (int)(roff[bb + 1] - ro);
    int lw = lr, ln = lr;   // the wave's longest and shortest candidates: the column loops are uniform
    for (int o = 32; o > 0; o >>= 1) {
        lw = max(lw, __shfl_xor(lw, o));
        ln = min(ln, __shfl_xor(ln, o));
    }
    lw = __builtin_amdgcn_readfirstlane(lw);
    ln = __builtin_amdgcn_readfirstlane(ln);
    const double ratio = A.window_ratio;
    const cip qo = (cip)qoff;
    for (int64_t a0 = (int64_t)blockIdx.y * QT; a0 < A.nA; a0 += (int64_t)gridDim.y * QT) {
        const int nqt = (int)((A.nA - a0) < QT ? (A.nA - a0) : QT);
        int64_t qb[QT];
        int lq[QT];
        double acc[QT], lbv[QT];
#pragma unroll
        for (int t = 0; t < QT; ++t) {
            qb[t] = t < nqt ? qo[a0 + t] : 0;
            lq[t] = t < nqt ? (int)(qo[a0 + t + 1] - qb[t]) : 1;
            const int L = lq[t] > lr ? lq[t] : lr, ld = lq[t] > lr ? lq[t] - lr : lr - lq[t];
            acc[t] = (ratio < 1.0 && (int)floor(ratio * (double)L) < ld) ? __builtin_huge_val() : 0.0;   // +inf: no path
            lbv[t] = 0.0;
        }
        // candidate values in chunks of CH (loads issued together, indexes
        // clamped into the series); the query extended by its last value and
        // the envelopes come in aligned chunks of 8 from rows of ld >= lw
        // entries, so their reads need no clamp; terms added in order.  Chunks
        // inside every lane's candidate (j0 + CH <= ln) need no mask; in the
        // others a column past a candidate's end adds +0 (the sums are >= 0,
        // so they do not change), by selects rather than per-lane branches.  A
        // full group of QT queries runs without a per-query guard, so the
        // compiler can issue the next queries' scalar loads while it computes.
        constexpr int CH = 8;
        auto chunk = [&](int j0, auto full_tag, auto mask_tag) {
            constexpr bool FULL = decltype(full_tag)::value, MASK = decltype(mask_tag)::value;
            double xv[CH];
            bool in[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                in[u] = !MASK || j0 + u < lr;
                const int jj = in[u] ? j0 + u : lr - 1;
                xv[u] = rv ? rv[ro + jj] : rT[(int64_t)jj * nB + bb];
            }
#pragma unroll
            for (int t = 0; t < QT; ++t) {
                if (!FULL && t >= nqt) continue;
                const int64_t base = (a0 + t) * ld + j0;
                const d8 Y = *(cd8p)(env_q + base), U = *(cd8p)(env_up + base), O = *(cd8p)(env_lo + base);
#pragma unroll
                for (int u = 0; u < CH; ++u) {
                    // the diagonal while both series last, then down the candidate
                    const double x = xv[u];
                    const double d = x - Y[u];
                    const double e = fmax(fmax(x - U[u], O[u] - x), 0.0);   // at most one side is positive
                    if (MASK) {
                        acc[t] = (in[u] ? d * d : 0.0) + acc[t];
                        lbv[t] = lbv[t] + (in[u] ? e * e : 0.0);
                    } else {
                        acc[t] = (d * d) + acc[t];
                        lbv[t] = lbv[t] + e * e;
                    }
                }
            }
        };
        auto sweep = [&](auto full_tag) {
            int j0 = 0;
            for (; j0 + CH <= ln; j0 += CH) chunk(j0, full_tag, std::false_type{});
            for (; j0 < lw; j0 += CH) chunk(j0, full_tag, std::true_type{});
        };
        if (nqt == QT) sweep(std::true_type{});
        else sweep(std::false_type{});
        // queries longer than the candidate: their tail against its last value
        // (not for a pair whose window admits no path: its bound stays +inf, and
        // the wave's loop then runs only as long as its feasible pairs' tails)
        const double xl = rv ? rv[ro + lr - 1] : rT[(int64_t)(lr - 1) * nB + bb];
#pragma unroll
        for (int t = 0; t < QT; ++t) {
            if (t >= nqt) continue;
            const int iend = (acc[t] < __builtin_huge_val()) ? lq[t] : lr;
            for (int i = lr; i < iend; ++i) {
                const double d = qv[qb[t] + i] - xl;
                acc[t] = (d * d) + acc[t];
            }
        }
        // LB_Kim (first and last points): the first and last columns take the
        // exact costs of the cells (1,1) and (L_q, L_r) that every path holds,
        // in place of their envelope terms (which are no larger: for a
        // feasible pair q_1 and q_{L_q} lie in those columns' ranges)
        const double x1 = rv ? rv[ro] : rT[bb];
#pragma unroll
        for (int t = 0; t < QT; ++t) {
            if (t >= nqt) continue;
            const int64_t eb = (a0 + t) * ld;
            const double q1 = qv[qb[t]], qL = qv[qb[t] + lq[t] - 1];
            const double e1 = fmax(fmax(x1 - env_up[eb], env_lo[eb] - x1), 0.0);
            const double d1 = x1 - q1, dL = xl - qL;
            double c = d1 * d1 - e1 * e1;
            if (lr >= 2) {
                const double eL = fmax(fmax(xl - env_up[eb + lr - 1], env_lo[eb + lr - 1] - xl), 0.0);
                c = c + (dL * dL - eL * eL);
            } else if (lq[t] >= 2) {
                c = c + dL * dL;   // column 1 also holds (L_q, 1)
            }
            lbv[t] = lbv[t] + c;
        }
        if (live) {
#pragma unroll
            for (int t = 0; t < QT; ++t) {
                if (t < nqt) {
                    ub[(a0 + t) * nB + b] = acc[t];
                    lb[(a0 + t) * nB + b] = lbv[t];
                }
            }
        }
    }
}

template <int KIND>
__device__ __forceinline__ double pair_ub(const SweepArgs& A, const double* x, int lx, const double* y, int ly) {
    return (lx >= ly) ? path_ub<KIND>(A, x, lx, y, ly) : path_ub<KIND>(A, y, ly, x, lx);
}

// The next double above a non-negative value (+inf stays +inf): its bit
// pattern plus one, since non-negative doubles order like their bits.
__device__ __forceinline__ double next_up(double u) {
    if (!(u < __builtin_huge_val())) return u;
    return bitsd(dbits(u) + 1ull);
}

// Prune-only cut-off for every condensed pair: one ulp above its path bound.
template <int KIND>
__global__ void ub_condensed_kernel(SweepArgs A, const double* v, const int64_t* off, int64_t n, double* cut) {
    const int64_t total = n * (n - 1) / 2;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        int64_t i, j;
        condensed_ij(p, n, i, j);
        const double* x = v + off[i];
        const double* y = v + off[j];
        const int lx = (int)(off[i + 1] - off[i]), ly = (int)(off[j + 1] - off[j]);
        cut[p] = next_up(pair_ub<KIND>(A, x, lx, y, ly));
    }
}

// Multivariate DTW and CDTW (points of ND channels, stored point after
// point): the same diagonal-then-straight path, each step's cost the
// channels' squared differences added in channel order, as the sweep adds
// them.  One thread per pair.
template <int KIND, int ND>
__device__ double path_ub_mv(const SweepArgs& A, const double* li, int Lli, const double* co, int Lco) {
    if (KIND == CDTW && A.window_ratio < 1.0) {
        const int w = (int)floor(A.window_ratio * (double)Lli);
        if (w < Lli - Lco) return __builtin_huge_val();
    }
    auto cost = [&](int i, int j) {
        const double* a = li + (int64_t)i * ND;
        const double* b = co + (int64_t)j * ND;
        double d = a[0] - b[0];
        double c = d * d;
#pragma unroll
        for (int ch = 1; ch < ND; ++ch) {
            const double e = a[ch] - b[ch];
            c = c + e * e;
        }
        return c;
    };
    double acc = 0.0;
    for (int k = 0; k < Lco; ++k) acc = cost(k, k) + acc;
    for (int i = Lco; i < Lli; ++i) acc = cost(i, Lco - 1) + acc;
    return acc;
}

template <int KIND, int ND>
__device__ __forceinline__ double pair_ub_mv(const SweepArgs& A, const double* x, int lx, const double* y, int ly) {
    return (lx >= ly) ? path_ub_mv<KIND, ND>(A, x, lx, y, ly) : path_ub_mv<KIND, ND>(A, y, ly, x, lx);
}

template <int KIND, int ND>
__global__ void ub_nn_mv_kernel(SweepArgs A, const double* qv, const int64_t* qoff, const double* rv,
                                const int64_t* roff, double* ub) {
    const int64_t total = A.nA * A.nB;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = p / A.nB, b = p - a * A.nB;
        ub[p] = pair_ub_mv<KIND, ND>(A, qv + qoff[a] * ND, (int)(qoff[a + 1] - qoff[a]), rv + roff[b] * ND,
                                     (int)(roff[b + 1] - roff[b]));
    }
}

template <int KIND, int ND>
__global__ void ub_condensed_mv_kernel(SweepArgs A, const double* v, const int64_t* off, int64_t n, double* cut) {
    const int64_t total = n * (n - 1) / 2;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        int64_t i, j;
        condensed_ij(p, n, i, j);
        cut[p] = next_up(pair_ub_mv<KIND, ND>(A, v + off[i] * ND, (int)(off[i + 1] - off[i]), v + off[j] * ND,
                                               (int)(off[j + 1] - off[j])));
    }
}

// Per-query scans over the nr candidates (seed choice, argmin, screen
// filter): TPQ threads per query (64, 256 or 1024, from nr), a block of
// max(256, TPQ) threads holding 256 / TPQ queries when TPQ < 256; queries by
// grid stride.  Lexicographic (value, index) minima: the combination of two
// partial minima is associative, so the order of the reduction does not
// change the result.
__device__ __forceinline__ bool lex_less(double v, int64_t i, double bv, int64_t bi) {
    return v < bv || (v == bv && i >= 0 && (bi < 0 || i < bi));
}

template <int TPQ>
__device__ __forceinline__ void group_min(double& bv, int64_t& bi, double* sv, int64_t* si) {
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o);
        const int64_t oi = __shfl_xor(bi, o);
        if (lex_less(ov, oi, bv, bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if constexpr (TPQ > 64) {
        // one query per block: the waves' minima through LDS, the result to all
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            sv[threadIdx.x >> 6] = bv;
            si[threadIdx.x >> 6] = bi;
        }
        __syncthreads();
        bv = sv[0];
        bi = si[0];
        for (int w = 1; w < TPQ / 64; ++w)
            if (lex_less(sv[w], si[w], bv, bi)) {
                bv = sv[w];
                bi = si[w];
            }
    }
}

// Per query: the candidate with the smallest upper bound (lowest index on
// ties) is swept first, with that bound as its cut-off.
template <int TPQ>
__global__ void seed_kernel(const double* ub, int64_t nq, int64_t nr, int32_t* seed_b, int32_t* items,
                            unsigned long long* best) {
    constexpr int QPB = TPQ >= 256 ? 1 : 256 / TPQ;
    __shared__ double sv[TPQ / 64];
    __shared__ int64_t si[TPQ / 64];
    const int tq = threadIdx.x % TPQ;
    for (int64_t q0 = (int64_t)blockIdx.x * QPB; q0 < nq; q0 += (int64_t)gridDim.x * QPB) {
        const int64_t q = q0 + threadIdx.x / TPQ;
        double bv = __builtin_huge_val();
        int64_t bi = -1;
        if (q < nq)
            for (int64_t r = tq; r < nr; r += TPQ) {
                const double u = ub[q * nr + r];
                if (lex_less(u, r, bv, bi)) {
                    bv = u;
                    bi = r;
                }
            }
        group_min<TPQ>(bv, bi, sv, si);
        if (tq == 0 && q < nq) {
            if (bi < 0) bi = 0;   // every bound +inf: any candidate, cut-off +inf
            seed_b[q] = (int32_t)bi;
            items[q] = (int32_t)(q * nr + bi);
            best[q] = dbits(bv);
        }
    }
}

// Alg. 1's result: the lexicographically smallest (distance, index) per query;
// index -1 and +inf when no candidate is finite.
template <int TPQ>
__global__ void argmin_kernel(const double* res, int64_t nq, int64_t nr, const int32_t* labels, int64_t* out_idx,
                              double* out_dist, int32_t* out_label) {
    constexpr int QPB = TPQ >= 256 ? 1 : 256 / TPQ;
    __shared__ double sv[TPQ / 64];
    __shared__ int64_t si[TPQ / 64];
    const int tq = threadIdx.x % TPQ;
    for (int64_t q0 = (int64_t)blockIdx.x * QPB; q0 < nq; q0 += (int64_t)gridDim.x * QPB) {
        const int64_t q = q0 + threadIdx.x / TPQ;
        double bv = __builtin_huge_val();
        int64_t bi = -1;
        if (q < nq)
            for (int64_t r = tq; r < nr; r += TPQ) {
                const double d = res[q * nr + r];
                if (d < bv) {   // r increases per thread, so strict '<' keeps the lowest index
                    bv = d;
                    bi = r;
                }
            }
        group_min<TPQ>(bv, bi, sv, si);
        if (tq == 0 && q < nq) {
            out_idx[q] = bi;
            out_dist[q] = bv;
            if (out_label) out_label[q] = (bi >= 0 && labels) ? labels[bi] : -1;
        }
    }
}

// A few queries with many candidates: each query's scan is split over S
// blocks, block (c, q) reducing chunk c to a (value, index) minimum, and a
// finishing pass (one wave per query) reduces the chunks.  MODE 0 is the seed
// scan (lexicographic over every value, +inf included), MODE 1 the NN argmin
// (finite values only); the result equals the single-pass kernels' since the
// lexicographic minimum is associative.
template <int MODE>
__global__ __launch_bounds__(256) void scan_part_kernel(const double* v, int64_t nr, int S, double* pv,
                                                        int64_t* pi) {
    __shared__ double sv[4];
    __shared__ int64_t si[4];
    const int64_t q = blockIdx.y;
    const int64_t per = (nr + S - 1) / S, r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < nr ? r0 + per : nr;
    double bv = __builtin_huge_val();
    int64_t bi = -1;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const double u = v[q * nr + r];
        if (MODE == 0 ? lex_less(u, r, bv, bi) : u < bv) {
            bv = u;
            bi = r;
        }
    }
    group_min<256>(bv, bi, sv, si);
    if (threadIdx.x == 0) {
        pv[q * S + blockIdx.x] = bv;
        pi[q * S + blockIdx.x] = bi;
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void scan_finish_kernel(const double* pv, const int64_t* pi, int64_t nq, int S,
                                                          int64_t nr, int32_t* seed_b, int32_t* items,
                                                          unsigned long long* best, const int32_t* labels,
                                                          int64_t* out_idx, double* out_dist, int32_t* out_label) {
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double bv = __builtin_huge_val();
    int64_t bi = -1;
    if (q < nq)
        for (int c = lane; c < S; c += 64)
            if (lex_less(pv[q * S + c], pi[q * S + c], bv, bi)) {
                bv = pv[q * S + c];
                bi = pi[q * S + c];
            }
    group_min<64>(bv, bi, nullptr, nullptr);
    if (lane != 0 || q >= nq) return;
    if (MODE == 0) {
        if (bi < 0) bi = 0;   // every bound +inf: any candidate, cut-off +inf
        seed_b[q] = (int32_t)bi;
        items[q] = (int32_t)(q * nr + bi);
        best[q] = dbits(bv);
    } else {
        out_idx[q] = bi;
        out_dist[q] = bv;
        if (out_label) out_label[q] = (bi >= 0 && labels) ? labels[bi] : -1;
    }
}

constexpr int kCompactPer = 8192;   // candidates per block of lb_compact_kernel (4 waves x 64 lanes x 32)

// CDTW NN: the pairs whose lower bound does not exceed the query's cut-off
// after the seed sweep (the seed itself excluded), listed for the main sweep;
// the others are +inf without a sweep, as are the pairs whose window admits no
// path (w = floor(ratio * max(L_q, L_r)) < |L_q - L_r|).  Wave-level
// compaction: one atomic per wave of 64 pairs.  The cut-off can only fall
// afterwards, so no NN is lost.
__global__ __launch_bounds__(256) void lb_compact_kernel(const double* lb, const unsigned long long* best,
                                                         const int32_t* seed, const int64_t* qoff,
                                                         const int64_t* roff, double ratio, int64_t nq, int64_t nr,
                                                         double* res, int32_t* items, unsigned int* count,
                                                         unsigned long long* pruned) {
    // block (c, q-stride): candidates [c * per, (c + 1) * per) of its queries;
    // a wave takes 2048 at a time, 32 per lane (coalesced, lane-minor), and
    // lists its kept pairs with one atomic on the shared list counter (a scan
    // of the lanes' counts gives each lane its place)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t per = (int64_t)kCompactPer, r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < nr ? r0 + per : nr;
    unsigned long long np = 0;
    for (int64_t q = blockIdx.y; q < nq; q += gridDim.y) {
        const int lq = (int)(qoff[q + 1] - qoff[q]);
        const double cut = bitsd(best[q]);
        const int64_t sb = seed ? (int64_t)seed[q] : -1;
        for (int64_t base = r0 + (int64_t)wv * 2048; base < r1; base += 4 * 2048) {
            unsigned int keep = 0;   // bit u: candidate base + 64 u + lane kept
#pragma unroll 8
            for (int u = 0; u < 32; ++u) {
                const int64_t r = base + 64 * u + lane;
                if (r < r1 && r != sb) {
                    const int64_t p = q * nr + r;
                    const int lr = (int)(roff[r + 1] - roff[r]);
                    const int L = lq > lr ? lq : lr, ld = lq > lr ? lq - lr : lr - lq;
                    const bool feasible = ratio >= 1.0 || (int)floor(ratio * (double)L) >= ld;
                    const bool drop = feasible && lb[p] * (1.0 - 1e-11) > cut;   // counted
                    if (feasible && !drop) keep |= 1u << u;
                    else res[p] = __builtin_huge_val();
                    np += drop ? 1 : 0;
                }
            }
            const unsigned int c = (unsigned int)__popc(keep);
            unsigned int pre = c;   // inclusive scan of the counts over the wave
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned int y = __shfl_up(pre, o);
                if (lane >= o) pre += y;
            }
            const unsigned int total = __shfl(pre, 63);
            unsigned int off = 0;
            if (lane == 63 && total) off = atomicAdd(count, total);
            off = __shfl(off, 63) + pre - c;
            for (unsigned int km = keep; km; km &= km - 1u)
                items[off++] = (int32_t)(q * nr + base + 64 * (__ffs(km) - 1) + lane);
        }
    }
    for (int o = 32; o > 0; o >>= 1) np += __shfl_xor(np, o);
    if (lane == 0 && np) atomicAdd(pruned, np);
}

// Largest |x| over a set, as the bit pattern of a non-negative double.
__global__ void absmax_kernel(const double* v, int64_t n, unsigned long long* out) {
    __shared__ double part[4];
    double m = 0.0;
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; x + 3 * st < n; x += 4 * st) {   // four independent loads in flight
        const double a = v[x], b = v[x + st], c = v[x + 2 * st], d = v[x + 3 * st];
        m = fmax(m, fmax(fmax(__builtin_fabs(a), __builtin_fabs(b)), fmax(__builtin_fabs(c), __builtin_fabs(d))));
    }
    for (; x < n; x += st) m = fmax(m, __builtin_fabs(v[x]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {   // one atomic per block
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, part[w]);
        atomicMax(out, dbits(m));
    }
}

// Widening of each query's FP32 cut-off during the screening sweep.  The
// best-so-far b is an FP32 distance (or the FP64 path bound UB >= b), so the
// exact NN distance is <= screen_bound(b) and any prefix of its path evaluates
// in FP32 to <= b + 2 eps(screen_bound(UB)).
__global__ void screen_widen_kernel(int kind, SweepArgs A, const int64_t* qoff, int64_t lr_max, double gap,
                                    const unsigned long long* absmax, double* widen_abs) {
    double Amax = bitsd(*absmax);
    if ((kind & 7) == ERP) Amax = fmax(Amax, __builtin_fabs(gap));
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < A.nA; q += (int64_t)gridDim.x * blockDim.x) {
        const double N = (double)(qoff[q + 1] - qoff[q] + lr_max);
        const double ub = bitsd(A.best[q]);
        widen_abs[q] = (ub < __builtin_huge_val()) ? 2.0 * screen_eps(kind, screen_bound(kind, ub, N, Amax), N, Amax)
                                                   : 0.0;
    }
}

// The screen's thresholds for one query from its FP32 cut-off b32: thr
// (FP32 results above it cannot be the NN) and cut64 (an upper bound on the
// FP64 NN distance); both +inf when b32 is.
__device__ __forceinline__ void screen_cut(int kind, const int64_t* qoff, int64_t q, int64_t lr_max, double gap,
                                           double Ab, double margin_rel, double b32, double& thr, double& cut64) {
    thr = __builtin_huge_val();
    cut64 = __builtin_huge_val();
    if (!(b32 < __builtin_huge_val())) return;
    const double N = (double)(qoff[q + 1] - qoff[q] + lr_max);
    const double Amax = ((kind & 7) == ERP) ? fmax(Ab, __builtin_fabs(gap)) : Ab;
    const double b = b32 * (1.0 + margin_rel);
    cut64 = screen_bound(kind, b, N, Amax);
    thr = b + 2.0 * screen_eps(kind, cut64, N, Amax);
}

// After the FP32 sweep: every candidate of query q whose FP32 distance is
// <= b + 2 eps(screen_bound(b)) is listed for the FP64 recheck, where b is the
// best-so-far (the least FP32 distance, or the seed's FP64 distance).  The
// FP64 NN cannot be elsewhere: its exact cost is <= that of the winner, which
// is <= screen_bound(b), and its FP32 value exceeds that by at most eps.  The
// margin m widens b by a relative (1 + m) on top.  The seed (seed[q], swept in
// FP64 before the screen) keeps its FP64 distance and is not listed; every
// other result slot is reset to +inf, and best[q] becomes the smaller of
// screen_bound(b) and the seed's distance, an upper bound on the FP64 NN
// distance that serves as the recheck's first cut-off.  TPQ threads per query.
template <int TPQ>
__global__ void screen_filter_kernel(int kind, SweepArgs A, const int64_t* qoff, int64_t lr_max, double gap,
                                     const unsigned long long* absmax, double margin_rel, double* res,
                                     unsigned long long* best, const int32_t* seed, int32_t* items,
                                     unsigned int* count, unsigned long long* rechecks) {
    constexpr int QPB = TPQ >= 256 ? 1 : 256 / TPQ;
    const int tq = threadIdx.x % TPQ;
    const double Ab = bitsd(*absmax);
    for (int64_t q0 = (int64_t)blockIdx.x * QPB; q0 < A.nA; q0 += (int64_t)gridDim.x * QPB) {
        const int64_t q = q0 + threadIdx.x / TPQ;
        const bool on = q < A.nA;
        double thr = __builtin_huge_val(), cut64 = __builtin_huge_val(), dseed = __builtin_huge_val();
        int64_t sb = -1;
        unsigned long long n = 0;
        if (on) {
            screen_cut(kind, qoff, q, lr_max, gap, Ab, margin_rel, bitsd(best[q]), thr, cut64);
            sb = seed ? (int64_t)seed[q] : -1;
            dseed = (sb >= 0) ? res[q * A.nB + sb] : __builtin_huge_val();
            for (int64_t r = tq; r < A.nB; r += TPQ) {
                if (r == sb) continue;
                const int64_t p = q * A.nB + r;
                if (res[p] <= thr) {
                    const unsigned int k = atomicAdd(count, 1u);
                    items[k] = (int32_t)p;
                    ++n;
                }
                res[p] = __builtin_huge_val();
            }
        }
        for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
        if ((threadIdx.x & 63) == 0 && n) atomicAdd(rechecks, n);
        // every thread of the query has read best[q] before it is replaced
        if constexpr (TPQ > 64) __syncthreads();
        if (on && tq == 0) best[q] = dbits(dseed < cut64 ? dseed : cut64);
    }
}

// The screen filter split for a few queries with many candidates: first the
// per-query thresholds (and the recheck's first cut-off into best[q], as
// screen_filter_kernel sets it), then block (c, q) lists the pairs of chunk c
// of query q at or below the threshold and resets every result slot but the
// seed's; wave-level compaction of the list.
__global__ void screen_prep_kernel(int kind, SweepArgs A, const int64_t* qoff, int64_t lr_max, double gap,
                                   const unsigned long long* absmax, double margin_rel, const double* res,
                                   unsigned long long* best, const int32_t* seed, double* thr_out) {
    const double Ab = bitsd(*absmax);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < A.nA; q += (int64_t)gridDim.x * blockDim.x) {
        double thr, cut64;
        screen_cut(kind, qoff, q, lr_max, gap, Ab, margin_rel, bitsd(best[q]), thr, cut64);
        const int64_t sb = seed ? (int64_t)seed[q] : -1;
        const double dseed = (sb >= 0) ? res[q * A.nB + sb] : __builtin_huge_val();
        thr_out[q] = thr;
        best[q] = dbits(dseed < cut64 ? dseed : cut64);
    }
}

__global__ __launch_bounds__(256) void screen_pick_kernel(const double* thr_in, int64_t nB, int S, double* res,
                                                          const int32_t* seed, int32_t* items, unsigned int* count,
                                                          unsigned long long* rechecks) {
    const int64_t q = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int64_t per = (nB + S - 1) / S, r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < nB ? r0 + per : nB;
    const double thr = thr_in[q];
    const int64_t sb = seed ? (int64_t)seed[q] : -1;
    unsigned long long n = 0;
    for (int64_t base = r0 + (threadIdx.x & ~63); base < r1; base += blockDim.x) {
        const int64_t r = base + lane;
        bool keep = false;
        if (r < r1 && r != sb) {
            const int64_t p = q * nB + r;
            keep = res[p] <= thr;
            res[p] = __builtin_huge_val();
        }
        const unsigned long long m = __ballot(keep);
        unsigned int off = 0;
        if (lane == 0 && m) off = atomicAdd(count, (unsigned int)__popcll(m));
        off = __shfl(off, 0);
        if (keep) items[off + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)(q * nB + r);
        n += keep ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
    if (lane == 0 && n) atomicAdd(rechecks, n);
}

// Threads per query for the per-query scans over nr candidates: one wave up
// to 1024 candidates, a 256-thread block up to 4096, else a 1024-thread block
// (with a few queries and many candidates a wave's chain of loads is the
// whole kernel's time).
static int scan_threads(int64_t nr) { return nr > 4096 ? 1024 : (nr > 1024 ? 256 : 64); }

// Blocks per query for the split scans: one per 4096 candidates, at most
// about 1024 blocks in all (so nq x S < scan_part_entries(nq)); 1 = no split.
static int scan_split(int64_t nq, int64_t nr) {
    if (nr <= 4096) return 1;
    const int64_t s = std::min<int64_t>((nr + 4095) / 4096, (1024 + nq - 1) / nq);
    return (int)std::max<int64_t>(s, 1);
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

hipError_t launch_derivative(const double* v, const int64_t* off, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(derivative_kernel, dim3((unsigned)std::min<int64_t>(n, 65535)), dim3(256), 0, s, v, off, n,
                       out);
    return hipGetLastError();
}

hipError_t launch_subseq_windows(const double* x, int64_t nw, int m, double* out, hipStream_t s) {
    const size_t lds = sizeof(double) * (size_t)(3 * kWinPerBlock + m - 1);
    hipLaunchKernelGGL(subseq_windows_kernel, dim3(blocks_for(nw, kWinPerBlock)), dim3(256), lds, s, x, nw, m, out);
    return hipGetLastError();
}

hipError_t launch_znorm(const double* v, const int64_t* off, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(znorm_kernel, dim3(blocks_for(n, 1)), dim3(256), 0, s, v, off, n, out);
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

hipError_t launch_next_up(double* x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(next_up_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_put_u64(unsigned long long* dst, const unsigned long long* src, int n, hipStream_t s) {
    if (n < 0 || n > kPutWords) return hipErrorInvalidValue;
    PutWords w;
    for (int x = 0; x < n; ++x) w.w[x] = src[x];
    hipLaunchKernelGGL(put_u64_kernel, dim3(1), dim3(kPutWords), 0, s, dst, n, w);
    return hipGetLastError();
}

hipError_t launch_interleave(const double* rv, const int64_t* roff, int64_t nr, int lr_max, double* rT, float* r32,
                             unsigned long long* absmax, hipStream_t s) {
    hipLaunchKernelGGL(interleave_kernel, dim3((unsigned)((nr + 63) / 64), (unsigned)((lr_max + 63) / 64)), dim3(256),
                       0, s, rv, roff, nr, lr_max, rT, r32, absmax);
    return hipGetLastError();
}

__global__ void max_u64_kernel(unsigned long long* dst, const unsigned long long* src) {
    if (threadIdx.x == 0) atomicMax(dst, *src);
}

hipError_t launch_max_u64(unsigned long long* dst, const unsigned long long* src, hipStream_t s) {
    hipLaunchKernelGGL(max_u64_kernel, dim3(1), dim3(64), 0, s, dst, src);
    return hipGetLastError();
}

hipError_t launch_lb_compact(const double* lb, const unsigned long long* best, const int32_t* seed,
                             const int64_t* qoff, const int64_t* roff, double ratio, int64_t nq, int64_t nr,
                             double* res, int32_t* items, unsigned int* count, unsigned long long* pruned,
                             hipStream_t s) {
    // about 4096 blocks: chunks of kCompactPer candidates times query groups
    const int64_t gx = (nr + kCompactPer - 1) / kCompactPer;
    const int64_t gy = std::min<int64_t>(nq, std::max<int64_t>(1, 4096 / gx));
    hipLaunchKernelGGL(lb_compact_kernel, dim3((unsigned)gx, (unsigned)std::min<int64_t>(gy, 65535)), dim3(256), 0,
                       s, lb, best, seed, qoff, roff, ratio, nq, nr, res, items, count, pruned);
    return hipGetLastError();
}

hipError_t launch_absmax(const double* v, int64_t n, unsigned long long* out, hipStream_t s) {
    hipLaunchKernelGGL(absmax_kernel, dim3(std::min(blocks_for(n, 256 * 16), 2048)), dim3(256), 0, s, v, n, out);
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
                                unsigned long long* best, const int32_t* seed, int32_t* items, unsigned int* count,
                                unsigned long long* rechecks, double* part, hipStream_t s) {
    const int S = scan_split(a.nA, a.nB);
    if (S >= 2 && part) {
        hipLaunchKernelGGL(screen_prep_kernel, dim3(blocks_for(a.nA, 256)), dim3(256), 0, s, kind, a, qoff, lr_max,
                           gap, absmax, margin_rel, res, best, seed, part);
        hipLaunchKernelGGL(screen_pick_kernel, dim3((unsigned)S, (unsigned)a.nA), dim3(256), 0, s, part, a.nB, S, res,
                           seed, items, count, rechecks);
        return hipGetLastError();
    }
    switch (scan_threads(a.nB)) {
    case 1024: hipLaunchKernelGGL(screen_filter_kernel<1024>, dim3(blocks_for(a.nA, 1)), dim3(1024), 0, s, kind, a,
                                  qoff, lr_max, gap, absmax, margin_rel, res, best, seed, items, count, rechecks); break;
    case 256: hipLaunchKernelGGL(screen_filter_kernel<256>, dim3(blocks_for(a.nA, 1)), dim3(256), 0, s, kind, a, qoff,
                                 lr_max, gap, absmax, margin_rel, res, best, seed, items, count, rechecks); break;
    default: hipLaunchKernelGGL(screen_filter_kernel<64>, dim3(blocks_for(a.nA, 4)), dim3(256), 0, s, kind, a, qoff,
                                lr_max, gap, absmax, margin_rel, res, best, seed, items, count, rechecks); break;
    }
    return hipGetLastError();
}

hipError_t launch_envelope(const double* v, const int64_t* off, int64_t n, int set_max, int other_max, int npos,
                           double ratio, double* up, double* lo, double* qx, int64_t s_stride, int64_t p_stride,
                           hipStream_t s) {
    const int cap = std::max(set_max, npos);
    int w = ratio >= 1.0 ? cap : (int)std::floor(ratio * (double)std::max(set_max, other_max));
    w = std::min(w, cap);
    const size_t lds = sizeof(double) * 2 * (size_t)(npos + 2 * w);
    static bool attr_set = false;
    if (!attr_set && lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&envelope_kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(envelope_kernel, dim3((unsigned)std::min<int64_t>(n, 65535)), dim3(256), lds, s, v, off, n, npos,
                       other_max, ratio, up, lo, qx, s_stride, p_stride);
    return hipGetLastError();
}

hipError_t launch_lb_reverse(const double* qv, const int64_t* qoff, const double* rv, const int64_t* roff, int64_t nr,
                             const double* cup, const double* clo, const int32_t* items, const unsigned int* count,
                             int64_t max_items, double* lb, hipStream_t s) {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((max_items + 255) / 256, 256 * 16));
    hipLaunchKernelGGL(lb_reverse_kernel, dim3((unsigned)blocks), dim3(256), 0, s, qv, qoff, rv, roff, nr, cup, clo,
                       items, count, lb);
    return hipGetLastError();
}

hipError_t launch_ub_nn(int kind, const SweepArgs& a, const double* qv, const int64_t* qoff, const double* rv,
                        const int64_t* roff, int lq_max, int lr_max, const double* rT, double* ub, double* env,
                        double* lb, hipStream_t s) {
    if ((kind == CDTW || kind == DTW) && lb && env) {
        // the query envelopes (upper, lower, and the query extended by its
        // last value: three arrays of env_stride doubles), then bound and
        // LB_Keogh of up to 16 queries per pass over the candidates
        const int64_t stride = env_stride(a.nA, lr_max), ld = env_ld(lr_max);
        double *up = env, *lo = env + stride, *qx = env + 2 * stride;
        hipError_t e = launch_envelope(qv, qoff, a.nA, lq_max, lr_max, lr_max, a.window_ratio, up, lo, qx, ld, 1, s);
        if (e != hipSuccess) return e;
        // queries per block: the most that still leaves at least 2 blocks per
        // CU (fewer reads of the candidates)
        const int64_t bx = (a.nB + 255) / 256;
        int cus = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        int qt = 1;
        for (int c : {16, 8, 4, 2})
            if (bx * ((a.nA + c - 1) / c) >= 2 * (int64_t)cus) {
                qt = c;
                break;
            }
        const dim3 gq((unsigned)bx, (unsigned)std::min<int64_t>((a.nA + qt - 1) / qt, 65535));
#define EAP_UBLB(QT) hipLaunchKernelGGL(ub_lb_kernel<QT>, gq, dim3(256), 0, s, a, qv, qoff, rv, rT, roff, ld, \
                                        up, lo, qx, lb, ub)
        switch (qt) {
        case 16: EAP_UBLB(16); break;
        case 8: EAP_UBLB(8); break;
        case 4: EAP_UBLB(4); break;
        case 2: EAP_UBLB(2); break;
        default: EAP_UBLB(1); break;
        }
#undef EAP_UBLB
        return hipGetLastError();
    }
    // queries per block: the most that still leaves at least 2 blocks per CU
    const int64_t bx = (a.nB + 255) / 256;
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    int qt = 1;
    for (int c : {8, 4, 2})
        if (bx * ((a.nA + c - 1) / c) >= 2 * (int64_t)cus) {
            qt = c;
            break;
        }
    const dim3 g((unsigned)bx, (unsigned)std::min<int64_t>((a.nA + qt - 1) / qt, 65535)), b(256);
    // WDTW's weight table in LDS: m = 2|d| - L within -lmax .. lmax
    const int ltab = std::max(lq_max, lr_max);
    const size_t lds = (kind == WDTW) ? sizeof(double) * (size_t)(2 * ltab + 1) : 0;
#define EAP_UBT(K, QT) \
    hipLaunchKernelGGL((ub_nn_t_kernel<K, QT>), g, b, lds, s, a, qv, qoff, rT, roff, lr_max, ltab, ub)
#define EAP_UBQ(K)             \
    switch (qt) {              \
    case 8: EAP_UBT(K, 8); break; \
    case 4: EAP_UBT(K, 4); break; \
    case 2: EAP_UBT(K, 2); break; \
    default: EAP_UBT(K, 1); break; \
    }
    switch (kind) {
    case DTW: EAP_UBQ(DTW); break;
    case CDTW: EAP_UBQ(CDTW); break;
    case WDTW: EAP_UBQ(WDTW); break;
    case ERP: EAP_UBQ(ERP); break;
    case MSM: EAP_UBQ(MSM); break;
    case TWE: EAP_UBQ(TWE); break;
    default: return hipErrorInvalidValue;
    }
#undef EAP_UBQ
#undef EAP_UBT
    return hipGetLastError();
}

template <int KIND>
static hipError_t ub_mv_launch(int nd, bool condensed, const SweepArgs& a, const double* qv, const int64_t* qoff,
                               const double* rv, const int64_t* roff, int64_t n, double* out, hipStream_t s) {
    const int64_t total = condensed ? n * (n - 1) / 2 : a.nA * a.nB;
    const dim3 g(blocks_for(total, 256)), b(256);
#define EAP_MV(ND)                                                                                              \
    if (condensed) hipLaunchKernelGGL((ub_condensed_mv_kernel<KIND, ND>), g, b, 0, s, a, qv, qoff, n, out);    \
    else hipLaunchKernelGGL((ub_nn_mv_kernel<KIND, ND>), g, b, 0, s, a, qv, qoff, rv, roff, out);
    switch (nd) {
    case 2: EAP_MV(2); break;
    case 3: EAP_MV(3); break;
    case 4: EAP_MV(4); break;
    default: return hipErrorInvalidValue;
    }
#undef EAP_MV
    return hipGetLastError();
}

hipError_t launch_ub_mv(int kind, int nd, bool condensed, const SweepArgs& a, const double* qv, const int64_t* qoff,
                        const double* rv, const int64_t* roff, int64_t n, double* out, hipStream_t s) {
    if (kind == DTW) return ub_mv_launch<DTW>(nd, condensed, a, qv, qoff, rv, roff, n, out, s);
    if (kind == CDTW) return ub_mv_launch<CDTW>(nd, condensed, a, qv, qoff, rv, roff, n, out, s);
    return hipErrorInvalidValue;
}

hipError_t launch_ub_condensed(int kind, const SweepArgs& a, const double* v, const int64_t* off, int64_t n,
                               double* cut, hipStream_t s) {
    const dim3 g(blocks_for(n * (n - 1) / 2, 256)), b(256);
    switch (kind) {
    case DTW: hipLaunchKernelGGL(ub_condensed_kernel<DTW>, g, b, 0, s, a, v, off, n, cut); break;
    case CDTW: hipLaunchKernelGGL(ub_condensed_kernel<CDTW>, g, b, 0, s, a, v, off, n, cut); break;
    case WDTW: hipLaunchKernelGGL(ub_condensed_kernel<WDTW>, g, b, 0, s, a, v, off, n, cut); break;
    case ERP: hipLaunchKernelGGL(ub_condensed_kernel<ERP>, g, b, 0, s, a, v, off, n, cut); break;
    case MSM: hipLaunchKernelGGL(ub_condensed_kernel<MSM>, g, b, 0, s, a, v, off, n, cut); break;
    case TWE: hipLaunchKernelGGL(ub_condensed_kernel<TWE>, g, b, 0, s, a, v, off, n, cut); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_seed(const double* ub, int64_t nq, int64_t nr, int32_t* seed_b, int32_t* items,
                       unsigned long long* best, double* part, hipStream_t s) {
    const int S = scan_split(nq, nr);
    if (S >= 2 && part) {
        int64_t* pi = reinterpret_cast<int64_t*>(part + scan_part_entries(nq));
        hipLaunchKernelGGL(scan_part_kernel<0>, dim3((unsigned)S, (unsigned)nq), dim3(256), 0, s, ub, nr, S, part, pi);
        hipLaunchKernelGGL(scan_finish_kernel<0>, dim3(blocks_for(nq, 4)), dim3(256), 0, s, part, pi, nq, S, nr,
                           seed_b, items, best, nullptr, nullptr, nullptr, nullptr);
        return hipGetLastError();
    }
    switch (scan_threads(nr)) {
    case 1024: hipLaunchKernelGGL(seed_kernel<1024>, dim3(blocks_for(nq, 1)), dim3(1024), 0, s, ub, nq, nr, seed_b,
                                  items, best); break;
    case 256: hipLaunchKernelGGL(seed_kernel<256>, dim3(blocks_for(nq, 1)), dim3(256), 0, s, ub, nq, nr, seed_b, items,
                                 best); break;
    default: hipLaunchKernelGGL(seed_kernel<64>, dim3(blocks_for(nq, 4)), dim3(256), 0, s, ub, nq, nr, seed_b, items,
                                best); break;
    }
    return hipGetLastError();
}

hipError_t launch_argmin(const double* res, int64_t nq, int64_t nr, const int32_t* labels, int64_t* out_idx,
                         double* out_dist, int32_t* out_label, double* part, hipStream_t s) {
    const int S = scan_split(nq, nr);
    if (S >= 2 && part) {
        int64_t* pi = reinterpret_cast<int64_t*>(part + scan_part_entries(nq));
        hipLaunchKernelGGL(scan_part_kernel<1>, dim3((unsigned)S, (unsigned)nq), dim3(256), 0, s, res, nr, S, part,
                           pi);
        hipLaunchKernelGGL(scan_finish_kernel<1>, dim3(blocks_for(nq, 4)), dim3(256), 0, s, part, pi, nq, S, nr,
                           nullptr, nullptr, nullptr, labels, out_idx, out_dist, out_label);
        return hipGetLastError();
    }
    switch (scan_threads(nr)) {
    case 1024: hipLaunchKernelGGL(argmin_kernel<1024>, dim3(blocks_for(nq, 1)), dim3(1024), 0, s, res, nq, nr, labels,
                                  out_idx, out_dist, out_label); break;
    case 256: hipLaunchKernelGGL(argmin_kernel<256>, dim3(blocks_for(nq, 1)), dim3(256), 0, s, res, nq, nr, labels,
                                 out_idx, out_dist, out_label); break;
    default: hipLaunchKernelGGL(argmin_kernel<64>, dim3(blocks_for(nq, 4)), dim3(256), 0, s, res, nq, nr, labels,
                                out_idx, out_dist, out_label); break;
    }
    return hipGetLastError();
}

}  // namespace eap
