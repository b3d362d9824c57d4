// Host-side launch interface between the C ABI (eap_api.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eap {

// How a sweep kernel enumerates its work items.
// A launch processes items[0..npairs) when `items` is given, else 0..npairs.
enum PairMode : int {
    PM_NN_ALL = 0,    // item p -> (a = p / nB, b = p % nB); skips b == skip_b[a]
    PM_CONDENSED = 1, // item p -> pair (i, j), i < j, of set A (B == A), condensed order
    PM_SINGLE = 3     // one pair (A[0], B[0])
};

struct SweepArgs {
    int mode;
    int64_t nA, nB, npairs;
    const int32_t* skip_b;
    const int32_t* items;
    // NN: best-so-far cut-off per query a (bits of a non-negative double),
    // atomically lowered by every pair that completes under it.
    unsigned long long* best;
    // Per-item cut-off (PM_CONDENSED: condensed index; PM_SINGLE: [0]); NULL = +inf.
    const double* pcut;
    // Result per item: NN modes at a*nB + b, PM_CONDENSED at the condensed
    // index, PM_SINGLE at [0].  +inf when abandoned.
    double* res;
    unsigned int* queue;             // work counter, zero at launch
    int chunk;                       // work slots taken per atomic on `queue` (>= 1)
    unsigned long long* counters;    // [0] cells executed, [1] pairs swept, [3] band overflows
    unsigned long long* stage;       // [0] cells of this launch's stage, [8] its pairs
    // plain DP: cut-off +inf for every item, no best-so-far, no abandoning
    int plain;
    // NN items under a per-item cut-off pcut[p] instead of the best-so-far
    // (prune-only: one ulp above the pair's path bound, so nothing is abandoned)
    int prune_only;
    // no pruning (EABase, Alg. 4): every strip of the row sweep starts at row 1
    // and runs to the last row; a pair is still abandoned once nothing on the
    // sweep's boundary is <= cut-off
    int no_prune;
    // distance parameters
    double gap, c, nu, lam;
    // Per-diagonal tables, indexed by (j - i) + tab_off:
    //   TWE: nu * (2|j-i|);  WDTW: weight of |j-i| for the pair's longer length
    const double* tab;
    int tab_off, tab_len;
    // WDTW: G[m] = 1/(1+exp(-g*m/2)) for m = 2k - L, indexed m + gtab_off
    // (zeros below m = -Lmax; covers every m the row sweep reads)
    const double* gtab;
    int gtab_off, gtab_len;
    // window (CDTW / ERP): ratio as given; <0 means none
    double window_ratio;
    // band kernel: half-width of the band for unconstrained distances
    int band_half;
    // band kernel: items whose band was too narrow are appended here
    int32_t* ovf_items;
    unsigned int* ovf_count;
    // when set, the number of work slots is read from here at run time
    const unsigned int* npairs_dev;
    // FP32 screen: the cut-off of query a is best[a] * (1 + widen_rel) + widen_abs[a]
    const double* widen_abs;
    double widen_rel;
    // row sweep: per-group edge buffers of edge_stride values (T), for pairs
    // whose shorter series is wider than one strip; NULL = no strips
    void* edge;
    int64_t edge_stride;
    // NN, CDTW: lower bound of each pair (at its result index); a pair whose
    // bound exceeds the cut-off is not swept.  NULL = none
    const double* lb;
    // latency-bound launch (a few pairs per query): its waves take a higher
    // issue priority than those of a throughput-bound sweep running beside it
    int prio;
};

// Shape of the row sweep: G lanes per pair (pairs per wave = 64 / G), C
// columns per lane, strips of W = G * C columns.
struct RowsShape {
    int g, c;
};

struct SeriesPtrs {
    const void* v;
    const int64_t* off;
    const void* border;
};

// Row sweep (kernel A): strips of W = G*C columns per pair (DTW, WDTW, ERP
// without a window, MSM, TWE).  Returns the launch error.  Pairs wider than
// one strip need a.edge with room for grid * 256 / G groups.  With `occ` set
// nothing is launched: *occ = blocks of this kernel one CU holds at once.
// xd: exact differences (FP32 WDTW only; A and B hold float64 values).
// nd > 1: multivariate series of nd channels (2..4; DTW, and CDTW with its
// window on the row sweep; FP64; shapes G in {8, 16, 32, 64} x 8).
hipError_t launch_rows(int kind, bool fp32, RowsShape sh, const SweepArgs& a, SeriesPtrs A, SeriesPtrs B, int grid,
                       hipStream_t s, int* occ = nullptr, bool xd = false, int nd = 1);
int rows_lds_bytes(int kind, bool fp32, const SweepArgs& a);
bool rows_shape_ok(int kind, RowsShape sh, bool fp32);

// Band sweep (kernel B): anti-diagonal sweep of a band of diags = 2*G*C
// diagonals with G lanes per pair (C in {4, 8, 16}).  `occ` as for the row sweep.
hipError_t launch_band(int kind, bool fp32, int diags, int g, const SweepArgs& a, SeriesPtrs A, SeriesPtrs B,
                       int grid, hipStream_t s, int* occ = nullptr);
bool band_shape_ok(int diags, int g);

// Auxiliary kernels.
hipError_t launch_erp_border(const double* v, const int64_t* off, int64_t n, double gap, double* out, hipStream_t s);
hipError_t launch_to_f32(const double* v, int64_t n, float* out, hipStream_t s);
// z-normalise each series of a ragged set (device offsets), see eap_znorm.
hipError_t launch_znorm(const double* v, const int64_t* off, int64_t n, double* out, hipStream_t s);
hipError_t launch_derivative(const double* v, const int64_t* off, int64_t n, double* out, hipStream_t s);
hipError_t launch_subseq_windows(const double* x, int64_t nw, int m, double* out, hipStream_t s);
// Candidates interleaved for coalesced reads: rT[k * nr + b] = value k of
// candidate b (0 past its end), k < lr_max (rT may be NULL when only the
// following are wanted).  With r32 also the FP32 copy
// (same layout as rv), with absmax also the largest |x| (atomicMax on the
// bit pattern of a non-negative double; clear it first).
hipError_t launch_interleave(const double* rv, const int64_t* roff, int64_t nr, int lr_max, double* rT, float* r32,
                             unsigned long long* absmax, hipStream_t s);
// *dst = max(*dst, *src) (u64), one thread.
hipError_t launch_max_u64(unsigned long long* dst, const unsigned long long* src, hipStream_t s);
// CDTW envelope area: three arrays (upper envelope, lower envelope, query
// extended by its last value), each nq rows of env_ld(lr_max) doubles, lr_max
// of them used: rows of a multiple of 8 doubles, so the UB + LB kernel reads
// them in aligned chunks of 8.
inline int64_t env_ld(int64_t lr_max) { return (lr_max + 7) & ~(int64_t)7; }
inline int64_t env_stride(int64_t nq, int64_t lr_max) { return nq * env_ld(lr_max); }
// Envelopes of a ragged set (device offsets) for LB_Keogh: positions 1..npos,
// window floor(ratio * max(L_s, other_max)) per series (ratio >= 1: the whole
// series), out[s * s_stride + (j-1) * p_stride]; qx (nullable): the series
// extended by its last value.  set_max: the set's longest series.
hipError_t launch_envelope(const double* v, const int64_t* off, int64_t n, int set_max, int other_max, int npos,
                           double ratio, double* up, double* lo, double* qx, int64_t s_stride, int64_t p_stride,
                           hipStream_t s);
// Reversed LB_Keogh over the listed pairs (items[0 .. *count)): the candidate
// envelopes cup / clo (interleaved, [position][nr]) against the query values;
// lb[p] becomes the larger of its two bounds.
hipError_t launch_lb_reverse(const double* qv, const int64_t* qoff, const double* rv, const int64_t* roff, int64_t nr,
                             const double* cup, const double* clo, const int32_t* items, const unsigned int* count,
                             int64_t max_items, double* lb, hipStream_t s);
// Path upper bound of every (query, candidate) pair from rT (launch_interleave);
// for DTW and CDTW with env (3 x env_stride doubles) and lb also the query
// envelopes and LB_Keogh with LB_Kim's corners, reading the candidates from rT, or with rv != NULL from rv /
// roff in their own layout (rT unused).
hipError_t launch_ub_nn(int kind, const SweepArgs& a, const double* qv, const int64_t* qoff, const double* rv,
                        const int64_t* roff, int lq_max, int lr_max, const double* rT, double* ub, double* env,
                        double* lb, hipStream_t s);
hipError_t launch_ub_condensed(int kind, const SweepArgs& a, const double* v, const int64_t* off, int64_t n,
                               double* cut, hipStream_t s);
// Multivariate DTW / CDTW (nd = 2..4 channels): the path bound of every
// (query, candidate) pair into out[a * nB + b] (condensed = false; qv / qoff
// and rv / roff the two sets, n unused), or one ulp above it for every
// condensed pair of the set qv / qoff of n series (condensed = true).
hipError_t launch_ub_mv(int kind, int nd, bool condensed, const SweepArgs& a, const double* qv, const int64_t* qoff,
                        const double* rv, const int64_t* roff, int64_t n, double* out, hipStream_t s);
// Scratch of the split per-query scans (seed, argmin, screen filter) for a
// few queries with many candidates: 2 x scan_part_entries(nq) doubles
// (partial values, then partial indexes); part == nullptr runs the
// single-pass kernels.
inline int64_t scan_part_entries(int64_t nq) { return 1024 + nq; }
hipError_t launch_seed(const double* ub, int64_t nq, int64_t nr, int32_t* seed_b, int32_t* list_a,
                       unsigned long long* best, double* part, hipStream_t s);
hipError_t launch_argmin(const double* res, int64_t nq, int64_t nr, const int32_t* labels, int64_t* out_idx,
                         double* out_dist, int32_t* out_label, double* part, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s);
// x[i] = the next double above x[i], in place (+inf unchanged).
hipError_t launch_next_up(double* x, int64_t n, hipStream_t s);
// Up to kPutWords host words written to dst by one kernel whose argument
// block carries them: a host-to-device transfer that needs no staging memory
// and no copy call (the call that allocates nothing uses it).
constexpr int kPutWords = 448;
struct PutWords {
    unsigned long long w[kPutWords];
};
hipError_t launch_put_u64(unsigned long long* dst, const unsigned long long* src, int n, hipStream_t s);
hipError_t launch_absmax(const double* v, int64_t n, unsigned long long* out, hipStream_t s);
hipError_t launch_lb_compact(const double* lb, const unsigned long long* best, const int32_t* seed,
                             const int64_t* qoff, const int64_t* roff, double ratio, int64_t nq, int64_t nr,
                             double* res, int32_t* items, unsigned int* count, unsigned long long* pruned,
                             hipStream_t s);
hipError_t launch_screen_filter(int kind, const SweepArgs& a, const int64_t* qoff, int64_t lr_max, double gap,
                                const unsigned long long* absmax, double margin_rel, double* res,
                                unsigned long long* best, const int32_t* seed, int32_t* items, unsigned int* count,
                                unsigned long long* rechecks, double* part, hipStream_t s);
hipError_t launch_screen_widen(int kind, const SweepArgs& a, const int64_t* qoff, int64_t lr_max, double gap,
                               const unsigned long long* absmax, double* widen_abs, hipStream_t s);

}  // namespace eap
