/*
 * eap.h - C ABI of libeap.so: EAPruned elastic distances on one MI355X (gfx950).
 *
 * Implements the distance computation with a cut-off of Herrmann & Webb,
 * "Early Abandoning and Pruning for Elastic Distances including Dynamic Time
 * Warping" (arXiv 2102.05221), for the six distances of its Section 2.3 (DTW,
 * CDTW, WDTW, ERP, MSM, TWE), and the two drivers the paper uses it in: NN
 * search (Alg. 1) and all-pairs distance matrices with pruning only.
 *
 * Conventions shared by every entry point
 *  - Series values are float64 arrays in DEVICE memory.  A set of n series is
 *    one concatenated array plus an offsets array of n+1 int64 in HOST memory:
 *    series k is values[off[k] .. off[k+1]), length >= 1.  Offsets must start
 *    at 0 and be non-decreasing with every length >= 1.  Lengths up to 2048
 *    (longer series are EINVAL).
 *  - Outputs are DEVICE arrays owned by the caller.  Nothing is freed or kept.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    runs asynchronously; outputs are valid once the stream has reached the
 *    call.  Host-to-device copies of offsets are issued on the same stream
 *    from library-owned pinned staging memory, so the caller's host arrays may
 *    be reused as soon as the call returns.
 *  - The library never allocates device memory inside these calls: each driver
 *    takes a caller-provided device workspace sized by its *_workspace()
 *    function and aligned to 256 bytes (hipMalloc's and torch's allocations
 *    are).  One workspace must not be used by two calls in flight.
 *  - Inputs must be finite; the library does not scan for NaN.
 *  - Errors: argument errors return EAP_EINVAL / EAP_EWORKSPACE synchronously,
 *    before anything is enqueued, and leave outputs untouched.  HIP failures
 *    return EAP_EDEVICE.  eap_last_error() returns a thread-local message for
 *    the last failing call.  No C++ exception crosses this boundary and nothing
 *    aborts.
 */
#ifndef EAP_H
#define EAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The six distances of Section 2.3 (eq. Common and the per-distance equations). */
typedef enum { EAP_DTW = 0, EAP_CDTW = 1, EAP_WDTW = 2, EAP_ERP = 3, EAP_MSM = 4, EAP_TWE = 5 } eap_kind;

typedef enum {
    EAP_OK = 0,
    EAP_EINVAL = -1,     /* bad argument */
    EAP_ENOMEM = -2,     /* host staging memory could not be obtained */
    EAP_EDEVICE = -3,    /* a HIP call failed */
    EAP_EWORKSPACE = -4  /* workspace missing, smaller than *_workspace() or not 256-byte aligned */
} eap_status;

/* Distance parameters (Section 2.3).
 *  window_ratio  CDTW and ERP only: Sakoe-Chiba window (Section 2.3.2) given
 *                as a ratio of the longer length, w = floor(ratio * max(L_x, L_y));
 *                >= 1 or +inf means no window; < 0 or NaN is EINVAL.
 *                Ignored by the other distances.
 *  g             WDTW weight steepness of eq. WDTW, finite, >= 0.
 *  gap           ERP gap value g of eq. ERP, finite.
 *  c             MSM split/merge cost of eq. MSMCost, finite, >= 0.
 *  nu, lambda    TWE stiffness and delete penalty of eq. TWECost, finite, >= 0;
 *                timestamps are the indices (tau_i = i).
 *  dims          channels per series point, 0 or 1 for univariate series.
 *                2..4: multivariate DTW and CDTW (EAP_EINVAL for the other
 *                distances): values are stored point after point (point i of
 *                a series is values[(off + i) * dims .. + dims)), lengths and
 *                offsets count points, and the cost of two points is their
 *                squared Euclidean distance, the channels' squared differences
 *                added in channel order (Section 2.3 names the squared
 *                Euclidean distance as the usual cost; the paper's conclusion
 *                names the multivariate case).  Multivariate searches run in
 *                FP64 without lower bounds (precision and lb are ignored) and
 *                are not taken by the request server.
 * Costs: DTW, CDTW, WDTW use the squared difference; ERP, MSM, TWE the
 * absolute difference. */
typedef struct {
    int32_t kind; /* eap_kind */
    double window_ratio;
    double g;
    double gap;
    double c;
    double nu;
    double lambda;
    int32_t dims;
} eap_params;

/* NN search options.
 *  precision   0 = FP64 throughout.  1 = FP32 screening sweep, then every
 *              candidate whose FP32 distance is within the screen margin of the
 *              query's FP32 best is recomputed in FP64; results equal the FP64
 *              ones (indices bit-exact, distances bit-exact): the margin is
 *              margin_rel * best32 plus twice a certified bound on the FP32
 *              rounding error of any warping path (input rounding, per-term
 *              rounding and the running sum), so the FP64 nearest neighbour is
 *              always among the candidates rechecked.  WDTW whose diagonal
 *              weight 1/(1+exp(g*L/2)) is below 1e-8 (L the longest length)
 *              screens with exact differences: the FP32 sweep reads the
 *              float64 series and rounds each difference once, so the bound
 *              has no input-rounding term (its distances, scaled by such
 *              weights, lie far below the rounding of the inputs); below a
 *              diagonal weight of 1e-30 it sweeps in FP64 throughout.
 *  margin_rel  relative part of the screen margin for precision 1 (>= 0,
 *              finite; 1e-4 by default in the binding).
 *  flags       bit 0: skip the seeding pass (every candidate starts from the
 *              path upper bound); for ablation only.
 *              bit 1: plain full dynamic programme for every pair (no cut-off,
 *              no pruning, no abandoning): the baseline the pruned search is
 *              measured against.  Same results.
 *              bit 2: prepared: a previous call on this workspace had the same
 *              offsets and parameters, so their host-to-device copies are
 *              skipped and the call enqueues kernels only.  Required while the
 *              stream is being captured into a graph (see eap_capture_begin).
 *              bit 3: candidates prepared: a previous call on this workspace
 *              had the same candidates (values, offsets), parameters and
 *              precision, with any queries; what it derived from the
 *              candidates alone (their device offsets, ERP borders,
 *              interleaved and FP32 copies, |x| maximum), which sits at the
 *              workspace's start, is reused (a CDTW search without LB_Keogh
 *              over 2^18 or more candidates rebuilds the interleaved copy,
 *              which searches with the bound over such sets do not make).  For a resident candidate set
 *              searched by batch after batch (the request server uses it).
 *              bit 4: prune only (Section 5's "Prune"): every pair is swept
 *              under its own cut-off, one ulp above the cost of its
 *              diagonal-then-straight warping path (an upper bound), with no
 *              best-so-far shared between pairs: cells are pruned, nothing
 *              is abandoned, every pair's value is exact.  Precision 0 only
 *              (EAP_EINVAL otherwise); no seed sweep, no lower bounds.  For
 *              ablation.  Same results.
 *              bit 5: no pruning (EABase, Alg. 4): the row sweep computes
 *              every row of every strip of a pair, abandoning the pair only
 *              once nothing on its sweep boundary is <= cut-off.  (The band
 *              sweep prunes nothing beyond the window anyway.)  For ablation.
 *              Same results.
 *              Other bits: EAP_EINVAL.
 *  lb          lower bounds in front of the sweep (DTW and CDTW only; the
 *              other distances ignore it), eap_lb_mode:
 *              EAP_LB_DEFAULT  CDTW: EAP_LB_KEOGH; DTW: EAP_LB_NONE.
 *              EAP_LB_NONE     every pair is swept under the cut-off.
 *              EAP_LB_KEOGH    LB_Keogh of the query's envelope against the
 *                              candidate, its first and last columns taking
 *                              the exact costs of the corner cells (LB_Kim).
 *              EAP_LB_KEOGH2   then, for the pairs it keeps, the reversed
 *                              LB_Keogh (the candidate's envelope against the
 *                              query, Section 5.2's "lb-keogh2").
 *              A pair whose bound exceeds the best-so-far is +inf without a
 *              sweep; envelopes use the widest window any pair of the series
 *              has (for DTW the series' range).  Results do not depend on it.
 *              Other values: EAP_EINVAL.
 *  main_wait   hipEvent_t or NULL: the stream waits for it before the main
 *              sweep (after the bounds, the seed sweep and the screen set-up).
 *  main_done   hipEvent_t or NULL: recorded on the stream right after the main
 *              sweep (and its band re-run), before the recheck and the argmin.
 *              Several searches, each on its own stream and chained by these
 *              events (search k waits for search k-1's main_done), run their
 *              throughput-bound main sweeps one at a time while the
 *              latency-bound stages of the neighbouring searches overlap
 *              them.  Both must be NULL while the stream is being captured.
 *              The caller owns the events; results do not depend on them. */
typedef enum { EAP_LB_DEFAULT = 0, EAP_LB_NONE = 1, EAP_LB_KEOGH = 2, EAP_LB_KEOGH2 = 3 } eap_lb_mode;
typedef struct {
    int32_t precision;
    double margin_rel;
    int32_t flags;
    void* main_wait;
    void* main_done;
    int32_t lb;
} eap_nn_opts;

/* Counters accumulated in a workspace by the calls that use it (zero them with
 * eap_reset_counters() before the first read).  Cells are counted per lane
 * slot the sweep kernels evaluate, including slots past a series' end or
 * outside a window.  Stages: 0 seed sweep, 1 its re-run, 2 main sweep, 3 its
 * re-run (NN; FP32 when precision = 1), 4 FP64 recheck, 5 its re-run;
 * pairwise and distance use stage 2. */
typedef struct {
    uint64_t cells;          /* DP cells executed by the sweep kernels */
    uint64_t pairs;          /* pairs swept (CDTW NN pairs that LB_Keogh drops before
                                the sweep are not counted here) */
    uint64_t rechecks;       /* FP64 recomputations after an FP32 screen */
    uint64_t overflows;      /* band sweeps that had to be redone wider */
    uint64_t stage_cells[8];
    uint64_t stage_pairs[8];
    uint64_t lb_pruned;      /* CDTW NN pairs given +inf without a sweep because their
                                LB_Keogh exceeds the cut-off: the seed's distance
                                before the sweep, the best-so-far within it */
} eap_counters;

/* Optional timing of the sweep kernels with HIP events (off by default).
 * While enabled, every sweep launch is bracketed by two events on its stream.
 * eap_profile_take() waits for the recorded launches, copies up to `cap`
 * records into `out` (host memory), returns their number in *n and forgets
 * them.  kernel: 0 row sweep, 1 band sweep; size: strip width (row sweep) or
 * band diagonals; group: lanes per pair; kind: eap_kind swept; exact_diff: 1
 * for an FP32 sweep that forms its differences from float64 values. */
typedef struct {
    int32_t stage;
    int32_t kernel;
    int32_t kind;
    int32_t size;
    int32_t fp32;
    float ms;
    int32_t group;
    int32_t exact_diff;
} eap_profile_rec;
eap_status eap_profile_enable(int32_t on);
eap_status eap_profile_take(eap_profile_rec* out, int32_t cap, int32_t* n);

/* Distance with cut-off (Alg. 5: "Input S, T, w, cut-off; Result D or +inf").
 *  x (lx), y (ly)  device float64 series, lengths >= 1.
 *  cutoff          >= 0 or +inf (NaN is EINVAL).
 *  out             device, 1 double: D(x,y) if D <= cutoff, else +inf
 *                  (+inf also when the window admits no alignment).
 *  ws, ws_bytes    device workspace of at least eap_distance_workspace() bytes. */
size_t eap_distance_workspace(int64_t lx, int64_t ly, const eap_params* p);
eap_status eap_distance(const double* x, int64_t lx, const double* y, int64_t ly, const eap_params* p,
                        double cutoff, double* out, void* ws, size_t ws_bytes, void* stream);

/* Distance with cut-off that allocates nothing, for callers that cannot
 * allocate device or pinned memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, result and
 * errors as eap_distance, without the workspace: the scratch lives in a
 * static device array of the library (2 MiB, one copy per GPU, held until the
 * process ends; its device address is taken once per device, on the first
 * call there).  The offsets, the TWE / WDTW table and the cut-off reach the
 * device through kernel arguments, so no staging buffer or copy call is used,
 * and no event is created.  Every call on one GPU shares that GPU's scratch,
 * which keeps the last call's contents (the call clears what must start at
 * zero): calls that overlap on one GPU - on two streams, or from two
 * threads - race and must not be issued.  A layout larger than the scratch
 * (impossible for lengths up to 2048) is EAP_EWORKSPACE. */
eap_status eap_distance_noalloc(const double* x, int64_t lx, const double* y, int64_t ly, const eap_params* p,
                                double cutoff, double* out, void* stream);

/* 1-NN search (Alg. 1): for each query, the candidate with the smallest
 * distance, lowest index on ties (the strict '<' of Alg. 1).
 *  q, q_off, nq        queries (device values, host offsets), nq >= 1.
 *  r, r_off, nr        candidates (device values, host offsets), nr >= 1.
 *  r_labels            device int32[nr] or NULL.
 *  out_idx             device int64[nq]: index, or -1 when no candidate has a
 *                      finite distance (window too small for every one).
 *  out_dist            device double[nq]: the distance, or +inf.
 *  out_label           device int32[nq] or NULL: r_labels[idx], -1 when idx < 0.
 * DTW and CDTW searches can put lower bounds in front of the DP (the
 * lower-bounded search of Section 2.1, Alg. 2; eap_nn_opts.lb): a pair whose
 * bound exceeds the cut-off is +inf without a sweep; results are those of the
 * search without them. */
size_t eap_nn1_workspace(const int64_t* q_off, int64_t nq, const int64_t* r_off, int64_t nr, const eap_params* p,
                         const eap_nn_opts* o);
eap_status eap_nn1(const double* q, const int64_t* q_off, int64_t nq, const double* r, const int64_t* r_off,
                   int64_t nr, const int32_t* r_labels, const eap_params* p, const eap_nn_opts* o, void* ws,
                   size_t ws_bytes, int64_t* out_idx, double* out_dist, int32_t* out_label, void* stream);

/* All pairs i < j of one set (Section 5, "Prune" and "Base").
 *  mode 0  prune-only EAPruned: each pair's cut-off is one ulp above the cost
 *          of its diagonal-then-straight warping path (an upper bound,
 *          Section 4 intro), so nothing is abandoned and every value is exact.
 *  mode 1  plain full dynamic programme.
 *  out     device double[n*(n-1)/2], condensed: pair (i,j), i<j, at
 *          n*i - i*(i+1)/2 + (j-i-1).  +inf where the window admits no path. */
size_t eap_pairwise_workspace(const int64_t* s_off, int64_t n, const eap_params* p);
eap_status eap_pairwise(const double* s, const int64_t* s_off, int64_t n, const eap_params* p, int32_t mode,
                        void* ws, size_t ws_bytes, double* out, void* stream);

/* Sub-sequence search (Section 5.3: the closest match of a query within a
 * long series) as NN search: every window of length m of the series,
 * z-normalised on its own as the UCR suite does, is a candidate.
 * out[w*m + k] = (s[w+k] - mean_w) / sd_w for w = 0..n-m, k < m, with
 * mean_w = (sum of s[w..w+m-1], left to right) / m and sd_w = sqrt((sum of
 * (s[w+k] - mean_w)^2, left to right) / m) in binary64 (population standard
 * deviation; a constant window gives zeros).  The search is then eap_nn1 of
 * the query, z-normalised the same way (this call with n = m), against the
 * n-m+1 candidates with offsets k*m; the NN index is the window's start.
 *  s, n, m     device double[n], 1 <= m <= 2048, m <= n, (n-m+1)*m < 2^31
 *              (longer series: search them in overlapping parts).
 *  out         device double[(n-m+1)*m], not overlapping s. */
eap_status eap_subseq_windows(const double* s, int64_t n, int64_t m, double* out, void* stream);

/* Z-normalisation of every series of a ragged set: the normalisation that
 * sub-sequence search (Section 5.3) applies to its queries.  For each series,
 * out = (v - mean) / sd with mean and sd as in eap_subseq_windows (sums left
 * to right in binary64, population standard deviation; a constant series
 * gives zeros), so a series of length m comes out equal to its single
 * window from eap_subseq_windows.  One launch for the whole set.
 *  v, off, n   device values, host offsets (n >= 1 series, lengths 1..2048
 *              as for every set).
 *  out         device double[off[n]], not overlapping v.
 *  ws          device workspace of eap_znorm_workspace(n) bytes.
 * Errors as for eap_derivative. */
size_t eap_znorm_workspace(int64_t n);
eap_status eap_znorm(const double* v, const int64_t* off, int64_t n, double* out, void* ws, size_t ws_bytes,
                     void* stream);

/* Derivative series, for the derivative variants DDTW, DCDTW and DWDTW
 * (Section 2.3 names them: the distance of the series' first derivatives,
 * with no formula given).  The estimate of Keogh and Pazzani: for 1 < i < m,
 * d_i = ((q_i - q_{i-1}) + (q_{i+1} - q_{i-1}) / 2) / 2 in that order in
 * binary64; d_1 = d_2 and d_m = d_{m-1}; m = 2 gives d_1 = d_2 = q_2 - q_1,
 * m = 1 gives 0.  A derivative variant is then eap_nn1 / eap_pairwise /
 * eap_distance of DTW, CDTW or WDTW on the derivative series.
 *  v, off, n   device values, host offsets (n >= 1 series, lengths >= 1).
 *  out         device double[off[n]], not overlapping v.
 *  ws          device workspace of eap_derivative_workspace(n) bytes. */
size_t eap_derivative_workspace(int64_t n);
eap_status eap_derivative(const double* v, const int64_t* off, int64_t n, double* out, void* ws, size_t ws_bytes,
                          void* stream);

/* Envelopes for LB_Keogh (Section 2.1), as the NN search builds them: for
 * every series s of a ragged set and positions j = 1..npos,
 * up[s*npos + j-1] / lo[s*npos + j-1] = max / min of s_i over i in [j-w, j+w]
 * and [1, L_s], with w = floor(window_ratio * max(L_s, other_max)) (the widest
 * window of any pair of s with series of length <= other_max; window_ratio
 * >= 1: the whole series); an empty range gives (+inf, -inf).  O(L) per
 * series (van Herk / Gil-Werman; the values are copies of inputs).
 *  v, off, n          device values, host offsets (n >= 1 series, lengths 1..2048).
 *  npos               1..2048; other_max 0..2048; window_ratio >= 0.
 *  up, lo             device double[n * npos] each.
 *  ws                 device workspace of eap_envelopes_workspace(n) bytes. */
size_t eap_envelopes_workspace(int64_t n);
eap_status eap_envelopes(const double* v, const int64_t* off, int64_t n, int64_t npos, int64_t other_max,
                         double window_ratio, double* up, double* lo, void* ws, size_t ws_bytes, void* stream);

/* Copies the counters accumulated in `ws` to host memory (synchronises `stream`).
 * eap_reset_counters() zeroes them (asynchronously, on `stream`). */
eap_status eap_read_counters(const void* ws, size_t ws_bytes, eap_counters* out, void* stream);
eap_status eap_reset_counters(void* ws, size_t ws_bytes, void* stream);

/* Row-sweep autotuner.  The row sweep runs each pair on G lanes (64/G pairs
 * per wavefront) with C columns per lane, in strips of G*C columns; every
 * shape gives the same results, bit for bit.  eap_tune_nn1() runs eap_nn1() on
 * the given problem (a sample of the real one, typically) once per shape, G in
 * {4, 8, 16, 32, 64} x C in {8, 16} (and C = 32 with G >= 16 for the FP32 sweep
 * of DTW and WDTW), at the precision of `o` (1: the shape of the
 * FP32 screening sweep; 0: of the FP64 sweep), checks that all shapes return
 * the same indices and distances (EAP_EDEVICE otherwise), times each over two
 * further runs, and records the fastest for (distance, precision, class of the
 * shorter series' longest length: <=128, <=256, <=512, <=1024, <=2048) in a
 * process-wide table that every later call consults; without an entry a
 * default shape is used.  Distances the band sweep runs (CDTW, ERP with a
 * window, WDTW in its narrow band) are tuned over the band sweep's lanes per
 * pair instead (two choices per band width of 128 to 512 diagonals, 2*G*C
 * diagonals with C = 4 or 8), per band width; records then give G and C.
 * Synchronises `stream`; not for use while other calls are in flight.
 *  ws, ws_bytes        as for eap_nn1 (its workspace fits every shape).
 *  out_idx, out_dist   device int64[nq], double[nq]: scratch outputs.
 *  recs, cap, n        host array receiving one record per shape timed. */
typedef struct {
    int32_t g, c;      /* lanes per pair, columns per lane */
    float ms;          /* fastest of three timed eap_nn1 calls */
    int32_t chosen;    /* 1 for the shape recorded in the table */
} eap_tune_rec;
eap_status eap_tune_nn1(const double* q, const int64_t* q_off, int64_t nq, const double* r, const int64_t* r_off,
                        int64_t nr, const eap_params* p, const eap_nn_opts* o, void* ws, size_t ws_bytes,
                        int64_t* out_idx, double* out_dist, void* stream, eap_tune_rec* recs, int32_t cap,
                        int32_t* n);
/* Records row-sweep shape g x c for (kind, precision 0/1, the length class of
 * lco_max, the shorter series' longest length), as eap_tune_nn1 would; lets
 * a caller reuse tuning results or pin a shape.  EINVAL for shapes that do
 * not exist.  The distance swept as DTW (CDTW without a window) is keyed as
 * DTW. */
eap_status eap_tune_set(int32_t kind, int32_t precision, int64_t lco_max, int32_t g, int32_t c);
/* Forgets every tuned shape (later calls use the defaults). */
eap_status eap_tune_reset(void);

/* HIP graphs of NN searches.  eap_capture_begin() starts capturing `stream`
 * (thread-local capture mode); every eap_nn1 call made on it until
 * eap_capture_end() must carry flags bit 2 (prepared: run once uncaptured
 * first, on the same workspace and inputs) and is recorded, not run.
 * eap_capture_end() instantiates the graph; eap_graph_launch() replays all the
 * recorded searches with one launch, on the buffers they were recorded with
 * (their contents may change between launches, their sizes and addresses may
 * not).  The graph contains kernels only (buffers are cleared by kernels, not
 * memset nodes).  eap_graph_destroy() frees it (NULL is accepted). */
typedef struct eap_graph eap_graph;
eap_status eap_capture_begin(void* stream);
eap_status eap_capture_end(void* stream, eap_graph** out);
eap_status eap_graph_launch(eap_graph* g, void* stream);
eap_status eap_graph_destroy(eap_graph* g);

/* Request server: 1-NN queries arriving one by one against a candidate set
 * resident on the device, answered in batches that overlap on the device.
 * The caller owns the candidate arrays (they must outlive the server); the
 * server allocates, once, in eap_server_create(), a device pool of
 * mem_budget bytes split evenly into `slots`, plus pinned host buffers.
 * Queries wait in a FIFO (host copies of their values).  eap_server_poll()
 * never blocks: it returns the results of batches that have completed, then
 * admits waiting queries into every free slot, as many (at most max_batch, in
 * arrival order) as fit the slot's bytes with their values, NN workspace and
 * outputs (admission by memory), and starts each such batch as one eap_nn1
 * call on the slot's own stream.  Each result is the one eap_nn1 gives for
 * that query alone (NN search does not couple queries).  One thread at a
 * time per server.  Errors of these calls are reported by
 * eap_server_last_error(). */
typedef struct eap_server eap_server;
typedef struct {
    int32_t slots;          /* batches in flight at most, 1..16 */
    int32_t max_batch;      /* queries per batch at most */
    int64_t max_query_len;  /* longest query accepted */
    size_t mem_budget;      /* device bytes for all slots */
    int32_t precision;      /* as eap_nn_opts */
    double margin_rel;
} eap_server_opts;
typedef struct {
    int64_t tag;      /* as submitted */
    int64_t idx;      /* NN index, -1 when no candidate is finite */
    double dist;      /* its distance, or +inf */
    int32_t label;    /* r_labels[idx], or -1 */
    int32_t status;   /* 0 */
} eap_result;
typedef struct {
    int64_t batches, queries, max_batch_seen, max_inflight, waiting;
} eap_server_stats;
eap_status eap_server_create(const double* refs, const int64_t* r_off, int64_t nr, const int32_t* r_labels,
                             const eap_params* p, const eap_server_opts* o, eap_server** out);
/* Queue a query of `len` host float64 values (copied). */
eap_status eap_server_submit(eap_server* s, const double* q, int64_t len, int64_t tag);
/* Up to `cap` results into `out` (host), their number in *n; see above. */
eap_status eap_server_poll(eap_server* s, eap_result* out, int32_t cap, int32_t* n);
eap_status eap_server_stats_get(const eap_server* s, eap_server_stats* out);
/* The sweep counters of every batch the server has run, summed over its
 * slots (see eap_counters; a slot's workspace keeps accumulating them).
 * Waits for the batches in flight. */
eap_status eap_server_counters(const eap_server* s, eap_counters* out);
/* Waits for the batches in flight and frees everything (NULL is accepted). */
eap_status eap_server_destroy(eap_server* s);
const char* eap_server_last_error(void);

/* Host utility: the WDTW weights the library uses for longer length L,
 * out[k] = w(k) = 1 / (1 + exp(-g * (k - L/2))) for k = 0..L-1 (eq. WDTW with
 * w_max = 1).  `out` is HOST memory of L doubles.  Lets a caller check the
 * library's weights against another implementation bit for bit. */
eap_status eap_wdtw_weights(double g, int64_t L, double* out);

/* Host utilities: the certified error bound of the FP32 screen (precision 1).
 * eap_screen_eps(kind, exact_diff, B, N, A) bounds |V32 - B| for any warping
 * path of exact cost B with at most N steps over values of magnitude <= A
 * (ERP: also >= |gap|), V32 being the path's cost evaluated in FP32 as the
 * recurrence adds it; exact_diff != 0 when each difference is formed in
 * float64 and rounded once (no input rounding).  eap_screen_bound(kind,
 * exact_diff, b, N, A) is the largest exact cost C with C <= b + eps(C).
 * The derivation is in the library's eap_screen.h.  NaN for an unknown kind. */
double eap_screen_eps(int32_t kind, int32_t exact_diff, double B, double N, double A);
double eap_screen_bound(int32_t kind, int32_t exact_diff, double b, double N, double A);

/* Thread-local text of the last error on this thread; valid until the next call. */
const char* eap_last_error(void);

/* Library version string. */
const char* eap_version(void);

/* Content hash (16 hex digits) of the sources the library was built from;
 * the Python binding refuses a library whose hash differs from the sources
 * beside it, so a stale build is never used silently. */
const char* eap_source_hash(void);

#ifdef __cplusplus
}
#endif
#endif /* EAP_H */
