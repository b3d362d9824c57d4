// C ABI of libeap (see include/eap.h): argument checks, workspace layout,
// kernel selection and the launch sequences of distance, NN search and
// pairwise matrices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "eap.h"
#include "eap_internal.h"
#include "eap_launch.h"
#include "eap_screen.h"

using namespace eap;

namespace {

thread_local std::string g_err;

eap_status fail(eap_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(EAP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int64_t kMaxLen = 2048;     // longest series the sweep kernels take
constexpr int kRowsBlocksPerCU = 4;   // persistent grid of the row sweep
constexpr size_t kAlign = 256;

// ---------------------------------------------------------------- parameters
eap_status check_params(const eap_params* p) {
    if (!p) return fail(EAP_EINVAL, "params is NULL");
    if (p->kind < EAP_DTW || p->kind > EAP_TWE) return fail(EAP_EINVAL, "unknown distance kind %d", p->kind);
    if (p->kind == EAP_CDTW || p->kind == EAP_ERP) {
        if (std::isnan(p->window_ratio) || p->window_ratio < 0)
            return fail(EAP_EINVAL, "window_ratio must be >= 0 (got %g)", p->window_ratio);
    }
    if (p->kind == EAP_WDTW && !(std::isfinite(p->g) && p->g >= 0))
        return fail(EAP_EINVAL, "WDTW g must be finite and >= 0");
    if (p->kind == EAP_ERP && !std::isfinite(p->gap)) return fail(EAP_EINVAL, "ERP gap must be finite");
    if (p->kind == EAP_MSM && !(std::isfinite(p->c) && p->c >= 0)) return fail(EAP_EINVAL, "MSM c must be >= 0");
    if (p->kind == EAP_TWE && !(std::isfinite(p->nu) && p->nu >= 0 && std::isfinite(p->lambda) && p->lambda >= 0))
        return fail(EAP_EINVAL, "TWE nu and lambda must be finite and >= 0");
    if (p->dims < 0 || p->dims > 4) return fail(EAP_EINVAL, "dims must be 0..4 (got %d)", p->dims);
    if (p->dims > 1 && p->kind != EAP_DTW && p->kind != EAP_CDTW)
        return fail(EAP_EINVAL, "multivariate series (dims > 1) are supported for DTW and CDTW only");
    return EAP_OK;
}

// Channels per series point (1: univariate).
int dims_of(const eap_params* p) { return p->dims > 1 ? p->dims : 1; }

bool windowed(const eap_params* p) {
    return (p->kind == EAP_CDTW || p->kind == EAP_ERP) && p->window_ratio < 1.0;
}

// Distance actually swept: CDTW without a window is DTW.
int effective_kind(const eap_params* p) {
    if (p->kind == EAP_CDTW && !windowed(p)) return EAP_DTW;
    return p->kind;
}

struct SetInfo {
    int64_t n = 0, total = 0, maxlen = 0, minlen = 0;
};

eap_status check_offsets(const int64_t* off, int64_t n, const char* what, SetInfo* info) {
    if (!off) return fail(EAP_EINVAL, "%s offsets are NULL", what);
    if (n < 1) return fail(EAP_EINVAL, "%s: need at least one series", what);
    if (off[0] != 0) return fail(EAP_EINVAL, "%s offsets must start at 0", what);
    int64_t mx = 0, mn = INT64_MAX;
    for (int64_t k = 0; k < n; ++k) {
        int64_t L = off[k + 1] - off[k];
        if (L < 1) return fail(EAP_EINVAL, "%s series %lld has length %lld (< 1)", what, (long long)k, (long long)L);
        mx = std::max(mx, L);
        mn = std::min(mn, L);
    }
    if (mx > kMaxLen) return fail(EAP_EINVAL, "%s: series longer than %lld are not supported", what, (long long)kMaxLen);
    if (off[n] > (int64_t)INT32_MAX) return fail(EAP_EINVAL, "%s: too many values", what);
    info->n = n;
    info->total = off[n];
    info->maxlen = mx;
    info->minlen = mn;
    return EAP_OK;
}

// --------------------------------------------------------- workspace layout
struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + kAlign - 1) / kAlign * kAlign;
        return o;
    }
};

// Header at the start of every workspace.
struct Header {
    // [0] cells, [1] pairs, [2] rechecks, [3] overflows, [8+s] cells and
    // [16+s] pairs of stage s (s < 8)
    unsigned long long counters[32];
    unsigned int queues[16];
    unsigned int ovf_count[4];   // [0] band overflows, [2] FP64 recheck items, [3] CDTW pairs past the
                                 // lower bound (u64 fills clear [0..1])
    unsigned long long absmax;   // FP32 screen: largest |value| (double bits)
    // kept across calls: largest |value| of the candidates (NN, precision 1),
    // reused by calls with the candidates-prepared flag
    unsigned long long absmax_r;
};
constexpr int kCounterWords = 32;
// Workspace checks shared by the drivers: present, 256-byte aligned (kernels
// read parts of it in aligned vectors), and at least `need` bytes.
static eap_status check_ws(const void* ws, size_t ws_bytes, size_t need) {
    if (!ws || ws_bytes < need) return fail(EAP_EWORKSPACE, "workspace of %zu bytes, need %zu", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0)
        return fail(EAP_EWORKSPACE, "workspace must be %zu-byte aligned", kAlign);
    return EAP_OK;
}

// Candidate sets from this size on are read in their own layout by the CDTW
// bound + LB_Keogh kernel (no interleaved copy).
constexpr int64_t kDirectReadMinCandidates = int64_t(1) << 18;

constexpr size_t kHeaderBytes = (sizeof(Header) + kAlign - 1) / kAlign * kAlign;
// header words cleared by every call: the queues, counts and absmax
constexpr int kClearedWords = (int)(offsetof(Header, absmax_r) / 8) - kCounterWords;

// ------------------------------------------------------------------ tables
// WDTW: G[m] = 1 / (1 + exp(-g * (m / 2))) for m = 2k - L; the weight of
// |i-j| = k for longer length L is G[2k - L] (eq. WDTW with w_max = 1:
// (double)k - (double)L / 2 equals m / 2 exactly).  Layout: kWdtwZero zeros,
// then m = -Lmax .. Lmax + kWdtwHi at index m + Lmax + kWdtwZero.  The row
// sweep reads its window without bounds checks, as the larger of the entries
// of 2d - L and -2d - L (entries never decrease for g >= 0): with rows from
// -(G + K) to L + G + 2K and columns up to L + W + C, |d| <= L + W + G + 3K +
// C <= L + 2240 (G <= 64, K <= 32, C <= 32, W <= 2048), so m <= Lmax + 4480;
// the other side of a window that crosses d = 0 reaches down to m = -L -
// 2 (C + K - 2) >= -Lmax - 92, inside the zeros.
constexpr int64_t kWdtwZero = 128, kWdtwHi = 4608;
int64_t wdtw_table_len(int64_t lmax) { return kWdtwZero + 2 * lmax + kWdtwHi + 1; }
int64_t wdtw_table_off(int64_t lmax) { return lmax + kWdtwZero; }
double wdtw_entry(double g, int64_t lmax, int64_t e) {
    if (e < kWdtwZero) return 0.0;
    const int64_t m = e - wdtw_table_off(lmax);
    return 1.0 / (1.0 + std::exp(-g * ((double)m / 2.0)));
}
void wdtw_table(double g, int64_t lmax, std::vector<double>& t, int& off) {
    off = (int)wdtw_table_off(lmax);
    t.resize((size_t)wdtw_table_len(lmax));
    for (size_t e = 0; e < t.size(); ++e) t[e] = wdtw_entry(g, lmax, (int64_t)e);
}

// TWE: nu * (2|k|) for k = j - i in [-Lmax, Lmax + 1024] (eq. TWECost with tau_i = i).
// TWE's per-diagonal term nu * 2|d| for d = j - i.  The row sweep reads a
// window of C + K - 1 consecutive entries per lane and block without bounds
// checks, also for cells outside the matrix: with rows from -(G + K) to
// L + G + 2K and first columns up to L + W, d stays within
// [-(lmax + G + 3K), lmax + W + G + K + C] = [-(lmax + 160), lmax + 1136] for
// G <= 64, K <= 32, C <= 16, W <= 1024, inside the table's range.
constexpr int64_t kTweLo = 256, kTweHi = 1280;
int64_t twe_table_len(int64_t lmax) { return 2 * lmax + kTweLo + kTweHi + 1; }
void twe_table(double nu, int64_t lmax, std::vector<double>& t, int& off) {
    off = (int)(lmax + kTweLo);
    t.resize((size_t)twe_table_len(lmax));
    for (int64_t k = -(lmax + kTweLo); k <= lmax + kTweHi; ++k)
        t[(size_t)(k + lmax + kTweLo)] = nu * (double)(2 * (k < 0 ? -k : k));
}

// Pinned staging for host-to-device copies: a ring of buffers, each reused
// only after the copy issued from it last time has completed, so calls on
// different streams do not wait for each other.
struct StagingSlot {
    void* buf = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};
struct Staging {
    std::mutex mu;
    StagingSlot slot[32];
    unsigned next = 0;
};
Staging g_stage;

eap_status upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return EAP_OK;
    std::lock_guard<std::mutex> lk(g_stage.mu);
    StagingSlot& sl = g_stage.slot[g_stage.next++ % 32];
    if (sl.pending) {
        HIPCHK(hipEventSynchronize(sl.ev));
        sl.pending = false;
    }
    if (!sl.ev) HIPCHK(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    if (sl.cap < bytes) {
        if (sl.buf) HIPCHK(hipHostFree(sl.buf));
        sl.buf = nullptr;
        sl.cap = 0;
        size_t cap = std::max<size_t>(bytes, 1 << 16);
        if (hipHostMalloc(&sl.buf, cap, hipHostMallocDefault) != hipSuccess)
            return fail(EAP_ENOMEM, "pinned staging buffer of %zu bytes", cap);
        sl.cap = cap;
    }
    std::memcpy(sl.buf, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, sl.buf, bytes, hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(sl.ev, s));
    sl.pending = true;
    return EAP_OK;
}

int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, dev) == hipSuccess) cus[dev] = pr.multiProcessorCount;
        else cus[dev] = 256;
    }
    return cus[dev];
}

int sweep_grid(int64_t items, int group_lanes) {
    const int groups_per_block = 256 / group_lanes;
    int64_t need = (items + groups_per_block - 1) / groups_per_block;
    int64_t cap = (int64_t)device_cus() * 8;
    return (int)std::max<int64_t>(1, std::min(need, cap));
}

int rows_grid(int64_t items, int group_lanes) {
    const int groups_per_block = 256 / group_lanes;
    int64_t need = (items + groups_per_block - 1) / groups_per_block;
    int64_t cap = (int64_t)device_cus() * kRowsBlocksPerCU;
    return (int)std::max<int64_t>(1, std::min(need, cap));
}

// Bytes of the row sweep's strip-edge buffers for a launch over `items` work
// slots: one column of L_li + 1 values per group, for the most groups any
// shape launches (4 lanes per pair, 64 groups per block); none when every
// pair fits one strip of the narrowest shape (32 columns).
size_t edge_bytes(int64_t items, int64_t lli_max, int64_t lco_max) {
    if (lco_max <= 32) return 0;
    const int64_t groups = std::min<int64_t>((items + 63) / 64 * 64, (int64_t)device_cus() * kRowsBlocksPerCU * 64);
    return (size_t)groups * (size_t)(lli_max + 1) * sizeof(double);
}

// Default lanes per pair of the band sweep: 8 diagonals per parity and lane
// for the narrow bands (32, 64), else 4 or 8 from the band's width.
int band_group(int diags) {
    return diags == 32 ? 2 : (diags == 64 ? 4 : (diags <= 256 ? 16 : (diags == 512 ? 32 : 64)));
}

int pick_diags(int64_t need) {
    for (int d : {32, 64, 128, 256, 512, 1024, 2048})
        if (need <= d) return d;
    return 0;
}

// Row-sweep shapes: defaults, the autotuned table, and the tuner's override.
int len_bucket(int64_t lco_max) {
    int b = 0;
    while (b < 5 && lco_max > ((int64_t)128 << b)) ++b;
    return b;
}

RowsShape default_shape(int kind, bool fp32, int64_t lco_max) {
    int c = 16;
    if (!fp32 && (kind == EAP_TWE || kind == EAP_WDTW)) c = 8;   // their FP64 registers
    for (int g : {16, 32, 64})
        if ((int64_t)g * c >= lco_max) return RowsShape{g, c};
    return RowsShape{64, c};
}

std::mutex g_tune_mu;
std::map<int, RowsShape> g_tuned;                // key: (kind * 2 + fp32) * 8 + bucket
std::map<int, int> g_tuned_band;                 // key: (kind * 2 + fp32) * 16 + log2(diagonals)
thread_local RowsShape g_force[2] = {{0, 0}, {0, 0}};   // [fp32], set while tuning
thread_local int g_force_band[2] = {0, 0};

RowsShape rows_shape(int kind, bool fp32, int64_t lco_max) {
    if (g_force[fp32].g) return g_force[fp32];
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find((kind * 2 + (fp32 ? 1 : 0)) * 8 + len_bucket(lco_max));
    if (it != g_tuned.end()) return it->second;
    return default_shape(kind, fp32, lco_max);
}

int log2i(int x) {
    int b = 0;
    while ((1 << (b + 1)) <= x) ++b;
    return b;
}

// Lanes per pair of the band sweep for a band of `diags` diagonals.
int band_lanes(int kind, bool fp32, int diags) {
    if (g_force_band[fp32] && band_shape_ok(diags, g_force_band[fp32])) return g_force_band[fp32];
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned_band.find((kind * 2 + (fp32 ? 1 : 0)) * 16 + log2i(diags));
    if (it != g_tuned_band.end()) return it->second;
    return band_group(diags);
}

// Shape for launches with few pairs (one per query: the seed and recheck
// sweeps, both FP64), which are bound by the latency of a pair's chain of
// steps rather than by throughput: 64 lanes per pair and the fewest columns
// per lane (steps take time in proportion to the columns a lane owns).  ERP,
// MSM and TWE keep 8 columns per lane at any length: with 16 their FP64 lanes
// spill registers inside the step loop.
RowsShape latency_shape(int kind, int64_t lco_max) {
    if (kind == EAP_ERP || kind == EAP_MSM || kind == EAP_TWE) return RowsShape{64, 8};
    return RowsShape{64, lco_max <= 512 ? 8 : 16};
}

// What the sweep of one distance needs, for sets whose longest series have
// lengths la_max and lb_max.
struct Plan {
    bool band = false;     // kernel B (true) or kernel A
    int size = 0;          // B: diagonals
    int band_half = 0;     // B, WDTW: half width of the certified narrow band
    bool rerun = false;    // B, WDTW: items the narrow band cannot certify go to kernel A
    RowsShape r64{16, 16}, r32{16, 16};   // kernel A shapes per precision
    int bg64 = 16, bg32 = 16;             // kernel B lanes per pair per precision
};

eap_status make_plan(const eap_params* p, int64_t la_max, int64_t lb_max, int64_t l_diff_max, bool narrow_first,
                     Plan* pl) {
    const int kind = effective_kind(p);
    const int64_t lmax = std::max(la_max, lb_max);
    const int64_t lco_max = std::min(la_max, lb_max);
    pl->r64 = rows_shape(kind, false, lco_max);
    pl->r32 = rows_shape(kind, true, lco_max);
    pl->band = false;
    pl->rerun = false;
    if (dims_of(p) > 1) {
        // multivariate DTW and CDTW: the row sweep, 8 columns per lane, the
        // narrowest group whose strip holds the shorter series
        int g = 64;
        for (int c : {8, 16, 32})
            if ((int64_t)c * 8 >= lco_max) {
                g = c;
                break;
            }
        pl->r64 = pl->r32 = RowsShape{g, 8};
        return EAP_OK;
    }
    if (kind == EAP_CDTW || (kind == EAP_ERP && windowed(p))) {
        pl->band = true;
        int64_t w = (int64_t)std::floor(p->window_ratio * (double)lmax);
        int64_t wb = std::min<int64_t>(w + (kind == EAP_ERP ? 1 : 0), lmax);
        pl->size = pick_diags(2 * wb + 2);
        if (!pl->size) return fail(EAP_EINVAL, "window too wide for the band sweep");
        pl->bg64 = band_lanes(kind, false, pl->size);
        pl->bg32 = band_lanes(kind, true, pl->size);
        return EAP_OK;
    }
    // WDTW in an NN search with lengths that differ little: a certified narrow
    // band around the diagonal first, the row sweep for the items it cannot certify
    if (kind == EAP_WDTW && narrow_first && l_diff_max <= 64) {
        pl->band = true;
        pl->size = 256;
        pl->band_half = (int)std::max<int64_t>(16, (256 - 2 - l_diff_max) / 2);
        pl->rerun = true;
        pl->bg64 = band_lanes(kind, false, pl->size);
        pl->bg32 = band_lanes(kind, true, pl->size);
    }
    return EAP_OK;
}

SweepArgs base_args(const eap_params* p) {
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.gap = p->gap;
    a.c = p->c;
    a.nu = p->nu;
    a.lam = p->lambda;
    a.window_ratio = windowed(p) ? p->window_ratio : 2.0;
    return a;
}

// Device regions shared by the drivers for one (set A, set B) problem.
struct Common {
    size_t hdr = 0, offA = 0, offB = 0, bordA = 0, bordB = 0, tab = 0, gtab = 0;
    std::vector<double> tabv, gtabv;   // host copies (empty when the tables are not built on the host)
    int tab_off = 0, gtab_off = 0, tab_len = 0, gtab_len = 0;
    int64_t lmax = 0;
};

// Region offsets of the common part; with build_tables the TWE / WDTW tables
// are also built on the host (for upload), else only their places are taken.
void plan_common(Layout& L, Common& c, const eap_params* p, const SetInfo& A, const SetInfo* B,
                 bool build_tables = true) {
    c.hdr = L.take(kHeaderBytes);
    c.offA = L.take(sizeof(int64_t) * (size_t)(A.n + 1));
    if (B) c.offB = L.take(sizeof(int64_t) * (size_t)(B->n + 1));
    const int64_t lmax = std::max(A.maxlen, B ? B->maxlen : 0);
    c.lmax = lmax;
    if (p->kind == EAP_ERP) {
        c.bordA = L.take(sizeof(double) * (size_t)A.total);
        if (B) c.bordB = L.take(sizeof(double) * (size_t)B->total);
    }
    if (p->kind == EAP_TWE) {
        if (build_tables) twe_table(p->nu, lmax, c.tabv, c.tab_off);
        c.tab_off = (int)(lmax + kTweLo);
        c.tab_len = (int)twe_table_len(lmax);
        c.tab = L.take(sizeof(double) * (size_t)c.tab_len);
    }
    if (p->kind == EAP_WDTW) {
        if (build_tables) wdtw_table(p->g, lmax, c.gtabv, c.gtab_off);
        c.gtab_off = (int)wdtw_table_off(lmax);
        c.gtab_len = (int)wdtw_table_len(lmax);
        c.gtab = L.take(sizeof(double) * (size_t)c.gtab_len);
    }
}

char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

eap_status setup_common(void* ws, const Common& c, const eap_params* p, const double* va, const int64_t* offa,
                        int64_t na, const double* vb, const int64_t* offb, int64_t nb, hipStream_t s,
                        SweepArgs& a, SeriesPtrs& SA, SeriesPtrs& SB, bool prepared = false,
                        bool b_ready = false) {
    eap_status st;
    // work queues and overflow counts start at zero; the counters keep accumulating
    HIPCHK(launch_fill_u64(reinterpret_cast<unsigned long long*>(at(ws, c.hdr)) + kCounterWords, 0ull,
                           kClearedWords, s));
    // offsets and tables: uploaded, unless a previous call with the same
    // inputs left them in this workspace (the only host-to-device copies, so a
    // prepared call enqueues kernels only and can be captured in a graph)
    if (!prepared && (st = upload(at(ws, c.offA), offa, sizeof(int64_t) * (size_t)(na + 1), s)) != EAP_OK)
        return st;
    // set B's offsets and ERP borders: also kept when a previous call left them
    // (b_ready: the NN candidates, unchanged since)
    if (!prepared && !b_ready && offb &&
        (st = upload(at(ws, c.offB), offb, sizeof(int64_t) * (size_t)(nb + 1), s)) != EAP_OK)
        return st;
    const int64_t* dA = reinterpret_cast<const int64_t*>(at(ws, c.offA));
    const int64_t* dB = offb ? reinterpret_cast<const int64_t*>(at(ws, c.offB)) : dA;
    SA = SeriesPtrs{va, dA, nullptr};
    SB = SeriesPtrs{vb ? vb : va, dB, nullptr};
    if (p->kind == EAP_ERP) {
        double* bA = reinterpret_cast<double*>(at(ws, c.bordA));
        HIPCHK(launch_erp_border(va, dA, na, p->gap, bA, s));
        SA.border = bA;
        if (offb) {
            double* bB = reinterpret_cast<double*>(at(ws, c.bordB));
            if (!b_ready) HIPCHK(launch_erp_border(vb, dB, nb, p->gap, bB, s));
            SB.border = bB;
        } else {
            SB.border = bA;
        }
    }
    if (p->kind == EAP_TWE) {
        if (!prepared && (st = upload(at(ws, c.tab), c.tabv.data(), sizeof(double) * c.tabv.size(), s)) != EAP_OK)
            return st;
        a.tab = reinterpret_cast<const double*>(at(ws, c.tab));
        a.tab_off = c.tab_off;
        a.tab_len = c.tab_len;
    }
    if (p->kind == EAP_WDTW) {
        if (!prepared && (st = upload(at(ws, c.gtab), c.gtabv.data(), sizeof(double) * c.gtabv.size(), s)) != EAP_OK)
            return st;
        a.gtab = reinterpret_cast<const double*>(at(ws, c.gtab));
        a.gtab_off = c.gtab_off;
        a.gtab_len = c.gtab_len;
    }
    Header* h = reinterpret_cast<Header*>(at(ws, c.hdr));
    a.counters = h->counters;
    return EAP_OK;
}

Header* hdr_of(void* ws, const Common& c) { return reinterpret_cast<Header*>(at(ws, c.hdr)); }

// Optional event timing of sweep launches.
struct ProfRec {
    eap_profile_rec r;
    hipEvent_t e0, e1;
};
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<ProfRec> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
Profiler g_prof;

// One sweep launch (kernel A or B) over `n` work slots, counted under `stage`.
// timed = false: never bracketed by profiling events (the call that makes no
// allocation of any kind may not create them).
eap_status sweep(const eap_params* p, const Plan& pl, bool band, SweepArgs a, Header* h, int stage,
                 unsigned int* queue, const int32_t* items, int64_t n, SeriesPtrs SA, SeriesPtrs SB, hipStream_t s,
                 bool fp32 = false, bool timed = true, bool xd = false) {
    if (xd && band) return fail(EAP_EINVAL, "exact-difference FP32 sweeps run on the row sweep only");
    a.queue = queue;
    a.items = items;
    a.npairs = n;
    a.stage = &h->counters[8 + stage];
    // seed stages (0, 1): a few pairs per query, and a search's main sweep
    // waits for them; rechecks (4, 5) keep the normal priority, so that beside
    // another search's main sweep they take only the issue slots it leaves
    a.prio = (stage == 0 || stage == 1) ? 1 : 0;
    const int kind = effective_kind(p);
    const RowsShape sh = fp32 ? pl.r32 : pl.r64;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
    if (cap == hipStreamCaptureStatusNone && timed) {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (g_prof.on) {
            e0 = g_prof.get();
            e1 = g_prof.get();
        }
    }
    if (e0 && e1) HIPCHK(hipEventRecord(e0, s));
    (void)hipGetLastError();   // launch errors below must be this launch's own
    hipError_t e;
    const int lanes = band ? (fp32 ? pl.bg32 : pl.bg64) : sh.g;
    int grid = band ? sweep_grid(n, lanes) : rows_grid(n, lanes);
    {
        // a persistent grid no larger than what the device holds at once:
        // blocks beyond it only start once the work has run out, yet
        // measurably slow the sweep (up to a quarter for the band sweep)
        int occ = 0;
        const hipError_t oe = band ? launch_band(kind, fp32, pl.size, lanes, a, SA, SB, grid, s, &occ)
                                   : launch_rows(kind, fp32, sh, a, SA, SB, grid, s, &occ, xd, dims_of(p));
        if (oe == hipSuccess && occ > 0) grid = std::min(grid, device_cus() * occ);
    }
    // slots per queue atomic: about 8 chunks per group, so that short items
    // (infeasible windows) do not serialise on the counter and long ones still
    // balance; one at a time when the count is only known on the device
    const int64_t groups = (int64_t)grid * (256 / lanes);
    a.chunk = a.npairs_dev ? 1 : (int)std::max<int64_t>(1, std::min<int64_t>(32, n / (groups * 8)));
    if (band) e = launch_band(kind, fp32, pl.size, lanes, a, SA, SB, grid, s);
    else e = launch_rows(kind, fp32, sh, a, SA, SB, grid, s, nullptr, xd, dims_of(p));
    if (e != hipSuccess) return fail(EAP_EDEVICE, "sweep launch: %s", hipGetErrorString(e));
    if (e0 && e1) {
        HIPCHK(hipEventRecord(e1, s));
        std::lock_guard<std::mutex> lk(g_prof.mu);
        ProfRec pr;
        pr.r = eap_profile_rec{stage, band ? 1 : 0, kind, band ? pl.size : sh.g * sh.c, fp32 ? 1 : 0, 0.0f,
                               lanes, xd ? 1 : 0};
        pr.e0 = e0;
        pr.e1 = e1;
        g_prof.pending.push_back(pr);
    }
    return EAP_OK;
}

// Items of the narrow band pass that could not be certified are swept again by
// the row sweep.  Their list and count stay on the device: the re-run reads
// the count at run time, so nothing synchronises the host.
eap_status rerun_overflow(const eap_params* p, const Plan& pl, SweepArgs a, Header* h, int stage,
                          unsigned int* ovf_count, const int32_t* ovf_items, int64_t max_items, unsigned int* queue,
                          SeriesPtrs SA, SeriesPtrs SB, hipStream_t s, bool fp32 = false, bool xd = false) {
    a.ovf_items = nullptr;
    a.ovf_count = nullptr;
    a.npairs_dev = ovf_count;
    a.skip_b = nullptr;
    return sweep(p, pl, false, a, h, stage, queue, ovf_items, max_items, SA, SB, s, fp32, true, xd);
}

}  // namespace

// ------------------------------------------- distance without allocation
// Scratch of eap_distance_noalloc: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends.  Its largest layout
// (two series of 2048 values: header, offsets, ERP borders or a distance
// table, and the row sweep's strip edges for one block of 64 groups) is
// about 1.2 MB.
constexpr size_t kNoAllocScratchBytes = size_t(2) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
// Device address of `scratch` per device, taken once with that device current
// (the array's name is only a host-side stand-in, not a device address).
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {nullptr};

eap_status scratch_ptr(void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(EAP_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(EAP_EDEVICE, "no device address for the static scratch");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return EAP_OK;
}

// n host words to dst through kernel arguments, kPutWords per launch.
eap_status put_words(void* dst, const unsigned long long* src, int64_t n, hipStream_t s) {
    for (int64_t o = 0; o < n; o += kPutWords) {
        const int m = (int)std::min<int64_t>(kPutWords, n - o);
        HIPCHK(launch_put_u64(static_cast<unsigned long long*>(dst) + o, src + o, m, s));
    }
    return EAP_OK;
}

// A per-diagonal table (TWE: nu * 2|k|; WDTW: the weights), built on the host
// with the same expressions eap_distance uploads, a chunk at a time on the
// stack, and delivered through kernel arguments.
eap_status put_table(int kind, const eap_params* p, int64_t lmax, double* dst, hipStream_t s) {
    const int64_t len = (kind == EAP_TWE) ? twe_table_len(lmax) : wdtw_table_len(lmax);
    double buf[kPutWords];
    for (int64_t o = 0; o < len; o += kPutWords) {
        const int m = (int)std::min<int64_t>(kPutWords, len - o);
        for (int x = 0; x < m; ++x) {
            const int64_t e = o + x;
            if (kind == EAP_TWE) {
                const int64_t k = e - (lmax + kTweLo);
                buf[x] = p->nu * (double)(2 * (k < 0 ? -k : k));
            } else {
                buf[x] = wdtw_entry(p->g, lmax, e);
            }
        }
        unsigned long long w[kPutWords];
        std::memcpy(w, buf, sizeof(double) * (size_t)m);
        HIPCHK(launch_put_u64(reinterpret_cast<unsigned long long*>(dst + o), w, m, s));
    }
    return EAP_OK;
}
}  // namespace

// ====================================================================== ABI
extern "C" {

const char* eap_last_error(void) { return g_err.c_str(); }

const char* eap_version(void) { return "eap-mi355x 0.2 (gfx950)"; }

#ifndef EAP_SOURCE_HASH
#define EAP_SOURCE_HASH "unknown"
#endif
const char* eap_source_hash(void) { return EAP_SOURCE_HASH; }

// ------------------------------------------------------------------ distance
static void distance_layout(int64_t lx, int64_t ly, const eap_params* p, Layout& L, Common& c, size_t* ovf,
                            size_t* edge, bool build_tables = true) {
    SetInfo A, B;
    A.n = 1; A.total = lx; A.maxlen = A.minlen = lx;
    B.n = 1; B.total = ly; B.maxlen = B.minlen = ly;
    plan_common(L, c, p, A, &B, build_tables);
    *ovf = L.take(sizeof(int32_t) * 8);
    *edge = L.take(edge_bytes(1, std::max(lx, ly), std::min(lx, ly)));
}

size_t eap_distance_workspace(int64_t lx, int64_t ly, const eap_params* p) {
    if (check_params(p) != EAP_OK || lx < 1 || ly < 1) return 0;
    Layout L;
    Common c;
    size_t ovf, edge;
    distance_layout(lx, ly, p, L, c, &ovf, &edge);
    return L.off;
}

eap_status eap_distance(const double* x, int64_t lx, const double* y, int64_t ly, const eap_params* p, double cutoff,
                        double* out, void* ws, size_t ws_bytes, void* stream) {
    eap_status st;
    if ((st = check_params(p)) != EAP_OK) return st;
    if (!x || !y || !out) return fail(EAP_EINVAL, "NULL series or output");
    if (lx < 1 || ly < 1) return fail(EAP_EINVAL, "series lengths must be >= 1");
    if (lx > kMaxLen || ly > kMaxLen) return fail(EAP_EINVAL, "series longer than %lld are not supported", (long long)kMaxLen);
    if (std::isnan(cutoff) || cutoff < 0) return fail(EAP_EINVAL, "cutoff must be >= 0 or +inf");
    Layout L;
    Common c;
    size_t ovf, edge;
    distance_layout(lx, ly, p, L, c, &ovf, &edge);
    if (eap_status st_ws = check_ws(ws, ws_bytes, L.off)) return st_ws;
    Plan pl;
    if ((st = make_plan(p, lx, ly, std::llabs(lx - ly), false, &pl)) != EAP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t offa[2] = {0, lx}, offb[2] = {0, ly};
    SweepArgs a = base_args(p);
    SeriesPtrs SA, SB;
    if ((st = setup_common(ws, c, p, x, offa, 1, y, offb, 1, s, a, SA, SB)) != EAP_OK) return st;
    // the cut-off travels in the result slot: the kernel reads it from pcut[0]
    if ((st = upload(out, &cutoff, sizeof cutoff, s)) != EAP_OK) return st;
    a.mode = PM_SINGLE;
    a.nA = a.nB = 1;
    a.pcut = out;
    a.res = out;
    a.band_half = pl.band_half;
    a.ovf_items = reinterpret_cast<int32_t*>(at(ws, ovf));
    a.ovf_count = &hdr_of(ws, c)->ovf_count[0];
    a.edge = edge_bytes(1, std::max(lx, ly), std::min(lx, ly)) ? at(ws, edge) : nullptr;
    a.edge_stride = std::max(lx, ly) + 1;
    return sweep(p, pl, pl.band, a, hdr_of(ws, c), 2, &hdr_of(ws, c)->queues[0], nullptr, 1, SA, SB, s);
}


// ------------------------------------------- distance without allocation
eap_status eap_distance_noalloc(const double* x, int64_t lx, const double* y, int64_t ly, const eap_params* p,
                                double cutoff, double* out, void* stream) {
    eap_status st;
    if ((st = check_params(p)) != EAP_OK) return st;
    if (!x || !y || !out) return fail(EAP_EINVAL, "NULL series or output");
    if (lx < 1 || ly < 1) return fail(EAP_EINVAL, "series lengths must be >= 1");
    if (lx > kMaxLen || ly > kMaxLen) return fail(EAP_EINVAL, "series longer than %lld are not supported", (long long)kMaxLen);
    if (std::isnan(cutoff) || cutoff < 0) return fail(EAP_EINVAL, "cutoff must be >= 0 or +inf");
    Layout L;
    Common c;
    size_t ovf, edge;
    distance_layout(lx, ly, p, L, c, &ovf, &edge, /*build_tables=*/false);
    if (L.off > kNoAllocScratchBytes)
        return fail(EAP_EWORKSPACE, "eap_distance_noalloc needs %zu bytes of scratch; its static area holds %zu",
                    L.off, kNoAllocScratchBytes);
    void* ws = nullptr;
    if ((st = scratch_ptr(&ws)) != EAP_OK) return st;
    Plan pl;
    if ((st = make_plan(p, lx, ly, std::llabs(lx - ly), false, &pl)) != EAP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // what eap_distance uploads from staging memory arrives here through
    // kernel arguments: the offsets, the per-diagonal table and the cut-off
    const unsigned long long offw[2][2] = {{0ull, (unsigned long long)lx}, {0ull, (unsigned long long)ly}};
    if ((st = put_words(at(ws, c.offA), offw[0], 2, s)) != EAP_OK) return st;
    if ((st = put_words(at(ws, c.offB), offw[1], 2, s)) != EAP_OK) return st;
    if (p->kind == EAP_TWE || p->kind == EAP_WDTW) {
        double* tab = reinterpret_cast<double*>(at(ws, p->kind == EAP_TWE ? c.tab : c.gtab));
        if ((st = put_table(p->kind, p, c.lmax, tab, s)) != EAP_OK) return st;
    }
    const int64_t offa[2] = {0, lx}, offb[2] = {0, ly};
    SweepArgs a = base_args(p);
    SeriesPtrs SA, SB;
    // prepared: nothing left to upload (queues are cleared by a fill kernel)
    if ((st = setup_common(ws, c, p, x, offa, 1, y, offb, 1, s, a, SA, SB, /*prepared=*/true)) != EAP_OK) return st;
    unsigned long long cw;
    std::memcpy(&cw, &cutoff, sizeof cw);
    if ((st = put_words(out, &cw, 1, s)) != EAP_OK) return st;
    a.mode = PM_SINGLE;
    a.nA = a.nB = 1;
    a.pcut = out;
    a.res = out;
    a.band_half = pl.band_half;
    a.ovf_items = reinterpret_cast<int32_t*>(at(ws, ovf));
    a.ovf_count = &hdr_of(ws, c)->ovf_count[0];
    a.edge = edge_bytes(1, std::max(lx, ly), std::min(lx, ly)) ? at(ws, edge) : nullptr;
    a.edge_stride = std::max(lx, ly) + 1;
    return sweep(p, pl, pl.band, a, hdr_of(ws, c), 2, &hdr_of(ws, c)->queues[0], nullptr, 1, SA, SB, s,
                 /*fp32=*/false, /*timed=*/false);
}

// ---------------------------------------------------------------------- NN
// How the FP32 screen forms its differences.  Its certified error bound with
// FP32 inputs carries their rounding, about u * max|x| per difference, at any
// weight; WDTW's weights near the diagonal, 1 / (1 + exp(g L / 2)), make its
// distances so small for long series that this bound would list most
// candidates for the recheck.  Such WDTW searches sweep in FP32 with exact
// differences instead (float64 series, each difference rounded once), whose
// bound is relative.  WDTW keeps a weight of at least 1e-30 there, far inside
// the FP32 normal range, so the relative bound holds for the weights too.
bool screen_exact_diff(const eap_params* p, int64_t lmax) {
    if (p->kind != EAP_WDTW) return false;
    return 1.0 / (1.0 + std::exp(p->g * (double)lmax / 2.0)) < 1e-8;
}
bool screen_possible(const eap_params* p, int64_t lmax) {
    if (p->kind != EAP_WDTW || !screen_exact_diff(p, lmax)) return true;
    return 1.0 / (1.0 + std::exp(p->g * (double)lmax / 2.0)) >= 1e-30;
}

// Lower bounds a search uses (eap_nn_opts.lb resolved for the distance swept).
int lb_mode(const eap_params* p, const eap_nn_opts* o) {
    const int k = effective_kind(p);
    if ((k != EAP_DTW && k != EAP_CDTW) || dims_of(p) > 1) return EAP_LB_NONE;
    const int m = o ? o->lb : EAP_LB_DEFAULT;
    if (m == EAP_LB_DEFAULT) return k == EAP_CDTW ? EAP_LB_KEOGH : EAP_LB_NONE;
    return m;
}

struct NNLayout {
    Layout L;
    Common c;
    size_t best = 0, seed = 0, seed_items = 0, res = 0, ovf = 0, edge = 0, rT = 0, part = 0;
    size_t env = 0, lb = 0;     // lower bounds: query envelopes (env_stride layout) and the bound per pair
    size_t cenv = 0;            // reversed LB_Keogh: candidate envelopes, [position][nr], upper then lower
    // FP32 screen
    size_t q32 = 0, r32 = 0, q32b = 0, r32b = 0, widen = 0, recheck = 0;
};

// NN workspace.  The candidate side comes first (header, candidate offsets,
// ERP borders, interleaved copy, FP32 copies when precision is 1): its place
// depends on the candidates alone, so a later call on the same workspace with
// other queries and the candidates-prepared flag finds what an earlier call
// derived.  Then the query side and the per-pair arrays.
static eap_status nn_layout(const SetInfo& Q, const SetInfo& R, const eap_params* p, bool prec1, bool screen,
                            int lbm, NNLayout& nl) {
    Layout& L = nl.L;
    Common& c = nl.c;
    c.hdr = L.take(kHeaderBytes);
    c.offB = L.take(sizeof(int64_t) * (size_t)(R.n + 1));
    if (p->kind == EAP_ERP) c.bordB = L.take(sizeof(double) * (size_t)R.total);
    nl.rT = L.take(sizeof(double) * (size_t)(R.n * R.maxlen));
    if (prec1) {
        nl.r32 = L.take(sizeof(float) * (size_t)R.total);
        if (p->kind == EAP_ERP) nl.r32b = L.take(sizeof(float) * (size_t)R.total);
    }
    c.offA = L.take(sizeof(int64_t) * (size_t)(Q.n + 1));
    if (p->kind == EAP_ERP) c.bordA = L.take(sizeof(double) * (size_t)Q.total);
    const int64_t lmax = std::max(Q.maxlen, R.maxlen);
    c.lmax = lmax;
    if (p->kind == EAP_TWE) {
        twe_table(p->nu, lmax, c.tabv, c.tab_off);
        c.tab_len = (int)c.tabv.size();
        c.tab = L.take(sizeof(double) * c.tabv.size());
    }
    if (p->kind == EAP_WDTW) {
        wdtw_table(p->g, lmax, c.gtabv, c.gtab_off);
        c.gtab_len = (int)c.gtabv.size();
        c.gtab = L.take(sizeof(double) * c.gtabv.size());
    }
    nl.best = nl.L.take(sizeof(unsigned long long) * (size_t)Q.n);
    nl.part = nl.L.take(sizeof(double) * 2 * (size_t)scan_part_entries(Q.n));
    nl.seed = nl.L.take(sizeof(int32_t) * (size_t)Q.n);
    nl.seed_items = nl.L.take(sizeof(int32_t) * (size_t)Q.n);
    nl.res = nl.L.take(sizeof(double) * (size_t)(Q.n * R.n));
    nl.ovf = nl.L.take(sizeof(int32_t) * (size_t)(Q.n * R.n));
    if (lbm >= EAP_LB_KEOGH) {
        nl.env = nl.L.take(sizeof(double) * 3 * (size_t)env_stride(Q.n, R.maxlen));
        nl.lb = nl.L.take(sizeof(double) * (size_t)(Q.n * R.n));
    }
    if (lbm == EAP_LB_KEOGH2) nl.cenv = nl.L.take(sizeof(double) * 2 * (size_t)(Q.maxlen * R.n));
    nl.edge = nl.L.take(edge_bytes(Q.n * R.n, std::max(Q.maxlen, R.maxlen), std::min(Q.maxlen, R.maxlen)));
    if (screen) {
        nl.q32 = nl.L.take(sizeof(float) * (size_t)Q.total);
        if (p->kind == EAP_ERP) nl.q32b = nl.L.take(sizeof(float) * (size_t)Q.total);
        nl.widen = nl.L.take(sizeof(double) * (size_t)Q.n);
        nl.recheck = nl.L.take(sizeof(int32_t) * (size_t)(Q.n * R.n));
    }
    return EAP_OK;
}

size_t eap_nn1_workspace(const int64_t* q_off, int64_t nq, const int64_t* r_off, int64_t nr, const eap_params* p,
                         const eap_nn_opts* o) {
    (void)o;
    SetInfo Q, R;
    if (check_params(p) != EAP_OK || check_offsets(q_off, nq, "queries", &Q) != EAP_OK ||
        check_offsets(r_off, nr, "candidates", &R) != EAP_OK)
        return 0;
    NNLayout nl;
    const bool prec1 = o && o->precision == 1 && dims_of(p) == 1;
    nn_layout(Q, R, p, prec1, prec1 && screen_possible(p, std::max(Q.maxlen, R.maxlen)), lb_mode(p, o), nl);
    return nl.L.off;
}

eap_status eap_nn1(const double* q, const int64_t* q_off, int64_t nq, const double* r, const int64_t* r_off,
                   int64_t nr, const int32_t* r_labels, const eap_params* p, const eap_nn_opts* o, void* ws,
                   size_t ws_bytes, int64_t* out_idx, double* out_dist, int32_t* out_label, void* stream) {
    eap_status st;
    if ((st = check_params(p)) != EAP_OK) return st;
    if (!q || !r || !out_idx || !out_dist) return fail(EAP_EINVAL, "NULL series or output");
    SetInfo Q, R;
    if ((st = check_offsets(q_off, nq, "queries", &Q)) != EAP_OK) return st;
    if ((st = check_offsets(r_off, nr, "candidates", &R)) != EAP_OK) return st;
    if ((int64_t)nq * nr > (int64_t)INT32_MAX) return fail(EAP_EINVAL, "nq * nr exceeds 2^31 - 1");
    if (o) {
        if (o->precision != 0 && o->precision != 1) return fail(EAP_EINVAL, "precision must be 0 or 1");
        if (!(std::isfinite(o->margin_rel) && o->margin_rel >= 0)) return fail(EAP_EINVAL, "margin_rel must be >= 0");
        if (o->flags & ~63) return fail(EAP_EINVAL, "unknown flags 0x%x", (unsigned)o->flags);
        if ((o->flags & 16) && o->precision != 0) return fail(EAP_EINVAL, "prune-only search runs in FP64 (precision 0)");
        if (o->lb < EAP_LB_DEFAULT || o->lb > EAP_LB_KEOGH2) return fail(EAP_EINVAL, "unknown lb mode %d", o->lb);
    }
    const bool prec1 = o && o->precision == 1 && dims_of(p) == 1;   // multivariate: FP64
    const bool screen = prec1 && screen_possible(p, std::max(Q.maxlen, R.maxlen));
    const bool xd = screen && screen_exact_diff(p, std::max(Q.maxlen, R.maxlen));
    const int skind = effective_kind(p) | (xd ? kScreenExactDiff : 0);   // the screen bound's mode
    const int lbm = lb_mode(p, o);
    NNLayout nl;
    nn_layout(Q, R, p, prec1, screen, lbm, nl);
    if (eap_status st_ws = check_ws(ws, ws_bytes, nl.L.off)) return st_ws;
    Plan pl;
    const int64_t ldiff = std::max(std::llabs(Q.maxlen - R.minlen), std::llabs(R.maxlen - Q.minlen));
    const bool plain = o && (o->flags & 2);
    const bool prune_only = !plain && o && (o->flags & 16);
    const bool seeded = !plain && !prune_only && !(o && (o->flags & 1));
    const bool prepared = o && (o->flags & 4);
    const bool cand_ready = o && (o->flags & 8);
    // exact-difference sweeps run on the row sweep only (no narrow WDTW band)
    if ((st = make_plan(p, Q.maxlen, R.maxlen, ldiff, !plain && !xd, &pl)) != EAP_OK) return st;

    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone && !prepared)
        return fail(EAP_EINVAL, "a captured eap_nn1 needs prepared inputs (flags bit 2)");
    hipEvent_t main_wait = o ? static_cast<hipEvent_t>(o->main_wait) : nullptr;
    hipEvent_t main_done = o ? static_cast<hipEvent_t>(o->main_done) : nullptr;
    if (cap != hipStreamCaptureStatusNone && (main_wait || main_done))
        return fail(EAP_EINVAL, "main_wait / main_done must be NULL while the stream is captured");
    SweepArgs a = base_args(p);
    SeriesPtrs SQ, SR;
    if ((st = setup_common(ws, nl.c, p, q, q_off, nq, r, r_off, nr, s, a, SQ, SR, prepared, cand_ready)) != EAP_OK)
        return st;
    Header* h = hdr_of(ws, nl.c);
    double* rT = reinterpret_cast<double*>(at(ws, nl.rT));
    // The bound kernels read the interleaved copy of the candidates, except
    // CDTW with LB_Keogh over a very large candidate set, whose kernel reads
    // them in their own layout (building the copy would cost a full extra read
    // and write of the set).  The choice depends on the candidates and the
    // flags only, so calls with flags bit 3 find the copy when they need it.
    const bool lbk = lbm >= EAP_LB_KEOGH && !plain && !prune_only;
    const bool direct = lbk && nr >= kDirectReadMinCandidates;
    const bool need_rT = !direct && dims_of(p) == 1;
    if (!cand_ready) {
        // what the candidates alone determine, kept for calls with flags bit 3:
        // the interleaved copy (when a bound kernel reads it), and for precision
        // 1 the FP32 copies and |x| maximum, all in one pass over the candidates
        if (prec1) HIPCHK(launch_fill_u64(&h->absmax_r, 0ull, 1, s));
        if (need_rT || prec1)
            HIPCHK(launch_interleave(r, SR.off, nr, (int)R.maxlen, need_rT ? rT : nullptr,
                                     prec1 ? reinterpret_cast<float*>(at(ws, nl.r32)) : nullptr,
                                     prec1 ? &h->absmax_r : nullptr, s));
        if (prec1 && p->kind == EAP_ERP)
            HIPCHK(launch_to_f32(static_cast<const double*>(SR.border), R.total,
                                 reinterpret_cast<float*>(at(ws, nl.r32b)), s));
    } else if (need_rT && (effective_kind(p) == EAP_CDTW || effective_kind(p) == EAP_DTW) &&
               nr >= kDirectReadMinCandidates) {
        // an earlier call with LB_Keogh over this large set made no interleaved copy
        HIPCHK(launch_interleave(r, SR.off, nr, (int)R.maxlen, rT, nullptr, nullptr, s));
    }
    unsigned long long* best = reinterpret_cast<unsigned long long*>(at(ws, nl.best));
    int32_t* seed = reinterpret_cast<int32_t*>(at(ws, nl.seed));
    int32_t* seed_items = reinterpret_cast<int32_t*>(at(ws, nl.seed_items));
    double* res = reinterpret_cast<double*>(at(ws, nl.res));
    double* part = reinterpret_cast<double*>(at(ws, nl.part));
    int32_t* ovf = reinterpret_cast<int32_t*>(at(ws, nl.ovf));
    a.mode = PM_NN_ALL;
    a.nA = nq;
    a.nB = nr;
    a.best = best;
    a.res = res;
    a.band_half = pl.band_half;
    a.ovf_items = ovf;
    a.ovf_count = &h->ovf_count[0];
    a.edge = edge_bytes(nq * nr, std::max(Q.maxlen, R.maxlen), std::min(Q.maxlen, R.maxlen)) ? at(ws, nl.edge)
                                                                                             : nullptr;
    a.edge_stride = std::max(Q.maxlen, R.maxlen) + 1;
    a.no_prune = (o && (o->flags & 32)) ? 1 : 0;
    if (plain) {
        // baseline: every pair by the full dynamic programme
        a.plain = 1;
        if (main_wait) HIPCHK(hipStreamWaitEvent(s, main_wait, 0));
        if ((st = sweep(p, pl, pl.band, a, h, 2, &h->queues[2], nullptr, nq * nr, SQ, SR, s)) != EAP_OK)
            return st;
        if (main_done) HIPCHK(hipEventRecord(main_done, s));
        HIPCHK(launch_argmin(res, nq, nr, r_labels, out_idx, out_dist, out_label, part, s));
        return EAP_OK;
    }
    // 1. upper bounds from the diagonal path, the best of them seeds each query
    double* lb = lbk ? reinterpret_cast<double*>(at(ws, nl.lb)) : nullptr;
    if (dims_of(p) > 1)
        HIPCHK(launch_ub_mv(effective_kind(p), dims_of(p), false, a, q, SQ.off, r, SR.off, 0, res, s));
    else
        HIPCHK(launch_ub_nn(effective_kind(p), a, q, SQ.off, direct ? r : nullptr, SR.off, (int)Q.maxlen,
                            (int)R.maxlen, rT, res, lbk ? reinterpret_cast<double*>(at(ws, nl.env)) : nullptr, lb,
                            s));
    a.lb = lb;
    if (prune_only) {
        // Section 5's "Prune": each pair under its own path bound (one ulp
        // above it), no best-so-far shared between pairs, so nothing is
        // abandoned and every result is exact
        HIPCHK(launch_next_up(res, nq * nr, s));
        a.prune_only = 1;
        a.pcut = res;
        if (main_wait) HIPCHK(hipStreamWaitEvent(s, main_wait, 0));
        if ((st = sweep(p, pl, pl.band, a, h, 2, &h->queues[2], nullptr, nq * nr, SQ, SR, s)) != EAP_OK) return st;
        if (pl.rerun) {
            if ((st = rerun_overflow(p, pl, a, h, 3, &h->ovf_count[0], ovf, nq * nr, &h->queues[3], SQ, SR, s)) !=
                EAP_OK)
                return st;
        }
        if (main_done) HIPCHK(hipEventRecord(main_done, s));
        HIPCHK(launch_argmin(res, nq, nr, r_labels, out_idx, out_dist, out_label, part, s));
        return EAP_OK;
    }
    HIPCHK(launch_seed(res, nq, nr, seed, seed_items, best, part, s));
    const bool rerun = pl.rerun;
    // the seed and recheck sweeps have one or a few pairs per query
    Plan few = pl;
    few.r64 = few.r32 =
        dims_of(p) > 1 ? RowsShape{64, 8} : latency_shape(effective_kind(p), std::min(Q.maxlen, R.maxlen));
    if (seeded) {
        // 2. sweep the seed candidate of every query under its bound, in FP64
        //    also when screening: its exact distance is the tightest start for
        //    both passes, and the recheck need not compute it again
        if ((st = sweep(p, few, pl.band, a, h, 0, &h->queues[0], seed_items, nq, SQ, SR, s)) != EAP_OK) return st;
        if (rerun) {
            if ((st = rerun_overflow(p, few, a, h, 1, &h->ovf_count[0], ovf, nq, &h->queues[1], SQ, SR, s)) !=
                EAP_OK)
                return st;
            HIPCHK(launch_fill_u64(reinterpret_cast<unsigned long long*>(&h->ovf_count[0]), 0ull, 1, s));
        }
        a.skip_b = seed;
    }
    // FP32 screen: sweep single-precision copies under a widened cut-off
    SeriesPtrs XQ = SQ, XR = SR;   // exact differences: the sweep reads the float64 series
    if (screen && !xd) {
        float* q32 = reinterpret_cast<float*>(at(ws, nl.q32));
        float* r32 = reinterpret_cast<float*>(at(ws, nl.r32));
        HIPCHK(launch_to_f32(q, Q.total, q32, s));
        XQ = SeriesPtrs{q32, SQ.off, nullptr};
        XR = SeriesPtrs{r32, SR.off, nullptr};
        if (p->kind == EAP_ERP) {
            float* qb = reinterpret_cast<float*>(at(ws, nl.q32b));
            float* rb = reinterpret_cast<float*>(at(ws, nl.r32b));
            HIPCHK(launch_to_f32(static_cast<const double*>(SQ.border), Q.total, qb, s));
            XQ.border = qb;
            XR.border = rb;
        }
    }
    if (screen) {
        // |x| maximum over queries and candidates (theirs computed above or kept)
        HIPCHK(launch_fill_u64(&h->absmax, 0ull, 1, s));
        HIPCHK(launch_absmax(q, Q.total, &h->absmax, s));
        HIPCHK(launch_max_u64(&h->absmax, &h->absmax_r, s));
        double* widen = reinterpret_cast<double*>(at(ws, nl.widen));
        // best[q] is now the seed's FP64 distance or the path bound: the widening
        // at it bounds every best-so-far of the FP32 pass
        HIPCHK(launch_screen_widen(skind, a, SQ.off, R.maxlen, p->gap, &h->absmax, widen, s));
        a.widen_abs = widen;
        a.widen_rel = o->margin_rel;
    }
    // 3. every other pair, under the per-query best-so-far (lowered as pairs
    //    complete); for CDTW only the pairs whose LB_Keogh does not already
    //    exceed the seed's distance (listed in `ovf`, which CDTW does not use)
    SweepArgs m = a;
    const int32_t* main_items = nullptr;
    if (lbk) {
        HIPCHK(launch_lb_compact(lb, best, seeded ? seed : nullptr, SQ.off, SR.off, a.window_ratio, nq, nr, res, ovf,
                                 &h->ovf_count[3], &h->counters[4], s));
        main_items = ovf;
        m.npairs_dev = &h->ovf_count[3];
        m.skip_b = nullptr;
        if (lbm == EAP_LB_KEOGH2) {
            // the reversed LB_Keogh for the pairs kept: the candidates' envelopes
            // at the queries' positions, then each kept pair's larger bound; the
            // sweep drops a pair whose bound exceeds its query's cut-off
            double* cup = reinterpret_cast<double*>(at(ws, nl.cenv));
            double* clo = cup + (size_t)(Q.maxlen * nr);
            HIPCHK(launch_envelope(r, SR.off, nr, (int)R.maxlen, (int)Q.maxlen, (int)Q.maxlen, a.window_ratio, cup, clo,
                                   nullptr, 1, nr, s));
            HIPCHK(launch_lb_reverse(q, SQ.off, r, SR.off, nr, cup, clo, ovf, &h->ovf_count[3], nq * nr, lb, s));
        }
    }
    if (main_wait) HIPCHK(hipStreamWaitEvent(s, main_wait, 0));
    if ((st = sweep(p, pl, pl.band, m, h, 2, &h->queues[2], main_items, nq * nr, XQ, XR, s, screen, true, xd)) !=
        EAP_OK)
        return st;
    if (rerun) {
        if ((st = rerun_overflow(p, pl, a, h, 3, &h->ovf_count[0], ovf, nq * nr, &h->queues[3], XQ, XR, s, screen,
                                 xd)) != EAP_OK)
            return st;
    }
    if (main_done) HIPCHK(hipEventRecord(main_done, s));
    if (screen) {
        // 3b. candidates within the certified FP32 error of each query's best are
        //     recomputed in FP64 (the seed keeps its FP64 distance); every other
        //     result becomes +inf
        int32_t* items = reinterpret_cast<int32_t*>(at(ws, nl.recheck));
        HIPCHK(launch_screen_filter(skind, a, SQ.off, R.maxlen, p->gap, &h->absmax, o->margin_rel, res,
                                    best, seeded ? seed : nullptr, items, &h->ovf_count[2], &h->counters[2], part,
                                    s));
        HIPCHK(launch_fill_u64(reinterpret_cast<unsigned long long*>(&h->ovf_count[0]), 0ull, 1, s));
        SweepArgs b = a;
        b.widen_abs = nullptr;
        b.widen_rel = 0.0;
        b.skip_b = nullptr;
        b.npairs_dev = &h->ovf_count[2];
        if ((st = sweep(p, few, pl.band, b, h, 4, &h->queues[4], items, nq * nr, SQ, SR, s)) != EAP_OK) return st;
        if (rerun) {
            if ((st = rerun_overflow(p, few, b, h, 5, &h->ovf_count[0], ovf, nq * nr, &h->queues[5], SQ, SR, s)) !=
                EAP_OK)
                return st;
        }
    }
    // 4. lexicographic (distance, index) minimum per query
    HIPCHK(launch_argmin(res, nq, nr, r_labels, out_idx, out_dist, out_label, part, s));
    return EAP_OK;
}

// ---------------------------------------------------------------- pairwise
struct PWLayout {
    Layout L;
    Common c;
    size_t cut = 0, ovf = 0, edge = 0;
};

static void pw_layout(const SetInfo& S, const eap_params* p, PWLayout& pl) {
    plan_common(pl.L, pl.c, p, S, nullptr);
    const int64_t np = S.n * (S.n - 1) / 2;
    pl.cut = pl.L.take(sizeof(double) * (size_t)std::max<int64_t>(np, 1));
    pl.ovf = pl.L.take(sizeof(int32_t) * (size_t)std::max<int64_t>(np, 1));
    pl.edge = pl.L.take(edge_bytes(std::max<int64_t>(np, 1), S.maxlen, S.maxlen));
}

eap_status eap_subseq_windows(const double* s, int64_t n, int64_t m, double* out, void* stream) {
    if (!s || !out) return fail(EAP_EINVAL, "NULL series or output");
    if (m < 1 || m > kMaxLen) return fail(EAP_EINVAL, "window length %lld outside 1..%lld", (long long)m,
                                          (long long)kMaxLen);
    if (n < m) return fail(EAP_EINVAL, "series of %lld values is shorter than the window", (long long)n);
    const int64_t nw = n - m + 1;
    if (nw > (int64_t)INT32_MAX / m)
        return fail(EAP_EINVAL, "%lld windows of %lld values exceed 2^31 - 1 values: search the series in parts",
                    (long long)nw, (long long)m);
    const char* sb = reinterpret_cast<const char*>(s);
    const char* ob = reinterpret_cast<const char*>(out);
    if (sb < ob + sizeof(double) * (size_t)(nw * m) && ob < sb + sizeof(double) * (size_t)n)
        return fail(EAP_EINVAL, "out overlaps the series");
    HIPCHK(launch_subseq_windows(s, nw, (int)m, out, (hipStream_t)stream));
    return EAP_OK;
}

size_t eap_derivative_workspace(int64_t n) {
    if (n < 1) return 0;
    return (sizeof(int64_t) * (size_t)(n + 1) + kAlign - 1) / kAlign * kAlign;
}

eap_status eap_derivative(const double* v, const int64_t* off, int64_t n, double* out, void* ws, size_t ws_bytes,
                          void* stream) {
    eap_status st;
    if (!v || !out) return fail(EAP_EINVAL, "NULL series or output");
    SetInfo S;
    if ((st = check_offsets(off, n, "series", &S)) != EAP_OK) return st;
    const size_t need = eap_derivative_workspace(n);
    if (eap_status st_ws = check_ws(ws, ws_bytes, need)) return st_ws;
    const char* vb = reinterpret_cast<const char*>(v);
    const char* ob = reinterpret_cast<const char*>(out);
    const size_t bytes = sizeof(double) * (size_t)S.total;
    if (vb < ob + bytes && ob < vb + bytes) return fail(EAP_EINVAL, "out overlaps the input values");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload(ws, off, sizeof(int64_t) * (size_t)(n + 1), s)) != EAP_OK) return st;
    HIPCHK(launch_derivative(v, reinterpret_cast<const int64_t*>(ws), n, out, s));
    return EAP_OK;
}

size_t eap_envelopes_workspace(int64_t n) { return eap_derivative_workspace(n); }

eap_status eap_envelopes(const double* v, const int64_t* off, int64_t n, int64_t npos, int64_t other_max,
                         double window_ratio, double* up, double* lo, void* ws, size_t ws_bytes, void* stream) {
    eap_status st;
    if (!v || !up || !lo) return fail(EAP_EINVAL, "NULL series or output");
    SetInfo S;
    if ((st = check_offsets(off, n, "series", &S)) != EAP_OK) return st;
    if (npos < 1 || npos > kMaxLen) return fail(EAP_EINVAL, "npos %lld outside 1..%lld", (long long)npos,
                                                (long long)kMaxLen);
    if (other_max < 0 || other_max > kMaxLen) return fail(EAP_EINVAL, "other_max outside 0..%lld", (long long)kMaxLen);
    if (std::isnan(window_ratio) || window_ratio < 0) return fail(EAP_EINVAL, "window_ratio must be >= 0");
    if (eap_status st_ws = check_ws(ws, ws_bytes, eap_envelopes_workspace(n))) return st_ws;
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload(ws, off, sizeof(int64_t) * (size_t)(n + 1), s)) != EAP_OK) return st;
    HIPCHK(launch_envelope(v, reinterpret_cast<const int64_t*>(ws), n, (int)S.maxlen, (int)other_max, (int)npos,
                           window_ratio, up, lo, nullptr, npos, 1, s));
    return EAP_OK;
}

size_t eap_znorm_workspace(int64_t n) { return eap_derivative_workspace(n); }

eap_status eap_znorm(const double* v, const int64_t* off, int64_t n, double* out, void* ws, size_t ws_bytes,
                     void* stream) {
    eap_status st;
    if (!v || !out) return fail(EAP_EINVAL, "NULL series or output");
    SetInfo S;
    if ((st = check_offsets(off, n, "series", &S)) != EAP_OK) return st;
    if (eap_status st_ws = check_ws(ws, ws_bytes, eap_znorm_workspace(n))) return st_ws;
    const char* vb = reinterpret_cast<const char*>(v);
    const char* ob = reinterpret_cast<const char*>(out);
    const size_t bytes = sizeof(double) * (size_t)S.total;
    if (vb < ob + bytes && ob < vb + bytes) return fail(EAP_EINVAL, "out overlaps the input values");
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload(ws, off, sizeof(int64_t) * (size_t)(n + 1), s)) != EAP_OK) return st;
    HIPCHK(launch_znorm(v, reinterpret_cast<const int64_t*>(ws), n, out, s));
    return EAP_OK;
}

size_t eap_pairwise_workspace(const int64_t* s_off, int64_t n, const eap_params* p) {
    SetInfo S;
    if (check_params(p) != EAP_OK || check_offsets(s_off, n, "series", &S) != EAP_OK) return 0;
    PWLayout pl;
    pw_layout(S, p, pl);
    return pl.L.off;
}

eap_status eap_pairwise(const double* s, const int64_t* s_off, int64_t n, const eap_params* p, int32_t mode, void* ws,
                        size_t ws_bytes, double* out, void* stream) {
    eap_status st;
    if ((st = check_params(p)) != EAP_OK) return st;
    if (!s || !out) return fail(EAP_EINVAL, "NULL series or output");
    if (mode != 0 && mode != 1) return fail(EAP_EINVAL, "mode must be 0 (prune-only) or 1 (plain DP)");
    SetInfo S;
    if ((st = check_offsets(s_off, n, "series", &S)) != EAP_OK) return st;
    if (n < 2) return fail(EAP_EINVAL, "pairwise needs at least two series");
    const int64_t np = n * (n - 1) / 2;
    if (np > (int64_t)INT32_MAX) return fail(EAP_EINVAL, "too many pairs");
    PWLayout pw;
    pw_layout(S, p, pw);
    if (eap_status st_ws = check_ws(ws, ws_bytes, pw.L.off)) return st_ws;
    Plan pl;
    if ((st = make_plan(p, S.maxlen, S.maxlen, S.maxlen - S.minlen, false, &pl)) != EAP_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    SweepArgs a = base_args(p);
    SeriesPtrs SA, SB;
    if ((st = setup_common(ws, pw.c, p, s, s_off, n, nullptr, nullptr, n, hs, a, SA, SB)) != EAP_OK) return st;
    Header* h = hdr_of(ws, pw.c);
    a.mode = PM_CONDENSED;
    a.nA = a.nB = n;
    a.res = out;
    a.band_half = pl.band_half;
    a.ovf_items = reinterpret_cast<int32_t*>(at(ws, pw.ovf));
    a.ovf_count = &h->ovf_count[0];
    a.edge = edge_bytes(np, S.maxlen, S.maxlen) ? at(ws, pw.edge) : nullptr;
    a.edge_stride = S.maxlen + 1;
    if (mode == 0) {
        double* cut = reinterpret_cast<double*>(at(ws, pw.cut));
        if (dims_of(p) > 1) HIPCHK(launch_ub_mv(effective_kind(p), dims_of(p), true, a, s, SA.off, nullptr, nullptr, n,
                                               cut, hs));
        else HIPCHK(launch_ub_condensed(effective_kind(p), a, s, SA.off, n, cut, hs));
        a.pcut = cut;
    }
    if (mode == 1) a.plain = 1;
    return sweep(p, pl, pl.band, a, h, 2, &h->queues[0], nullptr, np, SA, SB, hs);
}

eap_status eap_tune_nn1(const double* q, const int64_t* q_off, int64_t nq, const double* r, const int64_t* r_off,
                        int64_t nr, const eap_params* p, const eap_nn_opts* o, void* ws, size_t ws_bytes,
                        int64_t* out_idx, double* out_dist, void* stream, eap_tune_rec* recs, int32_t cap,
                        int32_t* n) {
    eap_status st;
    if (!n || (cap > 0 && !recs)) return fail(EAP_EINVAL, "bad tuning output");
    *n = 0;
    if ((st = check_params(p)) != EAP_OK) return st;
    if (!q || !r || !out_idx || !out_dist) return fail(EAP_EINVAL, "NULL series or output");
    SetInfo Q, R;
    if ((st = check_offsets(q_off, nq, "queries", &Q)) != EAP_OK) return st;
    if ((st = check_offsets(r_off, nr, "candidates", &R)) != EAP_OK) return st;
    // the timed runs use no pipelining events
    eap_nn_opts own{};
    if (o) {
        own = *o;
        own.main_wait = own.main_done = nullptr;
        o = &own;
    }
    if (dims_of(p) > 1) return EAP_OK;   // multivariate searches have one shape per length: nothing to tune
    const bool fp32 = o && o->precision == 1 && screen_possible(p, std::max(Q.maxlen, R.maxlen));
    const bool xd = fp32 && screen_exact_diff(p, std::max(Q.maxlen, R.maxlen));
    const bool plain = o && (o->flags & 2);
    const int64_t ldiff = std::max(std::llabs(Q.maxlen - R.minlen), std::llabs(R.maxlen - Q.minlen));
    Plan pl;
    if ((st = make_plan(p, Q.maxlen, R.maxlen, ldiff, !plain && !xd, &pl)) != EAP_OK) return st;
    const bool band = pl.band;
    hipStream_t s = (hipStream_t)stream;
    const RowsShape all[13] = {{4, 8},  {4, 16},  {8, 8},   {8, 16},  {16, 8},  {16, 16}, {32, 8},
                               {32, 16}, {64, 8}, {64, 16}, {16, 32}, {32, 32}, {64, 32}};
    std::vector<RowsShape> shapes;   // band sweep: {lanes, columns per lane}
    if (band) {
        for (int g : {2, 4, 8, 16, 32, 64})
            if (band_shape_ok(pl.size, g)) shapes.push_back(RowsShape{g, pl.size / (2 * g)});
    } else {
        for (const RowsShape& x : all)
            if (rows_shape_ok(effective_kind(p), x, fp32)) shapes.push_back(x);
    }
    std::vector<int64_t> idx0((size_t)nq), idx((size_t)nq);
    std::vector<double> d0((size_t)nq), d((size_t)nq);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best_ms = 0.0f;
    int best = -1, k = 0;
    st = EAP_OK;
    for (int v = 0; v < (int)shapes.size() && st == EAP_OK; ++v) {
        if (band) g_force_band[fp32] = shapes[v].g;
        else g_force[fp32] = shapes[v];
        st = eap_nn1(q, q_off, nq, r, r_off, nr, nullptr, p, o, ws, ws_bytes, out_idx, out_dist, nullptr, stream);
        if (st != EAP_OK) break;
        if (hipMemcpyAsync(idx.data(), out_idx, sizeof(int64_t) * (size_t)nq, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(d.data(), out_dist, sizeof(double) * (size_t)nq, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = fail(EAP_EDEVICE, "tuning: copying results back failed");
            break;
        }
        if (v == 0) {
            idx0 = idx;
            d0 = d;
        } else if (idx != idx0 || std::memcmp(d.data(), d0.data(), sizeof(double) * (size_t)nq) != 0) {
            st = fail(EAP_EDEVICE, "tuning: row-sweep shape %dx%d disagrees with %dx%d", shapes[v].g, shapes[v].c,
                      shapes[0].g, shapes[0].c);
            break;
        }
        // the fastest of three timed searches (the least disturbed one)
        float ms = 0.0f;
        for (int rep = 0; rep < 3 && st == EAP_OK; ++rep) {
            float one = 0.0f;
            if (hipEventRecord(e0, s) != hipSuccess) {
                st = fail(EAP_EDEVICE, "tuning: event record failed");
                break;
            }
            st = eap_nn1(q, q_off, nq, r, r_off, nr, nullptr, p, o, ws, ws_bytes, out_idx, out_dist, nullptr, stream);
            if (st != EAP_OK) break;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&one, e0, e1) != hipSuccess) {
                st = fail(EAP_EDEVICE, "tuning: event timing failed");
                break;
            }
            ms = (rep == 0 || one < ms) ? one : ms;
        }
        if (st != EAP_OK) break;
        if (best < 0 || ms < best_ms) {
            best = v;
            best_ms = ms;
        }
        if (k < cap) recs[k] = eap_tune_rec{shapes[v].g, shapes[v].c, ms, 0};
        ++k;
    }
    g_force[fp32] = RowsShape{0, 0};
    g_force_band[fp32] = 0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != EAP_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (band)
            g_tuned_band[(effective_kind(p) * 2 + (fp32 ? 1 : 0)) * 16 + log2i(pl.size)] = shapes[best].g;
        else
            g_tuned[(effective_kind(p) * 2 + (fp32 ? 1 : 0)) * 8 + len_bucket(std::min(Q.maxlen, R.maxlen))] =
                shapes[best];
    }
    if (best < cap) recs[best].chosen = 1;
    *n = k < cap ? k : cap;
    return EAP_OK;
}

struct eap_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

eap_status eap_capture_begin(void* stream) {
    HIPCHK(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return EAP_OK;
}

eap_status eap_capture_end(void* stream, eap_graph** out) {
    if (!out) return fail(EAP_EINVAL, "NULL graph output");
    *out = nullptr;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamEndCapture((hipStream_t)stream, &g));
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(EAP_EDEVICE, "hipGraphInstantiate failed");
    }
    eap_graph* r = new (std::nothrow) eap_graph;
    if (!r) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return fail(EAP_ENOMEM, "graph handle");
    }
    r->graph = g;
    r->exec = x;
    *out = r;
    return EAP_OK;
}

eap_status eap_graph_launch(eap_graph* g, void* stream) {
    if (!g || !g->exec) return fail(EAP_EINVAL, "NULL graph");
    HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return EAP_OK;
}

eap_status eap_graph_destroy(eap_graph* g) {
    if (!g) return EAP_OK;
    if (g->exec) HIPCHK(hipGraphExecDestroy(g->exec));
    if (g->graph) HIPCHK(hipGraphDestroy(g->graph));
    delete g;
    return EAP_OK;
}

eap_status eap_tune_set(int32_t kind, int32_t precision, int64_t lco_max, int32_t g, int32_t c) {
    if (kind < EAP_DTW || kind > EAP_TWE || (precision != 0 && precision != 1) || lco_max < 1 ||
        lco_max > kMaxLen)
        return fail(EAP_EINVAL, "bad tuning key");
    const RowsShape sh{g, c};
    if (!rows_shape_ok(kind, sh, precision == 1)) return fail(EAP_EINVAL, "no row-sweep shape %dx%d", g, c);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[(kind * 2 + precision) * 8 + len_bucket(lco_max)] = sh;
    return EAP_OK;
}

eap_status eap_tune_reset(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    g_tuned_band.clear();
    return EAP_OK;
}

double eap_screen_eps(int32_t kind, int32_t exact_diff, double B, double N, double A) {
    if (kind < EAP_DTW || kind > EAP_TWE) return NAN;
    return screen_eps(kind | (exact_diff ? kScreenExactDiff : 0), B, N, A);
}

double eap_screen_bound(int32_t kind, int32_t exact_diff, double b, double N, double A) {
    if (kind < EAP_DTW || kind > EAP_TWE) return NAN;
    return screen_bound(kind | (exact_diff ? kScreenExactDiff : 0), b, N, A);
}

eap_status eap_wdtw_weights(double g, int64_t L, double* out) {
    if (!out || L < 1 || !(std::isfinite(g) && g >= 0)) return fail(EAP_EINVAL, "bad WDTW weight arguments");
    std::vector<double> t;
    int off = 0;
    wdtw_table(g, L, t, off);
    for (int64_t k = 0; k < L; ++k) out[k] = t[(size_t)(2 * k - L + off)];
    return EAP_OK;
}

// ---------------------------------------------------------------- counters
eap_status eap_read_counters(const void* ws, size_t ws_bytes, eap_counters* out, void* stream) {
    if (!ws || ws_bytes < kHeaderBytes || !out) return fail(EAP_EINVAL, "bad workspace or output");
    Header h;
    HIPCHK(hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    out->cells = h.counters[0];
    out->pairs = h.counters[1];
    out->rechecks = h.counters[2];
    out->overflows = h.counters[3];
    out->lb_pruned = h.counters[4];
    for (int s = 0; s < 8; ++s) {
        out->stage_cells[s] = h.counters[8 + s];
        out->stage_pairs[s] = h.counters[16 + s];
    }
    return EAP_OK;
}

eap_status eap_reset_counters(void* ws, size_t ws_bytes, void* stream) {
    if (!ws || ws_bytes < kHeaderBytes) return fail(EAP_EINVAL, "bad workspace");
    HIPCHK(launch_fill_u64(reinterpret_cast<unsigned long long*>(ws), 0ull, kCounterWords, (hipStream_t)stream));
    return EAP_OK;
}

eap_status eap_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
    return EAP_OK;
}

eap_status eap_profile_take(eap_profile_rec* out, int32_t cap, int32_t* n) {
    if (!n || (cap > 0 && !out)) return fail(EAP_EINVAL, "bad profile output");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    int32_t k = 0;
    for (auto& pr : g_prof.pending) {
        HIPCHK(hipEventSynchronize(pr.e1));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, pr.e0, pr.e1));
        if (k < cap) {
            out[k] = pr.r;
            out[k].ms = ms;
        }
        ++k;
        g_prof.pool.push_back(pr.e0);
        g_prof.pool.push_back(pr.e1);
    }
    g_prof.pending.clear();
    *n = k < cap ? k : cap;
    return EAP_OK;
}

}  // extern "C"

namespace eap {

size_t nn1_workspace_sizes(const SetSizes& Q, const SetSizes& R, const eap_params* p, const eap_nn_opts* o) {
    if (check_params(p) != EAP_OK || Q.n < 1 || R.n < 1) return 0;
    SetInfo q, r;
    q.n = Q.n; q.total = Q.total; q.maxlen = Q.maxlen; q.minlen = Q.minlen;
    r.n = R.n; r.total = R.total; r.maxlen = R.maxlen; r.minlen = R.minlen;
    NNLayout nl;
    const bool prec1 = o && o->precision == 1 && dims_of(p) == 1;
    nn_layout(q, r, p, prec1, prec1 && screen_possible(p, std::max(q.maxlen, r.maxlen)), lb_mode(p, o), nl);
    return nl.L.off;
}

}  // namespace eap
