// Request server of libeap: 1-NN queries that arrive one by one against a
// reference set resident on the device (see the eap_server_* functions in
// include/eap.h).
//
// Design.  The server owns S slots; each has a stream, a completion event, a
// fixed share of one device memory pool and pinned host buffers.  Submitted
// queries wait in a FIFO.  poll() first collects every slot whose batch has
// completed (its results were copied back on its stream, behind the search),
// then fills every free slot with the longest prefix of the FIFO that fits
// the slot: at most max_batch queries whose values, NN workspace and outputs
// fit the slot's bytes (admission by memory).  Each batch is one eap_nn1 call
// on the slot's stream, so batches admitted while others are running overlap
// on the device.  A slot's NN workspace sits at the start of its bytes; what
// a search derives from the candidates alone sits at the workspace's start,
// so from the slot's second batch on it is reused (flags bit 3).  A query is
// answered by the same search whether it runs alone or in a batch: its result
// does not depend on the other queries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "eap.h"
#include "eap_internal.h"

namespace {

thread_local std::string s_err;

eap_status sfail(eap_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s_err = buf;
    return st;
}

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Query {
    int64_t tag;
    std::vector<double> v;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* dev = nullptr;
    size_t bytes = 0;
    double* hq = nullptr;        // pinned: query values of the batch
    int64_t* hidx = nullptr;     // pinned: results
    double* hdist = nullptr;
    int32_t* hlab = nullptr;
    bool busy = false;
    bool cand_ready = false;   // the slot's workspace holds the candidates' derived data
    std::vector<int64_t> tags;
};

}  // namespace

struct eap_server {
    eap_params p{};
    eap_server_opts o{};
    eap_nn_opts nn{};
    const double* refs = nullptr;
    std::vector<int64_t> r_off;
    int64_t nr = 0;
    eap::SetSizes rs;   // the candidates' sizes, checked once at creation
    const int32_t* labels = nullptr;
    char* pool = nullptr;
    std::vector<Slot> slots;
    std::deque<Query> fifo;
    eap_server_stats st{};
};

namespace {

void free_server(eap_server* s) {
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.hq) (void)hipHostFree(sl.hq);
        if (sl.hidx) (void)hipHostFree(sl.hidx);
        if (sl.hdist) (void)hipHostFree(sl.hdist);
        if (sl.hlab) (void)hipHostFree(sl.hlab);
    }
    if (s->pool) (void)hipFree(s->pool);
    delete s;
}

// Bytes a batch of queries of these sizes needs in a slot: NN workspace (at
// the slot's start, so that what it derived from the candidates stays in
// place from batch to batch), values, outputs.  From sizes alone: admission
// reads neither the candidates' offsets nor the queries' again.
size_t batch_bytes(const eap_server* s, const eap::SetSizes& q) {
    const size_t ws = eap::nn1_workspace_sizes(q, s->rs, &s->p, &s->nn);
    if (ws == 0) return SIZE_MAX;
    return up(ws) + up(sizeof(double) * (size_t)q.total) + up(sizeof(int64_t) * (size_t)q.n) +
           up(sizeof(double) * (size_t)q.n) + up(sizeof(int32_t) * (size_t)q.n);
}

// Fill `sl` with the longest FIFO prefix that fits and start its search.
eap_status launch_batch(eap_server* s, Slot& sl) {
    std::vector<int64_t> qoff{0};
    eap::SetSizes q;
    size_t k = 0;
    while (k < s->fifo.size() && (int64_t)k < s->o.max_batch) {
        const int64_t L = (int64_t)s->fifo[k].v.size();
        eap::SetSizes q2 = q;
        q2.n += 1;
        q2.total += L;
        q2.maxlen = std::max(q.maxlen, L);
        q2.minlen = q.n ? std::min(q.minlen, L) : L;
        if (batch_bytes(s, q2) > sl.bytes) break;
        q = q2;
        qoff.push_back(qoff.back() + L);
        ++k;
    }
    if (k == 0) return sfail(EAP_ENOMEM, "query %lld does not fit a slot of %zu bytes",
                             (long long)s->fifo.front().tag, sl.bytes);
    const int64_t nq = (int64_t)k;
    sl.tags.clear();
    for (size_t i = 0; i < k; ++i) {
        std::memcpy(sl.hq + qoff[i], s->fifo[i].v.data(), sizeof(double) * s->fifo[i].v.size());
        sl.tags.push_back(s->fifo[i].tag);
    }
    const size_t ws_bytes = eap::nn1_workspace_sizes(q, s->rs, &s->p, &s->nn);
    char* at = sl.dev;
    void* ws = at;
    at += up(ws_bytes);
    double* dq = reinterpret_cast<double*>(at);
    at += up(sizeof(double) * (size_t)qoff.back());
    int64_t* didx = reinterpret_cast<int64_t*>(at);
    at += up(sizeof(int64_t) * (size_t)nq);
    double* ddist = reinterpret_cast<double*>(at);
    at += up(sizeof(double) * (size_t)nq);
    int32_t* dlab = reinterpret_cast<int32_t*>(at);
    if (hipMemcpyAsync(dq, sl.hq, sizeof(double) * (size_t)qoff.back(), hipMemcpyHostToDevice, sl.stream) !=
        hipSuccess)
        return sfail(EAP_EDEVICE, "query upload failed");
    // after the slot's first batch, the candidates' derived data is reused
    eap_nn_opts nn = s->nn;
    if (sl.cand_ready) nn.flags |= 8;
    eap_status e = eap_nn1(dq, qoff.data(), nq, s->refs, s->r_off.data(), s->nr, s->labels, &s->p, &nn, ws,
                           ws_bytes, didx, ddist, s->labels ? dlab : nullptr, sl.stream);
    if (e != EAP_OK) {
        sl.cand_ready = false;
        return sfail(e, "batch search: %s", eap_last_error());
    }
    sl.cand_ready = true;
    if (hipMemcpyAsync(sl.hidx, didx, sizeof(int64_t) * (size_t)nq, hipMemcpyDeviceToHost, sl.stream) !=
            hipSuccess ||
        hipMemcpyAsync(sl.hdist, ddist, sizeof(double) * (size_t)nq, hipMemcpyDeviceToHost, sl.stream) !=
            hipSuccess ||
        (s->labels &&
         hipMemcpyAsync(sl.hlab, dlab, sizeof(int32_t) * (size_t)nq, hipMemcpyDeviceToHost, sl.stream) !=
             hipSuccess) ||
        hipEventRecord(sl.done, sl.stream) != hipSuccess)
        return sfail(EAP_EDEVICE, "result download failed");
    s->fifo.erase(s->fifo.begin(), s->fifo.begin() + (std::ptrdiff_t)k);
    sl.busy = true;
    s->st.batches += 1;
    s->st.queries += nq;
    s->st.max_batch_seen = std::max<int64_t>(s->st.max_batch_seen, nq);
    return EAP_OK;
}

}  // namespace

extern "C" {

const char* eap_server_last_error(void) { return s_err.c_str(); }

eap_status eap_server_create(const double* refs, const int64_t* r_off, int64_t nr, const int32_t* r_labels,
                             const eap_params* p, const eap_server_opts* o, eap_server** out) {
    if (!out) return sfail(EAP_EINVAL, "NULL server output");
    *out = nullptr;
    if (!refs || !r_off || nr < 1 || !p || !o) return sfail(EAP_EINVAL, "NULL or empty argument");
    if (o->slots < 1 || o->slots > 16 || o->max_batch < 1 || o->max_query_len < 1 || o->mem_budget == 0)
        return sfail(EAP_EINVAL, "slots must be 1..16, max_batch, max_query_len and mem_budget positive");
    if (p->dims > 1) return sfail(EAP_EINVAL, "the server takes univariate series only");
    eap_server* s = new (std::nothrow) eap_server;
    if (!s) return sfail(EAP_ENOMEM, "server object");
    s->p = *p;
    s->o = *o;
    s->nn.precision = o->precision;
    s->nn.margin_rel = o->margin_rel;
    s->nn.flags = 0;
    s->refs = refs;
    s->r_off.assign(r_off, r_off + nr + 1);
    s->nr = nr;
    // the candidates' offsets, checked once (the library's limits: lengths 1..2048)
    if (r_off[0] != 0) {
        delete s;
        return sfail(EAP_EINVAL, "candidate offsets must start at 0");
    }
    s->rs.n = nr;
    s->rs.minlen = INT64_MAX;
    for (int64_t k = 0; k < nr; ++k) {
        const int64_t L = r_off[k + 1] - r_off[k];
        if (L < 1 || L > 2048) {
            delete s;
            return sfail(EAP_EINVAL, "candidate %lld has length %lld (1..2048)", (long long)k, (long long)L);
        }
        s->rs.maxlen = std::max(s->rs.maxlen, L);
        s->rs.minlen = std::min(s->rs.minlen, L);
    }
    s->rs.total = r_off[nr];
    s->labels = r_labels;
    // the one allocation of the server: every slot's share of the pool
    const size_t per = o->mem_budget / (size_t)o->slots / kAlign * kAlign;
    if (per == 0) {
        delete s;
        return sfail(EAP_EINVAL, "mem_budget too small for %d slots", o->slots);
    }
    if (hipMalloc(&s->pool, per * (size_t)o->slots) != hipSuccess) {
        delete s;
        return sfail(EAP_ENOMEM, "device pool of %zu bytes", per * (size_t)o->slots);
    }
    s->slots.resize((size_t)o->slots);
    const size_t nb = (size_t)o->max_batch;
    for (int i = 0; i < o->slots; ++i) {
        Slot& sl = s->slots[(size_t)i];
        sl.dev = s->pool + per * (size_t)i;
        sl.bytes = per;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&sl.hq), sizeof(double) * nb * (size_t)o->max_query_len,
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&sl.hidx), sizeof(int64_t) * nb, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&sl.hdist), sizeof(double) * nb, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&sl.hlab), sizeof(int32_t) * nb, hipHostMallocDefault) !=
                hipSuccess) {
            free_server(s);
            return sfail(EAP_ENOMEM, "slot %d: stream, event or pinned buffers", i);
        }
    }
    *out = s;
    return EAP_OK;
}

eap_status eap_server_submit(eap_server* s, const double* q, int64_t len, int64_t tag) {
    if (!s || !q || len < 1) return sfail(EAP_EINVAL, "bad query");
    if (len > s->o.max_query_len) return sfail(EAP_EINVAL, "query longer than max_query_len");
    Query x;
    x.tag = tag;
    x.v.assign(q, q + len);
    s->fifo.push_back(std::move(x));
    return EAP_OK;
}

eap_status eap_server_poll(eap_server* s, eap_result* out, int32_t cap, int32_t* n) {
    if (!s || !n || (cap > 0 && !out)) return sfail(EAP_EINVAL, "bad poll arguments");
    *n = 0;
    // 1. completed batches (only while there is room for all their results)
    for (Slot& sl : s->slots) {
        if (!sl.busy) continue;
        if ((int64_t)*n + (int64_t)sl.tags.size() > (int64_t)cap) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return sfail(EAP_EDEVICE, "batch failed: %s", hipGetErrorString(q));
        for (size_t i = 0; i < sl.tags.size(); ++i)
            out[(*n)++] = eap_result{sl.tags[i], sl.hidx[i], sl.hdist[i], s->labels ? sl.hlab[i] : -1, 0};
        sl.busy = false;
    }
    // 2. admit waiting queries into free slots
    for (Slot& sl : s->slots) {
        if (s->fifo.empty()) break;
        if (sl.busy) continue;
        eap_status e = launch_batch(s, sl);
        if (e != EAP_OK) return e;
    }
    int64_t inflight = 0;
    for (const Slot& sl : s->slots) inflight += sl.busy ? 1 : 0;
    s->st.max_inflight = std::max(s->st.max_inflight, inflight);
    return EAP_OK;
}

eap_status eap_server_stats_get(const eap_server* s, eap_server_stats* out) {
    if (!s || !out) return sfail(EAP_EINVAL, "bad stats arguments");
    *out = s->st;
    out->waiting = (int64_t)s->fifo.size();
    return EAP_OK;
}

eap_status eap_server_counters(const eap_server* s, eap_counters* out) {
    if (!s || !out) return sfail(EAP_EINVAL, "bad counters arguments");
    std::memset(out, 0, sizeof *out);
    for (const Slot& sl : s->slots) {
        eap_counters c;
        if (eap_read_counters(sl.dev, sl.bytes, &c, sl.stream) != EAP_OK)
            return sfail(EAP_EDEVICE, "slot counters: %s", eap_last_error());
        out->cells += c.cells;
        out->pairs += c.pairs;
        out->rechecks += c.rechecks;
        out->overflows += c.overflows;
        for (int i = 0; i < 8; ++i) {
            out->stage_cells[i] += c.stage_cells[i];
            out->stage_pairs[i] += c.stage_pairs[i];
        }
        out->lb_pruned += c.lb_pruned;
    }
    return EAP_OK;
}

eap_status eap_server_destroy(eap_server* s) {
    if (s) free_server(s);
    return EAP_OK;
}

}  // extern "C"
