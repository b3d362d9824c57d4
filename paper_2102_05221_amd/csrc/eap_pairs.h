// Work-item decoding shared by the sweep kernels.
#pragma once
#include "eap_device.h"
#include "eap_launch.h"

namespace eap {

struct Item {
    int32_t a, b;     // series index in set A and set B
    int64_t out;      // result slot
    int64_t cutidx;   // index into pcut (non-NN modes)
    bool skip;
};

// Condensed index k -> (i, j), i < j < n, with k = n*i - i*(i+1)/2 + (j-i-1).
__device__ __forceinline__ void condensed_ij(int64_t k, int64_t n, int64_t& i, int64_t& j) {
    double nn = (double)(2 * n - 1);
    int64_t ii = (int64_t)((nn - sqrt(nn * nn - 8.0 * (double)k)) * 0.5);
    if (ii < 0) ii = 0;
    if (ii > n - 2) ii = n - 2;
    while (ii > 0 && n * ii - ii * (ii + 1) / 2 > k) --ii;
    while (ii < n - 2 && n * (ii + 1) - (ii + 1) * (ii + 2) / 2 <= k) ++ii;
    i = ii;
    j = k - (n * ii - ii * (ii + 1) / 2) + ii + 1;
}

__device__ __forceinline__ Item decode_item(const SweepArgs& A, int64_t p) {
    Item it;
    it.skip = false;
    it.cutidx = p;
    switch (A.mode) {
    case PM_NN_ALL: {
        int64_t a = p / A.nB, b = p - a * A.nB;
        it.a = (int32_t)a;
        it.b = (int32_t)b;
        it.out = p;
        it.skip = (A.skip_b != nullptr) && (A.skip_b[a] == (int32_t)b);
        break;
    }
    case PM_CONDENSED: {
        int64_t i, j;
        condensed_ij(p, A.nA, i, j);
        it.a = (int32_t)i;
        it.b = (int32_t)j;
        it.out = p;
        break;
    }
    default: {
        it.a = 0;
        it.b = 0;
        it.out = 0;
        break;
    }
    }
    return it;
}

__device__ __forceinline__ bool is_nn_mode(int mode) { return mode == PM_NN_ALL; }

// The item index behind work slot p of a launch.  An NN search over all
// pairs takes them candidate by candidate (slot p -> query p % nA, candidate
// p / nA): each query then has only a few pairs in flight at a time, and its
// best-so-far tightens as its candidates complete, as in Alg. 1's loop; in
// query order the pairs of one query would all start under the seed's
// cut-off.  The item (a * nB + b) and its result slot are unchanged.
__device__ __forceinline__ int64_t item_of(const SweepArgs& A, unsigned int p) {
    if (A.items) return (int64_t)A.items[p];
    if (A.mode == PM_NN_ALL && A.nA > 1) {
        const unsigned int na = (unsigned int)A.nA;
        const unsigned int b = p / na, a = p - b * na;
        return (int64_t)a * A.nB + (int64_t)b;
    }
    return (int64_t)p;
}

// The cut-off of query a in NN mode: the best-so-far, widened for an FP32
// screen (so that no candidate within the certified FP32 error of the best is
// abandoned) and rounded up to T.
template <typename T> __device__ __forceinline__ T nn_cut(const SweepArgs& A, int64_t a) {
    double c = bitsd(A.best[a]);
    if (A.widen_abs) c = c * (1.0 + A.widen_rel) + A.widen_abs[a];
    T t = (T)c;
    if ((double)t < c) t = round_up_next(t);
    return t;
}

// Work slots are handed to a group A.chunk at a time (consecutive slots);
// `next`/`end` are the group's current chunk.  The groups of a wave that need
// a chunk at the same time take theirs with one atomic (its first such group
// adds all of them, each group takes its chunk by rank), so that lists of
// many short items, taken one slot at a time, do not serialise on the counter.
__device__ __forceinline__ unsigned int fetch_slot(const SweepArgs& A, unsigned int& next, unsigned int& end,
                                                   int lane, int k) {
    const bool need = next >= end;
    const unsigned long long m = __ballot(need && k == 0);
    if (need) {
        const unsigned int ch = A.chunk > 0 ? (unsigned int)A.chunk : 1u;
        const int lead = __ffsll((long long)m) - 1;
        unsigned int base = 0;
        if (lane == lead) base = atomicAdd(A.queue, ch * (unsigned int)__popcll(m));
        base = __shfl(base, lead);
        const int g0 = lane - k;   // this group's first lane
        const unsigned int rank = (unsigned int)__popcll(m & ((1ull << g0) - 1ull));
        next = base + rank * ch;
        end = next + ch;
    }
    return next++;
}

// Sum of a per-lane counter over the wave, added once per wave.
__device__ __forceinline__ void wave_add_u64(unsigned long long* dst, unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

}  // namespace eap
