// Kernel B: anti-diagonal sweep of a band of diagonals, one pair per group of
// G lanes, with the cut-off and early abandoning of EAPruned (Alg. 5).
//
// Coordinates.  Cell (i, j) of the cost matrix lies on diagonal d = j - i and
// anti-diagonal a = i + j.  Rows are the longer series (Alg. 3/5).  The band
// is the 2*G*C diagonals dlo .. dlo + 2GC - 1; lane k owns diagonals
// dk .. dk + 2C - 1 with dk = dlo + 2kC and keeps the latest cell of each in a
// register.  Step a computes the cells of anti-diagonal a, one parity of
// diagonals at a time (C cells per lane): the diagonal dependency is the same
// register two steps earlier, the top and left ones are the neighbouring
// diagonals one step earlier - in the same lane except at strip ends, where
// one DPP wave shift brings the value from lane k+1 (odd steps) or k-1 (even
// steps).  Along a lane's diagonals the cells of one step sit on consecutive
// rows and columns, so the row and column values live in two C-entry
// register rings that advance by one row (one column) every two steps; the
// entering value comes from the neighbouring lane, or from memory at the
// group's ends.  A block of 2C steps returns the rings to their phase, so the
// block is unrolled and every register index is static.
//
// Window (CDTW, ERP).  Cells with |i - j| > w are outside the Sakoe-Chiba
// band (Section 2.3.2): their diagonals get an additive +inf penalty.  ERP's
// computed borders are kept on 1..w+1 (Alg. 4/5 initialise them there), so
// for ERP the penalty starts at anti-diagonal w+2, after the two border cells
// (0, w+1) and (w+1, 0) have been formed.
//
// Unconstrained distances (WDTW, DTW) sweep a band around the diagonal path.
// A warping path leaves the band only through one of its two edge diagonals
// and path costs never decrease, so when every cell computed on an edge
// diagonal is > cut-off, the band holds every cell <= cut-off and the result
// is exact.  Otherwise the item is appended to an overflow list and redone
// by the host with a wider band.
//
// Series values outside 1..L are 0 before the start and +inf after the end:
// cells before (0,0) stay +inf because their dependencies are, cells past the
// end become +inf through their cost, and s_0 = t_0 = 0 needs no special case.
//
// Abandoning: a warping path visits at least one of any two consecutive
// anti-diagonals, so when the cells of two consecutive steps are all > cut-off
// (and the band is certified) no path stays under it (Alg. 5's criterion for
// a dead row, applied to anti-diagonals).
#include "eap_pairs.h"

namespace eap {

__device__ __forceinline__ int shl1_i32(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float shl1(float v) {
    return __builtin_bit_cast(float, shl1_i32(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double shl1(double v) {
    long long b = __builtin_bit_cast(long long, v);
    int lo = shl1_i32((int)(unsigned long long)b);
    int hi = shl1_i32((int)((unsigned long long)b >> 32));
    unsigned long long r = (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32);
    return __builtin_bit_cast(double, r);
}

// Blocks per CU the register budget is sized for: the band sweep waits on a
// chain of dependent steps, so FP32 bands of up to 8 diagonals per parity and
// lane are held to 168 VGPRs (3 blocks of 256, 3 waves per SIMD).  Wider FP32
// lanes and FP64 take the registers they need (a tighter budget spills).
template <typename T, int C>
constexpr int band_min_blocks() { return (sizeof(T) == 4 && C <= 8) ? 3 : 1; }

template <int KIND, typename T, int G, int C>
__global__ __launch_bounds__(256, (band_min_blocks<T, C>())) void band_kernel(SweepArgs A, Series<T> SA,
                                                                             Series<T> SB) {
    constexpr bool WIN = (KIND == CDTW || KIND == ERP);
    constexpr int CB = C;        // ring length
    constexpr int M2 = 2 * C;    // diagonals per lane
    constexpr int NB = 2 * CB;   // steps per block
    if (A.prio) __builtin_amdgcn_s_setprio(2);
    // Edge values entering the rings: with small C the next block's are fetched
    // one block ahead; with large C a block is long enough to hide the fetch.
    constexpr bool AHEAD = (C <= 8);
    const T INF = inf_v<T>();
    const int lane = threadIdx.x & 63;
    const int k = lane & (G - 1);
    const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (lane - k));
    // NN search with a shared best-so-far (not the plain DP, not prune-only)
    const bool nn = is_nn_mode(A.mode) && !A.plain && !A.prune_only;
    const T gap = (T)A.gap;

    bool have = false, done = false, fin = false, ovf = false, lo_open = false, hi_open = false;
    unsigned int fnext = 0, fend = 0;   // this group's chunk of work slots
    int32_t qa = 0;
    int64_t out = 0, item = 0;
    const T* li = nullptr;
    const T* co = nullptr;
    int Lli = 0, Lco = 0, a = 0, a_end = 0, apen = 0, dk = 0, w = 0, ke = 0, me = 0, i0 = 0, j0 = 0;
    // cells counted as executed per step of either parity: the lane's
    // diagonals inside the window (CDTW, ERP: the band padded to the group's
    // width also sweeps diagonals that are +inf throughout), all of them for
    // the unconstrained distances
    int ncnt0 = C, ncnt1 = C;
    T cut = 0, res_v = 0;
    T val[M2], S[CB], Tt[CB], Sc[CB], Sn[CB], Tc[CB], Tn[CB], wt[M2], pen[M2];
    unsigned long long ncells = 0, npairs = 0, nlb = 0;
    unsigned int nblk = 0;   // blocks swept by the wave (the cut-off refresh)
#pragma unroll
    for (int m = 0; m < M2; ++m) val[m] = wt[m] = pen[m] = 0;
#pragma unroll
    for (int q = 0; q < CB; ++q) S[q] = Tt[q] = Sc[q] = Sn[q] = Tc[q] = Tn[q] = 0;

    auto sval = [&](int r) -> T { return r < 1 ? (T)0 : (r > Lli ? INF : li[r - 1]); };
    auto tval = [&](int c) -> T { return c < 1 ? (T)0 : (c > Lco ? INF : co[c - 1]); };

    constexpr bool PF = sizeof(T) == 8;
    // The group's next work item, fetched one stage per block while the
    // current pair is swept, so that a short pair's successor does not wait
    // on the chain of loads behind it (slot, item, offsets, lower bound) with
    // the whole wave: pf 0 none, 1 slot claimed (the atomic's result in the
    // group's first lane), 2 slot known, 3 item index loaded, 4 offsets and
    // bound loaded, 5 no work left for this group.  A list's length is fixed
    // before the launch, so it is read once.  FP64 instances only: the FP32
    // ones are held to 168 registers, where the fetch state spills.
    const int64_t n_items_pf = PF ? (A.npairs_dev ? (int64_t)*A.npairs_dev : A.npairs) : 0;
    const unsigned int ch = A.chunk > 0 ? (unsigned int)A.chunk : 1u;
    const int g0 = lane - k;
    int pf = 0;
    unsigned int pf_base = 0, pf_p = 0;
    int64_t pf_item = 0, pf_o0 = 0, pf_o1 = 0, pf_o2 = 0, pf_o3 = 0;
    double pf_lb = 0.0;
    Item pf_it{};
    // the offsets and the bound of the item decoded from pf_item
    auto pf_request = [&]() {
        pf_it = decode_item(A, pf_item);
        if (!pf_it.skip) {
            pf_o0 = SA.off[pf_it.a];
            pf_o1 = SA.off[pf_it.a + 1];
            pf_o2 = SB.off[pf_it.b];
            pf_o3 = SB.off[pf_it.b + 1];
            if (KIND == CDTW && nn && A.lb) pf_lb = A.lb[pf_it.out];
        }
    };

    for (;;) {
        if (!have && !done) {
            // FP64: the prefetched item, else one fetched now.  FP32: the plain
            // fetch (its own copy of the loop, so that the FP32 instances keep
            // their register allocation)
            if constexpr (PF) {
                for (;;) {
                    Item it;
                    int64_t oa, oa1, ob, ob1;
                    double lbv = 0.0;
                    if (pf != 0) {
                        // the prefetched item: finish the stages the blocks have not done
                        if (pf == 1) {
                            const unsigned int base = __shfl(pf_base, g0);
                            fnext = base;
                            fend = base + ch;
                            pf_p = fnext++;
                            pf = 2;
                        }
                        if (pf == 2) {
                            if ((int64_t)pf_p >= n_items_pf) pf = 5;
                            else {
                                pf_item = item_of(A, pf_p);
                                pf = 3;
                            }
                        }
                        if (pf == 3) {
                            pf_request();
                            pf = 4;
                        }
                        if (pf == 5) {
                            done = true;
                            break;
                        }
                        item = pf_item;
                        it = pf_it;
                        oa = pf_o0; oa1 = pf_o1; ob = pf_o2; ob1 = pf_o3;
                        lbv = pf_lb;
                        pf = 0;
                    } else {
                        const unsigned int p = fetch_slot(A, fnext, fend, lane, k);
                        if ((int64_t)p >= n_items_pf) {
                            done = true;
                            break;
                        }
                        item = item_of(A, p);
                        it = decode_item(A, item);
                        if (it.skip) continue;
                        oa = SA.off[it.a]; oa1 = SA.off[it.a + 1];
                        ob = SB.off[it.b]; ob1 = SB.off[it.b + 1];
                        if (KIND == CDTW && nn && A.lb) lbv = A.lb[it.out];
                    }
                    if (it.skip) continue;
                    const int La = (int)(oa1 - oa), Lb = (int)(ob1 - ob);
                    if (La >= Lb) {
                        li = SA.v + oa; Lli = La; co = SB.v + ob; Lco = Lb;
                    } else {
                        li = SB.v + ob; Lli = Lb; co = SA.v + oa; Lco = La;
                    }
                    qa = it.a;
                    out = it.out;
                    if (nn) cut = nn_cut<T>(A, it.a);
                    else cut = (A.pcut && !A.plain) ? (T)A.pcut[it.cutidx] : INF;
                    const int L = Lli > Lco ? Lli : Lco;
                    const int d_end = Lco - Lli;
                    int lo_need, hi_need;
                    if constexpr (WIN) {
                        const double r = A.window_ratio;
                        w = (r >= 1.0) ? L : (int)floor(r * (double)L);
                        if (w > L) w = L;
                        if (w < Lli - Lco) {   // the window admits no warping path
                            if (k == 0) {
                                A.res[out] = __builtin_huge_val();
                                ++npairs;
                            }
                            continue;
                        }
                        if constexpr (KIND == CDTW) {
                            // lower bound above the cut-off: D > cut-off, +inf without a sweep.
                            // The factor covers the rounding of the bound and of the DP
                            // (relative 1e-11 against under 1e-12 for 2 x 2048 terms).
                            if (nn && A.lb && lbv * (1.0 - 1e-11) > (double)cut) {
                                if (k == 0) {
                                    A.res[out] = __builtin_huge_val();
                                    ++npairs;
                                    ++nlb;
                                }
                                continue;
                            }
                        }
                        const int wb = (KIND == ERP) ? w + 1 : w;
                        lo_need = -(wb < Lli ? wb : Lli);
                        hi_need = wb < Lco ? wb : Lco;
                    } else {
                        const int H = A.band_half;
                        lo_need = d_end - H;
                        if (lo_need < 1 - Lli) lo_need = 1 - Lli;
                        hi_need = H < Lco - 1 ? H : Lco - 1;
                    }
                    int dlo = lo_need;
                    if (dlo & 1) dlo -= 1;   // first step a = 2 has even parity
                    const int dhi = dlo + 2 * G * C - 1;
                    if (dhi < hi_need) {     // this band is too narrow: hand the item back
                        if (k == 0) {
                            if (A.ovf_items) {
                                const unsigned int idx = atomicAdd(A.ovf_count, 1u);
                                A.ovf_items[idx] = (int32_t)item;
                            } else {
                                A.res[out] = __builtin_nan("");
                            }
                        }
                        continue;
                    }
                    if constexpr (WIN) {
                        ncnt0 = ncnt1 = 0;
    #pragma unroll
                        for (int m = 0; m < M2; ++m) {
                            const int d = dlo + 2 * k * C + m;
                            const int in = (d >= lo_need && d <= hi_need) ? 1 : 0;
                            if (m & 1) ncnt1 += in;
                            else ncnt0 += in;
                        }
                    }
                    lo_open = !WIN && dlo > 1 - Lli;
                    hi_open = !WIN && dhi < Lco - 1;
                    ke = (d_end - dlo) / M2;
                    me = (d_end - dlo) - ke * M2;
                    a_end = Lli + Lco;
                    a = 2;
                    dk = dlo + 2 * k * C;
                    const T H1 = (KIND == ERP) ? vabs(co[0] - gap) : INF;   // M(0,1)
                    const T V1 = (KIND == ERP) ? vabs(li[0] - gap) : INF;   // M(1,0)
    #pragma unroll
                    for (int m = 0; m < M2; ++m) {
                        const int d = dk + m;
                        val[m] = (d == 0) ? (T)0 : (d == 1 ? H1 : (d == -1 ? V1 : INF));
                        const int ad = d < 0 ? -d : d;
                        if constexpr (KIND == WDTW) {
                            int gi = 2 * ad - L + A.gtab_off;
                            gi = gi < 0 ? 0 : (gi >= A.gtab_len ? A.gtab_len - 1 : gi);
                            wt[m] = (T)A.gtab[gi];
                        }
                        if constexpr (KIND == CDTW) pen[m] = (ad > w) ? INF : (T)0;
                        if constexpr (KIND == ERP) pen[m] = (T)0;
                    }
                    apen = (KIND == ERP) ? w + 2 : 2;
                    if constexpr (KIND == ERP) {
                        if (apen <= 2) {
    #pragma unroll
                            for (int m = 0; m < M2; ++m) {
                                const int d = dk + m;
                                pen[m] = ((d < 0 ? -d : d) > w) ? INF : (T)0;
                            }
                        }
                    }
                    i0 = (2 - dk) / 2;
                    j0 = (2 + dk) / 2;
    #pragma unroll
                    for (int q = 0; q < CB; ++q) {
                        S[q] = sval(i0 - q);
                        Tt[q] = tval(j0 + q);
                    }
                    if (k == 0) {
    #pragma unroll
                        for (int n = 1; n <= CB; ++n) {
                            Sc[n - 1] = sval(i0 + n);
                            if constexpr (AHEAD) Sn[n - 1] = sval(i0 + CB + n);
                        }
                    }
                    if (k == G - 1) {
    #pragma unroll
                        for (int n = 1; n <= CB; ++n) {
                            Tc[n - 1] = tval(j0 + C - 1 + n);
                            if constexpr (AHEAD) Tn[n - 1] = tval(j0 + C - 1 + CB + n);
                        }
                    }
                    fin = false;
                    ovf = false;
                    have = true;
                    break;
                }
            } else {
                for (;;) {
                    const unsigned int p = fetch_slot(A, fnext, fend, lane, k);
                    const int64_t n_items = A.npairs_dev ? (int64_t)*A.npairs_dev : A.npairs;
                    if ((int64_t)p >= n_items) {
                        done = true;
                        break;
                    }
                    item = item_of(A, p);
                    Item it = decode_item(A, item);
                    if (it.skip) continue;
                    const int64_t oa = SA.off[it.a], ob = SB.off[it.b];
                    const int La = (int)(SA.off[it.a + 1] - oa), Lb = (int)(SB.off[it.b + 1] - ob);
                    if (La >= Lb) {
                        li = SA.v + oa; Lli = La; co = SB.v + ob; Lco = Lb;
                    } else {
                        li = SB.v + ob; Lli = Lb; co = SA.v + oa; Lco = La;
                    }
                    qa = it.a;
                    out = it.out;
                    if (nn) cut = nn_cut<T>(A, it.a);
                    else cut = (A.pcut && !A.plain) ? (T)A.pcut[it.cutidx] : INF;
                    const int L = Lli > Lco ? Lli : Lco;
                    const int d_end = Lco - Lli;
                    int lo_need, hi_need;
                    if constexpr (WIN) {
                        const double r = A.window_ratio;
                        w = (r >= 1.0) ? L : (int)floor(r * (double)L);
                        if (w > L) w = L;
                        if (w < Lli - Lco) {   // the window admits no warping path
                            if (k == 0) {
                                A.res[out] = __builtin_huge_val();
                                ++npairs;
                            }
                            continue;
                        }
                        if constexpr (KIND == CDTW) {
                            // lower bound above the cut-off: D > cut-off, +inf without a sweep.
                            // The factor covers the rounding of the bound and of the DP
                            // (relative 1e-11 against under 1e-12 for 2 x 2048 terms).
                            if (nn && A.lb && A.lb[out] * (1.0 - 1e-11) > (double)cut) {
                                if (k == 0) {
                                    A.res[out] = __builtin_huge_val();
                                    ++npairs;
                                    ++nlb;
                                }
                                continue;
                            }
                        }
                        const int wb = (KIND == ERP) ? w + 1 : w;
                        lo_need = -(wb < Lli ? wb : Lli);
                        hi_need = wb < Lco ? wb : Lco;
                    } else {
                        const int H = A.band_half;
                        lo_need = d_end - H;
                        if (lo_need < 1 - Lli) lo_need = 1 - Lli;
                        hi_need = H < Lco - 1 ? H : Lco - 1;
                    }
                    int dlo = lo_need;
                    if (dlo & 1) dlo -= 1;   // first step a = 2 has even parity
                    const int dhi = dlo + 2 * G * C - 1;
                    if (dhi < hi_need) {     // this band is too narrow: hand the item back
                        if (k == 0) {
                            if (A.ovf_items) {
                                const unsigned int idx = atomicAdd(A.ovf_count, 1u);
                                A.ovf_items[idx] = (int32_t)item;
                            } else {
                                A.res[out] = __builtin_nan("");
                            }
                        }
                        continue;
                    }
                    if constexpr (WIN) {
                        ncnt0 = ncnt1 = 0;
    #pragma unroll
                        for (int m = 0; m < M2; ++m) {
                            const int d = dlo + 2 * k * C + m;
                            const int in = (d >= lo_need && d <= hi_need) ? 1 : 0;
                            if (m & 1) ncnt1 += in;
                            else ncnt0 += in;
                        }
                    }
                    lo_open = !WIN && dlo > 1 - Lli;
                    hi_open = !WIN && dhi < Lco - 1;
                    ke = (d_end - dlo) / M2;
                    me = (d_end - dlo) - ke * M2;
                    a_end = Lli + Lco;
                    a = 2;
                    dk = dlo + 2 * k * C;
                    const T H1 = (KIND == ERP) ? vabs(co[0] - gap) : INF;   // M(0,1)
                    const T V1 = (KIND == ERP) ? vabs(li[0] - gap) : INF;   // M(1,0)
    #pragma unroll
                    for (int m = 0; m < M2; ++m) {
                        const int d = dk + m;
                        val[m] = (d == 0) ? (T)0 : (d == 1 ? H1 : (d == -1 ? V1 : INF));
                        const int ad = d < 0 ? -d : d;
                        if constexpr (KIND == WDTW) {
                            int gi = 2 * ad - L + A.gtab_off;
                            gi = gi < 0 ? 0 : (gi >= A.gtab_len ? A.gtab_len - 1 : gi);
                            wt[m] = (T)A.gtab[gi];
                        }
                        if constexpr (KIND == CDTW) pen[m] = (ad > w) ? INF : (T)0;
                        if constexpr (KIND == ERP) pen[m] = (T)0;
                    }
                    apen = (KIND == ERP) ? w + 2 : 2;
                    if constexpr (KIND == ERP) {
                        if (apen <= 2) {
    #pragma unroll
                            for (int m = 0; m < M2; ++m) {
                                const int d = dk + m;
                                pen[m] = ((d < 0 ? -d : d) > w) ? INF : (T)0;
                            }
                        }
                    }
                    i0 = (2 - dk) / 2;
                    j0 = (2 + dk) / 2;
    #pragma unroll
                    for (int q = 0; q < CB; ++q) {
                        S[q] = sval(i0 - q);
                        Tt[q] = tval(j0 + q);
                    }
                    if (k == 0) {
    #pragma unroll
                        for (int n = 1; n <= CB; ++n) {
                            Sc[n - 1] = sval(i0 + n);
                            if constexpr (AHEAD) Sn[n - 1] = sval(i0 + CB + n);
                        }
                    }
                    if (k == G - 1) {
    #pragma unroll
                        for (int n = 1; n <= CB; ++n) {
                            Tc[n - 1] = tval(j0 + C - 1 + n);
                            if constexpr (AHEAD) Tn[n - 1] = tval(j0 + C - 1 + CB + n);
                        }
                    }
                    fin = false;
                    ovf = false;
                    have = true;
                    break;
                }
            }
        }
        if (__all(done)) break;

        // one stage of the next item's fetch; its loads complete during the block
        if constexpr (PF) {
            if (have) {
                if (pf == 3) {
                    pf_request();
                    pf = 4;
                } else if (pf == 2) {
                    if ((int64_t)pf_p >= n_items_pf) pf = 5;
                    else {
                        pf_item = item_of(A, pf_p);
                        pf = 3;
                    }
                } else if (pf == 1) {
                    const unsigned int base = __shfl(pf_base, g0);
                    fnext = base;
                    fend = base + ch;
                    pf_p = fnext++;
                    pf = 2;
                } else if (pf == 0) {
                    if (fnext < fend) {
                        pf_p = fnext++;
                        pf = 2;
                    } else {
                        if (k == 0) pf_base = atomicAdd(A.queue, ch);
                        pf = 1;
                    }
                }
            }
        }

        // the query's best-so-far, read now and applied at the block end (a cut-off
        // one block old is only larger, so still safe); every eighth block only:
        // the read waits on memory that every group of every wave updates, at a
        // latency that a block of steps does not cover, and a cut-off a few
        // blocks old is still safe
        const bool refresh = (++nblk & 7) == 0;
        const T cut_next = (nn && have && refresh) ? nn_cut<T>(A, qa) : INF;
        bool live_any = false;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int p = t & 1;
            const int nr = t / 2, nc = (t + 1) / 2;
            // advance the row or column ring (entering value from the neighbour lane)
            if (t & 1) {
                const int n = (t + 1) / 2;
                T x = shl1(Tt[(n - 1) % CB]);
                if (k == G - 1) x = Tc[n - 1];
                Tt[(n + C - 1) % CB] = x;
            } else if (t > 0) {
                const int n = t / 2;
                T x = shr1(S[(C - n) % CB]);
                if (k == 0) x = Sc[n - 1];
                S[(CB - n) % CB] = x;
            }
            if constexpr (KIND == ERP) {
                if (have && !fin && a == apen) {
#pragma unroll
                    for (int m = 0; m < M2; ++m) {
                        const int d = dk + m;
                        pen[m] = ((d < 0 ? -d : d) > w) ? INF : (T)0;
                    }
                }
            }
            // the neighbouring diagonal across the strip end
            T xv;
            if (p == 0) {
                xv = shr1(val[M2 - 1]);
                if (k == 0) xv = INF;
            } else {
                xv = shl1(val[0]);
                if (k == G - 1) xv = INF;
            }
            if (have && !fin) {
                T mstep = INF;
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    const int m = p + 2 * q;
                    const T s = S[((q - nr) % CB + CB) % CB];
                    const T tt = Tt[(nc + q) % CB];
                    const T diag = val[m];
                    const T top = (m + 1 < M2) ? val[m + 1] : xv;
                    const T left = (m >= 1) ? val[m - 1] : xv;
                    const T d = s - tt;
                    T v;
                    if constexpr (sizeof(T) == 4 && (KIND == DTW || KIND == CDTW || KIND == WDTW)) {
                        // FP32 screen: the square (weighted) and the add fused; the
                        // window's penalty (0 or +inf) added to the minimum exactly
                        const T mn = vmin(vmin(diag, top), left);
                        if constexpr (KIND == DTW) v = __builtin_fmaf(d, d, mn);
                        if constexpr (KIND == CDTW) v = __builtin_fmaf(d, d, mn + pen[m]);
                        if constexpr (KIND == WDTW) v = __builtin_fmaf(wt[m] * d, d, mn);
                    } else if constexpr (KIND == DTW) {
                        v = (d * d) + vmin(vmin(diag, top), left);
                    } else if constexpr (KIND == CDTW) {
                        v = ((d * d) + pen[m]) + vmin(vmin(diag, top), left);
                    } else if constexpr (KIND == WDTW) {
                        v = (wt[m] * (d * d)) + vmin(vmin(diag, top), left);
                    } else if constexpr (KIND == ERP) {
                        v = vmin(vmin(diag + vabs(d), top + vabs(s - gap)), left + vabs(tt - gap)) + pen[m];
                    }
                    val[m] = v;
                    if (t >= NB - 2) mstep = vmin(mstep, v);
                }
                ncells += (p == 0) ? ncnt0 : ncnt1;
                if (t >= NB - 2) live_any = live_any || (mstep <= cut);
                if (p == 0) {
                    if (k == 0 && lo_open && val[0] <= cut) ovf = true;
                } else {
                    if (k == G - 1 && hi_open && val[M2 - 1] <= cut) ovf = true;
                }
                if (__builtin_expect(a == a_end, 0)) {   // once per pair: its code out of line
                    if (k == ke) {
                        T r = val[0];
#pragma unroll
                        for (int m = 1; m < M2; ++m)
                            if (m == me) r = val[m];
                        res_v = r;
                    }
                    fin = true;
                }
                a += 1;
            }
        }

        // the block's last row advance (n = CB), so that the next block starts in phase
        {
            T x = shr1(S[(C - CB + CB) % CB]);
            if (k == 0) x = Sc[CB - 1];
            S[0] = x;
        }

        const bool ovf_g = (ballot(have && ovf) & gmask) != 0;
        const bool alive = (ballot(live_any) & gmask) != 0;
        if (have) {
            if (fin && !ovf_g) {
                if (k == ke) {
                    const double D = (res_v <= cut) ? (double)res_v : __builtin_huge_val();
                    A.res[out] = D;
                    if (nn && D < __builtin_huge_val()) atomicMin(&A.best[qa], dbits(D));
                }
                have = false;
                if (k == 0) ++npairs;
            } else if (ovf_g) {
                if (k == 0) {
                    if (A.ovf_items) {
                        const unsigned int idx = atomicAdd(A.ovf_count, 1u);
                        A.ovf_items[idx] = (int32_t)item;
                    } else {
                        A.res[out] = __builtin_nan("");
                    }
                    atomicAdd(&A.counters[3], 1ull);
                }
                have = false;
            } else if (!alive) {
                if (k == 0) {
                    A.res[out] = __builtin_huge_val();
                    ++npairs;
                }
                have = false;
            } else {
                if (nn) cut = vmin(cut, cut_next);
                i0 += CB;
                j0 += CB;
                if constexpr (AHEAD) {
#pragma unroll
                    for (int q = 0; q < CB; ++q) {
                        Sc[q] = Sn[q];
                        Tc[q] = Tn[q];
                    }
                }
                if (k == 0) {
#pragma unroll
                    for (int n = 1; n <= CB; ++n) {
                        if constexpr (AHEAD) Sn[n - 1] = sval(i0 + CB + n);
                        else Sc[n - 1] = sval(i0 + n);
                    }
                }
                if (k == G - 1) {
#pragma unroll
                    for (int n = 1; n <= CB; ++n) {
                        if constexpr (AHEAD) Tn[n - 1] = tval(j0 + C - 1 + CB + n);
                        else Tc[n - 1] = tval(j0 + C - 1 + n);
                    }
                }
            }
        }
    }
    wave_add_u64(&A.counters[0], ncells);
    wave_add_u64(&A.counters[1], npairs);
    wave_add_u64(&A.counters[4], nlb);
    wave_add_u64(&A.stage[0], ncells);
    wave_add_u64(&A.stage[8], npairs);
}

template <int KIND, typename T, int G, int C>
static hipError_t gob(const SweepArgs& a, SeriesPtrs SA, SeriesPtrs SB, int grid, hipStream_t s, int* occ) {
    if (occ)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, reinterpret_cast<const void*>(&band_kernel<KIND, T, G, C>),
                                                            256, 0);
    Series<T> A{(const T*)SA.v, SA.off, (const T*)SA.border};
    Series<T> B{(const T*)SB.v, SB.off, (const T*)SB.border};
    hipLaunchKernelGGL((band_kernel<KIND, T, G, C>), dim3(grid), dim3(256), 0, s, a, A, B);
    return hipGetLastError();
}

template <int KIND, typename T>
static hipError_t gob_d(int diags, int g, const SweepArgs& a, SeriesPtrs SA, SeriesPtrs SB, int grid, hipStream_t s,
                        int* occ) {
    switch (diags * 100 + g) {
    case 3202: return gob<KIND, T, 2, 8>(a, SA, SB, grid, s, occ);
    case 3204: return gob<KIND, T, 4, 4>(a, SA, SB, grid, s, occ);
    case 6404: return gob<KIND, T, 4, 8>(a, SA, SB, grid, s, occ);
    case 6408: return gob<KIND, T, 8, 4>(a, SA, SB, grid, s, occ);
    case 12808: return gob<KIND, T, 8, 8>(a, SA, SB, grid, s, occ);
    case 12816: return gob<KIND, T, 16, 4>(a, SA, SB, grid, s, occ);
    case 25616: return gob<KIND, T, 16, 8>(a, SA, SB, grid, s, occ);
    case 25632: return gob<KIND, T, 32, 4>(a, SA, SB, grid, s, occ);
    case 51232: return gob<KIND, T, 32, 8>(a, SA, SB, grid, s, occ);
    case 51264: return gob<KIND, T, 64, 4>(a, SA, SB, grid, s, occ);
    case 102464: return gob<KIND, T, 64, 8>(a, SA, SB, grid, s, occ);
    case 204864: return gob<KIND, T, 64, 16>(a, SA, SB, grid, s, occ);
    }
    return hipErrorInvalidValue;
}

// The compiled band shapes: 4 or 8 diagonals per parity and lane (more only
// for the widest band; the band's rings and weights make wider lanes spill out
// of the register file).  16 diagonals on 2 lanes (4 per parity) were
// measured for the narrowest windows and were slower: their blocks of 8 steps
// fetch the entering series values too short a time ahead.
bool band_shape_ok(int diags, int g) {
    switch (diags * 100 + g) {
    case 3202: case 3204: case 6404: case 6408:
    case 12808: case 12816: case 25616: case 25632: case 51232: case 51264: case 102464: case 204864: return true;
    }
    return false;
}

hipError_t launch_band(int kind, bool fp32, int diags, int g, const SweepArgs& a, SeriesPtrs A, SeriesPtrs B,
                       int grid, hipStream_t s, int* occ) {
    if (!band_shape_ok(diags, g)) return hipErrorInvalidValue;
    if (fp32) {
        switch (kind) {
        case DTW: return gob_d<DTW, float>(diags, g, a, A, B, grid, s, occ);
        case CDTW: return gob_d<CDTW, float>(diags, g, a, A, B, grid, s, occ);
        case WDTW: return gob_d<WDTW, float>(diags, g, a, A, B, grid, s, occ);
        case ERP: return gob_d<ERP, float>(diags, g, a, A, B, grid, s, occ);
        }
    } else {
        switch (kind) {
        case DTW: return gob_d<DTW, double>(diags, g, a, A, B, grid, s, occ);
        case CDTW: return gob_d<CDTW, double>(diags, g, a, A, B, grid, s, occ);
        case WDTW: return gob_d<WDTW, double>(diags, g, a, A, B, grid, s, occ);
        case ERP: return gob_d<ERP, double>(diags, g, a, A, B, grid, s, occ);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace eap
