// Kernel A: row sweep of the cost matrix (eq. Common), one pair per group of
// G lanes, with the early abandoning and cut-off of EAPruned (Alg. 5).
//
// Layout.  The shorter series of a pair goes on the columns (Alg. 3/5).  Lane
// k of a group owns columns c0..c0+C-1 with c0 = 1 + k*C and keeps, in
// registers, its C cells of the last row it computed and the C column values
// t_j.  Rows are skewed across the group: at step s lane k computes row
// s - k, receiving the cell left of its strip, M(i, c0-1), and the row value
// s_i from lane k-1 through one DPP wave shift (lane 0 reads the left border
// and s_i from memory).  The previous left input is the diagonal of the
// strip's first cell.  Every dependency of a cell is thus in a register of
// its own lane or was computed by the left neighbour one step earlier.
//
// Abandoning.  Define sigma(i, k) = i + k, the step at which lane k computes
// row i.  Along any warping path sigma never decreases and grows by at most 2
// per step (the diagonal move across a strip boundary), so the cells of two
// consecutive steps s-1, s form a cut between M(0,0) and M(L_li, L_co).  When
// none of them is <= cut-off, no path to the end stays under the cut-off and
// the pair is abandoned - the same criterion as Alg. 5 ("no cell of a row
// stays under the cut-off"), applied to the staircase the group sweeps.
// Groups test it every K steps; cells are exact whenever they are <= cut-off,
// so the result is D when D <= cut-off and +inf otherwise.
//
// Columns beyond L_co in the last strip hold t = +inf, which makes their
// cells +inf for every distance, so they never count as alive.
#include "eap_pairs.h"

namespace eap {

template <int KIND, typename T, int G, int C>
__global__ __launch_bounds__(256) void rows_kernel(SweepArgs A, Series<T> SA, Series<T> SB) {
    constexpr int K = 8;  // steps between group decisions
    extern __shared__ unsigned char lds_raw[];
    T* tab = reinterpret_cast<T*>(lds_raw);
    if constexpr (KIND == TWE) {
        for (int m = threadIdx.x; m < A.tab_len; m += blockDim.x) tab[m] = (T)A.tab[m];
        __syncthreads();
    }
    const T INF = inf_v<T>();
    const int lane = threadIdx.x & 63;
    const int k = lane & (G - 1);
    const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (lane - k));
    const bool nn = is_nn_mode(A.mode) && !A.plain;
    const T gap = (T)A.gap, cc = (T)A.c, nu = (T)A.nu, lam = (T)A.lam;

    bool have = false, done = false;
    int32_t qa = 0;
    int64_t out = 0;
    const T* li = nullptr;
    const T* lib = nullptr;
    int Lli = 0, Lco = 0, kend = 0, uend = 0, row = 0;
    const int c0 = 1 + k * C;
    T cut = 0;
    T val[C], vb[C], tv[C], aux[C];
    T adv[KIND == TWE ? C : 1];   // TWE: |s_{i-1} - t_j| of the previous row
    T dg = 0, lout = 0, sout = 0, s_next = 0, b_next = 0, sp = 0, tpm = 0, brd0 = 0, s0 = 0;
    unsigned long long ncells = 0, npairs = 0;
#pragma unroll
    for (int u = 0; u < C; ++u) val[u] = vb[u] = tv[u] = aux[u] = 0;
#pragma unroll
    for (int u = 0; u < (KIND == TWE ? C : 1); ++u) adv[u] = 0;

    for (;;) {
        if (!have && !done) {
            // fetch the next work item for this group
            for (;;) {
                unsigned int p = 0;
                if (k == 0) p = atomicAdd(A.queue, 1u);
                p = __shfl(p, lane - k);
                const int64_t n_items = A.npairs_dev ? (int64_t)*A.npairs_dev : A.npairs;
                if ((int64_t)p >= n_items) {
                    done = true;
                    break;
                }
                Item it = decode_item(A, item_of(A, p));
                if (it.skip) continue;
                const int64_t oa = SA.off[it.a], ob = SB.off[it.b];
                const int La = (int)(SA.off[it.a + 1] - oa), Lb = (int)(SB.off[it.b + 1] - ob);
                const T* co;
                const T* cob;
                if (La >= Lb) {
                    li = SA.v + oa; lib = SA.border ? SA.border + oa : nullptr; Lli = La;
                    co = SB.v + ob; cob = SB.border ? SB.border + ob : nullptr; Lco = Lb;
                } else {
                    li = SB.v + ob; lib = SB.border ? SB.border + ob : nullptr; Lli = Lb;
                    co = SA.v + oa; cob = SA.border ? SA.border + oa : nullptr; Lco = La;
                }
                qa = it.a;
                out = it.out;
                if (Lco > G * C) {   // wider than this kernel's row: refuse rather than sweep part of it
                    if (k == 0) A.res[out] = __builtin_nan("");
                    continue;
                }
                if (nn) cut = nn_cut<T>(A, it.a);
                else cut = (A.pcut && !A.plain) ? (T)A.pcut[it.cutidx] : INF;
                kend = (Lco - 1) / C;
                uend = (Lco - 1) - kend * C;
                // column values t_j of the strip (+inf beyond L_co) and t_{c0-1} (t_0 = 0)
#pragma unroll
                for (int u = 0; u < C; ++u) tv[u] = (c0 + u <= Lco) ? co[c0 + u - 1] : INF;
                tpm = (c0 >= 2 && c0 - 1 <= Lco) ? co[c0 - 2] : (T)0;
#pragma unroll
                for (int u = 0; u < C; ++u) {
                    const T tprev = (u == 0) ? tpm : tv[u - 1];
                    const bool ghost = c0 + u > Lco;
                    if constexpr (KIND == ERP) aux[u] = ghost ? INF : vabs(tv[u] - gap);
                    if constexpr (KIND == MSM) aux[u] = ghost ? INF : tv[u] - tprev;
                    if constexpr (KIND == TWE) aux[u] = ghost ? INF : (vabs(tv[u] - tprev) + nu) + lam;
                    if constexpr (KIND == TWE) adv[u] = vabs((T)0 - tv[u]);   // row 0: s_0 = 0
                    // top border M(0, j): computed for ERP, +inf otherwise
                    if constexpr (KIND == ERP) val[u] = ghost ? INF : cob[c0 + u - 1];
                    else val[u] = INF;
                }
                // diagonal of the first cell of row 1: M(0, c0-1)
                if (k == 0) dg = 0;
                else if constexpr (KIND == ERP) dg = (c0 - 1 <= Lco) ? cob[c0 - 2] : INF;
                else dg = INF;
                // what a lane is fed until it reaches row 1 (see the step below):
                // ERP's border M(0, c0-1), which makes the lane recompute its own
                // top border exactly, or +inf, which keeps +inf borders at +inf
                if constexpr (KIND == ERP) brd0 = dg;
                else brd0 = INF;
                s0 = (KIND == ERP) ? gap : (T)0;
                // start late enough that the last cell, (L_li, L_co) in lane kend,
                // is computed by the last step of a block: the result is then read
                // once, at the block end, from the buffer that step wrote
                row = -k - (K - (Lli + kend) % K) % K;
                lout = val[C - 1];
                sout = 0;
                sp = 0;
                if (k == 0) {
                    s_next = li[0];
                    if constexpr (KIND == ERP) b_next = lib[0];
                    else b_next = INF;
                }
                have = true;
                break;
            }
        }
        if (__all(done)) break;

        bool live_any = false;
        // One step: every lane computes its strip for its current row, reading
        // the previous row from `src` and writing `dst` (the two buffers
        // alternate, so no value is copied).  Lanes that have not reached row 1
        // are fed their own left-border value and s = gap (ERP) or +inf inputs,
        // which reproduces their top border bit for bit; lanes past the last
        // row compute values nobody reads.
        auto step = [&](T (&src)[C], T (&dst)[C], bool check) {
            T lin = shr1(lout);
            T sin = shr1(sout);
            row += 1;
            if (k == 0) {
                lin = b_next;   // M(row, 0)
                sin = s_next;   // s_row
            }
            const bool ns = row <= 0;   // not started: keep the top border
            if (ns) {
                lin = brd0;
                sin = s0;
            }
            const bool act = have && row >= 1 && row <= Lli;
            if (k == 0 && act && row < Lli) {
                s_next = li[row];
                if constexpr (KIND == ERP) b_next = lib[row];
            }
            T diag = ns ? brd0 : dg;
            if (!ns) dg = lin;          // M(0, c0-1) stays the diagonal of row 1
            T left = lin;
            T sg = 0, ds = 0, gA = 0, carry = 0;
            const T* ntp = nullptr;
            if constexpr (KIND == ERP) sg = vabs(sin - gap);
            if constexpr (KIND == MSM) ds = sin - sp;
            if constexpr (KIND == TWE) {
                gA = (vabs(sin - sp) + nu) + lam;
                const int rr = row < 1 ? 1 : (row > Lli ? Lli : row);
                ntp = tab + (c0 - rr + A.tab_off);
            }
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const T top = src[u];
                const T d = sin - tv[u];
                T v;
                if constexpr (KIND == DTW || KIND == CDTW) {
                    v = (d * d) + vmin(vmin(diag, top), left);
                } else if constexpr (KIND == ERP) {
                    v = vmin(vmin(diag + vabs(d), top + sg), left + aux[u]);
                } else if constexpr (KIND == MSM) {
                    // C(s_i, s_{i-1}, t_j) and C(t_j, s_i, t_{j-1}) of eq. MSMCost as
                    // c + max(0, min(x,y) - np, np - max(x,y)), with the differences
                    // written through d = s_i - t_j, ds = s_i - s_{i-1}, dt = t_j - t_{j-1}.
                    // max(0, min(a,b), -max(a,b)) is |med3(a, b, 0)|, one instruction
                    // in FP32 (gfx950 has no FP64 med3); both select the same operand.
                    T c1, c2;
                    if constexpr (sizeof(T) == 4) {
                        c1 = cc + vabs(__builtin_amdgcn_fmed3f(ds, d, 0.0f));
                        c2 = cc + vabs(__builtin_amdgcn_fmed3f(d, -aux[u], 0.0f));
                    } else {
                        c1 = cc + vmax(vmax(vmin(-ds, -d), vmin(ds, d)), (T)0);
                        c2 = cc + vmax(vmax(vmin(d, -aux[u]), vmin(-d, aux[u])), (T)0);
                    }
                    v = vmin(vmin(diag + vabs(d), top + c1), left + c2);
                } else if constexpr (KIND == TWE) {
                    // |s_{i-1} - t_{j-1}| is the previous row's |d| one column to the
                    // left (rounded subtraction of the same operands)
                    const T ad = vabs(d);
                    const T adp = (u == 0) ? vabs(sp - tpm) : adv[u - 1];
                    if (u > 0) adv[u - 1] = carry;
                    carry = ad;
                    const T match = (ad + adp) + ntp[u];
                    v = vmin(vmin(diag + match, top + gA), left + aux[u]);
                }
                dst[u] = v;
                diag = top;
                left = v;
            }
            if constexpr (KIND == TWE) adv[C - 1] = carry;
            if (row >= 1) sp = sin;
            if (act) ncells += C;
            lout = dst[C - 1];
            sout = sin;
            if (check) {
                bool lv;
                if (!have || row > Lli) lv = false;
                else if (row < 1) lv = (KIND == ERP);   // top border row: +inf except for ERP
                else {
                    T m = lin;
#pragma unroll
                    for (int u = 0; u < C; ++u) m = vmin(m, dst[u]);
                    lv = (m <= cut);
                }
                live_any = live_any || lv;
            }
        };
#pragma unroll
        for (int t = 0; t < K; t += 2) {
            step(val, vb, t + 1 >= K - 2);
            step(vb, val, t + 2 >= K - 2);
        }

        // group decisions: finished, abandoned, or refresh the cut-off
        const bool fin_l = have && k == kend && row == Lli;
        const unsigned long long fm = ballot(fin_l);
        const unsigned long long lm = ballot(live_any);
        const bool fin = (fm & gmask) != 0;
        const bool alive = (lm & gmask) != 0;
        if (fin_l) {
            T r = val[0];
#pragma unroll
            for (int u = 1; u < C; ++u)
                if (u == uend) r = val[u];
            const double D = (r <= cut) ? (double)r : __builtin_huge_val();
            A.res[out] = D;
            if (nn && D < __builtin_huge_val()) atomicMin(&A.best[qa], dbits(D));
        }
        if (have && !fin && !alive && k == 0) A.res[out] = __builtin_huge_val();
        if (have && (fin || !alive)) {
            have = false;
            if (k == 0) ++npairs;
        } else if (have && nn) {
            cut = vmin(cut, nn_cut<T>(A, qa));
        }
    }
    wave_add_u64(&A.counters[0], ncells);
    wave_add_u64(&A.counters[1], npairs);
    wave_add_u64(&A.stage[0], ncells);
    wave_add_u64(&A.stage[8], npairs);
}

template <int KIND, typename T, int G, int C>
static hipError_t go(const SweepArgs& a, SeriesPtrs SA, SeriesPtrs SB, int grid, hipStream_t s) {
    Series<T> A{(const T*)SA.v, SA.off, (const T*)SA.border};
    Series<T> B{(const T*)SB.v, SB.off, (const T*)SB.border};
    size_t lds = (KIND == TWE) ? sizeof(T) * (size_t)a.tab_len : 0;
    hipLaunchKernelGGL((rows_kernel<KIND, T, G, C>), dim3(grid), dim3(256), lds, s, a, A, B);
    return hipGetLastError();
}

template <int KIND, typename T>
static hipError_t go_w(int width, const SweepArgs& a, SeriesPtrs SA, SeriesPtrs SB, int grid, hipStream_t s) {
    switch (width) {
    case 128: return go<KIND, T, 16, 8>(a, SA, SB, grid, s);
    case 256: return go<KIND, T, 16, 16>(a, SA, SB, grid, s);
    case 512: return go<KIND, T, 32, 16>(a, SA, SB, grid, s);
    case 1024: return go<KIND, T, 64, 16>(a, SA, SB, grid, s);
    }
    return hipErrorInvalidValue;
}

int rows_lds_bytes(int kind, bool fp32, const SweepArgs& a) {
    return kind == TWE ? (int)((fp32 ? 4 : 8) * (size_t)a.tab_len) : 0;
}

hipError_t launch_rows(int kind, bool fp32, int width, const SweepArgs& a, SeriesPtrs A, SeriesPtrs B, int grid,
                       hipStream_t s) {
    if (fp32) {
        switch (kind) {
        case DTW: case CDTW: return go_w<DTW, float>(width, a, A, B, grid, s);
        case ERP: return go_w<ERP, float>(width, a, A, B, grid, s);
        case MSM: return go_w<MSM, float>(width, a, A, B, grid, s);
        case TWE: return go_w<TWE, float>(width, a, A, B, grid, s);
        }
    } else {
        switch (kind) {
        case DTW: case CDTW: return go_w<DTW, double>(width, a, A, B, grid, s);
        case ERP: return go_w<ERP, double>(width, a, A, B, grid, s);
        case MSM: return go_w<MSM, double>(width, a, A, B, grid, s);
        case TWE: return go_w<TWE, double>(width, a, A, B, grid, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace eap
