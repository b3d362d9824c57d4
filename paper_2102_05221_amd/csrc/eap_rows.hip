// Kernel A: row sweep of the cost matrix (eq. Common), one pair per group of
// G lanes, with the early abandoning and cut-off of EAPruned (Alg. 5).
//
// Layout.  The shorter series of a pair goes on the columns (Alg. 3/5).  The
// columns are cut into strips of W = G*C; the group sweeps the strips of a
// pair one after the other.  In a strip, lane k owns columns c0..c0+C-1 with
// c0 = cb + 1 + k*C (cb = first column of the strip minus one) and keeps, in
// registers, its C cells of the last row it computed and the C column values
// t_j.  Rows are skewed across the group: at step s lane k computes row
// s - k, receiving the cell left of its columns, M(i, c0-1), and the row value
// s_i from lane k-1 through one DPP wave shift.  Lane 0 reads the left input
// from the left border (first strip) or from the edge buffer, where the last
// lane of the previous strip stored M(i, cb), one value per row.  The previous
// left input is the diagonal of a lane's first cell.  Every dependency of a
// cell is thus in a register of its own lane or was computed by the left
// neighbour one step earlier.
//
// Abandoning.  Define sigma(i, k) = i + k, the step at which lane k computes
// row i.  Along any warping path sigma never decreases and grows by at most 2
// per step (the diagonal move across a lane boundary), so the cells of two
// consecutive steps s-1, s form a cut between the strip's entry and its exit.
// When none of them is <= cut-off and no left input still to come is either,
// no path through the strip stays under the cut-off: the strip ends (its live
// edge rows are recorded for the next strip) or, in the last strip, the pair
// is abandoned - the criterion of Alg. 5 ("no cell of a row stays under the
// cut-off") applied to the staircase the group sweeps.  A strip also starts
// at the first row whose left input is <= cut-off (the cells above it only
// have inputs > cut-off), so each strip sweeps only the rows a live path can
// cross: column pruning at strip granularity.  Groups decide every K steps;
// cells are exact whenever they are <= cut-off, so the result is D when
// D <= cut-off and +inf otherwise.
//
// Columns beyond L_co in the last strip hold t = +inf, which makes their
// cells +inf for every distance, so they never count as alive.
//
// Per-diagonal terms (TWE's nu * 2|i-j|, WDTW's weight of |i-j|) come from an
// LDS table; each lane reads the C + K - 1 entries its next K steps need into
// registers at the start of every block.
//
// Exact differences (XD, FP32 WDTW only): the series stay in float64 (type V)
// and each cell rounds its difference s_i - t_j once to FP32 after forming it
// in float64, so the FP32 screen's error bound carries no input rounding (it
// is then relative: for long series WDTW's distances, scaled by weights near
// 1e-22, are far below the rounding of the inputs themselves).
#include <type_traits>

#include "eap_pairs.h"

namespace eap {

// Blocks per CU the register budget is sized for: 3 (168 VGPRs) for FP32,
// except TWE, ERP and MSM lanes of 16 or more columns (and exact-difference
// lanes), which spill at that budget - MSM into its step loop, a scratch
// reload and a wait on every step - and run with 256 VGPRs at 2 blocks per CU
// (measured on the 500 x 500, length-512 NN workload: TWE 8x16 3.49 against
// 4.87 ms); FP64: 2.
template <int KIND, typename T, int C, bool XD>
constexpr int rows_min_blocks() {
    return (sizeof(T) == 4 && !(C >= 16 && (KIND == TWE || KIND == ERP || KIND == MSM || XD))) ? 3 : 2;
}

template <typename T, bool XD> using RowValue = typename std::conditional<XD, double, T>::type;

template <int KIND, typename T, int G, int C, bool XD, int ND>
__global__ __launch_bounds__(256, (rows_min_blocks<KIND, T, C, XD>())) void rows_kernel(
    SweepArgs A, Series<RowValue<T, XD>> SA, Series<RowValue<T, XD>> SB) {
    using V = RowValue<T, XD>;   // type of the series values
    using P = Pt<V, ND>;         // one series point (ND channels for multivariate DTW / CDTW)
    constexpr bool DTAB = (KIND == TWE || KIND == WDTW);
    // steps between group decisions: long blocks share the block-end work
    // (ballots, cut-off, strip and pair bookkeeping) among more steps, and
    // stage more row inputs per lane (K / G) and, for TWE and WDTW, keep
    // C + K - 1 per-diagonal terms in registers; the distances with the most
    // registers per column (MSM, TWE, WDTW) take shorter blocks with wide lanes,
    // and so do multivariate lanes (K / G staged points of ND channels)
    constexpr int K = (ND > 1 || (C > 8 && (KIND == MSM || DTAB))) ? 16 : 32;
    constexpr int W = G * C;
    constexpr int NW = DTAB ? C + K - 1 : 1;
    if (A.prio) __builtin_amdgcn_s_setprio(2);
    extern __shared__ unsigned char lds_raw[];
    T* tab = reinterpret_cast<T*>(lds_raw);
    int tab_len = 1, tab_off = 0;
    if constexpr (DTAB) {
        const double* src = (KIND == TWE) ? A.tab : A.gtab;
        tab_len = (KIND == TWE) ? A.tab_len : A.gtab_len;
        tab_off = (KIND == TWE) ? A.tab_off : A.gtab_off;
        for (int m = threadIdx.x; m < tab_len; m += blockDim.x) tab[m] = (T)src[m];
        __syncthreads();
    }
    const T INF = inf_v<T>();
    const int lane = threadIdx.x & 63;
    const int k = lane & (G - 1);
    const int gaddr = (lane - k) * 4;   // byte address of the group's first lane (ds_bpermute)
    const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (lane - k));
    // NN search with a shared best-so-far (not the plain DP, not prune-only)
    const bool nn = is_nn_mode(A.mode) && !A.plain && !A.prune_only;
    const T gap = (T)A.gap, cc = (T)A.c, nu = (T)A.nu, lam = (T)A.lam;
    // this group's edge buffer: M(i, cb) of the previous strip, i = 0..L_li
    const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    T* const eb = A.edge ? reinterpret_cast<T*>(A.edge) + gid * A.edge_stride : nullptr;

    bool have = false, done = false;
    unsigned int nblk = 0;              // blocks swept by the wave (the cut-off refresh)
    unsigned int fnext = 0, fend = 0;   // this group's chunk of work slots
    int32_t qa = 0;
    int64_t out = 0;
    // Every lane loads its row inputs at every step, also in groups without a
    // pair: until a group fetches one, li and bp point at a valid one-value
    // range (the first value of set A), so those loads stay in bounds.
    const V* li = SA.v;
    const V* lib = nullptr;
    const V* co = nullptr;
    const V* cob = nullptr;
    int Lli = 1, Lco = 0, kend = 0, uend = 0, row = 0;
    int nstrip = 1, si = 0, cb = 0, c0 = 1, r_start = 1;
    int e_lo = 0, e_hi = -1;       // rows of the incoming edge that can be <= cut-off
    // the same for the edge this strip writes, over the rows this lane has
    // checked (reduced over the group when the strip ends)
    int rec_lo = 0, rec_hi = -1;
    // The last lane's right-edge values of the current block, one slot per
    // step (beside their store to the edge buffer), checked by the whole
    // group at the block end, K / G slots per lane: no per-step work beyond
    // the store.  A group never spans two waves, so no barrier.
    __shared__ T eblk[256 / G][K];
    const int gslot = threadIdx.x / G;
    bool last = true, full_top = true;
    T cut = 0;
    T val[C], vb[C], aux[C];
    P tv[C];
    T adv[KIND == TWE ? C : 1];   // TWE: |s_{i-1} - t_j| of the previous row
    T dwin[NW];                   // per-diagonal terms of this block
    T dg = 0, lout = 0, brd0 = 0;
    P sout = pt_fill<V, ND>(0), s0 = pt_fill<V, ND>(0);
    V sp = 0, tpm = 0;
    int wcap = 0;   // CDTW (multivariate, on the row sweep): the pair's window
    // Lane 0's inputs of a block's K rows (s_i and M(i, cb)) are staged across
    // the group: lane j holds rows R0 + 1 + j + G*i (i < RS; R0 = lane 0's row
    // before the block), loaded one block ahead, and lane 0 reads the one for
    // each step with a cross-lane permute.
    constexpr int RS = (K + G - 1) / G;
    P st_s[RS], nx_s[RS];
    T st_b[RS], nx_b[RS];
#pragma unroll
    for (int i = 0; i < RS; ++i) {
        st_s[i] = nx_s[i] = pt_fill<V, ND>(0);
        st_b[i] = nx_b[i] = 0;
    }
    // left inputs: bp[i] = M(i, cb) for e_lo <= i <= e_hi (until a pair is
    // fetched, and in the first strip of +inf borders, a valid dummy range)
    const T* bp = reinterpret_cast<const T*>(SA.v) - 1;
    unsigned long long ncells = 0, npairs = 0, nlb = 0;
#pragma unroll
    for (int u = 0; u < C; ++u) {
        val[u] = vb[u] = aux[u] = 0;
        tv[u] = pt_fill<V, ND>(0);
    }
#pragma unroll
    for (int u = 0; u < (KIND == TWE ? C : 1); ++u) adv[u] = 0;
#pragma unroll
    for (int m = 0; m < NW; ++m) dwin[m] = 0;

    // Row value s_r and left input M(r, cb) for lane 0: the left border (first
    // strip) or the previous strip's edge, +inf outside its live rows.  Every
    // lane loads (rows clamped into 1..L_li, so every address is in bounds) and
    // only lane 0's values are used: no branch in the step.
    auto load_row = [&](int r, P& sv, T& bv) {
        const unsigned rc = (unsigned)__builtin_elementwise_min(__builtin_elementwise_max(r, 1), Lli);
#pragma unroll
        for (int ch = 0; ch < ND; ++ch) sv.c[ch] = li[(rc - 1u) * ND + ch];
        const T x = load_nc(bp + rc);
        bv = (r >= e_lo && r <= e_hi) ? x : INF;   // e_hi < e_lo: no live row
    };

    // Set up the strip si of the current pair.
    auto start_strip = [&]() {
        cb = si * W;
        if (si == 0) {
            // the left border M(i, 0): computed for ERP, +inf otherwise
            e_lo = 1;
            e_hi = (KIND == ERP) ? Lli : 0;
            if constexpr (KIND == ERP) bp = lib - 1;
            else bp = reinterpret_cast<const T*>(li) - 1;
        } else {
            bp = eb;
        }
        c0 = cb + 1 + k * C;
        last = (si == nstrip - 1);
        // the first row: 1, unless the strip's top border and the incoming edge
        // are > cut-off down to some row (only for strips after the first)
        r_start = 1;
        if (si > 0 && !A.no_prune) {
            bool top_live = (e_lo <= 1);
            if constexpr (KIND == ERP) top_live = top_live || (cob[cb] <= cut);   // M(0, cb+1)
            if (!top_live) r_start = e_lo;
        }
        full_top = (r_start == 1);
        rec_lo = 1 << 30;
        rec_hi = -1;
        // column values t_j of the strip (+inf beyond L_co) and t_{c0-1} (t_0 = 0)
#pragma unroll
        for (int u = 0; u < C; ++u)
#pragma unroll
            for (int ch = 0; ch < ND; ++ch) tv[u].c[ch] = (c0 + u <= Lco) ? co[(c0 + u - 1) * ND + ch] : inf_v<V>();
        tpm = (c0 >= 2 && c0 - 1 <= Lco) ? co[(c0 - 2) * ND] : (V)0;
#pragma unroll
        for (int u = 0; u < C; ++u) {
            const T tprev = (u == 0) ? tpm : tv[u - 1].c[0];
            const bool ghost = c0 + u > Lco;
            if constexpr (KIND == ERP) aux[u] = ghost ? INF : vabs(tv[u].c[0] - gap);
            if constexpr (KIND == MSM) aux[u] = ghost ? INF : tv[u].c[0] - tprev;
            if constexpr (KIND == TWE) aux[u] = ghost ? INF : (vabs(tv[u].c[0] - tprev) + nu) + lam;
            if constexpr (KIND == TWE) adv[u] = vabs((T)0 - tv[u].c[0]);   // row 0: s_0 = 0
            // the row above the first: the top border M(0, j) (computed for ERP,
            // +inf otherwise), or +inf when the strip starts lower down
            if constexpr (KIND == ERP) val[u] = (ghost || !full_top) ? INF : cob[c0 + u - 1];
            else val[u] = INF;
        }
        // M(r_start - 1, c0 - 1): the diagonal of the lane's first cell
        T topl = INF;
        if (full_top) {
            if (c0 == 1) topl = 0;
            else if constexpr (KIND == ERP) topl = (c0 - 1 <= Lco) ? cob[c0 - 2] : INF;
        }
        dg = topl;
        // what a lane is fed until it reaches its first row (see the step below):
        // ERP's border M(0, c0-1), which makes the lane recompute its own top
        // border exactly, or +inf, which keeps +inf borders at +inf
        brd0 = (KIND == ERP) ? topl : INF;
        s0 = pt_fill<V, ND>((KIND == ERP) ? (V)gap : (V)0);
        // the last strip starts late enough that the last cell, (L_li, L_co) in
        // lane kend, is computed by the last step of a block: the result is then
        // read once, at the block end, from the buffer that step wrote
        int pad = 0;
        if (last) {
            const int lc = Lco - 1 - cb;
            kend = lc / C;
            uend = lc - kend * C;
            pad = (K - ((Lli - r_start + 1) + kend) % K) % K;
        }
        row = r_start - 1 - k - pad;
        lout = val[C - 1];
        sout = pt_fill<V, ND>(0);
        sp = 0;
        // the first block's row inputs (the loop stages each next block)
#pragma unroll
        for (int i = 0; i < RS; ++i) load_row(row + k + 1 + k + G * i, st_s[i], st_b[i]);
    };

    for (;;) {
        if (!have && !done) {
            // fetch the next work item for this group
            for (;;) {
                const unsigned int p = fetch_slot(A, fnext, fend, lane, k);
                const int64_t n_items = A.npairs_dev ? (int64_t)*A.npairs_dev : A.npairs;
                if ((int64_t)p >= n_items) {
                    done = true;
                    break;
                }
                Item it = decode_item(A, item_of(A, p));
                if (it.skip) continue;
                const int64_t oa = SA.off[it.a], ob = SB.off[it.b];
                const int La = (int)(SA.off[it.a + 1] - oa), Lb = (int)(SB.off[it.b + 1] - ob);
                if (La >= Lb) {
                    li = SA.v + oa * ND; lib = SA.border ? SA.border + oa : nullptr; Lli = La;
                    co = SB.v + ob * ND; cob = SB.border ? SB.border + ob : nullptr; Lco = Lb;
                } else {
                    li = SB.v + ob * ND; lib = SB.border ? SB.border + ob : nullptr; Lli = Lb;
                    co = SA.v + oa * ND; cob = SA.border ? SA.border + oa : nullptr; Lco = La;
                }
                if constexpr (KIND == CDTW) {
                    // the window of the pair; none that admits a path: +inf without a sweep
                    const int L = Lli;
                    const double wr = A.window_ratio;
                    wcap = (wr >= 1.0) ? L : (int)floor(wr * (double)L);
                    if (wcap > L) wcap = L;
                    if (wcap < Lli - Lco) {
                        if (k == 0) {
                            A.res[it.out] = __builtin_huge_val();
                            ++npairs;
                        }
                        continue;
                    }
                }
                qa = it.a;
                out = it.out;
                nstrip = (Lco + W - 1) / W;
                if (nstrip > 1 && (!eb || Lli >= A.edge_stride)) {
                    // no room for the strip edges: refuse rather than sweep part of the pair
                    if (k == 0) A.res[out] = __builtin_nan("");
                    continue;
                }
                if (nn) cut = nn_cut<T>(A, it.a);
                else cut = (A.pcut && !A.plain) ? (T)A.pcut[it.cutidx] : INF;
                // a lower bound above the cut-off (DTW searches with lower
                // bounds): D > cut-off, +inf without a sweep (the factor covers
                // the rounding of the bound and of the DP)
                if (nn && A.lb && A.lb[out] * (1.0 - 1e-11) > (double)cut) {
                    if (k == 0) {
                        A.res[out] = __builtin_huge_val();
                        ++npairs;
                        ++nlb;
                    }
                    continue;
                }
                si = 0;
                start_strip();
                have = true;
                break;
            }
        }
        if (__all(done)) break;

        if constexpr (DTAB) {
            // the per-diagonal terms of the next K steps: d = j - i runs over
            // c0 - row - K .. c0 + C - 2 - row.  A group without a pair reads
            // the window of d = 0 .. NW - 1 (its rows keep advancing while the
            // wave's other groups sweep, which would leave the table's range).
            const int base = have ? c0 - row - K : 0;
            if constexpr (KIND == TWE) {
                // the table covers every d this sweep forms (see its
                // construction): one address, the entries at fixed offsets
                const T* tp = tab + (base + tab_off);
#pragma unroll
                for (int m = 0; m < NW; ++m) dwin[m] = tp[m];
            } else {
                // WDTW: the weight of d is entry 2|d| - L_li + tab_off.  Entries
                // never decrease (g >= 0) and the table opens with zeros, so it
                // is the larger of the entries of 2d and -2d, two runs of NW
                // entries two apart read from fixed offsets: 2 (base + m) + c
                // upwards, and c - 2 (base + m) read from its far end.  A lane
                // whose window lies on one side of d = 0 points the other run at
                // the zeros.  Every entry read is inside the table: the table
                // covers |d| up to what the sweep forms, and the wrong side of a
                // window that crosses 0 stays at or above c - 2 (NW - 1) >= 0.
                const int c = tab_off - Lli;
                const T* const pp = tab + ((base + NW - 1 >= 0) ? 2 * base + c : 0);
                const T* const pn = tab + ((base <= 0) ? c - 2 * (base + NW - 1) : 0);
                // Eight entries at a time: their loads in flight together, and
                // each entry formed here (the empty asm keeps the maximum from
                // being sunk into the steps, where both runs would stay live).
                constexpr int CH = 8;
#pragma unroll
                for (int m0 = 0; m0 < NW; m0 += CH) {
                    T rp[CH], rn[CH];
#pragma unroll
                    for (int j = 0; j < CH; ++j)
                        if (m0 + j < NW) {
                            rp[j] = pp[2 * (m0 + j)];
                            rn[j] = pn[2 * (NW - 1 - m0 - j)];
                        }
#pragma unroll
                    for (int j = 0; j < CH; ++j)
                        if (m0 + j < NW) {
                            dwin[m0 + j] = vmax(rp[j], rn[j]);
                            asm volatile("" : "+v"(dwin[m0 + j]));
                        }
                }
            }
        }

        // stage the next block's row inputs (lane 0's row is row + k)
#pragma unroll
        for (int i = 0; i < RS; ++i) load_row(row + k + K + 1 + k + G * i, nx_s[i], nx_b[i]);
        // the query's best-so-far, read now and applied at the block end (a cut-off
        // one block old is only larger, so still safe); every eighth block only:
        // the read waits on memory that every group of every wave updates, and a
        // cut-off a few blocks old is still safe
        const bool refresh = (++nblk & 7) == 0;
        const T cut_next = (nn && have && refresh) ? nn_cut<T>(A, qa) : INF;

        bool live_any = false;
        // One step: every lane computes its columns for its current row, reading
        // the previous row from `src` and writing `dst` (the two buffers
        // alternate, so no value is copied).  Lanes that have not reached their
        // first row are fed their own left-border value and s = gap (ERP) or
        // +inf inputs, which reproduces their top border bit for bit; lanes past
        // the last row compute values nobody reads.  A block in which no lane
        // of the wave is before its first row or past the pair's last one (the
        // interior of a strip, nearly every block of a long one) runs a step
        // without those cases (FAST).
        // lane 0's row R0 + 1 + t is staged in lane t % G, slot t / G; each
        // step reads the next step's pair (M(row, cb), s_row) ahead, so the
        // cross-lane read overlaps a step of cell updates
        T pre_b = bperm(gaddr, st_b[0]);
        P pre_s = bperm(gaddr, st_s[0]);
        auto step = [&](T (&src)[C], T (&dst)[C], bool check, int t, auto fast_tag) {
            constexpr bool FAST = decltype(fast_tag)::value;
            T lin;
            P sin;
            row += 1;
            {
                const T bv = pre_b;   // M(row, cb)
                const P sv = pre_s;   // s_row
                if (t + 1 < K) {
                    pre_b = bperm(gaddr + 4 * ((t + 1) % G), st_b[(t + 1) / G]);
                    pre_s = bperm(gaddr + 4 * ((t + 1) % G), st_s[(t + 1) / G]);
                }
                if constexpr (G == 16) {
                    // a group is one DPP row: shift and feed lane 0 at once
                    lin = row_shr1_or(lout, bv);
                    sin = row_shr1_or(sout, sv);
                } else {
                    lin = shr1(lout);
                    sin = shr1(sout);
                    if (k == 0) {
                        lin = bv;
                        sin = sv;
                    }
                }
            }
            const bool ns = !FAST && row < r_start;   // not started: keep the top border
            if (ns) {
                lin = brd0;
                sin = s0;
            }
            const bool act = FAST ? have : (have && !ns && row <= Lli);
            T diag = ns ? brd0 : dg;
            if (!ns) dg = lin;          // M(r_start-1, c0-1) stays the diagonal of the first row
            T left = lin;
            T sg = 0, ds = 0, gA = 0, carry = 0;
            if constexpr (KIND == ERP) sg = vabs(sin.c[0] - gap);
            if constexpr (KIND == MSM) ds = sin.c[0] - sp;
            if constexpr (KIND == TWE) gA = (vabs(sin.c[0] - sp) + nu) + lam;
            const int wd = c0 - row;   // j - i of the lane's first cell (CDTW on the row sweep)
#pragma unroll
            for (int u = 0; u < C; ++u) {
                const T top = src[u];
                const T d = (T)(sin.c[0] - tv[u].c[0]);   // XD: formed in float64, rounded once
                T v;
                if constexpr (KIND == DTW || KIND == CDTW) {
                    // multivariate: the channels' squared differences added in channel order
                    T cost = d * d;
#pragma unroll
                    for (int ch = 1; ch < ND; ++ch) {
                        const T e = (T)(sin.c[ch] - tv[u].c[ch]);
                        cost = cost + e * e;
                    }
                    // CDTW on the row sweep: cells outside the window are +inf
                    if constexpr (KIND == CDTW) cost = cost + ((wd + u > wcap || wd + u < -wcap) ? INF : (T)0);
                    if constexpr (sizeof(T) == 4 && ND == 1 && KIND == DTW) {
                        // FP32 screen: the square and the add fused (one rounding
                        // fewer than the bound allows; an instruction fewer per cell)
                        v = __builtin_fmaf(d, d, vmin(vmin(diag, top), left));
                    } else {
                        v = cost + vmin(vmin(diag, top), left);
                    }
                } else if constexpr (KIND == WDTW) {
                    if constexpr (sizeof(T) == 4) {
                        v = __builtin_fmaf(dwin[u - t - 1 + K] * d, d, vmin(vmin(diag, top), left));
                    } else {
                        v = (dwin[u - t - 1 + K] * (d * d)) + vmin(vmin(diag, top), left);
                    }
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
                    const T match = (ad + adp) + dwin[u - t - 1 + K];
                    v = vmin(vmin(diag + match, top + gA), left + aux[u]);
                }
                dst[u] = v;
                diag = top;
                left = v;
            }
            if constexpr (KIND == TWE) adv[C - 1] = carry;
            if (!ns) sp = sin.c[0];
            // this strip's right edge, M(row, cb + W), for the next strip
            if (!last && k == G - 1 && act) {
                eb[row] = dst[C - 1];
                eblk[gslot][t] = dst[C - 1];
            }
            lout = dst[C - 1];
            sout = sin;
            if (check) {
                bool lv;
                if (!have || (!FAST && row > Lli)) lv = false;
                else if (ns) lv = (KIND == ERP) && full_top;   // the computed top border
                else {
                    T m = lin;
#pragma unroll
                    for (int u = 0; u < C; ++u) m = vmin(m, dst[u]);
                    lv = (m <= cut);
                }
                // left inputs still to come from the previous strip's live rows
                if (k == 0 && have && si > 0 && row < e_hi) lv = true;
                live_any = live_any || lv;
            }
        };
        // the staircase of the block's last two steps is the cut tested below
        auto block = [&](auto fast_tag) {
#pragma unroll
            for (int t = 0; t < K; t += 2) {
                step(val, vb, t >= K - 2, t, fast_tag);
                step(vb, val, t + 1 >= K - 2, t + 1, fast_tag);
            }
        };
        // rows row + 1 .. row + K of every lane with a pair within r_start..L_li
        if (__all(!have || (row + 1 >= r_start && row + K <= Lli))) block(std::true_type{});
        else block(std::false_type{});
#pragma unroll
        for (int i = 0; i < RS; ++i) {
            st_s[i] = nx_s[i];
            st_b[i] = nx_b[i];
        }
        if (have && !last) {
            // the rows of the edge written in this block that are <= cut-off:
            // lane G-1 computed rows R + 1 .. R + K (R its row before the block),
            // slot t holding row R + 1 + t where that step stored it
            const int r1 = row + k - (G - 1) - K + 1;
#pragma unroll
            for (int i = 0; i < (K + G - 1) / G; ++i) {
                const int t = k + G * i;
                if (t < K) {
                    const int r = r1 + t;
                    if (r >= r_start && r <= Lli && eblk[gslot][t] <= cut) {
                        rec_lo = vmin(rec_lo, r);
                        rec_hi = vmax(rec_hi, r);
                    }
                }
            }
        }
        if (have) {
            // rows of this block in r_start..L_li: the cells counted as executed
            const int lo = (row - K + 1 > r_start) ? row - K + 1 : r_start;
            const int hi = row < Lli ? row : Lli;
            if (hi >= lo) ncells += (unsigned long long)(C * (hi - lo + 1));
        }

        // group decisions: finished, strip done, abandoned, or refresh the cut-off
        const bool fin_l = have && last && k == kend && row == Lli;
        // never true (the last strip is aligned to end on a block end); a guard
        // that ends the pair with NaN rather than sweeping on past its last row
        const bool lost_l = have && last && k == kend && row > Lli;
        const bool send_l = have && !last && k == G - 1 && row >= Lli;
        const unsigned long long fm = ballot(fin_l);
        const unsigned long long sm = ballot(send_l);
        const unsigned long long lm = ballot(live_any);
        const bool lost = (ballot(lost_l) & gmask) != 0;
        const bool fin = (fm & gmask) != 0;
        const bool send = (sm & gmask) != 0;
        const bool alive = (lm & gmask) != 0;
        // a strip that ends (not the last one): its live edge rows over the group
        int nlo = rec_lo, nhi = rec_hi;
        if (__any(have && !last && (send || !alive))) {
#pragma unroll
            for (int o = 1; o < G; o <<= 1) {
                nlo = vmin(nlo, __shfl_xor(nlo, o));
                nhi = vmax(nhi, __shfl_xor(nhi, o));
            }
        }
        if (fin_l) {
            T r = val[0];
#pragma unroll
            for (int u = 1; u < C; ++u)
                if (u == uend) r = val[u];
            const double D = (r <= cut) ? (double)r : __builtin_huge_val();
            A.res[out] = D;
            if (nn && D < __builtin_huge_val()) atomicMin(&A.best[qa], dbits(D));
        }
        bool next_strip = false, drop = false;
        if (have && lost) {
            if (k == 0) A.res[out] = __builtin_nan("");
            have = false;
            if (k == 0) ++npairs;
        }
        if (have) {
            if (fin) {
                drop = true;
            } else if (!last && (send || !alive)) {
                if (nhi < nlo) drop = true;   // no edge row <= cut-off: no path goes on
                else if (send || !A.no_prune) next_strip = true;
                // without pruning the strip goes on to its last row
            } else if (!alive) {
                drop = true;
            }
        }
        if (drop) {
            if (!fin && k == 0) A.res[out] = __builtin_huge_val();
            have = false;
            if (k == 0) ++npairs;
        } else if (have && nn) {
            cut = vmin(cut, cut_next);
        }
        // the edge stores of this wave complete before the next strip reads them
        if (__any(next_strip)) __builtin_amdgcn_s_waitcnt(0);
        if (next_strip) {
            e_lo = nlo;
            e_hi = nhi;
            si += 1;
            start_strip();
        }
    }
    wave_add_u64(&A.counters[0], ncells);
    wave_add_u64(&A.counters[1], npairs);
    wave_add_u64(&A.stage[0], ncells);
    wave_add_u64(&A.stage[8], npairs);
    wave_add_u64(&A.counters[4], nlb);
}

template <int KIND, typename T, int G, int C, bool XD, int ND = 1>
static hipError_t go(const SweepArgs& a, SeriesPtrs SA, SeriesPtrs SB, int grid, hipStream_t s, int* occ) {
    using V = RowValue<T, XD>;
    const int lds = rows_lds_bytes(KIND, sizeof(T) == 4, a);
    if (occ)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            occ, reinterpret_cast<const void*>(&rows_kernel<KIND, T, G, C, XD, ND>), 256, (size_t)lds);
    Series<V> A{(const V*)SA.v, SA.off, (const V*)SA.border};
    Series<V> B{(const V*)SB.v, SB.off, (const V*)SB.border};
    hipLaunchKernelGGL((rows_kernel<KIND, T, G, C, XD, ND>), dim3(grid), dim3(256), lds, s, a, A, B);
    return hipGetLastError();
}

// Multivariate DTW and CDTW (FP64): G in {8, 16, 32, 64} x 8 columns per lane.
template <int KIND, int ND>
static hipError_t go_mv(RowsShape sh, const SweepArgs& a, SeriesPtrs SA, SeriesPtrs SB, int grid, hipStream_t s,
                        int* occ) {
    if (sh.c != 8) return hipErrorInvalidValue;
    switch (sh.g) {
    case 8: return go<KIND, double, 8, 8, false, ND>(a, SA, SB, grid, s, occ);
    case 16: return go<KIND, double, 16, 8, false, ND>(a, SA, SB, grid, s, occ);
    case 32: return go<KIND, double, 32, 8, false, ND>(a, SA, SB, grid, s, occ);
    case 64: return go<KIND, double, 64, 8, false, ND>(a, SA, SB, grid, s, occ);
    }
    return hipErrorInvalidValue;
}

template <int KIND>
static hipError_t go_mv_d(int nd, RowsShape sh, const SweepArgs& a, SeriesPtrs SA, SeriesPtrs SB, int grid,
                          hipStream_t s, int* occ) {
    switch (nd) {
    case 2: return go_mv<KIND, 2>(sh, a, SA, SB, grid, s, occ);
    case 3: return go_mv<KIND, 3>(sh, a, SA, SB, grid, s, occ);
    case 4: return go_mv<KIND, 4>(sh, a, SA, SB, grid, s, occ);
    }
    return hipErrorInvalidValue;
}

template <int KIND, typename T, bool XD = false>
static hipError_t go_w(RowsShape sh, const SweepArgs& a, SeriesPtrs SA, SeriesPtrs SB, int grid, hipStream_t s,
                       int* occ) {
    switch (sh.g * 1000 + sh.c) {
    case 4008: return go<KIND, T, 4, 8, XD>(a, SA, SB, grid, s, occ);
    case 4016: return go<KIND, T, 4, 16, XD>(a, SA, SB, grid, s, occ);
    case 8008: return go<KIND, T, 8, 8, XD>(a, SA, SB, grid, s, occ);
    case 8016: return go<KIND, T, 8, 16, XD>(a, SA, SB, grid, s, occ);
    case 16008: return go<KIND, T, 16, 8, XD>(a, SA, SB, grid, s, occ);
    case 16016: return go<KIND, T, 16, 16, XD>(a, SA, SB, grid, s, occ);
    case 32008: return go<KIND, T, 32, 8, XD>(a, SA, SB, grid, s, occ);
    case 32016: return go<KIND, T, 32, 16, XD>(a, SA, SB, grid, s, occ);
    case 64008: return go<KIND, T, 64, 8, XD>(a, SA, SB, grid, s, occ);
    case 64016: return go<KIND, T, 64, 16, XD>(a, SA, SB, grid, s, occ);
    }
    if constexpr (sizeof(T) == 4 && (KIND == DTW || KIND == WDTW)) {   // 32 columns per lane: registers
        switch (sh.g * 1000 + sh.c) {
        case 16032: return go<KIND, T, 16, 32, XD>(a, SA, SB, grid, s, occ);
        case 32032: return go<KIND, T, 32, 32, XD>(a, SA, SB, grid, s, occ);
        case 64032: return go<KIND, T, 64, 32, XD>(a, SA, SB, grid, s, occ);
        }
    }
    return hipErrorInvalidValue;
}

int rows_lds_bytes(int kind, bool fp32, const SweepArgs& a) {
    const size_t e = fp32 ? 4 : 8;
    if (kind == TWE) return (int)(e * (size_t)a.tab_len);
    if (kind == WDTW) return (int)(e * (size_t)a.gtab_len);
    return 0;
}

bool rows_shape_ok(int kind, RowsShape sh, bool fp32) {
    const bool c32 = fp32 && (kind == DTW || kind == CDTW || kind == WDTW);
    return (sh.g == 4 || sh.g == 8 || sh.g == 16 || sh.g == 32 || sh.g == 64) &&
           (sh.c == 8 || sh.c == 16 || (c32 && sh.g >= 16 && sh.c == 32));
}

hipError_t launch_rows(int kind, bool fp32, RowsShape sh, const SweepArgs& a, SeriesPtrs A, SeriesPtrs B, int grid,
                       hipStream_t s, int* occ, bool xd, int nd) {
    if (nd > 1) {   // multivariate: DTW, and CDTW (window on the row sweep), FP64
        if (fp32 || xd) return hipErrorInvalidValue;
        if (kind == DTW) return go_mv_d<DTW>(nd, sh, a, A, B, grid, s, occ);
        if (kind == CDTW) return go_mv_d<CDTW>(nd, sh, a, A, B, grid, s, occ);
        return hipErrorInvalidValue;
    }
    if (xd) {   // exact differences: FP32 WDTW on float64 series only
        if (fp32 && kind == WDTW) return go_w<WDTW, float, true>(sh, a, A, B, grid, s, occ);
        return hipErrorInvalidValue;
    }
    if (fp32) {
        switch (kind) {
        case DTW: case CDTW: return go_w<DTW, float>(sh, a, A, B, grid, s, occ);
        case WDTW: return go_w<WDTW, float>(sh, a, A, B, grid, s, occ);
        case ERP: return go_w<ERP, float>(sh, a, A, B, grid, s, occ);
        case MSM: return go_w<MSM, float>(sh, a, A, B, grid, s, occ);
        case TWE: return go_w<TWE, float>(sh, a, A, B, grid, s, occ);
        }
    } else {
        switch (kind) {
        case DTW: case CDTW: return go_w<DTW, double>(sh, a, A, B, grid, s, occ);
        case WDTW: return go_w<WDTW, double>(sh, a, A, B, grid, s, occ);
        case ERP: return go_w<ERP, double>(sh, a, A, B, grid, s, occ);
        case MSM: return go_w<MSM, double>(sh, a, A, B, grid, s, occ);
        case TWE: return go_w<TWE, double>(sh, a, A, B, grid, s, occ);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace eap
