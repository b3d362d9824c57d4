/*
 * CPU oracle for the six elastic distances of Herrmann & Webb, "Early
 * Abandoning and Pruning for Elastic Distances including Dynamic Time
 * Warping" (arXiv 2102.05221).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check
 * and the benchmark's CPU-baseline leg load this library.  It shares no code,
 * header, table or constant with the device library, and the device library
 * never loads it.
 *
 * Arithmetic: IEEE binary64, round to nearest even, built with
 * -ffp-contract=off (no fused multiply-add), no fast-math.  Cell formulas use
 * one fixed operation order per distance (documented at each formula).
 *
 * Contents
 *   orc_dp        the full cost matrix of eq. (Common) for each distance
 *                 (Section 2.3: eqs. DTW, ERP, MSM/MSMCost, TWE/TWECost, the
 *                 WDTW weight, and the Sakoe-Chiba window of Section 2.3.2);
 *                 the plain definition, O(L_S * L_T) memory.
 *   orc_brute     minimum over every monotone lattice path, enumerated
 *                 explicitly (the guarantees listed after eq. Common).
 *   orc_eap       EAPruned (Section 4), each row evaluated over the interval
 *                 of columns that the pruning rules of Sections 4.1-4.2 leave
 *                 live, with a cell counter.
 *   orc_eabase    EABase, Alg. 4: full rows, abandoned on a dead row.
 *   orc_ub        cost of the diagonal-then-straight warping path, an upper
 *                 bound usable as a prune-only cut-off (Section 4, intro).
 *   orc_envelope, orc_lb_keogh, orc_lb_kim
 *                 the lower bounds of Section 2.1 (definitions).
 *   orc_nn1       NN search, Alg. 1 (strict '<', lowest index wins ties); with
 *                 the full DP, EAPruned, EABase, or EAPruned behind the lower
 *                 bounds (Alg. 2).
 *   orc_pairwise  all pairs i<j, plain DP or prune-only EAPruned.
 *
 * Parity status: DTW, CDTW, ERP and MSM are pinned by the paper's worked
 * example, brute force and closed forms.  The WDTW recurrence (weight times
 * squared difference) and the TWE reading (L1 cost, s_0 = t_0 = 0, uniform
 * timestamps tau_i = i) are pinned by brute force and limit cases but the paper
 * prints no value for them: parity unpinned against the paper's numbers.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_DTW = 0, ORC_CDTW = 1, ORC_WDTW = 2, ORC_ERP = 3, ORC_MSM = 4, ORC_TWE = 5 };

/* prm[] layout used by every entry point: window_ratio, g, gap, c, nu, lambda,
 * dims.  dims > 1 (DTW and CDTW only) makes every series point a vector of
 * dims values, stored point after point; lengths and offsets count points. */
enum { P_WR = 0, P_G = 1, P_GAP = 2, P_C = 3, P_NU = 4, P_LAMBDA = 5, P_DIMS = 6 };

static int dims_of(const double* prm)
{
    int d = (int)prm[P_DIMS];
    return d < 1 ? 1 : d;
}

/* Squared Euclidean cost of two points of dims channels (Section 2.3: the
 * cost is "usually the squared Euclidean distance"; for multivariate series
 * it runs over the channels), added channel by channel from the first; one
 * channel gives d*d exactly as the univariate cost. */
static double sqcost(const double* x, int64_t i, const double* y, int64_t j, int dims)
{
    const double* a = x + (i - 1) * dims;
    const double* b = y + (j - 1) * dims;
    double d = a[0] - b[0];
    double s = d * d;
    for (int c = 1; c < dims; ++c) {
        double e = a[c] - b[c];
        s = s + e * e;
    }
    return s;
}

#define INF HUGE_VAL

static double dmin2(double a, double b) { return a < b ? a : b; }
static double dmin3(double a, double b, double c) { return dmin2(dmin2(a, b), c); }
static int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }
static int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t iabs(int64_t a) { return a < 0 ? -a : a; }

/* Window (Section 2.3.2): cells with |i - j| > w are outside the band.
 * Reading: the workloads give the window as a ratio of the longer length,
 * w = floor(ratio * max(L_S, L_T)); ratio >= 1 (or +inf) is no constraint.
 * Only CDTW and ERP take a window; the other distances are unconstrained.
 * "Unconstrained" is represented by w = max(L_S, L_T), which no |i-j| exceeds. */
int64_t orc_window(int kind, double ratio, int64_t lx, int64_t ly)
{
    int64_t L = imax(lx, ly);
    if (kind != ORC_CDTW && kind != ORC_ERP) return L;
    if (isnan(ratio) || ratio < 0) return -1;
    if (ratio >= 1.0) return L;
    int64_t w = (int64_t)floor(ratio * (double)L);
    return w > L ? L : w;
}

/* WDTW weight (eq. WDTW): w(d) = 1 / (1 + exp(-g * (d - L/2))), read with
 * w_max = 1 and L = the longer of the two lengths. */
void orc_wdtw_weights(double g, int64_t L, double* out)
{
    for (int64_t k = 0; k < L; ++k)
        out[k] = 1.0 / (1.0 + exp(-g * ((double)k - (double)L / 2.0)));
}

/* MSM split/merge cost (eq. MSMCost), written as defined: c when np lies
 * between x and y (either order, inclusive), else c plus the distance to the
 * nearer of the two. */
static double msm_cost(double np, double x, double y, double c)
{
    if ((x <= np && np <= y) || (x >= np && np >= y)) return c;
    double a = fabs(np - x), b = fabs(np - y);
    return c + dmin2(a, b);
}

/* ------------------------------------------------------------------------- */
/* Full cost matrix.  x (length lx) indexes rows i = 1..lx, y (length ly)
 * indexes columns j = 1..ly; x[i-1] is s_i.  M has (lx+1)*(ly+1) entries.
 *
 * Borders (eq. Common corner/vborder/hborder): M(0,0) = 0.  DTW, CDTW, WDTW,
 * MSM and TWE have +inf borders.  ERP computes them (eq. ERP):
 *   M(i,0) = M(i-1,0) + |s_i - gap|,  M(0,j) = M(0,j-1) + |t_j - gap|.
 * READING (window + computed borders): the border is computed on
 * 1..min(w+1, L), as Alg. 4/5 initialise it, and is +inf beyond.
 *
 * Interior cell (i,j), |i-j| <= w, with d = s_i - t_j (one rounding):
 *   DTW, CDTW  cost + min(diag, top, left),  cost = d*d      (eq. DTW)
 *   WDTW       cost + min(...),  cost = W[|i-j|] * (d*d)
 *   ERP        min(diag + |d|, top + |s_i - gap|, left + |t_j - gap|)
 *              (eq. ERP; its left term is read as cost(t_j, g))
 *   MSM        min(diag + |d|, top + C(s_i, s_{i-1}, t_j),
 *                  left + C(t_j, s_i, t_{j-1}))            (eq. MSM)
 *              the top term is +inf on row 1 and the left one on column 1
 *              (they would read s_0 / t_0 and sit on +inf borders)
 *   TWE        min(diag + ((|s_i - t_j| + |s_{i-1} - t_{j-1}|) + nu*(2|i-j|)),
 *                  top  + ((|s_i - s_{i-1}| + nu) + lambda),
 *                  left + ((|t_j - t_{j-1}| + nu) + lambda))  (eq. TWE/TWECost)
 *              with s_0 = t_0 = 0, L1 cost and timestamps tau_i = i, so
 *              nu(|tau_i - tau_j| + |tau_{i-1} - tau_{j-1}|) = nu * 2|i-j|.
 * Returns M(lx, ly) (+inf when the window forbids every path). */
static double cell_dp(int kind, const double* prm, const double* W, const double* x, const double* y,
                      int64_t i, int64_t j, double diag, double top, double left)
{
    double si = x[i - 1], tj = y[j - 1];
    double d = si - tj;
    switch (kind) {
    case ORC_DTW:
    case ORC_CDTW: {
        double cost = sqcost(x, i, y, j, dims_of(prm));
        return cost + dmin3(diag, top, left);
    }
    case ORC_WDTW: {
        double cost = W[iabs(i - j)] * (d * d);
        return cost + dmin3(diag, top, left);
    }
    case ORC_ERP: {
        double gap = prm[P_GAP];
        return dmin3(diag + fabs(d), top + fabs(si - gap), left + fabs(tj - gap));
    }
    case ORC_MSM: {
        double c = prm[P_C];
        double a = diag + fabs(d);
        double b = (i == 1) ? INF : top + msm_cost(si, x[i - 2], tj, c);
        double e = (j == 1) ? INF : left + msm_cost(tj, si, y[j - 2], c);
        return dmin3(a, b, e);
    }
    case ORC_TWE: {
        double nu = prm[P_NU], lam = prm[P_LAMBDA];
        double sp = (i == 1) ? 0.0 : x[i - 2];
        double tp = (j == 1) ? 0.0 : y[j - 2];
        double match = (fabs(d) + fabs(sp - tp)) + nu * (double)(2 * iabs(i - j));
        double delA = (fabs(si - sp) + nu) + lam;
        double delB = (fabs(tj - tp) + nu) + lam;
        return dmin3(diag + match, top + delA, left + delB);
    }
    }
    return NAN;
}

double orc_dp(int kind, const double* x, int64_t lx, const double* y, int64_t ly, const double* prm,
              double* M_out)
{
    if (lx < 1 || ly < 1) return NAN;
    int64_t w = orc_window(kind, prm[P_WR], lx, ly);
    if (w < 0) return NAN;
    int64_t nc = ly + 1;
    double* M = M_out ? M_out : (double*)malloc(sizeof(double) * (size_t)(lx + 1) * (size_t)nc);
    double* W = NULL;
    if (kind == ORC_WDTW) {
        W = (double*)malloc(sizeof(double) * (size_t)imax(lx, ly));
        orc_wdtw_weights(prm[P_G], imax(lx, ly), W);
    }
    double gap = prm[P_GAP];
    for (int64_t i = 0; i <= lx; ++i) {
        for (int64_t j = 0; j <= ly; ++j) {
            double v;
            if (i == 0 && j == 0) v = 0.0;
            else if (j == 0) v = (kind == ORC_ERP && i <= w + 1) ? M[(i - 1) * nc] + fabs(x[i - 1] - gap) : INF;
            else if (i == 0) v = (kind == ORC_ERP && j <= w + 1) ? M[j - 1] + fabs(y[j - 1] - gap) : INF;
            else if (iabs(i - j) > w) v = INF;
            else v = cell_dp(kind, prm, W, x, y, i, j, M[(i - 1) * nc + (j - 1)], M[(i - 1) * nc + j],
                             M[i * nc + (j - 1)]);
            M[i * nc + j] = v;
        }
    }
    double D = M[lx * nc + ly];
    free(W);
    if (!M_out) free(M);
    return D;
}

/* ------------------------------------------------------------------------- */
/* Brute force: every monotone lattice path from (0,0) to (lx,ly) with steps
 * diagonal (i+1,j+1), down (i+1,j) and right (i,j+1), its cost accumulated
 * step by step in path order with the same per-step term as the recurrence,
 * minimised over all paths.  Border cells are reachable only along row 0 or
 * column 0 (ERP: gap costs, within the w+1 border; others: +inf).  Paths
 * through a +inf cell are cut off early (their cost stays +inf). */
typedef struct {
    int kind;
    const double *prm, *W, *x, *y;
    int64_t lx, ly, w;
    double best;
    int64_t finite_paths;
} bf_ctx;

/* cost of stepping into (a,b) by move m (0 diag, 1 down, 2 right) with cost
 * so far acc; +inf when (a,b) may not be entered */
static double bf_step(const bf_ctx* b, int m, int64_t a, int64_t c, double acc)
{
    double gap = b->prm[P_GAP];
    if (a == 0 || c == 0) {
        if (b->kind != ORC_ERP) return INF;
        if (c == 0 && m == 1 && a <= b->w + 1) return acc + fabs(b->x[a - 1] - gap);
        if (a == 0 && m == 2 && c <= b->w + 1) return acc + fabs(b->y[c - 1] - gap);
        return INF;
    }
    if (iabs(a - c) > b->w) return INF;
    double si = b->x[a - 1], tj = b->y[c - 1], d = si - tj;
    switch (b->kind) {
    case ORC_DTW:
    case ORC_CDTW: return sqcost(b->x, a, b->y, c, dims_of(b->prm)) + acc;
    case ORC_WDTW: return (b->W[iabs(a - c)] * (d * d)) + acc;
    case ORC_ERP:
        if (m == 0) return acc + fabs(d);
        if (m == 1) return acc + fabs(si - gap);
        return acc + fabs(tj - gap);
    case ORC_MSM: {
        double cc = b->prm[P_C];
        if (m == 0) return acc + fabs(d);
        if (m == 1) return (a == 1) ? INF : acc + msm_cost(si, b->x[a - 2], tj, cc);
        return (c == 1) ? INF : acc + msm_cost(tj, si, b->y[c - 2], cc);
    }
    case ORC_TWE: {
        double nu = b->prm[P_NU], lam = b->prm[P_LAMBDA];
        double sp = (a == 1) ? 0.0 : b->x[a - 2];
        double tp = (c == 1) ? 0.0 : b->y[c - 2];
        if (m == 0) return acc + ((fabs(d) + fabs(sp - tp)) + nu * (double)(2 * iabs(a - c)));
        if (m == 1) return acc + ((fabs(si - sp) + nu) + lam);
        return acc + ((fabs(tj - tp) + nu) + lam);
    }
    }
    return NAN;
}

static void bf_rec(bf_ctx* b, int64_t i, int64_t j, double acc)
{
    if (acc == INF) return;
    if (i == b->lx && j == b->ly) {
        b->finite_paths++;
        if (acc < b->best) b->best = acc;
        return;
    }
    if (i < b->lx && j < b->ly) bf_rec(b, i + 1, j + 1, bf_step(b, 0, i + 1, j + 1, acc));
    if (i < b->lx) bf_rec(b, i + 1, j, bf_step(b, 1, i + 1, j, acc));
    if (j < b->ly) bf_rec(b, i, j + 1, bf_step(b, 2, i, j + 1, acc));
}

double orc_brute(int kind, const double* x, int64_t lx, const double* y, int64_t ly, const double* prm,
                 int64_t* n_finite_paths)
{
    if (lx < 1 || ly < 1 || lx > 12 || ly > 12) return NAN;
    bf_ctx b;
    b.kind = kind;
    b.prm = prm;
    b.x = x;
    b.y = y;
    b.lx = lx;
    b.ly = ly;
    b.w = orc_window(kind, prm[P_WR], lx, ly);
    if (b.w < 0) return NAN;
    double* W = NULL;
    if (kind == ORC_WDTW) {
        W = (double*)malloc(sizeof(double) * (size_t)imax(lx, ly));
        orc_wdtw_weights(prm[P_G], imax(lx, ly), W);
    }
    b.W = W;
    b.best = INF;
    b.finite_paths = 0;
    bf_rec(&b, 0, 0, 0.0);
    free(W);
    if (n_finite_paths) *n_finite_paths = b.finite_paths;
    return b.best;
}

/* ------------------------------------------------------------------------- */
/* The three additive terms of eq. (Common) for cell (i,j) of the matrix whose
 * rows are R (length lr) and columns C, in the same operation order as
 * cell_dp.  DTW-like distances add the same cost to every dependency:
 * cost + min(a,b,c) equals min(a+cost, b+cost, c+cost) exactly because
 * rounded addition is monotone. */
typedef struct {
    int kind;
    const double *prm, *W, *R, *C;
    int64_t lr, lc, w;
} eap_ctx;

static void terms(const eap_ctx* e, int64_t i, int64_t j, double* canon, double* arow, double* acol)
{
    double si = e->R[i - 1], tj = e->C[j - 1], d = si - tj;
    switch (e->kind) {
    case ORC_DTW:
    case ORC_CDTW: {
        double cost = sqcost(e->R, i, e->C, j, dims_of(e->prm));
        *canon = *arow = *acol = cost;
        return;
    }
    case ORC_WDTW: {
        double cost = e->W[iabs(i - j)] * (d * d);
        *canon = *arow = *acol = cost;
        return;
    }
    case ORC_ERP: {
        double gap = e->prm[P_GAP];
        *canon = fabs(d);
        *arow = fabs(si - gap);
        *acol = fabs(tj - gap);
        return;
    }
    case ORC_MSM: {
        double c = e->prm[P_C];
        *canon = fabs(d);
        *arow = (i == 1) ? INF : msm_cost(si, e->R[i - 2], tj, c);
        *acol = (j == 1) ? INF : msm_cost(tj, si, e->C[j - 2], c);
        return;
    }
    case ORC_TWE: {
        double nu = e->prm[P_NU], lam = e->prm[P_LAMBDA];
        double sp = (i == 1) ? 0.0 : e->R[i - 2];
        double tp = (j == 1) ? 0.0 : e->C[j - 2];
        *canon = (fabs(d) + fabs(sp - tp)) + nu * (double)(2 * iabs(i - j));
        *arow = (fabs(si - sp) + nu) + lam;
        *acol = (fabs(tj - tp) + nu) + lam;
        return;
    }
    }
}

/* Orientation shared by the cut-off variants: the shorter series on the
 * columns, the longer on the rows (Section 2.4); the window; the WDTW
 * weights.  Returns 0, or 1 when the window admits no path (result +inf),
 * or -1 on a bad argument. */
static int eap_setup(eap_ctx* e, int kind, const double* S, int64_t ls, const double* T, int64_t lt,
                     const double* prm, double** W)
{
    e->kind = kind;
    e->prm = prm;
    if (ls >= lt) {
        e->R = S; e->lr = ls; e->C = T; e->lc = lt;
    } else {
        e->R = T; e->lr = lt; e->C = S; e->lc = ls;
    }
    e->w = orc_window(kind, prm[P_WR], ls, lt);
    *W = NULL;
    e->W = NULL;
    if (e->w < 0) return -1;
    if (e->w < e->lr - e->lc) return 1;
    if (kind == ORC_WDTW) {
        *W = (double*)malloc(sizeof(double) * (size_t)e->lr);
        orc_wdtw_weights(prm[P_G], e->lr, *W);
        e->W = *W;
    }
    return 0;
}

/* One interior cell from whichever dependencies are given (+inf for the
 * others), in the operation order of cell_dp. */
static double cell_from(const eap_ctx* e, int64_t i, int64_t j, double diag, double top, double left)
{
    double canon, arow, acol;
    terms(e, i, j, &canon, &arow, &acol);
    return dmin3(diag + canon, top + arow, left + acol);
}

/* EAPruned (Section 4).  Returns D(S,T) when D <= cutoff, else +inf.
 *
 * Written from the definitions of Sections 4.1 and 4.2 rather than from the
 * staged loop of Alg. 5.  A cell is alive when its value is <= cutoff.
 * Costs are non-negative and rounded addition is monotone, so a cell's value
 * is never below its smallest dependency: a cell whose dependencies are all
 * dead is dead, and a dead cell never leads to an alive one.  Hence the only
 * cells worth evaluating in row i are those that have an alive dependency:
 *
 *  - pruning from the left (Section 4.1): left of the previous row's first
 *    alive cell, every top and diagonal dependency is dead (a discard zone or
 *    a run of discard points above), so row i starts at that column - or at
 *    column 1 when its own left border is computed and alive (ERP);
 *  - pruning on the right (Section 4.2): past the previous row's last alive
 *    cell p-1 (p is that row's pruning point), only the cell at p still has
 *    an alive (diagonal) dependency; beyond it a cell can only be alive
 *    through its left neighbour, so the row goes on while its last cell is
 *    alive;
 *  - early abandoning: when no cell of a row (left border included) is
 *    alive, no path to (L_li, L_co) stays under the cut-off.
 *
 * Every row is then the interval [lo, hi] of columns it evaluates, read from
 * the previous row's alive extent; dependencies outside the previous row's
 * evaluated interval are dead and read as +inf.  Alive cells come out exact
 * (their smallest dependency is alive, hence exact, by induction); dead cells
 * come out > cutoff, though not necessarily with their exact value.
 * Borders (eq. Common): M(0,0) = 0; the top border M(0,j) and the left
 * border M(i,0) are computed for ERP on 1..w+1 (Alg. 4's initialisation,
 * reading R5) and +inf otherwise; the left border of row i is evaluated only
 * while the one above it was alive (a dead border stays dead).  The result is
 * M(L_li, L_co) when the last row evaluated column L_co and it is alive.
 *
 * These intervals evaluate the same cells as the staged loop of Alg. 5 for
 * the distances with +inf borders (the worked example's counts of Section 4.2
 * follow: 5 and 16 cells saved, abandoned at (5,3)); with a live computed
 * left border (ERP) a row without an alive interior cell gets the pruning
 * point its definition gives, 1, where the printed loop keeps the previous
 * row's.
 *
 * cells (nullable) counts the interior cells evaluated; ab_i/ab_j (nullable)
 * receive the last cell evaluated in the row where the pair was abandoned
 * (0,0 when it was not). */
double orc_eap(int kind, const double* S, int64_t ls, const double* T, int64_t lt, const double* prm,
               double cutoff, int64_t* cells, int64_t* ab_i, int64_t* ab_j)
{
    if (ls < 1 || lt < 1 || isnan(cutoff)) return NAN;
    if (cells) *cells = 0;
    if (ab_i) *ab_i = 0;
    if (ab_j) *ab_j = 0;
    eap_ctx e;
    double* W;
    int st = eap_setup(&e, kind, S, ls, T, lt, prm, &W);
    if (st < 0) return NAN;
    if (st > 0) return INF;
    const int64_t Lco = e.lc, Lli = e.lr, w = e.w;
    const double gap = prm[P_GAP];
    double* prev = (double*)malloc(sizeof(double) * (size_t)(Lco + 1));
    double* curr = (double*)malloc(sizeof(double) * (size_t)(Lco + 1));
    int64_t n_cells = 0;

    /* row 0, the top border: evaluated on [0, hb] */
    int64_t hb = (kind == ORC_ERP) ? imin(w + 1, Lco) : 0;
    prev[0] = 0.0;
    for (int64_t j = 1; j <= hb; ++j) prev[j] = prev[j - 1] + fabs(e.C[j - 1] - gap);
    int64_t plo = 0, phi = hb;             /* evaluated interval of the previous row */
    int64_t first = 0, last = 0;           /* its first and last alive columns */
    for (int64_t j = 0; j <= hb; ++j)
        if (prev[j] <= cutoff) last = j;   /* M(0,0) = 0 is alive: cutoff >= 0 */

    double result = INF;
    int abandoned = 0;
    for (int64_t i = 1; i <= Lli; ++i) {
        /* left border of row i, evaluated while the border above is alive */
        double border = INF;
        if (kind == ORC_ERP && i <= w + 1 && plo == 0 && prev[0] <= cutoff)
            border = prev[0] + fabs(e.R[i - 1] - gap);
        const int64_t jmax = imin(i + w, Lco);
        int64_t lo = (border <= cutoff) ? 1 : imax(first, 1);
        lo = imax(lo, i - w);
        const int64_t reach = imin(last + 1, jmax);   /* last column with an alive top or diagonal */
        curr[lo - 1] = (lo == 1) ? border : INF;
        int64_t hi = lo - 1, nfirst = -1, nlast = -1;
        if (lo == 1 && border <= cutoff) nfirst = nlast = 0;
        for (int64_t j = lo; j <= jmax; ++j) {
            if (j > reach && curr[j - 1] > cutoff) break;   /* right of the pruning point, left dead */
            double diag = (j - 1 >= plo && j - 1 <= phi) ? prev[j - 1] : INF;
            double top = (j >= plo && j <= phi) ? prev[j] : INF;
            curr[j] = cell_from(&e, i, j, diag, top, curr[j - 1]);
            ++n_cells;
            hi = j;
            if (curr[j] <= cutoff) {
                if (nfirst < 0) nfirst = j;
                nlast = j;
            }
        }
        if (nfirst < 0) {                   /* no alive cell: abandon */
            abandoned = 1;
            if (ab_i) *ab_i = i;
            if (ab_j) *ab_j = hi;
            break;
        }
        double* t = prev; prev = curr; curr = t;
        plo = lo - 1;
        phi = hi;
        first = nfirst;
        last = nlast;
    }
    if (!abandoned && phi == Lco && prev[Lco] <= cutoff) result = prev[Lco];
    free(prev);
    free(curr);
    free(W);
    if (cells) *cells = n_cells;
    return result;
}

/* EABase (Alg. 4): the usual early abandoning, no pruning.  Every row is
 * evaluated in full within the window, with all three dependencies; the pair
 * is abandoned after the first row whose smallest value (left border
 * included, as Alg. 4 stores it in the row) exceeds the cut-off.  Returns
 * M(L_li, L_co) when no row is abandoned (which may exceed the cut-off: the
 * last row's minimum need not be its last cell), else +inf.  cells
 * (nullable) counts the interior cells evaluated. */
double orc_eabase(int kind, const double* S, int64_t ls, const double* T, int64_t lt, const double* prm,
                  double cutoff, int64_t* cells)
{
    if (ls < 1 || lt < 1 || isnan(cutoff)) return NAN;
    if (cells) *cells = 0;
    eap_ctx e;
    double* W;
    int st = eap_setup(&e, kind, S, ls, T, lt, prm, &W);
    if (st < 0) return NAN;
    if (st > 0) return INF;
    const int64_t Lco = e.lc, Lli = e.lr, w = e.w;
    const double gap = prm[P_GAP];
    double* prev = (double*)malloc(sizeof(double) * (size_t)(Lco + 1));
    double* curr = (double*)malloc(sizeof(double) * (size_t)(Lco + 1));
    for (int64_t j = 0; j <= Lco; ++j) prev[j] = curr[j] = INF;
    curr[0] = 0.0;
    for (int64_t j = 1; j <= imin(w + 1, Lco); ++j)
        curr[j] = (kind == ORC_ERP) ? curr[j - 1] + fabs(e.C[j - 1] - gap) : INF;
    int64_t n_cells = 0;
    double result = INF;
    int abandoned = 0;
    for (int64_t i = 1; i <= Lli; ++i) {
        double* t = prev; prev = curr; curr = t;
        const int64_t js = imax(1, i - w), je = imin(i + w, Lco);
        curr[js - 1] = (js == 1 && kind == ORC_ERP) ? prev[0] + fabs(e.R[i - 1] - gap) : INF;
        double mn = curr[js - 1];
        for (int64_t j = js; j <= je; ++j) {
            curr[j] = cell_from(&e, i, j, prev[j - 1], prev[j], curr[j - 1]);
            ++n_cells;
            mn = dmin2(mn, curr[j]);
        }
        if (mn > cutoff) {
            abandoned = 1;
            break;
        }
    }
    if (!abandoned) result = curr[Lco];
    free(prev);
    free(curr);
    free(W);
    if (cells) *cells = n_cells;
    return result;
}

/* ------------------------------------------------------------------------- */
/* Upper bound from one warping path (Section 4, intro: any path's cost bounds
 * the optimum): the diagonal (1,1)..(m,m), m = min(L_S, L_T), then straight
 * down (or right) along the last column (row) to (L_S, L_T).  Each step adds
 * its term exactly as the recurrence does, so the result is >= the distance
 * in floating point too.  +inf when the window forbids the path. */
double orc_ub(int kind, const double* x, int64_t lx, const double* y, int64_t ly, const double* prm)
{
    if (lx < 1 || ly < 1) return NAN;
    bf_ctx b;
    b.kind = kind;
    b.prm = prm;
    b.x = x;
    b.y = y;
    b.lx = lx;
    b.ly = ly;
    b.w = orc_window(kind, prm[P_WR], lx, ly);
    if (b.w < 0) return NAN;
    double* W = NULL;
    if (kind == ORC_WDTW) {
        W = (double*)malloc(sizeof(double) * (size_t)imax(lx, ly));
        orc_wdtw_weights(prm[P_G], imax(lx, ly), W);
    }
    b.W = W;
    double acc = 0.0;
    int64_t m = imin(lx, ly);
    for (int64_t k = 1; k <= m; ++k) acc = bf_step(&b, 0, k, k, acc);
    for (int64_t i = m + 1; i <= lx; ++i) acc = bf_step(&b, 1, i, m, acc);
    for (int64_t j = m + 1; j <= ly; ++j) acc = bf_step(&b, 2, m, j, acc);
    free(W);
    return acc;
}

/* ------------------------------------------------------------------------- */
/* NN search, Alg. 1: candidates in index order, replace on strictly smaller
 * distance, so the lowest index wins ties.  mode 0 evaluates every candidate
 * with the full DP; mode 1 with EAPruned using the current best as cut-off.
 * Out: index (-1 when no candidate has a finite distance) and distance.
 * cells_total (nullable) sums EAPruned's evaluated cells.  Queries run in
 * parallel over nthreads OpenMP threads (<= 0: the OpenMP default); the
 * count applies to this call only. */
/* ------------------------------------------------------------------------- */
/* Lower bounds for DTW and CDTW (Section 2.1: LB_Kim and LB_Keogh, used by
 * the lower-bounded NN search, Alg. 2; Section 5.2 runs LB_Keogh and a
 * second LB_Keogh with the arguments reversed, "lb-keogh2").  Both distances
 * use the squared difference, and every warping path starts at (1,1), ends at
 * (L_Q, L_C) and, under a window w, visits each column j of C only at rows i
 * with |i - j| <= w. */

/* Envelope of x (length L) under window w, at positions j = 1..n:
 * up[j-1] = max and lo[j-1] = min of x_i over i in [j-w, j+w] and [1, L];
 * an empty range (j > L + w) gives up = -inf, lo = +inf. */
void orc_envelope(const double* x, int64_t L, int64_t w, int64_t n, double* up, double* lo)
{
    for (int64_t j = 1; j <= n; ++j) {
        double u = -INF, l = INF;
        for (int64_t i = imax(1, j - w); i <= imin(L, j + w); ++i) {
            if (x[i - 1] > u) u = x[i - 1];
            if (x[i - 1] < l) l = x[i - 1];
        }
        up[j - 1] = u;
        lo[j - 1] = l;
    }
}

/* Squared distance of v to the range [lo, up] (0 inside it). */
static double dist_to_range(double v, double lo, double up)
{
    if (v > up) return (v - up) * (v - up);
    if (v < lo) return (lo - v) * (lo - v);
    return 0.0;
}

/* LB_Keogh(Q, C) under window w: the sum over the columns j = 1..L_C of C,
 * left to right, of the squared distance of c_j to the envelope of Q at j.
 * A path pays at least that much in column j.  +inf when the window admits
 * no path (w < |L_Q - L_C|). */
double orc_lb_keogh(const double* q, int64_t lq, const double* c, int64_t lc, int64_t w)
{
    if (w < (lq > lc ? lq - lc : lc - lq)) return INF;
    double* up = (double*)malloc(sizeof(double) * (size_t)lc);
    double* lo = (double*)malloc(sizeof(double) * (size_t)lc);
    orc_envelope(q, lq, w, lc, up, lo);
    double s = 0.0;
    for (int64_t j = 0; j < lc; ++j) s = s + dist_to_range(c[j], lo[j], up[j]);
    free(up);
    free(lo);
    return s;
}

/* LB_Kim in its first-and-last-points form: the costs of the cells (1,1)
 * and (L_Q, L_C), which every path contains (one cell when both series have
 * length 1). */
double orc_lb_kim(const double* q, int64_t lq, const double* c, int64_t lc)
{
    double a = q[0] - c[0];
    double s = a * a;
    if (lq > 1 || lc > 1) {
        double b = q[lq - 1] - c[lc - 1];
        s = s + b * b;
    }
    return s;
}

void orc_nn1(int kind, const double* prm, const double* q, const int64_t* q_off, int64_t nq, const double* r,
             const int64_t* r_off, int64_t nr, int mode, int64_t* out_idx, double* out_dist, int nthreads,
             int64_t* cells_total)
{
    int64_t cells_sum = 0;
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : cells_sum) num_threads(nt)
#endif
    for (int64_t a = 0; a < nq; ++a) {
        const int dims = dims_of(prm);
        const double* qa = q + q_off[a] * dims;
        int64_t la = q_off[a + 1] - q_off[a];
        double best = INF;
        int64_t bi = -1;
        for (int64_t b = 0; b < nr; ++b) {
            const double* rb = r + r_off[b] * dims;
            int64_t lb = r_off[b + 1] - r_off[b];
            double d;
            if (mode == 1) {
                int64_t c = 0;
                d = orc_eap(kind, qa, la, rb, lb, prm, best, &c, NULL, NULL);
                cells_sum += c;
            } else if (mode == 2) {
                int64_t c = 0;
                d = orc_eabase(kind, qa, la, rb, lb, prm, best, &c);
                cells_sum += c;
            } else if (mode == 3) {
                /* Alg. 2: a candidate is computed only while its lower bounds
                 * stay below the best-so-far (DTW and CDTW): LB_Kim, then
                 * LB_Keogh(Q, C), then LB_Keogh(C, Q), then EAPruned.  A bound
                 * is compared after scaling by 1 - 1e-11, which covers its own
                 * rounding and the distance's (sums of at most 2 x 2048 terms). */
                d = INF;
                int go = 1;
                if ((kind == ORC_DTW || kind == ORC_CDTW) && dims == 1) {
                    int64_t w = orc_window(kind, prm[P_WR], la, lb);
                    go = orc_lb_kim(qa, la, rb, lb) * (1.0 - 1e-11) < best &&
                         orc_lb_keogh(qa, la, rb, lb, w) * (1.0 - 1e-11) < best &&
                         orc_lb_keogh(rb, lb, qa, la, w) * (1.0 - 1e-11) < best;
                }
                if (go) {
                    int64_t c = 0;
                    d = orc_eap(kind, qa, la, rb, lb, prm, best, &c, NULL, NULL);
                    cells_sum += c;
                }
            } else {
                d = orc_dp(kind, qa, la, rb, lb, prm, NULL);
            }
            if (d < best) {
                best = d;
                bi = b;
            }
        }
        out_idx[a] = bi;
        out_dist[a] = best;
    }
    if (cells_total) *cells_total = cells_sum;
}

/* All pairs i < j, condensed: out[n*i - i*(i+1)/2 + (j-i-1)].  mode 1 is the
 * full DP; mode 0 is prune-only EAPruned with the path upper bound (one ulp
 * above it) as cut-off, which never abandons. */
void orc_pairwise(int kind, const double* prm, const double* s, const int64_t* s_off, int64_t n, int mode,
                  double* out, int nthreads)
{
#ifdef _OPENMP
    const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            const double* a = s + s_off[i] * dims_of(prm);
            const double* b = s + s_off[j] * dims_of(prm);
            int64_t la = s_off[i + 1] - s_off[i], lb = s_off[j + 1] - s_off[j];
            double d;
            if (mode == 1) d = orc_dp(kind, a, la, b, lb, prm, NULL);
            else {
                double ub = orc_ub(kind, a, la, b, lb, prm);
                d = (ub == INF) ? INF : orc_eap(kind, a, la, b, lb, prm, nextafter(ub, INF), NULL, NULL, NULL);
            }
            out[n * i - i * (i + 1) / 2 + (j - i - 1)] = d;
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
