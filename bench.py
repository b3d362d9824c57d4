"""Benchmark: 1-NN search with the six elastic distances on one MI355X.

One step is the whole hot path over one batch.  The default workload (4) is
batched 1-NN search with uneven lengths: for each of DTW, CDTW, WDTW, ERP, MSM
and TWE, the 1-NN of 1,000 queries among 10,000 candidates whose lengths are
uniform in 64..2048 (five time-warped sine classes, z-normalised; synthetic,
seeded stand-ins for the paper's NN classification over UCR-shaped data),
each search an FP32 screening sweep with an FP64 recheck of its near-ties
(margin 1e-4 relative plus a certified rounding bound), the six searches
captured in one HIP graph: a step is one graph launch.  Inputs are resident
in HBM before the timed region.  --workload 2 runs 500 x 500 series of length
512 (six pipelined searches per step), 3 all-pairs matrices, 5 a request
server, 6 sub-sequence search.

Reported (one JSON line on stdout):
  value        effective GCUPS: DP cells of the plain full programme (cells in
               the window for CDTW, none for pairs the window forbids) of all
               six searches, divided by the step time
  queries_per_s  1-NN searches per second (queries x six distances per step)
  plain_gpu_dp   the same searches with the plain full FP64 DP on the GPU
  roofline     the dominant sweep kernel: executed cells per launch over its
               mean launch time (HIP events on its stream), against the VALU
               cell-update peak for that distance and precision
  cpu_baseline the CPU oracle on bounded samples (EAPruned NN on all host
               threads, its full DP, one thread), NN answers compared
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCUPS (cell updates/s) & queries/s for 1-NN search vs plain GPU DP; p50/p99 latency"

# VALU roofline of gfx950: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12
# FP64 lane-ops/s (the published 78.6 TFLOP/s FP64 vector rate, FMA = 2 flops);
# FP32 issues up to two lane-ops per lane and cycle, 78.6e12/s (the published
# 157.3 TFLOP/s FP32 vector rate).  Minimal lane-ops per DP cell of each
# distance; FP32 has three-operand min3/max3/med3, FP64 does not.
LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
LANE_OPS_PER_S_F32 = 2 * LANE_OPS_PER_S
OPS_PER_CELL = {"dtw": 5, "cdtw": 5, "wdtw": 6, "erp": 6, "msm": 16, "twe": 8}
# FP32 sweeps fuse the squared costs' (weighted) square with the add (one
# lane-op for the FMA): DTW sub, min3, fma; CDTW (band) sub, min3, the window's
# add, fma; WDTW sub, weight mul, min3, fma
OPS_PER_CELL_F32 = {"dtw": 3, "cdtw": 4, "wdtw": 4, "erp": 5, "msm": 9, "twe": 7}
# FP32 WDTW with exact differences: the float64 subtraction, at half the FP32
# lane-op rate, counts as two FP32 operations, plus its conversion to FP32
OPS_PER_CELL_F32_XD = {"wdtw": 6}
HBM_PEAK_GBS = 8000.0
ROOFLINE_CONVENTION = ("achieved = executed cells of the dominant kernel's launch / its launch time; peak = VALU "
                       "lane-op rate / minimal lane-ops per cell of its distance and precision, with the lane-op "
                       "rate 39.3e12/s for FP64 (78.6 TFLOP/s / 2: min-plus cells have no FMA) and 78.6e12/s for "
                       "FP32 (157.3 TFLOP/s / 2); an FP32 sweep with exact differences counts its float64 "
                       "subtraction as two FP32 operations")


def say(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def band_cells(li, co, w):
    """Cells (i, j), 1 <= i <= li, 1 <= j <= co, with |i - j| <= w, for arrays
    li >= co with w >= li - co (closed form of the row-by-row count)."""
    li, co, w = (np.asarray(x, dtype=np.int64) for x in (li, co, w))
    m = np.clip(co - w, 0, li)
    s_up = m * (m + 1) // 2 + m * w + (li - m) * co                     # sum of min(i + w, co)
    n1 = np.minimum(li, w + 1)
    t = np.maximum(li - w, 1)
    s_lo = n1 + np.where(li >= w + 2, t * (t + 1) // 2 - 1, 0)          # sum of max(i - w, 1)
    return s_up - s_lo + li


def dense_cells(kind, p, q_off, r_off):
    """Cells of the plain full DP over all (query, candidate) pairs; for a
    windowed distance the cells inside the window (0 for infeasible pairs)."""
    lq = np.diff(q_off).astype(np.int64)
    lr = np.diff(r_off).astype(np.int64)
    ratio = p.get("window_ratio", math.inf)
    if kind not in ("cdtw", "erp") or ratio >= 1:
        return int(lq.sum() * lr.sum())
    uq, cq = np.unique(lq, return_counts=True)
    ur, cr = np.unique(lr, return_counts=True)
    A, B = np.meshgrid(uq, ur, indexing="ij")
    li, co = np.maximum(A, B), np.minimum(A, B)
    w = np.floor(ratio * li.astype(np.float64)).astype(np.int64)
    feas = w >= li - co
    cells = np.where(feas, band_cells(li, co, np.where(feas, w, li)), 0)
    return int((cells * np.outer(cq, cr)).sum())


def kernel_label(rec):
    """Name of a sweep launch: kernel, width (strip columns or band diagonals),
    lanes per pair x columns per lane (xd: exact differences)."""
    g = rec["group"]
    c = rec["size"] // g if rec["kernel"] == "rows" else rec["size"] // (2 * g)
    return f"{rec['kernel']}{rec['size']} {g}x{c}" + (" xd" if rec.get("exact_diff") else "")


def ops_per_cell(kind, fp32, xd=False):
    """Minimal lane-ops per cell of a sweep, in FP32 operations for FP32 sweeps."""
    if fp32 and xd:
        return OPS_PER_CELL_F32_XD[kind]
    return (OPS_PER_CELL_F32 if fp32 else OPS_PER_CELL)[kind]


def hbm_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/*_hbm.md), valid only while the kernel sources are the
    ones it was measured on; (None, reason) otherwise."""
    pdir = os.path.join(ROOT, "profiles")
    for fn in sorted(os.listdir(pdir)) if os.path.isdir(pdir) else []:
        if not fn.endswith("_hbm.md"):
            continue
        lines = open(os.path.join(pdir, fn)).read().splitlines()
        hashes = [ln.split(":", 1)[1].strip() for ln in lines if ln.startswith("source_hash:")]
        if not hashes or hashes[0] != _source_hash():
            continue
        for ln in lines:
            cells = [c.strip() for c in ln.strip().strip("|").split("|")]
            if len(cells) >= 2 and cells[0] == kernel:
                return float(cells[1]), f"HBM bytes per launch, profiles/{fn} (FETCH_SIZE + WRITE_SIZE, " \
                                        "copy-calibrated)"
    return None, "no counter summary for this kernel and these sources in profiles/"


def swept_kind(kind, p):
    """The distance the library sweeps (CDTW without a window is DTW)."""
    if kind == "cdtw" and p.get("window_ratio", math.inf) >= 1:
        return "dtw"
    return kind


def cpu_baseline(wl, kinds, gpu_idx, gpu_dist, eap_q, dp_q, dp_r=None, one_q=1, one_r=None, derivative=False):
    """The CPU oracle timed on the host, on bounded samples of the workload:
      value          EAPruned NN (Alg. 1 + Alg. 5) of the first eap_q queries
                     against every candidate, all host threads, as effective
                     GCUPS (dense cells of the sample / seconds); its NN
                     answers compared with the GPU's (nn_identical_to_gpu)
      full_dp_gcups  the oracle's full DP of the first dp_q queries against the
                     first dp_r candidates (all of them when None), all threads
      one_core_gcups EAPruned NN of the first one_q queries against the first
                     one_r candidates, one thread
    derivative: on the oracle's derivative series of the same inputs (the
    transform itself untimed)."""
    from oracle import oracle as orc
    if derivative:
        wl = dict(wl, queries=orc.derivative(wl["queries"], wl["query_off"]),
                  refs=orc.derivative(wl["refs"], wl["ref_off"]))
    nr = len(wl["ref_off"]) - 1
    dp_r = nr if dp_r is None else min(dp_r, nr)
    one_r = nr if one_r is None else min(one_r, nr)

    def head(off, vals, n):
        o = off[: n + 1]
        return vals[: o[-1]], o

    qv, qo = head(wl["query_off"], wl["queries"], eap_q)
    cells = 0
    secs = 0.0
    match = True
    seq_cells = {}   # cells the oracle's sequential EAPruned (Alg. 1 order) evaluates per distance
    for kind in kinds:
        p = wl["params"][kind]
        t0 = time.perf_counter()
        idx, dist, ocells = orc.nn1(p, qv, qo, wl["refs"], wl["ref_off"], "eap")
        secs += time.perf_counter() - t0
        seq_cells[kind] = int(ocells)
        cells += dense_cells(kind, p, qo, wl["ref_off"])
        match &= bool(np.array_equal(idx, gpu_idx[kind][:eap_q]) and np.array_equal(dist, gpu_dist[kind][:eap_q]))
    dv, do = head(wl["query_off"], wl["queries"], dp_q)
    rv, ro = head(wl["ref_off"], wl["refs"], dp_r)
    v1, o1 = head(wl["query_off"], wl["queries"], one_q)
    r1, ro1 = head(wl["ref_off"], wl["refs"], one_r)
    sd = dcells = 0.0
    c1 = s1 = 0.0
    for kind in kinds:
        p = wl["params"][kind]
        t0 = time.perf_counter()
        orc.nn1(p, dv, do, rv, ro, "dp")
        sd += time.perf_counter() - t0
        dcells += dense_cells(kind, p, do, ro)
        t0 = time.perf_counter()
        orc.nn1(p, v1, o1, r1, ro1, "eap", nthreads=1)
        s1 += time.perf_counter() - t0
        c1 += dense_cells(kind, p, o1, ro1)
    model = ""
    try:
        model = next(ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return dict(value=cells / secs / 1e9, unit="GCUPS", cores=orc.num_threads(), kind="oracle",
                host=dict(cpu_model=model, logical_cpus=os.cpu_count()),
                sample=f"EAPruned NN of the first {eap_q} queries against all {nr} candidates, {len(kinds)} "
                       f"distances, {secs:.1f} s on {orc.num_threads()} threads",
                seconds=secs,
                nn_identical_to_gpu=match,
                full_dp_gcups=dcells / sd / 1e9,
                full_dp_sample=f"full DP of the first {dp_q} queries against the first {dp_r} candidates, "
                               f"{len(kinds)} distances, {sd:.1f} s",
                sequential_eapruned_cells=seq_cells,
                one_core_gcups=c1 / s1 / 1e9,
                one_core_sample=f"EAPruned NN of the first {one_q} queries against the first {one_r} "
                                f"candidates, {len(kinds)} distances, one thread, {s1:.1f} s")


def run_pairwise(args, torch, eap, synth):
    """Workload 3: all pairs of 2,000 random walks of length 1024 (1,999,000
    pairs), DTW, CDTW (w = 5%) and MSM, FP64: prune-only EAPruned (each pair's
    cut-off one ulp above its path bound, so every value is exact) against the
    plain full DP."""
    dev = torch.device("cuda:0")
    wl = synth.make_workload(3, n_ref=args.refs or None)
    so = wl["ref_off"]
    n = len(so) - 1
    s = torch.from_numpy(wl["refs"]).to(dev)
    kinds = [k for k in args.kinds.split(",") if k in wl["params"]] or list(wl["params"])
    per = {}
    tot_cells = 0
    tot_ms = 0.0
    for k in kinds:
        p = wl["params"][k]
        ws = eap.workspace(eap.pairwise_workspace_bytes(so, p), dev)
        out = torch.empty(n * (n - 1) // 2, dtype=torch.float64, device=dev)
        res = {}
        for mode in ("prune", "full"):
            eap.pairwise(s, so, p, mode, ws=ws, out=out)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            eap.reset_counters(ws)
            eap.profile_take()
            eap.profile_enable(True)
            a.record()
            for _ in range(args.steps):
                eap.pairwise(s, so, p, mode, ws=ws, out=out)
            b.record()
            torch.cuda.synchronize()
            eap.profile_enable(False)
            recs = [x for x in eap.profile_take() if x["stage"] == 2]
            ms = a.elapsed_time(b) / args.steps
            c = eap.read_counters(ws)
            res[mode] = (ms, c["cells"] / args.steps, out.clone(), recs)
        # dense cells: all pairs (band cells for CDTW)
        lens = np.diff(so)
        if k == "cdtw":   # ordered pairs minus the diagonal, halved
            diag = sum(dense_cells(k, p, so[i:i + 2] - so[i], so[i:i + 2] - so[i]) for i in range(n))
            cells = (dense_cells(k, p, so, so) - diag) // 2
        else:
            cells = int((lens.sum() ** 2 - (lens ** 2).sum()) // 2)
        same = bool(torch.equal(res["prune"][2], res["full"][2]))
        recs = res["prune"][3]
        sweep_ms = sum(x["ms"] for x in recs) / max(len(recs), 1)
        per[k] = dict(prune_ms=res["prune"][0], full_ms=res["full"][0], speedup=res["full"][0] / res["prune"][0],
                      dense_cells=cells, prune_executed_fraction=res["prune"][1] / cells,
                      prune_gcups_effective=cells / (res["prune"][0] * 1e-3) / 1e9,
                      full_gcups=cells / (res["full"][0] * 1e-3) / 1e9, identical=same,
                      prune_sweep_ms=sweep_ms, prune_executed_cells=res["prune"][1],
                      prune_kernel=kernel_label(recs[0]) if recs else None)
        tot_cells += cells
        tot_ms += res["prune"][0]
        if args.cpu_queries:
            # the oracle's prune-only matrix of the first 64 series, compared element by element
            from oracle import oracle as orc
            m = min(64, n)
            sv = wl["refs"][: so[m]]
            t = time.perf_counter()
            want = orc.pairwise(p, sv, so[: m + 1], "prune")
            secs = time.perf_counter() - t
            got = eap.pairwise(s[: so[m]], so[: m + 1], p, "prune")
            torch.cuda.synchronize()
            mc = int(np.diff(so[: m + 1]).sum() ** 2 - (np.diff(so[: m + 1]) ** 2).sum()) // 2 if k != "cdtw" else None
            per[k]["cpu"] = dict(seconds=secs, pairs=m * (m - 1) // 2, dense_cells=mc,
                                 identical_to_gpu=bool(np.array_equal(got.cpu().numpy(), want)))
        del ws, out
    # roofline: the dominant prune-only sweep, executed cells per launch over its launch time
    dom = max(kinds, key=lambda k: per[k]["prune_sweep_ms"])
    d = per[dom]
    sk = swept_kind(dom, wl["params"][dom])
    peak = LANE_OPS_PER_S / OPS_PER_CELL[sk] / 1e9
    ach = d["prune_executed_cells"] / (d["prune_sweep_ms"] * 1e-3) / 1e9
    roofline = dict(bound="alu", achieved=ach, peak=peak, unit="GCUPS", frac=ach / peak, traffic=None,
                    kernel=f"{d['prune_kernel']} sweep, {sk.upper()} main stage, fp64",
                    ops_per_cell=OPS_PER_CELL[sk], launch_ms=d["prune_sweep_ms"], convention=ROOFLINE_CONVENTION)
    cpu = None
    if args.cpu_queries:
        from oracle import oracle as orc
        secs = sum(per[k]["cpu"]["seconds"] for k in kinds)
        cells_cpu = sum(per[k]["cpu"]["dense_cells"] or 0 for k in kinds if k != "cdtw")
        cpu = dict(value=cells_cpu / sum(per[k]["cpu"]["seconds"] for k in kinds if k != "cdtw") / 1e9,
                   unit="GCUPS", cores=orc.num_threads(), kind="oracle",
                   sample="prune-only matrix of the first 64 series (2,016 pairs) per distance; GCUPS over DTW "
                          "and MSM", seconds=secs,
                   identical_to_gpu=all(per[k]["cpu"]["identical_to_gpu"] for k in kinds))
    print(json.dumps(dict(
        metric=METRIC, value=tot_cells / (tot_ms * 1e-3) / 1e9, unit="GCUPS", n_gpus=1, steps=args.steps,
        warmup=1, ms_per_step=tot_ms, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
        data="synthetic",
        config=dict(workload=f"all pairs of {n} random walks, length 1024, prune-only EAPruned vs plain DP: "
                             + ", ".join(kinds), series=n, pairs=n * (n - 1) // 2, distances=kinds),
        roofline=roofline, cpu_baseline=cpu, per_distance=per)), flush=True)


ap_default_kinds = "dtw,cdtw,wdtw,erp,msm,twe"


ABLATION = [
    # name, precision, flags, lower bounds, distances it applies to (None: all)
    ("base_plain_dp_fp64", 0, "plain", "none", None),
    ("pruned_fp64", 0, "prune_only", "none", None),
    ("eabase_fp64", 0, "no_prune", "none", None),
    ("eapruned_fp64_no_seed", 0, "no_seed", "none", None),
    ("eapruned_fp64", 0, "", "none", None),
    ("eabase_fp64_lb_keogh2", 0, "no_prune", "keogh2", ("dtw", "cdtw")),
    ("eapruned_fp64_lb_keogh", 0, "", "keogh", ("dtw", "cdtw")),
    ("eapruned_fp64_lb_keogh2", 0, "", "keogh2", ("dtw", "cdtw")),
    ("eapruned_fp32_screen_default", 1, "", "default", None),
]


def ablation(torch, eap, stream, q, q_off, r, r_off, params, ref, dense, kinds):
    """The search with its parts switched off one at a time, on the GPU
    (Section 5.1's Base, Prune, EABase and EAPruned; Section 5.2's lower
    bounds lb-none, lb-keogh, lb-keogh2 for DTW and CDTW): every variant is
    one nn1 call per distance, timed with HIP events on the search's stream
    after an untimed run, its results checked against the default path's
    (`ref`, which the CPU-baseline leg checks against the oracle).
      base_plain_dp_fp64         Base: the full DP, no cut-off
      pruned_fp64                Prune: each pair under its own path bound (nothing
                                 abandoned), no shared best-so-far; at the GPU's strip
                                 granularity PrunedDTW's pruning is this too
      eabase_fp64                EABase: best-so-far cut-off, early abandoning, no
                                 pruning (every strip row is computed)
      eapruned_fp64_no_seed      EAPruned without the seed sweep
      eapruned_fp64              EAPruned, no lower bound (at strip granularity
                                 PrunedDTW+EA coincides with it)
      eabase_fp64_lb_keogh2      EABase behind LB_Keogh both ways
      eapruned_fp64_lb_keogh     EAPruned behind LB_Keogh (with LB_Kim's corners)
      eapruned_fp64_lb_keogh2    and the reversed LB_Keogh
      eapruned_fp32_screen_default  the default search (FP32 screen + FP64 recheck,
                                 LB_Keogh for CDTW)"""
    flag = {"": 0, "plain": eap.FLAG_PLAIN, "prune_only": eap.FLAG_PRUNE_ONLY, "no_prune": eap.FLAG_NO_PRUNE,
            "no_seed": eap.FLAG_NO_SEED}
    nq = len(q_off) - 1
    ws = {k: eap.workspace(eap.nn1_workspace_bytes(q_off, r_off, params[k], precision=1, lb="keogh2"), q.device)
          for k in kinds}
    out = {}
    for name, prec, fl, lb, only in ABLATION:
        per, total, same = {}, 0.0, True
        for k in kinds:
            if only is not None and params[k]["kind"] not in only:
                continue
            o = (torch.empty(nq, dtype=torch.int64, device=q.device),
                 torch.empty(nq, dtype=torch.float64, device=q.device), None)
            for rep in range(2):
                if rep:
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                eap.nn1(q, q_off, r, r_off, params[k], ws=ws[k], out=o, precision=prec, flags=flag[fl], lb=lb,
                        stream=stream)
                if rep:
                    b.record(stream)
                torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            total += ms
            per[k] = dict(ms=ms, gcups=dense[k] / (ms * 1e-3) / 1e9)
            same &= bool(np.array_equal(o[0].cpu().numpy(), ref[k][0]) and np.array_equal(o[1].cpu().numpy(), ref[k][1]))
        if per:
            out[name] = dict(ms=total, per_distance=per, nn_identical=same)
    del ws
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kinds", default=ap_default_kinds)
    ap.add_argument("--cpu-queries", type=int, default=None,
                    help="queries in the CPU-oracle EAPruned sample, each against every candidate (0: skip; "
                         "default 16 for workload 4, 500 for workload 2)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-DP comparison")
    ap.add_argument("--ablation", action="store_true",
                    help="workloads 2, 4 and 6: also time the search with its parts switched off one at a time "
                         "(Base, Prune, EABase, EAPruned, lower bounds lb-none / lb-keogh / lb-keogh2), after the "
                         "timed region; workload 4 on its first --ablation-queries queries")
    ap.add_argument("--ablation-queries", type=int, default=100)
    ap.add_argument("--precision", type=int, default=None,
                    help="0: FP64 sweep; 1: FP32 screen + FP64 recheck (default 1, and 0 for workload 6, where "
                         "LB_Keogh leaves so few pairs that the screen's extra stages cost more than they save)")
    ap.add_argument("--no-tune", action="store_true", help="skip the row-sweep autotuner (default shapes)")
    ap.add_argument("--shapes", default="",
                    help="workload 4: row-sweep shapes pinned instead of tuned, e.g. wdtw=4x16,msm=8x16 (the other "
                         "distances keep their defaults); lets a profiled run launch exactly the shapes of a timed "
                         "one without the tuner's own launches")
    ap.add_argument("--schedule", default="pipelined", choices=("pipelined", "serial", "concurrent"),
                    help="workload 2: how the six searches of a step share the GPU.  pipelined: three "
                         "streams (round-robin), main sweeps one at a time (chained by events), the "
                         "latency-bound stages overlapping them; serial: one after the other on one stream; "
                         "concurrent: six streams, no ordering")
    ap.add_argument("--batch-schedule", default="serial", choices=("serial", "concurrent"),
                    help="workload 4: the six searches of the captured step one after the other on one stream, "
                         "or each on its own stream (forked and joined inside the graph)")
    ap.add_argument("--derivative", action="store_true",
                    help="workload 2 with the derivative variants: the series' first derivatives computed "
                         "inside every step, then DDTW, DCDTW and DWDTW (default --kinds dtw,cdtw,wdtw)")
    ap.add_argument("--compare-precision", action="store_true",
                    help="also time the other precision's step (outside the timed region)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run 3 plain device copies of this many MiB (HBM counter calibration) and exit")
    ap.add_argument("--workload", type=int, default=4, choices=(2, 3, 4, 5, 6),
                    help="4 (default): 1-NN of 1,000 queries among 10,000 candidates of uneven lengths "
                         "(64..2048), six distances, FP32 screen + FP64 recheck, one graph launch per step; "
                         "2: 500 x 500, length 512; 3: all-pairs matrix; 5: served requests; 6: sub-sequence "
                         "search")
    ap.add_argument("--refs", type=int, default=0, help="workloads 3-6: series / candidate / window count (0: the full workload)")
    ap.add_argument("--queries", type=int, default=0, help="workloads 4-6: query count (0: the full workload)")
    args = ap.parse_args()
    if args.cpu_queries is None and args.workload != 5:   # workload 5: 500 CDTW / 20 MSM served queries
        args.cpu_queries = 16 if args.workload == 4 else 500
    if args.precision is None:
        args.precision = 0 if args.workload == 6 else 1
    if args.copy_mib > 0:
        import torch
        n = args.copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes_read=n * 8, copy_bytes_written=n * 8, copies=3)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is described "
              "but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2102_05221_amd as eap
    from paper_2102_05221_amd import synth

    if args.workload == 3:
        return run_pairwise(args, torch, eap, synth)
    if args.workload == 4:
        return run_batched(args, torch, eap, synth)
    if args.workload == 5:
        return run_served(args, torch, eap, synth)
    if args.workload == 6:
        return run_subseq(args, torch, eap, synth)

    dev = torch.device("cuda:0")
    if args.derivative and args.kinds == ap_default_kinds:
        args.kinds = "dtw,cdtw,wdtw"
    kinds = [k for k in args.kinds.split(",") if k]
    wl = synth.make_workload(2)
    q = torch.from_numpy(wl["queries"]).to(dev)
    r = torch.from_numpy(wl["refs"]).to(dev)
    labels = torch.from_numpy(wl["ref_labels"]).to(dev)
    derive = None
    if args.derivative:
        # the searches read the derivative series, recomputed at the start of
        # every step from the raw series (part of the timed work)
        q_raw, r_raw = q, r
        q, r = torch.empty_like(q_raw), torch.empty_like(r_raw)
        dws = eap.workspace(max(eap.lib().eap_derivative_workspace(len(wl["query_off"]) - 1),
                                eap.lib().eap_derivative_workspace(len(wl["ref_off"]) - 1)), dev)

        def derive():
            eap.derivative(q_raw, wl["query_off"], ws=dws, out=q)
            eap.derivative(r_raw, wl["ref_off"], ws=dws, out=r)

        derive()
    nq, nr = len(wl["query_off"]) - 1, len(wl["ref_off"]) - 1
    ws = {k: eap.workspace(eap.nn1_workspace_bytes(wl["query_off"], wl["ref_off"], wl["params"][k], precision=1), dev)
          for k in kinds}
    outs = {k: (torch.empty(nq, dtype=torch.int64, device=dev), torch.empty(nq, dtype=torch.float64, device=dev),
                torch.empty(nq, dtype=torch.int32, device=dev)) for k in kinds}
    dense = {k: dense_cells(k, wl["params"][k], wl["query_off"], wl["ref_off"]) for k in kinds}
    stream = torch.cuda.current_stream(dev)

    kstream = {k: torch.cuda.Stream(dev) for k in kinds}
    # pipelined: three streams, the searches round-robin over them.  HIP maps
    # streams onto a few hardware queues (4 by default, one taken by torch's
    # stream), and work on a queue runs in order: with six streams two
    # consecutive searches could share one, and the second's bound and seed
    # stages would wait behind the first's main sweep and recheck.  With three,
    # a queue's next search follows one whose main sweep ended two sweeps ago.
    pstream = [torch.cuda.Stream(dev) for _ in range(3)]
    main_done = {k: torch.cuda.Event() for k in kinds}

    def step(precision=args.precision, schedule=args.schedule):
        """One pass of the six searches.  The step starts and ends on `stream`
        (the other streams fork from it and join it again)."""
        if derive:
            derive()
        if schedule == "serial":
            for k in kinds:
                eap.nn1(q, wl["query_off"], r, wl["ref_off"], wl["params"][k], ref_labels=labels, ws=ws[k],
                        out=outs[k], precision=precision)
            return
        used = []
        for i, k in enumerate(kinds):
            chain = {}
            if schedule == "pipelined":
                ks = pstream[i % len(pstream)]
                chain = dict(main_wait=main_done[kinds[i - 1]] if i > 0 else None, main_done=main_done[k])
            else:
                ks = kstream[k]
            if ks not in used:
                ks.wait_stream(stream)
                used.append(ks)
            eap.nn1(q, wl["query_off"], r, wl["ref_off"], wl["params"][k], ref_labels=labels, ws=ws[k], out=outs[k],
                    precision=precision, stream=ks, **chain)
        for ks in used:
            stream.wait_stream(ks)

    # autotune the row sweep's shape per distance on this workload (setup, untimed)
    tuning = {}
    if not args.no_tune:
        for k in kinds:
            recs = eap.tune_nn1(q, wl["query_off"], r, wl["ref_off"], wl["params"][k], precision=args.precision,
                                ws=ws[k])
            if recs:
                tuning[k] = dict(chosen=next(f"{x['g']}x{x['c']}" for x in recs if x["chosen"]),
                                 ms={f"{x['g']}x{x['c']}": round(x["ms"], 3) for x in recs})

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for k in kinds:
        eap.reset_counters(ws[k])
    eap.profile_take()
    eap.profile_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        e_a = torch.cuda.Event(enable_timing=True)
        e_b = torch.cuda.Event(enable_timing=True)
        e_a.record(stream)
        step()
        e_b.record(stream)
        step_ms.append((e_a, e_b))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    eap.profile_enable(False)
    prof = eap.profile_take()
    step_ms = [a.elapsed_time(b) for a, b in step_ms]
    ms_per_step = wall * 1e3 / args.steps
    counters = {k: eap.read_counters(ws[k]) for k in kinds}

    # per-distance times of the main sweep and the dominant kernel
    per = {}
    for k in kinds:
        sk = swept_kind(k, wl["params"][k])
        main = [x for x in prof if x["kind"] == sk and x["stage"] == 2]
        rechk = [x for x in prof if x["kind"] == sk and x["stage"] in (4, 5)]
        per[k] = dict(
            sweep_ms_per_step=sum(x["ms"] for x in prof if x["kind"] == sk) / args.steps,
            main_sweep_ms=(sum(x["ms"] for x in main) / len(main)) if main else None,
            main_kernel=(kernel_label(main[0]) if main else None),
            main_fp32=bool(main[0]["fp32"]) if main else False,
            recheck_ms_per_step=sum(x["ms"] for x in rechk) / args.steps,
            executed_cells_per_step=counters[k]["cells"] / args.steps,
            main_cells_per_launch=counters[k]["stage_cells"][2] / args.steps,
            dense_cells=dense[k],
            executed_fraction=counters[k]["cells"] / args.steps / dense[k],
            overflows_per_step=counters[k]["overflows"] / args.steps,
            fp64_rechecks_per_step=counters[k]["rechecks"] / args.steps,
            lb_pruned_per_step=counters[k]["lb_pruned"] / args.steps,
        )
    gpu_idx = {k: outs[k][0].cpu().numpy() for k in kinds}
    gpu_dist = {k: outs[k][1].cpu().numpy() for k in kinds}
    gpu_lab = {k: outs[k][2].cpu().numpy() for k in kinds}
    qlab = wl["query_labels"]
    for k in kinds:
        per[k]["nn_accuracy"] = float(np.mean(gpu_lab[k] == qlab))

    # dominant kernel: the main sweep with the largest time per step
    dom_kind = max(kinds, key=lambda k: per[k]["main_sweep_ms"] or 0.0)
    d = per[dom_kind]
    achieved = d["main_cells_per_launch"] / (d["main_sweep_ms"] * 1e-3) / 1e9
    ops = (OPS_PER_CELL_F32 if d["main_fp32"] else OPS_PER_CELL)[dom_kind]
    peak = (LANE_OPS_PER_S_F32 if d["main_fp32"] else LANE_OPS_PER_S) / ops / 1e9
    roofline = dict(bound="alu", achieved=achieved, peak=peak, unit="GCUPS", frac=achieved / peak, traffic=None,
                    kernel=f"{d['main_kernel']} sweep, {dom_kind.upper()} main stage, "
                           f"{'fp32' if d['main_fp32'] else 'fp64'}",
                    ops_per_cell=ops, launch_ms=d["main_sweep_ms"],
                    cells_per_launch=d["main_cells_per_launch"])
    # HBM bytes per launch from the committed rocprofv3 counter summary, valid
    # only while the kernel sources are the ones it was measured on
    roofline["traffic"], roofline["traffic_note"] = hbm_traffic(roofline["kernel"])

    # plain full DP on the GPU, same searches (outside the timed region)
    plain = None
    if not args.no_plain:
        plain = {}
        total_plain_ms = 0.0
        same = True
        for k in kinds:
            pouts = (torch.empty(nq, dtype=torch.int64, device=dev), torch.empty(nq, dtype=torch.float64, device=dev),
                     None)
            eap.nn1(q, wl["query_off"], r, wl["ref_off"], wl["params"][k], ws=ws[k], out=pouts,
                    flags=eap.FLAG_PLAIN)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            eap.nn1(q, wl["query_off"], r, wl["ref_off"], wl["params"][k], ws=ws[k], out=pouts,
                    flags=eap.FLAG_PLAIN)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b)
            total_plain_ms += ms
            same &= bool(np.array_equal(pouts[0].cpu().numpy(), gpu_idx[k]) and
                         np.array_equal(pouts[1].cpu().numpy(), gpu_dist[k]))
            plain[k] = dict(ms=ms, gcups=dense[k] / (ms * 1e-3) / 1e9)
        plain = dict(per_distance=plain, ms_per_step=total_plain_ms,
                     gcups=sum(dense.values()) / (total_plain_ms * 1e-3) / 1e9,
                     speedup_of_eapruned=total_plain_ms / ms_per_step, nn_identical=same)

    abl = None
    if args.ablation:
        abl = ablation(torch, eap, stream, q, wl["query_off"], r, wl["ref_off"], wl["params"],
                       {k: (gpu_idx[k], gpu_dist[k]) for k in kinds}, dense, kinds)

    # the same step under the other schedules (secondary figures, after the
    # timed region; the kernel times above come from the timed schedule)
    schedules = {}
    if len(kinds) > 1:
        for sc in ("pipelined", "serial", "concurrent"):
            if sc == args.schedule:
                continue
            step(schedule=sc)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                step(schedule=sc)
            torch.cuda.synchronize()
            cms = (time.perf_counter() - t1) * 1e3 / args.steps
            csame = all(np.array_equal(outs[k][0].cpu().numpy(), gpu_idx[k]) and
                        np.array_equal(outs[k][1].cpu().numpy(), gpu_dist[k]) for k in kinds)
            schedules[sc] = dict(ms_per_step=cms, value=sum(dense.values()) / (cms * 1e-3) / 1e9,
                                 nn_identical=csame)

    other = None
    if args.compare_precision:
        op = 1 - args.precision
        step(op)
        torch.cuda.synchronize()
        a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        a.record(stream)
        for _ in range(reps):
            step(op)
        b_.record(stream)
        torch.cuda.synchronize()
        same = all(np.array_equal(outs[k][0].cpu().numpy(), gpu_idx[k]) and
                   np.array_equal(outs[k][1].cpu().numpy(), gpu_dist[k]) for k in kinds)
        other = dict(precision=op, ms_per_step=a.elapsed_time(b_) / reps, nn_identical=same)

    cpu = None
    if args.cpu_queries > 0:
        cpu = cpu_baseline(wl, kinds, gpu_idx, gpu_dist, eap_q=min(args.cpu_queries, nq), dp_q=min(args.cpu_queries, nq, 64),
                           derivative=args.derivative)
        if args.cpu_queries >= nq:
            # cells the GPU sweeps execute per step against those sequential
            # EAPruned evaluates on the same queries (Alg. 1's order and cut-off)
            for k in kinds:
                seq = cpu["sequential_eapruned_cells"].get(k)
                if seq:
                    per[k]["executed_vs_sequential_eapruned"] = per[k]["executed_cells_per_step"] / seq

    total_dense = sum(dense.values())
    line = dict(
        metric=METRIC,
        value=total_dense / (ms_per_step * 1e-3) / 1e9,
        unit="GCUPS",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=ms_per_step,
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype=("f32+f64" if args.precision else "f64"),
        data="synthetic",
        config=dict(workload="1-NN classification, 500 queries x 500 candidates, length 512, 5 warped-sine "
                             "classes; " + ("derivative variants (first-derivative series computed in every "
                                            "step) of " if args.derivative else "") + ", ".join(kinds) +
                             " (CDTW w=10%, WDTW g=0.05, ERP gap=0, MSM c=0.5, TWE nu=0.001 lambda=1)",
                    queries=nq, candidates=nr, length=512, distances=kinds,
                    precision=("fp32 screen + fp64 recheck" if args.precision else "fp64")),
        other_precision=other,
        schedule=args.schedule,
        other_schedules=schedules,
        tuning=tuning,
        queries_per_s=nq * len(kinds) / (ms_per_step * 1e-3),
        step_ms_p50=float(np.percentile(step_ms, 50)),
        step_ms_p99=float(np.percentile(step_ms, 99)),
        per_distance=per,
        plain_gpu_dp=plain,
        ablation=abl,
        roofline=roofline,
        cpu_baseline=cpu,
    )
    print(json.dumps(line), flush=True)


def run_batched(args, torch, eap, synth):
    """Workload 4: 10,000 candidates x 1,000 queries of uneven lengths (64..2048,
    warped-sine classes), six distances, FP32 screen + FP64 recheck, shapes
    autotuned on a sample, and the six searches of a step captured in one HIP
    graph: a step is one graph launch."""
    dev = torch.device("cuda:0")
    kinds = [k for k in args.kinds.split(",") if k]
    wl = synth.make_workload(4, n_ref=args.refs or None, n_query=args.queries or None)
    qo, ro = wl["query_off"], wl["ref_off"]
    nq, nr = len(qo) - 1, len(ro) - 1
    q = torch.from_numpy(wl["queries"]).to(dev)
    r = torch.from_numpy(wl["refs"]).to(dev)
    labels = torch.from_numpy(wl["ref_labels"]).to(dev)
    P = wl["params"]
    ws = {k: eap.workspace(eap.nn1_workspace_bytes(qo, ro, P[k], precision=1), dev) for k in kinds}
    outs = {k: (torch.empty(nq, dtype=torch.int64, device=dev), torch.empty(nq, dtype=torch.float64, device=dev),
                torch.empty(nq, dtype=torch.int32, device=dev)) for k in kinds}
    dense = {k: dense_cells(k, P[k], qo, ro) for k in kinds}

    say(f"workload 4: {nq} queries x {nr} candidates resident; shapes")
    # shapes tuned on a sample (100 queries x every candidate), untimed
    sq, sr = min(100, nq), nr
    tq, tr = q[: qo[sq]], r[: ro[sr]]
    tuning = {}
    if args.shapes:
        lco_max = int(min(np.diff(qo).max(), np.diff(ro).max()))
        for item in args.shapes.split(","):
            k, shp = item.split("=")
            g, c = (int(x) for x in shp.split("x"))
            for prec in (0, 1):
                eap.tune_set(swept_kind(k, P[k]), prec, lco_max, g, c)
            tuning[k] = f"{g}x{c} (pinned)"
    elif not args.no_tune:
        for k in kinds:
            recs = eap.tune_nn1(tq, qo[: sq + 1], tr, ro[: sr + 1], P[k], precision=1)
            if recs:
                tuning[k] = next(f"{x['g']}x{x['c']}" for x in recs if x["chosen"])

    s = torch.cuda.Stream(dev)
    kst = {k: torch.cuda.Stream(dev) for k in kinds}

    def issue(flags=0, schedule="serial"):
        """The six searches of a step on `s`: one after the other, or
        (concurrent) each on a stream of its own forked from `s` and joined
        back, so that one search's latency-bound stages (bounds, seed sweep,
        recheck) can run beside another's main sweep."""
        if schedule == "concurrent":
            for k in kinds:
                kst[k].wait_stream(s)
                eap.nn1(q, qo, r, ro, P[k], ref_labels=labels, precision=1, flags=flags, ws=ws[k], out=outs[k],
                        stream=kst[k])
            for k in kinds:
                s.wait_stream(kst[k])
        else:
            for k in kinds:
                eap.nn1(q, qo, r, ro, P[k], ref_labels=labels, precision=1, flags=flags, ws=ws[k], out=outs[k],
                        stream=s)

    def eager():
        issue()

    say("eager run and graph capture")
    eager()   # uploads offsets and tables into the workspaces
    s.synchronize()
    want = {k: (outs[k][0].clone(), outs[k][1].clone(), outs[k][2].clone()) for k in kinds}
    eap.capture_begin(s)
    issue(eap.FLAG_PREPARED, args.batch_schedule)
    graph = eap.capture_end(s)
    for _ in range(args.warmup):
        graph.launch(stream=s)
    s.synchronize()
    say(f"{args.steps} timed graph launches")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    step_ev = []
    t0 = time.perf_counter()
    ev0.record(s)
    for _ in range(args.steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        graph.launch(stream=s)
        b.record(s)
        step_ev.append((a, b))
    ev1.record(s)
    s.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    step_ms = [a.elapsed_time(b) for a, b in step_ev]
    same = all(torch.equal(outs[k][i], want[k][i]) for k in kinds for i in range(3))
    graph.close()

    # per-distance breakdown and the dominant kernel: eager steps right after the
    # timed graph launches, every sweep launch bracketed by HIP events on the
    # stream it runs on (the same kernels, inputs and launch shapes the graph
    # replays; the graph itself cannot carry timing events)
    prof_steps = 2
    say("per-kernel timing steps")
    for k in kinds:
        eap.reset_counters(ws[k], stream=s)
    eap.profile_take()
    eap.profile_enable(True)
    for _ in range(prof_steps):
        eager()
    s.synchronize()
    eap.profile_enable(False)
    prof = eap.profile_take()
    counters = {k: eap.read_counters(ws[k], stream=s) for k in kinds}
    per = {}
    for k in kinds:
        sk = swept_kind(k, P[k])
        main = [x for x in prof if x["kind"] == sk and x["stage"] == 2]
        mc = counters[k]["stage_cells"][2] / prof_steps
        mms = sum(x["ms"] for x in main) / prof_steps
        fp32 = bool(main[0]["fp32"]) if main else False
        xd = bool(main[0].get("exact_diff")) if main else False
        ops = ops_per_cell(sk, fp32, xd)
        peak = (LANE_OPS_PER_S_F32 if fp32 else LANE_OPS_PER_S) / ops / 1e9
        per[k] = dict(sweep_ms=sum(x["ms"] for x in prof if x["kind"] == sk) / prof_steps,
                      main_sweep_ms=mms, main_launches=len(main) // prof_steps,
                      main_kernel=(kernel_label(main[0]) if main else None), main_fp32=fp32, main_xd=xd,
                      main_cells=mc, dense_cells=dense[k],
                      main_gcups=(mc / (mms * 1e-3) / 1e9) if mms else None, main_peak_gcups=peak,
                      main_frac=(mc / (mms * 1e-3) / 1e9 / peak) if mms else None,
                      executed_fraction=counters[k]["cells"] / prof_steps / dense[k] if dense[k] else None,
                      fp64_rechecks=counters[k]["rechecks"] / prof_steps,
                      lb_pruned=counters[k]["lb_pruned"] / prof_steps,
                      nn_accuracy=float(np.mean(outs[k][2].cpu().numpy() == wl["query_labels"])))
    dom = max(kinds, key=lambda k: per[k]["main_sweep_ms"])
    d = per[dom]
    ops = ops_per_cell(swept_kind(dom, P[dom]), d["main_fp32"], d["main_xd"])
    kernel = f"{d['main_kernel']} sweep, {swept_kind(dom, P[dom]).upper()} main stage, " \
             f"{'fp32' if d['main_fp32'] else 'fp64'}"
    launch_ms = d["main_sweep_ms"] / max(d["main_launches"], 1)
    roofline = dict(bound="alu", achieved=d["main_gcups"], peak=d["main_peak_gcups"], unit="GCUPS",
                    frac=d["main_frac"], traffic=None, kernel=kernel, ops_per_cell=ops, launch_ms=launch_ms,
                    cells_per_launch=d["main_cells"] / max(d["main_launches"], 1),
                    convention=ROOFLINE_CONVENTION,
                    note=f"kernel time: mean of {prof_steps} eager steps right after the timed graph launches, "
                         "HIP events on the launch stream")
    roofline["traffic"], roofline["traffic_note"] = hbm_traffic(kernel)

    # plain FP64 DP on the GPU for the first queries against every candidate,
    # scaled to the whole workload by dense cells
    plain = None
    if not args.no_plain:
        say("plain FP64 DP sample")
        pq = min(50, nq)
        pqv = q[: qo[pq]]
        pms = 0.0
        pdense = 0
        pws = {k: eap.workspace(eap.nn1_workspace_bytes(qo[: pq + 1], ro, P[k]), dev) for k in kinds}
        for k in kinds:
            eap.nn1(pqv, qo[: pq + 1], r, ro, P[k], ws=pws[k], flags=eap.FLAG_PLAIN, stream=s)
            s.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            eap.nn1(pqv, qo[: pq + 1], r, ro, P[k], ws=pws[k], flags=eap.FLAG_PLAIN, stream=s)
            b.record(s)
            s.synchronize()
            pms += a.elapsed_time(b)
            pdense += dense_cells(k, P[k], qo[: pq + 1], ro)
        gcups = pdense / (pms * 1e-3) / 1e9
        est = sum(dense.values()) / (gcups * 1e9) * 1e3
        plain = dict(sample=f"first {pq} queries x all {nr} candidates", gcups=gcups,
                     ms_per_step_estimate=est, speedup_of_eapruned=est / ms_per_step)
        del pws

    abl = None
    if args.ablation:
        say("ablation")
        aq = min(args.ablation_queries, nq)
        aqo = qo[: aq + 1]
        abl = ablation(torch, eap, s, q[: qo[aq]], aqo, r, ro, P,
                       {k: (outs[k][0][:aq].cpu().numpy(), outs[k][1][:aq].cpu().numpy()) for k in kinds},
                       {k: dense_cells(k, P[k], aqo, ro) for k in kinds}, kinds)
        abl = dict(sample=f"first {aq} queries x all {nr} candidates", variants=abl)

    cpu = None
    if args.cpu_queries > 0:
        say("CPU oracle baseline")
        gi = {k: outs[k][0].cpu().numpy() for k in kinds}
        gd = {k: outs[k][1].cpu().numpy() for k in kinds}
        cpu = cpu_baseline(wl, kinds, gi, gd, eap_q=min(args.cpu_queries, nq), dp_q=min(16, nq), dp_r=250,
                           one_q=1, one_r=2000)
        # every cell the GPU search executes (seed, FP32 main sweep, FP64
        # rechecks) on the oracle's sample, against the cells sequential
        # EAPruned evaluates there (Alg. 1's order and cut-off)
        cq = min(args.cpu_queries, nq)
        ratio = {}
        for k in kinds:
            c0 = eap.read_counters(ws[k], stream=s)["cells"]
            eap.nn1(q[: qo[cq]], qo[: cq + 1], r, ro, P[k], ref_labels=labels, precision=1, ws=ws[k], stream=s)
            c1 = eap.read_counters(ws[k], stream=s)["cells"]
            seq = cpu["sequential_eapruned_cells"].get(k)
            if seq:
                ratio[k] = (c1 - c0) / seq
        cpu["gpu_executed_vs_sequential_eapruned"] = ratio

    total = sum(dense.values())
    print(json.dumps(dict(
        metric=METRIC, value=total / (ms_per_step * 1e-3) / 1e9, unit="GCUPS", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32+f64", data="synthetic",
        config=dict(workload=f"batched uneven lengths: 1-NN of {nq} queries among {nr} candidates, lengths "
                             "uniform in [64, 2048], 5 warped-sine classes, six distances (CDTW w=10%, WDTW "
                             "g=0.05, ERP gap=0, MSM c=0.5, TWE nu=0.001 lambda=1), FP32 screen + FP64 recheck "
                             "(margin 1e-4 relative), one HIP graph launch per step", queries=nq, candidates=nr,
                    lengths=[64, 2048], distances=kinds, precision="fp32 screen + fp64 recheck",
                    schedule=args.batch_schedule),
        queries_per_s=nq * len(kinds) / (ms_per_step * 1e-3),
        step_ms_p50=float(np.percentile(step_ms, 50)), step_ms_p99=float(np.percentile(step_ms, 99)),
        graph_results_identical_to_eager=same, tuning=tuning, per_distance=per, plain_gpu_dp=plain,
        ablation=abl, roofline=roofline, cpu_baseline=cpu)), flush=True)


def run_subseq(args, torch, eap, synth):
    """Workload 6: sub-sequence search (Section 5.3), the query slid along a
    long reference series as NN search over its z-normalised windows.  A
    random walk of 2^20 + 127 values (2^20 windows of 128), 16 queries of 128
    values (8 noisy, scaled and shifted copies of windows, 8 random walks),
    CDTW w = 5% (the usual UCR-suite window; --kinds dtw for full DTW), FP64
    sweeps unless --precision 1 asks for the FP32 screen.  A step builds the
    z-normalised windows (a GB of candidates, resident in HBM) and searches
    every query."""
    dev = torch.device("cuda:0")
    m, nw, nq = 128, (args.refs or (1 << 20)), (args.queries or 16)
    W = synth.subseq_workload(nw, m, nq)
    s, qs, starts = W["series"], W["queries"], W["starts"]
    n = nw + m - 1
    kinds = [k for k in args.kinds.split(",") if k in ("dtw", "cdtw")] if args.kinds != ap_default_kinds else ["cdtw"]
    P = {"dtw": dict(kind="dtw"), "cdtw": dict(kind="cdtw", window_ratio=0.05)}
    sd = torch.from_numpy(s).to(dev)
    qv = torch.from_numpy(np.concatenate(qs)).to(dev)
    q_off = np.arange(nq + 1, dtype=np.int64) * m
    r_off = np.arange(nw + 1, dtype=np.int64) * m
    w = torch.empty(nw * m, dtype=torch.float64, device=dev)
    zq = torch.empty(nq * m, dtype=torch.float64, device=dev)
    ws = {k: eap.workspace(eap.nn1_workspace_bytes(q_off, r_off, P[k], precision=1), dev) for k in kinds}   # fits both
    outs = {k: (torch.empty(nq, dtype=torch.int64, device=dev), torch.empty(nq, dtype=torch.float64, device=dev), None)
            for k in kinds}
    stream = torch.cuda.current_stream(dev)

    zws = eap.workspace(eap.lib().eap_znorm_workspace(nq), dev)
    flags = {k: 0 for k in kinds}

    def step():
        # the windows and queries are rebuilt every step; their offsets (2^20 + 1
        # of them) are the same each time, so after the first search they stay
        # on the device (flags bit 2) instead of being checked and uploaded again
        eap.subseq_windows(sd, m, out=w)
        eap.znorm(qv, q_off, ws=zws, out=zq)
        for k in kinds:
            eap.nn1(zq, q_off, w, r_off, P[k], ws=ws[k], out=outs[k], precision=args.precision, flags=flags[k])
            flags[k] = eap.FLAG_PREPARED

    step()
    if not args.no_tune:
        for k in kinds:
            eap.tune_nn1(zq, q_off, w, r_off, P[k], precision=args.precision, ws=ws[k])
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    eap.profile_take()
    eap.profile_enable(True)
    for k in kinds:
        eap.reset_counters(ws[k])
    steps = max(1, min(args.steps, 5))
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / steps
    eap.profile_enable(False)
    prof = eap.profile_take()
    dense = {k: dense_cells(k, P[k], q_off, r_off) for k in kinds}
    cnt = {k: eap.read_counters(ws[k]) for k in kinds}
    found = {k: int(sum(1 for i, st in enumerate(starts) if int(outs[k][0][i].item()) == int(st))) for k in kinds}
    per = {}
    for k in kinds:
        main = [x for x in prof if x["kind"] == k and x["stage"] == 2]
        per[k] = dict(main_sweep_ms=(sum(x["ms"] for x in main) / len(main)) if main else None,
                      main_kernel=(kernel_label(main[0]) if main else None),
                      main_fp32=bool(main[0]["fp32"]) if main else False,
                      main_cells_per_launch=cnt[k]["stage_cells"][2] / steps, dense_cells=dense[k],
                      executed_fraction=cnt[k]["cells"] / steps / dense[k],
                      lb_pruned_fraction=cnt[k]["lb_pruned"] / steps / (nq * nw),
                      fp64_rechecks_per_step=cnt[k]["rechecks"] / steps,
                      planted_found=found[k], planted=len(starts))
    # dominant kernel: the main sweep, executed cells per launch over its launch time
    dom = max(kinds, key=lambda k: per[k]["main_sweep_ms"] or 0.0)
    d = per[dom]
    roofline = None
    if d["main_sweep_ms"]:
        ops = (OPS_PER_CELL_F32 if d["main_fp32"] else OPS_PER_CELL)[dom]
        peak = (LANE_OPS_PER_S_F32 if d["main_fp32"] else LANE_OPS_PER_S) / ops / 1e9
        achieved = d["main_cells_per_launch"] / (d["main_sweep_ms"] * 1e-3) / 1e9
        kernel = f"{d['main_kernel']} sweep, {dom.upper()} main stage, {'fp32' if d['main_fp32'] else 'fp64'}"
        roofline = dict(bound="alu", achieved=achieved, peak=peak, unit="GCUPS", frac=achieved / peak,
                        traffic=None, kernel=kernel, ops_per_cell=ops, launch_ms=d["main_sweep_ms"],
                        cells_per_launch=d["main_cells_per_launch"])
        roofline["traffic"], roofline["traffic_note"] = hbm_traffic(kernel)
    abl = None
    if args.ablation:
        abl = ablation(torch, eap, stream, zq, q_off, w, r_off, P,
                       {k: (outs[k][0].cpu().numpy(), outs[k][1].cpu().numpy()) for k in kinds}, dense, kinds)
    # the oracle on the whole workload, timed like one step: the windows and
    # the queries normalised, then the NN search; the GPU answers compared
    cpu = None
    if args.cpu_queries > 0:
        from oracle import oracle as orc
        same, cells, secs = True, 0.0, 0.0
        for k in kinds:
            t1 = time.perf_counter()
            ow = orc.subseq_windows(s, m)
            oq = np.concatenate([orc.subseq_windows(x, m) for x in qs])
            oi, od, _ = orc.nn1(P[k], oq, q_off, ow, r_off, "eap")
            secs += time.perf_counter() - t1
            cells += dense[k]
            same &= bool(np.array_equal(outs[k][0].cpu().numpy(), oi)
                         and np.array_equal(outs[k][1].cpu().numpy(), od))
            del ow
        cpu = dict(value=cells / secs / 1e9, unit="GCUPS", cores=orc.num_threads(), kind="oracle",
                   sample=f"the whole workload: {nw} windows normalised and the EAPruned NN of the {nq} queries "
                          f"({secs:.1f} s)",
                   nn_identical_to_gpu=same)
    total = sum(dense.values())
    print(json.dumps(dict(
        metric=METRIC, value=total / (ms_per_step * 1e-3) / 1e9, unit="GCUPS", n_gpus=1, steps=steps, warmup=args.warmup,
        ms_per_step=ms_per_step, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype=("f32+f64" if args.precision else "f64"), data="synthetic",
        config=dict(workload=f"sub-sequence search: {nq} queries of {m} values in a random walk of {n} values "
                             f"({nw} z-normalised windows), " + ", ".join(
                                 f"{k}" + (" w=5%" if k == "cdtw" else "") for k in kinds),
                    queries=nq, windows=nw, length=m, distances=kinds),
        queries_per_s=nq * len(kinds) / (ms_per_step * 1e-3), per_distance=per, ablation=abl,
        roofline=roofline, cpu_baseline=cpu)), flush=True)


def run_served(args, torch, eap, synth):
    """Workload 5: a request server over 50,000 resident random walks (lengths
    128..1024); queries (lengths 128..1024) arrive as a Poisson process at
    2,000 q/s for 5 s of warm-up and 30 s measured, and are answered in
    batches on 4 slots (FP32 screen + FP64 recheck, admission by memory).
    Latency = arrival -> result on the host, over the queries that arrive in
    the measured 30 s.  Also the closed-loop capacity (a block of queries
    submitted at once) and, when the offered rate exceeds it, a run at 90% of
    it (the sustainable rate) with the same warm-up and window.  The roofline
    is the main sweeps' executed cells over their launch times (HIP events)
    during 2 s of the measured window, from the server's own counters."""
    dev = torch.device("cuda:0")
    rate, warm_s, meas_s = 2000.0, 5.0, 30.0
    nq_total = args.queries or int(rate * (warm_s + meas_s))
    wl = synth.make_workload(5, n_ref=args.refs or None, n_query=nq_total)
    ro, qo = wl["ref_off"], wl["query_off"]
    nr, nq = len(ro) - 1, len(qo) - 1
    r = torch.from_numpy(wl["refs"]).to(dev)
    qs = [wl["queries"][qo[i]: qo[i + 1]] for i in range(nq)]
    times = wl["arrivals"][:nq] - wl["arrivals"][0]
    kinds = [k for k in args.kinds.split(",") if k in wl["params"]] or list(wl["params"])
    out = {}
    for k in kinds:
        p = wl["params"][k]
        say(f"workload 5 {k}: {nq} queries over {nr} resident candidates")
        if not args.no_tune:   # shapes for this distance, on a sample of the traffic
            eap.tune_nn1(torch.from_numpy(wl["queries"][: qo[32]]).to(dev), qo[:33], r, ro, p, precision=1)

        def serve(tm, n, prof_window=None):
            """Queries 0..n-1 submitted at times tm (s from the start); returns
            completion times, results, stats and, for prof_window = (t0, t1),
            the main sweeps' cells and launches within it."""
            srv = eap.Server(r, ro, p, slots=4, max_batch=64, max_query_len=1024, mem_budget=8 << 30, precision=1)
            done, prof = {}, None
            try:
                t0 = time.perf_counter()
                i = 0
                phase = 0
                c0 = None
                while len(done) < n:
                    now = time.perf_counter() - t0
                    if prof_window and phase == 0 and now >= prof_window[0]:
                        c0 = srv.counters()
                        eap.profile_take()
                        eap.profile_enable(True)
                        phase = 1
                    elif prof_window and phase == 1 and now >= prof_window[1]:
                        c1 = srv.counters()
                        eap.profile_enable(False)
                        recs = [x for x in eap.profile_take() if x["stage"] == 2]
                        prof = dict(cells=c1["stage_cells"][2] - c0["stage_cells"][2], launches=recs)
                        phase = 2
                    while i < n and tm[i] <= now:
                        srv.submit(qs[i], i)
                        i += 1
                    res = srv.poll()
                    tnow = time.perf_counter() - t0
                    for tag, idx, dist, _ in res:
                        done[tag] = (tnow, idx, dist)
                    if not res and (i == n or tm[i] > tnow + 2e-4):
                        time.sleep(1e-4)
                st = srv.stats()
            finally:
                eap.profile_enable(False)
                srv.close()
            return done, st, prof

        def summary(tm, n, done):
            meas = [j for j in range(n) if warm_s <= tm[j] < warm_s + meas_s]
            lat = np.array([done[j][0] - tm[j] for j in meas]) * 1e3
            completed = sum(1 for v in done.values() if warm_s <= v[0] < warm_s + meas_s)
            return dict(offered_qps=len(meas) / meas_s, achieved_qps=completed / meas_s,
                        p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                        max_ms=float(lat.max()), measured_queries=len(meas)), meas

        ncap = min(nq, 4000)
        serve(np.zeros(min(nq, 500)), min(nq, 500))   # warm-up of the process: a first block
        say(f"{k}: closed-loop capacity on {ncap} queries")
        t = time.perf_counter()
        cap_done, _, _ = serve(np.zeros(ncap), ncap)
        cap_qps = ncap / max(v[0] for v in cap_done.values())
        say(f"{k}: offered {rate:.0f} q/s for {warm_s + meas_s:.0f} s")
        done, st, prof = serve(times, nq, prof_window=(warm_s + 5.0, warm_s + 7.0))
        res, meas = summary(times, nq, done)
        same = all(done[j][1:] == cap_done[j][1:] for j in range(ncap))
        res.update(capacity_qps=cap_qps, batches=st["batches"], max_batch=st["max_batch_seen"],
                   max_inflight=st["max_inflight"], results_identical_to_closed_loop=same)
        if rate > 0.9 * cap_qps:
            # the sustainable rate: the same arrival draws, slowed to 90% of capacity
            rs = 0.9 * cap_qps
            ts = times * (rate / rs)
            ns = int(np.searchsorted(ts, warm_s + meas_s))
            say(f"{k}: sustainable {rs:.0f} q/s for {warm_s + meas_s:.0f} s ({ns} queries)")
            sdone, _, _ = serve(ts, ns)
            sres, _ = summary(ts, ns, sdone)
            res["sustainable"] = dict(sres, rate_qps=rs)
        # roofline of the main sweeps inside the profiled window
        if prof and prof["launches"]:
            ms = sum(x["ms"] for x in prof["launches"])
            labels = {}
            for x in prof["launches"]:
                labels[kernel_label(x)] = labels.get(kernel_label(x), 0) + 1
            lab = max(labels, key=labels.get)
            fp32 = bool(prof["launches"][0]["fp32"])
            ops = ops_per_cell(swept_kind(k, p), fp32, bool(prof["launches"][0].get("exact_diff")))
            peak = (LANE_OPS_PER_S_F32 if fp32 else LANE_OPS_PER_S) / ops / 1e9
            ach = prof["cells"] / (ms * 1e-3) / 1e9
            res["roofline"] = dict(bound="alu", achieved=ach, peak=peak, unit="GCUPS", frac=ach / peak, traffic=None,
                                   kernel=f"{lab} sweep, {swept_kind(k, p).upper()} main stage, "
                                          f"{'fp32' if fp32 else 'fp64'}",
                                   launches=len(prof["launches"]), mean_launch_ms=ms / len(prof["launches"]),
                                   note="2 s of the measured window; launches of the 4 slots overlap, so each "
                                        "launch's time includes its share of the GPU",
                                   convention=ROOFLINE_CONVENTION)
        # the oracle on recorded served queries (the first measured ones)
        ncpu = args.cpu_queries if args.cpu_queries is not None else (500 if k == "cdtw" else 20)
        if ncpu > 0:
            from oracle import oracle as orc
            sel = meas[:ncpu]
            sq = np.concatenate([qs[j] for j in sel])
            so = np.concatenate([[0], np.cumsum([len(qs[j]) for j in sel])]).astype(np.int64)
            say(f"{k}: CPU oracle on {len(sel)} served queries")
            t = time.perf_counter()
            oi, od, _ = orc.nn1(p, sq, so, wl["refs"], ro, "eap")
            secs = time.perf_counter() - t
            gi = np.array([done[j][1] for j in sel])
            gd = np.array([done[j][2] for j in sel])
            res["cpu_baseline"] = dict(value=len(sel) / secs, unit="queries/s", cores=orc.num_threads(),
                                       kind="oracle", seconds=secs,
                                       sample=f"EAPruned NN of the first {len(sel)} measured served queries "
                                              f"against all {nr} candidates",
                                       nn_identical_to_gpu=bool(np.array_equal(gi, oi) and np.array_equal(gd, od)))
        out[k] = res
    k0 = kinds[0]
    print(json.dumps(dict(
        metric=METRIC, value=out[k0]["achieved_qps"], unit="queries/s", n_gpus=1, steps=1, warmup=1,
        ms_per_step=None, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32+f64",
        data="synthetic",
        config=dict(workload=f"served 1-NN: {nr} resident random walks (lengths 128..1024), queries (lengths "
                             "128..1024) arriving as a Poisson process at 2000 q/s, 5 s warm-up + 30 s measured, "
                             "CDTW w=5% and MSM c=0.5, FP32 screen + FP64 recheck, 4 slots x batches of at most 64",
                    candidates=nr, queries=nq, distances=kinds),
        roofline=out[k0].get("roofline"), cpu_baseline=out[k0].get("cpu_baseline"),
        per_distance=out)), flush=True)


def _source_hash():
    """Hash of the library sources the committed counter summaries must match
    (the one the build embeds in libeap.so)."""
    from paper_2102_05221_amd import srchash
    return srchash.source_hash()


if __name__ == "__main__":
    main()
