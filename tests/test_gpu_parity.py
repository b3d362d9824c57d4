"""Parity of the HIP path with the CPU oracle (GPU required).

Distances must agree to 1e-12 relative (the contract) and in practice bit for
bit, since both sides evaluate every cell with the same operation order; NN
indices and labels must agree exactly.  Inputs are seeded and synthetic.
"""
import math
import sys

import numpy as np
import pytest

import paper_2102_05221_amd as eap
from paper_2102_05221_amd import synth

pytestmark = pytest.mark.gpu

INF = math.inf
RTOL = 1e-12

ALL = [
    dict(kind="dtw"),
    dict(kind="cdtw", window_ratio=0.1),
    dict(kind="cdtw", window_ratio=0.0),
    dict(kind="cdtw", window_ratio=0.35),
    dict(kind="wdtw", g=0.05),
    dict(kind="wdtw", g=0.6),
    dict(kind="erp", gap=0.0),
    dict(kind="erp", gap=0.3, window_ratio=0.2),
    dict(kind="msm", c=0.5),
    dict(kind="twe", nu=0.001, lam=1.0),
    dict(kind="twe", nu=0.5, lam=0.0),
]


def pid(p):
    return "-".join(f"{k}={v}" for k, v in p.items())


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


def close(g, o):
    if math.isinf(o) or math.isinf(g):
        return math.isinf(o) and math.isinf(g)
    return abs(g - o) <= RTOL * max(abs(o), 1e-300)


@pytest.mark.parametrize("p", ALL, ids=pid)
def test_distance_parity_with_cutoffs(torch_dev, orc, p):
    torch, dev = torch_dev
    rng = np.random.default_rng(100 + synth.SIX.index(p["kind"]))
    lens = [(1, 1), (1, 7), (7, 1), (3, 5), (17, 16), (64, 64), (65, 130), (200, 199), (333, 512), (512, 500),
            (1000, 1024), (257, 1)]
    nbits = ntot = 0
    for (lx, ly) in lens:
        x = synth.znorm(np.cumsum(rng.normal(size=lx))) if lx > 1 else rng.normal(size=1)
        y = synth.znorm(np.cumsum(rng.normal(size=ly))) if ly > 1 else rng.normal(size=1)
        d = orc.dp(p, x, y)
        cuts = [INF]
        if d < INF:
            cuts += [d, float(np.nextafter(d, -INF)), 0.5 * d, 1.5 * d, 0.0]
        xd, yd = to_dev(torch, dev, x), to_dev(torch, dev, y)
        for c in cuts:
            log(f"distance {pid(p)} lx={lx} ly={ly} cut={c}")
            g = float(eap.distance(xd, yd, p, c).item())
            want = d if d <= c else INF
            assert close(g, want), (lx, ly, c, g, want)
            ntot += 1
            nbits += (g == want)
    assert nbits == ntot, f"{ntot - nbits} of {ntot} results not bit-identical"


@pytest.mark.parametrize("p", ALL, ids=pid)
def test_distance_parity_long_series(torch_dev, orc, p):
    """Series up to 2048: wider than one strip of the row sweep, so the pair is
    swept strip by strip through the edge buffer (and the band sweep takes the
    wide windows)."""
    torch, dev = torch_dev
    rng = np.random.default_rng(300 + synth.SIX.index(p["kind"]))
    nbits = ntot = 0
    for (lx, ly) in [(1500, 2048), (2048, 2048), (1100, 300), (2048, 1), (1025, 1030), (700, 1900)]:
        x = synth.znorm(np.cumsum(rng.normal(size=lx))) if lx > 1 else rng.normal(size=1)
        y = synth.znorm(np.cumsum(rng.normal(size=ly))) if ly > 1 else rng.normal(size=1)
        d = orc.dp(p, x, y)
        cuts = [INF]
        if d < INF:
            cuts += [d, float(np.nextafter(d, -INF)), 0.5 * d, 1.02 * d]
        xd, yd = to_dev(torch, dev, x), to_dev(torch, dev, y)
        for c in cuts:
            log(f"distance long {pid(p)} lx={lx} ly={ly} cut={c}")
            g = float(eap.distance(xd, yd, p, c).item())
            want = d if d <= c else INF
            assert close(g, want), (lx, ly, c, g, want)
            ntot += 1
            nbits += (g == want)
    assert nbits == ntot, f"{ntot - nbits} of {ntot} results not bit-identical"


@pytest.mark.parametrize("kind", synth.SIX)
def test_nn1_long_uneven_lengths(torch_dev, orc, kind):
    """Workload-4 shape (class templates, lengths uniform in [64, 2048]),
    subsampled; FP64 and FP32 screen + FP64 recheck."""
    torch, dev = torch_dev
    wl = synth.make_workload(4, n_ref=30, n_query=6)
    p = wl["params"][kind]
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, wl["refs"])
    oi, od, _ = orc.nn1(p, wl["queries"], wl["query_off"], wl["refs"], wl["ref_off"], "dp")
    for precision in (0, 1):
        log(f"nn1 long uneven {kind} precision={precision}")
        gi, gd, _ = eap.nn1(q, wl["query_off"], r, wl["ref_off"], p, precision=precision)
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), oi)
        assert np.array_equal(gd.cpu().numpy(), od)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kind", ["dtw", "wdtw", "erp", "msm", "twe"])
def test_tuner_shapes_agree(torch_dev, orc, kind, precision):
    """Every row-sweep shape (16/32/64 lanes per pair x 8/16 columns per lane,
    strips of 128..1024 columns) gives the same NN bit for bit (the tuner checks
    it), and the tuned shape gives the oracle's."""
    torch, dev = torch_dev
    rng = np.random.default_rng(44)
    qs = synth.random_walks(rng, 6, (100, 700))
    rs = synth.random_walks(rng, 30, (60, 700))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    p = dict(synth.DEFAULT_PARAMS[kind])
    q, r = to_dev(torch, dev, qv), to_dev(torch, dev, rv)
    log(f"tuner {kind} precision={precision}")
    try:
        recs = eap.tune_nn1(q, qo, r, ro, p, precision=precision)
        assert len(recs) >= 6 and sum(x["chosen"] for x in recs) == 1
        gi, gd, _ = eap.nn1(q, qo, r, ro, p, precision=precision)
        torch.cuda.synchronize()
    finally:
        eap.tune_reset()
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)


@pytest.mark.parametrize("forked", [False, True], ids=["one_stream", "forked_streams"])
def test_graph_replays_match_eager(torch_dev, orc, forked):
    """The six searches of a workload-4-shaped batch (FP32 screen + FP64
    recheck) captured in one HIP graph, on the capturing stream or each on a
    stream of its own forked from it and joined back: every replay, with eager
    work on the same buffers in between, gives the eager results, which are
    the oracle's."""
    torch, dev = torch_dev
    wl = synth.make_workload(4, n_ref=40, n_query=8, length=(64, 700))
    qo, ro = wl["query_off"], wl["ref_off"]
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, wl["refs"])
    P = wl["params"]
    nq = len(qo) - 1
    s = torch.cuda.Stream(dev)
    ws = {k: eap.workspace(eap.nn1_workspace_bytes(qo, ro, P[k], precision=1), dev) for k in synth.SIX}
    outs = {k: (torch.empty(nq, dtype=torch.int64, device=dev), torch.empty(nq, dtype=torch.float64, device=dev),
                None) for k in synth.SIX}
    log("graph: eager pass")
    for k in synth.SIX:
        eap.nn1(q, qo, r, ro, P[k], precision=1, ws=ws[k], out=outs[k], stream=s)
    s.synchronize()
    want = {k: (outs[k][0].clone(), outs[k][1].clone()) for k in synth.SIX}
    for k in synth.SIX:
        oi, od, _ = orc.nn1(P[k], wl["queries"], qo, wl["refs"], ro, "dp")
        assert np.array_equal(want[k][0].cpu().numpy(), oi) and np.array_equal(want[k][1].cpu().numpy(), od)
    log(f"graph: capture (forked={forked})")
    ks = {k: torch.cuda.Stream(dev) for k in synth.SIX}
    eap.capture_begin(s)
    for k in synth.SIX:
        st = s
        if forked:
            ks[k].wait_stream(s)
            st = ks[k]
        eap.nn1(q, qo, r, ro, P[k], precision=1, flags=eap.FLAG_PREPARED, ws=ws[k], out=outs[k], stream=st)
    if forked:
        for k in synth.SIX:
            s.wait_stream(ks[k])
    g = eap.capture_end(s)
    try:
        for rep in range(3):
            log(f"graph: replay {rep}")
            with torch.cuda.stream(s):
                for k in synth.SIX:
                    outs[k][0].fill_(-7)
                    outs[k][1].fill_(-1.0)
            # eager work on the same workspace between replays
            eap.nn1(q, qo, r, ro, P["msm"], precision=0, ws=ws["msm"], stream=s)
            g.launch(stream=s)
            s.synchronize()
            for k in synth.SIX:
                assert torch.equal(outs[k][0], want[k][0]) and torch.equal(outs[k][1], want[k][1]), (rep, k)
    finally:
        g.close()


def test_capture_needs_prepared_inputs(torch_dev):
    torch, dev = torch_dev
    qv, qo = synth.pack([np.linspace(0, 1, 30)])
    rv, ro = synth.pack([np.linspace(1, 0, 30), np.zeros(20)])
    q, r = to_dev(torch, dev, qv), to_dev(torch, dev, rv)
    s = torch.cuda.Stream(dev)
    ws = eap.workspace(eap.nn1_workspace_bytes(qo, ro, dict(kind="dtw")), dev)
    out = (torch.empty(1, dtype=torch.int64, device=dev), torch.empty(1, dtype=torch.float64, device=dev), None)
    ev = torch.cuda.Event()
    ev.record(torch.cuda.current_stream(dev))   # creates the event before the capture
    torch.cuda.synchronize()
    eap.capture_begin(s)
    with pytest.raises(eap.EapError, match="prepared"):
        eap.nn1(q, qo, r, ro, dict(kind="dtw"), ws=ws, stream=s, out=out)
    with pytest.raises(eap.EapError, match="captured"):
        eap.nn1(q, qo, r, ro, dict(kind="dtw"), ws=ws, stream=s, out=out, flags=eap.FLAG_PREPARED, main_done=ev)
    eap.capture_end(s).close()


def test_pipelined_searches_match_serial(torch_dev, orc):
    """Six searches on six streams, main sweeps chained by events (each waits
    for the previous search's), two passes in a row: every result equals the
    serial call's and the oracle's."""
    torch, dev = torch_dev
    wl = synth.make_workload(2, n_ref=120, n_query=16)
    qo, ro = wl["query_off"], wl["ref_off"]
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, wl["refs"])
    P = wl["params"]
    kinds = list(P)
    nq = len(qo) - 1
    ws = {k: eap.workspace(eap.nn1_workspace_bytes(qo, ro, P[k], precision=1), dev) for k in kinds}
    log("pipelined: serial reference")
    want = {}
    for k in kinds:
        gi, gd, _ = eap.nn1(q, qo, r, ro, P[k], precision=1, ws=ws[k])
        want[k] = (gi.cpu().numpy(), gd.cpu().numpy())
        oi, od, _ = orc.nn1(P[k], wl["queries"], qo, wl["refs"], ro, "dp")
        assert np.array_equal(want[k][0], oi) and np.array_equal(want[k][1], od), k
    main = torch.cuda.current_stream(dev)
    st = {k: torch.cuda.Stream(dev) for k in kinds}
    done = {k: torch.cuda.Event() for k in kinds}
    outs = {k: (torch.full((nq,), -7, dtype=torch.int64, device=dev), torch.empty(nq, dtype=torch.float64, device=dev),
                None) for k in kinds}
    for rep in range(2):
        log(f"pipelined: pass {rep}")
        for i, k in enumerate(kinds):
            st[k].wait_stream(main)
            eap.nn1(q, qo, r, ro, P[k], precision=1, ws=ws[k], out=outs[k], stream=st[k],
                    main_wait=done[kinds[i - 1]] if i > 0 else None, main_done=done[k])
        for k in kinds:
            main.wait_stream(st[k])
        torch.cuda.synchronize()
        for k in kinds:
            assert np.array_equal(outs[k][0].cpu().numpy(), want[k][0]), k
            assert np.array_equal(outs[k][1].cpu().numpy(), want[k][1]), k


@pytest.mark.parametrize("p", [dict(kind="cdtw", window_ratio=0.05), dict(kind="msm", c=0.5)], ids=pid)
def test_server_results_alone_and_in_the_mix(torch_dev, orc, p):
    """Workload-5 shape, reduced: queries of uneven lengths submitted while
    earlier batches run (several slots in flight, batches of several queries)
    get exactly the result each gets alone, which is the oracle's."""
    import time
    torch, dev = torch_dev
    rng = np.random.default_rng(55)
    rs = synth.random_walks(rng, 300, (128, 400))
    qs = synth.random_walks(rng, 40, (128, 400))
    rs[17] = qs[3].copy()
    rv, ro = synth.pack(rs)
    r = to_dev(torch, dev, rv)
    srv = eap.Server(r, ro, p, slots=3, max_batch=6, max_query_len=400, mem_budget=1 << 30, precision=1)
    got = {}
    try:
        log(f"server {pid(p)}: staggered submits")
        for i, qv in enumerate(qs):
            srv.submit(qv, i)
            if i % 4 == 3:
                for tag, idx, dist, _ in srv.poll():
                    got[tag] = (idx, dist)
        t0 = time.time()
        while len(got) < len(qs):
            assert time.time() - t0 < 120, "server did not finish"
            for tag, idx, dist, _ in srv.poll():
                got[tag] = (idx, dist)
            time.sleep(0.001)
        st = srv.stats()
    finally:
        srv.close()
    assert st["queries"] == len(qs) and st["batches"] >= 2 and st["max_batch_seen"] >= 2
    log(f"server {pid(p)}: alone")
    for i, qv in enumerate(qs):
        qd = to_dev(torch, dev, qv)
        gi, gd, _ = eap.nn1(qd, np.array([0, len(qv)]), r, ro, p, precision=1)
        torch.cuda.synchronize()
        assert got[i] == (int(gi.item()), float(gd.item())), i
    qv_all, qo_all = synth.pack(qs)
    oi, od, _ = orc.nn1(p, qv_all, qo_all, rv, ro, "dp")
    assert [got[i][0] for i in range(len(qs))] == list(oi)
    assert [got[i][1] for i in range(len(qs))] == list(od)
    assert got[3] == (17, 0.0)


@pytest.mark.parametrize("p", [dict(kind="cdtw", window_ratio=0.1), dict(kind="erp", gap=0.3, window_ratio=0.2),
                               dict(kind="wdtw", g=0.05)], ids=pid)
def test_tuner_band_shapes_agree(torch_dev, orc, p):
    """The band sweep's lane counts (windowed CDTW/ERP, WDTW's narrow band:
    lengths within 64 of each other) agree bit for bit and with the oracle."""
    torch, dev = torch_dev
    rng = np.random.default_rng(45)
    qs = synth.random_walks(rng, 6, (400, 440))
    rs = synth.random_walks(rng, 30, (400, 440))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    q, r = to_dev(torch, dev, qv), to_dev(torch, dev, rv)
    for precision in (0, 1):
        log(f"band tuner {pid(p)} precision={precision}")
        try:
            recs = eap.tune_nn1(q, qo, r, ro, p, precision=precision)
            assert len(recs) == 2 and sum(x["chosen"] for x in recs) == 1
            gi, gd, _ = eap.nn1(q, qo, r, ro, p, precision=precision)
            torch.cuda.synchronize()
        finally:
            eap.tune_reset()
        oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
        assert np.array_equal(gi.cpu().numpy(), oi)
        assert np.array_equal(gd.cpu().numpy(), od)


ROW_SHAPES64 = [(4, 8), (4, 16), (8, 8), (8, 16), (16, 8), (16, 16), (32, 8), (32, 16), (64, 8), (64, 16)]


def test_distance_random_shapes_and_cutoffs(torch_dev, orc):
    """Seeded random cases: distance, parameters, lengths 1..2048, a pinned
    row-sweep shape (so most pairs run in several strips) and a cut-off at,
    just below or under the distance: bit-identical to the oracle."""
    torch, dev = torch_dev
    rng = np.random.default_rng(2024)
    kinds = ["dtw", "wdtw", "erp", "msm", "twe", "cdtw"]
    nbad = 0
    try:
        for case in range(60):
            kind = kinds[case % len(kinds)]
            p = dict(kind=kind)
            if kind == "wdtw":
                p["g"] = float(rng.choice([0.0, 0.01, 0.05, 0.3]))
            if kind == "erp":
                p["gap"] = float(rng.normal())
            if kind == "msm":
                p["c"] = float(rng.choice([0.0, 0.1, 0.5, 2.0]))
            if kind == "twe":
                p["nu"], p["lam"] = float(rng.choice([0.0, 0.001, 0.1])), float(rng.choice([0.0, 0.5, 1.0]))
            if kind == "cdtw":
                p["window_ratio"] = float(rng.choice([0.02, 0.1, 0.3]))
            lx = int(rng.integers(1, 2049)) if case % 3 else int(rng.integers(1, 300))
            ly = int(rng.integers(max(1, lx // 3), 2049)) if case % 3 else int(rng.integers(1, 300))
            x = synth.znorm(np.cumsum(rng.normal(size=lx))) if lx > 1 else rng.normal(size=1)
            y = synth.znorm(np.cumsum(rng.normal(size=ly))) if ly > 1 else rng.normal(size=1)
            g, c = ROW_SHAPES64[int(rng.integers(len(ROW_SHAPES64)))]
            eap.tune_reset()
            eap.tune_set("dtw" if kind == "cdtw" else kind, 0, min(lx, ly), g, c)
            d = orc.dp(p, x, y)
            cut = [INF, d, float(np.nextafter(d, -INF)), 0.7 * d][case % 4] if d < INF else INF
            log(f"random case {case}: {pid(p)} lx={lx} ly={ly} shape {g}x{c} cut={cut}")
            got = float(eap.distance(to_dev(torch, dev, x), to_dev(torch, dev, y), p, cut).item())
            want = d if d <= cut else INF
            nbad += not (got == want)
            assert close(got, want), (case, got, want)
    finally:
        eap.tune_reset()
    assert nbad == 0


@pytest.mark.parametrize("kind", ["dtw", "wdtw", "erp", "msm", "twe"])
def test_nn1_every_row_shape(torch_dev, orc, kind):
    """NN over ragged sets (lengths 1..600) with every row-sweep shape pinned in
    turn, FP64 and FP32 screen: each gives the oracle's result."""
    torch, dev = torch_dev
    rng = np.random.default_rng(77)
    qs = synth.random_walks(rng, 5, (1, 600))
    rs = synth.random_walks(rng, 25, (1, 600))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    p = dict(synth.DEFAULT_PARAMS[kind])
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    q, r = to_dev(torch, dev, qv), to_dev(torch, dev, rv)
    lco = min(max(np.diff(qo)), max(np.diff(ro)))
    try:
        for precision in (0, 1):
            shapes = ROW_SHAPES64 + ([(16, 32), (32, 32), (64, 32)] if precision and kind in ("dtw", "wdtw") else [])
            for g, c in shapes:
                eap.tune_reset()
                eap.tune_set(kind, precision, lco, g, c)
                log(f"nn1 {kind} precision={precision} shape {g}x{c}")
                gi, gd, _ = eap.nn1(q, qo, r, ro, p, precision=precision)
                torch.cuda.synchronize()
                assert np.array_equal(gi.cpu().numpy(), oi), (g, c)
                assert np.array_equal(gd.cpu().numpy(), od), (g, c)
    finally:
        eap.tune_reset()


@pytest.mark.parametrize("kind", synth.SIX)
def test_nn1_parity_class_templates(torch_dev, orc, kind):
    """Workload-2 data (five warped sine classes, length 512), subsampled."""
    torch, dev = torch_dev
    wl = synth.make_workload(2, n_ref=96, n_query=24)
    p = wl["params"][kind]
    log(f"nn1 class templates {kind}")
    oi, od, _ = orc.nn1(p, wl["queries"], wl["query_off"], wl["refs"], wl["ref_off"], "eap")
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, wl["refs"])
    labels = torch.from_numpy(wl["ref_labels"]).to(dev)
    gi, gd, gl = eap.nn1(q, wl["query_off"], r, wl["ref_off"], p, ref_labels=labels)
    torch.cuda.synchronize()
    gi, gd, gl = gi.cpu().numpy(), gd.cpu().numpy(), gl.cpu().numpy()
    assert np.array_equal(gi, oi)
    assert np.array_equal(gd, od)
    assert np.array_equal(gl, wl["ref_labels"][oi])


@pytest.mark.parametrize("precision", [0, 1])
def test_cdtw_lower_bound_prunes_and_keeps_the_nn(torch_dev, orc, precision):
    """CDTW (w = 10%) on workload-2 data: LB_Keogh skips pairs whose bound is
    above the cut-off, and the NN is still the oracle's."""
    torch, dev = torch_dev
    wl = synth.make_workload(2, n_ref=120, n_query=16)
    p = wl["params"]["cdtw"]
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, wl["refs"])
    ws = eap.workspace(eap.nn1_workspace_bytes(wl["query_off"], wl["ref_off"], p, precision=1), dev)
    eap.reset_counters(ws)
    log(f"cdtw lower bound precision={precision}")
    gi, gd, _ = eap.nn1(q, wl["query_off"], r, wl["ref_off"], p, precision=precision, ws=ws)
    c = eap.read_counters(ws)
    oi, od, _ = orc.nn1(p, wl["queries"], wl["query_off"], wl["refs"], wl["ref_off"], "dp")
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)
    assert c["lb_pruned"] > 0
    # with the bound switched off every pair is swept, with the same results
    eap.reset_counters(ws)
    gi, gd, _ = eap.nn1(q, wl["query_off"], r, wl["ref_off"], p, precision=precision, ws=ws, lb="none")
    assert eap.read_counters(ws)["lb_pruned"] == 0
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)


@pytest.mark.parametrize("m", [1, 2, 37, 128])
def test_subseq_windows_bit_equal_to_oracle(torch_dev, orc, m):
    """Z-normalised windows of a long series (sums, square root and divisions
    in the same order as the oracle's) equal the oracle's bit for bit."""
    torch, dev = torch_dev
    rng = np.random.default_rng(m)
    s = np.cumsum(rng.standard_normal(1500)) * 2.0 + 5.0
    s[100:130] = 3.25   # constant stretch: constant windows give zeros
    log(f"subseq windows m={m}")
    g = eap.subseq_windows(to_dev(torch, dev, s), m).cpu().numpy()
    assert np.array_equal(g, orc.subseq_windows(s, m))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("p", [dict(kind="dtw"), dict(kind="cdtw", window_ratio=0.1)], ids=pid)
def test_subseq_search_parity(torch_dev, orc, p, precision):
    """Sub-sequence search over a 4,000-value series with noisy, scaled and
    shifted copies of windows planted as queries: the GPU's best window and
    distance equal the oracle's."""
    torch, dev = torch_dev
    rng = np.random.default_rng(21 + precision)
    s = np.cumsum(rng.standard_normal(4000))
    m = 64
    sd = to_dev(torch, dev, s)
    w_or = orc.subseq_windows(s, m)
    off = np.arange(0, len(w_or) + 1, m, dtype=np.int64)
    for start in (0, 1234, 3936):
        q = 1.7 * s[start:start + m] - 2.0 + 0.05 * rng.standard_normal(m)
        log(f"subseq search {pid(p)} precision={precision} start={start}")
        gi, gd = eap.subseq_search(to_dev(torch, dev, q), sd, p, precision=precision)
        oi, od, _ = orc.nn1(p, orc.subseq_windows(q, m), np.array([0, m], dtype=np.int64), w_or, off, "dp")
        assert int(gi.item()) == int(oi[0]) and float(gd.item()) == float(od[0])


def test_znorm_bit_equal_to_oracle(torch_dev, orc):
    """Ragged z-normalisation in one launch (lengths 1 to 2048, a constant
    series, more series than the grid covers in one pass): each series equals
    the oracle's single window over it, bit for bit."""
    torch, dev = torch_dev
    rng = np.random.default_rng(77)
    lens = [1, 2, 37, 128, 1000, 2048, 5] + list(rng.integers(1, 9, 70_000))
    xs = [np.cumsum(rng.standard_normal(int(L))) * 3.0 + 7.0 for L in lens]
    xs[4] = np.full(1000, 2.5)
    v, off = synth.pack(xs)
    log("znorm ragged")
    g = eap.znorm(to_dev(torch, dev, v), off).cpu().numpy()
    want = np.concatenate([orc.subseq_windows(x, len(x)) for x in xs])
    assert np.array_equal(g, want)
    assert np.array_equal(g[off[4]:off[5]], np.zeros(1000))


@pytest.mark.parametrize("precision", [0, 1])
def test_subseq_search_many_windows(torch_dev, orc, precision):
    """Sixteen queries over the 70,000 windows of 64 of a random walk (the
    scans split over blocks, several queries per bound pass), half of them
    planted copies: the GPU's windows and distances equal the oracle's."""
    torch, dev = torch_dev
    W = synth.subseq_workload(70_000, 64, 16)
    s, m = W["series"], W["m"]
    qv = np.concatenate(W["queries"])
    log(f"subseq search many windows precision={precision}")
    gi, gd = eap.subseq_search(to_dev(torch, dev, qv), to_dev(torch, dev, s), dict(kind="cdtw", window_ratio=0.05),
                               precision=precision, m=m)
    w_or = orc.subseq_windows(s, m)
    zq = np.concatenate([orc.subseq_windows(x, m) for x in W["queries"]])
    q_off = np.arange(17, dtype=np.int64) * m
    oi, od, _ = orc.nn1(dict(kind="cdtw", window_ratio=0.05), zq, q_off, w_or,
                        np.arange(len(w_or) // m + 1, dtype=np.int64) * m, "eap")
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)
    assert np.array_equal(oi[:8], W["starts"])


def test_derivative_series_bit_equal_to_oracle(torch_dev, orc):
    """The derivative series of ragged series (lengths 1 to 300, the short
    cases included) equal the oracle's bit for bit."""
    torch, dev = torch_dev
    rng = np.random.default_rng(12)
    lens = [1, 2, 3, 4] + list(rng.integers(1, 300, 60))
    s = [rng.standard_normal(int(m)) * 3.0 for m in lens]
    v, o = synth.pack(s)
    log("derivative series")
    g = eap.derivative(to_dev(torch, dev, v), o).cpu().numpy()
    assert np.array_equal(g, orc.derivative(v, o))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kind", ["dtw", "cdtw", "wdtw"])
def test_derivative_variant_nn_parity(torch_dev, orc, kind, precision):
    """DDTW / DCDTW / DWDTW: NN search over the derivative series (device
    transform, then the usual search) gives the oracle's NN on the oracle's
    derivative series."""
    torch, dev = torch_dev
    wl = synth.make_workload(2, n_ref=80, n_query=10)
    p = wl["params"][kind]
    qo, ro = wl["query_off"], wl["ref_off"]
    log(f"derivative variant {kind} precision={precision}")
    qd = eap.derivative(to_dev(torch, dev, wl["queries"]), qo)
    rd = eap.derivative(to_dev(torch, dev, wl["refs"]), ro)
    gi, gd, _ = eap.nn1(qd, qo, rd, ro, p, precision=precision)
    oq, orr = orc.derivative(wl["queries"], qo), orc.derivative(wl["refs"], ro)
    oi, od, _ = orc.nn1(p, oq, qo, orr, ro, "dp")
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kind", ["erp", "cdtw", "msm", "wdtw"])
def test_candidates_prepared_flag(torch_dev, orc, kind, precision):
    """One workspace, three query batches of different sizes and lengths
    against the same candidates; the second and third reuse what the first
    derived from the candidates (flags bit 3).  Every batch gets the oracle's
    NN."""
    torch, dev = torch_dev
    rng = np.random.default_rng(77 + precision)
    rs = synth.random_walks(rng, 60, (40, 160))
    rv, ro = synth.pack(rs)
    r = to_dev(torch, dev, rv)
    p = {"erp": dict(kind="erp", gap=0.3), "cdtw": dict(kind="cdtw", window_ratio=0.1),
         "msm": dict(kind="msm", c=0.5), "wdtw": dict(kind="wdtw", g=0.1)}[kind]
    batches = [synth.random_walks(rng, 5, (40, 160)), synth.random_walks(rng, 9, (100, 220)),
               synth.random_walks(rng, 3, (30, 60))]
    packed = [synth.pack(b) for b in batches]
    nbytes = max(eap.nn1_workspace_bytes(qo, ro, p, precision=precision) for _, qo in packed)
    ws = eap.workspace(nbytes, dev)
    for i, (qv, qo) in enumerate(packed):
        log(f"candidates prepared {kind} precision={precision} batch {i}")
        gi, gd, _ = eap.nn1(to_dev(torch, dev, qv), qo, r, ro, p, precision=precision, ws=ws,
                            flags=eap.FLAG_CANDIDATES if i > 0 else 0)
        oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
        assert np.array_equal(gi.cpu().numpy(), oi), i
        assert np.array_equal(gd.cpu().numpy(), od), i
    if kind == "cdtw":
        # the LB_Keogh calls above left no interleaved copy of the candidates;
        # a call without the bound that reuses the candidates rebuilds it
        qv, qo = packed[1]
        log(f"candidates prepared {kind} precision={precision} without LB_Keogh")
        gi, gd, _ = eap.nn1(to_dev(torch, dev, qv), qo, r, ro, p, precision=precision, ws=ws,
                            flags=eap.FLAG_CANDIDATES, lb="none")
        oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
        assert np.array_equal(gi.cpu().numpy(), oi)
        assert np.array_equal(gd.cpu().numpy(), od)


@pytest.mark.parametrize("precision", [0, 1])
def test_cdtw_very_many_candidates_read_in_place(torch_dev, orc, precision):
    """2^18 + 5 short ragged candidates (lengths 8..16): the CDTW bound + LB
    kernel reads them in their own layout; then, on the same workspace with
    the candidates prepared, a search without LB_Keogh (which rebuilds the
    interleaved copy) and one with it.  Every result is the oracle's."""
    torch, dev = torch_dev
    rng = np.random.default_rng(123 + precision)
    nr = (1 << 18) + 5
    lens = rng.integers(8, 17, nr)
    ro = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    rv = rng.standard_normal(int(ro[-1]))
    qs = [rng.standard_normal(int(L)) for L in (12, 9, 16)]
    qs[1] = rv[ro[nr - 2]:ro[nr - 1]].copy()        # an exact match near the end
    qv, qo = synth.pack(qs)
    p = dict(kind="cdtw", window_ratio=0.25)
    r = to_dev(torch, dev, rv)
    q = to_dev(torch, dev, qv)
    ws = eap.workspace(eap.nn1_workspace_bytes(qo, ro, p, precision=1), dev)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "eap")
    assert oi[1] == nr - 2 and od[1] == 0.0
    for flags, lb in ((0, "default"), (eap.FLAG_CANDIDATES, "none"), (eap.FLAG_CANDIDATES, "default")):
        log(f"cdtw very many candidates precision={precision} flags={flags} lb={lb}")
        gi, gd, _ = eap.nn1(q, qo, r, ro, p, precision=precision, ws=ws, flags=flags, lb=lb)
        assert np.array_equal(gi.cpu().numpy(), oi), flags
        assert np.array_equal(gd.cpu().numpy(), od), flags


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kind", ["dtw", "cdtw", "erp"])
def test_nn1_many_queries(torch_dev, orc, kind, precision):
    """300,000 short queries (more than the largest grid of the per-query
    kernels covers in one pass, so every one of them strides) against three
    candidates; every query gets the oracle's NN."""
    torch, dev = torch_dev
    rng = np.random.default_rng(5 + precision)
    nq = 300_000
    lq = rng.integers(2, 5, nq)
    qo = np.concatenate([[0], np.cumsum(lq)]).astype(np.int64)
    qv = rng.standard_normal(int(qo[-1]))
    rs = [rng.standard_normal(3), rng.standard_normal(4), rng.standard_normal(2)]
    rv, ro = synth.pack(rs)
    p = {"dtw": dict(kind="dtw"), "cdtw": dict(kind="cdtw", window_ratio=0.5), "erp": dict(kind="erp", gap=0.1)}[kind]
    log(f"nn1 many queries {kind} precision={precision}")
    gi, gd, _ = eap.nn1(to_dev(torch, dev, qv), qo, to_dev(torch, dev, rv), ro, p, precision=precision)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)


@pytest.mark.parametrize("nr", [2000, 5000])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kind", ["dtw", "cdtw", "msm"])
def test_nn1_many_candidates(torch_dev, orc, kind, precision, nr):
    """Thousands of short candidates (the per-query scans run 256 or 1024
    threads per query); duplicated candidates check the lowest-index rule."""
    torch, dev = torch_dev
    rng = np.random.default_rng(nr + precision)
    rs = synth.random_walks(rng, nr, (24, 40))
    qs = synth.random_walks(rng, 5, (24, 40))
    rs[nr - 3] = qs[1].copy()            # an exact match late in the set ...
    rs[nr - 1] = qs[1].copy()            # ... and its duplicate: the lower index wins
    rs[7] = rs[nr // 2].copy()
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    p = {"dtw": dict(kind="dtw"), "cdtw": dict(kind="cdtw", window_ratio=0.2), "msm": dict(kind="msm", c=0.5)}[kind]
    log(f"nn1 many candidates {kind} precision={precision} nr={nr}")
    gi, gd, _ = eap.nn1(to_dev(torch, dev, qv), qo, to_dev(torch, dev, rv), ro, p, precision=precision)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    assert oi[1] == nr - 3 and od[1] == 0.0
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nq,nr", [(256, 4096), (64, 8192), (16, 16384)])
def test_cdtw_nn_bound_and_scan_shapes(torch_dev, orc, nq, nr, precision):
    """CDTW NN at shapes that take the bound + LB_Keogh kernel through 8, 4
    and 2 queries per pass over the candidates (on a 256-CU device) and split
    the per-query scans over 2 to 4 blocks; ragged lengths 20..40.  Exact
    copies of query 0 sit at candidates 5 and nr - 1, in different chunks of
    the split scans: the lower index must win."""
    torch, dev = torch_dev
    rng = np.random.default_rng(nq + nr + precision)
    rs = synth.random_walks(rng, nr, (20, 40))
    qs = synth.random_walks(rng, nq, (20, 40))
    rs[5] = qs[0].copy()
    rs[nr - 1] = qs[0].copy()
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    p = dict(kind="cdtw", window_ratio=0.2)
    log(f"cdtw bound and scan shapes nq={nq} nr={nr} precision={precision}")
    gi, gd, _ = eap.nn1(to_dev(torch, dev, qv), qo, to_dev(torch, dev, rv), ro, p, precision=precision)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "eap")
    assert oi[0] == 5 and od[0] == 0.0
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)


@pytest.mark.parametrize("precision", [0, 1])
def test_cdtw_windows_without_a_path(torch_dev, orc, precision):
    """CDTW w = 5% over uneven lengths: pairs whose window admits no path are
    +inf without a sweep (and are not counted as lower-bound prunes); a query
    with no feasible candidate gets index -1 and +inf, the others the
    oracle's NN."""
    torch, dev = torch_dev
    rng = np.random.default_rng(31)
    rs = synth.random_walks(rng, 40, (100, 121)) + synth.random_walks(rng, 30, (300, 301))
    qs = synth.random_walks(rng, 1, (40, 41)) + synth.random_walks(rng, 6, (100, 121)) + \
        synth.random_walks(rng, 3, (290, 311))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    p = dict(kind="cdtw", window_ratio=0.05)
    ws = eap.workspace(eap.nn1_workspace_bytes(qo, ro, p, precision=1), dev)
    eap.reset_counters(ws)
    log(f"cdtw windows without a path precision={precision}")
    gi, gd, _ = eap.nn1(to_dev(torch, dev, qv), qo, to_dev(torch, dev, rv), ro, p, precision=precision, ws=ws)
    c = eap.read_counters(ws)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    assert oi[0] == -1 and np.isinf(od[0])
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)
    lq, lr = np.diff(qo), np.diff(ro)
    L = np.maximum(lq[:, None], lr[None, :])
    feasible = np.floor(0.05 * L) >= np.abs(lq[:, None] - lr[None, :])
    assert c["lb_pruned"] <= int(feasible.sum())


def test_nn1_parity_random_walk_workload_full(torch_dev, orc):
    """Workload 1 in full: DTW, 100 x 100 random walks of length 128."""
    torch, dev = torch_dev
    wl = synth.make_workload(1)
    p = wl["params"]["dtw"]
    log("nn1 workload 1 full")
    oi, od, _ = orc.nn1(p, wl["queries"], wl["query_off"], wl["refs"], wl["ref_off"], "dp")
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, wl["refs"])
    labels = torch.from_numpy(wl["ref_labels"]).to(dev)
    gi, gd, gl = eap.nn1(q, wl["query_off"], r, wl["ref_off"], p, ref_labels=labels)
    torch.cuda.synchronize()
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)
    assert np.array_equal(gl.cpu().numpy(), wl["ref_labels"][oi])


@pytest.mark.parametrize("p", ALL, ids=pid)
def test_nn1_parity_ragged_lengths(torch_dev, orc, p):
    """Uneven lengths (ragged tails of every strip and band size)."""
    torch, dev = torch_dev
    rng = np.random.default_rng(7)
    qs = synth.random_walks(rng, 9, (5, 300))
    rs = synth.random_walks(rng, 40, (1, 300))
    rs[3] = qs[0].copy()            # an exact match
    rs[11] = rs[10].copy()          # a duplicate: ties go to the lower index
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    log(f"nn1 ragged {pid(p)}")
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    gi, gd, _ = eap.nn1(to_dev(torch, dev, qv), qo, to_dev(torch, dev, rv), ro, p)
    torch.cuda.synchronize()
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy(), od)


def test_nn1_no_feasible_candidate(torch_dev, orc):
    torch, dev = torch_dev
    p = dict(kind="cdtw", window_ratio=0.05)
    qv, qo = synth.pack([np.zeros(10), np.linspace(0, 1, 40)])
    rv, ro = synth.pack([np.ones(80), np.ones(90), np.linspace(1, 0, 41)])
    log("nn1 infeasible windows")
    gi, gd, gl = eap.nn1(to_dev(torch, dev, qv), qo, to_dev(torch, dev, rv), ro, p,
                         ref_labels=torch.tensor([4, 5, 6], dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    assert list(gi.cpu().numpy()) == list(oi) == [-1, 2]
    assert gd.cpu().numpy()[0] == INF
    assert list(gl.cpu().numpy()) == [-1, 6]


@pytest.mark.parametrize("kind", ["dtw", "cdtw", "msm", "wdtw", "erp", "twe"])
@pytest.mark.parametrize("mode", ["prune", "full"])
def test_pairwise_parity(torch_dev, orc, kind, mode):
    """Workload-3 shape (random walks, all pairs), subsampled to 14 series of
    ragged lengths up to 1024."""
    torch, dev = torch_dev
    rng = np.random.default_rng(33)
    S = synth.random_walks(rng, 14, (700, 1024))
    sv, so = synth.pack(S)
    p = dict(synth.DEFAULT_PARAMS[kind])
    if kind == "cdtw":
        p["window_ratio"] = 0.05
    log(f"pairwise {kind} {mode}")
    want = orc.pairwise(p, sv, so, "full")
    got = eap.pairwise(to_dev(torch, dev, sv), so, p, mode).cpu().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("kind", synth.SIX)
def test_plain_dp_mode_gives_the_same_nn(torch_dev, kind):
    """The plain full-DP baseline (no cut-off) and the pruned search agree."""
    torch, dev = torch_dev
    wl = synth.make_workload(4, n_ref=60, n_query=10, length=(40, 260))
    p = wl["params"][kind]
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, wl["refs"])
    log(f"plain vs pruned {kind}")
    a = eap.nn1(q, wl["query_off"], r, wl["ref_off"], p)
    b = eap.nn1(q, wl["query_off"], r, wl["ref_off"], p, flags=eap.FLAG_PLAIN)
    c = eap.nn1(q, wl["query_off"], r, wl["ref_off"], p, flags=eap.FLAG_NO_SEED)
    torch.cuda.synchronize()
    for x in (b, c):
        assert torch.equal(a[0], x[0]) and torch.equal(a[1], x[1])


@pytest.mark.parametrize("margin", [1e-4, 0.0])
@pytest.mark.parametrize("kind", synth.SIX)
def test_fp32_screen_gives_fp64_results(torch_dev, orc, kind, margin):
    """Precision 1 (FP32 screen + FP64 recheck) returns the FP64 NN bit for bit,
    also when candidates differ by far less than FP32 can resolve; with margin
    0 only the certified rounding bound keeps the FP64 NN in the recheck."""
    torch, dev = torch_dev
    wl = synth.make_workload(2, n_ref=80, n_query=12, length=200)
    rs = synth.unpack(wl["refs"], wl["ref_off"])
    qs = synth.unpack(wl["queries"], wl["query_off"])
    rng = np.random.default_rng(5)
    # near-ties: copies of two queries, nudged by ~1e-9 (FP32 sees them as equal)
    rs[5] = qs[0].copy()
    rs[6] = qs[0].copy()
    rs[6][17] += 1e-9
    rs[9] = qs[1] + rng.normal(0, 1e-9, size=len(qs[1]))
    rs[2] = qs[1] + rng.normal(0, 1e-9, size=len(qs[1]))
    rv, ro = synth.pack(rs)
    p = wl["params"][kind]
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, rv)
    log(f"fp32 screen {kind} margin {margin}")
    ws = eap.workspace(eap.nn1_workspace_bytes(wl["query_off"], ro, p, precision=1), dev)
    eap.reset_counters(ws)
    a = eap.nn1(q, wl["query_off"], r, ro, p, precision=1, margin_rel=margin, ws=ws)
    c = eap.read_counters(ws)
    torch.cuda.synchronize()
    oi, od, _ = orc.nn1(p, wl["queries"], wl["query_off"], rv, ro, "dp")
    gi, gd = a[0].cpu().numpy(), a[1].cpu().numpy()
    bad = np.nonzero((gi != oi) | (gd != od))[0]
    assert bad.size == 0, [(int(i), int(gi[i]), float(gd[i]), int(oi[i]), float(od[i])) for i in bad]
    # the seed of each query is swept in FP64 first and not rechecked; the
    # nudged copies of queries 0 and 1 cannot be separated in FP32 and are
    assert c["rechecks"] >= 2
    # every listed candidate is recomputed once in FP64 (narrow-band overflows of
    # WDTW finish in the full-band rerun)
    assert c["stage_pairs"][4] + c["stage_pairs"][5] == c["rechecks"]


@pytest.mark.parametrize("margin", [1e-4, 0.0])
def test_fp32_screen_exact_differences_wdtw_long(torch_dev, orc, margin):
    """WDTW of long series (weights near the diagonal around 1e-22): the FP32
    screen forms its differences from the float64 values, and the NN must
    equal the FP64 oracle's bit for bit, near-ties included."""
    torch, dev = torch_dev
    rng = np.random.default_rng(31)
    qs = synth.random_walks(rng, 5, (1500, 2048))
    rs = synth.random_walks(rng, 36, (64, 2048))
    rs[3] = qs[0].copy()
    rs[4] = qs[0].copy()
    rs[4][100] += 1e-9
    rs[7] = qs[2] + rng.normal(0, 1e-9, size=len(qs[2]))
    rs[8] = qs[2] + rng.normal(0, 1e-9, size=len(qs[2]))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    p = dict(kind="wdtw", g=0.05)
    log(f"fp32 screen, exact differences, WDTW, margin {margin}")
    ws = eap.workspace(eap.nn1_workspace_bytes(qo, ro, p, precision=1), dev)
    eap.reset_counters(ws)
    eap.profile_take()
    eap.profile_enable(True)
    g = eap.nn1(to_dev(torch, dev, qv), qo, to_dev(torch, dev, rv), ro, p, precision=1, margin_rel=margin, ws=ws)
    torch.cuda.synchronize()
    eap.profile_enable(False)
    prof = eap.profile_take()
    c = eap.read_counters(ws)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    assert np.array_equal(g[0].cpu().numpy(), oi) and np.array_equal(g[1].cpu().numpy(), od)
    # the main sweep ran in FP32 with exact differences; the near-ties were rechecked
    main = [x for x in prof if x["stage"] == 2]
    assert main and all(x["fp32"] and x["exact_diff"] for x in main)
    assert c["rechecks"] >= 2


def test_exact_difference_row_shapes_wdtw_long(torch_dev, orc):
    """The FP32 WDTW sweep with float64 differences (long series: weights near
    the diagonal around 1e-22) with every row-sweep shape pinned in turn, strips
    of 32 to 2048 columns whose weight windows reach |j - i| near the longer
    length plus a strip: each gives the FP64 oracle's NN bit for bit, and its
    main stage ran as pinned."""
    torch, dev = torch_dev
    rng = np.random.default_rng(91)
    qs = synth.random_walks(rng, 3, (1500, 2048))
    rs = synth.random_walks(rng, 12, (64, 2048))
    rs[5] = qs[1] + rng.normal(0, 1e-9, size=len(qs[1]))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    p = dict(kind="wdtw", g=0.05)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    q, r = to_dev(torch, dev, qv), to_dev(torch, dev, rv)
    lco = min(max(np.diff(qo)), max(np.diff(ro)))
    try:
        for g, c in ROW_SHAPES64 + [(16, 32), (32, 32), (64, 32)]:
            eap.tune_reset()
            eap.tune_set("wdtw", 1, lco, g, c)
            log(f"exact-difference WDTW, shape {g}x{c}")
            eap.profile_take()
            eap.profile_enable(True)
            gi, gd, _ = eap.nn1(q, qo, r, ro, p, precision=1)
            torch.cuda.synchronize()
            eap.profile_enable(False)
            main = [x for x in eap.profile_take() if x["stage"] == 2]
            assert main and all(x["kernel"] == "rows" and x["fp32"] and x["exact_diff"] for x in main), main
            assert all(x["group"] == g and x["size"] == g * c for x in main), (g, c, main)
            assert np.array_equal(gi.cpu().numpy(), oi), (g, c)
            assert np.array_equal(gd.cpu().numpy(), od), (g, c)
    finally:
        eap.profile_enable(False)
        eap.tune_reset()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kind", ["erp", "msm", "twe"])
def test_every_row_shape_long_series(torch_dev, orc, kind, precision):
    """Long series (queries of 1500..2048 values, candidates of 64..2048) with
    every row-sweep shape pinned in turn: strips up to 1024 columns, TWE's
    per-diagonal window at the far ends of its table, the edge buffers of many
    strips.  Each shape gives the oracle's NN bit for bit."""
    torch, dev = torch_dev
    rng = np.random.default_rng(92 + precision)
    qs = synth.random_walks(rng, 3, (1500, 2048))
    rs = synth.random_walks(rng, 10, (64, 2048))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    p = dict(synth.DEFAULT_PARAMS[kind])
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    q, r = to_dev(torch, dev, qv), to_dev(torch, dev, rv)
    lco = min(max(np.diff(qo)), max(np.diff(ro)))
    try:
        for g, c in ROW_SHAPES64:
            eap.tune_reset()
            eap.tune_set(kind, precision, lco, g, c)
            log(f"long series {kind} precision={precision} shape {g}x{c}")
            gi, gd, _ = eap.nn1(q, qo, r, ro, p, precision=precision)
            torch.cuda.synchronize()
            assert np.array_equal(gi.cpu().numpy(), oi), (g, c)
            assert np.array_equal(gd.cpu().numpy(), od), (g, c)
    finally:
        eap.tune_reset()


def test_fp32_screen_ragged_windows(torch_dev, orc):
    torch, dev = torch_dev
    rng = np.random.default_rng(8)
    qs = synth.random_walks(rng, 7, (20, 400))
    rs = synth.random_walks(rng, 50, (10, 400))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    for p in (dict(kind="cdtw", window_ratio=0.1), dict(kind="erp", gap=0.2, window_ratio=0.3),
              dict(kind="wdtw", g=0.3)):
        log(f"fp32 screen ragged {p}")
        g = eap.nn1(to_dev(torch, dev, qv), qo, to_dev(torch, dev, rv), ro, p, precision=1)
        torch.cuda.synchronize()
        oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
        assert np.array_equal(g[0].cpu().numpy(), oi)
        assert np.array_equal(g[1].cpu().numpy(), od)


def test_profile_records_each_sweep(torch_dev):
    torch, dev = torch_dev
    wl = synth.make_workload(2, n_ref=30, n_query=4, length=64)
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, wl["refs"])
    eap.profile_take()
    eap.profile_enable(True)
    eap.nn1(q, wl["query_off"], r, wl["ref_off"], wl["params"]["msm"])
    eap.profile_enable(False)
    recs = eap.profile_take()
    assert [x["stage"] for x in recs] == [0, 2]
    assert all(x["kernel"] == "rows" and x["kind"] == "msm" and x["ms"] > 0 for x in recs)


def test_counters_accumulate(torch_dev):
    torch, dev = torch_dev
    wl = synth.make_workload(1, n_ref=20, n_query=5)
    p = wl["params"]["dtw"]
    ws = eap.workspace(eap.nn1_workspace_bytes(wl["query_off"], wl["ref_off"], p), dev)
    eap.reset_counters(ws)
    q, r = to_dev(torch, dev, wl["queries"]), to_dev(torch, dev, wl["refs"])
    eap.nn1(q, wl["query_off"], r, wl["ref_off"], p, ws=ws)
    c1 = eap.read_counters(ws)
    eap.nn1(q, wl["query_off"], r, wl["ref_off"], p, ws=ws)
    c2 = eap.read_counters(ws)
    assert c1["pairs"] > 0 and c1["cells"] > 0
    assert c2["pairs"] == 2 * c1["pairs"]


@pytest.mark.parametrize("ratio", [0.0, 0.05, 0.3, 0.99, 1.0, 2.0])
def test_envelopes_match_oracle(torch_dev, orc, ratio):
    """The O(L) envelope kernel (segmented scans) against the definition."""
    torch, dev = torch_dev
    rng = np.random.default_rng(int(ratio * 100) + 3)
    series = synth.random_walks(rng, 23, (1, 700)) + [rng.normal(size=1), rng.normal(size=2048)]
    v, off = synth.pack(series)
    vd = to_dev(torch, dev, v)
    for npos, other in ((700, 0), (2048, 2048), (64, 900), (1, 5)):
        log(f"envelopes ratio={ratio} npos={npos} other_max={other}")
        up, lo = eap.envelopes(vd, off, npos, ratio, other)
        torch.cuda.synchronize()
        up, lo = up.cpu().numpy(), lo.cpu().numpy()
        for i, x in enumerate(series):
            L = len(x)
            cap = max(L, npos)
            w = cap if ratio >= 1 else min(int(math.floor(ratio * max(L, other))), cap)
            ou, ol = orc.envelope(x, w, npos)
            empty = np.arange(1, npos + 1) > L + w
            assert np.array_equal(up[i][~empty], ou[~empty]) and np.array_equal(lo[i][~empty], ol[~empty]), (i, L)
            assert (up[i][empty] == INF).all() and (lo[i][empty] == -INF).all()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("p", [dict(kind="dtw"), dict(kind="cdtw", window_ratio=0.1),
                               dict(kind="cdtw", window_ratio=0.3)], ids=pid)
def test_nn_lower_bound_modes(torch_dev, orc, p, precision):
    """lb-none, lb-keogh (with LB_Kim's corners) and lb-keogh2 (plus the
    reversed LB_Keogh) give the oracle's NN, for DTW and CDTW, ragged lengths."""
    torch, dev = torch_dev
    rng = np.random.default_rng(77)
    qs = synth.random_walks(rng, 9, (20, 400))
    rs = synth.random_walks(rng, 150, (10, 420))
    rs[4] = qs[3].copy()                               # an exact match
    rs[9] = qs[5] + rng.normal(0, 1e-9, size=len(qs[5]))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    q, r = to_dev(torch, dev, qv), to_dev(torch, dev, rv)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    for lb in ("none", "keogh", "keogh2", "default"):
        log(f"nn lower bounds {pid(p)} lb={lb} precision={precision}")
        ws = eap.workspace(eap.nn1_workspace_bytes(qo, ro, p, precision=precision, lb=lb), dev)
        eap.reset_counters(ws)
        gi, gd, _ = eap.nn1(q, qo, r, ro, p, precision=precision, ws=ws, lb=lb)
        c = eap.read_counters(ws)
        assert np.array_equal(gi.cpu().numpy(), oi) and np.array_equal(gd.cpu().numpy(), od), lb
        if lb == "none":
            assert c["lb_pruned"] == 0
        elif lb in ("keogh", "keogh2"):
            assert c["lb_pruned"] > 0, lb


@pytest.mark.parametrize("p", ALL, ids=pid)
def test_nn_prune_only_and_no_pruning(torch_dev, orc, p):
    """Ablation modes: prune-only (each pair under its own path bound, FP64)
    and early abandoning without pruning (EABase), FP64 and FP32 screen."""
    torch, dev = torch_dev
    rng = np.random.default_rng(78)
    qs = synth.random_walks(rng, 7, (30, 700))
    rs = synth.random_walks(rng, 60, (20, 700))
    qv, qo = synth.pack(qs)
    rv, ro = synth.pack(rs)
    q, r = to_dev(torch, dev, qv), to_dev(torch, dev, rv)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    for flags, precision in ((eap.FLAG_PRUNE_ONLY, 0), (eap.FLAG_NO_PRUNE, 0), (eap.FLAG_NO_PRUNE, 1)):
        log(f"nn ablation mode {pid(p)} flags={flags} precision={precision}")
        gi, gd, _ = eap.nn1(q, qo, r, ro, p, precision=precision, flags=flags)
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), oi) and np.array_equal(gd.cpu().numpy(), od), (flags, precision)


def mv_series(rng, L, D):
    """A z-normalised random-walk series of L points and D channels, point-major."""
    x = np.cumsum(rng.normal(size=(L, D)), axis=0)
    return ((x - x.mean(axis=0)) / x.std(axis=0).clip(1e-12)).ravel()


MV = [dict(kind="dtw", dims=2), dict(kind="dtw", dims=3), dict(kind="dtw", dims=4),
      dict(kind="cdtw", window_ratio=0.1, dims=3), dict(kind="cdtw", window_ratio=0.3, dims=2),
      dict(kind="cdtw", window_ratio=0.0, dims=4)]


@pytest.mark.parametrize("p", MV, ids=pid)
def test_multivariate_distance_parity(torch_dev, orc, p):
    torch, dev = torch_dev
    D = p["dims"]
    rng = np.random.default_rng(90 + D)
    for lx, ly in [(1, 1), (7, 3), (64, 64), (65, 130), (333, 512), (700, 650)]:
        x, y = mv_series(rng, lx, D), mv_series(rng, ly, D)
        d = orc.dp(p, x, y)
        xd, yd = to_dev(torch, dev, x), to_dev(torch, dev, y)
        for c in [INF] + ([d, float(np.nextafter(d, -INF)), 0.5 * d] if 0 < d < INF else []):
            log(f"multivariate distance {pid(p)} lx={lx} ly={ly} cut={c}")
            g = float(eap.distance(xd, yd, p, c).item())
            want = d if d <= c else INF
            assert g == want or (math.isinf(g) and math.isinf(want)), (lx, ly, c, g, want)


@pytest.mark.parametrize("p", MV, ids=pid)
def test_multivariate_nn_and_pairwise_parity(torch_dev, orc, p):
    torch, dev = torch_dev
    D = p["dims"]
    rng = np.random.default_rng(95 + D)
    qs = [mv_series(rng, int(L), D) for L in rng.integers(20, 300, size=6)]
    rs = [mv_series(rng, int(L), D) for L in rng.integers(15, 320, size=70)]
    rs[5] = qs[2].copy()
    qv, rv = np.concatenate(qs), np.concatenate(rs)
    qo = np.concatenate([[0], np.cumsum([len(x) // D for x in qs])]).astype(np.int64)
    ro = np.concatenate([[0], np.cumsum([len(x) // D for x in rs])]).astype(np.int64)
    q, r = to_dev(torch, dev, qv), to_dev(torch, dev, rv)
    oi, od, _ = orc.nn1(p, qv, qo, rv, ro, "dp")
    for precision, flags in ((0, 0), (1, 0), (0, eap.FLAG_PRUNE_ONLY), (0, eap.FLAG_NO_PRUNE), (0, eap.FLAG_PLAIN)):
        log(f"multivariate nn {pid(p)} precision={precision} flags={flags}")
        gi, gd, _ = eap.nn1(q, qo, r, ro, p, precision=precision, flags=flags)
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), oi) and np.array_equal(gd.cpu().numpy(), od), (precision, flags)
    sv = np.concatenate(rs[:25])
    so = ro[:26]
    want = orc.pairwise(p, sv, so, "full")
    for mode in ("prune", "full"):
        log(f"multivariate pairwise {pid(p)} {mode}")
        g = eap.pairwise(to_dev(torch, dev, sv), so, p, mode=mode)
        torch.cuda.synchronize()
        assert np.array_equal(g.cpu().numpy(), want), mode
