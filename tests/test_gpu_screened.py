"""The screened split forms: a one-product BF16 screen over every tile (on all
coordinates for BF16X3S, on the first 64 for BF16X3P), the split form over the
tiles it cannot rule out.

Against the oracle on sampled rows at sizes where the screen flags some tiles
and passes others, against the unscreened split form (BF16X3G) everywhere, and
through the tile windows of a source range longer than 64 tiles (one split).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev, host, next_version

pytestmark = pytest.mark.gpu

yy = pytest.importorskip("paper_2509_16896_amd.yy")


@pytest.fixture(scope="module")
def ctx():
    c = yy.yy_create(0, torch.cuda.current_stream())
    yield c
    yy.yy_destroy(c)


def _case(r, n, q, dt, half, seed, scales=(1.0, 2.0, 4.0), stripes=0, zero_every=0):
    rng = np.random.default_rng(seed)
    lo, hi = -half * np.ones(r), half * np.ones(r)
    codes = oracle.sobol_codes(r, n, 0, True, seed)
    x = oracle.codes_to_points(codes, lo, hi)
    lw = -3.0 * rng.random(n) - 0.5 * np.sum((x / half) ** 2, axis=1)
    if stripes:
        # every other run of `stripes` nodes 3000 below the rest: the screen rules out the tiles
        # of heavy targets against light sources and keeps the others, an irregular tile pattern
        lw -= 3000.0 * ((np.arange(n) // stripes) % 2)
    if zero_every:
        # nodes of weight zero: as targets they still receive mass, and their self pair gives no
        # lower bound of their row maximum
        lw[::zero_every] = -np.inf
    gm = yy.Model(r, r, yy.YY_F_COS, None, yy.YY_H_IDENTITY, None, 0.0, q, 1.0)
    om = oracle.OModel(r, r, oracle.F_COS, None, oracle.H_IDENTITY, None, 0.0, q, 1.0)
    return dict(r=r, n=n, x=x, lo=lo, hi=hi, lw=lw, gm=gm, om=om, dt=dt, scales=scales)


def _run(ctx, c, prec):
    out = torch.empty(c["n"], dtype=torch.float64, device="cuda")
    yy.yy_propagate(ctx, c["gm"], yy.Scales(c["scales"]), prec, c["n"], dev(c["x"].ravel()), next_version(),
                    dev(c["lo"]), dev(c["hi"]), c["dt"], dev(c["lw"]), out)
    return host(out)


# Kernel widths from "every tile holds near pairs" to "only the self pairs are near";
# n spans several 256-target blocks and 128-source tiles with a ragged tail.
CASES = {
    "r64_n4000_wide": dict(r=64, n=4000, q=2.0, dt=0.05, half=0.25, seed=41),
    "r96_n6000_mid": dict(r=96, n=6000, q=0.3, dt=0.02, half=0.3, seed=42),
    "r200_n5000_narrow": dict(r=200, n=5000, q=0.09, dt=0.005, half=0.3, seed=43),
    "r33_n3000_s1": dict(r=33, n=3000, q=0.5, dt=0.02, half=0.5, seed=44),
    # a partial screen over source ranges longer than a 64-tile window (16 splits of 69 tiles)
    "r32_n140000_stripes": dict(r=32, n=140000, q=1.0, dt=0.05, half=0.25, seed=45, stripes=2560),
    "r100_n3000_zero_weights": dict(r=100, n=3000, q=0.3, dt=0.02, half=0.3, seed=46, zero_every=7),
    # more than 32 target blocks and r > 32: BF16X3P's symmetric screen (each pair of target blocks once,
    # the transposed orientation by a coarse bound per 64 rows), with a ragged last block and tile
    "r100_n12000_mid_sym": dict(r=100, n=12000, q=0.3, dt=0.02, half=0.3, seed=48),
    "r64_n20000_wide_sym": dict(r=64, n=20000, q=2.0, dt=0.05, half=0.25, seed=49),
    "r200_n8500_narrow_sym": dict(r=200, n=8500, q=0.09, dt=0.005, half=0.3, seed=50, zero_every=11),
    "r48_n9000_stripes_sym": dict(r=48, n=9000, q=1.0, dt=0.05, half=0.25, seed=51, stripes=640),
    # wide kernels over 547 target blocks: every group of the transposed orientation is doubted, about
    # 2.4 million units against a list of 2^20, so the groups past the list's end are flagged directly
    "r64_n140000_wide_sym": dict(r=64, n=140000, q=2.0, dt=0.05, half=0.25, seed=53),
    # the smallest n with 33 target blocks: the last block holds one node and one source tile
    "r40_n8193_edge_sym": dict(r=40, n=8193, q=0.5, dt=0.02, half=0.4, seed=54),
    # r <= 32 (a screen over 32 coordinates) keeps the one-sided screen at any size
    "r32_n9000_stripes": dict(r=32, n=9000, q=1.0, dt=0.05, half=0.25, seed=52, stripes=640),
}


@pytest.mark.parametrize("form", ["bf16x3s", "bf16x3p"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_screened_matches_split_form_and_oracle_rows(ctx, name, form):
    c = _case(**CASES[name])
    got = _run(ctx, c, form)
    ref = _run(ctx, c, "bf16x3g")
    f = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), f)
    # both forms keep every pair within 2^-80 of a row maximum exactly: they agree to FP32 rounding
    rel = np.abs(got[f] - ref[f]) / np.maximum(1.0, np.abs(ref[f]))
    print(f"{name}: max |{form} - x3g| / max(1, |x3g|) = {rel.max():.3g}")
    assert rel.max() < 2e-6
    assert np.array_equal(_run(ctx, c, form), got)   # deterministic
    flagged, tiles = yy.yy_screen_count(ctx)
    n = c["n"]
    assert tiles == ((n + 255) // 256) * ((n + 127) // 128)
    assert 0 <= flagged <= tiles
    print(f"{name}: {form} screen flagged {flagged} of {tiles} tiles")
    if "stripes" in CASES[name]:
        assert 0.2 * tiles < flagged < 0.9 * tiles
    # sampled rows against the oracle
    rng = np.random.default_rng(1)
    rows = np.unique(np.concatenate([[0, c["n"] - 1], rng.choice(c["n"], 24, replace=False)]))
    s = np.asarray(c["scales"])
    lo = oracle.propagate_rows(c["om"], s, oracle.kernel_coefficients(s), c["x"], c["lo"], c["hi"], c["dt"],
                               c["lw"], rows)[0]
    g = got[rows]
    ok = np.isfinite(lo)
    assert np.array_equal(np.isfinite(g), ok)
    z = np.log(np.sum(np.exp(got[f] - np.max(got[f])))) + np.max(got[f])
    err = np.abs(g[ok] - lo[ok]) / np.maximum(1.0, np.abs(lo[ok] - z))
    assert err.max() <= 1e-5, (name, err.max())


def test_screen_count_needs_a_screened_run():
    c = yy.yy_create(0, torch.cuda.current_stream())
    try:
        with pytest.raises(yy.YYError):
            yy.yy_screen_count(c)
    finally:
        yy.yy_destroy(c)


def test_screened_long_source_range_windows(ctx):
    """One source split of 160 tiles (three windows of the filtered pass, the last one
    ragged), through the batch call's split cap, against the single-run call."""
    from paper_2509_16896_amd import workloads as W
    from paper_2509_16896_amd.batch import Batch
    from paper_2509_16896_amd.filter import GpuFilter
    w = W.Workload("win_r64_n20480", r=64, n=20480, dt=0.01, K=2, drift=W.F_COS, obs=W.H_CUBE, q=0.09, rho2=0.09,
                   scales=(1.0, 2.0, 4.0), box_half=0.6, restart_every=2, R=0.3, seed=5)
    dys = W.simulate(w)[1]
    b = Batch([w], [dys], prec="bf16x3s", max_split=1)
    try:
        for _ in range(w.K):
            b.step()
        got = [host(t) for t in b.results(0)]
    finally:
        b.close()
    f = GpuFilter(w, prec="bf16x3s")
    try:
        f.set_observations(dys)
        f.init()
        for k in range(1, w.K + 1):
            f.step(k)
        ref = [host(f.hist), host(f.logZ_hist), host(f.ess_hist)]
    finally:
        f.close()
    for a, r in zip(got, ref):
        assert np.all(np.isfinite(a))
        # another split count changes only the summation order of the partial sums
        assert np.allclose(a, r, rtol=1e-9, atol=1e-9)


def test_deferred_planes_across_calls_on_one_node_set():
    """BF16X3P on one run writes the planes beyond its screen's first 64 coordinates only
    once the screen flags a tile for the node set.  Calls on one node set (same device array
    and version): source weights that flag no tile, then weights that flag some (the planes
    are written), then other flagging weights (the planes are reused), then a new node set
    in the same array under a new version (written again); each against the split form
    BF16X3G on another context."""
    c = _case(**CASES["r200_n5000_narrow"])
    n = c["n"]
    # light stripes far below the gap to their nearest neighbour (about 2e4 bits at this
    # kernel width): their rows' maxima come from heavy sources, so their tiles are flagged
    stripe = lambda w: 1e5 * ((np.arange(n) // w) % 2)
    seq = [(0, c["lw"]), (0, c["lw"] - stripe(640)), (0, c["lw"] - stripe(384)), (1, c["lw"] - stripe(640))]
    c1 = _case(**dict(CASES["r200_n5000_narrow"], seed=47))
    xs = [c["x"], c1["x"]]
    a = yy.yy_create(0, torch.cuda.current_stream())
    b = yy.yy_create(0, torch.cuda.current_stream())
    try:
        x = dev(xs[0].ravel())
        lo, hi = dev(c["lo"]), dev(c["hi"])
        versions = [next_version(), next_version()]
        counts = []
        for node_set, lw in seq:
            if node_set == 1:
                x.copy_(dev(xs[1].ravel()))
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            yy.yy_propagate(a, c["gm"], yy.Scales(c["scales"]), "bf16x3p", n, x, versions[node_set], lo, hi,
                            c["dt"], dev(lw), out)
            got = host(out)
            counts.append(yy.yy_screen_count(a)[0])
            ref_out = torch.empty(n, dtype=torch.float64, device="cuda")
            yy.yy_propagate(b, c["gm"], yy.Scales(c["scales"]), "bf16x3g", n, dev(xs[node_set].ravel()),
                            next_version(), dev(c["lo"]), dev(c["hi"]), c["dt"], dev(lw), ref_out)
            ref = host(ref_out)
            f = np.isfinite(ref)
            assert np.array_equal(np.isfinite(got), f)
            rel = np.abs(got[f] - ref[f]) / np.maximum(1.0, np.abs(ref[f]))
            assert rel.max() < 2e-6, (len(counts), counts[-1], rel.max())
        print(f"flagged tiles per call: {counts}")
        assert counts[0] == 0 and min(counts[1:]) > 0
    finally:
        yy.yy_destroy(a)
        yy.yy_destroy(b)


# A posterior collapsed onto one node j*: every other weight lies far below, so each row's maximum is
# its pair with j* (the self pair lies far below it). The row floor counts that pair exactly at
# initialisation and leaves it out of the tiles, so the screens flag no tile; j* in an inner tile, in
# the ragged last tile, and where it shares a tile with the self pairs of a target block.
COLLAPSED = {
    "r100_n3000_jstar_inner": dict(r=100, n=3000, q=0.5, dt=0.02, half=0.3, seed=51, jstar=1300),
    "r64_n9000_jstar_tail": dict(r=64, n=9000, q=1.0, dt=0.02, half=0.3, seed=52, jstar=8997),
    "r200_n2000_jstar_first": dict(r=200, n=2000, q=1.0, dt=0.01, half=0.3, seed=53, jstar=0),
}


@pytest.mark.parametrize("name", sorted(COLLAPSED))
def test_collapsed_posterior_flags_no_tile(ctx, name):
    kw = dict(COLLAPSED[name])
    jstar = kw.pop("jstar")
    c = _case(**kw)
    n = c["n"]
    rng = np.random.default_rng(kw["seed"])
    lw = -1e6 - 1e3 * rng.random(n)
    lw[jstar] = 0.0
    c["lw"] = lw
    s = np.asarray(c["scales"])
    ref = oracle.propagate(c["om"], s, oracle.kernel_coefficients(s), c["x"], c["lo"], c["hi"], c["dt"], lw)[0]
    from gpu_util import compare_logw
    g3 = _run(ctx, c, "bf16x3g")
    for form in ("bf16x3p", "bf16x3s"):
        got = _run(ctx, c, form)
        flagged, tiles = yy.yy_screen_count(ctx)
        print(f"{name}: {form} flagged {flagged} of {tiles} tiles")
        assert flagged == 0
        f = np.isfinite(g3)
        assert np.array_equal(np.isfinite(got), f)
        assert np.max(np.abs(got[f] - g3[f]) / np.maximum(1.0, np.abs(g3[f]))) < 2e-6
        worst, cnt = compare_logw(got, ref, 1e-5)
        print(f"{name}: {form} worst err/allowed = {worst:.3g} over {cnt} nodes")
        assert worst <= 1.0
        # every row's value is dominated by its pair with j*: against the oracle on all rows
        fr = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got), fr)
        assert np.max(np.abs(got[fr] - ref[fr]) / np.maximum(1.0, np.abs(ref[fr]))) < 1e-5
