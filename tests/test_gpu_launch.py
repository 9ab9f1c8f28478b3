"""Launch machinery of the batched path: HIP-graph capture and replay of the
forward launch (qs_set_graphs) and the launch tuner with its cache
(qs_tune).  Neither may change a result bit: graph replays are compared with
eager launches of the same arguments, several times, with other eager work
and synchronisations between them; tuned launches with untuned ones.
"""
import numpy as np
import pytest

from paper_2308_09348_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09348_amd as qs
    return qs


def _np(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def _same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), (what, k)


def _case(**kw):
    p = workloads.scaled(workloads.focused_3d(), n_samples=9037, n_steps=256)
    p.update(kw)
    return p


def test_graph_replays_match_eager(qs):
    import torch
    eager = qs.Context(0)
    graph = qs.Context(0)
    graph.set_graphs(True)
    p = _case()
    other = _case(n_samples=3000, n_steps=128, rr_model="classical")
    ref = _np(eager.forward(p))
    for r in range(4):
        got = _np(graph.forward(p))
        _same(got, ref, f"replay {r}")
        # eager work on the same context and on torch between the replays
        eager.forward(other)
        torch.cuda.synchronize()
        x = torch.arange(1 << 20, device="cuda", dtype=torch.float64).sum()
        assert x.item() > 0
    # new per-shot parameters, same shapes: the replay copies the new shot table
    q = dict(p, a0=37.0, x_off_um=-1.0, gamma0=2300.0)
    _same(_np(graph.forward(q)), _np(eager.forward(q)), "new parameters")
    # another class of launch on the graph context is captured separately
    _same(_np(graph.forward(other)), _np(eager.forward(other)), "second graph")
    _same(_np(graph.forward(p)), ref, "first graph again")
    eager.close()
    graph.close()


def test_graph_replays_match_eager_batched(qs):
    eager = qs.Context(0)
    graph = qs.Context(0)
    graph.set_graphs(True)
    shots = [_case(n_samples=n, a0=a, shot=0) for n, a in ((5000, 20.0), (777, 60.0),
                                                           (12001, 45.0))]
    shots = [dict(s, chi_fp64=0.1) for s in shots]
    ref = [_np(o) for o in eager.forward_batched(shots)]
    for r in range(3):
        got = [_np(o) for o in graph.forward_batched(shots)]
        for k in range(len(shots)):
            _same(got[k], ref[k], f"replay {r} shot {k}")
        eager.forward(shots[1])
    eager.close()
    graph.close()


def test_tuner_choice_cache_and_results(qs, tmp_path):
    p = _case(n_samples=1 << 17, n_steps=128)
    plain = qs.Context(0)
    ref = _np(plain.forward(p))
    tuned = qs.Context(0)
    cache = tmp_path / "tune.txt"
    t = tuned.tune(p, cache_path=str(cache))
    assert not t["from_cache"]
    assert t["dep_tile"] in (1024, 2048, 4096, 8192)
    assert t["phase_cap"] in (0, 2, 3) and t["dep_cap"] in (0, 2, 4)
    assert 0 < t["phase_ms"] < 1e3 and 0 < t["deposit_ms"] < 1e3
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("qscatter-tune-1 ")
    # the tuned launch gives the untuned bits
    _same(_np(tuned.forward(p)), ref, "tuned")
    # a new context reads the choice from the cache
    again = qs.Context(0)
    u = again.tune(p, cache_path=str(cache))
    assert u["from_cache"]
    assert (u["dep_tile"], u["phase_cap"], u["dep_cap"]) == (t["dep_tile"], t["phase_cap"],
                                                             t["dep_cap"])
    assert len(cache.read_text().splitlines()) == 1
    _same(_np(again.forward(p)), ref, "from cache")
    for c in (plain, tuned, again):
        c.close()


@pytest.mark.parametrize("tile", [1024, 8192])
def test_deposit_tile_leaves_results_unchanged(qs, tmp_path, tile):
    """A cache line forcing each extreme tile (and capped residency): the
    moments are summed per 1024-sample tile whatever the deposit item."""
    import re
    p = _case(n_samples=50001, deposit="gauss")
    plain = qs.Context(0)
    ref = _np(plain.forward(p))
    probe = qs.Context(0)
    cache = tmp_path / "tune.txt"
    probe.tune(p, cache_path=str(cache))
    line = cache.read_text().split()
    # replace the choice (fields 10-12 after the tag) with the forced one
    line[10:13] = [str(tile), "2", "2"]
    cache.write_text(" ".join(line) + "\n")
    forced = qs.Context(0)
    u = forced.tune(p, cache_path=str(cache))
    assert u["from_cache"] and u["dep_tile"] == tile and u["dep_cap"] == 2
    _same(_np(forced.forward(p)), ref, f"tile {tile}")
    assert re.match(r"qscatter-tune-1 \S+/\d+ ", cache.read_text())
    for c in (plain, probe, forced):
        c.close()


def test_tuner_on_a_batch(qs, tmp_path):
    """The class of a batch (shot count and total samples) is tuned as a
    whole; the tuned batched launch, replayed from a graph, gives the bits of
    the plain one."""
    shots = [_case(n_samples=n, a0=a) for n, a in ((3000, 15.0), (20000, 50.0), (9000, 80.0),
                                                   (1, 30.0))]
    plain = qs.Context(0)
    ref = [_np(o) for o in plain.forward_batched(shots)]
    tuned = qs.Context(0)
    cache = tmp_path / "tune.txt"
    t = tuned.tune(shots, cache_path=str(cache))
    assert not t["from_cache"] and t["dep_tile"] in (1024, 2048, 4096, 8192)
    key = cache.read_text().split()
    assert key[9] == "2"  # floor(log2 4 shots)
    tuned.set_graphs(True)
    for r in range(2):
        got = [_np(o) for o in tuned.forward_batched(shots)]
        for k in range(len(shots)):
            _same(got[k], ref[k], f"tuned batch, launch {r}, shot {k}")
    plain.close()
    tuned.close()


def test_graph_replays_follow_the_shadow_stride(qs):
    """The FP64-shadow launches of a captured batch take their item count from
    shadow_stride: a new stride that leaves every buffer size unchanged
    (16384 and 6400 samples, stride 64 then 63) must be captured anew, not
    replayed with the old count."""
    eager = qs.Context(0)
    graph = qs.Context(0)
    graph.set_graphs(True)
    base = [_case(n_samples=n, a0=a, shot=0, validate_fp64=True)
            for n, a in ((16384, 30.0), (6400, 45.0))]
    for stride in (64, 63, 64):
        shots = [dict(s, shadow_stride=stride) for s in base]
        ref = [_np(o) for o in eager.forward_batched(shots)]
        for r in range(2):
            got = [_np(o) for o in graph.forward_batched(shots)]
            for k in range(len(shots)):
                _same(got[k], ref[k], f"stride {stride} replay {r} shot {k}")
    eager.close()
    graph.close()


def test_profiled_calls_are_kept_for_the_sum(qs):
    """Kernel events are kept per profiled call (a ring of 64 sets): the sum
    over calls enqueued back to back equals the per-call durations read one
    by one, only the last 64 calls are summed, and profiled launches are
    never graph replays."""
    ctx = qs.Context(0)
    p = _case(n_samples=4000, n_steps=64)
    out = ctx.forward(p)
    with pytest.raises(qs.QScatterError):
        ctx.timings_sum()  # profiling off
    ctx.set_profiling(True)
    with pytest.raises(qs.QScatterError):
        ctx.timings_sum()  # no profiled call yet
    each = []
    for _ in range(3):
        ctx.forward(p, out=out, check=False)
        each.append(ctx.last_timings())
    n, tot = ctx.timings_sum()
    assert n == 3
    for k in tot:
        assert tot[k] == pytest.approx(sum(t[k] for t in each), rel=1e-12, abs=1e-9)
    assert tot["phase"] > 0 and tot["deposit"] > 0
    # back to back, read once: the ring keeps the last 64
    for _ in range(70):
        ctx.forward(p, out=out, check=False)
    n, tot = ctx.timings_sum()
    assert n == 64 and tot["phase"] > 0
    last = ctx.last_timings()
    assert 0 < last["phase"] <= tot["phase"]
    # switching profiling on again starts a new count
    ctx.set_profiling(True)
    ctx.forward(p, out=out, check=False)
    assert ctx.timings_sum()[0] == 1
    # profiled launches are not captured into graphs: they stay eager and count
    ctx.set_graphs(True)
    ctx.forward(p, out=out, check=False)
    ctx.forward(p, out=out, check=False)
    assert ctx.timings_sum()[0] == 3
    ctx.close()
