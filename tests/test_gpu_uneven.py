"""The uneven job mix on the GPU: sources of log-uniform length, 1..8
directions x 2 ears each, in one launch.  Checked against the FP64 oracle
row by row; persistent, graph-captured and autotuned launch shapes must give
the same bits as the default launch."""
import json
import os

import numpy as np
import pytest

import fp32bound
import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def test_uneven_mix_parity_and_shapes(dev, tmp_path):
    import torch
    import paper_1502_03162_amd as H
    n_src, F, K, lf, lg = 40, 60, 16, 32, 169
    lens = synth.uneven_lengths(301, n_src, 4096, 1 << 17)
    jr = synth.jobs_uneven(302, n_src, F // 2)
    jobs = [(int(a), int(b)) for a, b in jr]
    rng = np.random.default_rng(5)
    r = rng.standard_normal(lf).astype(np.float32)
    p, g = synth.random_taps(6, F, K, lg, nnz_min=12)
    plan = H.Plan(r, p, g, lg)
    srcs = [synth.pink(500 + i, int(n)) for i, n in enumerate(lens)]
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs)).to(dev)
    out_off, total = H.row_layout(plan, lens, jobs)
    rows_j = [(s, f, o) for (s, f), o in zip(jobs, out_off)]

    def render(**kw):
        out = torch.full((total,), float("nan"), dtype=torch.float32, device=dev)
        b = H.Batch(plan, off, lens, rows_j, **kw)
        for _ in range(2):
            b.render(src, out)
        torch.cuda.synchronize()
        b.close()
        return out.cpu().numpy()

    base = render()
    refs = oracle.sparse_render_jobs(r, np.concatenate(srcs), off, lens, p, g, lg, np.asarray(jobs, np.int32))
    worst = max(oracle.rel_l2(base[o:o + ref.size], ref) for o, ref in zip(out_off, refs))
    assert worst <= TOL, worst
    for kw in (dict(flags=H.SPCONV_PERSISTENT | H.SPCONV_GRAPH), dict(tile=4096, group=4),
               dict(tile=1024, group=16, flags=H.SPCONV_PERSISTENT)):
        assert np.array_equal(render(**kw), base, equal_nan=True), kw

    cache = str(tmp_path / "tune.json")
    scratch = torch.zeros(total, dtype=torch.float32, device=dev)
    best = H.autotune(plan, src, off, lens, rows_j, scratch, cache_path=cache)
    assert best["tile"] in (1024, 2048, 3072, 4096) and best["group"] in (0, 4, 8, 16) and best["ms"] > 0
    stored = json.load(open(cache))
    assert len(stored) == 1 and list(stored.values())[0][:3] == [best["tile"], best["group"], best["flags"]]
    again = H.autotune(plan, src, off, lens, rows_j, scratch, cache_path=cache)   # served from the cache
    assert {k: again[k] for k in ("tile", "group", "flags")} == {k: best[k] for k in ("tile", "group", "flags")}
    assert abs(again["ms"] - best["ms"]) <= 1e-9 * best["ms"]
    pers = H.autotune(plan, src, off, lens, rows_j, scratch, cache_path=cache, force_flags=H.SPCONV_PERSISTENT)
    assert pers["flags"] & H.SPCONV_PERSISTENT
    assert len(json.load(open(cache))) == 2
    assert np.array_equal(render(tile=best["tile"], group=best["group"], flags=best["flags"] | H.SPCONV_GRAPH),
                          base, equal_nan=True)


def test_full_size_uneven_config_sampled(dev):
    """The uneven workload at full size in the benchmark's launch form (one
    persistent launch replayed from a HIP graph, tile 3072): 512 pink
    sources of log-uniform length in [4096, 1048576], 1..8 directions x 2
    ears of a 1,250-direction tap table, K = 16; sampled outputs of 64 rows
    against the oracle's per-sample definition, with every row's first and
    last samples."""
    import torch
    import paper_1502_03162_amd as H
    n_src, F, K, lf, lg = 512, 2500, 16, 32, 169
    lens = synth.uneven_lengths(300, n_src)
    jobs = [(int(a), int(b)) for a, b in synth.jobs_uneven(300, n_src, F // 2)]
    rng = np.random.default_rng(7)
    r = rng.standard_normal(lf).astype(np.float32)
    p, g = synth.random_taps(8, F, K, lg, nnz_min=12)
    plan = H.Plan(r, p, g, lg)
    srcs = [synth.pink(1000 + i, int(n)) for i, n in enumerate(lens)]
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs)).to(dev)
    out_off, total = H.row_layout(plan, lens, jobs)
    out = torch.full((total,), float("nan"), dtype=torch.float32, device=dev)
    b = H.Batch(plan, off, lens, [(s, f, o) for (s, f), o in zip(jobs, out_off)], tile=3072,
                flags=H.SPCONV_PERSISTENT | H.SPCONV_GRAPH)
    for _ in range(2):                                   # the graph is replayed
        b.render(src, out)
    torch.cuda.synchronize()
    got, ref = [], []
    for j in rng.choice(len(jobs), size=64, replace=False):
        s, f = jobs[j]
        L = plan.out_len(lens[s])
        t = np.unique(np.concatenate([[0, 1, L - 1], rng.integers(0, L, 45)]))
        gj = out[torch.from_numpy(out_off[j] + t).to(dev)].cpu().numpy()
        rj = oracle.sparse_render_points(r, srcs[s], p[f], g[f].astype(np.float64), t)
        # every sample within the FP32 bound of its own fma chains
        assert np.all(np.abs(gj - rj) <= fp32bound.render_bound(r, srcs[s], p[f], g[f], t, K)), (j, s, f)
        got.append(gj)
        ref.append(rj)
    got, ref = np.concatenate(got), np.concatenate(ref)
    assert np.all(np.isfinite(got))
    assert oracle.rel_l2(got, ref) <= TOL
    b.close()
    plan.close()
    del out, src
    torch.cuda.empty_cache()
