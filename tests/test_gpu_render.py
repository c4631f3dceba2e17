"""GPU parity of the fused sparse renderer against the FP64 oracle.

Bar: relative L2 error <= 1e-5 per output row (FP32 kernels vs FP64 oracle
on the same float32 inputs).  Launch variants (tile size, job grouping,
persistent, unfused, graph replay, batch mixing) must agree bitwise, since
every output is summed in one fixed order."""
import numpy as np
import pytest

import fp32bound
import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def H():
    import paper_1502_03162_amd
    return paper_1502_03162_amd


def render_rows(plan, srcs, jobs_sf, dev, tile=0, group=0, flags=0, reps=1):
    """Render (src, filt) jobs through a Batch; returns host rows."""
    import torch
    h = H()
    lens = np.array([len(s) for s in srcs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs).astype(np.float32)).to(dev)
    out_off, total = h.row_layout(plan, lens, jobs_sf)
    out = torch.full((total + 64,), float("nan"), dtype=torch.float32, device=dev)
    b = h.Batch(plan, off, lens, [(s, f, o) for (s, f), o in zip(jobs_sf, out_off)], tile=tile, group=group,
                flags=flags)
    for _ in range(reps):
        b.render(src, out)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    rows = [host[o:o + plan.out_len(lens[s])] for (s, _), o in zip(jobs_sf, out_off)]
    # nothing outside the rows is written
    mask = np.ones(host.size, dtype=bool)
    for (s, _), o in zip(jobs_sf, out_off):
        mask[o:o + plan.out_len(lens[s])] = False
    assert np.all(np.isnan(host[mask]))
    b.close()
    return rows


def oracle_rows(r, srcs, p, g, lg, jobs_sf):
    lens = [len(s) for s in srcs]
    off = np.concatenate([[0], np.cumsum(lens)[:-1]])
    return oracle.sparse_render_jobs(np.asarray(r, np.float32), np.concatenate(srcs).astype(np.float32), off,
                                     lens, p, np.asarray(g, np.float32), lg, np.asarray(jobs_sf, np.int32))


def check(rows, refs):
    worst = 0.0
    for row, ref in zip(rows, refs):
        assert row.shape == ref.shape
        assert np.all(np.isfinite(row))
        e = oracle.rel_l2(row, ref)
        worst = max(worst, e)
    assert worst <= TOL, worst
    return worst


def test_config0_end_to_end(dev):
    """Small configuration: 50 directions x 2 ears, one white source of
    65,536 samples, factorized with lf = 32 and K = 16, all 100 filters."""
    h = H()
    hs = synth.hrir_set(0, 5, 10)
    fac = h.factorize(hs.h, 32, 600, 16, seed=7, lambda0=0.2, want_cost=False)
    r = fac["f"].astype(np.float32)
    plan = h.Plan(r, fac["p"], fac["g"], 169)
    s = synth.white(0, 65536)
    jobs = [(0, f) for f in range(100)]
    rows = render_rows(plan, [s], jobs, dev)
    worst = check(rows, oracle_rows(r, [s], fac["p"], fac["g"], 169, jobs))
    print(f"config0 worst rel L2 {worst:.3e}", flush=True)


@pytest.mark.parametrize("kernel", ["quad", "quad256", "lds_gather", "regwin"])
@pytest.mark.parametrize("lf,lg,k", [(32, 169, 16), (1, 1, 1), (5, 2, 2), (17, 40, 3), (33, 300, 32),
                                     (64, 2048, 64), (16, 169, 8), (32, 169, 64), (64, 169, 33)])
def test_ragged_lengths_and_shapes(dev, lf, lg, k, kernel):
    h = H()
    rng = np.random.default_rng(lf * 1000 + lg + k)
    r = rng.standard_normal(lf).astype(np.float32)
    F = 7
    kk = min(k, lg)
    p, g = synth.random_taps(lf + lg + k, F, kk, lg, nnz_min=1)
    # force both extreme positions into the table
    p[0, 0], p[1, kk - 1] = 0, lg - 1
    g[0, 0], g[1, kk - 1] = 1.0, 0.5
    lens = [1, 2, 31, 199, 1023, 1024, 1025, 4095, 4096, 4097, 8191, 10000]
    srcs = [synth.white(100 + i, n) for i, n in enumerate(lens)]
    jobs = [(i, (i + j) % F) for i in range(len(lens)) for j in range(2)]
    plan = h.Plan(r, p, g, lg)
    if kernel == "regwin" and lg > 169:
        # the register-window kernel serves lg <= 169: it refuses longer
        # filters before any device work (the default kernel renders them)
        lens = np.array([len(x) for x in srcs], dtype=np.int64)
        off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
        with pytest.raises(h.HrirError) as e:
            h.Batch(plan, off, lens, [(0, 0, 0)], flags=h.SPCONV_REGWIN)
        assert e.value.code == h.HRIR_EINVAL and "lg <=" in str(e.value)
        plan.close()
        return
    flags = {"quad": 0, "quad256": h.SPCONV_WG256, "lds_gather": h.SPCONV_LDS_GATHER,
             "regwin": h.SPCONV_REGWIN}[kernel]
    # 256-thread workgroups cover tile + lg + 2 <= 4096 z values: at lg = 2048
    # the largest tile they take is 1024
    tile = 1024 if kernel == "quad256" and lg > 2048 - 2 else 0
    rows = render_rows(plan, srcs, jobs, dev, flags=flags, tile=tile)
    check(rows, oracle_rows(r, srcs, p, g, lg, jobs))


def test_largest_tile_and_longest_filter(dev):
    """The default kernel at its limits: tile 4096 (the largest), lg = 2048
    (the longest reflection filter a plan takes), K = 64 and lf = 64, so one
    tile's z window spans 6,143 samples in four LDS copies (98 KB); plain
    and persistent launches against the oracle, and bitwise against each
    other and the default tile."""
    h = H()
    rng = np.random.default_rng(2048)
    lf, lg, k, F = 64, 2048, 64, 5
    r = rng.standard_normal(lf).astype(np.float32)
    p, g = synth.random_taps(77, F, k, lg, nnz_min=k)
    p[0, 0], p[1, k - 1] = 0, lg - 1
    srcs = [synth.white(300 + i, n) for i, n in enumerate([1, 4095, 4097, 12289])]
    jobs = [(i, (2 * i + j) % F) for i in range(len(srcs)) for j in range(3)]
    plan = h.Plan(r, p, g, lg)
    base = render_rows(plan, srcs, jobs, dev, tile=4096)
    check(base, oracle_rows(r, srcs, p, g, lg, jobs))
    for v in (dict(tile=4096, flags=h.SPCONV_PERSISTENT, reps=2), dict(), dict(tile=1024)):
        rows = render_rows(plan, srcs, jobs, dev, **v)
        for a, b in zip(rows, base):
            assert np.array_equal(a, b), v


def _variant_setup(seed=0):
    h = H()
    rng = np.random.default_rng(seed)
    lf, lg, k, F = 32, 169, 16, 12
    r = rng.standard_normal(lf).astype(np.float32)
    p, g = synth.random_taps(seed + 1, F, k, lg, nnz_min=4)
    lens = [3000, 17, 40000, 4096, 12345]
    srcs = [synth.pink(200 + i, n) for i, n in enumerate(lens)]
    jobs = [(i, (3 * i + j) % F) for i in range(len(lens)) for j in range(2 + i)]
    return h.Plan(r, p, g, lg), r, p, g, lg, srcs, jobs


def test_launch_variants_bitwise_identical(dev):
    h = H()
    plan, r, p, g, lg, srcs, jobs = _variant_setup()
    base = render_rows(plan, srcs, jobs, dev)
    check(base, oracle_rows(r, srcs, p, g, lg, jobs))
    L, R, PS, W = h.SPCONV_LDS_GATHER, h.SPCONV_REGWIN, h.SPCONV_PERSISTENT, h.SPCONV_WG256
    variants = [dict(tile=1024), dict(tile=2048), dict(tile=3072), dict(group=1), dict(group=3),
                dict(flags=PS), dict(flags=PS, tile=2048, reps=3),
                dict(flags=W), dict(flags=W, tile=1024), dict(flags=W, tile=3072), dict(flags=W, group=3),
                dict(flags=W | PS, reps=3), dict(flags=W | PS, tile=1024, reps=3),
                dict(flags=L), dict(flags=L, tile=1024), dict(flags=L, tile=8192), dict(flags=L, tile=16384),
                dict(flags=L, group=3), dict(flags=L | PS), dict(flags=L | PS, tile=2048, reps=3),
                dict(flags=R), dict(flags=R, tile=12288), dict(flags=R, group=3), dict(flags=R | PS, reps=3),
                dict(flags=h.SPCONV_UNFUSED)]
    for v in variants:
        rows = render_rows(plan, srcs, jobs, dev, **v)
        for a, b in zip(rows, base):
            assert np.array_equal(a, b), v


def test_lds_and_direct_stages_bitwise_identical(dev):
    """Tiles with many jobs stage the source window in LDS; batches whose
    tiles all have few jobs, and the persistent kernel, read the FIR windows
    from global memory.  Both form the same z, so the rows agree bit for bit
    (30 jobs per source: the one-tile kernel takes the LDS stage; group=3 and
    the persistent launch take the direct one), also at sources shorter than
    a tile and on tiles that reach past either end of the source."""
    h = H()
    rng = np.random.default_rng(5)
    lf, lg, k, F = 32, 169, 16, 40
    r = rng.standard_normal(lf).astype(np.float32)
    p, g = synth.random_taps(6, F, k, lg, nnz_min=4)
    lens = [9000, 100, 5000]
    srcs = [synth.pink(300 + i, n) for i, n in enumerate(lens)]
    jobs = [(i, (7 * i + j) % F) for i in range(len(lens)) for j in range(30)]
    plan = h.Plan(r, p, g, lg)
    base = render_rows(plan, srcs, jobs, dev)
    check(base, oracle_rows(r, srcs, p, g, lg, jobs))
    PS, W = h.SPCONV_PERSISTENT, h.SPCONV_WG256
    for v in (dict(group=3), dict(flags=PS), dict(group=3, flags=PS), dict(flags=W, group=3), dict(tile=1024)):
        rows = render_rows(plan, srcs, jobs, dev, **v)
        for a, b in zip(rows, base):
            assert np.array_equal(a, b), v
    plan.close()


def test_graph_replays_match_eager(dev):
    import torch
    h = H()
    plan, r, p, g, lg, srcs, jobs = _variant_setup(1)
    base = render_rows(plan, srcs, jobs, dev)
    lens = np.array([len(s) for s in srcs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs)).to(dev)
    out_off, total = h.row_layout(plan, lens, jobs)
    for flags in (h.SPCONV_GRAPH, h.SPCONV_GRAPH | h.SPCONV_PERSISTENT, h.SPCONV_GRAPH | h.SPCONV_LDS_GATHER,
                  h.SPCONV_GRAPH | h.SPCONV_REGWIN | h.SPCONV_PERSISTENT,
                  h.SPCONV_GRAPH | h.SPCONV_WG256 | h.SPCONV_PERSISTENT):
        out = torch.zeros(total, dtype=torch.float32, device=dev)
        b = h.Batch(plan, off, lens, [(s, f, o) for (s, f), o in zip(jobs, out_off)], flags=flags)
        for rep in range(4):
            out.fill_(-1.0)                      # eager work between replays
            torch.cuda.synchronize()
            b.render(src, out)
            torch.cuda.synchronize()
            host = out.cpu().numpy()
            for (s, _), o, ref in zip(jobs, out_off, base):
                assert np.array_equal(host[o:o + ref.size], ref), (flags, rep)
        other = torch.zeros_like(out)
        with pytest.raises(h.HrirError):
            b.render(src, other)                 # graph is bound to its buffers
        b.close()


def test_batch_mix_invariance(dev):
    """A job renders to the same bits alone and inside a large mixed batch."""
    plan, r, p, g, lg, srcs, jobs = _variant_setup(2)
    mixed = render_rows(plan, srcs, jobs, dev)
    for idx in (0, len(jobs) // 2, len(jobs) - 1):
        s, f = jobs[idx]
        alone = render_rows(plan, [srcs[s]], [(0, f)], dev)
        assert np.array_equal(alone[0], mixed[idx])


def test_one_shot_render_and_empty_batch(dev):
    import torch
    h = H()
    plan, r, p, g, lg, srcs, jobs = _variant_setup(3)
    lens = np.array([len(s) for s in srcs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs)).to(dev)
    out_off, total = h.row_layout(plan, lens, jobs)
    out = torch.zeros(total, dtype=torch.float32, device=dev)
    h.render(plan, src, off, lens, [(s, f, o) for (s, f), o in zip(jobs, out_off)], out)
    host = out.cpu().numpy()
    base = render_rows(plan, srcs, jobs, dev)
    for (s, _), o, ref in zip(jobs, out_off, base):
        assert np.array_equal(host[o:o + ref.size], ref)
    empty = h.Batch(plan, off, lens, [])
    empty.render(src, out)                        # no-op
    torch.cuda.synchronize()


def test_argument_errors(dev):
    import torch
    h = H()
    plan, r, p, g, lg, srcs, jobs = _variant_setup(4)
    lens = np.array([len(s) for s in srcs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    for bad_jobs, kw in [([(9, 0, 0)], {}), ([(0, 99, 0)], {}), ([(0, 0, -1)], {}), ([(0, 0, 0)], {"tile": 1000}),
                         ([(0, 0, 0)], {"tile": 32768}), ([(0, 0, 0)], {"tile": 8192}),
                         ([(0, 0, 0)], {"tile": 1000, "flags": h.SPCONV_LDS_GATHER}),
                         ([(0, 0, 0)], {"tile": 4096, "flags": h.SPCONV_REGWIN}),
                         ([(0, 0, 0)], {"flags": h.SPCONV_REGWIN | h.SPCONV_LDS_GATHER}),
                         ([(0, 0, 0)], {"flags": h.SPCONV_PERSISTENT | h.SPCONV_UNFUSED})]:
        with pytest.raises(h.HrirError) as e:
            h.Batch(plan, off, lens, bad_jobs, **kw)
        assert e.value.code == h.HRIR_EINVAL
    with pytest.raises(h.HrirError):
        h.Batch(plan, off, np.array([0, 5, 5, 5, 5]), [(0, 0, 0)])       # empty source
    b = h.Batch(plan, off, lens, [(2, 0, 100)])
    src = torch.zeros(int(lens.sum()), dtype=torch.float32, device=dev)
    small = torch.zeros(100 + plan.out_len(lens[2]) - 1, dtype=torch.float32, device=dev)
    with pytest.raises(h.HrirError) as e:
        b.render(src, small)                                               # row does not fit
    assert "too small" in str(e.value)
    b.close()
    b = h.Batch(plan, off, lens, [(len(lens) - 1, 0, 0)])                # reads the last source
    with pytest.raises(h.HrirError) as e:
        b.render(src[:-1], torch.zeros(10 ** 6, dtype=torch.float32, device=dev))
    assert "too small" in str(e.value)
    b.close()


def test_full_size_throughput_config_sampled(dev):
    """The throughput workload at full size in the benchmark's launch shape:
    64 pink sources x 1,048,576 samples, 20 directions x 2 ears each, K = 16,
    from a 1,250-direction set; sampled outputs against the oracle's
    per-sample definition, plus every row's first and last samples."""
    import torch
    h = H()
    hs = synth.hrir_set(0, 25, 50)
    fac = h.factorize(hs.h, 32, 100, 16, seed=7, lambda0=0.2, want_cost=False)
    r = fac["f"].astype(np.float32)
    plan = h.Plan(r, fac["p"], fac["g"], 169)
    n_src, ns = 64, 1 << 20
    srcs = [synth.pink(100 + i, ns) for i in range(n_src)]
    jr = synth.jobs_fixed(n_src, 1250, 20)
    jobs = [(int(a), int(b)) for a, b in jr]
    lens = np.full(n_src, ns, dtype=np.int64)
    off = (np.arange(n_src) * ns).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs)).to(dev)
    out_off, total = h.row_layout(plan, lens, jobs)
    out = torch.empty(total, dtype=torch.float32, device=dev)
    b = h.Batch(plan, off, lens, [(s, f, o) for (s, f), o in zip(jobs, out_off)])
    b.render(src, out)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    L = plan.out_len(ns)
    got, ref = [], []
    for j in rng.choice(len(jobs), size=48, replace=False):
        s, f = jobs[j]
        t = np.unique(np.concatenate([[0, 1, 168, 199, L - 200, L - 1], rng.integers(0, L, 40)]))
        idx = torch.from_numpy(out_off[j] + t).to(dev)
        gj = out[idx].cpu().numpy()
        pf, gf = fac["p"][f], fac["g"][f].astype(np.float64)
        rj = oracle.sparse_render_points(r, srcs[s], pf, gf, t)
        # every sample within the FP32 bound of its own fma chains
        assert np.all(np.abs(gj - rj) <= fp32bound.render_bound(r, srcs[s], pf, gf, t, 16)), (j, s, f)
        got.append(gj)
        ref.append(rj)
    got, ref = np.concatenate(got), np.concatenate(ref)
    e = oracle.rel_l2(got, ref)
    print(f"full-size sampled rel L2 {e:.3e} over {got.size} samples", flush=True)
    assert e <= TOL
    b.close()
    del out, src
    torch.cuda.empty_cache()
