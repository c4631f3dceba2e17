"""GPU tests of the device-side top-K (spconv_plan_topk) and of moving-source
rendering (moving_*) against the FP64 oracle on seeded inputs.

Top-K is an index decision on identical float32 values, so positions and
gains must agree exactly.  The moving render is floating point: 1e-5
relative L2 per (source, ear) row, the bar of every render."""
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


def _dense_rows(seed, n, width, stride):
    """Seeded dense rows [n][stride] with the cases that matter in the first
    `width` entries: no positive entry, fewer positives than slots with a
    tie, runs of equal values, a NaN, all positive."""
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((n, stride)).astype(np.float32)
    D[0] = -np.abs(D[0])
    D[1, :] = 0.0
    pos = sorted({min(5, width - 1), min(9, width - 1), width - 1})
    D[1, pos] = 0.5
    D[1, pos[0]] = 0.25
    D[2, :width:3] = 0.75
    D[3, width // 2] = np.nan
    D[4] = np.abs(D[4])
    return D, len(pos)


@pytest.mark.parametrize("k,lg,width,stride", [(16, 169, 169, 200), (4, 40, 33, 40), (64, 2048, 2048, 2048),
                                               (1, 7, 7, 9)])
def test_plan_topk_matches_oracle(dev, k, lg, width, stride):
    import torch
    h = H()
    n_static, n_dyn = 6, 37
    p0, g0 = synth.random_taps(3, n_static + n_dyn, k, lg, nnz_min=1)
    plan = h.Plan(np.ones(4, np.float32), p0, g0, lg)
    D, n_pos1 = _dense_rows(k + lg, n_dyn, width, stride)
    dense = torch.from_numpy(D).to(dev)
    h.plan_topk(plan, n_static, dense, width)
    torch.cuda.synchronize()
    p, g = h.plan_read(plan, 0, n_static + n_dyn)
    np.testing.assert_array_equal(p[:n_static], p0[:n_static])        # untouched rows
    np.testing.assert_array_equal(g[:n_static], g0[:n_static])
    po, go, nz = oracle.topk(D[:, :width].astype(np.float64), k)
    np.testing.assert_array_equal(p[n_static:], po)
    np.testing.assert_array_equal(g[n_static:].astype(np.float64), go)
    assert nz[0] == 0 and nz[1] == min(n_pos1, k)
    plan.close()


def _moving_case(seed, n_src, n, lf, lg, k, F):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(lf).astype(np.float32)
    p, g = synth.random_taps(seed + 1, F, k, lg, nnz_min=1)
    srcs = np.stack([synth.pink(seed + 10 + i, n) for i in range(n_src)])
    return r, p, g, srcs, rng


@pytest.mark.parametrize("n,seg,fade,lf,lg,k,tile", [(20000, 512, 64, 32, 169, 16, 0), (20000, 256, 0, 32, 169, 16, 0),
                                                      (9000, 256, 256, 5, 40, 3, 0), (5000, 768, 100, 64, 2048, 64, 0),
                                                      (100, 256, 64, 32, 169, 16, 0), (12000, 1024, 256, 16, 100, 8, 0),
                                                      (9000, 512, 256, 64, 2048, 64, 4096),
                                                      (20000, 512, 64, 32, 169, 16, 1536)])
def test_moving_render_matches_oracle(dev, n, seg, fade, lf, lg, k, tile):
    """Moving sources against the oracle; the last two cases: the largest
    tile with the longest filter (LDS near its limit), and a 512-output-item
    tile that is not a power of two."""
    import torch
    h = H()
    n_src, F = 3, 12
    r, p, g, srcs, rng = _moving_case(n + seg + fade, n_src, n, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    mv = h.Moving(plan, n_src, n, seg, fade, tile)
    n_seg = (n + seg - 1) // seg
    assert mv.n_seg == n_seg and mv.out_len == n + lf + lg - 2
    seg_filt = rng.integers(0, F, (n_src, n_seg, 2)).astype(np.int32)
    stride = mv.out_len + 13                                   # unaligned rows take the guarded store path
    src = torch.from_numpy(srcs.reshape(-1)).to(dev)
    out = torch.full((2 * n_src * stride,), float("nan"), device=dev)
    mv.render(src, seg_filt, out, stride)
    torch.cuda.synchronize()
    host = out.cpu().numpy().reshape(2 * n_src, stride)
    worst = 0.0
    for s in range(n_src):
        for e in range(2):
            ref = oracle.moving_render(r, srcs[s], p, g, lg, seg_filt[s, :, e], seg, fade)
            row = host[2 * s + e]
            assert np.all(np.isnan(row[mv.out_len:]))          # nothing written past the row
            worst = max(worst, oracle.rel_l2(row[:mv.out_len], ref))
    assert worst <= TOL, worst
    mv.close()
    plan.close()


def test_moving_sees_rows_rewritten_on_device(dev):
    """The render forms its tap table from the plan's rows on every call: rows
    that spconv_plan_topk rewrites on the device between two renders of one
    moving object are the ones the second render uses."""
    import torch
    h = H()
    n, seg, fade, lf, lg, k, F, n_src = 6000, 512, 64, 32, 169, 16, 10, 2
    r, p, g, srcs, rng = _moving_case(77, n_src, n, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    mv = h.Moving(plan, n_src, n, seg, fade)
    seg_filt = rng.integers(0, F, (n_src, mv.n_seg, 2)).astype(np.int32)
    stride = mv.out_len
    src = torch.from_numpy(srcs.reshape(-1)).to(dev)
    out = torch.empty(2 * n_src * stride, device=dev)
    mv.render(src, seg_filt, out, stride)
    first = out.cpu().numpy().copy()
    dense = torch.from_numpy(np.abs(rng.standard_normal((F, lg))).astype(np.float32)).to(dev)
    h.plan_topk(plan, 0, dense, lg)
    mv.render(src, seg_filt, out, stride)
    torch.cuda.synchronize()
    p2, g2 = h.plan_read(plan, 0, F)
    assert not np.array_equal(p2, p)
    host = out.cpu().numpy().reshape(2 * n_src, stride)
    assert not np.array_equal(host.reshape(-1), first)
    for s_ in range(n_src):
        for e in range(2):
            ref = oracle.moving_render(r, srcs[s_], p2, g2, lg, seg_filt[s_, :, e], seg, fade)
            assert oracle.rel_l2(host[2 * s_ + e], ref) <= TOL
    mv.close()
    plan.close()


def test_back_to_back_renders_keep_their_segment_tables(dev):
    """Renders issued back to back with different segment tables (uploads on
    the object's own stream, two staging halves) each use their own table:
    equal, bit for bit, to the same render issued alone after a sync."""
    import torch
    h = H()
    n, seg, fade, lf, lg, k, F, n_src = 7000, 512, 64, 32, 169, 16, 12, 3
    r, p, g, srcs, rng = _moving_case(91, n_src, n, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    mv = h.Moving(plan, n_src, n, seg, fade)
    tables = [rng.integers(0, F, (n_src, mv.n_seg, 2)).astype(np.int32) for _ in range(5)]
    stride = mv.out_len
    src = torch.from_numpy(srcs.reshape(-1)).to(dev)
    outs = [torch.empty(2 * n_src * stride, device=dev) for _ in tables]
    for t, o in zip(tables, outs):
        mv.render(src, t, o, stride)
    torch.cuda.synchronize()
    alone = torch.empty(2 * n_src * stride, device=dev)
    for t, o in zip(tables, outs):
        mv.render(src, t, alone, stride)
        torch.cuda.synchronize()
        assert torch.equal(o, alone)
    assert not torch.equal(outs[0], outs[1])
    mv.close()
    plan.close()


def test_moving_argument_errors(dev):
    import torch
    h = H()
    p, g = synth.random_taps(1, 4, 4, 40, nnz_min=1)
    plan = h.Plan(np.ones(8, np.float32), p, g, 40)
    for kw in [dict(seg_len=300, fade=10), dict(seg_len=0, fade=0), dict(seg_len=256, fade=257),
               dict(seg_len=256, fade=-1)]:
        with pytest.raises(h.HrirError):
            h.Moving(plan, 2, 1000, **kw)
    mv = h.Moving(plan, 2, 1000, 256, 16)
    src = torch.zeros(2000, device=dev)
    out = torch.zeros(2 * mv.out_len, device=dev)
    bad = np.zeros((2, mv.n_seg, 2), dtype=np.int32)
    bad[1, 2, 1] = 4                                           # past the plan's 4 filters
    with pytest.raises(h.HrirError):
        mv.render(src, bad, out, mv.out_len)
    with pytest.raises(h.HrirError):
        mv.render(src, np.zeros((2, mv.n_seg, 2), np.int32), out[:-1], mv.out_len)
    with pytest.raises(h.HrirError):
        mv.render(src[:-1], np.zeros((2, mv.n_seg, 2), np.int32), out, mv.out_len)
    with pytest.raises(h.HrirError):
        h.plan_topk(plan, 3, torch.zeros((2, 40), device=dev), 40)      # rows 3, 4: past the plan
    mv.close()
    plan.close()


def test_moving_tile_lengths_agree_bitwise(dev):
    import torch
    h = H()
    n, seg, fade, n_src, F = 7000, 512, 64, 2, 9
    r, p, g, srcs, rng = _moving_case(41, n_src, n, 32, 169, 16, F)
    plan = h.Plan(r, p, g, 169)
    src = torch.from_numpy(srcs.reshape(-1)).to(dev)
    outs = []
    for tile in (0, 256, 1024, 4096):
        mv = h.Moving(plan, n_src, n, seg, fade, tile)
        if not outs:
            seg_filt = rng.integers(0, F, (n_src, mv.n_seg, 2)).astype(np.int32)
        out = torch.zeros(2 * n_src * mv.out_len, device=dev)
        mv.render(src, seg_filt, out, mv.out_len)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
        mv.close()
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    with pytest.raises(h.HrirError):
        h.Moving(plan, n_src, n, seg, fade, 300)
    plan.close()


def test_full_size_moving_config(dev):
    """The moving-source workload at full size: 128 pink sources of 262,144
    samples, a direction every 512 samples with a 64-sample crossfade,
    K = 16, the default tile (3072 at these sizes; the benchmark sweeps
    2048..4096); 6
    sources (both ears, every sample) against the oracle."""
    import torch
    h = H()
    n_src, n, seg, fade, lf, lg, k, F = 128, 262144, 512, 64, 32, 169, 16, 2500
    rng = np.random.default_rng(11)
    r = rng.standard_normal(lf).astype(np.float32)
    p, g = synth.random_taps(12, F, k, lg, nnz_min=8)
    plan = h.Plan(r, p, g, lg)
    mv = h.Moving(plan, n_src, n, seg, fade)
    seg_filt = rng.integers(0, F, (n_src, mv.n_seg, 2)).astype(np.int32)
    srcs = np.stack([synth.pink(900 + i, n) for i in range(n_src)])
    stride = (mv.out_len + 63) // 64 * 64
    src = torch.from_numpy(srcs.reshape(-1)).to(dev)
    out = torch.full((2 * n_src * stride,), float("nan"), device=dev)
    mv.render(src, seg_filt, out, stride)
    torch.cuda.synchronize()
    worst = 0.0
    for s in (0, 1, 37, 64, 100, 127):
        rows = out[2 * s * stride:(2 * s + 2) * stride].cpu().numpy().reshape(2, stride)
        for e in range(2):
            ref = oracle.moving_render(r, srcs[s], p, g, lg, seg_filt[s, :, e], seg, fade)
            worst = max(worst, oracle.rel_l2(rows[e, :mv.out_len], ref))
            # every sample within the FP32 bound of its chains and crossfade
            bound = fp32bound.moving_bound(r, srcs[s], p, g, lg, seg_filt[s, :, e], seg, fade, k)
            assert np.all(np.abs(rows[e, :mv.out_len] - ref) <= bound), (s, e)
    assert worst <= TOL, worst
    mv.close()
    plan.close()
    del out, src
    torch.cuda.empty_cache()
