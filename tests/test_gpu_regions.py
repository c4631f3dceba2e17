"""GPU tests of plans with one resonance filter per region of space
(spconv_plan_multi): every (source, filter) row must match the FP64 oracle
rendered with its region's resonance filter (1e-5 relative L2); every launch
shape gives the same bits; a one-region plan built through the multi-region
entry equals the ordinary plan bit for bit; kernels that do not support
several resonance filters refuse such plans."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def H():
    import paper_1502_03162_amd
    return paper_1502_03162_amd


def _case(seed, lf=32, lg=169, k=16, F=30, R=3):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((R, lf)).astype(np.float32)
    p, g = synth.random_taps(seed + 1, F, k, lg, nnz_min=2)
    reg = rng.integers(0, R, F).astype(np.int32)
    lens = [1, 31, 2047, 2049, 5000, 12345]
    srcs = [synth.pink(seed + 10 + i, n) for i, n in enumerate(lens)]
    jobs = [(s, int(f)) for s in range(len(lens)) for f in rng.choice(F, 7, replace=False)]
    return r, p, g, reg, srcs, jobs, lg


def _render(h, plan, srcs, jobs, dev, **kw):
    import torch
    lens = np.array([len(s) for s in srcs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs)).to(dev)
    out_off, total = h.row_layout(plan, lens, jobs)
    out = torch.full((total + 64,), float("nan"), device=dev)
    b = h.Batch(plan, off, lens, [(s, f, o) for (s, f), o in zip(jobs, out_off)], **kw)
    b.render(src, out)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    b.close()
    return [host[o:o + plan.out_len(lens[s])] for (s, _), o in zip(jobs, out_off)]


def test_rows_match_oracle_with_their_regions_resonance(dev):
    h = H()
    r, p, g, reg, srcs, jobs, lg = _case(1)
    plan = h.Plan(r, p, g, lg, regions=reg)
    rows = _render(h, plan, srcs, jobs, dev)
    lens = [len(s) for s in srcs]
    off = np.concatenate([[0], np.cumsum(lens)[:-1]])
    cat = np.concatenate(srcs)
    worst = 0.0
    for (s, f), row in zip(jobs, rows):
        ref = oracle.sparse_render_jobs(r[reg[f]], cat, off, lens, p, g, lg, np.array([[s, f]], np.int32))[0]
        worst = max(worst, oracle.rel_l2(row, ref))
    assert worst <= TOL, worst
    plan.close()


def test_launch_shapes_agree_bitwise(dev):
    h = H()
    r, p, g, reg, srcs, jobs, lg = _case(2)
    plan = h.Plan(r, p, g, lg, regions=reg)
    base = _render(h, plan, srcs, jobs, dev)
    for kw in [dict(tile=1024), dict(tile=4096), dict(group=2), dict(flags=h.SPCONV_PERSISTENT),
               dict(flags=h.SPCONV_GRAPH | h.SPCONV_PERSISTENT, tile=3072)]:
        other = _render(h, plan, srcs, jobs, dev, **kw)
        for a, b in zip(base, other):
            np.testing.assert_array_equal(a, b)
    plan.close()


def test_one_region_equals_the_ordinary_plan(dev):
    h = H()
    r, p, g, reg, srcs, jobs, lg = _case(3, R=1)
    multi = h.Plan(r, p, g, lg, regions=np.zeros(len(p), np.int32))
    single = h.Plan(r[0], p, g, lg)
    for a, b in zip(_render(h, multi, srcs, jobs, dev), _render(h, single, srcs, jobs, dev)):
        np.testing.assert_array_equal(a, b)
    multi.close()
    single.close()


def test_other_paths_refuse_several_resonance_filters(dev):
    h = H()
    r, p, g, reg, srcs, jobs, lg = _case(4)
    plan = h.Plan(r, p, g, lg, regions=reg)
    lens = [len(s) for s in srcs]
    off = np.concatenate([[0], np.cumsum(lens)[:-1]])
    for flags in (h.SPCONV_LDS_GATHER, h.SPCONV_REGWIN, h.SPCONV_UNFUSED):
        with pytest.raises(h.HrirError):
            h.Batch(plan, off, lens, [(0, 0, 0)], flags=flags)
    with pytest.raises(h.HrirError):
        h.Streams(plan, 4)
    with pytest.raises(h.HrirError):
        h.Moving(plan, 1, 1000, 256, 0)
    plan.close()
