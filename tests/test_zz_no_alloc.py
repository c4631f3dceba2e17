"""The allocation-free one-shot render (spconv_render_noalloc) against the
allocating one (spconv_render), through the C ABI.

Both run the same kernel over the same tiles, so their outputs must agree bit
for bit (which is inside the 1e-5 relative L2 parity bar); each row is also
checked against the FP64 oracle at that bar.  Two calls in a row, the second
with a smaller input, show that the shared descriptor array carries nothing
from one call into the next.  The limits are refused before any device
work."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _setup():
    import paper_1502_03162_amd as H
    hs = synth.hrir_set(0, 5, 10)
    fac = H.factorize(hs.h, 32, 200, 16, seed=7, lambda0=0.2, want_cost=False)
    r = fac["f"].astype(np.float32)
    return H, fac, r, H.Plan(r, fac["p"], fac["g"], 169)


def _render_both(H, plan, srcs, jobs_sf, dev):
    import torch
    lens = np.array([len(s) for s in srcs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs).astype(np.float32)).to(dev)
    out_off, total = H.row_layout(plan, lens, jobs_sf)
    jobs = [(s, f, o) for (s, f), o in zip(jobs_sf, out_off)]
    outs = []
    for fn in (H.render, H.render_noalloc):
        out = torch.full((total + 64,), float("nan"), dtype=torch.float32, device=dev)
        fn(plan, src, off, lens, jobs, out)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    return lens, off, out_off, outs


def test_noalloc_equals_render_on_two_calls(dev):
    H, fac, r, plan = _setup()
    rng = np.random.default_rng(11)
    cases = [
        # first call: three sources of ragged lengths (several tiles, a
        # ragged tail, a source shorter than one tile), 60 jobs
        ([synth.white(1, 70001), synth.white(2, 4097), synth.white(3, 1025)],
         [(int(rng.integers(0, 3)), int(rng.integers(0, 100))) for _ in range(60)]),
        # second call, smaller: one short source, 5 jobs
        ([synth.white(4, 3000)], [(0, f) for f in (0, 17, 42, 77, 99)]),
    ]
    for call, (srcs, jobs_sf) in enumerate(cases):
        print(f"noalloc call {call}: {len(srcs)} sources, {len(jobs_sf)} jobs", flush=True)
        lens, off, out_off, (a, b) = _render_both(H, plan, srcs, jobs_sf, dev)
        # bit for bit, including the untouched (NaN) elements between rows
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"call {call}"
        refs = oracle.sparse_render_jobs(r, np.concatenate(srcs).astype(np.float32), off, lens, fac["p"],
                                         np.asarray(fac["g"], np.float32), 169, np.asarray(jobs_sf, np.int32))
        worst = max(oracle.rel_l2(b[o:o + ref.size], ref) for o, ref in zip(out_off, refs))
        assert worst <= TOL, (call, worst)


def test_noalloc_limits_refused_before_device_work(dev):
    import torch
    H, fac, r, plan = _setup()
    src = torch.zeros(16, dtype=torch.float32, device=dev)
    out = torch.zeros(16, dtype=torch.float32, device=dev)
    # too many jobs
    n = H.NOALLOC_MAX_JOBS + 1
    with pytest.raises(H.HrirError) as e:
        H.render_noalloc(plan, src, [0], [8], [(0, 0, 0)] * n, out)
    assert e.value.code == H.HRIR_EINVAL and "jobs exceed" in str(e.value)
    # too many tiles: one source whose output spans more than the tile limit
    long_len = H.NOALLOC_MAX_TILES * 2048
    with pytest.raises(H.HrirError) as e:
        H.render_noalloc(plan, src, [0], [long_len], [(0, 0, 0)], out)
    assert e.value.code == H.HRIR_EINVAL and "tiles" in str(e.value)
    # buffers too small for the job rows
    with pytest.raises(H.HrirError) as e:
        H.render_noalloc(plan, src, [0], [100], [(0, 0, 0)], out)
    assert e.value.code == H.HRIR_EINVAL and "too small" in str(e.value)
