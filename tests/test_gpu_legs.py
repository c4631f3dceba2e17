"""GPU parity of the comparison legs (dense direct convolution and FFT
overlap-add) against the FP64 oracle, and the exact-reconstruction identity
between the sparse renderer with every tap kept and dense rendering with the
full HRIR h = r * g (Eqs. (1), (2), (12))."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def H():
    import paper_1502_03162_amd
    return paper_1502_03162_amd


def _layout(out_len_fn, lens, jobs, align=64):
    off, pos = [], 0
    for s, _ in jobs:
        off.append(pos)
        pos += (out_len_fn(lens[s]) + align - 1) // align * align
    return np.array(off, dtype=np.int64), pos


def _run(leg, srcs, jobs, dev):
    import torch
    lens = [len(s) for s in srcs]
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs).astype(np.float32)).to(dev)
    out_off, total = _layout(leg.out_len, lens, jobs)
    out = torch.full((total + 64,), float("nan"), dtype=torch.float32, device=dev)
    runner = leg.make(off, lens, [(s, f, o) for (s, f), o in zip(jobs, out_off)])
    runner.render(src, out)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    rows = [host[o:o + leg.out_len(lens[s])] for (s, _), o in zip(jobs, out_off)]
    mask = np.ones(host.size, dtype=bool)
    for (s, _), o in zip(jobs, out_off):
        mask[o:o + leg.out_len(lens[s])] = False
    assert np.all(np.isnan(host[mask]))
    runner.close()
    return rows


class Dense:
    def __init__(self, h):
        self.plan = H().DensePlan(h)
        self.out_len = self.plan.out_len

    def make(self, off, lens, jobs):
        return H().DenseBatch(self.plan, off, lens, jobs)


class Fft:
    def __init__(self, h, nfft):
        self.h, self.nfft, self.m = h, nfft, h.shape[1]

    def out_len(self, n):
        return int(n) + self.m - 1

    def make(self, off, lens, jobs):
        return H().FftOla(self.h, self.nfft, off, lens, jobs)


def _check(rows, srcs, h, jobs):
    lens = [len(s) for s in srcs]
    off = np.concatenate([[0], np.cumsum(lens)[:-1]])
    refs = oracle.dense_render_jobs(np.concatenate(srcs).astype(np.float32), off, lens, h.astype(np.float32),
                                    np.asarray(jobs, np.int32))
    worst = 0.0
    for row, ref in zip(rows, refs):
        assert row.shape == ref.shape and np.all(np.isfinite(row))
        worst = max(worst, oracle.rel_l2(row, ref))
    assert worst <= TOL, worst
    return worst


@pytest.mark.parametrize("m", [1, 7, 64, 200])
def test_dense_direct_parity(dev, m):
    rng = np.random.default_rng(m)
    F = 5
    h = rng.standard_normal((F, m)).astype(np.float32)
    lens = [1, 2, 199, 200, 511, 512, 2047, 2048, 2049, 5000, 20000]
    srcs = [synth.white(300 + i, n) for i, n in enumerate(lens)]
    jobs = [(i, (i + j) % F) for i in range(len(lens)) for j in range(2)]
    # 17 jobs of one source exceed one tile's job group
    jobs += [(9, j % F) for j in range(17)]
    _check(_run(Dense(h), srcs, jobs, dev), srcs, h, jobs)


@pytest.mark.parametrize("nfft,m", [(512, 200), (4096, 200), (16384, 200), (64, 7)])
def test_fft_overlap_add_parity(dev, nfft, m):
    rng = np.random.default_rng(nfft + m)
    F = 4
    h = rng.standard_normal((F, m)).astype(np.float32)
    lens = [1, 3, nfft - m, nfft - m + 1, nfft - m + 2, 3 * nfft + 5, 40000]
    srcs = [synth.pink(400 + i, n) for i, n in enumerate(lens)]
    jobs = [(i, (2 * i + j) % F) for i in range(len(lens)) for j in range(2)]
    _check(_run(Fft(h, nfft), srcs, jobs, dev), srcs, h, jobs)


def test_sparse_full_taps_equals_dense_hrir(dev):
    """K = lg with the true reflection filters reproduces h = r * g exactly
    (no truncation since lf + lg - 1 = 200): sparse render == dense render."""
    import torch
    h = H()
    hs = synth.hrir_set(1, 2, 2)
    lf, lg = 32, 169
    F = hs.n_filters
    p = np.tile(np.arange(lg, dtype=np.int32), (F, 1))[:, :64]       # first 64 positions
    g = hs.g[:, :64].astype(np.float32)
    r = hs.r.astype(np.float32)
    g_full = np.zeros((F, lg), dtype=np.float32)
    g_full[:, :64] = g
    hrir = np.stack([np.convolve(r.astype(np.float64), g_full[f].astype(np.float64)) for f in range(F)])
    srcs = [synth.white(7, 30000)]
    jobs = [(0, f) for f in range(F)]
    plan = h.Plan(r, p, g, lg)
    lens = [len(srcs[0])]
    src = torch.from_numpy(srcs[0]).to(dev)
    off_s, tot_s = _layout(plan.out_len, lens, jobs)
    out_s = torch.zeros(tot_s, dtype=torch.float32, device=dev)
    b = h.Batch(plan, [0], lens, [(s, f, o) for (s, f), o in zip(jobs, off_s)])
    b.render(src, out_s)
    dense = Dense(hrir.astype(np.float32))
    rows_d = _run(dense, srcs, jobs, dev)
    torch.cuda.synchronize()
    host = out_s.cpu().numpy()
    for (s, f), o, rd in zip(jobs, off_s, rows_d):
        rs = host[o:o + plan.out_len(lens[0])]
        assert rs.size == rd.size
        assert oracle.rel_l2(rs, rd) <= 2 * TOL
    b.close()


def test_leg_argument_errors(dev):
    h = H()
    hh = np.ones((2, 10), dtype=np.float32)
    with pytest.raises(h.HrirError):
        h.DensePlan(np.ones((2, 201), dtype=np.float32))
    with pytest.raises(h.HrirError):
        h.FftOla(hh, 16, [0], [100], [(0, 0, 0)])        # nfft < 2m
    with pytest.raises(h.HrirError):
        h.FftOla(hh, 1000, [0], [100], [(0, 0, 0)])      # not a power of two
    with pytest.raises(h.HrirError):
        h.FftOla(hh, 64, [0], [100], [(0, 5, 0)])        # filter out of range
