"""Block rendering with device-resident stream history: any split of a
stream into blocks, interleaved with other streams in the same launches and
followed by a flush, reproduces the offline render of the whole stream bit
for bit (and the FP64 oracle within 1e-5)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _setup(dev, n_streams, seed):
    import paper_1502_03162_amd as H
    rng = np.random.default_rng(seed)
    lf, lg, K, F = 32, 169, 16, 20
    r = rng.standard_normal(lf).astype(np.float32)
    p, g = synth.random_taps(seed + 1, F, K, lg, nnz_min=8)
    plan = H.Plan(r, p, g, lg)
    lens = [int(x) for x in rng.integers(1, 12000, size=n_streams)]
    dirs = [(2 * int(d), 2 * int(d) + 1) for d in rng.integers(0, F // 2, size=n_streams)]
    srcs = [synth.white(900 + seed * 100 + i, n) for i, n in enumerate(lens)]
    return H, rng, plan, r, p, g, lg, lens, dirs, srcs


def _offline(H, plan, srcs, jobs, dev):
    import torch
    lens = [len(s) for s in srcs]
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    src = torch.from_numpy(np.concatenate(srcs)).to(dev)
    out_off, total = H.row_layout(plan, lens, jobs)
    out = torch.zeros(total, dtype=torch.float32, device=dev)
    b = H.Batch(plan, off, lens, [(s, f, o) for (s, f), o in zip(jobs, out_off)])
    b.render(src, out)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    b.close()
    return [host[o:o + plan.out_len(lens[s])] for (s, _), o in zip(jobs, out_off)]


def _stream_blocks(H, plan, srcs, dirs, splits, dev, streams=None, slot_of=None):
    """Render every stream by its block split; blocks of different streams
    share launches (one block per stream per launch)."""
    import torch
    n = len(srcs)
    st = streams or H.Streams(plan, max(n, 1) + 3)
    slot_of = slot_of or list(range(n))
    cat = np.concatenate(srcs)
    d_in = torch.from_numpy(cat).to(dev)
    base = np.concatenate([[0], np.cumsum([len(s) for s in srcs])[:-1]])
    outs = [[[], []] for _ in range(n)]
    pos = [0] * n
    bi = [0] * n
    done = [False] * n
    while not all(done):
        jobs, meta, o = [], [], 0
        for i in range(n):
            if done[i]:
                continue
            if bi[i] < len(splits[i]):
                m = splits[i][bi[i]]
                jobs.append((slot_of[i], m, dirs[i][0], dirs[i][1], base[i] + pos[i], o, False))
                pos[i] += m
            else:
                m = st.tail
                jobs.append((slot_of[i], 0, dirs[i][0], dirs[i][1], 0, o, True))
                done[i] = True
            meta.append((i, o, m))
            bi[i] += 1
            o += 2 * m
        d_out = torch.zeros(max(o, 1), dtype=torch.float32, device=dev)
        st.render(d_in, jobs, d_out)
        torch.cuda.synchronize()
        h = d_out.cpu().numpy()
        for i, oo, m in meta:
            outs[i][0].append(h[oo:oo + m])
            outs[i][1].append(h[oo + m:oo + 2 * m])
    return [(np.concatenate(a), np.concatenate(b)) for a, b in outs], st


def _random_splits(rng, n_total):
    sp, left = [], n_total
    while left > 0:
        b = int(min(left, rng.choice([1, 2, 7, 64, 100, 513, 1024, 4096])))
        sp.append(b)
        left -= b
    return sp


def test_block_splits_equal_offline_render(dev):
    H, rng, plan, r, p, g, lg, lens, dirs, srcs = _setup(dev, 9, 3)
    splits = [_random_splits(rng, n) for n in lens]
    got, st = _stream_blocks(H, plan, srcs, dirs, splits, dev)
    jobs = [(i, dirs[i][e]) for i in range(len(srcs)) for e in range(2)]
    off_rows = _offline(H, plan, srcs, jobs, dev)
    refs = oracle.sparse_render_jobs(r, np.concatenate(srcs), np.concatenate([[0], np.cumsum(lens)[:-1]]), lens,
                                     p, g, lg, np.asarray(jobs, np.int32))
    for i in range(len(srcs)):
        for e in range(2):
            row = got[i][e]
            assert row.size == plan.out_len(lens[i])
            assert np.array_equal(row, off_rows[2 * i + e]), (i, e)
            assert oracle.rel_l2(row, refs[2 * i + e]) <= 1e-5
    st.close()


def test_block_slot_reuse_after_reset(dev):
    H, rng, plan, r, p, g, lg, lens, dirs, srcs = _setup(dev, 3, 4)
    splits = [_random_splits(rng, n) for n in lens]
    first, st = _stream_blocks(H, plan, srcs, dirs, splits, dev)
    st.reset([0, 1, 2])                      # the same slots carry new streams
    whole = [[4096] * (n // 4096) + ([n % 4096] if n % 4096 else []) for n in lens]
    again, _ = _stream_blocks(H, plan, srcs, dirs, whole, dev, streams=st)
    for a, b in zip(first, again):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    st.close()


def test_block_argument_errors(dev):
    import torch
    H, rng, plan, r, p, g, lg, lens, dirs, srcs = _setup(dev, 2, 5)
    st = H.Streams(plan, 4)
    d_in = torch.zeros(100, dtype=torch.float32, device=dev)
    d_out = torch.zeros(1000, dtype=torch.float32, device=dev)
    for jobs in ([(0, 10, 0, 1, 0, 0, False), (0, 10, 0, 1, 10, 20, False)],   # slot twice
                 [(0, 0, 0, 1, 0, 0, False)],                                  # empty block
                 [(9, 10, 0, 1, 0, 0, False)],                                 # slot out of range
                 [(0, 10, 0, 99, 0, 0, False)],                                # filter out of range
                 [(0, 95, 0, 1, 10, 0, False)],                                # input outside buffer
                 [(0, 10, 0, 1, 0, 990, False)],                               # output outside buffer
                 [(0, 5000, 0, 1, 0, 0, False)]):                              # block too long
        with pytest.raises(H.HrirError) as e:
            st.render(d_in, jobs, d_out)
        assert e.value.code == H.HRIR_EINVAL
    st.close()
