"""GPU tests of the streaming request loop (stream_* in include/hrir.h).

Each stream's blocks, rendered through the continuous-batching loop, must
equal the FP64 oracle's partitioned render (Sec. IV-F, with Eq. (2) applied
per block and the direction taking effect at block boundaries) within the
1e-5 relative-L2 bar, and must be the same bits whether the stream runs alone
or mixed with many others, whichever launch form the loop uses."""
import threading
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def H():
    import paper_1502_03162_amd
    return paper_1502_03162_amd


def _taps(seed, lf, lg, k, F):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(lf).astype(np.float32)
    p, g = synth.random_taps(seed + 1, F, min(k, lg), lg, nnz_min=1)
    return r, p, g


def _script(seed, F, n_blocks, lo=1, hi=4096, change_every=3):
    """One stream: blocks of U{lo..hi} samples of pink noise, the direction
    (a pair of filters) changing every few blocks; then the end's pair."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, n_blocks)
    sig = synth.pink(seed, int(sizes.sum()))
    blocks = np.split(sig, np.cumsum(sizes)[:-1])
    out, d = [], int(rng.integers(0, F // 2))
    for i, b in enumerate(blocks):
        if i % change_every == 0:
            d = int(rng.integers(0, F // 2))
        out.append((b, 2 * d, 2 * d + 1))
    return out, (2 * d, 2 * d + 1)


def _oracle(r, p, g, lg, script, end_dirs):
    left = oracle.BlockRenderer(r, p[0], g[0], lg)
    right = oracle.BlockRenderer(r, p[0], g[0], lg)
    ys = [[], []]

    def taps(rd, f):
        # a direction change swaps the taps; the histories hold z, which no
        # direction touches (reading of Sec. IV-F)
        rd.p = np.ascontiguousarray(p[f], dtype=np.int32)
        rd.g = np.ascontiguousarray(g[f], dtype=np.float64)

    for blk, fl, fr in script:
        taps(left, fl)
        taps(right, fr)
        ys[0].append(left.push(blk))
        ys[1].append(right.push(blk))
    taps(left, end_dirs[0])
    taps(right, end_dirs[1])
    ys[0].append(left.flush())
    ys[1].append(right.flush())
    return np.concatenate(ys[0]), np.concatenate(ys[1])


def _drive(server, scripts, seed=0, deadline_s=60.0):
    """Submits every stream's blocks and end, interleaving streams at random
    (each stream in order), polling when refused and now and then.  Returns
    per stream the concatenated (left, right) outputs and the results'
    tags in arrival order."""
    rng = np.random.default_rng(seed)
    sids = list(scripts)
    nxt = {s: 0 for s in sids}
    got = {s: [] for s in sids}
    expected = sum(len(scripts[s][0]) + 1 for s in sids)
    n_got = 0

    def take(res):
        nonlocal n_got
        for tag, sid, y, t0, t1, t2, tail in res:
            assert t0 <= t1 <= t2
            got[sid].append((tag, y, tail))
            n_got += 1

    t_end = time.monotonic() + deadline_s
    live = [s for s in sids]
    while live:
        assert time.monotonic() < t_end, "submission did not finish"
        s = live[int(rng.integers(0, len(live)))]
        blocks, end_dirs = scripts[s]
        i = nxt[s]
        tag = (s << 32) | i
        if i < len(blocks):
            blk, fl, fr = blocks[i]
            ok = server.submit(s, blk, fl, fr, tag)
        else:
            ok = server.end(s, end_dirs[0], end_dirs[1], tag)
        if not ok:
            take(server.poll(timeout_us=2000))
            continue
        nxt[s] += 1
        if nxt[s] > len(blocks):
            live.remove(s)
        if rng.random() < 0.1:
            take(server.poll())
    while n_got < expected:
        assert time.monotonic() < t_end, f"only {n_got} of {expected} results"
        take(server.poll(timeout_us=20000))
    out = {}
    for s in sids:
        tags = [t for t, _, _ in got[s]]
        assert tags == [(s << 32) | i for i in range(len(scripts[s][0]) + 1)], "results out of order"
        assert [tl for _, _, tl in got[s]] == [False] * len(scripts[s][0]) + [True]
        out[s] = (np.concatenate([y[0] for _, y, _ in got[s]]), np.concatenate([y[1] for _, y, _ in got[s]]))
    return out


def _check_oracle(out, scripts, r, p, g, lg):
    worst = 0.0
    for s, (yl, yr) in out.items():
        blocks, end_dirs = scripts[s]
        rl, rr = _oracle(r, p, g, lg, blocks, end_dirs)
        total = sum(b.size for b, _, _ in blocks)
        assert yl.size == rl.size == total + r.size + lg - 2
        worst = max(worst, oracle.rel_l2(yl, rl), oracle.rel_l2(yr, rr))
    assert worst <= TOL, worst
    return worst


@pytest.mark.parametrize("flags", [0, 1, 2, 3], ids=["graph", "direct", "zero_copy_graph", "zero_copy_direct"])
def test_mix_matches_oracle_and_alone(dev, flags):
    h = H()
    lf, lg, k, F = 32, 169, 16, 40
    r, p, g = _taps(11, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    scripts = {s: _script(1000 + s, F, n_blocks=6, hi=1500) for s in range(48)}
    srv = h.Server(plan, max_streams=64, flags=flags)
    mixed = _drive(srv, scripts, seed=1)
    info = srv.info()
    srv.close()
    _check_oracle(mixed, scripts, r, p, g, lg)
    assert info["results"] == sum(len(b) + 1 for b, _ in scripts.values())
    assert info["max_batch"] > 1          # the loop did batch blocks of different streams
    for s in (0, 17, 47):
        alone_srv = h.Server(plan, max_streams=64, flags=flags)
        alone = _drive(alone_srv, {s: scripts[s]}, seed=2)
        alone_srv.close()
        assert np.array_equal(alone[s][0], mixed[s][0]) and np.array_equal(alone[s][1], mixed[s][1])
    plan.close()


def test_launch_forms_agree_bitwise(dev):
    """Graph or direct launch, device ring or zero-copy host ring, polling
    or sleeping completion: the same bits for every stream."""
    h = H()
    lf, lg, k, F = 32, 169, 16, 20
    r, p, g = _taps(12, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    scripts = {s: _script(2000 + s, F, n_blocks=5) for s in range(12)}
    outs = []
    for flags in (0, h.STREAM_DIRECT_LAUNCH, h.STREAM_ZERO_COPY, h.STREAM_ZERO_COPY | h.STREAM_DIRECT_LAUNCH,
                  h.STREAM_SLEEPING_COMPLETION, h.STREAM_SLEEPING_COMPLETION | h.STREAM_ZERO_COPY):
        srv = h.Server(plan, max_streams=16, flags=flags)
        outs.append(_drive(srv, scripts, seed=3))
        srv.close()
    for o in outs[1:]:
        for s in scripts:
            assert np.array_equal(outs[0][s][0], o[s][0]) and np.array_equal(outs[0][s][1], o[s][1])
    plan.close()


def test_full_size_streams(dev):
    """The serving workload's scale in the benchmark's launch form: 1,024
    streams of blocks U{64..1024} over a 1,250-direction tap table, K = 16,
    graph launch; every stream driven, 128 of them checked against the
    oracle."""
    h = H()
    lf, lg, k, F, ms = 32, 169, 16, 2500, 1024
    r, p, g = _taps(17, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    scripts = {s: _script(9000 + s, F, n_blocks=3, lo=64, hi=1024) for s in range(ms)}
    srv = h.Server(plan, max_streams=ms, hbm_budget=1 << 30)
    out = _drive(srv, scripts, seed=9, deadline_s=120.0)
    info = srv.info()
    srv.close()
    assert info["results"] == 4 * ms
    checked = {s: scripts[s] for s in range(0, ms, 8)}
    _check_oracle({s: out[s] for s in checked}, checked, r, p, g, lg)
    plan.close()


@pytest.mark.parametrize("lf,lg,k", [(1, 1, 1), (5, 2, 2), (64, 2048, 64), (17, 40, 3)])
def test_shapes_match_oracle(dev, lf, lg, k):
    h = H()
    F = 8
    r, p, g = _taps(lf * 100 + lg, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    scripts = {s: _script(3000 + s, F, n_blocks=4, lo=1, hi=4096, change_every=2) for s in range(6)}
    srv = h.Server(plan, max_streams=8)
    out = _drive(srv, scripts, seed=4)
    srv.close()
    _check_oracle(out, scripts, r, p, g, lg)
    plan.close()


@pytest.mark.parametrize("flags", [0, 2], ids=["device_ring", "zero_copy"])
def test_backpressure_small_budget(dev, flags):
    """A budget of exactly two generations of one maximal block: blocks are
    refused (EAGAIN) until polls free generations, and every result is
    still exact."""
    h = H()
    lf, lg, k, F, ms = 32, 169, 16, 10, 8
    r, p, g = _taps(13, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    hist = ms * 200 * 4                      # round_up(lf - 1 + lg - 1, 4) floats per stream
    per_gen = 64 + 32 * ms + 12 * 4096
    with pytest.raises(h.HrirError):
        h.Server(plan, max_streams=ms, hbm_budget=hist + 2 * per_gen - 1, flags=flags)
    srv = h.Server(plan, max_streams=ms, hbm_budget=hist + 2 * per_gen, flags=flags)
    info = srv.info()
    assert info["generations"] == 2 and info["gen_samples"] == 4096
    scripts = {s: _script(4000 + s, F, n_blocks=5, lo=900, hi=1100) for s in range(ms)}
    out = _drive(srv, scripts, seed=5)
    info = srv.info()
    srv.close()
    assert info["eagain"] > 0
    _check_oracle(out, scripts, r, p, g, lg)
    plan.close()


def test_stream_reuse_after_end(dev):
    """After stream_end the id starts a new stream from zero history."""
    h = H()
    lf, lg, k, F = 32, 169, 16, 10
    r, p, g = _taps(14, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    first, second = _script(5000, F, n_blocks=4), _script(5001, F, n_blocks=4)
    srv = h.Server(plan, max_streams=4)
    _drive(srv, {2: first}, seed=6)
    again = _drive(srv, {2: second}, seed=7)
    srv.close()
    fresh_srv = h.Server(plan, max_streams=4)
    fresh = _drive(fresh_srv, {2: second}, seed=8)
    fresh_srv.close()
    assert np.array_equal(again[2][0], fresh[2][0]) and np.array_equal(again[2][1], fresh[2][1])
    _check_oracle(again, {2: second}, r, p, g, lg)
    plan.close()


def test_threads_submit_concurrently(dev):
    """Four submitting threads on disjoint streams and one polling thread:
    every stream's output equals its single-threaded render bit for bit."""
    h = H()
    lf, lg, k, F = 32, 169, 16, 16
    r, p, g = _taps(15, lf, lg, k, F)
    plan = h.Plan(r, p, g, lg)
    scripts = {s: _script(6000 + s, F, n_blocks=6, hi=2048) for s in range(32)}
    ref_srv = h.Server(plan, max_streams=32)
    ref = _drive(ref_srv, scripts, seed=9)
    ref_srv.close()

    srv = h.Server(plan, max_streams=32)
    expected = sum(len(b) + 1 for b, _ in scripts.values())
    got = {s: [] for s in scripts}
    done = threading.Event()
    errors = []

    def submitter(sids):
        try:
            for s in sids:
                blocks, end_dirs = scripts[s]
                for i, (blk, fl, fr) in enumerate(blocks):
                    while not srv.submit(s, blk, fl, fr, (s << 32) | i):
                        time.sleep(1e-4)
                while not srv.end(s, end_dirs[0], end_dirs[1], (s << 32) | len(blocks)):
                    time.sleep(1e-4)
        except Exception as e:  # noqa: BLE001  (reported below)
            errors.append(e)

    def poller():
        n, t_end = 0, time.monotonic() + 60
        while n < expected and time.monotonic() < t_end and not errors:
            for tag, sid, y, *_ in srv.poll(timeout_us=5000):
                got[sid].append((tag, y))
                n += 1
        done.set()

    pt = threading.Thread(target=poller)
    pt.start()
    ths = [threading.Thread(target=submitter, args=(list(range(i, 32, 4)),)) for i in range(4)]
    for t in ths:
        t.start()
    for t in ths:
        t.join(60)
    pt.join(70)
    srv.close()
    assert not errors, errors
    assert done.is_set()
    for s in scripts:
        assert [t for t, _ in got[s]] == [(s << 32) | i for i in range(len(scripts[s][0]) + 1)]
        yl = np.concatenate([y[0] for _, y in got[s]])
        yr = np.concatenate([y[1] for _, y in got[s]])
        assert np.array_equal(yl, ref[s][0]) and np.array_equal(yr, ref[s][1])
    plan.close()


def test_argument_errors(dev):
    h = H()
    r, p, g = _taps(16, 32, 169, 16, 4)
    plan = h.Plan(r, p, g, 169)
    srv = h.Server(plan, max_streams=4)
    blk = np.zeros(100, dtype=np.float32)
    for args in [(4, blk, 0, 1), (-1, blk, 0, 1), (0, np.zeros(0, np.float32), 0, 1),
                 (0, np.zeros(4097, np.float32), 0, 1), (0, blk, 0, 4), (0, blk, -1, 0)]:
        with pytest.raises(h.HrirError) as ei:
            srv.submit(*args)
        assert ei.value.code == h.HRIR_EINVAL
    with pytest.raises(h.HrirError):
        srv.end(9, 0, 1)
    with pytest.raises(h.HrirError):
        srv.end(0, 0, 7)
    assert srv.poll(timeout_us=-1) == []            # nothing queued: returns at once
    srv.close()
    with pytest.raises(h.HrirError):
        h.Server(plan, max_streams=0)
    with pytest.raises(h.HrirError):
        h.Server(plan, max_streams=4, flags=8)
    with pytest.raises(h.HrirError) as ei:
        h.Server(plan, max_streams=4, hbm_budget=-1)
    assert ei.value.code == h.HRIR_EINVAL
    srv = h.Server(plan, max_streams=4, hbm_budget=1 << 50)   # a bound, not an allocation
    srv.close()
    plan.close()


def test_default_budget_from_free_memory(dev):
    """hbm_budget = 0 (the binding's default) sizes the ring from the free
    device memory: a full ring of generations, and blocks render as with an
    explicit budget."""
    h = H()
    r, p, g = _taps(16, 32, 169, 16, 4)
    plan = h.Plan(r, p, g, 169)
    outs = []
    for budget in (0, 1 << 30):
        srv = h.Server(plan, max_streams=8, hbm_budget=budget)
        assert srv.info()["generations"] >= 2
        assert srv.submit(3, synth.white(5, 1000), 0, 1)
        got = []
        while not got:
            got = srv.poll(timeout_us=-1)
        outs.append(got[0][2])
        srv.close()
    assert np.array_equal(outs[0], outs[1])
    plan.close()
