"""The seeded input generators: determinism and the shape of the data."""
import numpy as np

import synth


def test_hrir_set_shapes_and_determinism():
    a = synth.hrir_set(0, 5, 10)
    b = synth.hrir_set(0, 5, 10)
    assert a.h.shape == (100, 200) and a.g.shape == (100, 169) and a.r.shape == (32,)
    assert np.array_equal(a.h, b.h)
    assert abs(np.linalg.norm(a.r) - 1) < 1e-12
    assert np.all(a.g >= 0)
    assert np.all((a.onset >= 0) & (a.onset <= 40))
    # 12 significant taps (onset + 11 pinna) above the 1e-3 noise, unless offsets collide
    sig = np.sum(a.g > 0.01, axis=1)
    assert np.all(sig <= 12) and np.mean(sig) > 10
    # HRIR = resonance * reflection, full length 32 + 169 - 1 = 200
    assert np.allclose(a.h[3], np.convolve(a.r, a.g[3]))


def test_ears_onsets_follow_azimuth():
    hs = synth.hrir_set(1, 25, 2)
    left, right = hs.onset[0::2], hs.onset[1::2]
    # the ear facing the source hears it first; at az = 0 both are 20
    assert np.all((left - 20) == -(right - 20)) or np.max(np.abs((left - 20) + (right - 20))) <= 1


def test_signals():
    w = synth.white(0, 65536)
    assert w.dtype == np.float32 and abs(w.std() - 0.1) < 0.002
    p = synth.pink(100, 1 << 16)
    assert p.dtype == np.float32 and abs(np.sqrt(np.mean(p.astype(np.float64) ** 2)) - 0.1) < 1e-4
    # 1/f: power in an octave band is roughly constant
    P = np.abs(np.fft.rfft(p.astype(np.float64))) ** 2
    b1, b2 = P[100:200].sum(), P[1000:2000].sum()
    assert 0.5 < b1 / b2 < 2.0
    assert np.array_equal(synth.pink(100, 1000), synth.pink(100, 1000))


def test_job_lists():
    j = synth.jobs_fixed(4, 1250, 20)
    assert j.shape == (160, 2)
    for i in range(4):
        dirs = j[j[:, 0] == i, 1] // 2
        assert len(set(dirs.tolist())) == 20
    lens = synth.uneven_lengths(300, 512)
    assert lens.min() >= 4096 and lens.max() <= 1 << 20
    ju = synth.jobs_uneven(300, 512, 1250)
    per = np.bincount(ju[:, 0], minlength=512)
    assert per.min() >= 2 and per.max() <= 16 and np.all(per % 2 == 0)


def test_random_taps():
    p, g = synth.random_taps(0, 10, 16, 169, nnz_min=3)
    assert p.dtype == np.int32 and g.dtype == np.float32
    assert np.all((p >= 0) & (p < 169)) and np.all(g >= 0)
