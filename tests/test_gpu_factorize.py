"""Alg. 1 on the GPU (hrir_factorize with HRIR_FACTORIZE_DEVICE) against the
host iterations and the FP64 oracle on the same initial G.  The device code
keeps the host's arithmetic and order (no fused multiply-adds), so the two
agree to rounding; the oracle bar is the host's own (1e-10)."""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def H():
    import paper_1502_03162_amd
    return paper_1502_03162_amd


def test_device_iterations_match_host_and_oracle(dev):
    h = H()
    hs = synth.hrir_set(2, 2, 5)
    X = hs.h
    n, m = X.shape
    lf, k, T = 32, 16, 60
    G0 = oracle.rand_g0(9, n, m - lf + 1)
    host = h.factorize(X, lf, T, k, g0=G0, lambda0=0.2)
    devr = h.factorize(X, lf, T, k, g0=G0, lambda0=0.2, device=True)
    assert np.max(np.abs(devr["f"] - host["f"])) < 1e-12
    assert np.max(np.abs(devr["G"] - host["G"])) < 1e-12 * np.max(host["G"])
    assert np.max(np.abs(devr["cost"] - host["cost"]) / host["cost"]) < 1e-12
    assert np.array_equal(devr["p"], host["p"]) and np.array_equal(devr["nnz"], host["nnz"])
    f, G, tr = oracle.factorize(X, lf, T, G0, 0.2)
    assert np.max(np.abs(devr["f"] - f)) < 1e-10
    assert np.max(np.abs(devr["G"] - G)) < 1e-10 * np.max(G)
    assert np.max(np.abs(devr["cost"] - tr) / tr) < 1e-10
    assert np.all(np.diff(tr[T // 2:]) <= 1e-12 * tr[T // 2:-1])      # lambda = 0 half: monotone


def test_device_full_set_matches_host(dev):
    """The 1,250-direction set (2,500 rows), 200 iterations: device and host
    give the same factorization to rounding; the device is timed."""
    h = H()
    hs = synth.hrir_set(0, 25, 50)
    t0 = time.perf_counter()
    d = h.factorize(hs.h, 32, 200, 16, seed=7, lambda0=0.2, want_cost=False, device=True)
    t_dev = time.perf_counter() - t0
    t0 = time.perf_counter()
    c = h.factorize(hs.h, 32, 200, 16, seed=7, lambda0=0.2, want_cost=False)
    t_host = time.perf_counter() - t0
    print(f"factorize 2500 x 200, 200 iterations: device {t_dev:.3f} s, host {t_host:.3f} s", flush=True)
    rec_d = oracle.reconstruct(d["f"], d["G"])
    rec_c = oracle.reconstruct(c["f"], c["G"])
    assert np.linalg.norm(rec_d - rec_c) / np.linalg.norm(rec_c) < 1e-10
    assert np.array_equal(d["p"], c["p"])


def test_device_errors(dev):
    h = H()
    X = synth.hrir_set(1, 2, 2).h
    with pytest.raises(h.HrirError) as e:
        h.factorize(X, 65, 3, 2, device=True)                   # lf beyond the device path
    assert e.value.code == h.HRIR_EINVAL
    with pytest.raises(h.HrirError) as e:
        h.factorize(np.zeros((4, 20)), 5, 3, 2, device=True)    # f vanishes
    assert e.value.code == h.HRIR_ENOTPD
