"""Pins of the error metrics (Sec. IV-B) and the cost model (Sec. IV-F)."""
import json
import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_metric_identities():
    rng = np.random.default_rng(0)
    h = rng.standard_normal((4, 200))
    assert oracle.spectral_distortion(h[0], h[0]) == 0.0
    assert oracle.rel_l2(h, h) == 0.0
    assert oracle.e_db(h, np.zeros_like(h)) == 0.0          # no reconstruction: 0 dB
    assert abs(oracle.e_db(h, 0.9 * h) - 20 * math.log10(0.1)) < 1e-12
    # RMSE of Eq. (17) is the Frobenius norm over sqrt(M N)
    d = rng.standard_normal(h.shape) * 1e-3
    assert abs(oracle.rmse(h, h + d) - np.linalg.norm(d) / math.sqrt(h.size)) < 1e-15
    # a pure gain of 2 is 20 log10(2) dB at every bin
    assert abs(oracle.spectral_distortion(2 * h[1], h[1]) - 20 * math.log10(2)) < 1e-9
    assert list(oracle.nnze(np.array([[0.0, 1e-4, 2e-4, -0.5]]))) == [2]


def test_cost_model_crossovers():
    gold = json.load(open(os.path.join(GOLDEN, "cost_model.json")))
    for ny, nx in gold["formula_crossover"].items():
        ny = int(ny)
        assert oracle.crossover(ny) == nx
        assert oracle.direct_cost(nx, ny) < oracle.fft_cost(nx, ny)
        assert oracle.direct_cost(nx + 1, ny) >= oracle.fft_cost(nx + 1, ny)
    lat = gold["latency_50ms_samples"]
    assert round(lat["fs"] * lat["seconds"]) == lat["samples"]
    # the quoted values are within a few taps of the formula's own
    for ny, nx in gold["paper_quoted_crossover"].items():
        assert abs(oracle.crossover(int(ny)) - nx) <= 5
