"""Pins of the surrogate oracle: bfloat16 rounding against its definition's
boundary cases and torch's own conversion, the backward pass against
central finite differences of the forward pass, and Adam's first step
against its closed form."""
import numpy as np
import pytest

import oracle.mlp as M
import synth


def test_bf16_rounding_boundaries():
    u = 2.0 ** -7                     # bf16 spacing in [1, 2)
    cases = {1.0: 1.0, 1.0 + u / 2: 1.0, 1.0 + 1.5 * u: 1.0 + 2 * u, 1.0 + 0.51 * u: 1.0 + u,
             -(1.0 + 1.5 * u): -(1.0 + 2 * u), 0.0: 0.0, 3.0: 3.0, 2.0 ** -130: 2.0 ** -130}
    for x, want in cases.items():
        assert M.bf16(np.array([x]))[0] == want, x


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000), rng.standard_normal(2000) * 1e-20,
                        rng.standard_normal(2000) * 1e20]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x.astype(np.float64)), ref)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = synth.mlp_params(3, [4, 7, 6, 5])
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    X = rng.standard_normal((9, 4))
    T = np.abs(rng.standard_normal((9, 5)))
    _, grads = M.loss_and_grads(params, X, T, rounding=False)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = M.loss_and_grads(params, X, T, rounding=False)
                arr[idx] = old - h
                lm, _ = M.loss_and_grads(params, X, T, rounding=False)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (li, idx, fd, g[idx])


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(2)
    params = [(rng.standard_normal((3, 2)), rng.standard_normal(2))]
    grads = [(rng.standard_normal((3, 2)), rng.standard_normal(2))]
    lr = 1e-2
    new, _ = M.adam_step(params, grads, M.zero_state(params), 1, lr)
    for (p, g), q in zip(((params[0][0], grads[0][0]), (params[0][1], grads[0][1])), new[0]):
        # step 1: m_hat = g, v_hat = g^2, so the step is lr * g / (|g| + eps)
        np.testing.assert_allclose(q, p - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_forward_rounds_hidden_activations_only_and_output_is_linear():
    rng = np.random.default_rng(4)
    params = synth.mlp_params(5, [4, 16, 3])
    X = rng.standard_normal((5, 4))
    y, cache = M.forward(params, X)
    h1 = cache[1][0]
    np.testing.assert_array_equal(h1, M.bf16(h1))             # hidden activations are bf16 values
    np.testing.assert_array_equal(cache[0][0], M.bf16(X))      # and so is the input
    np.testing.assert_array_equal(y, h1 @ params[1][0] + params[1][1])   # linear output layer
