"""Pins for the float64 reference of the learned drift surrogate."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_round_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 20000).astype(np.float32),
                        np.array([1.0, 1.00390625, 1.01171875, -2.5, 0.0, 3.0e-39, 65504.0,
                                  1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9], np.float32)])
    ours = mlp.bf16_round(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))


def test_rounding_free_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(3)
    p["b1"] = rng.normal(0, 0.1, 64).astype(np.float32)
    p["b2"] = rng.normal(0, 0.1, 64).astype(np.float32)
    X = rng.uniform(0, 1, (40, 16))
    t = rng.uniform(0, 1, 40)
    g = mlp.backward_f64(p, X, t)
    for key, idx in [("W1", (3, 5)), ("W1", (15, 63)), ("b1", (7,)), ("W2", (10, 20)),
                     ("W2", (63, 0)), ("b2", (33,)), ("w3", (12,)), ("b3", (0,))]:
        fd = mlp.finite_difference(p, X, t, key, idx)
        assert abs(fd - g[key][idx]) <= 1e-6 * max(1.0, abs(fd)), (key, idx, fd, g[key][idx])


def test_model_backward_equals_rounding_free_one_on_the_bf16_grid():
    """With inputs, weights and activations exactly on the bfloat16 grid (small
    dyadic values) every rounding of the model is the identity, so its
    gradients equal those of the rounding-free network."""
    rng = np.random.default_rng(2)
    p = dict(W1=rng.choice([-0.5, -0.25, 0, 0.25, 0.5], (16, 64)).astype(np.float32),
             b1=rng.choice([-0.25, 0, 0.25], 64).astype(np.float32),
             W2=rng.choice([-0.25, 0, 0.25], (64, 64)).astype(np.float32),
             b2=rng.choice([-0.5, 0, 0.5], 64).astype(np.float32),
             w3=rng.choice([-0.5, 0.5], 64).astype(np.float32),
             b3=np.array([0.25], np.float32))
    X = rng.choice([0.0, 0.25, 0.5, 1.0], (32, 16))
    t = rng.choice([0.0, 0.5, 1.0], 32)
    _, gm = mlp.backward(p, X, t)
    gf = mlp.backward_f64(p, X, t)
    for k in gf:
        assert np.allclose(gm[k], gf[k], rtol=0, atol=1e-12), k


def test_adam_first_step_moves_by_the_learning_rate():
    p = dict(a=np.array([1.0, -2.0, 3.0], np.float32))
    g = dict(a=np.array([0.5, -4.0, 1e-3]))
    out = mlp.adam_step(p, g, {}, {}, step=1, lr=1e-2)
    assert np.allclose(out["a"], p["a"] - 1e-2 * np.sign(g["a"]), atol=1e-6)


def test_flat_layout_roundtrip():
    p = mlp.init_params(5)
    v = mlp.flat(p)
    assert v.shape == (5313,)
    q = mlp.unflat(v)
    for k in p:
        assert np.array_equal(p[k], q[k])


def test_abs_terms_bound_every_gradient_and_are_tight_without_cancellation():
    """gradient_abs_terms is the triangle-inequality bound of each gradient
    entry, and equals |gradient| when every term has the same sign (positive
    inputs and weights, outputs above their targets)."""
    rng = np.random.default_rng(4)
    p = mlp.init_params(6)
    X = rng.uniform(0, 1, (48, 16))
    t = rng.uniform(0, 1, 48)
    _, g = mlp.backward(p, X, t)
    a = mlp.gradient_abs_terms(p, X, t)
    for k in g:
        assert np.all(np.abs(g[k]) <= a[k] * (1 + 1e-12) + 1e-300), k
    q = {k: np.abs(v).astype(np.float32) for k, v in p.items()}
    q["b1"] = np.full(64, 0.1, np.float32)
    q["b2"] = np.full(64, 0.1, np.float32)
    t0 = np.full(48, -1.0)
    _, g0 = mlp.backward(q, X, t0)
    a0 = mlp.gradient_abs_terms(q, X, t0)
    for k in g0:
        assert np.allclose(np.abs(g0[k]), a0[k], rtol=1e-12, atol=0), k


def rounded_backward(p, X, t):
    """The backward with the two output gradients rounded to bfloat16 before
    their matrix products (the placement the matrix-core kernels use), built
    here from backward's own pieces for the bound check below."""
    y, c = mlp.forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - t) / n
    dz2 = np.outer(dy, c["w3"]) * (c["z2"] > 0)
    dz2m = mlp.bf16_round(dz2.astype(np.float32)).astype(np.float64)
    dz1 = (dz2m @ c["W2"].T) * (c["z1"] > 0)
    dz1m = mlp.bf16_round(dz1.astype(np.float32)).astype(np.float64)
    return dict(w3=c["h2"].T @ dy, b3=np.array([dy.sum()]), W2=c["h1"].T @ dz2m,
                b2=dz2.sum(0), W1=c["X"].T @ dz1m, b1=dz1.sum(0))


def test_bf16_output_gradients_stay_within_the_stated_bound():
    """Rounding the output gradients to bfloat16 (relative error at most
    u = 2^-9 each, two roundings on the W1 path) moves every entry by at most
    2 u times its absolute-term sum; the bound is not vacuous (the typical
    entry moves by a tenth of it or less, and by more than zero)."""
    rng = np.random.default_rng(5)
    p = mlp.init_params(7)
    p["b1"] = rng.normal(0, 0.2, 64).astype(np.float32)
    p["b2"] = rng.normal(0, 0.2, 64).astype(np.float32)
    X = rng.uniform(0, 1, (512, 16))
    t = rng.uniform(0, 1, 512)
    _, g = mlp.backward(p, X, t)
    r = rounded_backward(p, X, t)
    a = mlp.gradient_abs_terms(p, X, t)
    u = 2.0 ** -9
    moved = 0
    for k in g:
        err = np.abs(r[k] - g[k])
        assert np.all(err <= (2 * u + u * u) * a[k] * (1 + 1e-9)), k
        moved += int((err > 0).sum())
    assert moved > 1000
    ratio = np.abs(r["W1"] - g["W1"]) / np.maximum(2 * u * a["W1"], 1e-300)
    assert np.median(ratio) < 0.1
