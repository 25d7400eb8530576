"""Pins of the surrogate's CPU reference (oracle/mlp_ref.py), on the CPU: its
gradients against central differences, closed forms of the loss, GELU and the
BF16 rounding, so that the GPU comparison rests on something other than the
reference's own formulas."""
import numpy as np

from oracle import mlp_ref as M


def _params(rng, scale=0.08):
    layers = []
    for fin, fout in M.layer_shapes():
        W = rng.normal(0.0, scale, size=(fin, fout))
        b = rng.normal(0.0, 0.1, size=fout)
        layers.append((W, b))
    return M.pack(layers)


NORM = (np.zeros(9), np.ones(9), np.zeros(2), np.ones(2))


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    flat = _params(rng)
    feats = rng.normal(size=(6, 9))
    targets = rng.normal(size=(6, 2))
    loss, g = M.loss_and_grad(flat, feats, targets, NORM)
    # a spread of parameters: first layer (live rows), hidden, last layer (live columns), biases
    shapes = M.layer_shapes()
    offs = np.cumsum([0] + [fi * fo + fo for fi, fo in shapes])
    picks = []
    for l, (fi, fo) in enumerate(shapes):
        for _ in range(4):
            i = rng.integers(0, 9 if l == 0 else fi)
            o = rng.integers(0, 4 if l == len(shapes) - 1 else fo)
            picks.append(offs[l] + i * fo + o)
        picks.append(offs[l] + fi * fo + rng.integers(0, 4 if l == len(shapes) - 1 else fo))
    h = 1e-5
    for k in picks:
        p = flat.copy(); p[k] += h
        lp, _ = M.loss_and_grad(p, feats, targets, NORM)
        p[k] -= 2 * h
        lm, _ = M.loss_and_grad(p, feats, targets, NORM)
        fd = (lp - lm) / (2 * h)
        assert abs(g[k] - fd) <= 1e-7 + 1e-5 * abs(fd), (k, g[k], fd)


def test_padded_parameters_have_no_effect():
    rng = np.random.default_rng(4)
    flat = _params(rng)
    feats = rng.normal(size=(5, 9))
    targets = rng.normal(size=(5, 2))
    _, g = M.loss_and_grad(flat, feats, targets, NORM)
    layers = M.unpack(g)
    assert np.all(layers[0][0][9:] == 0.0)          # unused input rows
    assert np.all(layers[-1][0][:, 4:] == 0.0)      # unused output columns
    assert np.all(layers[-1][1][4:] == 0.0)


def test_loss_closed_form_at_zero_network():
    # zero weights and biases: mu = 0, ln sigma = 0, loss = mean of y^2 / 2
    flat = np.zeros(sum(fi * fo + fo for fi, fo in M.layer_shapes()))
    rng = np.random.default_rng(5)
    feats = rng.normal(size=(7, 9))
    y = rng.normal(size=(7, 2))
    loss, g = M.loss_and_grad(flat, feats, y, NORM)
    assert np.isclose(loss, np.mean(0.5 * y * y))
    bl = M.unpack(g)[-1][1]
    n = y.shape[0]
    assert np.allclose(bl[:2], -y.sum(axis=0) / (2 * n))
    assert np.allclose(bl[2:4], (1.0 - y * y).sum(axis=0) / (2 * n))
    # normalisation: targets shifted and scaled by the norm arrays
    norm = (np.zeros(9), np.ones(9), np.array([1.0, -2.0]), np.array([2.0, 0.5]))
    l2, _ = M.loss_and_grad(flat, feats, y * np.array([2.0, 0.5]) + np.array([1.0, -2.0]), norm)
    assert np.isclose(l2, loss)


def test_gelu_reference_values():
    assert M.gelu(0.0) == 0.0
    assert np.isclose(M.gelu(10.0), 10.0) and abs(M.gelu(-10.0)) < 1e-20
    assert np.isclose(M.gelu(1.0), 0.8413447460685429)  # Phi(1) = 0.8413447...
    z = np.linspace(-4, 4, 33)
    h = 1e-6
    assert np.allclose(M.gelu_grad(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h), atol=1e-8)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.14159, 1e-3])
    r = M.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0            # tie to even
    assert r[2] == 1.0 + 2 ** -6                  # tie rounds up to the even neighbour
    assert r[3] == -2.5 and r[4] == 3.140625
    assert abs(r[5] - 1e-3) / 1e-3 < 2 ** -8
