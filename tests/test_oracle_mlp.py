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
    # the beta-NLL's weights are held constant: differentiate the loss with the
    # weights frozen at this point
    w = M.elementwise_weights(flat, feats, NORM)
    assert np.isclose(M.loss_and_grad(flat, feats, targets, NORM, weights=w)[0], loss)
    # a spread of parameters: first layer (live rows), hidden, last layer (live columns), biases
    shapes = M.layer_shapes()
    offs = np.cumsum([0] + [fi * fo + fo for fi, fo in shapes])
    picks = []
    for l, (fi, fo) in enumerate(shapes):
        for _ in range(4):
            i = rng.integers(0, M.N_EMB if l == 0 else fi)
            o = rng.integers(0, 4 if l == len(shapes) - 1 else fo)
            picks.append(offs[l] + i * fo + o)
        picks.append(offs[l] + fi * fo + rng.integers(0, 4 if l == len(shapes) - 1 else fo))
    h = 1e-5
    for k in picks:
        p = flat.copy(); p[k] += h
        lp, _ = M.loss_and_grad(p, feats, targets, NORM, weights=w)
        p[k] -= 2 * h
        lm, _ = M.loss_and_grad(p, feats, targets, NORM, weights=w)
        fd = (lp - lm) / (2 * h)
        assert abs(g[k] - fd) <= 1e-7 + 1e-5 * abs(fd), (k, g[k], fd)


def test_padded_parameters_have_no_effect():
    rng = np.random.default_rng(4)
    flat = _params(rng)
    feats = rng.normal(size=(5, 9))
    targets = rng.normal(size=(5, 2))
    _, g = M.loss_and_grad(flat, feats, targets, NORM)
    layers = M.unpack(g)
    assert np.all(layers[0][0][M.N_EMB:] == 0.0)    # unused input rows
    assert np.all(layers[-1][0][:, 4:] == 0.0)      # unused output columns
    assert np.all(layers[-1][1][4:] == 0.0)


def test_loss_closed_form_at_zero_network():
    # zero weights and biases: mu = 0, ln sigma = 0 (weights 1), loss = mean of y^2 / 2
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


def _feat(alpha, beta, gamma, theta, phi, m=1.4):
    return np.array([[1.0, 1.1, 5.0, m, alpha, beta, gamma, theta, phi]])


def test_embedding_frame_at_identity():
    e = M.embed(_feat(0.0, 0.0, 0.0, 130.0, 40.0), np.zeros(9), np.ones(9))[0]
    th, ph = np.radians(130.0), np.radians(40.0)
    assert np.allclose(e[9:12], [0, 0, 1]) and np.allclose(e[12:15], [1, 0, 0]) and np.allclose(e[15:18], [0, 1, 0])
    assert np.allclose(e[18:21], [np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    assert np.allclose(e[21:23], [np.cos(ph), np.sin(ph)])
    assert e.size == M.N_EMB


def test_embedding_frame_is_orthonormal_and_right_handed():
    rng = np.random.default_rng(8)
    for _ in range(20):
        a, g = rng.uniform(-180, 180, 2)
        b = rng.uniform(0, 180)
        e = M.embed(_feat(a, b, g, rng.uniform(120, 170), rng.uniform(0, 360)), np.zeros(9), np.ones(9))[0]
        vz, vx, vy, vs = e[9:12], e[12:15], e[15:18], e[18:21]
        for v in (vz, vx, vy, vs):
            assert abs(np.linalg.norm(v) - 1.0) < 1e-12
        assert np.allclose(np.cross(vx, vy), vz, atol=1e-12)


def test_embedding_euler_convention_matches_the_particle_generator():
    from paper_2403_13856_amd import inputs as I
    rng = np.random.default_rng(9)
    for _ in range(10):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                      [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                      [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
        eul = I._quat_to_zyz_deg((w, x, y, z))
        assert np.allclose(M.rotation_zyz(*np.radians(eul)), R, atol=1e-12)


def test_embedding_symmetries():
    rng = np.random.default_rng(10)
    for _ in range(10):
        a, g, ph, d = rng.uniform(-180, 180, 4)
        b, th = rng.uniform(0, 180), rng.uniform(120, 170)
        e0 = M.embed(_feat(a, b, g, th, ph), np.zeros(9), np.ones(9))[0]
        # turning particle and cell together about the incident axis keeps the
        # incident and cell directions in the particle frame and the rainbow terms
        e1 = M.embed(_feat(a + d, b, g, th, ph + d), np.zeros(9), np.ones(9))[0]
        assert np.allclose(e0[9:12], e1[9:12], atol=1e-12) and np.allclose(e0[18:21], e1[18:21], atol=1e-12)
        # a half turn of the particle about its own first axis flips the second
        # and third particle-frame components of every vector
        R = M.rotation_zyz(*np.radians([a, b, g])) @ np.diag([1.0, -1.0, -1.0])
        beta = np.degrees(np.arccos(np.clip(R[2, 2], -1, 1)))
        alpha = np.degrees(np.arctan2(R[1, 2], R[0, 2]))
        gamma = np.degrees(np.arctan2(R[2, 1], -R[2, 0]))
        e2 = M.embed(_feat(alpha, beta, gamma, th, ph), np.zeros(9), np.ones(9))[0]
        for v in range(4):
            sl = slice(9 + 3 * v, 12 + 3 * v)
            assert np.allclose(e2[sl], e0[sl] * [1, -1, -1], atol=1e-9)


def test_loss_floor_of_log_sigma():
    # last-layer bias alone sets the outputs: mu = b0, ln sigma = b2 (normalised)
    flat = np.zeros(sum(fi * fo + fo for fi, fo in M.layer_shapes()))
    layers = M.unpack(flat)
    rng = np.random.default_rng(11)
    feats = rng.normal(size=(5, 9))
    y = rng.normal(size=(5, 2))
    for s_val, live in ((-20.0, False), (-3.0, True), (0.7, True)):
        b = layers[-1][1].copy()
        b[2:4] = s_val
        lay = [(W, bb) for W, bb in layers[:-1]] + [(layers[-1][0], b)]
        loss, g = M.loss_and_grad(M.pack(lay), feats, y, NORM)
        s_eff = max(s_val, np.log(1e-4))
        # weight sigma^2 = exp(2 s) times the NLL: 0.5 y^2 + s exp(2 s)
        assert np.isclose(loss, np.mean(0.5 * y * y + s_eff * np.exp(2 * s_eff)))
        gb = M.unpack(g)[-1][1]
        # mean gradient that of the squared error, whatever sigma
        assert np.allclose(gb[:2], -y.sum(axis=0) / (2 * y.shape[0]))
        expect = (np.exp(2 * s_eff) - y * y).sum(axis=0) / (2 * y.shape[0]) if live else np.zeros(2)
        assert np.allclose(gb[2:4], expect)
