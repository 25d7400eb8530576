"""Plain FP64 CPU reference of the surrogate network (test infrastructure only).

Only ``tests/`` and the benchmark's checks use this module; the HIP surrogate
never does.  It is written from the definitions, not from the GPU code:

* network: inputs x (9 features: b/a, c/a, ln k rbar, m, ZYZ Euler angles
  alpha, beta, gamma, cell theta, phi; angles in degrees) mapped to a fixed
  23-wide embedding (``embed``), six hidden layers a_l = GELU(a_{l-1} W_l +
  b_l) of width 512, a linear output layer giving (mu_x, mu_y, s_x, s_y) in
  normalised target units;
* embedding: (x - shift) / scale; the particle-frame unit vectors R^T z,
  R^T x, R^T y (incident direction, both polarisations) and R^T s (cell
  direction) with R = Rz(alpha) Ry(beta) Rz(gamma) taking particle to lab
  coordinates; cos phi, sin phi;
* GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 (the exact form);
* loss: mean over rows and the two outputs of the beta-NLL (Seitzer et al.,
  ICLR 2022) with beta = 1: the Gaussian negative log-likelihood
  0.5 (y - mu)^2 exp(-2 s') + s' (constants dropped) of each element times
  the weight w = exp(2 s') held constant, s' = max(s, S_MIN), S_MIN =
  ln 1e-4 (zero gradient in s below the floor);
* gradients by reverse-mode differentiation written out layer by layer.

Parameters use the library's flat order: for each layer W[in][out] then
bias[out], with in = 128 for the first layer (rows >= 23 unused) and out = 128
for the last (columns >= 4 unused).  With ``bf16=True`` the operands are
rounded where the GPU keeps them in BF16 (inputs, weights, activations,
pre-activations and back-propagated gradients), everything else in FP64.
"""
import numpy as np
from scipy.special import erf

N_IN, N_EMB, IN_PAD, WIDTH, DEPTH, N_OUT, OUT_PAD = 9, 23, 128, 512, 6, 4, 128
S_MIN = np.log(1e-4)


def layer_shapes():
    shapes = []
    for l in range(DEPTH + 1):
        fin = IN_PAD if l == 0 else WIDTH
        fout = OUT_PAD if l == DEPTH else WIDTH
        shapes.append((fin, fout))
    return shapes


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, off = [], 0
    for fin, fout in layer_shapes():
        W = flat[off:off + fin * fout].reshape(fin, fout)
        off += fin * fout
        b = flat[off:off + fout]
        off += fout
        out.append((W, b))
    assert off == flat.size
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def bf16(x):
    """Round to bfloat16 (round to nearest, ties to even) and back to float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def rotation_zyz(alpha, beta, gamma):
    """R = Rz(alpha) Ry(beta) Rz(gamma) (radians), particle to lab coordinates."""
    def rz(t):
        c, s = np.cos(t), np.sin(t)
        return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])

    def ry(t):
        c, s = np.cos(t), np.sin(t)
        return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])
    return rz(alpha) @ ry(beta) @ rz(gamma)


def embed(feats, fs, fc):
    """The fixed 23-wide embedding of feature rows [n, 9] (FP64)."""
    x = np.asarray(feats, np.float64)[:, :N_IN]
    n = x.shape[0]
    out = np.zeros((n, N_EMB))
    out[:, :N_IN] = (x - np.asarray(fs, np.float64)) / np.asarray(fc, np.float64)
    for j in range(n):
        R = rotation_zyz(*np.radians(x[j, 4:7]))
        th, ph = np.radians(x[j, 7]), np.radians(x[j, 8])
        s = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
        vz, vx, vy, vs = R.T @ np.array([0.0, 0.0, 1.0]), R.T @ np.array([1.0, 0.0, 0.0]), \
            R.T @ np.array([0.0, 1.0, 0.0]), R.T @ s
        out[j, 9:21] = np.concatenate([vz, vx, vy, vs])
        out[j, 21:23] = np.cos(ph), np.sin(ph)
    return out


def _round(x, on):
    return bf16(x) if on else x


def forward(flat, feats, norm, bf16_ops=False):
    """Returns (outputs in normalised units [n, 4], cache)."""
    fs, fc, ts, tc = norm
    layers = unpack(flat)
    x = embed(feats, fs, fc)
    a = np.zeros((x.shape[0], IN_PAD))
    a[:, :N_EMB] = x
    a = _round(a, bf16_ops)
    cache = [a]
    zs = []
    for l, (W, b) in enumerate(layers):
        z = a @ _round(W, bf16_ops) + b
        if l < DEPTH:
            zs.append(_round(z, bf16_ops))
            a = _round(gelu(z), bf16_ops)
            cache.append(a)
        else:
            out = z[:, :N_OUT]
    return out, (cache, zs)


def predict(flat, feats, norm, bf16_ops=False):
    """De-normalised predictions [n, 4]: ln I_x, ln I_y, ln sigma_x, ln sigma_y."""
    out, _ = forward(flat, feats, norm, bf16_ops)
    ts, tc = np.asarray(norm[2], np.float64), np.asarray(norm[3], np.float64)
    return np.concatenate([out[:, :2] * tc + ts, out[:, 2:] + np.log(tc)], axis=1)


def loss_and_grad(flat, feats, targets, norm, bf16_ops=False, weights=None):
    """Mean beta-NLL (beta = 1) over rows and outputs, and its gradient (flat
    order).  ``weights`` [n, 2], if given, replaces the per-element weights
    exp(2 s') (the loss is then a plain function of the parameters, whose
    central differences pin the gradient at the point the weights came from)."""
    ts, tc = np.asarray(norm[2], np.float64), np.asarray(norm[3], np.float64)
    out, (acts, zs) = forward(flat, feats, norm, bf16_ops)
    n = out.shape[0]
    y = (np.asarray(targets, np.float64) - ts) / tc
    mu, s_raw = out[:, :2], out[:, 2:]
    s = np.maximum(s_raw, S_MIN)
    e = np.exp(-2.0 * s)
    w = np.exp(2.0 * s) if weights is None else np.asarray(weights, np.float64)
    d = y - mu
    nll = 0.5 * d * d * e + s
    loss = np.sum(w * nll) / (2.0 * n)
    g = np.zeros((n, OUT_PAD))
    g[:, :2] = -w * d * e / (2.0 * n)
    g[:, 2:4] = np.where(s_raw > S_MIN, w * (1.0 - d * d * e) / (2.0 * n), 0.0)
    g = _round(g, bf16_ops)
    layers = unpack(flat)
    grads = [None] * len(layers)
    for l in range(DEPTH, -1, -1):
        W, b = layers[l]
        grads[l] = (acts[l].T @ g, g.sum(axis=0))
        if l > 0:
            g = _round((g @ _round(W, bf16_ops).T) * gelu_grad(zs[l - 1]), bf16_ops)
    return loss, pack(grads)


def elementwise_weights(flat, feats, norm):
    """The weights exp(2 max(s, S_MIN)) [n, 2] of the beta-NLL at these parameters."""
    out, _ = forward(flat, feats, norm)
    return np.exp(2.0 * np.maximum(out[:, 2:], S_MIN))
