"""FP64 reference of the learned TENO5 sub-stencil selector (TEST INFRASTRUCTURE ONLY).

The learned part is not in the paper; its definitions are this library's and are stated here
in full so that the GPU kernels can be checked against them:

* input: the 15 face-side features of ``ora_face_features`` (rho, normal velocity, p at the
  five upwind-ordered cells, each as deviations from the centre scaled to [-1, 1]);
* network: 15 -> 32 (ReLU) -> 32 (ReLU) -> 3 logits; parameters flattened as
  W1[15][32], b1[32], W2[32][32], b2[32], W3[32][3], b3[3] (1667 values);
* output: sigmoid(z_k) is the predicted probability that TENO5 keeps sub-stencil k for every
  conserved component (label of ``ora_face_label``); loss: binary cross-entropy with logits,
  averaged over samples and the three outputs; optimiser: Adam.
* BF16 emulation (``emulate=True``) reproduces the rounding points of the GPU kernels: inputs,
  weights, hidden activations and back-propagated deltas are rounded to bfloat16
  (round-to-nearest-even of their FP32 value); biases, accumulations and everything else stay
  in full precision.
"""
import numpy as np

NIN, NH, NOUT = 15, 32, 3
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NOUT)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) from the FP32 value; returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(seed, scale=1.0):
    """He-style seeded initialisation (weights ~ N(0, 2/fan_in), biases 0)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            p[name] = rng.normal(0.0, scale * np.sqrt(2.0 / shp[0]), size=shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p)


def forward(theta, X, emulate=False):
    """Logits z [n][3] and the cache for the backward pass."""
    P = unpack(theta)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    x = r(X)
    W1, W2, W3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    a1 = x @ W1 + P["b1"]
    h1 = r(np.maximum(a1, 0.0))
    a2 = h1 @ W2 + P["b2"]
    h2 = r(np.maximum(a2, 0.0))
    z = h2 @ W3 + P["b3"]
    return z, (x, W1, W2, W3, a1, h1, a2, h2)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def loss_and_grad(theta, X, Y, emulate=False):
    """Mean binary cross-entropy with logits over samples x 3 outputs, and its gradient."""
    z, (x, W1, W2, W3, a1, h1, a2, h2) = forward(theta, X, emulate)
    r = bf16 if emulate else (lambda a: a)
    Y = np.asarray(Y, dtype=np.float64)
    n = z.shape[0]
    loss = np.mean(np.logaddexp(0.0, z) - Y * z)
    dz = (sigmoid(z) - Y) / (n * NOUT)
    dzb = r(dz)
    g = {}
    g["W3"] = h2.T @ dzb
    g["b3"] = dz.sum(axis=0)
    d2 = (dzb @ W3.T) * (a2 > 0)
    d2b = r(d2)
    g["W2"] = h1.T @ d2b
    g["b2"] = d2.sum(axis=0)
    d1 = (d2b @ W2.T) * (a1 > 0)
    d1b = r(d1)
    g["W1"] = x.T @ d1b
    g["b1"] = d1.sum(axis=0)
    return loss, pack(g)


def adam(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new theta, m, v."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def keep_flags(z):
    """Predicted keep bits (bit k = logit k > 0) and confidence min_k |2 sigma(z_k) - 1|."""
    bits = ((z[:, 0] > 0).astype(int) | ((z[:, 1] > 0).astype(int) << 1) | ((z[:, 2] > 0).astype(int) << 2))
    conf = np.min(np.abs(2.0 * sigmoid(z) - 1.0), axis=1)
    return bits, conf
