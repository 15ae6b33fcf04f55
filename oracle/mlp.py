"""Plain FP64 oracle of the learned order/rank selector's network.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): used by ``tests/``
to check the GPU training and inference kernels, never by the product.

The network (the learned form added to the method): a multilayer perceptron
with three hidden layers of 64 ReLU units,

    z  = (x - mu) / sigma                       (fixed input standardisation)
    h1 = relu(W1 z  + b1)      W1: 64 x 8
    h2 = relu(W2 h1 + b2)      W2: 64 x 64
    h3 = relu(W3 h2 + b3)      W3: 64 x 64
    y  = W4 h3 + b4            W4: n_out x 64

trained on the mean squared error L = mean over samples and outputs of
(y - t)^2 with Adam (Kingma and Ba, 2015: bias-corrected first and second
moment estimates).  The parameter vector is laid out as

    [mu(8), sigma(8), W1, b1, W2, b2, W3, b3, W4, b4]

with every W row-major (W[o, k] at o * n_in + k).  mu and sigma are not
trained (their gradient is zero).
"""
import numpy as np

N_IN, N_HID = 8, 64


def layout(n_out):
    """[(name, shape)] in parameter order."""
    return [("mu", (N_IN,)), ("sigma", (N_IN,)),
            ("W1", (N_HID, N_IN)), ("b1", (N_HID,)),
            ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
            ("W3", (N_HID, N_HID)), ("b3", (N_HID,)),
            ("W4", (n_out, N_HID)), ("b4", (n_out,))]


def n_params(n_out):
    return int(sum(np.prod(s) for _, s in layout(n_out)))


def unpack(p, n_out):
    out, o = {}, 0
    for name, shape in layout(n_out):
        k = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d, n_out):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel()
                           for name, _ in layout(n_out)])


def init(n_out, seed, mu=None, sigma=None):
    """He-uniform weights, zero biases (seeded PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = {"mu": np.zeros(N_IN) if mu is None else mu,
         "sigma": np.ones(N_IN) if sigma is None else sigma}
    for k, (n_o, n_i) in (("1", (N_HID, N_IN)), ("2", (N_HID, N_HID)), ("3", (N_HID, N_HID)),
                          ("4", (n_out, N_HID))):
        lim = np.sqrt(6.0 / n_i)
        d["W" + k] = rng.uniform(-lim, lim, size=(n_o, n_i))
        d["b" + k] = np.zeros(n_o)
    return pack(d, n_out)


def forward(p, x, n_out):
    """Outputs y (n, n_out) and the activations needed by the backward pass."""
    P = unpack(p, n_out)
    z = (np.asarray(x, dtype=np.float64) - P["mu"]) / P["sigma"]
    a1 = z @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    a3 = h2 @ P["W3"].T + P["b3"]
    h3 = np.maximum(a3, 0.0)
    y = h3 @ P["W4"].T + P["b4"]
    return y, (z, a1, h1, a2, h2, a3, h3)


def loss(p, x, t, n_out):
    y, _ = forward(p, x, n_out)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(p, x, t, n_out):
    """Gradient of ``loss`` by the chain rule (reverse mode), and the loss."""
    P = unpack(p, n_out)
    y, (z, a1, h1, a2, h2, a3, h3) = forward(p, x, n_out)
    n = y.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / (n * n_out)
    g = {"mu": np.zeros(N_IN), "sigma": np.zeros(N_IN)}
    g["W4"] = dy.T @ h3
    g["b4"] = dy.sum(axis=0)
    d3 = (dy @ P["W4"]) * (a3 > 0)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(axis=0)
    d2 = (d3 @ P["W3"]) * (a2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (a1 > 0)
    g["W1"] = d1.T @ z
    g["b1"] = d1.sum(axis=0)
    return pack(g, n_out), float(np.mean((y - t) ** 2))


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
