"""FP64 oracle of the learned warm start (test infrastructure).

Plain numpy definitions, written independently of the GPU kernels:
  * the 130 per-state features of a 3-D m^3 GridWorld (normalised
    coordinates, the clamped 5x5x5 reward window, gamma, slip), built here by
    edge-padding the reward cube and slicing;
  * the 130 -> 256 -> 256 -> 1 ReLU MLP, its mean-squared-error loss on
    (1 - gamma) V*, and the gradient by backpropagation;
  * Adam (Kingma & Ba 2015: beta1 0.9, beta2 0.999, eps 1e-8, bias
    corrected);
  * SplitMix64 (Steele, Lea & Flood 2014), the counter-based generator that
    draws minibatch indices, and the sampling rule of a training step.
Parameter layout: W1 [130, 256], b1 [256], W2 [256, 256], b2 [256], w3 [256],
b3 [1], flattened in that order (99,585 values).
"""
import numpy as np

F, H = 130, 256
SIZES = [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
R_SCALE, G_MEAN, G_SCALE, S_MEAN, S_SCALE = 10.0, 0.945, 1 / 0.026, 0.175, 1 / 0.072
OUT_MEAN, OUT_SCALE = 0.2, 0.05       # (1 - gamma) V = OUT_MEAN + OUT_SCALE * y


def target(V, gamma):
    """Training target of the network output for value V."""
    return ((1.0 - gamma) * np.asarray(V, np.float64) - OUT_MEAN) / OUT_SCALE


def values(y, gamma):
    """Warm-start values from network outputs."""
    return (OUT_MEAN + OUT_SCALE * np.asarray(y, np.float64)) / (1.0 - gamma)


def unpack(p):
    out, off = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[off:off + n], np.float64).reshape(shape)
        off += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def features(R, m, gamma, slip, states):
    """Rows of the feature matrix for the listed states (row-major index of
    Def. 2: last coordinate fastest)."""
    cube = np.asarray(R, np.float64).reshape(m, m, m)
    padded = np.pad(cube, 2, mode="edge")       # clamped coordinates
    states = np.asarray(states, np.int64)
    i0, i1, i2 = states // (m * m), (states // m) % m, states % m
    X = np.empty((states.size, F))
    scale = 1.0 / (m - 1) if m > 1 else 0.0
    X[:, 0], X[:, 1], X[:, 2] = i0 * scale, i1 * scale, i2 * scale
    for r, (a, b, c) in enumerate(zip(i0, i1, i2)):
        X[r, 3:128] = R_SCALE * padded[a:a + 5, b:b + 5, c:c + 5].ravel()
    X[:, 128] = (gamma - G_MEAN) * G_SCALE
    X[:, 129] = (slip - S_MEAN) * S_SCALE
    return X


def forward(p, X):
    q = unpack(p)
    Z1 = X @ q["W1"] + q["b1"]
    H1 = np.maximum(Z1, 0)
    Z2 = H1 @ q["W2"] + q["b2"]
    H2 = np.maximum(Z2, 0)
    y = H2 @ q["w3"] + q["b3"][0]
    return y, (X, Z1, H1, Z2, H2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - t) ** 2))


def loss_grad(p, X, t):
    """Loss and its gradient (flat, FP64) by backpropagation."""
    q = unpack(p)
    y, (X, Z1, H1, Z2, H2) = forward(p, X)
    B = X.shape[0]
    dy = 2.0 * (y - t) / B
    g = {"w3": H2.T @ dy, "b3": np.array([dy.sum()])}
    dZ2 = np.outer(dy, q["w3"]) * (Z2 > 0)
    g["W2"], g["b2"] = H1.T @ dZ2, dZ2.sum(axis=0)
    dZ1 = (dZ2 @ q["W2"].T) * (Z1 > 0)
    g["W1"], g["b1"] = X.T @ dZ1, dZ1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), pack(g)


def adam(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


_MASK = (1 << 64) - 1


def splitmix64(x):
    """One SplitMix64 output for state x (Python ints, 64-bit wrap)."""
    z = (int(x) + 0x9E3779B97F4A7C15) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def sample(seed, step, i, n_inst, S):
    """(instance, state) of sample i of training step `step`."""
    r = splitmix64(int(seed) ^ splitmix64((int(step) * 0x100000001B3 + int(i)) & _MASK))
    return (r >> 32) % n_inst, (r & 0xFFFFFFFF) % S
