"""TEST INFRASTRUCTURE -- FP64 CPU oracle of the boiling-curve surrogate network.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this.

A plain numpy statement of what the GPU surrogate kernels compute, in float64: an MLP
4 -> 128 -> 128 -> 2 with exact GELU, g(z) = z Phi(z) = 0.5 z (1 + erf(z / sqrt 2)),
squared-error loss averaged over the batch (summed over the two outputs), its
gradients by the chain rule, and the bias-corrected Adam update (Kingma & Ba, 2015).

Parameter vector of one member (row-major, a layer computes z = h W + b for a row h):
  W1[4][128], b1[128], W2[128][128], b2[128], W3[128][2], b3[2]
"""
import numpy as np
from scipy.special import erf

IN, HID, OUT = 4, 128, 2
SHAPES = (("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, OUT)), ("b3", (OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(vec):
    """Split a parameter vector into named arrays (views)."""
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = vec[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    # d/dz [z Phi(z)] = Phi(z) + z phi(z)
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(vec, X):
    """Outputs [B][2] and the intermediate values the backward pass needs."""
    p = unpack(np.asarray(vec, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ p["W1"] + p["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ p["W2"] + p["b2"]
    H2 = gelu(Z2)
    Y = H2 @ p["W3"] + p["b3"]
    return Y, (X, Z1, H1, Z2, H2)


def loss_and_grad(vec, X, T):
    """Loss = mean over rows of the squared error summed over outputs, and its gradient
    with respect to the parameter vector."""
    p = unpack(np.asarray(vec, dtype=np.float64))
    Y, (X, Z1, H1, Z2, H2) = forward(vec, X)
    B = X.shape[0]
    E = Y - np.asarray(T, dtype=np.float64)
    loss = float((E * E).sum() / B)
    dY = 2.0 * E / B
    g = {"W3": H2.T @ dY, "b3": dY.sum(axis=0)}
    dZ2 = (dY @ p["W3"].T) * gelu_grad(Z2)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"].T) * gelu_grad(Z1)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return loss, pack(g)


def adam_step(vec, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Step t (1-based) of Adam: returns the new (vec, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return vec - lr * mh / (np.sqrt(vh) + eps), m, v
