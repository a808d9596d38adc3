"""FP64 reference of the velocity-surrogate MLP (TEST INFRASTRUCTURE ONLY).

Network 3 -> 64 -> 64 -> 64 -> 1 with the exact GELU, g(z) = z Phi(z) =
z (1 + erf(z / sqrt 2)) / 2, on inputs mapped by x' = (x - shift) / scale and
targets mapped the same way; loss = mean over points of (v' - y')^2.

With emulate_bf16 the reference rounds (round-to-nearest-even) exactly where
the GPU kernels round to bfloat16: the weights W1..W4, the hidden activations
h1..h3, and the back-propagated pre-activation gradients dz3, dz2 where they
enter the matrix products; everything else is float64.  Without it, the
function is the plain float64 network, whose gradient a central finite
difference can check.

Parameter vector layout (8641): W1[64][3] b1[64] W2[64][64] b2[64] W3[64][64]
b3[64] W4[64] b4.

adam_step is one step of Adam (Kingma and Ba, "Adam: a method for stochastic
optimization", ICLR 2015, Algorithm 1) in float64: exponential moving
averages of the gradient and of its square, both divided by their bias
corrections, and a step of lr times their ratio.
"""
import numpy as np
from scipy.special import erf

NPARAM = 8641
LAYOUT = [("W1", 0, (64, 3)), ("b1", 192, (64,)), ("W2", 256, (64, 64)), ("b2", 4352, (64,)),
          ("W3", 4416, (64, 64)), ("b3", 8512, (64,)), ("W4", 8576, (64,)), ("b4", 8640, ())]


def bf16(x):
    """Round to bfloat16 (via float32, round to nearest even) and return float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    out = {}
    for name, off, shape in LAYOUT:
        size = int(np.prod(shape)) if shape else 1
        out[name] = p[off:off + size].reshape(shape) if shape else p[off]
    return out


def pack(d):
    p = np.zeros(NPARAM)
    for name, off, shape in LAYOUT:
        size = int(np.prod(shape)) if shape else 1
        p[off:off + size] = np.asarray(d[name], dtype=np.float64).reshape(size)
    return p


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def _maps(in_shift, in_scale):
    return np.asarray(in_shift, np.float64), np.asarray(in_scale, np.float64)


def forward(params, X, in_shift=(0, 0, 0), in_scale=(1, 1, 1), out_shift=0.0, out_scale=1.0,
            emulate_bf16=True, log_target=False):
    """Predicted v (target units) for X [n, 3]; also returns the cache for backward.
    With log_target the output map is v = exp(v' scale + shift)."""
    P = unpack(params)
    rnd = bf16 if emulate_bf16 else (lambda a: np.asarray(a, np.float64))
    sh, sc = _maps(in_shift, in_scale)
    x = (np.asarray(X, np.float64) - sh) / sc
    W1, W2, W3, W4 = rnd(P["W1"]), rnd(P["W2"]), rnd(P["W3"]), rnd(P["W4"])
    z1 = x @ W1.T + P["b1"]
    h1 = rnd(gelu(z1))
    z2 = h1 @ W2.T + P["b2"]
    h2 = rnd(gelu(z2))
    z3 = h2 @ W3.T + P["b3"]
    h3 = rnd(gelu(z3))
    vp = h3 @ W4 + P["b4"]
    cache = dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3, vp=vp, W2=W2, W3=W3, W4=W4)
    o = vp * out_scale + out_shift
    return (np.exp(o) if log_target else o), cache


def loss_and_grad(params, X, y, in_shift=(0, 0, 0), in_scale=(1, 1, 1), out_shift=0.0,
                  out_scale=1.0, emulate_bf16=True, log_target=False):
    """(loss in mapped units, gradient [8641]) of the mean squared error; with
    log_target the targets are mapped as (log y - shift) / scale."""
    rnd = bf16 if emulate_bf16 else (lambda a: np.asarray(a, np.float64))
    _, C = forward(params, X, in_shift, in_scale, out_shift, out_scale, emulate_bf16)
    n = len(C["vp"])
    yv = np.asarray(y, np.float64)
    yt = ((np.log(yv) if log_target else yv) - out_shift) / out_scale
    e = C["vp"] - yt
    loss = float(np.mean(e * e))
    dv = 2.0 * e / n
    g = {}
    g["W4"] = C["h3"].T @ dv
    g["b4"] = dv.sum()
    dz3 = np.outer(dv, C["W4"]) * gelu_grad(C["z3"])
    g["b3"] = dz3.sum(0)
    dz3r = rnd(dz3)
    g["W3"] = dz3r.T @ C["h2"]
    dz2 = (dz3r @ C["W3"]) * gelu_grad(C["z2"])
    g["b2"] = dz2.sum(0)
    dz2r = rnd(dz2)
    g["W2"] = dz2r.T @ C["h1"]
    dz1 = (dz2r @ C["W2"]) * gelu_grad(C["z1"])
    g["b1"] = dz1.sum(0)
    g["W1"] = dz1.T @ C["x"]
    return loss, pack(g)


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at step number t >= 1 (the first step is t = 1).

    m <- beta1 m + (1 - beta1) g,  v <- beta2 v + (1 - beta2) g^2,
    params <- params - lr mhat / (sqrt(vhat) + eps) with the bias-corrected
    mhat = m / (1 - beta1^t) and vhat = v / (1 - beta2^t).
    Returns new (params, m, v) as float64 arrays."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    p = np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
