"""MLP surrogate of the greedy error indicator, oracle side (test infrastructure only).

Not part of the paper: the surrogate ranks the training-set candidates of the greedy
(the argmax of Alg. 4) so that the true indicator is only evaluated on a short list.
Network: P -> H -> H -> 1 with exact-erf GELU, MSE loss on log10(indicator), Adam.
Everything here is float64 and written out by hand (no autograd).

Random numbers (initial weights, exploration picks) come from SplitMix64 used as a
counter-based generator: value(seed, i) = mix(seed + (i + 1) * 0x9E3779B97F4A7C15),
with mix the SplitMix64 finaliser (Steele, Lea, Flood 2014).  The GPU library
implements the same published definition independently.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def splitmix64(seed: int, i: int) -> int:
    z = (seed + (i + 1) * GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def uniform01(seed: int, i: int) -> float:
    """Uniform double in [0, 1) from the top 53 bits."""
    return (splitmix64(seed, i) >> 11) * (1.0 / (1 << 53))


def gelu(x):
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def features(mu, lo, hi):
    """Inputs centred to [-1, 1]: (log10 mu - mid) / half-width of the log range."""
    l0, l1 = math.log10(lo), math.log10(hi)
    return (np.log10(mu) - 0.5 * (l0 + l1)) / (0.5 * (l1 - l0))


PARAM_NAMES = ("W1", "b1", "W2", "b2", "w3", "b3")


def init_params(P, H, seed):
    """Glorot-uniform weights (counter order W1, W2, w3, row-major), zero biases."""
    shapes = {"W1": (H, P), "W2": (H, H), "w3": (1, H)}
    params = {}
    counter = 0
    for name in ("W1", "W2", "w3"):
        fo, fi = shapes[name]
        a = math.sqrt(6.0 / (fi + fo))
        vals = np.array([uniform01(seed, counter + k) for k in range(fo * fi)])
        counter += fo * fi
        params[name] = ((2.0 * vals - 1.0) * a).reshape(fo, fi)
    params["b1"] = np.zeros(H)
    params["b2"] = np.zeros(H)
    params["b3"] = np.zeros(1)
    return params


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), returned as float64: the FP32 value
    keeps its top 16 bits after adding half an ulp of BF16 plus the tie-break bit."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _mm(A, B, bf16):
    """A @ B; in BF16 mode both operands are rounded to BF16 first and the result is
    kept in FP32 (products accumulated here in FP64, then rounded once)."""
    if not bf16:
        return A @ B
    return _f32(bf16_round(A) @ bf16_round(B))


def forward(params, X, cache=False, bf16=False):
    """Output of the network for the rows of X.  bf16: every product takes BF16 operands
    and every stored activation is FP32 (the reduced-precision mode of the surrogate)."""
    rnd = _f32 if bf16 else (lambda v: v)
    z1 = rnd(_mm(X, params["W1"].T, bf16) + params["b1"])
    a1 = rnd(gelu(z1))
    z2 = rnd(_mm(a1, params["W2"].T, bf16) + params["b2"])
    a2 = rnd(gelu(z2))
    out = rnd(_mm(a2, params["w3"].T, bf16) + params["b3"])
    out = out[:, 0]
    if cache:
        return out, (X, z1, a1, z2, a2)
    return out


def loss_and_grads(params, X, y, bf16=False):
    """MSE loss (mean over rows) and its gradients by hand-written backprop (bf16: the
    products' operands rounded to BF16 and the intermediates kept in FP32, as forward)."""
    rnd = _f32 if bf16 else (lambda v: v)
    out, (X, z1, a1, z2, a2) = forward(params, X, cache=True, bf16=bf16)
    m = X.shape[0]
    diff = out - y
    loss = float(np.mean(diff * diff))
    g_out = rnd((2.0 / m) * diff[:, None])             # d loss / d out
    g = {}
    g["w3"] = _mm(g_out.T, a2, bf16)
    g["b3"] = rnd(g_out.sum(axis=0))
    g_a2 = _mm(g_out, params["w3"], bf16)
    g_z2 = rnd(g_a2 * gelu_grad(z2))
    g["W2"] = _mm(g_z2.T, a1, bf16)
    g["b2"] = rnd(g_z2.sum(axis=0))
    g_a1 = _mm(g_z2, params["W2"], bf16)
    g_z1 = rnd(g_a1 * gelu_grad(z1))
    g["W1"] = _mm(g_z1.T, X, bf16)
    g["b1"] = rnd(g_z1.sum(axis=0))
    return loss, g


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for k in params:
            g = grads[k]
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * g * g
            mhat = self.m[k] / c1
            vhat = self.v[k] / c2
            params[k] = params[k] - self.lr * mhat / (np.sqrt(vhat) + self.eps)
        return params
