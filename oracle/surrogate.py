"""Convolutional warm-start surrogate -- oracle (test infrastructure only).

FP64 NumPy reference of every layer of the learned warm start and of its training step: the
3x3 'same' convolution (forward, input gradient, weight gradient), ReLU, 2x2 average pooling,
nearest 2x upsampling, channel concatenation, the 4x4 patch stem and pixel-shuffle head, the
mean-squared error and one Adam step.  The network maps the solver's own inputs (dynamic power,
leakage variation, conductivity) to a predicted converged rise, used as the fixed point's
starting iterate; the fixed-point solve still decides the result.  The paper has no learned
part: the architecture is this project's (a five-level encoder-decoder), described by
``NetSpec``.

Layout: activations are [B][H][W][C] (channels last); conv weights [Cout][3][3][Cin].

Parity: pinned -- the convolution against scipy.signal.correlate2d, every backward against
central finite differences, pooling / upsampling against their adjoint identities, Adam's
first step against its closed form.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------- layers
def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """z[b, y, x, o] = sum_{ky, kx, i} w[o, ky, kx, i] x[b, y + ky - 1, x + kx - 1, i] (+ b[o]),
    zero outside the image."""
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    z = np.zeros((B, H, W, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            z += xp[:, ky:ky + H, kx:kx + W, :] @ w[:, ky, kx, :].T
    if b is not None:
        z += b
    return z


def conv3x3_dgrad(dz: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of sum(dz * conv3x3(x, w)) with respect to x."""
    B, H, W, _ = dz.shape
    dxp = np.zeros((B, H + 2, W + 2, w.shape[3]))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + H, kx:kx + W, :] += dz @ w[:, ky, kx, :]
    return dxp[:, 1:H + 1, 1:W + 1, :]


def conv3x3_wgrad(x: np.ndarray, dz: np.ndarray) -> np.ndarray:
    """Gradient of sum(dz * conv3x3(x, w)) with respect to w, shape [Cout][3][3][Cin]."""
    B, H, W, cin = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros((dz.shape[3], 3, 3, cin))
    dzf = dz.reshape(-1, dz.shape[3])
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = dzf.T @ xp[:, ky:ky + H, kx:kx + W, :].reshape(-1, cin)
    return dw


def relu(z):
    return np.maximum(z, 0.0)


def relu_grad(da, a):
    """Gradient through a = relu(z), expressed with the output a (z > 0 <=> a > 0)."""
    return da * (a > 0)


def avgpool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_grad(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_grad(dy):
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def patchify4(f):
    """[B][n][n][3] -> [B][n/4][n/4][48], vector index (py * 4 + px) * 3 + c."""
    B, n, _, c = f.shape
    return f.reshape(B, n // 4, 4, n // 4, 4, c).transpose(0, 1, 3, 2, 4, 5).reshape(B, n // 4, n // 4, 16 * c)


def unpatchify4(p):
    """[B][n/4][n/4][16] -> [B][n][n], entry (py * 4 + px) of a coarse pixel to (4Y + py, 4X + px)."""
    B, m, _, _ = p.shape
    return p.reshape(B, m, m, 4, 4).transpose(0, 1, 3, 2, 4).reshape(B, 4 * m, 4 * m)


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def mse_grad(y, t):
    return 2.0 * (y - t) / y.size


@dataclass
class Adam:
    """Adam with bias correction: m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
    p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""
    lr: float = 1e-3
    b1: float = 0.9
    b2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: dict = field(default_factory=dict)
    v: dict = field(default_factory=dict)

    def step(self, params: dict, grads: dict):
        self.t += 1
        for k, g in grads.items():
            m = self.m.get(k, np.zeros_like(g))
            v = self.v.get(k, np.zeros_like(g))
            m = self.b1 * m + (1.0 - self.b1) * g
            v = self.b2 * v + (1.0 - self.b2) * g * g
            self.m[k], self.v[k] = m, v
            mh = m / (1.0 - self.b1 ** self.t)
            vh = v / (1.0 - self.b2 ** self.t)
            params[k] = params[k] - self.lr * mh / (np.sqrt(vh) + self.eps)


# ----------------------------------------------------------------------------- network
@dataclass
class NetSpec:
    """Five-level encoder-decoder on the 4x-patchified grid.

    features f = ((q / 1e6 - shift0) * scale0, (ln v - shift1) * scale1, (k0 m / 150 - shift2) * scale2)
    stem     : 4x4 patches of f (48 values) -> width[0], ReLU
    encoder  : level l: conv width[l-1] -> width[l], ReLU, conv width[l] -> width[l], ReLU
               (level 0 starts from the stem output; levels 1..4 from the 2x2 average pool of
               the previous level)
    decoder  : level l = 3..0: conv [upsample2(d_{l+1}), e_l] -> width[l], ReLU (d_4 = e_4)
    head     : per coarse pixel 16 = 4x4 outputs from width[0] channels (+ bias), times out_scale
    """
    n: int = 512
    width: tuple = (32, 48, 64, 96, 128)
    shift: tuple = (1.0, 0.0, 1.0)
    scale: tuple = (1.0, 1.0 / 0.73, 20.0)
    out_scale: float = 10.0
    k0: float = 150.0

    def shapes(self) -> dict:
        """Parameter name -> shape, in the flat parameter order."""
        w = self.width
        s = {"stem.w": (w[0], 48), "stem.b": (w[0],)}
        for l in range(5):
            cin = w[0] if l == 0 else w[l - 1]
            s[f"enc{l}a.w"] = (w[l], 3, 3, cin)
            s[f"enc{l}a.b"] = (w[l],)
            s[f"enc{l}b.w"] = (w[l], 3, 3, w[l])
            s[f"enc{l}b.b"] = (w[l],)
        for l in range(3, -1, -1):
            s[f"dec{l}.w"] = (w[l], 3, 3, w[l + 1] + w[l])
            s[f"dec{l}.b"] = (w[l],)
        s["head.w"] = (16, w[0])
        s["head.b"] = (16,)
        return s

    def param_count(self) -> int:
        return sum(int(np.prod(v)) for v in self.shapes().values())

    def unflatten(self, flat: np.ndarray) -> dict:
        out, o = {}, 0
        for k, shp in self.shapes().items():
            c = int(np.prod(shp))
            out[k] = np.asarray(flat[o:o + c], dtype=np.float64).reshape(shp)
            o += c
        assert o == flat.size
        return out

    def flatten(self, params: dict) -> np.ndarray:
        return np.concatenate([params[k].ravel() for k in self.shapes()])

    def init(self, seed: int = 0) -> dict:
        """He-normal weights (fan-in), zero biases."""
        rng = np.random.default_rng(seed)
        out = {}
        for k, shp in self.shapes().items():
            if k.endswith(".b"):
                out[k] = np.zeros(shp)
            else:
                fan_in = int(np.prod(shp[1:]))
                gain = 1.0 if k.startswith("head") else 2.0
                out[k] = rng.standard_normal(shp) * np.sqrt(gain / fan_in)
        return out


def features(spec: NetSpec, q, v, m):
    """[B][n][n] maps (W/m^2, -, -) -> standardized [B][n][n][3]."""
    f0 = (q / 1e6 - spec.shift[0]) * spec.scale[0]
    f1 = (np.log(v) - spec.shift[1]) * spec.scale[1]
    f2 = (spec.k0 * m / 150.0 - spec.shift[2]) * spec.scale[2]
    return np.stack([f0, f1, f2], axis=-1)


def forward(spec: NetSpec, p: dict, q, v, m):
    """Predicted rise [B][n][n] and the activations the backward pass needs."""
    a = {}
    f = features(spec, q, v, m)
    a["patch"] = patchify4(f)
    a["stem"] = relu(a["patch"] @ p["stem.w"].T + p["stem.b"])
    x = a["stem"]
    for l in range(5):
        if l > 0:
            a[f"pool{l}"] = x = avgpool2(a[f"enc{l - 1}b"])
        a[f"enc{l}a"] = relu(conv3x3(x, p[f"enc{l}a.w"], p[f"enc{l}a.b"]))
        a[f"enc{l}b"] = x = relu(conv3x3(a[f"enc{l}a"], p[f"enc{l}b.w"], p[f"enc{l}b.b"]))
    d = a["enc4b"]
    for l in range(3, -1, -1):
        a[f"cat{l}"] = np.concatenate([upsample2(d), a[f"enc{l}b"]], axis=-1)
        a[f"dec{l}"] = d = relu(conv3x3(a[f"cat{l}"], p[f"dec{l}.w"], p[f"dec{l}.b"]))
    a["head"] = d @ p["head.w"].T + p["head.b"]
    y = spec.out_scale * unpatchify4(a["head"])
    return y, a


def backward(spec: NetSpec, p: dict, a: dict, dy):
    """Gradients of sum(dy * y) with respect to every parameter."""
    g = {}
    w = spec.width
    dh = spec.out_scale * patchify4(dy[..., None])  # [B][m][m][16] (c = 1)
    d = a["dec0"]
    g["head.w"] = dh.reshape(-1, 16).T @ d.reshape(-1, w[0])
    g["head.b"] = dh.reshape(-1, 16).sum(axis=0)
    dd = dh @ p["head.w"]
    denc = {l: None for l in range(5)}
    for l in range(4):
        dz = relu_grad(dd, a[f"dec{l}"])
        g[f"dec{l}.w"] = conv3x3_wgrad(a[f"cat{l}"], dz)
        g[f"dec{l}.b"] = dz.sum(axis=(0, 1, 2))
        dcat = conv3x3_dgrad(dz, p[f"dec{l}.w"])
        cu = w[l + 1]
        denc[l] = dcat[..., cu:]
        dd = upsample2_grad(dcat[..., :cu])  # gradient of d_{l+1} (d_4 = e_4)
    de = dd  # level 4 output
    for l in range(4, -1, -1):
        if denc[l] is not None and l < 4:
            de = de + denc[l]
        dz = relu_grad(de, a[f"enc{l}b"])
        g[f"enc{l}b.w"] = conv3x3_wgrad(a[f"enc{l}a"], dz)
        g[f"enc{l}b.b"] = dz.sum(axis=(0, 1, 2))
        da = conv3x3_dgrad(dz, p[f"enc{l}b.w"])
        dz = relu_grad(da, a[f"enc{l}a"])
        xin = a["stem"] if l == 0 else a[f"pool{l}"]
        g[f"enc{l}a.w"] = conv3x3_wgrad(xin, dz)
        g[f"enc{l}a.b"] = dz.sum(axis=(0, 1, 2))
        dx = conv3x3_dgrad(dz, p[f"enc{l}a.w"])
        if l > 0:
            de = avgpool2_grad(dx)  # into enc{l-1}b, plus its skip gradient next round
        else:
            dstem = dx
    dz = relu_grad(dstem, a["stem"])
    g["stem.w"] = dz.reshape(-1, w[0]).T @ a["patch"].reshape(-1, 48)
    g["stem.b"] = dz.reshape(-1, w[0]).sum(axis=0)
    return g


def loss_and_grads(spec: NetSpec, p: dict, q, v, m, target):
    y, a = forward(spec, p, q, v, m)
    return mse(y, target), backward(spec, p, a, mse_grad(y, target)), y
