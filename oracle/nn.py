"""FP64 reference of the learned warm start: a spectral-convolution neural operator.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain NumPy, float64; the
backward pass is written from hand-derived adjoints and is pinned against
central finite differences in tests/test_oracle_nn.py.

Network (hyper-parameters in NNConfig; n x n tiles, W channels, M modes):
  inputs  f (B, cin, n, n) real
  lift    h_0 = P_w f + P_b                         (pointwise, cin -> W)
  layers  h_{l+1} = act_l(K_l h_l + W_l h_l + c_l),  l = 0 .. L-1,
          act = GELU (tanh form) except after the last layer (identity)
  project y = Q_w h_L + Q_b                         (pointwise, W -> 2)
  spectral convolution K h = Finv(R . Ftrunc(h)):
    Ftrunc  H[a, k] = sum_{y,x} h[y, x] exp(-2 pi i (ky(a) y + k x) / n)
            for k = 0..M-1 and ky(a) = a (a < M), n - 2M + a (a >= M)
    mixing  G[o, a, k] = sum_i R[i, o, a, k] H[i, a, k]       (complex R)
    Finv    g[y, x] = n^-2 Re sum_{a,k} w_k G[a, k] exp(+2 pi i (ky(a) y + k x) / n),
            w_0 = 1, w_k = 2 (k >= 1): the real field of the truncated
            Hermitian half-spectrum, equal to numpy.fft.irfft2 of it.
Loss: mean over samples of |y - t|^2 / |t|^2.  Optimiser: Adam on an FP32 master
copy of the parameters; the network computes with that copy rounded to BF16
(quantize_bf16), so its forward and gradients are evaluated at the rounded
weights (the callers pass them to forward/backward).

Gradients use the convention grad = dL/dRe + i dL/dIm for complex quantities:
  through Finv:   dG = w_k n^-2 Ftrunc(dg)
  through mixing: dH_i = sum_o conj(R_io) dG_o,   dR_io = sum_b conj(H_i) dG_o
  through Ftrunc: dh = Re(Ey^H dH Ex^H)
Parameter order of the flat vector (shared with the GPU library's layout):
  P_w (W, cin), P_b (W), then per layer Re R (W, W, 2M, M), Im R, W_l (W, W),
  c_l (W), then Q_w (2, W), Q_b (2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class NNConfig:
    n: int = 256        # tile side (nodes)
    width: int = 16     # channels W
    modes: int = 16     # M: kx in [0, M), ky in [-M, M)
    layers: int = 4     # L
    cin: int = 3        # input features

    def shapes(self):
        W, M, c = self.width, self.modes, self.cin
        s = [("P_w", (W, c)), ("P_b", (W,))]
        for l in range(self.layers):
            s += [("R%d_re" % l, (W, W, 2 * M, M)), ("R%d_im" % l, (W, W, 2 * M, M)),
                  ("W%d" % l, (W, W)), ("c%d" % l, (W,))]
        s += [("Q_w", (2, W)), ("Q_b", (2,))]
        return s

    def nparams(self):
        return int(sum(np.prod(sh) for _, sh in self.shapes()))


def unflatten(cfg, flat):
    out, o = {}, 0
    for name, sh in cfg.shapes():
        k = int(np.prod(sh))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(sh)
        o += k
    assert o == len(flat)
    return out


def flatten(cfg, d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in cfg.shapes()])


def ky_index(cfg):
    M, n = cfg.modes, cfg.n
    return np.array([a if a < M else n - 2 * M + a for a in range(2 * M)])


def dft_mats(cfg):
    n, M = cfg.n, cfg.modes
    x = np.arange(n)
    Ex = np.exp(-2j * np.pi * np.outer(x, np.arange(M)) / n)        # (n, M)
    Ey = np.exp(-2j * np.pi * np.outer(ky_index(cfg), x) / n)       # (2M, n)
    wk = np.full(M, 2.0)
    wk[0] = 1.0
    return Ex, Ey, wk


def ftrunc(cfg, h):
    """Truncated 2D DFT of real planes h (..., n, n) -> (..., 2M, M) complex."""
    Ex, Ey, _ = dft_mats(cfg)
    return Ey @ (h @ Ex)


def finv(cfg, G):
    """Real field of the truncated half-spectrum G (..., 2M, M) -> (..., n, n)."""
    Ex, Ey, wk = dft_mats(cfg)
    return np.real(np.conj(Ey).T @ (G * wk) @ np.conj(Ex).T) / cfg.n ** 2


_C = np.sqrt(2.0 / np.pi)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(_C * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    u = _C * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * _C * (1.0 + 3 * 0.044715 * x * x)


def _pw(Wm, h):
    return np.einsum("oi,biyx->boyx", Wm, h)


def forward(cfg, p, f):
    """Returns (y, cache).  p: dict from unflatten; f: (B, cin, n, n)."""
    h = _pw(p["P_w"], f) + p["P_b"][None, :, None, None]
    cache = {"f": f, "h": [h], "H": [], "pre": []}
    for l in range(cfg.layers):
        R = p["R%d_re" % l] + 1j * p["R%d_im" % l]
        H = ftrunc(cfg, h)                                        # (B, W, 2M, M)
        G = np.einsum("ioak,biak->boak", R, H)
        pre = finv(cfg, G) + _pw(p["W%d" % l], h) + p["c%d" % l][None, :, None, None]
        h = gelu(pre) if l < cfg.layers - 1 else pre
        cache["H"].append(H)
        cache["pre"].append(pre)
        cache["h"].append(h)
    y = _pw(p["Q_w"], h) + p["Q_b"][None, :, None, None]
    return y, cache


def loss_and_grad(y, t):
    """Mean relative squared error over samples and its gradient w.r.t. y."""
    B = y.shape[0]
    d = y - t
    den = np.sum(t * t, axis=(1, 2, 3))
    loss = float(np.mean(np.sum(d * d, axis=(1, 2, 3)) / den))
    return loss, 2.0 * d / (B * den[:, None, None, None])


def backward(cfg, p, cache, dy):
    """Gradients of a scalar loss with dL/dy = dy: (dict of parameter grads, dL/df)."""
    g = {}
    hL = cache["h"][-1]
    g["Q_w"] = np.einsum("boyx,biyx->oi", dy, hL)
    g["Q_b"] = dy.sum(axis=(0, 2, 3))
    dh = np.einsum("oi,boyx->biyx", p["Q_w"], dy)
    Ex, Ey, wk = dft_mats(cfg)
    for l in reversed(range(cfg.layers)):
        pre, h, H = cache["pre"][l], cache["h"][l], cache["H"][l]
        dpre = dh * gelu_grad(pre) if l < cfg.layers - 1 else dh
        g["c%d" % l] = dpre.sum(axis=(0, 2, 3))
        g["W%d" % l] = np.einsum("boyx,biyx->oi", dpre, h)
        dh = np.einsum("oi,boyx->biyx", p["W%d" % l], dpre)
        dG = wk * ftrunc(cfg, dpre) / cfg.n ** 2                 # (B, W, 2M, M)
        R = p["R%d_re" % l] + 1j * p["R%d_im" % l]
        dR = np.einsum("biak,boak->ioak", np.conj(H), dG)
        g["R%d_re" % l] = dR.real
        g["R%d_im" % l] = dR.imag
        dH = np.einsum("ioak,boak->biak", np.conj(R), dG)
        dh = dh + np.real(np.conj(Ey).T @ dH @ np.conj(Ex).T)
    g["P_w"] = np.einsum("boyx,biyx->oi", dh, cache["f"])
    g["P_b"] = dh.sum(axis=(0, 2, 3))
    df = np.einsum("oi,boyx->biyx", p["P_w"], dh)
    return g, df


def quantize_bf16(flat):
    """The weights the network computes with: every parameter rounded to FP32
    (the master copy's format), then to BF16, the upper 16 bits of an IEEE
    binary32 (8 exponent bits, 7 fraction bits), by round to nearest with ties
    to even; returned as float64 (exactly representable).  Finite inputs only."""
    u = np.ascontiguousarray(np.asarray(flat, dtype=np.float64).astype(np.float32)).view(np.uint32)
    u = u.astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def adam(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) on flat arrays; step counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Deployment: features of a tile and the blended initial guess.
# ---------------------------------------------------------------------------
EPS_SCALE = 0.25      # f0 = (Re eps_node - 1) * EPS_SCALE


def features(eps_node, b, y0, x0, n):
    """Input features (3, n, n) of the n x n tile with corner (y0, x0) (global
    node indices): (Re eps - 1) / 4, Re b, Im b."""
    e = eps_node[y0:y0 + n, x0:x0 + n]
    s = b[y0:y0 + n, x0:x0 + n]
    return np.stack([(e.real - 1.0) * EPS_SCALE, s.real, s.imag])


def tile_weight(n, first, last):
    """1D blending weight of a tile: sin^2(pi (i + 1/2) / n), held at 1 on the
    outer half of a first or last tile."""
    i = np.arange(n)
    w = np.sin(np.pi * (i + 0.5) / n) ** 2
    if first:
        w[: n // 2] = 1.0
    if last:
        w[n // 2:] = 1.0
    return w


def blend(pred, origins_y, origins_x, ny, nx, pml, n):
    """Initial guess on the (ny, nx) grid from tile predictions pred[ty][tx]
    (2, n, n): weighted sum over tiles divided by the summed weights on the
    interior (tile origins are interior coordinates), zero in the global PML."""
    acc = np.zeros((ny, nx), dtype=np.complex128)
    wsum = np.zeros((ny, nx))
    for a, oy in enumerate(origins_y):
        wy = tile_weight(n, a == 0, a == len(origins_y) - 1)
        for c, ox in enumerate(origins_x):
            wx = tile_weight(n, c == 0, c == len(origins_x) - 1)
            w = np.outer(wy, wx)
            y = pred[a][c]
            sl = (slice(pml + oy, pml + oy + n), slice(pml + ox, pml + ox + n))
            acc[sl] += w * (y[0] + 1j * y[1])
            wsum[sl] += w
    out = np.zeros((ny, nx), dtype=np.complex128)
    m = wsum > 0
    out[m] = acc[m] / wsum[m]
    return out
