"""Pins of the FP64 spectral-operator reference (oracle/nn.py).

* truncated forward DFT = numpy.fft.fft2 at the kept modes (library);
* inverse = numpy.fft.irfft2 of the zero-padded half spectrum (library);
* hand-derived gradients of every parameter block and of the input = central
  finite differences (brute force), so a dropped term, a wrong sign or a
  transposed operand in any block fails;
* GELU: odd-part identity gelu(x) - gelu(-x) = x and its derivative by
  finite differences; with one layer and no activation the network is affine;
* Adam: the first step moves every parameter by lr * sign(grad) (closed form);
* blending: constant tile predictions give that constant on the interior;
* BF16 rounding: values with 8 significant bits are fixed points, exact ties go to
  the even neighbour (hand-computed cases), every result is within 2^-8 relative,
  and the rounding equals torch's FP32 -> bfloat16 conversion (library).
"""
import numpy as np
import pytest

from oracle import nn
import workloads
from workloads import learned

TINY = nn.NNConfig(n=12, width=3, modes=3, layers=2, cin=3)


def _params(cfg, seed):
    return nn.unflatten(cfg, learned.init_params(cfg.width, cfg.modes, cfg.layers, cfg.cin, seed)
                        + 0.05 * np.random.default_rng(seed + 7).standard_normal(cfg.nparams()))


def test_layout_sizes_agree():
    cfg = nn.NNConfig()
    assert sum(k for k, _ in learned.param_blocks(16, 16, 4, 3)) == cfg.nparams()
    assert 1.0e6 < cfg.nparams() < 1.1e6        # about a million parameters


def test_ftrunc_matches_fft2():
    cfg = nn.NNConfig(n=16, width=2, modes=4, layers=1)
    h = np.random.default_rng(0).standard_normal((2, 16, 16))
    ref = np.fft.fft2(h)[:, nn.ky_index(cfg)][:, :, :cfg.modes]
    assert np.abs(nn.ftrunc(cfg, h) - ref).max() < 1e-11


def test_finv_matches_irfft2():
    cfg = nn.NNConfig(n=16, width=2, modes=4, layers=1)
    rng = np.random.default_rng(1)
    G = rng.standard_normal((2 * 4, 4)) + 1j * rng.standard_normal((2 * 4, 4))
    S = np.zeros((16, 9), dtype=complex)
    S[nn.ky_index(cfg), :4] = G
    ref = np.fft.irfft2(S, s=(16, 16))
    assert np.abs(nn.finv(cfg, G) - ref).max() < 1e-13


def test_gelu_identities():
    x = np.linspace(-4, 4, 41)
    assert np.allclose(nn.gelu(x) - nn.gelu(-x), x, atol=1e-14)
    e = 1e-6
    fd = (nn.gelu(x + e) - nn.gelu(x - e)) / (2 * e)
    assert np.abs(fd - nn.gelu_grad(x)).max() < 1e-8


def _loss(cfg, p, f, t):
    y, _ = nn.forward(cfg, p, f)
    return nn.loss_and_grad(y, t)[0]


@pytest.mark.parametrize("block", [name for name, _ in TINY.shapes()] + ["input"])
def test_gradients_match_finite_differences(block):
    cfg = TINY
    rng = np.random.default_rng(3)
    p = _params(cfg, 11)
    f = rng.standard_normal((2, cfg.cin, cfg.n, cfg.n))
    t = rng.standard_normal((2, 2, cfg.n, cfg.n))
    y, cache = nn.forward(cfg, p, f)
    _, dy = nn.loss_and_grad(y, t)
    g, df = nn.backward(cfg, p, cache, dy)
    base = f if block == "input" else p[block]
    grad = df if block == "input" else g[block]
    d = rng.standard_normal(base.shape)
    e = 1e-5

    def at(s):
        if block == "input":
            return _loss(cfg, p, f + s * d, t)
        q = dict(p)
        q[block] = p[block] + s * d
        return _loss(cfg, q, f, t)

    fd = (at(e) - at(-e)) / (2 * e)
    an = float(np.sum(grad * d))
    assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (fd, an)


def test_single_linear_layer_is_affine():
    cfg = nn.NNConfig(n=8, width=2, modes=2, layers=1, cin=3)
    p = _params(cfg, 5)
    rng = np.random.default_rng(2)
    f1, f2 = rng.standard_normal((2, 1, 3, 8, 8))
    z = np.zeros_like(f1)
    y = lambda f: nn.forward(cfg, p, f)[0]
    assert np.abs((y(f1 + f2) - y(z)) - (y(f1) - y(z)) - (y(f2) - y(z))).max() < 1e-12


def test_adam_first_step_is_sign_times_lr():
    g = np.array([3.0, -0.2, 1e-3, -50.0])
    p1, m, v = nn.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p1, -0.01 * np.sign(g), rtol=1e-4)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    p2, _, _ = nn.adam(p1, g, m, v, 2, 0.01)
    assert np.allclose(p2 - p1, -0.01 * np.sign(g), rtol=1e-4)


def test_blend_is_a_partition_of_unity():
    n, pml, interior = 8, 2, 20
    oy = learned.tile_origins(interior, n, n // 2)
    assert oy[-1] == interior - n
    pred = [[np.stack([np.full((n, n), 2.0), np.full((n, n), -1.0)]) for _ in oy] for _ in oy]
    x0 = nn.blend(pred, oy, oy, interior + 2 * pml, interior + 2 * pml, pml, n)
    inner = x0[pml:pml + interior, pml:pml + interior]
    assert np.abs(inner - (2.0 - 1.0j)).max() < 1e-14
    assert np.all(x0[:pml] == 0) and np.all(x0[:, -pml:] == 0)


def test_training_tile_shape():
    w = learned.tile_workload(50000, subcells=4)
    assert w.nx == w.ny == 296 and w.b.shape == (1, 296, 296)
    r = w.meta["source_row"]
    assert 4 <= r <= w.meta["substrate_rows"] - 4
    assert w.b[0, 20 + r].real.min() == 1.0 and np.count_nonzero(w.b) == 296
    # the sheet sits in the substrate (eps 2.13) and is reproducible from the seed
    assert abs(w.eps_cells[20 + r, 150].real - 2.13) < 1e-12
    w2 = learned.tile_workload(50000, subcells=4)
    assert np.array_equal(w.eps_cells, w2.eps_cells) and np.array_equal(w.b, w2.b)


def test_bf16_rounding():
    exact = np.array([0.0, 1.0, -2.5, 0.15625, 3.0 * 2.0 ** -20, 255.0, -1.0 / 128])
    assert np.array_equal(nn.quantize_bf16(exact), exact)
    one = 1.0
    # halfway between 1 and 1 + 2^-7: the even neighbour is 1
    assert nn.quantize_bf16([one + 2.0 ** -8])[0] == one
    # halfway between 1 + 2^-7 (odd last bit) and 1 + 2^-6: the even one is 1 + 2^-6
    assert nn.quantize_bf16([one + 3 * 2.0 ** -8])[0] == one + 2.0 ** -6
    # just above the half: rounds up; just below: down
    assert nn.quantize_bf16([one + 2.0 ** -8 + 2.0 ** -20])[0] == one + 2.0 ** -7
    assert nn.quantize_bf16([one + 2.0 ** -8 - 2.0 ** -20])[0] == one
    assert nn.quantize_bf16([-(one + 3 * 2.0 ** -8)])[0] == -(one + 2.0 ** -6)
    x = np.random.default_rng(3).standard_normal(20000) * np.exp(np.random.default_rng(4).uniform(-20, 20, 20000))
    q = nn.quantize_bf16(x)
    assert np.all(np.abs(q - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))   # unit roundoff, 8 bits
    torch = pytest.importorskip("torch")
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(q, ref)
