"""GPU parity of the learned warm start against the FP64 reference (oracle/nn.py).

The network runs in FP32 on the GPU; the bars below are FP32-level:
forward outputs 1e-4 relative (max-norm over the batch), gradients 2e-3
relative per parameter block (norm-wise; they sum ~1e5 FP32 products), the
Adam kernel 1e-6 against the FP64 update of the same gradient, the blended
initial guess 1e-4.  The trained network's guess has no reference (parity
unpinned): the solve tests check only what holds for any guess, namely that
the learned solve converges to the same field and that the fallback rule
picks the zero guess when the network's residual is not below |b|.
"""
import numpy as np
import pytest

import workloads
from oracle import fdfd, nn
from workloads import learned

pytestmark = pytest.mark.gpu

CFG = nn.NNConfig(n=32, width=8, modes=4, layers=3, cin=3)
# the deployed architecture (256^2 tiles, 16 channels, 16 modes, 4 layers),
# whose transforms run the kernels compiled for that shape
DEPLOY = nn.NNConfig(n=256, width=16, modes=16, layers=4, cin=3)


@pytest.fixture(scope="module")
def stf():
    import paper_2509_20801_amd as stf
    return stf


@pytest.fixture(scope="module")
def ctx(stf):
    return stf.Context(0)


def _flat(cfg, seed, noise=0.05):
    p = learned.init_params(cfg.width, cfg.modes, cfg.layers, cfg.cin, seed)
    p = p + noise * np.random.default_rng(seed + 3).standard_normal(p.size)
    return p.astype(np.float32).astype(np.float64)     # the values the GPU holds


def _net(stf, ctx, cfg, flat, max_batch=8):
    return stf.Network(ctx, flat, n=cfg.n, width=cfg.width, modes=cfg.modes, layers=cfg.layers,
                       cin=cfg.cin, max_batch=max_batch)


def _inputs(cfg, B, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((B, cfg.cin, cfg.n, cfg.n)).astype(np.float32)
    t = rng.standard_normal((B, 2, cfg.n, cfg.n)).astype(np.float32)
    return f, t


def test_param_count_matches_reference(stf):
    for c in [CFG, nn.NNConfig(), nn.NNConfig(n=64, width=4, modes=8, layers=2)]:
        assert stf.nn_param_count(c.n, c.width, c.modes, c.layers, c.cin) == c.nparams()


@pytest.mark.parametrize("cfg,batch", [(CFG, 3), (DEPLOY, 2)], ids=["small", "deployed"])
def test_forward_matches_reference(stf, ctx, cfg, batch):
    import torch
    flat = _flat(cfg, 1)
    net = _net(stf, ctx, cfg, flat)
    f, _ = _inputs(cfg, batch, 2)
    y = net.forward(torch.from_numpy(f).cuda()).cpu().numpy()
    yr, _ = nn.forward(cfg, nn.unflatten(cfg, nn.quantize_bf16(flat)), f.astype(np.float64))
    assert np.abs(y - yr).max() <= 1e-4 * np.abs(yr).max()
    net.close()


@pytest.mark.parametrize("cfg,batch", [(CFG, 3), (DEPLOY, 1)], ids=["small", "deployed"])
def test_gradient_matches_reference(stf, ctx, cfg, batch):
    import torch
    flat = _flat(cfg, 4)
    net = _net(stf, ctx, cfg, flat)
    f, t = _inputs(cfg, batch, 5)
    loss, g = net.loss_grad(torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda())
    p = nn.unflatten(cfg, nn.quantize_bf16(flat))          # gradients at the BF16 weights
    y, cache = nn.forward(cfg, p, f.astype(np.float64))
    lr_, dy = nn.loss_and_grad(y, t.astype(np.float64))
    gr, _ = nn.backward(cfg, p, cache, dy)
    assert abs(loss - lr_) <= 1e-5 * lr_
    gg = nn.unflatten(cfg, g.astype(np.float64))
    for name, _ in cfg.shapes():
        num = np.linalg.norm(gg[name] - gr[name])
        assert num <= 2e-3 * np.linalg.norm(gr[name]) + 1e-7, (name, num, np.linalg.norm(gr[name]))
    net.close()


def test_adam_step_matches_reference(stf, ctx):
    import torch
    flat = _flat(CFG, 6)
    net = _net(stf, ctx, CFG, flat)
    f, t = _inputs(CFG, 2, 7)
    fd, td = torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda()
    _, g = net.loss_grad(fd, td)
    net.set_params(flat)                     # resets the moments
    net.train_step(fd, td, 1e-3, 1)
    p1 = net.get_params().astype(np.float64)
    z = np.zeros_like(flat)
    ref, _, _ = nn.adam(flat, g.astype(np.float64), z, z, 1, 1e-3)
    assert np.abs(p1 - ref).max() <= 1e-6
    net.close()


def test_weights_are_rounded_to_bf16(stf, ctx):
    """The network computes with its parameters rounded to BF16 exactly as the
    oracle rounds them: the same outputs, bit for bit, from the FP32 parameters
    and from their BF16 rounding, at creation, after set_params and after an
    Adam step (whose rounding is fused into the update); get_params returns the
    FP32 master copy."""
    import torch
    flat = _flat(CFG, 11)
    q = nn.quantize_bf16(flat)
    assert np.count_nonzero(q != flat) > 0.9 * flat.size
    f, t = _inputs(CFG, 2, 12)
    fd, td = torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda()
    a, b = _net(stf, ctx, CFG, flat), _net(stf, ctx, CFG, q)
    assert torch.equal(a.forward(fd), b.forward(fd))
    assert np.array_equal(a.get_params().astype(np.float64), flat)
    b.set_params(flat)
    assert torch.equal(a.forward(fd), b.forward(fd))
    a.train_step(fd, td, 1e-3, 1)
    p1 = a.get_params().astype(np.float64)
    b.set_params(nn.quantize_bf16(p1))
    assert torch.equal(a.forward(fd), b.forward(fd))
    a.close()
    b.close()


def test_training_reduces_the_loss(stf, ctx):
    import torch
    flat = _flat(CFG, 8, noise=0.0)
    net = _net(stf, ctx, CFG, flat)
    f, t = _inputs(CFG, 4, 9)
    fd, td = torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda()
    first = net.train_step(fd, td, 3e-3, 1)
    for s in range(2, 60):
        last = net.train_step(fd, td, 3e-3, s)
    assert np.isfinite(last) and last < 0.8 * first
    net.close()


def _small_problem(nx=80, pml=8, seed=0):
    w = workloads.configs.small_random(nx=nx, ny=nx, pml=pml, lam=12.0, px=2, py=2, overlap=4,
                                       local_pml=6, seed=seed)
    return w


def _prm(w):
    p = w.params()
    return dict(nx=p["nx"], ny=p["ny"], k0=p["k0"], pml=p["pml"], pml_order=p["pml_order"],
                pml_R=p["pml_R"], px=p["px"], py=p["py"], overlap=p["overlap"],
                local_pml=p["local_pml"], local_pml_order=p["local_pml_order"],
                local_pml_R=p["local_pml_R"])


def test_initial_guess_and_tile_data_match_reference(stf, ctx):
    import torch
    flat = _flat(CFG, 10)
    net = _net(stf, ctx, CFG, flat, max_batch=3)          # several batches of tiles
    w = _small_problem()
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    b = w.b[0]
    x0 = pb.initial_guess(net, b)
    pml, n, interior = 8, CFG.n, w.nx - 16
    org = learned.tile_origins(interior, n, n // 2)
    eps_node = fdfd.node_eps(w.eps_cells)
    p = nn.unflatten(CFG, nn.quantize_bf16(flat))
    feats = np.stack([nn.features(eps_node, b, pml + oy, pml + ox, n) for oy in org for ox in org])
    y, _ = nn.forward(CFG, p, feats)
    pred = [[y[a * len(org) + c] for c in range(len(org))] for a in range(len(org))]
    ref = nn.blend(pred, org, org, w.ny, w.nx, pml, n)
    assert np.abs(x0 - ref).max() <= 1e-4 * np.abs(ref).max()
    # the same tiles as training data
    bd = torch.from_numpy(b).cuda()
    f, t = pb.tile_data(net, bd, bd)
    assert f.shape == (len(org) ** 2, 3, n, n)
    assert np.abs(f.cpu().numpy() - feats).max() <= 1e-6 * max(1.0, np.abs(feats).max())
    tt = t.cpu().numpy()
    assert np.abs(tt[1, 0] - b[pml:pml + n, pml + org[1]:pml + org[1] + n].real).max() < 1e-6
    pb.close()
    net.close()


def test_learned_solve_converges_and_falls_back(stf, ctx):
    flat = _flat(CFG, 12, noise=0.0)
    net = _net(stf, ctx, CFG, flat)
    ctx.set_nn(net)
    w = _small_problem(seed=1)
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    pb.factor()
    b = w.b[0]
    x_ref, inf_ref = pb.solve(b, tol=1e-10)
    x_l, inf_l = pb.solve(b, tol=1e-10, x0="learned")
    assert inf_l[0]["status"] == 0 and inf_l[0]["relres_true"] <= 1e-10
    assert np.linalg.norm(x_l - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    # the flag agrees with the rule
    assert inf_l[0]["used_learned"] == int(inf_l[0]["relres_x0"] < 1.0)
    # a network whose guess is far off is rejected: the run equals the zero-guess run
    bad = flat.copy()
    bad[-2:] = 1e4                                   # output biases
    net.set_params(bad)
    x_f, inf_f = pb.solve(b, tol=1e-10, x0="learned")
    assert inf_f[0]["used_learned"] == 0 and inf_f[0]["relres_x0"] > 1.0
    assert inf_f[0]["iters"] == inf_ref[0]["iters"]
    assert np.array_equal(x_f, x_ref)
    ctx.set_nn(None)
    pb.close()
    net.close()


def test_factor_solve_runs_the_guess_beside_the_factorisation(stf, ctx):
    """stf_factor_solve (the network on a second stream during the
    factorisation, device arrays) gives the same fields, bit for bit, and the
    same iterations and guess residuals as stf_factor followed by stf_solve, for
    two right-hand sides; with host arrays (no overlap) as well."""
    import torch
    flat = _flat(CFG, 12, noise=0.0)
    net = _net(stf, ctx, CFG, flat)
    ctx.set_nn(net)
    w = _small_problem(seed=1)
    b2 = np.stack([w.b[0], 0.5j * w.b[0] + 0.1])
    pb = stf.Problem(ctx, _prm(w), w.eps_cells)
    try:
        for dev in (True, False):
            b = torch.from_numpy(b2).cuda() if dev else b2
            pb.assemble(w.eps_cells)
            pb.factor()
            x1, inf1 = pb.solve(b, tol=1e-10, x0="learned")
            pb.assemble(w.eps_cells)
            x2, inf2 = pb.factor_solve(b, tol=1e-10, x0="learned")
            if dev:
                x1, x2 = x1.cpu().numpy(), x2.cpu().numpy()
            assert np.array_equal(x1, x2)
            for a, c in zip(inf1, inf2):
                assert a["status"] == 0 and c["status"] == 0
                assert (a["iters"], a["used_learned"], a["relres_x0"]) == \
                    (c["iters"], c["used_learned"], c["relres_x0"])
                assert c["t_factor_ms"] > 0.0 and c["t_nn_ms"] > 0.0
        # solve before factor is still refused; factor_solve factors itself
        pb.assemble(w.eps_cells)
        with pytest.raises(stf.StfError):
            pb.solve(b2, tol=1e-10)
        x3, inf3 = pb.factor_solve(b2, tol=1e-10)
        assert inf3[0]["status"] == 0 and inf3[0]["relres_true"] <= 1e-10
    finally:
        ctx.set_nn(None)
        pb.close()
        net.close()


@pytest.mark.parametrize("nr", [2, 5])
def test_batched_learned_guess_matches_the_solo_guess(stf, ctx, nr):
    """stf_batch_solve with the learned guess: the guesses (computed on the
    side stream during the factorisation when every problem has at most four
    right-hand sides, after it otherwise) have the residuals of the solo
    solve's guesses, the fallback takes the same decisions, and the fields
    converge to the solo fields (1e-8 relative at rel-res 1e-10)."""
    import torch
    flat = _flat(CFG, 12, noise=0.0)
    net = _net(stf, ctx, CFG, flat)
    ctx.set_nn(net)
    ws = [_small_problem(seed=1), _small_problem(nx=72, seed=2)]
    bs = [np.stack([(1.0 + 0.3j * r) * w.b[0] + 0.05 * r for r in range(nr if k == 0 else 2)])
          for k, w in enumerate(ws)]
    pbs = [stf.Problem(ctx, _prm(w), w.eps_cells) for w in ws]
    try:
        xs, infos = stf.batch_solve(ctx, pbs, [torch.from_numpy(b).cuda() for b in bs], tol=1e-10,
                                    restart=12, max_iter=400, x0="learned")
        for p, (pb, b) in enumerate(zip(pbs, bs)):
            pb.factor()
            xsolo, isolo = pb.solve(b, tol=1e-10, restart=12, max_iter=400, x0="learned")
            for r in range(b.shape[0]):
                got, ref = infos[p][r], isolo[r]
                assert got["status"] == 0 and got["relres_true"] <= 1e-10
                assert got["used_learned"] == ref["used_learned"]
                assert abs(got["relres_x0"] - ref["relres_x0"]) <= 1e-12 * max(1.0, ref["relres_x0"])
                assert got["t_nn_ms"] > 0.0
                x = xs[p][r].cpu().numpy()
                assert np.linalg.norm(x - xsolo[r]) <= 1e-8 * np.linalg.norm(xsolo[r])
    finally:
        ctx.set_nn(None)
        for pb in pbs:
            pb.close()
        net.close()


@pytest.mark.parametrize("interior,parts,seed", [(1024, 8, 5001), (2048, 16, 5002)],
                         ids=["1024", "2048"])
def test_trained_network_gain_on_the_deploy_grids(stf, ctx, interior, parts, seed):
    """What the committed trained network gains on the deploy metasurfaces
    (1024^2 at 8 x 8 subdomains, seed 5001; 2048^2 at 16 x 16, seed 5002; not
    training tiles): both solves converge to the same field; when the fallback
    rejects the guess the run is the zero-guess run."""
    import json
    from paper_2509_20801_amd import learned as L
    net = L.load_network(stf, ctx, max_batch=64)
    if net is None:
        pytest.skip("no trained weights in the package")
    w = workloads.configs.metasurface_sheet(interior=interior, parts=parts, seed=seed)
    out = L.evaluate(stf, ctx, net, w, log=lambda s: print(s))
    z, l = out["zero"], out["learned"]
    assert z["relres_true"] <= 1e-8 and l["relres_true"] <= 1e-8
    assert l["used_learned"] == int(l["relres_x0"] < 1.0)
    if not l["used_learned"]:
        assert l["iters"] == z["iters"]
    print(json.dumps({"iters_zero": z["iters"], "iters_learned": l["iters"],
                      "relres_guess": l["relres_x0"], "used": l["used_learned"]}))
    net.close()
