"""GPU checks of the learned troubled-cell indicator (not part of the paper's
method; parity against the oracle's FP64 MLP and features).

Tolerances: features are FP64 ratios stored in FP32 (1e-6 absolute on O(1)
values).  Logits come from the inference pass (FP32 matrix cores), compared
per sample with the oracle's FP64 network within twice the forward error
bound of binary32 evaluation (tests/helpers.mlp_fp32_bound).  Decisions are
compared where the FP64 logit is further than that bound from a threshold.
Gradients (FP32 training pass) 1e-4 relative L2 against FP64.
"""
import numpy as np
import pytest

import oracle as O
from paper_2307_06471_amd import workloads as W
from tests.helpers import mlp_fp32_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2307_06471_amd import crkdg
    return crkdg


@pytest.fixture(scope="module")
def ML(K):
    from paper_2307_06471_amd import mlp
    return mlp


def shock_state(K, n=96, k=2):
    import torch
    lm = K.make_mesh(2, n, n, bc=(1, 1, 1, 1), equation=K.EQ_EULER)
    om = O.Mesh(2, n, n, bc=(1, 1, 1, 1), equation=O.EQ_EULER, flux=O.FLUX_LLF)
    s = K.Solver(lm, k, K.FLUX_LLF, 3)
    p = W.quadrant_params(3, split=(0.507, 0.493))
    s.crkdg_project(K.IC_QUADRANT, p)
    s.crkdg_limit(50.0)
    for _ in range(5):
        s.crkdg_step(0.1 / s.crkdg_max_wavespeed())
    return s, om


def test_features_match_oracle(K):
    s, om = shock_state(K)
    u = s.crkdg_get_state()
    X = s.crkdg_mlp_features(50.0).cpu().numpy()
    Xo = O.mlp_features(om, 2, 50.0, u)
    assert np.abs(X - Xo).max() < 1e-6


def test_forward_grad_adam_match_oracle(K):
    import torch
    rng = np.random.default_rng(0)
    P = 0.4 * rng.standard_normal(O.N_MLP_PARAMS)
    X = rng.standard_normal((4096, 12))
    y = (rng.random(4096) < 0.2).astype(np.uint8)
    Pd = torch.from_numpy(P.astype(np.float32)).cuda()
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    yd = torch.from_numpy(y).cuda()
    # reference on the same FP32-rounded inputs
    P32, X32 = P.astype(np.float32).astype(float), X.astype(np.float32).astype(float)
    z = K.crkdg_mlp_forward(Pd, Xd).cpu().numpy()
    zo = O.mlp_forward(P32, X32)
    bound = mlp_fp32_bound(P32, X32)
    print(f"[mlp] forward: max |dz| {np.abs(z - zo).max():.3g}, max |dz|/bound "
          f"{(np.abs(z - zo) / bound).max():.3g}", flush=True)
    assert np.all(np.abs(z - zo) <= bound)
    assert np.abs(z - zo).max() > 0.0  # really evaluated in binary32
    g, loss = K.crkdg_mlp_grad(Pd, Xd, yd, 3.0)
    lo, go = O.mlp_loss_grad(P32, X32, y, 3.0)
    g = g.cpu().numpy()
    assert np.sqrt(((g - go) ** 2).sum() / (go ** 2).sum()) < 1e-4
    assert abs(loss.item() - lo) < 1e-5 * lo
    # one Adam step
    m1 = torch.zeros_like(Pd)
    m2 = torch.zeros_like(Pd)
    gd = torch.from_numpy(go.astype(np.float32)).cuda()
    K.crkdg_mlp_adam(Pd, m1, m2, gd, 1, lr=1e-3)
    Po, m1o, m2o = P32.copy(), np.zeros_like(P32), np.zeros_like(P32)
    O.adam(Po, m1o, m2o, go.astype(np.float32).astype(float), 1, lr=1e-3)
    assert np.abs(Pd.cpu().numpy() - Po).max() < 1e-6


def test_gradient_is_bitwise_reproducible(K):
    import torch
    rng = np.random.default_rng(1)
    Pd = torch.from_numpy((0.3 * rng.standard_normal(O.N_MLP_PARAMS)).astype(np.float32)).cuda()
    Xd = torch.from_numpy(rng.standard_normal((5000, 12)).astype(np.float32)).cuda()  # ragged
    yd = torch.from_numpy((rng.random(5000) < 0.3).astype(np.uint8)).cuda()
    g1, l1 = K.crkdg_mlp_grad(Pd, Xd, yd, 2.0)
    g2, l2 = K.crkdg_mlp_grad(Pd, Xd, yd, 2.0)
    assert torch.equal(g1, g2) and torch.equal(l1, l2)


def test_fallback_band_everywhere_equals_tvb(K):
    """with the band covering all probabilities every decision goes to the
    FP64 TVB test: the result is bit-identical to the TVB limiter"""
    import torch
    a, om = shock_state(K)
    b, _ = shock_state(K)
    P = torch.zeros(O.N_MLP_PARAMS, dtype=torch.float32, device="cuda")
    fa = torch.zeros(a.ncells, dtype=torch.uint8, device="cuda")
    fb = torch.zeros(a.ncells, dtype=torch.uint8, device="cuda")
    na = a.crkdg_limit(50.0, fa)
    nb, nfall = b.crkdg_limit_mlp(50.0, P, -1.0, 2.0, fb)
    assert na == nb and nfall == a.ncells
    assert torch.equal(fa | 8, fb)
    assert np.array_equal(a.crkdg_get_state(), b.crkdg_get_state())


def test_mlp_decisions_match_oracle(K):
    """band collapsed at 0.5: the MLP alone decides; compare with the oracle's
    FP64 network on the oracle's features wherever the logit is further from
    0 than the binary32 error bound"""
    import torch
    s, om = shock_state(K)
    u = s.crkdg_get_state()
    rng = np.random.default_rng(5)
    P = 0.5 * rng.standard_normal(O.N_MLP_PARAMS)
    P[-1] = 0.3
    Pd = torch.from_numpy(P.astype(np.float32)).cuda()
    flags = torch.zeros(s.ncells, dtype=torch.uint8, device="cuda")
    s.crkdg_limit_mlp(50.0, Pd, 0.5, 0.5, flags)
    Xo = O.mlp_features(om, 2, 50.0, u)
    P32 = P.astype(np.float32).astype(float)
    z = O.mlp_forward(P32, Xo)
    safe = np.abs(z) > mlp_fp32_bound(P32, Xo)
    fg = (flags.cpu().numpy() & 1) != 0
    print(f"[mlp] decisions compared on {safe.mean():.4f} of the cells", flush=True)
    assert safe.mean() > 0.99
    assert np.array_equal(fg[safe], (z >= 0.0)[safe])


@pytest.mark.slow
def test_training_reproducible_and_generalises(K, ML):
    """train on four-quadrant problems (seeds 0-5, 96^2), pick the band on
    seeds 64-65, check on unseen seeds 80-81: the band keeps the false
    negative rate against TVB small, and training is bitwise reproducible"""
    Xtr, ytr = ML.generate(range(6), n=96)
    Xva, yva = ML.generate([64, 65], n=96, sample_seed=1)
    Xte, yte = ML.generate([80, 81], n=96, sample_seed=2)
    assert ytr.sum() > 200
    P1, info = ML.train(Xtr, ytr, epochs=6, batch=2048, seed=0)
    P2, _ = ML.train(Xtr, ytr, epochs=6, batch=2048, seed=0)
    import torch
    assert torch.equal(P1, P2)
    lo, hi = ML.choose_band(P1, Xva, yva)
    rv = ML.rates(P1, Xva, yva, lo, hi)
    rt = ML.rates(P1, Xte, yte, lo, hi)
    assert rv["fn_rate"] <= 0.0101
    assert rt["fn_rate"] <= 0.05, rt
    assert rt["fallback_fraction"] < 0.6, rt
