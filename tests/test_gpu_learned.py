"""The GPU trainer of the learned position model against the float64 oracle
(oracle/learned.py): the Adam trajectory of the 1-16-1 MLP, the least-squares
PLA fit, and the measured search bound of both models, through the C ABI.

Tolerances (float32 GPU against float64 oracle):
- Adam: along the oracle's trajectory every nonzero gradient component has
  S_k / |g_k| <= 2 (S_k: the sum of the absolute per-sample terms,
  ``learned.mlp_grad_abs_sum``), so the float32 gradient is accurate to a few
  1e-6 relative and each step's update (at most lr per component) to about
  1e-5 lr; after K steps the parameters agree within K * lr * 1e-4 plus 4
  float32 ulps of the parameter.  A missing bias correction or a wrong beta
  moves a parameter by about lr (1e-2) in the first steps.
- PLA fit: the GPU sums in float64 in another order and rounds to float32, so
  c and g equal the float32 rounding of the oracle's values within one ulp;
  knots are integers and equal.
- Measured bounds: integers taken in the float32 inference arithmetic on both
  sides, so they are equal.
"""
import sys

import numpy as np
import pytest

import oracle
import sinetgen
from oracle import learned

pytestmark = pytest.mark.gpu

LR = 1e-2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sinet():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2106_12863_amd as s
    return s


def _xy32(B):
    """The float32 training set the GPU builds: x = float32(B) * 2^-32,
    y = float32(j / m), as float64 values."""
    x32 = B.astype(np.float32) * np.float32(2.0 ** -32)
    y32 = (np.arange(B.shape[0]) / B.shape[0]).astype(np.float32)
    return x32.astype(np.float64), y32.astype(np.float64)


def _ulp32(v):
    v = np.abs(np.asarray(v, np.float32))
    return np.spacing(np.maximum(v, np.float32(1e-30))).astype(np.float64)


def _mlp_bound(p, B):
    m = B.shape[0]
    return learned.max_error_rounded(lambda a: learned.mlp_position_f32(p, a, m), B)


def _pla_bound(model, B):
    knot, c, g = model
    m = B.shape[0]
    return learned.max_error_rounded(lambda a: learned.pla_position_f32(knot, c, g, a, m), B)


@pytest.mark.parametrize("init", ["hinges", "perturbed"])
def test_adam_trajectory_vs_oracle(sinet, init):
    """GPU Adam after K = 1, 2, 4, 8 full-batch steps equals the oracle's
    float64 Adam from the same float32 start on the same float32 training set;
    the reported first and last losses and both measured bounds agree."""
    wl = sinetgen.config(4, n=10)
    B, _ = oracle.endpoints(wl.pbase, wl.plen)
    x, y = _xy32(B)
    p0 = learned.mlp_init_hinges()
    if init == "perturbed":
        p0 = p0 + np.random.default_rng(7).normal(0.0, 0.05, learned.N_PARAMS)
    p0 = p0.astype(np.float32)
    tab = sinet.Table(wl.pbase, wl.plen, kind="mlp", inout_index=False)
    loss0, _ = learned.mlp_loss_grad(p0.astype(np.float64), x, y)
    # the tolerance's premise: no gradient component of the first 8 steps cancels
    for t in range(8):
        p_t = learned.adam_steps(p0.astype(np.float64), x, y, t, LR)
        _, g = learned.mlp_loss_grad(p_t, x, y)
        S = learned.mlp_grad_abs_sum(p_t, x, y)
        nz = g != 0.0
        assert np.all(S[nz] <= 2.0 * np.abs(g[nz])), (init, t)
    for K in (1, 2, 4, 8):
        _say("adam", init, K)
        rep = tab.train(steps=K, lr=LR, init=p0)
        kind, p_gpu, err = tab.get_model()
        assert kind == "mlp"
        p_ref = learned.adam_steps(p0.astype(np.float64), x, y, K, LR)
        tol = K * LR * 1e-4 + 4.0 * _ulp32(p_ref)
        diff = np.abs(p_gpu.astype(np.float64) - p_ref)
        assert np.all(diff <= tol), (init, K, int(np.argmax(diff / tol)), float(np.max(diff / tol)))
        # losses: float32 per-sample terms summed through float64
        assert abs(rep.loss_first - loss0) <= 1e-5 * loss0
        lossK, _ = learned.mlp_loss_grad(p_gpu.astype(np.float64), x, y)
        assert abs(rep.loss_last - lossK) <= 1e-5 * lossK
        # measured bounds with the inference arithmetic
        assert rep.max_err_untrained == _mlp_bound(p0, B)
        assert rep.max_err == err == tab.info().max_err == _mlp_bound(p_gpu, B)
    # eight steps move the model: the trained loss is below the start
    assert rep.loss_last < rep.loss_first


@pytest.mark.parametrize("cfg,segs", [(1, (1, 3, "m")), (2, (1, 7, 256, 1000)), (4, (256, 4096))])
def test_pla_fit_vs_oracle(sinet, cfg, segs):
    """k_pla_fit's equal-count knots equal the oracle's, its lines equal the
    oracle's least-squares lines rounded to float32 (within one ulp), and the
    GPU-measured bound equals the oracle's rounded-position bound of the same
    float32 model.  S = m gives one boundary per segment (flat lines)."""
    wl = sinetgen.config(cfg, n=10)
    B, _ = oracle.endpoints(wl.pbase, wl.plen)
    m = B.shape[0]
    tab = sinet.Table(wl.pbase, wl.plen, kind="pla", inout_index=False)
    for S in segs:
        S = m if S == "m" else S
        _say("pla fit cfg", cfg, "S", S)
        rep = tab.train(segments=S)
        kind, (knot, c, g), err = tab.get_model()
        assert kind == "pla" and knot.shape[0] == min(S, m)
        eknot, _, ec, eg = learned.pla_fit(B, S)
        assert np.array_equal(knot, eknot)
        ec32, eg32 = ec.astype(np.float32), eg.astype(np.float32)
        # c = mean j - g * mean u: float64 order effects reach about 1e-15 of mean j
        assert np.all(np.abs(c.astype(np.float64) - ec32) <= _ulp32(ec32) + 1e-9), S
        assert np.all(np.abs(g.astype(np.float64) - eg32) <= _ulp32(eg32)), S
        assert np.all(g >= 0)
        assert rep.max_err == err == tab.info().max_err == _pla_bound((knot, c, g), B)


@pytest.mark.parametrize("target", [0, 2, 16])
def test_error_bounded_pla_bound_vs_oracle(sinet, target):
    """The host's error-bounded segmentation of the 200,000-prefix table: the
    bound the GPU measures equals the oracle's rounded-position bound of the
    uploaded float32 model.  Target 0 aims at the window search (a bound of at
    most 6); a cone of +-16 boundaries fits in LDS, and the float32 line and
    its rounding add at most one; a target too fine for LDS is doubled, so
    target 2 is checked only against the oracle."""
    wl = sinetgen.config(4, n=10)
    B, _ = oracle.endpoints(wl.pbase, wl.plen)
    tab = sinet.Table(wl.pbase, wl.plen, kind="pla", inout_index=False)
    rep = tab.train(target_err=target)
    _, model, err = tab.get_model()
    assert rep.max_err == err == _pla_bound(model, B)
    assert np.all(model[2] >= 0) and model[0][0] == 0
    if target == 0:
        assert err <= 6 and tab.info().pla_window == 1
    if target == 16:
        assert err <= 17


def test_measured_bound_of_loaded_models_vs_oracle(sinet):
    """Models loaded from the host with the bound left to the GPU: the
    measured bound equals the oracle's, for random MLP weights and for an
    equal-count PLA whose lines are perturbed."""
    wl = sinetgen.config(4, n=10)
    B, _ = oracle.endpoints(wl.pbase, wl.plen)
    rng = np.random.default_rng(11)
    mlp = sinet.Table(wl.pbase, wl.plen, kind="mlp", inout_index=False)
    for trial in range(3):
        p = (learned.mlp_init_hinges() + rng.normal(0.0, 0.3, learned.N_PARAMS)).astype(np.float32)
        mlp.set_model(params=p)
        assert mlp.info().max_err == _mlp_bound(p, B), trial
    pla = sinet.Table(wl.pbase, wl.plen, kind="pla", inout_index=False)
    knot, _, c, g = learned.pla_fit(B, 512)
    c = (c + rng.normal(0.0, 3.0, c.shape)).astype(np.float32)
    g = (g * rng.uniform(0.9, 1.1, g.shape)).astype(np.float32)
    pla.set_model(pla=(knot, c, g))
    assert pla.info().max_err == _pla_bound((knot, c, g), B)
