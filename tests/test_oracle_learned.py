"""Pins of the float64 learned-index oracle: gradients against central
differences, the least-squares segment fit against numpy.polyfit, the
interval-end error bound against random addresses, and positions against
the longest-prefix-match definition."""
import numpy as np

import oracle
import sinetgen
from oracle import learned


def _table(n=3000, seed=5):
    b, l = sinetgen.table_nested(seed, n, 8, 30, 0.3)
    return b, l


def test_mlp_gradient_vs_central_differences():
    rng = np.random.default_rng(3)
    B, _ = oracle.endpoints(*_table())
    x, y = learned.training_set(B)
    p = learned.mlp_init_hinges() + rng.normal(0, 0.3, learned.N_PARAMS)
    loss, g = learned.mlp_loss_grad(p, x, y)
    h = 1e-6
    w1, b1, _, _ = learned.split(p)
    for k in range(learned.N_PARAMS):
        e = np.zeros_like(p)
        e[k] = h
        # skip a coordinate whose step moves some sample across a ReLU kink
        zp = x[:, None] * (w1 + e[:16]) + (b1 + e[16:32])
        zm = x[:, None] * (w1 - e[:16]) + (b1 - e[16:32])
        if np.any(np.sign(zp) != np.sign(zm)):
            continue
        fd = (learned.mlp_loss_grad(p + e, x, y)[0] - learned.mlp_loss_grad(p - e, x, y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])
    assert np.isclose(loss, np.mean((learned.mlp_forward(p, x) - y) ** 2))


def test_mlp_closed_form_special_case():
    """With one active hinge (w1_0 = 1, b1_0 = 0, others off) the model is the
    line f = w2_0 x + b2, whose least-squares gradient has a closed form."""
    p = np.zeros(learned.N_PARAMS)
    p[0] = 1.0
    p[16:32] = -2.0          # all other hinges start at x = 2: never active
    p[16] = 0.0
    p[32] = 0.7
    p[48] = 0.1
    x = np.linspace(0.0, 1.0, 101)
    y = x ** 2
    _, g = learned.mlp_loss_grad(p, x, y)
    r = 0.7 * x + 0.1 - y
    assert np.isclose(g[32], 2 * np.mean(r * x))
    assert np.isclose(g[48], 2 * np.mean(r))
    assert np.isclose(g[0], 2 * np.mean(r * 0.7 * x))
    assert np.allclose(g[1:16], 0) and np.allclose(g[33:48], 0)


def test_adam_first_step_is_lr_times_sign():
    """Adam's bias-corrected first step moves every coordinate with a non-zero
    gradient by lr * g / (|g| + eps), i.e. by about lr against the gradient."""
    B, _ = oracle.endpoints(*_table(500))
    x, y = learned.training_set(B)
    p0 = learned.mlp_init_hinges()
    _, g = learned.mlp_loss_grad(p0, x, y)
    p1 = learned.adam_steps(p0, x, y, 1, lr=1e-3)
    nz = np.abs(g) > 1e-12
    assert np.allclose((p0 - p1)[nz], 1e-3 * np.sign(g[nz]), rtol=1e-6)
    p50 = learned.adam_steps(p0, x, y, 300, lr=1e-2)
    assert learned.mlp_loss_grad(p50, x, y)[0] < learned.mlp_loss_grad(p0, x, y)[0]


def test_pla_fit_vs_polyfit_and_bound():
    b, l = _table(4000, 9)
    B, own = oracle.endpoints(b, l)
    knot, k, c, g = learned.pla_fit(B, 256)
    assert knot[0] == 0 and np.all(np.diff(knot.astype(np.int64)) > 0)
    for s in range(0, len(knot), 17):
        u = B[k[s]:k[s + 1]].astype(np.float64) - float(knot[s])
        j = np.arange(k[s], k[s + 1], dtype=np.float64)
        if len(j) >= 2:
            sl, ic = np.polyfit(u, j, 1)
            assert np.isclose(sl, g[s], rtol=1e-7, atol=1e-15)
            assert np.isclose(ic, c[s], rtol=1e-9, atol=1e-6)
    assert np.all(g >= 0)  # increasing data: non-negative least-squares slope
    e = learned.max_error(lambda a: learned.pla_predict(knot, c, g, a), B)
    rng = np.random.default_rng(2)
    a = rng.integers(0, 1 << 32, 200_000, dtype=np.uint64).astype(np.uint32)
    err = np.abs(learned.pla_predict(knot, c, g, a) - learned.positions(B, a))
    assert err.max() <= e + 1e-9


def test_positions_give_lpm():
    b, l = _table(2000, 4)
    B, own = oracle.endpoints(b, l)
    rng = np.random.default_rng(8)
    a = rng.integers(0, 1 << 32, 50_000, dtype=np.uint64).astype(np.uint32)
    a[:len(B)] = B
    lab, si, _ = oracle.classify(b, l, a, a, mode="scan")
    pos = learned.positions(B, a)
    assert np.array_equal((own[pos] != 0), (lab & 1) == 1)
    assert np.array_equal(np.where(own[pos] == 0, np.uint32(0xFFFFFFFF), own[pos] - 1), si)
