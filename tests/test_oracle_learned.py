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


def _per_sample_fd_abs_sum(p, x, y, h=1e-6):
    """sum_i |d L_i / d theta_k| with L_i = (f(x_i) - y_i)^2 / n, each
    derivative by central differences of the per-sample loss."""
    n = x.shape[0]
    out = np.zeros(learned.N_PARAMS)
    for i in range(n):
        for k in range(learned.N_PARAMS):
            e = np.zeros_like(p)
            e[k] = h
            lp = (learned.mlp_forward(p + e, x[i:i + 1])[0] - y[i]) ** 2 / n
            lm = (learned.mlp_forward(p - e, x[i:i + 1])[0] - y[i]) ** 2 / n
            out[k] += abs((lp - lm) / (2 * h))
    return out


def test_grad_abs_sum_vs_per_sample_differences():
    """The tolerance scale of the GPU gradient check: the sum over samples of
    the magnitudes of each sample's gradient term, against central
    differences of every sample's own loss on a tiny set (residuals and
    hinge sides of both signs, so terms cancel in the plain gradient)."""
    rng = np.random.default_rng(11)
    x = np.array([0.03, 0.21, 0.37, 0.52, 0.68, 0.81, 0.95])
    p = learned.mlp_init_hinges() + rng.normal(0, 0.4, learned.N_PARAMS)
    # targets on alternate sides of the model: residuals of both signs
    y = learned.mlp_forward(p, x) + np.array([0.5, -0.4, 0.3, -0.6, 0.2, -0.5, 0.4])
    w1, b1, _, _ = learned.split(p)
    # keep every pre-activation away from the kink so the differences are smooth
    z = x[:, None] * w1[None, :] + b1[None, :]
    assert np.min(np.abs(z)) > 1e-5   # a step of 1e-6 moves z by at most 2e-6
    S = learned.mlp_grad_abs_sum(p, x, y)
    fd = _per_sample_fd_abs_sum(p, x, y)
    assert np.allclose(S, fd, rtol=1e-6, atol=1e-9), np.max(np.abs(S - fd))
    # terms of mixed sign: the magnitude sum exceeds |g| somewhere
    _, g = learned.mlp_loss_grad(p, x, y)
    assert np.all(S >= np.abs(g) - 1e-12) and np.any(S > np.abs(g) * 1.5 + 1e-9)


def test_grad_abs_sum_equals_gradient_without_cancellation():
    """When every residual, output weight, input and active pre-activation is
    positive, no per-sample term changes sign, so the magnitude sum equals
    the gradient itself (pinned by central differences above)."""
    x = np.linspace(0.05, 1.0, 40)
    y = np.zeros_like(x) - 1.0                  # f > 0 > y: residuals all positive
    p = np.zeros(learned.N_PARAMS)
    p[0:16] = np.linspace(0.5, 2.0, 16)         # w1 > 0
    p[16:32] = np.linspace(0.0, 0.3, 16)        # b1 >= 0: z > 0 for x > 0
    p[32:48] = np.linspace(0.1, 1.0, 16)        # w2 > 0
    p[48] = 0.2
    S = learned.mlp_grad_abs_sum(p, x, y)
    _, g = learned.mlp_loss_grad(p, x, y)
    assert np.all(g > 0)
    assert np.allclose(S, g, rtol=1e-12, atol=0)


def test_grad_abs_sum_is_a_mean():
    """Duplicating every sample leaves a per-sample mean unchanged."""
    rng = np.random.default_rng(4)
    x = rng.random(50)
    y = rng.random(50)
    p = learned.mlp_init_hinges() + rng.normal(0, 0.3, learned.N_PARAMS)
    S1 = learned.mlp_grad_abs_sum(p, x, y)
    S2 = learned.mlp_grad_abs_sum(p, np.concatenate([x, x]), np.concatenate([y, y]))
    assert np.allclose(S1, S2, rtol=1e-12)


def test_f32_positions_hand_cases():
    """Hand-worked float32 cases: a one-segment line y = x / 16 over
    boundaries 0, 16, 32, ...; ties round to even; clamping at both ends;
    a value above 2^24 that float32 cannot hold exactly."""
    knot = np.array([0], np.uint32)
    c = np.array([0.0], np.float32)
    g = np.array([1.0 / 16], np.float32)
    a = np.array([0, 15, 16, 24, 40, 47, 48, 1000], np.uint32)
    # 24/16 = 1.5 -> 2 (even), 40/16 = 2.5 -> 2 (even), 47/16 = 2.9375 -> 3
    exp = np.array([0, 1, 1, 2, 2, 3, 3, 9], np.int64)   # 1000/16 = 62.5 clamps to m - 1 = 9
    assert np.array_equal(learned.pla_position_f32(knot, c, g, a, 10), exp)
    # a negative intercept clamps to 0
    assert learned.pla_position_f32(knot, np.array([-5.0], np.float32), g, np.array([16], np.uint32), 10)[0] == 0
    # 2^24 + 1 rounds to 2^24 in float32 before the multiply
    big = np.array([(1 << 24) + 1], np.uint32)
    assert learned.pla_position_f32(knot, c, np.array([1.0], np.float32), big, 1 << 30)[0] == 1 << 24
    # an MLP with one active hinge of slope 2 and b2 = 0.25: f(x) = 2x + 0.25
    p = np.zeros(learned.N_PARAMS, np.float32)
    p[0] = 1.0
    p[16:32] = -2.0
    p[16] = 0.0
    p[32] = 2.0
    p[48] = 0.25
    a = np.array([0, 1 << 29, 1 << 30, 3 << 29], np.uint32)     # x = 0, 1/8, 1/4, 3/8
    # m = 8: f * 8 = 2, 4, 6, 8 -> the last clamps to 7
    assert np.array_equal(learned.mlp_position_f32(p, a, 8), [2, 4, 6, 7])


def test_f32_positions_track_float64():
    """The float32 positions differ from the rounded float64 prediction only
    where float32 rounding can move it across a half-integer."""
    b, l = _table(3000, 6)
    B, _ = oracle.endpoints(b, l)
    m = len(B)
    knot, k, c, g = learned.pla_fit(B, 64)
    rng = np.random.default_rng(5)
    a = rng.integers(0, 1 << 32, 100_000, dtype=np.uint64).astype(np.uint32)
    p64 = learned.pla_predict(knot, c, g, a)
    p32 = learned.pla_position_f32(knot, c.astype(np.float32), g.astype(np.float32), a, m)
    r64 = np.rint(np.clip(p64, 0, m - 1))
    # float32 carries 24 bits: relative error of a few ulp on values below m
    assert np.max(np.abs(p32 - r64)) <= 1
    # and they agree wherever the float64 prediction is not within float32
    # rounding (a few ulp of m) of a half-integer
    frac = np.abs(np.clip(p64, 0, m - 1) % 1.0 - 0.5)
    far = frac > 16 * m * 2.0 ** -24
    assert np.array_equal(p32[far], r64[far].astype(np.int64))
    w = learned.mlp_init_hinges() + rng.normal(0, 0.1, learned.N_PARAMS)
    q64 = np.clip(learned.mlp_forward(w, a.astype(np.float64) / 2.0 ** 32) * m, 0, m - 1)
    q32 = learned.mlp_position_f32(w.astype(np.float32), a, m)
    assert np.max(np.abs(q32 - np.rint(q64))) <= 1


def test_rounded_bound_covers_every_address():
    """For PLA segments with non-negative slopes the rounded prediction is
    monotone inside each interval, so the bound measured at interval ends
    covers random addresses (against the sorted-search position)."""
    b, l = _table(4000, 12)
    B, _ = oracle.endpoints(b, l)
    m = len(B)
    knot, k, c, g = learned.pla_fit(B, 128)
    c32, g32 = c.astype(np.float32), g.astype(np.float32)
    e = learned.max_error_rounded(lambda a: learned.pla_position_f32(knot, c32, g32, a, m), B)
    rng = np.random.default_rng(9)
    a = rng.integers(0, 1 << 32, 300_000, dtype=np.uint64).astype(np.uint32)
    err = np.abs(learned.pla_position_f32(knot, c32, g32, a, m) - learned.positions(B, a))
    assert err.max() <= e
    # and the bound is attained at some interval end
    ends = np.concatenate([B, B[1:] - 1])
    jj = np.concatenate([np.arange(m), np.arange(m - 1)])
    assert np.max(np.abs(learned.pla_position_f32(knot, c32, g32, ends, m) - jj)) == e
