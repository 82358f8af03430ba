"""Pins of the network oracle (oracle/net.py) against facts that do not come
from the oracle itself: a library cross-correlation, closed forms of the grid
transfers on sine modes and linear functions, adjoint identities, central
finite differences of the loss, the closed form of Adam's first step, and
exactness of the time interpolation on functions linear in t."""
import numpy as np
import pytest
import scipy.signal

from oracle import net as N


def rand_params(channels, rng, scale=0.4):
    return rng.standard_normal(N.param_count(channels)) * scale


def test_conv3x3_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 7, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = N.conv3x3(x, w, b)
    for bb in range(2):
        for o in range(4):
            ref = b[o] + sum(scipy.signal.correlate2d(x[bb, c], w[o, c], mode="same", boundary="fill")
                             for c in range(3))
            np.testing.assert_allclose(y[bb, o], ref, rtol=1e-12, atol=1e-12)


def test_conv_input_and_weight_grads_are_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 6))
    w = rng.standard_normal((4, 3, 3, 3))
    dy = rng.standard_normal((2, 4, 5, 6))
    zero = np.zeros(4)
    # <dy, conv(x)> = <conv_input_grad(dy), x> = <conv_weight_grad(dy, x), w>
    lhs = float((dy * N.conv3x3(x, w, zero)).sum())
    assert abs(lhs - float((N.conv3x3_input_grad(dy, w, 5, 6) * x).sum())) < 1e-10 * max(1, abs(lhs))
    dw, db = N.conv3x3_weight_grad(dy, x)
    assert abs(lhs - float((dw * w).sum())) < 1e-10 * max(1, abs(lhs))
    np.testing.assert_allclose(db, dy.sum(axis=(0, 2, 3)))


@pytest.mark.parametrize("k", [1, 3, 6])
def test_restriction_of_sine_mode_closed_form(k):
    # full weighting of sin(k pi x) on h-points gives cos^2(k pi h / 2) sin(k pi x) on 2h-points
    n = 31
    h = 1.0 / (n + 1)
    xf = h * np.arange(1, n + 1)
    xc = 2 * h * np.arange(1, (n - 1) // 2 + 1)
    f = np.sin(k * np.pi * xf)[None, None, None, :]
    r = N.restrict(f, two_d=False)[0, 0, 0]
    np.testing.assert_allclose(r, np.cos(k * np.pi * h / 2) ** 2 * np.sin(k * np.pi * xc), atol=1e-14)
    f2 = np.outer(np.sin(k * np.pi * xf), np.sin(2 * np.pi * xf))[None, None]
    r2 = N.restrict(f2, two_d=True)[0, 0]
    ref = (np.cos(k * np.pi * h / 2) ** 2 * np.cos(2 * np.pi * h / 2) ** 2 *
           np.outer(np.sin(k * np.pi * xc), np.sin(2 * np.pi * xc)))
    np.testing.assert_allclose(r2, ref, atol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_prolongation_of_sine_mode_closed_form(k):
    # sin(k pi x) sampled on the coarse grid: coincident fine points keep it, the
    # cubic midpoint value is sin(k pi x) (9 cos(theta/2) - cos(3 theta/2)) / 8,
    # theta = k pi H, at every midpoint (the odd reflections make the boundary ones exact too)
    nc = 15
    H = 1.0 / (nc + 1)
    xc = H * np.arange(1, nc + 1)
    xf = 0.5 * H * np.arange(1, 2 * nc + 2)
    theta = k * np.pi * H
    fac = (9 * np.cos(theta / 2) - np.cos(3 * theta / 2)) / 8
    p = N.prolong(np.sin(k * np.pi * xc)[None, None, None, :], two_d=False)[0, 0, 0]
    ref = np.sin(k * np.pi * xf) * np.where(np.arange(2 * nc + 1) % 2 == 1, 1.0, fac)
    np.testing.assert_allclose(p, ref, atol=1e-14)
    p2 = N.prolong(np.outer(np.sin(k * np.pi * xc), np.sin(np.pi * xc))[None, None], two_d=True)[0, 0]
    fac1 = (9 * np.cos(np.pi * H / 2) - np.cos(3 * np.pi * H / 2)) / 8
    ry = np.sin(k * np.pi * xf) * np.where(np.arange(2 * nc + 1) % 2 == 1, 1.0, fac)
    rx = np.sin(np.pi * xf) * np.where(np.arange(2 * nc + 1) % 2 == 1, 1.0, fac1)
    np.testing.assert_allclose(p2, np.outer(ry, rx), atol=1e-14)


def test_prolongation_exact_on_cubics_in_the_interior():
    nc = 9
    H = 1.0 / (nc + 1)
    xc = H * np.arange(1, nc + 1)
    xf = 0.5 * H * np.arange(1, 2 * nc + 2)
    cub = np.array([0.7, -1.3, 0.4, 2.0])
    p = N.prolong(np.polyval(cub, xc)[None, None, None, :], two_d=False)[0, 0, 0]
    inner = slice(3, 2 * nc - 2)    # fine points whose four coarse neighbours are all interior
    np.testing.assert_allclose(p[inner], np.polyval(cub, xf)[inner], atol=1e-13)


@pytest.mark.parametrize("two_d", [False, True])
def test_prolong_adjoint_identity(two_d):
    rng = np.random.default_rng(3)
    nc, nf = 7, 15
    shape_c = (2, 3, nc, nc) if two_d else (2, 3, 1, nc)
    shape_f = (2, 3, nf, nf) if two_d else (2, 3, 1, nf)
    c = rng.standard_normal(shape_c)
    f = rng.standard_normal(shape_f)
    lhs = float((N.prolong(c, two_d) * f).sum())
    rhs = float((c * N.prolong_adjoint(f, two_d)).sum())
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("two_d", [False, True])
def test_bands_telescope_to_signal(two_d):
    rng = np.random.default_rng(4)
    W = 31
    x = rng.standard_normal((2, 4, W if two_d else 1, W))
    inputs, sizes, td = N.level_inputs(x, nsig=3, h=1.0 / 32)
    assert sizes == [31, 15, 7, 3] and td == two_d
    acc = None
    for l in reversed(range(len(sizes))):
        band = inputs[l][:, :3]
        acc = band if acc is None else band + N.prolong(acc, two_d)
    np.testing.assert_allclose(acc, x[:, :3], atol=1e-13)
    # extra channel sampled at the level's points, level value log2(1/h_l)/10
    np.testing.assert_allclose(inputs[2][:, 3], x[:, 3][:, 3::4, 3::4] if two_d else x[:, 3][:, :, 3::4])
    np.testing.assert_allclose(inputs[1][:, 4], np.log2(16.0) / 10.0)


@pytest.mark.parametrize("two_d", [False, True])
def test_gradient_matches_central_differences(two_d):
    rng = np.random.default_rng(5)
    channels = [6, 5, 4, 3]     # 3 signal + 2 extra + level
    W = 7
    H = W if two_d else 1
    x = rng.standard_normal((2, 5, H, W))
    t = rng.standard_normal((2, 3, H, W))
    p = rand_params(channels, rng)
    h = 1.0 / 8
    _, g = N.gradient(p, channels, x, t, 3, h)
    idx = rng.choice(p.size, size=40, replace=False)
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (N.loss(N.forward(pp, channels, x, 3, h), t) - N.loss(N.forward(pm, channels, x, 3, h), t)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (i, fd, g[i])


def test_output_scaling_by_level():
    # one linear layer with only a centre tap 1 on the signal channel: out_l = band_l,
    # so y = sum_l P^l (4 h_l^2 band_l); with W = 3 there is one level: y = 4 h^2 x
    channels = [3, 1]
    p = np.zeros(N.param_count(channels))
    p[4] = 1.0              # w[0, 0, 1, 1]
    x = np.random.default_rng(6).standard_normal((1, 2, 1, 3))
    h = 0.25
    y = N.forward(p, channels, x, 1, h)
    np.testing.assert_allclose(y[:, 0], 4 * h * h * x[:, 0], atol=1e-15)


def test_adam_first_step_closed_form():
    # bias-corrected first step: p - lr * g / (|g| + eps)
    rng = np.random.default_rng(7)
    g = rng.standard_normal(50)
    p = rng.standard_normal(50)
    p1, m, v = N.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_round_ties_and_exact_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1.0 + 2 ** -7], dtype=np.float32)
    out = N.bf16_round(vals)
    np.testing.assert_array_equal(out, np.array([1.0, 1.0, 1.0 + 2 ** -6, -2.5, 1.0 + 2 ** -7], dtype=np.float32))


def test_time_interp_exact_on_linear_in_t_power_alpha():
    t = np.linspace(0, 1, 65) ** 3
    rows = [7, 15, 40, 63]
    alpha = 0.4
    q = np.array([0.5, -1.0])
    g = np.array([0.25, -0.5])
    slices = np.array([g + q * t[r + 1] ** alpha for r in rows])
    U = N.time_interp(slices, rows, t, g, alpha=alpha)
    np.testing.assert_allclose(U, g[None, :] + np.outer(t[1:] ** alpha, q), atol=1e-14)


def test_time_interp_exact_on_linear_in_t():
    t = np.linspace(0, 1, 33) ** 2
    rows = [3, 9, 20, 31]
    q = np.array([0.5, -1.0, 2.0])
    g = np.array([0.1, 0.2, 0.3])
    slices = np.array([g + q * t[r + 1] for r in rows])
    U = N.time_interp(slices, rows, t, g)
    np.testing.assert_allclose(U, g[None, :] + np.outer(t[1:], q), atol=1e-14)
    # constant after the last slice
    rows2 = [3, 9]
    U2 = N.time_interp(slices[:2], rows2, t, g)
    np.testing.assert_allclose(U2[10:], np.broadcast_to(slices[1], U2[10:].shape))


def test_finest_cutoff_drops_the_fine_bands():
    # with h_min = 2h the finest level is skipped: y equals the coarse-level
    # part only, i.e. the prolongation of the output computed on the grid below
    rng = np.random.default_rng(8)
    channels = [4, 3, 2]
    p = rng.standard_normal(N.param_count(channels)) * 0.3
    W, h = 15, 1.0 / 16
    x = rng.standard_normal((1, 3, 1, W))
    y = N.forward(p, channels, x, 2, h, h_min=2 * h)
    # the same network on the restricted input, one level down, then interpolated
    xc = np.concatenate([N.restrict(x[:, :2], False), x[:, 2:][:, :, :, 1::2]], axis=1)
    yc = N.forward(p, channels, xc, 2, 2 * h)
    np.testing.assert_allclose(y, N.prolong(yc, False), atol=1e-14)
    _, g = N.gradient(p, channels, x, rng.standard_normal((1, 2, 1, W)), 2, h, h_min=2 * h)
    assert np.all(np.isfinite(g))


def test_warm_start_input_hand_built_case():
    """A worked example written out by hand: the slice rows of b divided by
    ||b||_inf, then the constant channels alpha and r/10 (1D: an image of
    height 1; 2D: row-major [iy][ix] with q = iy n + ix)."""
    b = np.array([[1.0, 2.0, 3.0],
                  [-4.0, 5.0, 6.0],
                  [7.0, 8.0, -9.0],
                  [2.0, 0.0, 1.0]])
    x, scale = N.warm_start_input(b, [1, 3], 0.25, 7.0, 1, 3)
    assert scale == 9.0
    assert x.shape == (1, 4, 1, 3)
    assert np.array_equal(x[0, 0, 0], np.array([-4.0, 5.0, 6.0]) / 9.0)
    assert np.array_equal(x[0, 1, 0], np.array([2.0, 0.0, 1.0]) / 9.0)
    assert np.all(x[0, 2] == 0.25) and np.all(x[0, 3] == 0.7)
    # 2D, n = 3: the value at flat index q = 5 lands at (iy, ix) = (1, 2)
    b2 = np.zeros((2, 9))
    b2[1, 5] = -2.0
    b2[0, 0] = 1.0
    x2, s2 = N.warm_start_input(b2, [1], 0.5, 3.0, 2, 3)
    assert s2 == 2.0 and x2.shape == (1, 3, 3, 3)
    want = np.zeros((3, 3))
    want[1, 2] = -1.0
    assert np.array_equal(x2[0, 0], want)
    assert np.all(x2[0, 1] == 0.5) and np.all(x2[0, 2] == 0.3)


def test_bf16_activations_leave_bf16_inputs_unchanged():
    """With one layer on a single-level grid (W = 3, h = 1: the band is the
    signal, the level value log2(1/h)/10 is 0) and inputs that are bfloat16
    numbers, rounding the convolution input changes nothing."""
    rng = np.random.default_rng(4)
    ch = [4, 3]
    params = N.bf16_round(rng.standard_normal(N.param_count(ch)).astype(np.float32)).astype(np.float64)
    x = N.bf16_round(rng.standard_normal((2, 3, 1, 3)).astype(np.float32)).astype(np.float64)
    assert np.array_equal(N.forward(params, ch, x, 2, 1.0, act_bf16=True), N.forward(params, ch, x, 2, 1.0))


def test_bf16_activations_stay_within_one_rounding_of_each_input():
    """One layer, general inputs: the output moves by at most the bfloat16
    half-step (2^-9 relative) of every input, weighted by |w| (h = 1, W = 3)."""
    rng = np.random.default_rng(5)
    ch = [4, 3]
    params = rng.standard_normal(N.param_count(ch))
    x = rng.standard_normal((2, 3, 1, 3))
    d = N.forward(params, ch, x, 2, 1.0, act_bf16=True) - N.forward(params, ch, x, 2, 1.0)
    (w, b), = N.unpack(params, ch)
    xin = N.level_inputs(x, 2, 1.0)[0][0]
    bound = 4.0 * N.conv3x3(np.abs(xin), np.abs(w), np.zeros_like(b)) * 2.0 ** -8
    assert np.all(np.abs(d) <= bound + 1e-15) and np.abs(d).max() > 0
