"""Plant plausible mistakes in the network oracle (on the CPU) and check that
one of its pins fails."""
import numpy as np
import pytest

import test_oracle_net as T
from oracle import net as N


def _conv_flipped(x, w, b):
    # convolution instead of cross-correlation (kernel flipped)
    return _orig_conv(x, w[:, :, ::-1, ::-1], b)


def _input_grad_unflipped(dy, w, H, W):
    # gradient through the conv that sends taps the wrong way
    B = dy.shape[0]
    dyp = np.zeros((B, dy.shape[1], H + 2, W + 2))
    dyp[:, :, 1:-1, 1:-1] = dy
    out = np.zeros((B, w.shape[1], H, W))
    for di in range(3):
        for dj in range(3):
            out += np.einsum("oc,bohw->bchw", w[:, :, di, dj], dyp[:, :, di:di + H, dj:dj + W])
    return out


def _adjoint_no_reflection(g, two_d):
    # the columns of P without the odd-reflection terms at the boundary
    def adj(a, axis):
        a = np.moveaxis(a, axis, -1)
        nf = a.shape[-1]
        nc = (nf - 1) // 2
        r = np.zeros(a.shape[:-1] + (nc,))
        for i in range(nc):
            for f, w in [(2 * i - 2, -1 / 16), (2 * i, 9 / 16), (2 * i + 1, 1.0), (2 * i + 2, 9 / 16),
                         (2 * i + 4, -1 / 16)]:
                if 0 <= f < nf:
                    r[..., i] += w * a[..., f]
        return np.moveaxis(r, -1, axis)
    r = adj(g, g.ndim - 1)
    return adj(r, g.ndim - 2) if two_d else r


def _prolong_linear(a, two_d):
    def p1(a, axis):
        a = np.moveaxis(a, axis, -1)
        nc = a.shape[-1]
        padded = np.concatenate([np.zeros(a.shape[:-1] + (1,)), a, np.zeros(a.shape[:-1] + (1,))], axis=-1)
        out = np.zeros(a.shape[:-1] + (2 * nc + 1,))
        out[..., 1::2] = a
        out[..., 0::2] = 0.5 * (padded[..., :-1] + padded[..., 1:])
        return np.moveaxis(out, -1, axis)
    p = p1(a, a.ndim - 1)
    return p1(p, a.ndim - 2) if two_d else p


def _restrict_injection(a, two_d):
    r = a[..., 1:-1:2]
    return r[..., 1:-1:2, :] if two_d else r


def _gradient_no_tanh_derivative(params, channels, x, t, nsig, h):
    layers = N.unpack(params, channels)
    y, (acts, sizes, two_d) = N.forward(params, channels, x, nsig, h, cache=True)
    B = y.shape[0]
    den = (t ** 2).sum(axis=(1, 2, 3))
    gy = 2.0 * (y - t) / (den[:, None, None, None] * B)
    grads = [(np.zeros_like(w), np.zeros_like(b)) for w, b in layers]
    for l in range(len(sizes)):
        if l > 0:
            gy = N.prolong_adjoint(gy, two_d)
        d = 4.0 * (h * 2 ** l) ** 2 * gy
        a = acts[l]
        for j in reversed(range(len(layers))):
            dw, db = N.conv3x3_weight_grad(d, a[j])
            grads[j][0][...] += dw
            grads[j][1][...] += db
            if j > 0:
                d = N.conv3x3_input_grad(d, layers[j][0], a[j].shape[2], a[j].shape[3])
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return N.loss(y, t), flat


def _adam_no_bias_correction(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    return p - lr * m / (np.sqrt(v) + eps), m, v


def _interp_in_index(slices, rows, t, g=None, alpha=1.0):
    M = len(t) - 1
    S, Nq = slices.shape
    g0 = np.zeros(Nq) if g is None else g
    kx = np.concatenate([[-1.0], np.asarray(rows, dtype=float)])
    ky = np.concatenate([g0[None, :], slices], axis=0)
    return np.array([np.interp(np.arange(M), kx, ky[:, q]) for q in range(Nq)]).T


_orig_conv = N.conv3x3

CASES = [
    ("conv3x3", _conv_flipped, [T.test_conv3x3_matches_library_correlation]),
    ("conv3x3_input_grad", _input_grad_unflipped, [T.test_conv_input_and_weight_grads_are_adjoint]),
    ("prolong_adjoint", _adjoint_no_reflection, [lambda: T.test_prolong_adjoint_identity(True)]),
    ("prolong", _prolong_linear, [lambda: T.test_prolongation_of_sine_mode_closed_form(2)]),
    ("restrict", _restrict_injection, [lambda: T.test_restriction_of_sine_mode_closed_form(3)]),
    ("gradient", _gradient_no_tanh_derivative, [lambda: T.test_gradient_matches_central_differences(False)]),
    ("adam_step", _adam_no_bias_correction, [T.test_adam_first_step_closed_form]),
    ("time_interp", _interp_in_index, [T.test_time_interp_exact_on_linear_in_t,
                                       T.test_time_interp_exact_on_linear_in_t_power_alpha]),
]


@pytest.mark.parametrize("name,mutant,pins", CASES, ids=[c[0] for c in CASES])
def test_mutant_is_caught(monkeypatch, name, mutant, pins):
    monkeypatch.setattr(N, name, mutant)
    failed = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed > 0, f"no pin caught the planted mistake in {name}"
