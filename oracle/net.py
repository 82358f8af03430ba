"""Oracle of the learned initial guess: the band-pyramid convolution network,
its loss, gradient and Adam update, and the time interpolation of its output,
in plain float64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The network is not part of the paper (whose iteration starts from a given
iterate, Sections 4-5); this module states what the library's network
computes so that its forward, backward and optimiser kernels can be checked:

* pyramid over grids of n_0 = W = 2^p - 1 points per side, n_{l+1} =
  (n_l - 1)/2 down to 3; coarse point i sits on fine point 2i + 1;
  restriction R is full weighting ((1/4)[1 2 1] per dimension), P the
  4-point (cubic) interpolation per dimension with the coarse values extended
  by zero boundary values and their odd reflections;
* c_0 = signal, c_{l+1} = R c_l, band_l = c_l - P c_{l+1}, band_last = c_last;
* at every level the same stack of 3x3 cross-correlations with zero padding
  (tanh between layers) maps [band_l, the extra channels sampled at the
  level's points, log2(1/h_l)/10] to out_l, and y = sum_l P^l (4 h_l^2 out_l)
  with h_l = 2^l h; levels finer than a cut-off h_min (bands finer than the
  grids the network was trained on) are left out;
* loss L = (1/B) sum_b ||y_b - t_b||^2 / ||t_b||^2;
* Adam (Kingma and Ba, 2015) with bias-corrected moments;
* the space-time initial iterate: slice s placed at t_{rows[s]+1},
  piecewise-linear in t^alpha from the initial value at t_0, constant after
  the last slice.
"""
from __future__ import annotations

import numpy as np


def pyramid_sizes(W: int) -> list[int]:
    """Points per side of every level: W, (W-1)/2, ..., 3."""
    if W < 3 or (W + 1) & W:
        raise ValueError("W must be 2^p - 1 >= 3")
    out = []
    n = W
    while n >= 3:
        out.append(n)
        n = (n - 1) // 2
    return out


def _restrict_1d(a: np.ndarray, axis: int) -> np.ndarray:
    a = np.moveaxis(a, axis, -1)
    r = 0.25 * (a[..., 0:-2:2] + 2.0 * a[..., 1:-1:2] + a[..., 2::2])
    return np.moveaxis(r, -1, axis)


def _prolong_1d(a: np.ndarray, axis: int) -> np.ndarray:
    """Fine points on coarse ones copy them; midpoints take the cubic value
    (-c[i-2] + 9 c[i-1] + 9 c[i] - c[i+1]) / 16 of the coarse values extended
    as an odd function about both zero boundary values."""
    a = np.moveaxis(a, axis, -1)
    nc = a.shape[-1]
    z = np.zeros(a.shape[:-1] + (1,))
    ext = np.concatenate([-a[..., :1], z, a, z, -a[..., -1:]], axis=-1)   # c[-2..nc+1]
    out = np.zeros(a.shape[:-1] + (2 * nc + 1,))
    out[..., 1::2] = a
    for i in range(nc + 1):            # midpoint between coarse i-1 and i is fine 2i
        cm2, cm1, c0, cp1 = (ext[..., i - 2 + 2], ext[..., i - 1 + 2], ext[..., i + 2], ext[..., i + 1 + 2])
        out[..., 2 * i] = (-cm2 + 9.0 * cm1 + 9.0 * c0 - cp1) / 16.0
    return np.moveaxis(out, -1, axis)


def restrict(a: np.ndarray, two_d: bool) -> np.ndarray:
    """Full weighting over the last axis (and the one before it in 2D)."""
    r = _restrict_1d(a, a.ndim - 1)
    return _restrict_1d(r, a.ndim - 2) if two_d else r


def prolong(a: np.ndarray, two_d: bool) -> np.ndarray:
    """4-point interpolation over the last axis (and the one before in 2D)."""
    p = _prolong_1d(a, a.ndim - 1)
    return _prolong_1d(p, a.ndim - 2) if two_d else p


def prolong_adjoint(g: np.ndarray, two_d: bool) -> np.ndarray:
    """P^T g, written from the columns of P: coarse i collects fine 2i+1
    (weight 1), 2i and 2i+2 (9/16), 2i-2 and 2i+4 (-1/16), and through the
    odd reflections 1/16 more of fine 0 (i = 0) and of fine 2nc (i = nc-1)."""
    def adj(a, axis):
        a = np.moveaxis(a, axis, -1)
        nf = a.shape[-1]
        nc = (nf - 1) // 2
        r = np.zeros(a.shape[:-1] + (nc,))
        for i in range(nc):
            taps = [(2 * i - 2, -1 / 16), (2 * i, 9 / 16), (2 * i + 1, 1.0), (2 * i + 2, 9 / 16), (2 * i + 4, -1 / 16)]
            for f, w in taps:
                if 0 <= f < nf:
                    r[..., i] += w * a[..., f]
        r[..., 0] += a[..., 0] / 16
        r[..., nc - 1] += a[..., nf - 1] / 16
        return np.moveaxis(r, -1, axis)
    r = adj(g, g.ndim - 1)
    return adj(r, g.ndim - 2) if two_d else r


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[n, o, i, j] = b[o] + sum_c sum_{di,dj} w[o, c, di, dj] x[n, c, i+di-1, j+dj-1]
    (cross-correlation, zero padding).  x [B][C][H][W], w [O][C][3][3]."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.broadcast_to(b[None, :, None, None], (B, w.shape[0], H, W)).copy()
    for di in range(3):
        for dj in range(3):
            y += np.einsum("oc,bchw->bohw", w[:, :, di, dj], xp[:, :, di:di + H, dj:dj + W])
    return y


def conv3x3_input_grad(dy: np.ndarray, w: np.ndarray, H: int, W: int) -> np.ndarray:
    """d(sum dy * conv3x3(x))/dx: every output (i, j) sends w[o, c, di, dj] dy
    back to input (i+di-1, j+dj-1)."""
    B = dy.shape[0]
    dxp = np.zeros((B, w.shape[1], H + 2, W + 2))
    for di in range(3):
        for dj in range(3):
            dxp[:, :, di:di + H, dj:dj + W] += np.einsum("oc,bohw->bchw", w[:, :, di, dj], dy)
    return dxp[:, :, 1:-1, 1:-1]


def conv3x3_weight_grad(dy: np.ndarray, x: np.ndarray):
    """Gradients of sum dy * conv3x3(x) with respect to w and b."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dw = np.zeros((dy.shape[1], C, 3, 3))
    for di in range(3):
        for dj in range(3):
            dw[:, :, di, dj] = np.einsum("bohw,bchw->oc", dy, xp[:, :, di:di + H, dj:dj + W])
    return dw, dy.sum(axis=(0, 2, 3))


def unpack(params: np.ndarray, channels: list[int]):
    """Flat parameters -> [(w [c_out][c_in][3][3], b [c_out])] per layer."""
    out, off = [], 0
    params = np.asarray(params, dtype=np.float64)
    for cin, cout in zip(channels[:-1], channels[1:]):
        w = params[off:off + cout * cin * 9].reshape(cout, cin, 3, 3)
        off += cout * cin * 9
        b = params[off:off + cout]
        off += cout
        out.append((w, b))
    if off != params.size:
        raise ValueError("parameter count does not match the channels")
    return out


def param_count(channels: list[int]) -> int:
    return sum(cout * cin * 9 + cout for cin, cout in zip(channels[:-1], channels[1:]))


def level_inputs(x: np.ndarray, nsig: int, h: float):
    """Per-level network inputs [band, extra channels at the level's points,
    level value] for x [B][S+E][H][W]."""
    B, C, H, W = x.shape
    two_d = H > 1
    if two_d and H != W:
        raise ValueError("a 2D grid must be square")
    sizes = pyramid_sizes(W)
    sig = [x[:, :nsig]]
    for _ in sizes[1:]:
        sig.append(restrict(sig[-1], two_d))
    inputs = []
    for l, n in enumerate(sizes):
        band = sig[l] - prolong(sig[l + 1], two_d) if l + 1 < len(sizes) else sig[l]
        stride = 2 ** l
        idx = stride * (np.arange(n) + 1) - 1
        extra = x[:, nsig:][:, :, idx][:, :, :, idx] if two_d else x[:, nsig:][:, :, :, idx]
        hl = h * stride
        lev = np.full((B, 1) + band.shape[2:], np.log2(1.0 / hl) / 10.0)
        inputs.append(np.concatenate([band, extra, lev], axis=1))
    return inputs, sizes, two_d


def forward(params: np.ndarray, channels: list[int], x: np.ndarray, nsig: int, h: float, cache: bool = False,
            h_min: float = 0.0, act_bf16: bool = False):
    """Network output y [B][c_L][H][W] (and the activations when cache).
    Levels with h_l < h_min are left out (out_l = 0).  act_bf16: the input of
    every convolution is rounded to float32 and then to the nearest bfloat16
    first (the precision of the library's matrix-core inference)."""
    layers = unpack(params, channels)
    inputs, sizes, two_d = level_inputs(np.asarray(x, dtype=np.float64), nsig, h)
    acts, outs = [], []
    for l, xin in enumerate(inputs):
        if h * 2 ** l < h_min * (1 - 1e-9):
            acts.append(None)
            outs.append(np.zeros((xin.shape[0], channels[-1]) + xin.shape[2:]))
            continue
        a = [xin]
        for j, (w, b) in enumerate(layers):
            inp = bf16_round(a[-1].astype(np.float32)).astype(np.float64) if act_bf16 else a[-1]
            z = conv3x3(inp, w, b)
            a.append(np.tanh(z) if j + 1 < len(layers) else z)
        acts.append(a)
        outs.append(a[-1])
    y = None
    for l in reversed(range(len(sizes))):
        hl = h * 2 ** l
        term = 4.0 * hl * hl * outs[l]
        y = term if y is None else term + prolong(y, two_d)
    return (y, (acts, sizes, two_d)) if cache else y


def loss(y: np.ndarray, t: np.ndarray) -> float:
    num = ((y - t) ** 2).sum(axis=(1, 2, 3))
    den = (t ** 2).sum(axis=(1, 2, 3))
    return float((num / den).mean())


def gradient(params: np.ndarray, channels: list[int], x: np.ndarray, t: np.ndarray, nsig: int, h: float,
             h_min: float = 0.0):
    """(loss, dL/dparams) by reverse-mode differentiation of forward()."""
    layers = unpack(params, channels)
    y, (acts, sizes, two_d) = forward(params, channels, x, nsig, h, cache=True, h_min=h_min)
    B = y.shape[0]
    den = (t ** 2).sum(axis=(1, 2, 3))
    gy = 2.0 * (y - t) / (den[:, None, None, None] * B)
    grads = [(np.zeros_like(w), np.zeros_like(b)) for w, b in layers]
    for l in range(len(sizes)):
        if l > 0:
            gy = prolong_adjoint(gy, two_d)
        hl = h * 2 ** l
        a = acts[l]
        if a is None:
            continue
        d = 4.0 * hl * hl * gy
        for j in reversed(range(len(layers))):
            dw, db = conv3x3_weight_grad(d, a[j])
            grads[j][0][...] += dw
            grads[j][1][...] += db
            if j > 0:
                d = conv3x3_input_grad(d, layers[j][0], a[j].shape[2], a[j].shape[3]) * (1.0 - a[j] ** 2)
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return loss(y, t), flat


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update; returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even)."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def time_interp(slices: np.ndarray, rows, t: np.ndarray, g: np.ndarray | None = None,
                alpha: float = 1.0) -> np.ndarray:
    """Space-time iterate [M][N] from slice values [S][N]: slice s at
    t[rows[s]+1], piecewise linear in the variable t^alpha from (t[0], g) to
    the first slice and between slices, constant after the last one."""
    M = len(t) - 1
    S, N = slices.shape
    g0 = np.zeros(N) if g is None else np.asarray(g, dtype=np.float64)
    s = np.asarray(t, dtype=np.float64) ** alpha
    knots_s = np.concatenate([[s[0]], s[np.asarray(rows) + 1]])
    knots_y = np.concatenate([g0[None, :], slices], axis=0)
    U = np.empty((M, N))
    for q in range(N):
        U[:, q] = np.interp(s[1:], knots_s, knots_y[:, q])
    return U


def warm_start_input(b: np.ndarray, rows, alpha: float, r: float, dim: int, n: int):
    """Network input [1][S+2][H][W] of one instance and the scale ||b||_inf."""
    scale = float(np.abs(b).max())
    S = len(rows)
    H = 1 if dim == 1 else n
    x = np.empty((1, S + 2, H, n))
    for s, row in enumerate(rows):
        x[0, s] = (b[row] / scale).reshape(H, n)
    x[0, S] = alpha
    x[0, S + 1] = r / 10.0
    return x, scale
