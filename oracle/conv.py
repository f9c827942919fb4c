"""CPU oracle of the learned preconditioner's network (forward, loss, backward).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU baseline use it. Plain numpy in float64,
direct sliding-window convolutions, backward written out by the chain rule.
The network is not from the paper; it is the small convolutional
approximate inverse used as a preconditioner for CG on the tensor-product
DoF lattice. Definition (node lattices of n = 4m + 1 points per direction,
channel-last arrays [z, y, x, c]):

  h0 = relu(conv_A(x))          n^3, 1 -> C
  c1 = R(h0)                    m1 = (n+1)/2
  h1 = relu(conv_B(c1))         C -> C
  c2 = R(h1)                    m2 = (m1+1)/2
  h2 = relu(conv_C(c2))         C -> C
  g2 = relu(conv_D(h2))         C -> C
  u1 = P(g2) + h1
  g1 = relu(conv_E(u1))         C -> C
  u0 = P(g1) + h0
  y  = conv_F(u0)               C -> 1

conv: 3x3x3 taps, zero padding, no bias; weight W[tap, cin, cout] with
tap = (dx+1) + 3 (dy+1) + 9 (dz+1) and out[v] = sum in[v + d] W[tap(d)].
R (full weighting): c[I] = sum_d prod_k w(d_k) f[2I + d], w(0)=1/2, w(+-1)=1/4,
values outside the fine lattice are 0. P (trilinear prolongation):
f[i] = sum_I prod_k l(i_k - 2 I_k) c[I], l(0)=1, l(+-1)=1/2, so P^T = 8 R.
Loss of a sample: |y - t|^2 / |t|^2; a batch averages the samples.
"""
from __future__ import annotations

import numpy as np

LAYERS = ("A", "B", "C", "D", "E", "F")


def layer_shapes(C: int):
    return {"A": (27, 1, C), "B": (27, C, C), "C": (27, C, C), "D": (27, C, C), "E": (27, C, C), "F": (27, C, 1)}


def unpack(theta: np.ndarray, C: int):
    out, o = {}, 0
    for name in LAYERS:
        sh = layer_shapes(C)[name]
        n = int(np.prod(sh))
        out[name] = theta[o:o + n].reshape(sh)
        o += n
    assert o == theta.size
    return out


def nparams(C: int) -> int:
    return sum(int(np.prod(s)) for s in layer_shapes(C).values())


def _taps():
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yield (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1), dz, dy, dx


def _shift(a: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """s[v] = a[v + d] with zeros outside (a: [..., z, y, x, c])."""
    out = np.zeros_like(a)
    Z, Y, X = a.shape[-4:-1]

    def rng(d, n):
        return (slice(max(0, -d), n - max(0, d)), slice(max(0, d), n - max(0, -d)))

    (oz, iz), (oy, iy), (ox, ix) = rng(dz, Z), rng(dy, Y), rng(dx, X)
    out[..., oz, oy, ox, :] = a[..., iz, iy, ix, :]
    return out


def conv(a: np.ndarray, W: np.ndarray) -> np.ndarray:
    out = np.zeros(a.shape[:-1] + (W.shape[2],))
    for t, dz, dy, dx in _taps():
        out += _shift(a, dz, dy, dx) @ W[t]
    return out


def conv_backward(a: np.ndarray, W: np.ndarray, g: np.ndarray):
    """For out = conv(a, W): returns (dL/da, dL/dW) given g = dL/dout."""
    da = np.zeros_like(a)
    dW = np.zeros_like(W)
    for t, dz, dy, dx in _taps():
        s = _shift(a, dz, dy, dx)
        dW[t] = s.reshape(-1, s.shape[-1]).T @ g.reshape(-1, g.shape[-1])
        # out[v] += a[v + d] W  =>  da[u] += g[u - d] W^T
        da += _shift(g @ W[t].T, -dz, -dy, -dx)
    return da, dW


def restrict(f: np.ndarray) -> np.ndarray:
    Z, Y, X = f.shape[-4:-1]
    mz, my, mx = (Z + 1) // 2, (Y + 1) // 2, (X + 1) // 2
    out = np.zeros(f.shape[:-4] + (mz, my, mx) + f.shape[-1:])
    w = {-1: 0.25, 0: 0.5, 1: 0.25}
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                s = _shift(f, dz, dy, dx)
                out += w[dz] * w[dy] * w[dx] * s[..., ::2, ::2, ::2, :]
    return out


def prolong(c: np.ndarray, shape) -> np.ndarray:
    """Trilinear interpolation from the coarse lattice to the fine one of `shape` (z, y, x)."""
    out = np.zeros(c.shape[:-4] + tuple(shape) + c.shape[-1:])
    out[..., ::2, ::2, ::2, :] = c
    # interpolate along x, then y, then z (odd points are averages of their two neighbours)
    for ax in (-2, -3, -4):
        n = out.shape[ax]
        idx_odd = [slice(None)] * out.ndim
        idx_lo = [slice(None)] * out.ndim
        idx_hi = [slice(None)] * out.ndim
        idx_odd[ax] = slice(1, n - 1, 2)
        idx_lo[ax] = slice(0, n - 2, 2)
        idx_hi[ax] = slice(2, n, 2)
        # only rows already filled along the earlier axes are interpolated here
        out[tuple(idx_odd)] = 0.5 * (out[tuple(idx_lo)] + out[tuple(idx_hi)])
    return out


def relu(a):
    return np.maximum(a, 0.0)


def forward(theta: np.ndarray, C: int, x: np.ndarray, keep: bool = False):
    """x: [B, n, n, n, 1] -> y: [B, n, n, n, 1]."""
    W = unpack(theta, C)
    n = x.shape[1:4]
    h0 = relu(conv(x, W["A"]))
    c1 = restrict(h0)
    h1 = relu(conv(c1, W["B"]))
    c2 = restrict(h1)
    h2 = relu(conv(c2, W["C"]))
    g2 = relu(conv(h2, W["D"]))
    u1 = prolong(g2, h1.shape[1:4]) + h1
    g1 = relu(conv(u1, W["E"]))
    u0 = prolong(g1, n) + h0
    y = conv(u0, W["F"])
    if keep:
        return y, dict(x=x, h0=h0, c1=c1, h1=h1, c2=c2, h2=h2, g2=g2, u1=u1, g1=g1, u0=u0)
    return y


def loss_and_grad(theta: np.ndarray, C: int, x: np.ndarray, t: np.ndarray):
    """Batch-mean relative squared error and its gradient with respect to theta."""
    W = unpack(theta, C)
    y, a = forward(theta, C, x, keep=True)
    B = x.shape[0]
    tt = np.sum(t.reshape(B, -1) ** 2, axis=1)
    diff = (y - t).reshape(B, -1)
    loss = float(np.mean(np.sum(diff ** 2, axis=1) / tt))
    gy = (2.0 / B) * (diff / tt[:, None]).reshape(y.shape)
    grads = {}
    gu0, grads["F"] = conv_backward(a["u0"], W["F"], gy)
    gh0 = gu0.copy()
    gg1 = restrict(gu0) * 8.0  # P^T = 8 R
    gg1 = gg1 * (a["g1"] > 0)
    gu1, grads["E"] = conv_backward(a["u1"], W["E"], gg1)
    gh1 = gu1.copy()
    gg2 = restrict(gu1) * 8.0
    gg2 = gg2 * (a["g2"] > 0)
    gh2, grads["D"] = conv_backward(a["h2"], W["D"], gg2)
    gh2 = gh2 * (a["h2"] > 0)
    gc2, grads["C"] = conv_backward(a["c2"], W["C"], gh2)
    gh1 = gh1 + prolong(gc2, a["h1"].shape[1:4]) / 8.0  # R^T = P / 8
    gh1 = gh1 * (a["h1"] > 0)
    gc1, grads["B"] = conv_backward(a["c1"], W["B"], gh1)
    gh0 = gh0 + prolong(gc1, a["h0"].shape[1:4]) / 8.0
    gh0 = gh0 * (a["h0"] > 0)
    _, grads["A"] = conv_backward(a["x"], W["A"], gh0)
    g = np.concatenate([grads[k].ravel() for k in LAYERS])
    return loss, g


def adam_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), step counted from 1; returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def precond_apply(theta, C, r, diag, grid_of_dof, shape, dirichlet=None):
    """z = D^{-1/2} N(D^{-1/2} r) on the lattice: dof i sits at linear index
    grid_of_dof[i] of a (z, y, x) lattice of `shape`; constrained dofs pass through."""
    s = 1.0 / np.sqrt(diag)
    g = np.zeros(int(np.prod(shape)))
    g[grid_of_dof] = s * r
    y = forward(theta, C, g.reshape((1,) + tuple(shape) + (1,)))
    z = s * y.reshape(-1)[grid_of_dof]
    if dirichlet is not None:
        z = np.where(dirichlet, r, z)
    return z
