"""CPU oracle of the learned preconditioner's network (forward, loss, backward).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline use it. Plain numpy in float64, direct sliding-window convolutions,
backward written out by the chain rule. The network is not from the paper; it
is the convolutional approximate inverse used as a preconditioner for CG on the
tensor-product DoF lattice. Definition (L >= 2 levels, C channels, lattices of
n points per direction with (n - 1) divisible by 2^(L-1), channel-last arrays
[batch, z, y, x, c]):

  h_0 = relu(conv_A(x))                              1 -> C
  c_l = R h_(l-1),  h_l = relu(conv_B_l(c_l))        l = 1 .. L-1, C -> C
  g_(L-1) = relu(conv_D(h_(L-1)))                    C -> C
  u_l = P g_(l+1) + h_l                              l = L-2 .. 0
  g_l = relu(conv_E_l(u_l))                          l = L-2 .. 1, C -> C
  y = x + conv_F(u_0)                                C -> 1

conv: 3x3x3 taps, zero padding, no bias; weight W[tap, cin, cout] with
tap = (dx+1) + 3 (dy+1) + 9 (dz+1) and out[v] = sum_d in[v + d] W[tap(d)].
R (full weighting): c[I] = sum_d prod_k w(d_k) f[2I + d], w(0)=1/2, w(+-1)=1/4,
values outside the fine lattice are 0. P (trilinear prolongation):
f[i] = sum_I prod_k l(i_k - 2 I_k) c[I], l(0)=1, l(+-1)=1/2, so P^T = 8 R.
Parameters in the order A, B_1 .. B_(L-1), D, E_(L-2) .. E_1, F.
Loss of a sample: |y - t|^2 / |t|^2; a batch averages the samples.
"""
from __future__ import annotations

import numpy as np


def layer_names(L: int):
    return ["A"] + [f"B{l}" for l in range(1, L)] + ["D"] + [f"E{l}" for l in range(L - 2, 0, -1)] + ["F"]


def layer_shapes(C: int, L: int):
    sh = {}
    for name in layer_names(L):
        sh[name] = (27, 1, C) if name == "A" else (27, C, 1) if name == "F" else (27, C, C)
    return sh


def unpack(theta: np.ndarray, C: int, L: int):
    out, o = {}, 0
    for name, sh in layer_shapes(C, L).items():
        n = int(np.prod(sh))
        out[name] = theta[o:o + n].reshape(sh)
        o += n
    assert o == theta.size
    return out


def nparams(C: int, L: int) -> int:
    return sum(int(np.prod(s)) for s in layer_shapes(C, L).values())


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
        out[tuple(idx_odd)] = 0.5 * (out[tuple(idx_lo)] + out[tuple(idx_hi)])
    return out


def relu(a):
    return np.maximum(a, 0.0)


def forward(theta: np.ndarray, C: int, L: int, x: np.ndarray, keep: bool = False):
    """x: [B, nz, ny, nx, 1] -> y: [B, nz, ny, nx, 1]."""
    W = unpack(theta, C, L)
    h = [relu(conv(x, W["A"]))]
    c = [None]
    for l in range(1, L):
        c.append(restrict(h[l - 1]))
        h.append(relu(conv(c[l], W[f"B{l}"])))
    g = [None] * L
    u = [None] * (L - 1)
    g[L - 1] = relu(conv(h[L - 1], W["D"]))
    for l in range(L - 2, -1, -1):
        u[l] = prolong(g[l + 1], h[l].shape[1:4]) + h[l]
        if l >= 1:
            g[l] = relu(conv(u[l], W[f"E{l}"]))
    y = x + conv(u[0], W["F"])
    if keep:
        return y, dict(x=x, h=h, c=c, g=g, u=u)
    return y


def backward(theta: np.ndarray, C: int, L: int, acts: dict, gy: np.ndarray) -> np.ndarray:
    """Gradient with respect to theta given gy = dLoss/dy and the kept activations."""
    W = unpack(theta, C, L)
    x, h, c, g, u = acts["x"], acts["h"], acts["c"], acts["g"], acts["u"]
    grads = {}
    # decoder, fine to coarse: y = x + F u_0 (the skip from x carries no weight)
    gu = [None] * (L - 1)
    gu[0], grads["F"] = conv_backward(u[0], W["F"], gy)
    gh = [None] * L
    for l in range(0, L - 1):
        gh[l] = gu[l].copy()  # u_l = P g_(l+1) + h_l
        gg = restrict(gu[l]) * 8.0 * (g[l + 1] > 0)  # P^T = 8 R, then the relu of g_(l+1)
        if l + 1 <= L - 2:
            gu[l + 1], grads[f"E{l + 1}"] = conv_backward(u[l + 1], W[f"E{l + 1}"], gg)
        else:
            gh[L - 1], grads["D"] = conv_backward(h[L - 1], W["D"], gg)
    # encoder, coarse to fine
    for l in range(L - 1, 0, -1):
        gpre = gh[l] * (h[l] > 0)
        gc, grads[f"B{l}"] = conv_backward(c[l], W[f"B{l}"], gpre)
        gh[l - 1] = gh[l - 1] + prolong(gc, h[l - 1].shape[1:4]) / 8.0  # R^T = P / 8
    _, grads["A"] = conv_backward(x, W["A"], gh[0] * (h[0] > 0))
    return np.concatenate([grads[k].ravel() for k in layer_names(L)])


def loss_and_grad(theta: np.ndarray, C: int, L: int, x: np.ndarray, t: np.ndarray):
    """Batch-mean relative squared error and its gradient with respect to theta."""
    y, acts = forward(theta, C, L, x, keep=True)
    B = x.shape[0]
    tt = np.sum(t.reshape(B, -1) ** 2, axis=1)
    diff = (y - t).reshape(B, -1)
    loss = float(np.mean(np.sum(diff ** 2, axis=1) / tt))
    gy = (2.0 / B) * (diff / tt[:, None]).reshape(y.shape)
    return loss, backward(theta, C, L, acts, gy)


def energy_loss_and_grad(theta, C, L, r, A, diag, grid_of_dof, shape, dirichlet):
    """Energy (Ritz) loss of the preconditioned residual z = M r for one residual r:
    (z^T A z - 2 z^T r) / (r^T D^{-1} r), i.e. the A-norm error of z against A^{-1} r
    up to the constant r^T A^{-1} r, and its gradient with respect to theta. A is a
    dense symmetric matrix; constrained dofs pass r through (z_B = r_B)."""
    s = 1.0 / np.sqrt(diag)
    g = np.zeros(int(np.prod(shape)))
    g[grid_of_dof] = s * r
    x = g.reshape((1,) + tuple(shape) + (1,))
    y, acts = forward(theta, C, L, x, keep=True)
    z = np.where(dirichlet, r, s * y.reshape(-1)[grid_of_dof])
    Az = A @ z
    ns = float(np.sum(r * r / diag))
    loss = float((z @ Az - 2.0 * z @ r) / ns)
    gz = np.where(dirichlet, 0.0, 2.0 * (Az - r) / ns)
    gyv = np.zeros(int(np.prod(shape)))
    gyv[grid_of_dof] = s * gz
    return loss, backward(theta, C, L, acts, gyv.reshape(y.shape))


def adam_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), step counted from 1; returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def precond_apply(theta, C, L, r, diag, grid_of_dof, shape, dirichlet=None):
    """z = D^{-1/2} N(D^{-1/2} r) on the lattice: dof i sits at linear index
    grid_of_dof[i] of a (z, y, x) lattice of `shape`; constrained dofs pass through."""
    s = 1.0 / np.sqrt(diag)
    g = np.zeros(int(np.prod(shape)))
    g[grid_of_dof] = s * r
    y = forward(theta, C, L, g.reshape((1,) + tuple(shape) + (1,)))
    z = s * y.reshape(-1)[grid_of_dof]
    if dirichlet is not None:
        z = np.where(dirichlet, r, z)
    return z
