"""Pins of the CPU oracle of the learned preconditioner's network (oracle/conv.py).

The network is not from the paper; its definition is the one stated in
oracle/conv.py. These pins check the oracle against things that do not reuse its
code: a brute-force point-by-point convolution, explicit interpolation formulas,
linear-function reproduction, homogeneity, and central finite differences of the
loss.
"""
import numpy as np
import pytest

from oracle import conv


def _brute_conv(a, W):
    # a: [B, Z, Y, X, Ci]; out[b, z, y, x, o] = sum_d sum_i a[b, z+dz, y+dy, x+dx, i] W[tap(d), i, o]
    B, Z, Y, X, Ci = a.shape
    Co = W.shape[2]
    out = np.zeros((B, Z, Y, X, Co))
    for b in range(B):
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    s = np.zeros(Co)
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, yy, xx = z + dz, y + dy, x + dx
                                if 0 <= zz < Z and 0 <= yy < Y and 0 <= xx < X:
                                    t = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
                                    for i in range(Ci):
                                        s += a[b, zz, yy, xx, i] * W[t, i, :]
                    out[b, z, y, x] = s
    return out


def test_conv_matches_brute_force():
    r = np.random.default_rng(1)
    a = r.standard_normal((2, 4, 5, 3, 2))
    W = r.standard_normal((27, 2, 3))
    np.testing.assert_allclose(conv.conv(a, W), _brute_conv(a, W), rtol=1e-13, atol=1e-13)


def test_conv_single_tap_is_a_shift():
    # a weight that is the identity at tap (dx, dy, dz) = (+1, 0, -1) reads a[z-1, y, x+1]
    a = np.arange(4 * 4 * 4, dtype=float).reshape(1, 4, 4, 4, 1)
    W = np.zeros((27, 1, 1))
    W[(1 + 1) + 3 * 1 + 9 * 0, 0, 0] = 1.0
    out = conv.conv(a, W)[0, ..., 0]
    for z in range(4):
        for y in range(4):
            for x in range(4):
                want = a[0, z - 1, y, x + 1, 0] if (z >= 1 and x <= 2) else 0.0
                assert out[z, y, x] == want


def _R1(n):
    """1D full-weighting matrix, (n+1)/2 x n."""
    m = (n + 1) // 2
    R = np.zeros((m, n))
    for I in range(m):
        for d, w in ((-1, 0.25), (0, 0.5), (1, 0.25)):
            if 0 <= 2 * I + d < n:
                R[I, 2 * I + d] = w
    return R


def _P1(n):
    """1D linear interpolation matrix, n x (n+1)/2."""
    m = (n + 1) // 2
    P = np.zeros((n, m))
    for i in range(n):
        if i % 2 == 0:
            P[i, i // 2] = 1.0
        else:
            P[i, i // 2] = P[i, i // 2 + 1] = 0.5
    return P


@pytest.mark.parametrize("n", [5, 9])
def test_restrict_prolong_are_tensor_products(n):
    r = np.random.default_rng(n)
    f = r.standard_normal((1, n, n, n, 2))
    R = _R1(n)
    want = np.einsum("Zz,Yy,Xx,bzyxc->bZYXc", R, R, R, f)
    np.testing.assert_allclose(conv.restrict(f), want, rtol=1e-13, atol=1e-14)
    m = (n + 1) // 2
    c = r.standard_normal((1, m, m, m, 2))
    P = _P1(n)
    want = np.einsum("zZ,yY,xX,bZYXc->bzyxc", P, P, P, c)
    np.testing.assert_allclose(conv.prolong(c, (n, n, n)), want, rtol=1e-13, atol=1e-14)
    # adjointness used by the backward pass: P^T = 8 R (per direction 2 R)
    np.testing.assert_allclose(_P1(n).T, 2.0 * _R1(n), atol=0)


def test_prolong_reproduces_linear_functions():
    n, m = 9, 5
    Z, Y, X = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    c = (1.0 + 2.0 * X - 0.5 * Y + 3.0 * Z)[None, ..., None]
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    want = (1.0 + 2.0 * x / 2 - 0.5 * y / 2 + 3.0 * z / 2)[None, ..., None]
    np.testing.assert_allclose(conv.prolong(c, (n, n, n)), want, rtol=1e-14)


def test_restrict_of_constant_interior():
    f = np.ones((1, 9, 9, 9, 1))
    c = conv.restrict(f)
    np.testing.assert_allclose(c[0, 1:-1, 1:-1, 1:-1, 0], 1.0, rtol=1e-15)
    # a corner coarse point sees only the (1/2 + 1/4)^3 of its in-lattice weights
    assert abs(c[0, 0, 0, 0, 0] - 0.75 ** 3) < 1e-15


def test_parameter_count_and_order():
    for C, L in ((4, 2), (8, 3), (16, 6)):
        assert conv.nparams(C, L) == 27 * (2 * C + (2 * L - 2) * C * C)
    assert conv.layer_names(4) == ["A", "B1", "B2", "B3", "D", "E2", "E1", "F"]


@pytest.mark.parametrize("L", [2, 3, 4])
def test_network_positively_homogeneous(L):
    C = 4
    r = np.random.default_rng(3)
    th = r.standard_normal(conv.nparams(C, L)) * 0.3
    x = r.standard_normal((1, 9, 9, 9, 1))
    y1 = conv.forward(th, C, L, x)
    y2 = conv.forward(th, C, L, 2.5 * x)
    np.testing.assert_allclose(y2, 2.5 * y1, rtol=1e-12, atol=1e-14)


def test_zero_weights_give_the_identity():
    x = np.random.default_rng(8).standard_normal((2, 9, 5, 9, 1))
    np.testing.assert_array_equal(conv.forward(np.zeros(conv.nparams(4, 3)), 4, 3, x), x)


@pytest.mark.parametrize("L", [2, 3])
def test_network_linear_part_matches_explicit_composition(L):
    # with every pre-activation positive the network is linear; check it against
    # composing brute-force convolutions and the explicit 1D transfer matrices
    C = 2
    r = np.random.default_rng(4)
    th = np.abs(r.standard_normal(conv.nparams(C, L))) * 0.2
    x = np.abs(r.standard_normal((1, 5, 5, 5, 1)))
    W = conv.unpack(th, C, L)
    rs = lambda f, M: np.einsum("Zz,Yy,Xx,bzyxc->bZYXc", M, M, M, f)
    sizes = [5, 3, 2][:L]
    h = [_brute_conv(x, W["A"])]
    for l in range(1, L):
        h.append(_brute_conv(rs(h[l - 1], _R1(sizes[l - 1])), W[f"B{l}"]))
    g = _brute_conv(h[L - 1], W["D"])
    for l in range(L - 2, -1, -1):
        u = rs(g, _P1(sizes[l])) + h[l]
        if l >= 1:
            g = _brute_conv(u, W[f"E{l}"])
    y = x + _brute_conv(u, W["F"])
    np.testing.assert_allclose(conv.forward(th, C, L, x), y, rtol=1e-12)


@pytest.mark.parametrize("C,L,n", [(2, 2, 5), (3, 3, 9), (2, 4, 9)])
def test_gradient_matches_central_differences(C, L, n):
    r = np.random.default_rng(10 + C + L)
    th = r.standard_normal(conv.nparams(C, L)) * 0.4
    x = r.standard_normal((2, n, n, n, 1))
    t = r.standard_normal((2, n, n, n, 1))
    loss, g = conv.loss_and_grad(th, C, L, x, t)
    idx = r.choice(th.size, size=40, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (conv.loss_and_grad(tp, C, L, x, t)[0] - conv.loss_and_grad(tm, C, L, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_loss_definition():
    C, L = 2, 2
    r = np.random.default_rng(5)
    th = r.standard_normal(conv.nparams(C, L))
    x = r.standard_normal((3, 5, 5, 5, 1))
    t = r.standard_normal((3, 5, 5, 5, 1))
    y = conv.forward(th, C, L, x)
    want = np.mean([np.sum((y[b] - t[b]) ** 2) / np.sum(t[b] ** 2) for b in range(3)])
    assert abs(conv.loss_and_grad(th, C, L, x, t)[0] - want) <= 1e-13 * want


def test_adam_first_step_closed_form():
    # after one step the bias-corrected moments are g and g^2, so the update is lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 1.0, 1.0, 1.0])
    t1, m, v = conv.adam_step(th, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(t1, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # constant gradient: the bias-corrected moments stay exactly g and g^2
    t2, _, _ = conv.adam_step(t1, g, m, v, 2, lr=0.01)
    np.testing.assert_allclose(t2, t1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_precond_apply_diagonal_scaling_and_passthrough():
    # with zero weights the network is the identity, so z = D^{-1/2} D^{-1/2} r = r / d
    C, L = 4, 2
    th = np.zeros(conv.nparams(C, L))
    n = 5
    r = np.random.default_rng(7)
    perm = r.permutation(n ** 3)
    res = r.standard_normal(n ** 3)
    d = r.uniform(0.5, 2.0, n ** 3)
    bc = np.zeros(n ** 3, bool)
    bc[:7] = True
    z = conv.precond_apply(th, C, L, res, d, perm, (n, n, n), bc)
    np.testing.assert_allclose(z[~bc], res[~bc] / d[~bc], rtol=1e-14)
    np.testing.assert_array_equal(z[bc], res[bc])


def test_energy_loss_gradient_matches_central_differences():
    # a random SPD matrix on a 5^3 lattice with a few pass-through dofs
    C, L, n = 2, 2, 5
    N = n ** 3
    r = np.random.default_rng(21)
    Q = r.standard_normal((N, N))
    A = Q @ Q.T / N + np.eye(N)
    diag = np.diag(A).copy()
    perm = r.permutation(N)
    bc = np.zeros(N, bool)
    bc[perm[:9]] = True
    res = r.standard_normal(N)
    th = r.standard_normal(conv.nparams(C, L)) * 0.3
    loss, g = conv.energy_loss_and_grad(th, C, L, res, A, diag, perm, (n, n, n), bc)
    for i in r.choice(th.size, size=30, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[i] += 1e-6
        tm[i] -= 1e-6
        fd = (conv.energy_loss_and_grad(tp, C, L, res, A, diag, perm, (n, n, n), bc)[0]
              - conv.energy_loss_and_grad(tm, C, L, res, A, diag, perm, (n, n, n), bc)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_energy_loss_of_the_exact_inverse_is_minus_one_in_the_scaled_units():
    # z = A^{-1} r gives z^T A z - 2 z^T r = -r^T A^{-1} r, and any other z is larger:
    # check the definition with zero weights (z = D^{-1} r) against the closed form
    n = 5
    N = n ** 3
    r = np.random.default_rng(22)
    Q = r.standard_normal((N, N))
    A = Q @ Q.T / N + np.eye(N)
    d = np.diag(A).copy()
    res = r.standard_normal(N)
    bc = np.zeros(N, bool)
    loss, _ = conv.energy_loss_and_grad(np.zeros(conv.nparams(4, 2)), 4, 2, res, A, d, np.arange(N), (n, n, n), bc)
    z = res / d
    want = (z @ A @ z - 2 * z @ res) / np.sum(res * res / d)
    assert abs(loss - want) <= 1e-12 * abs(want)
    best = -(res @ np.linalg.solve(A, res)) / np.sum(res * res / d)
    assert loss >= best
