"""Pins of the FP64 network oracle against independent facts: brute-force
loops on tiny inputs, delta kernels, the adjoint identities that define the
backward passes, central finite differences of the whole network, the
closed form of Adam's first step and the bfloat16 rounding rule."""
import itertools

import numpy as np
import pytest

from oracle import nn_oracle as nn


def _brute_conv3(x, W, b):
    Z, Y, X, ci = x.shape
    co = W.shape[0]
    y = np.zeros((Z, Y, X, co))
    for z, yy, xx, o in itertools.product(range(Z), range(Y), range(X), range(co)):
        acc = b[o]
        for t, (dz, dy, dx) in enumerate(itertools.product((-1, 0, 1), repeat=3)):
            zz, y2, x2 = z + dz, yy + dy, xx + dx
            if 0 <= zz < Z and 0 <= y2 < Y and 0 <= x2 < X:
                for c in range(ci):
                    acc += W[o, t, c] * x[zz, y2, x2, c]
        y[z, yy, xx, o] = acc
    return y


def _brute_down2(x, W, b):
    Z, Y, X, ci = x.shape
    co = W.shape[0]
    y = np.zeros((Z // 2, Y // 2, X // 2, co))
    for z, yy, xx, o in itertools.product(range(Z // 2), range(Y // 2), range(X // 2), range(co)):
        acc = b[o]
        for t, (tz, ty, tx) in enumerate(itertools.product((0, 1), repeat=3)):
            for c in range(ci):
                acc += W[o, t, c] * x[2 * z + tz, 2 * yy + ty, 2 * xx + tx, c]
        y[z, yy, xx, o] = acc
    return y


def _brute_up2(x, W, b):
    Z, Y, X, ci = x.shape
    co = W.shape[0]
    y = np.zeros((2 * Z, 2 * Y, 2 * X, co))
    for z, yy, xx, o in itertools.product(range(2 * Z), range(2 * Y), range(2 * X), range(co)):
        t = (z % 2) * 4 + (yy % 2) * 2 + (xx % 2)
        y[z, yy, xx, o] = b[o] + sum(W[o, t, c] * x[z // 2, yy // 2, xx // 2, c] for c in range(ci))
    return y


def test_conv3_matches_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 2))
    W = rng.standard_normal((3, 27, 2))
    b = rng.standard_normal(3)
    assert np.allclose(nn.conv3(x, W, b), _brute_conv3(x, W, b), rtol=0, atol=1e-13)


def test_down_up_match_brute_force():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 2, 6, 3))
    W = rng.standard_normal((2, 8, 3))
    b = rng.standard_normal(2)
    assert np.allclose(nn.down2(x, W, b), _brute_down2(x, W, b), rtol=0, atol=1e-13)
    xc = rng.standard_normal((2, 3, 1, 3))
    assert np.allclose(nn.up2(xc, W, b), _brute_up2(xc, W, b), rtol=0, atol=1e-13)


@pytest.mark.parametrize("t", [0, 4, 13, 22, 26])
def test_conv3_delta_kernel_is_a_shift(t):
    """A kernel that is the identity at one tap and zero elsewhere shifts the
    field by that tap's offset, with zeros entering at the boundary."""
    rng = np.random.default_rng(t)
    x = rng.standard_normal((4, 5, 6, 2))
    W = np.zeros((2, 27, 2))
    W[:, t, :] = np.eye(2)
    dz, dy, dx = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
    y = nn.conv3(x, W, np.zeros(2))
    ref = np.zeros_like(x)
    for z, yy, xx in itertools.product(range(4), range(5), range(6)):
        if 0 <= z + dz < 4 and 0 <= yy + dy < 5 and 0 <= xx + dx < 6:
            ref[z, yy, xx] = x[z + dz, yy + dy, xx + dx]
    assert np.array_equal(y, ref)


@pytest.mark.parametrize("kind", ["conv3", "down2", "up2"])
def test_backward_is_the_adjoint(kind):
    """dgrad is the adjoint of the linear map x -> layer(x) and wgrad the
    adjoint of W -> layer(W): <L(x), g> = <x, L^T g> = <W, dL/dW>."""
    rng = np.random.default_rng(7)
    ci, co = 3, 5
    fine, coarse = (4, 6, 2), (2, 3, 1)
    x = rng.standard_normal((coarse if kind == "up2" else fine) + (ci,))
    T = 27 if kind == "conv3" else 8
    W = rng.standard_normal((co, T, ci))
    fwd = {"conv3": nn.conv3, "down2": nn.down2, "up2": nn.up2}[kind]
    dg = {"conv3": nn.conv3_dgrad, "down2": nn.down2_dgrad, "up2": nn.up2_dgrad}[kind]
    wg = {"conv3": nn.conv3_wgrad, "down2": nn.down2_wgrad, "up2": nn.up2_wgrad}[kind]
    y = fwd(x, W, np.zeros(co))
    g = rng.standard_normal(y.shape)
    lhs = np.sum(y * g)
    assert np.isclose(lhs, np.sum(x * dg(g, W)), rtol=1e-12)
    gW, gb = wg(x, g)
    assert np.isclose(lhs, np.sum(W * gW), rtol=1e-12)
    assert np.allclose(gb, g.reshape(-1, co).sum(axis=0))


def test_network_gradient_matches_central_differences():
    """Reverse-mode gradient of the MSE loss vs central differences in FP64,
    at sampled entries of every layer's weights and bias and of the input."""
    rng = np.random.default_rng(3)
    theta = nn.init_params(5)
    theta[:] += 0.05 * rng.standard_normal(theta.size)  # non-zero biases too
    x = rng.standard_normal((8, 8, 16))
    target = rng.standard_normal((8, 8, 16, 3))
    loss, g, gx = nn.loss_and_grad(theta, x, target, want_dx=True)
    idx, off = [], 0
    for _, ws, bs in nn.layer_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        idx += list(off + rng.choice(nw, 2, replace=False)) + [off + nw + int(rng.integers(nb))]
        off += nw + nb
    h = 1e-6
    worst = 0.0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (nn.loss_and_grad(tp, x, target)[0] - nn.loss_and_grad(tm, x, target)[0]) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / max(abs(g[i]), 1e-3 * np.abs(g).max()))
    for _ in range(4):
        j = tuple(rng.integers(s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (nn.loss_and_grad(theta, xp, target)[0] - nn.loss_and_grad(theta, xm, target)[0]) / (2 * h)
        worst = max(worst, abs(fd - gx[j + (0,)]) / max(abs(gx[j + (0,)]), 1e-3 * np.abs(gx).max()))
    assert worst <= 1e-6, worst


def test_adam_first_step_closed_form():
    """After one step from m = v = 0 the bias-corrected moments are g and
    g^2, so the update is -lr * g / (|g| + eps)."""
    g = np.array([1e-3, -2.0, 0.0, 5e2])
    th, m, v = nn.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.1)
    assert np.allclose(th, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_minimises_a_quadratic():
    theta = np.array([3.0, -4.0])
    m = v = np.zeros(2)
    for k in range(1, 3001):
        theta, m, v = nn.adam_step(theta, m, v, 2 * theta, k, lr=0.01)
    assert np.abs(theta).max() < 1e-2


def test_bf16_rounding_rule():
    torch = pytest.importorskip("torch")
    ulp = 2.0 ** -7
    assert nn.bf16_round(np.array([1 + ulp / 2]))[0] == 1.0             # tie -> even
    assert nn.bf16_round(np.array([1 + 1.5 * ulp]))[0] == 1 + 2 * ulp  # tie -> even
    assert nn.bf16_round(np.array([1 + 0.51 * ulp]))[0] == 1 + ulp
    v = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).integers(-8, 8, 10000)
    ref = torch.from_numpy(v).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(nn.bf16_round(v), ref)


def test_prediction_scales_with_the_source():
    """x = s / max|s| makes the predicted fields exactly proportional to s."""
    rng = np.random.default_rng(2)
    theta = nn.init_params(1)
    s = np.abs(rng.standard_normal((8, 8, 8)))
    k2 = (1.0, 4.0, 9.0)
    a = nn.predict(theta, s, (1.0, 0.5, 2.0), k2)
    b = nn.predict(theta, 7.5 * s, (1.0, 0.5, 2.0), k2)
    for p, q in zip(a, b):
        assert np.abs(q - 7.5 * p).max() <= 1e-13 * np.abs(q).max()


def test_rejects_grids_that_do_not_coarsen_three_times():
    with pytest.raises(ValueError):
        nn.forward(nn.init_params(0), np.zeros((8, 12, 16)))


def test_storage_rounding_option():
    """rnd = identity reproduces the plain FP64 pass bit for bit; with
    bfloat16 rounding every stored activation is a bfloat16 value and the
    loss moves by no more than the storage precision allows."""
    rng = np.random.default_rng(12)
    theta = nn.init_params(3)
    x = rng.random((8, 8, 8))
    t = rng.standard_normal((8, 8, 8, 3))
    l0, g0 = nn.loss_and_grad(theta, x, t)
    l1, g1 = nn.loss_and_grad(theta, x, t, rnd=lambda a: a)
    assert l0 == l1 and np.array_equal(g0, g1)
    _, acts = nn.forward(theta, x, rnd=nn.bf16_round)
    for k, a in acts.items():
        if k not in ("head", "head_in", "x_head"):  # the head and its direct x path stay FP64
            assert np.array_equal(a, nn.bf16_round(a)), k
    l2, g2 = nn.loss_and_grad(theta, x, t, rnd=nn.bf16_round)
    assert abs(l2 - l0) <= 1e-2 * l0
    assert np.linalg.norm(g2 - g0) <= 0.1 * np.linalg.norm(g0)
