"""FP64 NumPy oracle of the learned initial guess — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct forward and backward pass of the 3D
convolutional U-net that predicts the three screened photon-group fields
kappa_i^2 Psi_i from the ionisation source s (the three Helmholtz equations
of the radiative-transfer model, paper Sec. 2), written from the textbook
definitions of cross-correlation, ReLU, mean-squared error and Adam (Kingma
& Ba, "Adam: a method for stochastic optimization", 2015, Algorithm 1).
The paper itself has no network; its architecture is fixed here:

    level 0 (n)    e0a conv3 1->16, e0b conv3 16->16          -> skip0
                   d0  down2 16->32
    level 1 (n/2)  e1a conv3 32->32, e1b conv3 32->32         -> skip1
                   d1  down2 32->64
    level 2 (n/4)  e2a conv3 64->64, e2b conv3 64->64         -> skip2
                   d2  down2 64->64
    level 3 (n/8)  b3a conv3 64->64, b3b conv3 64->64
                   u2  up2 64->64, concat skip2
    level 2        c2a conv3 128->64, c2b conv3 64->64
                   u1  up2 64->32, concat skip1
    level 1        c1a conv3 64->32, c1b conv3 32->32
                   u0  up2 32->16, concat skip0
    level 0        c0a conv3 32->16, c0b conv3 16->16
                   head: linear map of (c0b's 16 channels, the 27 values
                   of the scaled input x around the cell) -> 3

Every layer except the head adds a bias and applies ReLU.  conv3 is a
3x3x3 cross-correlation with zero padding; down2 is a 2x2x2 stride-2
cross-correlation; up2 is its transpose (each fine cell 2V+t receives
W[:, t, :] @ x[V]).  Concatenation puts the upsampled channels first.  The
head's direct path from x (a 3x3x3 stencil, zero padding) lets the local
part of the screened fields bypass the network.

Tensors are channels-last ``[z][y][x][c]``.  Weights of a layer are
``W[cout][tap][cin]`` with taps ``t = (dz+1)*9 + (dy+1)*3 + (dx+1)`` for
conv3 (offset (dz,dy,dx)) and ``t = tz*4 + ty*2 + tx`` for down2/up2; the
head is ``W[3][16 + 27]`` (c0b channels, then x at taps 0..26).  The flat
parameter vector lists the layers in the order above, each as W (C order)
followed by b.

Input and output scaling: x = s / max|s|; the network output y_i is in
units of ``scale_i`` so that the predicted field is
``kappa_i^2 Psi_i = max|s| * scale_i * y_i``.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

# (name, kind, cin, cout); kind in {"conv3", "down2", "up2", "head"}
LAYERS: List[Tuple[str, str, int, int]] = [
    ("e0a", "conv3", 1, 16), ("e0b", "conv3", 16, 16), ("d0", "down2", 16, 32),
    ("e1a", "conv3", 32, 32), ("e1b", "conv3", 32, 32), ("d1", "down2", 32, 64),
    ("e2a", "conv3", 64, 64), ("e2b", "conv3", 64, 64), ("d2", "down2", 64, 64),
    ("b3a", "conv3", 64, 64), ("b3b", "conv3", 64, 64), ("u2", "up2", 64, 64),
    ("c2a", "conv3", 128, 64), ("c2b", "conv3", 64, 64), ("u1", "up2", 64, 32),
    ("c1a", "conv3", 64, 32), ("c1b", "conv3", 32, 32), ("u0", "up2", 32, 16),
    ("c0a", "conv3", 32, 16), ("c0b", "conv3", 16, 16), ("head", "head", 16 + 27, 3),
]
NTAPS = {"conv3": 27, "down2": 8, "up2": 8}


def layer_shapes() -> List[Tuple[str, Tuple[int, ...], Tuple[int, ...]]]:
    out = []
    for name, kind, cin, cout in LAYERS:
        w = (cout, cin) if kind == "head" else (cout, NTAPS[kind], cin)
        out.append((name, w, (cout,)))
    return out


def num_params() -> int:
    return sum(int(np.prod(w)) + int(np.prod(b)) for _, w, b in layer_shapes())


def unflatten(theta: np.ndarray) -> Dict[str, Tuple[np.ndarray, np.ndarray]]:
    p, off = {}, 0
    for name, ws, bs in layer_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        p[name] = (theta[off:off + nw].reshape(ws), theta[off + nw:off + nw + nb].reshape(bs))
        off += nw + nb
    assert off == theta.size
    return p


def flatten(p: Dict[str, Tuple[np.ndarray, np.ndarray]]) -> np.ndarray:
    return np.concatenate([np.concatenate([p[n][0].ravel(), p[n][1].ravel()]) for n, _, _ in layer_shapes()])


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, kind, cin, cout in LAYERS:
        fan_in = cin * (1 if kind == "head" else NTAPS[kind])
        shape = (cout, cin) if kind == "head" else (cout, NTAPS[kind], cin)
        std = np.sqrt((1.0 if kind == "head" else 2.0) / fan_in)
        parts += [std * rng.standard_normal(shape).ravel(), np.zeros(cout)]
    return np.concatenate(parts)


# ----------------------------------------------------------------- layers
def _offsets3():
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shifted(x: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """out[z,y,x] = x[z+dz, y+dy, x+dx], zero outside the grid."""
    Z, Y, X = x.shape[:3]
    out = np.zeros_like(x)
    zs, ys, xs = slice(max(0, -dz), min(Z, Z - dz)), slice(max(0, -dy), min(Y, Y - dy)), slice(max(0, -dx), min(X, X - dx))
    zt = slice(zs.start + dz, zs.stop + dz)
    yt = slice(ys.start + dy, ys.stop + dy)
    xt = slice(xs.start + dx, xs.stop + dx)
    out[zs, ys, xs] = x[zt, yt, xt]
    return out


def conv3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[v, co] = b[co] + sum_{t, ci} W[co, t, ci] x[v + o_t, ci] (zero padding)."""
    y = np.broadcast_to(b, x.shape[:3] + (W.shape[0],)).astype(np.float64).copy()
    for t, (dz, dy, dx) in enumerate(_offsets3()):
        y += _shifted(x, dz, dy, dx) @ W[:, t, :].T
    return y


def conv3_dgrad(gy: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of conv3 in x: gx[u, ci] = sum_{t, co} W[co, t, ci] gy[u - o_t, co]."""
    gx = np.zeros(gy.shape[:3] + (W.shape[2],))
    for t, (dz, dy, dx) in enumerate(_offsets3()):
        gx += _shifted(gy, -dz, -dy, -dx) @ W[:, t, :]
    return gx


def conv3_wgrad(x: np.ndarray, gy: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """dL/dW[co, t, ci] = sum_v gy[v, co] x[v + o_t, ci]; dL/db = sum_v gy[v]."""
    co, ci = gy.shape[3], x.shape[3]
    gW = np.zeros((co, 27, ci))
    g2 = gy.reshape(-1, co)
    for t, (dz, dy, dx) in enumerate(_offsets3()):
        gW[:, t, :] = g2.T @ _shifted(x, dz, dy, dx).reshape(-1, ci)
    return gW, g2.sum(axis=0)


def _parities():
    return [(tz, ty, tx) for tz in (0, 1) for ty in (0, 1) for tx in (0, 1)]


def down2(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[V, co] = b[co] + sum_{t, ci} W[co, t, ci] x[2V + t, ci]."""
    Z, Y, X = (s // 2 for s in x.shape[:3])
    y = np.broadcast_to(b, (Z, Y, X, W.shape[0])).astype(np.float64).copy()
    for t, (tz, ty, tx) in enumerate(_parities()):
        y += x[tz::2, ty::2, tx::2] @ W[:, t, :].T
    return y


def down2_dgrad(gy: np.ndarray, W: np.ndarray) -> np.ndarray:
    Z, Y, X = gy.shape[:3]
    gx = np.zeros((2 * Z, 2 * Y, 2 * X, W.shape[2]))
    for t, (tz, ty, tx) in enumerate(_parities()):
        gx[tz::2, ty::2, tx::2] = gy @ W[:, t, :]
    return gx


def down2_wgrad(x: np.ndarray, gy: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    co, ci = gy.shape[3], x.shape[3]
    g2 = gy.reshape(-1, co)
    gW = np.zeros((co, 8, ci))
    for t, (tz, ty, tx) in enumerate(_parities()):
        gW[:, t, :] = g2.T @ x[tz::2, ty::2, tx::2].reshape(-1, ci)
    return gW, g2.sum(axis=0)


def up2(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[2V + t, co] = b[co] + sum_ci W[co, t, ci] x[V, ci]."""
    Z, Y, X = x.shape[:3]
    y = np.zeros((2 * Z, 2 * Y, 2 * X, W.shape[0]))
    for t, (tz, ty, tx) in enumerate(_parities()):
        y[tz::2, ty::2, tx::2] = x @ W[:, t, :].T + b
    return y


def up2_dgrad(gy: np.ndarray, W: np.ndarray) -> np.ndarray:
    gx = np.zeros(tuple(s // 2 for s in gy.shape[:3]) + (W.shape[2],))
    for t, (tz, ty, tx) in enumerate(_parities()):
        gx += gy[tz::2, ty::2, tx::2] @ W[:, t, :]
    return gx


def up2_wgrad(x: np.ndarray, gy: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    co, ci = gy.shape[3], x.shape[3]
    gW = np.zeros((co, 8, ci))
    x2 = x.reshape(-1, ci)
    for t, (tz, ty, tx) in enumerate(_parities()):
        gW[:, t, :] = gy[tz::2, ty::2, tx::2].reshape(-1, co).T @ x2
    return gW, gy.reshape(-1, co).sum(axis=0)


def head_features(a: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Input of the head: c0b's channels, then x at the 27 taps of the cell."""
    taps = [_shifted(x, dz, dy, dx) for dz, dy, dx in _offsets3()]
    return np.concatenate([a] + taps, axis=3)


_FWD = {"conv3": conv3, "down2": down2, "up2": up2}
_DGRAD = {"conv3": conv3_dgrad, "down2": down2_dgrad, "up2": up2_dgrad}
_WGRAD = {"conv3": conv3_wgrad, "down2": down2_wgrad, "up2": up2_wgrad}

# the layer graph: (layer, inputs); inputs name activations (concatenated
# in the order given); "x" is the scaled source
GRAPH = [
    ("e0a", ["x"]), ("e0b", ["e0a"]), ("d0", ["e0b"]),
    ("e1a", ["d0"]), ("e1b", ["e1a"]), ("d1", ["e1b"]),
    ("e2a", ["d1"]), ("e2b", ["e2a"]), ("d2", ["e2b"]),
    ("b3a", ["d2"]), ("b3b", ["b3a"]), ("u2", ["b3b"]),
    ("c2a", ["u2", "e2b"]), ("c2b", ["c2a"]), ("u1", ["c2b"]),
    ("c1a", ["u1", "e1b"]), ("c1b", ["c1a"]), ("u0", ["c1b"]),
    ("c0a", ["u0", "e0b"]), ("c0b", ["c0a"]), ("head", ["c0b"]),
]
KIND = {n: k for n, k, _, _ in LAYERS}


def check_shape(shape: Tuple[int, int, int]) -> None:
    if any(s % 8 != 0 or s < 8 for s in shape):
        raise ValueError("every grid axis must be a positive multiple of 8 (three 2x coarsenings)")


def forward(theta: np.ndarray, x: np.ndarray, rnd=None) -> Tuple[np.ndarray, Dict[str, np.ndarray]]:
    """Network output y [z,y,x,3] for the scaled input x [z,y,x] (or [z,y,x,1]);
    returns (y, activations).

    ``rnd`` (optional) rounds every stored tensor — the scaled input and
    each layer's activation — to a storage format (e.g. ``bf16_round``),
    the arithmetic itself staying FP64; None keeps everything in FP64."""
    check_shape(x.shape[:3])
    p = unflatten(theta)
    keep = rnd if rnd is not None else (lambda a: a)
    x1 = x.reshape(x.shape[:3] + (1,)).astype(np.float64)
    acts = {"x": keep(x1), "x_head": x1}
    for name, ins in GRAPH:
        inp = np.concatenate([acts[i] for i in ins], axis=3) if len(ins) > 1 else acts[ins[0]]
        W, b = p[name]
        if KIND[name] == "head":
            acts["head_in"] = head_features(inp, acts["x_head"])
            acts[name] = acts["head_in"] @ W.T + b
        else:
            acts[name] = keep(np.maximum(_FWD[KIND[name]](inp, W, b), 0.0))
    return acts["head"], acts


def loss_and_grad(theta: np.ndarray, x: np.ndarray, target: np.ndarray,
                  want_dx: bool = False, rnd=None):
    """MSE loss L = mean over cells and the 3 channels of (y - target)^2, and
    dL/dtheta (flat, same layout as theta) by reverse-mode differentiation.
    With want_dx also dL/dx.

    ``rnd`` (optional, see ``forward``) also rounds every stored gradient of
    a layer output: each consumer's contribution is masked by the layer's
    ReLU and rounded, and a second contribution is added to the stored
    first one and the sum rounded again."""
    y, acts = forward(theta, x, rnd)
    p = unflatten(theta)
    diff = y - target
    loss = float(np.mean(diff * diff))
    g_act: Dict[str, np.ndarray] = {"head": 2.0 * diff / diff.size}
    grads: Dict[str, Tuple[np.ndarray, np.ndarray]] = {}
    for name, ins in reversed(GRAPH):
        g = g_act.pop(name)
        inp = np.concatenate([acts[i] for i in ins], axis=3) if len(ins) > 1 else acts[ins[0]]
        W, _ = p[name]
        kind = KIND[name]
        if kind == "head":
            hin = acts["head_in"]
            grads[name] = (g.reshape(-1, 3).T @ hin.reshape(-1, hin.shape[3]), g.reshape(-1, 3).sum(axis=0))
            c16 = inp.shape[3]
            gin = g @ W[:, :c16]
            # the direct path: x at tap t of cell v feeds y(v)
            gx = np.zeros(acts["x"].shape)
            for t, (dz, dy, dx) in enumerate(_offsets3()):
                gx += _shifted(g @ W[:, c16 + t:c16 + t + 1], -dz, -dy, -dx)
            g_act["x"] = g_act["x"] + gx if "x" in g_act else gx
        else:
            g = g * (acts[name] > 0.0)   # through the ReLU of this layer
            grads[name] = _WGRAD[kind](inp, g)
            gin = _DGRAD[kind](g, W)
        c0 = 0
        for i in ins:
            c = acts[i].shape[3]
            part = gin[..., c0:c0 + c]
            c0 += c
            if rnd is not None and i != "x":
                part = rnd(part * (acts[i] > 0.0))
                g_act[i] = rnd(g_act[i] + part) if i in g_act else part
            else:
                g_act[i] = g_act[i] + part if i in g_act else part
    gx = g_act.get("x")
    flat = flatten(grads)
    return (loss, flat, gx) if want_dx else (loss, flat)


def adam_step(theta: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, step: int,
              lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1); step counts from 1.
    Returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def scaled_input(s: np.ndarray) -> Tuple[np.ndarray, float]:
    """x = s / max|s| and the scale (1 for an all-zero source)."""
    m = float(np.max(np.abs(s)))
    m = m if m > 0 else 1.0
    return s / m, m


def predict(theta: np.ndarray, s: np.ndarray, scales, kappa2) -> List[np.ndarray]:
    """Initial guesses Psi_i = max|s| * scale_i * y_i / kappa_i^2, [z][y][x] each."""
    x, m = scaled_input(s)
    y, _ = forward(theta, x)
    return [m * scales[i] * y[..., i] / kappa2[i] for i in range(3)]


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP64 values to the nearest bfloat16 (ties to even), via FP32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
