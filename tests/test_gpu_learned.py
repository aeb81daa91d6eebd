"""GPU parity of the learned initial guess against the FP64 network oracle,
through the mgl_* C ABI.

Per-kernel checks feed the oracle the GPU's own bfloat16 tensors (the
inputs of one layer) so that the only differences are FP32 accumulation
order and the final rounding to bfloat16: outputs agree to one bfloat16
unit in the last place (2^-7 relative; a sum that lands next to a rounding
boundary may round the other way) plus 1e-5 of the layer's largest value;
weight gradients and the prediction entry by entry within the FP32
summation bound of their terms.  End to end the gradients agree to 2e-2
relative per layer with the FP64 oracle run with the same bfloat16 storage
rounding (activations and activation gradients), and the prediction with
the plain FP64 oracle to 2e-2."""
import numpy as np
import pytest

from oracle import nn_oracle as nn
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1809_08857_amd import learned as L  # noqa: E402
from paper_1809_08857_amd import mg  # noqa: E402

ULP = 2.0 ** -7
GRAPH = dict(nn.GRAPH)
KIND = nn.KIND
NAMES = [n for n, _ in nn.GRAPH]


def _params(seed):
    rng = np.random.default_rng(seed)
    th = nn.init_params(seed)
    off = 0
    for _, ws, bs in nn.layer_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        th[off + nw:off + nw + nb] = 0.05 * rng.standard_normal(nb)
        off += nw + nb
    return nn.bf16_round(th)


def _source(shape, seed):
    rng = np.random.default_rng(seed)
    s = np.exp(0.5 * rng.standard_normal(shape)) * (rng.random(shape) < 0.5)
    s[shape[0] // 2, shape[1] // 2, shape[2] // 2] = 40.0
    return s


def _layer_ref(name, p, acts_in):
    W, b = p[name]
    inp = np.concatenate(acts_in, axis=3) if len(acts_in) > 1 else acts_in[0]
    Wb = nn.bf16_round(W)
    if KIND[name] == "conv3":
        y = nn.conv3(inp, Wb, b)
    elif KIND[name] == "down2":
        y = nn.down2(inp, Wb, b)
    else:
        y = nn.up2(inp, Wb, b)
    return np.maximum(y, 0.0)


def _gpu_acts(net):
    acts = {"x": L.mgl_read_tensor(net, 0, -1)[..., :1].astype(np.float64)}
    for i, n in enumerate(NAMES[:-1]):
        acts[n] = L.mgl_read_tensor(net, 0, i).astype(np.float64)
    return acts


def _close_bf16(got, ref, what):
    tol = ULP * np.abs(ref) + 1e-5 * max(np.abs(ref).max(), 1e-30)
    bad = np.abs(got - ref) > tol
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} off, worst {np.abs(got - ref).max():.3e}"


def _run_case(shape, pseed, sseed, tseed):
    theta = _params(pseed)
    s = _source(shape, sseed)
    rng = np.random.default_rng(tseed)
    target = rng.standard_normal(shape + (3,)) * 0.1
    net = L.mgl_create(shape[2], shape[1], shape[0])
    L.mgl_set_params(net, theta.astype(np.float32))
    sd = dev(s)
    td = torch.from_numpy(target.astype(np.float32)).cuda()
    loss = L.mgl_train_step(net, [sd], [td])
    return dict(theta=theta, s=s, target=target, loss=loss, acts=_gpu_acts(net),
                gacts={n: L.mgl_read_tensor(net, 1, i).astype(np.float64) for i, n in enumerate(NAMES[:-1])},
                grads=L.mgl_get_grads(net).astype(np.float64), net=net)


@pytest.fixture(scope="module")
def case():
    """One forward + backward (gradients only) on a ragged 16x8x24 grid
    (levels 16x8x24 .. 2x1x3: small tiles, partial tiles on every axis)."""
    out = _run_case((24, 8, 16), 11, 3, 4)
    yield out
    L.mgl_destroy(out["net"])


@pytest.fixture(scope="module")
def case_big():
    """128x64x32: the finest level takes the large-tile path."""
    out = _run_case((32, 64, 128), 12, 5, 6)
    yield out
    L.mgl_destroy(out["net"])


BIG_LAYERS = ["e0a", "e0b", "d0", "u0", "c0a", "c0b"]


@pytest.fixture(scope="module")
def case_ragged():
    """56x40x24: x and y are not multiples of the 16-cell convolution
    tiles on any level, the 64-channel layers run on 14x10x6 and 7x5x3, and
    the head's 64-wide tile is partial."""
    out = _run_case((24, 40, 56), 13, 7, 8)
    yield out
    L.mgl_destroy(out["net"])


@pytest.mark.parametrize("name", NAMES[:-1])
def test_forward_layer_ragged(case_ragged, name):
    test_forward_layer(case_ragged, name)


@pytest.mark.parametrize("name", NAMES[:-2])
def test_input_gradient_ragged(case_ragged, name):
    test_input_gradient(case_ragged, name)


@pytest.mark.parametrize("name", NAMES)
def test_weight_gradient_ragged(case_ragged, name):
    test_weight_gradient(case_ragged, name)


def test_prediction_ragged(case_ragged):
    test_prediction_matches_oracle(case_ragged)


@pytest.mark.parametrize("name", BIG_LAYERS)
def test_forward_layer_large_tiles(case_big, name):
    test_forward_layer(case_big, name)


@pytest.mark.parametrize("name", ["e0a", "e0b", "u0", "c0a"])
def test_input_gradient_large_tiles(case_big, name):
    test_input_gradient(case_big, name)


@pytest.mark.parametrize("name", ["e0a", "e0b", "c0a", "c0b", "head"])
def test_weight_gradient_large_tiles(case_big, name):
    test_weight_gradient(case_big, name)


def test_input_scaling(case):
    x = case["acts"]["x"][..., 0]
    s = case["s"]
    assert np.array_equal(x, nn.bf16_round(s / np.abs(s).max()))


@pytest.mark.parametrize("name", NAMES[:-1])
def test_forward_layer(case, name):
    p = nn.unflatten(case["theta"])
    ins = [case["acts"][i] for i in GRAPH[name]]
    ref = nn.bf16_round(_layer_ref(name, p, ins))
    _close_bf16(case["acts"][name], ref, name)


def _head_in(case):
    """The head's features as the kernel forms them: c0b's bfloat16 channels
    and x = s / max|s| in FP32 at the 27 taps."""
    s = case["s"]
    x = (s / np.abs(s).max()).astype(np.float32).astype(np.float64)[..., None]
    return nn.head_features(case["acts"]["c0b"], x)


def test_head_gradient(case):
    p = nn.unflatten(case["theta"])
    W, b = p["head"]
    a = case["acts"]["c0b"]
    y = _head_in(case) @ W.T + b
    gy = 2.0 * (y - case["target"].astype(np.float32)) / y.size
    ga = (gy @ W[:, :16]) * (a > 0)
    _close_bf16(case["gacts"]["c0b"], nn.bf16_round(ga), "head input gradient")
    loss = float(np.mean((y - case["target"].astype(np.float32)) ** 2))
    assert abs(case["loss"] - loss) <= 1e-5 * loss


def _consumers(name):
    return [(n, ins) for n, ins in nn.GRAPH if name in ins and n != "head"]


@pytest.mark.parametrize("name", NAMES[:-2])
def test_input_gradient(case, name):
    """Gradient of a layer's pre-activation output = sum over its consumers
    of their data gradient, masked by the layer's ReLU."""
    p = nn.unflatten(case["theta"])
    tot, mag = 0.0, 0.0
    for n, ins in _consumers(name):
        W, _ = p[n]
        g = case["gacts"][n]
        dg = {"conv3": nn.conv3_dgrad, "down2": nn.down2_dgrad, "up2": nn.up2_dgrad}[KIND[n]]
        gin = dg(g, nn.bf16_round(W))
        c0 = 0
        for i in ins:
            c = case["acts"][i].shape[3]
            if i == name:
                part = nn.bf16_round(gin[..., c0:c0 + c] * (case["acts"][name] > 0))
                tot = tot + part
                mag = mag + np.abs(part)
            c0 += c
    got = case["gacts"][name]
    n_parts = len(_consumers(name))
    tol = n_parts * ULP * mag + 1e-5 * max(np.abs(tot).max(), 1e-30)
    assert np.all(np.abs(got - tot) <= tol), (name, np.abs(got - tot).max())


U32 = 2.0 ** -24


@pytest.mark.parametrize("name", NAMES)
def test_weight_gradient(case, name):
    """FP32 accumulation of the GPU's own bfloat16 tensors vs FP64, entry by
    entry.  Every term x * g is a product of two bfloat16 values, exact in
    FP32, so the only error is the summation over the n cells of the layer:
    at most n * 2^-24 times the sum of the terms' magnitudes (the bound of
    any summation order), which the oracle evaluates with |x| and |g|.  The
    head's gradient dL/dy is formed from the FP32 output y (43 fused
    multiply-adds), whose error bound enters the same way."""
    shapes = {n: (w, b) for n, w, b in nn.layer_shapes()}
    off = 0
    for n, ws, bs in nn.layer_shapes():
        if n == name:
            break
        off += int(np.prod(ws)) + int(np.prod(bs))
    ws, bs = shapes[name]
    nw = int(np.prod(ws))
    gW = case["grads"][off:off + nw].reshape(ws)
    gb = case["grads"][off + nw:off + nw + bs[0]]
    ins = [case["acts"][i] for i in GRAPH[name]]
    inp = np.concatenate(ins, axis=3) if len(ins) > 1 else ins[0]
    if name == "head":
        p = nn.unflatten(case["theta"])
        W, b = p["head"]
        hin = _head_in(case)
        t = case["target"].astype(np.float32).astype(np.float64)
        y = hin @ W.T + b
        g = 2.0 * (y - t) / y.size
        h2 = hin.reshape(-1, hin.shape[3])
        habs = np.abs(h2)
        rW, rb = g.reshape(-1, 3).T @ h2, g.reshape(-1, 3).sum(axis=0)
        n = h2.shape[0]
        yabs = np.abs(hin) @ np.abs(W).T + np.abs(b)
        dg = (2.0 / y.size) * (45 * U32 * yabs + U32 * np.abs(t))  # bound on |g_gpu - g|
        gabs = np.abs(g).reshape(-1, 3)
        tolW = n * U32 * (gabs.T @ habs) + dg.reshape(-1, 3).T @ habs
        tolb = n * U32 * gabs.sum(axis=0) + dg.reshape(-1, 3).sum(axis=0)
    else:
        g = case["gacts"][name]
        wg = {"conv3": nn.conv3_wgrad, "down2": nn.down2_wgrad, "up2": nn.up2_wgrad}[KIND[name]]
        rW, rb = wg(inp, g)
        mW, mb = wg(np.abs(inp), np.abs(g))
        n = g.shape[0] * g.shape[1] * g.shape[2]
        tolW, tolb = n * U32 * mW, n * U32 * mb
    badW = np.abs(gW - rW) > tolW + 1e-30
    badb = np.abs(gb - rb) > tolb + 1e-30
    assert not badW.any(), (name, int(badW.sum()), float(np.abs(gW - rW).max()))
    assert not badb.any(), (name, int(badb.sum()), float(np.abs(gb - rb).max()))


def _per_layer_rel(a, b):
    out, off = {}, 0
    for n, ws, bs in nn.layer_shapes():
        k = int(np.prod(ws)) + int(np.prod(bs))
        out[n] = np.linalg.norm(a[off:off + k] - b[off:off + k]) / np.linalg.norm(b[off:off + k])
        off += k
    return out


def test_gradients_end_to_end(case):
    """The whole backward pass against the FP64 oracle run with the kernels'
    bfloat16 storage rounding.  Deep layers of a randomly initialised net
    sum many cancelling terms across ReLU kinks, so their gradients move by
    several per cent when the values before each rounding change at FP32
    level; the bar per layer is 2e-2 or three times that sensitivity of the
    oracle itself (measured here by a 3e-7 relative perturbation before each
    rounding), whichever is larger.  Against the plain FP64 oracle (no
    storage rounding) the gradient as a whole stays within 1e-1."""
    s = case["s"]
    x, _ = nn.scaled_input(s)
    t = case["target"].astype(np.float32).astype(np.float64)
    _, g_bf = nn.loss_and_grad(case["theta"], x, t, rnd=nn.bf16_round)
    wig = lambda a: nn.bf16_round(a * (1 + 3e-7 * np.sin(np.arange(a.size).reshape(a.shape))))
    _, g_wig = nn.loss_and_grad(case["theta"], x, t, rnd=wig)
    _, g64 = nn.loss_and_grad(case["theta"], x, t)
    e_bf = _per_layer_rel(case["grads"], g_bf)
    sens = _per_layer_rel(g_wig, g_bf)
    print("vs bf16-storage oracle", {k: f"{v:.1e}" for k, v in e_bf.items()})
    print("oracle sensitivity", {k: f"{v:.1e}" for k, v in sens.items()})
    bad = {k: (e_bf[k], sens[k]) for k in e_bf if e_bf[k] > max(2e-2, 3 * sens[k])}
    assert not bad, bad
    assert np.linalg.norm(case["grads"] - g64) <= 0.1 * np.linalg.norm(g64)


def test_prediction_matches_oracle(case):
    """Entry by entry: the prediction is the head (FP32, 43 fused
    multiply-adds) on the GPU's own bfloat16 features of c0b and the FP32
    input taps, times max|s| * scale_i / kappa_i^2 in FP64; its error is at
    most 45 * 2^-24 times the sum of the magnitudes of the head's terms.  End
    to end (the whole bfloat16 network) it stays within 2e-2 of the plain
    FP64 oracle in relative L2."""
    shape = case["s"].shape
    net = case["net"]
    scales = (0.5, 2.0, 1.5)
    L.mgl_set_scales(net, scales)
    k2 = (3.0, 50.0, 700.0)
    gs = [torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(3)]
    L.mgl_predict(net, dev(case["s"]), k2, gs)
    L.mgl_set_scales(net, (1.0, 1.0, 1.0))
    p = nn.unflatten(case["theta"])
    W, b = p["head"]
    hin = _head_in(case)
    y = hin @ W.T + b
    yabs = np.abs(hin) @ np.abs(W).T + np.abs(b)
    m = float(np.abs(case["s"]).max())
    ref_e2e = nn.predict(case["theta"], case["s"], scales, k2)
    for i, (g, r) in enumerate(zip(gs, ref_e2e)):
        g = g.cpu().numpy()
        c = m * scales[i] / k2[i]
        ref = c * y[..., i]
        tol = abs(c) * 45 * U32 * yabs[..., i] + 1e-15 * np.abs(ref)
        bad = np.abs(g - ref) > tol
        assert not bad.any(), (i, int(bad.sum()), float(np.abs(g - ref).max()))
        assert np.linalg.norm(g - r) <= 2e-2 * np.linalg.norm(r)


def test_adam_step_matches_oracle():
    shape = (8, 8, 16)
    theta = _params(2)
    s = _source(shape, 5)
    t = np.random.default_rng(6).standard_normal(shape + (3,)).astype(np.float32)
    net = L.mgl_create(16, 8, 8)
    try:
        L.mgl_set_params(net, theta.astype(np.float32))
        sd, td = dev(s), torch.from_numpy(t).cuda()
        L.mgl_train_step(net, [sd, sd], [td, td])          # gradients only, 2 samples
        g = L.mgl_get_grads(net).astype(np.float64)
        L.mgl_set_params(net, theta.astype(np.float32))     # resets Adam
        L.mgl_train_step(net, [sd, sd], [td, td], lr=1e-3)
        got = L.mgl_get_params(net).astype(np.float64)
        ref, _, _ = nn.adam_step(theta, np.zeros_like(theta), np.zeros_like(theta), g / 2, 1, 1e-3)
        assert np.abs(got - ref).max() <= 1e-6 + 1e-6 * np.abs(ref).max()
        # summed gradient of two identical samples is twice one sample's
        L.mgl_set_params(net, theta.astype(np.float32))
        L.mgl_train_step(net, [sd], [td])
        g1 = L.mgl_get_grads(net).astype(np.float64)
        assert np.allclose(g, 2 * g1, rtol=1e-5, atol=1e-7 * np.abs(g).max())
    finally:
        L.mgl_destroy(net)


def test_training_lowers_the_loss():
    shape = (16, 16, 16)
    s = _source(shape, 7)
    x = s / np.abs(s).max()
    t = np.stack([x, 0.5 * x, 0.25 + 0.0 * x], axis=3).astype(np.float32)  # learnable: local maps of x
    net = L.mgl_create(16, 16, 16)
    try:
        L.mgl_init_params(net, 3)
        sd, td = dev(s), torch.from_numpy(t).cuda()
        l0 = L.mgl_eval_loss(net, sd, td)
        for _ in range(30):
            L.mgl_train_step(net, [sd], [td], lr=3e-3)
        l1 = L.mgl_eval_loss(net, sd, td)
        print("loss", l0, "->", l1)
        assert l1 < 0.5 * l0
    finally:
        L.mgl_destroy(net)


def test_save_load_roundtrip(tmp_path):
    net = L.mgl_create(8, 8, 8)
    net2 = L.mgl_create(16, 8, 8)
    try:
        L.mgl_init_params(net, 9)
        L.mgl_set_scales(net, (0.25, 0.5, 4.0))
        path = str(tmp_path / "w.mglw")
        L.mgl_save(net, path)
        L.mgl_load(net2, path)
        assert np.array_equal(L.mgl_get_params(net), L.mgl_get_params(net2))
        assert L.mgl_get_scales(net2) == (0.25, 0.5, 4.0)
        with open(path, "r+b") as f:
            f.write(b"XXXX")
        with pytest.raises(mg.MgError):
            L.mgl_load(net2, path)
    finally:
        L.mgl_destroy(net)
        L.mgl_destroy(net2)


def test_invalid_arguments():
    net = L.mgl_create(8, 8, 8)
    try:
        with pytest.raises(mg.MgError):
            L.mgl_set_params(net, np.zeros(5, np.float32))
        bad = np.zeros(L.mgl_num_params(), np.float32)
        bad[7] = np.nan
        with pytest.raises(mg.MgError):
            L.mgl_set_params(net, bad)
        with pytest.raises(mg.MgError):
            L.mgl_set_scales(net, (1.0, 0.0, 1.0))
        s = dev(np.ones((8, 8, 8)))
        gs = [torch.empty((8, 8, 8), dtype=torch.float64, device="cuda") for _ in range(3)]
        with pytest.raises(mg.MgError):
            L.mgl_predict(net, s, (1.0, -1.0, 1.0), gs)
    finally:
        L.mgl_destroy(net)
