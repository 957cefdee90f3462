"""The FP64 reference network (oracle side) against finite differences and
its own invariants; and the packing helpers of the binding."""
import numpy as np

from oracle import mlp_ref as R


def test_reference_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    params = R.init(rng, 16, width=8, depth=4)
    params = [(W, rng.normal(0, 0.1, b.shape)) for W, b in params]
    x = rng.normal(size=(32, 16))
    t = rng.normal(size=32) * 0.1
    loss, grads = R.loss_and_grads(params, x, t)
    h = 1e-6
    for li in range(len(params)):
        W, b = params[li]
        for (i, j) in [(0, 0), (W.shape[0] - 1, W.shape[1] - 1), (3 % W.shape[0], 0)]:
            Wp = W.copy(); Wp[i, j] += h
            Wm = W.copy(); Wm[i, j] -= h
            pp = list(params); pp[li] = (Wp, b)
            pm = list(params); pm[li] = (Wm, b)
            fd = (R.loss_and_grads(pp, x, t)[0] - R.loss_and_grads(pm, x, t)[0]) / (2 * h)
            assert abs(fd - grads[li][0][i, j]) < 1e-7 + 1e-6 * abs(fd)
        bp = b.copy(); bp[0] += h
        bm = b.copy(); bm[0] -= h
        pp = list(params); pp[li] = (W, bp)
        pm = list(params); pm[li] = (W, bm)
        fd = (R.loss_and_grads(pp, x, t)[0] - R.loss_and_grads(pm, x, t)[0]) / (2 * h)
        assert abs(fd - grads[li][1][0]) < 1e-7 + 1e-6 * abs(fd)


def test_gelu_tanh_form_properties():
    z = np.linspace(-6, 6, 1001)
    g = R.gelu(z)
    assert abs(R.gelu(np.array([0.0]))[0]) == 0.0
    assert np.all(np.abs(g[z > 5] - z[z > 5]) < 1e-6) and np.all(np.abs(g[z < -5]) < 1e-6)
    h = 1e-6
    fd = (R.gelu(z + h) - R.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - R.gelu_grad(z))) < 1e-8


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(1)
    params = R.init(rng, 4, width=4, depth=1)
    grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in params]
    new = R.adam_step(params, grads, R.adam_state(params), lr=1e-3, step=1)
    for (W, b), (W2, b2), (gW, gb) in zip(params, new, grads):
        assert np.allclose(W - W2, 1e-3 * np.sign(gW), atol=1e-8)


def test_parameter_count_and_packing():
    from paper_2410_05408_amd import gl
    rng = np.random.default_rng(2)
    params = R.init(rng, 16)
    assert R.n_params(params) == 16 * 256 + 256 + 3 * (256 * 256 + 256) + 256 + 1
    packed = gl.pack_params(params)
    assert packed.size == gl.gl_mlp_num_params()
    back = gl.unpack_params(packed)
    for (W, b), (W2, b2) in zip(params, back):
        assert np.allclose(W, W2, rtol=1e-7) and np.allclose(b, b2)


# ---------------------------------------------------------------- pins of the reference network
def _hand_network(width=256):
    """A network whose every pre-activation is 0 or at least 10 in magnitude:
    there the tanh-form GELU is exactly max(z, 0) in FP64 (tanh of an argument
    above 19 rounds to 1), so its output can be added up by hand."""
    dims = [16] + [width] * 4 + [1]
    P = [(np.zeros((a, b)), np.zeros(b)) for a, b in zip(dims[:-1], dims[1:])]
    (W0, b0), (W1, b1), (W2, b2), (W3, b3), (w4, b4) = P
    W0[0, 0], b0[0] = 2.0, 10.0     # unit 0 of layer 0: 2 x0 + 10
    W0[1, 1], b0[1] = 1.0, -30.0    # unit 1: x1 - 30
    W0[2, 2] = 3.0                  # unit 2: 3 x2
    W1[0, 5] = W1[2, 5] = 1.0       # layer 1, unit 5: h0 + h2
    W1[1, 7], b1[7] = 100.0, 10.0   # unit 7: 100 h1 + 10
    W1[0, 9] = -1.0                 # unit 9: -h0
    W2[5, 3], W2[7, 3] = 0.5, 1.0   # layer 2, unit 3: h5 / 2 + h7
    W2[9, 4], b2[4] = 1000.0, 11.0  # unit 4: 1000 h9 + 11
    W3[3, 0], W3[4, 0] = 1.0, -1.0  # layer 3, unit 0: h3 - h4
    W3[3, 1] = -1.0                 # unit 1: -h3
    w4[0, 0], w4[1, 0], b4[0] = 2.0, 5.0, -30.0  # output (linear): 2 h0 + 5 h1 - 30
    return P


def test_forward_on_a_hand_added_network():
    x = np.zeros((2, 16))
    x[0, :3] = [1.0, 5.0, 4.0]
    x[1, :3] = [-10.0, 45.0, 4.0]
    y, _ = R.forward(_hand_network(), x)
    # row 0: layer 0 -> (12, 0, 12); layer 1 -> h5 = 24, h7 = 10, h9 = 0;
    #        layer 2 -> h3 = 22, h4 = 11; layer 3 -> (11, 0); out 22 - 30
    # row 1: layer 0 -> (0, 15, 12); layer 1 -> h5 = 12, h7 = 1510, h9 = 0;
    #        layer 2 -> h3 = 1516, h4 = 11; layer 3 -> (1505, 0); out 3010 - 30
    assert y[0] == -8.0 and y[1] == 2980.0


def _torch_net(params):
    import torch
    layers = []
    for i, (W, b) in enumerate(params):
        lin = torch.nn.Linear(W.shape[0], W.shape[1], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W.T.copy()))  # torch keeps [out, in]
            lin.bias.copy_(torch.from_numpy(b))
        layers.append(lin)
        if i + 1 < len(params):
            layers.append(torch.nn.GELU(approximate="tanh"))
    return torch.nn.Sequential(*layers)


def test_forward_and_gradients_match_torch_autograd():
    """The reference against an independent implementation: torch's own
    linear layers and tanh-form GELU in FP64, gradients by autograd."""
    import torch
    rng = np.random.default_rng(3)
    params = R.init(rng, 16, width=32, depth=4)
    params = [(W, rng.normal(0, 0.2, b.shape)) for W, b in params]
    x = rng.normal(size=(40, 16))
    t = rng.normal(size=40) * 0.3
    net = _torch_net(params)
    xt = torch.from_numpy(x)
    yt = net(xt)[:, 0]
    y, _ = R.forward(params, x)
    assert np.max(np.abs(y - yt.detach().numpy())) < 1e-13
    loss_t = torch.mean((yt - torch.from_numpy(t)) ** 2)
    loss_t.backward()
    loss, grads = R.loss_and_grads(params, x, t)
    assert abs(loss - loss_t.item()) < 1e-14
    lins = [m for m in net if isinstance(m, torch.nn.Linear)]
    for (gW, gb), lin in zip(grads, lins):
        assert np.max(np.abs(gW - lin.weight.grad.numpy().T)) < 1e-13 * max(1.0, np.abs(gW).max())
        assert np.max(np.abs(gb - lin.bias.grad.numpy())) < 1e-13 * max(1.0, np.abs(gb).max())


def test_adam_matches_torch_over_many_steps():
    """Twelve steps with changing gradients against torch.optim.Adam (same
    definition: Kingma & Ba's bias-corrected moments, eps outside the root)."""
    import torch
    rng = np.random.default_rng(4)
    params = R.init(rng, 6, width=5, depth=2)
    ref = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for W, b in params for a in (W, b)]
    opt = torch.optim.Adam(ref, lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    state = R.adam_state(params)
    for step in range(1, 13):
        grads = [(rng.normal(size=W.shape) * 10 ** rng.uniform(-3, 1), rng.normal(size=b.shape))
                 for W, b in params]
        params = R.adam_step(params, grads, state, lr=3e-3, step=step)
        for tp, g in zip(ref, [a for gw in grads for a in gw]):
            tp.grad = torch.from_numpy(np.array(g))
        opt.step()
    for (W, b), tW, tb in zip(params, ref[0::2], ref[1::2]):
        assert np.max(np.abs(W - tW.detach().numpy())) < 1e-14
        assert np.max(np.abs(b - tb.detach().numpy())) < 1e-14


def test_adam_closed_form_for_alternating_gradients():
    """With g_s = (-1)^s g the recurrences sum in closed form: the first
    moment is (1-b1) g (-1)^s (1 - (-b1)^s)/(1 + b1), the second (1 - b2^s) g^2,
    so the bias-corrected root is |g| and each update is
    lr (m_s / (1 - b1^s)) / (|g| + eps).  A wrong bias-correction exponent or
    swapped moment roles changes every step after the first."""
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 1e-2
    g = np.array([[0.5, -2.0], [1e-3, 7.0]])
    params = [(np.zeros((2, 2)), np.zeros(2))]
    state = R.adam_state(params)
    w = np.zeros((2, 2))
    for s in range(1, 21):
        gs = (-1.0) ** s * g
        params = R.adam_step(params, [(gs, np.zeros(2))], state, lr=lr, step=s, b1=b1, b2=b2, eps=eps)
        m = (1 - b1) * g * (-1.0) ** s * (1 - (-b1) ** s) / (1 + b1)
        w = w - lr * (m / (1 - b1 ** s)) / (np.abs(g) + eps)
        assert np.allclose(params[0][0], w, rtol=1e-12, atol=1e-16), s
