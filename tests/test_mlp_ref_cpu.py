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
