"""GPU: the BF16-MFMA surrogate network against the FP64 reference network."""
import sys

import numpy as np
import pytest

from oracle import mlp_ref as R

pytestmark = pytest.mark.gpu


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup(gpu_lib):
    import torch
    gl = gpu_lib
    rng = np.random.default_rng(7)
    params = R.init(rng, 16)
    params = [(W, rng.normal(0, 0.05, b.shape)) for W, b in params]
    net = gl.MLP(0, max_batch=1024)
    net.set_weights(gl.pack_params(params))
    x = rng.uniform(-1, 1, (1024, 16))
    x[:, 12:] = 0.0
    t = np.tanh(x[:, 0] * 2 + x[:, 1] * x[:, 2]) * 0.3
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    yield gl, net, params, x, t, xd, td
    net.close()


def test_weights_round_trip(setup):
    gl, net, params, *_ = setup
    assert np.array_equal(net.get_weights(), gl.pack_params(params))


def test_forward_matches_reference(setup):
    import torch
    gl, net, params, x, t, xd, td = setup
    say("case: BF16 MFMA forward vs FP64 reference, 1024 rows")
    y = net.forward(xd)
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    # the reference sees the same BF16-rounded inputs and weights
    xb = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    ref, _ = R.forward(params, xb)
    err = np.abs(y - ref)
    scale = np.abs(ref).max()
    say(f"  max |y - ref| {err.max():.3e}, scale {scale:.3e}, corr {np.corrcoef(y, ref)[0, 1]:.6f}")
    assert err.max() <= 2e-2 * scale
    assert np.corrcoef(y, ref)[0, 1] > 0.9999


def test_gradients_match_reference(setup):
    gl, net, params, x, t, xd, td = setup
    say("case: BF16 MFMA gradients vs FP64 reference")
    g, loss = net.grads(xd, td)
    import torch
    xb = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    ref_loss, ref_grads = R.loss_and_grads(params, xb, t.astype(np.float32).astype(np.float64))
    got = gl.unpack_params(g.astype(np.float64))
    say(f"  loss {loss:.6e} ref {ref_loss:.6e}")
    assert abs(loss - ref_loss) <= 2e-2 * ref_loss
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(got, ref_grads)):
        for a, r, name in ((gW, rW, "W"), (gb, rb, "b")):
            rel = np.linalg.norm(a - r) / np.linalg.norm(r)
            cos = float(np.dot(a.ravel(), r.ravel()) / (np.linalg.norm(a) * np.linalg.norm(r)))
            say(f"  layer {li} {name}: rel {rel:.2e} cos {cos:.6f}")
            # BF16 operands, FP32 accumulation: relative error per tensor below
            # 1e-2 and cosine similarity above 0.999
            assert rel < 1e-2 and cos > 0.999


def test_adam_matches_reference(gpu_lib):
    """Adam on the FP32 master weights: over several steps, each update of the
    GPU equals the reference recurrence (FP64) fed the same GPU gradient and
    the GPU's weights before the step, to 1e-6 relative on the weights."""
    import torch
    gl = gpu_lib
    say("case: Adam steps vs FP64 reference recurrence")
    rng = np.random.default_rng(13)
    params = R.init(rng, 16)
    params = [(W, rng.normal(0, 0.05, b.shape)) for W, b in params]
    net = gl.MLP(0, max_batch=512)
    net.set_weights(gl.pack_params(params))
    x = rng.uniform(-1, 1, (512, 16))
    t = np.cos(3 * x[:, 0]) * 0.2 + 0.1 * x[:, 1]
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    lr = 2e-3
    w_prev = net.get_weights().astype(np.float64)
    state = R.adam_state(gl.unpack_params(w_prev))
    try:
        for step in range(1, 9):
            g, _ = net.grads(xd, td)      # the gradient the step will use (deterministic)
            net.train_step(xd, td, lr)
            torch.cuda.synchronize()
            w_gpu = net.get_weights().astype(np.float64)
            ref = R.adam_step(gl.unpack_params(w_prev), gl.unpack_params(g.astype(np.float64)), state,
                              lr=lr, step=step)
            w_ref = np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in ref])
            d_gpu, d_ref = w_gpu - w_prev, w_ref - w_prev
            rel_w = np.max(np.abs(w_gpu - w_ref) / np.maximum(np.abs(w_ref), lr))
            rel_u = np.linalg.norm(d_gpu - d_ref) / np.linalg.norm(d_ref)
            say(f"  step {step}: max rel weight err {rel_w:.2e}, update rel err {rel_u:.2e}")
            assert rel_w <= 1e-6
            assert rel_u <= 1e-4
            w_prev = w_gpu
    finally:
        net.close()


def test_training_reduces_loss(gpu_lib):
    import torch
    gl = gpu_lib
    say("case: Adam training on a smooth target")
    rng = np.random.default_rng(3)
    net = gl.MLP(0, max_batch=4096)
    net.set_weights(gl.pack_params(R.init(rng, 16)))
    x = rng.uniform(-1, 1, (4096, 16))
    x[:, 8:] = 0
    t = np.sin(2 * x[:, 0]) * np.cos(x[:, 1]) * 0.5 + 0.1 * x[:, 2]
    xd = torch.tensor(x, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    _, l0 = net.grads(xd, td)
    for i in range(300):
        net.train_step(xd, td, 1e-3)
    torch.cuda.synchronize()
    _, l1 = net.grads(xd, td)
    say(f"  loss {l0:.3e} -> {l1:.3e}")
    assert l1 < 0.05 * l0
    net.close()
