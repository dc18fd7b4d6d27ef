"""GPU parity of the surrogate network (BF16 MFMA forward, backward, Adam) against
the FP64 reference of oracle/mlp.py, through the C ABI.

Two comparisons per quantity:
  * "same storage": the reference rounds the weights, the inputs, every hidden
    activation and every hidden pre-activation gradient to bfloat16 where the
    kernels store them.  What is left is FP32 (matrix-core) versus FP64
    accumulation and the bfloat16 rounding flips it causes: a sum of K terms
    carries a relative error of about sqrt(K) 2^-24 times its condition number
    (about sqrt(K) for random signs), i.e. about K 2^-24 = 3.4e-5 for K = 576,
    so about K 2^-16 ~ 1 % of the stored values sit close enough to a rounding
    boundary to round the other way (one bfloat16 ulp, at most 2^-7 relative).
    With ~15 such flips among the 1536 hidden values of a row, the output moves
    by about sqrt(15 / 512) 2^-7 ~ 1.3e-3 of its size (rms); the bounds are
    rms <= 3e-3 and max <= 1e-2 of the largest output, and 2e-2 on the relative
    norm of every gradient tensor.
  * "exact": the plain FP64 network on the FP32 parameters; this measures what
    bfloat16 storage costs (each stored value carries a relative error of at
    most 2^-9): outputs within 3e-2 of the largest, gradients pointing the same
    way (cosine >= 0.995).
A wrong index, operand or lane layout moves results by O(1) and fails both.
Batches of 300 rows span three 128-row tiles with a ragged 44-row tail.
"""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_09972_amd as sc
    sc.load()
    from paper_2112_09972_amd import mlp
    return torch, mlp


def rounded_params(p32):
    """Weights rounded to bfloat16, biases kept in float32, as float64."""
    ts = ref.unflatten(np.asarray(p32, dtype=np.float64))
    return ref.flatten([ref.round_bf16(t) if t.ndim == 2 else t for t in ts])


def make_batch(seed, n, scale=1.0):
    rng = np.random.default_rng(seed)
    w = ref.round_bf16(rng.standard_normal((n, 576)) * scale).astype(np.float32)   # exact in bfloat16
    t = (1.0 + 0.05 * rng.standard_normal((n, 3))).astype(np.float32)
    return w, t


OUT_SHIFT = np.ones(3, dtype=np.float32)
OUT_SCALE = np.full(3, 16.0, dtype=np.float32)   # powers of two: the normalisation is exact


def setup_net(torch, mlp, seed, max_batch=512):
    net = mlp.Network(max_batch=max_batch)
    p = mlp.init_params(seed)
    for b in ref.unflatten(np.arange(p.size))[1::2]:
        p[b] = 0.01                                  # small non-zero biases
    net.set_params(p)
    net.set_normalization(np.zeros(576), np.ones(576), OUT_SHIFT, OUT_SCALE)
    return net, p


def test_predict_matches_reference(env):
    torch, mlp = env
    net, p = setup_net(torch, mlp, 11)
    w, _ = make_batch(1, 300)
    out = net.predict(torch.from_numpy(w).cuda()).cpu().numpy().astype(np.float64)
    y_same, _ = ref.forward(rounded_params(p), w.astype(np.float64), round_hidden=ref.round_bf16)
    a_same = ref.denormalize_outputs(y_same, OUT_SHIFT, OUT_SCALE)
    y_exact, _ = ref.forward(p.astype(np.float64), w.astype(np.float64))
    a_exact = ref.denormalize_outputs(y_exact, OUT_SHIFT, OUT_SCALE)
    # compare the normalised outputs (the semi-axis offset of 1 would hide errors)
    d_same = (out - a_same) * OUT_SCALE
    e_same = np.max(np.abs(d_same)) / np.max(np.abs(y_same))
    r_same = np.sqrt(np.mean(d_same ** 2) / np.mean(y_same ** 2))
    e_exact = np.max(np.abs((out - a_exact) * OUT_SCALE)) / np.max(np.abs(y_exact))
    print("predict: same-storage max %.2e rms %.2e, exact max %.2e" % (e_same, r_same, e_exact))
    assert e_same <= 1e-2 and r_same <= 3e-3
    assert e_exact <= 3e-2
    # a batch of one row and an empty batch
    one = net.predict(torch.from_numpy(w[:1]).cuda()).cpu().numpy()
    assert np.array_equal(one, out[:1].astype(np.float32))
    assert net.predict(torch.empty((0, 576), dtype=torch.float32, device="cuda")).shape == (0, 3)


def test_predict_normalisation(env):
    torch, mlp = env
    net, p = setup_net(torch, mlp, 12)
    rng = np.random.default_rng(3)
    shift = rng.standard_normal(576).astype(np.float32) * 0.1
    scale = (1.0 + rng.random(576)).astype(np.float32)
    oshift = np.array([1.0, 0.9, 0.8], dtype=np.float32)
    oscale = np.array([10.0, 20.0, 30.0], dtype=np.float32)
    net.set_normalization(shift, scale, oshift, oscale)
    w = (rng.standard_normal((200, 576)) * 0.5).astype(np.float32)
    out = net.predict(torch.from_numpy(w).cuda()).cpu().numpy().astype(np.float64)
    x = ref.round_bf16((w.astype(np.float64) - shift) * scale)
    y, _ = ref.forward(rounded_params(p), x, round_hidden=ref.round_bf16)
    expect = ref.denormalize_outputs(y, oshift, oscale)
    err = np.max(np.abs((out - expect) * oscale)) / np.max(np.abs(y))
    print("normalised predict %.2e" % err)
    assert err <= 1e-2


def test_predict_one_launch_equals_layer_path(env):
    """Inference of 16-byte-aligned windows runs the four layers in one launch
    (k_forward, activations in LDS); any other alignment takes the layer-by-layer
    path (input kernel, three GEMMs, output kernel).  Both give the same bits, on a
    ragged batch and on one that fills the padded rows, with a non-trivial input
    and output normalisation."""
    torch, mlp = env
    net, p = setup_net(torch, mlp, 13, max_batch=1024)
    rng = np.random.default_rng(21)
    shift = rng.standard_normal(576).astype(np.float32) * 0.1
    scale = (1.0 + rng.random(576)).astype(np.float32)
    net.set_normalization(shift, scale, np.array([1.0, 0.9, 0.8], np.float32), np.array([10.0, 20.0, 30.0], np.float32))
    for n in (1000, 77, 1024):
        w = (rng.standard_normal((n, 576)) * 0.5).astype(np.float32)
        aligned = torch.from_numpy(w).cuda()
        buf = torch.zeros(n * 576 + 1, dtype=torch.float32, device="cuda")
        buf[1:].copy_(aligned.reshape(-1))
        shifted = buf[1:].view(n, 576)
        assert aligned.data_ptr() % 16 == 0 and shifted.data_ptr() % 16 != 0
        a = net.predict(aligned).cpu().numpy()
        b = net.predict(shifted).cpu().numpy()
        assert np.array_equal(a, b), (n, np.abs(a - b).max())


def check_grads(g_gpu, g_ref, rel, label):
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"], ref.unflatten(g_gpu), ref.unflatten(g_ref)):
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        print("%s %s: rel norm err %.2e" % (label, name, e))
        assert e <= rel, name


def test_gradients_match_reference(env):
    torch, mlp = env
    net, p = setup_net(torch, mlp, 13)
    w, t = make_batch(2, 300)
    loss = net.gradients(torch.from_numpy(w).cuda(), torch.from_numpy(t).cuda()).item()
    g = net.grads().astype(np.float64)
    tn = (t.astype(np.float64) - OUT_SHIFT) * OUT_SCALE
    l_same, g_same = ref.backward(rounded_params(p), w.astype(np.float64), tn, round_hidden=ref.round_bf16,
                                  round_grad=ref.round_bf16)
    l_exact, g_exact = ref.backward(p.astype(np.float64), w.astype(np.float64), tn)
    assert loss == pytest.approx(l_same, rel=5e-3)
    check_grads(g, g_same, 2e-2, "same-storage")
    cos = float(g @ g_exact / np.linalg.norm(g) / np.linalg.norm(g_exact))
    print("exact: loss %.6g vs %.6g, cosine %.6f" % (loss, l_exact, cos))
    assert cos >= 0.995
    assert loss == pytest.approx(l_exact, rel=5e-2)


def test_index_gather_and_bad_rows(env):
    torch, mlp = env
    net, p = setup_net(torch, mlp, 14)
    w, t = make_batch(4, 500)
    rng = np.random.default_rng(9)
    idx = rng.choice(500, size=200, replace=False).astype(np.int32)
    idx_bad = idx.copy()
    idx_bad[[3, 77]] = [-1, 500]          # out of range: skipped and counted
    dw, dt = torch.from_numpy(w).cuda(), torch.from_numpy(t).cuda()
    net.gradients(dw, dt, torch.from_numpy(idx).cuda())
    g_idx = net.grads()
    net.gradients(dw[torch.from_numpy(idx).long().cuda()].contiguous(), dt[torch.from_numpy(idx).long().cuda()].contiguous())
    g_copy = net.grads()
    assert np.array_equal(g_idx, g_copy)
    assert net.bad_rows() == 0
    net.gradients(dw, dt, torch.from_numpy(idx_bad).cuda())
    g_bad = net.grads().astype(np.float64)
    assert net.bad_rows() == 2
    keep = np.ones(200, bool)
    keep[[3, 77]] = False
    tn = (t[idx[keep]].astype(np.float64) - OUT_SHIFT) * OUT_SCALE
    _, g_ref = ref.backward(rounded_params(p), w[idx[keep]].astype(np.float64), tn, round_hidden=ref.round_bf16,
                            round_grad=ref.round_bf16)
    check_grads(g_bad, g_ref * (198.0 / 200.0), 2e-2, "skipped rows")


def test_adam_two_steps_match_reference(env):
    torch, mlp = env
    net, p = setup_net(torch, mlp, 15)
    w, t = make_batch(5, 256)
    dw, dt = torch.from_numpy(w).cuda(), torch.from_numpy(t).cuda()
    pr = p.astype(np.float64).copy()
    m = np.zeros_like(pr)
    v = np.zeros_like(pr)
    lr = 1e-3
    for step in (1, 2):
        net.gradients(dw, dt)
        g = net.grads().astype(np.float64)
        net.adam(lr)
        ref.adam_step(pr, g, m, v, step, lr)
        got = net.params().astype(np.float64)
        err = np.max(np.abs(got - pr))
        print("adam step %d: max |dp| err %.2e" % (step, err))
        assert err <= 1e-6 * max(1.0, np.max(np.abs(pr)))
    assert net.step_count == 2
    # the BF16 copies (incl. the transposed ones of the backward pass) follow the update
    w2, t2 = make_batch(6, 300)
    net.gradients(torch.from_numpy(w2).cuda(), torch.from_numpy(t2).cuda())
    got = net.params()
    tn = (t2.astype(np.float64) - OUT_SHIFT) * OUT_SCALE
    _, g_ref = ref.backward(rounded_params(got), w2.astype(np.float64), tn, round_hidden=ref.round_bf16,
                            round_grad=ref.round_bf16)
    check_grads(net.grads().astype(np.float64), g_ref, 2e-2, "after update")


def test_full_batch_8192_sampled_rows(env):
    """The inference batch of 8192 rows at the launch shape the benchmark uses;
    64 sampled rows against the reference."""
    torch, mlp = env
    net = mlp.Network(max_batch=8192)
    p = mlp.init_params(16)
    net.set_params(p)
    net.set_normalization(np.zeros(576), np.ones(576), OUT_SHIFT, OUT_SCALE)
    w, _ = make_batch(7, 8192)
    out = net.predict(torch.from_numpy(w).cuda()).cpu().numpy().astype(np.float64)
    rows = np.random.default_rng(8).choice(8192, 64, replace=False)
    y, _ = ref.forward(rounded_params(p), w[rows].astype(np.float64), round_hidden=ref.round_bf16)
    a = ref.denormalize_outputs(y, OUT_SHIFT, OUT_SCALE)
    err = np.max(np.abs((out[rows] - a) * OUT_SCALE)) / np.max(np.abs(y))
    print("8192 batch sampled rows %.2e" % err)
    assert err <= 1e-2


def test_training_reduces_loss(env):
    """Adam through the GPU kernels fits a smooth teacher function of the windows."""
    torch, mlp = env
    net, _ = setup_net(torch, mlp, 17, max_batch=256)
    rng = np.random.default_rng(10)
    w = rng.standard_normal((2048, 576)).astype(np.float32)
    B = rng.standard_normal((576, 3)) / np.sqrt(576)
    t = (1.0 + 0.05 * np.tanh(w.astype(np.float64) @ B)).astype(np.float32)
    dw, dt = torch.from_numpy(w).cuda(), torch.from_numpy(t).cuda()
    losses = []
    for it in range(400):
        idx = torch.from_numpy(rng.choice(2048, 256, replace=False).astype(np.int32)).cuda()
        losses.append(net.train_step(dw, dt, idx, lr=1e-3).item())
    print("loss %.4g -> %.4g" % (np.mean(losses[:10]), np.mean(losses[-10:])))
    assert np.mean(losses[-10:]) < 0.05 * np.mean(losses[:10])


def test_errors(env):
    torch, mlp = env
    import paper_2112_09972_amd as sc
    net, _ = setup_net(torch, mlp, 18, max_batch=100)
    w = torch.zeros((200, 576), dtype=torch.float32, device="cuda")
    o = torch.zeros((200, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(sc.SclbmError):
        mlp.sclmlp_predict(net.ctx, w, 101, o)
    with pytest.raises(sc.SclbmError):
        mlp.sclmlp_gradients(net.ctx, w, o, None, None, 0, 200)
    with pytest.raises(sc.SclbmError):
        net.adam(-1.0)
    with pytest.raises(sc.SclbmError):
        net.set_normalization(np.zeros(576), np.zeros(576), OUT_SHIFT, OUT_SCALE)
    bad = mlp.init_params(1)
    bad[5] = np.nan
    with pytest.raises(sc.SclbmError):
        net.set_params(bad)
