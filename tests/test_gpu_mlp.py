"""GPU parity of the learned-initial-guess kernels: the BF16 matrix-core GEMM (exact on
integer data), the network's forward pass, loss gradient and Adam step against the FP64
oracle with the same BF16 roundings, and a short training run."""
import numpy as np
import pytest

import bec_inputs as bi
import paper_2603_05194_amd as bec
from oracle import mlp as om
from tests.gpu_util import dev, host, torch_mod

pytestmark = pytest.mark.gpu


def bf16_bits(x):
    """int16 bit patterns of values that are exactly representable in BF16."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    assert np.array_equal(om.bf16_round(x32.astype(np.float64)), x32.astype(np.float64))
    return (x32.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def bf16_values(bits):
    return (np.asarray(bits).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K,splits,bias", [(200, 136, 72, 1, True), (200, 136, 72, 3, False),
                                               (256, 384, 1024, 4, True), (1, 8, 8, 1, False),
                                               (130, 129, 520, 2, True), (37, 512, 512, 1, True)])
def test_gemm_exact_on_integers(M, N, K, splits, bias):
    torch = torch_mod()
    rng = np.random.default_rng(M * 7919 + N * 31 + K)
    A = rng.integers(-8, 9, (M, K))
    B = rng.integers(-8, 9, (N, K))
    b = rng.integers(-50, 51, N).astype(np.float32)
    dA, dB = dev(bf16_bits(A)), dev(bf16_bits(B))
    C = torch.full((M, N), np.nan, dtype=torch.float32, device="cuda")
    part = torch.empty(splits * M * N, dtype=torch.float32, device="cuda")
    db = dev(b) if bias else None
    s = torch.cuda.current_stream().cuda_stream
    print(f"gemm M={M} N={N} K={K} splits={splits}", flush=True)
    bec.bec_gemm_bf16_nt(M, N, K, dA.data_ptr(), K, dB.data_ptr(), K, C.data_ptr(), N,
                         db.data_ptr() if bias else None, splits, part.data_ptr(), s)
    torch.cuda.synchronize()
    ref = A @ B.T + (b[None, :] if bias else 0)
    assert np.array_equal(host(C), ref.astype(np.float32))


DIMS = (6, 512, 32768)


def make_net(dims, seed):
    net = bec.Mlp(*dims)
    p = bi.mlp_init(dims, seed)
    rng = np.random.default_rng(seed + 1)
    offs = np.cumsum([0, dims[1] * dims[0], dims[1], dims[1] ** 2, dims[1], dims[2] * dims[1], dims[2]])
    for blk in (1, 3, 5):   # nonzero biases so that every term is exercised
        p[offs[blk]:offs[blk + 1]] = rng.uniform(-0.2, 0.2, offs[blk + 1] - offs[blk])
    net.load_params(p)
    return net, p.astype(np.float64)


def batch_inputs(B, dims, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (B, dims[0])).astype(np.float32)
    t = (0.1 * rng.standard_normal((B, dims[2]))).astype(np.float32)
    return x, t


def test_bf16_copies_and_transposes():
    torch = torch_mod()
    dims = (6, 64, 256)
    net, p = make_net(dims, 3)
    torch.cuda.synchronize()
    pb = bf16_values(host(net.params_bf16))
    assert np.array_equal(pb, om.bf16_round(p))
    o = net.offsets()
    W2 = host(net.params_bf16)[o["W2"][0]:o["W2"][1]].reshape(64, 64)
    W3 = host(net.params_bf16)[o["W3"][0]:o["W3"][1]].reshape(256, 64)
    assert np.array_equal(host(net.w2t).reshape(64, 64), W2.T)
    assert np.array_equal(host(net.w3t).reshape(64, 256), W3.T)


@pytest.mark.parametrize("B", [37, 64])
def test_forward_and_gradient_match_oracle(B):
    torch = torch_mod()
    net, p = make_net(DIMS, 11)
    x, t = batch_inputs(B, DIMS, 12)
    print(f"mlp forward/backward B={B}", flush=True)
    y_fw = host(net.forward(dev(x)))
    loss, y = net.loss_grad(dev(x), dev(t), want_y=True)
    torch.cuda.synchronize()
    g = host(net.grads).astype(np.float64)
    ref_loss, ref_g, ref_y = om.loss_grad(p, x, t, DIMS, bf16=True)
    y = host(y)
    assert np.array_equal(y, y_fw)
    assert np.linalg.norm(y - ref_y) <= 1e-4 * np.linalg.norm(ref_y)
    assert np.max(np.abs(y - ref_y)) <= 1e-3 * np.max(np.abs(ref_y))
    assert abs(host(loss)[0] - ref_loss) <= 1e-5 * ref_loss
    o = net.offsets()
    for k, (a, b) in o.items():
        err = np.linalg.norm(g[a:b] - ref_g[a:b]) / np.linalg.norm(ref_g[a:b])
        assert err <= 1e-3, (k, err)


def test_index_gather_equals_contiguous_batch():
    torch = torch_mod()
    dims = (6, 64, 256)
    net, p = make_net(dims, 5)
    x, t = batch_inputs(40, dims, 6)
    idx = np.array([3, 17, 0, 39, 22, 8, 8, 30, 1, 12], dtype=np.int32)
    l1 = net.loss_grad(dev(x), dev(t), idx=dev(idx))
    g1 = host(net.grads).copy()
    l2 = net.loss_grad(dev(x[idx]), dev(t[idx]))
    g2 = host(net.grads)
    torch.cuda.synchronize()
    assert host(l1)[0] == host(l2)[0]
    assert np.array_equal(g1, g2)


def test_adam_step_matches_oracle():
    torch = torch_mod()
    dims = (6, 64, 256)
    net, p = make_net(dims, 7)
    rng = np.random.default_rng(8)
    P = p.size
    g = (rng.standard_normal(P) * 10.0 ** rng.uniform(-6, 0, P)).astype(np.float32)
    m = (0.1 * rng.standard_normal(P)).astype(np.float32)
    v = (0.01 * rng.random(P)).astype(np.float32)
    net.grads.copy_(dev(g))
    net.adam_m.copy_(dev(m))
    net.adam_v.copy_(dev(v))
    net.step_count = 2
    net.adam_step(1e-3, 0.9, 0.999, 1e-8)     # step t = 3
    torch.cuda.synchronize()
    rp, rm, rv = om.adam_step(p, g, m, v, 3, 1e-3, 0.9, 0.999, 1e-8)
    gp, gm, gv = host(net.params), host(net.adam_m), host(net.adam_v)
    assert np.all(np.abs(gm - rm) <= 1e-6 * (0.9 * np.abs(m) + 0.1 * np.abs(g)) + 1e-30)
    assert np.all(np.abs(gv - rv) <= 1e-6 * np.abs(rv) + 1e-15)
    step = np.abs(rp - p)
    assert np.all(np.abs(gp - rp) <= 1e-5 * step + 1.2e-7 * np.abs(rp) + 1e-12)
    pb = bf16_values(host(net.params_bf16))
    assert np.all(np.abs(pb - gp) <= 2.0 ** -8 * np.abs(gp))


def test_short_training_run_tracks_oracle():
    torch = torch_mod()
    dims = (6, 64, 256)
    net, p = make_net(dims, 9)
    x, t = batch_inputs(16, dims, 10)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    gl, ol = [], []
    for step in range(1, 21):
        loss = net.loss_grad(dev(x), dev(t))
        net.adam_step(3e-3)
        torch.cuda.synchronize()
        gl.append(host(loss)[0])
        lo, go, _ = om.loss_grad(p, x, t, dims, bf16=True)
        ol.append(lo)
        p, m, v = om.adam_step(p, go, m, v, step, 3e-3)
    assert gl[-1] < 0.5 * gl[0]
    assert abs(gl[0] - ol[0]) <= 1e-5 * ol[0]
    assert np.all(np.abs(np.array(gl) - np.array(ol)) <= 3e-2 * np.array(ol))


def test_gradients_across_batch_sizes_on_one_network():
    """One network called at batch sizes whose row grouping and split-K plans differ (and whose
    scratch need is not monotone in the batch): every call matches the oracle."""
    torch = torch_mod()
    dims = (6, 64, 256)
    net, p = make_net(dims, 13)
    for B in (9, 8, 1, 129, 128, 300):
        x, t = batch_inputs(B, dims, 100 + B)
        print(f"mlp loss_grad dims={dims} B={B}", flush=True)
        loss = net.loss_grad(dev(x), dev(t))
        torch.cuda.synchronize()
        g = host(net.grads).astype(np.float64)
        ref_loss, ref_g, _ = om.loss_grad(p, x, t, dims, bf16=True)
        assert abs(host(loss)[0] - ref_loss) <= 1e-5 * ref_loss
        for k, (a, b) in net.offsets().items():
            err = np.linalg.norm(g[a:b] - ref_g[a:b]) / np.linalg.norm(ref_g[a:b])
            assert err <= 1e-3, (B, k, err)
