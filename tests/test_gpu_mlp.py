"""Warm-start network on the matrix cores, through the C ABI.

Bounds: with small-integer inputs and weights every bfloat16 operand and
every FP32 sum is exact, so one linear layer's forward pass and its
gradient must equal the FP64 reference bit for bit (this pins the matrix
cores' operand and result layouts, the transposed operands of the backward
products and the edge guards).  Deep tanh networks are compared with the
bfloat16 emulator (the same roundings; FP32 summation order and rare
one-ulp bfloat16 flips differ: 1e-2 normwise) and with FP64 (bfloat16
operands: 5e-2 normwise).
"""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2108_07031_amd import qlskum
    return torch, qlskum


def _say(msg):
    print(msg, flush=True)


def _dev(torch, a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda").contiguous()


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - b)) / max(np.max(np.abs(b)), 1e-30))


@pytest.mark.parametrize("K,N,n", [(6, 4, 1), (6, 128, 17), (128, 128, 1000), (37, 33, 70),
                                   (128, 4, 300), (32, 16, 64)])
def test_linear_layer_exact(env, K, N, n):
    torch, ql = env
    _say(f"linear forward K={K} N={N} n={n}")
    rng = np.random.default_rng(K * 1000 + N)
    w = rng.integers(-8, 9, mlp.n_params([K, N])).astype(np.float64)
    X = rng.integers(-8, 9, (n, K)).astype(np.float64)
    m = ql.Mlp([K, N], max_batch=max(n, 8))
    m.set_weights(w)
    Y = m.forward(_dev(torch, X)).cpu().numpy()
    _, ref = mlp.forward(w, [K, N], X)
    np.testing.assert_array_equal(Y, ref)
    m.close()


@pytest.mark.parametrize("K,N,n", [(5, 4, 32), (6, 16, 64), (128, 128, 256), (37, 32, 64),
                                   (128, 128, 1024), (6, 4, 2048)])
def test_linear_gradient_exact(env, K, N, n):
    """n >= 512: the weight gradient's product is split along the batch
    (slices of 256 rows added in slice order); on integer data every
    partial sum is exact, so the result is the same bit for bit."""
    torch, ql = env
    _say(f"linear gradient K={K} N={N} n={n}")
    rng = np.random.default_rng(7 * K + N)
    w = rng.integers(-8, 9, mlp.n_params([K, N])).astype(np.float64)
    X = rng.integers(-8, 9, (n, K)).astype(np.float64)
    _, y = mlp.forward(w, [K, N], X)
    T = y - rng.integers(-4, 5, y.shape)
    m = ql.Mlp([K, N], max_batch=n)
    m.set_weights(w)
    loss, g = m.gradient(_dev(torch, X), _dev(torch, T))
    lref, gref = mlp.loss_grad(w, [K, N], X, T)
    assert loss == lref
    np.testing.assert_array_equal(g, gref.astype(np.float32))
    m.close()


def _xavier(rng, widths):
    parts = []
    for fi, fo in zip(widths[:-1], widths[1:]):
        parts.append(rng.normal(0.0, np.sqrt(1.0 / fi), fi * fo))
        parts.append(rng.normal(0.0, 0.1, fo))
    return np.concatenate(parts)


@pytest.mark.parametrize("n", [2048, 1500])
def test_deep_network_matches_emulator(env, n):
    """n = 1500: the split weight-gradient products end on a short slice
    (six slices of 256 rows, the last of 220)."""
    torch, ql = env
    _say(f"deep network forward and gradient, {n} rows")
    widths = [6, 128, 128, 128, 128, 4]
    rng = np.random.default_rng(2108)
    w = _xavier(rng, widths).astype(np.float32)
    X = rng.normal(0.0, 1.0, (n, 6)).astype(np.float32)
    T = rng.normal(0.0, 1.0, (n, 4)).astype(np.float32)
    m = ql.Mlp(widths, max_batch=n)
    m.set_weights(w)
    assert m.num_params == 50948
    np.testing.assert_array_equal(m.get_weights(), w)
    Y = m.forward(_dev(torch, X)).cpu().numpy()
    e_emu = _rel(Y, mlp.forward_bf16(w, widths, X))
    e_64 = _rel(Y, mlp.forward(w.astype(np.float64), widths, X)[1])
    loss, g = m.gradient(_dev(torch, X), _dev(torch, T))
    lemu, gemu = mlp.loss_grad_bf16(w, widths, X, T)
    l64, g64 = mlp.loss_grad(w.astype(np.float64), widths, X, T)
    ge_emu, ge_64 = _rel(g, gemu), _rel(g, g64)
    _say(f"  forward vs emulator {e_emu:.2e}, vs FP64 {e_64:.2e}; gradient vs emulator "
         f"{ge_emu:.2e}, vs FP64 {ge_64:.2e}; loss {loss:.6f} / {lemu:.6f} / {l64:.6f}")
    assert e_emu <= 1e-2 and e_64 <= 5e-2
    assert ge_emu <= 1e-2 and ge_64 <= 5e-2
    assert abs(loss - lemu) <= 1e-3 * lemu
    m.close()


def test_training_tracks_fp64(env):
    torch, ql = env
    _say("training")
    widths = [2, 32, 32, 1]
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (512, 2))
    T = np.sin(2 * X[:, :1]) * np.cos(X[:, 1:])
    w0 = _xavier(rng, widths)
    m = ql.Mlp(widths, max_batch=512)
    m.set_weights(w0)
    Xd, Td = _dev(torch, X), _dev(torch, T)
    w, mm, vv = w0.copy(), np.zeros_like(w0), np.zeros_like(w0)
    l0 = mlp.loss_grad(w0, widths, X, T)[0]
    for t in range(1, 301):
        lg = m.train_step(Xd, Td, 1e-2, want_loss=(t == 300))
        _, g = mlp.loss_grad(w, widths, X, T)
        w, mm, vv = mlp.adam(w, g, mm, vv, t, 1e-2)
    l64 = mlp.loss_grad(w, widths, X, T)[0]
    lgpu = mlp.loss_grad(m.get_weights().astype(np.float64), widths, X, T)[0]
    _say(f"  loss {l0:.4e} -> GPU {lgpu:.4e} (reported {lg:.4e}), FP64 {l64:.4e}")
    assert lgpu < 0.05 * l0 and l64 < 0.05 * l0
    assert lgpu < 3.0 * l64 + 1e-4
    m.close()


def test_network_errors(env):
    torch, ql = env
    _say("network errors")
    with pytest.raises(ql.QLError):
        ql.Mlp([6], max_batch=4)
    with pytest.raises(ql.QLError):
        ql.Mlp([6, 0, 4], max_batch=4)
    m = ql.Mlp([3, 5, 2], max_batch=4)
    X = _dev(torch, np.zeros((4, 3)))
    with pytest.raises(ql.QLError):
        m.forward(X)  # no weights yet
    w = np.zeros(m.num_params, np.float32)
    w[0] = np.nan
    with pytest.raises(ql.QLError):
        m.set_weights(w)
    m.set_weights(np.zeros(m.num_params, np.float32))
    with pytest.raises(ql.QLError):
        m.gradient(_dev(torch, np.zeros((5, 3))), _dev(torch, np.zeros((5, 2))))  # > max_batch
    with pytest.raises(ql.QLError):
        m.train_step(X, _dev(torch, np.zeros((4, 2))), -1.0)
    m.close()
