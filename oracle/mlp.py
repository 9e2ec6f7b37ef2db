"""FP64 reference of the warm-start network, and an emulator of its BF16
arithmetic.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark may
import this module.  The solver package never does.

The network is a plain multilayer perceptron with widths w_0 .. w_L:
    a_0 = x,   z_l = a_{l-1} W_l + b_l,   a_l = tanh(z_l)  (l < L),   y = z_L
with W_l of shape (w_{l-1}, w_l).  The loss of a batch of B samples is the
mean squared error over samples and outputs,
    loss = 1/(B w_L) sum (y - t)^2 .
Gradients are the layer-by-layer chain rule written out (reverse mode):
    d_L = 2 (y - t) / (B w_L),   dW_l = a_{l-1}^T d_l,   db_l = sum_rows d_l,
    d_{l-1} = (d_l W_l^T) * (1 - a_{l-1}^2).
The optimiser is Adam (Kingma and Ba, 2015) with bias-corrected moments.

Flat parameter layout (shared with the device library's weight vector):
for l = 1 .. L, W_l row-major (w_{l-1} x w_l), then b_l (w_l).

parity unpinned: none -- every function here is checked against finite
differences, closed-form properties of Adam, or the bfloat16 format's
definition in tests/test_mlp_oracle.py.
"""
import numpy as np


def n_params(widths):
    """Number of parameters of the network."""
    return sum(widths[l - 1] * widths[l] + widths[l] for l in range(1, len(widths)))


def unflatten(w, widths):
    """Flat parameter vector -> list of (W_l, b_l) views, l = 1 .. L."""
    out, o = [], 0
    for l in range(1, len(widths)):
        fi, fo = widths[l - 1], widths[l]
        W = w[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        b = w[o:o + fo]
        o += fo
        out.append((W, b))
    assert o == len(w)
    return out


def flatten(params):
    """List of (W_l, b_l) -> flat vector."""
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def forward(w, widths, X):
    """Activations a_0 .. a_{L-1} and the output y, all FP64."""
    acts = [np.asarray(X, np.float64)]
    layers = unflatten(np.asarray(w, np.float64), widths)
    for l, (W, b) in enumerate(layers):
        z = acts[-1] @ W + b
        if l < len(layers) - 1:
            acts.append(np.tanh(z))
        else:
            return acts, z
    raise AssertionError("network without layers")


def loss_grad(w, widths, X, T):
    """Mean squared error of the batch and its gradient (flat, FP64)."""
    acts, y = forward(w, widths, X)
    B, nout = y.shape
    d = 2.0 * (y - T) / (B * nout)
    loss = float(np.mean((y - T) ** 2))
    layers = unflatten(np.asarray(w, np.float64), widths)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_prev = acts[l]
        grads[l] = (a_prev.T @ d, d.sum(axis=0))
        if l > 0:
            d = (d @ W.T) * (1.0 - a_prev ** 2)
    return loss, flatten(grads)


def adam(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --- bfloat16 -----------------------------------------------------------------

def bf16(x):
    """Round FP32 values to bfloat16 (8 exponent, 7 fraction bits), round to
    nearest, ties to even; returned as FP32 values.  NaN stays NaN."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).copy()
    nan = np.isnan(f)
    out[nan] = np.nan
    return out


def forward_bf16(w, widths, X):
    """The device's inference arithmetic: inputs, weights and hidden
    activations rounded to bfloat16, products accumulated in FP32, bias and
    tanh in FP32.  Returns FP32 outputs (FP32 accumulation order differs from
    the device's by FP32 rounding only)."""
    layers = unflatten(np.asarray(w, np.float32), widths)
    a = bf16(X)
    for l, (W, b) in enumerate(layers):
        z = (a.astype(np.float64) @ bf16(W).astype(np.float64)).astype(np.float32) + b
        if l < len(layers) - 1:
            a = bf16(np.tanh(z))
        else:
            return z
    raise AssertionError("network without layers")


def loss_grad_bf16(w, widths, X, T):
    """The device's training arithmetic: the forward pass of forward_bf16
    (hidden activations kept in bfloat16), output error
    d_L = bf16(2 (y - t) / (B w_L)), and for each layer
        dW_l = a_{l-1}^T d_l,   db_l = sum_rows d_l         (FP32 results)
        d_{l-1} = bf16((d_l bf16(W_l)^T) * (1 - a_{l-1}^2))
    with bfloat16 operands of every product.  Returns (loss, flat FP32
    gradient); products are formed in FP64 and rounded once to FP32."""
    layers = unflatten(np.asarray(w, np.float32), widths)
    acts = [bf16(X)]
    for l, (W, b) in enumerate(layers):
        z = (acts[-1].astype(np.float64) @ bf16(W).astype(np.float64)).astype(np.float32) + b
        if l < len(layers) - 1:
            acts.append(bf16(np.tanh(z)))
        else:
            y = z
    T = np.asarray(T, np.float32)
    cnt = y.size
    diff = (y - T).astype(np.float32)
    loss = float(np.sum(diff.astype(np.float64) ** 2) / cnt)
    d = bf16(np.float32(2.0 / cnt) * diff)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        a_prev = acts[l]
        gW = (a_prev.T.astype(np.float64) @ d.astype(np.float64)).astype(np.float32)
        gb = d.astype(np.float64).sum(axis=0).astype(np.float32)
        grads[l] = (gW, gb)
        if l > 0:
            v = (d.astype(np.float64) @ bf16(W).T.astype(np.float64)).astype(np.float32)
            d = bf16(v * (np.float32(1.0) - a_prev * a_prev))
    return loss, flatten(grads)
