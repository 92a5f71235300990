"""Oracle for the learned sketch-size policy: a plain FP64 multilayer
perceptron with ReLU, its mean-squared-error gradient by the chain rule, and
the Adam update (Kingma and Ba, 2015, Algorithm 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The policy maps F features of one core update to two outputs (log J, log
lambda).  The paper fixes J only through the bound of Corollary 3 (Sec. 4)
and calls that bound conservative (Sec. 5); the network is an addition to
the method, so the oracle follows the textbook definitions, not the paper.

Parameter vector layout (shared with the C ABI, float32 there):
    for each layer l = 1..L with fan-in a and fan-out b:
        W_l (b x a, row-major: W_l[j, i] at offset + j * a + i), then b_l (b)
Network: z_1 = W_1 x + b_1, h_1 = relu(z_1), ..., output y = W_L h_{L-1} + b_L.
Loss over a batch of B samples: mean over the B x O outputs of (y - t)^2.
"""
import numpy as np


def layer_sizes(F, H, O, hidden_layers=3):
    """[(fan_in, fan_out)] for F -> H -> ... -> H -> O."""
    dims = [F] + [H] * hidden_layers + [O]
    return list(zip(dims[:-1], dims[1:]))


def param_count(F, H, O, hidden_layers=3):
    return sum(a * b + b for a, b in layer_sizes(F, H, O, hidden_layers))


def unpack(theta, F, H, O, hidden_layers=3):
    """Views (W_l, b_l) into the flat parameter vector."""
    out, off = [], 0
    for a, b in layer_sizes(F, H, O, hidden_layers):
        W = theta[off:off + a * b].reshape(b, a)
        off += a * b
        bias = theta[off:off + b]
        off += b
        out.append((W, bias))
    return out


def forward(theta, X, F, H, O, hidden_layers=3):
    """X: B x F.  Returns (Y: B x O, list of pre-activations z_l)."""
    layers = unpack(np.asarray(theta, dtype=np.float64), F, H, O, hidden_layers)
    h = np.asarray(X, dtype=np.float64)
    zs = []
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        h = z if li == len(layers) - 1 else np.maximum(z, 0.0)
    return h, zs


def loss(theta, X, T, F, H, O, hidden_layers=3):
    Y, _ = forward(theta, X, F, H, O, hidden_layers)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def loss_grad(theta, X, T, F, H, O, hidden_layers=3):
    """(loss, gradient w.r.t. the flat parameter vector), by backpropagation:
    dL/dy = 2 (y - t) / (B O); for a layer z = W h + b, dL/dW = delta^T h,
    dL/db = sum_B delta, dL/dh = delta W; through a ReLU, delta = dL/dh * [z > 0]."""
    theta = np.asarray(theta, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    layers = unpack(theta, F, H, O, hidden_layers)
    Y, zs = forward(theta, X, F, H, O, hidden_layers)
    B = X.shape[0]
    L = float(np.mean((Y - T) ** 2))
    # inputs of each layer
    ins = [X] + [np.maximum(z, 0.0) for z in zs[:-1]]
    grads = [None] * len(layers)
    delta = 2.0 * (Y - T) / (B * O)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        gW = delta.T @ ins[li]
        gb = delta.sum(axis=0)
        grads[li] = (gW, gb)
        if li > 0:
            delta = (delta @ W) * (zs[li - 1] > 0.0)
    flat = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])
    return L, flat


def adam_step(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v).
    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
    theta <- theta - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def finite_difference_grad(theta, X, T, F, H, O, hidden_layers=3, h=1e-6, idx=None):
    """Central differences of the loss for the entries idx of theta."""
    theta = np.asarray(theta, dtype=np.float64)
    idx = range(theta.size) if idx is None else idx
    out = []
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        out.append((loss(tp, X, T, F, H, O, hidden_layers) - loss(tm, X, T, F, H, O, hidden_layers)) / (2 * h))
    return np.array(out)
