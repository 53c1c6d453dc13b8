"""Oracle of the learned-bounds network (test infrastructure only): a plain
FP64 NumPy multilayer perceptron with the exact GELU, its mean-squared-error
gradient by backpropagation written out layer by layer, and the Adam update
(Kingma & Ba, bias-corrected).

Parameter layout, the interface of the device network: for layer l = 0..depth,
W_l [out_l][in_l] row-major, then b_l [out_l]; in_0 = n_in, out_l = width for
hidden layers, out_depth = n_out.  Hidden layers apply GELU, the last layer is
linear.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def layer_shapes(n_in: int, width: int, depth: int, n_out: int) -> list[tuple[int, int]]:
    shapes = []
    for l in range(depth + 1):
        fan_in = n_in if l == 0 else width
        fan_out = width if l < depth else n_out
        shapes.append((fan_out, fan_in))
    return shapes


def n_params(n_in: int, width: int, depth: int, n_out: int) -> int:
    return sum(o * i + o for o, i in layer_shapes(n_in, width, depth, n_out))


def unpack(params: np.ndarray, n_in: int, width: int, depth: int, n_out: int):
    """List of (W, b) views of the flat parameter vector."""
    out, k = [], 0
    for o, i in layer_shapes(n_in, width, depth, n_out):
        W = params[k:k + o * i].reshape(o, i)
        k += o * i
        b = params[k:k + o]
        k += o
        out.append((W, b))
    assert k == params.size
    return out


def gelu(x):
    """x Phi(x), Phi the standard normal distribution function."""
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_prime(x):
    """Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(params, X, n_in, width, depth, n_out):
    """Network output and the per-layer inputs / pre-activations."""
    layers = unpack(np.asarray(params, dtype=np.float64), n_in, width, depth, n_out)
    A = np.asarray(X, dtype=np.float64)
    acts, pre = [A], []
    for l, (W, b) in enumerate(layers):
        Z = A @ W.T + b
        pre.append(Z)
        A = gelu(Z) if l < depth else Z
        acts.append(A)
    return A, (acts, pre)


def loss_grad(params, X, T, n_in, width, depth, n_out):
    """Mean over all B x n_out entries of (net(X) - T)^2 and its gradient."""
    params = np.asarray(params, dtype=np.float64)
    Y, (acts, pre) = forward(params, X, n_in, width, depth, n_out)
    D = Y - np.asarray(T, dtype=np.float64)
    loss = float(np.mean(D * D))
    layers = unpack(params, n_in, width, depth, n_out)
    grads = [None] * len(layers)
    dA = 2.0 * D / D.size
    for l in range(depth, -1, -1):
        dZ = dA * gelu_prime(pre[l]) if l < depth else dA
        W, _ = layers[l]
        grads[l] = (dZ.T @ acts[l], dZ.sum(axis=0))
        dA = dZ @ W
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at step count t (1-based); returns (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
