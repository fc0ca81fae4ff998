"""The warm-start network in float64: forward, backward, MSE loss and Adam (test infrastructure).

The network (not in the paper; W0 is only an input of Alg. 2) is a multilayer
perceptron with SiLU activations, silu(z) = z sigmoid(z), between dense layers
of widths sizes = [D + 2, H, H, H, 1].  Its parameters are one flat vector,
layer by layer: the weight matrix W_l (out x in, row-major) and then the bias b_l
(out).  A layer maps a row-batch A (m x in) to Z = A W_l^T + b_l; every layer
but the last applies silu to Z.

Loss: the mean squared error (1/m) sum_i (f(a_i) - t_i)^2.  Its gradient is
obtained by the chain rule, layer by layer from the output back (reverse-mode
differentiation), using silu'(z) = s(z) (1 + z (1 - s(z))) with s the logistic
sigmoid.  Adam (Kingma and Ba) with bias-corrected first and second moments
updates the parameters.
"""
import numpy as np


def layer_shapes(sizes):
    """[(out, in)] of the dense layers."""
    return [(sizes[i + 1], sizes[i]) for i in range(len(sizes) - 1)]


def param_count(sizes):
    return sum(o * i + o for o, i in layer_shapes(sizes))


def unpack(params, sizes):
    """[(W_l, b_l)] views into the flat parameter vector."""
    out, off = [], 0
    for o, i in layer_shapes(sizes):
        W = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((W, b))
    return out


def sigmoid(z):
    """Logistic function, evaluated as 1 / (1 + e^-|z|) mirrored, so no branch cancels."""
    z = np.asarray(z, dtype=np.float64)
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params, sizes, A):
    """Network output f(a_i) for the rows of A, plus the pre-activations of every layer."""
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    act = np.asarray(A, dtype=np.float64)
    acts, pre = [act], []
    for li, (W, b) in enumerate(layers):
        z = act @ W.T + b
        pre.append(z)
        act = silu(z) if li < len(layers) - 1 else z
        acts.append(act)
    return act[:, 0], (acts, pre)


def mse(out, target):
    r = np.asarray(out, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(r * r))


def loss_and_grad(params, sizes, A, target):
    """(loss, d loss / d params) for one batch."""
    params = np.asarray(params, dtype=np.float64)
    out, (acts, pre) = forward(params, sizes, A)
    m = out.shape[0]
    layers = unpack(params, sizes)
    grads = [None] * len(layers)
    dz = (2.0 / m) * (out - np.asarray(target, dtype=np.float64))[:, None]
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads[li] = (dz.T @ acts[li], dz.sum(axis=0))
        if li > 0:
            dz = (dz @ W) * silu_grad(pre[li - 1])
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return mse(out, target), flat


class Adam:
    """Adam state for a flat parameter vector (step counter starts at 1)."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps

    def step(self, params, grad):
        """Returns the updated parameters."""
        self.t += 1
        self.m = self.beta1 * self.m + (1.0 - self.beta1) * grad
        self.v = self.beta2 * self.v + (1.0 - self.beta2) * grad * grad
        mhat = self.m / (1.0 - self.beta1 ** self.t)
        vhat = self.v / (1.0 - self.beta2 ** self.t)
        return params - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def train(params, sizes, A, target, epochs, batch, lr, seed, order=None):
    """Minibatch Adam.  Epoch e visits the rows in the order order(seed, e, m), in
    consecutive batches of `batch` rows (the last one may be shorter).  Returns the
    parameters and the mean loss of each epoch (average of the batch losses, each
    weighted by its row count)."""
    from . import rng

    order = order or (lambda s, e, m: rng.permutation(s, rng.PURPOSE_MINIBATCH, e, m))
    params = np.array(params, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    m = A.shape[0]
    opt = Adam(params.size, lr=lr)
    losses = []
    for e in range(epochs):
        perm = order(seed, e, m)
        tot = 0.0
        for i0 in range(0, m, batch):
            idx = perm[i0:i0 + batch]
            loss, g = loss_and_grad(params, sizes, A[idx], target[idx])
            params = opt.step(params, g)
            tot += loss * idx.size
        losses.append(tot / m)
    return params, np.array(losses)
