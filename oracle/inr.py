"""INR f_theta, the evaluation operator E, and the exact Jacobian-transpose
product (Sec. III: grad L = sum_i v_i grad_theta f_theta(x_i); Eq. (2);
Eq. (3)).

Architectures (Sec. IV names FFN, SIREN and hash encoding):
  * FFN (Fourier features + ReLU MLP): a_0 = [sin(2 pi B x); cos(2 pi B x)]
    (sin block first), z_l = W_l a_{l-1} + b_l, a_l = max(z_l, 0) for
    l = 1..L, f = w_out . a_L + b_out.  B is fixed (not trained).
  * SIREN: a_0 = x, a_l = sin(omega0 z_l) for l = 1..L, same linear output.
  * hash encoding: a_0 = the multi-resolution hash encoding of x (module
    ``hashenc``, whose tables are trained), then the FFN's ReLU MLP.

Parameter vector layout: for each affine layer in order, W (fan_out x
fan_in, row-major) then b; the output layer last.  The hash encoding's
tables come before the MLP.

The backward pass is textbook reverse mode (chain rule applied layer by
layer), with ReLU'(0) taken as 0.
"""
import numpy as np

from . import hashenc


def _enc_dim(arch):
    if arch.kind == "ffn":
        return 2 * arch.n_freq
    if arch.kind == "hash":
        return arch.hash_levels * arch.hash_feats
    return arch.in_dim


def _n_tab(arch):
    return hashenc.n_table_params(arch) if arch.kind == "hash" else 0


def layer_dims(arch):
    enc = _enc_dim(arch)
    dims = [(enc, arch.width)] + [(arch.width, arch.width)] * (arch.depth - 1)
    return dims + [(arch.width, 1)]


def n_params(arch):
    return _n_tab(arch) + sum(i * o + o for i, o in layer_dims(arch))


def unpack(theta, arch):
    theta = np.asarray(theta, np.float64)
    layers, off = [], _n_tab(arch)
    for fi, fo in layer_dims(arch):
        W = theta[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = theta[off:off + fo]
        off += fo
        layers.append((W, b))
    if off != theta.size:
        raise ValueError("theta has %d entries, architecture needs %d"
                         % (theta.size, off))
    return layers


def pack(grads):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in grads])


def encode(X, B, arch, theta=None):
    X = np.asarray(X, np.float64)
    if arch.kind == "hash":
        return hashenc.encode(theta, X, arch)
    if arch.kind == "ffn":
        ph = 2.0 * np.pi * (X @ np.asarray(B, np.float64).T)
        return np.concatenate([np.sin(ph), np.cos(ph)], axis=1)
    return X


def _act(z, arch):
    return np.maximum(z, 0.0) if arch.kind != "siren" else np.sin(arch.omega0 * z)


def _act_grad(z, arch):
    if arch.kind != "siren":
        return (z > 0.0).astype(np.float64)
    return arch.omega0 * np.cos(arch.omega0 * z)


def forward(theta, B, X, arch, keep=False):
    """f_theta at the points X (k x d).  With keep=True also returns the
    layer inputs a_0..a_L and pre-activations z_1..z_L."""
    layers = unpack(theta, arch)
    a = encode(X, B, arch, theta)
    acts, pre = [a], []
    for W, b in layers[:-1]:
        z = a @ W.T + b
        a = _act(z, arch)
        pre.append(z)
        acts.append(a)
    W, b = layers[-1]
    f = a @ W[0] + b[0]
    return (f, acts, pre) if keep else f


def vjp(theta, B, X, cot, arch):
    """sum_i cot_i * grad_theta f_theta(x_i), as a flat vector."""
    layers = unpack(theta, arch)
    cot = np.asarray(cot, np.float64)
    _, acts, pre = forward(theta, B, X, arch, keep=True)
    L = len(layers) - 1
    grads = [None] * (L + 1)
    W_out = layers[-1][0]
    grads[L] = ((cot @ acts[L])[None, :], np.array([cot.sum()]))
    g_a = cot[:, None] * W_out[0][None, :]          # dL/da_L
    for l in range(L - 1, -1, -1):
        g_z = g_a * _act_grad(pre[l], arch)         # dL/dz_{l+1}
        grads[l] = (g_z.T @ acts[l], g_z.sum(axis=0))
        if l > 0:
            g_a = g_z @ layers[l][0]                # dL/da_l
    if arch.kind == "hash":                         # dL/da_0 into the tables
        g_enc = g_z @ layers[0][0]
        return np.concatenate([hashenc.encode_vjp(X, g_enc, arch), pack(grads)])
    return pack(grads)


def eval_grid(theta, B, arch, dim, N, fov_idx, coords_fn):
    """E{f_theta} on the full grid: f at FOV points, 0 elsewhere."""
    u = np.zeros(N ** dim)
    u[fov_idx] = forward(theta, B, coords_fn(dim, N, fov_idx), arch)
    return u.reshape([N] * dim)
