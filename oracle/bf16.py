"""BF16 form of the coordinate-MLP forward and backward pass, float64 oracle.

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this package.

The paper trains in full precision and stores 16-bit weights (Sec. 4);
lower-precision arithmetic is named as future work (Sec. 5, Discussion).  The
BF16 form is this implementation's reading of that direction for training and
decoding, and this module defines it:
  * bf16(v) rounds a value to bfloat16 (8 significant bits, the float32
    exponent range) to nearest, ties to an even last bit;
  * the operands of every hidden layer's product are bfloat16: the weights
    bf16(W_l) and the layer input (bf16 of the mapped features gamma(x) for
    the first layer, the stored activations for the others); the products are
    summed exactly and the float32 bias added;
  * each hidden activation is stored as h_l = bf16(act(z_l)) (ReLU, or
    sin(omega z_l) with its derivative factor stored as d_l = bf16(omega cos(omega z_l)));
  * the identity head multiplies the stored h_H by its unrounded weights;
  * backward, with the output gradient gy unrounded: the head's input
    gradient g_H = bf16((W_head^T gy) * 1[z_H > 0]) is stored in bfloat16,
    dW_head = sum gy h_H^T, db_head = sum gy; for each hidden layer
    dW_l = sum g_l h_{l-1}^T and db_l = sum g_l of the stored bfloat16 values,
    and g_{l-1} = bf16((bf16(W_l)^T g_l) * d_{l-1}) with d = 1[z > 0] for ReLU
    (the head's input gradient likewise).
Where all of these values are already bfloat16 numbers the form equals the
plain float64 pass of oracle.mlp.
"""
import numpy as np

from . import mlp


def round_bf16(v):
    """Nearest bfloat16 value of each float64 entry, ties to an even last bit
    (values beyond the largest finite bfloat16 round to infinity).

    A float64 carries 53 significant bits, a bfloat16 8: in bfloat16's normal
    range the 45 low bits of the float64 significand are dropped, rounding to
    nearest with ties to an even kept part (a carry out of the significand
    moves into the exponent, as in the float64 encoding itself).  Values below
    the smallest normal bfloat16 (2^-126) round on the fixed step 2^-133 of
    its subnormals."""
    v = np.asarray(v, np.float64)
    bits = v.view(np.uint64)
    keep = (bits >> np.uint64(45)) & np.uint64(1)
    r = (bits + np.uint64((1 << 44) - 1) + keep) & ~np.uint64((1 << 45) - 1)
    out = r.view(np.float64).copy()
    a = np.abs(v)
    small = (a < 2.0 ** -126) & (a > 0)
    if np.any(small):
        q = a[small] * 2.0 ** 133                       # exact: a power-of-two scaling
        f = np.floor(q)
        d = q - f
        up = (d > 0.5) | ((d == 0.5) & (np.mod(f, 2) == 1))
        out[small] = np.sign(v[small]) * (f + up) * 2.0 ** -133
    big = np.isfinite(v) & (np.abs(out) >= 2.0 ** 128)   # rounded past the largest finite value
    out[big] = np.sign(v[big]) * np.inf
    nonfin = ~np.isfinite(v)
    out[nonfin] = v[nonfin]
    return out


def forward_bf16(params, z0):
    """Forward pass of the BF16 form on mapped features z0 (n, K).  Returns the
    output (n, c) and the cache [h_0, z_1, h_1, ..., z_H, h_H] of stored values."""
    omega = getattr(params, "omega", 0.0)
    h = round_bf16(z0)
    cache = [h]
    for Wl, bl in params[:-1]:
        z = h @ round_bf16(Wl).T + bl
        h = round_bf16(mlp.activation(z, omega))
        cache += [z, h]
    Wo, bo = params[-1]
    return h @ Wo.T + bo, cache


def backward_bf16(params, cache, gy):
    """Parameter gradient [(dW_l, db_l)] of the BF16 form for output gradients gy (n, c)."""
    H = len(params) - 1
    omega = getattr(params, "omega", 0.0)

    def factor(z):  # the stored derivative factor d of a hidden layer
        d = mlp.activation_grad(z, omega)
        return d if omega == 0 else round_bf16(d)
    gy = np.asarray(gy, np.float64)
    Wo, _ = params[H]
    grads = [None] * (H + 1)
    grads[H] = (gy.T @ cache[2 * H], gy.sum(axis=0))
    g = round_bf16((gy @ Wo) * factor(cache[2 * H - 1]))
    for l in range(H - 1, -1, -1):
        grads[l] = (g.T @ cache[2 * l], g.sum(axis=0))
        if l > 0:
            Wl, _ = params[l]
            g = round_bf16((g @ round_bf16(Wl)) * factor(cache[2 * l - 1]))
    return grads
