"""FP8 (OCP e4m3) form of the coordinate-MLP forward pass, float64 oracle.

Test infrastructure: only the tests, the smoke check and the CPU baseline of
the benchmark use this package.

The paper stores networks in 16 bits and names mixed-precision inference as
future work (Sec. 5, Discussion); the FP8 form is this implementation's reading of that
direction for decoding.  Its definition:
  * a value is rounded to e4m3 (1 sign, 4 exponent bits with bias 7, 3 mantissa
    bits, subnormals, largest finite 448, no infinities) to nearest, ties to an
    even mantissa, after clamping to [-448, 448];
  * each hidden layer's weight matrix W_l is quantised as q(W_l * s_w) with one
    scale s_w = 448 / max|W_l| per layer;
  * the input of each hidden layer (the encoding for the first) is quantised
    per sample as q(h * s_a), s_a = 448 / max_f |h_f| over that sample's
    features;
  * the product is accumulated exactly and divided by s_w * s_a, the bias added
    and ReLU applied; the identity head works on the unquantised last hidden
    activations.
Where a quantised code is decided, the decision is taken in float32, the
precision in which the device forms the scaled values: scales are float32
quotients, W * s_w and h * s_a are float32 products of float32 operands.
"""
import numpy as np

E4M3_MAX = 448.0


def e4m3_decode(code):
    """Value of an 8-bit e4m3 code (NaN for the two NaN codes)."""
    code = int(code) & 0xFF
    s, e, m = code >> 7, (code >> 3) & 15, code & 7
    if e == 15 and m == 7:
        return float("nan")
    v = (m / 8.0) * 2.0 ** -6 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return -v if s else v


def e4m3_values():
    """All finite e4m3 values, ascending, each once (+0 only)."""
    vals = {e4m3_decode(c) for c in range(256)}
    return np.array(sorted(v for v in vals if v == v))


def e4m3_round(x):
    """Round to the nearest e4m3 value, ties to an even mantissa, saturating at 448."""
    x = np.clip(np.asarray(x, np.float64), -E4M3_MAX, E4M3_MAX)
    _, e = np.frexp(x)                        # |x| = f 2^e with 0.5 <= f < 1
    e = np.maximum(e - 1, -6)                 # exponent of the binade (normal or subnormal)
    quantum = np.ldexp(1.0, e - 3)            # three mantissa bits
    return np.rint(x / quantum) * quantum


def _f32(a):
    return np.asarray(a, np.float32)


def layer_weight_scale(W):
    amax = np.float32(np.max(np.abs(_f32(W)))) if np.size(W) else np.float32(0)
    return np.float32(1.0) if amax == 0 else np.float32(E4M3_MAX) / amax


def quantize_weights(W):
    """(quantised values as float64, scale) of one layer's weights."""
    s = layer_weight_scale(W)
    return e4m3_round((_f32(W) * s).astype(np.float32)), s


def quantize_activations(h):
    """Per-sample quantisation of float32 activations h (n, f): (values, scales)."""
    h = _f32(h)
    amax = np.max(np.abs(h), axis=1).astype(np.float32)
    s = np.where(amax == 0, np.float32(1.0), np.float32(E4M3_MAX) / np.where(amax == 0, np.float32(1), amax))
    s = s.astype(np.float32)
    return e4m3_round((h * s[:, None]).astype(np.float32)), s


def forward_fp8(params, z0):
    """FP8-form forward of an MLP given as [(W_1, b_1), ..., (W_H, b_H), (W_out, b_out)]
    (ReLU networks only)."""
    if getattr(params, "omega", 0.0) != 0:
        raise ValueError("the FP8 form is defined for ReLU networks only")
    h = np.asarray(z0, np.float64)
    for Wl, bl in params[:-1]:
        Wq, sw = quantize_weights(Wl)
        hq, sa = quantize_activations(h)
        acc = hq @ Wq.T
        z = acc / (np.float64(sw) * sa.astype(np.float64))[:, None] + np.asarray(bl, np.float64)
        h = np.maximum(z, 0.0)
    Wo, bo = params[-1]
    return h @ np.asarray(Wo, np.float64).T + bo
