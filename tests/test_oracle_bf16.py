"""Pins of the BF16-form oracle (oracle/bf16.py): its rounding against torch's
float32 -> bfloat16 conversion (round to nearest even) and hand-checked ties;
equality with the plain float64 pass when every value is a bfloat16 number;
the rounding points (layer inputs and hidden weights rounded, head weights and
output gradient not) on a hand-computed case."""
import numpy as np
import torch

from oracle import bf16, mlp


def test_round_matches_torch_rne():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        rng.standard_normal(1000) * 1e-39,             # float32 subnormals
                        np.float32([3.3895e38, -3.39e38, 1e-45, 0.0, -0.0])])
    v = v.astype(np.float32)
    # exact ties: a bfloat16 value plus half its last-place step, with both parities of the last bit
    base = torch.from_numpy(rng.standard_normal(2000).astype(np.float32)).to(torch.bfloat16).float().numpy()
    bits = base.view(np.uint32)
    ties = (bits | np.uint32(0x8000)).view(np.float32)
    v = np.concatenate([v, ties])
    want = torch.from_numpy(v).to(torch.bfloat16).float().numpy().astype(np.float64)
    got = bf16.round_bf16(v.astype(np.float64))
    assert np.array_equal(got, want)


def test_round_hand_cases():
    # 1 + 2^-8 is the tie between 1 and 1 + 2^-7: even last bit -> 1; 1 + 3 2^-8 -> 1 + 2^-6
    assert bf16.round_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0
    assert bf16.round_bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6
    assert bf16.round_bf16(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7
    assert bf16.round_bf16(np.array([-(255.5)]))[0] == -256.0
    assert bf16.round_bf16(np.array([3.0 * 2.0 ** 125]))[0] == 3.0 * 2.0 ** 125


def _dyadic_net(rng, K, W, H, c):
    shapes = mlp.layer_shapes(K, W, H, c)
    params = [(rng.integers(-2, 3, s).astype(np.float64) * 0.5, rng.integers(-2, 3, s[0]).astype(np.float64) * 0.25)
              for s in shapes]
    return shapes, params


def test_equals_float64_pass_on_bf16_numbers():
    """Small dyadic weights, inputs and output gradients keep every sum a bfloat16 number:
    then the BF16 form is the plain pass, forward and backward."""
    rng = np.random.default_rng(3)
    shapes, params = _dyadic_net(rng, 6, 5, 3, 2)
    z0 = rng.integers(-4, 5, (40, 6)) * 0.5
    gy = rng.integers(-3, 4, (40, 2)) * 0.25
    y, c = mlp.forward(params, z0)
    yb, cb = bf16.forward_bf16(params, z0)
    assert np.array_equal(y, yb)
    assert all(np.array_equal(a, b) for a, b in zip(c, cb))
    g = mlp.flatten(mlp.backward(params, c, gy))
    gb = mlp.flatten(bf16.backward_bf16(params, cb, gy))
    assert np.array_equal(g, gb)
    assert np.any(g != 0)


def test_rounding_points():
    """One hidden layer of one unit, one input: z = bf16(w) bf16(x) + b, h = bf16(relu z),
    y = w_o h + b_o with the head weight unrounded; backward g = bf16(w_o gy) for z > 0."""
    e = 2.0 ** -8
    w, b, wo, bo = 1 + 3 * e, 2.0 ** -10, 1 + e, 0.5
    x = 1 + e                                            # rounds to 1 (tie, even)
    params = [(np.array([[w]]), np.array([b])), (np.array([[wo]]), np.array([bo]))]
    y, c = bf16.forward_bf16(params, np.array([[x]]))
    zw = (1 + 2 * 2 ** -7) * 1.0 + b                     # bf16(w) = 1 + 2^-6, bf16(x) = 1
    assert c[1][0, 0] == zw
    h = bf16.round_bf16(np.array([zw]))[0]
    assert h == 1 + 2.0 ** -6 and c[2][0, 0] == h
    assert y[0, 0] == wo * h + bo
    gy = np.array([[1 + 2.0 ** -9]])
    (dW1, db1), (dWo, dbo) = bf16.backward_bf16(params, c, gy)
    assert dWo[0, 0] == gy[0, 0] * h and dbo[0] == gy[0, 0]
    # (1 + 2^-8)(1 + 2^-9) = 1 + 2^-8 + 2^-9 + 2^-17 lies above the tie 1 + 2^-8: up to 1 + 2^-7
    g = 1 + 2.0 ** -7
    assert bf16.round_bf16(np.array([wo * gy[0, 0]]))[0] == g
    assert dW1[0, 0] == g * 1.0 and db1[0] == g
    # a negative pre-activation stops the gradient
    params[0] = (np.array([[-w]]), np.array([b]))
    _, c = bf16.forward_bf16(params, np.array([[x]]))
    (dW1, db1), _ = bf16.backward_bf16(params, c, gy)
    assert dW1[0, 0] == 0 and db1[0] == 0
