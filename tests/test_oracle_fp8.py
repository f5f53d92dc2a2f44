"""Pins of the FP8 (e4m3) oracle: the format from its definition, rounding by
brute force over all codes, and forward passes that reduce to the exact one."""
import numpy as np

import workloads
from oracle import fp8, mlp


def test_e4m3_format_constants():
    v = fp8.e4m3_values()
    pos = v[v > 0]
    assert pos.max() == 448.0                      # largest finite value
    assert pos.min() == 2.0 ** -9                  # smallest subnormal
    assert np.min(pos[pos >= 2.0 ** -6]) == 2.0 ** -6  # smallest normal
    assert len(v) == 253                           # 256 codes - 2 NaN - duplicate zero
    assert np.isnan(fp8.e4m3_decode(0x7F)) and np.isnan(fp8.e4m3_decode(0xFF))
    assert fp8.e4m3_decode(0x38) == 1.0 and fp8.e4m3_decode(0x7E) == 448.0


def test_e4m3_round_is_nearest_even_by_brute_force():
    v = fp8.e4m3_values()
    assert np.array_equal(fp8.e4m3_round(v), v)  # every value maps to itself
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-500, 500, 4000), rng.uniform(-0.05, 0.05, 4000),
                        (v[:-1] + v[1:]) / 2.0])     # include every tie
    q = fp8.e4m3_round(x)
    xc = np.clip(x, -448, 448)
    d = np.abs(xc[:, None] - v[None, :])
    dmin = d.min(axis=1)
    assert np.allclose(np.abs(q - xc), dmin, rtol=0, atol=0)
    # ties go to the neighbour with an even mantissa (even code index)
    codes = {val: c for c in range(256) for val in [fp8.e4m3_decode(c)] if val == val and not (val == 0 and c)}
    mid = (v[:-1] + v[1:]) / 2.0
    for m_, qq in zip(mid, fp8.e4m3_round(mid)):
        assert codes[qq] % 2 == 0, (m_, qq)
    assert fp8.e4m3_round(464.0) == 448.0 and fp8.e4m3_round(1e9) == 448.0
    assert fp8.e4m3_round(2.0 ** -10) == 0.0 and fp8.e4m3_round(3 * 2.0 ** -10) == 2.0 ** -8


def test_forward_fp8_exact_when_everything_is_representable():
    """Weights in {0, +-1} and inputs in {0, 1/2, 1/4} (maximum 1/2 in every
    sample, so both scales are exact) quantise without error: the FP8 form
    equals the float64 forward."""
    rng = np.random.default_rng(1)
    shapes = mlp.layer_shapes(8, 16, 1, 1)
    W1 = rng.choice([-1.0, 0.0, 1.0], size=(16, 8))
    W1[0, 0] = 1.0
    params = [(W1, rng.normal(size=16)), (rng.normal(size=(1, 16)), rng.normal(size=1))]
    x = rng.choice([0.0, 0.5, 0.25], size=(50, 8))
    x[:, 0] = 0.5
    assert np.allclose(fp8.forward_fp8(params, x), mlp.forward(params, x)[0], rtol=1e-12, atol=1e-12)
    assert shapes[0] == (16, 8)


def test_forward_fp8_error_within_format_bound():
    """Random networks: the FP8 form stays within a few e4m3 roundings (relative
    2^-4 each) of the exact forward."""
    K, W, H = 128, 64, 3
    theta = workloads.init_params(K, W, H, 1, seed=3).astype(np.float64)
    params = mlp.unflatten(theta, mlp.layer_shapes(K, W, H, 1))
    x = np.random.default_rng(2).uniform(0, 1, (300, 3))
    z0 = mlp.encode(x, workloads.ffm_matrix(K // 2, 3.0, seed=4).astype(np.float64))
    y8 = fp8.forward_fp8(params, z0)
    y = mlp.forward(params, z0)[0]
    rel = np.linalg.norm(y8 - y) / np.linalg.norm(y)
    assert 1e-4 < rel < 0.1, rel
