"""Pins for the oracle's number formats (BF16, OCP FP8 E4M3) and the FP64
predictor network.  The formats and the network are not in the paper; they
are pinned against torch's own conversions and against finite differences."""
import numpy as np
import pytest
import torch

from oracle import oracle as O


def test_bf16_decode_all_codes_roundtrip():
    """Every finite BF16 code decodes to a float that encodes back to itself."""
    codes = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    vals = O.bf16_decode(codes)
    fin = np.isfinite(vals)
    back = O.bf16_encode(vals[fin])
    assert np.array_equal(back, codes[fin])


def test_bf16_matches_torch_rne():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.normal(0, 1, 20000), rng.normal(0, 1e30, 2000), rng.normal(0, 1e-38, 2000),
        np.array([0.0, -0.0, 1.0, -1.0, 3.3895314e38, -3.3895314e38, 3.4e38, 1e-45]),
    ]).astype(np.float32)
    # exact halfway points between adjacent BF16 values: ties go to the even code
    base = rng.integers(0x3000, 0x5000, size=4000).astype(np.uint32) << 16
    half = (base | 0x8000).view(np.float32)
    x = np.concatenate([x, half])
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = O.bf16_encode(x)
    assert np.array_equal(got, want)
    # spot-check ties by hand: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7 -> 1 (even)
    assert O.bf16_encode(np.array([1.0 + 2 ** -8], np.float32))[0] == 0x3F80
    assert O.bf16_encode(np.array([1.0 + 3 * 2 ** -8], np.float32))[0] == 0x3F82


def test_e4m3_decode_table_matches_torch():
    codes = torch.arange(256, dtype=torch.int16).to(torch.uint8)
    want = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = np.array([O.e4m3_value(c) for c in range(256)])
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], want[~nan])
    assert O.e4m3_value(0x7E) == 448.0 and O.e4m3_value(0x01) == 2.0 ** -9


def test_e4m3_encode_matches_torch_in_range():
    rng = np.random.default_rng(1)
    y = np.concatenate([rng.uniform(-448, 448, 5000), rng.normal(0, 1, 5000),
                        rng.normal(0, 0.01, 2000)]).astype(np.float32)
    # every midpoint between adjacent codes (ties to the even code)
    vals = np.array([O.e4m3_value(c) for c in range(0x7F)])
    mids = ((vals[1:] + vals[:-1]) / 2).astype(np.float32)
    y = np.concatenate([y, mids, -mids])
    want = torch.from_numpy(y).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = np.array([O.e4m3_encode(v) for v in y], dtype=np.uint8)
    assert np.array_equal(got, want)


def test_e4m3_saturates():
    assert O.e4m3_encode(1e6) == 0x7E and O.e4m3_encode(-1e6) == 0xFE
    assert O.e4m3_encode(448.5) == 0x7E


def test_fp8_rows_scale_and_error():
    rng = np.random.default_rng(2)
    X = rng.normal(0, 3, size=(200, 100)).astype(np.float32)
    X[7] = 0
    codes, scales = O.fp8_encode_rows(X)
    assert scales[7] == 1.0 and np.all(codes[7] == 0)
    np.testing.assert_array_equal(scales[:7], (np.abs(X[:7]).max(1) / np.float32(448)).astype(np.float32))
    # the largest-magnitude element maps to +-448 exactly
    i = np.abs(X[3]).argmax()
    assert O.e4m3_value(codes[3, i]) in (448.0, -448.0)
    Y = O.fp8_decode_rows(codes, scales)
    nz = np.arange(200) != 7
    rel = np.abs(Y[nz] - X[nz]) / np.abs(X[nz]).max(1, keepdims=True)
    assert rel.max() <= 16.0 / 448.0 * 1.0001  # half a unit (32) in the top binade, over 448
    # decode = FP32 product of the scale and the code value
    assert Y[3, 5] == np.float32(np.float64(scales[3]) * O.e4m3_value(codes[3, 5]))


def _params(seed):
    rng = np.random.default_rng(seed)
    P = np.zeros(O.N_PARAMS)
    P[:1024] = rng.normal(0, 0.4, 1024)
    P[1024:1088] = rng.normal(0, 0.1, 64)
    P[1088:5184] = rng.normal(0, 0.15, 4096)
    P[5184:5248] = rng.normal(0, 0.1, 64)
    P[5248:5312] = rng.normal(0, 0.2, 64)
    P[5312] = 0.3
    return P


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    P = _params(4)
    X = rng.normal(size=(32, 16))
    T = rng.normal(size=32) * 2
    loss, G, _ = O.mlp_loss_grad(P, X, T)
    h = 1e-6
    idx = np.concatenate([rng.choice(1024, 40, replace=False), 1024 + np.arange(0, 64, 7),
                          1088 + rng.choice(4096, 60, replace=False), 5184 + np.arange(0, 64, 9),
                          5248 + np.arange(0, 64, 5), [5312]])
    for j in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[j] += h
        Pm[j] -= h
        num = (O.mlp_loss_grad(Pp, X, T)[0] - O.mlp_loss_grad(Pm, X, T)[0]) / (2 * h)
        assert abs(num - G[j]) <= 1e-6 * max(1.0, abs(num)), (j, num, G[j])


def test_mlp_forward_matches_torch_float64():
    rng = np.random.default_rng(5)
    P = _params(6)
    X = rng.normal(size=(64, 16))
    T = rng.normal(size=64)
    loss, G, Y = O.mlp_loss_grad(P, X, T)
    W1 = torch.tensor(P[:1024].reshape(64, 16), requires_grad=True)
    b1 = torch.tensor(P[1024:1088], requires_grad=True)
    W2 = torch.tensor(P[1088:5184].reshape(64, 64), requires_grad=True)
    b2 = torch.tensor(P[5184:5248], requires_grad=True)
    w3 = torch.tensor(P[5248:5312], requires_grad=True)
    b3 = torch.tensor(P[5312:5313], requires_grad=True)
    x = torch.tensor(X)
    y = torch.relu(torch.relu(x @ W1.T + b1) @ W2.T + b2) @ w3 + b3
    lt = ((y - torch.tensor(T)) ** 2).mean()
    lt.backward()
    np.testing.assert_allclose(Y, y.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert abs(loss - lt.item()) < 1e-12
    gt = np.concatenate([W1.grad.numpy().ravel(), b1.grad.numpy(), W2.grad.numpy().ravel(),
                         b2.grad.numpy(), w3.grad.numpy(), b3.grad.numpy()])
    np.testing.assert_allclose(G, gt, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("v", [0.0, 1.0, 4.0])
def test_mlp_zero_net_is_bias(v):
    P = np.zeros(O.N_PARAMS)
    P[5312] = v
    loss, G, Y = O.mlp_loss_grad(P, np.ones((3, 16)), np.zeros(3))
    assert np.all(Y == v) and loss == v * v
