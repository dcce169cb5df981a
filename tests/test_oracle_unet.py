"""Pins of the FP64 U-Net oracle: brute-force convolution, adjoint identities,
complex-step gradients of the whole network, and the Adam update in closed form."""
import numpy as np
import pytest

from oracle import unet as U


def test_conv3x3_matches_brute_force_sum():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 6, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = U.conv3x3(x, w, b)
    N, H, W, Ci = x.shape
    for n in range(N):
        for i in range(H):
            for j in range(W):
                for o in range(4):
                    acc = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            ii, jj = i + ky - 1, j + kx - 1
                            if 0 <= ii < H and 0 <= jj < W:
                                acc += np.dot(w[o, ky, kx], x[n, ii, jj])
                    assert abs(acc - y[n, i, j, o]) < 1e-12


def test_adjoint_identities():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 8, 6, 3))
    w = rng.normal(size=(5, 3, 3, 3))
    y = rng.normal(size=(2, 8, 6, 5))
    gx, gw, gb = U.conv3x3_backward(x, w, y)
    # <conv(x), y> = <x, conv^T y> = <w, dconv/dw^T y>  (bias off)
    lhs = np.sum(U.conv3x3(x, w, np.zeros(5)) * y)
    assert lhs == pytest.approx(np.sum(x * gx), rel=1e-12)
    assert lhs == pytest.approx(np.sum(w * gw), rel=1e-12)
    assert gb == pytest.approx(y.sum(axis=(0, 1, 2)))
    p = rng.normal(size=(2, 4, 3, 3))
    assert np.sum(U.avgpool2(x) * p) == pytest.approx(np.sum(x * U.avgpool2_backward(p)), rel=1e-12)
    q = rng.normal(size=(2, 16, 12, 3))
    assert np.sum(U.upsample2(x) * q) == pytest.approx(np.sum(x * U.upsample2_backward(q)), rel=1e-12)
    w1 = rng.normal(size=(4, 3))
    y1 = rng.normal(size=(2, 8, 6, 4))
    g1x, g1w, _ = U.conv1x1_backward(x, w1, y1)
    l1 = np.sum(U.conv1x1(x, w1, np.zeros(4)) * y1)
    assert l1 == pytest.approx(np.sum(x * g1x), rel=1e-12)
    assert l1 == pytest.approx(np.sum(w1 * g1w), rel=1e-12)


def _loss(P, x, t, levels):
    out, _ = U.forward(P, x, levels)
    d = out - t
    return np.mean(d * d)


@pytest.mark.parametrize("levels", [2, 3])
def test_network_gradient_matches_complex_step(levels):
    rng = np.random.default_rng(2)
    P = U.init_params(seed=3, levels=levels, base=4, cin=2, cout=3)
    for k in P:
        if k.endswith(".b"):
            P[k] = 0.1 * rng.normal(size=P[k].shape)
    H = 2 ** levels * 2
    x = rng.normal(size=(2, H, H, 2))
    t = rng.normal(size=(2, H, H, 3))
    out, cache = U.forward(P, x, levels)
    _, g = U.mse(out, t)
    G = U.backward(P, cache, g, levels)
    eps = 1e-30
    for name in P:
        flat = P[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            Pc = {k: v.astype(complex) for k, v in P.items()}
            Pc[name].reshape(-1)[idx] += 1j * eps
            d = _loss(Pc, x.astype(complex), t, levels).imag / eps
            assert d == pytest.approx(G[name].reshape(-1)[idx], rel=1e-9, abs=1e-13), (name, idx)
    # input gradient too
    xc = x.astype(complex)
    xc[1, 3, 2, 1] += 1j * eps
    d = _loss({k: v.astype(complex) for k, v in P.items()}, xc, t, levels).imag / eps
    assert d == pytest.approx(G["input"][1, 3, 2, 1], rel=1e-9, abs=1e-13)


def test_adam_first_step_closed_form():
    P = {"w": np.array([1.0, -2.0, 0.5])}
    G = {"w": np.array([0.3, -4.0, 1e-3])}
    st = {}
    U.adam_step(P, G, st, lr=0.01)
    # first step: m_hat = g, v_hat = g^2, so the update is lr * g / (|g| + eps)
    want = np.array([1.0, -2.0, 0.5]) - 0.01 * G["w"] / (np.abs(G["w"]) + 1e-8)
    assert np.allclose(P["w"], want, rtol=0, atol=1e-15)
    assert st["t"] == 1


def test_silu_hand_values():
    """SiLU z / (1 + e^-z) (Elfwing, Uchibe and Doya 2018) at points worked by hand:
    0 at 0; ln 2 / (1 + 1/2) at z = ln 2; -ln 2 / 3 at z = -ln 2 (e^{ln 2} = 2);
    z -> z for large z, -> 0 for very negative z."""
    ln2 = np.log(2.0)
    z = np.array([0.0, ln2, -ln2, 50.0, -50.0])
    want = np.array([0.0, ln2 / 1.5, -ln2 / 3.0, 50.0, 0.0])
    got = U.silu(z)
    assert np.abs(got - want).max() < 1e-15 * 50 + 1e-20
    assert abs(got[4]) < 1e-19  # -50 e^-50
    # derivative at 0 is 1/2 (s = 1/2, 1 + 0) and at ln 2: s = 2/3, 2/3 (1 + ln2/3)
    assert U.silu_grad(np.array([0.0]))[0] == 0.5
    assert U.silu_grad(np.array([ln2]))[0] == pytest.approx(2.0 / 3.0 * (1.0 + ln2 / 3.0), rel=1e-15)


def test_avgpool_and_upsample_hand_values():
    """2x2 average pooling and nearest upsampling of small arrays worked by hand."""
    x = np.arange(16.0).reshape(1, 4, 4, 1)  # rows 0..3, 4..7, 8..11, 12..15
    pooled = U.avgpool2(x)[0, :, :, 0]
    assert pooled.tolist() == [[2.5, 4.5], [10.5, 12.5]]  # (0+1+4+5)/4, (2+3+6+7)/4, ...
    # two channels pool independently
    y = np.stack([x[..., 0], -2.0 * x[..., 0]], axis=-1)
    assert U.avgpool2(y)[0, :, :, 1].tolist() == [[-5.0, -9.0], [-21.0, -25.0]]
    up = U.upsample2(np.array([[1.0, 2.0], [3.0, 4.0]]).reshape(1, 2, 2, 1))[0, :, :, 0]
    assert up.tolist() == [[1, 1, 2, 2], [1, 1, 2, 2], [3, 3, 4, 4], [3, 3, 4, 4]]
    # pooling undoes upsampling
    assert np.array_equal(U.avgpool2(U.upsample2(x)), x)
