"""Element-by-element parity of every U-Net kernel, layer by layer.

Each layer is checked on its own BF16 inputs, read back from the GPU
(ssn_read_tensor), so errors do not compound: the FP64 oracle (oracle/unet.py)
takes the GPU's BF16 input of a layer and its BF16 weights, and the GPU's
result must lie within a per-element bound derived from the arithmetic:
  * FP32 accumulation of K terms (products of BF16 numbers are exact in FP32):
    |error| <= gamma_K * sum |terms|, gamma_K = K 2^-24;
  * each rounding of a stored value to BF16 (round to nearest even, 8
    significant bits): |error| <= 2^-8 |value| (half an ulp, relative);
  * SiLU and SiLU' evaluated in FP32 with a fast exponential: 1e-5 relative.
Bounds are summed per element (the triangle inequality). Forward: pre-activation,
activation, pooling, upsampling and concatenation, head. Backward: head, weight and
bias gradients, backward-data passes (with the fused SiLU'), upsampling and pooling
backward. Shapes: the direct-operand kernels (large and one-wave blocks), the
LDS-tiled kernels, a channel count that is not a multiple of 32 (ragged output
blocks), and the production network (4 levels, widths 32..256, 128^2 image).
"""
import numpy as np
import pytest

from oracle import unet as U

pytestmark = pytest.mark.gpu

T_IN, T_Z, T_A, T_GZ, T_GD = 0, 1, 2, 3, 4
U32 = 2.0 ** -24
HALF_BF16 = 2.0 ** -8
SILU_EPS = 1e-5
TINY = 1e-30


def _bf16(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _check(name, got, ref, bound, stats):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    bad = err > bound
    assert not bad.any(), (f"{name}: {int(bad.sum())} of {bad.size} elements out of bound; worst "
                           f"err {err[bad].max():.3e} at bound {bound[bad][np.argmax(err[bad])]:.3e}")
    sig = np.abs(ref) > 1e-3 * max(np.abs(ref).max(), TINY)
    if sig.any():
        stats.append((name, float(np.median(bound[sig] / np.abs(ref[sig]))), float(np.median(err[sig] / np.abs(ref[sig])))))


def _layer_names(levels, base, cin, cout):
    shp = U.layer_shapes(levels, base, cin, cout)
    return [(shp[2 * k][0], shp[2 * k + 1][0]) for k in range((len(shp) - 2) // 2)]


def _net(ss, levels, base, N, H, seed):
    cin, cout = 2, 4
    rng = np.random.default_rng(seed)
    P = U.init_params(seed=seed, levels=levels, base=base, cin=cin, cout=cout)
    for k in P:
        if k.endswith(".b"):
            P[k] = 0.05 * rng.normal(size=P[k].shape)
    flat = np.concatenate([P[n].reshape(-1) for n, _ in U.layer_shapes(levels, base, cin, cout)]).astype(np.float32)
    net = ss.Net(levels=levels, base=base, cin=cin, cout=cout, N=N, H=H, W=H)
    net.set_weights(flat)
    x = rng.normal(size=(N, H, H, cin))
    t = rng.normal(size=(N, H, H, cout)) * 0.5
    return net, P, x, t


def _grads(net, levels, base):
    v = net.get_grads().astype(np.float64)
    out, o = {}, 0
    for name, shp in U.layer_shapes(levels, base, 2, 4):
        k = int(np.prod(shp))
        out[name] = v[o:o + k].reshape(shp)
        o += k
    return out


def _run_layers(ss, levels, base, N, H, seed):
    net, P, x, t = _net(ss, levels, base, N, H, seed)
    out = net.forward(x).cpu().numpy().astype(np.float64)
    net.backward(t)
    G = _grads(net, levels, base)
    names = _layer_names(levels, base, 2, 4)
    L = levels - 1
    R = lambda kind, k: net.read_tensor(kind, k).astype(np.float64)
    stats = []
    enc_a = lambda l: 2 * l
    enc_b = lambda l: 2 * l + 1
    mid_a, mid_b = 2 * L, 2 * L + 1
    dec_a = lambda l: 2 * L + 2 + 2 * (L - 1 - l)
    dec_b = lambda l: dec_a(l) + 1
    # ------------------------------------------------------------ forward
    for k, (wn, bn) in enumerate(names):
        w = _bf16(_f32(P[wn]))
        b = _f32(P[bn])
        xin = R(T_IN, k)[..., :w.shape[3]]  # layer 0's input is padded to 16 channels
        z_ref = U.conv3x3(xin, w, b)
        S = U.conv3x3(np.abs(xin), np.abs(w), np.abs(b))
        g = (9 * w.shape[3] + 1) * U32 * S
        _check(f"z[{k}]", R(T_Z, k), z_ref, g + HALF_BF16 * (np.abs(z_ref) + g) + TINY, stats)
        a_ref = U.silu(z_ref)
        ga = 1.1 * g + SILU_EPS * np.abs(a_ref)
        _check(f"a[{k}]", R(T_A, k), a_ref, ga + HALF_BF16 * (np.abs(a_ref) + ga) + TINY, stats)
    for l in range(L):  # pooling: FP32 sums of 4 BF16 values, rounded once
        skip = R(T_A, enc_b(l))
        nxt = enc_a(l + 1) if l + 1 < L else mid_a
        p_ref = U.avgpool2(skip)
        _check(f"pool[{l}]", R(T_IN, nxt), p_ref, HALF_BF16 * np.abs(p_ref) + 4 * U32 * U.avgpool2(np.abs(skip)) + TINY,
               stats)
    for l in range(L):  # upsampling and concatenation move bits
        prev = R(T_A, mid_b) if l == L - 1 else R(T_A, dec_b(l + 1))
        cat = R(T_IN, dec_a(l))
        cn = prev.shape[-1]
        assert np.array_equal(cat[..., :cn], U.upsample2(prev)), f"upsample[{l}]"
        assert np.array_equal(cat[..., cn:], R(T_A, enc_b(l))), f"concat[{l}]"
    hw, hb = _f32(P["head.w"]), _f32(P["head.b"])
    top = R(T_A, dec_b(0))
    o_ref = U.conv1x1(top, hw, hb)
    So = U.conv1x1(np.abs(top), np.abs(hw), np.abs(hb))
    _check("head", out, o_ref, (top.shape[-1] + 1) * U32 * So + U32 * np.abs(o_ref) + TINY, stats)
    # ------------------------------------------------------------ backward
    t32 = _f32(t)  # the GPU holds the target in FP32
    nout = out.size
    gout = 2.0 * (out - t32) / nout  # the GPU forms it in FP32 from the same output
    gout_err = 3 * U32 * np.abs(gout)  # a difference, a product and a quotient, each rounded once
    cz = np.zeros(hw.shape[1])
    ztop = R(T_Z, dec_b(0))
    gh = U.conv1x1(gout, hw.T.copy(), cz)
    Sh = U.conv1x1(np.abs(gout), np.abs(hw).T.copy(), cz)
    Eh = U.conv1x1(gout_err, np.abs(hw).T.copy(), cz)
    ref = U.silu_grad(ztop) * gh
    bnd = 1.1 * (hw.shape[0] * U32 * Sh + Eh) + SILU_EPS * np.abs(ref)
    _check("head_bwd", R(T_GZ, dec_b(0)), ref, bnd + HALF_BF16 * (np.abs(ref) + bnd) + TINY, stats)
    # head weight and bias gradients (FP32 sums over pixels)
    npix = top.shape[0] * top.shape[1] * top.shape[2]
    gw_ref = np.einsum("nhwo,nhwi->oi", gout, top)
    bw = 2 * npix * U32 * np.einsum("nhwo,nhwi->oi", np.abs(gout), np.abs(top)) + np.einsum(
        "nhwo,nhwi->oi", gout_err, np.abs(top))
    _check("head.w grad", G["head.w"], gw_ref, bw + TINY, stats)
    gb_ref = gout.sum(axis=(0, 1, 2))
    bb = 2 * npix * U32 * np.abs(gout).sum(axis=(0, 1, 2)) + gout_err.sum(axis=(0, 1, 2))
    _check("head.b grad", G["head.b"], gb_ref, bb + TINY, stats)
    for k, (wn, bn) in enumerate(names):
        w = _bf16(_f32(P[wn]))
        gz = R(T_GZ, k)
        xin = R(T_IN, k)[..., :w.shape[3]]
        gx_ref, gw_ref, gb_ref = U.conv3x3_backward(xin, w, gz)
        _, Sw, Sb = U.conv3x3_backward(np.abs(xin), np.abs(w), np.abs(gz))
        P_ = gz.shape[0] * gz.shape[1] * gz.shape[2]
        _check(f"w grad[{k}]", G[wn], gw_ref, 2 * P_ * U32 * Sw + TINY, stats)
        _check(f"b grad[{k}]", G[bn], gb_ref, 2 * P_ * U32 * Sb + TINY, stats)
        if k == 0:
            continue
        Sx, _, _ = U.conv3x3_backward(np.abs(xin), np.abs(w), np.abs(gz))
        gsum = (9 * w.shape[0]) * U32 * Sx
        second = (k % 2) == 1
        got = R(T_GD, k)
        if second:  # fused SiLU' of the pair's first layer
            sg = U.silu_grad(R(T_Z, k - 1))
            ref = sg * gx_ref
            bnd = 1.1 * gsum + SILU_EPS * np.abs(ref)
        else:
            ref, bnd = gx_ref, gsum
        if k in [dec_a(l) for l in range(L)]:  # the skip half was overwritten by the encoder's backward
            cn = got.shape[-1] - R(T_A, enc_b([l for l in range(L) if dec_a(l) == k][0])).shape[-1]
            got, ref, bnd = got[..., :cn], ref[..., :cn], bnd[..., :cn]
        _check(f"bwd data[{k}]", got, ref, bnd + HALF_BF16 * (np.abs(ref) + bnd) + TINY, stats)
    # upsampling backward (+ SiLU') into the level below
    for l in range(L):
        gcat = R(T_GD, dec_a(l))
        dst_layer = mid_b if l == L - 1 else dec_b(l + 1)
        cn = R(T_A, dst_layer).shape[-1]
        s4 = U.upsample2_backward(gcat[..., :cn])
        ref = U.silu_grad(R(T_Z, dst_layer)) * s4
        bnd = 4 * U32 * U.upsample2_backward(np.abs(gcat[..., :cn])) * 1.1 + HALF_BF16 * 1.1 * np.abs(s4)
        bnd = bnd + SILU_EPS * np.abs(ref)
        _check(f"up bwd[{l}]", R(T_GZ, dst_layer), ref, bnd + HALF_BF16 * (np.abs(ref) + bnd) + TINY, stats)
    # pooling backward + the skip half of the decoder's backward-data, then SiLU'
    for l in range(L):
        w = _bf16(_f32(P[names[dec_a(l)][0]]))
        gz = R(T_GZ, dec_a(l))
        cat_in = R(T_IN, dec_a(l))
        gx_ref, _, _ = U.conv3x3_backward(cat_in, w, gz)
        Sx, _, _ = U.conv3x3_backward(np.abs(cat_in), np.abs(w), np.abs(gz))
        cn = cat_in.shape[-1] - R(T_A, enc_b(l)).shape[-1]
        A, SA = gx_ref[..., cn:], (9 * w.shape[0]) * U32 * Sx[..., cn:]
        gp = R(T_GD, enc_a(l + 1)) if l + 1 < L else R(T_GD, mid_a)
        q = U.avgpool2_backward(gp)  # gP / 4 spread over 2x2 (exact in FP32; rounded to BF16 once)
        s = A + q
        e_s = SA + HALF_BF16 * (np.abs(A) + SA) + HALF_BF16 * np.abs(q) + HALF_BF16 * (np.abs(s) + SA + HALF_BF16 * (np.abs(A) + np.abs(q)))
        ref = U.silu_grad(R(T_Z, enc_b(l))) * s
        bnd = 1.1 * e_s + SILU_EPS * np.abs(ref)
        _check(f"pool bwd[{l}]", R(T_GZ, enc_b(l)), ref, bnd + HALF_BF16 * (np.abs(ref) + bnd) + TINY, stats)
    net.close()
    return stats


def _report(stats):
    worst = max(stats, key=lambda s: s[2])
    loosest = max(stats, key=lambda s: s[1])
    print(f"[unet layers] {len(stats)} checks; worst median relative error {worst[2]:.2e} ({worst[0]}); "
          f"loosest median bound {loosest[1]:.2e} ({loosest[0]})", flush=True)
    # the bounds are tight enough to see a wrong tap or channel block (O(1) relative)
    assert loosest[1] < 0.05


@pytest.mark.parametrize("shape", ["1", "2", "3"])
def test_every_layer_element_by_element(ss_net, shape, monkeypatch):
    """levels 3, base 16, two 64^2 images, with each convolution launch shape forced
    (1: direct 4-wave blocks, 2: direct one-wave blocks, 3: LDS-tiled)."""
    monkeypatch.setenv("SSN_CONV_SHAPE", shape)
    _report(_run_layers(ss_net, 3, 16, 2, 64, seed=3))


def test_ragged_channel_blocks_element_by_element(ss_net):
    """48 base channels (96, 192 below): output channel blocks of 32 end part-way."""
    _report(_run_layers(ss_net, 2, 48, 1, 64, seed=5))


def test_production_network_element_by_element(ss_net):
    """The learned start's network (4 levels, widths 32..256, concatenations of up to
    384 channels) on one 128^2 image, launch shapes chosen by problem size."""
    _report(_run_layers(ss_net, 4, 32, 1, 128, seed=7))


@pytest.fixture(scope="module")
def ss_net():
    import torch
    assert torch.cuda.is_available()
    import paper_2603_24370_amd as m
    m.lib()
    return m
