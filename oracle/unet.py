"""FP64 NumPy oracle of the learned initialiser's network (test infrastructure only).

The network is a U-Net (Ronneberger, Fischer and Brox 2015) with `levels`
resolution levels and `base` channels at the top, doubling per level:
  encoder level l:  conv3x3 -> SiLU -> conv3x3 -> SiLU   (kept as skip_l), then 2x2 average pool
  bottleneck:       conv3x3 -> SiLU -> conv3x3 -> SiLU
  decoder level l:  nearest 2x upsample, concatenate [upsampled, skip_l] along channels,
                    conv3x3 -> SiLU -> conv3x3 -> SiLU
  head:             1x1 conv to `cout` channels (no activation)
Convolutions are 'same' (zero padding 1), with bias. Activations are NHWC; a
3x3 kernel is stored as w[co, ky, kx, ci] (ky, kx = 0..2 for offsets -1..1).

Every function is written for reading, not speed; backward passes apply the
chain rule to each forward step in reverse order. Pins: tests check the
backward against central differences and complex steps of the forward, and
the adjoint identities <A x, y> = <x, A^T y> of each linear piece.
"""
from __future__ import annotations

import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def conv3x3(x, w, b):
    """x: (N, H, W, Ci), w: (Co, 3, 3, Ci), b: (Co,) -> (N, H, W, Co)."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci), dtype=x.dtype)
    xp[:, 1:H + 1, 1:W + 1, :] = x
    out = np.zeros((N, H, W, w.shape[0]), dtype=np.result_type(x, w))
    for ky in range(3):
        for kx in range(3):
            out += xp[:, ky:ky + H, kx:kx + W, :] @ w[:, ky, kx, :].T
    return out + b


def conv3x3_backward(x, w, gout):
    """Gradients of conv3x3 w.r.t. x, w, b given gout = dL/d(out)."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci), dtype=x.dtype)
    xp[:, 1:H + 1, 1:W + 1, :] = x
    gxp = np.zeros_like(xp, dtype=np.result_type(x, gout))
    gw = np.zeros_like(w, dtype=np.result_type(w, gout))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + H, kx:kx + W, :]
            gw[:, ky, kx, :] = np.einsum("nhwo,nhwi->oi", gout, patch)
            gxp[:, ky:ky + H, kx:kx + W, :] += gout @ w[:, ky, kx, :]
    gb = gout.sum(axis=(0, 1, 2))
    return gxp[:, 1:H + 1, 1:W + 1, :], gw, gb


def conv1x1(x, w, b):
    """x: (N, H, W, Ci), w: (Co, Ci)."""
    return x @ w.T + b


def conv1x1_backward(x, w, gout):
    return gout @ w, np.einsum("nhwo,nhwi->oi", gout, x), gout.sum(axis=(0, 1, 2))


def avgpool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_backward(gout):
    return np.repeat(np.repeat(gout, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_backward(gout):
    N, H, W, C = gout.shape
    return gout.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def layer_shapes(levels=4, base=32, cin=2, cout=4):
    """Ordered list of (name, shape) of all parameters."""
    shapes = []
    ch = [base * (2 ** l) for l in range(levels)]
    c_prev = cin
    for l in range(levels - 1):
        shapes += [(f"enc{l}a.w", (ch[l], 3, 3, c_prev)), (f"enc{l}a.b", (ch[l],)),
                   (f"enc{l}b.w", (ch[l], 3, 3, ch[l])), (f"enc{l}b.b", (ch[l],))]
        c_prev = ch[l]
    L = levels - 1
    shapes += [("mid.a.w", (ch[L], 3, 3, c_prev)), ("mid.a.b", (ch[L],)),
               ("mid.b.w", (ch[L], 3, 3, ch[L])), ("mid.b.b", (ch[L],))]
    c_prev = ch[L]
    for l in reversed(range(levels - 1)):
        shapes += [(f"dec{l}a.w", (ch[l], 3, 3, c_prev + ch[l])), (f"dec{l}a.b", (ch[l],)),
                   (f"dec{l}b.w", (ch[l], 3, 3, ch[l])), (f"dec{l}b.b", (ch[l],))]
        c_prev = ch[l]
    shapes += [("head.w", (cout, c_prev)), ("head.b", (cout,))]
    return shapes


def init_params(seed=0, levels=4, base=32, cin=2, cout=4):
    """He-uniform weights from a seeded generator, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, shp in layer_shapes(levels, base, cin, cout):
        if name.endswith(".b"):
            P[name] = np.zeros(shp)
        else:
            fan_in = int(np.prod(shp[1:]))
            lim = np.sqrt(6.0 / fan_in)
            P[name] = rng.uniform(-lim, lim, size=shp)
    return P


def forward(P, x, levels=4):
    """Returns (output, cache) for x of shape (N, H, W, cin)."""
    cache = {"x": x}
    h = x
    skips = []
    for l in range(levels - 1):
        za = conv3x3(h, P[f"enc{l}a.w"], P[f"enc{l}a.b"]); a = silu(za)
        zb = conv3x3(a, P[f"enc{l}b.w"], P[f"enc{l}b.b"]); s = silu(zb)
        cache[f"enc{l}"] = (h, za, a, zb)
        skips.append(s)
        h = avgpool2(s)
    za = conv3x3(h, P["mid.a.w"], P["mid.a.b"]); a = silu(za)
    zb = conv3x3(a, P["mid.b.w"], P["mid.b.b"]); h2 = silu(zb)
    cache["mid"] = (h, za, a, zb)
    h = h2
    for l in reversed(range(levels - 1)):
        u = upsample2(h)
        cat = np.concatenate([u, skips[l]], axis=-1)
        za = conv3x3(cat, P[f"dec{l}a.w"], P[f"dec{l}a.b"]); a = silu(za)
        zb = conv3x3(a, P[f"dec{l}b.w"], P[f"dec{l}b.b"]); h2 = silu(zb)
        cache[f"dec{l}"] = (cat, za, a, zb, u.shape[-1])
        h = h2
    out = conv1x1(h, P["head.w"], P["head.b"])
    cache["head_in"] = h
    return out, cache


def backward(P, cache, gout, levels=4):
    """Gradients of a scalar loss with dL/d(out) = gout, for every parameter."""
    G = {}
    gh, G["head.w"], G["head.b"] = conv1x1_backward(cache["head_in"], P["head.w"], gout)
    gskips = {}
    for l in range(levels - 1):
        cat, za, a, zb, cu = cache[f"dec{l}"]
        gzb = gh * silu_grad(zb)
        ga, G[f"dec{l}b.w"], G[f"dec{l}b.b"] = conv3x3_backward(a, P[f"dec{l}b.w"], gzb)
        gza = ga * silu_grad(za)
        gcat, G[f"dec{l}a.w"], G[f"dec{l}a.b"] = conv3x3_backward(cat, P[f"dec{l}a.w"], gza)
        gskips[l] = gcat[..., cu:]
        gh = upsample2_backward(gcat[..., :cu])
    h_in, za, a, zb = cache["mid"]
    gzb = gh * silu_grad(zb)
    ga, G["mid.b.w"], G["mid.b.b"] = conv3x3_backward(a, P["mid.b.w"], gzb)
    gza = ga * silu_grad(za)
    gh, G["mid.a.w"], G["mid.a.b"] = conv3x3_backward(h_in, P["mid.a.w"], gza)
    for l in reversed(range(levels - 1)):
        h_in, za, a, zb = cache[f"enc{l}"]
        gs = avgpool2_backward(gh) + gskips[l]
        gzb = gs * silu_grad(zb)
        ga, G[f"enc{l}b.w"], G[f"enc{l}b.b"] = conv3x3_backward(a, P[f"enc{l}b.w"], gzb)
        gza = ga * silu_grad(za)
        gh, G[f"enc{l}a.w"], G[f"enc{l}a.b"] = conv3x3_backward(h_in, P[f"enc{l}a.w"], gza)
    G["input"] = gh
    return G


def mse(out, target):
    """Mean squared error over all elements, and its gradient."""
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(P, G, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in P:
        m = state.setdefault("m_" + k, np.zeros_like(P[k]))
        v = state.setdefault("v_" + k, np.zeros_like(P[k]))
        m[...] = beta1 * m + (1 - beta1) * G[k]
        v[...] = beta2 * v + (1 - beta2) * G[k] * G[k]
        mhat = m / (1 - beta1 ** t)
        vhat = v / (1 - beta2 ** t)
        P[k] -= lr * mhat / (np.sqrt(vhat) + eps)
