"""FP64 oracle of the small convolutional network that predicts a diagonal PCG preconditioner.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network (a project addition; the paper uses the analytic diagonal of App. B or
a stochastic estimate, Sec. 6):  L layers of 3x3 "same" convolutions with zero
padding, ReLU after every layer but the last.  Input: C_in feature maps on the
object grid; output: C_out maps r, the log of the object block of the GGN
diagonal relative to a per-problem scale s (the preconditioner is s * exp(r),
positive by construction; s is the largest entry of the App. B object diagonal,
so that only the scale, not the spatial shape, comes from the analytic formula).
Loss on a mask of illuminated pixels:
    L = sum_mask (r - t)^2 / (2 * count)
with t = log(d_exact / s).  Gradients are written out by the chain rule.

Parameter vector layout (shared with the GPU library by definition, not code):
for each layer l: W_l (C_out_l, C_in_l, 3, 3) row-major, then b_l (C_out_l).
"""
from __future__ import annotations

import numpy as np


def layer_shapes(cin: int, cmid: int, cout: int, layers: int):
    chans = [cin] + [cmid] * (layers - 1) + [cout]
    return [(chans[i + 1], chans[i]) for i in range(layers)]


def param_count(cin, cmid, cout, layers) -> int:
    return sum(co * ci * 9 + co for co, ci in layer_shapes(cin, cmid, cout, layers))


def unpack(params: np.ndarray, cin, cmid, cout, layers):
    out, o = [], 0
    for co, ci in layer_shapes(cin, cmid, cout, layers):
        W = params[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = params[o:o + co]
        o += co
        out.append((W, b))
    return out


def init_params(rng, cin, cmid, cout, layers) -> np.ndarray:
    """He-normal weights, zero biases; the last layer starts at zero (r = 0: d_paper)."""
    parts = []
    shapes = layer_shapes(cin, cmid, cout, layers)
    for i, (co, ci) in enumerate(shapes):
        if i == len(shapes) - 1:
            W = np.zeros((co, ci, 3, 3))
        else:
            W = rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (ci * 9))
        parts += [W.ravel(), np.zeros(co)]
    return np.concatenate(parts)


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[n,o,i,j] = b[o] + sum_{c,u,v} W[o,c,u,v] x[n,c,i+u-1,j+v-1] (zero outside)."""
    n, c, h, w = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    y = np.zeros((n, W.shape[0], h, w))
    for u in range(3):
        for v in range(3):
            y += np.einsum("oc,nchw->nohw", W[:, :, u, v], xp[:, :, u:u + h, v:v + w])
    return y + b[None, :, None, None]


def forward(params, x, cin, cmid, cout, layers, keep=False):
    acts = [x]
    a = x
    Ws = unpack(params, cin, cmid, cout, layers)
    for i, (W, b) in enumerate(Ws):
        z = conv3x3(a, W, b)
        a = np.maximum(z, 0.0) if i < len(Ws) - 1 else z
        acts.append(a)
    return (a, acts) if keep else a


def loss(params, x, t, mask, cin, cmid, cout, layers) -> float:
    r = forward(params, x, cin, cmid, cout, layers)
    cnt = max(float(mask.sum()), 1.0)
    return float(np.sum(mask * (r - t) ** 2) / (2.0 * cnt))


def grad(params, x, t, mask, cin, cmid, cout, layers):
    """(loss, dL/dparams) by reverse accumulation through the layers."""
    r, acts = forward(params, x, cin, cmid, cout, layers, keep=True)
    cnt = max(float(mask.sum()), 1.0)
    L = float(np.sum(mask * (r - t) ** 2) / (2.0 * cnt))
    Ws = unpack(params, cin, cmid, cout, layers)
    gz = mask * (r - t) / cnt                      # dL/dz of the last (linear) layer
    grads = [None] * len(Ws)
    for i in range(len(Ws) - 1, -1, -1):
        W, b = Ws[i]
        a_in = acts[i]
        n, c, h, w = a_in.shape
        ap = np.pad(a_in, ((0, 0), (0, 0), (1, 1), (1, 1)))
        gW = np.zeros_like(W)
        for u in range(3):
            for v in range(3):
                gW[:, :, u, v] = np.einsum("nohw,nchw->oc", gz, ap[:, :, u:u + h, v:v + w])
        gb = gz.sum(axis=(0, 2, 3))
        grads[i] = (gW, gb)
        if i > 0:
            # d a_in = correlation of gz with the flipped kernel, channels transposed
            gzp = np.pad(gz, ((0, 0), (0, 0), (1, 1), (1, 1)))
            ga = np.zeros_like(a_in)
            for u in range(3):
                for v in range(3):
                    ga += np.einsum("oc,nohw->nchw", W[:, :, 2 - u, 2 - v], gzp[:, :, u:u + h, v:v + w])
            gz = ga * (acts[i] > 0.0)             # ReLU of layer i-1
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, flat


def adam(params, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def features(P, pos, obj_shape) -> np.ndarray:
    """The network's 3 input maps on the object grid (illumination overlap, overlap-weighted
    |P|^2, overlap-weighted arg P), each normalised as in the GPU library's definition:
    f0 = ov / max ov, f1 = (sum S^T|P|^4 / ov) / max|P|^2, f2 = (sum S^T(|P|^2 arg P) / ov) / pi."""
    from .ptycho import extract_adjoint
    K = len(pos)
    q = np.abs(P) ** 2
    ov = extract_adjoint(np.broadcast_to(q[None], (K,) + P.shape), pos, obj_shape)
    s4 = extract_adjoint(np.broadcast_to((q * q)[None], (K,) + P.shape), pos, obj_shape)
    sp = extract_adjoint(np.broadcast_to((q * np.angle(P))[None], (K,) + P.shape), pos, obj_shape)
    with np.errstate(invalid="ignore", divide="ignore"):
        f1 = np.where(ov > 0, s4 / ov, 0.0) / q.max()
        f2 = np.where(ov > 0, sp / ov, 0.0) / np.pi
    return np.stack([ov / ov.max(), f1, f2])


def learned_scale(dO_paper) -> float:
    """s: the largest entry of the App. B object diagonal (both real coordinates)."""
    return float(np.max(dO_paper))


def target(d_exact, dO_paper, floor=1e-6) -> np.ndarray:
    """Training target t = log(d / s) of the network, (2, ny, nx): the exact object diagonal d
    (real coordinates on the last axis, floored at floor * its largest entry as the LM floors
    its diagonals) relative to the scale s of ``learned_scale``."""
    d = np.maximum(d_exact, floor * d_exact.max())
    t = np.log(d / learned_scale(dO_paper))
    return np.stack([t[..., 0], t[..., 1]])


def learned_diag(dO_paper, dP_paper, r, floor=1e-6):
    """Learned PCG diagonal: object part s * exp(r) with r clamped to [log(floor), 2] (so the
    floor of the LM's diagonals holds) and s = ``learned_scale(dO_paper)``; the probe part
    stays the App. B one floored at floor * its block maximum.  With r = 0 (an untrained
    network, whose last layer starts at zero) the object part is the constant s.  Returns the
    flat (n, 2) real-coordinate diagonal (object entries, then probe)."""
    rr = np.clip(r, np.log(floor), 2.0)
    dO = learned_scale(dO_paper) * np.exp(np.stack([rr[0], rr[1]], axis=-1))
    parts = [dO.reshape(-1, 2)]
    if dP_paper is not None:
        parts.append(np.maximum(dP_paper, floor * dP_paper.max()).reshape(-1, 2))
    return np.concatenate(parts, axis=0)
