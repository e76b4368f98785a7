"""Learned diagonal PCG preconditioner: training data, training loop and evaluation helpers.

Everything runs through the library's HIP kernels:
* samples come from LM runs (D = Dg(G), Jacobi PCG) on seeded proxies of the joint
  512x512 / 128x128 workload (same probe recipe and scan step, 256x256 object, 8x8
  raster); at every iterate the input maps are ``ptlm_cnn_features`` and the target is
  t = log(d_exact / d_paper) on illuminated object pixels (``ptlm_diag`` exact and App. B);
* training is Adam on the masked squared error with ``ptlm_cnn_loss_grad`` /
  ``ptlm_cnn_adam``.

    python -m paper_2103_01767_amd.learned train [--problems 40 --iters 5 --steps 400]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

import paper_2103_01767_amd as pt

HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(HERE, "data", "cnn_params.npy")
META_PATH = os.path.join(HERE, "data", "cnn_params.json")
ARCH = dict(cin=3, cmid=32, cout=2, layers=4)


def proxy(seed: int):
    import synth
    return synth.make_scaled("proxy%d" % seed, 50000 + seed, 256, 128, 8, 8, 36, 1, 40.0, 1e4, 4.0, T=10)


def _c64(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)


def poisson_data(prob, pr, seed, dev):
    zeta = prob.forward(_c64(pr.O_true, dev), _c64(pr.P_true, dev))
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    return torch.poisson((zeta.double() ** 2).float(), generator=g).contiguous()


def target_from_diagonals(d_exact, d_paper, floor=1e-6):
    """(2, ny, nx) log ratio of floored exact and App. B diagonals (object part)."""
    e = torch.clamp(d_exact, min=floor * float(d_exact.max()))
    p = torch.clamp(d_paper, min=floor * float(d_paper.max()))
    return torch.log(e / p).permute(2, 0, 1).contiguous()


def samples_from_run(pr, iters, dev, seed=0):
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, metric="gauss", mode="joint",
                      background=pr.background, device=dev)
    y = poisson_data(prob, pr, seed, dev)
    O, P = _c64(pr.O_init, dev), _c64(pr.P_init, dev)
    params = pt.default_params(scaling=1, precond=1)
    st = prob.new_state()
    prob.lm_init(params, st)
    out = []
    for _ in range(iters):
        prob.linearize(O, P, y)
        feat = pt.cnn_features(prob)
        d_ex, _ = prob.diag(exact=True)
        d_pa, _ = prob.diag(exact=False)
        t = target_from_diagonals(d_ex, d_pa)
        mask = (feat[0:1] > 0.05).float().expand(2, -1, -1).contiguous()
        out.append((feat, t, mask))
        prob.lm_step(O, P, y, params, st)
    return out


def build_samples(n_problems, iters, dev):
    samples = []
    for p in range(n_problems):
        samples += samples_from_run(proxy(p), iters, dev, seed=p)
    return samples


def he_params(seed, dev):
    """He-normal hidden weights, zero biases, zero last layer (r = 0: the App. B diagonal)."""
    rng = np.random.default_rng(seed)
    chans = [ARCH["cin"]] + [ARCH["cmid"]] * (ARCH["layers"] - 1) + [ARCH["cout"]]
    parts = []
    for i in range(ARCH["layers"]):
        ci, co = chans[i], chans[i + 1]
        W = (np.zeros((co, ci, 3, 3)) if i == ARCH["layers"] - 1
             else rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (ci * 9)))
        parts += [W.ravel(), np.zeros(co)]
    return torch.from_numpy(np.concatenate(parts).astype(np.float32)).to(dev)


def train_cnn(samples, steps=400, batch=4, lr=2e-3, seed=0, dev="cuda", log=None):
    """Adam on minibatches of samples; returns (network, loss history)."""
    n = len(samples)
    h, w = samples[0][0].shape[1:]
    batch = min(batch, n)
    cnn = pt.Cnn(batch, h, w, device=dev, params=he_params(seed, dev), **ARCH)
    gen = torch.Generator()
    gen.manual_seed(seed)
    hist = []
    for s in range(steps):
        idx = torch.randperm(n, generator=gen)[:batch].tolist()
        x = torch.stack([samples[i][0] for i in idx]).contiguous()
        t = torch.stack([samples[i][1] for i in idx]).contiguous()
        m = torch.stack([samples[i][2] for i in idx]).contiguous()
        loss, g = cnn.loss_grad(x, t, m)
        cnn.adam(g, lr=lr)
        if s % 20 == 0 or s == steps - 1:
            hist.append((s, float(loss.item())))
            if log:
                log("step %d loss %.5f" % hist[-1])
    return cnn, hist


def mean_loss(cnn_params, samples, dev="cuda"):
    h, w = samples[0][0].shape[1:]
    net = pt.Cnn(1, h, w, device=dev, params=cnn_params, **ARCH)
    tot = 0.0
    for x, t, m in samples:
        loss, _ = net.loss_grad(x[None].contiguous(), t[None].contiguous(), m[None].contiguous())
        tot += float(loss.item())
    return tot / len(samples)


def lm_net(cnn_params, obj_shape, dev="cuda"):
    """Network instance for an LM on an object grid of ``obj_shape`` (fully convolutional)."""
    return pt.Cnn(1, obj_shape[0], obj_shape[1], device=dev, params=cnn_params, **ARCH)


def save(params, meta):
    os.makedirs(os.path.dirname(PARAMS_PATH), exist_ok=True)
    np.save(PARAMS_PATH, params.detach().cpu().numpy().astype(np.float32))
    json.dump(meta, open(META_PATH, "w"), indent=1)


def load(dev="cuda"):
    return torch.from_numpy(np.load(PARAMS_PATH)).to(dev)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--problems", type=int, default=40)
    ap.add_argument("--iters", type=int, default=5)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    a = ap.parse_args()
    dev = torch.device("cuda:0")
    t0 = time.time()
    train_s = build_samples(a.problems, a.iters, dev)
    held = []
    for p in range(1000, 1004):
        held += samples_from_run(proxy(p), a.iters, dev, seed=p)
    t1 = time.time()
    print("samples %d (+%d held out) in %.1fs" % (len(train_s), len(held), t1 - t0), flush=True)
    base = mean_loss(he_params(0, dev), held, dev)
    cnn, hist = train_cnn(train_s, a.steps, a.batch, a.lr, dev=dev, log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    t2 = time.time()
    held_loss = mean_loss(cnn.params, held, dev)
    meta = {"arch": ARCH, "problems": a.problems, "iters": a.iters, "steps": a.steps, "batch": a.batch,
            "lr": a.lr, "train_seconds": round(t2 - t1, 2), "sample_seconds": round(t1 - t0, 2),
            "heldout_loss_untrained": base, "heldout_loss": held_loss, "history": hist}
    save(cnn.params, meta)
    print(json.dumps({k: v for k, v in meta.items() if k != "history"}), flush=True)


if __name__ == "__main__":
    main()
