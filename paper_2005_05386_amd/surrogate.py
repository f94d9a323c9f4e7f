"""Training and loading of the learned crossing surrogate.

One network per bump shape maps a ray's entry on the bump's support sphere
(radius 3 sigma) to its exit point and direction, in the canonical frame
where a bump of amplitude a and width sigma becomes kappa exp(-|u|^2/2),
kappa = |a| / sigma (Sec. 5.1's graph metric, Eq. 5.4).  Every step runs in
the library's kernels: crossing data from the RK4 integrator, the MLP
forward and backward on the matrix cores, the MSE gradient, AdamW, the
calibration of per-bin error bounds.  This module only sequences the calls
and holds the hyper-parameters.

Training draws fresh crossings for every step (sin^2 of the entry angle
uniform, i.e. entry points uniform over the disc of impact parameters), so
`samples` is the number of distinct crossings each network sees.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import rt as _rt

MLP_PARAMS = _rt.MLP_PARAMS
_SIZES = [(256, 6), (256, 256), (256, 256), (6, 256)]


def init_params(n_nets, seed):
    """He-style uniform initialisation (fan-in bound sqrt(6 / fan_in), half
    of it for the output layer), zero biases; [n_nets, MLP_PARAMS] float32."""
    rng = np.random.default_rng(seed)
    p = np.zeros((n_nets, MLP_PARAMS), np.float32)
    for i in range(n_nets):
        k = 0
        for li, (o, fan) in enumerate(_SIZES):
            lim = math.sqrt(6.0 / fan) * (0.5 if li == 3 else 1.0)
            p[i, k:k + o * fan] = rng.uniform(-lim, lim, size=o * fan)
            k += o * fan + o
    return p


def shapes_of(bumps):
    """Distinct |a| / sigma of a bump list (rows a, cx, cy, cz, sigma) and the
    network index of every bump (-1 for a zero amplitude)."""
    b = np.asarray(bumps, np.float64).reshape(-1, 5)
    kap = np.abs(b[:, 0]) / b[:, 4]
    kap32 = kap.astype(np.float32)
    uniq = sorted({float(k) for k, a in zip(kap32, b[:, 0]) if a != 0.0})
    index = {k: i for i, k in enumerate(uniq)}
    net = np.array([index.get(float(k), -1) if a != 0.0 else -1 for k, a in zip(kap32, b[:, 0])], np.int32)
    return np.array(uniq, np.float32), net


@dataclass
class Surrogate:
    kappa: np.ndarray           # [n] shapes
    scale: np.ndarray           # [n] target scales
    params: object              # torch [n, P] float32 (master)
    w_bf16: object              # torch [n, P] bfloat16
    arc: object                 # torch [n, n_tab] arc length in units of sigma on the cos-theta grid
    err: object                 # torch [n, n_bins, 2] calibrated error bounds
    h: float = 0.01
    losses: list = field(default_factory=list)
    train_s: float = 0.0
    gen_s: float = 0.0
    steps: int = 0
    samples: int = 0

    def state(self):
        """Tensors and scalars for torch.save (load with weights_only=True)."""
        import torch
        return {"kappa": torch.tensor(self.kappa), "scale": torch.tensor(self.scale), "params": self.params.cpu(),
                "w_bf16": self.w_bf16.cpu(), "arc": self.arc.cpu(), "err": self.err.cpu(), "h": self.h,
                "steps": self.steps, "samples": self.samples}

    @staticmethod
    def from_state(d, device):
        return Surrogate(kappa=d["kappa"].numpy(), scale=d["scale"].numpy(), params=d["params"].to(device),
                         w_bf16=d["w_bf16"].to(device), arc=d["arc"].to(device), err=d["err"].to(device),
                         h=float(d["h"]), steps=int(d["steps"]), samples=int(d["samples"]))


def train(tracer, kappa, samples=10_000_000, batch=1024, h=0.01, lr=2e-3, lr_min=1e-5, warmup=200, seed=0,
          n_tab=4097, n_bins=64, n_cal=8192, log_every=500, log=None, sampling=0):
    """Train one network per shape in kappa (all in one grouped launch per
    layer) and calibrate it.  Returns a Surrogate."""
    import torch
    kappa = np.ascontiguousarray(kappa, np.float32)
    n = len(kappa)
    dev = torch.device("cuda", tracer.device)
    t0 = time.perf_counter()
    # target scale per shape from a pilot sample (scale 1)
    _, ypil, _ = tracer.surrogate_gen(kappa, np.ones(n, np.float32), 4096, h, grid=False, seed=seed ^ 0x5EED)
    ypil = ypil.cpu().numpy()
    scale = np.maximum(np.abs(ypil).reshape(n, -1).max(axis=1), 1e-6).astype(np.float32)

    params = torch.tensor(init_params(n, seed), device=dev)
    wb = params.to(torch.bfloat16)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    steps = max(1, (samples + batch - 1) // batch)
    log_every = min(log_every, steps)
    # the library runs the whole loop (data, forward, loss, backward, AdamW)
    loss_log, _work = tracer.surrogate_train(kappa, scale, params, wb, m, v, batch, steps, h=h, mode=sampling,
                                             seed=seed, lr=lr, lr_min=lr_min, warmup=warmup, log_every=log_every)
    tracer.sync()
    train_s = time.perf_counter() - t0
    # loss per network of every logged step (64 partial sums of squares each)
    sums = loss_log.cpu().numpy().astype(np.float64).sum(axis=1) / (batch * n)
    losses = [((i + 1) * log_every, float(v_)) for i, v_ in enumerate(sums)]
    if log:
        for st_, l_ in losses:
            log("surrogate step %d/%d loss/net %.3e" % (st_, steps, l_))
    gen_s = 0.0

    # calibration on a cos-theta grid; the arc table comes from the same grid
    xg, yg, auxg = tracer.surrogate_gen(kappa, scale, n_cal, h, grid=True)
    work_c = tracer.mlp_work(n, n_cal)
    pg = tracer.mlp_fwd(wb, params, xg, work_c)
    err = tracer.surrogate_calibrate(xg, pg, yg, scale, n_bins)
    if n_tab == n_cal:
        arc = auxg[:, :, 1].contiguous()
    else:
        _, _, auxt = tracer.surrogate_gen(kappa, scale, n_tab, h, grid=True)
        arc = auxt[:, :, 1].contiguous()
    tracer.sync()
    return Surrogate(kappa=kappa, scale=scale, params=params, w_bf16=wb, arc=arc, err=err, h=h, losses=losses,
                     train_s=train_s, gen_s=gen_s, steps=steps, samples=steps * batch)


def load(tracer, model, net_of_bump, tol=1e-3):
    """Give the trained networks to the tracer; net_of_bump maps every bump of
    the current metric to a network (-1: none)."""
    tracer.surrogate_load(model.w_bf16, model.params, model.scale, model.arc, model.err, net_of_bump, tol)
