"""Orchestration of the learned control variate through the C ABI.

The sequence (every computation runs in libpdd's kernels; this module only
sequences calls and marshals tensors):
  1. plain float32 assembly of G, b and the solve for the knot values u0;
  2. training pairs (path point, tail score) from the first paths of every
     knot, scored with u0 at the exits (pdd_collect_training);
  3. Adam on the 2-64-64-1 network from seeded Glorot weights (pdd_mlp_train);
  4. optionally grad v baked into a table (pdd_mlp_bake_grad_lut).
"""
import time

import numpy as np

from . import pdd, workloads


def fit(ctx, w, u0, paths_per_knot=256, points_per_path=32, epochs=8, batch=256, lr=3e-3, seed=0, lut=None):
    """Train the control-variate network on pathwise estimates of workload w.

    Returns (params tensor, info dict with the number of pairs, the loss
    history and the GPU time of collection and training in milliseconds)."""
    torch = ctx.torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(ctx.stream)
    xy, t = ctx.collect(w, u0, paths_per_knot, points_per_path, lut=lut)
    ev[1].record(ctx.stream)
    valid = torch.nonzero(~torch.isnan(t)).flatten()
    n_pairs = int(valid.numel())
    xy, t = xy.index_select(0, valid).contiguous(), t.index_select(0, valid).contiguous()
    order = torch.from_numpy(workloads.minibatch_order(n_pairs, epochs, seed)).to(ctx.device)
    steps = order.numel() // batch
    params = torch.from_numpy(workloads.mlp_init(seed).astype(np.float32)).to(ctx.device)
    m = torch.zeros_like(params)
    s = torch.zeros_like(params)
    t0 = time.perf_counter()
    ev_t = torch.cuda.Event(enable_timing=True)
    ev_t.record(ctx.stream)
    losses = ctx.mlp_train(params, m, s, xy, t, order, batch, steps, 0, lr)
    ev[2].record(ctx.stream)
    ev[2].synchronize()
    info = dict(pairs=n_pairs, steps=steps, losses=losses.cpu().numpy(),
                collect_ms=ev[0].elapsed_time(ev[1]), train_ms=ev_t.elapsed_time(ev[2]),
                wall_s=time.perf_counter() - t0)
    return params, info
