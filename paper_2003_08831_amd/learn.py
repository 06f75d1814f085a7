"""Network proposing each element's first relaxation trial point.

The per-element root solve of the local relaxation (Sec. 2) is always run to
the same tolerance; the network only chooses the trial point that follows
phi_k(1).  This module logs training samples from locally relaxed steps,
trains the network and measures what it gains.  Feature logging, the
normalization, the gradient, the Adam update and the inference all run in the
library's kernels (esrk_set_step_model, esrk_mlp_prepare, esrk_mlp_grad,
esrk_mlp_adam, esrk_local_relaxation_solve_ml); torch only holds the buffers,
selects samples and gathers mini-batches.
"""
from __future__ import annotations

import torch

from . import esrk, inputs

NF = esrk.MLP_IN


def collect(ctx: esrk.Context, u: torch.Tensor, t: torch.Tensor, nsteps: int, model=None):
    """Advance u (in place) by nsteps CFL steps and log (features, gamma_k).

    Returns the raw features (float32 [S][5]) and the solved gamma_k (float64
    [S]) of every active element of every step (inactive elements, whose
    gamma_k is +inf, carry no target and are left out)."""
    dev = u.device
    feats = torch.empty(ctx.ne, NF, dtype=torch.float32, device=dev)
    gk = torch.empty(ctx.ne, dtype=torch.float64, device=dev)
    F, G = [], []
    ctx.set_step_model(model, feats)
    try:
        for _ in range(nsteps):
            ctx.step(u, t, 0.0, gk)
            F.append(feats.clone())
            G.append(gk.clone())
    finally:
        ctx.set_step_model(None, None)
    rc, bad = ctx.sync_status()
    if rc != 0:
        raise esrk.EsrkError(rc, f"collect (element {bad})")
    F = torch.cat(F)
    G = torch.cat(G)
    keep = torch.isfinite(G) & (G > 0)
    return F[keep].contiguous(), G[keep].contiguous()


def split_runs(runs, val_frac: float = 0.2):
    """Per run, the last val_frac of its samples (its latest steps) are held out."""
    tr_x, tr_g, va_x, va_g = [], [], [], []
    for raw, g in runs:
        n = raw.shape[0]
        cut = int(round(n * (1.0 - val_frac)))
        tr_x.append(raw[:cut])
        tr_g.append(g[:cut])
        va_x.append(raw[cut:])
        va_g.append(g[cut:])
    return (torch.cat(tr_x).contiguous(), torch.cat(tr_g).contiguous(),
            torch.cat(va_x).contiguous(), torch.cat(va_g).contiguous())


def loss_of(model, x_norm, t_norm):
    """Mean squared error of the network on normalized samples (kernel-computed)."""
    grad = torch.empty(esrk.MLP_TRAINED, dtype=torch.float32, device=model.device)
    loss = torch.zeros(1, dtype=torch.float32, device=model.device)
    esrk.mlp_grad(model, x_norm, t_norm, grad, loss)
    return float(loss.item())


def train(runs, steps: int = 2000, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          val_frac: float = 0.2, log_every: int = 0):
    """Train on logged runs [(raw, gamma), ...]; returns (model, history).

    The normalization is fitted on the training part; Adam on mini-batches of
    the shuffled training samples, reshuffled each epoch (seeded)."""
    raw_tr, g_tr, raw_va, g_va = split_runs(runs, val_frac)
    dev = raw_tr.device
    model = torch.from_numpy(inputs.mlp_init(seed)).to(dev)
    x_tr = torch.empty(raw_tr.shape[0], NF, dtype=torch.float32, device=dev)
    t_tr = torch.empty(raw_tr.shape[0], dtype=torch.float32, device=dev)
    esrk.mlp_prepare(model, raw_tr, x_tr, g_tr, t_tr, fit=True)
    x_va = torch.empty(max(raw_va.shape[0], 1), NF, dtype=torch.float32, device=dev)
    t_va = torch.empty(max(raw_va.shape[0], 1), dtype=torch.float32, device=dev)
    if raw_va.shape[0] > 0:
        esrk.mlp_prepare(model, raw_va, x_va, g_va, t_va, fit=False)
    grad = torch.empty(esrk.MLP_TRAINED, dtype=torch.float32, device=dev)
    m = torch.zeros(esrk.MLP_TRAINED, dtype=torch.float32, device=dev)
    v = torch.zeros(esrk.MLP_TRAINED, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    S = x_tr.shape[0]
    B = min(batch, S)
    perm, pos = None, S
    work = torch.empty(esrk.mlp_grad_work_size(B), dtype=torch.float32, device=dev)
    hist = {"train": [], "val": []}
    for it in range(1, steps + 1):
        if pos + B > S:
            perm = torch.randperm(S, generator=gen).to(dev)
            pos = 0
        idx = perm[pos:pos + B]
        pos += B
        xb = x_tr.index_select(0, idx).contiguous()
        tb = t_tr.index_select(0, idx).contiguous()
        esrk.mlp_grad(model, xb, tb, grad, loss, work)
        esrk.mlp_adam(model, grad, m, v, it, lr)
        if log_every and (it % log_every == 0 or it == steps):
            hist["train"].append((it, float(loss.item())))
    hist["train_final"] = loss_of(model, x_tr, t_tr)
    hist["val_final"] = loss_of(model, x_va, t_va) if raw_va.shape[0] > 0 else None
    hist["n_train"], hist["n_val"] = int(S), int(raw_va.shape[0])
    return model, hist


def _events():
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def gain(ctx: esrk.Context, u: torch.Tensor, t: torch.Tensor, nsteps: int, model,
         dt: float | None = None, reps: int = 3):
    """Relaxation solve with the plain first trial point, with the previous
    step's gamma_k as first trial point, and with the network's, on the same
    increments of nsteps consecutive steps (u advances in place).

    Returns per variant: mean phi evaluations per active element, mean solve
    time per step (ms), and the largest |gamma_k - gamma_k(plain)| over active
    elements."""
    dev = u.device
    st = torch.cuda.current_stream()
    nv, N, ne = ctx.nv, ctx.N, ctx.ne
    s = 3 if ctx.cfg.tableau == esrk.SSPRK33 else 4
    ns = ctx.cfg.mu > 0.0
    if dt is None:
        stats = torch.zeros(8, dtype=torch.float64, device=dev)
        probe = u.clone()
        tp = t.clone()
        ctx.step(probe, tp, 0.0, None, stats, stream=st)
        dt = float(stats[1].item())
        del probe, tp
    ya = torch.empty_like(u)
    yb = torch.empty_like(u)
    du = torch.empty(nv * N, dtype=torch.float64, device=dev)
    deta = torch.empty(ne, dtype=torch.float64, device=dev)
    scratch = torch.empty_like(u)
    vd = torch.zeros(ne, dtype=torch.float64, device=dev) if ns else None
    prev = torch.full((ne,), 1.0, dtype=torch.float32, device=dev)
    out = {k: {"evals": 0.0, "ms": 0.0, "dgamma": 0.0, "n": 0} for k in ("plain", "warm", "net")}
    gk = {k: torch.empty(ne, dtype=torch.float64, device=dev) for k in out}
    gam = torch.empty(1, dtype=torch.float64, device=dev)
    its = {k: torch.empty(ne, dtype=torch.int32, device=dev) for k in out}
    gk_step = torch.empty(ne, dtype=torch.float64, device=dev)
    for n in range(nsteps):
        y_in, y_out = u, ya
        for i in range(s):
            if ns and i == s - 1:
                ctx.rhs_ns(y_in, scratch, None, vd, stream=st)
            ctx.rk_stage(i, dt, u, y_in, y_out if i < s - 1 else None, du, deta, stream=st)
            if i < s - 1:
                y_in, y_out = y_out, (yb if y_out is ya else ya)
        for k in ("plain", "warm", "net"):
            e0, e1 = _events()
            e0.record(st)
            for _ in range(reps):
                if k == "plain":
                    ctx.local_relaxation_solve(u, du, deta, gk[k], gam, None, its[k], stream=st)
                elif k == "warm":
                    ctx.local_relaxation_solve(u, du, deta, gk[k], gam, prev if n > 0 else None,
                                               its[k], stream=st)
                else:
                    ctx.local_relaxation_solve_ml(u, du, deta, dt, gk[k], gam, vd, model, None,
                                                  its[k], stream=st)
            e1.record(st)
            e1.synchronize()
            out[k]["ms"] += e0.elapsed_time(e1) / reps
        act = torch.isfinite(gk["plain"])
        for k in out:
            out[k]["evals"] += float(its[k][act].double().mean().item()) if act.any() else 0.0
            d = (gk[k] - gk["plain"])[act].abs().max().item() if act.any() else 0.0
            out[k]["dgamma"] = max(out[k]["dgamma"], float(d))
            out[k]["n"] += 1
        ctx.step(u, t, dt, gk_step, stream=st)
        prev.copy_(gk_step)
    rc, bad = ctx.sync_status()
    if rc != 0:
        raise esrk.EsrkError(rc, f"gain (element {bad})")
    for k in out:
        n = max(out[k].pop("n"), 1)
        out[k]["evals"] /= n
        out[k]["ms"] /= n
    return out
