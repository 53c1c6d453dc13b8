"""Learned filter bounds: the self-consistent-step driver around the library's
network (chebfilter_mlp_*) and guard (chebfilter_bounds_predict).

Each step of a sequence changes the potential (synth.perturb), so the
operator H~ changes a little from step to step; one filter pass and a
Rayleigh-Ritz projection per step follow it.  The filter needs (a, b, m):
a = theta_N from the last projection, b an upper bound of the spectrum
(Lanczos, Sec. V), m the degree.  The network maps the last 8 steps' spectrum
summaries (8 numbers each) to (a, b, m); the guard falls back to Lanczos.

Labels for training, per step (chebfilter_bounds_label): a* = theta_N of the
projection of the step's operator, b* = the upper bound of a 40-step Lanczos
run on it, and m* = the library's degree rule at (theta_1, theta_Nw, a*, b*);
the network inputs are the scale-free features of
chebfilter_bounds_features and its outputs
(alpha, beta, m) with a = theta_N + alpha w, b = theta_N + beta w, w the last
step's b - theta_N, so one network serves clusters of different sizes.  Host code here only marshals arrays,
keeps histories and normalisation constants; every operator application,
Lanczos step, projection and network evaluation runs in the library.
"""
from __future__ import annotations

import time

import numpy as np

FEATURES = 8          # per step
HISTORY = 8           # steps fed to the network
N_IN = FEATURES * HISTORY
N_OUT = 3             # a, b, m
WIDTH, DEPTH = 128, 3


def degree_rule(theta_1: float, theta_w: float, a: float, b: float, rho: float = 100.0,
                m_min: int = 8, m_max: int = 120) -> int:
    """The library's degree rule (chebfilter_degree_rule)."""
    from .binding import degree_rule as lib_rule
    return lib_rule(theta_1, theta_w, a, b, rho, m_min, m_max)


def step_features(theta, theta_prev, wanted: int, b_used: float, m_used: int, res) -> np.ndarray:
    """The library's step summary (chebfilter_step_summary)."""
    from .binding import step_summary
    return step_summary(theta, theta_prev, wanted, b_used, m_used, res)


def history_vector(feats: list) -> np.ndarray:
    """The last HISTORY feature rows, oldest first (the earliest row repeated
    while fewer steps exist)."""
    rows = list(feats[-HISTORY:])
    while len(rows) < HISTORY:
        rows.insert(0, rows[0])
    return np.concatenate(rows)


def init_params(seed: int = 0, n_in: int = N_IN, width: int = WIDTH, depth: int = DEPTH,
                n_out: int = N_OUT) -> np.ndarray:
    """Seeded initial parameters (layout of chebfilter_mlp_*): W ~ N(0, 1/fan_in)
    (2/fan_in before GELU layers), b = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(depth + 1):
        fi = n_in if l == 0 else width
        fo = width if l < depth else n_out
        scale = np.sqrt((2.0 if l < depth else 1.0) / fi)
        parts.append(rng.standard_normal(fo * fi) * scale)
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def run_sequence(ctx, prob, N: int, wanted: int, steps: int, seed: int, chooser, v0,
                 label_k: int = 0, X0=None, log=None, lanczos_fallback=None):
    """One self-consistent-step sequence on a context.  chooser(step, feats,
    theta) -> (a, b, m, used_lanczos).  If the projection after the filter
    finds the block rank deficient and lanczos_fallback is given, the step is
    redone with it ("rescued").  Returns per-step records with the features,
    the bounds used, timings and (if label_k) the labels."""
    import torch
    from .binding import ChebFilterError
    from synth import configs, perturb
    dev = v0.device
    X = torch.tensor(configs.initial_block(prob, N, seed=seed) if X0 is None else X0,
                     dtype=torch.float64, device=dev)
    Y = torch.empty_like(X)
    theta = ctx.rayleigh_ritz(X)
    feats, recs = [], []
    seq = perturb.sequence(prob, steps, seed=seed)
    for s, Hs in enumerate(seq):
        ctx.update_H_cc(Hs)
        # the projection of the new operator on the current subspace
        theta_cur = ctx.rayleigh_ritz(X)
        if not feats:
            res = ctx.residual_norms(X, theta_cur)
            _, b0 = ctx.lanczos_bounds(v0, 10)
            feats.append(step_features(theta_cur, theta_cur, wanted, b0, 40, res))
        rec = {"step": s}
        if label_k:
            rec["input"], rec["target"] = ctx.bounds_label(history_vector(feats), theta_cur, wanted,
                                                           v0, k=label_k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a, b, m, fb = chooser(s, feats, theta_cur)
        t1 = time.perf_counter()
        ctx.filter(X, m, a, b, Y=Y)
        rescued = False
        try:
            th = ctx.rayleigh_ritz(Y)
        except ChebFilterError as exc:
            # the filtered block lost rank (interval or degree too aggressive):
            # redo the step from X with the Lanczos bound and the degree rule
            if exc.status != 3 or lanczos_fallback is None:
                raise
            a, b, m, fb = lanczos_fallback(s, feats, theta_cur)
            ctx.filter(X, m, a, b, Y=Y)
            th = ctx.rayleigh_ritz(Y)
            rescued = True
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = ctx.residual_norms(Y, th)
        feats.append(step_features(th, theta_cur, wanted, b, m, res))
        rec.update(a=a, b=b, m=m, fallback=bool(fb), rescued=rescued, t_bounds=t1 - t0,
                   t_pass=t2 - t1,
                   theta=th.copy(), res_max=float(np.max(res[:wanted])))
        recs.append(rec)
        X, Y = Y, X
        theta = th
        if log:
            log(f"step {s}: a={a:.4f} b={b:.3f} m={m} lanczos={bool(fb)} "
                f"res_max={rec['res_max']:.3e}")
    return recs, X


def lanczos_chooser(ctx, v0, wanted: int, k: int = 10):
    """The baseline: Lanczos b, a = theta_N, degree by degree_rule."""
    def choose(step, feats, theta):
        _, b = ctx.lanczos_bounds(v0, k)
        a = float(theta[-1])
        return a, b, degree_rule(float(theta[0]), float(theta[wanted - 1]), a, b), True
    return choose


def mlp_chooser(ctx, mlp, v0, k: int = 10):
    def choose(step, feats, theta):
        return ctx.bounds_predict(mlp, history_vector(feats), v0, lanczos_k=k)
    return choose


def train(mlp, inputs: np.ndarray, targets: np.ndarray, steps: int = 2000, batch: int = 64,
          lr: float = 1e-3, seed: int = 0, log=None, lr_end: float | None = None):
    """Adam on minibatches of the normalised corpus, all arithmetic in the
    library's network kernels; with lr_end the step size follows a cosine
    from lr to lr_end.  Returns the loss per step."""
    import torch
    mlp.fit_normalization(inputs, targets)
    Xn = mlp.normalize_inputs(inputs)
    Tn = mlp.normalize_targets(targets)
    rng = np.random.default_rng(seed)
    S = Xn.shape[0]
    B = min(batch, S, mlp.max_batch)
    losses = []
    for it in range(steps):
        idx = torch.tensor(rng.choice(S, size=B, replace=False), device=mlp.device)
        xb, tb = Xn[idx].contiguous(), Tn[idx].contiguous()
        losses.append(mlp.loss_grad(xb, tb))
        lr_it = lr if lr_end is None else \
            lr_end + 0.5 * (lr - lr_end) * (1.0 + np.cos(np.pi * it / max(steps - 1, 1)))
        mlp.adam_step(lr_it)
        if log and (it % 250 == 0 or it == steps - 1):
            log(f"train step {it}: loss {losses[-1]:.4e}")
    return np.array(losses)
