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
                 label_k: int = 0, X0=None, log=None, lanczos_fallback=None, apply_step=None):
    """One self-consistent-step sequence on a context.  chooser(step, feats,
    theta) -> (a, b, m, used_lanczos).  If the projection after the filter
    finds the block rank deficient and lanczos_fallback is given, the step is
    redone with it ("rescued").  The operator of step s is the host
    perturbation sequence of `seed` (re-uploaded cell blocks), or whatever
    apply_step(s) sets on the device.  Returns per-step records with the
    features, the bounds used, timings and (if label_k) the labels."""
    import torch
    from .binding import ChebFilterError, empty_block
    from synth import configs, perturb
    dev = v0.device
    X = empty_block(prob.n, N, dev)
    X.copy_(torch.as_tensor(configs.initial_block(prob, N, seed=seed) if X0 is None else X0))
    Y = empty_block(prob.n, N, dev)
    theta = ctx.rayleigh_ritz(X)
    feats, recs = [], []
    if apply_step is None:
        def host_steps():
            for Hs in perturb.sequence(prob, steps, seed=seed):
                ctx.update_H_cc(Hs)
                yield
    else:
        def host_steps():
            for s in range(steps):
                apply_step(s)
                yield
    for s, _ in enumerate(host_steps()):
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


class DeviceSteps:
    """Operator update of a self-consistent-step sequence on the device: every
    plain cell's block assembled once from the base potential V0 at its Gauss
    points (chebfilter_assemble_cells), then per step the far plain cells'
    blocks (cells sharing no DOF with an enriched cell) from V0 + dV, dV a
    fresh seeded smooth field (synth.perturb.field_draw / field_at)."""

    def __init__(self, ctx, prob, plain, far, V0_plain):
        import torch
        from synth.assemble import plain_points, plain_tables
        B, w, K, _ = plain_tables(prob)
        ctx.assembly_tables(B, w, K)
        dev = torch.device("cuda", torch.cuda.current_device())
        V0 = torch.tensor(np.asarray(V0_plain).reshape(len(plain), -1), dtype=torch.float64,
                          device=dev)
        ctx.assemble_cells(plain, V0)
        pos = torch.as_tensor(np.searchsorted(plain, far), device=dev)
        self.V0f = V0[pos].contiguous()
        del V0
        self.pts = torch.tensor(plain_points(prob, far).reshape(-1, 3), dtype=torch.float64,
                                device=dev)
        self.ctx, self.far, self.nq = ctx, np.asarray(far, dtype=np.int32), B.shape[0]
        mesh = prob.meta["mesh"]
        self.lo, self.length = mesh.lo, mesh.length
        self.rng = np.random.default_rng(0)

    def start(self, seed: int):
        """Begin a new sequence (its fields drawn from `seed`)."""
        self.rng = np.random.default_rng(seed)
        return self

    def __call__(self, s: int):
        from synth import perturb
        c, a, sg = perturb.field_draw(self.rng, self.lo, self.length)
        dV = perturb.field_at(self.pts, c, a, sg).reshape(len(self.far), self.nq)
        self.ctx.assemble_cells(self.far, self.V0f + dV)


def run_paths(ctx, prob, N: int, wanted: int, steps: int, seed: int, choosers: dict, v0,
              apply_step, ref_steps=(), ref_passes: int = 10, ref_tol: float = 1e-9, log=None,
              lanczos_fallback=None):
    """Several choosers on one operator sequence in lockstep (one context, one
    block per path plus a spare): at each step the operator is updated once,
    then every path takes its filter pass and projection from its own
    subspace.  At the steps in ref_steps (1-based) a reference is formed from
    a copy of the first path's block: FP64 passes with the Lanczos bound and
    the degree rule until the wanted Ritz values change by < ref_tol.
    Returns ({name: records}, {step: reference Ritz values})."""
    import torch
    from .binding import ChebFilterError, empty_block
    from synth import configs
    dev = v0.device
    X0 = torch.as_tensor(configs.initial_block(prob, N, seed=seed))
    st = {}
    for name in choosers:
        X = empty_block(prob.n, N, dev)
        X.copy_(X0)
        st[name] = {"X": X, "feats": [], "recs": [], "theta": ctx.rayleigh_ritz(X)}
    del X0
    spare = empty_block(prob.n, N, dev)
    refs = {}
    first = next(iter(choosers))
    for s in range(steps):
        apply_step(s)
        for name, chooser in choosers.items():
            p = st[name]
            theta_cur = ctx.rayleigh_ritz(p["X"])
            if not p["feats"]:
                res = ctx.residual_norms(p["X"], theta_cur)
                _, b0 = ctx.lanczos_bounds(v0, 10)
                p["feats"].append(step_features(theta_cur, theta_cur, wanted, b0, 40, res))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a, b, m, fb = chooser(s, p["feats"], theta_cur)
            t1 = time.perf_counter()
            ctx.filter(p["X"], m, a, b, Y=spare)
            rescued = False
            try:
                th = ctx.rayleigh_ritz(spare)
            except ChebFilterError as exc:
                if exc.status != 3 or lanczos_fallback is None:
                    raise
                a, b, m, fb = lanczos_fallback(s, p["feats"], theta_cur)
                ctx.filter(p["X"], m, a, b, Y=spare)
                th = ctx.rayleigh_ritz(spare)
                rescued = True
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            res = ctx.residual_norms(spare, th)
            p["feats"].append(step_features(th, theta_cur, wanted, b, m, res))
            p["recs"].append(dict(step=s, a=a, b=b, m=m, fallback=bool(fb), rescued=rescued,
                                  t_bounds=t1 - t0, t_pass=t2 - t1, theta=th.copy(),
                                  res_max=float(np.max(res[:wanted]))))
            p["X"], spare = spare, p["X"]
            if log:
                log(f"step {s} {name}: a={a:.4f} b={b:.3f} m={m} lanczos={bool(fb)} "
                    f"res_max={p['recs'][-1]['res_max']:.3e} pass {t2 - t1:.2f}s")
        if s + 1 in ref_steps:
            R = empty_block(prob.n, N, dev)
            R.copy_(st[first]["X"])
            th = ctx.rayleigh_ritz(R)
            for it in range(ref_passes):
                _, b = ctx.lanczos_bounds(v0, 10)
                mref = degree_rule(float(th[0]), float(th[wanted - 1]), float(th[-1]), b)
                ctx.filter(R, mref, float(th[-1]), b, Y=spare)
                thn = ctx.rayleigh_ritz(spare)
                R, spare = spare, R
                d = float(np.abs(thn[:wanted] - th[:wanted]).max())
                th = thn
                if d < ref_tol and it >= 1:
                    break
            refs[s + 1] = th[:wanted].copy()
            del R                       # the other of the two buffers stays the spare
            if log:
                log(f"reference at step {s + 1}: {it + 1} passes, last change {d:.2e}")
    return {k: v["recs"] for k, v in st.items()}, refs


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
