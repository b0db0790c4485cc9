"""Learned model of the work-item order (training driver over the C ABI).

The persistent build kernel takes work items <A,B> by an atomic ticket in the
order the plan uploads; the longest-first greedy rule of the paper's machine
scheduling (Sec. III D 1, Algorithm 6) then needs per-item costs.  The static
cost |N(A)| |N(B)| ignores screening, block shapes and memory effects; this
module fits a small perceptron with two outputs to labels the build kernel
itself records per item: its wall-clock ticks (the cost the plan orders by) and
its contribution bound (the summed screening bounds of its kept units, which
bounds the size of its contribution to Sigma).  The inputs are features the
library computes on the GPU.  The forward pass, the gradient of the squared
error and Adam are the library's kernels (hfx_mlp_train); Python only stacks
samples and standardises them.

    samples = [profile_samples(plan)]            # after one or more builds
    model = train(samples)
    save(model, "sched.bin")
    plan = Plan(..., scheduler=SCHED_MLP, mlp_weights="sched.bin")
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np

from . import _abi as A

N_IN = A.ITEM_FEATURES
N_OUT = A.ITEM_TARGETS
MAGIC = b"HFXMLP02"
TARGETS = ("log ticks", "log1p(contribution bound / eps)")


@dataclasses.dataclass
class CostModel:
    hidden: int
    mu: np.ndarray       # feature standardisation (N_IN,)
    sd: np.ndarray
    params: np.ndarray   # float32, layout of hfx_mlp_n_params(N_IN, hidden, N_OUT)
    loss: np.ndarray     # training loss per epoch
    t_mu: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(N_OUT, np.float32))
    t_sd: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(N_OUT, np.float32))


def n_params(hidden: int) -> int:
    return int(A.lib().hfx_mlp_n_params(N_IN, hidden, N_OUT))


def profile_samples(plan):
    """Raw features (host float32 [n_items, N_IN]) and the two labels [n_items, 2] of the plan's
    last build: log(ticks) and log1p(contribution bound / eps_cs_mat)."""
    X = plan.item_features(np.zeros(N_IN, np.float32), np.ones(N_IN, np.float32)).cpu().numpy()
    cyc, _, contrib = plan.item_profile()
    scale = plan.eps_mat if plan.eps_mat > 0 else 1e-12
    T = np.stack([np.log(np.maximum(cyc, 1).astype(np.float64)), np.log1p(contrib / scale)], axis=1)
    return X, T


def init_params(hidden: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    H, F, O = hidden, N_IN, N_OUT
    p = np.zeros(n_params(hidden), np.float32)
    o = 0
    p[o:o + H * F] = rng.uniform(-1, 1, H * F) / np.sqrt(F)
    o += H * F + H
    p[o:o + H * H] = rng.uniform(-1, 1, H * H) / np.sqrt(H)
    o += H * H + H
    p[o:o + O * H] = rng.uniform(-1, 1, O * H) / np.sqrt(H)
    return p


def train(samples, hidden: int = 32, epochs: int = 2000, lr: float = 3e-3, seed: int = 0) -> CostModel:
    """Full-batch Adam on the GPU over the concatenated (features, labels) samples; features and
    both labels are standardised, the loss is the sum of the two outputs' mean squared errors."""
    import torch
    X = np.concatenate([s[0] for s in samples]).astype(np.float64)
    T = np.concatenate([np.asarray(s[1], np.float64).reshape(len(s[0]), -1) for s in samples])
    if T.shape[1] != N_OUT:
        raise ValueError(f"labels need {N_OUT} columns")
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[sd < 1e-6] = 1.0
    t_mu = T.mean(axis=0)
    t_sd = T.std(axis=0)
    t_sd[t_sd < 1e-12] = 1.0
    Xn = torch.from_numpy(((X - mu) / sd).astype(np.float32)).cuda()
    Tn = torch.from_numpy(((T - t_mu) / t_sd).astype(np.float32)).contiguous().cuda()
    P = torch.from_numpy(init_params(hidden, seed)).cuda()
    loss = np.zeros(epochs, np.float32)
    stream = torch.cuda.current_stream()
    A.check(A.lib().hfx_mlp_train(N_IN, hidden, N_OUT, ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(Xn.data_ptr()),
                                  ctypes.c_void_p(Tn.data_ptr()), Xn.shape[0], epochs, lr,
                                  loss.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(stream.cuda_stream)))
    return CostModel(hidden, mu.astype(np.float32), sd.astype(np.float32), P.cpu().numpy(), loss,
                     t_mu.astype(np.float32), t_sd.astype(np.float32))


def predict(model: CostModel, X_raw):
    """Standardised predictions [n, 2] (log cost, log contribution bound) of raw feature rows,
    on the GPU; ``model.t_mu + model.t_sd * y`` gives the labels' own scale."""
    import torch
    Xn = torch.from_numpy(((np.asarray(X_raw, np.float64) - model.mu) / model.sd).astype(np.float32)).cuda()
    P = torch.from_numpy(model.params).cuda()
    y = torch.empty((Xn.shape[0], N_OUT), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    A.check(A.lib().hfx_mlp_predict(N_IN, model.hidden, N_OUT, ctypes.c_void_p(P.data_ptr()),
                                    ctypes.c_void_p(Xn.data_ptr()), Xn.shape[0], ctypes.c_void_p(y.data_ptr()),
                                    ctypes.c_void_p(stream.cuda_stream)))
    return y.cpu().numpy()


def save(model: CostModel, path) -> None:
    """The library's model file, followed by the target standardisation (which the library does
    not read)."""
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(np.array([N_IN, model.hidden, N_OUT], np.int32).tobytes())
        f.write(model.mu.astype(np.float32).tobytes())
        f.write(model.sd.astype(np.float32).tobytes())
        f.write(model.params.astype(np.float32).tobytes())
        f.write(np.asarray(model.t_mu, np.float32).tobytes())
        f.write(np.asarray(model.t_sd, np.float32).tobytes())


def load(path) -> CostModel:
    with open(path, "rb") as f:
        raw = f.read()
    if raw[:8] != MAGIC:
        raise ValueError(f"{path}: not a scheduler model file")
    n_in, hidden, n_out = (int(x) for x in np.frombuffer(raw[8:20], np.int32))
    if n_in != N_IN or n_out != N_OUT:
        raise ValueError(f"{path}: {n_in} inputs / {n_out} outputs, expected {N_IN} / {N_OUT}")
    v = np.frombuffer(raw[20:], np.float32)
    npar = hidden * n_in + hidden + hidden * hidden + hidden + n_out * hidden + n_out
    if v.size != 2 * N_IN + npar + 2 * N_OUT:
        raise ValueError(f"{path}: truncated or oversized model file")
    o = 2 * N_IN + npar
    return CostModel(hidden, v[:N_IN].copy(), v[N_IN:2 * N_IN].copy(), v[2 * N_IN:o].copy(), np.zeros(0),
                     v[o:o + N_OUT].copy(), v[o + N_OUT:].copy())


def choose_by_build_time(make_plan, D, kinds, reps: int = 3):
    """The fallback rule: build with each scheduler kind (one warm-up build, whose order is the
    static one for the kinds that learn from a previous build, then ``reps`` timed builds) and
    keep the kind with the smallest median main-kernel time.  ``make_plan(kind)`` returns a Plan.
    Returns (best kind, {kind: median ms}, {kind: [ms of the timed builds]})."""
    import torch
    med, runs = {}, {}
    for kind in kinds:
        plan = make_plan(kind)
        plan.build(D, stats=True)
        ms = []
        for _ in range(reps):
            plan.build(D, stats=True)
            ms.append(plan.last_stats["ms_main"])
        runs[kind] = ms
        med[kind] = float(np.median(ms))
        del plan
        torch.cuda.empty_cache()
    best = min(med, key=med.get)
    return best, med, runs


def list_schedule_makespan(costs, order, n_machines: int) -> float:
    """Makespan of greedy list scheduling: items taken in `order`, each by the machine that
    frees first (what the atomic ticket of the persistent kernel does)."""
    import heapq
    h = [0.0] * n_machines
    for i in order:
        heapq.heapreplace(h, h[0] + float(costs[i]))
    return max(h)
