"""Learned cost model of the work-item order (training driver over the C ABI).

The persistent build kernel takes work items <A,B> by an atomic ticket in the
order the plan uploads; the longest-first greedy rule of the paper's machine
scheduling (Sec. III D 1, Algorithm 6) then needs per-item costs.  The static
cost |N(A)| |N(B)| ignores screening, block shapes and memory effects; this
module fits a small perceptron to the per-item wall-clock ticks that the build
kernel itself records, from features the library computes on the GPU.  The
forward pass, the gradient of the squared error and Adam are the library's
kernels (hfx_mlp_train); Python only stacks samples and normalises them.

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

N_IN = 8
MAGIC = b"HFXMLP01"


@dataclasses.dataclass
class CostModel:
    hidden: int
    mu: np.ndarray       # feature normalisation (8,)
    sd: np.ndarray
    params: np.ndarray   # float32, layout of hfx_mlp_n_params
    loss: np.ndarray     # training loss per epoch


def n_params(hidden: int) -> int:
    return int(A.lib().hfx_mlp_n_params(N_IN, hidden))


def profile_samples(plan):
    """Raw features (host float32 [n_items, 8]) and labels log(ticks) of the plan's last build."""
    X = plan.item_features(np.zeros(N_IN, np.float32), np.ones(N_IN, np.float32)).cpu().numpy()
    cyc, _ = plan.item_profile()
    return X, np.log(np.maximum(cyc, 1).astype(np.float64))


def init_params(hidden: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    H, F = hidden, N_IN
    p = np.zeros(n_params(hidden), np.float32)
    o = 0
    p[o:o + H * F] = rng.uniform(-1, 1, H * F) / np.sqrt(F)
    o += H * F + H
    p[o:o + H * H] = rng.uniform(-1, 1, H * H) / np.sqrt(H)
    o += H * H + H
    p[o:o + H] = rng.uniform(-1, 1, H) / np.sqrt(H)
    return p


def train(samples, hidden: int = 32, epochs: int = 2000, lr: float = 3e-3, seed: int = 0) -> CostModel:
    """Full-batch Adam on the GPU over the concatenated (features, log ticks) samples."""
    import torch
    X = np.concatenate([s[0] for s in samples]).astype(np.float64)
    t = np.concatenate([s[1] for s in samples])
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd[sd < 1e-6] = 1.0
    Xn = torch.from_numpy(((X - mu) / sd).astype(np.float32)).cuda()
    tn = torch.from_numpy(((t - t.mean()) / max(t.std(), 1e-12)).astype(np.float32)).cuda()
    P = torch.from_numpy(init_params(hidden, seed)).cuda()
    loss = np.zeros(epochs, np.float32)
    stream = torch.cuda.current_stream()
    A.check(A.lib().hfx_mlp_train(N_IN, hidden, ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(Xn.data_ptr()),
                                  ctypes.c_void_p(tn.data_ptr()), Xn.shape[0], epochs, lr,
                                  loss.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(stream.cuda_stream)))
    return CostModel(hidden, mu.astype(np.float32), sd.astype(np.float32), P.cpu().numpy(), loss)


def predict(model: CostModel, X_raw):
    """Predicted (normalised) log cost of raw feature rows, on the GPU."""
    import torch
    Xn = torch.from_numpy(((np.asarray(X_raw, np.float64) - model.mu) / model.sd).astype(np.float32)).cuda()
    P = torch.from_numpy(model.params).cuda()
    y = torch.empty(Xn.shape[0], dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    A.check(A.lib().hfx_mlp_predict(N_IN, model.hidden, ctypes.c_void_p(P.data_ptr()),
                                    ctypes.c_void_p(Xn.data_ptr()), Xn.shape[0], ctypes.c_void_p(y.data_ptr()),
                                    ctypes.c_void_p(stream.cuda_stream)))
    return y.cpu().numpy()


def save(model: CostModel, path) -> None:
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(np.array([N_IN, model.hidden], np.int32).tobytes())
        f.write(model.mu.astype(np.float32).tobytes())
        f.write(model.sd.astype(np.float32).tobytes())
        f.write(model.params.astype(np.float32).tobytes())


def load(path) -> CostModel:
    with open(path, "rb") as f:
        raw = f.read()
    if raw[:8] != MAGIC:
        raise ValueError(f"{path}: not a scheduler model file")
    n_in, hidden = np.frombuffer(raw[8:16], np.int32)
    if n_in != N_IN:
        raise ValueError(f"{path}: {n_in} inputs, expected {N_IN}")
    v = np.frombuffer(raw[16:], np.float32)
    return CostModel(int(hidden), v[:N_IN].copy(), v[N_IN:2 * N_IN].copy(), v[2 * N_IN:].copy(), np.zeros(0))


def list_schedule_makespan(costs, order, n_machines: int) -> float:
    """Makespan of greedy list scheduling: items taken in `order`, each by the machine that
    frees first (what the atomic ticket of the persistent kernel does)."""
    import heapq
    h = [0.0] * n_machines
    for i in order:
        heapq.heapreplace(h, h[0] + float(costs[i]))
    return max(h)
