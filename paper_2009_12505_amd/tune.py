"""Autotuner of the build's tile shape and precision tiers (driver over the C ABI).

For one plan key (the species present, the CS-matrix threshold and the precision form, as
hfx_tune_key reports it) it times the candidate column widths of the terms-3/4 output blocks
(tile_r 128, 64 or 32) and, for the tiered forms, candidate tier bounds (tier_tau; tier_tau_bf for the
split-BF16x3 tier) on a calibration subset of home atoms.  A candidate is admitted only if its
Sigma and E_x on that subset differ from the FP64 build of the same subset by at most a third of
the method's targets (1e-7 max-abs in Sigma, 1e-8 Ha per home atom in E_x); the fastest admitted
candidate (median main-kernel time) is appended to a text tuning file, which hfx_plan_create
reads (hfx_options.tuning_db):

    hfxtune1 species=13x60 eps=1e-06 prec=tiered tile_r=64 tier_tau=0.001 tier_tau_bf=0

Python only loops over candidates and compares results; every build runs in the library.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import _abi as A
from .plan import Plan

SIGMA_BUDGET = 1e-7 / 3.0  # a third of the method's max-abs Sigma target
EX_BUDGET = 1e-8 / 3.0     # a third of the method's |dE_x| per atom target
FORM_NAMES = {A.PREC_FP64: "fp64", A.PREC_TIERED: "tiered", A.PREC_FP32: "fp32", A.PREC_BF16X3: "bf16x3"}


@dataclasses.dataclass
class Candidate:
    tile_r: int
    tier_tau: float
    tier_tau_bf: float
    ms: float = float("nan")         # median main-kernel time
    max_dsigma: float = float("nan")  # against the FP64 build of the subset
    de_x_atom: float = float("nan")
    admitted: bool = False


def _builds(plan, D, reps):
    import torch
    plan.build(D, stats=True)
    ms = []
    for _ in range(reps):
        sig = plan.build(D, stats=True)
        ms.append(plan.last_stats["ms_main"])
    torch.cuda.synchronize()
    return sig, float(np.median(ms))


def tune(cells, C, V, D_pattern, D, thresholds, precision, home_subset, db_path=None, tiles=(128, 64, 32),
         taus=(1e-4, 1e-3, 1e-2), taus_bf=(1e-6, 1e-5, 1e-4), reps: int = 2, log=print):
    """Tune one plan key on the given home subset; returns (key, best Candidate, all candidates).
    The best choice is appended to ``db_path`` when given."""
    import torch
    n_home = len(home_subset)
    ref = Plan(cells, C, V, D_pattern, thresholds, home_subset=home_subset)
    sig64, _ = _builds(ref, D, 1)
    e64 = sum(ref.energy(D, sig64))
    ref64 = [s.cpu().numpy() for s in sig64]
    del ref, sig64
    torch.cuda.empty_cache()
    if precision in (A.PREC_TIERED, A.PREC_FP32):
        grid = [(t, 0.0) for t in taus] if precision == A.PREC_TIERED else [(0.0, 0.0)]
    elif precision == A.PREC_BF16X3:
        grid = [(t, tb) for t in taus for tb in taus_bf if tb <= t]
    else:
        grid = [(0.0, 0.0)]
    cands, key = [], None
    for tile in tiles:
        for tau, tau_bf in grid:
            c = Candidate(tile, tau, tau_bf)
            plan = Plan(cells, C, V, D_pattern, thresholds, precision=precision, tier_tau=tau, tier_tau_bf=tau_bf,
                        tile_r=tile, home_subset=home_subset)
            key = plan.tune_key
            sig, c.ms = _builds(plan, D, reps)
            e = sum(plan.energy(D, sig))
            c.max_dsigma = max(float(np.abs(s.cpu().numpy() - r).max()) if r.size else 0.0 for s, r in zip(sig, ref64))
            c.de_x_atom = abs(e - e64) / max(n_home, 1)
            c.admitted = c.max_dsigma <= SIGMA_BUDGET and c.de_x_atom <= EX_BUDGET
            log(f"tune {key}: tile_r {tile} tau {tau:g} tau_bf {tau_bf:g}: {c.ms:.1f} ms, max|dSigma| "
                f"{c.max_dsigma:.2e}, |dE_x|/atom {c.de_x_atom:.2e}, {'admitted' if c.admitted else 'rejected'}")
            cands.append(c)
            del plan, sig
            torch.cuda.empty_cache()
    ok = [c for c in cands if c.admitted]
    if not ok:
        raise RuntimeError(f"no candidate of {key} meets the accuracy gate")
    best = min(ok, key=lambda c: c.ms)
    if db_path is not None:
        with open(db_path, "a") as f:
            f.write(f"hfxtune1 {key} tile_r={best.tile_r} tier_tau={best.tier_tau:.6g} "
                    f"tier_tau_bf={best.tier_tau_bf:.6g}\n")
    return key, best, cands
