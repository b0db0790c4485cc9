"""Locality groups (k-means on the midpoints of the atom pairs, one group per XCD, Algorithm 7
mapped onto one GPU): the same units are computed in a different order, so Sigma equals the LPT
build to FP64 summation order; the build times of both orders are reported."""
import numpy as np
import pytest

import hfx_synth as hs
from test_gpu_parity import log

pytestmark = pytest.mark.gpu


def _build(w, **opt):
    import torch
    from paper_2009_12505_amd import Plan
    plan = Plan(w.cells, w.C, w.V, w.D, w.thresholds, **opt)
    ms = []
    for _ in range(3):
        sig = plan.build(w.D, stats=True)
        ms.append(plan.last_stats["ms_main"])
    torch.cuda.synchronize()
    out = [s.cpu().numpy() for s in sig]
    del plan, sig
    torch.cuda.empty_cache()
    return out, ms


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["cfg3", "cfg4"])
def test_kmeans_groups_leave_sigma_unchanged(name):
    from paper_2009_12505_amd import SCHED_KMEANS, SCHED_LPT
    w = hs.make_workload(name, eps=1e-6 if name == "cfg3" else None)
    offs = np.cumsum([0] + [c.n_atoms for c in w.cells])
    rng = np.random.default_rng(5)
    if name == "cfg3":
        home = sorted(rng.choice(w.cells[0].n_atoms, size=64, replace=False).tolist())
    else:
        home = [int(offs[c] + rng.integers(w.cells[c].n_atoms)) for c in range(len(w.cells))]
    log(f"case k-means groups {name}, {len(home)} home atoms")
    a, ms_lpt = _build(w, scheduler=SCHED_LPT, home_subset=home)
    b, ms_km = _build(w, scheduler=SCHED_KMEANS, home_subset=home)
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) <= 1e-12 * max(np.max(np.abs(x)), 1e-300)
    log(f"{name}: main kernel ms, LPT {[round(t, 1) for t in ms_lpt]}, k-means groups {[round(t, 1) for t in ms_km]}")
