"""Graph mode: the whole device-side build captured once as a HIP graph and replayed.

Each replay is checked against an eager build of the same inputs, with other eager GPU work
and synchronisations between replays; D changed in place between replays is picked up (the
graph holds pointers, not values), new Sigma buffers force a re-capture."""
import sys

import numpy as np
import pytest

import hfx_synth as hs

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _workload():
    parts = [hs.make_workload("tiny", kind="conventional", species_table=((5, 9),), r_c=7.0, r_v=9.0, r_d=10.0,
                              eps=1e-6, seed=21),
             hs.make_workload("tiny", kind="primitive", species_table=((18, 21), (3, 5)), species=[0, 1], r_c=6.0,
                              r_v=7.0, r_d=8.0, eps=1e-6, seed=22)]
    import dataclasses
    return dataclasses.replace(parts[0], cells=[w.cells[0] for w in parts], C=[w.C[0] for w in parts],
                               V=[w.V[0] for w in parts], D=[w.D[0] for w in parts])


def _dev(D):
    import torch
    return [hs.Blocks(b.row, b.col, b.R, b.off, torch.from_numpy(np.array(b.data)).cuda(), "D") for b in D]


def _close(a, b):
    for x, y in zip(a, b):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.max(np.abs(x - y)) <= 1e-12 * max(np.max(np.abs(y)), 1e-300)


def test_graph_replays_match_eager():
    import torch
    from paper_2009_12505_amd import HfxError, Plan
    log("case graph replays")
    w = _workload()
    eager = Plan(w.cells, w.C, w.V, w.D, w.thresholds)
    graph = Plan(w.cells, w.C, w.V, w.D, w.thresholds, use_graph=True)
    Dd = _dev(w.D)
    ref = eager.build(Dd, stats=True)
    ref_stats = eager.last_stats
    sig = graph.alloc_sigma()
    for rep in range(4):
        graph.build(Dd, sig, stats=(rep % 2 == 0))
        torch.cuda.synchronize()
        _close(sig, ref)
        if rep % 2 == 0:
            for t in (1, 2, 3, 4):
                assert graph.last_stats[f"kept_s3_t{t}"] == ref_stats[f"kept_s3_t{t}"]
        # unrelated eager work between replays
        x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
        assert torch.isfinite(x.sum()).item()
        eager.build(Dd, stats=False)
        torch.cuda.synchronize()
        log(f"  replay {rep}: equal to eager")
    # D changed in place: the same graph reads the new values
    for b in Dd:
        b.data.mul_(0.5)
    ref_half = eager.build(Dd)
    graph.build(Dd, sig)
    torch.cuda.synchronize()
    _close(sig, ref_half)
    # new Sigma buffers: re-captured
    sig2 = graph.alloc_sigma()
    graph.build(Dd, sig2)
    torch.cuda.synchronize()
    _close(sig2, ref_half)
    e_g, e_e = graph.energy(Dd, sig2), eager.energy(Dd, ref_half)
    assert all(abs(a - b) <= 1e-11 * abs(b) for a, b in zip(e_g, e_e))
    # host D is refused in graph mode
    with pytest.raises(HfxError):
        graph.build(w.D, sig2)
