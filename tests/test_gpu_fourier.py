"""GPU parity of the real-space to k-space sum (hfx_sigma_to_k) against the FP64 oracle
(oracle.fourier), element by element, on seeded Sigma values in each plan's layout.

Bound: each element of H(k) is a sum of products Sigma_R exp(i k.R); FP64 summation in another
order differs by a few ulps of the sum of the terms' magnitudes, so |dH| <= 1e-13 * sum_R |Sigma_R|
for every element (the k = 0 transform of |Sigma|)."""
import numpy as np
import pytest

import hfx_synth as hs
from oracle import fourier
from test_gpu_parity import TINY, _combine, log

pytestmark = pytest.mark.gpu


def _plan(w):
    from paper_2009_12505_amd import Plan
    return Plan(w.cells, w.C, w.V, w.D, w.thresholds)


def _seeded_sigma(plan, cell, seed):
    return np.random.default_rng(seed).normal(size=plan.sizes[cell])


def _check(cell, D, sig, k, got, label, pairs=None):
    ref = fourier.sigma_to_k(cell, D, sig, k, pairs=pairs)
    mag = fourier.sigma_to_k(cell, D, np.abs(sig), np.zeros((1, 3)), pairs=pairs)
    if pairs is None:
        err = np.abs(got - ref)
        bound = 1e-13 * mag[0].real + 1e-300
        worst = float(np.max(err / bound)) if err.size else 0.0
        log(f"{label}: n_k {k.shape[0]} n_basis {ref.shape[1]} max|H| {np.abs(ref).max():.3e} "
            f"max|dH| {err.max():.3e} (worst / bound {worst:.3f})")
        assert np.all(err <= bound)
    else:
        bo, _ = fourier.basis_offsets(cell)
        nao = [cell.species_table[int(s)][0] for s in cell.species]
        worst = 0.0
        for (I, J), r in ref.items():
            g = got[:, bo[I]:bo[I] + nao[I], bo[J]:bo[J] + nao[J]]
            err = np.abs(g - r)
            bound = 1e-13 * mag[(I, J)][0].real + 1e-300
            worst = max(worst, float(np.max(err / bound)))
            assert np.all(err <= bound), (I, J)
        log(f"{label}: {len(ref)} sampled blocks, worst |dH| / bound {worst:.3f}")


@pytest.mark.parametrize("cfg", range(len(TINY)))
def test_tiny_sigma_to_k(cfg):
    import torch
    log(f"case fourier tiny[{cfg}]")
    w = hs.make_workload("tiny", **TINY[cfg])
    plan = _plan(w)
    sig = _seeded_sigma(plan, 0, 100 + cfg)
    rng = np.random.default_rng(cfg)
    n_k = 70 if cfg == 2 else 13  # more than one launch of 64 k-points, and a ragged batch of 8
    k = rng.uniform(-2.0, 2.0, size=(n_k, 3))
    k[0] = 0.0
    H = plan.sigma_to_k(torch.from_numpy(sig).cuda(), k, cell=0)
    torch.cuda.synchronize()
    _check(w.cells[0], w.D[0], sig, k, H.cpu().numpy(), f"tiny[{cfg}]")


def test_multicell_second_cell_and_edges():
    import torch
    from paper_2009_12505_amd import HfxError
    log("case fourier multicell")
    parts = [hs.make_workload("tiny", kind="primitive", species_table=((2, 3), (3, 4)), species=[0, 1],
                              r_c=8.0, r_v=6.0, r_d=9.0, seed=11),
             hs.make_workload("tiny", kind="conventional", species_table=((5, 9),), r_c=7.0, r_v=9.0, r_d=10.0,
                              eps=1e-6, seed=12)]
    w = _combine(parts)
    plan = _plan(w)
    for c in range(2):
        sig = _seeded_sigma(plan, c, 7 + c)
        k = np.random.default_rng(c).uniform(-1, 1, size=(9, 3))
        H = plan.sigma_to_k(torch.from_numpy(sig).cuda(), k, cell=c)
        torch.cuda.synchronize()
        _check(w.cells[c], w.D[c], sig, k, H.cpu().numpy(), f"multicell[{c}]")
    # no k-points: nothing to do; bad cell: rejected before any launch
    s0 = torch.from_numpy(_seeded_sigma(plan, 0, 1)).cuda()
    assert plan.sigma_to_k(s0, np.zeros((0, 3)), cell=0).shape[0] == 0
    with pytest.raises(HfxError):
        plan.sigma_to_k(s0, np.zeros((1, 3)), cell=2)


@pytest.mark.timeout(600)
def test_cfg3_sigma_to_k_sampled_blocks():
    """The 512-atom supercell at the eight k-points of the 2x2x2 grid, the launch bench.py
    times; 40 seeded atom pairs (and every pair of atom 0) checked block by block."""
    import torch
    log("case fourier cfg3")
    w = hs.make_workload("cfg3", eps=1e-6)
    plan = _plan(w)
    sig = _seeded_sigma(plan, 0, 2009)
    k = np.array([[a, b, c] for a in (0.0, 0.5) for b in (0.0, 0.5) for c in (0.0, 0.5)])
    H = plan.sigma_to_k(torch.from_numpy(sig).cuda(), k, cell=0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    n = w.cells[0].n_atoms
    pairs = {(int(i), int(j)) for i, j in rng.integers(0, n, size=(40, 2))} | {(0, j) for j in range(n)}
    got = H.cpu().numpy()
    _check(w.cells[0], w.D[0], sig, k, got, "cfg3", pairs=sorted(pairs))
