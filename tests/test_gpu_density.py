"""GPU parity of the density matrix from eigenvectors (hfx_density_from_k) against the FP64
oracle (oracle.density), element by element, on seeded eigenvectors and occupations; and the
GPU round trip Sigma(R) -> H(k) (hfx_sigma_to_k) -> eigenvectors -> D(R) = Sigma(R).

Bound: each element of D is (1/N_k) sum over k and bands of f c conj(c) exp(-i k.R); FP64
summation in another order differs by a few ulps of the sum of the terms' magnitudes, so
|dD| <= 1e-13 * (1/N_k) sum_k sum_n |f| |c_i| |c_j| for every element."""
import numpy as np
import pytest

import hfx_synth as hs
from oracle import density, fourier
from test_gpu_parity import TINY, log

pytestmark = pytest.mark.gpu


def _plan(w):
    from paper_2009_12505_amd import Plan
    return Plan(w.cells, w.C, w.V, w.D, w.thresholds)


def _inputs(nb, n_k, n_occ, seed):
    rng = np.random.default_rng(seed)
    ck = rng.normal(size=(n_k, nb, n_occ)) + 1j * rng.normal(size=(n_k, nb, n_occ))
    occ = rng.uniform(0.0, 2.0, size=(n_k, n_occ))
    k = rng.uniform(-1.5, 1.5, size=(n_k, 3))
    return ck, occ, k


def _run(plan, ck, occ, k, cell=0):
    import torch
    d = plan.density_from_k(torch.from_numpy(ck).cuda(), torch.from_numpy(occ).cuda(), k, cell=cell)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def _check(cell, D, k, ck, occ, got, label, pairs=None):
    ref = density.density_from_k(cell, D, k, ck, occ, pairs=pairs)
    mag = density.density_from_k(cell, D, np.zeros_like(k), np.abs(ck), np.abs(occ), pairs=pairs)
    if pairs is not None:
        off = density.sigma_offsets(cell, D)
        keep = np.zeros(ref.size, bool)
        for b in range(D.n_blocks):
            if (int(D.row[b]), int(D.col[b])) in set(pairs):
                keep[off[b]:off[b + 1]] = True
        got, ref, mag = got[keep], ref[keep], mag[keep]
    err = np.abs(got - ref)
    bound = 1e-13 * mag + 1e-300
    log(f"{label}: {ref.size} elements, max|D| {np.abs(ref).max():.3e} max|dD| {err.max():.3e} "
        f"(worst / bound {float(np.max(err / bound)):.3f})")
    assert np.all(err <= bound)


@pytest.mark.parametrize("cfg,n_k,n_occ", [(0, 5, 3), (2, 70, 4), (4, 9, 40), (6, 4, 33), (5, 3, 0)])
def test_tiny_density(cfg, n_k, n_occ):
    log(f"case density tiny[{cfg}] n_k={n_k} n_occ={n_occ}")
    w = hs.make_workload("tiny", **TINY[cfg])
    plan = _plan(w)
    nb = plan.n_basis[0]
    ck, occ, k = _inputs(nb, n_k, n_occ, 50 + cfg)
    got = _run(plan, ck, occ, k)
    if n_occ == 0:
        assert not np.any(got)
        return
    _check(w.cells[0], w.D[0], k, ck, occ, got, f"tiny[{cfg}]")


def test_round_trip_through_k_space():
    """Sigma(R) (seeded, made Hermitian on the pattern) -> H(k) on a 6^3 grid on the GPU ->
    eigenvectors (host) with their eigenvalues as occupations -> D(R) on the GPU == Sigma(R)."""
    import torch
    log("case density round trip")
    w = hs.make_workload("tiny", **TINY[1])
    plan = _plan(w)
    D = w.D[0]
    off = density.sigma_offsets(w.cells[0], D)
    idx = {(int(D.row[b]), int(D.col[b]), tuple(int(x) for x in D.R[b])): b for b in range(D.n_blocks)}
    assert max(abs(int(x)) for x in D.R.ravel()) < 3  # no aliasing on the 6^3 grid
    rng = np.random.default_rng(8)
    sig = np.zeros(plan.sizes[0])
    nao = [w.cells[0].species_table[int(s)][0] for s in w.cells[0].species]
    for (i, j, R), b in idx.items():
        bm = idx[(j, i, tuple(-x for x in R))]
        if bm < b:
            continue
        blk = rng.normal(size=(nao[i], nao[j]))
        if bm == b:
            blk = 0.5 * (blk + blk.T)
        sig[off[b]:off[b + 1]] = blk.ravel()
        sig[off[bm]:off[bm + 1]] = blk.T.ravel()
    N = 6
    k = np.array([[a / N, b / N, c / N] for a in range(N) for b in range(N) for c in range(N)])
    H = plan.sigma_to_k(torch.from_numpy(sig).cuda(), k).cpu().numpy()
    lam, U = np.linalg.eigh(H)
    got = _run(plan, U, lam, k)
    err = float(np.max(np.abs(got - sig)))
    log(f"round trip: max|Sigma| {np.abs(sig).max():.3e} max|D - Sigma| {err:.3e}")
    assert err <= 1e-11 * np.abs(sig).max()


@pytest.mark.timeout(600)
def test_cfg3_gamma_sampled_blocks():
    """The 512-atom supercell at the Gamma point with 64 bands: 40 seeded atom pairs (and every
    pair of atom 0) checked block by block."""
    log("case density cfg3 Gamma")
    w = hs.make_workload("cfg3", eps=1e-6)
    plan = _plan(w)
    ck, occ, _ = _inputs(plan.n_basis[0], 1, 64, 2009)
    k = np.zeros((1, 3))
    got = _run(plan, ck, occ, k)
    n = w.cells[0].n_atoms
    rng = np.random.default_rng(4)
    pairs = {(int(i), int(j)) for i, j in rng.integers(0, n, size=(40, 2))} | {(0, j) for j in range(n)}
    _check(w.cells[0], w.D[0], k, ck, occ, got, "cfg3 Gamma", pairs=sorted(pairs))
