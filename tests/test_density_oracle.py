"""Pins of the FP64 reference of the real-space density matrix from eigenvectors
(oracle.density):

- full occupation: with unitary eigenvector matrices on a uniform N^3 grid the density matrix is
  the identity at R = 0 and zero at every other R of the pattern (|R_i| < N);
- inverse of the k-space sum: eigenvectors of H(k) = sum_R exp(i k.R) H(R) with their eigenvalues
  as occupations give back H(R) (no aliasing: the pattern spans less than half the grid);
- band energy: (1/N_k) sum_k sum_n f_nk e_nk equals the real-space trace sum_R <D(R), H(R)> --
  an identity between k space and real space that fixes the sign of the phase (the operator has
  no inversion symmetry).
"""
import numpy as np

from oracle import density, fourier
from test_fourier_oracle import _pattern, _primitive_operator


def _grid(N):
    return np.array([[a / N, b / N, c / N] for a in range(N) for b in range(N) for c in range(N)])


def test_full_occupation_gives_identity():
    cell, blocks = _primitive_operator()
    D, _ = _pattern(blocks, cell)
    k = _grid(4)
    nb = 5
    rng = np.random.default_rng(0)
    ck = np.stack([np.linalg.qr(rng.normal(size=(nb, nb)) + 1j * rng.normal(size=(nb, nb)))[0] for _ in k])
    occ = np.ones((len(k), nb))
    d = density.density_from_k(cell, D, k, ck, occ)
    off = density.sigma_offsets(cell, D)
    nao = [cell.species_table[int(s)][0] for s in cell.species]
    for b in range(D.n_blocks):
        blk = d[off[b]:off[b + 1]]
        on_site = D.row[b] == D.col[b] and not np.any(D.R[b])
        want = np.eye(nao[D.row[b]]).ravel() if on_site else np.zeros(blk.size)
        assert np.max(np.abs(blk - want)) <= 1e-13


def test_inverse_of_the_k_space_sum():
    cell, blocks = _primitive_operator()
    D, h = _pattern(blocks, cell)
    k = _grid(8)
    Hk = fourier.sigma_to_k(cell, D, h, k)
    lam, U = np.linalg.eigh(Hk)
    d = density.density_from_k(cell, D, k, U, lam)
    assert np.max(np.abs(d - h)) <= 1e-12 * np.max(np.abs(h))


def test_band_energy_equals_real_space_trace():
    cell, blocks = _primitive_operator(seed=9)
    D, h = _pattern(blocks, cell)
    k = _grid(6)
    Hk = fourier.sigma_to_k(cell, D, h, k)
    lam, U = np.linalg.eigh(Hk)
    n_occ = 2
    occ = np.full((len(k), n_occ), 2.0)
    e_k = float(np.sum(occ * lam[:, :n_occ])) / len(k)
    d = density.density_from_k(cell, D, k, U[:, :, :n_occ], occ)
    e_r = float(np.dot(d, h))
    assert abs(e_k - e_r) <= 1e-11 * max(1.0, abs(e_k))
    # the same with the phase sign flipped would pair D(-R) with H(R): not equal here
    d_flip = np.zeros_like(d)
    off = density.sigma_offsets(cell, D)
    idx = {(int(D.row[b]), int(D.col[b]), tuple(int(x) for x in D.R[b])): b for b in range(D.n_blocks)}
    for (i, j, R), b in idx.items():
        bm = idx[(i, j, tuple(-x for x in R))] if (i, j, tuple(-x for x in R)) in idx else None
        if bm is not None:
            d_flip[off[b]:off[b + 1]] = d[off[bm]:off[bm + 1]]
    assert abs(float(np.dot(d_flip, h)) - e_k) > 1e-6 * max(1.0, abs(e_k))
