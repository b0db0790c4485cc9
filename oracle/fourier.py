"""FP64 reference of the lattice Fourier sum that takes the real-space exchange matrix to
k space (test infrastructure only; shares no code with the GPU path).

The band-structure step of the paper (the real-space to k-space equation, Ham_rs2kspace)
builds the matrix at any k from the real-space blocks:

    H_{Ii,Jj}(k) = sum_R exp(i k.R) H_{Ii,Jj}(R),

with R the lattice vector of the column atom J (the row atom I in the home cell).  Here k is
given in fractional coordinates of the reciprocal lattice, so k.R = 2 pi (k_frac . n_R) with
n_R the integer coordinates of R.  The sum runs over the blocks the caller's pattern holds
(the pattern of D, on which Sigma is produced).  Plain loops over blocks; numpy exponentials.
"""
from __future__ import annotations

import numpy as np

from . import sigma_offsets


def basis_offsets(cell):
    """First basis index of every atom of the cell, and the basis size."""
    nao = np.asarray([cell.species_table[int(s)][0] for s in cell.species], np.int64)
    off = np.concatenate([[0], np.cumsum(nao)])
    return off[:-1], int(off[-1])


def sigma_to_k(cell, D, sigma, kfrac, pairs=None):
    """H(k) for every row of ``kfrac`` ([n_k, 3] fractional), as a complex array
    [n_k, n_basis, n_basis]; with ``pairs`` (an iterable of (I, J) atom pairs) only those
    blocks, as a dict (I, J) -> [n_k, n_ao(I), n_ao(J)]."""
    kfrac = np.asarray(kfrac, np.float64).reshape(-1, 3)
    bo, nbas = basis_offsets(cell)
    nao = [cell.species_table[int(s)][0] for s in cell.species]
    off = sigma_offsets(cell, D)
    want = None if pairs is None else {(int(i), int(j)) for i, j in pairs}
    if want is None:
        H = np.zeros((kfrac.shape[0], nbas, nbas), np.complex128)
    else:
        H = {p: np.zeros((kfrac.shape[0], nao[p[0]], nao[p[1]]), np.complex128) for p in want}
    for b in range(D.n_blocks):
        I, J = int(D.row[b]), int(D.col[b])
        if want is not None and (I, J) not in want:
            continue
        blk = np.asarray(sigma[off[b]:off[b + 1]], np.float64).reshape(nao[I], nao[J])
        phase = np.exp(2j * np.pi * (kfrac @ np.asarray(D.R[b], np.float64)))
        if want is None:
            H[:, bo[I]:bo[I] + nao[I], bo[J]:bo[J] + nao[J]] += phase[:, None, None] * blk
        else:
            H[(I, J)] += phase[:, None, None] * blk
    return H
