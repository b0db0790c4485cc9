"""FP64 reference of the real-space density matrix from Kohn-Sham eigenvectors (test
infrastructure only; shares no code with the GPU path).

Sec. II, eq. DM_realspace: D is the Brillouin-zone average over k of the occupied projector
P(k) = sum_n f_nk c_n(k) c_n(k)^H with a lattice phase.  The printed phase
exp(-i k.(R_K - R_L)) and the k-space Hamiltonian H(k) = sum_R exp(i k.R) H(R) of the
band-structure section fix opposite Bloch conventions; this reference takes the one that makes
the two steps each other's inverse (eigenvectors of that H(k); band energy in k space equal to
the real-space trace sum_R <D(R), H(R)>):

    D_{Ii,Jj}(R) = Re (1/N_k) sum_k exp(-i 2 pi k.R) sum_n f_nk c_{Ii,n}(k) conj(c_{Jj,n}(k)),

with R the integer lattice vector of the column atom J, k in fractional coordinates of the
reciprocal lattice and N_k the number of k-points given.  The real part is taken: it is the whole
value when the k-set is closed under k -> -k with P(-k) = conj(P(k)) (time reversal).
The result is laid out on the caller's block pattern, like Sigma.
"""
from __future__ import annotations

import numpy as np

from . import sigma_offsets
from .fourier import basis_offsets


def projector(ck, occ):
    """P(k) = sum_n f_nk c_n(k) c_n(k)^H for ck [n_k, n_basis, n_occ], occ [n_k, n_occ]."""
    ck = np.asarray(ck, np.complex128)
    occ = np.asarray(occ, np.float64)
    return np.einsum("kin,kn,kjn->kij", ck, occ, np.conj(ck))


def projector_block(ci, cj, occ):
    """Rows i of ci against rows j of cj: sum_n f_nk ci[k, i, n] conj(cj[k, j, n])."""
    return np.einsum("kin,kn,kjn->kij", np.asarray(ci, np.complex128), np.asarray(occ, np.float64),
                     np.conj(np.asarray(cj, np.complex128)))


def density_from_k(cell, D, kfrac, ck, occ, pairs=None):
    """The flat D on the pattern ``D`` (offsets of ``sigma_offsets``); with ``pairs`` only the
    blocks of those (I, J) atom pairs are filled (others left at 0)."""
    kfrac = np.asarray(kfrac, np.float64).reshape(-1, 3)
    ck = np.asarray(ck, np.complex128)
    bo, _ = basis_offsets(cell)
    nao = [cell.species_table[int(s)][0] for s in cell.species]
    off = sigma_offsets(cell, D)
    want = None if pairs is None else {(int(i), int(j)) for i, j in pairs}
    out = np.zeros(int(off[-1]), np.float64)
    nk = kfrac.shape[0]
    P = {}  # the blocks of P(k) the pattern needs, one atom pair at a time
    for b in range(D.n_blocks):
        I, J = int(D.row[b]), int(D.col[b])
        if want is not None and (I, J) not in want:
            continue
        if (I, J) not in P:
            P[(I, J)] = projector_block(ck[:, bo[I]:bo[I] + nao[I]], ck[:, bo[J]:bo[J] + nao[J]], occ)
        phase = np.exp(-2j * np.pi * (kfrac @ np.asarray(D.R[b], np.float64)))
        blk = (phase[:, None, None] * P[(I, J)]).sum(axis=0) / nk
        out[off[b]:off[b + 1]] = blk.real.ravel()
    return out
