"""Definition-level checker: explicit four-centre integrals (tiny inputs only).

TEST INFRASTRUCTURE ONLY.  Follows the <I,J>-outer loop of Algorithm 1 with
the full ERIs assembled from the pair expansion of eq. LRI:

    (Ii Kk | Jj Ll) = sum_{A in S(I,K)} sum_{B in S(J,L)} sum_{alpha,beta}
                      C^{A alpha}_{Ii,Kk} V_{A alpha, B beta} C^{B beta}_{Jj,Ll}

(eq. HFX_LRI / eq. ERI_split), where S(I,K) is the set {I, K} of atom images
(a single element when K is I itself), C^{I alpha}_{Ii,Kk} is the stored block
C(I,K)[alpha,i,k] and C^{K alpha}_{Ii,Kk} is C(K,I)[alpha,k,i].  Then

    K_{Ii,Jj}(R) = sum_{K,L} sum_{k,l} (Ii Kk | Jj Ll) D_{Kk,Ll}     (eq. HFX_ERIs)
    Sigma^X = -K, returned on the D block pattern.

No screening of any kind: this is the plain definition the screened method
approximates.  Blocks are translation invariant: the block between X at R1 and
Y at R2 is the stored (X, Y, R2 - R1).
"""
from __future__ import annotations

import numpy as np


def _tkey(r, c, R):
    return (int(r), int(c), (int(R[0]), int(R[1]), int(R[2])))


def _lookup(dct, X, Y):
    """Block between atom-images X=(x,Rx) and Y=(y,Ry)."""
    (x, Rx), (y, Ry) = X, Y
    return dct.get((x, y, (Ry[0] - Rx[0], Ry[1] - Rx[1], Ry[2] - Rx[2])))


def _pair_expansion(Cd, I, K):
    """[(ABF atom-image, E[alpha,i,k])] for the product phi_I i * phi_K k."""
    out = []
    c_ik = _lookup(Cd, I, K)
    if I == K:
        if c_ik is not None:
            out.append((I, c_ik))
        return out
    if c_ik is not None:
        out.append((I, c_ik))
    c_ki = _lookup(Cd, K, I)
    if c_ki is not None:
        out.append((K, c_ki.transpose(0, 2, 1)))
    return out


def eri(Cd, Vd, I, K, J, L):
    """(I i K k | J j L l) as an array [i,k,j,l]."""
    e1 = _pair_expansion(Cd, I, K)
    e2 = _pair_expansion(Cd, J, L)
    out = None
    for A, E in e1:
        for B, F in e2:
            v = _lookup(Vd, A, B)
            if v is None:
                continue
            t = np.einsum("aik,ab,bjl->ikjl", E, v, F, optimize=True)
            out = t if out is None else out + t
    return out


def sigma(cell, C, V, D):
    """Sigma^X on the D pattern, keyed (I, J, R) with I a home atom."""
    Cd, Vd, Dd = C.as_dict(cell), V.as_dict(cell), D.as_dict(cell)
    z = (0, 0, 0)
    # neighbours K of a home atom I: atom images that share a C block with I (either orientation)
    nbr = {}
    for (r, c, R) in Cd:
        nbr.setdefault(r, set()).add((c, R))
        nbr.setdefault(c, set()).add((r, (-R[0], -R[1], -R[2])))
    out = {}
    for (i, j, R), dblk in Dd.items():
        I = (i, z)
        J = (j, R)
        acc = np.zeros((dblk.shape[0], dblk.shape[1]))
        for (k, RK) in nbr.get(i, ()):
            K = (k, RK)
            for (l, RL0) in nbr.get(j, ()):
                L = (l, (RL0[0] + R[0], RL0[1] + R[1], RL0[2] + R[2]))
                dkl = _lookup(Dd, K, L)
                if dkl is None:
                    continue
                e = eri(Cd, Vd, I, K, J, L)
                if e is None:
                    continue
                acc += np.einsum("ikjl,kl->ij", e, dkl)
        out[(i, j, R)] = -acc
    return out


def energy(cell, D, sig: dict) -> float:
    Dd = D.as_dict(cell)
    return 0.5 * float(sum(np.sum(Dd[k] * v) for k, v in sig.items()))
