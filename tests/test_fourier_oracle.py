"""Pins of the FP64 reference of the real-space to k-space sum (oracle.fourier).

- a one-orbital simple-cubic tight-binding model, whose H(k) has the textbook closed form
  e0 + 2 t (cos 2 pi kx + cos 2 pi ky + cos 2 pi kz);
- band folding: the eigenvalues of a 2x2x2 supercell's H(K) are the union of the primitive
  cell's eigenvalues at the eight k = (K + m) / 2 (m in {0,1}^3), and H(K) maps Bloch vectors
  of the supercell to those of H(k) -- fixes the phase sign, the R of the column atom and the
  block placement;
- Hermiticity when H_JI(-R) = H_IJ(R)^T, periodicity H(k + G) = H(k), and the block subset
  agreeing with the full matrix.
"""
import itertools

import numpy as np

import hfx_synth as hs
from oracle import fourier


def _pattern(blocks, cell):
    """Blocks from a dict (I, J, R tuple) -> matrix, in a fixed order."""
    keys = sorted(blocks)
    nao = [cell.species_table[int(s)][0] for s in cell.species]
    data, off, o = [], [], 0
    for (i, j, R) in keys:
        b = np.asarray(blocks[(i, j, R)], np.float64)
        assert b.shape == (nao[i], nao[j])
        off.append(o)
        data.append(b.ravel())
        o += b.size
    D = hs.Blocks(np.array([k[0] for k in keys], np.int32), np.array([k[1] for k in keys], np.int32),
                  np.array([k[2] for k in keys], np.int32).reshape(-1, 3), np.array(off, np.int64),
                  np.concatenate(data), "D")
    return D, D.data


def test_tight_binding_closed_form():
    cell = hs.Cell(np.eye(3) * 5.0, np.zeros((1, 3)), np.zeros(1, np.int32), [(1, 1)])
    e0, t = -0.7, 0.25
    blocks = {(0, 0, (0, 0, 0)): [[e0]]}
    for ax in range(3):
        for s in (1, -1):
            R = [0, 0, 0]
            R[ax] = s
            blocks[(0, 0, tuple(R))] = [[t]]
    D, sig = _pattern(blocks, cell)
    k = np.random.default_rng(1).uniform(-1.5, 1.5, size=(17, 3))
    H = fourier.sigma_to_k(cell, D, sig, k)
    want = e0 + 2 * t * np.cos(2 * np.pi * k).sum(axis=1)
    assert np.max(np.abs(H[:, 0, 0] - want)) <= 1e-14


def _primitive_operator(seed=3):
    """A real-space operator on a 2-atom fcc cell (2 and 3 orbitals) with blocks within 9 bohr,
    H_JI(-R) = H_IJ(R)^T."""
    a = 6.0
    L = np.array([[0, a / 2, a / 2], [a / 2, 0, a / 2], [a / 2, a / 2, 0]])
    pos = np.array([[0.0, 0.0, 0.0], [a / 4, a / 4, a / 4]])
    cell = hs.Cell(L, pos, np.array([0, 1], np.int32), [(2, 1), (3, 1)])
    nao = [2, 3]
    rng = np.random.default_rng(seed)
    blocks = {}
    rng_R = range(-3, 4)
    for i, j in itertools.product(range(2), range(2)):
        for R in itertools.product(rng_R, rng_R, rng_R):
            d = pos[j] + np.asarray(R) @ L - pos[i]
            if np.linalg.norm(d) > 9.0 or (i, j, R) in blocks:
                continue
            b = rng.normal(size=(nao[i], nao[j])) * np.exp(-np.linalg.norm(d) / 3)
            mR = tuple(-x for x in R)
            if (i, j, R) == (j, i, mR):
                b = 0.5 * (b + b.T)
            blocks[(i, j, R)] = b
            blocks[(j, i, mR)] = b.T
    return cell, blocks


def test_hermitian_and_periodic():
    cell, blocks = _primitive_operator()
    D, sig = _pattern(blocks, cell)
    k = np.random.default_rng(2).uniform(-1, 1, size=(6, 3))
    H = fourier.sigma_to_k(cell, D, sig, k)
    assert np.max(np.abs(H - np.conj(np.transpose(H, (0, 2, 1))))) <= 1e-13
    G = np.array([[1, 0, -2], [0, 3, 1], [-1, -1, -1], [2, 0, 0], [0, 0, 5], [1, 1, 1]])
    H2 = fourier.sigma_to_k(cell, D, sig, k + G)
    assert np.max(np.abs(H2 - H)) <= 1e-11
    sub = fourier.sigma_to_k(cell, D, sig, k, pairs=[(0, 1), (1, 1)])
    bo, _ = fourier.basis_offsets(cell)
    assert np.array_equal(sub[(0, 1)], H[:, 0:2, 2:5]) and np.array_equal(sub[(1, 1)], H[:, 2:5, 2:5])


def test_band_folding_supercell_vs_primitive():
    cp, bp = _primitive_operator()
    Lp = cp.lattice
    # 2x2x2 supercell: atom (m, i) at r_i + m.Lp, lattice 2 Lp
    ms = list(itertools.product(range(2), repeat=3))
    pos = np.array([cp.pos[i] + np.asarray(m) @ Lp for m in ms for i in range(2)])
    spec = np.array([i for m in ms for i in range(2)], np.int32)
    cs = hs.Cell(2 * Lp, pos, spec, cp.species_table)
    sc = {}
    for (i, j, n), b in bp.items():
        n = np.asarray(n)
        for mi, mI in enumerate(ms):
            t = n + np.asarray(mI)
            mJ = tuple(int(x) % 2 for x in t)
            Rs = tuple(int(x) for x in (t - np.asarray(mJ)) // 2)
            I, J = 2 * mi + i, 2 * ms.index(mJ) + j
            sc[(I, J, Rs)] = b
    Ds, ss = _pattern(sc, cs)
    Dp, sp = _pattern(bp, cp)
    for K in (np.zeros(3), np.array([0.13, -0.31, 0.27])):
        Hs = fourier.sigma_to_k(cs, Ds, ss, K[None])[0]
        ev_s = np.linalg.eigvalsh(Hs)
        kp = np.array([(K + np.asarray(m)) / 2 for m in ms])
        Hp = fourier.sigma_to_k(cp, Dp, sp, kp)
        ev_p = np.sort(np.concatenate([np.linalg.eigvalsh(h) for h in Hp]))
        assert ev_s.shape == ev_p.shape
        assert np.max(np.abs(ev_s - ev_p)) <= 1e-11 * max(1.0, np.max(np.abs(ev_p)))
        # Bloch vectors: x_(m,j) = exp(i 2 pi k.m) y_j is mapped by H_sc(K) to
        # exp(i 2 pi k.m) (H_p(k) y)_i -- this fixes the sign of the phase, not only the spectrum
        y = np.random.default_rng(5).normal(size=5) + 1j * np.random.default_rng(6).normal(size=5)
        for q, k in enumerate(kp):
            ph = np.exp(2j * np.pi * np.array([np.dot(k, m) for m in ms]))
            x = np.concatenate([p * y for p in ph])
            want = np.concatenate([p * (Hp[q] @ y) for p in ph])
            assert np.max(np.abs(Hs @ x - want)) <= 1e-11 * max(1.0, np.max(np.abs(want)))
