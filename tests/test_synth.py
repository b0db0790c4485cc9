"""Invariants of the seeded synthetic inputs (hfx_synth), which both the oracle and the GPU
path consume: V(R) = V(-R)^T and D(R) = D(-R)^T block by block; V and D positive definite as
Bloch sums at Gamma and at random k (V is a positive-definite kernel matrix plus a diagonal
shift, D a tapered positive-definite kernel times a Gram matrix); and translation keying:
every block of a supercell equals the primitive cell's block of the same atom pair and
displacement."""
import numpy as np
import pytest

import hfx_synth as hs
from oracle import fourier


def _as_ao(cell, which):
    """The cell with the block dimension of ``which`` (0: AO, 1: ABF) as its 'AO' count, so that
    the k-space sum of the oracle can form Bloch sums of V as well as D."""
    tab = [(s[which], s[which]) for s in cell.species_table]
    return hs.Cell(cell.lattice, cell.pos, cell.species, tab)


def _transpose_partners(B, cell, which):
    n = [cell.species_table[int(s)][which] for s in cell.species]
    idx = {(int(B.row[b]), int(B.col[b]), tuple(int(x) for x in B.R[b])): b for b in range(B.n_blocks)}
    worst = 0.0
    for (i, j, R), b in idx.items():
        bm = idx[(j, i, tuple(-x for x in R))]
        x = B.data[B.off[b]:B.off[b] + n[i] * n[j]].reshape(n[i], n[j])
        y = B.data[B.off[bm]:B.off[bm] + n[j] * n[i]].reshape(n[j], n[i])
        worst = max(worst, float(np.abs(x - y.T).max()))
    return worst


def _compact(B, cell, which):
    """Block data in the compact order of the pattern (what the k-space sum expects)."""
    n = [cell.species_table[int(s)][which] for s in cell.species]
    return np.concatenate([B.data[B.off[b]:B.off[b] + n[B.row[b]] * n[B.col[b]]] for b in range(B.n_blocks)])


@pytest.mark.parametrize("name,kw", [("cfg1", {}), ("tiny", dict(kind="conventional", species_table=((4, 7), (6, 10)),
                                                                   species=[0, 1] * 4, r_c=7.0, r_v=9.0, r_d=10.0))])
def test_symmetry_and_positive_definiteness(name, kw):
    w = hs.make_workload(name, **kw)
    cell = w.cells[0]
    k = np.vstack([np.zeros(3), np.random.default_rng(1).uniform(-0.5, 0.5, size=(4, 3))])
    for B, which in ((w.V[0], 1), (w.D[0], 0)):
        assert _transpose_partners(B, cell, which) == 0.0
        c = _as_ao(cell, which)
        H = fourier.sigma_to_k(c, B, _compact(B, cell, which), k)
        for h in H:
            assert np.abs(h - h.conj().T).max() <= 1e-12 * np.abs(h).max()
            assert np.linalg.eigvalsh(h).min() > 0.0


def test_supercell_blocks_equal_primitive_blocks():
    ws, wp = hs.make_workload("cfg2"), hs.make_workload("cfg2prim")
    cs, cp = ws.cells[0], wp.cells[0]
    pi, pR = hs.map_to_primitive(cs, cp)
    conv = np.rint(cs.lattice @ np.linalg.inv(cp.lattice)).astype(np.int64)
    for which, Bs, Bp in ((1, ws.V[0], wp.V[0]), (0, ws.D[0], wp.D[0])):
        n = [cp.species_table[int(s)][which] for s in cp.species]
        prim = {(int(Bp.row[b]), int(Bp.col[b]), tuple(int(x) for x in Bp.R[b])): b for b in range(Bp.n_blocks)}
        rng = np.random.default_rng(which)
        for b in rng.choice(Bs.n_blocks, size=200, replace=False):
            i, j = int(Bs.row[b]), int(Bs.col[b])
            Rp = tuple(int(x) for x in (np.asarray(Bs.R[b]) @ conv + pR[j] - pR[i]))
            q = prim[(int(pi[i]), int(pi[j]), Rp)]
            m = n[pi[i]] * n[pi[j]]
            assert np.array_equal(Bs.data[Bs.off[b]:Bs.off[b] + m], Bp.data[Bp.off[q]:Bp.off[q] + m])


def test_keyed_stream_is_splitmix64():
    """The counter-based stream behind every keyed block is SplitMix64 (Steele, Lea & Flood 2014):
    key 0 at counters 0..3 gives the first four outputs of the published generator seeded with 0."""
    b = hs._bits(np.array([0], np.uint64), np.arange(4, dtype=np.uint64))[0]
    assert [int(x) for x in b] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
