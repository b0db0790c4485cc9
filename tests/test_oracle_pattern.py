"""The reading that Sigma is produced on the block pattern of D (a contribution whose target
block is outside that pattern is not formed) does not change the result on the workloads: with
D's pattern zero-extended to every pair any unit can reach (|F - G| <= C range + V range + C
range), no unit with a target outside the original pattern survives the screening of
Sec. III C, so every added Sigma block stays exactly zero.  The zero-valued D blocks added to the
pattern are removed by the D pre-screen (Sec. III B) and so never serve as an operand; the
in-pattern result is therefore unchanged."""
import numpy as np
import pytest

import hfx_synth as hs
import oracle


def _extend_pattern(cell, D, radius):
    row, col, R, _ = hs.enumerate_pairs(cell.lattice, cell.pos, radius)
    have = {(int(r), int(c), tuple(int(x) for x in RR)) for r, c, RR in zip(D.row, D.col, D.R)}
    extra = [k for k in range(row.shape[0]) if (int(row[k]), int(col[k]), tuple(int(x) for x in R[k])) not in have]
    nao = np.asarray([cell.species_table[s][0] for s in cell.species], np.int64)
    sizes = nao[row[extra]] * nao[col[extra]]
    base = D.data.shape[0]
    data = np.concatenate([D.data, np.zeros(int(sizes.sum()))])
    off = base + np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if extra else np.zeros(0, np.int64)
    ext = hs.Blocks(np.r_[D.row, row[extra]].astype(np.int32), np.r_[D.col, col[extra]].astype(np.int32),
                    np.r_[D.R, R[extra]].astype(np.int32), np.r_[D.off, off].astype(np.int64), data, "D")
    return ext, D.n_blocks, len(extra)


def _check(w, cell_idx, home, radius):
    cell = w.cells[cell_idx]
    De, n0, n_extra = _extend_pattern(cell, w.D[cell_idx], radius)
    assert n_extra > 0
    r = oracle.run(cell, w.C[cell_idx], w.V[cell_idx], De, w.thresholds, home=home, n_threads=8)
    off = r.sig_off
    outside = r.sigma[off[n0]:]
    inside = r.sigma[:off[n0]]
    assert r.stats["units_formed"] > 0 and np.abs(inside).max() > 0
    assert np.count_nonzero(outside) == 0, "a unit with a target outside D's pattern survived the screening"


@pytest.mark.parametrize("eps", [1e-4, pytest.param(1e-6, marks=pytest.mark.slow)])
def test_cfg3_sigma_stays_on_the_density_pattern(eps):
    """512-atom crystal's primitive cell (same keyed blocks): C within 16 bohr, V within 36, D
    within 45; targets can lie up to 16 + 36 + 16 = 68 bohr away, the pattern is extended to 70."""
    w = hs.make_workload("cfg3prim", eps=eps)
    _check(w, 0, [0], 70.0)


def test_cfg4_sigma_stays_on_the_density_pattern():
    """A two-species cell of the batched workload (C within 12 bohr, V 24, D 30, eps 1e-4), one
    home atom of each species; targets can lie up to 48 bohr away, the pattern is extended to 50."""
    w = hs.make_workload("cfg4", n_cells=1)
    cell = w.cells[0]
    homes = [int(np.nonzero(cell.species == s)[0][0]) for s in (0, 1) if np.any(cell.species == s)]
    assert len(homes) == 2
    _check(w, 0, homes, 50.0)
