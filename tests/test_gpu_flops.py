"""The build's FLOP counters against the oracle's counts.

flops_paper is the numerator of the benchmark's TFLOP/s; flops_contract the library's own count.
On cells of one species (n_ao = n, n_abf = P) both follow from the number of kept units of each
term and the number of (A,B,G) whose Y = V C is formed, with the product sizes of Algorithm 3
(2 FLOPs per multiply-add):

* Algorithm 3: per kept unit of terms 1, 2 the products T_t = Y D and Htilde_t = C T_t, of terms
  3, 4 Htilde_t (T3 and T4 are formed once per G), each 2 P n^3; per formed Y: Y itself, 2 P^2 n^2,
  and T3, T4, 2 P n^3 each;
* the library: one block product per kept unit, 2 P n^3; per formed Y: Y, T3, T4, the two Gram
  matrices Y_b^T Y_b and Y_g^T Y_g (2 P n^3 each) and the two contractions with Y (2 P n^3 each).

The counts come from the oracle (kept units after stage 3, Y formed), and the GPU's count of G's
whose Y it forms must equal the oracle's."""
import pytest

import hfx_synth as hs
import oracle
from test_gpu_parity import TINY, gpu_build, log

pytestmark = pytest.mark.gpu

CASES = {"eps0": TINY[1], "eps1e-6": TINY[4], "eps1e-3": dict(TINY[4], eps=1e-3)}


@pytest.mark.parametrize("name", list(CASES))
def test_flop_counts_follow_the_kept_units(name):
    log(f"case FLOP counters {name}")
    w = hs.make_workload("tiny", **CASES[name])
    cell = w.cells[0]
    assert len(cell.species_table) == 1
    n, P = cell.species_table[0]
    ref = oracle.run(cell, w.C[0], w.V[0], w.D[0], w.thresholds, n_threads=8)
    _, _, st = gpu_build(w)
    k = [ref.stats[f"kept_s3_t{t}"] for t in (1, 2, 3, 4)]
    y = ref.stats["y_formed"]
    unit = 2 * P * n ** 3
    y_cost = 2 * P * P * n * n
    paper = 2 * unit * (k[0] + k[1]) + unit * (k[2] + k[3]) + y * (y_cost + 2 * unit)
    contract = unit * sum(k) + y * (y_cost + 6 * unit)
    log(f"  kept {k}, Y formed {y} (GPU {st['g_alive']}); flops_paper {st['flops_paper']:.6e} "
        f"(expected {paper:.6e}), flops_contract {st['flops_contract']:.6e} (expected {contract:.6e})")
    assert sum(k) > 0
    assert [st[f"kept_s3_t{t}"] for t in (1, 2, 3, 4)] == k
    assert st["g_alive"] == y
    assert st["flops_paper"] == pytest.approx(paper, rel=1e-12)
    assert st["flops_contract"] == pytest.approx(contract, rel=1e-12)
