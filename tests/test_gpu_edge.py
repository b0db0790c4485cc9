"""Degenerate and extreme inputs on the GPU against the oracle: everything screened out, no
home atoms, a single isolated atom (one work item, on-site units only), and the largest block
the kernels take (32 AOs per atom)."""
import numpy as np
import pytest

import hfx_synth as hs
import oracle
from test_gpu_parity import check_close, gpu_build, log

pytestmark = pytest.mark.gpu


def _ref(w, **kw):
    return oracle.run(w.cells[0], w.C[0], w.V[0], w.D[0], w.thresholds, n_threads=8, **kw)


def test_everything_screened_out():
    log("case all screened")
    w = hs.make_workload("tiny", kind="conventional", species_table=((5, 9),), r_c=7.0, r_v=9.0, r_d=10.0, eps=1e3)
    ref = _ref(w)
    sig, e, st = gpu_build(w)
    assert not np.any(ref.sigma) and not np.any(sig[0])
    assert e[0] == 0.0
    assert all(st[f"kept_s3_t{t}"] == 0 for t in (1, 2, 3, 4))


def test_no_home_atoms():
    log("case empty home subset")
    w = hs.make_workload("tiny", kind="conventional", species_table=((4, 7),), r_c=7.0, r_v=9.0, r_d=10.0, eps=1e-6)
    ref = _ref(w, home=[])
    sig, e, st = gpu_build(w, home_subset=[])
    assert st["items"] == 0
    assert not np.any(ref.sigma) and not np.any(sig[0])


def test_isolated_atom_single_item():
    log("case isolated atom")
    w = hs.make_workload("tiny", kind="custom", lattice=np.eye(3) * 400.0, pos=[[0.0, 0.0, 0.0]],
                         species_table=((6, 11),), r_c=6.0, r_v=6.0, r_d=6.0)
    ref = _ref(w)
    sig, e, st = gpu_build(w)
    assert st["items"] == 1
    check_close(sig[0], ref.sigma, label="isolated atom")


def test_largest_block_size():
    log("case n_ao = 32")
    w = hs.make_workload("tiny", kind="primitive", species_table=((32, 48), (7, 12)), species=[0, 1], r_c=5.0,
                         r_v=6.0, r_d=6.0, eps=1e-5)
    ref = _ref(w)
    sig, e, st = gpu_build(w)
    check_close(sig[0], ref.sigma, label="n_ao 32")
    for t in (1, 2, 3, 4):
        assert st[f"kept_s3_t{t}"] == ref.stats[f"kept_s3_t{t}"]
