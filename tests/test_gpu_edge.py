"""Degenerate and extreme inputs on the GPU against the oracle: everything screened out, no
home atoms, a single isolated atom (one work item, on-site units only), the largest block the
kernels take (32 AOs per atom) and the smallest (one AO or one ABF per atom)."""
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


@pytest.mark.parametrize("table", [((1, 1), (1, 3)), ((3, 1), (2, 1)), ((1, 2), (3, 5))])
def test_smallest_block_sizes(table):
    """One AO or one ABF per atom (blocks from 1x1 up): the degenerate end of the block shapes, next
    to slightly larger ones, in a two-species conventional cell."""
    log(f"case smallest blocks {table}")
    w = hs.make_workload("tiny", kind="conventional", species_table=table, species=[0, 1] * 4, r_c=6.0, r_v=7.0,
                         r_d=8.0, eps=1e-6)
    ref = _ref(w)
    sig, e, st = gpu_build(w)
    check_close(sig[0], ref.sigma, label=f"blocks {table}")
    assert abs(e[0] - oracle.energy(w.cells[0], w.D[0], ref.sigma)) <= 1e-11 * abs(e[0]) + 1e-300
    for t in (1, 2, 3, 4):
        assert st[f"kept_s3_t{t}"] == ref.stats[f"kept_s3_t{t}"]


def test_density_pattern_mismatch_is_a_state_error():
    """hfx_build checks that D carries the plan's pattern: a different block count, different
    offsets or a different block structure is HFX_ERR_STATE, and the plan stays usable."""
    import hfx_synth as hs2
    from paper_2009_12505_amd import Plan, _abi as A
    log("case D pattern mismatch")
    w = hs.make_workload("tiny", kind="primitive", species_table=((3, 5),), r_c=6.0, r_v=6.0, r_d=7.0, eps=1e-6)
    plan = Plan(w.cells, w.C, w.V, w.D, w.thresholds)
    D = w.D[0]
    short = hs2.Blocks(D.row[:-1], D.col[:-1], D.R[:-1], D.off[:-1], D.data, "D")
    with pytest.raises(A.HfxError) as e:
        plan.build([short])
    assert e.value.status == A.HFX_ERR_STATE
    moved = hs2.Blocks(D.row, D.col, D.R, D.off + 1, np.r_[0.0, D.data], "D")
    with pytest.raises(A.HfxError) as e:
        plan.build([moved])
    assert e.value.status == A.HFX_ERR_STATE
    swapped = hs2.Blocks(D.row.copy(), D.col.copy(), D.R.copy(), D.off, D.data, "D")
    k = int(np.nonzero(np.any(D.R != 0, axis=1))[0][0])
    swapped.R[k] = -swapped.R[k] + 7
    with pytest.raises(A.HfxError) as e:
        plan.build([swapped])
    assert e.value.status == A.HFX_ERR_STATE
    sig = plan.build(w.D, stats=True)  # still usable
    ref = _ref(w)
    check_close(sig[0].cpu().numpy(), ref.sigma, label="after rejected builds")


def test_host_pointers_are_rejected_before_any_launch():
    """Arrays the kernels dereference must be GPU-accessible: pageable host memory passed where the
    header asks for device memory is HFX_ERR_ARG, checked before any launch."""
    import ctypes
    import torch
    from paper_2009_12505_amd import Plan, _abi as A
    log("case host pointers at the C ABI")
    w = hs.make_workload("tiny", kind="primitive", species_table=((3, 5),), r_c=6.0, r_v=6.0, r_d=7.0)
    plan = Plan(w.cells, w.C, w.V, w.D, w.thresholds)
    L = A.lib()
    sig = plan.build(w.D)
    torch.cuda.synchronize()
    k = np.zeros(3)
    nb = plan.n_basis[0]
    host_hk = np.zeros(2 * nb * nb)
    st = L.hfx_sigma_to_k(plan._h, 0, ctypes.c_void_p(sig[0].data_ptr()), 1, k.ctypes.data, host_hk.ctypes.data)
    assert st == A.HFX_ERR_ARG and "GPU-accessible" in L.hfx_last_error().decode()
    host_sig = sig[0].cpu().numpy()
    hk = torch.empty((1, nb, nb), dtype=torch.complex128, device="cuda")
    st = L.hfx_sigma_to_k(plan._h, 0, host_sig.ctypes.data, 1, k.ctypes.data, ctypes.c_void_p(hk.data_ptr()))
    assert st == A.HFX_ERR_ARG
    ck = np.zeros(2 * nb * 2)
    occ = torch.ones((1, 2), dtype=torch.float64, device="cuda")
    d = torch.empty(plan.sizes[0], dtype=torch.float64, device="cuda")
    st = L.hfx_density_from_k(plan._h, 0, 1, k.ctypes.data, 2, ck.ctypes.data, ctypes.c_void_p(occ.data_ptr()),
                              ctypes.c_void_p(d.data_ptr()))
    assert st == A.HFX_ERR_ARG
    with pytest.raises(A.HfxError) as e:
        plan.energy(w.D, [torch.from_numpy(host_sig)])
    assert e.value.status == A.HFX_ERR_ARG
    # the plan is not poisoned by the rejected calls
    plan.sigma_to_k(sig[0], k.reshape(1, 3), out=hk)
    torch.cuda.synchronize()
