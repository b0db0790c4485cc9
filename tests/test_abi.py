"""Host-side checks of the C ABI: the library loads, exports every declared entry
point, and rejects bad arguments before touching the device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import hfx_synth as hs
from paper_2009_12505_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hfx.h")).read()
    return sorted(set(re.findall(r"\b(hfx_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = A.lib()
    names = _declared()
    assert set(names) == set(A.EXPORTED)
    for n in names:
        assert hasattr(L, n), n
    assert L.hfx_abi_version() == A.ABI_VERSION == 3


def _cstructs(w, th=None):
    cell = w.cells[0]
    keep = []
    pos = np.ascontiguousarray(cell.pos.reshape(-1))
    sp = np.ascontiguousarray(cell.species, np.int32)
    tab = (A.Species * len(cell.species_table))(*[A.Species(a, b) for a, b in cell.species_table])
    c = A.Cell()
    c.n_atoms = cell.n_atoms
    for k, v in enumerate(cell.lattice.reshape(-1)):
        c.lattice[k] = v
    c.pos, c.species, c.n_species, c.sp = pos.ctypes.data, sp.ctypes.data, len(cell.species_table), tab
    keep += [pos, sp, tab]

    def blk(b, data=True):
        arrs = [np.ascontiguousarray(b.row, np.int32), np.ascontiguousarray(b.col, np.int32),
                np.ascontiguousarray(b.R, np.int32).reshape(-1), np.ascontiguousarray(b.off, np.int64),
                np.ascontiguousarray(b.data, np.float64)]
        keep.extend(arrs)
        return A.Blocks(b.n_blocks, *[a.ctypes.data for a in arrs[:4]], arrs[4].ctypes.data if data else None, 0)

    t = th or w.thresholds
    return keep, c, blk(w.C[0]), blk(w.V[0]), blk(w.D[0], False), A.Thresholds(
        t["eps_C"], t["eps_V"], t["eps_D"], t["eps_cs_eri"], t["eps_cs_mat"])


def _create(c, C, V, D, th, opt=None):
    L = A.lib()
    h = ctypes.c_void_p()
    st = L.hfx_plan_create(1, ctypes.byref(c), ctypes.byref(C), ctypes.byref(V), ctypes.byref(D),
                           ctypes.byref(th), None if opt is None else ctypes.byref(opt), ctypes.byref(h))
    return st, L.hfx_last_error().decode()


def _tiny():
    return hs.make_workload("tiny", kind="primitive", species_table=((2, 3),), r_c=5.0, r_v=5.0, r_d=5.0)


@pytest.mark.parametrize("bad", ["nan", "neg"])
def test_rejects_bad_thresholds(bad):
    w = _tiny()
    t = dict(w.thresholds, eps_cs_mat=float("nan") if bad == "nan" else -1.0)
    keep, c, C, V, D, th = _cstructs(w, t)
    st, msg = _create(c, C, V, D, th)
    assert st == A.HFX_ERR_ARG and "threshold" in msg


def test_rejects_asymmetric_v():
    w = _tiny()
    V = w.V[0].compact(w.cells[0])
    k = int(np.nonzero(V.row != V.col)[0][0])
    V.data[V.off[k]] += 1e-3
    w.V[0] = V
    keep, c, C, Vs, D, th = _cstructs(w)
    st, msg = _create(c, C, Vs, D, th)
    assert st == A.HFX_ERR_SYMMETRY, msg


def test_rejects_nonsymmetric_onsite_c():
    w = _tiny()
    C = w.C[0].compact(w.cells[0])
    k = int(np.nonzero((C.row == C.col) & np.all(C.R == 0, axis=1))[0][0])
    C.data[C.off[k] + 1] += 1e-2  # element [0][0][1] but not [0][1][0]
    w.C[0] = C
    keep, c, Cs, V, D, th = _cstructs(w)
    st, msg = _create(c, Cs, V, D, th)
    assert st == A.HFX_ERR_SYMMETRY, msg


def test_rejects_out_of_range_atoms_and_duplicates():
    w = _tiny()
    C = w.C[0]
    bad = hs.Blocks(C.row.copy(), C.col.copy(), C.R.copy(), C.off.copy(), C.data, "C")
    bad.col[0] = 7
    w.C[0] = bad
    keep, c, Cs, V, D, th = _cstructs(w)
    st, msg = _create(c, Cs, V, D, th)
    assert st == A.HFX_ERR_SHAPE, msg
    w = _tiny()
    D = w.D[0]
    dup = hs.Blocks(np.r_[D.row, D.row[:1]], np.r_[D.col, D.col[:1]], np.r_[D.R, D.R[:1]], np.r_[D.off, D.off[:1]],
                    D.data, "D")
    w.D[0] = dup
    keep, c, Cs, V, Ds, th = _cstructs(w)
    st, msg = _create(c, Cs, V, Ds, th)
    assert st in (A.HFX_ERR_SHAPE, A.HFX_ERR_HIP), msg


def test_rejects_unknown_scheduler_and_null_out():
    w = _tiny()
    keep, c, C, V, D, th = _cstructs(w)
    opt = A.Options()
    opt.scheduler = 9
    st, msg = _create(c, C, V, D, th, opt)
    assert st == A.HFX_ERR_ARG
    L = A.lib()
    assert L.hfx_plan_create(1, ctypes.byref(c), ctypes.byref(C), ctypes.byref(V), ctypes.byref(D),
                             ctypes.byref(th), None, None) == A.HFX_ERR_ARG
    assert L.hfx_build(None, None, None, None) == A.HFX_ERR_ARG


def test_rejects_invalid_precision_tiles_and_tuning():
    w = _tiny()
    keep, c, C, V, D, th = _cstructs(w)
    opt = A.Options()
    opt.precision = A.PREC_BF16X3
    opt.tier_tau_bf = -1.0  # < 0 needs a tuning file entry
    opt.tier_tau = 1e-3
    st, msg = _create(c, C, V, D, th, opt)
    assert st == A.HFX_ERR_ARG and "tier_tau_bf" in msg
    opt = A.Options()
    opt.tile_r = 48
    st, msg = _create(c, C, V, D, th, opt)
    assert st == A.HFX_ERR_ARG and "tile_r" in msg
    opt = A.Options()
    opt.tuning_db = b"/nonexistent/tuning.txt"
    st, msg = _create(c, C, V, D, th, opt)
    assert st == A.HFX_ERR_ARG and "tuning_db" in msg
    opt = A.Options()
    opt.precision = 7
    st, msg = _create(c, C, V, D, th, opt)
    assert st == A.HFX_ERR_ARG
    opt = A.Options()
    opt.precision = A.PREC_TIERED
    opt.tier_tau = -1.0
    st, msg = _create(c, C, V, D, th, opt)
    assert st == A.HFX_ERR_ARG and "tier_tau" in msg


def test_mlp_entry_points_validate_before_launch():
    L = A.lib()
    assert L.hfx_mlp_n_params(8, 32, 1) == 32 * 8 + 32 + 32 * 32 + 32 + 32 + 1
    assert L.hfx_mlp_n_params(10, 32, 2) == 32 * 10 + 32 + 32 * 32 + 32 + 2 * 32 + 2
    P = ctypes.c_void_p(1)  # never dereferenced: the sizes are rejected first
    assert L.hfx_mlp_predict(0, 32, 1, P, P, 1, P, None) == A.HFX_ERR_ARG
    assert L.hfx_mlp_predict(8, 65, 1, P, P, 1, P, None) == A.HFX_ERR_ARG
    assert L.hfx_mlp_predict(8, 32, 0, P, P, 1, P, None) == A.HFX_ERR_ARG
    assert L.hfx_mlp_predict(8, 32, 5, P, P, 1, P, None) == A.HFX_ERR_ARG
    assert L.hfx_mlp_loss_grad(8, 32, 2, None, P, P, 1, P, P, None) == A.HFX_ERR_ARG
    assert L.hfx_mlp_train(8, 32, 2, P, P, P, 1, 10, ctypes.c_float(0.0), None, None) == A.HFX_ERR_ARG
    assert L.hfx_item_features(None, None, None, None) == A.HFX_ERR_ARG
    n = ctypes.c_int64()
    assert L.hfx_item_profile(None, ctypes.byref(n), None, None, None) == A.HFX_ERR_ARG
    k = np.zeros(3)
    assert L.hfx_sigma_to_k(None, 0, P, 1, k.ctypes.data, P) == A.HFX_ERR_ARG
    assert L.hfx_density_from_k(None, 0, 1, k.ctypes.data, 1, P, P, P) == A.HFX_ERR_ARG


def test_scheduler_model_file_roundtrip_and_list_schedule(tmp_path):
    from paper_2009_12505_amd import sched
    F = sched.N_IN
    m = sched.CostModel(4, np.arange(F, dtype=np.float32), np.ones(F, np.float32),
                        np.linspace(-1, 1, sched.n_params(4)).astype(np.float32), np.zeros(0),
                        np.array([1.5, -2.0], np.float32), np.array([0.5, 3.0], np.float32))
    sched.save(m, tmp_path / "m.bin")
    m2 = sched.load(tmp_path / "m.bin")
    assert m2.hidden == 4 and np.array_equal(m2.params, m.params) and np.array_equal(m2.mu, m.mu)
    assert np.array_equal(m2.t_mu, m.t_mu) and np.array_equal(m2.t_sd, m.t_sd)
    # the header the library reads: magic, n_in = 10, n_hidden, n_out = 2
    raw = (tmp_path / "m.bin").read_bytes()
    assert raw[:8] == b"HFXMLP02" and list(np.frombuffer(raw[8:20], np.int32)) == [10, 4, 2]
    (tmp_path / "short.bin").write_bytes(raw[:-4])
    with pytest.raises(ValueError):
        sched.load(tmp_path / "short.bin")
    # greedy list scheduling: longest first on 2 machines is optimal here, plan order is not
    costs = np.array([1.0, 1.0, 2.0])
    assert sched.list_schedule_makespan(costs, [2, 0, 1], 2) == 2.0
    assert sched.list_schedule_makespan(costs, [0, 1, 2], 2) == 3.0
    with pytest.raises(ValueError):
        (tmp_path / "bad.bin").write_bytes(b"NOTAMODEL" + bytes(64))
        sched.load(tmp_path / "bad.bin")


def test_rejects_blocks_beyond_the_kernel_limits():
    w = hs.make_workload("tiny", kind="primitive", species_table=((33, 5),), r_c=5.0, r_v=5.0, r_d=5.0)
    keep, c, C, V, D, th = _cstructs(w)
    st, msg = _create(c, C, V, D, th)
    assert st == A.HFX_ERR_UNSUPPORTED and "n_ao" in msg


def test_device_footprint_cap_gives_oom_before_any_allocation():
    """max_device_bytes: plan creation fails with HFX_ERR_OOM at the first device buffer that would
    exceed the cap (the check precedes hipMalloc, so no device is needed)."""
    w = _tiny()
    keep, c, C, V, D, th = _cstructs(w)
    opt = A.Options()
    opt.max_device_bytes = 4
    st, msg = _create(c, C, V, D, th, opt)
    assert st == A.HFX_ERR_OOM and "max_device_bytes" in msg, msg


def test_library_shares_torchs_hip_runtime():
    """Loading the library before torch must not map a second HIP runtime into the process (device
    pointers and streams of one runtime are invalid in the other)."""
    import subprocess
    import sys
    code = ("import paper_2009_12505_amd as p; p.lib(); import torch; "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.check_output([sys.executable, "-c", code], cwd=ROOT, text=True).strip().splitlines()[-1]
    assert out == "1", out


def test_mfma_peak_rejects_bad_arguments_before_any_launch():
    tf = ctypes.c_double(0.0)
    assert A.lib().hfx_mfma_peak(3, None, ctypes.byref(tf), None) == A.HFX_ERR_ARG
    assert A.lib().hfx_mfma_peak(-1, None, ctypes.byref(tf), None) == A.HFX_ERR_ARG
    assert A.lib().hfx_mfma_peak(0, None, None, None) == A.HFX_ERR_ARG
    assert "kind" in A.lib().hfx_last_error().decode()
