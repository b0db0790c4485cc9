"""GPU parity: the HIP build (through the C ABI) against the FP64 CPU oracle.

Element-by-element on the same seeded inputs.  FP64 GPU path: Sigma within
1e-11 of max|Sigma| (different summation order only) and the target of the
method: max-abs Sigma error <= 1e-7 and |dE_x| <= 1e-8 Ha per atom.
"""
import sys
import time

import numpy as np
import pytest

import hfx_synth as hs
import oracle

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_build(w, **opt):
    from paper_2009_12505_amd import Plan
    torch = _torch()
    plan = Plan(w.cells, w.C, w.V, w.D, w.thresholds, **opt)
    sig = plan.build(w.D, stats=True)
    e = plan.energy(w.D, sig)
    torch.cuda.synchronize()
    return [s.cpu().numpy() for s in sig], e, plan.last_stats


def check_close(got, ref, rel=1e-11, label=""):
    scale = float(np.abs(ref).max()) if ref.size else 0.0
    err = float(np.abs(got - ref).max()) if ref.size else 0.0
    log(f"{label}: max|Sigma|={scale:.4e} max|dSigma|={err:.3e} (rel {err / max(scale, 1e-300):.2e})")
    assert err <= rel * scale + 1e-300, (err, scale)
    assert err <= 1e-7
    return err


TINY = [
    dict(kind="primitive", species_table=((2, 3),), r_c=5.0, r_v=5.0, r_d=5.0),
    dict(kind="primitive", species_table=((3, 5),), r_c=8.0, r_v=8.0, r_d=9.0),
    dict(kind="primitive", species_table=((2, 3), (3, 4)), species=[0, 1], r_c=8.0, r_v=6.0, r_d=9.0),
    dict(kind="conventional", species_table=((2, 4),), r_c=5.0, r_v=4.5, r_d=6.0),
    dict(kind="conventional", species_table=((5, 9),), r_c=7.0, r_v=9.0, r_d=10.0, eps=1e-6),
    dict(kind="conventional", species_table=((4, 7), (6, 10)), species=[0, 1] * 4, r_c=7.0, r_v=9.0, r_d=10.0,
         eps=1e-4),
    # blocks wider than one 16x16 matrix-core tile, next to narrow ones
    dict(kind="primitive", species_table=((18, 21), (3, 5)), species=[0, 1], r_c=6.0, r_v=7.0, r_d=8.0, eps=1e-3),
]


@pytest.mark.parametrize("cfg", range(len(TINY)))
def test_tiny_parity(cfg):
    log(f"case tiny[{cfg}] {TINY[cfg]}")
    w = hs.make_workload("tiny", **TINY[cfg])
    cell = w.cells[0]
    ref = oracle.run(cell, w.C[0], w.V[0], w.D[0], w.thresholds, n_threads=8)
    sig, e, st = gpu_build(w)
    check_close(sig[0], ref.sigma, label=f"tiny[{cfg}]")
    e_ref = oracle.energy(cell, w.D[0], ref.sigma)
    assert abs(e[0] - e_ref) <= 1e-11 * abs(e_ref)
    for s in (1, 2, 3):
        for t in (1, 2, 3, 4):
            assert st[f"kept_s{s}_t{t}"] == ref.stats[f"kept_s{s}_t{t}"], (s, t)
    assert st["kept_cs_eri"] == ref.stats["kept_cs_eri"]


@pytest.mark.parametrize("stages", [1, 3, 7, 15, 31])
def test_stage_switches(stages):
    """Each screening stage can be switched off; the oracle honours the same switches."""
    from paper_2009_12505_amd import Plan
    log(f"case stages={stages}")
    w = hs.make_workload("tiny", kind="conventional", species_table=((5, 9),), r_c=7.0, r_v=9.0, r_d=10.0, eps=1e-3)
    cell = w.cells[0]
    ref = oracle.run(cell, w.C[0], w.V[0], w.D[0], w.thresholds, stages=stages, n_threads=8)
    sig, e, st = gpu_build(w, stages=stages)
    check_close(sig[0], ref.sigma, label=f"stages={stages}")


def test_home_subset():
    log("case home subset")
    w = hs.make_workload("tiny", kind="conventional", species_table=((5, 9),), r_c=7.0, r_v=9.0, r_d=10.0, eps=1e-6)
    cell = w.cells[0]
    home = [1, 4, 6]
    ref = oracle.run(cell, w.C[0], w.V[0], w.D[0], w.thresholds, home=home, n_threads=8)
    sig, e, st = gpu_build(w, home_subset=home)
    check_close(sig[0], ref.sigma, label="home subset")


def test_cfg1_full():
    """2-atom primitive cell, 13 AO / 40 ABF, every block within 12 bohr, no screening."""
    log("case cfg1")
    w = hs.make_workload("cfg1")
    cell = w.cells[0]
    t = time.time()
    ref = oracle.run(cell, w.C[0], w.V[0], w.D[0], w.thresholds, n_threads=16)
    log(f"cfg1 oracle {time.time() - t:.1f}s")
    sig, e, st = gpu_build(w)
    check_close(sig[0], ref.sigma, label="cfg1")
    e_ref = oracle.energy(cell, w.D[0], ref.sigma)
    assert abs(e[0] - e_ref) / cell.n_atoms <= 1e-8
    assert e[0] < 0


def _supercell_vs_primitive(name, eps, rel, **opt):
    torch = _torch()
    log(f"case {name} eps={eps} {opt}: GPU full supercell vs oracle primitive cell")
    wp = hs.make_workload(name + "prim", eps=eps)
    t = time.time()
    ref = oracle.run(wp.cells[0], wp.C[0], wp.V[0], wp.D[0], wp.thresholds, n_threads=16)
    log(f"{name} oracle (2 home atoms) {time.time() - t:.1f}s")
    ws = hs.make_workload(name, eps=eps)
    t = time.time()
    sig, e, st = gpu_build(ws, **opt)
    log(f"{name} gpu plan+build {time.time() - t:.1f}s stats {st}")
    cs, cp = ws.cells[0], wp.cells[0]
    pi, pR = hs.map_to_primitive(cs, cp)
    D = ws.D[0]
    shift = np.rint(D.R @ cs.lattice @ np.linalg.inv(cp.lattice)).astype(np.int64)
    Rp = pR[D.col] + shift - pR[D.row]
    # primitive block index for every supercell block
    Dp = wp.D[0]
    key = lambda r, c, R: ((r * 4 + c) * 1000 + (R[:, 0] + 500)) * 1000000 + (R[:, 1] + 500) * 1000 + (R[:, 2] + 500)
    kp = key(Dp.row.astype(np.int64), Dp.col.astype(np.int64), Dp.R.astype(np.int64))
    order = np.argsort(kp)
    ks = key(pi[D.row], pi[D.col], Rp)
    pos = np.searchsorted(kp[order], ks)
    assert np.all(kp[order][pos] == ks)
    pidx = order[pos]
    soff = oracle.sigma_offsets(cs, D)
    poff = ref.sig_off
    n = 169
    assert np.all(np.diff(soff) == n)
    got = sig[0].reshape(-1, n)
    want = ref.sigma.reshape(-1, n)[pidx]
    err = check_close(got, want, rel=rel, label=f"{name} eps={eps}")
    e_ref_atom = oracle.energy(cp, Dp, ref.sigma) / cp.n_atoms
    e_gpu_atom = e[0] / cs.n_atoms
    log(f"{name}: E_x/atom gpu {e_gpu_atom:.12f} oracle {e_ref_atom:.12f} diff {abs(e_gpu_atom - e_ref_atom):.3e}")
    assert abs(e_gpu_atom - e_ref_atom) <= 1e-8
    for t in (1, 2, 3, 4):
        # every home atom of the crystal keeps the same units as a primitive home atom
        assert st[f"kept_s3_t{t}"] * cp.n_atoms == ref.stats[f"kept_s3_t{t}"] * cs.n_atoms
    del torch
    return err


@pytest.mark.timeout(900)
def test_cfg3_eps1e4_full_vs_primitive():
    """512-atom supercell (4^3 conventional cells), 13 AO / 60 ABF, eps 1e-4: every Sigma block
    of the GPU build equals the oracle's primitive-cell block of the same atom pair."""
    _supercell_vs_primitive("cfg3", 1e-4, 1e-11)


@pytest.mark.timeout(900)
def test_cfg3_eps1e6_full_vs_primitive():
    """The benchmark workload itself (512 atoms, eps 1e-6, FP64, the launch configuration bench.py
    times): every Sigma block against the oracle's primitive-cell block of the same atom pair."""
    _supercell_vs_primitive("cfg3", 1e-6, 1e-11)


@pytest.mark.timeout(900)
def test_cfg2_full_vs_primitive():
    """64-atom supercell (2^3 conventional cells), 13 AO / 40 ABF, C within 16 bohr, eps 1e-6."""
    _supercell_vs_primitive("cfg2", 1e-6, 1e-11)


def _combine(ws):
    """One batched workload from several single-cell workloads."""
    import dataclasses
    return dataclasses.replace(ws[0], cells=[w.cells[0] for w in ws], C=[w.C[0] for w in ws],
                               V=[w.V[0] for w in ws], D=[w.D[0] for w in ws])


def test_multicell_tiny():
    """Several independent cells of different shapes and species in one launch: each cell's
    Sigma equals the oracle of that cell alone."""
    log("case multicell tiny")
    parts = [hs.make_workload("tiny", kind="primitive", species_table=((2, 3), (3, 4)), species=[0, 1],
                              r_c=8.0, r_v=6.0, r_d=9.0, seed=11),
             hs.make_workload("tiny", kind="conventional", species_table=((5, 9),), r_c=7.0, r_v=9.0, r_d=10.0,
                              eps=1e-6, seed=12),
             hs.make_workload("tiny", kind="custom", lattice=np.eye(3) * 300.0,
                              pos=[[0.0, 0.0, 0.0], [2.5, 1.0, -0.5]], species_table=((2, 3), (3, 2)),
                              species=[0, 1], r_c=6.0, r_v=6.0, r_d=6.0, seed=13)]
    w = _combine(parts)
    w = w.__class__(**{**w.__dict__, "thresholds": parts[1].thresholds})
    sig, e, st = gpu_build(w)
    for c, p in enumerate(parts):
        ref = oracle.run(p.cells[0], p.C[0], p.V[0], p.D[0], w.thresholds, n_threads=8)
        check_close(sig[c], ref.sigma, label=f"multicell[{c}]")
        assert abs(e[c] - oracle.energy(p.cells[0], p.D[0], ref.sigma)) <= 1e-11 * abs(e[c])


@pytest.mark.timeout(900)
def test_cfg4_batched_cells_home_subset():
    """48 cells of 1..3 x 1..3 x 1..3 conventional cells (8..216 atoms), two species (13 AO / 60 ABF
    and 27 AO / 100 ABF) drawn per site, all built in one persistent launch with one seeded home
    atom per cell; three seeded cells are checked against the oracle of that cell with the same
    home atom (the other cells' items run in the same launch)."""
    log("case cfg4")
    w = hs.make_workload("cfg4")
    rng = np.random.default_rng(2009)
    home_local = [int(rng.integers(c.n_atoms)) for c in w.cells]
    offs = np.cumsum([0] + [c.n_atoms for c in w.cells])
    home = [int(offs[k] + a) for k, a in enumerate(home_local)]
    t = time.time()
    sig, e, st = gpu_build(w, home_subset=home)
    log(f"cfg4 gpu {time.time() - t:.1f}s items {st['items']} units {[st[f'kept_s3_t{t}'] for t in (1, 2, 3, 4)]}")
    checked = sorted(rng.choice(len(w.cells), size=3, replace=False).tolist())
    for k in checked:
        cell = w.cells[k]
        t = time.time()
        ref = oracle.run(cell, w.C[k], w.V[k], w.D[k], w.thresholds, home=[home_local[k]], n_threads=16)
        log(f"cfg4 cell {k}: oracle {time.time() - t:.1f}s")
        check_close(sig[k], ref.sigma, label=f"cfg4 cell {k} ({cell.n_atoms} atoms)")


@pytest.mark.parametrize("seed", range(6))
def test_random_shapes_parity(seed):
    """Seeded random block shapes (one or two species, 1..3 AOs and 1..5 ABFs per atom, random C, V
    and D ranges; the cells the oracle is pinned on against brute force), at eps 0 and 1e-4."""
    from test_oracle import _random_shape
    cfg = dict(_random_shape(seed), eps=(0.0, 1e-4)[seed % 2])
    log(f"case random shape {seed}: {cfg}")
    w = hs.make_workload("tiny", **cfg)
    ref = oracle.run(w.cells[0], w.C[0], w.V[0], w.D[0], w.thresholds, n_threads=8)
    sig, e, st = gpu_build(w)
    check_close(sig[0], ref.sigma, label=f"random shape {seed}")
    for t in (1, 2, 3, 4):
        assert st[f"kept_s3_t{t}"] == ref.stats[f"kept_s3_t{t}"]
    assert st["g_alive"] == ref.stats["y_formed"]
