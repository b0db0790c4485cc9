"""The 4096-atom cell (8^3 conventional diamond cells, 13 AO / 60 ABF per atom, C within 16 bohr,
eps 1e-6) built in full on one GPU: every Sigma block against the oracle's primitive-cell block of
the same atom pair (identical keyed blocks, Sec. IV A: a k-point mesh of the unit cell and the
Gamma-only supercell give the same blocks), and E_x per atom.  Each step prints when it ends."""
import time

import numpy as np
import pytest

import hfx_synth as hs
import oracle
from test_gpu_parity import check_close, log

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1500)
def test_cfg5_full_vs_primitive():
    import torch
    from paper_2009_12505_amd import Plan
    log("case cfg5: 4096 atoms, eps 1e-6, FP64, full build against the primitive-cell oracle")
    t = time.time()
    wp = hs.make_workload("cfg5prim")
    ref = oracle.run(wp.cells[0], wp.C[0], wp.V[0], wp.D[0], wp.thresholds, n_threads=16)
    log(f"cfg5 oracle (2 home atoms of the primitive cell) {time.time() - t:.1f}s")
    t = time.time()
    ws = hs.make_workload("cfg5")
    log(f"cfg5 inputs generated in {time.time() - t:.1f}s: C {ws.C[0].n_blocks}, V {ws.V[0].n_blocks}, "
        f"D {ws.D[0].n_blocks} blocks")
    t = time.time()
    plan = Plan(ws.cells, ws.C, ws.V, ws.D, ws.thresholds)
    torch.cuda.synchronize()
    log(f"cfg5 plan created in {time.time() - t:.1f}s")
    t = time.time()
    sig = plan.build(ws.D, stats=True)
    st = plan.last_stats
    log(f"cfg5 build {time.time() - t:.1f}s (main kernel {st['ms_main']:.0f} ms, {st['items']} items, "
        f"{st['flops_paper'] / 1e12:.1f} TFLOP Algorithm-3 count)")
    e = plan.energy(ws.D, sig)[0]
    got = sig[0].cpu().numpy()
    del sig, plan
    torch.cuda.empty_cache()
    cs, cp = ws.cells[0], wp.cells[0]
    pi, pR = hs.map_to_primitive(cs, cp)
    D, Dp = ws.D[0], wp.D[0]
    shift = np.rint(D.R @ cs.lattice @ np.linalg.inv(cp.lattice)).astype(np.int64)
    Rp = pR[D.col] + shift - pR[D.row]
    key = lambda r, c, R: ((r * 4 + c) * 1000 + (R[:, 0] + 500)) * 1000000 + (R[:, 1] + 500) * 1000 + (R[:, 2] + 500)
    kp = key(Dp.row.astype(np.int64), Dp.col.astype(np.int64), Dp.R.astype(np.int64))
    order = np.argsort(kp)
    ks = key(pi[D.row], pi[D.col], Rp)
    pos = np.searchsorted(kp[order], ks)
    assert np.all(kp[order][pos] == ks)
    n = 169
    got = got.reshape(-1, n)
    want = ref.sigma.reshape(-1, n)[order[pos]]
    check_close(got, want, rel=1e-11, label="cfg5 eps=1e-06")
    e_ref_atom = oracle.energy(cp, Dp, ref.sigma) / cp.n_atoms
    log(f"cfg5: E_x/atom gpu {e / cs.n_atoms:.12f} oracle {e_ref_atom:.12f}")
    assert abs(e / cs.n_atoms - e_ref_atom) <= 1e-8
    for t_ in (1, 2, 3, 4):
        assert st[f"kept_s3_t{t_}"] * cp.n_atoms == ref.stats[f"kept_s3_t{t_}"] * cs.n_atoms
