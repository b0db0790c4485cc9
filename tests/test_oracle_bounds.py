"""Pins of the oracle's screening-bound factors from both sides (Sec. III C 1, eq.
CS_upper_bounds, Algorithms 4 and 5).

The rigour test in test_oracle.py shows that no dropped unit exceeds its bound, which
catches a factor that is too small but not one that is too large.  These tests fix the
factors from the other side:

* a construction in which Hoelder's inequality for the trace of four matrices holds
  with equality, so every stage's bound must equal the exact max|Htilde| of the unit;
* the factors themselves against their definitions, evaluated independently through
  singular values (sqrt||X X^T||_F is the Schatten-4 norm (sum sigma^4)^(1/4));
* per-stage, per-term kept counts against a brute-force numpy enumeration of the
  three bounds on a tiny periodic cell, and the CS-ERI kept count against an enumeration
  of Q_AF Q_BG > eps (Sec. III C 2);
* the max-abs pre-screening of C, V and D (Sec. III B) against its plain definition:
  the unscreened build of the same tensors with the dropped blocks set to zero.
"""
import numpy as np
import pytest

import hfx_synth as hs
import oracle

STAGES_CS = oracle.CS1 | oracle.CS2 | oracle.CS3


def _blocks(entries, kind):
    """Blocks from a list of (row, col, R, array)."""
    sizes = [a.size for *_, a in entries]
    off = np.zeros(len(entries), np.int64)
    if entries:
        off[1:] = np.cumsum(sizes)[:-1]
    data = np.concatenate([a.ravel() for *_, a in entries]).astype(np.float64)
    return hs.Blocks(np.array([e[0] for e in entries], np.int32), np.array([e[1] for e in entries], np.int32),
                     np.array([e[2] for e in entries], np.int32).reshape(-1, 3), off, data, kind)


def s4(x):
    """Schatten-4 norm from the singular values: (sum sigma^4)^(1/4) = sqrt(||X X^T||_F)."""
    sv = np.linalg.svd(np.atleast_2d(x), compute_uv=False)
    return float(np.sum(sv ** 4) ** 0.25)


def _tight_workload():
    """Two atoms 20 bohr apart in a 500-bohr cell (no images), n_ao = n_abf = 3, on-site C only:
    C_00[al,a,f] = delta(al,f) w_a (every fixed-a slice is w_a I) and C_11[al,a,f] = delta(al,a) w_f
    (every fixed-f slice is w_f I); every V and D block is the identity.  Each of the four terms
    then has a unit whose factors are all scaled identities, where the trace inequality of
    Sec. III C 1 is an equality: term 1 in item (0,0), term 4 in (1,1), term 2 in (0,1),
    term 3 in (1,0)."""
    n = 3
    w = np.array([0.5, -1.25, 0.75])
    c00 = np.zeros((n, n, n))
    c11 = np.zeros((n, n, n))
    for al in range(n):
        for a in range(n):
            for f in range(n):
                c00[al, a, f] = w[a] * (al == f)
                c11[al, a, f] = w[f] * (al == a)
    eye = np.eye(n)
    z = (0, 0, 0)
    C = _blocks([(0, 0, z, c00), (1, 1, z, c11)], "C")
    V = _blocks([(r, c, z, eye) for r in (0, 1) for c in (0, 1)], "V")
    D = _blocks([(r, c, z, eye) for r in (0, 1) for c in (0, 1)], "D")
    cell = hs.Cell(np.eye(3) * 500.0, np.array([[0.0, 0.0, 0.0], [20.0, 0.0, 0.0]]), np.zeros(2, np.int32),
                   [(n, n)])
    return cell, C, V, D, w


@pytest.mark.parametrize("stage", [1, 2, 3])
def test_bounds_attained_in_the_tight_case(stage):
    """With only one screening stage on and a threshold above every bound, every unit is dropped
    at that stage and the oracle compares its exact Htilde with the bound: the largest ratio of
    every term must be exactly 1 (the bound is attained), not below it (a looser factor)."""
    cell, C, V, D, w = _tight_workload()
    th = dict(eps_C=0.0, eps_V=0.0, eps_D=0.0, eps_cs_eri=0.0, eps_cs_mat=1e300)
    st = {1: oracle.CS1, 2: oracle.CS2, 3: oracle.CS3}[stage]
    r = oracle.run(cell, C, V, D, th, stages=st, diag=True, n_threads=1)
    ratios = r.diag[2 + 4 * (stage - 1): 6 + 4 * (stage - 1)]
    assert r.diag[1] > 0
    np.testing.assert_allclose(ratios, 1.0, rtol=0, atol=1e-12)
    # the attained value: 3 max|w|^2 for every term (the identity blocks have Tr I = 3)
    th_lo = dict(th, eps_cs_mat=3 * np.max(np.abs(w)) ** 2 * (1 - 1e-9))
    th_hi = dict(th, eps_cs_mat=3 * np.max(np.abs(w)) ** 2 * (1 + 1e-9))
    kept_lo = oracle.run(cell, C, V, D, th_lo, stages=st, n_threads=1).stats
    kept_hi = oracle.run(cell, C, V, D, th_hi, stages=st, n_threads=1).stats
    for t in (1, 2, 3, 4):
        assert kept_lo[f"kept_s{stage}_t{t}"] > kept_hi[f"kept_s{stage}_t{t}"], t


def _random_workload():
    return hs.make_workload("tiny", kind="conventional", species_table=((3, 5), (2, 4)), species=[0, 1] * 4,
                            r_c=6.0, r_v=6.0, r_d=8.0)


def test_factors_equal_their_definitions():
    """nA = max_a ||C[:,a,:]||_F, gA = max_a ||C[:,a,:]||_S4, nF, gF likewise over the last AO
    index, gV = ||V||_S4, gD = ||D||_S4 (Sec. III C 1), evaluated from singular values."""
    w = _random_workload()
    cell = w.cells[0]
    r = oracle.run(cell, w.C[0], w.V[0], w.D[0], w.thresholds, norms=True, n_threads=2)
    for k in range(w.C[0].n_blocks):
        c = w.C[0].block(cell, k)
        nA = max(np.linalg.norm(c[:, a, :]) for a in range(c.shape[1]))
        gA = max(s4(c[:, a, :]) for a in range(c.shape[1]))
        nF = max(np.linalg.norm(c[:, :, f]) for f in range(c.shape[2]))
        gF = max(s4(c[:, :, f]) for f in range(c.shape[2]))
        got = [r.norms[x][k] for x in ("nA", "gA", "nF", "gF")]
        np.testing.assert_allclose(got, [nA, gA, nF, gF], rtol=1e-12)
    for k in range(w.V[0].n_blocks):
        assert r.norms["gV"][k] == pytest.approx(s4(w.V[0].block(cell, k)), rel=1e-12)
    for k in range(w.D[0].n_blocks):
        assert r.norms["gD"][k] == pytest.approx(s4(w.D[0].block(cell, k)), rel=1e-12)


def _enumerate_kept(w, eps):
    """Per-stage, per-term kept counts of Algorithm 5 by brute force: every <A,B> item (A home, B
    any image), every F of A and G of B, every term with its density block and target in the
    pattern; stage 1 b1 = gi gV gj gD, stage 2 b2 = gi ||Y_j|| gD, stage 3 b3 = ni ||T_j||."""
    cell = w.cells[0]
    Cd, Vd, Dd = (x.as_dict(cell) for x in (w.C[0], w.V[0], w.D[0]))
    cby = {}
    for (r, c, R), blk in Cd.items():
        cby.setdefault(r, []).append((c, np.array(R), blk))

    def fac(c):
        return dict(nA=max(np.linalg.norm(c[:, a, :]) for a in range(c.shape[1])),
                    gA=max(s4(c[:, a, :]) for a in range(c.shape[1])),
                    nF=max(np.linalg.norm(c[:, :, f]) for f in range(c.shape[2])),
                    gF=max(s4(c[:, :, f]) for f in range(c.shape[2])))

    cf = {k: fac(v) for k, v in Cd.items()}
    kept = np.zeros((3, 4), np.int64)
    t3 = lambda R: tuple(int(x) for x in R)
    for (A, B, RB), V in Vd.items():
        RB = np.array(RB)
        gV = s4(V)
        for (G, RCG, Cbg) in cby.get(B, []):
            RG = RB + RCG
            Y = np.einsum("ab,bcg->acg", V, Cbg)              # Y[al][b][g]
            yb = max(np.linalg.norm(Y[:, b, :]) for b in range(Y.shape[1]))
            yg = max(np.linalg.norm(Y[:, :, g]) for g in range(Y.shape[2]))
            fg = cf[(B, G, t3(RCG))]
            for (F, RF, Caf) in cby.get(A, []):
                ff = cf[(A, F, t3(RF))]
                spec = [((F, G, t3(RG - RF)), (A, B, t3(RB))),
                        ((F, B, t3(RB - RF)), (A, G, t3(RG))),
                        ((A, G, t3(RG)), (F, B, t3(RB - RF))),
                        ((A, B, t3(RB)), (F, G, t3(RG - RF)))]
                for t, (dk, tk) in enumerate(spec):
                    if dk not in Dd or tk not in Dd:
                        continue
                    Dt = Dd[dk]
                    gi = ff["gA"] if t < 2 else ff["gF"]
                    gj = fg["gA"] if t in (0, 2) else fg["gF"]
                    ni = ff["nA"] if t < 2 else ff["nF"]
                    b1 = gi * gV * gj * s4(Dt)
                    if not b1 > eps:
                        continue
                    kept[0, t] += 1
                    b2 = gi * (yb if t in (0, 2) else yg) * s4(Dt)
                    if not b2 > eps:
                        continue
                    kept[1, t] += 1
                    if t == 0:
                        T = np.einsum("abg,fg->afb", Y, Dt)
                    elif t == 1:
                        T = np.einsum("abg,fb->afg", Y, Dt)
                    elif t == 2:
                        T = np.einsum("xbg,ag->xab", Y, Dt)
                    else:
                        T = np.einsum("xbg,ab->xag", Y, Dt)
                    tmax = max(np.linalg.norm(T[:, :, j]) for j in range(T.shape[2]))
                    if ni * tmax > eps:
                        kept[2, t] += 1
    return kept


@pytest.mark.parametrize("eps", [1e-4, 3e-3, 1e-2, 0.3])
def test_kept_counts_equal_bruteforce_enumeration(eps):
    """The oracle's per-stage, per-term kept counts (no pre-screen, no CS-ERI) equal a plain
    enumeration of the three Cauchy-Schwarz bounds with factors from singular values."""
    w = _random_workload()
    th = {k: eps for k in w.thresholds}
    r = oracle.run(w.cells[0], w.C[0], w.V[0], w.D[0], th, stages=STAGES_CS, n_threads=2)
    want = _enumerate_kept(w, eps)
    got = np.array([[r.stats[f"kept_s{s}_t{t}"] for t in (1, 2, 3, 4)] for s in (1, 2, 3)])
    assert want[0].sum() > want[2].sum() > 0, want
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("quantile", [0.2, 0.5, 0.8])
def test_cs_eri_counts_equal_bruteforce_enumeration(quantile):
    """With only the CS-ERI test on (eq. CS-ERI, Sec. III C 2), a quartet (A a, F f | B b, G g) is
    kept iff Q_AF Q_BG > eps: the oracle's visited and kept counts equal a plain enumeration over
    every <A,B> item, F of A and G of B, with Q_AF taken from the oracle's per-block values (which
    test_cs_eri_q_is_max_diagonal_eri pins against the explicit four-centre integrals).  The
    threshold sits at a quantile of the products, so both outcomes occur."""
    w = _random_workload()
    cell = w.cells[0]
    C = w.C[0]
    r0 = oracle.run(cell, C, w.V[0], w.D[0], {k: 0.0 for k in w.thresholds}, stages=oracle.CS_ERI, norms=True,
                    n_threads=2)
    Q = {(int(C.row[k]), int(C.col[k]), tuple(int(x) for x in C.R[k])): r0.norms["Q"][k] for k in range(C.n_blocks)}
    by_row = {}
    for (a, f, R), q in Q.items():
        by_row.setdefault(a, []).append(q)
    prods = [qf * qg for (A, B, _R) in w.V[0].as_dict(cell) for qf in by_row.get(A, []) for qg in by_row.get(B, [])]
    eps = float(np.quantile(prods, quantile))
    th = {k: 0.0 for k in w.thresholds}
    th["eps_cs_eri"] = eps
    r = oracle.run(cell, C, w.V[0], w.D[0], th, stages=oracle.CS_ERI, n_threads=2)
    assert r.stats["candidates"] == len(prods)
    want = sum(1 for p in prods if p > eps)
    assert 0 < want < len(prods)
    assert r.stats["kept_cs_eri"] == want


def _zeroed(X, cell, ks):
    data = X.data.copy()
    for k in ks:
        o = int(X.off[k])
        data[o:o + X.block(cell, k).size] = 0.0
    return hs.Blocks(X.row, X.col, X.R, X.off, data, X.kind)


@pytest.mark.parametrize("which", ["C", "V", "D"])
def test_prescreen_is_dropping_small_blocks(which):
    """Pre-screening (Sec. III B: a C, V or D block whose largest element is at most its threshold
    is discarded) gives exactly the unscreened Sigma of the same tensors with those blocks set to
    zero.  The threshold of the tensor under test sits at the median of its block maxima; the
    others are 0 (keep every non-zero block); no Cauchy-Schwarz stage is on."""
    w = _random_workload()
    cell = w.cells[0]
    X = {"C": w.C[0], "V": w.V[0], "D": w.D[0]}
    mx = np.array([np.abs(X[which].block(cell, k)).max() for k in range(X[which].n_blocks)])
    eps = float(np.median(mx))
    small = np.nonzero(mx <= eps)[0]
    assert 0 < len(small) < len(mx)
    th = {k: 0.0 for k in w.thresholds}
    th[f"eps_{which}"] = eps
    r_pre = oracle.run(cell, w.C[0], w.V[0], w.D[0], th, stages=oracle.PRE, n_threads=2)
    X[which] = _zeroed(X[which], cell, small)
    r_zero = oracle.run(cell, X["C"], X["V"], X["D"], {k: 0.0 for k in w.thresholds}, stages=0, n_threads=2)
    assert np.abs(r_zero.sigma).max() > 0
    np.testing.assert_allclose(r_pre.sigma, r_zero.sigma, rtol=0, atol=1e-14 * np.abs(r_zero.sigma).max())
    assert r_pre.stats["units_formed"] < r_zero.stats["units_formed"]
