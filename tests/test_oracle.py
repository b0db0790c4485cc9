"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's own
arithmetic: they compare it with the plain definition (explicit four-centre
integrals, Algorithm 1), closed forms, textbook special cases, exact
invariants, and the rigour of the Cauchy-Schwarz bounds.
"""
import numpy as np
import pytest

import hfx_synth as hs
import oracle
from oracle import bruteforce as bf

TINY = [
    # one species, primitive cell, nearest shell only
    dict(kind="primitive", species_table=((2, 3),), r_c=5.0, r_v=5.0, r_d=5.0),
    # second shell, D reaching further than C
    dict(kind="primitive", species_table=((3, 5),), r_c=8.0, r_v=8.0, r_d=9.0),
    # two species with different block shapes
    dict(kind="primitive", species_table=((2, 3), (3, 4)), species=[0, 1], r_c=8.0, r_v=6.0, r_d=9.0),
    # conventional cell: more home atoms, V shorter than C
    dict(kind="conventional", species_table=((2, 4),), r_c=5.0, r_v=4.5, r_d=6.0),
]


def _run(w, **kw):
    return oracle.run(w.cells[0], w.C[0], w.V[0], w.D[0], w.thresholds, n_threads=4, **kw)


def _maxdiff(d1, d2):
    keys = set(d1) | set(d2)
    m = 0.0
    for k in keys:
        a = d1.get(k)
        b = d2.get(k)
        if a is None:
            a = np.zeros_like(b)
        if b is None:
            b = np.zeros_like(a)
        m = max(m, float(np.abs(a - b).max()))
    return m


@pytest.mark.parametrize("cfg", range(len(TINY)))
def test_oracle_equals_bruteforce(cfg):
    """eq. HFX_ERIs with the ERIs of eq. ERI_split (Algorithm 1) == Algorithms 2/3 at eps = 0."""
    w = hs.make_workload("tiny", **TINY[cfg])
    cell = w.cells[0]
    ref = bf.sigma(cell, w.C[0], w.V[0], w.D[0])
    r = _run(w)
    got = oracle.sigma_dict(cell, w.D[0], r.sigma)
    scale = max(float(np.abs(v).max()) for v in ref.values())
    assert _maxdiff(got, ref) <= 1e-12 * scale
    e_ref = bf.energy(cell, w.D[0], ref)
    assert abs(oracle.energy(cell, w.D[0], r.sigma) - e_ref) <= 1e-12 * abs(e_ref)


def test_isolated_atom_is_plain_ri_k():
    """One atom far from its images: only the on-site pair survives, and the
    build reduces to the textbook RI exchange  K_ij = sum C^a_ik V_ab C^b_jl D_kl."""
    w = hs.make_workload("tiny", kind="primitive", a=200.0, species_table=((4, 6),), r_c=5.0, r_v=5.0, r_d=5.0)
    cell = w.cells[0]
    assert w.C[0].n_blocks == 2  # two primitive atoms, 86 bohr apart: on-site blocks only
    r = _run(w)
    got = oracle.sigma_dict(cell, w.D[0], r.sigma)
    for i in range(2):
        k = (i, i, (0, 0, 0))
        C = w.C[0].as_dict(cell)[k]
        V = w.V[0].as_dict(cell)[k]
        D = w.D[0].as_dict(cell)[k]
        Kmat = np.einsum("aik,ab,bjl,kl->ij", C, V, C, D)
        np.testing.assert_allclose(got[k], -Kmat, rtol=1e-13, atol=1e-13 * np.abs(Kmat).max())


def test_one_function_closed_form():
    """n_ao = n_abf = 1, isolated atom: Sigma = -c^2 v d."""
    w = hs.make_workload("tiny", kind="custom", lattice=np.eye(3) * 500.0, pos=[[0.0, 0.0, 0.0]],
                         species_table=((1, 1),), r_c=3.0, r_v=3.0, r_d=3.0)
    cell = w.cells[0]
    r = _run(w)
    c = w.C[0].data[w.C[0].off[0]]
    v = w.V[0].data[w.V[0].off[0]]
    d = w.D[0].data[w.D[0].off[0]]
    assert r.sigma[0] == pytest.approx(-c * c * v * d, rel=1e-15)
    assert oracle.energy(cell, w.D[0], r.sigma) == pytest.approx(-0.5 * c * c * v * d * d, rel=1e-15)


def test_two_atom_molecule_erisplit():
    """Two atoms without images: both C_IK and C_KI enter, the four partial ERIs
    of eq. ERI_split add to the full ERI, and on-site pairs count once."""
    w = hs.make_workload("tiny", kind="custom", lattice=np.eye(3) * 300.0,
                         pos=[[0.0, 0.0, 0.0], [2.5, 1.0, -0.5]], species_table=((2, 3), (3, 2)),
                         species=[0, 1], r_c=6.0, r_v=6.0, r_d=6.0)
    cell = w.cells[0]
    ref = bf.sigma(cell, w.C[0], w.V[0], w.D[0])
    got = oracle.sigma_dict(cell, w.D[0], _run(w).sigma)
    scale = max(float(np.abs(v).max()) for v in ref.values())
    assert _maxdiff(got, ref) <= 1e-13 * scale
    assert len(ref) == 4


def test_symmetry_and_negative_energy():
    """Sigma_IJ(R) = Sigma_JI(-R)^T for symmetric V and D, and E_x = 1/2 <D,Sigma> <= 0
    for positive-definite V and positive-semi-definite D (eps = 0)."""
    w = hs.make_workload("tiny", kind="conventional", species_table=((3, 4),), r_c=6.0, r_v=6.0, r_d=7.0)
    cell = w.cells[0]
    r = _run(w)
    sd = oracle.sigma_dict(cell, w.D[0], r.sigma)
    m = 0.0
    for (i, j, R), blk in sd.items():
        t = sd[(j, i, (-R[0], -R[1], -R[2]))]
        m = max(m, float(np.abs(blk - t.T).max()))
    assert m <= 1e-12 * max(float(np.abs(b).max()) for b in sd.values())
    assert oracle.energy(cell, w.D[0], r.sigma) < 0


def test_linearity_and_scaling():
    """Sigma is linear in D and in V and quadratic in C (eq. HFX_LRI)."""
    w = hs.make_workload("tiny", kind="primitive", species_table=((2, 3),), r_c=6.0, r_v=6.0, r_d=6.0)
    cell = w.cells[0]
    th = w.thresholds
    base = oracle.run(cell, w.C[0], w.V[0], w.D[0], th).sigma

    def scaled(b, s):
        return hs.Blocks(b.row, b.col, b.R, b.off, b.data * s, b.kind)

    s_d = oracle.run(cell, w.C[0], w.V[0], scaled(w.D[0], -2.5), th).sigma
    s_v = oracle.run(cell, w.C[0], scaled(w.V[0], 3.0), w.D[0], th).sigma
    s_c = oracle.run(cell, scaled(w.C[0], 0.5), w.V[0], w.D[0], th).sigma
    np.testing.assert_allclose(s_d, -2.5 * base, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(s_v, 3.0 * base, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(s_c, 0.25 * base, rtol=1e-12, atol=1e-13)
    # D = D1 + D2
    D2 = hs.Blocks(w.D[0].row, w.D[0].col, w.D[0].R, w.D[0].off, np.cos(w.D[0].data * 7.0), "D")
    s_2 = oracle.run(cell, w.C[0], w.V[0], D2, th).sigma
    Ds = hs.Blocks(w.D[0].row, w.D[0].col, w.D[0].R, w.D[0].off, w.D[0].data + D2.data, "D")
    s_s = oracle.run(cell, w.C[0], w.V[0], Ds, th).sigma
    np.testing.assert_allclose(s_s, base + s_2, rtol=1e-12, atol=1e-12)


def test_cs_eri_q_is_max_diagonal_eri():
    """Q_AF^2 = max_{a,f} (Aa Ff | Aa Ff) (eq. CS-ERI), the diagonal of the
    explicit four-centre integral of the pair expansion."""
    w = hs.make_workload("tiny", kind="primitive", species_table=((3, 4),), r_c=8.0, r_v=8.0, r_d=8.0)
    cell = w.cells[0]
    r = _run(w, norms=True)
    Cd, Vd = w.C[0].as_dict(cell), w.V[0].as_dict(cell)
    for k in range(w.C[0].n_blocks):
        A, F, R = int(w.C[0].row[k]), int(w.C[0].col[k]), tuple(int(x) for x in w.C[0].R[k])
        e = bf.eri(Cd, Vd, (A, (0, 0, 0)), (F, R), (A, (0, 0, 0)), (F, R))
        diag = np.einsum("ikik->ik", e)
        assert r.norms["Q"][k] == pytest.approx(np.sqrt(diag.max()), rel=1e-12)


def test_home_atom_additivity():
    """Sigma is additive over home atoms A of the <A,B> loop (Algorithm 2)."""
    w = hs.make_workload("tiny", kind="conventional", species_table=((2, 3),), r_c=5.0, r_v=5.0, r_d=6.0,
                         eps=1e-4)
    full = _run(w).sigma
    parts = sum(_run(w, home=[i]).sigma for i in range(w.cells[0].n_atoms))
    np.testing.assert_allclose(parts, full, rtol=1e-12, atol=1e-12 * np.abs(full).max())


@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_supercell_equals_primitive_with_images(eps):
    """Unit cell with images == Gamma-only supercell (Sec. IV A, k mesh vs supercell):
    with translation-keyed blocks, every block of the 8-atom conventional cell equals
    the block of the 2-atom primitive cell between the same two atom positions, and every
    count of the screening (candidates, kept per stage and term, Y and units formed) is
    the primitive cell's per atom (the linear scaling of Sec. III B)."""
    kw = dict(species_table=((2, 3),), r_c=6.0, r_v=6.0, r_d=7.0, seed=77, eps=eps)
    wp = hs.make_workload("tiny", kind="primitive", **kw)
    ws = hs.make_workload("tiny", kind="conventional", **kw)
    rp, rs = _run(wp), _run(ws)
    sp = oracle.sigma_dict(wp.cells[0], wp.D[0], rp.sigma)
    ss = oracle.sigma_dict(ws.cells[0], ws.D[0], rs.sigma)
    # linear scaling: every home atom of the crystal keeps the same work at every stage
    for k in oracle.STAT_NAMES:
        assert rs.stats[k] * wp.cells[0].n_atoms == rp.stats[k] * ws.cells[0].n_atoms, k
    pi, pR = hs.map_to_primitive(ws.cells[0], wp.cells[0])
    Lsup, Lp_inv = ws.cells[0].lattice, np.linalg.inv(wp.cells[0].lattice)
    m = 0.0
    for (i, j, R), blk in ss.items():
        shift = np.rint(np.asarray(R) @ Lsup @ Lp_inv).astype(int)
        Rp = tuple(int(x) for x in pR[j] + shift - pR[i])
        m = max(m, float(np.abs(blk - sp[(int(pi[i]), int(pi[j]), Rp)]).max()))
    assert len(ss) == 4 * len(sp)
    assert m <= 1e-12 * max(float(np.abs(b).max()) for b in sp.values())


def test_screening_bounds_are_rigorous():
    """Every unit dropped by stages 1-3 satisfies max|Htilde| <= its Cauchy-Schwarz
    bound (eq. CS_upper_bounds, with the trace inequalities of Sec. III C 1), and the
    screened Sigma differs from the unscreened one by at most the dropped bounds."""
    w = hs.make_workload("tiny", kind="conventional", species_table=((3, 5),), r_c=6.0, r_v=6.0, r_d=8.0)
    cell = w.cells[0]
    stages = oracle.CS1 | oracle.CS2 | oracle.CS3      # no pre-screen, no CS-ERI: only rigorous gates
    exact = oracle.run(cell, w.C[0], w.V[0], w.D[0], w.thresholds, stages=stages).sigma
    for eps in (1e-3, 1e-2, 1e-1):
        th = dict(w.thresholds, eps_cs_mat=eps)
        r = oracle.run(cell, w.C[0], w.V[0], w.D[0], th, stages=stages, diag=True, dropped=True)
        assert r.diag[1] > 0, "eps too small to drop anything"
        assert r.diag[0] <= 1.0 + 1e-12
        off = r.sig_off
        for k in range(w.D[0].n_blocks):
            dmax = np.abs(r.sigma[off[k]:off[k + 1]] - exact[off[k]:off[k + 1]]).max()
            assert dmax <= r.dropped_bound[k] * (1 + 1e-12) + 1e-14


def test_raising_eps_never_keeps_more():
    w = hs.make_workload("tiny", kind="conventional", species_table=((3, 5),), r_c=6.0, r_v=6.0, r_d=8.0)
    prev = first = None
    for eps in (0.0, 1e-4, 1e-3, 1e-2, 1e-1):
        th = {k: eps for k in w.thresholds}
        st = _run(dataclass_replace(w, thresholds=th)).stats
        cur = np.array([st["kept_cs_eri"]] + [st[f"kept_s{s}_t{t}"] for s in (1, 2, 3) for t in (1, 2, 3, 4)])
        if prev is not None:
            assert np.all(cur <= prev)
        else:
            first = cur
        prev = cur
    assert prev.sum() < first.sum()


def dataclass_replace(w, **kw):
    import dataclasses
    return dataclasses.replace(w, **kw)


def test_stage_counts_are_nested():
    """Algorithm 5 gates stage 2 on stage 1 and stage 3 on stage 2."""
    w = hs.make_workload("tiny", kind="conventional", species_table=((3, 5),), r_c=6.0, r_v=6.0, r_d=8.0, eps=1e-3)
    st = _run(w).stats
    for t in (1, 2, 3, 4):
        assert st[f"kept_s1_t{t}"] >= st[f"kept_s2_t{t}"] >= st[f"kept_s3_t{t}"]
    assert st["units_formed"] == sum(st[f"kept_s3_t{t}"] for t in (1, 2, 3, 4))
    assert st["candidates"] >= st["kept_cs_eri"]


def _random_shape(seed):
    """A seeded tiny cell of random shape: one or two species with n_ao in 1..3 and n_abf in 1..5
    (fewer ABFs than AOs allowed), random ranges for C, V and D."""
    rng = np.random.default_rng(seed)
    n_sp = int(rng.integers(1, 3))
    table = tuple((int(rng.integers(1, 4)), int(rng.integers(1, 6))) for _ in range(n_sp))
    r_c = float(rng.uniform(4.5, 7.5))
    cfg = dict(kind="primitive", species_table=table, r_c=r_c, r_v=float(rng.uniform(4.0, 8.0)),
               r_d=float(rng.uniform(r_c, r_c + 2.5)), seed=1000 + seed)
    if n_sp == 2:
        cfg["species"] = [0, 1]
    return cfg


@pytest.mark.parametrize("seed", range(6))
def test_oracle_equals_bruteforce_random_shapes(seed):
    """As test_oracle_equals_bruteforce, on seeded random block shapes and ranges (Algorithm 1 against
    Algorithms 2/3 at eps = 0)."""
    w = hs.make_workload("tiny", **_random_shape(seed))
    cell = w.cells[0]
    ref = bf.sigma(cell, w.C[0], w.V[0], w.D[0])
    r = _run(w)
    got = oracle.sigma_dict(cell, w.D[0], r.sigma)
    scale = max(float(np.abs(v).max()) for v in ref.values())
    assert scale > 0
    assert _maxdiff(got, ref) <= 1e-12 * scale
