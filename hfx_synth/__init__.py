"""Seeded synthetic inputs for the periodic exchange-matrix build.

This module only draws inputs: diamond-Si-like periodic cells and the block-sparse
expansion coefficients C, ABF interaction matrix V and density matrix D that the
build consumes.  It holds none of the exchange-build arithmetic, and both the
CPU oracle and the GPU library are fed from it.

Data model (paper Sec. II, eq. AO and eq. ABF): every atom reference is a pair
(home-cell atom index, integer lattice vector R).  A block-sparse periodic
tensor is a list of dense blocks, one per (row atom, column atom, R), where the
row atom sits in the home cell and the column atom in cell R.  Block shapes:

    C (row A, col F):  [n_abf(A)][n_ao(A)][n_ao(F)]   expansion coefficients C^{A alpha}_{Aa,Ff}
    V (row A, col B):  [n_abf(A)][n_abf(B)]           (P_{A alpha} | P_{B beta})
    D (row K, col L):  [n_ao(K)][n_ao(L)]             density matrix

Every block is a pure function of (seed, species of both atoms, displacement
vector quantised to 1e-6 bohr), drawn from a counter-based hash (SplitMix64
finaliser), so blocks are translation invariant and identical in a primitive
cell and in any supercell built from it.  Identical blocks may therefore share
storage: ``Blocks.off`` may alias (the consumer treats blocks as read-only).

Value distributions (the stand-in for the paper's HSE06 Si workloads):

* C entries are N(0,1) * exp(-d/2) for pair distance d within the pair cutoff;
  on-site blocks (d = 0) are symmetrised in the two AO indices.
* V = (1-lam) * K_V(|r_A + s_alpha - r_B - s_beta|) * <w_alpha, w_beta> + lam * delta.
  K_V is the screened Coulomb potential (omega = 0.11/bohr) of a Gaussian-smeared
  charge, normalised to K_V(0) = 1, times a Wendland psi_{3,1} taper; it behaves
  as erfc(0.11 d)/d beyond a few bohr.  K_V is a positive-definite function on
  R^3 and <w,w> is a Gram matrix, so the global V is positive definite (Schur
  product theorem) with unit diagonal.  The per-ABF offsets s_alpha make the
  off-site blocks non-symmetric while V(R) = V(-R)^T holds exactly.
* D = K_D(|r_K + t_k - r_L - t_l|) * <u_k, u_l> with K_D = exp(-d/3) times a
  Wendland taper: positive semi-definite with unit diagonal.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

A_SI = 10.26          # diamond Si lattice constant (bohr)
_QUANT = 1e-6         # displacement quantum for block keys (bohr)

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_GOLD = np.uint64(0x9E3779B97F4A7C15)

TAG_C, TAG_W, TAG_S, TAG_U, TAG_T, TAG_OCC, TAG_DIMS = 11, 12, 13, 14, 15, 16, 17


# ----------------------------------------------------------------------------- hashing
def _u64(x) -> np.ndarray:
    a = np.asarray(x)
    if a.dtype == np.uint64:
        return a
    return np.ascontiguousarray(a.astype(np.int64)).view(np.uint64)


def _mix(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014) on uint64 arrays."""
    x = x ^ (x >> np.uint64(30))
    x = x * _M1
    x = x ^ (x >> np.uint64(27))
    x = x * _M2
    return x ^ (x >> np.uint64(31))


def key(*parts) -> np.ndarray:
    """Combine integer parts (scalars or equal-length arrays) into uint64 keys."""
    h = None
    for p in parts:
        v = _u64(np.atleast_1d(p))
        h = _mix(v + _GOLD) if h is None else _mix(h ^ _mix(v + _GOLD))
    return h


def _bits(k: np.ndarray, counter: np.ndarray) -> np.ndarray:
    return _mix(k[:, None] + (counter[None, :].astype(np.uint64) + np.uint64(1)) * _GOLD)


def _uniform01(k: np.ndarray, counter: np.ndarray) -> np.ndarray:
    """Uniform on the open interval (0,1), shape (len(k), len(counter))."""
    b = _bits(k, counter) >> np.uint64(11)
    return (b.astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def keyed_normal(k: np.ndarray, n: int) -> np.ndarray:
    """n standard normals per key (Box-Muller on two keyed uniforms)."""
    c = np.arange(n, dtype=np.uint64)
    u1 = _uniform01(k, 2 * c)
    u2 = _uniform01(k, 2 * c + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def keyed_uniform(k: np.ndarray, n: int, lo: float, hi: float) -> np.ndarray:
    c = np.arange(n, dtype=np.uint64)
    return lo + (hi - lo) * _uniform01(k, c)


# ----------------------------------------------------------------------------- containers
@dataclass
class Cell:
    """One periodic home cell: lattice rows a1,a2,a3 (bohr), cartesian positions, species."""
    lattice: np.ndarray            # (3,3)
    pos: np.ndarray                # (n,3)
    species: np.ndarray            # (n,) int32 index into species_table
    species_table: list            # [(n_ao, n_abf), ...]

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    def n_ao(self, i):
        return np.asarray([self.species_table[s][0] for s in self.species])[i]

    def n_abf(self, i):
        return np.asarray([self.species_table[s][1] for s in self.species])[i]


@dataclass
class Blocks:
    """Block-sparse periodic tensor: block k is (row[k], col[k], R[k]) at data[off[k]:]."""
    row: np.ndarray    # (nb,) int32
    col: np.ndarray    # (nb,) int32
    R: np.ndarray      # (nb,3) int32
    off: np.ndarray    # (nb,) int64
    data: np.ndarray   # float64 flat
    kind: str = ""     # "C", "V" or "D"

    @property
    def n_blocks(self) -> int:
        return int(self.row.shape[0])

    def shape_of(self, cell: Cell, k: int):
        r, c = int(self.row[k]), int(self.col[k])
        nr_ao, nr_abf = cell.species_table[int(cell.species[r])]
        nc_ao, nc_abf = cell.species_table[int(cell.species[c])]
        if self.kind == "C":
            return (nr_abf, nr_ao, nc_ao)
        if self.kind == "V":
            return (nr_abf, nc_abf)
        return (nr_ao, nc_ao)

    def block(self, cell: Cell, k: int) -> np.ndarray:
        shp = self.shape_of(cell, k)
        n = int(np.prod(shp))
        o = int(self.off[k])
        return self.data[o:o + n].reshape(shp)

    def as_dict(self, cell: Cell) -> dict:
        return {(int(self.row[k]), int(self.col[k]), tuple(int(x) for x in self.R[k])): self.block(cell, k)
                for k in range(self.n_blocks)}

    def compact(self, cell: Cell) -> "Blocks":
        """Copy with every block stored separately (no aliasing), in block order."""
        sizes = np.array([int(np.prod(self.shape_of(cell, k))) for k in range(self.n_blocks)], np.int64)
        off = np.zeros(self.n_blocks, np.int64)
        if self.n_blocks:
            off[1:] = np.cumsum(sizes)[:-1]
        data = np.empty(int(sizes.sum()), np.float64)
        for k in range(self.n_blocks):
            data[off[k]:off[k] + sizes[k]] = self.data[int(self.off[k]):int(self.off[k]) + sizes[k]]
        return Blocks(self.row.copy(), self.col.copy(), self.R.copy(), off, data, self.kind)

    def select(self, mask: np.ndarray) -> "Blocks":
        m = np.asarray(mask, bool)
        return Blocks(self.row[m], self.col[m], self.R[m], self.off[m], self.data, self.kind)


@dataclass
class Params:
    """Generator parameters for one workload."""
    r_c: float = 12.0        # C pair cutoff (2 x NAO cutoff)
    r_v: float = 12.0        # V taper radius (blocks beyond are exactly zero, not emitted)
    r_d: float = 12.0        # D taper radius
    omega: float = 0.11      # range-separation parameter of the screened interaction (1/bohr)
    sigma: float = 1.0       # Gaussian smearing width of the ABF charge (bohr)
    lam: float = 1e-2        # ridge weight keeping V positive definite
    c_decay: float = 2.0     # C ~ exp(-d / c_decay)
    d_decay: float = 3.0     # D ~ exp(-d / d_decay)
    abf_offset: float = 0.25  # per-ABF centre offsets, uniform in [-x, x]^3 (bohr)
    ao_offset: float = 0.25   # per-AO centre offsets for D
    gram_dim: int = 128      # dimension of the unit vectors w (ABF) and u (AO)


@dataclass
class Workload:
    name: str
    seed: int
    cells: list
    C: list
    V: list
    D: list
    thresholds: dict
    params: Params
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------- geometry
def diamond_primitive(a: float = A_SI):
    lat = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    pos = np.array([[0.0, 0.0, 0.0], [0.25 * a, 0.25 * a, 0.25 * a]])
    return lat, pos


def diamond_conventional(n1: int, n2: int, n3: int, a: float = A_SI):
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    basis = np.concatenate([fcc, fcc + 0.25])          # 8 atoms, fractional in the cube
    pos = []
    for i in range(n1):
        for j in range(n2):
            for k in range(n3):
                pos.append((basis + np.array([i, j, k])) * a)
    lat = np.diag([n1 * a, n2 * a, n3 * a]).astype(np.float64)
    return lat, np.concatenate(pos)


def enumerate_pairs(lattice: np.ndarray, pos: np.ndarray, cutoff: float, rows=None):
    """All (i home, j, R) with |pos[j] + R.lattice - pos[i]| <= cutoff.

    Returns row, col, R (n,3), displacement (n,3), sorted by (row, col, R)."""
    from scipy.spatial import cKDTree
    n = pos.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    vol = abs(np.linalg.det(lattice))
    h = np.array([vol / np.linalg.norm(np.cross(lattice[(i + 1) % 3], lattice[(i + 2) % 3])) for i in range(3)])
    nr = np.ceil(cutoff / h).astype(int) + 1
    rng = [np.arange(-m, m + 1) for m in nr]
    Rs = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)
    img = (pos[None, :, :] + (Rs @ lattice)[:, None, :]).reshape(-1, 3)
    tree = cKDTree(img)
    out_r, out_c, out_R = [], [], []
    lists = tree.query_ball_point(pos[rows], cutoff + 1e-9)
    for ii, lst in zip(rows, lists):
        lst = np.asarray(lst, np.int64)
        out_r.append(np.full(lst.shape, ii, np.int64))
        out_c.append(lst % n)
        out_R.append(Rs[lst // n])
    row = np.concatenate(out_r) if out_r else np.zeros(0, np.int64)
    col = np.concatenate(out_c) if out_c else np.zeros(0, np.int64)
    R = np.concatenate(out_R) if out_R else np.zeros((0, 3), np.int64)
    order = np.lexsort((R[:, 2], R[:, 1], R[:, 0], col, row))
    row, col, R = row[order], col[order], R[order]
    d = pos[col] + R @ lattice - pos[row]
    return row.astype(np.int32), col.astype(np.int32), R.astype(np.int32), d


# ----------------------------------------------------------------------------- kernels
def _wendland(x: np.ndarray) -> np.ndarray:
    """Wendland psi_{3,1}(x) = (1-x)^4 (4x+1) on [0,1], 0 beyond (positive definite on R^3)."""
    y = np.clip(1.0 - x, 0.0, None)
    return y ** 4 * (4.0 * x + 1.0)


def kernel_v(r: np.ndarray, p: Params) -> np.ndarray:
    """Screened (erfc, omega) potential of a Gaussian charge, K_V(0) = 1, tapered at r_v."""
    from scipy.special import erf
    r = np.asarray(r, np.float64)
    k0 = 2.0 / math.sqrt(math.pi) * (1.0 / p.sigma - p.omega)
    small = r < 1e-8
    rs = np.where(small, 1.0, r)
    val = (erf(rs / p.sigma) - erf(p.omega * rs)) / rs / k0
    val = np.where(small, 1.0, val)
    return val * _wendland(r / p.r_v)


def kernel_d(r: np.ndarray, p: Params) -> np.ndarray:
    return np.exp(-np.asarray(r) / p.d_decay) * _wendland(np.asarray(r) / p.r_d)


# ----------------------------------------------------------------------------- species data
class _SpeciesData:
    def __init__(self, seed: int, sid: int, n_ao: int, n_abf: int, p: Params):
        self.n_ao, self.n_abf = n_ao, n_abf
        w = keyed_normal(key(seed, TAG_W, sid, np.arange(n_abf)), p.gram_dim)
        self.w = w / np.linalg.norm(w, axis=1, keepdims=True)
        self.s = keyed_uniform(key(seed, TAG_S, sid, np.arange(n_abf)), 3, -p.abf_offset, p.abf_offset)
        u = keyed_normal(key(seed, TAG_U, sid, np.arange(n_ao)), p.gram_dim)
        self.u = u / np.linalg.norm(u, axis=1, keepdims=True)
        self.t = keyed_uniform(key(seed, TAG_T, sid, np.arange(n_ao)), 3, -p.ao_offset, p.ao_offset)


def _quant(d: np.ndarray) -> np.ndarray:
    return np.rint(d / _QUANT).astype(np.int64)


def _unique_keys(sr, sc, q):
    rows = np.concatenate([sr[:, None].astype(np.int64), sc[:, None].astype(np.int64), q], axis=1)
    uniq, inv = np.unique(rows, axis=0, return_inverse=True)
    return uniq, inv.reshape(-1)


def _draw(kind, tab, sr, sc, d, seed, p, spd):
    """Block data for pairs with row/column species sr, sc and displacement d: one draw per
    distinct (species pair, quantised displacement), vectorised over the draws of a species
    pair.  Returns (data, offset of each pair's block)."""
    q = _quant(d)
    uniq, inv = _unique_keys(sr, sc, q)
    nu = uniq.shape[0]
    a_all, b_all, q_all = uniq[:, 0].copy(), uniq[:, 1].copy(), uniq[:, 2:5].copy()
    flip = np.zeros(nu, bool)
    if kind in ("V", "D"):
        # V(R) = V(-R)^T and D(R) = D(-R)^T exactly: draw the canonical orientation, transpose
        # (canonical: (species of col, -q) does not precede (species of row, q) lexicographically)
        nq = -q_all
        lt = (nq[:, 0] < q_all[:, 0]) | ((nq[:, 0] == q_all[:, 0]) & (
            (nq[:, 1] < q_all[:, 1]) | ((nq[:, 1] == q_all[:, 1]) & (nq[:, 2] < q_all[:, 2]))))
        flip = (b_all < a_all) | ((b_all == a_all) & lt)
        a_all[flip], b_all[flip] = uniq[flip, 1], uniq[flip, 0]
        q_all[flip] = nq[flip]
    if kind == "C":
        sizes = np.array([tab[int(x)][1] * tab[int(x)][0] * tab[int(y)][0] for x, y in zip(uniq[:, 0], uniq[:, 1])],
                         np.int64)
    elif kind == "V":
        sizes = np.array([tab[int(x)][1] * tab[int(y)][1] for x, y in zip(uniq[:, 0], uniq[:, 1])], np.int64)
    else:
        sizes = np.array([tab[int(x)][0] * tab[int(y)][0] for x, y in zip(uniq[:, 0], uniq[:, 1])], np.int64)
    uoff = np.zeros(nu, np.int64)
    if nu:
        uoff[1:] = np.cumsum(sizes)[:-1]
    data = np.empty(int(sizes.sum()), np.float64)
    for a in np.unique(a_all):
        for b in np.unique(b_all):
            sel = np.nonzero((a_all == a) & (b_all == b))[0]
            if sel.size == 0:
                continue
            A, B = spd[int(a)], spd[int(b)]
            qd = q_all[sel]
            dv = qd.astype(np.float64) * _QUANT                      # (n,3)
            if kind == "C":
                z = keyed_normal(key(seed, TAG_C, a, b, qd[:, 0], qd[:, 1], qd[:, 2]), A.n_abf * A.n_ao * B.n_ao)
                z = z.reshape(-1, A.n_abf, A.n_ao, B.n_ao)
                onsite = np.all(qd == 0, axis=1)
                if np.any(onsite):
                    z[onsite] = (z[onsite] + z[onsite].transpose(0, 1, 3, 2)) / math.sqrt(2.0)
                blk = z * np.exp(-np.linalg.norm(dv, axis=1) / p.c_decay)[:, None, None, None]
            elif kind == "V":
                rv = np.linalg.norm(dv[:, None, None, :] + B.s[None, None, :, :] - A.s[None, :, None, :], axis=3)
                blk = (1.0 - p.lam) * kernel_v(rv, p) * (A.w @ B.w.T)[None]
                onsite = np.all(qd == 0, axis=1) & (a == b)
                if np.any(onsite):
                    blk[onsite] += p.lam * np.eye(A.n_abf)
            else:
                rd = np.linalg.norm(dv[:, None, None, :] + B.t[None, None, :, :] - A.t[None, :, None, :], axis=3)
                blk = kernel_d(rd, p) * (A.u @ B.u.T)[None]
            n = sel.size
            size = int(blk[0].size)
            out = np.empty((n, size), np.float64)
            fl = flip[sel]
            out[~fl] = blk[~fl].reshape(-1, size)
            if np.any(fl):
                out[fl] = blk[fl].transpose(0, 2, 1).reshape(-1, size)
            pos = uoff[sel][:, None] + np.arange(size)[None, :]
            data[pos] = out
    return data, uoff[inv]


def build_blocks_multi(cells, seed: int, p: Params):
    """C, V and D blocks for cells that share one species table and one keyed draw:
    identical blocks (same species pair and displacement) share storage within and
    across cells."""
    tab = cells[0].species_table
    spd = [_SpeciesData(seed, s, na, nb, p) for s, (na, nb) in enumerate(tab)]
    out = {"C": [], "V": [], "D": []}
    for kind, rc in (("C", p.r_c), ("V", p.r_v), ("D", p.r_d)):
        pairs = [enumerate_pairs(c.lattice, c.pos, rc - 1e-9 if kind != "C" else rc) for c in cells]
        sr = np.concatenate([c.species[pr[0]] for c, pr in zip(cells, pairs)])
        sc = np.concatenate([c.species[pr[1]] for c, pr in zip(cells, pairs)])
        d = np.concatenate([pr[3] for pr in pairs])
        data, off = _draw(kind, tab, sr, sc, d, seed, p, spd)
        k0 = 0
        for (row, col, R, _), c in zip(pairs, cells):
            n = row.shape[0]
            out[kind].append(Blocks(row.astype(np.int32), col.astype(np.int32), R.astype(np.int32), off[k0:k0 + n],
                                    data, kind))
            k0 += n
    return out["C"], out["V"], out["D"]


def build_blocks(cell: Cell, seed: int, p: Params):
    """C, V and D blocks for one cell (aliased storage for identical blocks)."""
    C, V, D = build_blocks_multi([cell], seed, p)
    return C[0], V[0], D[0]


# ----------------------------------------------------------------------------- configs
SEED0 = 2009_12505


def make_cell(kind: str, n=(1, 1, 1), species_table=((13, 40),), species=None, a: float = A_SI,
              lattice=None, pos=None) -> Cell:
    if kind == "primitive":
        lat, pos = diamond_primitive(a)
    elif kind == "custom":
        lat, pos = np.asarray(lattice, np.float64), np.asarray(pos, np.float64)
    else:
        lat, pos = diamond_conventional(*n, a=a)
    sp = np.zeros(pos.shape[0], np.int32) if species is None else np.asarray(species, np.int32)
    return Cell(lat, pos, sp, [tuple(s) for s in species_table])


def make_workload(name: str, seed: int | None = None, eps: float | None = None, **kw) -> Workload:
    """Named workloads.

    cfg1      2-atom primitive cell, 13/40, all blocks within 12 bohr, no screening
    cfg2      64 atoms (2^3 conventional cells), 13/40, C within 16 bohr, eps 1e-6
    cfg3      512 atoms (4^3 conventional cells), 13/60, C within 16 bohr, eps 1e-6 (or 1e-4)
    cfg2prim  the 2-atom primitive cell of cfg2 with identical keyed blocks
    cfg3prim  the 2-atom primitive cell of cfg3 with identical keyed blocks
    cfg4      48 cells of 1..3 x 1..3 x 1..3 conventional cells, species 13/60 and 27/100
              drawn per site with p = 1/2, C within 12 bohr, V within 24, D within 30, eps 1e-4
    cfg5      4096 atoms (8^3 conventional cells), 13/60, eps 1e-6
    lr        full-range Coulomb variant: 64 atoms (2^3 conventional cells), 13/60, C within 12 bohr,
              V the unscreened (omega = 0) smeared Coulomb interaction tapered at 50 bohr, D within
              45 bohr, eps 1e-4
    lrprim    the 2-atom primitive cell of lr with identical keyed blocks
    tiny      user-sized cells for tests (keywords: kind, n, species_table, r_c, r_v, r_d, eps)
    """
    idx = {"cfg1": 0, "cfg2": 1, "cfg2prim": 1, "cfg3": 2, "cfg3prim": 2, "cfg4": 3, "cfg5": 4, "cfg5prim": 4,
           "lr": 5, "lrprim": 5, "tiny": 9}[name]
    seed = SEED0 + idx if seed is None else seed
    if name == "cfg1":
        p = Params(r_c=12.0, r_v=12.0, r_d=12.0)
        cells = [make_cell("primitive", species_table=((13, 40),))]
        th = 0.0 if eps is None else eps
    elif name in ("cfg2", "cfg2prim", "cfg3", "cfg3prim", "cfg5", "cfg5prim"):
        p = Params(r_c=16.0, r_v=36.0, r_d=45.0)
        nabf = 40 if name.startswith("cfg2") else 60
        if name.endswith("prim"):
            cells = [make_cell("primitive", species_table=((13, nabf),))]
        else:
            n = {"cfg2": 2, "cfg3": 4, "cfg5": 8}[name]
            cells = [make_cell("conventional", (n, n, n), species_table=((13, nabf),))]
        th = 1e-6 if eps is None else eps
    elif name in ("lr", "lrprim"):
        p = Params(r_c=12.0, r_v=50.0, r_d=45.0, omega=0.0)
        if name == "lrprim":
            cells = [make_cell("primitive", species_table=((13, 60),))]
        else:
            cells = [make_cell("conventional", (2, 2, 2), species_table=((13, 60),))]
        th = 1e-4 if eps is None else eps
    elif name == "cfg4":
        # eps 1e-4: V beyond ~20 bohr and D beyond ~28 bohr are below it before tapering
        p = Params(r_c=12.0, r_v=24.0, r_d=30.0)
        ncell = kw.pop("n_cells", 48)
        cells = []
        for c in range(ncell):
            dims = (1 + (key(seed, TAG_DIMS, c, np.arange(3)) % np.uint64(3))).astype(int)
            lat, pos = diamond_conventional(*dims)
            occ = (key(seed, TAG_OCC, c, np.arange(pos.shape[0])) >> np.uint64(63)).astype(np.int32)
            cells.append(Cell(lat, pos, occ, [(13, 60), (27, 100)]))
        th = 1e-4 if eps is None else eps
    else:
        p = Params(r_c=kw.pop("r_c", 8.0), r_v=kw.pop("r_v", 8.0), r_d=kw.pop("r_d", 8.0))
        for f in ("c_decay", "d_decay", "lam", "abf_offset", "ao_offset"):
            if f in kw:
                setattr(p, f, kw.pop(f))
        cells = [make_cell(kw.pop("kind", "primitive"), kw.pop("n", (1, 1, 1)),
                           species_table=kw.pop("species_table", ((3, 5),)), species=kw.pop("species", None),
                           a=kw.pop("a", A_SI), lattice=kw.pop("lattice", None), pos=kw.pop("pos", None))]
        th = 0.0 if eps is None else eps
    if kw:
        raise TypeError(f"unknown keywords {sorted(kw)}")
    C, V, D = build_blocks_multi(cells, seed, p)
    thr = dict(eps_C=th, eps_V=th, eps_D=th, eps_cs_eri=th, eps_cs_mat=th)
    return Workload(name, seed, cells, C, V, D, thr, p)


def map_to_primitive(cell: Cell, prim: Cell):
    """For each atom of a diamond supercell: (primitive atom index, integer lattice vector of
    the primitive cell holding it).  Used to compare a supercell result with the primitive one."""
    inv = np.linalg.inv(prim.lattice)
    out_i = np.zeros(cell.n_atoms, np.int64)
    out_R = np.zeros((cell.n_atoms, 3), np.int64)
    for i, x in enumerate(cell.pos):
        for j, y in enumerate(prim.pos):
            f = (x - y) @ inv
            if np.allclose(f, np.rint(f), atol=1e-8):
                out_i[i], out_R[i] = j, np.rint(f).astype(np.int64)
                break
        else:
            raise ValueError("atom does not map onto the primitive cell")
    return out_i, out_R
