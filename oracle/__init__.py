"""FP64 CPU oracle for the screened periodic exchange-matrix build.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark, never by the GPU library.  It shares no code with
the GPU path; both are fed by the seeded input generator ``hfx_synth``.

``build_lib()`` compiles ``hfxref.c`` (plain C, OpenMP) into ``libhfxref.so``;
``run()`` calls it on the block-sparse inputs.  ``bruteforce`` holds the
definition-level checker (explicit four-centre integrals, Algorithm 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libhfxref.so")
SRC = os.path.join(HERE, "hfxref.c")

PRE, CS_ERI, CS1, CS2, CS3 = 1, 2, 4, 8, 16
ALL_STAGES = PRE | CS_ERI | CS1 | CS2 | CS3
DIAG_N = 14  # diag: overall max ratio, count, then per (stage, term) max ratio

_lib = None


def build_lib(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_lib()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.hfxref_build.restype = ctypes.c_int
        L.hfxref_build.argtypes = ([ctypes.c_int32, P, P] + [ctypes.c_int64, P, P, P, P, P] * 3 +
                                   [P, ctypes.c_uint32, P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P])
        L.hfxref_energy.restype = ctypes.c_double
        L.hfxref_energy.argtypes = [ctypes.c_int64, P, P, P, P, P, P]
        L.hfxref_sigma_size.restype = ctypes.c_int64
        L.hfxref_sigma_size.argtypes = [ctypes.c_int64, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _blk_args(b):
    row = np.ascontiguousarray(b.row, np.int32)
    col = np.ascontiguousarray(b.col, np.int32)
    R = np.ascontiguousarray(b.R, np.int32).reshape(-1)
    off = np.ascontiguousarray(b.off, np.int64)
    data = np.ascontiguousarray(b.data, np.float64)
    keep = (row, col, R, off, data)
    return keep, [ctypes.c_int64(b.n_blocks), _p(row), _p(col), _p(R), _p(off), _p(data)]


STAT_NAMES = (["candidates", "kept_cs_eri"] + [f"kept_s{s}_t{t}" for s in (1, 2, 3) for t in (1, 2, 3, 4)] +
              ["y_formed", "units_formed"])


@dataclass
class Result:
    sigma: np.ndarray        # flat, D-pattern layout
    sig_off: np.ndarray      # (nD+1,) offsets
    stats: dict
    diag: np.ndarray | None
    dropped_bound: np.ndarray | None
    norms: dict | None


def sigma_offsets(cell, D):
    nao = np.asarray([cell.species_table[s][0] for s in cell.species], np.int64)
    sz = nao[D.row] * nao[D.col]
    off = np.zeros(D.n_blocks + 1, np.int64)
    off[1:] = np.cumsum(sz)
    return off


def run(cell, C, V, D, thresholds: dict, stages: int = ALL_STAGES, home=None, n_threads: int = 0,
        diag: bool = False, dropped: bool = False, norms: bool = False) -> Result:
    """Oracle build of Sigma^X for one cell.  Sigma is returned on the D pattern."""
    L = lib()
    nao = np.asarray([cell.species_table[s][0] for s in cell.species], np.int32)
    nabf = np.asarray([cell.species_table[s][1] for s in cell.species], np.int32)
    kc, ac = _blk_args(C)
    kv, av = _blk_args(V)
    kd, ad = _blk_args(D)
    eps = np.array([thresholds["eps_C"], thresholds["eps_V"], thresholds["eps_D"], thresholds["eps_cs_eri"],
                    thresholds["eps_cs_mat"]], np.float64)
    off = sigma_offsets(cell, D)
    sigma = np.zeros(int(off[-1]), np.float64)
    stats = np.zeros(16, np.int64)
    dg = np.zeros(DIAG_N, np.float64) if diag else None
    drop = np.zeros(D.n_blocks, np.float64) if dropped else None
    nrm = np.zeros(6 * C.n_blocks + V.n_blocks + D.n_blocks, np.float64) if norms else None
    h = None if home is None else np.ascontiguousarray(home, np.int32)
    rc = L.hfxref_build(ctypes.c_int32(cell.n_atoms), _p(nao), _p(nabf), *ac, *av, *ad, _p(eps),
                        ctypes.c_uint32(stages), _p(h), ctypes.c_int32(0 if h is None else len(h)),
                        ctypes.c_int32(n_threads), _p(sigma), _p(stats), _p(dg), _p(drop), _p(nrm))
    if rc != 0:
        raise RuntimeError(f"hfxref_build failed ({rc})")
    del kc, kv, kd
    nd = None
    if norms:
        nC, nV = C.n_blocks, V.n_blocks
        nd = dict(nA=nrm[:nC], gA=nrm[nC:2 * nC], nF=nrm[2 * nC:3 * nC], gF=nrm[3 * nC:4 * nC],
                  Q=nrm[4 * nC:5 * nC], keepC=nrm[5 * nC:6 * nC] > 0.5, gV=nrm[6 * nC:6 * nC + nV],
                  gD=nrm[6 * nC + nV:])
    return Result(sigma, off, dict(zip(STAT_NAMES, stats.tolist())), dg, drop, nd)


def energy(cell, D, sigma) -> float:
    """E_x = 1/2 <D, Sigma^X> over the D pattern (compensated sum)."""
    L = lib()
    nao = np.asarray([cell.species_table[s][0] for s in cell.species], np.int32)
    k, a = _blk_args(D)
    s = np.ascontiguousarray(sigma, np.float64)
    return float(L.hfxref_energy(a[0], a[1], a[2], a[4], a[5], _p(nao), _p(s)))


def sigma_dict(cell, D, sigma) -> dict:
    off = sigma_offsets(cell, D)
    nao = np.asarray([cell.species_table[s][0] for s in cell.species], np.int64)
    out = {}
    for k in range(D.n_blocks):
        r, c = int(D.row[k]), int(D.col[k])
        out[(r, c, tuple(int(x) for x in D.R[k]))] = sigma[off[k]:off[k + 1]].reshape(nao[r], nao[c])
    return out
