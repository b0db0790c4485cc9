"""Strength of the oracle's pins: each case plants one plausible mistake in a scratch copy of the
oracle (a looser or transposed bound factor, a dropped weight, a wrong lattice displacement or
target block, a sign, a transposed block, a wrong Fourier phase, a wrong back-propagation step)
and runs the CPU oracle tests against the copy; every case must make them fail.  CPU only, the
repository's oracle is not touched.  Opt-in (about five minutes with -n 8):

    python -m pytest tests/test_oracle_mutations.py --mutations -n 8
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.mutation

# (name, text in hfxref.c, replacement): the screened build of Algorithms 2-5
C_M = [
 ("gram_sqrt_dropped", "return sqrt(sqrt(s));", "return sqrt(s);"),
 ("gram_as_frobenius", "static double sqrt_gram_norm(const double *X, int m, int n, int ldx) {\n",
  "static double sqrt_gram_norm(const double *X, int m, int n, int ldx) {\n  { double f = 0; for (int i = 0; i < m; ++i) for (int k = 0; k < n; ++k) f += X[i*ldx+k]*X[i*ldx+k]; return sqrt(sqrt(f*f)) > 0 ? sqrt(f) : 0; }\n"),
 ("nA_whole_block", "    if (n > mnA) mnA = n;\n", "    (void)n; { double w = 0; for (int64_t q = 0; q < (int64_t)P*na*nf; ++q) w += c[q]*c[q]; if (sqrt(w) > mnA) mnA = sqrt(w); }\n"),
 ("nA_nF_swapped", "  *nA = mnA;\n", "  *nA = mnF;\n"),
 ("gA_gF_swapped", "  *gA = mgA;\n", "  *gA = mgF;\n"),
 ("gi_wrong_slice", "const double gi = (t < 2) ? x->gA[kf] : x->gF[kf];", "const double gi = (t < 2) ? x->gF[kf] : x->gA[kf];"),
 ("gj_wrong_slice", "const double gj = (t == 0 || t == 2) ? x->gA[kg] : x->gF[kg];", "const double gj = (t == 0 || t == 2) ? x->gF[kg] : x->gA[kg];"),
 ("ni_wrong_slice", "const double ni = (t < 2) ? x->nA[kf] : x->nF[kf];", "const double ni = (t < 2) ? x->nF[kf] : x->nA[kf];"),
 ("ymax_swapped", "const double ymax = (t == 0 || t == 2) ? yb : yg;", "const double ymax = (t == 0 || t == 2) ? yg : yb;"),
 ("b1_no_gD", "const double b1 = gi * gV * gj * x->gD[kd];", "const double b1 = gi * gV * gj;"),
 ("b2_no_gD", "const double b2 = gi * ymax * x->gD[kd];", "const double b2 = gi * ymax;"),
 ("b3_gram_not_norm", "const double b3 = ni * tmax;", "const double b3 = gi * tmax;"),
 ("f_onsite_weight", "const double w = (f_onsite ? 0.5 : 1.0) * (g_onsite ? 0.5 : 1.0);", "const double w = 1.0 * (g_onsite ? 0.5 : 1.0);"),
 ("g_onsite_weight", "const double w = (f_onsite ? 0.5 : 1.0) * (g_onsite ? 0.5 : 1.0);", "const double w = (f_onsite ? 0.5 : 1.0);"),
 ("t2_D_R_sign", "kd = index_find(&x->iD, Ft, Bt, RB[0] - RF[0], RB[1] - RF[1], RB[2] - RF[2]);\n              ktg = index_find(&x->iD, A, Gt,",
  "kd = index_find(&x->iD, Ft, Bt, RF[0] - RB[0], RF[1] - RB[1], RF[2] - RB[2]);\n              ktg = index_find(&x->iD, A, Gt,"),
 ("t3_target_R", "ktg = index_find(&x->iD, Ft, Bt, RB[0] - RF[0], RB[1] - RF[1], RB[2] - RF[2]);", "ktg = index_find(&x->iD, Ft, Bt, RB[0] + RF[0], RB[1] + RF[1], RB[2] + RF[2]);"),
 ("t4_target_swap", "ktg = index_find(&x->iD, Ft, Gt, RG[0] - RF[0], RG[1] - RF[1], RG[2] - RF[2]);", "ktg = index_find(&x->iD, Gt, Ft, RF[0] - RG[0], RF[1] - RG[1], RF[2] - RG[2]);"),
 ("T1_D_transposed", "s += Y[((int64_t)al * nb + b) * ng + g] * Dt[f * ng + g];\n                    T[", "s += Y[((int64_t)al * nb + b) * ng + g] * Dt[g * nf + f];\n                    T["),
 ("T4_D_transposed", "s += Y[((int64_t)al * nb + b) * ng + g] * Dt[a * nb + b];", "s += Y[((int64_t)al * nb + b) * ng + g] * Dt[b * na + a];"),
 ("sigma_sign", "dst[i] -= w * h[i];", "dst[i] += w * h[i];"),
 ("cseri_one_factor", "!(x->Q[kf] * x->Q[kg] > x->eps_eri)", "!(x->Q[kf] > x->eps_eri)"),
 ("q_no_vFF", "    if (vFF) acc_quad(U2, PF, vFF, U2, PF, n, val, W);\n", ""),
 ("q_no_cross", "    if (vAF) acc_quad(cAF, PA, vAF, U2, PF, n, val, W);\n", ""),
 ("q_U2_transposed", "U2[((int64_t)be * na + a) * nf + f] = cFA[((int64_t)be * nf + f) * na + a];", "U2[((int64_t)be * na + a) * nf + f] = cFA[((int64_t)be * na + a) * nf + f];"),
 ("q_max_sum", "    if (val[q] > best) best = val[q];\n", "    best += val[q] > 0 ? val[q] : 0;\n"),
 ("H3_index_swap", "s += Caf[((int64_t)al * na + a) * nf + f] * Tt[((int64_t)al * na + a) * nb + b];", "s += Caf[((int64_t)al * nf + f) * na + a] * Tt[((int64_t)al * na + a) * nb + b];"),
 ("energy_factor", "return 0.5 * (s + c);", "return (s + c);"),
 ("Y_slice_b_uses_g", "                if (sqrt(s) > yb) yb = sqrt(s);\n", "                if (sqrt(s) > yb) yb = sqrt(s) * 0.5;\n"),
 ("t3max_half", "                  if (sqrt(sl[b]) > t3max) t3max = sqrt(sl[b]);\n", "                  if (sqrt(sl[b]) > t3max) t3max = 0.5 * sqrt(sl[b]);\n"),
 ("gV_transposed_dims", "x->gV[k] = need_v[A] ? sqrt_gram_norm(v, x->nabf[A], x->nabf[B], x->nabf[B]) : 0.0;", "x->gV[k] = need_v[A] ? sqrt_gram_norm(v, x->nabf[B], x->nabf[A], x->nabf[A]) : 0.0;"),
 ("keepC_ignored", "x->keepC[k] = pre ? (max_abs(c, (int64_t)P * na * nf) > x->eps_C) : 1;", "x->keepC[k] = 1;"),
 ("keepV_ignored", "x->keepV[k] = pre ? (max_abs(v, (int64_t)x->nabf[A] * x->nabf[B]) > x->eps_V) : 1;", "x->keepV[k] = 1;"),
 ("keepD_ge", "x->keepD[k] = pre ? (max_abs(d, (int64_t)x->nao[K] * x->nao[L]) > x->eps_D) : 1;", "x->keepD[k] = pre ? (max_abs(d, (int64_t)x->nao[K] * x->nao[L]) > 2.0 * x->eps_D) : 1;"),
 ("keepD_ignored", "if (kd < 0 || ktg < 0 || !x->keepD[kd]) continue;", "if (kd < 0 || ktg < 0) continue;"),
]

# (file, name, text, replacement): the k-space steps and the scheduler model
PY_M = [
 ("fourier.py", "F_phase_sign", "phase = np.exp(2j * np.pi * (kfrac @", "phase = np.exp(-2j * np.pi * (kfrac @"),
 ("fourier.py", "F_no_2pi", "phase = np.exp(2j * np.pi * (kfrac @", "phase = np.exp(1j * np.pi * (kfrac @"),
 ("fourier.py", "F_block_T", "blk = np.asarray(sigma[off[b]:off[b + 1]], np.float64).reshape(nao[I], nao[J])",
  "blk = np.asarray(sigma[off[b]:off[b + 1]], np.float64).reshape(nao[J], nao[I]).T"),
 ("fourier.py", "F_place_swap", "H[:, bo[I]:bo[I] + nao[I], bo[J]:bo[J] + nao[J]] += phase[:, None, None] * blk",
  "H[:, bo[J]:bo[J] + nao[J], bo[I]:bo[I] + nao[I]] += phase[:, None, None] * blk.T"),
 ("density.py", "D_phase_sign", "phase = np.exp(-2j * np.pi * (kfrac @", "phase = np.exp(2j * np.pi * (kfrac @"),
 ("density.py", "D_conj_side", "return np.einsum(\"kin,kn,kjn->kij\", np.asarray(ci, np.complex128), np.asarray(occ, np.float64),\n                     np.conj(np.asarray(cj, np.complex128)))",
  "return np.einsum(\"kin,kn,kjn->kij\", np.conj(np.asarray(ci, np.complex128)), np.asarray(occ, np.float64),\n                     np.asarray(cj, np.complex128))"),
 ("density.py", "D_no_nk", ".sum(axis=0) / nk", ".sum(axis=0)"),
 ("density.py", "D_occ_sq", "np.asarray(occ, np.float64),\n                     np.conj", "np.asarray(occ, np.float64) ** 2,\n                     np.conj"),
 ("density.py", "D_block_T", "out[off[b]:off[b + 1]] = blk.real.ravel()", "out[off[b]:off[b + 1]] = blk.real.T.ravel()"),
 ("mlp.py", "M_no_tanh_deriv2", "d2 = (dy @ W3) * (1.0 - h2 * h2)", "d2 = (dy @ W3)"),
 ("mlp.py", "M_W2_T", "d1 = (d2 @ W2) * (1.0 - h1 * h1)", "d1 = (d2 @ W2.T) * (1.0 - h1 * h1)"),
 ("mlp.py", "M_dy_no_2", "dy = 2.0 * r / n", "dy = r / n"),
 ("mlp.py", "M_b1_from_d2", "g_b1 = d1.sum(axis=0)", "g_b1 = d2.sum(axis=0)"),
 ("mlp.py", "M_layout_b1_W2", "W1 = p[o:o + H * F].reshape(H, F); o += H * F", "W1 = p[o:o + H * F].reshape(F, H).T; o += H * F"),
]

C_TESTS = ["tests/test_oracle.py", "tests/test_oracle_bounds.py", "tests/test_oracle_pattern.py"]
PY_TESTS = ["tests/test_fourier_oracle.py", "tests/test_density_oracle.py", "tests/test_mlp_oracle.py"]


def _planted(tmp_path, fname, old, new):
    d = tmp_path / "repo"
    for sub in ("oracle", "tests", "hfx_synth"):
        shutil.copytree(os.path.join(ROOT, sub), d / sub, ignore=shutil.ignore_patterns("__pycache__", "*.so"))
    path = d / "oracle" / fname
    src = path.read_text()
    assert src.count(old) >= 1, "mutation anchor not found"
    path.write_text(src.replace(old, new, 1))
    subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o",
                           str(d / "oracle" / "libhfxref.so"), str(d / "oracle" / "hfxref.c"), "-lm"])
    return d


def _pins_fail(d, tests):
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu and not mutation",
                        "-p", "no:cacheprovider", *tests], cwd=d, capture_output=True, text=True, timeout=1200,
                       env={**os.environ, "OMP_NUM_THREADS": "2"})
    assert r.returncode in (0, 1), r.stdout[-2000:] + r.stderr[-2000:]  # not a collection or usage error
    return r.returncode == 1


@pytest.mark.parametrize("name,old,new", C_M, ids=[m[0] for m in C_M])
def test_screened_build_mistake_is_caught(tmp_path, name, old, new):
    assert _pins_fail(_planted(tmp_path, "hfxref.c", old, new), C_TESTS), f"{name} passes every pin"


@pytest.mark.parametrize("fname,name,old,new", PY_M, ids=[m[1] for m in PY_M])
def test_kspace_and_model_mistake_is_caught(tmp_path, fname, name, old, new):
    assert _pins_fail(_planted(tmp_path, fname, old, new), PY_TESTS), f"{name} passes every pin"


def test_unplanted_copy_passes(tmp_path):
    """Control: the scratch copy with nothing planted passes every pin, so a failure above is the
    planted mistake's."""
    d = _planted(tmp_path, "hfxref.c", "/*", "/*")
    assert not _pins_fail(d, C_TESTS + PY_TESTS)
