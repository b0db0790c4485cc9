"""Tile shapes, the split-BF16x3 tier and the autotuner against the FP64 oracle.

* tile_r = 32 and 128 (narrower and wider terms-3/4 output blocks) give the same Sigma as the
  oracle to FP64 summation order, like the default 64.
* HFX_PREC_BF16X3: three tiers (FP64 / FP32 / split-BF16x3 by the stage-2 bounds of a block's
  kept units) meet the method's target (1e-7 max-abs Sigma, 1e-8 Ha per atom) with small tier
  bounds; with every terms-3/4 block forced into split-BF16x3 the error stays within a bound of
  its rounding (about 2^-16 relative per product), i.e. the product is right, only less accurate.
* The autotuner times candidates on a calibration subset, admits only those within a third of the
  accuracy targets, writes its choice to a tuning file, and a plan created with that file (tile_r
  0, tier_tau < 0) builds with the filed choice and matches the oracle."""
import numpy as np
import pytest

import hfx_synth as hs
import oracle
from test_gpu_parity import TINY, check_close, gpu_build, log

pytestmark = pytest.mark.gpu


def _ref(w):
    cell = w.cells[0]
    ref = oracle.run(cell, w.C[0], w.V[0], w.D[0], w.thresholds, n_threads=8)
    return ref, oracle.energy(cell, w.D[0], ref.sigma)


@pytest.mark.parametrize("tile", [32, 128])
@pytest.mark.parametrize("cfg", [1, 4, 5, 6])
def test_tile_r_matches_oracle(cfg, tile):
    log(f"case tile_r {tile} tiny[{cfg}]")
    w = hs.make_workload("tiny", **TINY[cfg])
    ref, e_ref = _ref(w)
    sig, e, st = gpu_build(w, tile_r=tile)
    assert st["tile_r"] == tile
    check_close(sig[0], ref.sigma, label=f"tile_r {tile} tiny[{cfg}]")
    assert abs(e[0] - e_ref) <= 1e-11 * abs(e_ref)
    for t in (1, 2, 3, 4):
        assert st[f"kept_s3_t{t}"] == ref.stats[f"kept_s3_t{t}"]


@pytest.mark.parametrize("cfg,tile", [(1, 64), (4, 128), (5, 32), (6, 64)])
def test_bf16x3_tiers_meet_the_target(cfg, tile):
    from paper_2009_12505_amd import PREC_BF16X3
    log(f"case bf16x3 tiny[{cfg}] tile_r {tile}")
    w = hs.make_workload("tiny", **TINY[cfg])
    ref, e_ref = _ref(w)
    sig, e, st = gpu_build(w, precision=PREC_BF16X3, tier_tau=1e-3, tier_tau_bf=1e-5, tile_r=tile)
    err = float(np.abs(sig[0] - ref.sigma).max())
    de = abs(e[0] - e_ref) / w.cells[0].n_atoms
    log(f"  max|dSigma| {err:.3e}, |dE|/atom {de:.3e}, BF16 MFMA FLOPs {st['mfma_flops_bf16']:.3e}, "
        f"FP32 {st['mfma_flops_fp32']:.3e}")
    assert err <= 1e-7 and de <= 1e-8
    for t in (1, 2, 3, 4):
        assert st[f"kept_s3_t{t}"] == ref.stats[f"kept_s3_t{t}"]


@pytest.mark.parametrize("cfg", [1, 5])
def test_bf16x3_everywhere_within_its_rounding(cfg):
    from paper_2009_12505_amd import PREC_BF16X3
    log(f"case bf16x3 everywhere tiny[{cfg}]")
    w = hs.make_workload("tiny", **TINY[cfg])
    ref, e_ref = _ref(w)
    sig, e, st = gpu_build(w, precision=PREC_BF16X3, tier_tau=1e30, tier_tau_bf=1e30)
    err = float(np.abs(sig[0] - ref.sigma).max())
    scale = float(np.abs(ref.sigma).max())
    log(f"  max|dSigma| {err:.3e} of max|Sigma| {scale:.3e}; BF16 MFMA FLOPs {st['mfma_flops_bf16']:.3e}")
    assert st["mfma_flops_bf16"] > 0
    assert err <= 1e-3 * scale  # 2^-16 relative per product over K <= 10^3 terms: not a wrong result


def test_tuner_files_a_choice_the_plan_uses(tmp_path):
    from paper_2009_12505_amd import PREC_TIERED, tune
    log("case autotuner round trip")
    w = hs.make_workload("tiny", **TINY[5])
    home = list(range(w.cells[0].n_atoms))
    db = tmp_path / "tune.txt"
    key, best, cands = tune.tune(w.cells, w.C, w.V, w.D, w.D, w.thresholds, PREC_TIERED, home, db_path=db,
                                 tiles=(128, 64), taus=(1e-4, 1e-3), reps=1, log=log)
    assert len(cands) == 4 and best.admitted
    line = db.read_text().strip().splitlines()[-1]
    assert line.startswith(f"hfxtune1 {key} tile_r={best.tile_r} ")
    ref, e_ref = _ref(w)
    sig, e, st = gpu_build(w, precision=PREC_TIERED, tier_tau=-1.0, tuning_db=str(db))
    assert st["tile_r"] == best.tile_r and abs(st["tier_tau"] - best.tier_tau) <= 1e-12
    err = float(np.abs(sig[0] - ref.sigma).max())
    assert err <= 1e-7 and abs(e[0] - e_ref) / w.cells[0].n_atoms <= 1e-8
