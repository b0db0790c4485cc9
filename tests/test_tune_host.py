"""Host logic of the autotuner (no GPU): the candidate grid of each precision form, the accuracy
gate against the FP64 build of the subset, the choice of the fastest admitted candidate and the
tuning-file line, with the library's Plan replaced by a stand-in whose timings and errors are
known."""
import numpy as np
import pytest
import torch

from paper_2009_12505_amd import PREC_BF16X3, PREC_FP64, PREC_TIERED, tune

TILE_MS = {128: 30.0, 64: 20.0, 32: 25.0}


class FakePlan:
    """Sigma = 1 everywhere for the FP64 build; a tiered build with bound tau is off by
    err_per_tau * (tau + tau_bf) in every element and saves 1000 * tau ms."""
    made = []
    err_per_tau = 1e-4
    e_scale = 1e-3  # E_x of the fake build = e_scale * sum(Sigma)

    def __init__(self, cells, C, V, D_pattern, thresholds, precision=PREC_FP64, tier_tau=0.0, tier_tau_bf=0.0,
                 tile_r=64, home_subset=None):
        self.precision, self.tau, self.tau_bf, self.tile = precision, tier_tau, tier_tau_bf, tile_r
        self.tune_key = f"species=13x60 eps=1e-06 prec={tune.FORM_NAMES[precision]}"
        self.last_stats = {}
        FakePlan.made.append((precision, tile_r, tier_tau, tier_tau_bf))

    def build(self, D, stats=False):
        dev = self.err_per_tau * (self.tau + self.tau_bf) if self.precision != PREC_FP64 else 0.0
        self.last_stats = {"ms_main": TILE_MS.get(self.tile, 20.0) - 1000.0 * self.tau}
        return [torch.full((5,), 1.0 + dev, dtype=torch.float64)]

    def energy(self, D, sig):
        return [float(s.sum()) * self.e_scale for s in sig]


@pytest.fixture
def fake(monkeypatch):
    FakePlan.made = []
    FakePlan.err_per_tau = 1e-4
    FakePlan.e_scale = 1e-3
    monkeypatch.setattr(tune, "Plan", FakePlan)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(torch.cuda, "empty_cache", lambda *a, **k: None)
    return FakePlan


def _tune(precision, **kw):
    return tune.tune(None, None, None, None, None, None, precision, list(range(4)), log=lambda *_: None, **kw)


def test_fp64_form_times_tiles_only(fake, tmp_path):
    db = tmp_path / "t.txt"
    key, best, cands = _tune(PREC_FP64, db_path=db, tiles=(128, 64, 32))
    assert [(c.tile_r, c.tier_tau, c.tier_tau_bf) for c in cands] == [(128, 0, 0), (64, 0, 0), (32, 0, 0)]
    assert best.tile_r == 64 and all(c.admitted for c in cands)
    assert db.read_text() == f"hfxtune1 {key} tile_r=64 tier_tau=0 tier_tau_bf=0\n"
    assert fake.made[0] == (PREC_FP64, 64, 0.0, 0.0)  # the FP64 reference build of the subset


def test_tiered_gate_rejects_inaccurate_bounds(fake):
    # errors 1e-6, 1e-7, 1e-8 for tau 1e-2, 1e-3, 1e-4: only the last is within a third of 1e-7
    key, best, cands = _tune(PREC_TIERED, tiles=(64, 32), taus=(1e-4, 1e-3, 1e-2))
    adm = {(c.tile_r, c.tier_tau): c.admitted for c in cands}
    assert adm == {(64, 1e-4): True, (64, 1e-3): False, (64, 1e-2): False,
                   (32, 1e-4): True, (32, 1e-3): False, (32, 1e-2): False}
    c = next(c for c in cands if c.tile_r == 64 and c.tier_tau == 1e-3)
    assert c.max_dsigma == pytest.approx(1e-7, rel=1e-6)
    assert (best.tile_r, best.tier_tau) == (64, 1e-4)  # the faster tau=1e-2 is not admitted


def test_bf16x3_grid_keeps_tau_bf_at_most_tau(fake):
    fake.err_per_tau = 1e-6
    _, best, cands = _tune(PREC_BF16X3, tiles=(64,), taus=(1e-4, 1e-3), taus_bf=(1e-5, 1e-4, 1e-3))
    pairs = [(c.tier_tau, c.tier_tau_bf) for c in cands]
    assert pairs == [(1e-4, 1e-5), (1e-4, 1e-4), (1e-3, 1e-5), (1e-3, 1e-4), (1e-3, 1e-3)]
    assert best.tier_tau == 1e-3 and best.admitted


def test_no_admitted_candidate_is_an_error(fake, tmp_path):
    fake.err_per_tau = 1.0
    db = tmp_path / "t.txt"
    with pytest.raises(RuntimeError, match="accuracy gate"):
        _tune(PREC_TIERED, db_path=db, tiles=(64,), taus=(1e-3,))
    assert not db.exists()


def test_energy_gate_per_home_atom(fake):
    # Sigma within budget but E_x off by more than a third of 1e-8 Ha per home atom (4 atoms)
    fake.err_per_tau = 1e-5
    fake.e_scale = 0.5
    _, _, cands = _tune(PREC_TIERED, tiles=(64,), taus=(2e-3, 1e-4))
    by_tau = {c.tier_tau: c for c in cands}
    assert by_tau[2e-3].max_dsigma <= tune.SIGMA_BUDGET
    assert by_tau[2e-3].de_x_atom == pytest.approx(5 * 2e-8 * 0.5 / 4, rel=1e-6)
    assert by_tau[2e-3].de_x_atom > tune.EX_BUDGET and not by_tau[2e-3].admitted
    assert by_tau[1e-4].admitted
    assert np.isfinite(by_tau[1e-4].ms)
