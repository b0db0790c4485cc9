"""The 4096-atom cell (8^3 conventional diamond cells, 13 AO / 60 ABF per atom, C within 16 bohr,
eps 1e-6) built in full on one GPU: every Sigma block against the oracle's primitive-cell block of
the same atom pair (identical keyed blocks), and E_x per atom."""
import pytest

from test_gpu_parity import _supercell_vs_primitive

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1500)
def test_cfg5_full_vs_primitive():
    _supercell_vs_primitive("cfg5", 1e-6, 1e-11)
