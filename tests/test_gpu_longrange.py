"""The full-range Coulomb variant (the unscreened, Gaussian-smeared 1/r interaction tapered at
50 bohr instead of the HSE-screened one): far more V blocks survive the pre-screen (3917 partners
per atom within 50 bohr against 1419 within 36) and the quartet screening keeps far more units,
which stresses the same kernels.  The 64-atom supercell built on the GPU against the oracle's
primitive cell with identical keyed blocks, every Sigma block."""
import pytest

from test_gpu_parity import _supercell_vs_primitive

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_longrange_64_atoms_vs_primitive():
    _supercell_vs_primitive("lr", 1e-4, 1e-11)
