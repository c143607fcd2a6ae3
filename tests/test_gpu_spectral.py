"""The approximate dispersion relation computed with the GPU operator (paper_1808_00037_amd.spectral)
against the oracle's, mode by mode (the oracle side with its own grid and FFT projection)."""
import numpy as np
import pytest

from paper_1808_00037_amd import spectral as S

from test_oracle_spectral import oracle_adr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,scheme", [(256, 0), (128, 1)])
def test_adr_matches_the_oracle(orc, n, scheme):
    phi_g, Phi_g = S.adr(n, scheme=scheme)
    phi_o, Phi_o, _ = oracle_adr(orc, n, scheme=scheme)
    assert np.allclose(phi_g, phi_o, rtol=0, atol=1e-15)
    assert np.abs(Phi_g - Phi_o).max() < 1e-12 * max(1.0, np.abs(Phi_o).max())
