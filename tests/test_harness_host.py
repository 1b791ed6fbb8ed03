"""Host-side pieces of the penalty-scan harness (no GPU): unit conversion of the
paper's couplings and penalties."""
import numpy as np
import pytest

from paper_1603_03755_amd import harness as H


def test_paper_instance_values():
    """Sec. III: J_ij uniform over {+-0.1, ..., +-1}, h = 0; times 10 in integers."""
    J = H.paper_instance(16, 3)
    iu = np.triu_indices(16, 1)
    vals = J[iu]
    assert set(np.unique(vals).tolist()) <= set(range(-10, 0)) | set(range(1, 11))
    assert len(np.unique(vals)) >= 15
    assert (np.tril(J) == 0).all()


def test_penalty_coefficient_and_units():
    assert H.penalty_coefficient(0.5) == -5
    assert H.penalty_coefficient(2.0) == -20
    assert H.penalty_coefficient(0.0) == 0
    with pytest.raises(ValueError):
        H.penalty_coefficient(0.25)
    cfg = H.ScanConfig()
    # beta' J' = beta J and beta' Gamma' = beta Gamma
    beta_p = cfg.beta_eff / H.SCALE
    assert beta_p * 10 == pytest.approx(cfg.beta_eff * 1.0)
    assert beta_p * (H.SCALE * cfg.gamma_start) == pytest.approx(cfg.beta_eff * cfg.gamma_start)
    assert cfg.slices == 64 and cfg.sweeps == 10_000 and cfg.reads == 1000
