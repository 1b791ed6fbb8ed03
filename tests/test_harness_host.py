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


def test_critical_penalty_is_the_first_half_crossing():
    """Fig. 7's critical penalty: where p_s at beta = 20 (slot 0) first reaches 0.5,
    interpolated linearly between the scan points around the crossing."""
    pen = [0.5, 1.0, 1.5, 2.0]
    ps = np.zeros((4, 4, 2))
    ps[0, :, 0] = [0.0, 0.2, 0.8, 0.9]          # crosses between 1.0 and 1.5: 1.0 + 0.3 / 0.6 * 0.5
    ps[1, :, 0] = [0.6, 0.7, 0.9, 1.0]          # already above at the first point
    ps[2, :, 0] = [0.1, 0.2, 0.3, 0.4]          # never
    ps[3, :, 0] = [0.0, 0.5, 0.1, 0.9]          # first crossing counts, exactly 0.5 at 1.0
    ps[:, :, 1] = 1.0                           # another slot is not looked at
    res = H.PTScanResult(pen, np.array([20.0, 0.1]), [0, 0, 0, 0], {"lhz": ps})
    c = res.critical("lhz")
    assert c[0] == pytest.approx(1.25)
    assert c[1] == 0.5
    assert np.isnan(c[2])
    assert c[3] == pytest.approx(1.0)
    assert res.critical("lhz", slot=1) == [0.5] * 4
    cfg = H.PTScanConfig()
    assert cfg.temps == 64 and cfg.beta_max == 20.0 and cfg.beta_min == 0.1 and cfg.sweeps_per_swap == 10
    assert len({H.pt_seed(cfg, i, k, kind, r) for i in range(3) for k in range(5) for kind in range(3)
                for r in range(40)}) == 3 * 5 * 3 * 40
