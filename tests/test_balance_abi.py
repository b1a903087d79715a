"""Correction-coefficient update (Section "Load balancing") through the C-ABI
against the oracle: host-only code, so it runs without a GPU."""
import numpy as np
import pytest

import oracle.partition as op
from paper_2005_05899_amd import lesasm


def _hist(rng, P, K, R=lambda s: s + 0.2 * s ** 2):
    lams = rng.uniform(0.5, 1.5, (K, P))
    lams *= P / lams.sum(axis=1, keepdims=True)
    edges = np.concatenate([np.zeros((K, 1)), np.cumsum(lams, axis=1)], axis=1)
    ts = np.diff(R(edges), axis=1) * rng.uniform(0.9, 1.1, (K, P))
    return lams, ts


@pytest.mark.parametrize("P,K", [(2, 1), (4, 1), (8, 2), (8, 5), (33, 7), (256, 4)])
@pytest.mark.parametrize("growth", [1.0, 1.5])
def test_update_matches_oracle(P, K, growth):
    rng = np.random.default_rng(P * 100 + K)
    lams, ts = _hist(rng, P, K)
    got = lesasm.balance_update(lams, ts, growth)
    want = op.balance_update(lams, ts, growth)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * P)
    assert abs(got.sum() - P) < 1e-9 * P and (got >= 0).all()


def test_degenerate_and_clamped_cases_match_oracle():
    rng = np.random.default_rng(3)
    P = 6
    # the same coefficients twice: no spread, fall back to the newest point
    lam = rng.uniform(0.5, 1.5, P)
    lam *= P / lam.sum()
    ts = rng.uniform(1, 2, (2, P))
    for g in (1.0, 1.5):
        assert np.allclose(lesasm.balance_update([lam, lam], ts, g), op.balance_update([lam, lam], ts, g),
                           rtol=1e-12, atol=1e-12)
    # noisy, non-monotone times: negative slopes and clamping
    lams = rng.uniform(0.2, 1.8, (4, P))
    lams *= P / lams.sum(axis=1, keepdims=True)
    ts = rng.uniform(0.0, 3.0, (4, P))
    ts[1, :2] = 0.0
    assert np.allclose(lesasm.balance_update(lams, ts, 1.5), op.balance_update(lams, ts, 1.5), rtol=1e-12,
                       atol=1e-12)


def test_balanced_history_is_a_fixed_point():
    lam = np.array([0.5, 1.5, 1.0, 1.0])
    got = lesasm.balance_update([lam], [[3.0, 3.0, 3.0, 3.0]])
    assert np.allclose(got, lam, rtol=0, atol=1e-14)


def test_update_errors():
    with pytest.raises(lesasm.LesasmError):
        lesasm.balance_update([[1.0, 1.0]], [[1.0, -1.0]])
    with pytest.raises(lesasm.LesasmError):
        lesasm.balance_update([[1.0, np.nan]], [[1.0, 1.0]])
    with pytest.raises(lesasm.LesasmError):
        lesasm.balance_update([[1.0, 1.0]], [[0.0, 0.0]])
    with pytest.raises(lesasm.LesasmError):
        lesasm.balance_update([[1.0, 1.0]], [[1.0, 1.0]], growth=0.0)
    with pytest.raises(ValueError):
        lesasm.balance_update([[1.0, 1.0]], [[1.0, 1.0, 1.0]])
