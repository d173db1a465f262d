"""The transfer-function parity checker (tests/transfer_checks.py) on the CPU:
it must pass the oracle's own H, and fail on a NaN, an inf, a small error
planted in one pair, and a vacuous pair whose sample row carries no energy.
Also: every input the GPU test feeds it holds the pulse inside its window."""
import numpy as np
import pytest

import synth
from transfer_checks import check_transfer


def _case(orc, N, M, seed=1001):
    fs = 20e12
    x = synth.pairs(3, N=N, fs=fs, t0=min(15e-12, 0.3 * N / fs), seed=seed).astype(np.float64)
    w = (2.5e12 - 0.2e12) / (M * fs)
    W, A = np.exp(-2j * np.pi * w), np.exp(2j * np.pi * 0.2e12 / fs)
    X = orc.czt(x, M, W, A)
    return x, X, X[1::2] / X[0::2]


@pytest.mark.parametrize("N,M", [(4096, 512), (300, 200), (1500, 900)])
def test_checker_passes_exact_H_on_the_gpu_test_inputs(orc, N, M):
    _, X, H = _case(orc, N, M)
    w, b = check_transfer(H.astype(np.complex64), X, 1e-6, 1e-5, say=lambda m: None)
    assert w <= 1e-6 and b <= 1e-5


def test_checker_rejects_nan_inf_and_error(orc):
    _, X, H = _case(orc, 300, 200)
    bad = H.copy()
    bad[1, 7] = np.nan
    with pytest.raises(AssertionError, match="non-finite"):
        check_transfer(bad, X, 1e-6, 1e-5, say=lambda m: None)
    bad = H.copy()
    bad[2, 0] = np.inf
    with pytest.raises(AssertionError, match="non-finite"):
        check_transfer(bad, X, 1e-6, 1e-5, say=lambda m: None)
    # an error of 1e-3 relative at the strongest reference bin of pair 1 only
    bad = H.copy()
    k = int(np.argmax(np.abs(X[2])))
    bad[1, k] *= 1 + 1e-3
    with pytest.raises(AssertionError, match="pair 1"):
        check_transfer(bad, X, 1e-6, 1e-5, say=lambda m: None)


def test_checker_rejects_vacuous_pair(orc):
    x, X, H = _case(orc, 300, 200)
    X = X.copy()
    X[3] *= 1e-6  # the sample of pair 1 almost empty: any H passes a weighted bar
    with pytest.raises(AssertionError, match="vacuous"):
        check_transfer(X[1::2] / X[0::2], X, 1e-6, 1e-5, say=lambda m: None)


def test_short_window_pulses_are_inside():
    """The 300-sample pairs keep the reference and the delayed sample pulse
    well inside the 15 ps window (each row's peak is far above its noise)."""
    fs, N = 20e12, 300
    x = synth.pairs(3, N=N, fs=fs, t0=0.3 * N / fs)
    for row in x:
        peak = np.abs(row).max()
        assert peak > 0.05
        assert int(np.argmax(np.abs(row))) < N - 5
