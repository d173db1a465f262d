"""Parity checker of the transfer function H = X_sample / X_reference of
reference/sample row pairs (Section 1), shared by the GPU test and the CPU
test that proves the checker itself rejects bad output.

For each pair p, with X the FP64 oracle's CZT of every row (references on
even rows, samples on odd rows):
  weighted error  ||X_r (H_gpu - H)|| / ||X_s||   (the error of X_r H)
  strong bins     max |H_gpu - H| / |H| over bins with |X_r| >= 0.1 max |X_r|
Every pair is asserted on its own (no folding through max(), which drops NaN),
H_gpu must be finite everywhere, and both rows of a pair must carry energy
(a vacuous pair with X_s ~ 0 would pass any weighted bar).
"""
import numpy as np

# a pair whose sample spectrum holds less than this share of the reference's
# energy does not test anything
MIN_ENERGY_RATIO = 1e-3


def check_transfer(Hg, X, tol_w, tol_b, say=print, what=""):
    Hg = np.asarray(Hg)
    X = np.asarray(X)
    Xr, Xs = X[0::2], X[1::2]
    assert Hg.shape == Xr.shape, f"{what}: H has shape {Hg.shape}, expected {Xr.shape}"
    assert np.isfinite(Hg).all(), f"{what}: H holds {np.count_nonzero(~np.isfinite(Hg))} non-finite values"
    worst_w, worst_b = 0.0, 0.0
    for p in range(Xr.shape[0]):
        nr, ns = np.linalg.norm(Xr[p]), np.linalg.norm(Xs[p])
        assert nr > 0 and np.isfinite(nr), f"{what}: pair {p}: reference spectrum is zero"
        assert ns >= MIN_ENERGY_RATIO * nr, \
            f"{what}: pair {p}: sample spectrum holds {ns / nr:.2e} of the reference's norm (vacuous pair)"
        H = Xs[p] / Xr[p]
        ew = float(np.linalg.norm(Xr[p] * (Hg[p] - H)) / ns)
        strong = np.abs(Xr[p]) >= 0.1 * np.abs(Xr[p]).max()
        eb = float(np.max(np.abs(Hg[p][strong] - H[strong]) / np.abs(H[strong])))
        assert np.isfinite(ew) and ew <= tol_w, f"{what}: pair {p}: weighted rel L2 {ew:.3e} > {tol_w}"
        assert np.isfinite(eb) and eb <= tol_b, f"{what}: pair {p}: strong-bin rel error {eb:.3e} > {tol_b}"
        worst_w, worst_b = max(worst_w, ew), max(worst_b, eb)
    say(f"  {what}: weighted rel L2 {worst_w:.3e}, strong-bin max rel {worst_b:.3e} over {Xr.shape[0]} pairs")
    return worst_w, worst_b
