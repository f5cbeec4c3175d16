"""Image-quality metrics of Sec. 4.1 (test oracle).

Test infrastructure only.
  interpolation fraction = #interpolated / (n_x n_y)          (Eq. 7)
  flux error             = |F - F_hat| / F                    (Eq. 8)
  mean squared error     = sum |I - I_hat|^2 / sum |I|^2      (Eq. 9)
Fluxes are plain pixel sums on the common grid (the constant pixel area
cancels in the ratio).
"""
import numpy as np


def interp_fraction(level):
    return float((np.asarray(level) < 0).sum()) / float(np.asarray(level).size)


def flux_error(truth, approx):
    F = float(np.sum(truth, dtype=np.float64))
    Fh = float(np.sum(approx, dtype=np.float64))
    return abs(F - Fh) / abs(F)


def mse(truth, approx):
    t = np.asarray(truth, dtype=np.float64)
    d = np.asarray(approx, dtype=np.float64) - t
    return float(np.sum(d * d) / np.sum(t * t))


def residual_image(truth, approx, ibar):
    """|I_hat - I| / Ibar (Sec. 4.2, residual images)."""
    return np.abs(np.asarray(approx) - np.asarray(truth)) / ibar
