"""The error report on hand-built cases."""
import numpy as np

from paper_1912_05494_amd.report import error_report


def test_report_counts_flips_and_errors():
    o = np.full((4, 4, 3), 2.0)
    g = o.copy()
    assert error_report(g, o) == {"max_rel": 0.0, "mean_rel": 0.0, "flips": 0, "frac_within_tol": 1.0,
                                  "mean_ratio": 1.0, "spectral_pixels": 48}
    g[0, 0, 0] = 2.0 * (1 + 5e-5)          # inside 1e-4
    g[1, 2, 1] = 3.0                       # a flip: relative error 0.5
    r = error_report(g, o)
    assert r["flips"] == 1 and abs(r["max_rel"] - 0.5) < 1e-12
    assert abs(r["mean_rel"] - (0.5 + 5e-5) / 48) < 1e-12
    assert abs(r["frac_within_tol"] - 47 / 48) < 1e-12
    # dark pixels are judged against the floor of the image mean
    o2 = np.array([1.0, 1e-9]); g2 = np.array([1.0, 1e-9 + 4e-8])
    assert error_report(g2, o2)["flips"] == 0
