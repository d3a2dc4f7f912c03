"""Per-image error report of a render against a reference render (analysis of
results, not part of the render): the mixed-precision form is judged by
these figures against the FP64 oracle."""
import numpy as np


def error_report(image, reference, rtol=1e-4, floor=1e-3):
    """image, reference: spectral images (..., nl).  A spectral pixel is within
    tolerance when |g - o| <= rtol * max(|o|, floor * mean |o|); the ones
    outside are path flips (a decision taken the other way moves a pixel by
    one path weight / spp).  Relative errors use the same floor."""
    g = np.asarray(image, dtype=np.float64)
    o = np.asarray(reference, dtype=np.float64)
    scale = np.maximum(np.abs(o), floor * np.abs(o).mean())
    rel = np.abs(g - o) / np.where(scale > 0, scale, 1.0)
    ok = np.abs(g - o) <= rtol * scale
    return {
        "max_rel": float(rel.max()) if rel.size else 0.0,
        "mean_rel": float(rel.mean()) if rel.size else 0.0,
        "flips": int((~ok).sum()),
        "frac_within_tol": float(ok.mean()) if ok.size else 1.0,
        "mean_ratio": float(g.mean() / o.mean()) if o.size and o.mean() != 0 else 1.0,
        "spectral_pixels": int(o.size),
    }
