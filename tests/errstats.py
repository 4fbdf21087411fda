"""Error statistics used by the parity tests (test helper)."""
import numpy as np


def err_stats(a, ref):
    """Normalised rms error sqrt(sum|a-ref|^2 / sum|ref|^2) plus the paper's
    per-particle fractional-error summary (median, fraction above 1e-4;
    Sec. 4.4 and 4.5 report forces this way)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm(a - ref, axis=1)
    m = np.linalg.norm(ref, axis=1)
    rms = float(np.sqrt((d ** 2).sum() / max((m ** 2).sum(), 1e-300)))
    with np.errstate(divide="ignore", invalid="ignore"):
        frac = np.where(m > 0, d / m, np.where(d > 0, np.inf, 0.0))
    return {
        "rms": rms,
        "median": float(np.median(frac)) if frac.size else 0.0,
        "p99": float(np.percentile(frac, 99)) if frac.size else 0.0,
        "max": float(frac.max()) if frac.size else 0.0,
        "frac_gt_1e-4": float((frac > 1e-4).mean()) if frac.size else 0.0,
    }
