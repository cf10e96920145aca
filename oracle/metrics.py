"""Error metrics of Section 4.2 (oracle; test use only).

For reference coefficients f and reconstructed g over all (l, m):
max |f-g|, mean |f-g|, median |f-g|, rms = sqrt(mean |f-g|^2) and the relative
rms = sqrt(sum |f-g|^2 / sum |f|^2).  The last one is the "relative l2" error
used for every parity bar.
"""

from __future__ import annotations

import numpy as np


def error_metrics(f: np.ndarray, g: np.ndarray) -> dict:
    f = np.asarray(f).ravel()
    g = np.asarray(g).ravel()
    d = np.abs(f - g)
    den = float(np.sum(np.abs(f) ** 2))
    return {
        "max": float(d.max()) if d.size else 0.0,
        "mean": float(d.mean()) if d.size else 0.0,
        "median": float(np.median(d)) if d.size else 0.0,
        "rms": float(np.sqrt(np.mean(d ** 2))) if d.size else 0.0,
        "rel_rms": float(np.sqrt(np.sum(d ** 2) / den)) if den > 0 else float(np.sqrt(np.sum(d ** 2))),
    }


def rel_l2(f: np.ndarray, g: np.ndarray) -> float:
    """Relative rms error sqrt(sum|f-g|^2 / sum|f|^2), f the reference."""
    return error_metrics(f, g)["rel_rms"]
