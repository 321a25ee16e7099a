"""Comparison helpers of the GPU parity tests (no map-making arithmetic).

``err`` is the larger of two figures, so that a test bound holds for both:
the relative L2 norm of the difference over the whole vector, and for each
component (I, Q, U of a pixel-domain vector, or the lone component of a
timeline) the element-wise max |a - b| / max |b|.  A Q/U error far above the
bar cannot hide under the I-dominated joint norm this way.
"""
import numpy as np


def _np(a):
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.asarray(a, dtype=np.float64)


def joint_rel(a, b):
    a, b = _np(a).reshape(-1), _np(b).reshape(-1)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def comp_rel(a, b, nc=1):
    """Per component: max |a - b| / max |b| (max |a - b| where b is all zero)."""
    a, b = _np(a).reshape(-1, nc), _np(b).reshape(-1, nc)
    if a.shape != b.shape:
        raise ValueError(f"shapes differ: {a.shape} vs {b.shape}")
    if a.size == 0:
        return np.zeros(nc)
    num = np.abs(a - b).max(axis=0)
    den = np.abs(b).max(axis=0)
    return num / np.where(den > 0, den, 1.0)


def err(a, b, nc=1):
    """max(joint relative L2, every per-component element-wise ratio)."""
    return max(joint_rel(a, b), float(np.max(comp_rel(a, b, nc))))
