"""Euclidean projection onto the second-order cone {(t, eta) : ||eta||_2 <= t}.

Closed form of supplementary section II-C, with a = ||eta||_2 and the three
cases tested in the printed order:
    a <= t        -> (t, eta)
    a <= -t       -> (0, 0)
    otherwise     -> ((t + a) / 2, (t + a) / (2 a) * eta)
A length-1 segment (no eta) is the ray t >= 0 and follows the same rule with a = 0.
"""
from __future__ import annotations

import numpy as np


def project(t: float, eta: np.ndarray):
    a = float(np.sqrt(np.sum(eta * eta))) if eta.size else 0.0
    if a <= t:
        return t, eta.copy()
    if a <= -t:
        return 0.0, np.zeros_like(eta)
    s = (t + a) / 2.0
    return s, (s / a) * eta


def project_rows(S: np.ndarray) -> np.ndarray:
    """Row-wise projection of S[:, 0] = t, S[:, 1:] = eta (all rows the same length)."""
    out = np.empty_like(S)
    for j in range(S.shape[0]):
        t, e = project(S[j, 0], S[j, 1:])
        out[j, 0] = t
        out[j, 1:] = e
    return out


def project_rows_vec(S: np.ndarray) -> np.ndarray:
    """Same rule as `project_rows`, evaluated with array operations."""
    t = S[:, 0]
    eta = S[:, 1:]
    a = np.sqrt(np.sum(eta * eta, axis=1))
    out = np.empty_like(S)
    c1 = a <= t
    c2 = (~c1) & (a <= -t)
    c3 = ~(c1 | c2)
    out[c1] = S[c1]
    out[c2] = 0.0
    s = (t[c3] + a[c3]) / 2.0
    out[c3, 0] = s
    out[c3, 1:] = (s / a[c3])[:, None] * eta[c3]
    return out


def project_segments(x: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """Projection of a concatenation of cones; cone i is x[offsets[i]:offsets[i+1]],
    its first entry is t.  Empty segments are allowed and left untouched."""
    out = np.empty_like(x)
    for i in range(len(offsets) - 1):
        a, b = int(offsets[i]), int(offsets[i + 1])
        if b <= a:
            continue
        t, e = project(float(x[a]), x[a + 1:b])
        out[a] = t
        out[a + 1:b] = e
    return out
