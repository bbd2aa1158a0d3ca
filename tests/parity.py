"""Element-wise and per-field comparison of a GPU result with the oracle's.

A whole-vector norm can hide an error confined to one field (the pressure
block, one velocity component) or to a few DoFs, so every parity check
bounds
  * each element:  |z_i - ref_i| <= tol * ||ref||_inf, and
  * each field f (velocity components, pressure): ||z_f - ref_f||_2 <= tol * ||ref_f||_2.
"""
from __future__ import annotations

import numpy as np


def parity_errors(z: np.ndarray, ref: np.ndarray, field: np.ndarray) -> dict:
    z = np.asarray(z, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    d = np.abs(z - ref)
    out = {"elem": float(d.max() / max(np.abs(ref).max(), 1e-300)) if ref.size else 0.0}
    for f in np.unique(field):
        m = field == f
        nrm = np.linalg.norm(ref[m])
        out[f"field{int(f)}"] = float(np.linalg.norm(z[m] - ref[m]) / nrm) if nrm > 0 else float(np.abs(z[m]).max())
    return out


def assert_parity(z, ref, field, tol: float, label: str = "") -> dict:
    e = parity_errors(z, ref, field)
    print(f"  {label} parity: " + ", ".join(f"{k} {v:.1e}" for k, v in e.items()), flush=True)
    bad = {k: v for k, v in e.items() if not v <= tol}
    assert not bad, f"{label}: {bad} above {tol:g}"
    return e
