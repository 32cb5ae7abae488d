"""Shared comparison helpers for the parity tests."""
import numpy as np

FAMILIES = [[0], [1], [2, 3, 4], [5, 6, 7], [8], [9]]


def family_scale(P):
    """Per-variable denominator field: max(|P_v|, RMS over the grid of P_v's family)."""
    nvar = P.shape[0]
    out = np.empty_like(P)
    for fam in FAMILIES:
        fam = [v for v in fam if v < nvar]
        if not fam:
            continue
        rms = np.sqrt(np.mean(np.stack([P[v] ** 2 for v in fam])))
        for v in fam:
            out[v] = np.maximum(np.abs(P[v]), rms)
    return np.where(out > 0, out, 1.0)


def prim_rel_err(A, B):
    """Per-primitive error of A against reference B, normalised by family_scale(B)."""
    A = np.asarray(A, dtype=np.float64).reshape(B.shape)
    return np.abs(A - B) / family_scale(B)
