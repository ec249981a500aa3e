"""Shared test helpers: oracle <-> library layout permutation and error norms (no method arithmetic)."""
import numpy as np

import synth


def rel(a, b):
    """Normwise relative difference ||a - b||_2 / ||b||_2."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def to_lib(S):
    """Oracle dense (M, nrc, nz) -> library packed (tau, nz)."""
    return synth.to_packed(S)


def from_lib(P, M, nrc):
    return synth.from_packed(P, M, nrc)
