"""Shared set-up of the GPU parity tests: seeded inputs handed to both the HIP
path and the oracle, and the tolerances the comparisons use.

Tolerances (binary32 kernels against the binary64 oracle):
  energy:   |E_gpu - E_ref| <= 1e-3 + 1e-4 |E_ref|          (kcal/mol)
  gradient: |g_gpu,k - g_ref,k| <= 1e-3 + 1e-4 |g_ref,k| for every
            component k (translation, quaternion, torsion and coordinate
            components alike)
A pose with an atom within 1e-4 A of a lattice plane, or an intra pair within
1e-4 A of the cutoff or of a term kink, sits where binary32 and binary64 may
pick different one-sided derivatives (coordinates differ by ~1e-5 A): a
gradient mismatch there is excused, counted, and must stay rare.  A mismatch
anywhere else fails.
"""
import numpy as np

KINK = 1e-4


def e_tol(ref):
    return 1e-3 + 1e-4 * np.abs(ref)


def g_tol(ref):
    """Per-component gradient tolerance (an array shaped like ref)."""
    return 1e-3 + 1e-4 * np.abs(ref)


def g_ok(got, ref):
    return bool(np.all(np.abs(np.asarray(got, np.float64) - ref) <= g_tol(ref)))


def near_kink(r):
    return min(r["min_face"], r["min_cut"], r["min_kink"]) < KINK


def cpu_dof(dof):
    return np.asarray(dof, np.float64)
