"""Shared set-up of the GPU parity tests: seeded inputs handed to both the HIP
path and the oracle, and the tolerances the comparisons use.

Tolerances (binary32 kernels against the binary64 oracle):
  energy:   |E_gpu - E_ref| <= 1e-3 + 1e-4 |E_ref|          (kcal/mol)
  gradient: |g_gpu,k - g_ref,k| <= 1e-3 + 1e-4 |g_ref,k| for every
            translation, torsion and coordinate component k; for the four
            raw-quaternion components of a DOF gradient the scale is the
            block's norm, 1e-3 + 1e-4 |g_ref,q|: they are four linear
            combinations of the three torque components, so a component
            that cancels to near zero still carries the torque's rounding
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


def g_tol(ref, dof=False):
    """Per-component gradient tolerance (an array shaped like ref); with
    dof=True, ref is a DOF gradient [t(3), q(4), psi(T)] and the quaternion
    components take the quaternion block's norm as their scale."""
    t = 1e-3 + 1e-4 * np.abs(np.asarray(ref, np.float64))
    if dof:
        t[3:7] = 1e-3 + 1e-4 * np.linalg.norm(ref[3:7])
    return t


def g_ok(got, ref, dof=False):
    return bool(np.all(np.abs(np.asarray(got, np.float64) - ref) <= g_tol(ref, dof)))


def near_kink(r):
    return min(r["min_face"], r["min_cut"], r["min_kink"]) < KINK


def cpu_dof(dof):
    return np.asarray(dof, np.float64)
