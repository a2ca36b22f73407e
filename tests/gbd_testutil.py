"""Shared helpers of the test-suite (error metrics, library build check)."""
import os

import numpy as np


def rel_l2(E, ref):
    """Raw relative L2 error ||E - ref|| / ||ref||."""
    E = np.asarray(E, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.linalg.norm(E - ref) / np.linalg.norm(ref))


def rel_l2_phase_aligned(E, ref):
    """min over a global phase phi of ||E e^{i phi} - ref|| / ||ref||, with
    phi = arg sum(conj(E) ref)."""
    E = np.asarray(E, np.complex128)
    ref = np.asarray(ref, np.complex128)
    phi = np.angle(np.vdot(E, ref))
    return float(np.linalg.norm(E * np.exp(1j * phi) - ref) / np.linalg.norm(ref))


def ensure_library():
    """Build the HIP library only if nothing is built yet."""
    from paper_2404_12454_amd import build, library_path
    if not os.path.exists(library_path()):
        build.build()
    return library_path()
