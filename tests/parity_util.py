"""Comparison helpers shared by the GPU parity tests."""
import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def max_abs(a, b):
    return float(np.abs(np.asarray(a).ravel() - np.asarray(b).ravel()).max())


def compare_states(gpu, ref, tol_l2=1e-10, tol_alpha=1e-10, label=""):
    """Spec bar: relative L2 on p_rgh and U, max-abs on alpha."""
    e = {
        "alpha_maxabs": max_abs(gpu["alpha"], ref["alpha"]),
        "U_relL2": rel_l2(gpu["U"], ref["U"]),
        "p_rgh_relL2": rel_l2(gpu["p_rgh"], ref["p_rgh"]),
        "F_relL2": rel_l2(np.concatenate(gpu["F"]), np.concatenate(ref["F"])),
    }
    print(label, e, flush=True)
    assert e["alpha_maxabs"] <= tol_alpha, (label, e)
    assert e["U_relL2"] <= tol_l2, (label, e)
    assert e["p_rgh_relL2"] <= tol_l2, (label, e)
    return e
