"""Per-field error bound shared by the GPU parity tests.

A field f is compared in L1: sum |G_f - R_f| <= tol * sum |R_f| + floor *
sum |R_vec| where R_vec is the whole vector (momentum or face field) that a
component belongs to (a scalar field is its own vector).  The floor states
what rounding alone produces in a component that is much smaller than its
vector (m_x of an Alfven wave, b_y grown from zero by the edge fields): such a
component is formed from products of the vector's full magnitude, so its
absolute error scales with the vector, not with itself.  The floor is a few
tens of units in the last place of the stored precision (FP64 1e-14, FP32
1e-6), far below the per-field tolerance, so it only matters for components
many orders of magnitude below their vector.
"""
import numpy as np

FLOOR = {"f64": 1e-14, "f32": 1e-6}


def vector_slice(f):
    if 1 <= f <= 3:
        return slice(1, 4)
    if 6 <= f <= 8:
        return slice(6, 9)
    return slice(f, f + 1)


def field_error(G, R, f, floor):
    """(L1 error / own L1 norm, L1 error / bound denominator, max abs error);
    the second figure is <= tol exactly when the bound holds."""
    d = np.abs(G[f] - R[f])
    own = float(np.abs(R[f]).sum())
    vec = float(np.abs(R[vector_slice(f)]).sum())
    err = float(d.sum())
    rel_own = err / own if own > 0 else (0.0 if err == 0 else float("inf"))
    return rel_own, err, own, vec, float(d.max())


def within(err, own, vec, tol, floor):
    return err <= tol * own + floor * vec
