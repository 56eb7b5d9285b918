"""Oracle: constrained degrees of freedom beyond the clamped plane.  TEST
INFRASTRUCTURE ONLY.

Eq. (2) prescribes the displacement on part of the boundary.  The voxel
assembly eliminates the clamped plane z = 0; other constraints with zero
prescribed displacement (a roller fixes one component of a node) are kept in
the system as identity rows: the rows and columns of the fixed dofs become
those of the identity and the load is zero there.  Then A x = b has x = 0 at
the fixed dofs and the other dofs solve the reduced system A_ff x_f = b_f,
and A stays symmetric positive definite.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def constrain(A, b, fixed):
    """(A with identity rows and columns at the fixed dofs, b with zeros there)."""
    fixed = np.asarray(fixed, dtype=bool).reshape(-1)
    keep = sp.diags((~fixed).astype(float))
    Ac = (keep @ A @ keep + sp.diags(fixed.astype(float))).tocsr()
    return Ac, np.where(fixed, 0.0, b)
