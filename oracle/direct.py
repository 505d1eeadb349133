"""Direct reference solutions of A f = b (dense LU for tiny grids, sparse LU).

Test infrastructure (oracle): see the package docstring.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def dense_solve(A, b):
    return np.linalg.solve(A.toarray(), np.asarray(b, np.complex128))


def sparse_solve(A, b):
    lu = spla.splu(A.tocsc())
    return lu.solve(np.asarray(b, np.complex128))
