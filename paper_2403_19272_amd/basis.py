"""Rest-shape subspace for the library (scene set-up, not part of the step).

Section 5 of the paper builds U from the eigenvectors of the rest global
matrix H with the r smallest eigenvalues, once, on the CPU (the paper uses
the Spectra library).  This helper does the same on the host: it reads the
library's own H back through cloth_system_matrix and solves the symmetric
eigenproblem on the free vertices (dense LAPACK for small meshes, shift-
invert Lanczos otherwise).  Pinned rows of U are zero.
"""
from __future__ import annotations

import numpy as np


def rest_eigenbasis(H, pinned, r: int, dense_limit: int = 3000) -> np.ndarray:
    import scipy.sparse.linalg as spla
    nv = H.shape[0]
    pinned = np.zeros(nv, bool) if pinned is None else np.asarray(pinned).astype(bool)
    free = np.flatnonzero(~pinned)
    Hff = H[free][:, free]
    if len(free) <= dense_limit:
        w, V = np.linalg.eigh(Hff.toarray())
        V = V[:, :r]
    else:
        lu = spla.splu(Hff.tocsc(), permc_spec="MMD_AT_PLUS_A", options=dict(SymmetricMode=True))
        op = spla.LinearOperator(Hff.shape, matvec=lu.solve, dtype=np.float64)
        w, V = spla.eigsh(Hff, k=r, sigma=0.0, which="LM", OPinv=op, tol=1e-10)
        V = V[:, np.argsort(w)]
    U = np.zeros((nv, r))
    U[free] = V
    return U
