"""Independent (SciPy) construction of the regularised operator, used to
check properties of GPU outputs without feeding them to the oracle."""
import numpy as np
import scipy.sparse as sp


def path_laplacian(k):
    """Sparse graph Laplacian of a path with k nodes."""
    main = np.full(k, 2.0)
    if k > 0:
        main[0] = main[-1] = 1.0
    if k == 1:
        main[0] = 0.0
    off = -np.ones(max(k - 1, 0))
    return sp.diags([off, main, off], [-1, 0, 1], shape=(k, k), format="csr")


def laplacian(nx, ny, nz):
    """-(grid-graph Laplacian) in the unknown order (iy, ix, iz), depth fastest."""
    Iy, Ix, Iz = sp.identity(ny), sp.identity(nx), sp.identity(nz)
    L = (sp.kron(sp.kron(path_laplacian(ny), Ix), Iz) + sp.kron(sp.kron(Iy, path_laplacian(nx)), Iz)
         + sp.kron(sp.kron(Iy, Ix), path_laplacian(nz)))
    return (-L).tocsr()


def sparse_abar(s):
    G = sp.csr_matrix((s.val, s.col, s.row_ptr), shape=(s.m, s.n))
    return sp.vstack([G, s.smooth * laplacian(s.nx, s.ny, s.nz),
                      s.damp * sp.identity(s.n)]).tocsr()


def eta_explicit(s, x, A=None):
    """|Abar^T (bbar - Abar x)| / |Abar^T bbar| and |bbar - Abar x|."""
    A = sparse_abar(s) if A is None else A
    b = np.r_[s.dt, np.zeros(2 * s.n)]
    r = b - A @ x
    return np.linalg.norm(A.T @ r) / np.linalg.norm(A.T @ b), np.linalg.norm(r)
