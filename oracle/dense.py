"""Dense matrices of the lattice operators, for brute-force checks on tiny lattices."""
import numpy as np


def dense_matrix(apply_op, shape):
    """Matrix M with M[:, j] = apply_op(e_j) for the unit vectors of a field of `shape`."""
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        M[:, j] = apply_op(e.reshape(shape)).ravel()
    return M
