"""Explicit sparse-matrix assembly of the three operators, written
independently of the oracle (numpy/scipy only), for brute-force pins.

CONST27 is built offset by offset with boolean masks; VAR7 is built as
sum_d D_d^T K_d D_d from the paper's difference matrix D and padding matrix
P (Sec. 4.1) through Kronecker products; BLOCK7 as sum_d S_d (x) B_d with
1-D shift matrices.  Flattening is C order of (nz, ny, nx[, 5]).
"""
import numpy as np
import scipy.sparse as sp


def const27(nx, ny, nz, diag=26.0, off=-1.0):
    n = nx * ny * nz
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                          indexing="ij")
    rows, cols, vals = [], [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ii, jj, kk = i + dx, j + dy, k + dz
                m = ((ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) &
                     (kk >= 0) & (kk < nz))
                p = (k * ny + j) * nx + i
                q = (kk * ny + jj) * nx + ii
                rows.append(p[m])
                cols.append(q[m])
                v = diag if (dx, dy, dz) == (0, 0, 0) else off
                vals.append(np.full(int(m.sum()), v))
    return sp.csr_matrix((np.concatenate(vals),
                          (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def diff_matrix(m):
    """The paper's D_(m): (m-1) x m, rows [.. -1 1 ..]."""
    return sp.diags([-np.ones(m - 1), np.ones(m - 1)], [0, 1],
                    shape=(m - 1, m))


def pad_matrix(n):
    """The paper's P = [0; I; 0]: (n+2) x n."""
    return sp.vstack([sp.csr_matrix((1, n)), sp.eye(n),
                      sp.csr_matrix((1, n))])


def padded_diff(n):
    """D_(n+2) P: the n+1 face differences of [0; u; 0]."""
    return (diff_matrix(n + 2) @ pad_matrix(n)).tocsr()


def var7(kx, ky, kz):
    nz, ny, nx1 = kx.shape
    nx = nx1 - 1
    Ix, Iy, Iz = sp.eye(nx), sp.eye(ny), sp.eye(nz)
    Dx = sp.kron(Iz, sp.kron(Iy, padded_diff(nx)))
    Dy = sp.kron(Iz, sp.kron(padded_diff(ny), Ix))
    Dz = sp.kron(padded_diff(nz), sp.kron(Iy, Ix))
    A = (Dx.T @ sp.diags(kx.ravel()) @ Dx + Dy.T @ sp.diags(ky.ravel()) @ Dy
         + Dz.T @ sp.diags(kz.ravel()) @ Dz)
    return A.tocsr()


def block7(nx, ny, nz, blocks):
    Ix, Iy, Iz = sp.eye(nx), sp.eye(ny), sp.eye(nz)
    shifts = [
        sp.kron(Iz, sp.kron(Iy, Ix)),
        sp.kron(Iz, sp.kron(Iy, sp.eye(nx, k=-1))),
        sp.kron(Iz, sp.kron(Iy, sp.eye(nx, k=1))),
        sp.kron(Iz, sp.kron(sp.eye(ny, k=-1), Ix)),
        sp.kron(Iz, sp.kron(sp.eye(ny, k=1), Ix)),
        sp.kron(sp.eye(nz, k=-1), sp.kron(Iy, Ix)),
        sp.kron(sp.eye(nz, k=1), sp.kron(Iy, Ix)),
    ]
    A = sum(sp.kron(S, sp.csr_matrix(blocks[d])) for d, S in
            enumerate(shifts))
    return A.tocsr()


def split_ldu(A):
    """Strict lower, diagonal, strict upper parts (scalar)."""
    return sp.tril(A, -1).tocsr(), sp.diags(A.diagonal()).tocsr(), \
        sp.triu(A, 1).tocsr()


def split_block_ldu(A, bs=5):
    """Strict block-lower, block-diagonal, strict block-upper parts."""
    A = A.tocoo()
    br, bc = A.row // bs, A.col // bs
    low = br > bc
    dia = br == bc
    up = br < bc
    mk = lambda m: sp.csr_matrix((A.data[m], (A.row[m], A.col[m])),  # noqa
                                 shape=A.shape)
    return mk(low), mk(dia), mk(up)
