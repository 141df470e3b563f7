"""Independent numpy references used to pin the oracle on tiny lattices.

Nothing here is imported by the oracle or by the GPU library.  The gamma
matrices are defined here a second time, on their own, so that a mistake in
either definition shows up as a disagreement.
"""
import numpy as np

# Pauli matrices and the chiral-basis gammas, mu = x, y, z, t
PAULI = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128)
GAMMA = np.zeros((4, 4, 4), dtype=np.complex128)
for _k in range(3):
    GAMMA[_k][:2, 2:] = -1j * PAULI[_k]
    GAMMA[_k][2:, :2] = 1j * PAULI[_k]
GAMMA[3][:2, 2:] = -np.eye(2)
GAMMA[3][2:, :2] = -np.eye(2)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]


def sigma(mu, nu):
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


def coords(L):
    """(V, 4) integer coordinates of every site, site = x + Lx(y + Ly(z + Lz t))."""
    V = int(np.prod(L))
    i = np.arange(V)
    x = i % L[0]
    y = (i // L[0]) % L[1]
    z = (i // (L[0] * L[1])) % L[2]
    t = i // (L[0] * L[1] * L[2])
    return np.stack([x, y, z, t], axis=1)


def index(L, c):
    return c[..., 0] + L[0] * (c[..., 1] + L[1] * (c[..., 2] + L[2] * c[..., 3]))


def shift(L, mu, step):
    """site index of x + step*mu for every x (periodic wrap)."""
    c = coords(L).copy()
    c[:, mu] = (c[:, mu] + step) % L[mu]
    return index(L, c)


def dense_operator(apply, n):
    """Assemble the n x n matrix of a linear map on flat complex vectors."""
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1
        M[:, j] = apply(e).reshape(-1)
        e[j] = 0
    return M


def domain_ids(L, b):
    c = coords(L)
    n = [L[m] // b[m] for m in range(4)]
    X = c // np.array(b)
    return X[:, 0] + n[0] * (X[:, 1] + n[1] * (X[:, 2] + n[2] * X[:, 3])), X.sum(axis=1) % 2


def site_parity(L):
    return coords(L).sum(axis=1) % 2


def textbook_mr(M, rhs, n_iter):
    """Minimal residual iteration for M x = rhs from x = 0 (Saad, Iterative
    Methods for Sparse Linear Systems, Sec. 5.3.2)."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    for _ in range(n_iter):
        p = M @ r
        pp = np.vdot(p, p).real
        a = np.vdot(p, r) / pp if pp > 0 else 0
        x = x + a * r
        r = r - a * p
    return x, r


def dense_block_solve(Ablk, par_dof, rho, n_mr):
    """Even-odd preconditioned MR on one domain from its dense matrix.

    Ablk: dense matrix of D restricted to the domain (dof ordering arbitrary);
    par_dof: site parity of each dof.  Returns (delta, block residual)."""
    e = np.where(par_dof == 0)[0]
    o = np.where(par_dof == 1)[0]
    Dee, Deo = Ablk[np.ix_(e, e)], Ablk[np.ix_(e, o)]
    Doe, Doo = Ablk[np.ix_(o, e)], Ablk[np.ix_(o, o)]
    Dooi = np.linalg.inv(Doo) if len(o) else Doo
    S = Dee - Deo @ Dooi @ Doe
    rt = rho[e] - Deo @ (Dooi @ rho[o])
    x, r = textbook_mr(S, rt, n_mr)
    delta = np.zeros_like(rho)
    delta[e] = x
    delta[o] = Dooi @ (rho[o] - Doe @ x)
    res = np.zeros_like(rho)
    res[e] = r
    return delta, res
