"""Seeded synthetic inputs for the Wilson-clover solver.

Gauge links U = exp(i*eps*H), one per (site, direction), with H a Gaussian
Hermitian traceless 3x3 matrix, and Gaussian or point spinor sources.  This
module only draws inputs; it holds none of the solver's arithmetic and is the
one piece shared by the oracle's checks, the GPU tests and the benchmark.

Canonical layouts (what the C-ABI takes):
  site index   i = x + Lx*(y + Ly*(z + Lz*t))
  gauge field  [site][mu=x,y,z,t][row][col]  complex128
  spinor field [site][spin][colour]          complex128

The paper's runs use production gauge ensembles (Sec. IV-C); those are
replaced by these synthetic fields of the same shapes.
"""
import os

import numpy as np

# Gell-Mann matrices lambda_1..lambda_8 (standard su(3) generators).
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1] = -1j
_GM[1][1, 0] = 1j
_GM[2][0, 0] = 1
_GM[2][1, 1] = -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2] = -1j
_GM[4][2, 0] = 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2] = -1j
_GM[6][2, 1] = 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)


def volume(L):
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _expi_hermitian(H, eps):
    """exp(i*eps*H) for a batch of Hermitian 3x3 matrices, via eigh."""
    w, v = np.linalg.eigh(H)
    return (v * np.exp(1j * eps * w)[..., None, :]) @ v.conj().swapaxes(-1, -2)


def random_gauge(L, eps, seed, chunk=1 << 16):
    """U_mu(x) = exp(i*eps*H), H = sum_a w_a lambda_a / 2, w_a ~ N(0,1) i.i.d.

    Drawn as w of shape (Lt, Lz, Ly, Lx, 4, 8) in C order from PCG64(seed), so
    the field is a fixed function of (L, eps, seed).  Returns (V, 4, 3, 3)
    complex128 in the canonical layout.  Chunks are exponentiated in a thread
    pool (the result does not depend on the chunking).
    """
    from concurrent.futures import ThreadPoolExecutor
    V = volume(L)
    rng = _rng(seed)
    w = rng.standard_normal((V * 4, 8))
    U = np.empty((V * 4, 3, 3), dtype=np.complex128)
    gm = (_GM / 2).reshape(8, 9)

    def work(a):
        b = min(V * 4, a + chunk)
        H = (w[a:b] @ gm).reshape(-1, 3, 3)
        U[a:b] = _expi_hermitian(H, eps)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(work, range(0, V * 4, chunk)))
    return U.reshape(V, 4, 3, 3)


def unit_gauge(L):
    V = volume(L)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1
    return U


def random_su3(n, seed):
    """n Haar-like random SU(3) matrices (QR of a complex Gaussian, phase-fixed, det 1)."""
    rng = _rng(seed)
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q[:, :, 0] /= det[:, None]          # multiply one column by conj(det) -> det 1
    return q


def gaussian_source(L, seed):
    """Complex spinor with Re and Im ~ N(0,1); drawn as (Lt,Lz,Ly,Lx,4,3,2)."""
    V = volume(L)
    g = _rng(seed).standard_normal((V, 4, 3, 2))
    return (g[..., 0] + 1j * g[..., 1]).astype(np.complex128)


def point_source(L, site, spin, colour):
    V = volume(L)
    f = np.zeros((V, 4, 3), dtype=np.complex128)
    f[site, spin, colour] = 1.0
    return f


def gaussian_spinor(V, seed):
    g = _rng(seed).standard_normal((V, 4, 3, 2))
    return (g[..., 0] + 1j * g[..., 1]).astype(np.complex128)
