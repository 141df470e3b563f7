"""FP64 CPU oracle (test infrastructure only).

Python bindings over oracle/liboracle.so (built from oracle/ddqcd_oracle.c by
oracle/build_oracle.py).  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.

All fields are numpy complex128 in the canonical layouts:
  gauge  (V, 4, 3, 3)   spinor (V, 4, 3)   clover (V, 12, 12)
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, ERR_ARG, ERR_GEOMETRY, ERR_NOMEM, ERR_NOT_CONVERGED = 0, 1, 2, 5, 6


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build_oracle
            build_oracle.build()
        _LIB = ctypes.CDLL(path)
    return _LIB


def _i4(a):
    return (ctypes.c_int * 4)(*[int(v) for v in a])


def _d4(a):
    return (ctypes.c_double * 4)(*[float(v) for v in a])


def _p(a):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a, shape):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.reshape(shape)


def volume(L):
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def clover_field(L, U, kappa, csw):
    """Dense site matrices C(x) = 1/(2 kappa) + D_cl(x), shape (V, 12, 12)."""
    V = volume(L)
    U = _c128(U, (V, 4, 3, 3))
    C = np.empty((V, 12, 12), dtype=np.complex128)
    lib().oracle_clover_field(_i4(L), _p(U), ctypes.c_double(kappa), ctypes.c_double(csw), _p(C))
    return C


def clover_inverse(C):
    C = np.ascontiguousarray(C, dtype=np.complex128)
    Ci = np.empty_like(C)
    st = lib().oracle_clover_inverse_field(ctypes.c_long(C.shape[0]), _p(C), _p(Ci))
    if st != OK:
        raise ValueError("singular clover block")
    return Ci


def apply_A(L, bc, U, C, psi):
    V = volume(L)
    U = _c128(U, (V, 4, 3, 3))
    psi = _c128(psi, (V, 4, 3))
    C = _c128(C, (V, 12, 12))
    out = np.empty((V, 4, 3), dtype=np.complex128)
    lib().oracle_apply_A(_i4(L), _d4(bc), _p(U), _p(C), _p(psi), _p(out))
    return out


def apply_A_sites(L, bc, U, kappa, csw, psi, sites):
    V = volume(L)
    U = _c128(U, (V, 4, 3, 3))
    psi = _c128(psi, (V, 4, 3))
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    lib().oracle_apply_A_sites(_i4(L), _d4(bc), _p(U), ctypes.c_double(kappa), ctypes.c_double(csw), _p(psi),
                               ctypes.c_long(len(sites)), _p(sites), _p(out))
    return out


def _split(fn, L, b, bc, U, C, psi):
    V = volume(L)
    out = np.empty((V, 4, 3), dtype=np.complex128)
    st = fn(_i4(L), _i4(b), _d4(bc), _p(_c128(U, (V, 4, 3, 3))), _p(_c128(C, (V, 12, 12))),
            _p(_c128(psi, (V, 4, 3))), _p(out))
    if st != OK:
        raise ValueError(f"oracle status {st}")
    return out


def apply_Dblock(L, b, bc, U, C, psi):
    return _split(lib().oracle_apply_Dblock, L, b, bc, U, C, psi)


def apply_R(L, b, bc, U, C, psi):
    return _split(lib().oracle_apply_R, L, b, bc, U, C, psi)


def blocksolve(L, b, U, C, Cinv, d, n_mr, rho):
    """Block solve of domain d; returns (delta, block residual) as full fields
    that are zero outside the domain."""
    V = volume(L)
    delta = np.zeros((V, 4, 3), dtype=np.complex128)
    res = np.zeros((V, 4, 3), dtype=np.complex128)
    st = lib().oracle_blocksolve(_i4(L), _i4(b), _p(_c128(U, (V, 4, 3, 3))), _p(_c128(C, (V, 12, 12))),
                                 _p(_c128(Cinv, (V, 12, 12))), ctypes.c_long(d), ctypes.c_int(n_mr),
                                 _p(_c128(rho, (V, 4, 3))), _p(delta), _p(res))
    if st != OK:
        raise ValueError(f"oracle status {st}")
    return delta, res


def sap(L, b, bc, U, C, Cinv, n_cycles, n_mr, eta):
    V = volume(L)
    psi = np.empty((V, 4, 3), dtype=np.complex128)
    st = lib().oracle_sap(_i4(L), _i4(b), _d4(bc), _p(_c128(U, (V, 4, 3, 3))), _p(_c128(C, (V, 12, 12))),
                          _p(_c128(Cinv, (V, 12, 12))), ctypes.c_int(n_cycles), ctypes.c_int(n_mr),
                          _p(_c128(eta, (V, 4, 3))), _p(psi))
    if st != OK:
        raise ValueError(f"oracle status {st}")
    return psi


def sap_additive(L, b, bc, U, C, Cinv, n_cycles, n_mr, eta):
    """Additive Schwarz (Eq. 4): all domains from the same residual each cycle."""
    V = volume(L)
    psi = np.empty((V, 4, 3), dtype=np.complex128)
    st = lib().oracle_sap_additive(_i4(L), _i4(b), _d4(bc), _p(_c128(U, (V, 4, 3, 3))), _p(_c128(C, (V, 12, 12))),
                                   _p(_c128(Cinv, (V, 12, 12))), ctypes.c_int(n_cycles), ctypes.c_int(n_mr),
                                   _p(_c128(eta, (V, 4, 3))), _p(psi))
    if st != OK:
        raise ValueError(f"oracle status {st}")
    return psi


def fgcr(L, b, bc, U, C, Cinv, f, precond=True, n_cycles=16, n_mr=5, restart=16, tol=1e-10, max_cycles=64,
         x0=None, history=False, additive=False):
    """Returns (x, status, n_steps, relres[, history])."""
    V = volume(L)
    f = _c128(f, (V, 4, 3))
    x = np.zeros((V, 4, 3), dtype=np.complex128) if x0 is None else _c128(x0, (V, 4, 3)).copy()
    steps = ctypes.c_int(0)
    rel = ctypes.c_double(0)
    hist = np.zeros(max_cycles * restart + 1)
    b = b if b is not None else (1, 1, 1, 1)
    Cinv = Cinv if Cinv is not None else C
    st = lib().oracle_fgcr(_i4(L), _i4(b), _d4(bc), _p(_c128(U, (V, 4, 3, 3))), _p(_c128(C, (V, 12, 12))),
                           _p(_c128(Cinv, (V, 12, 12))), ctypes.c_int((2 if additive else 1) if precond else 0),
                           ctypes.c_int(n_cycles),
                           ctypes.c_int(n_mr), ctypes.c_int(restart), ctypes.c_double(tol), ctypes.c_int(max_cycles),
                           _p(f), _p(x), ctypes.c_int(0 if x0 is None else 1), ctypes.byref(steps), ctypes.byref(rel),
                           _p(hist))
    out = (x, st, steps.value, rel.value)
    if history:
        n = int(np.count_nonzero(hist))
        return out + (hist[:n],)
    return out


def fgmres_dr(L, b, bc, U, C, Cinv, f, m, k, precond=True, n_cycles=16, n_mr=5, tol=1e-10, max_cycles=64,
              x0=None, history=False, additive=False):
    """Flexible GMRES with deflated restarts (basis m, k deflation vectors).
    Returns (x, status, n_steps, relres[, history])."""
    V = volume(L)
    f = _c128(f, (V, 4, 3))
    x = np.zeros((V, 4, 3), dtype=np.complex128) if x0 is None else _c128(x0, (V, 4, 3)).copy()
    steps = ctypes.c_int(0)
    rel = ctypes.c_double(0)
    hist = np.zeros(max_cycles * m + 1)
    b = b if b is not None else (1, 1, 1, 1)
    Cinv = Cinv if Cinv is not None else C
    st = lib().oracle_fgmres_dr(_i4(L), _i4(b), _d4(bc), _p(_c128(U, (V, 4, 3, 3))), _p(_c128(C, (V, 12, 12))),
                                _p(_c128(Cinv, (V, 12, 12))), ctypes.c_int((2 if additive else 1) if precond else 0),
                                ctypes.c_int(n_cycles), ctypes.c_int(n_mr), ctypes.c_int(m), ctypes.c_int(k),
                                ctypes.c_double(tol), ctypes.c_int(max_cycles), _p(f), _p(x),
                                ctypes.c_int(0 if x0 is None else 1), ctypes.byref(steps), ctypes.byref(rel), _p(hist))
    out = (x, st, steps.value, rel.value)
    if history:
        n = int(np.count_nonzero(hist))
        return out + (hist[:n],)
    return out


def harmonic_ritz(Hbar, k):
    """The oracle's k harmonic Ritz pairs of smallest magnitude of the flexible
    Arnoldi relation with Hessenberg-like Hbar ((m+1) x m): (theta, P), P an
    orthonormal m x k basis of their vectors."""
    Hbar = np.ascontiguousarray(Hbar, dtype=np.complex128)
    m = Hbar.shape[1]
    assert Hbar.shape == (m + 1, m)
    P = np.zeros((m, k), dtype=np.complex128)
    th = np.zeros(k, dtype=np.complex128)
    st = lib().oracle_harmonic_ritz(ctypes.c_int(m), _p(Hbar), ctypes.c_int(k), _p(P), _p(th))
    if st != OK:
        raise ValueError(f"oracle status {st}")
    return th, P


def num_threads():
    return int(lib().oracle_num_threads())
