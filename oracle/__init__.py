"""FP64 CPU oracle (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The GPU library never imports it.  It wraps ``oracle.c`` (plain C,
OpenMP over sites) with ctypes and adds ``expr``, a numpy interpreter for
site-local lattice expressions.

Function index (what each follows; section numbers are the paper's):
- ``shift``          QDP shift over lattice objects (section 4.2: expressions)
- ``smear``          Jacobi source/sink smearing, SRC/SNK of section 5 and
                     Figure 4; operator reading (1 + kappa H)^N
- ``meson``          mesonic hadron spectrum (HAD, section 5): all 16 gamma
                     bilinears, zero-momentum time-slice sums
- ``timeslice_sum``, ``norm2``, ``inner``   FP64 global / time-slice sums
- ``gamma``          dense DeGrand-Rossi gamma products

Pins (tests/test_oracle_pins.py): free-field Fourier closed form, exact
rational values, gauge covariance and invariance, Hermiticity, time-slice
locality, dense brute force on a 2^4 lattice, gamma algebra, Fierz
completeness and gamma_5 hermiticity of the contraction.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.or_shift.argtypes = [_i32p, ctypes.c_int32, _dp, _dp, ctypes.c_int32, ctypes.c_int32]
    lib.or_shift.restype = None
    lib.or_smear_step.argtypes = [_i32p, _dp, _dp, _dp, ctypes.c_double]
    lib.or_smear_step.restype = None
    lib.or_smear.argtypes = [_i32p, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]
    lib.or_smear.restype = ctypes.c_int32
    lib.or_meson.argtypes = [_i32p, _dp, _dp, _dp]
    lib.or_meson.restype = ctypes.c_int32
    lib.or_meson_mom.argtypes = [_i32p, _dp, _dp, ctypes.c_int32, _i32p, _dp]
    lib.or_meson_mom.restype = ctypes.c_int32
    lib.or_nucleon.argtypes = [_i32p, _dp, _dp, ctypes.c_int32, _dp]
    lib.or_nucleon.restype = ctypes.c_int32
    lib.or_delta.argtypes = [_i32p, _dp, ctypes.c_int32, _dp]
    lib.or_delta.restype = ctypes.c_int32
    lib.or_timeslice_sum.argtypes = [_i32p, ctypes.c_int32, _dp, _dp]
    lib.or_timeslice_sum.restype = None
    lib.or_norm2.argtypes = [ctypes.c_int64, _dp]
    lib.or_norm2.restype = ctypes.c_double
    lib.or_inner.argtypes = [ctypes.c_int64, _dp, _dp, _dp]
    lib.or_inner.restype = None
    lib.or_gamma.argtypes = [ctypes.c_int32, _dp]
    lib.or_gamma.restype = None
    lib.or_neighbour.argtypes = [_i32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    lib.or_neighbour.restype = ctypes.c_int64
    _lib = lib
    return lib


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,)
    return d


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def volume(dims) -> int:
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def neighbour(dims, site: int, mu: int, step: int) -> int:
    d = _dims(dims)
    return int(_load().or_neighbour(d.ctypes.data_as(_i32p), site, mu, step))


def shift(field, dims, mu: int, sign: int) -> np.ndarray:
    """dest(x) = field(x + sign * mu_hat); field has shape (V, ...)."""
    f = _c128(field)
    V = volume(dims)
    assert f.shape[0] == V
    ncomplex = f.size // V
    out = np.empty_like(f)
    d = _dims(dims)
    _load().or_shift(d.ctypes.data_as(_i32p), ncomplex, _dptr(f.view(np.float64)),
                     _dptr(out.view(np.float64)), mu, sign)
    return out


def smear_step(U, psi, dims, kappa: float) -> np.ndarray:
    """One application of (1 + kappa H) to one column of shape (V, 4, 3)."""
    U = _c128(U)
    p = _c128(psi)
    out = np.empty_like(p)
    d = _dims(dims)
    _load().or_smear_step(d.ctypes.data_as(_i32p), _dptr(U.view(np.float64)),
                          _dptr(p.view(np.float64)), _dptr(out.view(np.float64)), kappa)
    return out


def smear(U, psi, dims, kappa: float, niter: int) -> np.ndarray:
    """(1 + kappa H)^niter applied to columns of shape (ncols, V, 4, 3)."""
    U = _c128(U)
    p = _c128(psi)
    V = volume(dims)
    assert U.shape == (4, V, 3, 3), U.shape
    if p.ndim == 3:
        p = p[None]
    assert p.shape[1:] == (V, 4, 3), p.shape
    out = np.empty_like(p)
    d = _dims(dims)
    rc = _load().or_smear(d.ctypes.data_as(_i32p), _dptr(U.view(np.float64)),
                          _dptr(p.view(np.float64)), _dptr(out.view(np.float64)),
                          kappa, niter, p.shape[0])
    if rc != 0:
        raise MemoryError("oracle smear: allocation failed")
    return out


def meson(S1, S2, dims) -> np.ndarray:
    """C_n(t) for n = 0..15, shape (16, Lt) complex128; S has shape (12, V, 4, 3)."""
    a = _c128(S1)
    b = _c128(S2)
    V = volume(dims)
    assert a.shape == (12, V, 4, 3) and b.shape == a.shape
    out = np.zeros((16, int(dims[3])), dtype=np.complex128)
    d = _dims(dims)
    rc = _load().or_meson(d.ctypes.data_as(_i32p), _dptr(a.view(np.float64)),
                          _dptr(b.view(np.float64)), _dptr(out.view(np.float64)))
    if rc != 0:
        raise MemoryError("oracle meson: allocation failed")
    return out


def meson_mom(S1, S2, dims, moms) -> np.ndarray:
    """Momentum-projected C_n(p, t), shape (nmom, 16, Lt) complex128, for the
    integer momenta `moms` (sequence of (k0, k1, k2), p_i = 2 pi k_i / L_i)."""
    a = _c128(S1)
    b = _c128(S2)
    V = volume(dims)
    assert a.shape == (12, V, 4, 3) and b.shape == a.shape
    k = np.ascontiguousarray(np.asarray(moms, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((k.shape[0], 16, int(dims[3])), dtype=np.complex128)
    d = _dims(dims)
    rc = _load().or_meson_mom(d.ctypes.data_as(_i32p), _dptr(a.view(np.float64)), _dptr(b.view(np.float64)),
                              int(k.shape[0]), k.ctypes.data_as(_i32p), _dptr(out.view(np.float64)))
    if rc != 0:
        raise MemoryError("oracle meson_mom: allocation failed")
    return out


def nucleon(Su, Sd, dims, parity=1) -> np.ndarray:
    """Proton two-point function C(t), shape (Lt,) complex128, with the
    parity projector (1 + parity gamma_4)/2; Su, Sd have shape (12, V, 4, 3)."""
    a = _c128(Su)
    b = _c128(Sd)
    V = volume(dims)
    assert a.shape == (12, V, 4, 3) and b.shape == a.shape and parity in (1, -1)
    out = np.zeros(int(dims[3]), dtype=np.complex128)
    d = _dims(dims)
    rc = _load().or_nucleon(d.ctypes.data_as(_i32p), _dptr(a.view(np.float64)), _dptr(b.view(np.float64)),
                            int(parity), _dptr(out.view(np.float64)))
    if rc != 0:
        raise MemoryError("oracle nucleon: allocation failed")
    return out


def delta(S, dims, parity=1) -> np.ndarray:
    """Delta++ two-point function C(t), shape (Lt,) complex128, summed over
    the spatial mu and projected with (1 + parity gamma_4)/2; S has shape
    (12, V, 4, 3) (the u propagator)."""
    a = _c128(S)
    V = volume(dims)
    assert a.shape == (12, V, 4, 3) and parity in (1, -1)
    out = np.zeros(int(dims[3]), dtype=np.complex128)
    d = _dims(dims)
    rc = _load().or_delta(d.ctypes.data_as(_i32p), _dptr(a.view(np.float64)), int(parity),
                          _dptr(out.view(np.float64)))
    if rc != 0:
        raise MemoryError("oracle delta: allocation failed")
    return out


def timeslice_sum(field, dims) -> np.ndarray:
    """Per-slice sums of every component, shape (Lt, ncomplex) complex128."""
    f = _c128(field)
    V = volume(dims)
    ncomplex = f.size // V
    out = np.zeros((int(dims[3]), ncomplex), dtype=np.complex128)
    d = _dims(dims)
    _load().or_timeslice_sum(d.ctypes.data_as(_i32p), ncomplex, _dptr(f.view(np.float64)),
                             _dptr(out.view(np.float64)))
    return out


def norm2(field) -> float:
    f = _c128(field)
    return float(_load().or_norm2(f.size, _dptr(f.view(np.float64))))


def inner(a, b) -> complex:
    x = _c128(a)
    y = _c128(b)
    assert x.shape == y.shape
    out = np.zeros(2)
    _load().or_inner(x.size, _dptr(x.view(np.float64)), _dptr(y.view(np.float64)), _dptr(out))
    return complex(out[0], out[1])


def gamma(n: int) -> np.ndarray:
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().or_gamma(n, _dptr(out.view(np.float64)))
    return out
