"""Seeded synthetic inputs: SU(3) gauge links, Gaussian propagators, point
sources and gauge transformations.

This module holds input generation only; none of the smearing, contraction or
summation arithmetic lives here.  It is used by the tests (to feed the oracle
and the GPU library the same arrays) and by the benchmark.

Random numbers come from a counter-based generator, Philox4x32-10 (Salmon,
Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11),
so that any element of any field can be generated on its own: complex normal
number ``e`` of stream ``sid`` under ``seed`` is the Box-Muller transform of
the Philox block with counter ``(e mod 2^32, e div 2^32, sid, 0)`` and key
``(seed mod 2^32, seed div 2^32)``.  The GPU library implements the same
published generator independently for full-size benchmark inputs; the two
agree to the last few bits of the transcendental functions.

Layouts are the canonical host layouts (lexicographic sites, x fastest):
gauge ``(4, V, 3, 3)``, fermion columns ``(ncols, V, 4, 3)``.

Recipes (the paper uses real gauge ensembles that are not available; these
synthetic fields have the same shapes and the structure the method needs):
- link U_mu(x): 3x3 complex Gaussian, orthonormalised column by column
  (Gram-Schmidt with re-orthogonalisation, which equals QR with a positive
  real diagonal of R, i.e. the Haar-distributed unitary), then divided by the principal cube root of its
  determinant so that det U = 1;
- synthetic propagator: 12 columns of i.i.d. complex Gaussians whose real and
  imaginary parts are N(0, 1), scaled by 1/sqrt(24 V) so each column has unit
  expected norm (a fixed factor, so that any time slice can be generated
  without the rest of the field);
- point source: 1 at (site, spin, colour) of the given column, 0 elsewhere.
"""

from __future__ import annotations

import numpy as np

# Philox4x32 constants from the published definition.
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

STREAM_LINKS = 1
STREAM_PROPAGATOR = 2
STREAM_GAUGE_TRANSFORM = 3


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32 with 10 rounds.

    Arguments are uint64 arrays (or scalars) holding 32-bit values; returns
    four uint64 arrays holding the 32-bit output words.
    """
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    k0 = np.uint64(k0) & _MASK
    k1 = np.uint64(k1) & _MASK
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0  # exact: both factors < 2^32
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def _uniform53(hi, lo):
    """Two 32-bit words -> a double in (0, 1) with 53 random bits."""
    k = ((hi >> np.uint64(5)) << np.uint64(26)) | (lo >> np.uint64(6))
    return (k.astype(np.float64) + 0.5) * 2.0**-53


def complex_normals(seed: int, stream: int, index) -> np.ndarray:
    """Complex numbers whose real and imaginary parts are independent N(0, 1).

    ``index`` is an integer array of element numbers within (seed, stream).
    """
    e = np.asarray(index, dtype=np.uint64)
    w0, w1, w2, w3 = philox4x32_10(
        e & _MASK, e >> _S32, np.uint64(stream), np.uint64(0),
        np.uint64(seed) & _MASK, np.uint64(seed) >> _S32)
    u1 = _uniform53(w0, w1)
    u2 = _uniform53(w2, w3)
    r = np.sqrt(-2.0 * np.log(u1))
    theta = 2.0 * np.pi * u2
    return r * np.cos(theta) + 1j * (r * np.sin(theta))


def volume(dims) -> int:
    return int(dims[0]) * int(dims[1]) * int(dims[2]) * int(dims[3])


def _site_range(dims, t_range):
    vs = volume(dims) // int(dims[3])
    t0, t1 = (0, int(dims[3])) if t_range is None else t_range
    return np.arange(t0 * vs, t1 * vs, dtype=np.uint64)


def _su3_from_gaussian(z: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on the columns of each 3x3 matrix, then det -> 1."""
    q = np.empty_like(z)
    for j in range(3):
        v = z[..., :, j].copy()
        # Two projection passes keep the columns orthonormal to rounding level
        # even for nearly singular draws.
        for _ in range(2):
            for k in range(j):
                proj = np.sum(np.conj(q[..., :, k]) * v, axis=-1)
                v = v - proj[..., None] * q[..., :, k]
        nrm = np.sqrt(np.sum((v * np.conj(v)).real, axis=-1))
        q[..., :, j] = v / nrm[..., None]
    det = np.linalg.det(q)
    phase = np.angle(det)  # principal branch, in (-pi, pi]
    fix = np.exp(-1j * phase / 3.0)
    return q * fix[..., None, None]


def su3_links(dims, seed: int, t_range=None) -> np.ndarray:
    """Gauge field U_mu(x), shape (4, V_sub, 3, 3), complex128.

    With ``t_range=(t0, t1)`` only the sites of slices t0..t1-1 are returned,
    identical to the corresponding rows of the full field.
    """
    V = volume(dims)
    sites = _site_range(dims, t_range)
    out = np.empty((4, sites.size, 3, 3), dtype=np.complex128)
    comp = np.arange(9, dtype=np.uint64)
    for mu in range(4):
        idx = ((np.uint64(mu) * np.uint64(V) + sites)[:, None] * np.uint64(9) + comp[None, :])
        z = complex_normals(seed, STREAM_LINKS, idx).reshape(-1, 3, 3)
        out[mu] = _su3_from_gaussian(z)
    return out


def gauge_transform(dims, seed: int, t_range=None) -> np.ndarray:
    """Per-site SU(3) matrices g(x), shape (V_sub, 3, 3)."""
    sites = _site_range(dims, t_range)
    comp = np.arange(9, dtype=np.uint64)
    idx = sites[:, None] * np.uint64(9) + comp[None, :]
    z = complex_normals(seed, STREAM_GAUGE_TRANSFORM, idx).reshape(-1, 3, 3)
    return _su3_from_gaussian(z)


def gaussian_propagator(dims, seed: int, ncols: int = 12, t_range=None,
                        columns=None) -> np.ndarray:
    """Synthetic propagator columns, shape (ncols, V_sub, 4, 3), complex128."""
    V = volume(dims)
    sites = _site_range(dims, t_range)
    cols = list(range(ncols)) if columns is None else list(columns)
    out = np.empty((len(cols), sites.size, 4, 3), dtype=np.complex128)
    comp = np.arange(12, dtype=np.uint64)
    scale = 1.0 / np.sqrt(24.0 * V)
    for i, j in enumerate(cols):
        idx = ((np.uint64(j) * np.uint64(V) + sites)[:, None] * np.uint64(12) + comp[None, :])
        out[i] = (complex_normals(seed, STREAM_PROPAGATOR, idx) * scale).reshape(-1, 4, 3)
    return out


def point_source(dims, columns=range(12), site: int = 0) -> np.ndarray:
    """Point-source columns: column j has 1 at (site, spin j//3, colour j%3)."""
    V = volume(dims)
    cols = list(columns)
    out = np.zeros((len(cols), V, 4, 3), dtype=np.complex128)
    for i, j in enumerate(cols):
        out[i, site, j // 3, j % 3] = 1.0
    return out


def lattice_sizes_batch(count: int = 64, seed: int = 4000):
    """Uneven lattice sizes for the multi-lattice batch: drawn uniformly from
    8^3x16, 12^3x24, 16^3x32 and 24^3x48 with numpy's default generator."""
    choices = [(8, 8, 8, 16), (12, 12, 12, 24), (16, 16, 16, 32), (24, 24, 24, 48)]
    draw = np.random.default_rng(seed).integers(0, 4, count)
    return [choices[int(k)] for k in draw]


def to_interleaved(a: np.ndarray) -> np.ndarray:
    """complex128 array -> contiguous float64 array with a trailing (re, im)."""
    return np.ascontiguousarray(np.ascontiguousarray(a).view(np.float64))


def from_interleaved(a: np.ndarray, shape) -> np.ndarray:
    return np.ascontiguousarray(a).view(np.complex128).reshape(shape)
