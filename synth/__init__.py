"""Seeded synthetic inputs for the triangular-inverse workloads.

This module holds only the random draws that build input matrices. It holds
none of the method's arithmetic (no inverse, no product, no residual) and it is
the one piece of code that the CPU oracle and the GPU path both use.

The paper measures on "non-singular triangular matrices" of unstated
distribution (Section 6, Table tab:combrit); these generators stand in for
them with a well-conditioned family:

* diagonal entries ``(1 + u) * s`` with ``u ~ U[0,1)`` and a random sign ``s``,
* strictly-lower entries ``(2u - 1) / n`` (uniform in ``[-1, 1) / n``),
* the strict upper part is zero unless the caller asks for garbage there
  (the inversion must ignore it).

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: the ``c``-th output for seed ``s`` is ``mix(s + (c + 1) * GAMMA)``
modulo 2**64, and a double in ``[0, 1)`` is ``(x >> 11) * 2**-53``. Every
matrix element has a fixed counter, so any element can be regenerated alone
and the bytes do not depend on the generation order or block size.

Counter assignment for an ``n x n`` matrix with seed ``s``:

* element ``(i, j)`` of the strict lower part: counter ``i * n + j``;
* diagonal ``i``: magnitude counter ``i * n + i``, sign counter ``n * n + i``;
* garbage in the strict upper part ``(i, j)``: counter ``i * n + j``
  (the same counter as a lower slot would use, which is unused there).
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_ROWS_PER_CHUNK = 512


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, counters) -> np.ndarray:
    """Raw 64-bit outputs of SplitMix64 for ``seed`` at the given counters."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * GAMMA)


def uniform01(seed: int, counters) -> np.ndarray:
    """Doubles in [0, 1) with 53 random bits, one per counter."""
    return (splitmix64(seed, counters) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def lower_triangular(n: int, seed: int, *, unit: bool = False, positive_diag: bool = False,
                     upper_garbage: bool = False, dtype=np.float64) -> np.ndarray:
    """Dense ``n x n`` row-major lower-triangular test matrix.

    ``unit`` puts ones on the diagonal; ``positive_diag`` drops the random sign;
    ``upper_garbage`` fills the strict upper part with values in [-8, 8) that a
    correct inversion never reads. ``dtype=float32`` rounds the FP64 draws to
    nearest-even, so FP32 paths and the oracle see the same (rounded) matrix.
    """
    n = int(n)
    out = np.zeros((n, n), dtype=np.float64)
    if n == 0:
        return out.astype(dtype)
    cols = np.arange(n, dtype=np.uint64)
    for r0 in range(0, n, _ROWS_PER_CHUNK):
        r1 = min(n, r0 + _ROWS_PER_CHUNK)
        rows = np.arange(r0, r1, dtype=np.uint64)
        ctr = rows[:, None] * np.uint64(n) + cols[None, :]
        u = uniform01(seed, ctr)
        blk = (2.0 * u - 1.0) / n
        ri = np.arange(r0, r1)[:, None]
        cj = np.arange(n)[None, :]
        low = cj < ri
        if upper_garbage:
            blk = np.where(low, blk, 16.0 * u - 8.0)
        else:
            blk = np.where(low, blk, 0.0)
        out[r0:r1] = blk
    idx = np.arange(n, dtype=np.uint64)
    if unit:
        diag = np.ones(n)
    else:
        mag = 1.0 + uniform01(seed, idx * np.uint64(n) + idx)
        if positive_diag:
            diag = mag
        else:
            sgn = uniform01(seed, np.uint64(n) * np.uint64(n) + idx)
            diag = np.where(sgn < 0.5, -mag, mag)
    out[np.arange(n), np.arange(n)] = diag
    return out.astype(dtype)


def upper_triangular(n: int, seed: int, *, unit: bool = False, positive_diag: bool = True,
                     dtype=np.float64) -> np.ndarray:
    """Upper-triangular factor: the transpose of a lower draw with the same seed.

    Diagonal ``1 + u`` (positive by default), strict upper ``(2u - 1) / n``.
    """
    return np.ascontiguousarray(
        lower_triangular(n, seed, unit=unit, positive_diag=positive_diag, dtype=np.float64).T
    ).astype(dtype)


def batch_sizes(batch: int, seed: int = 6, lo: int = 16, hi: int = 512) -> np.ndarray:
    """Sizes ``n_i = lo + (splitmix64(seed, i) mod (hi - lo + 1))`` for i < batch."""
    raw = splitmix64(seed, np.arange(batch, dtype=np.uint64))
    return (np.uint64(lo) + raw % np.uint64(hi - lo + 1)).astype(np.int64)


def batch_offsets(sizes) -> np.ndarray:
    """Element offsets of dense row-major blocks packed back to back."""
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes) > 1:
        off[1:] = np.cumsum(sizes[:-1] * sizes[:-1])
    return off


def packed_batch(sizes, first_seed: int = 1000, dtype=np.float32) -> np.ndarray:
    """All matrices of a batch packed densely; matrix i uses seed first_seed + i."""
    sizes = np.asarray(sizes, dtype=np.int64)
    total = int(np.sum(sizes * sizes))
    out = np.empty(total, dtype=dtype)
    off = batch_offsets(sizes)
    for i, n in enumerate(sizes):
        n = int(n)
        out[off[i]:off[i] + n * n] = lower_triangular(n, first_seed + i, dtype=dtype).ravel()
    return out


def normal(n_rows: int, n_cols: int, seed: int, dtype=np.float64) -> np.ndarray:
    """i.i.d. N(0, 1) by the Box-Muller transform; element (i, j) uses counters
    ``2 (i n_cols + j)`` and ``2 (i n_cols + j) + 1``."""
    k = np.arange(n_rows * n_cols, dtype=np.uint64)
    u1 = uniform01(seed, k * np.uint64(2))
    u2 = uniform01(seed, k * np.uint64(2) + np.uint64(1))
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    return z.reshape(n_rows, n_cols).astype(dtype)


def integer_unit_lower(n: int, seed: int, lo: int = -3, hi: int = 3) -> np.ndarray:
    """Unit lower-triangular matrix with integer strict-lower entries in [lo, hi]."""
    ctr = np.arange(n * n, dtype=np.uint64).reshape(n, n)
    raw = splitmix64(seed, ctr)
    vals = (raw % np.uint64(hi - lo + 1)).astype(np.int64) + lo
    out = np.tril(vals.astype(np.float64), -1)
    out[np.arange(n), np.arange(n)] = 1.0
    return out


def diag_dominant(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Dense ``n x n`` general matrix with the distribution of the triangular
    generator on both sides of the diagonal: off-diagonal ``(2u - 1) / n``
    (counter ``i n + j``), diagonal ``1 + u`` (counter ``i n + i``), positive.
    Strictly diagonally dominant, so it has a Crout factorization without
    pivoting."""
    k = np.arange(n * n, dtype=np.uint64)
    u = uniform01(seed, k).reshape(n, n)
    A = (2.0 * u - 1.0) / n
    idx = np.arange(n)
    A[idx, idx] = 1.0 + u[idx, idx]
    return A.astype(dtype)

