"""Seeded synthetic operands for recursive fast matrix multiplication.

This module is the only thing the oracle and the GPU library's callers share:
it draws random matrices and holds none of the method's arithmetic.  Every
array is a pure function of (seed, shape, kind), so the oracle regenerates
exactly what the GPU multiplied.

Distributions (the workloads described for the method's measurements):
* ``uniform``  -- i.i.d. uniform on [-1, 1)
* ``integer``  -- i.i.d. uniform on the integers {-8, ..., 8} (stored as
  floating point; products of such matrices are exact in binary64 at the
  sizes used, so every path must reproduce them bit for bit)
* ``normal_rowscaled`` -- i.i.d. normal(0, 1) with a seeded 10% of the rows
  multiplied by 1e3 (a dynamic-range stress)

Generator: numpy's PCG64 bit generator (O'Neill, 2014) seeded with
(seed, stream), where stream separates A from B and the row-scaling choice.
"""
import numpy as np

KINDS = ("uniform", "integer", "normal_rowscaled")

_STREAM_A = 1
_STREAM_B = 2
_STREAM_ROWS_A = 3
_STREAM_ROWS_B = 4


def _rng(seed, stream):
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


def matrix(seed, stream, rows, cols, kind="uniform", dtype=np.float64,
           scaled_fraction=0.1, scale=1e3):
    """One rows x cols matrix of the given kind, C-contiguous."""
    g = _rng(seed, stream)
    if kind == "uniform":
        X = g.uniform(-1.0, 1.0, size=(rows, cols))
    elif kind == "integer":
        X = g.integers(-8, 9, size=(rows, cols)).astype(np.float64)
    elif kind == "normal_rowscaled":
        X = g.standard_normal(size=(rows, cols))
        nsel = int(round(scaled_fraction * rows))
        if nsel:
            sel = _rng(seed, stream + 100).choice(rows, size=nsel, replace=False)
            X[sel, :] *= scale
    else:
        raise ValueError(f"unknown kind {kind!r}")
    return np.ascontiguousarray(X.astype(dtype, copy=False))


def operands(seed, m, k, n, kind="uniform", dtype=np.float64):
    """(A, B) with A m x k and B k x n, drawn from independent streams."""
    A = matrix(seed, _STREAM_A, m, k, kind, dtype)
    B = matrix(seed, _STREAM_B, k, n, kind, dtype)
    return A, B


def scaled_rows(seed, rows, which="A", scaled_fraction=0.1):
    """The row indices that ``normal_rowscaled`` multiplied, for reporting the
    error on scaled and unscaled rows separately."""
    stream = (_STREAM_A if which == "A" else _STREAM_B) + 100
    nsel = int(round(scaled_fraction * rows))
    if not nsel:
        return np.zeros(0, dtype=np.int64)
    return np.sort(_rng(seed, stream).choice(rows, size=nsel, replace=False))


def sample_rows(seed, m, count, must=()):
    """A seeded sorted set of distinct row indices of an m-row product, always
    containing the rows in ``must`` (e.g. block and peel boundaries)."""
    g = _rng(seed, 99)
    base = set(int(r) for r in must if 0 <= r < m)
    extra = g.choice(m, size=min(m, count), replace=False)
    for r in extra:
        if len(base) >= count:
            break
        base.add(int(r))
    return np.array(sorted(base), dtype=np.int64)
