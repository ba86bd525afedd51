"""ctypes front end of the oracle's C Ryser (``ryser.c``).  Test infrastructure only.

Every function takes a numpy array holding one n x n matrix in row-major
order (complex128, float64 or uint32 residues) and returns a Python scalar.
The library is built on first use if it is missing.
"""
import concurrent.futures as cf
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        dp, u32p, u64 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64
        c_int, c_u32 = ctypes.c_int, ctypes.c_uint32
        for name, args in [
            ("oracle_ryser_c128", [dp, c_int, c_int, dp]),
            ("oracle_ryser_c128_ld", [dp, c_int, dp]),
            ("oracle_ryser_f64", [dp, c_int, c_int, dp]),
            ("oracle_ryser_modp", [u32p, c_int, c_u32, u32p]),
            ("oracle_ryser_modp_prefix", [u32p, c_int, c_u32, u64, u32p]),
            ("oracle_ryser_modp_range", [u32p, c_int, c_u32, u64, u64, u32p]),
            ("oracle_ryser_c128_range", [dp, c_int, u64, u64, dp]),
            ("oracle_ryser_f64_range", [dp, c_int, u64, u64, dp]),
            ("oracle_glynn_range_c128", [dp, c_int, u64, u64, dp]),
            ("oracle_glynn_range_f64", [dp, c_int, u64, u64, dp]),
            ("oracle_glynn_range_modp", [u32p, c_int, c_u32, u64, u64, u32p]),
            ("oracle_ryser_c128_many", [dp, c_int, c_int, c_int, dp]),
            ("oracle_ryser_f64_many", [dp, c_int, c_int, c_int, dp]),
        ]:
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c_int
        _lib = L
    return _lib


def _mat(A, dtype):
    A = np.ascontiguousarray(A, dtype=dtype)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square matrix")
    return A, A.shape[0]


def _check(rc):
    if rc != 0:
        raise ValueError("oracle rejected its arguments")


def ryser_c128(A, kahan=True) -> complex:
    """perm(A) for complex A by Ryser's formula in double precision."""
    A, n = _mat(A, np.complex128)
    out = np.zeros(2)
    _check(lib().oracle_ryser_c128(A.ctypes.data, n, int(bool(kahan)), out.ctypes.data))
    return complex(out[0], out[1])


def ryser_c128_longdouble(A) -> complex:
    """The same walk as ``ryser_c128`` carried out in long double."""
    A, n = _mat(A, np.complex128)
    out = np.zeros(2)
    _check(lib().oracle_ryser_c128_ld(A.ctypes.data, n, out.ctypes.data))
    return complex(out[0], out[1])


def ryser_f64(A, kahan=True) -> float:
    """perm(A) for real A by Ryser's formula in double precision."""
    A, n = _mat(A, np.float64)
    out = np.zeros(1)
    _check(lib().oracle_ryser_f64(A.ctypes.data, n, int(bool(kahan)), out.ctypes.data))
    return float(out[0])


def ryser_modp(A, p: int) -> int:
    """perm(A) mod p for residues A in [0, p)."""
    A, n = _mat(A, np.uint32)
    out = np.zeros(1, dtype=np.uint32)
    _check(lib().oracle_ryser_modp(A.ctypes.data, n, int(p), out.ctypes.data))
    return int(out[0])


def ryser_modp_prefix(A, p: int, x_end: int) -> int:
    """Signed Ryser sum mod p over the first x_end - 1 Gray-ordered subsets."""
    A, n = _mat(A, np.uint32)
    out = np.zeros(1, dtype=np.uint32)
    _check(lib().oracle_ryser_modp_prefix(A.ctypes.data, n, int(p), x_end, out.ctypes.data))
    return int(out[0])


def ryser_modp_range(A, p: int, x0: int, x1: int) -> int:
    """Signed Ryser sum mod p over the Gray-ordered subsets x in [x0, x1),
    1 <= x0 <= x1 <= 2^n, without the final (-1)^n."""
    A, n = _mat(A, np.uint32)
    out = np.zeros(1, dtype=np.uint32)
    _check(lib().oracle_ryser_modp_range(A.ctypes.data, n, int(p), x0, x1, out.ctypes.data))
    return int(out[0])


def _spans(x0, x1, parts):
    """[x0, x1) cut into at most `parts` contiguous pieces."""
    parts = max(1, min(parts, x1 - x0))
    cuts = [x0 + (x1 - x0) * i // parts for i in range(parts + 1)]
    return [(a, b) for a, b in zip(cuts, cuts[1:]) if a < b]


def default_threads() -> int:
    return min(16, os.cpu_count() or 1)


def ryser_modp_threaded(A, p: int, threads: int = None) -> int:
    """perm(A) mod p by Ryser's formula, the subset range [1, 2^n) split into
    contiguous pieces summed on host threads (the C calls release the GIL)."""
    A, n = _mat(A, np.uint32)
    if n == 0:
        return 1 % p
    threads = threads or default_threads()
    with cf.ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda s: ryser_modp_range(A, p, *s), _spans(1, 1 << n, 4 * threads)))
    tot = sum(parts) % p
    return (p - tot) % p if n % 2 else tot


def ryser_float_range(A, x0: int, x1: int):
    """Signed Ryser sum (complex128 or float64 walk, Kahan-summed) over the
    Gray-ordered subsets x in [x0, x1), 1 <= x0 <= x1 <= 2^n, without the
    final (-1)^n."""
    if np.iscomplexobj(A):
        A, n = _mat(A, np.complex128)
        out = np.zeros(2)
        _check(lib().oracle_ryser_c128_range(A.ctypes.data, n, x0, x1, out.ctypes.data))
        return complex(out[0], out[1])
    A, n = _mat(A, np.float64)
    out = np.zeros(1)
    _check(lib().oracle_ryser_f64_range(A.ctypes.data, n, x0, x1, out.ctypes.data))
    return float(out[0])


def ryser_float_threaded(A, threads: int = None):
    """perm(A) for a complex128 or float64 matrix by Ryser's formula, the
    subset range [1, 2^n) split into contiguous pieces on host threads; the
    pieces' sums are added with math.fsum per component."""
    import math
    cplx = np.iscomplexobj(A)
    A = np.ascontiguousarray(A, dtype=np.complex128 if cplx else np.float64)
    n = A.shape[0]
    if n == 0:
        return 1.0
    threads = threads or default_threads()
    with cf.ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda s: ryser_float_range(A, *s), _spans(1, 1 << n, 4 * threads)))
    sign = -1.0 if n % 2 else 1.0
    if cplx:
        return sign * complex(math.fsum(z.real for z in parts), math.fsum(z.imag for z in parts))
    return sign * math.fsum(parts)


def glynn_range_threaded(A, x0: int, x1: int, field: str, p: int = 0, threads: int = None):
    """glynn_range_{c128,f64,modp} over [x0, x1) split into pieces on host
    threads; the pieces' sums are added (mod p for F_p)."""
    threads = threads or default_threads()
    fn = {"c128": lambda s: glynn_range_c128(A, *s), "f64": lambda s: glynn_range_f64(A, *s),
          "modp": lambda s: glynn_range_modp(A, p, *s)}[field]
    with cf.ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(fn, _spans(x0, x1, 4 * threads)))
    if field == "modp":
        return sum(parts) % p
    return sum(parts) if parts else 0.0


def glynn_range_c128(A, x0: int, x1: int) -> complex:
    """sum_{x in [x0,x1)} (-1)^x prod_i r_i(x), each term evaluated from scratch."""
    A, n = _mat(A, np.complex128)
    out = np.zeros(2)
    _check(lib().oracle_glynn_range_c128(A.ctypes.data, n, x0, x1, out.ctypes.data))
    return complex(out[0], out[1])


def glynn_range_f64(A, x0: int, x1: int) -> float:
    A, n = _mat(A, np.float64)
    out = np.zeros(1)
    _check(lib().oracle_glynn_range_f64(A.ctypes.data, n, x0, x1, out.ctypes.data))
    return float(out[0])


def glynn_range_modp(A, p: int, x0: int, x1: int) -> int:
    A, n = _mat(A, np.uint32)
    out = np.zeros(1, dtype=np.uint32)
    _check(lib().oracle_glynn_range_modp(A.ctypes.data, n, int(p), x0, x1, out.ctypes.data))
    return int(out[0])


def ryser_many(mats, kahan=True):
    """perm of each matrix of a (count, n, n) stack; complex128 or float64."""
    mats = np.ascontiguousarray(mats)
    count, n = mats.shape[0], mats.shape[1]
    if mats.dtype == np.complex128:
        out = np.zeros((count, 2))
        _check(lib().oracle_ryser_c128_many(mats.ctypes.data, n, count, int(bool(kahan)),
                                            out.ctypes.data))
        return out[:, 0] + 1j * out[:, 1]
    mats = mats.astype(np.float64, copy=False)
    out = np.zeros(count)
    _check(lib().oracle_ryser_f64_many(mats.ctypes.data, n, count, int(bool(kahan)),
                                       out.ctypes.data))
    return out
