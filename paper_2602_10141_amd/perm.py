"""Python binding of libperm (include/perm.h): argument marshalling only.

Every function has the name of the C entry point it calls.  Matrices may be
given as torch CUDA tensors (the call then passes device pointers and runs on
torch's current stream, PyTorch owning the memory) or as host numpy arrays
(the library copies them to the device).  No arithmetic of the permanent
happens here: results come back from the HIP kernels.

torch is imported before the library is loaded so that libperm binds to the
HIP runtime torch already holds (same soname) instead of loading a second one.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libperm.so")

PERM_OK, PERM_EINVAL, PERM_ERANGE, PERM_ENOMEM, PERM_EDEVICE, PERM_EAGAIN, PERM_ENOTFOUND, \
    PERM_ECANCELED = range(8)
PERM_C128, PERM_F64, PERM_MODP = 0, 1, 2
PERM_DEVICE_PTRS, PERM_NO_KAHAN, PERM_MONTGOMERY, PERM_SHARED_PARTITION = 0x1, 0x2, 0x4, 0x8
PERM_NMAX = 48
FIELDS = {"c128": PERM_C128, "f64": PERM_F64, "modp": PERM_MODP}

ITEM_DTYPE = np.dtype([("offset", "<u8"), ("n", "<i4"), ("field", "<i4"), ("p", "<u4"),
                       ("reserved", "<u4")])


class PermError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class perm_tune(ctypes.Structure):
    _fields_ = [("log2_chunk", ctypes.c_int), ("grid_per_cu", ctypes.c_int)]


class perm_srv_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_int),
                ("max_pending", ctypes.c_int), ("slice_us", ctypes.c_double),
                ("flags", ctypes.c_uint)]


class perm_srv_times(ctypes.Structure):
    _fields_ = [("queued_us", ctypes.c_double), ("admitted_us", ctypes.c_double),
                ("running_us", ctypes.c_double), ("latency_us", ctypes.c_double)]


class perm_srv_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("canceled", ctypes.c_uint64), ("slices", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("terms", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("items", ctypes.c_uint64), ("rate", ctypes.c_double)]


_lib = None
_P, _I, _U, _U64, _D, _SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_uint64,
                             ctypes.c_double, ctypes.c_size_t)
_SIGS = {
    "perm_ctx_create": ([_I, _SZ, _P], _I),
    "perm_ctx_destroy": ([_P], None),
    "perm_strerror": ([_I], ctypes.c_char_p),
    "perm_last_error": ([], ctypes.c_char_p),
    "perm_c128": ([_P, _P, _I, _P, _U, _P], _I),
    "perm_c128_noalloc": ([_P, _P, _I, _P, _U, _P], _I),
    "perm_f64": ([_P, _P, _I, _P, _U, _P], _I),
    "perm_modp": ([_P, _P, _I, ctypes.c_uint32, _P, _U, _P], _I),
    "perm_crt_int": ([_P, _P, _P, _I, _I, _D, _P, _I, _P, _P, _P, _U, _P], _I),
    "perm_batch": ([_P, _P, _I, _P, _P, _P, _U, _P], _I),
    "perm_range": ([_P, _P, _P, _U64, _U64, _P, _U, _P], _I),
    "perm_prof_enable": ([_P, _I], _I),
    "perm_prof_read": ([_P, _P, _P], _I),
    "perm_schur_primes": ([_I, _I, _P, _I, _P], _I),
    "perm_schur_residues": ([_I, ctypes.c_uint32, _P], _I),
    "perm_pick_primes": ([_I, _I, _P, _I, _P], _I),
    "perm_crt_lift": ([_P, _P, _I, _D, _P, _I, _P, _P], _I),
    "perm_crt_check": ([_P, _P, _I, _D, _P, _I, _P, _P, _P], _I),
    "perm_tune_get": ([_P, _I, _I, _P], _I),
    "perm_tune_set": ([_P, _I, _I, _P], _I),
    "perm_autotune": ([_P, _I, _I, _I, _I], _I),
    "perm_tune_save": ([_P, ctypes.c_char_p], _I),
    "perm_tune_load": ([_P, ctypes.c_char_p], _I),
    "perm_job_create": ([_P, _P, _P, _I, _I, _D, _I, ctypes.c_char_p, _P], _I),
    "perm_job_run": ([_P, _D, _P, _P], _I),
    "perm_job_result": ([_P, _P, _P, _I, _P, _P], _I),
    "perm_job_destroy": ([_P], None),
    "perm_srv_create": ([_P, _P, _P], _I),
    "perm_srv_submit": ([_P, _P, _P, _P], _I),
    "perm_srv_poll": ([_P, _U64, _P, _P, _P], _I),
    "perm_srv_wait": ([_P, _U64, _D, _P, _P, _P], _I),
    "perm_srv_wait_times": ([_P, _U64, _D, _P, _P, _P], _I),
    "perm_srv_cancel": ([_P, _U64], _I),
    "perm_srv_get_stats": ([_P, _P], _I),
    "perm_srv_destroy": ([_P], None),
}


def lib():
    """Load libperm.so (built in-tree); raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(or python paper_2602_10141_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != PERM_OK:
        raise PermError(rc, lib().perm_last_error().decode(errors="replace"))


def _is_dev(x):
    return isinstance(x, torch.Tensor) and x.is_cuda


# The current stream's raw handle without building a torch.cuda.Stream
# object (about 3 us per call, a fifth of a small permanent's call time).
_current_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(stream, device=None):
    """A hipStream_t for the library: `stream` (torch.cuda.Stream or a raw
    handle), or torch's current stream on `device` (default: the current
    device) when it is None."""
    if stream is None:
        if _current_raw_stream is not None:
            dev = torch.cuda.current_device() if device is None else device
            return ctypes.c_void_p(_current_raw_stream(dev))
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(stream)


class Context:
    """An owned perm_ctx on one device."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self.ptr = ctypes.c_void_p()
        self.device = device
        _check(lib().perm_ctx_create(device, hbm_budget, ctypes.byref(self.ptr)))

    def close(self):
        if self.ptr:
            lib().perm_ctx_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def perm_ctx_create(device: int = 0, hbm_budget: int = 0) -> Context:
    return Context(device, hbm_budget)


def perm_ctx_destroy(ctx: Context):
    ctx.close()


def perm_strerror(status: int) -> str:
    return lib().perm_strerror(status).decode()


def perm_last_error() -> str:
    return lib().perm_last_error().decode()


# ----------------------------------------------------------- single matrix
def _single(fn, ctx, A, n_out, dtype_out, extra, flags, stream):
    if _is_dev(A):
        if A.dim() != 2 or A.shape[0] != A.shape[1] or not A.is_contiguous():
            raise ValueError("expected a contiguous square CUDA tensor")
        out = torch.empty(n_out, dtype=dtype_out, device=A.device)
        _check(fn(ctx.ptr, ctypes.c_void_p(A.data_ptr()), A.shape[0], *extra,
                  ctypes.c_void_p(out.data_ptr()), flags | PERM_DEVICE_PTRS,
                  _stream(stream, A.device.index)))
        return out
    return None


def perm_c128(ctx, A, flags=0, stream=None):
    """perm(A), A complex128 n x n.  CUDA tensor -> CUDA tensor [re, im] (async);
    numpy array -> Python complex."""
    if _is_dev(A):
        if A.dtype != torch.complex128:
            raise TypeError("perm_c128 needs complex128")
        return _single(lib().perm_c128, ctx, A, 2, torch.float64, (), flags, stream)
    A = np.ascontiguousarray(A, dtype=np.complex128)
    out = np.zeros(2)
    _check(lib().perm_c128(ctx.ptr, A.ctypes.data, A.shape[0] if A.ndim == 2 else 0,
                           out.ctypes.data, flags & ~PERM_DEVICE_PTRS, None))
    return complex(out[0], out[1])


def perm_c128_noalloc(ctx, A, out=None, flags=0, stream=None):
    """perm(A) with no allocation inside the library (static device scratch).
    A: contiguous complex128 CUDA tensor, n <= 32.  out: a CUDA float64 tensor
    of 2 elements to write (re, im) into, or None for a new one; asynchronous
    on torch's current stream (or `stream`)."""
    if not _is_dev(A) or A.dtype != torch.complex128:
        raise TypeError("perm_c128_noalloc needs a complex128 CUDA tensor")
    if A.dim() != 2 or A.shape[0] != A.shape[1] or not A.is_contiguous():
        raise ValueError("expected a contiguous square CUDA tensor")
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=A.device)
    _check(lib().perm_c128_noalloc(ctx.ptr, ctypes.c_void_p(A.data_ptr()), A.shape[0],
                                   ctypes.c_void_p(out.data_ptr()), flags | PERM_DEVICE_PTRS,
                                   _stream(stream, A.device.index)))
    return out


def perm_f64(ctx, A, flags=0, stream=None):
    if _is_dev(A):
        if A.dtype != torch.float64:
            raise TypeError("perm_f64 needs float64")
        return _single(lib().perm_f64, ctx, A, 1, torch.float64, (), flags, stream)
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.zeros(1)
    _check(lib().perm_f64(ctx.ptr, A.ctypes.data, A.shape[0] if A.ndim == 2 else 0,
                          out.ctypes.data, flags & ~PERM_DEVICE_PTRS, None))
    return float(out[0])


def perm_modp(ctx, A, p: int, flags=0, stream=None):
    """perm(A) mod p.  A: uint32 residues (numpy) or an int32 CUDA tensor of
    residues below 2^31."""
    if _is_dev(A):
        if A.dtype != torch.int32:
            raise TypeError("perm_modp on the device takes int32 residues")
        return _single(lib().perm_modp, ctx, A, 1, torch.int32, (ctypes.c_uint32(p),), flags, stream)
    A = np.ascontiguousarray(A, dtype=np.uint32)
    out = np.zeros(1, dtype=np.uint32)
    _check(lib().perm_modp(ctx.ptr, A.ctypes.data, A.shape[0] if A.ndim == 2 else 0, p,
                           out.ctypes.data, flags & ~PERM_DEVICE_PTRS, None))
    return int(out[0])


# --------------------------------------------------------------------- CRT
def _limbs_to_int(limbs, nl, sign):
    v = 0
    for i in range(nl - 1, -1, -1):
        v = (v << 64) | int(limbs[i])
    return sign * v


def perm_crt_int(ctx, mats, primes, log2_bound: float, flags=0, stream=None):
    """Exact perm from k residue matrices; returns (integer, residues)."""
    primes_a = np.ascontiguousarray(primes, dtype=np.uint32)
    k = len(primes_a)
    limbs = np.zeros(64, dtype=np.uint64)
    nl, sg = ctypes.c_int(), ctypes.c_int()
    res = np.zeros(k, dtype=np.uint32)
    if _is_dev(mats):
        if mats.dtype != torch.int32 or not mats.is_contiguous():
            raise TypeError("device matrices must be a contiguous int32 tensor (k, n, n)")
        n = mats.shape[-1]
        ptr, fl = ctypes.c_void_p(mats.data_ptr()), flags | PERM_DEVICE_PTRS
        st = _stream(stream, mats.device.index)
    else:
        m = np.ascontiguousarray(mats, dtype=np.uint32)
        n = m.shape[-1]
        ptr, fl, st = m.ctypes.data, flags & ~PERM_DEVICE_PTRS, None
    _check(lib().perm_crt_int(ctx.ptr, ptr, primes_a.ctypes.data, k, n, float(log2_bound),
                              limbs.ctypes.data, len(limbs), ctypes.byref(nl), ctypes.byref(sg),
                              res.ctypes.data, fl, st))
    return _limbs_to_int(limbs, nl.value, sg.value), [int(r) for r in res]


def perm_crt_lift(residues, primes, log2_bound: float) -> int:
    r = np.ascontiguousarray(residues, dtype=np.uint32)
    p = np.ascontiguousarray(primes, dtype=np.uint32)
    limbs = np.zeros(64, dtype=np.uint64)
    nl, sg = ctypes.c_int(), ctypes.c_int()
    _check(lib().perm_crt_lift(r.ctypes.data, p.ctypes.data, len(p), float(log2_bound),
                               limbs.ctypes.data, len(limbs), ctypes.byref(nl), ctypes.byref(sg)))
    return _limbs_to_int(limbs, nl.value, sg.value)


def perm_crt_check(residues, primes, log2_bound: float):
    """Redundant-prime check: returns (integer, index of the corrupted
    residue or None); raises PermError (PERM_ERANGE) when the residues are
    inconsistent beyond one corrupted residue."""
    r = np.ascontiguousarray(residues, dtype=np.uint32)
    p = np.ascontiguousarray(primes, dtype=np.uint32)
    limbs = np.zeros(64, dtype=np.uint64)
    nl, sg, bad = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().perm_crt_check(r.ctypes.data, p.ctypes.data, len(p), float(log2_bound),
                                limbs.ctypes.data, len(limbs), ctypes.byref(nl), ctypes.byref(sg),
                                ctypes.byref(bad)))
    return _limbs_to_int(limbs, nl.value, sg.value), (None if bad.value < 0 else bad.value)


def perm_schur_primes(n: int, extra: int = 0):
    buf = np.zeros(128, dtype=np.uint32)
    k = ctypes.c_int()
    _check(lib().perm_schur_primes(n, extra, buf.ctypes.data, len(buf), ctypes.byref(k)))
    return [int(p) for p in buf[:k.value]]


def perm_pick_primes(n: int, extra: int = 0):
    buf = np.zeros(128, dtype=np.uint32)
    k = ctypes.c_int()
    _check(lib().perm_pick_primes(n, extra, buf.ctypes.data, len(buf), ctypes.byref(k)))
    return [int(p) for p in buf[:k.value]]


def perm_schur_residues(n: int, p: int) -> np.ndarray:
    out = np.zeros((n, n), dtype=np.uint32)
    _check(lib().perm_schur_residues(n, p, out.ctypes.data))
    return out


# ------------------------------------------------------------------- batch
def make_items(specs):
    """specs: list of (offset_bytes, n, field, p) -> perm_item array."""
    it = np.zeros(len(specs), dtype=ITEM_DTYPE)
    for i, (off, n, field, p) in enumerate(specs):
        it[i] = (off, n, FIELDS.get(field, field), p or 0, 0)
    return it


def pack_matrices(mats):
    """mats: list of (array, field, p).  Returns (items, data bytes as uint8
    numpy) with every matrix 16-byte aligned."""
    chunks, specs, off = [], [], 0
    for A, field, p in mats:
        f = FIELDS.get(field, field)
        dt = {PERM_C128: np.complex128, PERM_F64: np.float64, PERM_MODP: np.uint32}[f]
        a = np.ascontiguousarray(A, dtype=dt)
        b = a.tobytes()
        pad = (-len(b)) % 16
        specs.append((off, a.shape[0] if a.ndim == 2 else 0, f, p))
        chunks.append(b + b"\0" * pad)
        off += len(b) + pad
    data = np.frombuffer(b"".join(chunks) or b"\0" * 16, dtype=np.uint8).copy()
    return make_items(specs), data


def perm_batch(ctx, items, data, out=None, flags=0, stream=None):
    """Ragged batch.  data: CUDA uint8 tensor (device path, returns the CUDA
    float64 tensor `out` of shape (count, 2), async) or numpy bytes (returns a
    (count, 2) float64 numpy array; F_p residues are in the low 32 bits of
    column 0's bit pattern -- use batch_values() to decode)."""
    items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
    count = len(items)
    bad = ctypes.c_int(-1)
    if _is_dev(data):
        if out is None:
            out = torch.zeros((max(count, 1), 2), dtype=torch.float64, device=data.device)
        rc = lib().perm_batch(ctx.ptr, items.ctypes.data, count, ctypes.c_void_p(data.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()), ctypes.byref(bad),
                              flags | PERM_DEVICE_PTRS, _stream(stream, data.device.index))
    else:
        d = np.ascontiguousarray(data)
        out = np.zeros((max(count, 1), 2), dtype=np.float64)
        rc = lib().perm_batch(ctx.ptr, items.ctypes.data, count, d.ctypes.data, out.ctypes.data,
                              ctypes.byref(bad), flags & ~PERM_DEVICE_PTRS, None)
    if rc != PERM_OK:
        raise PermError(rc, f"{perm_last_error()} (item {bad.value})")
    return out


def batch_values(items, out):
    """Decode 16-byte result slots into Python complex / float / int."""
    o = out.detach().cpu().numpy() if isinstance(out, torch.Tensor) else np.asarray(out)
    o = np.ascontiguousarray(o, dtype=np.float64)
    u = o.view(np.uint32).reshape(len(o), 4)
    vals = []
    for i, it in enumerate(np.asarray(items, dtype=ITEM_DTYPE)):
        f = int(it["field"])
        if f == PERM_C128:
            vals.append(complex(o[i, 0], o[i, 1]))
        elif f == PERM_F64:
            vals.append(float(o[i, 0]))
        else:
            vals.append(int(u[i, 0]))
    return vals


def perm_range(ctx, item, data, x0: int, x1: int, flags=0):
    """Unscaled Glynn partial sum over [x0, x1) of one matrix (host data)."""
    it = np.ascontiguousarray(np.asarray(item, dtype=ITEM_DTYPE).reshape(1))
    d = np.ascontiguousarray(data)
    out = np.zeros(2, dtype=np.float64)
    _check(lib().perm_range(ctx.ptr, it.ctypes.data, d.ctypes.data, x0, x1, out.ctypes.data,
                            flags & ~PERM_DEVICE_PTRS, None))
    return batch_values(it, out.reshape(1, 2))[0]


# --------------------------------------------------------------- profiling
def perm_prof_enable(ctx, on=True):
    """on: False/0 disables; True or an int enables, with at least that many
    event pairs (256 at least) created up front."""
    _check(lib().perm_prof_enable(ctx.ptr, int(on)))


def perm_prof_read(ctx):
    """(summed walk-kernel milliseconds, launches) since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_uint64()
    _check(lib().perm_prof_read(ctx.ptr, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ------------------------------------------------------------------ tuning
def perm_tune_get(ctx, field, n):
    t = perm_tune()
    _check(lib().perm_tune_get(ctx.ptr, FIELDS.get(field, field), n, ctypes.byref(t)))
    return t.log2_chunk, t.grid_per_cu


def perm_tune_set(ctx, field, n, log2_chunk, grid_per_cu=0):
    t = perm_tune(log2_chunk, grid_per_cu)
    _check(lib().perm_tune_set(ctx.ptr, FIELDS.get(field, field), n, ctypes.byref(t)))


def perm_autotune(ctx, field, n_lo, n_hi, batch=1):
    _check(lib().perm_autotune(ctx.ptr, FIELDS.get(field, field), n_lo, n_hi, batch))


def perm_tune_save(ctx, path):
    _check(lib().perm_tune_save(ctx.ptr, str(path).encode()))


def perm_tune_load(ctx, path):
    _check(lib().perm_tune_load(ctx.ptr, str(path).encode()))


# ------------------------------------------------------- checkpointed job
class Job:
    """Exact integer permanent from k residue matrices, run in pieces whose
    partial sums go to `checkpoint` (resumed if the file exists)."""

    def __init__(self, ctx, mats, primes, log2_bound: float, piece_log2=0, checkpoint=None):
        m = np.ascontiguousarray(mats, dtype=np.uint32)
        p = np.ascontiguousarray(primes, dtype=np.uint32)
        if m.ndim != 3 or m.shape[0] != len(p) or m.shape[1] != m.shape[2]:
            raise ValueError("mats must have shape (k, n, n) with k = len(primes)")
        self.k = len(p)
        self.ptr = ctypes.c_void_p()
        path = str(checkpoint).encode() if checkpoint else None
        _check(lib().perm_job_create(ctx.ptr, m.ctypes.data, p.ctypes.data, len(p), m.shape[1],
                                     float(log2_bound), int(piece_log2), path,
                                     ctypes.byref(self.ptr)))

    def run(self, seconds=1e30):
        """Run pieces for about `seconds` (at least one batch); (done, total)."""
        d, t = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().perm_job_run(self.ptr, float(seconds), ctypes.byref(d), ctypes.byref(t)))
        return d.value, t.value

    def result(self):
        """(integer, residues); PermError(PERM_EAGAIN) while pieces remain."""
        limbs = np.zeros(64, dtype=np.uint64)
        nl, sg = ctypes.c_int(), ctypes.c_int()
        res = np.zeros(self.k, dtype=np.uint32)
        _check(lib().perm_job_result(self.ptr, res.ctypes.data, limbs.ctypes.data, len(limbs),
                                     ctypes.byref(nl), ctypes.byref(sg)))
        return _limbs_to_int(limbs, nl.value, sg.value), [int(r) for r in res]

    def close(self):
        if self.ptr:
            lib().perm_job_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ----------------------------------------------------------------- serving
class Server:
    """Owned perm_srv: submit host matrices, poll or wait for results."""

    def __init__(self, ctx, hbm_budget=0, max_inflight=0, max_pending=0, slice_us=0.0, flags=0):
        self.ctx = ctx
        self.ptr = ctypes.c_void_p()
        cfg = perm_srv_cfg(hbm_budget, max_inflight, max_pending, slice_us, flags)
        _check(lib().perm_srv_create(ctx.ptr, ctypes.byref(cfg), ctypes.byref(self.ptr)))

    def submit(self, A, field, p=0):
        f = FIELDS.get(field, field)
        dt = {PERM_C128: np.complex128, PERM_F64: np.float64, PERM_MODP: np.uint32}[f]
        a = np.ascontiguousarray(A, dtype=dt)
        it = make_items([(0, a.shape[0] if a.ndim == 2 else 0, f, p)])
        t = ctypes.c_uint64()
        _check(lib().perm_srv_submit(self.ptr, it.ctypes.data, a.ctypes.data, ctypes.byref(t)))
        return t.value, it

    def _decode(self, it, buf):
        return batch_values(it, np.frombuffer(buf, dtype=np.float64).reshape(1, 2))[0]

    def poll(self, ticket, it):
        buf = ctypes.create_string_buffer(16)
        done = ctypes.c_int()
        rc = lib().perm_srv_poll(self.ptr, ticket, buf, ctypes.byref(done), None)
        if rc != PERM_OK:
            raise PermError(rc, perm_last_error() if rc != PERM_ECANCELED else "cancelled")
        return (True, self._decode(it, buf.raw)) if done.value else (False, None)

    def wait(self, ticket, it, timeout_s=60.0, with_latency=False, with_times=False):
        """Result of a ticket; with_latency: (result, submit-to-result us);
        with_times: (result, dict of the latency's phases in us, as
        perm_srv_wait_times reports them)."""
        buf = ctypes.create_string_buffer(16)
        done = ctypes.c_int()
        lat = ctypes.c_double()
        tm = perm_srv_times()
        if with_times:
            rc = lib().perm_srv_wait_times(self.ptr, ticket, float(timeout_s), buf,
                                           ctypes.byref(done), ctypes.byref(tm))
        else:
            rc = lib().perm_srv_wait(self.ptr, ticket, float(timeout_s), buf, ctypes.byref(done),
                                     ctypes.byref(lat))
        if rc != PERM_OK:
            raise PermError(rc, perm_last_error() if rc != PERM_ECANCELED else "cancelled")
        if not done.value:
            raise TimeoutError(f"ticket {ticket} not done after {timeout_s} s")
        v = self._decode(it, buf.raw)
        if with_times:
            return v, {k: getattr(tm, k) for k, _ in perm_srv_times._fields_}
        return (v, lat.value) if with_latency else v

    def cancel(self, ticket):
        _check(lib().perm_srv_cancel(self.ptr, ticket))

    def stats(self):
        s = perm_srv_stats()
        _check(lib().perm_srv_get_stats(self.ptr, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in perm_srv_stats._fields_}

    def close(self):
        if self.ptr:
            lib().perm_srv_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
