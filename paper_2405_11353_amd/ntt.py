"""ctypes binding of libntt.so with the C ABI's names (include/ntt.h).

Argument marshalling only: every step of a transform runs in the HIP
kernels. Device buffers are passed as torch tensors (or raw device pointers)
and streams as torch streams (or raw hipStream_t handles). If the library
is not built this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(PKG, "libntt.so")

NTT_WORD32 = 0x1
NTT_ORDER_BITREV = 0x2
NTT_CYCLIC = 0x4
NTT_DEBUG_CHECK = 0x8
NTT_ROW_TWIST_FWD, NTT_ROW_TWIST_INV = 0x1, 0x2
NTT_ROW_TWIST_DEFAULT = NTT_ROW_TWIST_FWD | NTT_ROW_TWIST_INV
NTT_PATH_AUTO, NTT_PATH_TINY, NTT_PATH_LDS, NTT_PATH_FOURSTEP = 0, 1, 2, 3
NTT_PATH_PAPER_DIT, NTT_PATH_PAPER_DIF, NTT_PATH_PAPER_PEASE, NTT_PATH_PAPER_PEASE_NC, NTT_PATH_PAPER_STOCKHAM = \
    4, 5, 6, 7, 8

_lib = None

NTT_JOB_FORWARD, NTT_JOB_INVERSE = 0, 1
NTT_BATCH_NO_GRAPH = 0x1
NTT_BATCH_BRANCHES = 0x2
NTT_BATCH_SERIAL = 0x4


class JobDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("L", ctypes.c_uint32), ("op", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("moduli", ctypes.POINTER(ctypes.c_uint64)),
                ("d_data", ctypes.c_void_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("items", ctypes.c_uint32), ("buckets", ctypes.c_uint32), ("kernels", ctypes.c_uint32),
                ("uses_graph", ctypes.c_uint32), ("scratch_bytes", ctypes.c_uint64),
                ("twiddle_pool_bytes", ctypes.c_uint64)]


NTT_REQ_NTT, NTT_REQ_INTT, NTT_REQ_POLYMUL = 0, 1, 2
NTT_SERVER_SIMULATE = 0x1
# status codes (include/ntt.h)
NTT_OK = 0
NTT_ERR_ARG = -1
NTT_ERR_N = -2
NTT_ERR_MODULUS = -3
NTT_ERR_NOMEM = -4
NTT_ERR_HIP = -5
NTT_ERR_BUDGET = -6
NTT_ERR_UNSUPPORTED = -7
NTT_ERR_STATE = -8
NTT_ERR_TIMEOUT = -9
NTT_ERR_SCRATCH = -10
NTT_ERR_RANGE = -11
NTT_NOALLOC_SCRATCH_BYTES = 64 << 20


class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("N", ctypes.c_uint32), ("L", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("moduli", ctypes.POINTER(ctypes.c_uint64)),
                ("d_a", ctypes.c_void_p), ("d_b", ctypes.c_void_p), ("d_out", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("n_streams", ctypes.c_uint32),
                ("max_batch_items", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("simulate_ns_per_item", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("queued", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("items", ctypes.c_uint64), ("ntts", ctypes.c_uint64), ("admission_stalls", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("max_inflight_batches", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("table_bytes", ctypes.c_uint64), ("table_uploads", ctypes.c_uint64),
                ("table_evictions", ctypes.c_uint64)]


class TuneChoice(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("log_n1", ctypes.c_int32), ("exact", ctypes.c_int32),
                ("us_per_call", ctypes.c_float), ("row_twist", ctypes.c_int32), ("lv_col", ctypes.c_int32),
                ("col_tile", ctypes.c_int32)]


class NttError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = ntt_strerror(code) if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


def library_path() -> str:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """Load libntt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(_LIB_PATH)
        vp, u32, u64p, i32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int, ctypes.c_size_t
        sig = {
            "ntt_plan_create": (vp, [u32, u64p, u32]),
            "ntt_plan_create_ex": (vp, [u32, u64p, u32, u32, u64p]),
            "ntt_plan_destroy": (None, [vp]),
            "ntt_forward": (i32, [vp, vp, u32, vp]),
            "ntt_forward_noalloc": (i32, [vp, vp, u32, vp]),
            "ntt_inverse": (i32, [vp, vp, u32, vp]),
            "ntt_pointwise_mul": (i32, [vp, vp, vp, vp, u32, vp]),
            "ntt_pointwise_mul_inverse": (i32, [vp, vp, vp, vp, u32, vp]),
            "ntt_tensor_product": (i32, [vp, vp, vp, vp, u32, vp]),
            "ntt_polymul": (i32, [vp, vp, vp, vp, u32, vp]),
            "ntt_bconv_create": (vp, [u32, u64p, u32, u64p, u32]),
            "ntt_bconv_destroy": (None, [vp]),
            "ntt_bconv_get_info": (i32, [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]),
            "ntt_base_conv": (i32, [vp, vp, vp, u32, vp]),
            "ntt_mod_down": (i32, [vp, vp, vp, vp, u32, vp]),
            "ntt_pointwise_mul_inverse_stage": (i32, [vp, vp, vp, vp, u32, i32, vp]),
            "ntt_forward_stage": (i32, [vp, vp, u32, i32, vp]),
            "ntt_inverse_stage": (i32, [vp, vp, u32, i32, vp]),
            "ntt_plan_get_psi": (i32, [vp, u64p]),
            "ntt_plan_get_variant": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "ntt_plan_set_variant": (i32, [vp, i32, i32]),
            "ntt_plan_set_quotient": (i32, [vp, i32]),
            "ntt_plan_set_row_twist": (i32, [vp, i32]),
            "ntt_workspace_bytes": (sz, [vp, u32]),
            "ntt_last_error": (i32, []),
            "ntt_set_last_error": (None, [i32]),
            "ntt_plan_get_variant_for": (i32, [vp, u32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "ntt_plan_get_row_form": (i32, [vp, u32, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "ntt_plan_get_col_tile": (i32, [vp, u32, ctypes.POINTER(i32)]),
            "ntt_autotune": (i32, [u32, u32, u32, u32, ctypes.POINTER(TuneChoice)]),
            "ntt_tune_save": (i32, [ctypes.c_char_p]),
            "ntt_tune_load": (i32, [ctypes.c_char_p]),
            "ntt_tune_clear": (i32, []),
            "ntt_batch_create": (vp, [ctypes.POINTER(JobDesc), u32, u32]),
            "ntt_batch_run": (i32, [vp, vp]),
            "ntt_batch_get_info": (i32, [vp, ctypes.POINTER(BatchInfo)]),
            "ntt_batch_destroy": (None, [vp]),
            "ntt_server_create": (vp, [ctypes.POINTER(ServerConfig)]),
            "ntt_server_submit": (i32, [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
            "ntt_server_wait": (i32, [vp, ctypes.c_uint64, ctypes.c_int64]),
            "ntt_server_get_stats": (i32, [vp, ctypes.POINTER(ServerStats)]),
            "ntt_server_reset_stats": (i32, [vp]),
            "ntt_server_destroy": (None, [vp]),
            "ntt_strerror": (ctypes.c_char_p, [i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def ntt_strerror(code: int) -> str:
    return lib().ntt_strerror(code).decode()


def ntt_last_error() -> int:
    return lib().ntt_last_error()


def _u64_array(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_uint64 * len(vals))(*vals)


def _ptr(x) -> int:
    """Device pointer of a tensor (or an int address)."""
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError(f"expected a tensor or a device address, got {type(x)}")


def _stream(s) -> int | None:
    if s is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:  # pragma: no cover
            pass
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(rc: int, what: str):
    if rc != NTT_OK:
        raise NttError(rc, what)


# ---- C ABI names ----------------------------------------------------------------
def ntt_plan_create(N: int, moduli, L: int | None = None) -> int:
    L = len(moduli) if L is None else L
    h = lib().ntt_plan_create(N, _u64_array(moduli), L)
    if not h:
        raise NttError(ntt_last_error(), "ntt_plan_create")
    return h


def ntt_plan_create_ex(N: int, moduli, L: int | None = None, flags: int = 0, psi=None) -> int:
    L = len(moduli) if L is None else L
    h = lib().ntt_plan_create_ex(N, _u64_array(moduli), L, flags, _u64_array(psi) if psi is not None else None)
    if not h:
        raise NttError(ntt_last_error(), "ntt_plan_create_ex")
    return h


def ntt_plan_destroy(plan: int) -> None:
    lib().ntt_plan_destroy(plan)


def ntt_forward(plan: int, data, batch: int, stream=None) -> None:
    _check(lib().ntt_forward(plan, _ptr(data), batch, _stream(stream)), "ntt_forward")


def ntt_inverse(plan: int, data, batch: int, stream=None) -> None:
    _check(lib().ntt_inverse(plan, _ptr(data), batch, _stream(stream)), "ntt_inverse")


def ntt_forward_stage(plan: int, data, batch: int, stage: int, stream=None) -> None:
    _check(lib().ntt_forward_stage(plan, _ptr(data), batch, stage, _stream(stream)), "ntt_forward_stage")


def ntt_inverse_stage(plan: int, data, batch: int, stage: int, stream=None) -> None:
    _check(lib().ntt_inverse_stage(plan, _ptr(data), batch, stage, _stream(stream)), "ntt_inverse_stage")


def ntt_pointwise_mul(plan: int, a, b, c, batch: int, stream=None) -> None:
    _check(lib().ntt_pointwise_mul(plan, _ptr(a), _ptr(b), _ptr(c), batch, _stream(stream)), "ntt_pointwise_mul")


def ntt_pointwise_mul_inverse(plan: int, a, b, c, batch: int, stream=None) -> None:
    _check(lib().ntt_pointwise_mul_inverse(plan, _ptr(a), _ptr(b), _ptr(c), batch, _stream(stream)),
           "ntt_pointwise_mul_inverse")


def ntt_pointwise_mul_inverse_stage(plan: int, a, b, c, batch: int, stage: int, stream=None) -> None:
    _check(lib().ntt_pointwise_mul_inverse_stage(plan, _ptr(a), _ptr(b), _ptr(c), batch, stage, _stream(stream)),
           "ntt_pointwise_mul_inverse_stage")


def ntt_polymul(plan: int, a, b, c, batch: int, stream=None) -> None:
    _check(lib().ntt_polymul(plan, _ptr(a), _ptr(b), _ptr(c), batch, _stream(stream)), "ntt_polymul")


def ntt_tensor_product(plan: int, a, b, d, batch: int, stream=None) -> None:
    _check(lib().ntt_tensor_product(plan, _ptr(a), _ptr(b), _ptr(d), batch, _stream(stream)), "ntt_tensor_product")


def ntt_bconv_create(N: int, src, dst) -> int:
    h = lib().ntt_bconv_create(N, _u64_array(src), len(src), _u64_array(dst), len(dst))
    if not h:
        raise NttError(ntt_last_error(), "ntt_bconv_create")
    return h


def ntt_bconv_destroy(conv: int) -> None:
    lib().ntt_bconv_destroy(conv)


def ntt_base_conv(conv: int, x, out, batch: int, stream=None) -> None:
    _check(lib().ntt_base_conv(conv, _ptr(x), _ptr(out), batch, _stream(stream)), "ntt_base_conv")


def ntt_mod_down(conv: int, x, y, out, batch: int, stream=None) -> None:
    _check(lib().ntt_mod_down(conv, _ptr(x), _ptr(y), _ptr(out), batch, _stream(stream)), "ntt_mod_down")


def ntt_plan_get_psi(plan: int, L: int) -> list[int]:
    out = (ctypes.c_uint64 * L)()
    _check(lib().ntt_plan_get_psi(plan, out), "ntt_plan_get_psi")
    return [int(v) for v in out]


def ntt_plan_get_variant(plan: int) -> tuple[int, int]:
    p, n1 = ctypes.c_int(), ctypes.c_int()
    _check(lib().ntt_plan_get_variant(plan, ctypes.byref(p), ctypes.byref(n1)), "ntt_plan_get_variant")
    return p.value, n1.value


def ntt_plan_set_variant(plan: int, path: int, log_n1: int = 0) -> None:
    _check(lib().ntt_plan_set_variant(plan, path, log_n1), "ntt_plan_set_variant")


def ntt_plan_set_quotient(plan: int, exact: bool) -> None:
    _check(lib().ntt_plan_set_quotient(plan, 1 if exact else 0), "ntt_plan_set_quotient")


def ntt_plan_set_row_twist(plan: int, mask: int) -> None:
    _check(lib().ntt_plan_set_row_twist(plan, int(mask)), "ntt_plan_set_row_twist")


def ntt_workspace_bytes(plan: int, batch: int) -> int:
    return int(lib().ntt_workspace_bytes(plan, batch))


def ntt_plan_get_variant_for(plan: int, batch: int) -> tuple[int, int, int]:
    p, n1, ex = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().ntt_plan_get_variant_for(plan, batch, ctypes.byref(p), ctypes.byref(n1), ctypes.byref(ex)),
           "ntt_plan_get_variant_for")
    return p.value, n1.value, ex.value


def ntt_plan_get_row_form(plan: int, batch: int) -> tuple[int, int]:
    """(row-twist mask, log2 values per thread of the column passes) a call runs with."""
    tw, lv = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().ntt_plan_get_row_form(plan, batch, ctypes.byref(tw), ctypes.byref(lv)), "ntt_plan_get_row_form")
    return tw.value, lv.value


def ntt_plan_get_col_tile(plan: int, batch: int) -> int:
    """Columns per tile of the four-step column passes a call on `batch`
    polynomials runs with (0 off the four-step path)."""
    c = ctypes.c_int32()
    _check(lib().ntt_plan_get_col_tile(plan, batch, ctypes.byref(c)), "ntt_plan_get_col_tile")
    return c.value


def ntt_autotune(N: int, items: int, reps: int = 20, flags: int = 0) -> dict:
    out = TuneChoice()
    _check(lib().ntt_autotune(N, flags, items, reps, ctypes.byref(out)), "ntt_autotune")
    return {"path": out.path, "log_n1": out.log_n1, "exact": out.exact, "us_per_call": out.us_per_call,
            "row_twist": out.row_twist, "lv_col": out.lv_col, "col_tile": out.col_tile}


def ntt_tune_save(path: str) -> None:
    _check(lib().ntt_tune_save(path.encode()), "ntt_tune_save")


def ntt_tune_load(path: str) -> None:
    _check(lib().ntt_tune_load(path.encode()), "ntt_tune_load")


def ntt_tune_clear() -> None:
    _check(lib().ntt_tune_clear(), "ntt_tune_clear")


class Batch:
    """ntt_batch_create / run / destroy over a list of jobs.

    jobs: iterable of (N, moduli, op, tensor) with tensor holding [L][N] 64-bit words
    on the GPU. The tensors must outlive the batch (the captured graph holds their
    addresses); the Batch keeps references to them.
    """

    def __init__(self, jobs, flags: int = 0):
        jobs = list(jobs)
        self._keep = []
        arr = (JobDesc * len(jobs))()
        for i, (N, moduli, op, t) in enumerate(jobs):
            mods = _u64_array(moduli)
            self._keep.append((mods, t))
            if t.element_size() != 8 or not t.is_cuda or t.numel() < len(moduli) * N:
                raise ValueError("job tensor must hold [L][N] 64-bit words on the GPU")
            arr[i] = JobDesc(N, len(moduli), op, 0, mods, _ptr(t))
        self.handle = lib().ntt_batch_create(arr, len(jobs), flags)
        if not self.handle:
            raise NttError(ntt_last_error(), "ntt_batch_create")

    def run(self, stream=None):
        _check(lib().ntt_batch_run(self.handle, _stream(stream)), "ntt_batch_run")

    @property
    def info(self) -> dict:
        i = BatchInfo()
        _check(lib().ntt_batch_get_info(self.handle, ctypes.byref(i)), "ntt_batch_get_info")
        return {k: getattr(i, k) for k, _ in BatchInfo._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().ntt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """ntt_server_* wrapper. submit() takes device tensors (or int addresses)."""

    def __init__(self, hbm_budget_bytes=4 << 30, n_streams=4, max_batch_items=2048, flags=0,
                 simulate_ns_per_item=0.0):
        self.simulate = bool(flags & NTT_SERVER_SIMULATE)
        cfg = ServerConfig(hbm_budget_bytes, n_streams, max_batch_items, flags, 0, simulate_ns_per_item)
        self.handle = lib().ntt_server_create(ctypes.byref(cfg))
        if not self.handle:
            raise NttError(ntt_last_error(), "ntt_server_create")
        self._keep = {}

    def _check_buffers(self, op, N, moduli, a, out, b):
        """Each buffer must be a contiguous GPU tensor of 64-bit words holding
        at least L*N of them (b only for products): the kernels index L*N
        words of each, so anything smaller is refused before the C call. A
        simulating server never touches its buffers and takes anything (the
        C call still checks what it can)."""
        if self.simulate:
            return
        need = len(moduli) * int(N)
        named = [("a", a), ("out", out)] + ([("b", b)] if op == NTT_REQ_POLYMUL or b is not None else [])
        for name, t in named:
            if t is None or not hasattr(t, "data_ptr"):
                raise ValueError(f"{name} must be a GPU tensor of 64-bit words")
            if not t.is_cuda or t.element_size() != 8:
                raise ValueError(f"{name} must hold 64-bit words on the GPU")
            if t.numel() < need:
                raise ValueError(f"{name} holds {t.numel()} words, the request needs L*N = {need}")

    def submit(self, op, N, moduli, a, out, b=None) -> int:
        self._check_buffers(op, N, moduli, a, out, b)
        mods = _u64_array(moduli)
        req = Request(op, N, len(moduli), 0, mods, _ptr(a), _ptr(b) if b is not None else None, _ptr(out))
        t = ctypes.c_uint64()
        _check(lib().ntt_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)), "ntt_server_submit")
        self._keep[t.value] = (mods, a, b, out)
        return t.value

    def make_request(self, op, N, moduli, a, out, b=None):
        """A prepared request (ctypes struct) for submit_request: builds the
        moduli array and resolves the device pointers once."""
        self._check_buffers(op, N, moduli, a, out, b)
        mods = _u64_array(moduli)
        req = Request(op, N, len(moduli), 0, mods, _ptr(a), _ptr(b) if b is not None else None, _ptr(out))
        return (req, mods, a, b, out)

    def submit_request(self, prepared) -> int:
        t = ctypes.c_uint64()
        _check(lib().ntt_server_submit(self.handle, ctypes.byref(prepared[0]), ctypes.byref(t)), "ntt_server_submit")
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> int:
        """Returns NTT_OK or an error code (NTT_ERR_TIMEOUT if still pending)."""
        rc = lib().ntt_server_wait(self.handle, ticket, timeout_us)
        if rc != NTT_ERR_TIMEOUT:
            self._keep.pop(ticket, None)
        return rc

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().ntt_server_get_stats(self.handle, ctypes.byref(st)), "ntt_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_ if k != "reserved"}

    def reset_stats(self):
        _check(lib().ntt_server_reset_stats(self.handle), "ntt_server_reset_stats")

    def close(self):
        if getattr(self, "handle", None):
            lib().ntt_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class BaseConv:
    """Owns an ntt_bconv*: fast RNS basis conversion from `src` primes to
    `dst` primes (and ModDown, the division by prod(src)), 64-bit words."""

    def __init__(self, N: int, src, dst):
        self.N = int(N)
        self.src = [int(q) for q in src]
        self.dst = [int(q) for q in dst]
        self.L, self.K = len(self.src), len(self.dst)
        self.handle = ntt_bconv_create(self.N, self.src, self.dst)

    def close(self):
        if getattr(self, "handle", None):
            ntt_bconv_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _batch(self, t, limbs, batch):
        per = limbs * self.N
        if batch is None:
            if t.numel() % per:
                raise ValueError("tensor size is not a multiple of limbs*N")
            batch = t.numel() // per
        if not t.is_cuda or t.element_size() != 8 or t.numel() < per * batch:
            raise ValueError("tensor shape/dtype/device mismatch")
        return batch

    def convert(self, x, out, batch=None, stream=None):
        """out [batch][K][N] = conv(x [batch][L][N])."""
        batch = self._batch(x, self.L, batch)
        self._batch(out, self.K, batch)
        ntt_base_conv(self.handle, x, out, batch, stream)
        return out

    def mod_down(self, x, y, out=None, batch=None, stream=None):
        """out [batch][K][N] = (y - conv(x)) * prod(src)^-1; out defaults to y."""
        out = y if out is None else out
        batch = self._batch(x, self.L, batch)
        self._batch(y, self.K, batch)
        self._batch(out, self.K, batch)
        ntt_mod_down(self.handle, x, y, out, batch, stream)
        return out


# ---- convenience object ------------------------------------------------------
class Plan:
    """Owns an ntt_plan*; methods check tensor shape/dtype/device, then call the C ABI."""

    def __init__(self, N: int, moduli, flags: int = 0, psi=None):
        self.N = int(N)
        self.moduli = [int(q) for q in moduli]
        self.L = len(self.moduli)
        self.flags = flags
        self.word = 32 if flags & NTT_WORD32 else 64
        self.handle = ntt_plan_create_ex(self.N, self.moduli, self.L, flags, psi)

    def close(self):
        if getattr(self, "handle", None):
            ntt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def psi(self) -> list[int]:
        return ntt_plan_get_psi(self.handle, self.L)

    @property
    def variant(self) -> tuple[int, int]:
        return ntt_plan_get_variant(self.handle)

    def set_variant(self, path: int, log_n1: int = 0):
        ntt_plan_set_variant(self.handle, path, log_n1)

    def set_exact_quotient(self, exact: bool):
        ntt_plan_set_quotient(self.handle, exact)

    def set_row_twist(self, mask):
        """Directions whose four-step row pass is twisted: a mask of
        NTT_ROW_TWIST_FWD / NTT_ROW_TWIST_INV (True: both, False: neither)."""
        if mask is True:
            mask = NTT_ROW_TWIST_FWD | NTT_ROW_TWIST_INV
        elif mask is False:
            mask = 0
        ntt_plan_set_row_twist(self.handle, mask)

    def _batch(self, t, batch):
        if batch is None:
            n = t.numel()
            if n % (self.L * self.N):
                raise ValueError("tensor size is not a multiple of L*N")
            batch = n // (self.L * self.N)
        if not t.is_cuda:
            raise ValueError("tensor must be on the GPU")
        if t.element_size() * 8 != self.word:
            raise ValueError(f"tensor words must be {self.word}-bit")
        if t.numel() < batch * self.L * self.N:
            raise ValueError("tensor smaller than batch*L*N")
        return batch

    def forward(self, t, batch=None, stream=None):
        ntt_forward(self.handle, t, self._batch(t, batch), stream)
        return t

    def inverse(self, t, batch=None, stream=None):
        ntt_inverse(self.handle, t, self._batch(t, batch), stream)
        return t

    def forward_stage(self, t, stage: int, batch=None, stream=None):
        ntt_forward_stage(self.handle, t, self._batch(t, batch), stage, stream)
        return t

    def inverse_stage(self, t, stage: int, batch=None, stream=None):
        ntt_inverse_stage(self.handle, t, self._batch(t, batch), stage, stream)
        return t

    def pointwise(self, a, b, out=None, batch=None, stream=None):
        out = a if out is None else out
        bt = self._batch(a, batch)
        self._batch(b, bt)
        self._batch(out, bt)
        ntt_pointwise_mul(self.handle, a, b, out, bt, stream)
        return out

    def pointwise_inverse(self, a, b, out=None, batch=None, stream=None):
        """out = inverse(a * b); out defaults to a."""
        out = a if out is None else out
        bt = self._batch(a, batch)
        self._batch(b, bt)
        self._batch(out, bt)
        ntt_pointwise_mul_inverse(self.handle, a, b, out, bt, stream)
        return out

    def pointwise_inverse_stage(self, a, b, out, stage: int, batch=None, stream=None):
        bt = self._batch(a, batch)
        ntt_pointwise_mul_inverse_stage(self.handle, a, b, out, bt, stage, stream)
        return out

    def polymul(self, a, b, out, batch=None, stream=None):
        """out = a * b (negacyclic, or cyclic for NTT_CYCLIC plans) for batch
        pairs of [L][N] coefficient-domain polynomials; a and b are kept."""
        bt = self._batch(a, batch)
        self._batch(b, bt)
        self._batch(out, bt)
        ntt_polymul(self.handle, a, b, out, bt, stream)
        return out

    def tensor_product(self, a, b, d, batch=None, stream=None):
        """d [batch][3][L][N] = tensor product of ciphertexts a, b [batch][2][L][N]."""
        per = self.L * self.N
        if batch is None:
            batch = a.numel() // (2 * per)
        for t, k in ((a, 2), (b, 2), (d, 3)):
            if not t.is_cuda or t.element_size() * 8 != self.word or t.numel() < k * per * batch:
                raise ValueError("tensor shape/dtype/device mismatch")
        ntt_tensor_product(self.handle, a, b, d, batch, stream)
        return d

    def workspace_bytes(self, batch: int) -> int:
        return ntt_workspace_bytes(self.handle, batch)
