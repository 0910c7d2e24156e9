"""ctypes binding of libpir (include/pir.h): argument marshalling only.

Every step of the scan runs in libpir's HIP kernels; this module converts
Python/torch arguments to the C ABI and raises ``PirError`` on a non-OK
status.  Device buffers are torch tensors on the ROCm device (uint32 data is
held in int32 storage); streams default to torch's current stream.

If ``libpir.so`` has not been built the import fails loudly: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes as ct
import os
import weakref
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpir.so")

MAX_PRIMES = 4
STATUS = {
    0: "PIR_OK", 1: "PIR_ERR_INVALID_ARG", 2: "PIR_ERR_UNSUPPORTED", 3: "PIR_ERR_OUT_OF_MEMORY",
    4: "PIR_ERR_BUDGET", 5: "PIR_ERR_DEVICE", 6: "PIR_ERR_NOT_READY",
}

# Declared C functions: name -> (restype, argtypes).  Mirrors include/pir.h.
_P = ct.c_void_p
_U32 = ct.c_uint32
_U32P = ct.POINTER(ct.c_uint32)


class CParams(ct.Structure):
    _fields_ = [("log2_n", ct.c_uint32), ("n_primes", ct.c_uint32),
                ("primes", ct.c_uint32 * MAX_PRIMES), ("plain_log2", ct.c_uint32)]


class CJob(ct.Structure):
    _fields_ = [("db", ct.c_void_p), ("B", ct.c_uint32), ("query_coeff", ct.c_void_p),
                ("answer_coeff", ct.c_void_p), ("switch_bits", ct.c_uint32)]


SIGNATURES = {
    "pir_status_string": (ct.c_char_p, [ct.c_int]),
    "pir_version": (ct.c_char_p, []),
    "pir_find_primes": (ct.c_int, [_U32, _U32, _U32, _U32P]),
    "pir_params_check": (ct.c_int, [ct.POINTER(CParams), _U32P]),
    "pir_ctx_create": (ct.c_int, [ct.c_int, ct.c_size_t, ct.POINTER(ct.c_void_p)]),
    "pir_ctx_destroy": (None, [_P]),
    "pir_last_error": (ct.c_char_p, [_P]),
    "pir_ctx_device_bytes": (ct.c_size_t, [_P]),
    "pir_ctx_reserve": (ct.c_int, [_P, ct.c_size_t]),
    "pir_db_load_ntt": (ct.c_int, [_P, ct.POINTER(CParams), _P, ct.c_int, _U32, _U32, _P,
                                   ct.POINTER(ct.c_void_p)]),
    "pir_db_info": (ct.c_int, [_P, ct.POINTER(CParams), _U32P, _U32P,
                               ct.POINTER(ct.c_size_t)]),
    "pir_db_read_ntt": (ct.c_int, [_P, _P, _U32, _U32, _U32, _U32, _P, _P]),
    "pir_db_free": (None, [_P]),
    "pir_ntt": (ct.c_int, [_P, ct.POINTER(CParams), _P, ct.c_size_t, _P]),
    "pir_intt": (ct.c_int, [_P, ct.POINTER(CParams), _P, ct.c_size_t, _P]),
    "pir_intt_modswitch": (ct.c_int, [_P, ct.POINTER(CParams), _P, ct.c_size_t, _U32, _P, _P]),
    "pir_sdb_load": (ct.c_int, [_P, _P, ct.c_int, _U32, _U32, _P, ct.POINTER(ct.c_void_p)]),
    "pir_sdb_mul": (ct.c_int, [_P, _P, _P, _U32, _P, _P]),
    "pir_sdb_free": (None, [_P]),
    "pir_db_mul": (ct.c_int, [_P, _P, _P, _U32, _P, _P]),
    "pir_answer_batch": (ct.c_int, [_P, ct.POINTER(CJob), ct.c_size_t, _P]),
    "pir_answer_batch_static": (ct.c_int, [_P, ct.POINTER(CJob), ct.c_size_t, _P]),
    "pir_pack_load": (ct.c_int, [_P, ct.POINTER(CParams), _P, ct.c_int, _U32, _U32, _P,
                                 ct.POINTER(ct.c_void_p)]),
    "pir_pack": (ct.c_int, [_P, _P, _U32, _P, _P, _P, _U32, _P]),
    "pir_expand_keys_load": (ct.c_int, [_P, ct.POINTER(CParams), _P, ct.c_int, _U32, _U32, _U32,
                                        _U32, _P, ct.POINTER(ct.c_void_p)]),
    "pir_expand_keys_free": (None, [_P]),
    "pir_expand": (ct.c_int, [_P, _P, _P, _U32, _P, _P]),
    "pir_fold": (ct.c_int, [_P, ct.POINTER(CParams), _P, _U32, _P, _U32, _U32, _U32, _P, _P]),
    "pir_scan_variants": (ct.c_uint32, [_U32]),
    "pir_scan_select": (ct.c_int, [_P, _P, _U32, _U32]),
    "pir_scan_kernel": (ct.c_char_p, [_P, _P, _U32]),
    "pir_profile_stages": (ct.c_int, [_P, _U32]),
    "pir_tune": (ct.c_int, [_P, _P, _U32, _P, ct.c_char_p, ct.c_size_t]),
    "pir_tune_batch": (ct.c_int, [_P, ct.POINTER(CJob), ct.c_size_t, _P, ct.c_char_p,
                                  ct.c_size_t]),
    "pir_plan_create": (ct.c_int, [_P, ct.POINTER(CJob), ct.c_size_t, _P,
                                   ct.POINTER(ct.c_void_p)]),
    "pir_plan_launch": (ct.c_int, [_P, _P]),
    "pir_plan_destroy": (None, [_P]),
    "pir_server_create": (ct.c_int, [_P, _P, _U32, _U32, ct.POINTER(ct.c_void_p)]),
    "pir_server_destroy": (None, [_P]),
    "pir_server_submit": (ct.c_int, [_P, _P, _P, ct.POINTER(ct.c_uint64)]),
    "pir_server_step": (ct.c_int, [_P, _P, _U32P, _U32P]),
    "pir_server_poll": (ct.c_int, [_P, ct.c_uint64, ct.POINTER(ct.c_int)]),
    "pir_server_info": (ct.c_int, [_P, _U32P, _U32P, _U32P, _U32P]),
    "pir_server_capacity": (ct.c_int, [ct.POINTER(CParams), _U32, _U32, ct.c_size_t, ct.c_size_t,
                                       _U32, _U32P, ct.POINTER(ct.c_size_t)]),
    "pir_server_simulate": (ct.c_int, [_U32, _U32, _U32, _U32P, _U32, _U32, _U32P, _U32P, _U32P,
                                       _U32P]),
    "pir_profile_enable": (ct.c_int, [_P, ct.c_int]),
    "pir_profile_read": (ct.c_int, [_P, _U32, ct.POINTER(ct.c_double),
                                    ct.POINTER(ct.c_uint64)]),
}

STAGES = {"ntt": 0, "pack": 1, "scan": 2, "intt": 3, "unpack": 4}


class PirError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _load() -> ct.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2606_11536_amd.build`")
    # PyTorch ships its own HIP runtime (same soname as the system one).  Load it
    # first so libpir binds to the runtime that owns torch's device memory and
    # streams; a second HIP/HSA runtime in the process would not see the GPU.
    import torch  # noqa: F401
    lib = ct.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(st: int, ctx=None) -> None:
    if st != 0:
        msg = lib.pir_last_error(ctx).decode()
        raise PirError(st, msg or lib.pir_status_string(st).decode())


@dataclass
class Params:
    """RNS parameters: N = 2**log2_n, primes q_k, p = 2**plain_log2."""
    log2_n: int
    primes: list[int]
    plain_log2: int = 8
    _c: CParams = field(default=None, repr=False, compare=False)

    @property
    def N(self) -> int:
        return 1 << self.log2_n

    @property
    def K(self) -> int:
        return len(self.primes)

    def c(self) -> CParams:
        if self._c is None:
            arr = (ct.c_uint32 * MAX_PRIMES)(*(list(self.primes) + [0] * (MAX_PRIMES - self.K)))
            self._c = CParams(self.log2_n, self.K, arr, self.plain_log2)
        return self._c


def find_primes(log2_n: int, count: int, bound_log2: int = 28) -> list[int]:
    out = (ct.c_uint32 * count)()
    _check(lib.pir_find_primes(log2_n, count, bound_log2, out))
    return list(out)


def params_check(params: Params) -> list[int]:
    """Validate; return psi_k for every prime."""
    out = (ct.c_uint32 * MAX_PRIMES)()
    _check(lib.pir_params_check(ct.byref(params.c()), out))
    return list(out)[: params.K]


def _stream(stream):
    if stream is None:
        import torch
        return ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ct.c_void_p(stream)
    return ct.c_void_p(stream.cuda_stream)


def _ptr(t) -> ct.c_void_p:
    return ct.c_void_p(t.data_ptr())


class ScalarDatabase:
    """A device-resident int8 D1 x D0 database for the scalar-HE GEMM, owned by libpir."""

    def __init__(self, ctx: "Context", handle: ct.c_void_p, D1: int, D0: int):
        self.ctx, self.handle, self.D1, self.D0 = ctx, handle, D1, D0

    def free(self) -> None:
        if self.handle and self.ctx.handle:
            lib.pir_sdb_free(self.handle)
        self.handle = None


class ExpandKeys:
    """Key-switching keys of B clients for pir_expand, held in NTT form by libpir."""

    def __init__(self, ctx: "Context", handle: ct.c_void_p, params: Params, B: int, levels: int,
                 base_log: int, n_digits: int):
        self.ctx, self.handle, self.params = ctx, handle, params
        self.B, self.levels, self.base_log, self.n_digits = B, levels, base_log, n_digits

    def free(self) -> None:
        if self.handle and self.ctx.handle:
            lib.pir_expand_keys_free(self.handle)
        self.handle = None


class Database:
    """A device-resident NTT-form database owned by libpir."""

    def __init__(self, ctx: "Context", handle: ct.c_void_p, params: Params, R: int, C: int):
        self.ctx, self.handle, self.params, self.R, self.C = ctx, handle, params, R, C

    @property
    def device_bytes(self) -> int:
        n = ct.c_size_t()
        _check(lib.pir_db_info(self.handle, None, None, None, ct.byref(n)))
        return n.value

    def read_ntt(self, i0: int, ni: int, j0: int, nj: int, stream=None):
        """Canonical NTT form of rows [i0, i0+ni) x cols [j0, j0+nj): int32 tensor [ni][nj][K][N]."""
        import torch
        out = torch.empty((ni, nj, self.params.K, self.params.N), dtype=torch.int32,
                          device=f"cuda:{self.ctx.device}")
        _check(lib.pir_db_read_ntt(self.ctx.handle, self.handle, i0, ni, j0, nj, _ptr(out),
                                   _stream(stream)), self.ctx.handle)
        return out

    def free(self) -> None:
        if self.handle and self.ctx.handle:
            lib.pir_db_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """One libpir context on one device (tables, workspace, HBM budget)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ct.c_void_p()
        self.handle = None
        _check(lib.pir_ctx_create(device, hbm_budget_bytes, ct.byref(h)))
        self.handle, self.device = h, device
        self._dbs = weakref.WeakSet()
        self._servers = weakref.WeakSet()

    def close(self) -> None:
        """Free this context's databases, then the context."""
        if self.handle:
            for srv in list(self._servers):
                srv.close()
            for db in list(self._dbs):
                db.free()
            lib.pir_ctx_destroy(self.handle)
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
    def device_bytes(self) -> int:
        return lib.pir_ctx_device_bytes(self.handle)

    def reserve(self, nbytes: int) -> None:
        _check(lib.pir_ctx_reserve(self.handle, nbytes), self.handle)

    def load_db(self, params: Params, raw, R: int, C: int, stream=None) -> Database:
        """Offline transform of a raw [R][C][N] uint8 database (numpy array or torch tensor)."""
        h = ct.c_void_p()
        if hasattr(raw, "data_ptr"):
            is_dev = int(raw.is_cuda)
            assert raw.is_contiguous() and raw.numel() == R * C * params.N
            ptr = ct.c_void_p(raw.data_ptr())
        else:
            import numpy as np
            raw = np.ascontiguousarray(raw, dtype=np.uint8)
            assert raw.size == R * C * params.N
            is_dev = 0
            ptr = raw.ctypes.data_as(ct.c_void_p)
        _check(lib.pir_db_load_ntt(self.handle, ct.byref(params.c()), ptr, is_dev, R, C,
                                   _stream(stream), ct.byref(h)), self.handle)
        db = Database(self, h, params, R, C)
        self._dbs.add(db)
        return db

    def load_pack(self, params: Params, A, D1: int, n: int, stream=None) -> Database:
        """Offline transform of an LWE matrix A [D1][n] (uint32; numpy array or torch
        tensor) into a ring-packing hint (pir_pack_load)."""
        h = ct.c_void_p()
        if hasattr(A, "data_ptr"):
            assert A.is_contiguous() and A.numel() == D1 * n and A.element_size() == 4
            is_dev, ptr = int(A.is_cuda), ct.c_void_p(A.data_ptr())
        else:
            import numpy as np
            A = np.ascontiguousarray(A, dtype=np.uint32)
            assert A.size == D1 * n
            is_dev, ptr = 0, A.ctypes.data_as(ct.c_void_p)
        _check(lib.pir_pack_load(self.handle, ct.byref(params.c()), ptr, is_dev, D1, n,
                                 _stream(stream), ct.byref(h)), self.handle)
        H = Database(self, h, params, n, -(-D1 // params.N))
        H.D1 = D1
        self._dbs.add(H)
        return H

    def pack(self, H: Database, B: int, special_coeff, lwe_b, out, switch_bits: int = 0,
             stream=None) -> None:
        """Ring packing: special_coeff [B][n][2][K][N], lwe_b [B][D1] -> out
        [B][C'][2][K][N] (or [B][C'][2][N] mod 2^switch_bits); device tensors."""
        _check(lib.pir_pack(self.handle, H.handle, B, _ptr(special_coeff), _ptr(lwe_b), _ptr(out),
                            switch_bits, _stream(stream)), self.handle)

    def load_expand_keys(self, params: Params, keys, B: int, levels: int, base_log: int,
                         n_digits: int, stream=None) -> ExpandKeys:
        """Key-switching keys [B][levels][n_digits][2][K][N] (coefficient form; numpy array
        or torch tensor) for pir_expand."""
        h = ct.c_void_p()
        if hasattr(keys, "data_ptr"):
            assert keys.is_contiguous() and keys.element_size() == 4
            is_dev, ptr = int(keys.is_cuda), ct.c_void_p(keys.data_ptr())
        else:
            import numpy as np
            keys = np.ascontiguousarray(keys, dtype=np.uint32)
            is_dev, ptr = 0, keys.ctypes.data_as(ct.c_void_p)
        _check(lib.pir_expand_keys_load(self.handle, ct.byref(params.c()), ptr, is_dev, B, levels,
                                        base_log, n_digits, _stream(stream), ct.byref(h)),
               self.handle)
        k = ExpandKeys(self, h, params, B, levels, base_log, n_digits)
        self._dbs.add(k)
        return k

    def expand(self, keys: ExpandKeys, ct_coeff, n: int, out, stream=None) -> None:
        """Expansion: ct_coeff [B][2][K][N] -> out [B][n][2][K][N] (device tensors)."""
        _check(lib.pir_expand(self.handle, keys.handle, _ptr(ct_coeff), n, _ptr(out),
                              _stream(stream)), self.handle)

    def fold(self, params: Params, cts, D: int, rgsw, base_log: int, n_digits: int, B: int, out,
             stream=None) -> None:
        """RGSW folding: cts [B][D][2][K][N], rgsw [B][log2 D][2 n_digits][2][K][N] -> out
        [B][2][K][N] (device tensors, coefficient form)."""
        _check(lib.pir_fold(self.handle, ct.byref(params.c()), _ptr(cts), D,
                            _ptr(rgsw) if rgsw is not None else None, base_log, n_digits, B,
                            _ptr(out), _stream(stream)), self.handle)

    def load_sdb(self, db, D1: int, D0: int, stream=None) -> ScalarDatabase:
        """Tile an int8 [D1][D0] database (numpy array or torch tensor) for pir_sdb_mul."""
        h = ct.c_void_p()
        if hasattr(db, "data_ptr"):
            assert db.is_contiguous() and db.numel() == D1 * D0 and db.element_size() == 1
            is_dev, ptr = int(db.is_cuda), ct.c_void_p(db.data_ptr())
        else:
            import numpy as np
            db = np.ascontiguousarray(db, dtype=np.int8)
            assert db.size == D1 * D0
            is_dev, ptr = 0, db.ctypes.data_as(ct.c_void_p)
        _check(lib.pir_sdb_load(self.handle, ptr, is_dev, D1, D0, _stream(stream), ct.byref(h)),
               self.handle)
        sdb = ScalarDatabase(self, h, D1, D0)
        self._dbs.add(sdb)
        return sdb

    def sdb_mul(self, db: ScalarDatabase, query, B: int, out, stream=None) -> None:
        """out [B][D1] = query [B][D0] x db^T mod 2^32 (uint32 device tensors as int32)."""
        _check(lib.pir_sdb_mul(self.handle, db.handle, _ptr(query), B, _ptr(out), _stream(stream)),
               self.handle)

    def ntt(self, params: Params, polys, n_polys: int | None = None, stream=None) -> None:
        """In-place forward NTT of [n_polys][K][N] residues (device tensor)."""
        n = polys.numel() // (params.K * params.N) if n_polys is None else n_polys
        _check(lib.pir_ntt(self.handle, ct.byref(params.c()), _ptr(polys), n, _stream(stream)),
               self.handle)

    def intt(self, params: Params, polys, n_polys: int | None = None, stream=None) -> None:
        """In-place inverse NTT (with N^-1) of [n_polys][K][N] residues (device tensor)."""
        n = polys.numel() // (params.K * params.N) if n_polys is None else n_polys
        _check(lib.pir_intt(self.handle, ct.byref(params.c()), _ptr(polys), n, _stream(stream)),
               self.handle)

    def intt_modswitch(self, params: Params, answer_ntt, out, bits: int = 29,
                       n_polys: int | None = None, stream=None) -> None:
        """Inverse NTT fused with modulus switching: answer_ntt [P][K][N] (NTT form,
        device) -> out [P][N] (device), nearest integer to x 2^bits / Q mod 2^bits."""
        n = answer_ntt.numel() // (params.K * params.N) if n_polys is None else n_polys
        _check(lib.pir_intt_modswitch(self.handle, ct.byref(params.c()), _ptr(answer_ntt), n,
                                      bits, _ptr(out), _stream(stream)), self.handle)

    def db_mul(self, db: Database, query_ntt, B: int, answer_ntt, stream=None) -> None:
        """NTT-form scan: query [B][R][2][K][N] -> answer [B][C][2][K][N] (device tensors)."""
        _check(lib.pir_db_mul(self.handle, db.handle, _ptr(query_ntt), B, _ptr(answer_ntt),
                              _stream(stream)), self.handle)

    @staticmethod
    def _jobs(jobs):
        arr = (CJob * len(jobs))()
        for n, job in enumerate(jobs):
            db, B, qc, ac = job[:4]
            bits = job[4] if len(job) > 4 else 0
            arr[n] = CJob(db.handle, B, qc.data_ptr(), ac.data_ptr(), bits)
        return arr

    def answer_batch(self, jobs, stream=None) -> None:
        """Fused batch: jobs = [(db, B, query_coeff, answer_coeff[, switch_bits]), ...]
        (coefficient form; with switch_bits the answers are [B][C][2][N] mod 2^bits)."""
        _check(lib.pir_answer_batch(self.handle, self._jobs(jobs), len(jobs), _stream(stream)),
               self.handle)

    def answer_batch_static(self, jobs, stream=None) -> None:
        """answer_batch with its workspace in the library's fixed device scratch
        array: allocates nothing (see pir_answer_batch_static)."""
        _check(lib.pir_answer_batch_static(self.handle, self._jobs(jobs), len(jobs),
                                           _stream(stream)), self.handle)

    def plan(self, jobs, stream=None) -> "Plan":
        """Capture answer_batch(jobs) into a HIP graph (see pir_plan_create)."""
        return Plan(self, jobs, stream)

    def tune_batch(self, jobs, stream=None) -> str:
        """Autotune the fused scan launches for this job list; returns the report."""
        buf = ct.create_string_buffer(8192)
        _check(lib.pir_tune_batch(self.handle, self._jobs(jobs), len(jobs), _stream(stream), buf,
                                  len(buf)), self.handle)
        return buf.value.decode()

    def profile(self, enable: bool = True, stages=None) -> None:
        """Turn per-stage HIP-event timing on (resets the sums) or off; `stages`
        (names) limits the timing to those stages."""
        if stages is None:
            _check(lib.pir_profile_enable(self.handle, int(enable)), self.handle)
        else:
            mask = sum(1 << STAGES[st] for st in stages) if enable else 0
            _check(lib.pir_profile_stages(self.handle, mask), self.handle)

    def profile_read(self, stage: str) -> tuple[float, int]:
        """(summed ms, launches) of a stage since profiling was enabled; waits for the events."""
        ms, n = ct.c_double(), ct.c_uint64()
        _check(lib.pir_profile_read(self.handle, STAGES[stage], ct.byref(ms), ct.byref(n)),
               self.handle)
        return ms.value, n.value

    def scan_select(self, db: Database, B: int, index: int) -> None:
        """Use scan variant `index` for databases shaped like `db` at batch size B."""
        _check(lib.pir_scan_select(self.handle, db.handle, B, index), self.handle)

    def scan_kernel(self, db: Database, B: int) -> str:
        """Name of the kernel a scan of (db, B) launches with the current choice."""
        name = lib.pir_scan_kernel(self.handle, db.handle, B)
        if name is None:
            raise PirError(f"pir_scan_kernel: bad arguments (B={B})")
        return name.decode()

    def tune(self, db: Database, B: int, stream=None) -> str:
        """Time every scan variant for (db, B), keep the fastest; returns the report."""
        buf = ct.create_string_buffer(4096)
        _check(lib.pir_tune(self.handle, db.handle, B, _stream(stream), buf, len(buf)),
               self.handle)
        return buf.value.decode()


def scan_variants(B: int) -> int:
    return lib.pir_scan_variants(B)


def server_capacity(params: Params, R: int, C: int, held_bytes: int, budget_bytes: int,
                    max_batch: int) -> tuple[int, int]:
    """(admitted batch, its state bytes) under an HBM budget (host only)."""
    a, b = ct.c_uint32(), ct.c_size_t()
    _check(lib.pir_server_capacity(ct.byref(params.c()), R, C, held_bytes, budget_bytes, max_batch,
                                   ct.byref(a), ct.byref(b)))
    return a.value, b.value


def server_simulate(max_batch: int, n_slots: int, n_chunks: int, submits, cover: bool = True):
    """The server's schedule on the host: returns (admit_step, admit_slot,
    finish_step, cover) numpy arrays (cover [n_queries][n_slots] or None)."""
    import numpy as np
    sub = np.ascontiguousarray(submits, dtype=np.uint32)
    nq = int(sub.sum())
    a_step, a_slot, f_step = (np.empty(nq, dtype=np.uint32) for _ in range(3))
    cov = np.empty((nq, n_slots), dtype=np.uint32) if cover else None
    p = ct.POINTER(ct.c_uint32)
    _check(lib.pir_server_simulate(max_batch, n_slots, n_chunks, sub.ctypes.data_as(p), len(sub), nq,
                                   a_step.ctypes.data_as(p), a_slot.ctypes.data_as(p),
                                   f_step.ctypes.data_as(p),
                                   cov.ctypes.data_as(p) if cover else None))
    return a_step, a_slot, f_step, cov


class Server:
    """Continuous-batching server over one database (see pir_server_* in pir.h)."""

    def __init__(self, ctx: Context, db: Database, max_batch: int, n_chunks: int):
        h = ct.c_void_p()
        self.handle = None
        _check(lib.pir_server_create(ctx.handle, db.handle, max_batch, n_chunks, ct.byref(h)),
               ctx.handle)
        self.handle, self.ctx, self.db = h, ctx, db
        self._keep = {}
        ctx._servers.add(self)

    def close(self) -> None:
        if self.handle and self.ctx.handle:
            lib.pir_server_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, query_coeff, answer_coeff) -> int:
        t = ct.c_uint64()
        _check(lib.pir_server_submit(self.handle, _ptr(query_coeff), _ptr(answer_coeff),
                                     ct.byref(t)), self.ctx.handle)
        self._keep[t.value] = (query_coeff, answer_coeff)
        return t.value

    def step(self, stream=None) -> tuple[int, int]:
        a, f = ct.c_uint32(), ct.c_uint32()
        _check(lib.pir_server_step(self.handle, _stream(stream), ct.byref(a), ct.byref(f)),
               self.ctx.handle)
        return a.value, f.value

    def poll(self, ticket: int) -> bool:
        d = ct.c_int()
        _check(lib.pir_server_poll(self.handle, ticket, ct.byref(d)), self.ctx.handle)
        if d.value:
            self._keep.pop(ticket, None)
        return bool(d.value)

    def info(self) -> dict:
        v = [ct.c_uint32() for _ in range(4)]
        _check(lib.pir_server_info(self.handle, *[ct.byref(x) for x in v]), self.ctx.handle)
        return dict(zip(["max_batch", "active", "queued", "next_chunk"], [x.value for x in v]))


class Plan:
    """A job list captured into a HIP graph; launch() replays it."""

    def __init__(self, ctx: Context, jobs, stream=None):
        h = ct.c_void_p()
        self.handle = None
        _check(lib.pir_plan_create(ctx.handle, Context._jobs(jobs), len(jobs), _stream(stream),
                                   ct.byref(h)), ctx.handle)
        self.handle, self.ctx, self._jobs = h, ctx, list(jobs)
        ctx._servers.add(self)

    def launch(self, stream=None) -> None:
        _check(lib.pir_plan_launch(self.handle, _stream(stream)), self.ctx.handle)

    def close(self) -> None:
        if self.handle and self.ctx.handle:
            lib.pir_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
