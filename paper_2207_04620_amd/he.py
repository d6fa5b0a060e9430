"""Python binding of libhe (include/he.h): argument marshalling only.

Every homomorphic step runs in the HIP kernels of libhe.so; this module converts
numpy arrays and torch device tensors to pointers and status codes to exceptions.
There is no fallback: if the library is missing the import of a context fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhe.so")

STATUS = ["HE_OK", "HE_EINVAL", "HE_ENOMEM", "HE_ELEVEL", "HE_ESCALE", "HE_EKEY", "HE_ESHAPE",
          "HE_EMISMATCH", "HE_EDEVICE", "HE_EUNSUPPORTED"]
SCHED_RELIN_EACH = 0
SCHED_RELIN_ONCE = 1
SCHED_HOIST_MODDOWN = 2
SCHED_RESCALE_LATE = 4
SCHED_STEP3_BSGS = 8
SCHED_FAST = SCHED_RELIN_ONCE | SCHED_HOIST_MODDOWN | SCHED_RESCALE_LATE | SCHED_STEP3_BSGS
SIGN = 0
RELU = 1
REQ_MATMUL = 0
REQ_SIGN = 1
REQ_POWER = 2


class HEError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        self.name = STATUS[code] if 0 <= code < len(STATUS) else str(code)
        super().__init__(f"{what}: {self.name}")


class _Params(C.Structure):
    _fields_ = [("log_n", C.c_uint32), ("n_q", C.c_uint32), ("q_bits", C.POINTER(C.c_uint32)),
                ("n_p", C.c_uint32), ("p_bits", C.POINTER(C.c_uint32)), ("alpha", C.c_uint32),
                ("log_scale", C.c_double), ("seed", C.c_uint64), ("n_h", C.c_uint32),
                ("h_list", C.POINTER(C.c_uint32)), ("schedule", C.c_uint32)]


class _Device(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("alloc", C.c_void_p), ("free", C.c_void_p), ("user", C.c_void_p)]


class _ServeConfig(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_uint64), ("max_batch", C.c_uint32), ("min_batch", C.c_uint32),
                ("max_wait_us", C.c_uint32)]


class _Tuning(C.Structure):
    _fields_ = [("pair_batch", C.c_uint32), ("max_group", C.c_uint32), ("overlap", C.c_uint32),
                ("concurrent_groups", C.c_uint32)]


class _Request(C.Structure):
    _fields_ = [("op", C.c_uint32), ("h", C.c_uint32), ("d", C.c_uint32), ("k", C.c_uint32),
                ("mode", C.c_uint32), ("a", C.c_void_p), ("b", C.c_void_p)]


_lib = None

# name -> (restype, argtypes); every entry point of include/he.h
SIGNATURES = {
    "he_ctx_create": (C.c_int, [C.POINTER(_Params), C.POINTER(_Device), C.POINTER(C.c_void_p)]),
    "he_ctx_destroy": (None, [C.c_void_p]),
    "he_ctx_moduli": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.c_size_t]),
    "he_sync": (C.c_int, [C.c_void_p]),
    "he_counters": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int]),
    "he_memory": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "he_encrypt": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_size_t, C.c_uint32, C.c_uint64,
                             C.POINTER(C.c_void_p)]),
    "he_encrypt_coeffs": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_uint32, C.c_double, C.c_uint64,
                                    C.POINTER(C.c_void_p)]),
    "he_decrypt": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_size_t]),
    "he_decrypt_coeffs": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_size_t]),
    "he_encode": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_size_t, C.c_double, C.POINTER(C.c_int64)]),
    "he_ct_free": (None, [C.c_void_p]),
    "he_ct_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_double)]),
    "he_ct_export": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64), C.c_size_t]),
    "he_ct_import": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.c_size_t, C.c_uint32, C.c_uint32, C.c_double,
                               C.POINTER(C.c_void_p)]),
    "he_add": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "he_sub": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "he_drop": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(C.c_void_p)]),
    "he_mul_plain": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.c_double, C.POINTER(C.c_void_p)]),
    "he_mul_int": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_void_p)]),
    "he_tensor": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "he_relin": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "he_mul": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "he_rescale": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "he_rotate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_void_p)]),
    "he_gen_rotation_key": (C.c_int, [C.c_void_p, C.c_int64]),
    "he_matmul": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(C.c_void_p)]),
    "he_matmul_batch": (C.c_int, [C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_uint32), C.POINTER(C.c_void_p)]),
    "he_matmul_ex": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "he_matmul_batch_ex": (C.c_int, [C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.c_void_p, C.POINTER(C.c_void_p)]),
    "he_transpose": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(C.c_void_p)]),
    "he_appmax": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(C.c_void_p)]),
    "he_appmax_batch": (C.c_int, [C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_uint32,
                                  C.c_uint32, C.POINTER(C.c_void_p)]),
    "he_maxpool2": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_void_p)]),
    "he_maxpool2_batch": (C.c_int, [C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p), C.c_uint32, C.c_uint32,
                                    C.c_uint32, C.POINTER(C.c_void_p)]),
    "he_fl_update": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p), C.c_double,
                               C.POINTER(C.c_void_p)]),
    "he_transpose_batch": (C.c_int, [C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p), C.c_uint32, C.c_uint32,
                                     C.POINTER(C.c_void_p)]),
    "he_sign_approx": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32,
                                 C.POINTER(C.c_void_p)]),
    "he_sign_approx_batch": (C.c_int, [C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p), C.c_uint32, C.c_uint32,
                                       C.c_uint32, C.POINTER(C.c_void_p)]),
    "he_ntt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(C.c_uint32), C.c_int]),
    "he_serve_start": (C.c_int, [C.c_void_p, C.POINTER(_ServeConfig), C.POINTER(C.c_void_p)]),
    "he_serve_submit": (C.c_int, [C.c_void_p, C.POINTER(_Request), C.POINTER(C.c_uint64)]),
    "he_serve_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_void_p),
                                C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "he_serve_stop": (C.c_int, [C.c_void_p]),
    "he_serve_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                 C.c_size_t, C.POINTER(C.c_uint64), C.POINTER(C.c_size_t)]),
    "he_profile_enable": (C.c_int, [C.c_void_p, C.c_int, C.c_char_p]),
    "he_profile_report": (C.c_int, [C.c_void_p, C.c_char_p, C.c_size_t]),
    "he_status_string": (C.c_char_p, [C.c_int]),
    "he_debug_fail_launch": (C.c_int, [C.c_uint64]),
    "he_matmul_batch_capture": (C.c_int, [C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                          C.POINTER(C.c_uint32), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "he_graph_launch": (C.c_int, [C.c_void_p]),
    "he_graph_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_uint64)]),
    "he_graph_destroy": (None, [C.c_void_p]),
    "he_tuning_get": (C.c_int, [C.c_void_p, C.POINTER(_Tuning)]),
    "he_tuning_set": (C.c_int, [C.c_void_p, C.POINTER(_Tuning)]),
    "he_autotune": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_char_p, C.POINTER(_Tuning),
                              C.c_char_p, C.c_size_t]),
    "he_rotate_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_int64, C.c_void_p]),
    "he_pool_limit": (C.c_int, [C.c_void_p, C.c_uint64]),
    "he_pack_beta": (C.c_int, [C.c_size_t, C.c_size_t, C.c_void_p, C.POINTER(C.c_double)]),
    "he_pool_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.c_int]),
    "he_stream_probe": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                  C.c_uint32, C.POINTER(C.c_double)]),
}


def lib():
    """Load libhe.so (built in-tree by ``python -m paper_2207_04620_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libhe.so not built: run `python -m paper_2207_04620_amd.build` ({LIB_PATH})")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _chk(code, what):
    if code != 0:
        raise HEError(code, what)


def _u64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _i64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Ciphertext:
    __slots__ = ("ctx", "ptr")

    def __init__(self, ctx: "Context", ptr):
        self.ctx, self.ptr = ctx, ptr

    def __del__(self):
        # the context holds the free function, so this also works while the interpreter
        # tears down module globals
        if getattr(self, "ptr", None) and self.ctx.ptr:
            self.ctx._ct_free(self.ptr)
            self.ptr = None

    def info(self):
        lv, dg, sc = C.c_uint32(), C.c_uint32(), C.c_double()
        _chk(lib().he_ct_info(self.ptr, C.byref(lv), C.byref(dg), C.byref(sc)), "he_ct_info")
        return lv.value, dg.value, sc.value

    @property
    def level(self):
        return self.info()[0]

    @property
    def degree(self):
        return self.info()[1]

    @property
    def scale(self):
        return self.info()[2]


class _MatShape(C.Structure):
    _fields_ = [("h", C.c_uint32), ("t", C.c_uint32), ("beta", C.c_uint32)]


def pack_beta(mats):
    """the packing iota_beta (App. E) as a slot vector: matrix m's entry (i, j) at
    position beta (h i + j) + m (he_pack_beta)"""
    mats = [np.ascontiguousarray(np.asarray(m, np.float64).ravel()) for m in mats]
    beta, n = len(mats), mats[0].size
    if any(m.size != n for m in mats):
        raise ValueError("pack_beta: matrices of different sizes")
    ptrs = (C.POINTER(C.c_double) * beta)(*[m.ctypes.data_as(C.POINTER(C.c_double)) for m in mats])
    v = np.empty(beta * n)
    _chk(lib().he_pack_beta(beta, n, ptrs, v.ctypes.data_as(C.POINTER(C.c_double))), "he_pack_beta")
    return v


class Context:
    """An RNS-CKKS context on the current HIP device (see include/he.h)."""

    def __init__(self, params, schedule: int = SCHED_RELIN_EACH, h_list=None, stream=None):
        L = lib()
        self._ct_free, self._ctx_destroy = L.he_ct_free, L.he_ctx_destroy
        self.params = params
        self.n = 1 << params.log_n
        qb = (C.c_uint32 * len(params.q_bits))(*params.q_bits)
        pb = (C.c_uint32 * len(params.p_bits))(*params.p_bits)
        hl = list(params.h_list if h_list is None else h_list)
        ha = (C.c_uint32 * max(1, len(hl)))(*hl)
        self._keep = (qb, pb, ha)
        p = _Params(params.log_n, len(params.q_bits), qb, len(params.p_bits), pb, params.alpha,
                    float(params.log_scale), params.seed, len(hl), ha, schedule)
        dev = _Device(stream, None, None, None)
        out = C.c_void_p()
        self.ptr = None
        _chk(L.he_ctx_create(C.byref(p), C.byref(dev), C.byref(out)), "he_ctx_create")
        self.ptr = out.value
        m = np.zeros(len(params.q_bits) + len(params.p_bits), np.uint64)
        _chk(L.he_ctx_moduli(self.ptr, _u64p(m), len(m)), "he_ctx_moduli")
        self.moduli = [int(x) for x in m]
        self.max_level = len(params.q_bits) - 1
        self.scale = 2.0 ** params.log_scale

    def close(self):
        if getattr(self, "ptr", None):
            self._ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        self.close()

    def _ct(self, fn, *args, what=""):
        out = C.c_void_p()
        _chk(fn(self.ptr, *args, C.byref(out)), what or fn.__name__)
        return Ciphertext(self, out.value)

    # -- housekeeping
    def sync(self):
        _chk(lib().he_sync(self.ptr), "he_sync")

    def counters(self, reset=False):
        o = np.zeros(6, np.int64)
        _chk(lib().he_counters(self.ptr, _i64p(o), int(reset)), "he_counters")
        return dict(zip(["rot", "keyswitch", "mul_pt", "mul_ct", "add", "rescale"], (int(x) for x in o)))

    def tuning(self):
        t = _Tuning()
        _chk(lib().he_tuning_get(self.ptr, C.byref(t)), "he_tuning_get")
        return {"pair_batch": t.pair_batch, "max_group": t.max_group, "overlap": t.overlap,
                "concurrent_groups": t.concurrent_groups}

    def set_tuning(self, pair_batch: int, max_group: int, overlap: int = 0, concurrent_groups: int = 1):
        t = _Tuning(pair_batch, max_group, overlap, concurrent_groups)
        _chk(lib().he_tuning_set(self.ptr, C.byref(t)), "he_tuning_set")

    def autotune(self, h: int, level: int, batch: int, cache_path: str | None = None):
        """time the batched product under each candidate tuning, apply the fastest; returns the
        report (candidates' times and the choice)"""
        import json
        t = _Tuning()
        buf = C.create_string_buffer(1 << 14)
        _chk(lib().he_autotune(self.ptr, h, level, batch, cache_path.encode() if cache_path else None, C.byref(t),
                               buf, len(buf)), "he_autotune")
        return json.loads(buf.value.decode())

    def pool_limit(self, nbytes: int):
        _chk(lib().he_pool_limit(self.ptr, int(nbytes)), "he_pool_limit")

    def pool_stats(self, reset=False):
        """(bytes in use, peak bytes in use since the last reset)"""
        a, b = C.c_uint64(), C.c_uint64()
        _chk(lib().he_pool_stats(self.ptr, C.byref(a), C.byref(b), int(reset)), "he_pool_stats")
        return a.value, b.value

    def memory(self):
        k, p = C.c_uint64(), C.c_uint64()
        _chk(lib().he_memory(self.ptr, C.byref(k), C.byref(p)), "he_memory")
        return k.value, p.value

    def profile(self, on: bool, only: str | None = None):
        """time every launch (or only launches of the kernel kind named) with HIP events"""
        _chk(lib().he_profile_enable(self.ptr, int(on), None if only is None else only.encode()),
             "he_profile_enable")

    def profile_report(self):
        import json
        buf = C.create_string_buffer(1 << 16)
        _chk(lib().he_profile_report(self.ptr, buf, len(buf)), "he_profile_report")
        return json.loads(buf.value.decode())

    # -- encode / encrypt / decrypt
    def encode(self, vals, scale=None):
        v = np.ascontiguousarray(np.ravel(vals), np.float64)
        o = np.zeros(self.n, np.int64)
        _chk(lib().he_encode(self.ptr, _f64p(v), len(v), float(scale or self.scale), _i64p(o)), "he_encode")
        return o

    def encrypt(self, vals, level=None, nonce=0):
        v = np.ascontiguousarray(np.ravel(vals), np.float64)
        lvl = self.max_level if level is None else level
        return self._ct(lib().he_encrypt, _f64p(v), len(v), lvl, nonce)

    def encrypt_coeffs(self, coeffs, level, scale, nonce):
        m = np.ascontiguousarray(coeffs, np.int64)
        return self._ct(lib().he_encrypt_coeffs, _i64p(m), level, float(scale), nonce)

    def decrypt(self, ct, n=None):
        n = self.n // 2 if n is None else n
        o = np.zeros(n, np.float64)
        _chk(lib().he_decrypt(self.ptr, ct.ptr, _f64p(o), n), "he_decrypt")
        return o

    def decrypt_coeffs(self, ct):
        o = np.zeros(self.n, np.float64)
        _chk(lib().he_decrypt_coeffs(self.ptr, ct.ptr, _f64p(o), self.n), "he_decrypt_coeffs")
        return o

    def export(self, ct):
        lv, dg, _ = ct.info()
        o = np.zeros((dg + 1, lv + 1, self.n), np.uint64)
        _chk(lib().he_ct_export(self.ptr, ct.ptr, _u64p(o), o.size), "he_ct_export")
        return o

    def import_(self, arr, level, scale, degree=1):
        a = np.ascontiguousarray(arr, np.uint64)
        return self._ct(lib().he_ct_import, _u64p(a), a.size, level, degree, float(scale))

    # -- Fig. 1 operations
    def add(self, a, b):
        return self._ct(lib().he_add, a.ptr, b.ptr)

    def sub(self, a, b):
        return self._ct(lib().he_sub, a.ptr, b.ptr)

    def drop(self, a, level):
        return self._ct(lib().he_drop, a.ptr, level)

    def mul_plain(self, a, coeffs, pt_scale):
        m = np.ascontiguousarray(coeffs, np.int64)
        return self._ct(lib().he_mul_plain, a.ptr, _i64p(m), float(pt_scale))

    def mul_int(self, a, k):
        return self._ct(lib().he_mul_int, a.ptr, int(k))

    def tensor(self, a, b):
        return self._ct(lib().he_tensor, a.ptr, b.ptr)

    def relin(self, a):
        return self._ct(lib().he_relin, a.ptr)

    def mul(self, a, b):
        return self._ct(lib().he_mul, a.ptr, b.ptr)

    def rescale(self, a):
        return self._ct(lib().he_rescale, a.ptr)

    def rotate(self, a, k):
        return self._ct(lib().he_rotate, a.ptr, int(k))

    def gen_rotation_key(self, k):
        _chk(lib().he_gen_rotation_key(self.ptr, int(k)), "he_gen_rotation_key")

    # -- the packed product and the sign approximation
    def rotate_noalloc(self, in_ptr: int, level: int, k: int, out_ptr: int):
        """Rot by k on caller device memory (u64[2][level+1][N], evaluation domain); allocates
        nothing"""
        _chk(lib().he_rotate_noalloc(self.ptr, C.c_void_p(in_ptr), level, k, C.c_void_p(out_ptr)),
             "he_rotate_noalloc")

    def matmul(self, a, b, h):
        return self._ct(lib().he_matmul, a.ptr, b.ptr, int(h))

    def matmul_batch(self, As, Bs, hs):
        n = len(As)
        pa = (C.c_void_p * n)(*[x.ptr for x in As])
        pb = (C.c_void_p * n)(*[x.ptr for x in Bs])
        ph = (C.c_uint32 * n)(*[int(h) for h in hs])
        out = (C.c_void_p * n)()
        _chk(lib().he_matmul_batch(self.ptr, n, pa, pb, ph, out), "he_matmul_batch")
        return [Ciphertext(self, out[i]) for i in range(n)]

    def matmul_batch_graph(self, As, Bs, hs):
        """capture the batched product into a HIP graph: (Graph, first results)"""
        n = len(As)
        pa = (C.c_void_p * n)(*[x.ptr for x in As])
        pb = (C.c_void_p * n)(*[x.ptr for x in Bs])
        ph = (C.c_uint32 * n)(*hs)
        po = (C.c_void_p * n)()
        g = C.c_void_p()
        _chk(lib().he_matmul_batch_capture(self.ptr, n, pa, pb, ph, C.byref(g), po), "he_matmul_batch_capture")
        return Graph(self, g.value, (As, Bs)), [Ciphertext(self, po[i]) for i in range(n)]

    def matmul_ex(self, a, b, h, t=None, beta=1):
        """HE-MatMult (t = h) / HE-RMatMult (t < h, a holds h/t copies of a t x h matrix) on
        beta matrix pairs packed by iota_beta"""
        return self.matmul_batch_ex([a], [b], [(h, h if t is None else t, beta)])[0]

    def matmul_batch_ex(self, As, Bs, shapes):
        n = len(As)
        pa = (C.c_void_p * n)(*[x.ptr for x in As])
        pb = (C.c_void_p * n)(*[x.ptr for x in Bs])
        sh = (_MatShape * n)(*[_MatShape(int(h), int(t), int(bt)) for h, t, bt in shapes])
        out = (C.c_void_p * n)()
        _chk(lib().he_matmul_batch_ex(self.ptr, n, pa, pb, sh, out), "he_matmul_batch_ex")
        return [Ciphertext(self, out[i]) for i in range(n)]

    def transpose(self, a, h, beta=1):
        return self.transpose_batch([a], h, beta)[0]

    def transpose_batch(self, xs, h, beta=1):
        n = len(xs)
        px = (C.c_void_p * n)(*[x.ptr for x in xs])
        out = (C.c_void_p * n)()
        _chk(lib().he_transpose_batch(self.ptr, n, px, int(h), int(beta), out), "he_transpose_batch")
        return [Ciphertext(self, out[i]) for i in range(n)]

    def appmax(self, a, b, d, k):
        """AppMax (Alg. 5): max(a, b) by the composite sign g_d^(k)"""
        return self.appmax_batch([a], [b], d, k)[0]

    def appmax_batch(self, As, Bs, d, k):
        n = len(As)
        pa = (C.c_void_p * n)(*[x.ptr for x in As])
        pb = (C.c_void_p * n)(*[x.ptr for x in Bs])
        out = (C.c_void_p * n)()
        _chk(lib().he_appmax_batch(self.ptr, n, pa, pb, int(d), int(k), out), "he_appmax_batch")
        return [Ciphertext(self, out[i]) for i in range(n)]

    def maxpool2(self, x, h, d, k):
        return self.maxpool2_batch([x], h, d, k)[0]

    def maxpool2_batch(self, xs, h, d, k):
        n = len(xs)
        px = (C.c_void_p * n)(*[x.ptr for x in xs])
        out = (C.c_void_p * n)()
        _chk(lib().he_maxpool2_batch(self.ptr, n, px, int(h), int(d), int(k), out), "he_maxpool2_batch")
        return [Ciphertext(self, out[i]) for i in range(n)]

    def fl_update(self, w, grads, coeff):
        """Alg. 6 aggregation: W - coeff sum_i G_i"""
        n = len(grads)
        pg = (C.c_void_p * n)(*[g.ptr for g in grads])
        out = C.c_void_p()
        _chk(lib().he_fl_update(self.ptr, w.ptr, n, pg, float(coeff), C.byref(out)), "he_fl_update")
        return Ciphertext(self, out.value)

    def sign_approx(self, x, d, k, mode=SIGN):
        return self._ct(lib().he_sign_approx, x.ptr, int(d), int(k), int(mode))

    def sign_approx_batch(self, xs, d, k, mode=SIGN):
        n = len(xs)
        px = (C.c_void_p * n)(*[x.ptr for x in xs])
        out = (C.c_void_p * n)()
        _chk(lib().he_sign_approx_batch(self.ptr, n, px, int(d), int(k), int(mode), out), "he_sign_approx_batch")
        return [Ciphertext(self, out[i]) for i in range(n)]

    def ntt(self, dev_tensor, mod_idx, inverse=False):
        """in-place limb-batched NTT of a (n_limbs, N) uint64/int64 torch tensor on the GPU"""
        n_limbs = dev_tensor.shape[0]
        mi = (C.c_uint32 * n_limbs)(*[int(x) for x in mod_idx])
        _chk(lib().he_ntt(self.ptr, C.c_void_p(dev_tensor.data_ptr()), n_limbs, mi, int(inverse)), "he_ntt")

    def stream_probe(self, pattern, a, b, c, reps):
        """he_stream_probe over 64-bit torch tensors on the GPU (a, c and, for pattern 2, b of
        equal word counts; pattern 0 writes 2^20 partial-sum words to c): mean ms per launch"""
        for t in (a, b, c):
            if t is not None and (t.element_size() != 8 or not t.is_contiguous()):
                raise ValueError("stream_probe: contiguous tensors of 64-bit words")
        if b is not None and b.numel() != a.numel():
            raise ValueError("stream_probe: a and b of different sizes")
        need = 2 * ((a.numel() + 4095) // 4096) if pattern == 0 else a.numel()
        if c.numel() < need:
            raise ValueError(f"stream_probe: c holds {c.numel()} words, the pattern writes {need}")
        ms = C.c_double()
        bp = C.c_void_p(b.data_ptr()) if b is not None else None
        _chk(lib().he_stream_probe(self.ptr, int(pattern), C.c_void_p(a.data_ptr()), bp, C.c_void_p(c.data_ptr()),
                                   a.numel(), int(reps), C.byref(ms)), "he_stream_probe")
        return ms.value


class Graph:
    """A captured batched product (he_matmul_batch_capture): launch() replays it on the context
    stream, rewriting the results the capture returned."""

    def __init__(self, ctx, ptr, keep):
        self.ctx, self.ptr, self._keep = ctx, ptr, keep
        self._destroy = lib().he_graph_destroy

    def launch(self):
        _chk(lib().he_graph_launch(self.ptr), "he_graph_launch")

    def info(self):
        n, b = C.c_size_t(), C.c_uint64()
        _chk(lib().he_graph_info(self.ptr, C.byref(n), C.byref(b)), "he_graph_info")
        return {"nodes": n.value, "bytes": b.value}

    def close(self):
        if getattr(self, "ptr", None):
            self._destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        self.close()


def fail_launch(n: int):
    """error-path testing: the n-th kernel launch from now on fails before it is queued (the
    call that issued it returns HE_EDEVICE); 0 disarms"""
    _chk(lib().he_debug_fail_launch(int(n)), "he_debug_fail_launch")


def sign_depth(d: int, k: int, mode: int = SIGN) -> int:
    """levels consumed by k compositions of g_d (1 + floor(log2 d) + 1 each), +1 for ReLU"""
    return k * (d.bit_length() + 1) + (1 if mode == RELU else 0)


def smallest_ring(contexts, h: int = 0, depth: int = 3):
    """the context of the smallest ring that holds an h x h matrix (h^2 <= N/2) and has
    'depth' levels to spend from its top level; None if none does"""
    for ctx in sorted(contexts, key=lambda c: c.n):
        if h * h <= ctx.n // 2 and depth <= ctx.max_level:
            return ctx
    return None


class Server:
    """Continuous-batching request loop of libhe (he_serve_*)."""

    def __init__(self, ctx: Context, mem_budget_bytes=0, max_batch=0, min_batch=0, max_wait_us=0):
        self.ctx = ctx
        cfg = _ServeConfig(mem_budget_bytes, max_batch, min_batch, max_wait_us)
        out = C.c_void_p()
        self.ptr = None
        self._stop = lib().he_serve_stop
        _chk(lib().he_serve_start(ctx.ptr, C.byref(cfg), C.byref(out)), "he_serve_start")
        self.ptr = out.value
        self._inputs = {}

    def submit(self, op, a, b=None, h=0, d=3, k=1, mode=0):
        req = _Request(op, h, d, k, mode, a.ptr, b.ptr if b is not None else None)
        t = C.c_uint64()
        _chk(lib().he_serve_submit(self.ptr, C.byref(req), C.byref(t)), "he_serve_submit")
        self._inputs[t.value] = (a, b)
        return t.value

    def poll(self, ticket):
        done, res, st, lat = C.c_int(), C.c_void_p(), C.c_int(), C.c_double()
        _chk(lib().he_serve_poll(self.ptr, ticket, C.byref(done), C.byref(res), C.byref(st), C.byref(lat)),
             "he_serve_poll")
        if not done.value:
            return None
        self._inputs.pop(ticket, None)
        if st.value != 0:
            raise HEError(st.value, "request")
        return Ciphertext(self.ctx, res.value), lat.value

    def stats(self):
        """dict: bytes in flight, largest measured cohort footprint, the allocation cache's peak
        in-use bytes while serving, measured per-member footprints"""
        a, b, c, n = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_size_t()
        buf = (C.c_uint64 * 64)()
        _chk(lib().he_serve_stats(self.ptr, C.byref(a), C.byref(b), C.byref(c), 64, buf, C.byref(n)),
             "he_serve_stats")
        return {"inflight": a.value, "peak_cohort": b.value, "peak_in_use": c.value,
                "per_member": [buf[i] for i in range(min(64, n.value))]}

    def stop(self):
        if getattr(self, "ptr", None):
            code = self._stop(self.ptr)
            self.ptr = None
            if code != 0:
                raise HEError(code, "he_serve_stop")

    def __del__(self):
        self.stop()
