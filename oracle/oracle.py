"""ctypes front-end of the CPU oracle (ckks_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use this module; the GPU library never does.
It shares no code with the GPU library.  See ckks_oracle.h for the paper
passages each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "libckks_oracle.so")

RELIN_EACH = 0
RELIN_ONCE = 1
HOIST_MODDOWN = 2
RESCALE_LATE = 4
STEP3_BSGS = 8
FAST = RELIN_ONCE | HOIST_MODDOWN | RESCALE_LATE | STEP3_BSGS


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, libquadmath)."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "ckks_oracle.h"))
    ):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall",
             "-Wno-unused-function", "-o", tmp, _SRC, "-lquadmath", "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def build_sanitized() -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only),
    for the sanitizer run of the pins; load it by setting ORACLE_LIB to the returned path in a
    process started with the sanitizer runtimes preloaded."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    out = os.path.join(_LIB_DIR, "libckks_oracle_san.so")
    tmp = out + f".tmp{os.getpid()}"
    subprocess.check_call(
        ["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
         "-o", tmp, _SRC, "-lquadmath", "-lm"]
    )
    os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(os.environ.get("ORACLE_LIB") or build())
        _declare(_lib)
    return _lib


def _declare(L):
    vp, u64, i64, i32, dbl = C.c_void_p, C.c_uint64, C.c_int64, C.c_int, C.c_double
    P = C.POINTER
    sig = {
        "orc_create": (vp, [i32, i32, P(i32), i32, P(i32), i32, dbl, u64, i32]),
        "orc_destroy": (None, [vp]),
        "orc_n_moduli": (i32, [vp]),
        "orc_moduli": (None, [vp, P(u64)]),
        "orc_psi": (u64, [vp, i32]),
        "orc_mulmod": (u64, [u64, u64, u64]),
        "orc_is_prime": (i32, [u64]),
        "orc_chacha20_block": (None, [P(C.c_uint32), C.c_uint32, P(C.c_uint32), P(C.c_uint32)]),
        "orc_word": (u64, [u64, C.c_uint32, u64, u64]),
        "orc_gauss_table": (None, [P(u64)]),
        "orc_sample_ternary": (None, [u64, C.c_uint32, u64, i64, P(i64)]),
        "orc_sample_gauss": (None, [u64, C.c_uint32, u64, i64, P(i64)]),
        "orc_sample_uniform": (None, [u64, C.c_uint32, u64, u64, i64, P(u64)]),
        "orc_poly_mul": (None, [vp, i32, P(u64), P(u64), P(u64)]),
        "orc_eval_bitrev": (None, [vp, i32, P(u64), P(u64)]),
        "orc_base_conv": (None, [vp, i32, P(i32), i32, P(u64), P(u64)]),
        "orc_encode": (dbl, [vp, P(dbl), i64, dbl, P(i64)]),
        "orc_decode": (None, [vp, P(dbl), dbl, P(dbl)]),
        "orc_encrypt_coeffs": (vp, [vp, P(i64), i32, dbl, u64]),
        "orc_encrypt": (vp, [vp, P(dbl), i64, i32, u64]),
        "orc_decrypt_coeffs": (i32, [vp, vp, P(dbl)]),
        "orc_decrypt": (i32, [vp, vp, P(dbl)]),
        "orc_ct_free": (None, [vp]),
        "orc_ct_level": (i32, [vp]),
        "orc_ct_scale": (dbl, [vp]),
        "orc_ct_degree": (i32, [vp]),
        "orc_ct_export": (None, [vp, P(u64)]),
        "orc_ct_import": (vp, [vp, P(u64), i32, dbl]),
        "orc_add": (vp, [vp, vp, vp]),
        "orc_sub": (vp, [vp, vp, vp]),
        "orc_drop": (vp, [vp, vp, i32]),
        "orc_mul_plain": (vp, [vp, vp, P(i64), dbl]),
        "orc_mul_int": (vp, [vp, vp, i64]),
        "orc_tensor": (vp, [vp, vp, vp]),
        "orc_relin": (vp, [vp, vp]),
        "orc_mul": (vp, [vp, vp, vp]),
        "orc_rescale": (vp, [vp, vp]),
        "orc_rotate": (vp, [vp, vp, i64]),
        "orc_rotate_hoisted": (None, [vp, vp, i32, P(i64), P(vp)]),
        "orc_matmul": (vp, [vp, vp, vp, i32, i32]),
        "orc_mask_slots": (None, [i32, i32, i32, P(dbl)]),
        "orc_matmul_rotations": (i32, [vp, i32, i32, P(i64), i32]),
        "orc_matmul_ex": (vp, [vp, vp, vp, i32, i32, i32, i32]),
        "orc_transpose": (vp, [vp, vp, i32, i32, i32]),
        "orc_matmul_rotations_ex": (i32, [vp, i32, i32, i32, i32, P(i64), i32]),
        "orc_transpose_rotations": (i32, [vp, i32, i32, P(i64), i32]),
        "orc_counters": (None, [vp, P(i64)]),
        "orc_reset_counters": (None, [vp]),
        "orc_sign": (vp, [vp, vp, i32, i32, i32]),
        "orc_appmax": (vp, [vp, vp, vp, i32, i32]),
        "orc_maxpool2": (vp, [vp, vp, i32, i32, i32]),
        "orc_fl_update": (vp, [vp, vp, P(vp), i32, dbl]),
        "orc_gd_numerators": (None, [i32, P(i64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def u64p(a):
    return _p(a, C.c_uint64)


def i64p(a):
    return _p(a, C.c_int64)


def f64p(a):
    return _p(a, C.c_double)


# --------------------------------------------------------------------------
# free functions
# --------------------------------------------------------------------------
def mulmod(a: int, b: int, q: int) -> int:
    return lib().orc_mulmod(a, b, q)


def is_prime(n: int) -> bool:
    return bool(lib().orc_is_prime(n))


def chacha20_block(key_words, counter, nonce_words):
    k = (C.c_uint32 * 8)(*key_words)
    n = (C.c_uint32 * 3)(*nonce_words)
    o = (C.c_uint32 * 16)()
    lib().orc_chacha20_block(k, counter, n, o)
    return list(o)


def word(seed, purpose, index, w):
    return lib().orc_word(seed, purpose, index, w)


def gauss_table():
    o = np.zeros(19, np.uint64)
    lib().orc_gauss_table(u64p(o))
    return o


def sample_ternary(seed, purpose, index, n):
    o = np.zeros(n, np.int64)
    lib().orc_sample_ternary(seed, purpose, index, n, i64p(o))
    return o


def sample_gauss(seed, purpose, index, n):
    o = np.zeros(n, np.int64)
    lib().orc_sample_gauss(seed, purpose, index, n, i64p(o))
    return o


def sample_uniform(seed, purpose, index, q, n):
    o = np.zeros(n, np.uint64)
    lib().orc_sample_uniform(seed, purpose, index, q, n, u64p(o))
    return o


def gd_numerators(d: int) -> list:
    """numerators of g_d's coefficients of x, x^3, ..., x^(2d+1), each over 2^(2d-1)"""
    o = np.zeros(d + 1, np.int64)
    lib().orc_gd_numerators(d, i64p(o))
    return [int(x) for x in o]


def mask_slots(kind: int, h: int, k: int) -> np.ndarray:
    o = np.zeros(h * h, np.float64)
    lib().orc_mask_slots(kind, h, k, f64p(o))
    return o


# --------------------------------------------------------------------------
# context and ciphertexts
# --------------------------------------------------------------------------
class Ct:
    def __init__(self, ctx: "Ctx", ptr):
        if not ptr:
            raise ValueError("oracle operation failed (level, shape or degree)")
        self.ctx, self.ptr = ctx, ptr

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_ct_free(self.ptr)
            self.ptr = None

    @property
    def level(self):
        return lib().orc_ct_level(self.ptr)

    @property
    def scale(self):
        return lib().orc_ct_scale(self.ptr)

    @property
    def degree(self):
        return lib().orc_ct_degree(self.ptr)

    def export(self) -> np.ndarray:
        """coefficient-domain residues [deg+1][level+1][N]"""
        o = np.zeros((self.degree + 1, self.level + 1, self.ctx.n), np.uint64)
        lib().orc_ct_export(self.ptr, u64p(o))
        return o


class Ctx:
    def __init__(self, log_n, q_bits, p_bits, alpha, log_scale, seed, threads=0):
        self.log_n, self.n = log_n, 1 << log_n
        self.q_bits, self.p_bits = list(q_bits), list(p_bits)
        self.alpha, self.log_scale, self.seed = alpha, log_scale, seed
        qb = (C.c_int * len(q_bits))(*q_bits)
        pb = (C.c_int * len(p_bits))(*p_bits)
        self.ptr = lib().orc_create(log_n, len(q_bits), qb, len(p_bits), pb, alpha, float(log_scale), seed, threads)
        if not self.ptr:
            raise ValueError("bad parameters")
        m = np.zeros(len(q_bits) + len(p_bits), np.uint64)
        lib().orc_moduli(self.ptr, u64p(m))
        self.moduli = [int(x) for x in m]
        self.q = self.moduli[: len(q_bits)]
        self.p = self.moduli[len(q_bits):]
        self.max_level = len(q_bits) - 1

    @classmethod
    def from_params(cls, prm, threads=0):
        return cls(prm.log_n, prm.q_bits, prm.p_bits, prm.alpha, prm.log_scale, prm.seed, threads)

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_destroy(self.ptr)
            self.ptr = None

    @property
    def scale(self):
        return 2.0 ** self.log_scale

    def psi(self, i):
        return lib().orc_psi(self.ptr, i)

    # primitives
    def poly_mul(self, mi, a, b):
        a = np.ascontiguousarray(a, np.uint64)
        b = np.ascontiguousarray(b, np.uint64)
        o = np.zeros(self.n, np.uint64)
        lib().orc_poly_mul(self.ptr, mi, u64p(a), u64p(b), u64p(o))
        return o

    def eval_bitrev(self, mi, a):
        a = np.ascontiguousarray(a, np.uint64)
        o = np.zeros(self.n, np.uint64)
        lib().orc_eval_bitrev(self.ptr, mi, u64p(a), u64p(o))
        return o

    def base_conv(self, src_idx, dst_idx, x):
        x = np.ascontiguousarray(x, np.uint64)
        s = (C.c_int * len(src_idx))(*src_idx)
        o = np.zeros(self.n, np.uint64)
        lib().orc_base_conv(self.ptr, len(src_idx), s, dst_idx, u64p(x), u64p(o))
        return o

    def encode(self, vals, scale=None):
        v = np.ascontiguousarray(vals, np.float64)
        o = np.zeros(self.n, np.int64)
        tie = lib().orc_encode(self.ptr, f64p(v), len(v), float(scale or self.scale), i64p(o))
        return o, tie

    def decode(self, coeffs, scale):
        c = np.ascontiguousarray(coeffs, np.float64)
        o = np.zeros(self.n // 2, np.float64)
        lib().orc_decode(self.ptr, f64p(c), float(scale), f64p(o))
        return o

    # ciphertexts
    def encrypt_coeffs(self, m, level, scale, nonce):
        m = np.ascontiguousarray(m, np.int64)
        return Ct(self, lib().orc_encrypt_coeffs(self.ptr, i64p(m), level, float(scale), nonce))

    def encrypt(self, vals, level=None, nonce=0):
        v = np.ascontiguousarray(np.ravel(vals), np.float64)
        lvl = self.max_level if level is None else level
        return Ct(self, lib().orc_encrypt(self.ptr, f64p(v), len(v), lvl, nonce))

    def decrypt(self, ct: Ct, n=None):
        o = np.zeros(self.n // 2, np.float64)
        rc = lib().orc_decrypt(self.ptr, ct.ptr, f64p(o))
        if rc != 0:
            raise ValueError("plaintext exceeds the two-limb CRT range")
        return o if n is None else o[:n]

    def decrypt_coeffs(self, ct: Ct):
        o = np.zeros(self.n, np.float64)
        rc = lib().orc_decrypt_coeffs(self.ptr, ct.ptr, f64p(o))
        if rc != 0:
            raise ValueError("plaintext exceeds the two-limb CRT range")
        return o

    def ct_import(self, arr, level, scale):
        a = np.ascontiguousarray(arr, np.uint64)
        return Ct(self, lib().orc_ct_import(self.ptr, u64p(a), level, float(scale)))

    def add(self, a, b):
        return Ct(self, lib().orc_add(self.ptr, a.ptr, b.ptr))

    def sub(self, a, b):
        return Ct(self, lib().orc_sub(self.ptr, a.ptr, b.ptr))

    def drop(self, a, level):
        return Ct(self, lib().orc_drop(self.ptr, a.ptr, level))

    def mul_plain(self, a, pt, pt_scale):
        pt = np.ascontiguousarray(pt, np.int64)
        return Ct(self, lib().orc_mul_plain(self.ptr, a.ptr, i64p(pt), float(pt_scale)))

    def mul_int(self, a, k):
        return Ct(self, lib().orc_mul_int(self.ptr, a.ptr, int(k)))

    def tensor(self, a, b):
        return Ct(self, lib().orc_tensor(self.ptr, a.ptr, b.ptr))

    def relin(self, a):
        return Ct(self, lib().orc_relin(self.ptr, a.ptr))

    def mul(self, a, b):
        return Ct(self, lib().orc_mul(self.ptr, a.ptr, b.ptr))

    def rescale(self, a):
        return Ct(self, lib().orc_rescale(self.ptr, a.ptr))

    def rotate(self, a, k):
        return Ct(self, lib().orc_rotate(self.ptr, a.ptr, int(k)))

    def rotate_hoisted(self, a, ks):
        ks = np.ascontiguousarray(ks, np.int64)
        out = (C.c_void_p * len(ks))()
        lib().orc_rotate_hoisted(self.ptr, a.ptr, len(ks), i64p(ks), out)
        return [Ct(self, out[i]) for i in range(len(ks))]

    def matmul(self, a, b, h, relin_mode=RELIN_EACH):
        return Ct(self, lib().orc_matmul(self.ptr, a.ptr, b.ptr, h, relin_mode))

    def matmul_ex(self, a, b, h, t=None, beta=1, mode=RELIN_EACH):
        """Alg. 3 (t = h) / HE-RMatMult (Alg. 6, t < h) on beta matrices packed by iota_beta"""
        return Ct(self, lib().orc_matmul_ex(self.ptr, a.ptr, b.ptr, h, h if t is None else t, beta, mode))

    def transpose(self, a, h, beta=1, mode=RELIN_EACH):
        return Ct(self, lib().orc_transpose(self.ptr, a.ptr, h, beta, mode))

    def matmul_rotations_ex(self, h, t, beta=1, mode=RELIN_EACH):
        o = np.zeros(8192, np.int64)
        n = lib().orc_matmul_rotations_ex(self.ptr, h, t, beta, mode, i64p(o), 8192)
        return sorted(int(x) for x in o[:n])

    def transpose_rotations(self, h, beta=1):
        o = np.zeros(8192, np.int64)
        n = lib().orc_transpose_rotations(self.ptr, h, beta, i64p(o), 8192)
        return sorted(int(x) for x in o[:n])

    def matmul_rotations(self, h, mode=RELIN_EACH):
        o = np.zeros(8192, np.int64)
        n = lib().orc_matmul_rotations(self.ptr, h, mode, i64p(o), 8192)
        return sorted(int(x) for x in o[:n])

    def counters(self):
        o = np.zeros(6, np.int64)
        lib().orc_counters(self.ptr, i64p(o))
        return dict(zip(["rot", "keyswitch", "mul_pt", "mul_ct", "add", "rescale"], (int(x) for x in o)))

    def reset_counters(self):
        lib().orc_reset_counters(self.ptr)

    def appmax(self, a, b, d, k):
        return Ct(self, lib().orc_appmax(self.ptr, a.ptr, b.ptr, d, k))

    def maxpool2(self, x, h, d, k):
        return Ct(self, lib().orc_maxpool2(self.ptr, x.ptr, h, d, k))

    def fl_update(self, w, grads, coeff):
        arr = (C.c_void_p * len(grads))(*[g.ptr for g in grads])
        return Ct(self, lib().orc_fl_update(self.ptr, w.ptr, arr, len(grads), float(coeff)))

    def sign(self, x, d, k, relu=False):
        return Ct(self, lib().orc_sign(self.ptr, x.ptr, d, k, int(bool(relu))))
