"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only; GPU code is
not instrumented): the oracle, built with both sanitizers, runs a subset of its pins in a
child process with the sanitizer runtimes preloaded, and the library's host number theory and
encoder (csrc/host_math.hpp), built the same way into a small driver, must agree with the
oracle's primes and encoding.  Any sanitizer report ends the child with a nonzero status."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle as O
from paper_2207_04620_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _runtime(name):
    path = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return os.path.realpath(path)


@pytest.fixture(scope="module")
def host_driver():
    exe = os.path.join(ROOT, "oracle", "_build", "host_math_check_san")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                           "-o", exe, os.path.join(ROOT, "tests", "host_math_check.cpp")])
    return exe


def test_oracle_pins_under_sanitizers():
    lib = O.build_sanitized()
    syms = subprocess.check_output(["nm", "-D", "--undefined-only", lib], text=True)
    assert "__asan_" in syms and "__ubsan_" in syms  # the instrumented build is the one loaded
    env = dict(os.environ, ORACLE_LIB=lib, **SAN_ENV,
               LD_PRELOAD=" ".join([_runtime("libasan.so"), _runtime("libubsan.so")]))
    subset = ("mulmod or is_prime or psi or poly_mul or eval_bitrev or chacha or stream_word or gauss "
              "or sampler or base_conversion or encode or decode or slotwise or roundtrip or rotation_matches "
              "or hoisted or mul_relin or add_level or fig2 or eq2 or matmul_decrypts or relin_once "
              "or gd_numerators or g4_decrypts or transpose_decrypts or appmax or fl_update or noise_model")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", subset],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail


@pytest.mark.parametrize("prm", [I.C1P, I.C2, I.C3, I.C4], ids=lambda p: p.name)
def test_host_primes_match_oracle(host_driver, prm):
    out = subprocess.run([host_driver, "primes", str(prm.log_n), *map(str, prm.q_bits + prm.p_bits)],
                         capture_output=True, text=True, timeout=120, env=dict(os.environ, **SAN_ENV))
    assert out.returncode == 0, out.stderr[-2000:]
    got = [int(x) for x in out.stdout.split()]
    assert got == O.Ctx.from_params(prm).moduli


@pytest.mark.parametrize("log_n,n_vals", [(10, 64), (12, 2048), (15, 4096)])
def test_host_encoder_matches_oracle(host_driver, log_n, n_vals):
    vals = np.random.default_rng(log_n).uniform(-1, 1, n_vals)
    out = subprocess.run([host_driver, "encode", str(log_n), "40"], input="\n".join(repr(float(v)) for v in vals),
                         capture_output=True, text=True, timeout=300, env=dict(os.environ, **SAN_ENV))
    assert out.returncode == 0, out.stderr[-2000:]
    lines = out.stdout.split()
    n = 1 << log_n
    tie = float(lines[0])
    m = np.array([int(x) for x in lines[1:1 + n]], np.int64)
    dec = np.array([float(x) for x in lines[1 + n:1 + n + n // 2]])
    c = O.Ctx(log_n, [50, 40], [50], 1, 40.0, 1)
    want, otie = c.encode(vals)
    assert tie > 1e-9 and np.array_equal(m, want)
    assert np.abs(dec - np.tile(vals, n // 2 // n_vals)).max() < 1e-9
