"""CPU oracle for the negacyclic NTT -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's cpu_baseline leg may
import this package. It wraps liboracle.so (plain C, 128-bit products and '%'
reductions; see ntt_oracle.h for the definitions and the readings of the
paper's listings) and shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "ntt_oracle.c")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (OpenMP for the batched drivers)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None
_lib_path = None  # None: the default build


def use_library(path=None):
    """Load another build of the oracle (the mutation test's planted
    mistakes); None returns to the default build."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def build_variant(out_path: str, defines=()) -> str:
    """Compile ntt_oracle.c with extra -D definitions into out_path."""
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", out_path, _SRC] +
                          [f"-D{d}" for d in defines])
    return out_path


def lib():
    global _lib
    if _lib is None:
        if _lib_path is None and not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_lib_path or _SO)
        u64, u32, p64 = ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)
        sig = {
            "orc_addmod": (u64, [u64, u64, u64]),
            "orc_submod": (u64, [u64, u64, u64]),
            "orc_mulmod": (u64, [u64, u64, u64]),
            "orc_powmod": (u64, [u64, u64, u64]),
            "orc_invmod": (u64, [u64, u64]),
            "orc_smallest_qnr": (u64, [u64]),
            "orc_psi": (u64, [u64, u32]),
            "orc_bit_reverse": (None, [p64, u32]),
            "orc_ntt_forward": (None, [p64, u32, u64, u64]),
            "orc_ntt_inverse": (None, [p64, u32, u64, u64]),
            "orc_ntt_direct": (None, [p64, p64, u32, u64, u64]),
            "orc_ntt_direct_coeff": (u64, [p64, u32, u64, u64, u32]),
            "orc_intt_direct_coeff": (u64, [p64, u32, u64, u64, u32]),
            "orc_pointwise": (None, [p64, p64, p64, u32, u64]),
            "orc_negacyclic_mul": (None, [p64, p64, p64, u32, u64]),
            "orc_negacyclic_coeff": (u64, [p64, p64, u32, u64, u32]),
            "orc_omega": (u64, [u64, u32]),
            "orc_ntt_cyclic_forward": (None, [p64, u32, u64, u64]),
            "orc_ntt_cyclic_inverse": (None, [p64, u32, u64, u64]),
            "orc_ntt_cyclic_direct_coeff": (u64, [p64, u32, u64, u64, u32]),
            "orc_pease_cyclic_forward": (None, [p64, u32, u64, u64]),
            "orc_stockham_cyclic_forward": (None, [p64, u32, u64, u64]),
            "orc_ntt_forward_batch": (ctypes.c_int, [p64, u32, u32, u32, p64, p64, ctypes.c_int]),
            "orc_ntt_inverse_batch": (ctypes.c_int, [p64, u32, u32, u32, p64, p64, ctypes.c_int]),
            "orc_pointwise_batch": (ctypes.c_int, [p64, p64, p64, u32, u32, u32, p64, ctypes.c_int]),
            "orc_tensor_batch": (ctypes.c_int, [p64, p64, p64, u32, u32, u32, p64, ctypes.c_int]),
            "orc_base_conv_batch": (ctypes.c_int, [p64, p64, u32, u32, p64, u32, p64, u32, ctypes.c_int]),
            "orc_mod_down_batch": (ctypes.c_int, [p64, p64, p64, u32, u32, p64, u32, p64, u32, ctypes.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _u64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


# ---- scalar helpers ----------------------------------------------------------
def mulmod(a, b, q):
    return int(lib().orc_mulmod(a, b, q))


def powmod(a, e, q):
    return int(lib().orc_powmod(a, e, q))


def invmod(a, q):
    return int(lib().orc_invmod(a, q))


def smallest_qnr(q):
    return int(lib().orc_smallest_qnr(q))


def psi(q, N):
    return int(lib().orc_psi(q, N))


# ---- single-vector transforms (return new arrays) ------------------------------
def bit_reverse(x):
    y = _u64(x).copy()
    lib().orc_bit_reverse(_p(y), y.size)
    return y


def ntt_forward(x, q, root=None):
    y = _u64(x).copy()
    lib().orc_ntt_forward(_p(y), y.size, q, root if root is not None else psi(q, y.size))
    return y


def ntt_inverse(X, q, root=None):
    y = _u64(X).copy()
    lib().orc_ntt_inverse(_p(y), y.size, q, root if root is not None else psi(q, y.size))
    return y


def ntt_direct(x, q, root=None):
    x = _u64(x)
    X = np.empty_like(x)
    lib().orc_ntt_direct(_p(x), _p(X), x.size, q, root if root is not None else psi(q, x.size))
    return X


def ntt_direct_coeff(x, q, k, root=None):
    x = _u64(x)
    return int(lib().orc_ntt_direct_coeff(_p(x), x.size, q, root if root is not None else psi(q, x.size), k))


def intt_direct_coeff(X, q, j, root=None):
    X = _u64(X)
    return int(lib().orc_intt_direct_coeff(_p(X), X.size, q, root if root is not None else psi(q, X.size), j))


def pointwise(a, b, q):
    a, b = _u64(a), _u64(b)
    c = np.empty_like(a)
    lib().orc_pointwise(_p(a), _p(b), _p(c), a.size, q)
    return c


def negacyclic_mul(a, b, q):
    a, b = _u64(a), _u64(b)
    c = np.empty_like(a)
    lib().orc_negacyclic_mul(_p(a), _p(b), _p(c), a.size, q)
    return c


def negacyclic_coeff(a, b, q, k):
    a, b = _u64(a), _u64(b)
    return int(lib().orc_negacyclic_coeff(_p(a), _p(b), a.size, q, k))


# ---- cyclic transform (Eq. 3) ------------------------------------------------------
def omega(q, N):
    return int(lib().orc_omega(q, N))


def cyclic_forward(x, q, root=None):
    y = _u64(x).copy()
    lib().orc_ntt_cyclic_forward(_p(y), y.size, q, root if root is not None else omega(q, y.size))
    return y


def cyclic_inverse(X, q, root=None):
    y = _u64(X).copy()
    lib().orc_ntt_cyclic_inverse(_p(y), y.size, q, root if root is not None else omega(q, y.size))
    return y


def pease_forward(x, q, root=None):
    y = _u64(x).copy()
    lib().orc_pease_cyclic_forward(_p(y), y.size, q, root if root is not None else omega(q, y.size))
    return y


def stockham_forward(x, q, root=None):
    y = _u64(x).copy()
    lib().orc_stockham_cyclic_forward(_p(y), y.size, q, root if root is not None else omega(q, y.size))
    return y


def cyclic_direct_coeff(x, q, k, root=None):
    x = _u64(x)
    return int(lib().orc_ntt_cyclic_direct_coeff(_p(x), x.size, q, root if root is not None else omega(q, x.size), k))


# ---- batched [B][L][N] drivers (in place on a copy) ------------------------------
def _roots(moduli, N):
    return _u64([psi(int(q), N) for q in moduli])


def ntt_forward_batch(x, moduli, nthreads=0):
    y = _u64(x).copy()
    B, L, N = y.shape
    q = _u64(moduli)
    r = _roots(moduli, N)
    used = lib().orc_ntt_forward_batch(_p(y), B, L, N, _p(q), _p(r), nthreads)
    return y, used


def ntt_inverse_batch(X, moduli, nthreads=0):
    y = _u64(X).copy()
    B, L, N = y.shape
    q = _u64(moduli)
    r = _roots(moduli, N)
    used = lib().orc_ntt_inverse_batch(_p(y), B, L, N, _p(q), _p(r), nthreads)
    return y, used


def pointwise_batch(a, b, moduli, nthreads=0):
    a, b = _u64(a), _u64(b)
    c = np.empty_like(a)
    B, L, N = a.shape
    q = _u64(moduli)
    used = lib().orc_pointwise_batch(_p(a), _p(b), _p(c), B, L, N, _p(q), nthreads)
    return c, used


# ---- HE steps (definitions in ntt_oracle.h) -----------------------------------------
def tensor_product(a, b, moduli, nthreads=0):
    """a, b: [B][2][L][N] ciphertexts in the evaluation domain -> d [B][3][L][N]."""
    a, b = _u64(a), _u64(b)
    B, two, L, N = a.shape
    assert two == 2 and b.shape == a.shape and len(moduli) == L
    d = np.empty((B, 3, L, N), np.uint64)
    lib().orc_tensor_batch(_p(a), _p(b), _p(d), B, L, N, _p(_u64(moduli)), nthreads)
    return d


def base_conv(x, src, dst, nthreads=0):
    """x: [B][L][N] residues over src (L primes) -> [B][K][N] over dst (K primes)."""
    x = _u64(x)
    B, L, N = x.shape
    assert len(src) == L
    out = np.empty((B, len(dst), N), np.uint64)
    lib().orc_base_conv_batch(_p(x), _p(out), B, N, _p(_u64(src)), L, _p(_u64(dst)), len(dst), nthreads)
    return out


def mod_down(x, y, src, dst, nthreads=0):
    """x: [B][L][N] over src, y: [B][K][N] over dst -> (y - conv(x)) * S^-1 over dst."""
    x, y = _u64(x), _u64(y)
    B, L, N = x.shape
    assert len(src) == L and y.shape == (B, len(dst), N)
    out = np.empty_like(y)
    lib().orc_mod_down_batch(_p(x), _p(y), _p(out), B, N, _p(_u64(src)), L, _p(_u64(dst)), len(dst), nthreads)
    return out
