"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds input generation only: a counter-based random generator,
rejection sampling of uniform residues, the prime sets the workloads name,
the uneven job mix of the batched workload and the arrival process of the
serving workload. It contains none of the transform arithmetic, and neither
the oracle nor the GPU library is imported here.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; the constants are Stafford's "Mix13"
variant as used in the public-domain splitmix64.c). Output k of the stream
with seed s mixes s + (k+1)*0x9E3779B97F4A7C15.

Residues: a coefficient mod q is the next output shifted right by
64 - bitlen(q), drawn again while >= q (uniform on [0, q)). Streams are
consumed in memory order [poly][limb][coef].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1
BASE_SEED = 20240518


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream with `seed`."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + k * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_scalar(seed: int, k: int) -> int:
    """Output k of the stream, in Python integers (cross-check of the above)."""
    z = (seed + (k + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class Stream:
    """A SplitMix64 stream with a position counter."""

    def __init__(self, seed: int):
        self.seed = seed & MASK64
        self.pos = 0

    def raw(self, count: int) -> np.ndarray:
        out = splitmix64(self.seed, self.pos, count)
        self.pos += count
        return out

    def uniform_mod(self, q: int, n: int) -> np.ndarray:
        """n residues uniform on [0, q) by rejection on the top bitlen(q) bits."""
        shift = np.uint64(64 - q.bit_length())
        out = np.empty(n, dtype=np.uint64)
        filled = 0
        while filled < n:
            need = n - filled
            draw = need + need // 16 + 64
            cand = splitmix64(self.seed, self.pos, draw) >> shift
            ok = np.flatnonzero(cand < np.uint64(q))
            take = min(need, ok.size)
            out[filled:filled + take] = cand[ok[:take]]
            filled += take
            # advance past the last candidate consumed (or the whole draw)
            self.pos += int(ok[take - 1]) + 1 if take == need else draw
        return out

    def uniform_int(self, lo: int, hi: int) -> int:
        """One integer uniform on [lo, hi] (rejection, no modulo bias)."""
        span = hi - lo + 1
        bits = max(1, (span - 1).bit_length())
        while True:
            v = int(self.raw(1)[0]) >> (64 - bits)
            if v < span:
                return lo + v

    def uniform01(self, count: int) -> np.ndarray:
        """count doubles uniform on [0, 1) from the top 53 bits."""
        return (self.raw(count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def poly_batch(seed: int, batch: int, moduli, N: int, dtype=np.uint64) -> np.ndarray:
    """A [batch][L][N] array, limb l uniform on [0, moduli[l])."""
    s = Stream(seed)
    L = len(moduli)
    out = np.empty((batch, L, N), dtype=np.uint64)
    for b in range(batch):
        for l, q in enumerate(moduli):
            out[b, l] = s.uniform_mod(int(q), N)
    return out.astype(dtype)


# --------------------------------------------------------------------------
# Prime sets named by the workloads: the largest primes below 2^bits that are
# 1 mod 2^s. Primality by Miller-Rabin with the first 12 prime bases, which is
# deterministic for every n < 3.3e24 (so for all 64-bit n).
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(bits: int, s: int, count: int) -> list[int]:
    """The `count` largest primes q < 2^bits with q = 1 mod 2^s, descending."""
    out = []
    step = 1 << s
    q = ((1 << bits) - 1) // step * step + 1
    if q >= 1 << bits:
        q -= step
    while len(out) < count and q > step:
        if is_prime(q):
            out.append(q)
        q -= step
    return out


# --------------------------------------------------------------------------
# Workload definitions (sizes from the evaluation configurations).
Q_SMALL = 998244353  # 119 * 2^23 + 1, the 32-bit prime of the single-NTT case


@dataclass
class Workload:
    name: str
    N: int
    moduli: list
    batch: int
    word: int = 64
    seed: int = BASE_SEED
    note: str = ""


def workload_single_u32() -> Workload:
    return Workload("single_ntt_n1024_u32", 1024, [Q_SMALL], 1, word=32, seed=BASE_SEED + 0,
                    note="one negacyclic NTT+INTT, N=1024, q=998244353, uint32")


def workload_ct_n14() -> Workload:
    return Workload("ciphertext_n16384_l8", 1 << 14, ntt_primes(60, 15, 8), 2, seed=BASE_SEED + 1,
                    note="one ciphertext: 2 polys x 8 limbs, N=2^14, q=1 mod 2^15")


def workload_polymul_n16() -> Workload:
    return Workload("polymul_n65536_l24", 1 << 16, ntt_primes(60, 17, 24), 4, seed=BASE_SEED + 2,
                    note="2 ciphertexts x 2 components x 24 limbs, N=2^16, q=1 mod 2^17")


@dataclass
class Job:
    N: int
    L: int
    op: str = "ntt"          # "ntt" (forward) or "polymul"
    arrival_s: float = 0.0


def batched_jobs(seed: int = BASE_SEED + 3, count: int = 256, logn_lo: int = 12, logn_hi: int = 16,
                 l_max: int = 32) -> list[Job]:
    """The uneven batch: N uniform over {2^logn_lo..2^logn_hi}, L uniform on 1..l_max."""
    s = Stream(seed)
    jobs = []
    for _ in range(count):
        N = 1 << s.uniform_int(logn_lo, logn_hi)
        L = s.uniform_int(1, l_max)
        jobs.append(Job(N, L))
    return jobs


def batched_primes() -> list[int]:
    """32 primes, 1 mod 2^17, so every N up to 2^16 is supported by every limb."""
    return ntt_primes(60, 17, 32)


def serving_primes() -> list[int]:
    """40 primes, 1 mod 2^18, so every N up to 2^17 is supported by every limb."""
    return ntt_primes(60, 18, 40)


def serving_trace(seed: int = BASE_SEED + 4, count: int = 2000, rate_per_s: float = 2000.0,
                  logn_lo: int = 12, logn_hi: int = 17, l_max: int = 40,
                  polymul_frac: float = 0.5) -> list[Job]:
    """Poisson arrivals (exponential gaps) of forward-NTT and poly-mult jobs."""
    s = Stream(seed)
    t = 0.0
    jobs = []
    for _ in range(count):
        u = float(s.uniform01(1)[0])
        t += -math.log1p(-u) / rate_per_s
        N = 1 << s.uniform_int(logn_lo, logn_hi)
        L = s.uniform_int(1, l_max)
        op = "polymul" if float(s.uniform01(1)[0]) < polymul_frac else "ntt"
        jobs.append(Job(N, L, op, t))
    return jobs
