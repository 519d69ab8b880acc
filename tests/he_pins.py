"""Pins of the oracle's HE steps (tensor product, basis conversion, ModDown)
against the Chinese remainder theorem and ring algebra, computed with Python
integers; none of them calls the oracle's own formula a second time.

Each check returns a list of the pins that failed (empty when all hold), so
the same battery serves the direct tests and the mutation test."""
import numpy as np

import oracle
import seeded_inputs as si


def crt(res, moduli):
    """The integer in [0, prod(moduli)) with the given residues (Garner's
    mixed-radix reconstruction, unrelated to the shat form of conversion)."""
    x, M = 0, 1
    for r, m in zip(res, moduli):
        k = ((int(r) - x) * pow(M, -1, m)) % m
        x += k * M
        M *= m
    return x


def prod(ms):
    p = 1
    for m in ms:
        p *= int(m)
    return p


def wide(s, bits):
    """A random integer of `bits` bits from 64-bit draws of the stream."""
    v = 0
    for w in s.raw((bits + 63) // 64):
        v = (v << 64) | int(w)
    return v


def check_tensor(seed=5, N=32, moduli=(si.Q_SMALL, 7681)):
    s = si.Stream(seed)
    L = len(moduli)
    a = np.stack([np.stack([[s.uniform_mod(q, N) for q in moduli] for _ in range(2)])])
    b = np.stack([np.stack([[s.uniform_mod(q, N) for q in moduli] for _ in range(2)])])
    d = oracle.tensor_product(a, b, list(moduli))
    failed = []
    for l, q in enumerate(moduli):
        sk = [int(v) for v in s.uniform_mod(q, N)]
        for n in range(N):
            a0, a1 = int(a[0, 0, l, n]), int(a[0, 1, l, n])
            b0, b1 = int(b[0, 0, l, n]), int(b[0, 1, l, n])
            lhs = (a0 + a1 * sk[n]) * (b0 + b1 * sk[n]) % q
            rhs = (int(d[0, 0, l, n]) + int(d[0, 1, l, n]) * sk[n] + int(d[0, 2, l, n]) * sk[n] ** 2) % q
            if lhs != rhs or any(int(d[0, c, l, n]) >= q for c in range(3)):
                failed.append("tensor: decryption identity")
                return failed
    if L and int(d[0, 0, 0, 0]) != int(a[0, 0, 0, 0]) * int(b[0, 0, 0, 0]) % moduli[0]:
        failed.append("tensor: d0 = a0 b0")
    return failed


def check_base_conv(seed=6, N=24, L=5, K=4, bits=60):
    ps = si.ntt_primes(bits, 17, L + K)
    src, dst = ps[:L], ps[L:]
    S = prod(src)
    s = si.Stream(seed)
    # the first coefficients are 0, 1, S-1 and a value just above S/2; the
    # rest come from wide random integers reduced mod S
    Xs = [0, 1, S - 1, S // 2 + 1][:N]
    while len(Xs) < N:
        Xs.append(wide(s, 64 * (L + 1)) % S)
    x = np.array([[[X % q for X in Xs] for q in src]], np.uint64)
    out = oracle.base_conv(x, src, dst)
    failed, alphas = [], set()
    for n, X in enumerate(Xs):
        got = [int(out[0, j, n]) for j in range(K)]
        hits = [a for a in range(L) if all(got[j] == (X + a * S) % t for j, t in enumerate(dst))]
        if len(hits) != 1:
            failed.append("conv: X + alpha S for one alpha < L")
            break
        alphas.add(hits[0])
    if not failed and len(alphas) < 2:
        failed.append("conv: alpha never varies")
    # one source prime: conv is the plain reduction X mod t_j
    x1 = np.array([[[X % src[0] for X in Xs]]], np.uint64)
    o1 = oracle.base_conv(x1, src[:1], dst)
    if any(int(o1[0, j, n]) != (Xs[n] % src[0]) % t for j, t in enumerate(dst) for n in range(N)):
        failed.append("conv: one source prime")
    return failed


def check_mod_down(seed=7, N=20, L=3, K=5, bits=60):
    ps = si.ntt_primes(bits, 17, L + K)
    src, dst = ps[:L], ps[L:]          # divide by S = prod(src), keep the dst residues
    S, T = prod(src), prod(dst)
    s = si.Stream(seed)
    Xs, Es = [], []
    for n in range(N):
        X = wide(s, 64 * (K + 1)) % T
        E = 0 if n < 4 else wide(s, 64 * (L + 1)) % S
        Xs.append(X)
        Es.append(E)
    Z = [X * S + E for X, E in zip(Xs, Es)]
    x = np.array([[[z % q for z in Z] for q in src]], np.uint64)
    y = np.array([[[z % t for z in Z] for t in dst]], np.uint64)
    out = oracle.mod_down(x, y, src, dst)
    failed = []
    for n in range(N):
        got = [int(out[0, j, n]) for j in range(K)]
        hits = [b for b in range(L) if all(got[j] == (Xs[n] - b) % t for j, t in enumerate(dst))]
        if len(hits) != 1 or (Es[n] == 0 and hits[0] != 0):
            failed.append("moddown: (X S + E) -> X - beta, exact for E = 0")
            break
    return failed


def battery():
    return check_tensor() + check_base_conv() + check_mod_down()
