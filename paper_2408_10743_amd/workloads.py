"""Seeded synthetic inputs shaped like the paper's workloads.

The paper's data sets (random normalizer matrices) are not public, so the
benchmarks and tests draw codes of the same kind from a counter-free
SplitMix64 stream (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014).  This module draws bits and symbols only; it holds
none of the distance computation and is shared by the library tests and the
oracle tests alike.

Layout of the matrices (the C ABI's):
  field 2: uint8 array (m, 2n), row = x_1..x_n | z_1..z_n, entries in {0,1}
  field 4: uint8 array (k, n), entry a + 2b for the F4 symbol a + alpha*b
Bits are drawn row-major, x then z, low bit of each 64-bit draw first.
"""
import math

import numpy as np

_MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64: state += golden gamma; output = mix(state)."""

    def __init__(self, seed):
        self.state = seed & _MASK

    def next(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def bits(self, count):
        out = np.empty(count, dtype=np.uint8)
        i = 0
        while i < count:
            v = self.next()
            take = min(64, count - i)
            for b in range(take):
                out[i + b] = (v >> b) & 1
            i += take
        return out

    def uniform_int(self, lo, hi):
        """Integer in [lo, hi] (inclusive) by rejection."""
        span = hi - lo + 1
        limit = (1 << 64) - ((1 << 64) % span)
        while True:
            v = self.next()
            if v < limit:
                return lo + v % span

    def uniform01(self):
        return (self.next() >> 11) * (1.0 / (1 << 53))


def config_seed(config, index):
    return ((config & 0xFFFFFFFF) << 32) | (index & 0xFFFFFFFF)


def additive(n, m, seed):
    """m x 2n i.i.d. Bernoulli(1/2) binary symplectic generator."""
    rng = SplitMix64(seed)
    return rng.bits(m * 2 * n).reshape(m, 2 * n)


def f4_linear(n, k, seed):
    """k x n generator with i.i.d. uniform F4 entries (codes 0..3)."""
    rng = SplitMix64(seed)
    b = rng.bits(k * n * 2).reshape(k * n, 2)
    return (b[:, 0] | (b[:, 1] << 1)).astype(np.uint8).reshape(k, n)


# The five benchmark configurations --------------------------------------

def config1(index=0):
    """Plain single code: n = 20, m = 20, Bernoulli(1/2) bits."""
    return additive(20, 20, config_seed(1, index)), 2


def config2(index=0):
    """F4-linear [n=48, k=24] code with uniform symbols."""
    return f4_linear(48, 24, config_seed(2, index)), 4


def config3(index=0):
    """Plain single additive code: n = 72, m = 72, Bernoulli(1/2) bits."""
    return additive(72, 72, config_seed(3, index)), 2


def config4(count=512, index=0, n_lo=24, n_hi=96):
    """Batch of codes: n ~ U{n_lo..n_hi}; even entries additive with
    m ~ U{n-8..n+8}; odd entries F4-linear with k = n // 2."""
    rng = SplitMix64(config_seed(4, index))
    codes = []
    for i in range(count):
        n = rng.uniform_int(n_lo, n_hi)
        s = rng.next()
        if i % 2 == 0:
            m = rng.uniform_int(max(1, n - 8), n + 8)
            codes.append((additive(n, m, s), 2))
        else:
            codes.append((f4_linear(n, n // 2, s), 4))
    return codes


def config5(count, rate_hz, index=0, n_lo=16, n_hi=96):
    """Request stream: Poisson arrivals at rate_hz (exponential gaps),
    n = round(exp(U(ln n_lo, ln n_hi))), alternately additive (m = n) and
    F4-linear (k = n // 2).  Returns [(arrival_s, G, field), ...]."""
    rng = SplitMix64(config_seed(5, index))
    t = 0.0
    out = []
    for i in range(count):
        t += -math.log(1.0 - rng.uniform01()) / rate_hz
        n = int(round(math.exp(math.log(n_lo) + rng.uniform01() * (math.log(n_hi) - math.log(n_lo)))))
        s = rng.next()
        if i % 2 == 0:
            out.append((t, additive(n, n, s), 2))
        else:
            out.append((t, f4_linear(n, n // 2, s), 4))
    return out


def random_packages(P, n, seed, two_dim_fraction=1.0):
    """Random generator-matrix layout for one enumeration round: P packages
    of random rows, each of dimension 2 with probability two_dim_fraction
    (else 1).  Returns (rows (2P, 2n) uint8, dims (P,) int32); row 2i+1 is
    zero for a one-row package."""
    rng = SplitMix64(seed)
    rows = rng.bits(2 * P * 2 * n).reshape(2 * P, 2 * n)
    dims = np.empty(P, dtype=np.int32)
    for i in range(P):
        two = rng.uniform01() < two_dim_fraction
        dims[i] = 2 if two else 1
        if not two:
            rows[2 * i + 1, :] = 0
    return rows, dims


def tiny_code(seed, n_max=7, m_max=None):
    """Small random additive code for exhaustive cross-checks."""
    rng = SplitMix64(seed)
    n = rng.uniform_int(1, n_max)
    m_hi = m_max if m_max is not None else 2 * n + 1
    m = rng.uniform_int(1, m_hi)
    return additive(n, m, rng.next())


def random_stabilizer(n, k, seed):
    """Normalizer matrix (n + k) x 2n of a random [[n, k]] stabilizer code.

    The canonical code with stabilizer Z_1..Z_{n-k} has the normalizer rows
    Z_1..Z_n and X_{n-k+1}..X_n; every row is mapped by the same product of
    4n symplectic transvections x -> x + <x, v>_s v with random nonzero v,
    which preserves symplectic products, so the image is the normalizer of
    a random stabilizer code.  Rows: n - k stabilizer generators first, then
    the 2k logical operators."""
    if not 0 <= k <= n:
        raise ValueError("need 0 <= k <= n")
    rng = SplitMix64(seed)
    A = np.zeros((n + k, 2 * n), dtype=np.uint8)
    for i in range(n):
        A[i, n + i] = 1  # Z_{i+1}
    for j in range(k):
        A[n + j, n - k + j] = 1  # X_{n-k+1+j}
    order = list(range(n - k)) + list(range(n - k, n)) + list(range(n, n + k))
    A = A[order]
    for _ in range(4 * n):
        v = rng.bits(2 * n)
        if not v.any():
            continue
        # <a, v>_s = a_x . v_z + a_z . v_x (mod 2), for every row at once
        prod = ((A[:, :n].astype(np.int64) @ v[n:].astype(np.int64)) +
                (A[:, n:].astype(np.int64) @ v[:n].astype(np.int64))) & 1
        A ^= (prod[:, None].astype(np.uint8) & v[None, :])
    return A


def textbook_code(name):
    """Normalizer matrices of textbook stabilizer codes, from their Pauli
    strings (stabilizer generators, then logical operators)."""
    paulis = {
        # five-qubit code: cyclic shifts of XZZXI; logicals X^5, Z^5
        "[[5,1,3]]": ["XZZXI", "IXZZX", "XIXZZ", "ZXIXZ", "XXXXX", "ZZZZZ"],
        # Shor's nine-qubit code (degenerate: weight-2 stabilizers)
        "[[9,1,3]]": ["ZZIIIIIII", "IZZIIIIII", "IIIZZIIII", "IIIIZZIII", "IIIIIIZZI", "IIIIIIIZZ",
                      "XXXXXXIII", "IIIXXXXXX", "ZZZZZZZZZ", "XXXXXXXXX"],
        # Steane's seven-qubit code; logicals X^7, Z^7
        "[[7,1,3]]": ["IIIXXXX", "IXXIIXX", "XIXIXIX", "IIIZZZZ", "IZZIIZZ", "ZIZIZIZ", "XXXXXXX", "ZZZZZZZ"],
        # four-qubit error-detecting code; logicals XXII, XIXI, ZZII... one choice
        "[[4,2,2]]": ["XXXX", "ZZZZ", "XXII", "ZIZI", "XIXI", "ZZII"],
        # a k = 0 code (self-dual): the three-qubit GHZ state
        "[[3,0,2]]": ["XXX", "ZZI", "IZZ"],
    }[name]
    n = len(paulis[0])
    A = np.zeros((len(paulis), 2 * n), dtype=np.uint8)
    for i, p in enumerate(paulis):
        for q, ch in enumerate(p):
            A[i, q] = ch in "XY"
            A[i, n + q] = ch in "ZY"
    return A


def config_stab(index=0):
    """Random stabilizer codes shaped like the paper's larger data sets:
    n ~ U{32..64}, K/N = (n + k) / 2n ~ U[0.586, 0.758] (so K x N <= 12,416
    elements), normalizer matrix as input, field 2."""
    rng = SplitMix64(config_seed(6, index))
    n = rng.uniform_int(32, 64)
    ratio = 0.586 + (0.758 - 0.586) * rng.uniform01()
    k = max(1, min(n - 1, int(round((2 * ratio - 1) * n))))
    return random_stabilizer(n, k, rng.next()), 2
