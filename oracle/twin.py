"""Pure-Python restatement of the RAMBO oracle for tiny inputs -- TEST
INFRASTRUCTURE ONLY.

Independent of ``oracle.c`` (no shared code): Python integers for the 128-bit
hash arithmetic, Python sets for the Bloom filters (a BFU is the set of its
set bit positions). Same definitions and readings as the C oracle:
Section 2.1 (Bloom filter), Section 3 and Algorithm 1 (construction),
Section 3.3 and Algorithm 2 (query), Section 3.3.1 (sequence query).
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
P61 = (1 << 61) - 1
K = 31
CODE = {ord(c): i for i, c in enumerate("ACGT")}
CODE.update({ord(c): i for i, c in enumerate("acgt")})


def splitmix64(seed: int, n: int) -> list[int]:
    s, out = seed & MASK64, []
    for _ in range(n):
        s = (s + 0x9E3779B97F4A7C15) & MASK64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out.append(z ^ (z >> 31))
    return out


def kmer_terms(seq: bytes) -> list[int]:
    """Canonical codes of the valid 31-windows, in order."""
    out = []
    for p in range(len(seq) - K + 1):
        w = seq[p:p + K]
        if all(c in CODE for c in w):
            codes = [CODE[c] for c in w]
            fwd = 0
            for c in codes:
                fwd = fwd * 4 + c
            rc = 0
            for c in reversed(codes):
                rc = rc * 4 + (3 - c)
            out.append(min(fwd, rc))
    return out


def canon_code(x: int) -> int:
    codes = [(x >> (2 * (K - 1 - i))) & 3 for i in range(K)]
    rc = 0
    for c in reversed(codes):
        rc = rc * 4 + (3 - c)
    return min(x, rc)


class Twin:
    def __init__(self, K_docs, B, R, m, eta, seed):
        self.K, self.B, self.R, self.m, self.eta = K_docs, B, R, m, eta
        draws = iter(splitmix64(seed, 2 * R + 4 * R * eta))
        self.phi_ab = []
        for _ in range(R):
            a = 1 + next(draws) % (P61 - 1)
            b = next(draws) % P61
            self.phi_ab.append((a, b))
        self.hAC = []
        for _ in range(R * eta):
            alo, ahi, clo, chi = next(draws), next(draws), next(draws), next(draws)
            self.hAC.append(((ahi << 64) | alo, (chi << 64) | clo))
        self.bfu = [[set() for _ in range(B)] for _ in range(R)]

    def phi(self, r, d):
        a, b = self.phi_ab[r]
        return ((a * d + b) % P61) % self.B

    def h(self, r, j, x):
        A, C = self.hAC[r * self.eta + j]
        y = ((A * x + C) % (1 << 128)) >> 64
        return (y * self.m) >> 64

    def insert_terms(self, d, terms):
        for r in range(self.R):
            f = self.bfu[r][self.phi(r, d)]
            for x in terms:
                for j in range(self.eta):
                    f.add(self.h(r, j, x))

    def passes(self, r, b, x):
        f = self.bfu[r][b]
        return all(self.h(r, j, x) in f for j in range(self.eta))

    def query_terms(self, Q) -> set[int]:
        """Algorithm 2: per repetition, union of the documents of BFUs that
        hold every term; intersection across repetitions."""
        A = set(range(self.K))
        for r in range(self.R):
            G = set()
            for b in range(self.B):
                if all(self.passes(r, b, x) for x in Q):
                    G |= {d for d in range(self.K) if self.phi(r, d) == b}
            A &= G
        return A
