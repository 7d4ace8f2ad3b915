"""Minimal Goldbach prime of even n beyond 64 bits -- TEST INFRASTRUCTURE ONLY.

The paper's arbitrary-precision checker (section "Arbitrary Precision
Checker") scans small primes p and tests q = n - p with Miller-Rabin.  This
is that scan written out with Python integers, returning the first p in
ascending order (the minimal p in the sense below):

  * p runs over the odd primes 3, 5, 7, ... (n >= 6; 4 = 2 + 2);
  * q = n - p counts as prime when it passes the strong probable-prime test
    to each of the 25 prime bases 2, 3, 5, ..., 97 (the paper uses 25
    Miller-Rabin rounds).  A q that fails one base is certainly composite,
    so every p below the one returned certainly fails; the returned q is a
    probable prime (deterministic below 3.3e24 already with the first 12
    bases).

Only tests, the smoke check and the benchmark's CPU leg may import this.
"""
from __future__ import annotations

BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71,
         73, 79, 83, 89, 97)


def strong_probable_prime(q: int, a: int) -> bool:
    """q odd > a: a^d = 1 or a^(d 2^r) = -1 (mod q) for some r < s, q - 1 = d 2^s."""
    d, s = q - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    x = pow(a, d, q)
    if x == 1 or x == q - 1:
        return True
    for _ in range(s - 1):
        x = x * x % q
        if x == q - 1:
            return True
    return False


def probable_prime(q: int) -> bool:
    if q < 2:
        return False
    for a in BASES:
        if q == a:
            return True
        if q % a == 0:
            return False
    return all(strong_probable_prime(q, a) for a in BASES)


def _odd_primes(limit: int):
    sieve = bytearray([1]) * (limit + 1)
    sieve[0:2] = b"\x00\x00"
    for i in range(2, int(limit ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = bytearray(len(range(i * i, limit + 1, i)))
    return [i for i in range(3, limit + 1, 2) if sieve[i]]


def pmin_big(n: int, limit: int = 1 << 20) -> int:
    """Smallest odd prime p <= limit with n - p a probable prime (n even >= 6),
    2 for n = 4, 0 if none up to the limit."""
    if n % 2 or n < 4:
        raise ValueError("n must be even and at least 4")
    if n == 4:
        return 2
    for p in _odd_primes(min(limit, n // 2)):
        if probable_prime(n - p):
            return p
    return 0
