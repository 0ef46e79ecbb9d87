"""Pins for the oracle's GF(2^64) arithmetic, keyed hash and determinants.

Nothing here compares the oracle with itself: the checks are field axioms,
known answers, irreducibility of the modulus, published SplitMix64 outputs and
textbook determinant identities.
"""
import random

import pytest

N_RANDOM = 3000
MASK = (1 << 64) - 1
MODULUS = (1 << 64) | 0x1B  # x^64 + x^4 + x^3 + x + 1


def rnd(r):
    return r.getrandbits(64)


def test_known_answers(oracle_mod):
    O = oracle_mod
    # x^63 * x = x^64 = x^4 + x^3 + x + 1
    assert O.gf_mul(1 << 63, 2) == 0x1B
    for i in range(64):
        for j in range(64 - i):
            assert O.gf_mul(1 << i, 1 << j) == 1 << (i + j)
    # x^127 would need two folds: x^126 = x^62 * x^64
    assert O.gf_mul(1 << 63, 1 << 63) == O.gf_mul(1 << 62, 0x1B)
    r = random.Random(1)
    for _ in range(200):
        a = rnd(r)
        assert O.gf_mul(a, 1) == a
        assert O.gf_mul(a, 0) == 0


def test_field_axioms(oracle_mod):
    O = oracle_mod
    r = random.Random(2)
    for _ in range(N_RANDOM):
        a, b, c = rnd(r), rnd(r), rnd(r)
        ab = O.gf_mul(a, b)
        assert ab == O.gf_mul(b, a)
        assert O.gf_mul(ab, c) == O.gf_mul(a, O.gf_mul(b, c))
        assert O.gf_mul(a, b ^ c) == ab ^ O.gf_mul(a, c)


def test_two_formulations_agree(oracle_mod):
    O = oracle_mod
    r = random.Random(3)
    for _ in range(20 * N_RANDOM):
        a, b = rnd(r), rnd(r)
        assert O.gf_mul(a, b) == O.gf_mul_nibble(a, b)
    for a in [0, 1, MASK, 1 << 63, 0x8000000000000001]:
        for b in [0, 1, MASK, 1 << 63, 0x1B]:
            assert O.gf_mul(a, b) == O.gf_mul_nibble(a, b)


def test_frobenius_and_order(oracle_mod):
    O = oracle_mod
    r = random.Random(4)
    for _ in range(300):
        a, b = rnd(r), rnd(r)
        sq = lambda x: O.gf_mul(x, x)
        assert sq(a ^ b) == sq(a) ^ sq(b)
        x = a
        for _ in range(64):
            x = sq(x)
        assert x == a  # a^(2^64) = a in GF(2^64)
        if a:
            assert O.gf_mul(a, O.gf_inv(a)) == 1


def _clmod(a, p):
    """Remainder of GF(2)[x] division (python ints as bit polynomials)."""
    dp = p.bit_length()
    while a.bit_length() >= dp:
        a ^= p << (a.bit_length() - dp)
    return a


def _clgcd(a, b):
    while b:
        a, b = b, _clmod(a, b)
    return a


def test_modulus_irreducible(oracle_mod):
    """Rabin's test for degree 64 (only prime divisor 2): x^(2^64) = x mod p and
    gcd(x^(2^32) - x, p) = 1, with powers taken in the oracle's field."""
    O = oracle_mod
    x = 2
    y = x
    for i in range(64):
        y = O.gf_mul(y, y)
        if i == 31:
            h = y
    assert y == x
    assert _clgcd(MODULUS, h ^ x) == 1


def test_splitmix64_published_outputs(oracle_mod):
    """SplitMix64 seeded with 0 emits mix64(i * golden) for i = 1, 2, ...;
    these are the generator's published first outputs."""
    O = oracle_mod
    g = 0x9E3779B97F4A7C15
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
              0xF88BB8A8724C81EC, 0x1B39896A51A8749B]
    assert [O.mix64((i * g) & MASK) for i in range(1, 6)] == expect


def test_keyed_hash_definition(oracle_mod):
    O = oracle_mod
    g = 0x9E3779B97F4A7C15
    seed, tag, w = 12345, ord("Y"), [7 | (9 << 32), 3 | (2 << 32)]
    h = O.mix64((seed + tag * g) & MASK)
    for x in w:
        h = O.mix64(h ^ ((x + g) & MASK))
    assert O.keyed_hash(seed, tag, w) == h


def _mat_mul(O, A, B):
    k = len(A)
    C = [[0] * k for _ in range(k)]
    for i in range(k):
        for j in range(k):
            s = 0
            for t in range(k):
                s ^= O.gf_mul(A[i][t], B[t][j])
            C[i][j] = s
    return C


def test_determinant(oracle_mod):
    O = oracle_mod
    r = random.Random(5)
    for k in range(1, 7):
        for _ in range(10):
            A = [[rnd(r) for _ in range(k)] for _ in range(k)]
            B = [[rnd(r) for _ in range(k)] for _ in range(k)]
            dA = O.gf_det(A)
            assert dA == O.gf_det_leibniz(A)
            assert O.gf_det(_mat_mul(O, A, B)) == O.gf_mul(dA, O.gf_det(B))
            if k >= 2:
                A2 = [row[:] for row in A]
                A2[1] = A2[0][:]
                assert O.gf_det(A2) == 0
    # triangular: product of the diagonal
    k = 5
    T = [[(rnd(r) if j >= i else 0) for j in range(k)] for i in range(k)]
    d = 1
    for i in range(k):
        d = O.gf_mul(d, T[i][i])
    assert O.gf_det(T) == d


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_sieve_identity(oracle_mod, k):
    """Inclusion-exclusion over L of prod_p z^L_p equals the permanent, which
    is the determinant in characteristic 2 (multilinear sieving, Sec. 4.3)."""
    O = oracle_mod
    r = random.Random(10 + k)
    Z = [[rnd(r) for _ in range(k)] for _ in range(k)]
    total = 0
    for L in range(1 << k):
        prod = 1
        for p in range(k):
            zl = 0
            for j in range(k):
                if (L >> j) & 1:
                    zl ^= Z[p][j]
            prod = O.gf_mul(prod, zl)
        total ^= prod
    assert total == O.gf_det_leibniz(Z)
    # repeated row (a walk revisiting a vertex) sieves to zero
    if k >= 2:
        Z[k - 1] = Z[0][:]
        total = 0
        for L in range(1 << k):
            prod = 1
            for p in range(k):
                zl = 0
                for j in range(k):
                    if (L >> j) & 1:
                        zl ^= Z[p][j]
                prod = O.gf_mul(prod, zl)
            total ^= prod
        assert total == 0
