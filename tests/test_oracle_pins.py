"""Pins of the CPU oracle against facts fixed outside it: published known-answer vectors,
closed forms, invariants, brute force on tiny rings and plain numpy/mpmath definitions.

Each test names the mistake class it is meant to catch.  None of these tests touches the
GPU or the HIP library.
"""
import os

import mpmath
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------------------
# independent Python helpers (big integers, written from the definitions)
# --------------------------------------------------------------------------------------
def _is_prime(n):
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def schoolbook_negacyclic(a, b, q):
    n = len(a)
    r = [0] * n
    for i in range(n):
        ai = int(a[i])
        for j in range(n):
            k = i + j
            v = ai * int(b[j])
            if k >= n:
                r[k - n] -= v
            else:
                r[k] += v
    return [x % q for x in r]


def crt_lift_centered(residues, moduli):
    Q = 1
    for m in moduli:
        Q *= int(m)
    x = 0
    for r, m in zip(residues, moduli):
        m = int(m)
        Mi = Q // m
        x += int(r) * Mi * pow(Mi, -1, m)
    x %= Q
    return x - Q if x > Q // 2 else x


def centered(v, q):
    v = int(v) % q
    return v - q if v > q // 2 else v


# --------------------------------------------------------------------------------------
# primes and Philox
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("log_n,count", [(12, 3), (13, 4), (14, 6)])
def test_prime_rule(orc, log_n, count):
    """Primes are the largest q = k*2N+1 < 2^50, scanned downward (catches an off-by-one
    in the scan start, a non-prime, a wrong congruence or a skipped prime)."""
    got = [int(x) for x in orc.primes(log_n, count)]
    two_n = 2 << log_n
    want, k = [], ((1 << 50) - 2) // two_n
    while len(want) < count:
        q = k * two_n + 1
        if _is_prime(q):
            want.append(q)
        k -= 1
    assert got == want
    for q in got:
        assert q < (1 << 50) and q % two_n == 1


def test_prime_values_hand_checked(orc):
    """The first primes for N = 4096 / 8192 / 16384, checked by hand outside the oracle."""
    assert [hex(int(x)) for x in orc.primes(12, 3)] == ["0x3ffffffffc001", "0x3fffffffcc001", "0x3fffffff9a001"]
    assert [hex(int(x)) for x in orc.primes(13, 4)] == ["0x3ffffffffc001", "0x3fffffffcc001", "0x3ffffffef4001",
                                                        "0x3ffffffe94001"]
    assert [hex(int(x)) for x in orc.primes(14, 6)] == ["0x3ffffffdf0001", "0x3ffffffd48001", "0x3ffffffd20001",
                                                        "0x3ffffffd18001", "0x3ffffffcd0001", "0x3ffffffc70001"]


def test_philox_known_answers(orc):
    """Philox4x32-10 against the published Random123 known-answer vectors."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_gaussian_cdt_matches_mpmath(orc):
    """CDT thresholds floor(2^63 P(|x| <= k)) of the discrete Gaussian sigma = 3.2 on |x| <= 19,
    recomputed with mpmath at 60 digits (catches a wrong sigma, a missing factor 2 for +-x,
    or a normalisation over the wrong support)."""
    mpmath.mp.dps = 60
    sigma = mpmath.mpf("3.2")
    rho = [mpmath.e ** (-(mpmath.mpf(x) ** 2) / (2 * sigma ** 2)) for x in range(20)]
    z = rho[0] + 2 * sum(rho[1:])
    cum, want = mpmath.mpf(0), []
    for x in range(20):
        cum += (1 if x == 0 else 2) * rho[x] / z
        want.append(min(int(mpmath.floor(cum * 2 ** 63)), 2 ** 63 - 1))
    want[19] = 2 ** 63 - 1
    got = [int(v) for v in orc.cdt_table()]
    assert got == want


def test_samplers_statistics(orc):
    """Uniform mod q (chi^2 over 16 buckets), ternary frequencies, Gaussian variance."""
    q = int(orc.primes(13, 1)[0])
    n = 1 << 16
    u = orc.sample_uniform(7, 0, 0, orc.TAG_MASK, q, n).astype(object)
    assert all(0 <= int(x) < q for x in u[:1000])
    buckets = np.bincount([int(x) * 16 // q for x in u], minlength=16)
    chi2 = float(((buckets - n / 16) ** 2 / (n / 16)).sum())
    assert chi2 < 45.0  # 15 dof, p ~ 1e-4
    t = orc.sample_ternary(11, n)
    freq = np.bincount(t + 1, minlength=3) / n
    assert np.all(np.abs(freq - 1 / 3) < 0.01)
    g = orc.sample_gauss(13, 0, orc.TAG_ENC_E, n).astype(np.float64)
    assert abs(g.mean()) < 0.05
    assert abs(g.std() - 3.2) < 0.05
    assert np.abs(g).max() <= 19
    # different tags / objects give different streams
    assert not np.array_equal(orc.sample_gauss(13, 1, orc.TAG_ENC_E, 64), orc.sample_gauss(13, 0, orc.TAG_ENC_E, 64))


# --------------------------------------------------------------------------------------
# ring arithmetic
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("log_n", [2, 4, 6])
def test_polymul_equals_schoolbook(orc, log_n):
    """Ring product via the textbook NTT equals the negacyclic schoolbook convolution
    (catches a cyclic instead of negacyclic wrap, a wrong twist or a missing 1/N)."""
    c = orc.Context(log_n, 2, 1, 1)
    rng = np.random.default_rng(log_n)
    for m in range(3):
        q = int(c.moduli[m])
        a = rng.integers(0, q, c.n, dtype=np.uint64)
        b = rng.integers(0, q, c.n, dtype=np.uint64)
        assert [int(x) for x in c.polymul(m, a, b)] == schoolbook_negacyclic(a, b, q)
        assert np.array_equal(c.ntt_inverse(m, c.ntt_forward(m, a)), a)


def test_polymul_full_size_sampled(orc):
    """At N = 8192, sampled coefficients of the product equal the O(N) convolution sum."""
    c = orc.Context(13, 1, 0, 1)
    q = int(c.moduli[0])
    rng = np.random.default_rng(3)
    a = rng.integers(0, q, c.n, dtype=np.uint64)
    b = rng.integers(0, q, c.n, dtype=np.uint64)
    r = c.polymul(0, a, b)
    ai = [int(x) for x in a]
    bi = [int(x) for x in b]
    n = c.n
    for k in [0, 1, 77, n // 2, n - 1]:
        s = 0
        for i in range(n):
            j = k - i
            s += ai[i] * bi[j] if j >= 0 else -ai[i] * bi[j + n]
        assert int(r[k]) == s % q


def test_ntt_evaluates_at_odd_powers(orc):
    """The forward transform is evaluation at psi^(2t+1): the product of two transforms is
    the transform of the product, and the all-ones polynomial's transform at t matches a
    geometric series (catches an ordering mistake in the textbook NTT)."""
    c = orc.Context(4, 1, 0, 1)
    q = int(c.moduli[0])
    x = np.zeros(c.n, np.uint64)
    x[1] = 1  # X
    fx = [int(v) for v in c.ntt_forward(0, x)]  # values psi^(2t+1)
    psi = fx[0]
    assert pow(psi, 2 * c.n, q) == 1 and pow(psi, c.n, q) == q - 1
    for t in range(c.n):
        assert fx[t] == pow(psi, 2 * t + 1, q)


def test_automorphism_definition_and_group(orc):
    """sigma_g maps X^k to X^(kg mod 2N) with a sign flip past N; sigma_g o sigma_h = sigma_gh;
    5 has order N/2 modulo 2N."""
    c = orc.Context(5, 1, 0, 1)
    q = int(c.moduli[0])
    n = c.n
    rng = np.random.default_rng(1)
    a = rng.integers(0, q, n, dtype=np.uint64)
    g, h = 5, 2 * n - 1
    ra = c.automorphism(0, a, g)
    want = [0] * n
    for k in range(n):
        e = k * g % (2 * n)
        if e < n:
            want[e] = int(a[k])
        else:
            want[e - n] = (-int(a[k])) % q
    assert [int(x) for x in ra] == want
    assert np.array_equal(c.automorphism(0, c.automorphism(0, a, h), g), c.automorphism(0, a, g * h % (2 * n)))
    assert pow(5, n // 2, 2 * n) == 1 and all(pow(5, t, 2 * n) != 1 for t in range(1, n // 2))
    assert c.galois_elt(3) == pow(5, 3, 2 * n)
    assert c.galois_elt(-1) == pow(5, n // 2 - 1, 2 * n)


# --------------------------------------------------------------------------------------
# encode / decode (eq. ckks_encode)
# --------------------------------------------------------------------------------------
def test_encode_constant_vector(orc):
    """A constant slot vector encodes to the constant polynomial (c*Delta, 0, ..., 0):
    sum_j cos(pi e_j k / N) vanishes for 0 < k < N because {+-e_j} are all odd residues."""
    c = orc.Context(10, 1, 0, 1)
    for val, delta in [(0.75, 2.0 ** 30), (-1.25, 2.0 ** 40), (3.0, 2.0 ** 20)]:
        p = c.encode(np.full(c.slots, val), delta)
        assert int(p[0]) == int(round(val * delta))
        assert not p[1:].any()


@pytest.mark.parametrize("log_n", [3, 4, 5])
def test_encode_matches_direct_formula(orc, log_n):
    """At tiny N the encoding equals the direct formula
    p_k = round_half_away((2 Delta / N) sum_j m_j cos(pi 5^j k / N)) evaluated in mpmath."""
    mpmath.mp.dps = 50
    c = orc.Context(log_n, 1, 0, 1)
    n, s = c.n, c.slots
    rng = np.random.default_rng(log_n)
    m = rng.normal(0, 1, s)
    delta = 2.0 ** 40
    got = c.encode(m, delta)
    for k in range(n):
        acc = mpmath.mpf(0)
        for j in range(s):
            acc += mpmath.mpf(m[j]) * mpmath.cos(mpmath.pi * (pow(5, j, 2 * n) * k) / n)
        v = 2 * mpmath.mpf(delta) / n * acc
        r = int(mpmath.floor(abs(v) + mpmath.mpf("0.5")))
        assert int(got[k]) == (r if v >= 0 else -r)


def test_encode_matches_direct_formula_sampled_n4096(orc):
    """At N = 4096 (the smallest measured ring) 32 sampled coefficients, the first, the last, the
    middle ones and random ones, equal the direct formula in mpmath at 40 digits (catches an error
    in the fast transform that only shows at full size: a wrong twiddle index, a slot-order slip
    past the first few powers of 5, lost precision in a long sum)."""
    mpmath.mp.dps = 40
    c = orc.Context(12, 1, 0, 1)
    n, s = c.n, c.slots
    rng = np.random.default_rng(4096)
    m = rng.normal(0, 1, s)
    delta = 2.0 ** 40
    got = c.encode(m, delta)
    ks = sorted(set([0, 1, 2, n // 2 - 1, n // 2, n // 2 + 1, n - 2, n - 1] + [int(k) for k in rng.integers(0, n, 24)]))
    e = [pow(5, j, 2 * n) for j in range(s)]
    mm = [mpmath.mpf(float(x)) for x in m]
    for k in ks:
        acc = mpmath.mpf(0)
        for j in range(s):
            acc += mm[j] * mpmath.cos(mpmath.pi * ((e[j] * k) % (2 * n)) / n)
        v = 2 * mpmath.mpf(delta) / n * acc
        r = int(mpmath.floor(abs(v) + mpmath.mpf("0.5")))
        assert int(got[k]) == (r if v >= 0 else -r), k


def test_decode_inverts_encode(orc):
    """Decode(Encode(m)) = m within the rounding bound (no rounding before pi): each slot error is
    Delta^-1 sum_k eps_k cos(.), |eps_k| <= 1/2, so it is below N/(2 Delta) always and, with
    eps_k uniform (variance 1/12), below 8 sqrt(N/24)/Delta in practice."""
    c = orc.Context(13, 3, 0, 1)
    rng = np.random.default_rng(2)
    m = rng.normal(0, 1, c.slots)
    delta = 2.0 ** 40
    pt = c.encode_rns(m, delta, 2)
    err = np.abs(c.decode(pt, 2, delta) - m).max()
    assert err < c.n / (2 * delta)
    assert err < 8 * np.sqrt(c.n / 24) / delta
    # decode of the direct-formula definition at tiny N
    ct = orc.Context(4, 2, 0, 1)
    mm = rng.normal(0, 1, ct.slots)
    p = ct.encode_rns(mm, 2.0 ** 30, 1)
    lift = [crt_lift_centered([p[0, k], p[1, k]], ct.moduli[:2]) for k in range(ct.n)]
    for j in range(ct.slots):
        v = sum(lift[k] * np.cos(np.pi * pow(5, j, 2 * ct.n) * k / ct.n) for k in range(ct.n)) / 2.0 ** 30
        assert abs(ct.decode(p, 1, 2.0 ** 30)[j] - v) < 1e-9


def test_crt_centered_matches_bigint(orc):
    c = orc.Context(4, 4, 0, 1)
    rng = np.random.default_rng(9)
    for level in range(4):
        poly = np.stack([rng.integers(0, int(c.moduli[i]), c.n, dtype=np.uint64) for i in range(level + 1)])
        got = c.crt_centered(poly, level)
        for k in range(c.n):
            want = crt_lift_centered(poly[:, k], c.moduli[: level + 1])
            assert abs(got[k] - float(want)) <= abs(float(want)) * 1e-15 + 1e-9


# --------------------------------------------------------------------------------------
# encryption, keys, key switching, rescale
# --------------------------------------------------------------------------------------
def test_encrypt_decrypt_exact_error(orc):
    """Dec(Enc(pt)) - pt equals exactly the Gaussian sample e drawn for (seed, ct_id, enc-e)
    (catches a sign error in -a*s, a wrong tag, or per-limb instead of per-coefficient e)."""
    c = orc.Context(11, 3, 1, 3)
    k = orc.Keys(c, 5)
    rng = np.random.default_rng(0)
    pt = np.stack([rng.integers(0, int(q), c.n, dtype=np.uint64) for q in c.q])
    ct = k.encrypt(pt, 2, 42, 7)
    e = orc.sample_gauss(42, 7, orc.TAG_ENC_E, c.n)
    d = k.decrypt(ct, 2)
    for i, q in enumerate(c.q):
        q = int(q)
        diff = (d[i].astype(object) - pt[i].astype(object)) % q
        assert [centered(x, q) for x in diff] == [int(x) for x in e]
    # c1 is the uniform sample of tag enc-a for each limb
    assert np.array_equal(ct[1, 1], orc.sample_uniform(42, 1, 7, orc.TAG_ENC_A, int(c.q[1]), c.n))


def test_switching_key_structure(orc):
    """b_j + a_j s - [P]_{q_i} s' 1{i in D_j} equals the digit's Gaussian error exactly, on every
    modulus (catches a missing P factor, a wrong digit partition or an s' mix-up)."""
    c = orc.Context(6, 4, 2, 2)
    g = c.galois_elt(1)
    k = orc.Keys(c, 77, [g])
    s = [int(x) for x in k.secret]
    n = c.n
    # s' for the rotation key: sigma_g(s) over the integers
    sp = [0] * n
    for i in range(n):
        e = i * g % (2 * n)
        if e < n:
            sp[e] = s[i]
        else:
            sp[e - n] = -s[i]
    P = int(c.p[0]) * int(c.p[1])
    swk = k.switching_key(g)
    for j in range(c.dnum):
        e = [int(x) for x in orc.sample_gauss(77, g * 64 + j, orc.TAG_KEY_E, n)]
        for m in range(6):
            q = int(c.moduli[m])
            b = [int(x) for x in swk[j, 0, m]]
            a = [int(x) for x in swk[j, 1, m]]
            as_ = schoolbook_negacyclic(a, [x % q for x in s], q)
            in_digit = m < 4 and m // c.alpha == j
            for i in range(n):
                v = (b[i] + as_[i] - (P * sp[i] if in_digit else 0)) % q
                assert centered(v, q) == e[i]


def _noise(ctx, diff, level):
    """max |centred CRT lift| of a polynomial given by residues"""
    lift = ctx.crt_centered(diff, level)
    return np.abs(lift).max()


@pytest.mark.parametrize("params", [(11, 3, 1, 3), (11, 4, 2, 2)])
def test_rotation_keyswitch_invariant(orc, params):
    """Dec(Rot_g(ct)) - sigma_g(Dec(ct)) has a small centred norm at every level: the hybrid key
    switch (ModUp, hoisted automorphism, inner product, ModDown) adds only error of order
    N*sigma*Q_digit/P (catches a wrong ModUp factor, a wrong ModDown sign or P^-1, or a
    rotation applied before ModUp with the wrong key)."""
    log_n, n_q, n_sp, dnum = params
    c = orc.Context(log_n, n_q, n_sp, dnum)
    gal = [c.galois_elt(1), c.galois_elt(-3)]
    k = orc.Keys(c, 3, gal)
    rng = np.random.default_rng(1)
    m = rng.normal(0, 1, c.slots)
    for level in range(n_q - 1, -1, -1):
        delta = 2.0 ** 30
        ct = k.encrypt(c.encode_rns(m, delta, level), level, 1000 + level, 0)
        for steps, g in [(1, gal[0]), (-3, gal[1])]:
            r = k.rotate(ct, level, steps)
            d_rot = k.decrypt(r, level)
            d = k.decrypt(ct, level)
            sd = np.stack([c.automorphism(i, d[i], g) for i in range(level + 1)])
            diff = np.stack([(d_rot[i].astype(object) - sd[i].astype(object)) % int(c.q[i]) for i in range(level + 1)]).astype(np.uint64)
            assert _noise(c, diff, level) < 2.0 ** 30  # vs Q >= 2^49
            dec = c.decode(d_rot, level, delta)
            assert np.abs(dec - np.roll(m, -steps)).max() < 1e-3


# --------------------------------------------------------------------------------------
# the hybrid key switch written out over the integers (no RNS limbs, no NTT): every word
# of the oracle's rotations and relinearisations at tiny N
# --------------------------------------------------------------------------------------
def _prod(xs):
    r = 1
    for x in xs:
        r *= int(x)
    return r


def _crt(res, mods):
    M = _prod(mods)
    x = 0
    for r, m in zip(res, mods):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M


def _negacyclic_int(a, b, M):
    n = len(a)
    r = [0] * n
    for i in range(n):
        if a[i] == 0:
            continue
        for j in range(n):
            k = i + j
            if k >= n:
                r[k - n] -= a[i] * b[j]
            else:
                r[k] += a[i] * b[j]
    return [x % M for x in r]


def _sigma_int(a, g):
    """X^k -> X^(k g) on an integer polynomial of Z[X]/(X^N + 1)"""
    n = len(a)
    r = [0] * n
    for k in range(n):
        e = k * g % (2 * n)
        if e < n:
            r[e] = a[k]
        else:
            r[e - n] = -a[k]
    return r


def _keyswitch_int(ctx, swk, d, level, g):
    """KS(d) from the formulas of the hybrid key switch, with Python integers:
    ModUp of digit j without centring is the integer X_j = sum_{i in D_j} [d_i (Q_D/q_i)^-1]_{q_i}
    (Q_D/q_i); sigma_g acts on X_j (after ModUp); u = sum_j sigma_g(X_j) key_j over Z_{Q_l P};
    ModDown without centring is (u - v) / P with v = sum_t [u (P/p_t)^-1]_{p_t} (P/p_t).
    Returns (u_0, u_1) as residues [2][l+1][N]."""
    n, nl, alpha = ctx.n, level + 1, ctx.alpha
    qs = [int(x) for x in ctx.q[:nl]]
    ps = [int(x) for x in ctx.p]
    P, QP = _prod(ps), _prod(qs) * _prod(ps)
    key_mods = qs + ps
    key_idx = list(range(nl)) + [ctx.n_q + t for t in range(len(ps))]
    u = [[0] * n, [0] * n]
    for j in range((nl + alpha - 1) // alpha):
        lo, hi = j * alpha, min((j + 1) * alpha, nl)
        D = qs[lo:hi]
        QD = _prod(D)
        X = [sum((int(d[lo + t][k]) * pow(QD // qi, -1, qi)) % qi * (QD // qi) for t, qi in enumerate(D)) for k in range(n)]
        if g:
            X = _sigma_int(X, g)
        for p in range(2):
            key = [_crt([swk[j, p, m, k] for m in key_idx], key_mods) for k in range(n)]
            prod = _negacyclic_int(X, key, QP)
            u[p] = [(x + y) % QP for x, y in zip(u[p], prod)]
    out = np.zeros((2, nl, n), np.uint64)
    for p in range(2):
        for k in range(n):
            x = u[p][k]
            v = sum((x % pt) * pow(P // pt, -1, pt) % pt * (P // pt) for pt in ps)
            w = (x - v) // P
            assert w * P == x - v
            for i, qi in enumerate(qs):
                out[p, i, k] = w % qi
    return out


@pytest.mark.parametrize("params", [(4, 3, 1, 3), (5, 4, 2, 2), (6, 5, 2, 3)])
def test_keyswitch_matches_integer_formulas(orc, params):
    """Every word of the oracle's rotations (left and right) and relinearisations, at every level,
    equals the hybrid key switch written out over the integers (catches centring in ModUp or
    ModDown, sigma_g applied before ModUp instead of after, a lazy or missing ModDown, a digit
    partition slip at a partial last digit, a wrong key limb at a lower level)."""
    log_n, n_q, n_sp, dnum = params
    c = orc.Context(log_n, n_q, n_sp, dnum)
    n = c.n
    steps = [1, -3]
    gal = [c.galois_elt(t) for t in steps]
    k = orc.Keys(c, 1234 + log_n, gal)
    swk = {g: k.switching_key(g) for g in gal}
    swk[0] = k.switching_key(0)
    rng = np.random.default_rng(log_n)
    for level in range(n_q - 1, -1, -1):
        nl = level + 1
        qs = [int(x) for x in c.q[:nl]]
        ct = np.stack([np.stack([rng.integers(0, q, n, dtype=np.uint64) for q in qs]) for _ in range(3)])
        for t, g in zip(steps, gal):
            u = _keyswitch_int(c, swk[g], ct[1], level, g)
            want = u.copy()
            for i, q in enumerate(qs):
                s0 = _sigma_int([int(x) for x in ct[0, i]], g)
                want[0, i] = [(int(a) + b) % q for a, b in zip(u[0, i], s0)]
            assert np.array_equal(k.rotate(ct[:2], level, t), want), f"rotation {t} at level {level}"
        u = _keyswitch_int(c, swk[0], ct[2], level, 0)
        want = np.stack([np.stack([(u[p, i].astype(object) + ct[p, i].astype(object)) % q for i, q in enumerate(qs)]) for p in range(2)]).astype(np.uint64)
        assert np.array_equal(k.relinearize(ct, level), want), f"relinearisation at level {level}"


def test_relinearize_invariant(orc):
    """Relin(d0, d1, d2) decrypts like (d0, d1, d2) under (1, s, s^2) up to key-switch noise."""
    c = orc.Context(11, 3, 1, 3)
    k = orc.Keys(c, 8)
    rng = np.random.default_rng(4)
    level = 2
    m1, m2 = rng.normal(0, 1, c.slots), rng.normal(0, 1, c.slots)
    a = k.encrypt(c.encode_rns(m1, 2.0 ** 30, level), level, 1, 0)
    b = k.encrypt(c.encode_rns(m2, 2.0 ** 30, level), level, 2, 0)
    ct3 = np.zeros((3, level + 1, c.n), np.uint64)
    for i in range(level + 1):
        q = int(c.q[i])
        ct3[0, i] = c.polymul(i, a[0, i], b[0, i])
        t1 = c.polymul(i, a[0, i], b[1, i]).astype(object) + c.polymul(i, a[1, i], b[0, i]).astype(object)
        ct3[1, i] = (t1 % q).astype(np.uint64)
        ct3[2, i] = c.polymul(i, a[1, i], b[1, i])
    r = k.relinearize(ct3, level)
    d3 = k.decrypt(ct3, level)
    d2 = k.decrypt(r, level)
    diff = np.stack([(d2[i].astype(object) - d3[i].astype(object)) % int(c.q[i]) for i in range(level + 1)]).astype(np.uint64)
    assert _noise(c, diff, level) < 2.0 ** 30
    dec = c.decode(d2, level, 2.0 ** 60)
    assert np.abs(dec - m1 * m2).max() < 1e-3


@pytest.mark.parametrize("log_n", [3, 10])
def test_rescale_equals_rounded_division(orc, log_n):
    """Rescale equals round(c~ / q_l) mod Q_{l-1} for the CRT lift c~ in [0, Q_l) (any lift gives
    the same result because q_l is odd)."""
    c = orc.Context(log_n, 3, 0, 1)
    rng = np.random.default_rng(log_n)
    level = 2
    ct = np.stack([np.stack([rng.integers(0, int(q), c.n, dtype=np.uint64) for q in c.q]) for _ in range(2)])
    out = c.rescale(ct, level)
    Q = int(c.q[0]) * int(c.q[1]) * int(c.q[2])
    ql = int(c.q[2])
    for p in range(2):
        for kk in range(0, c.n, max(1, c.n // 64)):
            x = crt_lift_centered(ct[p, :, kk], c.q) % Q
            r = (2 * x + ql) // (2 * ql)  # round half up; no ties since q_l is odd
            for i in range(2):
                assert int(out[p, i, kk]) == r % int(c.q[i])


# --------------------------------------------------------------------------------------
# matmul_cp and mask-to-share
# --------------------------------------------------------------------------------------
def _unpack(ctx, g, vecs, L, D):
    out = np.zeros((L, D))
    for col in range(D):
        b, u = divmod(col, g["c"]) if g["c_out"] == g["c"] else (0, col)
        out[:, col] = vecs[b][u * g["Lp"]: u * g["Lp"] + L]
    return out


@pytest.mark.parametrize("shape", [(32, 32, 32), (20, 40, 24), (5, 96, 70)])
def test_matmul_cp_decodes_to_fp64_matmul(orc, shape):
    """Decoded matmul_cp output equals X @ W (FP64) within 2^-10 at Delta = 2^30, including
    ragged L, D_in, D_out and replicated packings."""
    L, d_in, d_out = shape
    c = orc.Context(12, 2, 1, 2)
    rng = np.random.default_rng(sum(shape))
    X = rng.uniform(-1, 1, (L, d_in))
    W = rng.normal(0, 0.02, (d_in, d_out))
    g = c.cp_geometry(L, d_in, d_out)
    k = orc.Keys(c, 9, c.cp_galois(L, d_in, d_out))
    cts = np.stack([k.encrypt(c.encode_rns(c.pack_spatial(X, a), 2.0 ** 30, 1), 1, 100, a) for a in range(g["n_in"])])
    Y = k.matmul_cp(cts, 1, W, L)
    vecs = [c.decode(k.decrypt(Y[b], 0), 0, 2.0 ** 30) for b in range(g["n_out"])]
    got = _unpack(c, g, vecs, L, d_out)
    assert np.abs(got - X @ W).max() < 2.0 ** -10
    # rows >= L of the output block are (near) zero, replicated blocks agree
    if g["c_out"] < g["c"]:
        v = vecs[0]
        assert np.abs(v[: g["Lp"] * g["c_out"]] - v[g["Lp"] * g["c_out"]: 2 * g["Lp"] * g["c_out"]]).max() < 2.0 ** -10


def test_matmul_cp_identity_and_counts(orc):
    """W = I gives back X; BSGS geometry for the BERT-base shape gives B = 8, G = 4 and
    n_in (B-1) + n_out (G-1) = 240 rotations on 10 Galois keys."""
    c = orc.Context(12, 2, 1, 2)
    L, D = 32, 64
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (L, D))
    g = c.cp_geometry(L, D, D)
    k = orc.Keys(c, 9, c.cp_galois(L, D, D))
    cts = np.stack([k.encrypt(c.encode_rns(c.pack_spatial(X, a), 2.0 ** 30, 1), 1, 100, a) for a in range(g["n_in"])])
    Y = k.matmul_cp(cts, 1, np.eye(D), L)
    vecs = [c.decode(k.decrypt(Y[b], 0), 0, 2.0 ** 30) for b in range(g["n_out"])]
    assert np.abs(_unpack(c, g, vecs, L, D) - X).max() < 2.0 ** -12
    c2 = orc.Context(13, 3, 1, 3)
    g2 = c2.cp_geometry(128, 768, 768)
    assert (g2["Lp"], g2["c"], g2["c_eff"], g2["n_in"], g2["n_out"], g2["B"], g2["G"]) == (128, 32, 32, 24, 24, 8, 4)
    assert g2["n_in"] * (g2["B"] - 1) + g2["n_out"] * (g2["G"] - 1) == 240
    assert len(c2.cp_galois(128, 768, 768)) == 10
    # modular multiplications of the plaintext MACs: 2 polys * n_q limbs * N per plaintext
    n_pt = g2["n_in"] * g2["n_out"] * g2["c_eff"]
    assert n_pt == 18432
    assert n_pt * 2 * 3 * 8192 == 905969664


def test_mask_to_share_identity_and_uniformity(orc):
    """Dec(masked) + share == Dec(ct) (mod Q) word for word; Dec(masked) is uniform (chi^2 on
    its top bits); the share is -r for the mask stream of (seed, ct_id)."""
    c = orc.Context(12, 3, 1, 3)
    k = orc.Keys(c, 4)
    rng = np.random.default_rng(7)
    m = rng.normal(0, 1, c.slots)
    ct = k.encrypt(c.encode_rns(m, 2.0 ** 40, 2), 2, 5, 0)
    for target in (2, 1):
        masked, share = c.mask_to_share(ct, 2, target, 99, 3)
        d_m = k.decrypt(masked, target)
        d = k.decrypt(ct, 2)[: target + 1]
        for i in range(target + 1):
            q = int(c.q[i])
            assert np.array_equal((d_m[i].astype(object) + share[i].astype(object)) % q, d[i].astype(object))
            r = orc.sample_uniform(99, i, 3, orc.TAG_MASK, q, c.n)
            assert np.array_equal(share[i], ((q - r.astype(object)) % q).astype(np.uint64))
            top = (d_m[i].astype(object) * 16 // q).astype(np.int64)
            cnt = np.bincount(top, minlength=16)
            chi2 = float(((cnt - c.n / 16) ** 2 / (c.n / 16)).sum())
            assert chi2 < 45.0


def test_mpc_to_ckks_server_addition(orc):
    """Algorithm mpc2ckks, the server's step: Enc(tmp_0) + tmp_1 decrypts to Dec(Enc(tmp_0)) + tmp_1
    in every limb (a big-integer CRT check), decodes to x when tmp_0 + tmp_1 = Encode(x) mod Q, and
    undoes mask-to-share word for word (masked ciphertext plus the share -r is the original)."""
    c = orc.Context(12, 3, 1, 3)
    k = orc.Keys(c, 4)
    rng = np.random.default_rng(9)
    x = rng.normal(0, 1, c.slots)
    level, scale = 2, 2.0 ** 40
    pt = c.encode_rns(x, scale, level)
    # additive shares of the encoded message over Z_Q: tmp_1 uniform per limb, tmp_0 = pt - tmp_1
    tmp1 = np.stack([orc.sample_uniform(123, i, 0, orc.TAG_MASK, int(c.q[i]), c.n) for i in range(level + 1)])
    tmp0 = np.stack([((pt[i].astype(object) - tmp1[i].astype(object)) % int(c.q[i])).astype(np.uint64) for i in range(level + 1)])
    ct0 = k.encrypt(tmp0, level, 6, 0)
    ct = c.add_share(ct0, level, tmp1)
    d, d0 = k.decrypt(ct, level), k.decrypt(ct0, level)
    for i in range(level + 1):
        q = int(c.q[i])
        assert np.array_equal(d[i].astype(object), (d0[i].astype(object) + tmp1[i].astype(object)) % q)
    assert np.abs(c.decode(d, level, scale) - x).max() < 2.0 ** -20
    # round trip with the CKKS-to-MPC step
    ctx_ = k.encrypt(pt, level, 7, 1)
    masked, share = c.mask_to_share(ctx_, level, level, 55, 2)
    assert np.array_equal(c.add_share(masked, level, share), ctx_)


@pytest.mark.parametrize("bits", [32, 40])
def test_rerandomize_adds_flooded_encryption_of_zero(orc, bits):
    """Dec(rerand(ct)) - Dec(ct) = v e_pk + e0 + e1 s, the same integer in every limb (CRT
    consistency, so the term is a genuine small polynomial); it lies within 2^F + 2 * 19 * N and is
    uniform over [-2^F, 2^F] (chi^2 over 16 bins, standard deviation 2^F / sqrt(3)); c1 moves by a
    value that looks uniform mod q; other seeds or object ids give other noise; the message
    decodes within 8 sqrt(N) 2^F / Delta (the slot sums of N flooding coefficients)."""
    c = orc.Context(12, 3, 1, 3)
    k = orc.Keys(c, 4)
    rng = np.random.default_rng(8)
    m = rng.normal(0, 1, c.slots)
    lvl, delta = 2, 2.0 ** 40
    ct = k.encrypt(c.encode_rns(m, delta, lvl), lvl, 5, 0)
    rr = k.rerandomize(ct, lvl, 1234, 3, bits)
    diff = (k.decrypt(rr, lvl).astype(object) - k.decrypt(ct, lvl).astype(object))
    vals = []
    for i in range(lvl + 1):
        q = int(c.q[i])
        vals.append([(int(x) % q) if (int(x) % q) <= q // 2 else (int(x) % q) - q for x in diff[i]])
    vals = np.array(vals, dtype=np.int64)
    assert all(np.array_equal(vals[0], vals[i]) for i in range(1, lvl + 1))
    e = vals[0].astype(np.float64)
    B = float(2 ** bits)
    assert np.abs(e).max() <= B + 2 * 19 * c.n
    assert np.abs(e).max() > 0.95 * B
    assert abs(e.std() / (B / np.sqrt(3)) - 1) < 0.05
    cnt = np.bincount(np.clip(((e + B) * 16 / (2 * B + 1)).astype(np.int64), 0, 15), minlength=16)
    assert float(((cnt - c.n / 16) ** 2 / (c.n / 16)).sum()) < 45.0
    q0 = int(c.q[0])
    dc1 = (rr[1, 0].astype(object) - ct[1, 0].astype(object)) % q0
    top = np.array([int(x) * 16 // q0 for x in dc1])
    assert float(((np.bincount(top, minlength=16) - c.n / 16) ** 2 / (c.n / 16)).sum()) < 45.0
    assert not np.array_equal(k.rerandomize(ct, lvl, 1234, 4, bits), rr)
    assert not np.array_equal(k.rerandomize(ct, lvl, 1235, 3, bits), rr)
    got = c.decode(k.decrypt(rr, lvl), lvl, delta)
    assert np.abs(got - m).max() < 8 * np.sqrt(c.n) * B / delta
    with pytest.raises(ValueError):
        k.rerandomize(ct, lvl, 1, 0, 31)


def test_encoded_mask_concentration_negative_control(orc):
    """The insecure MP2ML mask Encode(Delta^-1 r), r uniform in Z_q^(N/2), has coefficients with
    standard deviation q / sqrt(12 N) (N = 8192, q ~ 2^60 as in Figure distribution): far
    narrower than the uniform q / sqrt(12) of the secure mask."""
    n = 8192
    c = orc.Context(13, 1, 0, 1)
    q = float(2 ** 60 - 2 ** 40)
    rng = np.random.default_rng(11)
    r = rng.uniform(0, q, n // 2)
    p = c.encode(r - q / 2, 1.0).astype(np.float64)  # centred uniform; only the spread matters
    p = p[1:]  # coefficient 0 carries the mean
    ratio = p.std() / (q / np.sqrt(12 * n))
    assert abs(ratio - 1) < 0.05
    assert p.std() < q / np.sqrt(12) / 50


# --------------------------------------------------------------------------------------
# matmul_cc (multi-head, diagonal-packed output)
# --------------------------------------------------------------------------------------
def _unrotated_b(mats, H_g, L, d, a, slots):
    """slot i + L'(h + H_g kappa) <- B_h{a c + kappa, i}: the B operand before step 1 (built
    here by hand, independently of the packing helpers)"""
    lp = 1 << int(np.ceil(np.log2(L)))
    cc = slots // (lp * H_g)
    v = np.zeros(slots)
    for h in range(H_g):
        for kap in range(cc):
            k = a * cc + kap
            if k < d:
                v[lp * (h + H_g * kap): lp * (h + H_g * kap) + L] = mats[h][k, :]
    return v


def _cc_small(orc, H_g, L, d, seed, prerot=True):
    c = orc.Context(12, 4, 2, 2) if prerot else orc.Context(12, 5, 2, 3)  # digits of at most K = 2 primes
    g = c.cc_geometry(H_g, L, d)
    rng = np.random.default_rng(seed)
    Q = [rng.normal(0, 1, (L, d)) for _ in range(H_g)]
    K = [rng.normal(0, 1, (L, d)) for _ in range(H_g)]
    Bm = [k.T.copy() for k in K]
    keys = orc.Keys(c, 5, c.cc_galois(H_g, L, d))
    level, scale = (3 if prerot else 4), 2.0 ** 40
    A = np.stack([keys.encrypt(c.encode_rns(c.pack_mhp(Q, H_g, L, d, a, "A"), scale, level), level, 10, a) for a in range(g["n_ct"])])
    if prerot:
        bv = [c.pack_mhp(Bm, H_g, L, d, a, "Bp") for a in range(g["n_ct"])]
    else:
        bv = [_unrotated_b(Bm, H_g, L, d, a, c.slots) for a in range(g["n_ct"])]
    Bp = np.stack([keys.encrypt(c.encode_rns(v, scale, level), level, 11, a) for a, v in enumerate(bv)])
    return c, g, keys, Q, K, A, Bp, level, scale


@pytest.mark.parametrize("H_g,L,d,prerot", [(2, 32, 64, True), (4, 20, 32, True), (2, 32, 64, False), (4, 20, 32, False)])
def test_matmul_cc_decodes_to_qkt(orc, H_g, L, d, prerot):
    """Decoded diagonal-packed output equals Q_h K_h^T (FP64) for every head, within 2^-20 at
    the final scale ~2^40 (catches a wrong inner-rotation mask, a wrong step-3 block rotation
    or a wrong output index g+1 for the wrapped blocks).  prerot=False feeds B without the
    client-side row rotation and runs step 1 homomorphically (one more level, five primes);
    a wrong step-1 mask or rotation direction breaks the same check."""
    c, g, keys, Q, K, A, Bp, level, scale = _cc_small(orc, H_g, L, d, H_g + L, prerot)
    O = keys.matmul_cc(A, Bp, level, H_g, L, d, b_prerotated=prerot)
    if not prerot:
        level -= 1  # steps 2-3 run one level lower; step 1 keeps the scale
    lp, cc = g["Lp"], g["c"]
    # scale after the schedule: scale * (q3 2^10 / q3) * scale / q2 * (q1 / q1)
    out_scale = scale * 1024.0 * scale / float(c.q[2])
    got = [[np.zeros((lp, lp)) for _ in range(H_g)]]
    for gi in range(g["n_out"]):
        v = c.decode(keys.decrypt(O[gi], 0), 0, out_scale)
        for h in range(H_g):
            for kap in range(cc):
                D = gi * cc + kap
                for i in range(lp):
                    got[0][h][i, (i + D) % lp] = v[i + lp * (h + H_g * kap)]
    for h in range(H_g):
        ref = Q[h] @ K[h].T
        assert np.abs(got[0][h][:L, :L] - ref).max() < 2.0 ** -20
        if L < lp:
            assert np.abs(got[0][h][L:, :]).max() < 1e-4 and np.abs(got[0][h][:, L:]).max() < 1e-4


def _bsgs_rotation_count(lp, cc, n_ct, B, G, b1, g1, n_dense, hom1):
    """Rotations of one head group's BSGS schedule, counted from its definition: two per inner
    rotation of B' (i < B) and of A (0 < j < G), one step-3 rotation per t with tau != 0, one
    postponed giant rotation per (output, giant step j > 0, half) that receives a term, and for
    step 1 on the server b1 - 1 baby plus 2 g1 - 1 giant rotations per B ciphertext."""
    n_diag = lp // cc
    r = 2 * n_ct * (B - 1) + 2 * n_ct * (G - 1) + sum(1 for t in range(lp) if t % cc)
    for j in range(1, G):
        outs = set()
        for t in range(j * B, j * B + B):
            outs.add((t // cc) % n_dense)
            if t % cc:
                outs.add(((t // cc + 1) % n_diag) % n_dense)
        r += 2 * len(outs)
    if hom1:
        r += n_ct * ((b1 - 1) + (g1 - 1) + g1 - (1 if b1 == 1 else 0))
    return r


@pytest.mark.parametrize("H_g,L,d,prerot", [(2, 32, 64, True), (4, 20, 32, True), (4, 20, 32, False), (8, 16, 16, False)])
def test_matmul_cc_bsgs_decodes_to_qkt(orc, H_g, L, d, prerot):
    """The BSGS schedule (Appendix "BSGS Optimization": baby-step inner rotations of B', giant
    steps taken on A and postponed into step 3 with one more mask product and one rotation per
    giant-step accumulator; step 1 split into baby and giant rotations) decodes to Q_h K_h^T
    within 2^-20 for every head, with the plain schedule's levels and output scale, and performs
    exactly the rotations its closed form counts (and L' relinearisations).  A giant rotation in
    the wrong direction, a product mask on the wrong half of a block or a mask pre-rotated the
    wrong way breaks the decoded check."""
    c, g, keys, Q, K, A, Bp, level, scale = _cc_small(orc, H_g, L, d, H_g + L, prerot)
    keys = orc.Keys(c, 5, c.cc_galois(H_g, L, d, schedule=1))
    sp = c.cc_bsgs_split(H_g, L, d)
    assert sp["B"] * sp["G"] == g["Lp"] and sp["b1"] * sp["g1"] == g["c"]
    orc.ks_counts(reset=True)
    O = keys.matmul_cc(A, Bp, level, H_g, L, d, b_prerotated=prerot, schedule=1)
    n_rot, n_relin = orc.ks_counts(reset=True)
    assert n_relin == g["Lp"]
    assert n_rot == _bsgs_rotation_count(g["Lp"], g["c"], g["n_ct"], sp["B"], sp["G"], sp["b1"], sp["g1"], g["n_out"], not prerot)
    lp, cc = g["Lp"], g["c"]
    out_scale = scale * 1024.0 * scale / float(c.q[2 if prerot else 3])
    got = [np.zeros((lp, lp)) for _ in range(H_g)]
    for gi in range(g["n_out"]):
        v = c.decode(keys.decrypt(O[gi], 0), 0, out_scale)
        for h in range(H_g):
            for kap in range(cc):
                D = gi * cc + kap
                for i in range(lp):
                    got[h][i, (i + D) % lp] = v[i + lp * (h + H_g * kap)]
    for h in range(H_g):
        ref = Q[h] @ K[h].T
        assert np.abs(got[h][:L, :L] - ref).max() < 2.0 ** -20
        if L < lp:
            assert np.abs(got[h][L:, :]).max() < 1e-4 and np.abs(got[h][:, L:]).max() < 1e-4


def test_matmul_cc_bsgs_selected_outputs_match_full_run(orc):
    """Computing only some outputs of the BSGS schedule (the sampled full-size checks do this)
    gives the same words as the full run for those outputs."""
    c, g, keys, Q, K, A, Bp, level, scale = _cc_small(orc, 4, 20, 32, 3, True)
    keys = orc.Keys(c, 5, c.cc_galois(4, 20, 32, schedule=1))
    full = keys.matmul_cc(A, Bp, level, 4, 20, 32, schedule=1)
    for o in range(g["n_out"]):
        part = keys.matmul_cc(A, Bp, level, 4, 20, 32, outputs=[o], schedule=1)
        assert np.array_equal(part[o], full[o])


@pytest.mark.parametrize("log_n,H_g,L,d_v", [(12, 4, 32, 16), (12, 4, 20, 12)])
def test_softmax_v_bsgs_dense_diagonals(orc, log_n, H_g, L, d_v):
    """Softmax x V_h through the BSGS schedule: the fold of the diagonal accumulators happens after
    the postponed giant rotations, and every dense output decodes to (S_h V_h) within 2^-20."""
    c, g, keys, Sm, Vm, A, Bv, level, scale = _sv_small(orc, log_n, 4, H_g, L, d_v, log_n + L + d_v)
    keys = orc.Keys(c, 5, c.cc_galois(H_g, L, L, schedule=1))
    O = keys.matmul_cc_sv(A, Bv, level, H_g, L, d_v, schedule=1)
    out_scale = scale * 1024.0 * scale / float(c.q[2])
    lp, cg, dvp = g["Lp"], g["c"], g["dvp"]
    ref = [Sm[h] @ Vm[h] for h in range(H_g)]
    worst = 0.0
    for o in range(g["n_out"]):
        v = c.decode(keys.decrypt(O[o], 0), 0, out_scale)
        want = _dense_diag_vec(ref, 0, H_g, lp, cg, o, L, d_v, dvp, c.slots)
        worst = max(worst, np.abs(v - want).max())
    assert worst < 2.0 ** -20


def test_matmul_cc_bsgs_counts_bert_base():
    """Closed-form rotation counts of the 12-head BERT-base Q_h K_h^T (L' = 128, d_head = 64,
    8192 slots, groups 8 + 4): the plain schedule makes 2 (L' - 1) inner-rotation key switches per
    B' ciphertext (3048) plus 232 step-3 rotations; the BSGS schedule (B = 16, G = 8) makes 830,
    i.e. B + G - 2 = 22 inner rotations per operand pair instead of L' - 1 = 127, plus the
    postponed giant rotations (70)."""
    plain = sum(2 * n * 127 + (128 - 128 // c) for c, n in ((8, 8), (16, 4)))
    assert plain == 3048 + 232
    bsgs = sum(_bsgs_rotation_count(128, c, n, 16, 8, 4, 4 if c == 16 else 2, 128 // c, False) for c, n in ((8, 8), (16, 4)))
    assert bsgs == 830
    giant = sum(_bsgs_rotation_count(128, c, n, 16, 8, 4, 2, 128 // c, False) - 2 * n * (15 + 7) - (128 - 128 // c)
                for c, n in ((8, 8), (16, 4)))
    assert giant == 70


def test_matmul_cc_counts():
    """Theoretical ct-ct multiplication count m^2 d / s of the paper's Table complexity_compare
    (BERT-large, s = 16384): 1024 for Q_h K_h^T and m^3 H / s = 2048 for Softmax x V_h; the
    12-head BERT-base group split 8 + 4 at N = 16384 gives 1536 tensors (= 128^2 * 768 / 8192) and
    2 x 128 relinearisations."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "complexity_bert_large.txt")) if l.strip() and l[0] != "#"]
    for name, m, d, H, s, cm in rows:
        m, d, H, s, cm = int(m), int(d), int(H), int(s), int(cm)
        if name == "QK":
            assert m * m * d // s == cm
        else:
            assert m ** 3 * H // s == cm
    # the pinned schedule: tensors = sum over groups of L' * n_ct
    n_tensor = 0
    for H_g in (8, 4):
        c_ = 8192 // (128 * H_g)
        n_tensor += 128 * (64 // c_)
    assert n_tensor == 1536 == 128 * 128 * 768 // 8192


# --------------------------------------------------------------------------------------
# Softmax x V_h (zero padding, dense diagonal packing) and the diagonal-input matmul_cp
# --------------------------------------------------------------------------------------
def _groups(heads):
    out, h = [], heads
    while h:
        g = 1 << (h.bit_length() - 1)
        out.append(g)
        h -= g
    return out


def _softmax_rows(rng, L):
    z = rng.normal(0, 1, (L, L))
    e = np.exp(z - z.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def _dense_diag_vec(att, h0, H_g, lp, cg, o, L, d_v, dvp, slots):
    """slot i + L'(h + H_g kappa) <- Att_{h0+h}{i, (i + o c_g + kappa) mod d_v'} (0 past d_v or L),
    written element by element from the definition"""
    v = np.zeros(slots)
    for h in range(H_g):
        for kap in range(cg):
            for i in range(L):
                col = (i + o * cg + kap) % dvp
                if col < d_v:
                    v[i + lp * (h + H_g * kap)] = att[h0 + h][i, col]
    return v


def _sv_small(orc, log_n, n_q, H_g, L, d_v, seed):
    c = orc.Context(log_n, n_q, 2, (n_q + 1) // 2)
    g = c.cc_sv_geometry(H_g, L, d_v)
    rng = np.random.default_rng(seed)
    Sm = [_softmax_rows(rng, L) for _ in range(H_g)]
    Vm = [rng.normal(0, 1, (L, d_v)) for _ in range(H_g)]
    keys = orc.Keys(c, 5, c.cc_galois(H_g, L, L))
    level, scale = n_q - 1, 2.0 ** 40
    A = np.stack([keys.encrypt(c.encode_rns(c.pack_mhp(Sm, H_g, L, L, a, "A"), scale, level), level, 10, a) for a in range(g["n_ct"])])
    Bv = np.stack([keys.encrypt(c.encode_rns(c.pack_mhp(Vm, H_g, L, L, a, "Bp"), scale, level), level, 11, a)
                   for a in range(g["n_ct"])])
    return c, g, keys, Sm, Vm, A, Bv, level, scale


@pytest.mark.parametrize("log_n,H_g,L,d_v", [(12, 4, 32, 16), (12, 4, 20, 12), (11, 4, 32, 16)])
def test_softmax_v_dense_diagonals(orc, log_n, H_g, L, d_v):
    """Softmax x V_h through the ct-ct protocol with V_h zero-padded to L' columns, the diagonal
    ciphertexts folded mod d_v' (figure diag (b)): output o decodes to Att_h{i, (i + o c + kappa)
    mod d_v'} = (S_h V_h){i, .} for every head, zero past d_v and past row L.  Covers a fold of 2
    (L' = 2 d_v'), a ragged L with d_v = 12 (d_v' = 16, the padded columns stay zero) and two dense
    outputs per group (c < d_v' at N = 2048).  A wrong fold index, a lost wrap term or a
    non-complementary pair of diagonals breaks the check."""
    c, g, keys, Sm, Vm, A, Bv, level, scale = _sv_small(orc, log_n, 4, H_g, L, d_v, log_n + L + d_v)
    assert g["n_out"] == g["dvp"] // g["c"] >= 1
    O = keys.matmul_cc_sv(A, Bv, level, H_g, L, d_v)
    out_scale = scale * 1024.0 * scale / float(c.q[2])
    lp, cg, dvp = g["Lp"], g["c"], g["dvp"]
    ref = [Sm[h] @ Vm[h] for h in range(H_g)]
    worst, zero = 0.0, 0.0
    for o in range(g["n_out"]):
        v = c.decode(keys.decrypt(O[o], 0), 0, out_scale)
        want = _dense_diag_vec(ref, 0, H_g, lp, cg, o, L, d_v, dvp, c.slots)
        worst = max(worst, np.abs(v - want).max())
    assert worst < 2.0 ** -20
    # the fold really covers every column: each (i, col < d_v) appears in exactly one dense slot
    seen = np.zeros((H_g, L, d_v), int)
    for o in range(g["n_out"]):
        for h in range(H_g):
            for kap in range(cg):
                for i in range(L):
                    col = (i + o * cg + kap) % dvp
                    if col < d_v:
                        seen[h, i, col] += 1
    assert (seen == 1).all()


def test_softmax_v_geometry_limits(orc):
    """The fold needs d_v' <= L' and c <= d_v' (one output ciphertext gathers whole diagonals);
    the ct-ct multiplication count of Softmax x V_h is m^3 H / s (Table complexity_compare)."""
    c = orc.Context(14, 2, 1, 2)
    g = c.cc_sv_geometry(8, 128, 64)
    assert (g["Lp"], g["c"], g["n_ct"], g["n_out"]) == (128, 8, 16, 8)
    g4 = c.cc_sv_geometry(4, 128, 64)
    assert (g4["c"], g4["n_ct"], g4["n_out"]) == (16, 8, 4)
    # 12 heads = 8 + 4: tensors = L' * sum n_ct = 128 * 24 = 3072 = m^3 H / s at s = 8192 slots
    assert 128 * (g["n_ct"] + g4["n_ct"]) == 128 ** 3 * 12 // 8192
    # the 12 dense outputs hold Concat(Att_h) (128 x 768) tightly: 12 = 768 * 128 / 8192
    assert g["n_out"] + g4["n_out"] == 768 * 128 // 8192
    assert c.cc_sv_geometry(1, 64, 64)["n_out"] == 0      # c = 128 > d_v' = 64
    assert c.cc_sv_geometry(8, 32, 64)["n_out"] == 0      # d_v' = 64 > L' = 32


def _diag_inputs(c, keys, att, heads, L, d_v, level, scale, seed):
    lp = 1 << int(np.ceil(np.log2(L)))
    dvp = 1 << int(np.ceil(np.log2(d_v)))
    cts, h0, a = [], 0, 0
    for H_g in _groups(heads):
        cg = c.slots // (lp * H_g)
        for o in range(dvp // cg):
            v = _dense_diag_vec(att, h0, H_g, lp, cg, o, L, d_v, dvp, c.slots)
            cts.append(keys.encrypt(c.encode_rns(v, scale, level), level, seed, a))
            a += 1
        h0 += H_g
    return np.stack(cts)


def _unpack_spatial_by_hand(vecs, lp, cc, L, D):
    out = np.zeros((L, D))
    for col in range(D):
        b, u = divmod(col, cc)
        out[:, col] = vecs[b][u * lp: u * lp + L]
    return out


@pytest.mark.parametrize("heads,L,d_v,d_out", [(3, 64, 32, 48), (2, 50, 24, 40), (4, 32, 16, 70)])
def test_matmul_cp_diag_decodes(orc, heads, L, d_v, d_out):
    """Diagonal-input ct-pt matmul: inputs in the dense diagonal packing (head groups
    concatenated, 3 heads = 2 + 1 with different c per group), output spatial-first, decodes to
    Concat(Att_h) @ W in FP64; W = I returns Concat(Att_h) itself, which pins the row map
    (head, (i + tau) mod d_v') of the plaintext diagonals on its own."""
    c = orc.Context(12, 2, 1, 2)
    rng = np.random.default_rng(heads + L + d_v)
    att = [rng.uniform(-1, 1, (L, d_v)) for _ in range(heads)]
    Cm = np.concatenate(att, axis=1)
    dvp = 1 << int(np.ceil(np.log2(d_v)))
    g = c.cp_geometry(L, heads * dvp, d_out)
    gi = c.cp_geometry(L, heads * dvp, heads * d_v)
    gal = sorted(set(c.cp_galois(L, heads * dvp, d_out)) | set(c.cp_galois(L, heads * dvp, heads * d_v)))
    keys = orc.Keys(c, 9, gal)
    X = _diag_inputs(c, keys, att, heads, L, d_v, 1, 2.0 ** 30, 100)
    assert X.shape[0] == g["n_in"]
    W = rng.normal(0, 0.05, (heads * d_v, d_out))
    Y = keys.matmul_cp_diag(X, 1, W, L, heads, d_v)
    vecs = [c.decode(keys.decrypt(Y[b], 0), 0, 2.0 ** 30) for b in range(g["n_out"])]
    assert np.abs(_unpack_spatial_by_hand(vecs, g["Lp"], g["c"], L, d_out) - Cm @ W).max() < 2.0 ** -10
    # rows past L of every output block stay (near) zero
    if L < g["Lp"]:
        for v in vecs:
            for u in range(g["c"]):
                assert np.abs(v[u * g["Lp"] + L: (u + 1) * g["Lp"]]).max() < 2.0 ** -10
    Yi = keys.matmul_cp_diag(X, 1, np.eye(heads * d_v), L, heads, d_v)
    vi = [c.decode(keys.decrypt(Yi[b], 0), 0, 2.0 ** 30) for b in range(gi["n_out"])]
    assert np.abs(_unpack_spatial_by_hand(vi, gi["Lp"], gi["c"], L, heads * d_v) - Cm).max() < 2.0 ** -12


def test_attention_output_pipeline(orc):
    """Softmax x V_h (ct-ct, zero padding, dense fold) followed by the diagonal-input ct-pt matmul
    decodes to (S_h V_h)_h concatenated times W_O: the two operators compose with no repacking."""
    H_g, L, d_v, d_out = 4, 32, 16, 24
    c, g, keys, Sm, Vm, A, Bv, level, scale = _sv_small(orc, 11, 5, H_g, L, d_v, 3)
    O = keys.matmul_cc_sv(A, Bv, level, H_g, L, d_v)
    lvl = level - 3
    out_scale = scale * 1024.0 * scale / float(c.q[level - 1])
    gcp = c.cp_geometry(L, H_g * g["dvp"], d_out)
    keys2 = orc.Keys(c, 5, sorted(set(c.cc_galois(H_g, L, L)) | set(c.cp_galois(L, H_g * g["dvp"], d_out))))
    assert np.array_equal(keys2.secret, keys.secret)
    rng = np.random.default_rng(8)
    W = rng.normal(0, 0.1, (H_g * d_v, d_out))
    E = keys2.matmul_cp_diag(O, lvl, W, L, H_g, d_v)
    vecs = [c.decode(keys2.decrypt(E[b], lvl - 1), lvl - 1, out_scale) for b in range(gcp["n_out"])]
    ref = np.concatenate([Sm[h] @ Vm[h] for h in range(H_g)], axis=1) @ W
    assert np.abs(_unpack_spatial_by_hand(vecs, gcp["Lp"], gcp["c"], L, d_out) - ref).max() < 2.0 ** -16


# --------------------------------------------------------------------------------------
# Column-reordered W_Q / W_K: matmul_cp emits the multi-head packing; fused Q K^T from X
# --------------------------------------------------------------------------------------
def _mhp_by_hand(Y, heads, d_head, L, slots):
    """operand vectors of the multi-head packing of Y_h = Y[:, h d_head:(h+1) d_head], written from
    the definition: group of H heads from h0, c = slots / (L' H), ciphertext a, block h + H kappa
    holds column a c + kappa of Y_{h0+h}"""
    lp = 1 << int(np.ceil(np.log2(L)))
    vecs, h0 = [], 0
    for H in _groups(heads):
        c = slots // (lp * H)
        for a in range(-(-d_head // c)):
            v = np.zeros(slots)
            for h in range(H):
                for kap in range(c):
                    col = a * c + kap
                    if col < d_head:
                        v[lp * (h + H * kap): lp * (h + H * kap) + L] = Y[:, (h0 + h) * d_head + col]
            vecs.append(v)
        h0 += H
    return vecs


@pytest.mark.parametrize("heads,L,d_in,d_head", [(3, 64, 40, 48), (12, 32, 64, 8)])
def test_mhp_weight_makes_cp_emit_multihead_packing(orc, heads, L, d_in, d_head):
    """matmul_cp with the column-reordered weight decodes, ciphertext by ciphertext, to the
    multi-head packing of X W (3 heads = 2 + 1 with a ragged last operand ciphertext; 12 heads =
    8 + 4, both groups with a ragged operand ciphertext); the reordering only permutes (and
    zero-pads) columns."""
    c = orc.Context(12, 2, 1, 2)
    rng = np.random.default_rng(heads + L)
    X = rng.uniform(-1, 1, (L, d_in))
    W = rng.normal(0, 0.05, (d_in, heads * d_head))
    Wp = c.mhp_weight(W, heads, d_head, L)
    nz = Wp[:, np.abs(Wp).sum(axis=0) > 0]
    assert sorted(map(tuple, nz.T)) == sorted(map(tuple, W.T))
    g = c.cp_geometry(L, d_in, Wp.shape[1])
    k = orc.Keys(c, 9, c.cp_galois(L, d_in, Wp.shape[1]))
    cts = np.stack([k.encrypt(c.encode_rns(c.pack_spatial(X, a), 2.0 ** 30, 1), 1, 100, a) for a in range(g["n_in"])])
    Y = k.matmul_cp(cts, 1, Wp, L)
    want = _mhp_by_hand(X @ W, heads, d_head, L, c.slots)
    assert len(want) == g["n_out"]
    for b in range(g["n_out"]):
        assert np.abs(c.decode(k.decrypt(Y[b], 0), 0, 2.0 ** 30) - want[b]).max() < 2.0 ** -10


def test_fused_qk_from_x(orc):
    """X -> Q = X W_Q', K = X W_K' (reordered columns) -> the ct-ct product with step 1 on the
    server, with no repacking: decodes to Q_h K_h^T for every head (six primes: one level for
    matmul_cp, four for the ct-ct product)."""
    c = orc.Context(11, 6, 2, 3)
    heads, L, d_in, d_head = 4, 32, 32, 16
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (L, d_in))
    WQ = rng.normal(0, 0.2, (d_in, heads * d_head))
    WK = rng.normal(0, 0.2, (d_in, heads * d_head))
    WQp, WKp = c.mhp_weight(WQ, heads, d_head, L), c.mhp_weight(WK, heads, d_head, L)
    g = c.cp_geometry(L, d_in, WQp.shape[1])
    gal = sorted(set(c.cp_galois(L, d_in, WQp.shape[1])) | set(c.cc_galois(heads, L, d_head)))
    k = orc.Keys(c, 7, gal)
    level, scale = 5, 2.0 ** 40
    xc = np.stack([k.encrypt(c.encode_rns(c.pack_spatial(X, a), scale, level), level, 100, a) for a in range(g["n_in"])])
    Qc = k.matmul_cp(xc, level, WQp, L)
    Kc = k.matmul_cp(xc, level, WKp, L)
    O = k.matmul_cc(Qc, Kc, level - 1, heads, L, d_head, b_prerotated=False)
    out_scale = scale * 1024.0 * scale / float(c.q[level - 3])
    geo = c.cc_geometry(heads, L, d_head)
    lp, cg = geo["Lp"], geo["c"]
    Qm, Km = X @ WQ, X @ WK
    for gi in range(geo["n_out"]):
        v = c.decode(k.decrypt(O[gi], 0), 0, out_scale)
        for h in range(heads):
            ref = Qm[:, h * d_head:(h + 1) * d_head] @ Km[:, h * d_head:(h + 1) * d_head].T
            for kap in range(cg):
                D = gi * cg + kap
                i = np.arange(L)
                got = v[i + lp * (h + heads * kap)]
                assert np.abs(got - ref[i, (i + D) % lp]).max() < 2.0 ** -14


# --------------------------------------------------------------------------------------
# Rotate-and-sum summation and broadcast; MPC-to-CKKS server step
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("block,n_blocks", [(32, 8), (16, 64)])
def test_rotate_sum_closed_forms(orc, block, n_blocks):
    """Summation: slot j < block holds sum_k m[j + k block] and every other slot 0 (the first-block
    mask); without the mask, every slot j holds sum_k m[(j + k block) mod S] (at block x n_blocks = S
    that is the row sum in every block: mask and broadcast can be skipped).  Broadcast of a vector
    living in the first block fills the first n_blocks blocks with it.  Row sums of a spatial-first
    X equal X.sum(axis=1)."""
    c = orc.Context(12, 3, 1, 3)
    S = c.slots
    steps = []
    st = block
    while st < block * n_blocks:
        steps += [st, -st]
        st *= 2
    k = orc.Keys(c, 5, sorted({c.galois_elt(x) for x in steps}))
    rng = np.random.default_rng(block)
    level, scale = 2, 2.0 ** 40
    m = rng.uniform(-1, 1, S)
    ct = k.encrypt(c.encode_rns(m, scale, level), level, 3, 0)
    idx = np.arange(S)
    cyc = sum(m[(idx + j * block) % S] for j in range(n_blocks))
    got = c.decode(k.decrypt(k.rotate_sum(ct, level, block, n_blocks, 0, mask=True), level - 1), level - 1, scale)
    want = np.where(idx < block, cyc, 0.0)
    assert np.abs(got - want).max() < 2.0 ** -20
    got = c.decode(k.decrypt(k.rotate_sum(ct, level, block, n_blocks, 0, mask=False), level), level, scale)
    assert np.abs(got - cyc).max() < 2.0 ** -20
    b0 = np.where(idx < block, m, 0.0)
    ctb = k.encrypt(c.encode_rns(b0, scale, level), level, 4, 0)
    got = c.decode(k.decrypt(k.rotate_sum(ctb, level, block, n_blocks, 1), level), level, scale)
    assert np.abs(got - np.where(idx < block * n_blocks, b0[idx % block], 0.0)).max() < 2.0 ** -20
    # row sums of a spatial-first L x D matrix (D = n_blocks columns, L' = block)
    L = block - 3
    X = rng.normal(0, 1, (L, n_blocks))
    v = np.zeros(S)
    for j in range(n_blocks):
        v[j * block: j * block + L] = X[:, j]
    ctx_ = k.encrypt(c.encode_rns(v, scale, level), level, 5, 0)
    got = c.decode(k.decrypt(k.rotate_sum(ctx_, level, block, n_blocks, 0), level - 1), level - 1, scale)
    assert np.abs(got[:L] - X.sum(axis=1)).max() < 2.0 ** -18
    assert np.abs(got[L:]).max() < 2.0 ** -18


# --------------------------------------------------------------------------------------
# Identity and Expansion operators: element-wise ct-ct / ct-pt, scalar by broadcast
# --------------------------------------------------------------------------------------
def _lift_limbs(words, mods):
    return [[int(x) for x in words[i]] for i in range(len(mods))]


def test_elementwise_add_and_plain_ops_decrypt_exactly(orc):
    """ewadd_cc, ewadd_cp and ewmul_cp against decryption, limb by limb and exactly: Dec(a + b) =
    Dec(a) + Dec(b); Dec(a + p) = Dec(a) + p; Dec(a p) = Dec(a) p with the product taken as the
    schoolbook negacyclic convolution at N = 16 (decryption is linear, so these hold word for word)."""
    for log_n in (4, 12):
        c = orc.Context(log_n, 3, 1, 3)
        k = orc.Keys(c, 9, [])
        rng = np.random.default_rng(log_n)
        level = 2
        mods = [int(q) for q in c.moduli[:level + 1]]
        a = k.encrypt(c.encode_rns(rng.normal(0, 1, c.slots), 2.0 ** 30, level), level, 1, 0)
        b = k.encrypt(c.encode_rns(rng.normal(0, 1, c.slots), 2.0 ** 30, level), level, 1, 1)
        p = np.stack([rng.integers(0, q, c.n, dtype=np.uint64) for q in mods])
        da, db = k.decrypt(a, level), k.decrypt(b, level)
        for i, q in enumerate(mods):
            assert [int(x) for x in k.decrypt(c.ew_add(a, b, level), level)[i]] == [(int(x) + int(y)) % q for x, y in zip(da[i], db[i])]
            assert [int(x) for x in k.decrypt(c.ew_add_plain(a, p, level), level)[i]] == [(int(x) + int(y)) % q for x, y in zip(da[i], p[i])]
            if log_n == 4:
                assert [int(x) for x in k.decrypt(c.ew_mul_plain(a, p, level), level)[i]] == schoolbook_negacyclic(da[i], p[i], q)


def test_elementwise_mul_relin(orc):
    """ewmul_cc: the relinearised tensor decrypts to Dec(a) Dec(b) (schoolbook at N = 16) up to a small
    key-switch term, and at N = 4096 decodes to the slot-wise product (scale Delta^2)."""
    c = orc.Context(4, 3, 1, 3)
    k = orc.Keys(c, 9, [])
    rng = np.random.default_rng(1)
    level = 2
    a = k.encrypt(c.encode_rns(rng.normal(0, 1, c.slots), 2.0 ** 20, level), level, 1, 0)
    b = k.encrypt(c.encode_rns(rng.normal(0, 1, c.slots), 2.0 ** 20, level), level, 1, 1)
    da, db = k.decrypt(a, level), k.decrypt(b, level)
    got = k.decrypt(k.ew_mul_relin(a, b, level), level)
    diff = np.zeros_like(got)
    for i in range(level + 1):
        q = int(c.moduli[i])
        prod = schoolbook_negacyclic(da[i], db[i], q)
        diff[i] = [(int(x) - y) % q for x, y in zip(got[i], prod)]
    assert _noise(c, diff, level) < 2.0 ** 20
    c = orc.Context(12, 3, 1, 3)
    k = orc.Keys(c, 9, [])
    x, y = rng.uniform(-1, 1, c.slots), rng.uniform(-1, 1, c.slots)
    a = k.encrypt(c.encode_rns(x, 2.0 ** 40, level), level, 1, 0)
    b = k.encrypt(c.encode_rns(y, 2.0 ** 40, level), level, 1, 1)
    got = c.decode(k.decrypt(k.ew_mul_relin(a, b, level), level), level, 2.0 ** 80)
    assert np.abs(got - x * y).max() < 2.0 ** -20


@pytest.mark.parametrize("op", [0, 1])
def test_scalar_ops_closed_forms_and_counts(orc, op):
    """sadd / smul (Expansion) on the spatial-first packing, L' = 32, D = 64 blocks (the whole
    ciphertext): with a scalar column s in the first block, out[j + k L'] = a[j + k L'] (+ or x) s[j];
    after a summation, out[j] = a[j] (+ or x) sum_k z[(j mod L') + k L'].  Operation counts of
    Table packing_scalar (summation followed by a scalar operator): without fusion, the masked sum
    and the broadcast take 2 log2 D rotations, one product and one level; with fusion, log2 D
    rotations, no product and no level."""
    c = orc.Context(12, 3, 1, 3)
    S, blk, D = c.slots, 32, 64
    steps = []
    st = blk
    while st < blk * D:
        steps += [st, -st]
        st *= 2
    k = orc.Keys(c, 5, sorted({c.galois_elt(x) for x in steps}))
    rng = np.random.default_rng(op)
    level, scale = 2, 2.0 ** 40
    a = rng.uniform(-1, 1, S)
    z = rng.uniform(-1, 1, S) / 8
    idx = np.arange(S)
    rowsum = sum(z[(idx % blk) + j * blk] for j in range(D))
    A = k.encrypt(c.encode_rns(a, scale, level), level, 3, 0)
    Z = k.encrypt(c.encode_rns(z, scale, level), level, 3, 1)
    out_scale = scale if op == 0 else scale * scale
    # with fusion: summation then scalar operator, no mask, no broadcast
    orc.ks_counts(reset=True)
    fused = k.scalar_op(A, Z, level, blk, D, op, from_sum=True)
    assert orc.ks_counts(reset=True)[0] == int(np.log2(D))
    got = c.decode(k.decrypt(fused, level), level, out_scale)
    want = a + rowsum if op == 0 else a * rowsum
    assert np.abs(got - want).max() < 2.0 ** -20
    # without fusion: masked summation (one product, one level), then broadcast of its first block
    s_ct = k.rotate_sum(Z, level, blk, D, 0, mask=True)
    A1 = k.encrypt(c.encode_rns(a, scale, level - 1), level - 1, 3, 2)
    out = k.scalar_op(A1, s_ct, level - 1, blk, D, op)
    assert orc.ks_counts(reset=True)[0] == 2 * int(np.log2(D))
    got = c.decode(k.decrypt(out, level - 1), level - 1, out_scale)
    assert np.abs(got - want).max() < 2.0 ** -20
    # the broadcast form on its own: a column in the first block reaches every block
    col = np.where(idx < blk, rng.uniform(-1, 1, S), 0.0)
    Sc = k.encrypt(c.encode_rns(col, scale, level), level, 3, 3)
    got = c.decode(k.decrypt(k.scalar_op(A, Sc, level, blk, D, op), level), level, out_scale)
    want = a + col[idx % blk] if op == 0 else a * col[idx % blk]
    assert np.abs(got - want).max() < 2.0 ** -20


# --------------------------------------------------------------------------------------
# complex slots and the complex-slot output packing of matmul_cp
# --------------------------------------------------------------------------------------
def test_encode_cplx_imaginary_constant_is_x_half(orc):
    """i b in every slot encodes to b Delta X^(N/2): zeta^(e N/2) = i^e = i for every slot
    exponent e = 5^j = 1 (mod 4) and -i at the conjugate exponents (catches a conjugate written to
    the wrong half or with the wrong sign)."""
    c = orc.Context(10, 1, 0, 1)
    for b, delta in [(0.5, 2.0 ** 30), (-1.75, 2.0 ** 40)]:
        p = c.encode_cplx(np.zeros(c.slots), np.full(c.slots, b), delta)
        want = np.zeros(c.n, np.int64)
        want[c.n // 2] = int(round(b * delta))
        assert np.array_equal(p, want)
        # and a real constant a plus i b gives a Delta + b Delta X^(N/2)
        p2 = c.encode_cplx(np.full(c.slots, 0.25), np.full(c.slots, b), delta)
        want[0] = int(round(0.25 * delta))
        assert np.array_equal(p2, want)


@pytest.mark.parametrize("log_n", [3, 4, 5])
def test_encode_cplx_matches_direct_formula(orc, log_n):
    """At tiny N the complex encoding equals the direct formula
    p_k = round_half_away((2 Delta / N) sum_j [a_j cos(pi 5^j k / N) + b_j sin(pi 5^j k / N)]),
    the real part of (1/N) sum over all odd r of z_r zeta^(-r k) with z at -5^j the conjugate of
    z at 5^j, evaluated in mpmath (catches a sign slip of the sine term)."""
    mpmath.mp.dps = 50
    c = orc.Context(log_n, 1, 0, 1)
    n, s = c.n, c.slots
    rng = np.random.default_rng(100 + log_n)
    a = rng.normal(0, 1, s)
    b = rng.normal(0, 1, s)
    delta = 2.0 ** 40
    got = c.encode_cplx(a, b, delta)
    for k in range(n):
        acc = mpmath.mpf(0)
        for j in range(s):
            th = mpmath.pi * (pow(5, j, 2 * n) * k) / n
            acc += mpmath.mpf(a[j]) * mpmath.cos(th) + mpmath.mpf(b[j]) * mpmath.sin(th)
        v = 2 * mpmath.mpf(delta) / n * acc
        r = int(mpmath.floor(abs(v) + mpmath.mpf("0.5")))
        assert int(got[k]) == (r if v >= 0 else -r)


def test_encode_cplx_is_real_encodings_joined_by_x_half(orc):
    """Before rounding, Encode(a + i b) = Encode(a) + X^(N/2) Encode(b) (multiplying by
    X^(N/2) multiplies every slot by i; negacyclic, so coefficient k >= N/2 wraps with a minus
    sign).  Each side rounds once per coefficient, so at N = 4096 the two differ by at most 1
    everywhere; ties aside they mostly agree exactly.  This ties the complex encoding to the real
    one pinned above."""
    c = orc.Context(12, 1, 0, 1)
    n, h = c.n, c.n // 2
    rng = np.random.default_rng(7)
    a = rng.normal(0, 1, c.slots)
    b = rng.normal(0, 1, c.slots)
    delta = 2.0 ** 38
    pa, pb = c.encode(a, delta), c.encode(b, delta)
    shifted = np.concatenate([-pb[h:], pb[:h]])  # X^(N/2) pb mod X^N + 1
    d = c.encode_cplx(a, b, delta) - (pa + shifted)
    assert np.abs(d).max() <= 1
    assert np.count_nonzero(d) < n // 2


def test_decode_cplx_inverts_encode_cplx(orc):
    """Decode of a complex encoding returns both parts within the rounding bound of the real
    decode; the real parts equal the real decode of the same polynomial; Delta X^(N/2) decodes
    to i in every slot; and the imaginary part of a decoded real encoding is (near) zero."""
    c = orc.Context(13, 3, 0, 1)
    rng = np.random.default_rng(3)
    a = rng.normal(0, 1, c.slots)
    b = rng.normal(0, 1, c.slots)
    delta = 2.0 ** 40
    pt = c.encode_rns_cplx(a, b, delta, 2)
    re, im = c.decode_cplx(pt, 2, delta)
    bound = 8 * np.sqrt(c.n / 24) / delta
    assert np.abs(re - a).max() < bound and np.abs(im - b).max() < bound
    assert np.array_equal(re, c.decode(pt, 2, delta))
    x_half = np.zeros((3, c.n), np.uint64)
    x_half[:, c.n // 2] = int(delta)
    re1, im1 = c.decode_cplx(x_half, 2, delta)
    assert np.abs(re1).max() < 1e-12 and np.abs(im1 - 1.0).max() < 1e-12
    _, im0 = c.decode_cplx(c.encode_rns(a, delta, 2), 2, delta)
    assert np.abs(im0).max() < bound


@pytest.mark.parametrize("shape", [(32, 64, 96), (20, 40, 24), (5, 96, 70), (16, 64, 160)])
def test_matmul_cp_cplx_decodes_to_fp64_matmul(orc, shape):
    """Complex-slot output packing: output ciphertext b decodes, real part, to column block 2b of
    X @ W and, imaginary part, to block 2b + 1 (FP64, within 2^-10 at Delta = 2^30); an odd block
    count leaves the last imaginary part (near) zero; a replicated packing (one block) leaves the
    whole imaginary part (near) zero.  A conjugate slip in the plaintext encoding flips the sign of
    every odd block and fails here."""
    L, d_in, d_out = shape
    c = orc.Context(12, 2, 1, 2)
    rng = np.random.default_rng(sum(shape) + 1)
    X = rng.uniform(-1, 1, (L, d_in))
    W = rng.normal(0, 0.02, (d_in, d_out))
    g = c.cp_geometry(L, d_in, d_out)
    k = orc.Keys(c, 9, c.cp_galois(L, d_in, d_out))
    cts = np.stack([k.encrypt(c.encode_rns(c.pack_spatial(X, a), 2.0 ** 30, 1), 1, 100, a) for a in range(g["n_in"])])
    Y = k.matmul_cp(cts, 1, W, L, cplx=True)
    assert Y.shape[0] == (g["n_out"] + 1) // 2
    vecs = []
    for b in range(Y.shape[0]):
        re, im = c.decode_cplx(k.decrypt(Y[b], 0), 0, 2.0 ** 30)
        vecs += [re, im]
    got = _unpack(c, g, vecs[: g["n_out"]], L, d_out)
    assert np.abs(got - X @ W).max() < 2.0 ** -10
    if g["n_out"] % 2:
        assert np.abs(vecs[g["n_out"]]).max() < 2.0 ** -10


def test_matmul_cp_cplx_counts(orc):
    """At the BERT-base shape (L = 128, 768 x 768, N = 16384) the complex packing keeps the baby
    steps and halves the plaintexts, the output ciphertexts and the giant-step rotations:
    24 x 12 x 32 = 9216 plaintexts (18432 real), 24 x 7 + 12 x 3 = 204 rotations (240 real)."""
    c2 = orc.Context(13, 3, 1, 3)
    g = c2.cp_geometry(128, 768, 768)
    n_out_c = (g["n_out"] + 1) // 2
    assert n_out_c == 12
    assert g["n_in"] * n_out_c * g["c_eff"] == 9216
    assert g["n_in"] * (g["B"] - 1) + n_out_c * (g["G"] - 1) == 204


@pytest.mark.parametrize("heads,L,d_v,d_out", [(3, 64, 32, 48), (4, 32, 16, 70)])
def test_matmul_cp_diag_cplx_decodes(orc, heads, L, d_v, d_out):
    """The diagonal-input ct-pt matmul in the complex-slot output packing decodes to
    Concat(Att_h) @ W, real parts block 2b and imaginary parts block 2b + 1."""
    c = orc.Context(12, 2, 1, 2)
    rng = np.random.default_rng(heads + L + d_v + 1)
    att = [rng.uniform(-1, 1, (L, d_v)) for _ in range(heads)]
    Cm = np.concatenate(att, axis=1)
    dvp = 1 << int(np.ceil(np.log2(d_v)))
    g = c.cp_geometry(L, heads * dvp, d_out)
    keys = orc.Keys(c, 9, c.cp_galois(L, heads * dvp, d_out))
    X = _diag_inputs(c, keys, att, heads, L, d_v, 1, 2.0 ** 30, 100)
    W = rng.normal(0, 0.05, (heads * d_v, d_out))
    Y = keys.matmul_cp_diag(X, 1, W, L, heads, d_v, cplx=True)
    assert Y.shape[0] == (g["n_out"] + 1) // 2
    vecs = []
    for b in range(Y.shape[0]):
        re, im = c.decode_cplx(keys.decrypt(Y[b], 0), 0, 2.0 ** 30)
        vecs += [re, im]
    assert np.abs(_unpack_spatial_by_hand(vecs, g["Lp"], g["c"], L, d_out) - Cm @ W).max() < 2.0 ** -10
