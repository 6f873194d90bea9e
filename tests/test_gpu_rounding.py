"""Correctly rounded binary64 division and square root in device code
(paper_2104_04347_amd/csrc/wcc_rn.hpp).

The binary64 results of the kernels equal the oracle's bit for bit only if
every quotient and square root is the IEEE round-to-nearest-even value, as on
the CPU.  The operands that separate a faithful routine from a correctly
rounded one are those whose exact result lies very near the midpoint of two
binary64 neighbours; random operands almost never do.  The generators below
build such operands in exact integer arithmetic, the CPU tests check that
they are what they claim and that numpy's results are the exactly rounded
ones, and the GPU test runs the device helpers on them (tests/rn/rn_check,
built by build()) and compares bit for bit with numpy."""
import math
import os
import random
import subprocess
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "rn", "rn_check")
TWO53 = 1 << 53
# the quotient that the compiler's division returned one unit low in a limited
# Sod run (a denominator just below a power of two)
OBSERVED = (float.fromhex("0x1.6666666666663p-2"), float.fromhex("0x1.ffffffffffffbp-4"))


def near_tie_quotients(n: int, seed: int, family: str = "random"):
    """n pairs (a, b) whose exact quotient lies within |t| / (2 B) units in
    the last place of a rounding midpoint (|t| <= 4000, B >= 2^52).

    With B the 53-bit odd significand of b and M an odd integer in
    [2^53, 2^54), choose M = t B^-1 (mod 2^53); then B M - t is a multiple
    of 2^53 and A = (B M - t) / 2^53 gives A / B = M / 2^53 - t / (B 2^53):
    M / 2^53 is the midpoint between two binary64 numbers of [1, 2), and the
    quotient misses it by t / (B 2^53).  family: "random" B, "below" B =
    2^53 - k or "above" B = 2^52 + k for small odd k (divisors next to a
    power of two)."""
    rng = random.Random(seed)
    out = []
    while len(out) < n:
        if family == "random":
            B = rng.randrange(TWO53 // 2, TWO53) | 1
        elif family == "below":
            B = TWO53 - (2 * rng.randrange(0, 2000) + 1)
        else:
            B = TWO53 // 2 + (2 * rng.randrange(0, 2000) + 1)
        t = rng.randint(-4000, 4000)
        if t == 0:
            continue
        M = (t * pow(B, -1, TWO53)) % TWO53 + TWO53
        if M % 2 == 0:
            continue
        A, rem = divmod(B * M - t, TWO53)
        assert rem == 0
        if not TWO53 // 2 <= A < TWO53:
            continue
        a = math.ldexp(float(A), rng.randint(-40, 40))
        b = math.ldexp(float(B), rng.randint(-40, 40))
        out.append((-a if rng.random() < 0.5 else a, -b if rng.random() < 0.5 else b))
    return np.array(out, dtype=np.float64).reshape(-1, 2)


def _sqrt_mod_pow2(t: int, k: int) -> int:
    """r with r^2 = t (mod 2^k), for t = 1 (mod 8): lift a root mod 2^j to
    one mod 2^(j+1) by adding 2^(j-1) where needed."""
    assert t % 8 == 1
    r = 1
    for j in range(3, k):
        if (r * r - t) % (1 << (j + 1)):
            r += 1 << (j - 1)
    return r % (1 << k)


def near_tie_square_roots(n: int, seed: int):
    """n operands x whose exact square root lies within ~t / 2^55 units in
    the last place of a rounding midpoint.

    With M odd in [2^53, 2^53.5) and M^2 = t (mod 2^54), X = (M^2 - t) / 2^54
    is a 53-bit integer and sqrt(X) = (M / 2^27) sqrt(1 - t / M^2): M / 2^27
    is an odd multiple of half the spacing of binary64 numbers at sqrt(X)."""
    rng = random.Random(seed)
    lo, hi = TWO53, int(math.isqrt(2 * TWO53 * TWO53)) + 1   # [2^53, 2^53.5)
    out = []
    while len(out) < n:
        t = 8 * rng.randrange(0, 3000) + 1
        r = _sqrt_mod_pow2(t, 54)
        for M in {r, (1 << 54) - r, (r + TWO53) % (1 << 54), (TWO53 - r) % (1 << 54)}:
            if not (lo <= M < hi and M % 2 == 1 and (M * M - t) % (1 << 54) == 0):
                continue
            X = (M * M - t) >> 54
            if TWO53 // 2 <= X < TWO53:
                out.append(math.ldexp(float(X), 2 * rng.randint(-60, 60)))
    return np.array(out[:n], dtype=np.float64)


def rn_fraction(x: Fraction) -> float:
    """The binary64 number nearest to the positive rational x (normal range;
    ties to even), by integer arithmetic."""
    assert x > 0
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    s = x / Fraction(2) ** (e - 52)          # in [2^52, 2^53)
    m, rem = divmod(s.numerator, s.denominator)
    r2 = 2 * rem
    if r2 > s.denominator or (r2 == s.denominator and m % 2 == 1):
        m += 1
    return math.ldexp(float(m), e - 52)


def ulps_to_midpoint(x: Fraction) -> Fraction:
    """Distance of x > 0 from the nearest midpoint of binary64 neighbours, in
    units in the last place."""
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    s = x / Fraction(2) ** (e - 52)
    frac = s - math.floor(s)
    return abs(frac - Fraction(1, 2))


# -- CPU: the generators make near-ties, and numpy rounds them correctly ------


@pytest.mark.parametrize("family", ["random", "below", "above"])
def test_quotient_generator_makes_near_ties(family):
    ab = near_tie_quotients(300, seed=11, family=family)
    for a, b in ab:
        x = abs(Fraction(a) / Fraction(b))
        assert 0 < ulps_to_midpoint(x) < Fraction(1, 1 << 40)
        assert abs(np.float64(a) / np.float64(b)) == rn_fraction(x)


def test_square_root_generator_makes_near_ties():
    xs = near_tie_square_roots(300, seed=12)
    assert len(xs) == 300
    for x in xs:
        s = float(np.sqrt(np.float64(x)))
        # bracket sqrt(x) between the midpoints next to s, exactly: the
        # correctly rounded s satisfies (s - h)^2 < x < (s + h)^2
        h = Fraction(math.ulp(s)) / 2
        fs, fx = Fraction(s), Fraction(x)
        assert (fs - h) ** 2 < fx < (fs + h) ** 2
        # and the exact root is near one of the two midpoints
        d = min(abs(fx - (fs - h) ** 2), abs((fs + h) ** 2 - fx)) / (2 * fs * 2 * h)
        assert d < Fraction(1, 1 << 40)


def test_observed_case_is_a_near_tie():
    a, b = OBSERVED
    x = Fraction(a) / Fraction(b)
    assert ulps_to_midpoint(x) < Fraction(1, 1 << 20)
    assert a / b == rn_fraction(x) == float.fromhex("0x1.6666666666667p+1")


def test_rn_fraction_against_known_values():
    assert rn_fraction(Fraction(1, 3)) == 1 / 3
    assert rn_fraction(Fraction(2, 3)) == 2 / 3
    # the midpoint between 1 and 1 + 2^-52 rounds to even (1.0); just above it, up
    assert rn_fraction(1 + Fraction(1, 1 << 53)) == 1.0
    assert rn_fraction(1 + Fraction(1, 1 << 53) + Fraction(1, 1 << 80)) == 1 + 2.0 ** -52
    # 1 + 1.5 units: a tie between 1 + 2^-52 (odd) and 1 + 2^-51 (even)
    assert rn_fraction(1 + Fraction(3, 1 << 53)) == 1 + 2.0 ** -51
    assert rn_fraction(1 + Fraction(5, 1 << 53)) == 1 + 2.0 ** -51


# -- GPU ---------------------------------------------------------------------


def _special_quotients():
    big, tiny = 2.0 ** 1000, 2.0 ** -1000
    vals = [0.0, -0.0, 1.0, -3.0, np.inf, -np.inf, np.nan, big, tiny, 5e-324]
    return np.array([(a, b) for a in vals for b in vals], dtype=np.float64)


def _special_roots():
    return np.array([0.0, -0.0, 1.0, 4.0, 2.0, -1.0, np.inf, -np.inf, np.nan, 5e-324, 2.0 ** -1030, 2.0 ** -960,
                     2.0 ** 1000, 2.0 ** 1023, np.finfo(np.float64).max], dtype=np.float64)


def _run(tmp_path, ab, xs):
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built (run __graft_entry__.build())")
    ab.T.copy().tofile(tmp_path / "div.bin")            # n numerators, then n denominators
    xs.tofile(tmp_path / "sqrt.bin")
    print("rn_check:", len(ab), "quotients,", len(xs), "square roots", flush=True)
    r = subprocess.run([EXE, str(tmp_path / "div.bin"), str(tmp_path / "sqrt.bin"), str(tmp_path / "out.bin")],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = np.fromfile(tmp_path / "out.bin", dtype=np.float64)
    n, m = len(ab), len(xs)
    assert out.size == 2 * n + 2 * m
    return out[:n], out[n:2 * n], out[2 * n:2 * n + m], out[2 * n + m:]


def _same_bits(x, y):
    return (x.view(np.uint64) == y.view(np.uint64)) | (np.isnan(x) & np.isnan(y))


@pytest.mark.gpu
def test_device_division_and_square_root_are_correctly_rounded(tmp_path):
    rng = np.random.default_rng(5)
    ties = np.concatenate([near_tie_quotients(60000, 1, "random"), near_tie_quotients(20000, 2, "below"),
                           near_tie_quotients(20000, 3, "above"), np.array([OBSERVED])])
    # random significands over exponents where the remainder is exact
    rand = np.ldexp(rng.uniform(1.0, 2.0, (100000, 2)) * rng.choice([-1.0, 1.0], (100000, 2)),
                    rng.integers(-400, 400, (100000, 2)))
    special = _special_quotients()
    ab = np.concatenate([ties, rand, special])
    xs_ties = near_tie_square_roots(40000, 4)
    xs_rand = np.ldexp(rng.uniform(1.0, 2.0, 100000), rng.integers(-900, 900, 100000))
    xs = np.concatenate([xs_ties, xs_rand, _special_roots()])
    q_rn, q_hw, s_rn, s_hw = _run(tmp_path, ab, xs)
    with np.errstate(all="ignore"):
        q_ref = ab[:, 0] / ab[:, 1]
        s_ref = np.sqrt(xs)
    print("compiler's division: %d of %d near-tie quotients not correctly rounded; sqrt: %d of %d"
          % ((~_same_bits(q_hw[:len(ties)], q_ref[:len(ties)])).sum(), len(ties),
             (~_same_bits(s_hw[:len(xs_ties)], s_ref[:len(xs_ties)])).sum(), len(xs_ties)), flush=True)

    # bit for bit: zero, infinite and NaN operands, overflowing quotients,
    # and |a| >= 2^-969 with a normal quotient; elsewhere (subnormal or
    # underflowing quotients, tiny numerators) within one unit in the last place
    a, b = ab[:, 0], ab[:, 1]
    special = (a == 0) | (b == 0) | ~np.isfinite(a) | ~np.isfinite(b) | np.isinf(q_ref)
    in_dom = special | ((np.abs(a) >= 2.0 ** -969) & (np.abs(q_ref) >= np.finfo(np.float64).tiny))
    bad = np.flatnonzero(in_dom & ~_same_bits(q_rn, q_ref))
    assert bad.size == 0, [(a[i].hex(), b[i].hex(), q_ref[i].hex(), q_rn[i].hex()) for i in bad[:5]]
    assert np.isinf(q_ref).sum() >= 4          # overflows among the special cases
    out_dom = np.flatnonzero(~in_dom)
    assert out_dom.size > 0
    d = np.abs(q_rn[out_dom].view(np.int64) - q_ref[out_dom].view(np.int64))
    assert (d <= 1).all()

    s_dom = ((xs >= 2.0 ** -960) & (xs < 2.0 ** 1000)) | ~np.isfinite(xs) | (xs <= 0)
    bad = np.flatnonzero(s_dom & ~_same_bits(s_rn, s_ref))
    assert bad.size == 0, [(xs[i].hex(), s_ref[i].hex(), s_rn[i].hex()) for i in bad[:5]]
    out_dom = np.flatnonzero(~s_dom)
    d = np.abs(s_rn[out_dom].view(np.int64) - s_ref[out_dom].view(np.int64))
    assert (d <= 1).all()
