"""CPU checks of the exact member sums of the mean step
(paper_1805_00569_amd/csrc/exact_sum.hpp), through tests/exact_sum_check.cpp:
the limbs, their normalisation, the combination of partial limb sets and the
final rounding give the exactly rounded sum -- the rational sum of the values
(Python's Fraction) rounded to the nearest double, ties to even -- for FP32
and FP64 values over their whole range: subnormals, the largest finite
values, cancellation to zero and to tiny remainders, exact halfway cases in
both rounding directions, sums that carry into the next binade, and
thousands of terms spread over many accumulators."""
import os
import shutil
import struct
import subprocess
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path_factory.mktemp("xs") / "exact_sum_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "exact_sum_check.cpp")], check=True,
                   capture_output=True)
    return exe


def _gpu_style_sum(exe, vals, kind, accs):
    if kind == "f":
        lines = [f"{struct.unpack('<I', struct.pack('<f', float(v)))[0]:x}" for v in vals]
    else:
        lines = [f"{struct.unpack('<Q', struct.pack('<d', float(v)))[0]:x}" for v in vals]
    r = subprocess.run([exe], input=f"{kind} {accs}\n" + "\n".join(lines) + "\n", capture_output=True, text=True,
                       timeout=60)
    assert r.returncode == 0, r.stderr
    return struct.unpack("<d", struct.pack("<Q", int(r.stdout.strip(), 16)))[0]


def _exactly_rounded(vals, kind):
    conv = (lambda v: Fraction(float(np.float32(v)))) if kind == "f" else (lambda v: Fraction(float(v)))
    s = sum((conv(v) for v in vals), Fraction(0))
    return float(s)   # int / int true division: correctly rounded, ties to even


def _check(exe, vals, kind, accs=(1, 7, 64)):
    want = _exactly_rounded(vals, kind)
    for a in accs:
        got = _gpu_style_sum(exe, vals, kind, a)
        assert got == want and (got != 0 or struct.pack("<d", got) == struct.pack("<d", 0.0)), (kind, a, got, want)


@pytest.mark.parametrize("kind", ["f", "d"])
def test_random_wide_range(checker, kind):
    g = np.random.default_rng(1 if kind == "f" else 2)
    lo, hi = (-140, 120) if kind == "f" else (-1060, 1000)
    for case in range(6):
        n = int(g.integers(1, 3000))
        e = g.integers(lo, hi, n) if case % 2 == 0 else g.integers(-20, 20, n)
        vals = g.standard_normal(n) * np.exp2(e.astype(float))
        if kind == "f":
            vals = vals.astype(np.float32)
        _check(checker, vals.tolist(), kind)


@pytest.mark.parametrize("kind", ["f", "d"])
def test_special_values(checker, kind):
    if kind == "f":
        tiny, big = float(np.float32(2.0 ** -149)), float(np.finfo(np.float32).max)
    else:
        tiny, big = 2.0 ** -1074, float(np.finfo(np.float64).max) / 4
    cases = [
        [0.0], [-0.0, -0.0], [tiny], [-tiny, tiny], [tiny] * 1000, [big, big, -big],
        [big, -big, tiny],   # cancellation to the smallest subnormal
        [1.0, -1.0] * 500,   # exact zero after many terms
        [3.0, -1.0, 2.0 ** -30, -(2.0 ** -30)],
    ]
    for vals in cases:
        _check(checker, vals, kind)


def test_halfway_cases_round_to_even(checker):
    # 1 + 2^-53 lies halfway between 1 and 1 + 2^-52: ties go to the even 1;
    # 1 + 3 * 2^-53 lies halfway between 1 + 2^-52 and 1 + 2^-51: ties to the latter
    for vals, want in [([1.0, 2.0 ** -53], 1.0), ([1.0 + 2.0 ** -52, 2.0 ** -53], 1.0 + 2.0 ** -51),
                       ([1.0, 2.0 ** -53, 2.0 ** -200], 1.0 + 2.0 ** -52),   # sticky bit breaks the tie
                       ([-1.0, -(2.0 ** -53)], -1.0)]:
        assert _exactly_rounded(vals, "d") == want
        _check(checker, vals, "d")
    # FP32 terms whose exact sum needs more than 53 bits
    vals = [float(np.float32(2.0 ** 100)), float(np.float32(1.0)), float(np.float32(2.0 ** -100))]
    _check(checker, vals, "f")


def test_carry_into_next_binade_and_long_sums(checker):
    _check(checker, [1.0 - 2.0 ** -53] * 3, "d")   # 3 - 3 * 2^-53 rounds across the binade
    g = np.random.default_rng(7)
    vals = (g.uniform(0.5, 2.0, 20000) * g.choice([-1.0, 1.0], 20000)).astype(np.float32)
    _check(checker, vals.tolist(), "f", accs=(1, 16, 256))
