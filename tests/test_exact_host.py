"""The device exact accumulator's arithmetic, run on the host.

`paper_1708_07859_amd/csrc/exact.h` is compiled with g++ against a host
stand-in for its few HIP builtins (tests/exact_host/hip/hip_runtime.h) and
checked against exact rational sums (`fractions.Fraction`, whose float()
rounds correctly, ties to even).  This pins the parts a GPU test can only
reach at huge sizes: row multiplicities up to 2^64 - 1, and shared slots
that wrap modulo 2^64 and must carry into the next slot.
"""
import os
import random
import struct
import subprocess
from fractions import Fraction

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER_SRC = os.path.join(HERE, "exact_host", "driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("exact") / "driver")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", os.path.join(HERE, "exact_host"), "-o", exe,
                           DRIVER_SRC])
    return exe


def bits_of(v):
    return struct.unpack("<Q", struct.pack("<d", v))[0]


def run(exe, D, lsb, terms, init=None):
    """terms: (mode, value, mult); init: D unsigned slot values."""
    init = init or [0] * D
    lines = [f"{D} {lsb}", " ".join(str(u) for u in init)]
    lines += [f"{m} {bits_of(v)} {mult}" for m, v, mult in terms]
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    ok, ovf, rb, *parts = out.stdout.split()
    run.parts = [struct.unpack("<d", struct.pack("<Q", int(p)))[0] for p in parts]
    return int(ok), int(ovf), struct.unpack("<d", struct.pack("<Q", int(rb)))[0]


def slot_value(init, lsb):
    """Value of shared-form slots: all but the top unsigned, the top signed."""
    D = len(init)
    tot = 0
    for i, u in enumerate(init):
        if i == D - 1 and u >= 1 << 63:
            u -= 1 << 64
        tot += u << (32 * i)
    return Fraction(tot) * Fraction(2) ** lsb


def want(terms, lsb=0, init=None):
    s = sum((Fraction(v) * m for _, v, m in terms), Fraction(0))
    if init:
        s += slot_value(init, lsb)
    return float(s)


def test_single_terms_both_paths(driver):
    for mode in (0, 1):
        for v in (0.5, -0.25, 1.0, -(2.0 ** -100), 3.0 * 2 ** -106):
            ok, ovf, got = run(driver, 5, -106, [(mode, v, 1)])
            assert ok == 1 and ovf == 0 and got == v


def test_multiplicity_beyond_2_30(driver):
    # a term repeated 2^32 and 2^64 - 1 times (rows of unannotated bag relations)
    v = 1.0 - 2.0 ** -53            # full 53-bit mantissa
    for mode in (0, 1):
        for mult in (1 << 30, 1 << 32, (1 << 32) + 12345, (1 << 64) - 1):
            terms = [(mode, v, mult), (mode, -v / 3, 7)]
            D = 6
            ok, ovf, got = run(driver, D, -106, terms)
            assert ok == 1 and ovf == 0
            assert got == want(terms), (mode, mult)


def test_random_terms_order_free(driver):
    rng = random.Random(7)
    terms = []
    for _ in range(400):
        e = rng.randint(-40, 10)
        v = (rng.random() * 2 - 1) * 2.0 ** e
        terms.append((rng.randint(0, 1), v, rng.choice([1, 1, 2, 1 << 20, 1 << 33])))
    # lsb low enough for every term: multiples of 2^(e - 53) with e >= -40
    lsb = -100
    ok, ovf, got = run(driver, 6, lsb, terms)
    assert ok == 1 and ovf == 0
    assert got == want(terms)
    rng.shuffle(terms)
    ok2, _, got2 = run(driver, 6, lsb, terms)
    assert bits_of(got2) == bits_of(got)


def test_cancellation_to_tiny(driver):
    big = 2.0 ** 30
    terms = [(1, big, 1 << 40), (0, -big, 1 << 40), (1, 2.0 ** -90, 3)]
    ok, ovf, got = run(driver, 6, -106, terms)
    assert ok == 1 and ovf == 0 and got == 3 * 2.0 ** -90


@pytest.mark.parametrize("start", [(1 << 64) - 5, (1 << 63) - 3, (1 << 64) - (1 << 32)])
def test_shared_slot_wraps_carry(driver, start):
    # slot 0 (and 1) start at the edge of 2^64: additions that wrap them
    # must move 2^32 into the next slot, subtractions that borrow take it back
    D, lsb = 4, 0
    init = [start, start, 0, 0]
    terms = [(1, 7.0, 1), (1, 2.0 ** 32 * 3, 1), (1, 123456789.0, 1 << 40), (1, -5.0, 1), (1, -(2.0 ** 40), 9)]
    ok, ovf, got = run(driver, D, lsb, terms, init)
    assert ok == 1 and ovf == 0
    assert got == want(terms, lsb, init)


def test_borrow_below_zero(driver):
    # a negative term on zeroed slots borrows through every lower slot into
    # the signed top slot
    D, lsb = 4, 0
    terms = [(1, -1.0, 1), (1, -(2.0 ** 50), 3), (1, 2.0 ** 20, 1)]
    ok, ovf, got = run(driver, D, lsb, terms)
    assert ok == 1 and ovf == 0
    assert got == want(terms)


def test_term_below_window_reported(driver):
    for mode in (0, 1):
        ok, _, _ = run(driver, 4, -10, [(mode, 2.0 ** -20, 1)])
        assert ok == 0


def test_value_above_window_flags_overflow(driver):
    # D = 2 digits at lsb 0 hold |x| < 2^63: four terms of 2^62 do not fit
    ok, ovf, _ = run(driver, 2, 0, [(1, 2.0 ** 62, 1)] * 4)
    assert ok == 1 and ovf == 1


def test_exact_parts_sum_to_the_value(driver):
    # the parts a multi-node plan hands up: their exact sum is the value, the
    # first is the correctly rounded sum, and they do not overlap
    rng = random.Random(11)
    for trial in range(30):
        terms = [(1, (rng.random() * 2 - 1) * 2.0 ** rng.randint(-45, 20), rng.choice([1, 3, 1 << 40]))
                 for _ in range(rng.randint(1, 60))]
        D, lsb = 8, -110
        ok, ovf, got = run(driver, D, lsb, terms)
        parts = run.parts
        exact = sum((Fraction(v) * m for _, v, m in terms), Fraction(0))
        assert ok == 1 and ovf == 0
        assert got == float(exact) == parts[0]
        assert sum((Fraction(p) for p in parts), Fraction(0)) == exact
        nz = [p for p in parts if p != 0.0]
        assert parts[:len(nz)] == nz                     # zeros only at the end
        for a, b in zip(nz, nz[1:]):
            assert abs(b) <= abs(a) * 2.0 ** -53         # each below half an ulp of the one before
