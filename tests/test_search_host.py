"""The device key searches of `paper_1708_07859_amd/csrc/search.h`, run on
the host (compiled with g++ against the host stand-in of
tests/exact_host/hip) and checked against numpy's searchsorted: counts of
keys <= x in any sub-range, and lower bounds through the line samples, on
sorted sets with duplicates, gaps, single keys, empty ranges, ranges that
start or end inside a line, and keys at 0 and 2^32 - 1."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER_SRC = os.path.join(HERE, "search_host", "driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("search") / "driver")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", os.path.join(HERE, "exact_host"), "-o", exe,
                           DRIVER_SRC])
    return exe


def run(exe, keys, queries):
    lines = [str(len(keys)), " ".join(str(int(k)) for k in keys), str(len(queries))]
    lines += [f"{b} {e} {x}" for b, e, x in queries]
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    return np.array([[int(t) for t in ln.split()] for ln in out.stdout.split("\n") if ln], dtype=np.int64)


def check(exe, keys, queries):
    got = run(exe, keys, queries)
    for (b, e, x), (c, lb) in zip(queries, got):
        seg = keys[b:e]
        assert c == int(np.searchsorted(seg, x, side="right")), (b, e, x, c)
        assert lb == b + int(np.searchsorted(seg, x, side="left")), (b, e, x, lb)


@pytest.mark.parametrize("seed,n,universe,dup", [(1, 1, 10, False), (2, 31, 100, False), (3, 33, 100, True),
                                                  (4, 1000, 1 << 20, False), (5, 4097, 10000, True),
                                                  (6, 20000, 1 << 32, False)])
def test_searches_match_searchsorted(driver, seed, n, universe, dup):
    rng = np.random.default_rng(seed)
    if dup:
        keys = np.sort(rng.integers(0, universe, n, dtype=np.uint64))
    else:
        keys = np.sort(rng.choice(universe, n, replace=False).astype(np.uint64))
    if universe == 1 << 32:
        keys[0], keys[-1] = 0, (1 << 32) - 1
    queries = []
    for _ in range(400):
        b = int(rng.integers(0, n + 1))
        e = int(rng.integers(b, n + 1))
        kind = rng.integers(0, 4)
        if kind == 0 and e > b:
            x = int(keys[rng.integers(b, e)])          # a present key
        elif kind == 1 and e > b:
            x = int(keys[rng.integers(b, e)]) + 1      # just past one
        elif kind == 2:
            x = int(rng.choice([0, 1, (1 << 32) - 1]))
        else:
            x = int(rng.integers(0, 1 << 32))
        queries.append((b, e, min(x, (1 << 32) - 1)))
    # whole set, line-aligned and unaligned bounds
    queries += [(0, n, int(keys[n // 2])), (0, n, 0), (0, n, (1 << 32) - 1)]
    if n > 70:
        queries += [(32, 64, int(keys[40])), (31, 65, int(keys[64])), (5, 70, int(keys[5]) - 1 if keys[5] else 0)]
    check(driver, keys, queries)
