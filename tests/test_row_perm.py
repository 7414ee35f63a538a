"""The learned pruner's epoch order (csrc/row_perm.h), checked on the host:
built with g++ from the same header the device code includes, the order of
every (n, seed, epoch) visits each row exactly once (a bijection of 0..n-1),
different epochs and seeds give different orders, and the Feistel domain is
below 4n, which bounds the mean cycle walk."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_17118_amd", "csrc")
SIZES = [1, 2, 3, 5, 127, 128, 129, 1000, 4096, 65537, 1_000_003]


@pytest.fixture(scope="module")
def rows(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path_factory.mktemp("rp") / "row_perm_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "row_perm_check.cpp"), "-o", exe],
                   check=True)
    out = subprocess.run([exe] + [str(n) for n in SIZES], check=True, capture_output=True,
                         text=True).stdout
    return [line.split() for line in out.strip().splitlines()]


def test_every_order_is_a_bijection(rows):
    assert len(rows) == len(SIZES) * 3 * 3
    bad = [r for r in rows if r[3] != "1"]
    assert not bad, bad


def test_domain_bounds_the_walk(rows):
    for n, _, _, _, ratio, _, _, dom in rows:
        assert int(dom) >= int(n) and float(ratio) < 4.0 + 1e-12, (n, dom)


def test_orders_differ_between_epochs_and_seeds(rows):
    # the first index of the order, over 9 (seed, epoch) pairs, for large n
    for n in (65537, 1_000_003):
        firsts = {r[6] for r in rows if int(r[0]) == n}
        assert len(firsts) >= 8, (n, firsts)
        # a shuffle leaves about one fixed point on average, never most rows
        assert all(int(r[5]) < 50 for r in rows if int(r[0]) == n)
