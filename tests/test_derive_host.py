"""The cascade-input derivation shared by the host cascade and the
device-resident one (csrc/derive.hpp), compiled on the host with g++: the
128-bit radicand's conversion rounds exactly like the compiler's own
(double)(__int128), and the nine derived inputs equal the oracle's on
random integer feature vectors, bit for bit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from helpers import ROOT

DRIVER = r"""
#include <cstdio>
#include <cstdint>
#include <cstring>
#include "derive.hpp"
int main() {
    char mode[8];
    while (scanf("%7s", mode) == 1) {
        if (mode[0] == 'c') {            // conversion: hi lo (unsigned)
            unsigned long long hi, lo;
            if (scanf("%llu %llu", &hi, &lo) != 2) return 1;
            unsigned __int128 v = ((unsigned __int128)hi << 64) | lo;
            double a = ck::u128_to_double(v), b = (double)(__int128)v;
            unsigned long long ua, ub;
            memcpy(&ua, &a, 8); memcpy(&ub, &b, 8);
            printf("%llu %llu\n", ua, ub);
        } else {                         // derivation: 28 integers
            int64_t I[28];
            for (int k = 0; k < 28; ++k)
                if (scanf("%lld", (long long *)&I[k]) != 1) return 1;
            double d[9];
            ck::derive_inputs(I, d);
            for (int k = 0; k < 9; ++k) {
                unsigned long long u;
                memcpy(&u, &d[k], 8);
                printf("%llu ", u);
            }
            printf("\n");
        }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("derive")
    src = d / "derive_driver.cpp"
    src.write_text(DRIVER)
    exe = d / "derive_driver"
    subprocess.run([gxx, "-std=c++17", "-O2", "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas",
                    "-I", os.path.join(ROOT, "paper_2411_10143_amd", "csrc"), str(src), "-o",
                    str(exe)], check=True)
    return str(exe)


def test_u128_conversion_rounds_to_nearest_even(driver):
    rng = np.random.default_rng(3)
    vals = []
    for bits in list(range(50, 128)):
        for _ in range(40):
            v = int(rng.integers(0, 2 ** 62)) << max(0, bits - 62) | int(rng.integers(0, 2 ** 62))
            v &= (1 << bits) - 1
            v |= 1 << (bits - 1)
            vals.append(v)
        # exact halfway cases and their neighbours (ties to even, both parities)
        if bits > 54:
            s = bits - 53
            for m in (2 ** 52 + 1, 2 ** 52 + 2, 2 ** 53 - 1):
                for off in (-1, 0, 1):
                    vals.append((m << s) + (1 << (s - 1)) + off)
    vals = [v for v in vals if 0 <= v < 2 ** 127]
    inp = "\n".join(f"c {v >> 64} {v & (2 ** 64 - 1)}" for v in vals) + "\n"
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout
    for v, line in zip(vals, out.splitlines()):
        a, b = line.split()
        assert a == b, v
    assert len(out.splitlines()) == len(vals)


def test_derivation_equals_oracle(driver, orc):
    rng = np.random.default_rng(4)
    rows = []
    for _ in range(3000):
        n = int(rng.integers(1, 3_000_000))
        ncols = int(rng.integers(1, 3_000_000))
        mean = float(rng.uniform(0.1, 500.0))
        nnz = int(n * mean)
        kmin = max(1, -(-nnz // n))                 # sum_r2 >= sum_r^2 / n (Cauchy-Schwarz)
        mx = int(rng.integers(kmin, 20_000))
        sum_r2 = nnz * int(rng.integers(kmin, mx + 1))
        ints = [n, ncols, nnz, nnz, sum_r2, mx, int(rng.integers(0, 3)),
                int(rng.integers(0, n * 1000)), int(rng.integers(n, n * 10)),
                int(rng.integers(1, n + ncols)), int(rng.integers(0, n))] + [0] * 16 + [0]
        rows.append(ints)
    rows.append([0] * 28)                                  # no rows
    rows.append([5, 7, 0, 0, 0, 0, 0, 0, 0, 0, 0] + [5] + [0] * 15 + [1])   # no entries
    inp = "\n".join("d " + " ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout
    for r, line in zip(rows, out.splitlines()):
        got = np.array([int(u) for u in line.split()], dtype=np.uint64).view(np.float64)
        ref = orc.derive(np.array(r, dtype=np.int64))
        assert np.array_equal(got.view(np.uint64), np.asarray(ref, dtype=np.float64).view(np.uint64)), r
