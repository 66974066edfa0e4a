"""The request loop's admission scan (csrc/admit.hpp), compiled on the host
with g++ and run on scripted queues: each path first-come first-served, a
request waiting for a slot or worker does not hold back the other path, and
one waiting for memory holds back both."""
import os
import shutil
import subprocess

import pytest

from helpers import ROOT

DRIVER = r"""
#include <cstdio>
#include <deque>
#include "admit.hpp"
// request: path (0 small, 1 large) and bytes; the simulated loop has free
// slots per path and a memory budget
struct Req { int id, path, bytes; };
int main() {
    int cases;
    if (scanf("%d", &cases) != 1) return 1;
    for (int c = 0; c < cases; ++c) {
        int n, slots[2], mem;
        if (scanf("%d %d %d %d", &n, &slots[0], &slots[1], &mem) != 4) return 1;
        std::deque<Req> q;
        for (int i = 0; i < n; ++i) {
            Req r{i, 0, 0};
            if (scanf("%d %d", &r.path, &r.bytes) != 2) return 1;
            q.push_back(r);
        }
        ck::admit_scan(q, [&](const Req &r, const bool *blocked) {
            if (blocked[r.path] || slots[r.path] == 0)
                return std::make_pair(r.path, ck::WAIT_CLASS);
            if (r.bytes < 0) {                // can never fit: rejected
                printf("x%d ", r.id);
                return std::make_pair(r.path, ck::REJECTED);
            }
            if (r.bytes > mem)
                return std::make_pair(r.path, ck::WAIT_MEMORY);
            slots[r.path] -= 1;
            mem -= r.bytes;
            printf("%d ", r.id);
            return std::make_pair(r.path, ck::ADMITTED);
        });
        printf("| left");
        for (const Req &r : q) printf(" %d", r.id);
        printf("\n");
    }
    return 0;
}
"""

# (slots small, slots large, memory, [(path, bytes) ...]) -> admitted ids, ids left in order
CASES = [
    # the second large request waits for a worker; the small ones behind it go
    ((4, 1, 100, [(1, 10), (1, 10), (0, 1), (0, 1)]), ([0, 2, 3], [1])),
    # small slots full: the large request behind them still goes, small stay in order
    ((1, 2, 100, [(0, 1), (0, 1), (1, 5), (0, 1)]), ([0, 2], [1, 3])),
    # the head waits for memory: nothing behind it passes
    ((4, 4, 10, [(1, 20), (0, 1), (0, 1)]), ([], [0, 1, 2])),
    # a large request blocked on its worker, then a small one blocked on memory: scan stops
    ((4, 0, 5, [(1, 1), (0, 9), (0, 1)]), ([], [0, 1, 2])),
    # both paths blocked on slots: the scan ends early, order kept
    ((0, 0, 100, [(0, 1), (1, 1), (0, 1)]), ([], [0, 1, 2])),
    # everything fits: arrival order
    ((8, 8, 100, [(0, 1), (1, 1), (0, 1), (1, 1)]), ([0, 1, 2, 3], [])),
    # empty queue
    ((1, 1, 1, []), ([], [])),
    # a request that can never fit is rejected and leaves the queue; the scan goes on
    ((4, 4, 10, [(0, -1), (0, 1), (1, -1), (1, 2)]), (["x0", 1, "x2", 3], [])),
    # a rejection does not take a slot
    ((1, 1, 10, [(0, -1), (0, 1), (0, 1)]), (["x0", 1], [2])),
]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("admit")
    src = d / "admit_driver.cpp"
    src.write_text(DRIVER)
    exe = d / "admit_driver"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I",
                    os.path.join(ROOT, "paper_2411_10143_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True)
    return str(exe)


def test_admission_scan_cases(driver):
    lines = [str(len(CASES))]
    for (s0, s1, mem, reqs), _ in CASES:
        lines.append(f"{len(reqs)} {s0} {s1} {mem}")
        lines += [f"{p} {b}" for p, b in reqs]
    out = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.strip().splitlines()
    assert len(out) == len(CASES)
    for line, (_, (adm, left)) in zip(out, CASES):
        a, l = line.split("| left")
        assert [v if v.startswith("x") else int(v) for v in a.split()] == adm, line
        assert [int(v) for v in l.split()] == left, line
