"""The serving arena's row allocator (paper_2509_04390_amd/csrc/arena.hpp),
built for the host with g++, against a row-by-row model: first fit over the
maximal free runs, release only of allocated rows, free runs merged."""
import os
import random
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("arena") / "arena_driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_2509_04390_amd", "csrc"),
                    os.path.join(ROOT, "tests", "arena_driver.cpp"), "-o", exe], check=True)
    return exe


def run(driver, cmds):
    out = subprocess.run([driver], input="\n".join(cmds) + "\n", capture_output=True,
                         text=True, check=True).stdout.split("\n")
    return out[:len(cmds)]


class Model:
    def __init__(self, cap):
        self.used = [False] * cap

    def runs(self):
        out, i, n = [], 0, len(self.used)
        while i < n:
            if self.used[i]:
                i += 1
                continue
            j = i
            while j < n and not self.used[j]:
                j += 1
            out.append((i, j - i))
            i = j
        return out

    def alloc(self, n):
        if n < 1:
            return -1
        for s, ln in self.runs():
            if ln >= n:
                for k in range(s, s + n):
                    self.used[k] = True
                return s
        return -1

    def release(self, s, n):
        if n < 1 or s < 0 or s + n > len(self.used) or not all(self.used[s:s + n]):
            return 0
        for k in range(s, s + n):
            self.used[k] = False
        return 1

    def state(self):
        r = self.runs()
        used = sum(self.used)
        largest = max([ln for _, ln in r], default=0)
        return " ".join([str(used), str(largest)] + [f"{s}:{ln}" for s, ln in r])


@pytest.mark.parametrize("seed", range(6))
def test_random_alloc_release_matches_row_model(driver, seed):
    rng = random.Random(seed)
    cap = rng.choice([1, 7, 64, 1000])
    m = Model(cap)
    cmds, want = [f"c {cap}"], ["ok"]
    live = []
    for _ in range(400):
        r = rng.random()
        if r < 0.45:
            n = rng.randint(0, max(1, cap // 3))
            s = m.alloc(n)
            cmds.append(f"a {n}")
            want.append(str(s))
            if s >= 0:
                live.append((s, n))
        elif r < 0.8 and live:
            s, n = live.pop(rng.randrange(len(live)))
            cmds.append(f"r {s} {n}")
            want.append(str(m.release(s, n)))
        elif r < 0.9:
            # invalid or partly free ranges must be refused without change
            s, n = rng.randint(-2, cap), rng.randint(-1, 5)
            cmds.append(f"r {s} {n}")
            want.append(str(m.release(s, n)))
            if want[-1] == "1":
                # a valid release of rows owned by several live allocations:
                # drop those allocations from the live list
                live = [(a, b) for a, b in live if a + b <= s or a >= s + n]
        else:
            cmds.append("s")
            want.append(m.state())
    cmds.append("s")
    want.append(m.state())
    assert run(driver, cmds) == want


def test_free_ranges_merge_back_into_one(driver):
    cmds = ["c 100", "a 10", "a 20", "a 30", "r 10 20", "r 0 10", "r 30 30", "s"]
    assert run(driver, cmds) == ["ok", "0", "10", "30", "1", "1", "1", "0 100 0:100"]
