"""Host logic of the serving loop: the arena allocator that admits requests by result
memory (csrc/arena.hpp), compiled with the host compiler and driven by random
allocate/release sequences.  Checked against a plain model of first fit over 256-byte
units: every granted range is the lowest-offset free gap that fits, ranges never overlap
or leave the arena, a request larger than every free gap is refused, and releasing
everything leaves one free range of the whole arena."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = r'''
#include <cstdio>
#include "arena.hpp"
int main() {
    vbh::Arena a;
    long long total;
    if (scanf("%lld", &total) != 1) return 1;
    a.init(total);
    char op;
    long long x, y;
    while (scanf(" %c %lld %lld", &op, &x, &y) == 3) {
        if (op == 'a') printf("%lld\n", (long long)a.alloc(x));
        else { a.release(x, y); printf("ok\n"); }
    }
    printf("free %zu", a.free_.size());
    for (auto &kv : a.free_) printf(" %lld:%lld", (long long)kv.first, (long long)kv.second);
    printf("\n");
    return 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("arena")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_1805_03709_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)
    return str(exe)


def first_fit(used, total, n):
    """Lowest offset (256-byte units) of a free gap of n units, or -1."""
    pos = 0
    for off, size in sorted(used.items()):
        if off - pos >= n:
            return pos
        pos = off + size
    return pos if total - pos >= n else -1


@pytest.mark.parametrize("seed", range(6))
def test_first_fit_against_model(driver, seed):
    rng = np.random.default_rng(seed)
    total_units = int(rng.integers(64, 4096))
    total = total_units * 256 + int(rng.integers(0, 256))  # a ragged arena size
    ops, model, live = [], {}, []
    expect = []
    for _ in range(600):
        if live and rng.random() < 0.45:
            off, nbytes = live.pop(int(rng.integers(len(live))))
            ops.append(f"r {off} {nbytes}")
            del model[off // 256]
            expect.append("ok")
        else:
            nbytes = int(rng.integers(1, total // 8 + 2))
            units = (nbytes + 255) // 256
            off = first_fit(model, total // 256, units)
            if off >= 0 and (off + units) * 256 > total:
                off = -1
            ops.append(f"a {nbytes} 0")
            expect.append(str(off * 256 if off >= 0 else -1))
            if off >= 0:
                model[off] = units
                live.append((off * 256, nbytes))
    for off, nbytes in live:  # release everything
        ops.append(f"r {off} {nbytes}")
        expect.append("ok")
    out = subprocess.run([driver], input=f"{total}\n" + "\n".join(ops) + "\n", capture_output=True, text=True,
                         check=True).stdout.split("\n")
    got = out[:len(expect)]
    assert got == expect
    assert out[len(expect)] == f"free 1 0:{total}"
