"""Host logic of the serving loop's rounds form: the gate between serving and the MC update
of fused frames (McGate in csrc/sched.hpp), compiled with the host compiler and driven by
real threads: an updater thread rewrites a shared "MC pool" once per frame (the MC update)
and publishes a new version under the gate, while the serving thread runs rounds on worker
threads (standing in for the streams) that read the pool while in flight.  Checked: no
round is in flight while an update runs, every round reads a pool of one version that is
at least the version it was admitted under, every update happens, and the run ends.  The
same driver runs under ThreadSanitizer, which also checks that the gate orders the pool's
plain reads and writes.  A gate that grants while rounds are in flight, planted in a copy
of the header, fails."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = r'''
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>
#include "sched.hpp"

using namespace vbh;

int main(int argc, char **argv) {
    const unsigned seed = unsigned(atoi(argv[1]));
    const int n_updates = atoi(argv[2]), n_rounds = atoi(argv[3]);
    McGate gate;
    std::vector<int> pool(256, 0);  // the MC pool: written by updates, read by rounds in flight
    uint64_t end_pub = 0;           // published under the gate
    uint32_t ver_pub = 0;
    std::atomic<int> in_update{0}, in_flight{0};
    std::atomic<bool> bad{false}, upd_done{false};
    std::thread upd([&] {
        std::mt19937 rng(seed);
        for (int u = 1; u <= n_updates; ++u) {
            std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));  // the frame's fusion
            gate.acquire();
            in_update = 1;
            if (in_flight.load() != 0) bad = true;
            for (auto &x : pool) x = u;  // the MC update rewrites the pool
            in_update = 0;
            gate.release([&] {
                end_pub = uint64_t(u) * 100;
                ver_pub = uint32_t(u);
            });
        }
        upd_done = true;
        gate.finish();
    });
    struct Round {
        std::thread t;
        std::atomic<bool> done{false};
    };
    std::vector<Round *> flight;
    std::mt19937 rng(seed * 7u + 1u);
    int launched = 0;
    uint32_t last_ver = 0;
    while (launched < n_rounds || !flight.empty()) {
        uint64_t e = 0;
        uint32_t ver = 0;
        const bool closed = gate.poll(flight.empty(), [&] {
            e = end_pub;
            ver = ver_pub;
        });
        if (e != uint64_t(ver) * 100 || ver < last_ver) bad = true;
        last_ver = ver;
        if (!closed && launched < n_rounds && flight.size() < 4 && rng() % 2 == 0) {
            Round *r = new Round;
            const unsigned d = rng() % 100;
            in_flight++;
            r->t = std::thread([&, r, ver, d] {
                if (in_update.load() != 0) bad = true;
                const int first = pool[0];
                std::this_thread::sleep_for(std::chrono::microseconds(d));
                for (int x : pool)
                    if (x != first || x < int(ver)) bad = true;  // one version, not older than admitted
                in_flight--;
                r->done = true;
            });
            flight.push_back(r);
            ++launched;
        }
        for (size_t i = 0; i < flight.size();) {
            if (flight[i]->done) {
                flight[i]->t.join();
                delete flight[i];
                flight.erase(flight.begin() + long(i));
            } else {
                ++i;
            }
        }
        std::this_thread::yield();
    }
    while (!upd_done) {  // serving is over: grant what remains
        (void)gate.poll(true, [] {});
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    upd.join();
    if (bad) {
        printf("violation\n");
        return 1;
    }
    printf("ok %d rounds %d updates\n", launched, n_updates);
    return 0;
}
'''


def build(tmp_path, hdr_dir, sanitize=False):
    src, exe = tmp_path / "drv.cpp", tmp_path / ("drv_tsan" if sanitize else "drv")
    src.write_text(DRIVER)
    cmd = ["g++", "-std=c++17", "-pthread", "-I", str(hdr_dir), "-o", str(exe), str(src)]
    cmd[1:1] = ["-O1", "-g", "-fsanitize=thread"] if sanitize else ["-O2"]
    subprocess.run(cmd, check=True)
    return str(exe)


CSRC = os.path.join(ROOT, "paper_1805_03709_amd", "csrc")


@pytest.mark.parametrize("seed", range(4))
def test_gate_excludes_updates_and_rounds(tmp_path, seed):
    exe = build(tmp_path, CSRC)
    out = subprocess.run([exe, str(seed), "40", "400"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr


def test_gate_under_thread_sanitizer(tmp_path):
    exe = build(tmp_path, CSRC, sanitize=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    for seed in range(2):
        out = subprocess.run([exe, str(seed), "30", "300"], capture_output=True, text=True, timeout=300, env=env)
        assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr[-3000:]


def test_gate_granting_with_rounds_in_flight_fails(tmp_path):
    hdr = open(os.path.join(CSRC, "sched.hpp")).read()
    old = "if (request_ && !granted_ && idle) grant = granted_ = true;"
    assert old in hdr
    (tmp_path / "sched.hpp").write_text(hdr.replace(old, "if (request_ && !granted_) grant = granted_ = true;"))
    (tmp_path / "arena.hpp").write_text(open(os.path.join(CSRC, "arena.hpp")).read())
    exe = build(tmp_path, tmp_path)
    fails = [subprocess.run([exe, str(seed), "40", "400"], capture_output=True, text=True, timeout=120).returncode != 0
             for seed in range(4)]
    assert any(fails)
