"""Host-side logic of the serving form, no GPU: the arena allocator the
server admits simulations against (compiled from its header with the host
compiler and driven here), and the server's argument checks, which run
before any device call."""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1805_11169_amd import icwf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ARENA_HPP = os.path.join(ROOT, "paper_1805_11169_amd", "csrc", "arena.hpp")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <random>
#include "arena.hpp"
#define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); return 1; } } while (0)
int main() {
    using icwf::Arena;
    // sizes round up to 256 and blocks are 256-aligned, first fit from the bottom
    Arena a(10000);
    CHECK(a.size() == 9984);
    size_t x = a.alloc(1), y = a.alloc(300), z = a.alloc(256);
    CHECK(x == 0 && y == 256 && z == 768);
    CHECK(a.in_use() == 256 + 512 + 256);
    CHECK(a.alloc(0) == Arena::kFail);
    CHECK(a.alloc(9984) == Arena::kFail);
    // freeing the middle block leaves a hole that the next fitting request takes
    CHECK(a.release(y));
    CHECK(!a.release(y));                 // not live any more
    CHECK(!a.release(12345));
    CHECK(a.alloc(512) == 256);
    CHECK(a.release(256));
    // coalescing: free x, then z; x, the hole and z merge with the tail into one block
    CHECK(a.release(x) && a.release(z));
    CHECK(a.in_use() == 0 && a.free_blocks() == 1 && a.largest_free() == 9984);
    CHECK(a.peak() == 1024);
    // random alloc / release keeps the books consistent and ends fully merged
    std::mt19937 rng(7);
    Arena b(1 << 20);
    std::vector<size_t> live;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 2) {
            size_t o = b.alloc(1 + rng() % 40000);
            if (o != Arena::kFail) { CHECK(o % 256 == 0 && o < b.size()); live.push_back(o); }
        } else {
            size_t k = rng() % live.size();
            CHECK(b.release(live[k]));
            live[k] = live.back(); live.pop_back();
        }
        CHECK(b.in_use() <= b.size() && b.live_blocks() == live.size());
    }
    for (size_t o : live) CHECK(b.release(o));
    CHECK(b.in_use() == 0 && b.free_blocks() == 1 && b.largest_free() == b.size());
    std::printf("OK\n");
    return 0;
}
"""


def test_arena_allocator(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "arena_driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "arena_driver"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined", "-I",
                    os.path.dirname(ARENA_HPP), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout + out.stderr


def test_server_rejects_bad_arguments_before_touching_the_device():
    L = icwf.lib()
    h = ctypes.c_void_p()
    good = icwf.ServerConfig(4, 10, 2, 0)
    for cfg in (icwf.ServerConfig(0, 10, 2, 0), icwf.ServerConfig(65, 10, 2, 0), icwf.ServerConfig(4, 0, 2, 0),
                icwf.ServerConfig(4, 10, 0, 0), icwf.ServerConfig(4, 10, 5, 0), icwf.ServerConfig(4, 10, 2, -1)):
        assert L.icwf_server_create(ctypes.byref(cfg), ctypes.c_void_p(256), 1 << 20, ctypes.byref(h)) == icwf.EINVAL
    assert L.icwf_server_create(ctypes.byref(good), None, 1 << 20, ctypes.byref(h)) == icwf.EINVAL
    assert L.icwf_server_create(ctypes.byref(good), ctypes.c_void_p(257), 1 << 20, ctypes.byref(h)) == icwf.EINVAL
    assert L.icwf_server_create(ctypes.byref(good), ctypes.c_void_p(256), 100, ctypes.byref(h)) == icwf.EINVAL
    rid = ctypes.c_int64()
    assert L.icwf_server_submit(None, None, None, None, None, None, None, None, None, 1, ctypes.byref(rid)) \
        == icwf.EINVAL
    assert L.icwf_server_wait(None, 1, 0.0) == icwf.EINVAL
    assert L.icwf_server_result(None, 1, None, None) == icwf.EINVAL
    assert L.icwf_server_clock(None) == 0.0
    L.icwf_server_destroy(None)
    assert icwf.status_string(icwf.ETIMEDOUT) == "ICWF_ETIMEDOUT"
