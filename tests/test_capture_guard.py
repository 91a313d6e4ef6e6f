"""The library's capture guard on the CPU (host code only, built with g++): a
lock-step batch opens a graph capture only while no setup, destruction or
allocation runs on any thread, and those calls wait while a capture is open.
This is the invariant that keeps device-synchronising calls of one host thread
out of another thread's open stream capture."""
import os
import shutil
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_20496_amd", "csrc")

DRIVER = textwrap.dedent(r"""
    #include "capture_guard.h"
    #include <atomic>
    #include <chrono>
    #include <cstdio>
    #include <thread>
    using namespace coarse;
    using clk = std::chrono::steady_clock;
    static double ms_since(clk::time_point t) {
      return std::chrono::duration<double, std::milli>(clk::now() - t).count();
    }
    #define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); return 1; } } while (0)
    int main() {
      CaptureGuard g;
      // 1. a device call made while a capture is open waits for its end
      {
        std::atomic<int> opened{0};
        clk::time_point t_end;
        std::thread cap([&] {
          if (!g.try_begin_capture()) return;
          opened = 1;
          std::this_thread::sleep_for(std::chrono::milliseconds(200));
          t_end = clk::now();
          g.end_capture();
        });
        while (!opened) std::this_thread::yield();
        const auto t0 = clk::now();
        g.begin_device_call();
        const double waited = ms_since(t0);
        CHECK(g.captures() == 0);
        CHECK(waited >= 150.0);
        CHECK(clk::now() >= t_end);
        g.end_device_call();
        cap.join();
      }
      // 2. no capture opens while a device call (of any thread) is in progress
      {
        std::atomic<int> held{0}, release{0};
        std::thread dev([&] {
          DeviceCallScope s(g);
          held = 1;
          while (!release) std::this_thread::yield();
        });
        while (!held) std::this_thread::yield();
        CHECK(!g.try_begin_capture());
        CHECK(g.device_calls() == 1);
        release = 1;
        dev.join();
        CHECK(g.device_calls() == 0);
        CHECK(g.try_begin_capture());
        g.end_capture();
      }
      // 3. device calls nest (a setup that allocates the block-solve vectors)
      {
        DeviceCallScope a(g);
        DeviceCallScope b(g);
        CHECK(g.device_calls() == 2);
        CHECK(!g.try_begin_capture());
      }
      CHECK(g.device_calls() == 0 && g.captures() == 0);
      // 4. many threads: captures and device calls never overlap
      {
        std::atomic<int> in_cap{0}, in_dev{0}, bad{0};
        std::thread ts[8];
        for (int k = 0; k < 8; ++k)
          ts[k] = std::thread([&, k] {
            for (int i = 0; i < 2000; ++i) {
              if (k % 2 == 0) {
                if (g.try_begin_capture()) {
                  ++in_cap;
                  if (in_dev.load()) bad = 1;
                  --in_cap;
                  g.end_capture();
                }
              } else {
                DeviceCallScope s(g);
                ++in_dev;
                if (in_cap.load()) bad = 1;
                --in_dev;
              }
            }
          });
        for (auto &t : ts) t.join();
        CHECK(!bad);
      }
      std::printf("OK\n");
      return 0;
    }
""")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_capture_guard(tmp_path):
    src = tmp_path / "guard_test.cpp"
    exe = tmp_path / "guard_test"
    src.write_text(DRIVER)
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-pthread", f"-I{CSRC}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr
