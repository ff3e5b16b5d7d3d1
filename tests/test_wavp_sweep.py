"""Host logic of the batched victim choice (Sec. 4.3, Alg. 2) against a
literal clock walk.

The library scores a full cache once per batch and answers each eviction
from a min tree over 64-slot blocks, skipping blocks and runs of bitmap
words without set reference bits.  Here the same class, compiled on the
host, is driven through many evictions on random caches and compared with
a plain walk written from the algorithm: F_min over the residents whose
bit is clear (after one clearing round when every bit is set), then from
the hand, a set bit is cleared and passed, and the first clear slot holding
F_min is replaced, the hand staying on it.  Victims, hands and bits must
agree after every eviction.  Scores are drawn from a few levels so that
ties are common, and bit densities range from none to all set."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2601_08528_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdint>
#include <random>
#include <vector>
#include "wavp.hpp"

// Alg. 2 as a literal walk over the slots.
static int64_t walk(std::vector<double>& f, std::vector<uint8_t>& ref, int64_t& hand) {
  const int64_t C = (int64_t)f.size();
  double fmin = 0.0;
  bool any = false;
  for (int64_t s = 0; s < C; ++s)
    if (!ref[s] && (!any || f[s] < fmin)) { fmin = f[s]; any = true; }
  if (!any) {                                  // one round clears every bit
    for (int64_t s = 0; s < C; ++s) ref[s] = 0;
    fmin = f[0];
    for (int64_t s = 1; s < C; ++s) fmin = f[s] < fmin ? f[s] : fmin;
  }
  for (int64_t s = hand;; s = (s + 1) % C) {
    if (ref[s]) { ref[s] = 0; continue; }
    if (f[s] == fmin) { hand = s; return s; }
  }
}

int main(int argc, char** argv) {
  std::mt19937_64 rng(12345);
  int cases = 0;
  const int64_t sizes[] = {1, 2, 63, 64, 65, 640, 4096, 4097, 70000, 300000};
  const double dens[] = {0.0, 0.001, 0.05, 0.5, 0.95, 1.0};
  for (int64_t C : sizes)
    for (double d : dens)
      for (int rep = 0; rep < 2; ++rep) {
        std::vector<double> f(C), f2;
        std::vector<uint8_t> ref(C), ref2;
        std::uniform_int_distribution<int> lvl(0, 7);
        std::uniform_real_distribution<double> u(0.0, 1.0);
        for (int64_t s = 0; s < C; ++s) {
          f[s] = 0.25 * lvl(rng);
          ref[s] = u(rng) < d ? 1 : 0;
        }
        f2 = f;
        ref2 = ref;
        int64_t hand = (int64_t)(rng() % (uint64_t)C), hand2 = hand;
        svf::WavpSweep sw;
        sw.begin(C, [&](int64_t s) { return f[s]; }, [](int64_t) {}, ref.data(),
                 C > 100000 ? 4 : 1);
        const int evictions = (int)std::min<int64_t>(3 * C + 5, 2000);
        for (int e = 0; e < evictions; ++e) {
          const int64_t v = sw.evict(hand, ref.data());
          const int64_t v2 = walk(f2, ref2, hand2);
          if (v != v2 || hand != hand2) {
            std::printf("mismatch C=%lld d=%g eviction %d: %lld/%lld vs %lld/%lld\n",
                        (long long)C, d, e, (long long)v, (long long)hand, (long long)v2,
                        (long long)hand2);
            return 1;
          }
          const double fx = 0.25 * lvl(rng);
          f[v] = fx;
          f2[v] = fx;
          sw.place(v, fx);
          if (ref != ref2) {
            std::printf("bits differ C=%lld d=%g eviction %d\n", (long long)C, d, e);
            return 1;
          }
        }
        sw.end();
        ++cases;
      }
  std::printf("ok %d\n", cases);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("wavp")
    src = d / "drive.cpp"
    src.write_text(DRIVER)
    exe = d / "drive"
    subprocess.run([cxx, "-O2", "-std=c++17", "-pthread", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    return str(exe)


def test_victims_match_a_literal_clock_walk(driver):
    out = subprocess.run([driver], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
