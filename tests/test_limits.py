"""Index limits of one launch and the list groups of the rotation path, compiled for the
host from the library's own header (ar_limits.h) and checked on synthetic counts.

Counts are scanned in 32 bits on the device; the library sums them in 64 bits beside the
scan and hands the 64-bit totals to these checks before any buffer is sized, so a total
at or beyond 2^32 must be rejected (or split into groups), never used.
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR_DIR = os.path.join(ROOT, "paper_2503_00308_amd", "csrc")

PROG = r"""
#include <cstdio>
#include <cstdint>
#include <vector>
#include "ar_limits.h"
using namespace ar;
static int bad = 0;
#define CHECK(c) do { if (!(c)) { printf("FAIL line %d: %s\n", __LINE__, #c); ++bad; } } while (0)
int main() {
  // launch limits: items (scanned n + 1) and list entries (int indices)
  CHECK(launch_limit(0, 0) == nullptr);
  CHECK(launch_limit(kMaxItems, kMaxEntries) == nullptr);
  CHECK(launch_limit(kMaxItems + 1, 0) != nullptr);
  CHECK(launch_limit(1000, kMaxEntries + 1) != nullptr);
  CHECK(launch_limit(1000, 0xFFFFFFFFull) != nullptr);          // would wrap a uint32 total
  CHECK(launch_limit(1000, 0x100000000ull + 5) != nullptr);     // a total that wrapped to 5
  CHECK(kMaxEntries <= 0x7FFFFFFFull);
  // run totals of a group: uint32 offsets
  CHECK(group_runs_limit(0) == nullptr);
  CHECK(group_runs_limit(0xFFFFFFFFull) == nullptr);
  CHECK(group_runs_limit(0x100000000ull) != nullptr);
  CHECK(group_runs_limit(4200000000ull * 2) != nullptr);
  // a group's run counts are scanned in 2 n + 1 elements
  CHECK(2 * kMaxGroupEntries + 1 <= kScanMax);
  // groups: synthetic lists near the limits
  {
    // 5 lists of 3, 0, 4, 2, 6 entries (an empty list has the range [0, 0))
    const uint32_t r[] = {0, 3, 0, 0, 3, 7, 7, 9, 9, 15};
    std::vector<size_t> b;
    CHECK(plan_groups(r, 5, 100, b));
    CHECK(b.size() == 2 && b[0] == 0 && b[1] == 5);
    CHECK(plan_groups(r, 5, 7, b));                    // {3, 0, 4} {2} {6}: 7, then 2 + 6 > 7
    CHECK(b.size() == 4 && b[0] == 0 && b[1] == 3 && b[2] == 4 && b[3] == 5);
    CHECK(plan_groups(r, 5, 1, b));                    // every nonempty list alone
    CHECK(b.size() == 5 && b[1] == 2 && b[2] == 3 && b[3] == 4 && b[4] == 5);
    // each group holds at most cap entries unless it is one list
    CHECK(plan_groups(r, 5, 5, b));
    for (size_t g = 0; g + 1 < b.size(); ++g) {
      uint64_t n = 0; size_t ne = 0;
      for (size_t l = b[g]; l < b[g + 1]; ++l) { n += r[2 * l + 1] - r[2 * l]; ne += r[2 * l + 1] > r[2 * l]; }
      CHECK(n <= 5 || ne == 1);
    }
  }
  {
    // lists whose entries sum past 2^32 as uint32 would wrap; groups keep every group small
    std::vector<uint32_t> r;
    uint64_t pos = 0;
    const uint64_t per = 0x30000000ull;               // 805M entries per list
    for (int l = 0; l < 5; ++l) { r.push_back((uint32_t)pos); pos += per; r.push_back((uint32_t)pos); }
    std::vector<size_t> b;
    // the positions themselves wrap past list 5, so only 5 lists are representable;
    // one list longer than a group can be is rejected
    CHECK(!plan_groups(r.data(), 5, 1ull << 27, b));
    std::vector<uint32_t> r2 = {0, (uint32_t)kMaxGroupEntries, (uint32_t)kMaxGroupEntries,
                                (uint32_t)(kMaxGroupEntries + 10)};
    CHECK(plan_groups(r2.data(), 2, 1ull << 27, b));
    CHECK(b.size() == 3 && b[1] == 1);
  }
  {
    // many small lists: group entry totals never exceed the cap
    std::vector<uint32_t> r;
    uint32_t pos = 0;
    for (int l = 0; l < 100000; ++l) { r.push_back(pos); pos += (uint32_t)(l * 7919 % 97); r.push_back(pos); }
    std::vector<size_t> b;
    CHECK(plan_groups(r.data(), 100000, 1000, b));
    size_t lists = 0;
    for (size_t g = 0; g + 1 < b.size(); ++g) {
      uint64_t n = 0;
      for (size_t l = b[g]; l < b[g + 1]; ++l) n += r[2 * l + 1] - r[2 * l];
      CHECK(n <= 1000);
      CHECK(b[g + 1] > b[g]);
      lists += b[g + 1] - b[g];
    }
    CHECK(lists == 100000 && b.front() == 0 && b.back() == 100000);
  }
  printf("bad %d\n", bad);
  return bad != 0;
}
"""


def test_limits_and_groups(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(PROG)
    exe = tmp_path / "t"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", HDR_DIR, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
