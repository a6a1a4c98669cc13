// Index limits of one launch of cells and the plan of list groups of the rotation path
// (plain C++: also compiled for the host by the unit tests).
//
// Counts are scanned in 32 bits and several kernels index list entries with int, so
// every total is checked in 64 bits before it sizes a buffer: a total that would wrap
// is either split (list groups of the rotation path) or rejected with AR_E_UNSUPPORTED,
// never used.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace ar {

// largest exclusive scan of the library (elements): 16 x 32768 blocks of 1024
constexpr uint64_t kScanMax = 1ull << 29;
// items (cells x Gaussians) of one launch: n + 1 tile counts are scanned
constexpr uint64_t kMaxItems = kScanMax - 1;
// (tile, Gaussian) list entries of one launch: radix-sorted and indexed as int
constexpr uint64_t kMaxEntries = 0x7FFFFFF0ull;
// entries of one list group of the rotation path: 2 n + 1 run counts are scanned
constexpr uint64_t kMaxGroupEntries = (kScanMax - 1) / 2;
// runs of one list group: their offsets are uint32
constexpr uint64_t kMaxGroupRuns = 0xFFFFFFFFull;

// Returns nullptr when a launch of `items` items with `entries` list entries fits the
// index types of its kernels, else the reason it does not.
inline const char *launch_limit(uint64_t items, uint64_t entries) {
  if (items > kMaxItems) return "more Gaussian items (cells x Gaussians) than one launch indexes";
  if (entries > kMaxEntries) return "more (tile, Gaussian) list entries than one launch indexes";
  return nullptr;
}

// Returns nullptr when the runs of one list group fit their uint32 offsets.
inline const char *group_runs_limit(uint64_t runs) {
  return runs > kMaxGroupRuns ? "more Ind runs in one list group than uint32 offsets hold" : nullptr;
}

// Groups of consecutive tile lists for the rotation path.  ranges: [nlists][2] begin /
// end list positions (lists are contiguous and in order).  Lists are gathered while a
// group holds at most `cap` entries (cap <= kMaxGroupEntries); a longer single list
// gets a group of its own.  bounds receives the first list of each group, then nlists.
// Returns false (bounds unspecified) when a single list exceeds kMaxGroupEntries.
inline bool plan_groups(const uint32_t *ranges, size_t nlists, uint64_t cap, std::vector<size_t> &bounds) {
  bounds.clear();
  if (cap < 1) cap = 1;
  if (cap > kMaxGroupEntries) cap = kMaxGroupEntries;
  bounds.push_back(0);
  uint64_t held = 0;
  for (size_t l = 0; l < nlists; ++l) {
    const uint64_t n = (uint64_t)ranges[2 * l + 1] - (uint64_t)ranges[2 * l];
    if (n > kMaxGroupEntries) return false;
    if (held > 0 && n > 0 && held + n > cap) {
      bounds.push_back(l);
      held = 0;
    }
    held += n;
  }
  bounds.push_back(nlists);
  return true;
}

}  // namespace ar
