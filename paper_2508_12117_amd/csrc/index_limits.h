// Index limits of the step kernels.  Every chain set numbers its minibatch
// entries (two per observation and chain: events i and j) with 32-bit
// integers in the sort values, node numbers and solver lists, so a set may
// hold at most INT32_MAX entries; sets advanced together in fused steps are
// bounded the same way in total.
#pragma once
#include <stdint.h>

namespace spider {

constexpr int64_t kMaxEntries = 2147483647;  // INT32_MAX
// Station-phase groups of a catalog: the exact whitening counts each
// position block's nodes per group in LDS (4 bytes a group, 160 KB).
constexpr int32_t kMaxGroups = 40960;

// True iff `chains` chains with minibatch `batch` each fit the 32-bit entry
// numbering (2 chains batch <= kMaxEntries), for chains, batch >= 1.
inline bool entries_fit(int64_t chains, int64_t batch) {
  return chains >= 1 && batch >= 1 && batch <= kMaxEntries / 2 / chains;
}

}  // namespace spider
