// Size limits of the library's device data structures, checked on the host.
// Plain C++ (no HIP), so the limits can be exercised by a CPU-only test.
#pragma once

#include <cstdint>

namespace fmm {

// Interaction lists are grouped into int32 CSR arrays (offsets and sources)
// and the walk's frontier is indexed by int; a list or frontier longer than
// this is rejected with FMM_EUNSUPPORTED before anything indexes it.
constexpr long long kMaxWalkEntries = 0x7fffffffLL - 64;

inline bool walk_list_fits(long long entries) { return entries >= 0 && entries <= kMaxWalkEntries; }

}  // namespace fmm
