// Device scratch of the allocation-free entry point (defined in noalloc.hip).
#pragma once
#include <stddef.h>

namespace qsv {

// Size of the per-device scratch array: term tables, reduced columns and the per-workgroup
// partial sums of one expectation.
constexpr size_t kNoallocScratchBytes = (size_t)4 << 20;
// Largest Pauli sum the allocation-free expectation accepts (tables: 24 bytes per term,
// reduced columns: 16 bytes per group of terms sharing an x mask).
constexpr size_t kNoallocMaxTerms = 8192;
// Groups whose partial sums share the scratch at one time (2 * 64 * 2048 doubles = 2 MiB).
constexpr int kNoallocChunk = 64;

// Device address of the current device's scratch array, looked up with
// hipGetSymbolAddress on the first call on each device (the device must be current).
void* noalloc_scratch();

}  // namespace qsv
