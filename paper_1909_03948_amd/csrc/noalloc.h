// Fixed per-device scratch of the no-allocation entry points.
#pragma once

#include "common.h"

namespace hinv {

// Capacity of the fixed scratch in doubles (64 MiB per device).
constexpr size_t kNoAllocScratchDoubles = size_t(8) << 20;

// Looks up the device address of the scratch array on `device`, which must be
// the current device; once per device, later calls return at once.
void noalloc_init(int device);

// Device address of the scratch array on `device` (noalloc_init ran before).
double* noalloc_scratch(int device);

}  // namespace hinv
