// Limits of the staging of x (an extension of the ARG-CSR storage for
// banded matrices), shared by the staging kernels and the SpMV.
#pragma once

#include <cstdint>

namespace argcsr {

// Tiles of 64 columns one group may stage: positions 64*q + i stay below
// 4096, far from the 0xFFFF that marks an artificial zero.
constexpr int kStageMaxTiles = 64;
// Columns one group's smallest and largest column may span: the staging
// kernel marks the group's columns in a bitmap of this many bits in LDS.
constexpr int kStageSpanBits = 1 << 18;
constexpr uint16_t kStagePad = 0xFFFF;

}  // namespace argcsr
