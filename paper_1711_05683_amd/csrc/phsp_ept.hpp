// phsp_ept.hpp -- default events per thread of the single-channel kernels.
//
// FP64 generation with every column on the 128-byte line grid, by daughter
// count, and integration: the fastest of 1, 2 and 4 in warmed sweeps on MI355X
// (about 10 GB of output per launch).  The host's launch defaults and the batch
// kernel that runs every N in one launch at these settings both read them, so
// a channel's tiles in that launch are the blocks of a default single-channel
// call.
#pragma once

namespace hphsp {

constexpr int kEptLineFp64[11] = {0, 0, 2, 1, 2, 2, 4, 4, 4, 4, 4};
constexpr int kEptIntegrate = 4;

} // namespace hphsp
