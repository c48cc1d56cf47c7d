// Host launchers of the frame kernels (kernels.hip).  `cls` selects the
// batch class (padded ensemble size, storage precision); row and item counts
// are the launch's upper bounds (blocks past the class's work exit at once).
#pragma once
#include <hip/hip_runtime.h>

#include "desc.hpp"

namespace letkf {

void launch_slopes(int cls, int slope_rows, const InstDesc* tab, BatchHdr* hdr, hipStream_t s);
// mode 0: merge, 1: forecast, 2: merge + forecast
void launch_rows(int cls, int mode, int act_rows, const InstDesc* tab, BatchHdr* hdr, hipStream_t s);
void launch_analysis(int cls, int domain_items, const InstDesc* tab, BatchHdr* hdr, hipStream_t s);

}  // namespace letkf
