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
// Differential pistons of the instances created with LETKF_FLAG_PISTONS (the
// others are skipped): overlap mismatches, then pistons; between the analysis
// and the merge.
void launch_pistons(int cls, int domain_items, const InstDesc* tab, BatchHdr* hdr, hipStream_t s);
// max_grid > 0 splits the items into consecutive launches of at most max_grid
// workgroups (one workgroup per item in every case).
void launch_analysis(int cls, int domain_items, const InstDesc* tab, BatchHdr* hdr, hipStream_t s, int max_grid = 0);

}  // namespace letkf
