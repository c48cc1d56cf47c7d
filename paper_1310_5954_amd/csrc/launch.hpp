// Host launchers of the frame kernels (kernels.hip).  `cls` selects the
// batch class (padded ensemble size, storage precision).  Row and item counts
// size the grids (capped): every kernel reads the class's actual work from the
// batch header and loops grid-stride over it, so a grid sized for more work
// than the batch holds is still correct (its spare blocks exit at once).
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
// The persistent analysis kernel with `grid` workgroups: they share the
// class's domain items through its work counter, which the slope kernel
// launched before it zeroes, so any grid >= 1 covers every item.  fair != 0:
// progress-ordered issue priorities, for launches whose workgroups start
// together at most two to a CU (analysis_fair_grid).
void launch_analysis(int cls, int grid, const InstDesc* tab, BatchHdr* hdr, hipStream_t s, int fair = 0);
// Whether a plain launch of `grid` workgroups on `num_cu` CUs takes the
// progress-ordered priorities: at most two of its workgroups share a CU.
inline int analysis_fair_grid(int grid, int num_cu) { return grid <= 2 * num_cu ? 1 : 0; }
// Analysis workgroups of the class one CU holds at once (LDS and registers).
int analysis_blocks_per_cu(int cls);

// ---- the allocation-free frame (letkf_step_noalloc) ----
// Byte offsets, inside the library's static device array, of the scratch of
// one frame run without the instance workspace's scratch: copies of the
// instance descriptor and batch header pointing the kernels there, the slope
// perturbations, the innovation, the per-domain analysis rows, the packed
// copies of A (FP64) and the analysis means.
constexpr size_t kScratchBytes = size_t(32) << 20;
struct NoallocLayout {
  size_t desc, hdr, Yp, d, Z, Ascr, amean, total;
};
// The array's address on the current device (looked up once per device and
// kept); LETKF_EDEVICE-style HIP error otherwise.
hipError_t scratch_address(int device, unsigned char** out);
// Builds the descriptor and header copies in the array at sp (device address):
// the instance's descriptor with Yp, d, Z and Ascr moved into the array, and a
// one-entry header of class cls reading y (device) and writing the prediction
// means to pred (device), the analysis means into the array.
void launch_noalloc_setup(const InstDesc* src, const BatchHdr* src_hdr, unsigned char* sp, const NoallocLayout& lay,
                          const double* y, double* pred, int cls, hipStream_t s);
// The analysis of the m > 128 class (FP64): a fixed sequence of launches over
// the domains' scratch (rows_max: most state rows of a domain, m_max: most
// members of an instance in the batch).
void launch_big_analysis(int items, int rows_max, int m_max, const InstDesc* tab, BatchHdr* hdr, hipStream_t s);

}  // namespace letkf
