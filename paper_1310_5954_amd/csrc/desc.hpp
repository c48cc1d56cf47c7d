// Device-resident descriptors shared by the runtime and the kernels.
//
// An instance is one resident AO filter (its ensemble, D, domain map and
// scratch live in one workspace).  A batch is a list of instances that have
// one frame each in the current launch sequence; kernels are launched once
// per (padded ensemble size, storage precision) class and walk the class's
// entries, so the frames of several instances share every launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace letkf {

constexpr int kMaxBatch = 64;   // frames per batch
// classes 0..15: 4 padded sizes (16, 32, 64, 128) x 4 arithmetic variants
// (index variant x 4 + size): FP64, FP32, BF16, and BF16 with the Jacobi
// rotations in FP32 (LETKF_FLAG_FP32_ROTATIONS); class 16: 129..256 members,
// FP64 only
constexpr int kVariants = 4;
constexpr int kNumClasses = 4 * kVariants + 1;
constexpr int kBigClass = 4 * kVariants;

struct InstState {           // mutated on the device by the forecast kernel
  int32_t cur;               // ring slot holding phi_k (the other holds phi_{k-1})
  int32_t unconverged;       // domains that hit the Jacobi sweep cap in the last analysis
  uint64_t frame;            // forecasts done so far (Philox counter word 2..3)
  unsigned long long sweeps; // Jacobi sweeps summed over every domain solve
  unsigned long long solves; // domain solves
};

struct InstDesc {
  int32_t n_act, n_sub, m, n_dom;
  int32_t prec, flags, zrows, nnz;
  int32_t obs_inst;          // ring slot offset of the observed instant: 0 = phi_k, 1 = phi_{k-1}
  int32_t pad0;
  double sigma_v;
  double a_diag;             // (m-1)/rho
  uint64_t seed;
  void* ens;                 // [2][n_act][m]   storage type (double for FP64, float otherwise)
  void* Yp;                  // [p][m]          slope perturbations D X'_phi
  double* d;                 // [p]             innovation y - D xbar_phi
  void* Z;                   // [zrows][m]      per-domain analysis rows before the merge
  const double* a1;          // [n_act]
  const double* a2;          // [n_act]
  const int32_t* d_rowptr;   // [p+1]
  const int32_t* d_col;      // [nnz]
  const double* d_val;       // [nnz]
  const int32_t* dom;        // [n_dom][4]: est_off, e, obs_off, s  (Z rows of l start at 2*est_off)
  const int32_t* order;      // [n_dom] domains by decreasing estimated cost
  const int32_t* est_act;    // [sum e]
  const int32_t* obs_row;    // [2 sum s]: slope row of each observation (x rows then y rows per domain)
  const double* obs_r;       // [2 sum s]: taper * R^-1 of each observation
  const double* obs_sr;      // [2 sum s]: its square root (the weight of the staged rows of C)
  const int32_t* mptr;       // [n_act+1] merge CSR: covering (domain, position) entries per actuator
  const int32_t* mrow;       // [2*entries]: Z row of the phi_k copy and of the phi_{k-1} copy
  const double* mw;          // [entries]: merge weight
  const int32_t* mdom;       // [entries]: domain of each merge entry
  const double* pist_op;     // [n_dom][n_dom] piston operator (NULL unless LETKF_FLAG_PISTONS)
  const int32_t* pist_ptr;   // [n_dom+1] CSR of each domain's mismatch terms
  const int32_t* pist_row;   // [2*terms]: Z row of the term at phi_k and at phi_{k-1}
  const double* pist_coef;   // [terms]: its coefficient (1, or 1 - k_j for the domain's own row)
  double* pist_r;            // [n_dom][2][m] overlap mismatch of each domain, instant, member
  double* pist_c;            // [n_dom][2][m] pistons added before the merge
  double* bigA;              // m > 128: [n_dom][256][256] A (row-major), then T
  double* bigB;              // m > 128: [n_dom][256][256] L, then B = L J, then U (column-major)
  double* bigv;              // m > 128: [n_dom][5][256] b, wbar, lambda, spare
  int32_t* bigf;             // m > 128: [n_dom][4] converged, rounds that rotated, sweeps, spare
  uint32_t* dom_sweeps;      // [n_dom] Jacobi sweeps of each domain, summed over every analysis
  double* Ascr;              // FP64, m <= 128: [n_dom][m(m+1)/2] each domain's A (lower triangle packed by rows), for refining wbar
  double* dbg;               // [n_dom][2*m*m + m] C, lambda, T (NULL unless debug)
  int32_t* dbg_sweeps;       // [n_dom]
  InstState* st;
};

// Entries of one class in a batch.  Prefix arrays index the flattened work of
// the class: actuator rows, slope rows and domains of every entry.
struct ClassBatch {
  int32_t n;
  int32_t inst[kMaxBatch];        // index into the instance table
  int32_t ent[kMaxBatch];         // batch entry (position of y / outputs)
  int32_t act_off[kMaxBatch + 1];
  int32_t slope_off[kMaxBatch + 1];
  int32_t dom_off[kMaxBatch + 1];
  uint32_t next;                  // analysis work counter: items claimed past the first grid (k_slopes zeroes it)
  uint32_t pad;
};

struct BatchHdr {
  const double* yptr[kMaxBatch];  // slopes of entry e (device memory: staging slot or caller's buffer)
  double* amean;                  // analysis means (phi_k), entry e at out_off[e]
  double* pmean;                  // prediction means (phi_{k+1}), entry e at out_off[e]
  int32_t out_off[kMaxBatch];
  // check_y != 0 (server batches): the slope kernel sets bad[e] when entry e's
  // slopes hold a non-finite value, and the merge/forecast kernels then leave
  // that instance's ensemble and frame counter as they were.  The host uploads
  // the header with bad[] zeroed for every batch.
  int32_t check_y;
  int32_t bad[kMaxBatch];
  ClassBatch cls[kNumClasses];
};

// Per-domain debug record (LETKF_FLAG_DEBUG): C [m*m], lambda [m], T [m*m],
// then kDbgTail slots: 0-5 shader-clock stamps at the 6 phase boundaries,
// 6 HW_ID, 7 XCC_ID, 8 the workgroup index that ran the domain, 10-12 stamps
// inside the wbar/W/T phase (after U, after wbar, after its refinement).
constexpr int kDbgTail = 16;

// Arithmetic variant of an instance: its precision path, or 3 for the BF16
// path with FP32 rotations (fp32_rot: LETKF_FLAG_FP32_ROTATIONS, validated to
// come with LETKF_BF16).
inline int variant_of(int prec, bool fp32_rot) { return fp32_rot ? 3 : prec; }

inline int class_of(int padded_m, int prec, bool fp32_rot) {
  if (padded_m > 128) return kBigClass;  // validated to be FP64
  int s = padded_m <= 16 ? 0 : padded_m <= 32 ? 1 : padded_m <= 64 ? 2 : 3;
  return variant_of(prec, fp32_rot) * 4 + s;
}

// Entries of the packed lower triangle of an n x n matrix (row i starts at tri_size(i)).
__host__ __device__ inline int tri_size(int n) { return n * (n + 1) / 2; }

inline int padded_members(int m) {
  int p = 16;
  while (p < m) p *= 2;
  return p;
}

}  // namespace letkf
