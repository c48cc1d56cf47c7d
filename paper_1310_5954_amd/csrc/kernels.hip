// HIP kernels of the local ETKF frame (gfx950).
//
//   k_slopes    a3: Y' = D X'_phi and d = y - D xbar_phi, one thread per
//               (slope row, member), row means by wavefront shuffles.
//   k_rows      a1/a2/a8-merge: weighted merge of the per-domain analysis
//               rows into the ensemble, optionally fused with the AR forecast
//               (Philox4x32-10 + Box-Muller model noise) and the output means.
//   k_analysis  a4-a8: one workgroup per domain: gather, C and b, FP64
//               one-sided Jacobi eigensolver in LDS, wbar, W, T, update.
//
// All kernels walk the entries of one batch class (same padded ensemble size
// and storage precision) so that frames of several instances share a launch.
#include <hip/hip_runtime.h>

#include <mutex>

#include "desc.hpp"
#include "launch.hpp"

namespace letkf {

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and one Box-Muller normal per counter.
// ----------------------------------------------------------------------------
__device__ __forceinline__ double philox_normal(uint64_t seed, uint64_t frame, uint32_t act,
                                                uint32_t member) {
  uint32_t c0 = member, c1 = act, c2 = (uint32_t)frame, c3 = (uint32_t)(frame >> 32);
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  const uint64_t v1 = ((uint64_t)c0 << 21) | (c1 >> 11);
  const uint64_t v2 = ((uint64_t)c2 << 21) | (c3 >> 11);
  const double u1 = ((double)v1 + 0.5) * 0x1.0p-53;
  const double u2 = ((double)v2 + 0.5) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// Loads through a pointer into device memory taken from a descriptor.  Such a
// pointer is generic, and a generic (flat) load also counts against the LDS
// counter, so every LDS wait (s_waitcnt lgkmcnt) after a prefetch would wait
// for the prefetch too.  Reading through the global address space makes it a
// global load that only the vector-memory counter tracks.
template <typename T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
// The same for stores (a flat store also holds up the next LDS wait).
template <typename T>
__device__ __forceinline__ void gstore(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
// ... and for device-scope atomic adds whose result is not used.
template <typename T>
__device__ __forceinline__ void gatomic_add(T* p, T v) {
  (void)__hip_atomic_fetch_add((__attribute__((address_space(1))) T*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cross-lane moves of a double with DPP (VALU, no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  // Every pattern used here reads a valid lane, so no "old" value is needed.
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over aligned groups of G consecutive lanes (G = 2, 4, 8 or 16); every
// lane of a group ends with the group total.  Stages: swap neighbours, swap
// pairs (quad permutes), then mirror within 8 and within 16 lanes.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
  if constexpr (G >= 16) v += dpp_f64<0x140>(v); // row_mirror
  static_assert(G <= 16, "group_sum supports up to 16 lanes");
  return v;
}

// Sum of v over the MP lanes of a member row (MP <= 64: one wavefront segment;
// MP >= 128: wavefronts combined through LDS).  Every thread participates.
// Within 16 lanes by DPP (group_sum), across 16-lane rows by lane shuffles.
template <int MP>
__device__ __forceinline__ double row_sum(double v, double* red) {
  constexpr int W = MP < 64 ? MP : 64;
  v = group_sum<(W < 16 ? W : 16)>(v);
#pragma unroll
  for (int off = 16; off < W; off <<= 1) v += __shfl_xor(v, off, 64);
  if constexpr (MP > 64) {
    const int t = threadIdx.x;
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    const int base = (t / MP) * (MP / 64);
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < MP / 64; ++w) s += red[base + w];
    __syncthreads();
    v = s;
  }
  return v;
}

__device__ __forceinline__ int find_entry(const int32_t* off, int n, int g) {
  int b = 0;
  while (b + 1 < n && off[b + 1] <= g) ++b;
  return b;
}

template <typename T> __device__ __forceinline__ double ld(const T* p) { return (double)*p; }
template <typename T> __device__ __forceinline__ void st(T* p, double v) { *p = (T)v; }

// ----------------------------------------------------------------------------
// a3: slope perturbations and innovation of every slope row of the class,
// Y' = D X'_obs and d = y - D xbar_obs, X_obs the observed instant's rows.
// ----------------------------------------------------------------------------
template <typename T, int MP>
__global__ __launch_bounds__(256) void k_slopes(const InstDesc* __restrict__ tab,
                                                BatchHdr* __restrict__ hdr, int cls) {
  constexpr int RPB = 256 / MP;
  __shared__ double red[4];
  ClassBatch& cb = hdr->cls[cls];
  if (blockIdx.x == 0) {
    if ((int)threadIdx.x < cb.n) tab[cb.inst[threadIdx.x]].st->unconverged = 0;
    if (threadIdx.x == 0) cb.next = 0;  // the analysis launch that follows claims items from zero
  }
  const int j = threadIdx.x % MP;
  const int total = cb.slope_off[cb.n];
  // grid-stride over row groups (the trip count is uniform within a block)
  for (int base = blockIdx.x * RPB; base < total; base += gridDim.x * RPB) {
    const int g = base + threadIdx.x / MP;
    const bool active = g < total;
    const int b = find_entry(cb.slope_off, cb.n, active ? g : 0);
    const InstDesc& I = tab[cb.inst[b]];
    const int m = I.m;
    const int o = g - cb.slope_off[b];
    double v = 0.0;
    if (active && j < m) {
      // the observed instant: phi_k (ring slot cur) or phi_{k-1} (H = [0 D])
      const T* ens = (const T*)I.ens + (size_t)(I.st->cur ^ I.obs_inst) * I.n_act * m;
      for (int k = I.d_rowptr[o]; k < I.d_rowptr[o + 1]; ++k)
        v += I.d_val[k] * ld(ens + (size_t)I.d_col[k] * m + j);
    }
    const double ybar = row_sum<MP>(v, red) / (double)m;
    if (active) {
      if (j < m) st((T*)I.Yp + (size_t)o * m + j, v - ybar);
      if (j == 0) {
        const double yo = hdr->yptr[cb.ent[b]][o];
        I.d[o] = yo - ybar;
        if (hdr->check_y && !isfinite(yo)) hdr->bad[cb.ent[b]] = 1;  // every writer stores the same value
      }
    }
  }
}

// ----------------------------------------------------------------------------
// a8 merge and/or a1 forecast, per actuator row (both time instants).
//   MODE 0: merge only         -> ensemble = analysis, amean
//   MODE 1: forecast only      -> phi_{k+1} into the lagged slot, pmean, advance
//   MODE 2: merge + forecast   -> both, amean and pmean, advance
// ----------------------------------------------------------------------------
template <typename T, int MP, int MODE>
__global__ __launch_bounds__(256) void k_rows(const InstDesc* __restrict__ tab,
                                              BatchHdr* __restrict__ hdr, int cls) {
  constexpr int RPB = 256 / MP;
  __shared__ double red[4];
  ClassBatch& cb = hdr->cls[cls];
  const int j = threadIdx.x % MP;
  const int total = cb.act_off[cb.n];
  // grid-stride over row groups (the trip count is uniform within a block)
  for (int base = blockIdx.x * RPB; base < total; base += gridDim.x * RPB) {
    const int g = base + threadIdx.x / MP;
    const bool active = g < total;
    const int b = find_entry(cb.act_off, cb.n, active ? g : 0);
    const InstDesc& I = tab[cb.inst[b]];
    const int m = I.m;
    const int a = g - cb.act_off[b];
    const int cur = I.st->cur;
    const size_t slot = (size_t)I.n_act * m;
    T* ens = (T*)I.ens;
    T* e_cur = ens + (size_t)cur * slot;
    T* e_prev = ens + (size_t)(cur ^ 1) * slot;
    // an entry whose slopes were not finite keeps its ensemble (group-uniform:
    // the MP lanes of a row share the entry)
    const bool skip = hdr->check_y && hdr->bad[cb.ent[b]];
    const bool live = active && j < m && !skip;
    double vk = 0.0, vkm1 = 0.0;
    if (live) {
      if (MODE == 1) {
        vk = ld(e_cur + (size_t)a * m + j);
        vkm1 = ld(e_prev + (size_t)a * m + j);
      } else {
        const T* Z = (const T*)I.Z;
        for (int q = I.mptr[a]; q < I.mptr[a + 1]; ++q) {
          const double w = I.mw[q];
          double z0 = ld(Z + (size_t)I.mrow[2 * q] * m + j);
          double z1 = ld(Z + (size_t)I.mrow[2 * q + 1] * m + j);
          if (I.pist_c) {  // differential pistons of the covering domain (both instants)
            const double* c = I.pist_c + (size_t)I.mdom[q] * 2 * m;
            z0 += c[j];
            z1 += c[m + j];
          }
          vk += w * z0;
          vkm1 += w * z1;
        }
        // stored value (rounded to the storage type) is what the forecast uses
        vk = (double)(T)vk;
        vkm1 = (double)(T)vkm1;
        st(e_cur + (size_t)a * m + j, vk);
        if (MODE == 0) st(e_prev + (size_t)a * m + j, vkm1);
      }
    }
    const int ent = cb.ent[b];
    if (MODE != 1) {
      const double s = row_sum<MP>(live ? vk : 0.0, red);
      if (active && !skip && j == 0) hdr->amean[hdr->out_off[ent] + a] = s / (double)m;
    }
    if (MODE != 0) {
      double nx = 0.0;
      if (live) {
        nx = I.a1[a] * vk + I.a2[a] * vkm1;
        if (I.sigma_v != 0.0) nx += I.sigma_v * philox_normal(I.seed, I.st->frame, (uint32_t)a, (uint32_t)j);
        nx = (double)(T)nx;
        st(e_prev + (size_t)a * m + j, nx);
      }
      const double s = row_sum<MP>(nx, red);
      if (active && !skip && j == 0) hdr->pmean[hdr->out_off[ent] + a] = s / (double)m;
    }
  }
}

// ---- Differential pistons (Sec. 3.2), between the analysis and the merge ----
// One workgroup per (instance, domain) work item, thread (t, i) for instant t
// and member i.  k_piston_rhs: the overlap mismatch
//   r_l[t, i] = sum over the domain's actuators j of
//               (sum of the covering domains' rows at j) - k_j (own row at j),
// k_piston_solve: c_l = sum_l' G[l, l'] r_l' with the host-formed operator G.
// Instances created without LETKF_FLAG_PISTONS are skipped.
template <typename T>
__global__ __launch_bounds__(256) void k_piston_rhs(const InstDesc* __restrict__ tab, const BatchHdr* __restrict__ hdr,
                                                    int cls) {
  const ClassBatch& cb = hdr->cls[cls];
  const int total = cb.dom_off[cb.n], tid = threadIdx.x;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int eb = find_entry(cb.dom_off, cb.n, item);
    const InstDesc& I = tab[cb.inst[eb]];
    const int m = I.m;
    if (!I.pist_op || tid >= 2 * m) continue;
    const int l = item - cb.dom_off[eb], t = tid / m, i = tid % m;
    const T* Z = (const T*)I.Z;
    // terms precomputed at create (row, coefficient): independent loads
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    const int q0 = I.pist_ptr[l], q1 = I.pist_ptr[l + 1];
    int q = q0;
    for (; q + 8 <= q1; q += 8)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        acc[u] = fma(I.pist_coef[q + u], ld(Z + (size_t)I.pist_row[2 * (q + u) + t] * m + i), acc[u]);
    for (; q < q1; ++q) acc[0] = fma(I.pist_coef[q], ld(Z + (size_t)I.pist_row[2 * q + t] * m + i), acc[0]);
    double rsum = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) rsum += acc[u];
    I.pist_r[((size_t)l * 2 + t) * m + i] = rsum;
  }
}

__global__ __launch_bounds__(256) void k_piston_solve(const InstDesc* __restrict__ tab,
                                                      const BatchHdr* __restrict__ hdr, int cls) {
  const ClassBatch& cb = hdr->cls[cls];
  const int total = cb.dom_off[cb.n], tid = threadIdx.x;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int eb = find_entry(cb.dom_off, cb.n, item);
    const InstDesc& I = tab[cb.inst[eb]];
    const int m = I.m;
    if (!I.pist_op || tid >= 2 * m) continue;
    const int l = item - cb.dom_off[eb], t = tid / m, i = tid % m, n = I.n_dom;
    const double* g = I.pist_op + (size_t)l * n;
    // 16 independent partial sums keep that many L2 loads in flight
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    const double* r = I.pist_r + (size_t)t * m + i;
    int k = 0;
    for (; k + 16 <= n; k += 16)
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = fma(g[k + u], r[(size_t)(k + u) * 2 * m], acc[u]);
    for (; k < n; ++k) acc[0] = fma(g[k], r[(size_t)k * 2 * m], acc[0]);
    double c = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) c += acc[u];
    I.pist_c[((size_t)l * 2 + t) * m + i] = c;
  }
}

// After a forecast launch: the new instant becomes phi_k (ring swap) and the
// frame counter advances, for every instance of the class.  A launch of its
// own, ordered after k_rows on the stream, instead of a "last block" counter
// in k_rows: a completion counter that every block of k_rows increments
// serialises on one address and cost more than the whole merge.
__global__ __launch_bounds__(64) void k_advance(const InstDesc* __restrict__ tab, const BatchHdr* __restrict__ hdr,
                                                int cls) {
  const ClassBatch& cb = hdr->cls[cls];
  for (int e = threadIdx.x; e < cb.n; e += blockDim.x) {
    if (hdr->check_y && hdr->bad[cb.ent[e]]) continue;  // the frame was refused: nothing advanced
    InstState* S = tab[cb.inst[e]].st;
    S->cur ^= 1;
    S->frame += 1;
  }
}

// ----------------------------------------------------------------------------
// a4-a8: per-domain analysis, one 256-thread workgroup (4 wavefronts) per domain.
//
// P selects the contraction path: 0 = FP64 vector FMA, 1 = FP32 MFMA
// (v_mfma_f32_16x16x4f32), 2 = BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation, 3 = the BF16 path with its Jacobi rotations in FP32 (an
// opt-in variant, LETKF_FLAG_FP32_ROTATIONS).  The eigensolve, wbar and W are
// FP64 on paths 0-2; path 3 rotates in FP32 and keeps the Cholesky, lambda,
// wbar and W in FP64.  On the BF16 paths C uses split operands (hi + lo, three
// products): a single BF16 rounding of sqrt(r) Y' perturbs C by ~1e-3 of its
// largest eigenvalue, which exceeds the smallest ones ((m-1)/rho) that
// dominate W.
// ----------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// The thread index as a value the compiler may not move: every phase of the
// analysis derives its index arithmetic from it afresh.  Otherwise, inside the
// persistent item loop, the arithmetic of all phases (invariant across items)
// is hoisted out of the loop and stays live through the whole body, which
// costs registers and so occupancy.
__device__ __forceinline__ int phase_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

template <int M> struct AnaCfg {
  static constexpr int NT = 256;
  static constexpr int KC = 16;                    // FP64 path: rows per staged chunk (keeps m = 64 at 3 workgroups/CU)
  static constexpr int TM = M / 16;                // FP64 path: TM x TM outputs per thread
  static constexpr int TPP = (2 * NT / M) < M ? (2 * NT / M) : M;  // threads per Jacobi pair
  // Column stride of the M x M matrix in LDS: shifting consecutive columns by
  // one pair-group span (min(TPP, 8) doubles) spreads the pair groups of a
  // wavefront over all banks in every Jacobi step.
  static constexpr int LDB = M + (TPP < 8 ? TPP : 8);
  static constexpr int ACTIVE = (M / 2) * TPP;
  static constexpr int RPT = M / TPP;              // rows per thread in a Jacobi step
  static constexpr int MAX_SWEEPS = 40;
  // MFMA paths
  static constexpr int KCF = M <= 64 ? 32 : 16;    // FP32: observations per staged chunk
  // row stride (floats) of the transposed chunk: 2 mod 32, so that the 16 rows
  // and 2 k-offsets of a 32-lane operand load fall in 32 different banks
  static constexpr int LDKF = KCF + 2;
  static constexpr int KCB = 32;                   // BF16: observations per chunk (one k-step)
  static constexpr int LDKB = KCB + 8;             // row stride (bf16) of the transposed chunk
  static constexpr int KR = M <= 64 ? 32 : 16;     // update: state rows per chunk (16-row tiles)
  static constexpr size_t STAGE_BYTES = [] {
    size_t a = (size_t)KC * M * 8, b = (size_t)M * LDKF * 4, c = (size_t)M * LDKB * 2 * 2, d = (size_t)KR * M * 4;
    size_t x = a > b ? a : b;
    x = x > c ? x : c;
    return x > d ? x : d;
  }();
};

template <int M> struct AnaSmem {
  using C = AnaCfg<M>;
  double Bm[M * C::LDB];                              // A, then U, then T (row-major)
  alignas(16) unsigned char stage[C::STAGE_BYTES];    // chunk staging (phase-dependent type)
  double rc[32], dc[32];
  double bvec[M], nrm[M], lam[M], zv[M], wbar[M];
  double pcol[2][M];                                  // Cholesky pivot column (double buffer)
  int perm[M <= 64 ? M : 1];                          // FP64, M <= 64: A's symmetric permutation
  int s_rot;
  __device__ double* red() { return (double*)stage; }  // NT partial sums, aliases the staging area
};

// The entry (i, j) of A = (m-1)/rho I + C into LDS at (i, j) only: for the FP64
// gather, whose 16 tiles cover both halves and compute C_ij and C_ji with the
// same products summed in the same order (bitwise equal), so every entry is
// written once and along rows (the mirrored write went down a column, an 8-way
// bank conflict).
template <int M>
__device__ __forceinline__ void put_A_own(AnaSmem<M>& sm, int i, int j, int m, double c, double a_diag, double* dbg) {
  double v = c;
  if (i >= m || j >= m) v = (i == j) ? 1.0 : 0.0;
  else {
    if (dbg) dbg[i * m + j] = c;
    if (i == j) v += a_diag;
  }
  sm.Bm[i * AnaCfg<M>::LDB + j] = v;
}

// Writes the entry (i, j) of A = (m-1)/rho I + C into LDS (symmetrically: only
// the producer of i <= j writes, to both halves), padded members -> identity.
template <int M>
__device__ __forceinline__ void put_A(AnaSmem<M>& sm, int i, int j, int m, double c, double a_diag, double* dbg) {
  if (i > j) return;
  double v = c;
  if (i >= m || j >= m) v = (i == j) ? 1.0 : 0.0;
  else {
    if (dbg) { dbg[i * m + j] = c; dbg[j * m + i] = c; }
    if (i == j) v += a_diag;
  }
  sm.Bm[j * AnaCfg<M>::LDB + i] = v;
  sm.Bm[i * AnaCfg<M>::LDB + j] = v;
}

// ---- a4/a5 on the FP64 path: C = Y'^T diag(r) Y', b = Y'^T diag(r) d -------
template <int M>
__device__ void gather_C_fp64(AnaSmem<M>& sm, const InstDesc& I, int obs_off, int s, double* dbg) {
  using C = AnaCfg<M>;
  constexpr int NT = C::NT, KC = C::KC, TM = C::TM;
  double* Xc = (double*)sm.stage;
  const int m = I.m, tid = phase_tid(), ti = tid / 16, tj = tid % 16;
  double acc[TM][TM];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TM; ++y) acc[x][y] = 0.0;
  double bacc = 0.0;
  const double* Yp = (const double*)I.Yp;
  const int nobs = 2 * s;
  for (int q0 = 0; q0 < nobs; q0 += KC) {
    const int kc = min(KC, nobs - q0);
    for (int idx = tid; idx < KC * M; idx += NT) {
      const int qq = idx / M, j = idx % M;
      double v = 0.0;
      if (qq < kc && j < m) v = Yp[(size_t)I.obs_row[2 * obs_off + q0 + qq] * m + j];
      Xc[idx] = v;
    }
    if (tid < KC) {
      double r = 0.0, dd = 0.0;
      if (tid < kc) {
        r = I.obs_r[2 * obs_off + q0 + tid];
        dd = I.d[I.obs_row[2 * obs_off + q0 + tid]];
      }
      sm.rc[tid] = r;
      sm.dc[tid] = dd;
    }
    __syncthreads();
    for (int qq = 0; qq < kc; ++qq) {
      const double r = sm.rc[qq];
      double yi[TM], yj[TM];
#pragma unroll
      for (int x = 0; x < TM; ++x) {
        yi[x] = r * Xc[qq * M + ti + 16 * x];
        yj[x] = Xc[qq * M + tj + 16 * x];
      }
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TM; ++y) acc[x][y] += yi[x] * yj[y];
    }
    if (tid < M)
      for (int qq = 0; qq < kc; ++qq) bacc += sm.rc[qq] * sm.dc[qq] * Xc[qq * M + tid];
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TM; ++y) put_A<M>(sm, ti + 16 * x, tj + 16 * y, m, acc[x][y], I.a_diag, dbg);
  if (tid < M) sm.bvec[tid] = tid < m ? bacc : 0.0;
  __syncthreads();
}

// ---- a4/a5 on the FP64 path with FP64 MFMA (M <= 64) -------------------------
// As on the MFMA paths below, a chunk of KCH observations is staged transposed
// as At[j][k] = sqrt(r_k) Y'[k][j] (FP64), and wave w owns a WT x WT block of
// 16 x 16 tiles of C, accumulated by v_mfma_f64_16x16x4f64 in FP64 registers.
// A single wavefront per SIMD issues a VALU instruction only every ~8.5
// cycles, so the matrix core reaches the FP64 rate that the FMA loop cannot.
// (M = 128 would need 64 accumulators per lane and keeps the FMA loop.)
// Lane layout of v_mfma_f64_16x16x4f64 (measured on gfx950): A[i][k] in lane
// i + 16 k, B[k][j] in lane j + 16 k, and result register v of lane l holds
// D[l / 16 + 4 v][l % 16] (rows interleaved, unlike the FP32 16x16x4 form).
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int M>
__device__ void gather_C_fp64_mfma(AnaSmem<M>& sm, const InstDesc& I, int obs_off, int s, double* dbg) {
  using C = AnaCfg<M>;
  constexpr int NT = C::NT, KCH = 16, LDK = KCH + 1;  // LDK odd: the 16 rows of an operand load in 16 bank pairs
  constexpr int TILES = M / 16;
  constexpr int WT = TILES >= 2 ? TILES / 2 : 1;
  static_assert(M <= 64 && (size_t)M * LDK * 8 <= C::STAGE_BYTES, "staging");
  double* At = (double*)sm.stage;
  const int m = I.m, tid = phase_tid(), w = tid / 64, lane = tid % 64;
  const bool wave_on = TILES >= 2 || w == 0;
  const int tr0 = TILES >= 2 ? (w / 2) * WT : 0;
  const int tc0 = TILES >= 2 ? (w % 2) * WT : 0;
  f64x4 acc[WT][WT];
#pragma unroll
  for (int a = 0; a < WT; ++a)
#pragma unroll
    for (int b = 0; b < WT; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  double bpart = 0.0;
  const double* Yp = (const double*)I.Yp;
  const int nobs = 2 * s;
  // The domain's observation table (row of Y', sqrt(r), sqrt(r) d) is staged
  // in LDS, in the space A takes only once the products are done, by segments
  // of SEG observations (one segment on the ELT maps).  The chunk loop then
  // issues only the loads of Y' rows, three chunks of them in flight: with the
  // index, r and d loads in the loop, each chunk's loads waited on the
  // previous chunk's and a chunk spent ~5k cycles for ~1k of products.
  constexpr int SEG = (M * C::LDB * 8 / 20) / KCH * KCH;
  static_assert(SEG >= KCH && SEG % 2 == 0 && (size_t)SEG * (4 + 8 + 8) <= sizeof(sm.Bm), "observation table");
  int* rowT = reinterpret_cast<int*>(sm.Bm);
  double* sT = sm.Bm + SEG / 2;
  double* sdT = sT + SEG;
  const int32_t* obs_row = I.obs_row + 2 * obs_off;
  const double* obs_sr = I.obs_sr + 2 * obs_off;
  const double* dvec = I.d;
  // Thread (kk0 = tid / M, j = tid % M) stages observations kk0 + e NT / M of
  // every chunk for member j.
  constexpr int EPT = KCH * M / NT;
  static_assert(KCH * M % NT == 0, "whole chunks per thread");
  // M >= 64: a wavefront's lanes share kk0, so their table reads are broadcasts
  const int kk0 = M >= 64 ? __builtin_amdgcn_readfirstlane(tid / M) : tid / M, j = tid % M;
  for (int g0 = 0; g0 < nobs; g0 += SEG) {
    const int gn = nobs - g0 < SEG ? nobs - g0 : SEG;
    const int gr = (gn + KCH - 1) / KCH * KCH;
    // (the previous segment's last chunk ended with a barrier)
    for (int q = tid; q < gr; q += NT) {
      int rw = 0;
      double sr = 0.0, sd = 0.0;
      if (q < gn) {
        rw = gload(obs_row + g0 + q);
        sr = gload(obs_sr + g0 + q);
        sd = sr * gload(dvec + rw);
      }
      rowT[q] = rw;
      sT[q] = sr;
      sdT[q] = sd;
    }
    __syncthreads();
    auto fetch = [&](double (&y)[EPT], int q0) {  // Y' of chunk q0 (segment-relative)
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int q = q0 + kk0 + e * (NT / M);
        y[e] = 0.0;
        if (q < gn && j < m) y[e] = gload(Yp + (size_t)rowT[q] * m + j);
      }
    };
    auto chunk = [&](const double (&y)[EPT], double (&next)[EPT], int q0) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int q = q0 + kk0 + e * (NT / M);  // < gr: the table's tail is zero
        const double sy = sT[q] * y[e];
        bpart = fma(sdT[q], sy, bpart);  // r d y with r = sqrt(r)^2
        At[j * LDK + kk0 + e * (NT / M)] = sy;
      }
      __syncthreads();
      if (q0 + 2 * KCH < gn) fetch(next, q0 + 2 * KCH);
      if (wave_on) {
#pragma unroll
        for (int ks = 0; ks < KCH / 4; ++ks) {
          double av[WT], bv[WT];
#pragma unroll
          for (int a = 0; a < WT; ++a) {
            av[a] = At[((tr0 + a) * 16 + lane % 16) * LDK + ks * 4 + lane / 16];
            bv[a] = At[((tc0 + a) * 16 + lane % 16) * LDK + ks * 4 + lane / 16];
          }
#pragma unroll
          for (int a = 0; a < WT; ++a)
#pragma unroll
            for (int b = 0; b < WT; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
      }
      __syncthreads();
    };
    double ya[EPT], yb[EPT], yc[EPT];
    fetch(ya, 0);
    if (KCH < gn) fetch(yb, KCH);
    for (int q0 = 0; q0 < gn; q0 += 3 * KCH) {
      chunk(ya, yc, q0);
      if (q0 + KCH < gn) chunk(yb, ya, q0 + KCH);
      if (q0 + 2 * KCH < gn) chunk(yc, yb, q0 + 2 * KCH);
    }
  }
  if (wave_on) {
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
      for (int b = 0; b < WT; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          put_A_own<M>(sm, (tr0 + a) * 16 + lane / 16 + 4 * v, (tc0 + b) * 16 + lane % 16, m, acc[a][b][v], I.a_diag, dbg);
  }
  // b: threads sharing j = tid % M hold partial sums
  sm.red()[tid] = bpart;
  __syncthreads();
  if (tid < M) {
    double t = 0.0;
    for (int q = tid; q < NT; q += M) t += sm.red()[q];
    sm.bvec[tid] = tid < m ? t : 0.0;
  }
  __syncthreads();
}

// ---- a4/a5 on the MFMA paths ------------------------------------------------
// The chunk of observations is staged transposed, At[j][k] = sqrt(r_k) Y'[k][j],
// so that C = At At^T is one MFMA product per 16 x 16 tile.  Wave w owns a
// WT x WT block of tiles.  b is accumulated in FP64 from the FP32 slopes.
template <int P, int M>
__device__ void gather_C_mfma(AnaSmem<M>& sm, const InstDesc& I, int obs_off, int s, double* dbg) {
  using C = AnaCfg<M>;
  constexpr int NT = C::NT;
  constexpr int KCH = P == 1 ? C::KCF : C::KCB;
  constexpr int TILES = M / 16;
  constexpr int WT = TILES >= 2 ? TILES / 2 : 1;
  const int m = I.m, tid = phase_tid(), w = tid / 64, lane = tid % 64;
  const bool wave_on = TILES >= 2 || w == 0;
  const int tr0 = TILES >= 2 ? (w / 2) * WT : 0;
  const int tc0 = TILES >= 2 ? (w % 2) * WT : 0;
  f32x4 acc[WT][WT];
#pragma unroll
  for (int a = 0; a < WT; ++a)
#pragma unroll
    for (int b = 0; b < WT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  double bpart = 0.0;
  const float* Yp = (const float*)I.Yp;
  const int nobs = 2 * s;
  // FP32 path: every k-step's product (4 observations) comes out of the MFMA
  // on its own and is added into an FP64 accumulator in LDS (Bm, row-major,
  // each entry owned by one lane).  A single FP32 accumulator over all p_l
  // observations carries ~sqrt(p_l / 4) 2^-24 of |C|, which the inverse square
  // root amplifies by up to kappa(A) / 2 (~1e4 on the ELT workloads).
  constexpr int LDB = C::LDB;
  if constexpr (P == 1)
    for (int idx = tid; idx < M * LDB; idx += NT) sm.Bm[idx] = 0.0;
  // Thread (kk0 = tid / M, j = tid % M) stages observations kk0 + e NT / M of
  // every chunk for member j; the next chunk's rows are loaded into registers
  // before the current chunk's MFMAs, so their latency overlaps the products.
  constexpr int EPT = KCH * M / NT;
  static_assert(KCH * M % NT == 0, "whole chunks per thread");
  const int kk0 = M >= 64 ? __builtin_amdgcn_readfirstlane(tid / M) : tid / M, j = tid % M;
  float yv[EPT];
  double sv[EPT], dv[EPT];  // sqrt(r) (host-computed) and d; fetch() only issues loads
  const int32_t* obs_row = I.obs_row + 2 * obs_off;
  const double* obs_sr = I.obs_sr + 2 * obs_off;
  const double* dvec = I.d;
  auto fetch = [&](int q0) {
    if constexpr (M <= 64) {
      // global loads (see gload), the row indices first, then what depends on them
      int row[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int q = q0 + kk0 + e * (NT / M);
        row[e] = (q < nobs && j < m) ? gload(obs_row + q) : -1;
        sv[e] = q < nobs ? gload(obs_sr + q) : 0.0;
      }
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        yv[e] = 0.f;
        dv[e] = 0.0;
        if (row[e] >= 0) {
          dv[e] = gload(dvec + row[e]);
          yv[e] = gload(Yp + (size_t)row[e] * m + j);
        }
      }
    } else {  // M = 128: the indices of every value at once would not fit in the registers
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int q = q0 + kk0 + e * (NT / M);
        yv[e] = 0.f;
        sv[e] = dv[e] = 0.0;
        if (q < nobs && j < m) {
          const int row = gload(obs_row + q);
          sv[e] = gload(obs_sr + q);
          dv[e] = gload(dvec + row);
          yv[e] = gload(Yp + (size_t)row * m + j);
        }
      }
    }
  };
  fetch(0);
  for (int q0 = 0; q0 < nobs; q0 += KCH) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int kk = kk0 + e * (NT / M);
      const double y = (double)yv[e];
      const double sy = sv[e] * y;
      bpart += (sv[e] * dv[e]) * sy;  // r d y with r = sqrt(r)^2
      if constexpr (P == 1) ((float*)sm.stage)[j * C::LDKF + kk] = (float)sy;
      else {
        // split BF16: x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
        const float xf = (float)sy;
        const __bf16 hi = (__bf16)xf;
        ((__bf16*)sm.stage)[j * C::LDKB + kk] = hi;
        ((__bf16*)sm.stage)[M * C::LDKB + j * C::LDKB + kk] = (__bf16)(xf - (float)hi);
      }
    }
    __syncthreads();
    if (q0 + KCH < nobs) fetch(q0 + KCH);
    if (wave_on) {
      if constexpr (P == 1) {
        const float* At = (const float*)sm.stage;
#pragma unroll
        for (int ks = 0; ks < KCH / 4; ++ks) {
          float av[WT], bv[WT];
#pragma unroll
          for (int a = 0; a < WT; ++a) {
            av[a] = At[((tr0 + a) * 16 + lane % 16) * C::LDKF + ks * 4 + lane / 16];
            bv[a] = At[((tc0 + a) * 16 + lane % 16) * C::LDKF + ks * 4 + lane / 16];
          }
#pragma unroll
          for (int a = 0; a < WT; ++a)
#pragma unroll
            for (int b = 0; b < WT; ++b) {
              const f32x4 part = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
              double* cr = sm.Bm + ((tr0 + a) * 16 + 4 * (lane / 16)) * LDB + (tc0 + b) * 16 + lane % 16;
#pragma unroll
              for (int v = 0; v < 4; ++v) cr[v * LDB] += (double)part[v];
            }
        }
      } else {
        // C += hi hi^T + hi lo^T + lo hi^T (the lo lo^T term is below FP32 rounding)
        const __bf16* Ah = (const __bf16*)sm.stage;
        const __bf16* Al = Ah + M * C::LDKB;
        bf16x8 ah[WT], al[WT], bh[WT], bl[WT];
#pragma unroll
        for (int a = 0; a < WT; ++a) {
          const int ra = ((tr0 + a) * 16 + lane % 16) * C::LDKB + 8 * (lane / 16);
          const int rb = ((tc0 + a) * 16 + lane % 16) * C::LDKB + 8 * (lane / 16);
          ah[a] = *(const bf16x8*)(Ah + ra);
          al[a] = *(const bf16x8*)(Al + ra);
          bh[a] = *(const bf16x8*)(Ah + rb);
          bl[a] = *(const bf16x8*)(Al + rb);
        }
#pragma unroll
        for (int a = 0; a < WT; ++a)
#pragma unroll
          for (int b = 0; b < WT; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          }
      }
    }
    __syncthreads();
  }
  if (wave_on) {
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
      for (int b = 0; b < WT; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = (tr0 + a) * 16 + 4 * (lane / 16) + v, j = (tc0 + b) * 16 + lane % 16;
          // FP32 path: put_A of (i <= j) overwrites only (i, j), which this lane
          // owns, and (j, i), whose owner does not use its value; so every value
          // that is used is read before anything overwrites it.
          const double c = P == 1 ? sm.Bm[i * LDB + j] : (double)acc[a][b][v];
          put_A<M>(sm, i, j, m, c, I.a_diag, dbg);
        }
  }
  // b: threads sharing j = tid % M hold partial sums
  sm.red()[tid] = bpart;
  __syncthreads();
  if (tid < M) {
    double t = 0.0;
    for (int q = tid; q < NT; q += M) t += sm.red()[q];
    sm.bvec[tid] = tid < m ? t : 0.0;
  }
  __syncthreads();
}

// The BF16 paths at M <= 64: the same products as gather_C_mfma, with the
// observation table staged in LDS first (as in the FP64 gather: row of Y',
// sqrt(r), sqrt(r) d, in the space A takes afterwards), so that the chunk
// loop issues only the FP32 loads of Y' rows, three chunks in flight.  With
// the index, r and d loads in the loop a chunk of 32 observations spent
// ~6.6k cycles for a few hundred cycles of products.
template <int P, int M>
__device__ void gather_C_bf16_tab(AnaSmem<M>& sm, const InstDesc& I, int obs_off, int s, double* dbg) {
  using C = AnaCfg<M>;
  static_assert(P >= 2 && M <= 64, "BF16 paths, M <= 64");
  constexpr int NT = C::NT, KCH = C::KCB, LDKB = C::LDKB;
  constexpr int TILES = M / 16;
  constexpr int WT = TILES >= 2 ? TILES / 2 : 1;
  const int m = I.m, tid = phase_tid(), w = tid / 64, lane = tid % 64;
  const bool wave_on = TILES >= 2 || w == 0;
  const int tr0 = TILES >= 2 ? (w / 2) * WT : 0;
  const int tc0 = TILES >= 2 ? (w % 2) * WT : 0;
  f32x4 acc[WT][WT];
#pragma unroll
  for (int a = 0; a < WT; ++a)
#pragma unroll
    for (int b = 0; b < WT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  double bpart = 0.0;
  const float* Yp = (const float*)I.Yp;
  const int nobs = 2 * s;
  constexpr int SEG = (M * C::LDB * 8 / 20) / KCH * KCH;
  static_assert(SEG >= KCH && SEG % 2 == 0 && (size_t)SEG * (4 + 8 + 8) <= sizeof(sm.Bm), "observation table");
  int* rowT = reinterpret_cast<int*>(sm.Bm);
  double* sT = sm.Bm + SEG / 2;
  double* sdT = sT + SEG;
  const int32_t* obs_row = I.obs_row + 2 * obs_off;
  const double* obs_sr = I.obs_sr + 2 * obs_off;
  const double* dvec = I.d;
  // Thread (kk0 = tid / M, j = tid % M) stages observations kk0 + e NT / M of
  // every chunk for member j.
  constexpr int EPT = KCH * M / NT;
  static_assert(KCH * M % NT == 0, "whole chunks per thread");
  const int kk0 = M >= 64 ? __builtin_amdgcn_readfirstlane(tid / M) : tid / M, j = tid % M;
  __bf16* Ah = (__bf16*)sm.stage;
  __bf16* Al = Ah + M * LDKB;
  for (int g0 = 0; g0 < nobs; g0 += SEG) {
    const int gn = nobs - g0 < SEG ? nobs - g0 : SEG;
    const int gr = (gn + KCH - 1) / KCH * KCH;
    // (the previous segment's last chunk ended with a barrier)
    for (int q = tid; q < gr; q += NT) {
      int rw = 0;
      double sr = 0.0, sd = 0.0;
      if (q < gn) {
        rw = gload(obs_row + g0 + q);
        sr = gload(obs_sr + g0 + q);
        sd = sr * gload(dvec + rw);
      }
      rowT[q] = rw;
      sT[q] = sr;
      sdT[q] = sd;
    }
    __syncthreads();
    auto fetch = [&](float (&y)[EPT], int q0) {  // Y' of chunk q0 (segment-relative)
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int q = q0 + kk0 + e * (NT / M);
        y[e] = 0.f;
        if (q < gn && j < m) y[e] = gload(Yp + (size_t)rowT[q] * m + j);
      }
    };
    auto chunk = [&](const float (&y)[EPT], float (&next)[EPT], int q0) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int q = q0 + kk0 + e * (NT / M);  // < gr: the table's tail is zero
        const int kk = kk0 + e * (NT / M);
        const double sy = sT[q] * (double)y[e];
        bpart += sdT[q] * sy;  // r d y with r = sqrt(r)^2
        // split BF16: x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
        const float xf = (float)sy;
        const __bf16 hi = (__bf16)xf;
        Ah[j * LDKB + kk] = hi;
        Al[j * LDKB + kk] = (__bf16)(xf - (float)hi);
      }
      __syncthreads();
      if (q0 + 2 * KCH < gn) fetch(next, q0 + 2 * KCH);
      if (wave_on) {
        // C += hi hi^T + hi lo^T + lo hi^T (the lo lo^T term is below FP32 rounding)
        bf16x8 ah[WT], al[WT], bh[WT], bl[WT];
#pragma unroll
        for (int a = 0; a < WT; ++a) {
          const int ra = ((tr0 + a) * 16 + lane % 16) * LDKB + 8 * (lane / 16);
          const int rb = ((tc0 + a) * 16 + lane % 16) * LDKB + 8 * (lane / 16);
          ah[a] = *(const bf16x8*)(Ah + ra);
          al[a] = *(const bf16x8*)(Al + ra);
          bh[a] = *(const bf16x8*)(Ah + rb);
          bl[a] = *(const bf16x8*)(Al + rb);
        }
#pragma unroll
        for (int a = 0; a < WT; ++a)
#pragma unroll
          for (int b = 0; b < WT; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          }
      }
      __syncthreads();
    };
    float ya[EPT], yb[EPT], yc[EPT];
    fetch(ya, 0);
    if (KCH < gn) fetch(yb, KCH);
    for (int q0 = 0; q0 < gn; q0 += 3 * KCH) {
      chunk(ya, yc, q0);
      if (q0 + KCH < gn) chunk(yb, ya, q0 + KCH);
      if (q0 + 2 * KCH < gn) chunk(yc, yb, q0 + 2 * KCH);
    }
  }
  if (wave_on) {
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
      for (int b = 0; b < WT; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = (tr0 + a) * 16 + 4 * (lane / 16) + v, jj = (tc0 + b) * 16 + lane % 16;
          put_A<M>(sm, i, jj, m, (double)acc[a][b][v], I.a_diag, dbg);
        }
  }
  // b: threads sharing j = tid % M hold partial sums
  sm.red()[tid] = bpart;
  __syncthreads();
  if (tid < M) {
    double t = 0.0;
    for (int q = tid; q < NT; q += M) t += sm.red()[q];
    sm.bvec[tid] = tid < m ? t : 0.0;
  }
  __syncthreads();
}

// ---- a6 (first half): Cholesky factor A = L L^T (FP64) ----------------------
// Right-looking, by panels of 16 columns.  Wavefront 0 factors a panel on its
// own: lane l holds rows c0 + l (and c0 + 64 + l at M = 128) of the panel's
// 16 columns, the pivot of column j is read from lane j (readlane), column j is scaled by
// 1/sqrt(a_jj) (one rsqrt) and the later panel columns take its outer product
// with the entries L[c0+jj][c0+j] read from the lanes that hold them - no
// workgroup barrier inside the panel.  Then every wavefront subtracts the
// panel's rank-16 product from the lower triangle of the trailing matrix, in
// 16 x 16 tiles on v_mfma_f64_16x16x4f64 (accumulating onto the tile, with
// the right operand negated).  Two barriers per panel, against one per
// column for a column-at-a-time form.  L is left column-major in Bm (column c
// at Bm[c LDB ..]) with its upper triangle zeroed for the Jacobi phase.  A is
// SPD (all eigenvalues >= (m-1)/rho), so every pivot is positive.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int M>
__device__ __forceinline__ void cholesky(AnaSmem<M>& sm) {
  using C = AnaCfg<M>;
  constexpr int LDB = C::LDB, NT = C::NT, NP = M / 16;
  constexpr int RS = (M + 63) / 64;  // rows per lane: c0 + lane + 64 s, s < RS
  static_assert(M % 16 == 0 && M <= 128, "panels of 16 columns, at most two rows per lane");
  const int tid = phase_tid(), w = tid / 64, lane = tid % 64;
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    const int c0 = 16 * p;
    if (w == 0) {
      double a[RS][16];
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int r = c0 + lane + 64 * s;
        const bool on = r < M;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) a[s][jj] = on ? sm.Bm[(c0 + jj) * LDB + r] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double d = readlane_f64(a[0][j], j);  // a_jj after the earlier columns
        const double rs = rsqrt(d);
        double lj[RS];
        lj[0] = lane > j ? a[0][j] * rs : (lane == j ? d * rs : 0.0);
#pragma unroll
        for (int s = 1; s < RS; ++s) lj[s] = a[s][j] * rs;  // rows past the panel's diagonal block
#pragma unroll
        for (int s = 0; s < RS; ++s) a[s][j] = lj[s];
#pragma unroll
        for (int jj = j + 1; jj < 16; ++jj) {
          const double l = readlane_f64(lj[0], jj);
#pragma unroll
          for (int s = 0; s < RS; ++s) a[s][jj] = fma(-lj[s], l, a[s][jj]);
        }
      }
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int r = c0 + lane + 64 * s;
        if (r < M)
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) sm.Bm[(c0 + jj) * LDB + r] = a[s][jj];
      }
    }
    __syncthreads();
    // trailing lower triangle: tile (R, Cc), R >= Cc, of the blocks past the panel
    const int nt = NP - p - 1;
    int t = 0;
    for (int R = 0; R < nt; ++R)
      for (int Cc = 0; Cc <= R; ++Cc, ++t) {
        if (t % 4 != w) continue;
        const int rb = c0 + 16 * (R + 1), cb = c0 + 16 * (Cc + 1);
        // the tile transposed, D[i][j] = B(rb + j, cb + i): a lane's accumulators
        // then lie along one column of the column-major B, consecutive across
        // the 16 lanes (along a row they would be LDB apart, an 8-way bank
        // conflict on every load and store)
        f64x4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = sm.Bm[(cb + lane / 16 + 4 * v) * LDB + rb + lane % 16];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int k = c0 + 4 * ks + lane / 16;
          const double av = -sm.Bm[k * LDB + cb + lane % 16];
          const double bv = sm.Bm[k * LDB + rb + lane % 16];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) sm.Bm[(cb + lane / 16 + 4 * v) * LDB + rb + lane % 16] = acc[v];
      }
    __syncthreads();
  }
  for (int idx = tid; idx < M * M; idx += NT) {
    const int c = idx / M, r = idx % M;
    if (r < c) sm.Bm[c * LDB + r] = 0.0;
  }
  __syncthreads();
}

// 1/sqrt(x) for x in [1, 2] (no zero, infinity or denormal input): the
// hardware estimate e0 (relative error ~2^-23) refined by one third-order step
// c = c0 (1 + e/2 + 3e^2/8), e = 1 - x c0^2, which leaves a relative error of
// order e^3, below the rounding of the result.
__device__ __forceinline__ double rsqrt_1_2(double x) {
  const double c0 = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * c0, c0, 1.0);
  return fma(c0 * e, fma(e, 0.375, 0.5), c0);
}

// Rotation arithmetic in either precision.  approx_*: the hardware estimates
// (FP64: relative error ~2^-23; FP32: about 1 ulp); rsqrt_acc: 1/sqrt(x) for x
// in [1, 2] to the rounding of the type (FP32: the estimate already is).
__device__ __forceinline__ double approx_rsq(double x) { return __builtin_amdgcn_rsq(x); }
__device__ __forceinline__ float approx_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double approx_rcp(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float approx_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsqrt_acc(double x) { return rsqrt_1_2(x); }
// Issue priority of the calling wavefront (0..3; wavefront-uniform argument).
__device__ __forceinline__ void set_issue_prio(int p) {
  if (p >= 3) __builtin_amdgcn_s_setprio(3);
  else if (p == 2) __builtin_amdgcn_s_setprio(2);
  else if (p == 1) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}
// the word holding the sign: non-negative exactly when x >= +0
__device__ __forceinline__ int sign_word(double x) { return (int)(__double_as_longlong(x) >> 32); }
__device__ __forceinline__ int sign_word(float x) { return __float_as_int(x); }
__device__ __forceinline__ float rsqrt_acc(float x) { return __builtin_amdgcn_rsqf(x); }

// Group sum of a float (same lane patterns as the double form).
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
// lanes l and l ^ 8 exchange v (row_ror:8 within each row of 16 lanes)
__device__ __forceinline__ double swap_lanes8(double v) { return dpp_f64<0x128>(v); }
__device__ __forceinline__ float swap_lanes8(float v) { return dpp_f32<0x128>(v); }
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (G >= 2) v += dpp_f32<0xB1>(v);
  if constexpr (G >= 4) v += dpp_f32<0x4E>(v);
  if constexpr (G >= 8) v += dpp_f32<0x141>(v);
  if constexpr (G >= 16) v += dpp_f32<0x140>(v);
  static_assert(G <= 16, "group_sum supports up to 16 lanes");
  return v;
}

// True when every pair of columns of the current B satisfies
// (b_i.b_j)^2 <= tol2 |b_i|^2 |b_j|^2, i.e. when a further sweep would not
// rotate.  Each thread forms a TM x TM block of B^T B from LDS (the norms are
// the ones the sweep kept current).  Block-uniform result; ends with a barrier.
// B: column c at B[c * LD], element type R.
template <typename R, int M, int LD>
__device__ __forceinline__ bool gram_converged(const R* B, const R* nrm, R tol2) {
  constexpr int TM = AnaCfg<M>::TM;
  const int tid = phase_tid(), ti = tid / 16, tj = tid % 16;
  R g[TM][TM];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TM; ++y) g[x][y] = 0;
  // lane tj visits the rows from tj on (mod M): the 16 columns tj + 16 x that
  // a pass of lanes reads then fall in 16 bank pairs (all at one row they sat
  // in two, a column being LD doubles apart)
#pragma unroll 2
  for (int r0 = 0; r0 < M; ++r0) {
    const int r = (r0 + tj) & (M - 1);
    R u[TM], v[TM];
#pragma unroll
    for (int x = 0; x < TM; ++x) {
      u[x] = B[(ti + 16 * x) * LD + r];
      v[x] = B[(tj + 16 * x) * LD + r];
    }
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TM; ++y) g[x][y] = fma(u[x], v[y], g[x][y]);
  }
  bool bad = false;
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TM; ++y) {
      const int i = ti + 16 * x, j = tj + 16 * y;
      bad |= i < j && g[x][y] * g[x][y] > tol2 * (nrm[i] * nrm[j]);
    }
  return !__syncthreads_or(bad);
}

// The same test for FP64 columns at M = 64 with the products on the matrix
// cores: wavefront w forms the 2 x 2 tiles (16 x 16 each) of B^T B at tile rows
// 2 (w / 2), 2 (w / 2) + 1 and tile columns 2 (w % 2), 2 (w % 2) + 1.  Each lane
// reads two consecutive rows of its column with one 16-byte load, the A / B
// operands of two k-steps (rows r0 + 2 k and r0 + 2 k + 1 for the operand's
// k = lane / 16).  The VALU form spent ~25k cycles per test on 512 LDS loads
// and 1024 FMAs per thread; this one 64 MFMAs and 32 loads per wavefront.
template <int LD>
__device__ __forceinline__ bool gram_converged_mfma64(const double* B, const double* nrm, double tol2) {
  const int tid = phase_tid(), w = tid / 64, lane = tid % 64;
  const int tr0 = (w >> 1) * 2, tc0 = (w & 1) * 2;
  const int kq = lane / 16, cl = lane % 16;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (int r0 = 0; r0 < 64; r0 += 8) {
    const int r = r0 + 2 * kq;
    double2 av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      av[a] = *(const double2*)&B[((tr0 + a) * 16 + cl) * LD + r];
      bv[a] = *(const double2*)&B[((tc0 + a) * 16 + cl) * LD + r];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].y, acc[a][b], 0, 0, 0);
      }
  }
  bool bad = false;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = (tr0 + a) * 16 + kq + 4 * v, j = (tc0 + b) * 16 + cl;
        const double g = acc[a][b][v];
        bad |= i < j && g * g > tol2 * (nrm[i] * nrm[j]);
      }
  return !__syncthreads_or(bad);
}

// ---- a6 (second half): one-sided (Hestenes) Jacobi on the columns of L ------
// L J = U Sigma with U the eigenvectors of A = L L^T and lambda = sigma^2, so
// no rotation accumulator is needed; rounding scales with sqrt(lambda), and
// the Cholesky factor's columns start closer to orthogonal than those of A.
// A sweep visits the pairs (i, i^k), k = 1..M-1 (M-1 perfect matchings that
// cover every pair once).  Steps are grouped by the highest set bit h of k:
// within a group every pair joins a column with bit h clear (the "lower"
// column) to one with bit h set, and each lower column meets all its
// partners in that group, so its pair slot keeps it in registers for the
// whole group and only the partner column goes through LDS each step.
// The columns are B[c * LD ..] (element type R: FP64, or FP32 for the BF16
// path), their squared norms nrm[c]; tol is the rotation threshold.  Returns
// the sweeps done; `converged` is set when a sweep rotated nothing or the
// Gram test passed, and stays false when the sweep cap ended the loop.
template <typename R, int M, int LD>
__device__ __forceinline__ int jacobi_core(AnaSmem<M>& sm, int m, R* B, R* nrm, R tol, bool& converged, bool fair) {
  using C = AnaCfg<M>;
  constexpr int NT = C::NT, TPP = C::TPP;
  constexpr int PSW = 64 / TPP;  // pair slots per wavefront
  static_assert(TPP <= 64 && 64 % TPP == 0, "pair slots tile the wavefront");
  const int tid = phase_tid();
  const bool active = C::ACTIVE >= NT || tid < C::ACTIVE;
  const int q = tid / TPP, sub = tid % TPP;
  const R tol2 = tol * tol;
  // Once no rotation of a sweep had a relative off-diagonal above trig, the
  // next sweep is likely to find nothing to do, and the Gram test (a fraction
  // of a sweep's cost) is tried instead.  trig = tol^(1/3) / 5: on a CPU
  // replay of the 375 domains of the 84 x 84 map this is where fewer wasted
  // final sweeps stop paying for more failed Gram tests (FP64, tol 4.5e-13:
  // 7.63 -> 7.08 sweeps and 0.44 -> 1.03 Gram tests per domain against the
  // former 1e-7; tol 1e-6: 6.96 -> 6.3 sweeps; tol 1e-4 stays at 6.0).
  const R trig = (R)0.2 * cbrt(tol);
  const R trig2 = trig * trig;
  const R tol4 = (R)4 * tol2, trig4 = (R)4 * trig2;
  constexpr bool PREFETCH = C::RPT <= 16;
  // partners exchanged between slots q and q ^ 1 by a lane swap within 16-lane rows
  constexpr bool SWAP = PREFETCH && TPP == 8;
  // the step's column and norm accesses through LDS-typed pointers, so that
  // their addresses are 32-bit offsets (a generic pointer makes every partner
  // address a 64-bit multiply-add)
  using LR = __attribute__((address_space(3))) R;
  LR* const LB = (LR*)B;
  LR* const LN = (LR*)nrm;
  int sweeps = 0;
  converged = false;
  for (; sweeps < C::MAX_SWEEPS;) {
    // progress-ordered issue (see k_analysis): the priority falls as the sweeps go by
    if (fair) set_issue_prio(sweeps < 3 ? 3 : sweeps < 5 ? 2 : sweeps < 6 ? 1 : 0);
    {
      constexpr int TPC = NT / M;  // threads per column for the norms
      const int c = tid / TPC, part = tid % TPC;
      // de Rijk's ordering: every sweep starts with the m columns sorted by
      // decreasing norm (the padded unit columns stay at m..M-1), which saves
      // about one sweep in twelve on the ELT domains (CPU replay).  A column's
      // rank is counted by its TPC threads over interleaved norms; the columns
      // move, in passes of at most 16 values per thread, only when the order
      // changed (late sweeps mostly keep it).
      constexpr int PER = M / TPC, CH = PER < 16 ? PER : 16;
      R ss = 0;
      // column c's threads start at a row that shifts with c, so that the four
      // columns a pass of lanes reads fall in different banks
      for (int j0 = 0; j0 < PER; ++j0) {
        const R v = B[c * LD + part + TPC * ((j0 + c) & (PER - 1))];
        ss = fma(v, v, ss);
      }
      ss = group_sum<TPC>(ss);
      if (part == 0) nrm[c] = ss;
      if (tid == 0) sm.s_rot = 0;  // last read before the previous sweep's closing barrier
      __syncthreads();
      R ahead = 0;  // columns ahead of c among this thread's share (exact small integers)
      if (c < m)
        for (int c2 = part; c2 < m; c2 += TPC) {
          const R n2 = nrm[c2];
          ahead += (n2 > ss || (n2 == ss && c2 < c)) ? (R)1 : (R)0;
        }
      ahead = group_sum<TPC>(ahead);
      const int rank = c < m ? (int)ahead : c;
      if (__syncthreads_or(rank != c)) {
        for (int k0 = 0; k0 < PER; k0 += CH) {
          // rows rotated by c within the pass, as in the norms: the reads then
          // avoid bank conflicts, and the writes (to the rank's column, same
          // rows) mostly do
          R v[CH];
#pragma unroll
          for (int k = 0; k < CH; ++k) v[k] = B[c * LD + part + TPC * (k0 + ((k + c) & (CH - 1)))];
          // every read of this pass's rows (rows TPC k0 .. TPC (k0 + CH) - 1, which no
          // other pass touches) is done before any column moves; the sweep reads
          // the moved columns after the barrier that follows
          __syncthreads();
          // the write addresses recomputed from a copy of c the compiler cannot
          // see through: kept from the reads, the CH addresses stayed live
          // across the barrier and raised the kernel's register count
          int cw = c;
          __asm__ volatile("" : "+v"(cw));
#pragma unroll
          for (int k = 0; k < CH; ++k) B[rank * LD + part + TPC * (k0 + ((k + cw) & (CH - 1)))] = v[k];
        }
        if (part == 0) nrm[rank] = ss;
        __syncthreads();  // the moved columns and norms before the sweep reads them
      }
    }
    int big = INT_MIN;
#pragma unroll
    for (int h = 0; (1 << h) < M; ++h) {
      const int i = ((q >> h) << (h + 1)) | (q & ((1 << h) - 1));
      const int kend = 2 << h;
      R xi[C::RPT];
      R al = 0;
      // One step k: pair (i, i ^ k) with the partner column in xc (norm bc).
      // With PREFETCH the next step's partner arrives in xn (norm bn) before
      // this step rotates the lower column (registers only), so that its
      // latency overlaps that arithmetic instead of stalling the next dot
      // product; two register sets alternate between consecutive steps.
      // (M = 128 holds 32 rows per lane: a second set would spill, so there
      // each step loads its own partner.)
      // Between an even step k and k + 1 the slots exchange partners in pairs
      // (slot q takes the column slot q ^ 1 just rotated), so with SWAP the
      // rotated partner goes to its next slot by a lane swap and not through
      // LDS; the odd step after it writes that column back, rotated or not,
      // since its LDS copy is then out of date.
      auto step = [&](const int k, R (&xc)[C::RPT], R& bc, R (&xn)[C::RPT], R& bn) {
        // the lower column index as a value the compiler may not carry across
        // steps: unrolled, it would otherwise keep every step's partner
        // address live from the start of the group (registers, occupancy)
        int iv = i;
        __asm__ volatile("" : "+v"(iv));
        iv &= M - 1;  // a known range: 24-bit multiply-adds for the addresses
        const int jj = iv ^ k;
        const bool swp = SWAP && (k & 1) == 0 && k + 1 < kend;
        const bool stale = SWAP && (k & 1) == 1 && k > (1 << h);
        R c = 1, sn = 0;
        bool rot = false;
        if (!PREFETCH && active) {
#pragma unroll
          for (int t = 0; t < C::RPT; ++t) xc[t] = LB[jj * LD + sub + t * TPP];
          bc = LN[jj];
        }
        if (active) {
          R g0 = 0, g1 = 0;
#pragma unroll
          for (int t = 0; t < C::RPT; ++t) {
            if (t & 1) g1 = fma(xi[t], xc[t], g1);
            else g0 = fma(xi[t], xc[t], g0);
          }
          const R gsum = group_sum<TPP>(g0 + g1);
          // (2 gsum)^2 serves both the test, against 4 tol^2 al bc, and the angle
          const R ab = al * bc, g2 = gsum + gsum, g4 = g2 * g2;
          if (swp) {
            // A step whose partner leaves by the lane exchange: when any pair of
            // the wavefront rotates, every lane takes the step, a lane whose pair
            // does not with t = 0, c = 1, sn = 0 (an exact identity).  The branch
            // is wavefront-uniform, so the rotated columns need no merge with
            // the unrotated ones of masked lanes (that merge cost a register move
            // per value).
            rot = g4 > tol4 * ab;
            if (__builtin_amdgcn_ballot_w64(rot) != 0) {
              big = max(big, sign_word(fma(-trig4, ab, g4)));  // negative where no rotation
              const R dd = bc - al;
              const R q2 = fma(dd, dd, g4);
              const R den = fma(q2, approx_rsq(q2), fabs(dd));
              const R t = rot ? copysign((R)1, dd) * g2 * approx_rcp(den) : (R)0;
              c = rot ? rsqrt_acc(fma(t, t, (R)1)) : (R)1;
              sn = c * t;
#pragma unroll
              for (int u = 0; u < C::RPT; ++u) {
                const R a = xi[u], b = xc[u];
                xi[u] = c * a - sn * b;
                xc[u] = sn * a + c * b;
              }
              al -= t * gsum;
              bc += t * gsum;
              sm.s_rot = 1;
              // the exchange on both sides of the branch, so that the rotated
              // partner goes from the registers it was computed in
#pragma unroll
              for (int u = 0; u < C::RPT; ++u) xn[u] = swap_lanes8(xc[u]);
              bn = swap_lanes8(bc);
            } else {
#pragma unroll
              for (int u = 0; u < C::RPT; ++u) xn[u] = swap_lanes8(xc[u]);
              bn = swap_lanes8(bc);
            }
          } else if (g4 > tol4 * ab) {
            rot = true;
            // the largest sign word of g4 - 4 trig^2 al bc: non-negative once a
            // rotation of this sweep had a cosine above trig (an integer
            // maximum: no exec-mask update, no NaN handling)
            big = max(big, sign_word(fma(-trig4, ab, g4)));
            // t = tan(theta), the smaller root of t^2 + 2 zeta t - 1 = 0 with
            // zeta = (be - al) / (2 gsum), written without the quotient zeta.
            // c = (1 + t^2)^(-1/2) to the rounding of R keeps c^2 + s^2 = 1 to
            // rounding for whatever t is used, so t itself comes from the
            // hardware's approximate rsq / rcp: its error only changes how far
            // this rotation reduces gsum, never orthogonality.
            const R dd = bc - al;
            const R q2 = fma(dd, dd, g4);
            const R den = fma(q2, approx_rsq(q2), fabs(dd));
            const R t = copysign((R)1, dd) * g2 * approx_rcp(den);
            c = rsqrt_acc(fma(t, t, (R)1));
            sn = c * t;
            // the partner first: the slot that pairs it next reads it from LDS
            LR* bj = LB + jj * LD;
#pragma unroll
            for (int u = 0; u < C::RPT; ++u) bj[sub + u * TPP] = sn * xi[u] + c * xc[u];
            al -= t * gsum;
            bc += t * gsum;
            // one lane of the slot stores the norm and the flag (all eight storing
            // the same value saved an exec-mask region but cost ~1 % of the sweep)
            if (sub == 0) {
              LN[jj] = bc;
              sm.s_rot = 1;
            }
          }
          if (stale && !rot) {
            LR* bj = LB + jj * LD;
#pragma unroll
            for (int u = 0; u < C::RPT; ++u) bj[sub + u * TPP] = xc[u];
            LN[jj] = bc;
          }
        }
        // Step k + 1 reads a partner column (and its norm) that step k wrote:
        // the writer's lower column differs from this slot's in the low bits
        // where k and k + 1 differ, so it is a pair slot of the same wavefront
        // unless k + 1 is a multiple of PSW, and the LDS operations of one
        // wavefront take effect in order.  Only those steps need the
        // workgroup barrier (the group's last step is followed by one anyway);
        // the others only keep the compiler from moving LDS accesses across.
        if ((k + 1) % PSW == 0 && k + 1 < kend) __syncthreads();
        else __asm__ volatile("" ::: "memory");
        if (PREFETCH && active && !swp && k + 1 < kend) {
          const LR* bk = LB + (iv ^ (k + 1)) * LD;
#pragma unroll
          for (int t = 0; t < C::RPT; ++t) xn[t] = bk[sub + t * TPP];
          bn = LN[iv ^ (k + 1)];
        }
        if (rot && !swp) {
#pragma unroll
          for (int u = 0; u < C::RPT; ++u) xi[u] = c * xi[u] - sn * xc[u];
        }
      };
      R xa[C::RPT], xb[PREFETCH ? C::RPT : 1];
      R ba = 0, bb = 0;
      if (active) {
        const R* b0 = B + (i ^ (1 << h)) * LD;  // the group's first partner
#pragma unroll
        for (int t = 0; t < C::RPT; ++t) {
          xi[t] = B[i * LD + sub + t * TPP];
          if (PREFETCH) xa[t] = b0[sub + t * TPP];
        }
        al = nrm[i];
        if (PREFETCH) ba = nrm[i ^ (1 << h)];
      }
      if constexpr (PREFETCH) {
#pragma unroll
        for (int k = 1 << h; k < kend; k += 2) {
          step(k, xa, ba, xb, bb);
          if (k + 1 < kend) step(k + 1, xb, bb, xa, ba);
        }
      } else {
        for (int k = 1 << h; k < kend; ++k) step(k, xa, ba, xa, ba);
      }
      if (active) {
#pragma unroll
        for (int t = 0; t < C::RPT; ++t) B[i * LD + sub + t * TPP] = xi[t];
        if (sub == 0) nrm[i] = al;
      }
      __syncthreads();
    }
    ++sweeps;
    const int any = sm.s_rot;
    const int any_big = __syncthreads_or(big >= 0);
    bool gram = false;
    if (any && !any_big) {
      if constexpr (sizeof(R) == 8 && M == 64 && LD % 2 == 0) gram = gram_converged_mfma64<LD>((const double*)B, (const double*)nrm, (double)tol2);
      else gram = gram_converged<R, M, LD>(B, nrm, tol2);
    }
    if (!any || gram) {
      converged = true;
      break;
    }
  }
  return sweeps;
}

// Rotations are skipped once |b_i.b_j| <= tol |b_i| |b_j|; the W and T this
// leaves behind are off by about 4 tol (relative).  FP64 path: tol = 32 M eps
// (2.3e-13 at M = 64).  The rounding of the eigenvectors (eps |L| per column,
// amplified by the conditioning) leaves W about 2e-12 off whatever the
// tolerance, so this one adds nothing measurable: over the 375 domains of the
// 84x84 map, W stays within 2.05e-12 of the exact one against 2.00e-12 at
// tol = M eps, in at most 8 sweeps instead of 11 (CPU replay).  The FP32 and
// BF16 paths form C with relative errors ~5e-8 and ~4e-6, which put their T
// about 6e-5 and 4e-3 from the FP64 result whatever the eigensolver does;
// their tolerances, 1e-6 and 1e-4, keep the eigensolver's share an order of
// magnitude below that.  At 1e-4 the rotations themselves can run in FP32
// (rounding ~6e-8 per rotation, a converged off-diagonal of a few 1e-6), which
// the opt-in BF16 variant (P = 3) does: L is rounded to FP32 in place (float
// columns at stride M + TPP inside the double storage), rotated, and widened
// back.  The other paths rotate in FP64.
template <int P, int M>
__device__ int jacobi(AnaSmem<M>& sm, int m, bool& converged, bool fair) {
  using C = AnaCfg<M>;
  if constexpr (P == 3) {
    // In-place width change by chunks of CC columns (at most 16 values per
    // thread in flight).  A float column c ends at or below the start of
    // double column c + 1 (LDF <= 2 LDB and M <= 2 LDB), so narrowing in
    // increasing column order, and widening in decreasing order, never
    // overwrites a value that a later chunk still has to read; each chunk
    // reads everything before its barrier and writes after it.
    constexpr int NT = C::NT, LDB = C::LDB, LDF = M + C::TPP;
    constexpr int CC = M * M / NT <= 16 ? M : 16 * NT / M, PER = CC * M / NT;
    static_assert(LDF <= 2 * LDB && M <= 2 * LDB && M % CC == 0 && (CC * M) % NT == 0,
                  "float columns fit in the double storage");
    float* Bf = reinterpret_cast<float*>(sm.Bm);
    float* nf = reinterpret_cast<float*>(sm.nrm);
    const int tid = phase_tid();
    for (int c0 = 0; c0 < M; c0 += CC) {
      float v[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = tid + NT * k, c = c0 + idx / M, r = idx % M;
        v[k] = (float)sm.Bm[c * LDB + r];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = tid + NT * k, c = c0 + idx / M, r = idx % M;
        Bf[c * LDF + r] = v[k];
      }
    }
    __syncthreads();
    const int sweeps = jacobi_core<float, M, LDF>(sm, m, Bf, nf, 1e-4f, converged, fair);
    for (int c0 = M - CC; c0 >= 0; c0 -= CC) {
      float v[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = tid + NT * k, c = c0 + idx / M, r = idx % M;
        v[k] = Bf[c * LDF + r];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = tid + NT * k, c = c0 + idx / M, r = idx % M;
        sm.Bm[c * LDB + r] = (double)v[k];
      }
    }
    __syncthreads();
    return sweeps;
  } else {
    const double tol = P == 0 ? 32.0 * (double)M * 1.1102230246251565e-16 : (P == 1 ? 1e-6 : 1e-4);
    return jacobi_core<double, M, C::LDB>(sm, m, sm.Bm, sm.nrm, tol, converged, fair);
  }
}

// Products with the M x M matrix in LDS (column c at Bm[c * LDB ..]), by
// TPC = NT / M lanes per output reduced by DPP: lane group o = tid / TPC,
// lane part = tid % TPC takes every TPC-th term (two accumulators), and every
// lane of the group gets the sum.  With the column stride LDB the lanes of a
// wavefront read distinct banks in both forms.
// colsum: sum over r of Bm[o LDB + r] v[r]   (U^T v for U in the columns)
template <int M>
__device__ __forceinline__ double colsum(const AnaSmem<M>& sm, const double* v, int o, int part) {
  using C = AnaCfg<M>;
  constexpr int TPC = C::NT / M, PER = M / TPC, LDB = C::LDB;
  double t0 = 0.0, t1 = 0.0;
#pragma unroll 8
  for (int k = 0; k < PER; k += 2) {
    t0 = fma(sm.Bm[o * LDB + part + TPC * k], v[part + TPC * k], t0);
    if (k + 1 < PER) t1 = fma(sm.Bm[o * LDB + part + TPC * (k + 1)], v[part + TPC * (k + 1)], t1);
  }
  return group_sum<TPC>(t0 + t1);
}
// rowsum: sum over c of Bm[c LDB + o] z[c]   (U z)
template <int M>
__device__ __forceinline__ double rowsum(const AnaSmem<M>& sm, const double* z, int o, int part) {
  using C = AnaCfg<M>;
  constexpr int TPC = C::NT / M, PER = M / TPC, LDB = C::LDB;
  double t0 = 0.0, t1 = 0.0;
#pragma unroll 8
  for (int k = 0; k < PER; k += 2) {
    t0 = fma(sm.Bm[(part + TPC * k) * LDB + o], z[part + TPC * k], t0);
    if (k + 1 < PER) t1 = fma(sm.Bm[(part + TPC * (k + 1)) * LDB + o], z[part + TPC * (k + 1)], t1);
  }
  return group_sum<TPC>(t0 + t1);
}

// One step of iterative refinement of wbar = A^-1 b (FP64 path).  U from the
// one-sided Jacobi carries rounding of order eps |L| in every column, which the
// weights 1/lambda of U Lambda^-1 U^T b amplify for the small eigenvalues
// (wbar relative errors ~1e-10 at m = 100 against ~1e-12 for W).  The
// residual res = b - A wbar is therefore formed with A itself, as the gather
// built it (Ag: the domain's copy of A = (m-1)/rho I + C taken before the
// Cholesky, its lower triangle packed by rows), not through the eigenvectors,
// and wbar += U Lambda^-1 U^T res.  Uses pcol[0] (residual) and pcol[1].
template <int M>
__device__ void refine_wbar(AnaSmem<M>& sm, const double* __restrict__ Ag, int m) {
  constexpr int TPC = AnaCfg<M>::NT / M, PER = M / TPC;
  const int tid = phase_tid(), o = tid / TPC, part = tid % TPC;
  double* res = sm.pcol[0];
  double* z = sm.pcol[1];
  __syncthreads();  // wbar complete
  {
    // (A wbar)_o: row o of the symmetric A; entry (o, c) is packed at row
    // max(o, c), column min(o, c).  Padded rows and columns read entry 0 and
    // are masked by arithmetic (res is zero past m anyway).
    double a[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int c = part + TPC * k;
      const bool in = c < m && o < m;
      const int hi = c > o ? c : o, lo = c > o ? o : c;
      a[k] = (in ? 1.0 : 0.0) * gload(Ag + (in ? tri_size(hi) + lo : 0));
    }
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int k = 0; k < PER; k += 2) {
      t0 = fma(a[k], sm.wbar[part + TPC * k], t0);
      if (k + 1 < PER) t1 = fma(a[k + 1], sm.wbar[part + TPC * (k + 1)], t1);
    }
    const double t = group_sum<TPC>(t0 + t1);
    if (part == 0) res[o] = o < m ? sm.bvec[o] - t : 0.0;
  }
  __syncthreads();
  {
    const double t = colsum<M>(sm, res, o, part);
    if (part == 0) z[o] = o < m ? t / sm.lam[o] : 0.0;
  }
  __syncthreads();
  {
    const double w = rowsum<M>(sm, z, o, part);
    if (part == 0 && o < m) sm.wbar[o] += w;
  }
  __syncthreads();
}

// One step of iterative refinement of wbar on the FP32 / BF16 paths, whose
// Jacobi stops at a looser tolerance: there U^T is a poorer inverse of U, and
// the 1/lambda weights make wbar = U Lambda^-1 U^T b some 1e3 - 1e4 tol off,
// while W stays within 4 tol.  The normalised columns of L J still satisfy
// U Lambda U^T = (L J)(L J)^T = L L^T = A to rounding whether or not the
// sweeps converged, so res = b - U (Lambda (U^T wbar)) is an accurate residual
// from LDS alone, and each wbar += U Lambda^-1 U^T res shrinks the error by a
// factor of order tol kappa(A): two steps at tol 1e-6 and three at 1e-4 leave
// wbar below 1e-8 and 2e-5 on the 15x15 (m = 100) and 84x84 workloads.
template <int M>
__device__ void refine_wbar_lj(AnaSmem<M>& sm, int m) {
  constexpr int TPC = AnaCfg<M>::NT / M;
  const int tid = phase_tid(), o = tid / TPC, part = tid % TPC;
  double* z = sm.pcol[0];
  double* res = sm.pcol[1];
  __syncthreads();  // wbar complete
  {
    const double t = colsum<M>(sm, sm.wbar, o, part);
    if (part == 0) z[o] = o < m ? sm.lam[o] * t : 0.0;
  }
  __syncthreads();
  {
    const double t = rowsum<M>(sm, z, o, part);
    if (part == 0) res[o] = o < m ? sm.bvec[o] - t : 0.0;
  }
  __syncthreads();
  {
    const double t = colsum<M>(sm, res, o, part);
    if (part == 0) z[o] = o < m ? t / sm.lam[o] : 0.0;
  }
  __syncthreads();
  {
    const double w = rowsum<M>(sm, z, o, part);
    if (part == 0 && o < m) sm.wbar[o] += w;
  }
  __syncthreads();
}

// ---- a7: lambda, U, wbar = U Lambda^-1 U^T b, T = U sqrt((m-1)/Lambda) U^T + wbar 1^T
// (from the converged columns sigma_i u_i of L J)
// Leaves T row-major in Bm (T[k][j] at Bm[k*LDB + j], zero outside m x m).
template <int P, int M>
__device__ void transform(AnaSmem<M>& sm, const InstDesc& I, int l, double* dbg) {
  const int m = I.m;
  using C = AnaCfg<M>;
  constexpr int NT = C::NT, LDB = C::LDB, TM = C::TM;
  const int tid = phase_tid(), ti = tid / 16, tj = tid % 16;
  // debug: shader-clock stamps inside this phase (after U, after wbar, after its refinement)
  auto substamp = [&](int k) {
    if (dbg && threadIdx.x == 0) dbg[2 * m * m + m + 10 + k] = (double)clock64();
  };
  {
    constexpr int TPC = NT / M;
    const int c = tid / TPC, part = tid % TPC;
    double ss = 0.0;
    for (int r = part; r < M; r += TPC) { const double v = sm.Bm[c * LDB + r]; ss += v * v; }
    ss = group_sum<TPC>(ss);
    if (part == 0) {
      sm.lam[c] = ss;          // columns of L J are sigma_i u_i and lambda_i = sigma_i^2
      sm.nrm[c] = 1.0 / sqrt(ss);
    }
  }
  __syncthreads();
  for (int idx = tid; idx < M * M; idx += NT) {
    const int c = idx / M, r = idx % M;
    sm.Bm[c * LDB + r] *= sm.nrm[c];
  }
  __syncthreads();
  substamp(0);
  {
    // wbar = U Lambda^-1 U^T b
    constexpr int TPC = NT / M;
    const int o = tid / TPC, part = tid % TPC;
    const double t = colsum<M>(sm, sm.bvec, o, part);
    if (part == 0) {
      sm.zv[o] = o < m ? t / sm.lam[o] : 0.0;
      sm.nrm[o] = o < m ? sqrt((double)(m - 1) / sm.lam[o]) : 0.0;
    }
    __syncthreads();
    const double w = rowsum<M>(sm, sm.zv, o, part);
    if (part == 0) sm.wbar[o] = o < m ? w : 0.0;
  }
  __syncthreads();
  substamp(1);
  if constexpr (P == 0) {
    refine_wbar<M>(sm, I.Ascr + (size_t)l * tri_size(m), m);
  } else {
#pragma unroll 1
    for (int k = 0; k < (P == 1 ? 2 : 3); ++k) refine_wbar_lj<M>(sm, m);
  }
  substamp(2);
  if constexpr (M <= 64) {
    // T = (U S) U^T on v_mfma_f64_16x16x4f64 (S = diag sqrt((m-1)/lambda), zero
    // past m): k-steps over 4 columns c of U; wave w owns the same WT x WT block
    // of 16 x 16 tiles as in the FP64 gather.  Column c of U is Bm[c LDB ..],
    // so A[i][k] = U[i][c] s_c and B[k][j] = U[j][c] are rows of LDS columns.
    constexpr int TILES = M / 16, WT = TILES >= 2 ? TILES / 2 : 1;
    const int w = tid / 64, lane = tid % 64;
    const bool wave_on = TILES >= 2 || w == 0;
    const int tr0 = TILES >= 2 ? (w / 2) * WT : 0;
    const int tc0 = TILES >= 2 ? (w % 2) * WT : 0;
    f64x4 acc[WT][WT];
#pragma unroll
    for (int a = 0; a < WT; ++a)
#pragma unroll
      for (int b = 0; b < WT; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    if (wave_on) {
#pragma unroll 4
      for (int ks = 0; ks < M / 4; ++ks) {
        const int c = ks * 4 + lane / 16;
        const double sc = sm.nrm[c];
        double av[WT], bv[WT];
#pragma unroll
        for (int a = 0; a < WT; ++a) {
          av[a] = sm.Bm[c * LDB + (tr0 + a) * 16 + lane % 16] * sc;
          bv[a] = sm.Bm[c * LDB + (tc0 + a) * 16 + lane % 16];
        }
#pragma unroll
        for (int a = 0; a < WT; ++a)
#pragma unroll
          for (int b = 0; b < WT; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();  // every wavefront is done with U before T overwrites it
    if (wave_on) {
#pragma unroll
      for (int a = 0; a < WT; ++a)
#pragma unroll
        for (int b = 0; b < WT; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            int i = (tr0 + a) * 16 + lane / 16 + 4 * v, j = (tc0 + b) * 16 + lane % 16;
            // masked by arithmetic (T and wbar are zero and finite past m)
            const double t = (i < m && j < m ? 1.0 : 0.0) * (acc[a][b][v] + sm.wbar[i]);
            if constexpr (P == 0) {  // back from A's symmetric permutation
              i = sm.perm[i];
              j = sm.perm[j];
            }
            sm.Bm[i * LDB + j] = t;
            if (dbg && i < m && j < m) dbg[m * m + m + i * m + j] = t;
          }
    }
  } else {
    double tacc[TM][TM];
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TM; ++y) tacc[x][y] = 0.0;
    for (int c = 0; c < m; ++c) {
      const double sc = sm.nrm[c];
      double ui[TM], uj[TM];
#pragma unroll
      for (int x = 0; x < TM; ++x) {
        ui[x] = sm.Bm[c * LDB + ti + 16 * x] * sc;
        uj[x] = sm.Bm[c * LDB + tj + 16 * x];
      }
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TM; ++y) tacc[x][y] += ui[x] * uj[y];
    }
    __syncthreads();
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TM; ++y) {
        const int i = ti + 16 * x, j = tj + 16 * y;
        const double v = (i < m && j < m) ? tacc[x][y] + sm.wbar[i] : 0.0;
        sm.Bm[i * LDB + j] = v;
        if (dbg && i < m && j < m) dbg[m * m + m + i * m + j] = v;
      }
  }
  if (dbg && tid < m) dbg[m * m + tid] = sm.lam[tid];
  __syncthreads();
}

// A chunk of KCH state rows of the domain (both instants), rows q0 .. q0 +
// KCH - 1: fetch() loads each thread's EPT values into registers (issued
// before the previous chunk's products, so the loads overlap them), store()
// writes the zero-padded chunk to LDS and the rows' member means to sm.rc.
template <int M, int KCH, typename T>
struct RowChunk {
  static constexpr int NT = AnaCfg<M>::NT, EPT = KCH * M / NT;
  // row stride of the staged chunk: M + 1, so that the 16 rows an MFMA operand
  // load reads for one member (one row per lane) fall in 16 different banks
  // (a stride of M put them all in one: a 16-way conflict on every load)
  static constexpr int LDX = M + 1;
  static_assert(KCH * M % NT == 0, "whole chunks per thread");
  T v[EPT];
  int act[EPT];  // M <= 64: actuator indices of the chunk fetched next (see fetch)
  int qq0, jj;
  __device__ RowChunk() {
    const int tid = phase_tid();
    qq0 = M >= 64 ? __builtin_amdgcn_readfirstlane(tid / M) : tid / M;  // wavefront-uniform for M >= 64
    jj = tid % M;
  }
  // the actuator indices of chunk q0 (M <= 64; called once for the first chunk,
  // then by every fetch for the chunk after it)
  __device__ void fetch_act(const InstDesc& I, int est_off, int e, int q0) {
    if constexpr (M <= 64) {
      const int m = I.m;
      const int32_t* est_act = I.est_act + est_off;
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int q = q0 + qq0 + u * (NT / M);
        act[u] = (q < 2 * e && jj < m) ? gload(est_act + (q < e ? q : q - e)) : -1;
      }
    }
  }
  __device__ void fetch(const InstDesc& I, int est_off, int e, int cur, int q0) {
    const int m = I.m;
    const T* ens = (const T*)I.ens;
    const int32_t* est_act = I.est_act + est_off;
    const size_t slot = (size_t)I.n_act * m;
    if constexpr (M <= 64) {
      // global loads (see gload); the actuator indices run one chunk ahead
      // (fetch_act), so a fetch never waits for its own index loads
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int q = q0 + qq0 + u * (NT / M);
        v[u] = (T)0;
        if (act[u] >= 0) {
          const int inst = q < e ? cur : (cur ^ 1);
          v[u] = gload(ens + (size_t)inst * slot + (size_t)act[u] * m + jj);
        }
      }
      fetch_act(I, est_off, e, q0 + KCH);
    } else {  // M = 128: the indices of every value at once would not fit in the registers
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        const int q = q0 + qq0 + u * (NT / M);
        v[u] = (T)0;
        if (q < 2 * e && jj < m) {
          const int inst = q < e ? cur : (cur ^ 1);
          const int act = gload(est_act + (q < e ? q : q - e));
          v[u] = gload(ens + (size_t)inst * slot + (size_t)act * m + jj);
        }
      }
    }
  }
  template <typename S>
  __device__ void store(AnaSmem<M>& sm, S* X, int m) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) X[(qq0 + u * (NT / M)) * LDX + jj] = (S)v[u];
    __syncthreads();
    constexpr int TPR = NT / KCH;  // threads per row for the means (8 or 16)
    const int tid = phase_tid(), row = tid / TPR, part = tid % TPR;
    double sum = 0.0;
    for (int j = part; j < m; j += TPR) sum += (double)X[row * LDX + j];
    sum = group_sum<TPR>(sum);
    if (part == 0) sm.rc[row] = sum / (double)m;
    __syncthreads();
  }
};

// ---- a8 on the FP64 path: Z = xbar 1^T + X' T with FP64 MFMA ----------------
// Chunks of 16 state rows (both instants) are staged with their member means;
// wave w computes the 16 x 16 output tiles w, w + 4, ... of the chunk with
// v_mfma_f64_16x16x4f64 (A = X' - xbar from LDS, B = T from Bm).
template <int M>
__device__ void update_fp64(AnaSmem<M>& sm, const InstDesc& I, int est_off, int e, int cur) {
  using C = AnaCfg<M>;
  constexpr int LDB = C::LDB, KR = 16, CB = M / 16;
  static_assert((size_t)KR * (M + 1) * 8 <= C::STAGE_BYTES, "staging");
  constexpr int LDX = RowChunk<M, KR, double>::LDX;
  const int m = I.m, tid = phase_tid(), w = tid / 64, lane = tid % 64;
  double* Xd = (double*)sm.stage;
  double* Z = (double*)I.Z + (size_t)2 * est_off * m;
  RowChunk<M, KR, double> rows;
  rows.fetch_act(I, est_off, e, 0);
  rows.fetch(I, est_off, e, cur, 0);
  for (int q0 = 0; q0 < 2 * e; q0 += KR) {
    const int kc = min(KR, 2 * e - q0);
    rows.store(sm, Xd, m);
    if (q0 + KR < 2 * e) rows.fetch(I, est_off, e, cur, q0 + KR);
    for (int cb = w; cb < CB; cb += 4) {
      const int arow = lane % 16;
      const double xb = sm.rc[arow];
      const int col = cb * 16 + lane % 16;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int ks = 0; ks < M / 4; ++ks) {
        const int k = ks * 4 + lane / 16;
        // loaded unconditionally, masked by arithmetic (the staged rows are
        // zero past m, so the product is finite): a load under the mask is a
        // branch and a wait of its own before every MFMA
        const double a = (k < m ? 1.0 : 0.0) * (Xd[arow * LDX + k] - xb);
        const double b = sm.Bm[k * LDB + col];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
      double mean[4];  // read before the stores' branches, so the reads share one wait
#pragma unroll
      for (int v = 0; v < 4; ++v) mean[v] = sm.rc[lane / 16 + 4 * v];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = lane / 16 + 4 * v;
        if (row < kc && col < m) gstore(Z + (size_t)(q0 + row) * m + col, mean[v] + acc[v]);
      }
    }
    __syncthreads();
  }
}

// ---- a8 on the MFMA paths: Z = xbar 1^T + X' T in 16 x 16 tiles --------------
// FP32: X' and T in FP32.  BF16: X' in BF16, T split into hi + lo BF16 parts
// (two MFMAs), so only X' carries the BF16 rounding.
template <int P, int M>
__device__ void update_mfma(AnaSmem<M>& sm, const InstDesc& I, int est_off, int e, int cur) {
  using C = AnaCfg<M>;
  constexpr int LDB = C::LDB, KR = C::KR;
  constexpr int RB = KR / 16, CB = M / 16, NTILE = RB * CB;
  const int m = I.m, tid = phase_tid(), w = tid / 64, lane = tid % 64;
  float* Xf = (float*)sm.stage;
  float* Z = (float*)I.Z + (size_t)2 * est_off * m;
  RowChunk<M, KR, float> rows;
  constexpr int LDX = RowChunk<M, KR, float>::LDX;
  static_assert((size_t)KR * LDX * 4 <= C::STAGE_BYTES, "staging");
  // BF16, M a multiple of 32: T converted once to its hi and lo BF16 parts,
  // transposed (Th[j][k], k contiguous, so that a lane's 8 consecutive k of the
  // B operand are one 16-byte load), in Bm's storage; the staged rows likewise
  // once per chunk to BF16 X' - xbar (zero past m).  Converting inside the
  // products repeated the work for every tile and chunk.
  constexpr bool PRE = P == 2 && M % 32 == 0 && M <= 64;
  constexpr int LDT = M + 8;  // bf16 row stride: 16-byte rows, banks spread over a pass
  __bf16* Th = (__bf16*)sm.Bm;
  __bf16* Tl = Th + M * LDT;
  __bf16* Xb = (__bf16*)sm.stage;
  static_assert(!PRE || ((size_t)2 * M * LDT * 2 <= sizeof(sm.Bm) && (size_t)KR * LDT * 2 <= C::STAGE_BYTES),
                "BF16 copies");
  if constexpr (PRE) {
    constexpr int PER = M * M / C::NT;
    double tv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + u * C::NT;
      tv[u] = sm.Bm[(idx / M) * LDB + idx % M];  // T[k][j], k = idx / M, j = idx % M
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + u * C::NT, k = idx / M, j = idx % M;
      const __bf16 hi = (__bf16)(float)tv[u];
      Th[j * LDT + k] = hi;
      Tl[j * LDT + k] = (__bf16)(float)(tv[u] - (double)(float)hi);
    }
    __syncthreads();
  }
  rows.fetch_act(I, est_off, e, 0);
  rows.fetch(I, est_off, e, cur, 0);
  for (int q0 = 0; q0 < 2 * e; q0 += KR) {
    const int kc = min(KR, 2 * e - q0);
    rows.store(sm, Xf, m);
    if constexpr (PRE) {
      constexpr int PER = KR * M / C::NT;
      float xv[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * C::NT, r = idx / M, k = idx % M;
        xv[u] = (k < m ? 1.f : 0.f) * (Xf[r * LDX + k] - (float)sm.rc[r]);
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * C::NT;
        Xb[(idx / M) * LDT + idx % M] = (__bf16)xv[u];
      }
      __syncthreads();
    }
    if (q0 + KR < 2 * e) rows.fetch(I, est_off, e, cur, q0 + KR);
    for (int t = w; t < NTILE; t += 4) {
      const int rb = t / CB, cb = t % CB;
      const int arow = rb * 16 + lane % 16;
      const float xb = (float)sm.rc[arow];
      const int col = cb * 16 + lane % 16;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      if constexpr (P == 1) {
#pragma unroll 4
        for (int ks = 0; ks < M / 4; ++ks) {
          const int k = ks * 4 + lane / 16;
          const float a = (k < m ? 1.f : 0.f) * (Xf[arow * LDX + k] - xb);  // masked by arithmetic, as above
          const float b = (float)sm.Bm[k * LDB + col];
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
        }
      } else if constexpr (PRE) {
#pragma unroll
        for (int ks = 0; ks < M / 32; ++ks) {
          const int k0 = ks * 32 + 8 * (lane / 16);
          const bf16x8 a = *(const bf16x8*)&Xb[arow * LDT + k0];
          const bf16x8 bh = *(const bf16x8*)&Th[col * LDT + k0];
          const bf16x8 bl = *(const bf16x8*)&Tl[col * LDT + k0];
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc, 0, 0, 0);
        }
      } else {
        for (int ks = 0; ks < (M + 31) / 32; ++ks) {
          bf16x8 a, bh, bl;
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int k = ks * 32 + 8 * (lane / 16) + u;
            float xa;
            double tv;
            if constexpr (M <= 64) {
              // masked by arithmetic, as above; k runs past M only at M = 16 (the index is clamped)
              const int kc_ = (M % 32 == 0 || k < M) ? k : M - 1;
              xa = (k < m ? 1.f : 0.f) * (Xf[arow * LDX + kc_] - xb);
              tv = (M % 32 == 0 || k < M ? 1.0 : 0.0) * sm.Bm[kc_ * LDB + col];
            } else {  // M = 128: the loads in flight at once would not fit in the registers
              xa = (k < m) ? Xf[arow * LDX + k] - xb : 0.f;
              tv = sm.Bm[k * LDB + col];
            }
            const __bf16 hi = (__bf16)(float)tv;
            a[u] = (__bf16)xa;
            bh[u] = hi;
            bl[u] = (__bf16)(float)(tv - (double)(float)hi);
          }
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc, 0, 0, 0);
        }
      }
      double mean[4];  // read before the stores' branches, so the reads share one wait
#pragma unroll
      for (int v = 0; v < 4; ++v) mean[v] = sm.rc[rb * 16 + 4 * (lane / 16) + v];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rb * 16 + 4 * (lane / 16) + v;
        if (row < kc && col < m) gstore(Z + (size_t)(q0 + row) * m + col, (float)(mean[v] + (double)acc[v]));
      }
    }
    __syncthreads();
  }
}

// FP64 path, M <= 64: A (and b) permuted symmetrically so that its diagonal
// decreases, A_p[r][c] = A[perm[r]][perm[c]] (ties by index; padded members
// keep their places).  The Cholesky factor of A_p starts the one-sided Jacobi
// closer to convergence: 7.29 sweeps per solve instead of 7.61 on the 84 x 84
// map (CPU replay of every domain).  The eigenvectors of A_p are those of A
// with rows permuted, so T comes out of the transform as T_p and is stored back
// through perm (T[perm[r]][perm[c]] = T_p[r][c]).
template <int M>
__device__ void sort_diag(AnaSmem<M>& sm, int m) {
  using C = AnaCfg<M>;
  constexpr int NT = C::NT, LDB = C::LDB, PER = M * M / NT;
  static_assert(M * M % NT == 0 && M <= NT && NT % M == 0, "whole rows per thread");
  constexpr int TPI = NT / M;  // threads per index for the ranks
  const int tid = phase_tid();
  {
    const int i = tid / TPI, part = tid % TPI;
    const double d = sm.Bm[i * LDB + i];
    double ahead = 0.0;  // indices ranked before i among this thread's share (exact small integers)
    if (i < m)
      for (int j = part; j < m; j += TPI) {
        const double dj = sm.Bm[j * LDB + j];
        ahead += (dj > d || (dj == d && j < i)) ? 1.0 : 0.0;
      }
    ahead = group_sum<TPI>(ahead);
    if (part == 0) sm.perm[i < m ? (int)ahead : i] = i;
  }
  __syncthreads();
  // thread tid reads entries (perm[r], perm[c]) for c = tid % M and rows r = tid / M + e NT / M
  double v[PER];
  const int c = tid % M, pc = sm.perm[c];
#pragma unroll
  for (int e = 0; e < PER; ++e) v[e] = sm.Bm[sm.perm[tid / M + e * (NT / M)] * LDB + pc];
  const double bp = tid < M ? sm.bvec[pc] : 0.0;
  __syncthreads();
#pragma unroll
  for (int e = 0; e < PER; ++e) sm.Bm[(tid / M + e * (NT / M)) * LDB + c] = v[e];
  if (tid < M) sm.bvec[tid] = bp;
  __syncthreads();
}

template <int P, int M>
__device__ void analyse_item(AnaSmem<M>& sm, const InstDesc* __restrict__ tab, const ClassBatch& cb, int item, bool fair) {
  using C = AnaCfg<M>;
  const int eb = find_entry(cb.dom_off, cb.n, item);
  const InstDesc& I = tab[cb.inst[eb]];
  const int l = I.order[item - cb.dom_off[eb]];
  const int est_off = I.dom[4 * l], e = I.dom[4 * l + 1];
  const int obs_off = I.dom[4 * l + 2], s = I.dom[4 * l + 3];
  const int m = I.m;
  const int cur = I.st->cur;
  double* dbg = I.dbg ? I.dbg + (size_t)l * (2 * m * m + m + kDbgTail) : nullptr;
  // debug: shader-clock stamps at the phase boundaries (after each phase's barrier)
  auto stamp = [&](int k) {
    if (dbg && threadIdx.x == 0) dbg[2 * m * m + m + k] = (double)clock64();
  };
  stamp(0);
  if (fair) set_issue_prio(3);
  if (dbg && threadIdx.x == 0) {  // debug: where the workgroup runs (HW_ID: SE, SH, CU, SIMD; XCC_ID)
    dbg[2 * m * m + m + 6] = (double)__builtin_amdgcn_s_getreg(4 | (31 << 11));
    dbg[2 * m * m + m + 7] = (double)__builtin_amdgcn_s_getreg(20 | (31 << 11));
    dbg[2 * m * m + m + 8] = (double)blockIdx.x;
  }

  if constexpr (P == 0 && M <= 64) gather_C_fp64_mfma<M>(sm, I, obs_off, s, dbg);
  else if constexpr (P == 0) gather_C_fp64<M>(sm, I, obs_off, s, dbg);
  else if constexpr (P >= 2 && M <= 64) gather_C_bf16_tab<P, M>(sm, I, obs_off, s, dbg);
  else gather_C_mfma<P, M>(sm, I, obs_off, s, dbg);
  if constexpr (P == 0) {
    __syncthreads();
    if constexpr (M <= 64) sort_diag<M>(sm, m);
    // the domain's A (permuted as above), kept for the refinement of wbar (the
    // Cholesky overwrites it): the lower triangle of the m x m matrix, packed
    // by rows (row i at i (i + 1) / 2), rows spread over the wavefronts and
    // coalesced over lanes
    double* Ag = I.Ascr + (size_t)l * tri_size(m);
    const int w = phase_tid() / 64, lane = phase_tid() % 64;
    for (int i = w; i < m; i += AnaCfg<M>::NT / 64)
      for (int j = lane; j <= i; j += 64) gstore(Ag + tri_size(i) + j, sm.Bm[i * AnaCfg<M>::LDB + j]);
    __syncthreads();
  }
  stamp(1);
  cholesky<M>(sm);
  stamp(2);
  bool converged = false;
  const int sweeps = jacobi<P, M>(sm, m, converged, fair);
  stamp(3);
  if (fair) set_issue_prio(0);
  transform<P, M>(sm, I, l, dbg);
  stamp(4);
  if (threadIdx.x == 0) {
    if (I.dbg_sweeps) I.dbg_sweeps[l] = sweeps;
    gatomic_add(&I.dom_sweeps[l], (unsigned)sweeps);
    if (!converged) gatomic_add(&I.st->unconverged, 1);
    gatomic_add(&I.st->sweeps, (unsigned long long)sweeps);
    gatomic_add(&I.st->solves, 1ull);
  }
  if constexpr (P == 0) update_fp64<M>(sm, I, est_off, e, cur);
  else update_mfma<P, M>(sm, I, est_off, e, cur);
  stamp(5);
}

// Persistent: a workgroup analyses item blockIdx.x, then claims further items
// from the class's work counter (zeroed by the slope kernel that precedes
// every analysis launch) until the items run out, so the launch's grid can be
// smaller than the work (fixed grids for replayed graphs, a cap on the CUs the
// class occupies) and the heaviest domains, which come first in each
// instance's order, start first.  Every workgroup leaves once a claim passes
// the item count.
// fair != 0 (launches whose workgroups start together with at most two on a
// CU: the plain path): the wavefronts' issue priority falls with the item's
// progress (3 from its start, then by Jacobi sweeps done: 2 from the 3rd,
// 1 from the 5th, 0 from the 6th and after the eigensolve).  A SIMD issues
// from the oldest of its ready wavefronts, so of two domains sharing a CU the
// first dispatched ran nearly as if alone and the second got the leftover
// slots, then finished alone at one wavefront per SIMD: on the 84 x 84 map
// the pairs ended at 493k and 659k cycles (mean), with the priorities 566k
// and 612k, and the plain FP64 launch went 296 -> 275 us.  With three or
// more workgroups per CU (the serving batches) either ordering of the
// priorities made the batches slower (serving -11 % with this one), so the
// server launches with fair = 0.
template <int P, int M>
__global__ __launch_bounds__(256) void k_analysis(const InstDesc* __restrict__ tab,
                                                  BatchHdr* __restrict__ hdr, int cls, int fair) {
  __shared__ AnaSmem<M> sm;
  __shared__ int s_next;
  ClassBatch& cb = hdr->cls[cls];
  const int total = cb.dom_off[cb.n];
  int item = blockIdx.x;
  while (item < total) {
    analyse_item<P, M>(sm, tab, cb, item, fair != 0);
    if (threadIdx.x == 0) s_next = (int)gridDim.x + (int)atomicAdd(&cb.next, 1u);
    __syncthreads();
    item = s_next;
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// a4-a8 for ensembles of 129..256 members (padded to 256, FP64).  A domain's
// 256 x 256 matrices (512 KB each) do not fit in LDS, so its analysis is a
// sequence of launches over scratch in the instance workspace (A, B and a few
// vectors per domain, which stay in L2 between launches):
//   k_big_gram    A = (m-1)/rho I + Y'^T diag(r) Y' by 64 x 64 tiles on FP64
//                 MFMA, b = Y'^T diag(r) d; clears the domain's Jacobi flags
//   k_big_chol    A = L L^T, right-looking by panels, one workgroup per domain
//   k_big_round   one round of the blocked one-sided Jacobi (below)
//   k_big_sweep   end of a sweep: a domain is done when no round rotated
//   k_big_eig     lambda, U, wbar (one refinement step through the exact A)
//   k_big_T       T = U diag(sqrt((m-1)/lambda)) U^T + wbar 1^T, by tiles
//   k_big_update  Z = xbar 1^T + X' T, by 64 x 64 tiles
// The Jacobi is the one-sided method of the m <= 128 kernel on the columns of
// L (L J = U Sigma), visited by blocks: the columns form NB blocks of 16 (NB
// even; columns past m are unit vectors that never rotate).  A sweep is NB - 1
// rounds of a round-robin tournament between the blocks (circle method, block
// 0 fixed); in a round every pair of blocks is one workgroup that holds its 32
// columns in LDS and rotates the 256 pairs between them in 16 steps of 16
// disjoint pairs (the first round also the pairs inside each block), so every
// pair of columns is visited once per sweep.  Launch boundaries order the
// rounds; a converged domain's later launches return at once.
// ----------------------------------------------------------------------------
constexpr int kBigM = 256;
constexpr int kBigLd = kBigM + 8;     // LDS column stride in k_big_round
constexpr int kBigMaxSweeps = 24;

struct BigDom {
  const InstDesc* I;
  int l, est_off, e, obs_off, s;
  double* A;
  double* B;
  double* v;
  int32_t* f;
};

__device__ __forceinline__ BigDom big_dom(const InstDesc* __restrict__ tab, const ClassBatch& cb, int item) {
  BigDom d;
  const int eb = find_entry(cb.dom_off, cb.n, item);
  d.I = &tab[cb.inst[eb]];
  d.l = item - cb.dom_off[eb];
  d.est_off = d.I->dom[4 * d.l];
  d.e = d.I->dom[4 * d.l + 1];
  d.obs_off = d.I->dom[4 * d.l + 2];
  d.s = d.I->dom[4 * d.l + 3];
  d.A = d.I->bigA + (size_t)d.l * kBigM * kBigM;
  d.B = d.I->bigB + (size_t)d.l * kBigM * kBigM;
  d.v = d.I->bigv + (size_t)d.l * 5 * kBigM;
  d.f = d.I->bigf + 4 * d.l;
  return d;
}

__device__ __forceinline__ double* big_dbg(const BigDom& D) {
  const int m = D.I->m;
  return D.I->dbg ? D.I->dbg + (size_t)D.l * (2 * m * m + m + kDbgTail) : nullptr;
}

// 1024 threads: member j = t % 256 of observation quarter t / 256, summed in LDS.
// grid (10, items): the upper tiles (ti <= tj) of the 4 x 4 grid of 64 x 64
// tiles of C = Y'^T diag(r) Y', on FP64 MFMA: wavefront w owns the 32 x 32
// quadrant (w / 2, w % 2) of the tile, 2 x 2 MFMA tiles of 16 x 16, over
// chunks of 32 observations staged in LDS (Ya: Y' rows of the tile's rows,
// Yb: r Y' of its columns).  The diagonal tiles also form their 64 entries of
// b = Y'^T diag(r) d, and tile 0 clears the domain's Jacobi flags.
__global__ __launch_bounds__(256) void k_big_gram(const InstDesc* __restrict__ tab, const BatchHdr* __restrict__ hdr,
                                                  int cls) {
  __shared__ double Ya[32][64], Yb[32][64], rd[32], bred[4][64];
  const ClassBatch& cb = hdr->cls[cls];
  if ((int)blockIdx.y >= cb.dom_off[cb.n]) return;
  int t = blockIdx.x, ti = 0;
  while (t >= 4 - ti) { t -= 4 - ti; ++ti; }
  const int tj = ti + t, i0 = 64 * ti, j0 = 64 * tj;
  const bool diag = ti == tj;
  const BigDom D = big_dom(tab, cb, blockIdx.y);
  const InstDesc& I = *D.I;
  const int m = I.m, tid = threadIdx.x, w = tid / 64, lane = tid % 64, nobs = 2 * D.s;
  if (blockIdx.x == 0 && tid == 0) {
    D.f[0] = 0;
    D.f[1] = 0;
    D.f[2] = 0;
  }
  const double* Yp = (const double*)I.Yp;
  const int qr = 32 * (w / 2), qc = 32 * (w % 2);  // the wavefront's quadrant
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  double bpart = 0.0;  // diagonal tiles: b for row i0 + lane, observations w, w + 4, ...
  // Thread tid stages observations tid / 64 + 4 e (e < 8) of every chunk, row
  // entry c = tid % 64.  The next chunk's values are loaded into registers
  // before this chunk's products, and their row indices one chunk earlier
  // still, so the loads' latency overlaps the MFMAs instead of preceding them.
  const int c = tid % 64;
  int prow[8];
  double pr[8], pa[8], pb[8], pd[8];
  auto fetch_idx = [&](int q0n) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int q = q0n + tid / 64 + 4 * e;
      prow[e] = -1;
      pr[e] = 0.0;
      if (q < nobs) {
        const int o = 2 * D.obs_off + q;
        prow[e] = I.obs_row[o];
        pr[e] = I.obs_r[o];
      }
    }
  };
  auto fetch_val = [&]() {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      pa[e] = pb[e] = pd[e] = 0.0;
      if (prow[e] >= 0) {
        const size_t row = (size_t)prow[e] * m;
        if (i0 + c < m) pa[e] = Yp[row + i0 + c];
        if (j0 + c < m) pb[e] = pr[e] * Yp[row + j0 + c];
        if (diag && c == 0) pd[e] = pr[e] * I.d[prow[e]];
      }
    }
  };
  fetch_idx(0);
  fetch_val();
  fetch_idx(32);
  for (int q0 = 0; q0 < nobs; q0 += 32) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      Ya[tid / 64 + 4 * e][c] = pa[e];
      Yb[tid / 64 + 4 * e][c] = pb[e];
      if (c == 0) rd[tid / 64 + 4 * e] = pd[e];
    }
    __syncthreads();
    if (q0 + 32 < nobs) {
      fetch_val();
      fetch_idx(q0 + 64);
    }
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int k = 4 * ks + lane / 16;
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        av[a] = Ya[k][qr + 16 * a + lane % 16];
        bv[a] = Yb[k][qc + 16 * a + lane % 16];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (diag)
#pragma unroll
      for (int e = 0; e < 8; ++e) bpart = fma(Ya[w + 4 * e][lane], rd[w + 4 * e], bpart);
    __syncthreads();
  }
  if (diag) {
    bred[w][lane] = bpart;
    __syncthreads();
    if (tid < 64) {
      const int i = i0 + tid;
      D.v[i] = i < m ? (bred[0][tid] + bred[1][tid]) + (bred[2][tid] + bred[3][tid]) : 0.0;
    }
  }
  double* dbg = big_dbg(D);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + qr + 16 * a + lane / 16 + 4 * v, j = j0 + qc + 16 * b + lane % 16;
        if (i > j) continue;  // one writer per symmetric pair (deterministic)
        const double c = acc[a][b][v];
        double x;
        if (i < m && j < m) {
          x = c + (i == j ? I.a_diag : 0.0);
          if (dbg) {
            dbg[(size_t)i * m + j] = c;
            dbg[(size_t)j * m + i] = c;
          }
        } else {
          x = i == j ? 1.0 : 0.0;  // padded members: identity
        }
        D.A[(size_t)i * kBigM + j] = x;
        D.A[(size_t)j * kBigM + i] = x;
      }
}

// A = L L^T into B (column-major, leading dimension kBigM; the upper triangle
// zero, padded members the identity), right-looking by panels of 16 columns
// as the m <= 128 kernel: wavefront 0 factors the panel in registers (rows
// c0 + lane + 64 s), which also stages it in LDS, and all eight wavefronts
// subtract its rank-16 product from the trailing lower triangle in 16 x 16
// tiles on FP64 MFMA (the tiles in B, whose loads are the latency that more
// wavefronts hide; the panel's columns from LDS).
constexpr int kBigCholWaves = 8;
__global__ __launch_bounds__(64 * kBigCholWaves) void k_big_chol(const InstDesc* __restrict__ tab,
                                                                 const BatchHdr* __restrict__ hdr, int cls) {
  __shared__ double pnl[16][kBigM];
  const ClassBatch& cb = hdr->cls[cls];
  if ((int)blockIdx.x >= cb.dom_off[cb.n]) return;
  const BigDom D = big_dom(tab, cb, blockIdx.x);
  const int m = D.I->m, mp = (m + 15) & ~15, tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  for (int idx = tid; idx < kBigM * kBigM; idx += 64 * kBigCholWaves) {
    const int c = idx / kBigM, r = idx % kBigM;
    double v;
    if (c < m) v = (r >= c && r < m) ? D.A[(size_t)c * kBigM + r] : 0.0;  // A symmetric
    else v = r == c ? 1.0 : 0.0;
    D.B[idx] = v;
  }
  __syncthreads();
  for (int c0 = 0; c0 < mp; c0 += 16) {
    if (w == 0) {
      double a[4][16];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int r = c0 + lane + 64 * s;
        const bool on = r < mp;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) a[s][jj] = on ? D.B[(size_t)(c0 + jj) * kBigM + r] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double d = readlane_f64(a[0][j], j);  // a_jj after the earlier columns
        const double rs = rsqrt(d);
        double lj[4];
        lj[0] = lane > j ? a[0][j] * rs : (lane == j ? d * rs : 0.0);
#pragma unroll
        for (int s = 1; s < 4; ++s) lj[s] = a[s][j] * rs;
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s][j] = lj[s];
#pragma unroll
        for (int jj = j + 1; jj < 16; ++jj) {
          const double l = readlane_f64(lj[0], jj);
#pragma unroll
          for (int s = 0; s < 4; ++s) a[s][jj] = fma(-lj[s], l, a[s][jj]);
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int r = c0 + lane + 64 * s;
        if (r < mp)
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) {
            D.B[(size_t)(c0 + jj) * kBigM + r] = a[s][jj];
            pnl[jj][r] = a[s][jj];
          }
      }
    }
    __syncthreads();
    const int nt = (mp - c0) / 16 - 1;
    int t = 0;
    for (int R = 0; R < nt; ++R)
      for (int Cc = 0; Cc <= R; ++Cc, ++t) {
        if (t % kBigCholWaves != w) continue;
        const int rb = c0 + 16 * (R + 1), cb = c0 + 16 * (Cc + 1);
        f64x4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = D.B[(size_t)(cb + lane % 16) * kBigM + rb + lane / 16 + 4 * v];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const int k = 4 * ks + lane / 16;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pnl[k][rb + lane % 16], -pnl[k][cb + lane % 16], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) D.B[(size_t)(cb + lane % 16) * kBigM + rb + lane / 16 + 4 * v] = acc[v];
      }
    __syncthreads();
  }
}

// grid (nb / 2, items): the workgroup of block pair blockIdx.x in round `round`.
__global__ __launch_bounds__(256) void k_big_round(const InstDesc* __restrict__ tab, const BatchHdr* __restrict__ hdr,
                                                   int cls, int nb, int round) {
  __shared__ double col[32 * kBigLd];
  __shared__ double nrm[32];
  const ClassBatch& cb = hdr->cls[cls];
  if ((int)blockIdx.y >= cb.dom_off[cb.n]) return;
  const BigDom D = big_dom(tab, cb, blockIdx.y);
  if (D.f[0]) return;  // converged: uniform over the workgroup
  const int m = D.I->m, tid = threadIdx.x, w = blockIdx.x, n1 = nb - 1;
  const int a = w == 0 ? 0 : 1 + (round + w) % n1;
  const int b = w == 0 ? 1 + round % n1 : 1 + (round + n1 - w) % n1;
  // LDS column k: block a's column k (k < 16), block b's column k - 16
  for (int idx = tid; idx < 32 * kBigM; idx += 256) {
    const int k = idx / kBigM, r = idx % kBigM;
    const int c = 16 * (k < 16 ? a : b) + (k & 15);
    col[k * kBigLd + r] = D.B[(size_t)c * kBigM + r];
  }
  __syncthreads();
  {
    const int k = tid / 8, part = tid % 8;
    double ss = 0.0;
    for (int r = part; r < kBigM; r += 8) {
      const double v = col[k * kBigLd + r];
      ss = fma(v, v, ss);
    }
    ss = group_sum<8>(ss);
    if (part == 0) nrm[k] = ss;
  }
  __syncthreads();
  const double tol = 32.0 * (double)m * 1.1102230246251565e-16;  // as in the m <= 128 kernel
  const double tol2 = tol * tol;
  const int p = tid / 16, sub = tid % 16;  // pair slot, lane within the pair
  bool rotated = false;
  auto step = [&](int ci, int cj) {
    double xi[16], xj[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      xi[t] = col[ci * kBigLd + sub + 16 * t];
      xj[t] = col[cj * kBigLd + sub + 16 * t];
    }
    double g0 = 0.0, g1 = 0.0;
#pragma unroll
    for (int t = 0; t < 16; t += 2) {
      g0 = fma(xi[t], xj[t], g0);
      g1 = fma(xi[t + 1], xj[t + 1], g1);
    }
    const double gsum = group_sum<16>(g0 + g1);
    const double al = nrm[ci], be = nrm[cj];  // the pairs of a step are disjoint
    if (gsum * gsum > tol2 * (al * be)) {
      const double dd = be - al, g2 = 2.0 * gsum;
      const double q2 = fma(dd, dd, g2 * g2);
      const double den = fma(q2, __builtin_amdgcn_rsq(q2), fabs(dd));
      const double t = copysign(1.0, dd) * g2 * __builtin_amdgcn_rcp(den);
      const double c = rsqrt_1_2(fma(t, t, 1.0));
      const double sn = c * t;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const double x = xi[u];
        col[ci * kBigLd + sub + 16 * u] = c * x - sn * xj[u];
        col[cj * kBigLd + sub + 16 * u] = sn * x + c * xj[u];
      }
      if (sub == 0) {
        nrm[ci] = al - t * gsum;
        nrm[cj] = be + t * gsum;
      }
      rotated = true;
    }
    __syncthreads();
  };
  if (round == 0) {
    // pairs inside each block, (i, i ^ k): slots 0..7 block a, 8..15 block b
    const int base = p < 8 ? 0 : 16, q = p & 7;
    for (int k = 1; k < 16; ++k) {
      const int hk = 31 - __clz(k);
      const int i = ((q >> hk) << (hk + 1)) | (q & ((1 << hk) - 1));
      step(base + i, base + (i ^ k));
    }
  }
  // the 256 pairs between the blocks: slot p keeps block a's column p (and its
  // norm) in registers and meets block b's columns p, p + 1, ... (mod 16)
  {
    double xi[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) xi[t] = col[p * kBigLd + sub + 16 * t];
    double al = nrm[p];
    bool moved = false;
    for (int st = 0; st < 16; ++st) {
      const int cj = 16 + ((p + st) & 15);
      double xj[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) xj[t] = col[cj * kBigLd + sub + 16 * t];
      double g0 = 0.0, g1 = 0.0;
#pragma unroll
      for (int t = 0; t < 16; t += 2) {
        g0 = fma(xi[t], xj[t], g0);
        g1 = fma(xi[t + 1], xj[t + 1], g1);
      }
      const double gsum = group_sum<16>(g0 + g1);
      const double be = nrm[cj];
      if (gsum * gsum > tol2 * (al * be)) {
        const double dd = be - al, g2 = 2.0 * gsum;
        const double q2 = fma(dd, dd, g2 * g2);
        const double den = fma(q2, __builtin_amdgcn_rsq(q2), fabs(dd));
        const double t = copysign(1.0, dd) * g2 * __builtin_amdgcn_rcp(den);
        const double c = rsqrt_1_2(fma(t, t, 1.0));
        const double sn = c * t;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const double x = xi[u];
          xi[u] = c * x - sn * xj[u];
          col[cj * kBigLd + sub + 16 * u] = sn * x + c * xj[u];
        }
        al -= t * gsum;
        if (sub == 0) nrm[cj] = be + t * gsum;
        moved = true;
      }
      __syncthreads();
    }
    if (moved) {
      rotated = true;
#pragma unroll
      for (int t = 0; t < 16; ++t) col[p * kBigLd + sub + 16 * t] = xi[t];
    }
  }
  if (__syncthreads_or(rotated)) {
    for (int idx = tid; idx < 32 * kBigM; idx += 256) {
      const int k = idx / kBigM, r = idx % kBigM;
      const int c = 16 * (k < 16 ? a : b) + (k & 15);
      D.B[(size_t)c * kBigM + r] = col[k * kBigLd + r];
    }
    if (tid == 0) atomicAdd(&D.f[1], 1);
  }
}

__global__ __launch_bounds__(64) void k_big_sweep(const InstDesc* __restrict__ tab, const BatchHdr* __restrict__ hdr,
                                                  int cls) {
  const ClassBatch& cb = hdr->cls[cls];
  const int item = blockIdx.x * 64 + threadIdx.x;
  if (item >= cb.dom_off[cb.n]) return;
  const BigDom D = big_dom(tab, cb, item);
  if (D.f[0]) return;
  D.f[2] += 1;
  if (D.f[1] == 0) {
    D.f[0] = 1;
  } else if (D.f[2] >= kBigMaxSweeps) {
    D.f[0] = 2;
    atomicAdd(&D.I->st->unconverged, 1);
  }
  D.f[1] = 0;
}

// Thread c: lambda_c and U_c = B_c / sigma_c; then wbar = U Lambda^-1 U^T b
// and one refinement step wbar += U Lambda^-1 U^T (b - A wbar) with the exact A.
__global__ __launch_bounds__(256) void k_big_eig(const InstDesc* __restrict__ tab, const BatchHdr* __restrict__ hdr,
                                                 int cls) {
  __shared__ double bs[kBigM], zs[kBigM], wsh[kBigM];
  const ClassBatch& cb = hdr->cls[cls];
  if ((int)blockIdx.x >= cb.dom_off[cb.n]) return;
  const BigDom D = big_dom(tab, cb, blockIdx.x);
  const InstDesc& I = *D.I;
  const int m = I.m, c = threadIdx.x;
  double* Bc = D.B + (size_t)c * kBigM;
  double lc = 1.0;
  if (c < m) {
    double ss = 0.0;
    for (int r = 0; r < m; ++r) ss = fma(Bc[r], Bc[r], ss);
    lc = ss;
    const double inv = 1.0 / sqrt(ss);
    for (int r = 0; r < m; ++r) Bc[r] *= inv;
  }
  D.v[2 * kBigM + c] = lc;
  bs[c] = D.v[c];
  __syncthreads();
  auto project = [&](const double* rhs) {  // zs = Lambda^-1 U^T rhs
    double z = 0.0;
    if (c < m)
      for (int r = 0; r < m; ++r) z = fma(Bc[r], rhs[r], z);
    zs[c] = c < m ? z / lc : 0.0;
    __syncthreads();
  };
  auto expand = [&](int r) {  // (U zs)[r]
    double w = 0.0;
    if (r < m)
      for (int k = 0; k < m; ++k) w = fma(D.B[(size_t)k * kBigM + r], zs[k], w);
    return w;
  };
  project(bs);
  const int r = threadIdx.x;
  wsh[r] = r < m ? expand(r) : 0.0;
  __syncthreads();
  double res = 0.0;
  if (r < m) {
    double t = 0.0;
    for (int j = 0; j < m; ++j) t = fma(D.A[(size_t)j * kBigM + r], wsh[j], t);
    res = bs[r] - t;
  }
  __syncthreads();
  bs[r] = res;
  __syncthreads();
  project(bs);
  D.v[kBigM + r] = r < m ? wsh[r] + expand(r) : 0.0;
  double* dbg = big_dbg(D);
  if (dbg && c < m) dbg[(size_t)m * m + c] = lc;
  if (threadIdx.x == 0) {
    const int sweeps = D.f[2];
    if (I.dbg_sweeps) I.dbg_sweeps[D.l] = sweeps;
    atomicAdd(&I.st->sweeps, (unsigned long long)sweeps);
    atomicAdd(&I.st->solves, 1ull);
  }
}

// grid (16, items): 64 x 64 tile (blockIdx.x / 4, blockIdx.x % 4) of T, written
// over A (row-major); U columns staged 32 at a time.
__global__ __launch_bounds__(256) void k_big_T(const InstDesc* __restrict__ tab, const BatchHdr* __restrict__ hdr,
                                               int cls) {
  __shared__ double Ua[32][64], Ub[32][64];
  __shared__ double sc[kBigM];
  const ClassBatch& cb = hdr->cls[cls];
  if ((int)blockIdx.y >= cb.dom_off[cb.n]) return;
  const BigDom D = big_dom(tab, cb, blockIdx.y);
  const int m = D.I->m, tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int i0 = 64 * (blockIdx.x / 4), j0 = 64 * (blockIdx.x % 4);
  if (i0 >= m || j0 >= m) return;
  sc[tid] = tid < m ? sqrt((double)(m - 1) / D.v[2 * kBigM + tid]) : 0.0;
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
  for (int c0 = 0; c0 < m; c0 += 32) {
    for (int idx = tid; idx < 32 * 64; idx += 256) {
      const int cc = idx / 64, q = idx % 64, c = c0 + cc;
      const double* Uc = D.B + (size_t)c * kBigM;
      Ua[cc][q] = (c < m && i0 + q < m) ? Uc[i0 + q] * sc[c] : 0.0;
      Ub[cc][q] = (c < m && j0 + q < m) ? Uc[j0 + q] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int cc = 0; cc < 32; ++cc) {
      double a[4], b[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) a[x] = Ua[cc][ty + 16 * x];
#pragma unroll
      for (int y = 0; y < 4; ++y) b[y] = Ub[cc][tx + 16 * y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
  double* dbg = big_dbg(D);
  const double* wbar = D.v + kBigM;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int i = i0 + ty + 16 * x, j = j0 + tx + 16 * y;
      if (i < m && j < m) {
        const double tv = acc[x][y] + wbar[i];
        D.A[(size_t)i * kBigM + j] = tv;
        if (dbg) dbg[(size_t)m * m + m + (size_t)i * m + j] = tv;
      }
    }
}

// grid (row tiles, member tiles, items): Z rows q0..q0+63 of the domain (both
// instants), members j0..j0+63; X' staged 32 members at a time.
__global__ __launch_bounds__(256) void k_big_update(const InstDesc* __restrict__ tab, const BatchHdr* __restrict__ hdr,
                                                    int cls) {
  __shared__ double Xs[64][33], Ts[32][64], xb[64];
  const ClassBatch& cb = hdr->cls[cls];
  if ((int)blockIdx.z >= cb.dom_off[cb.n]) return;
  const BigDom D = big_dom(tab, cb, blockIdx.z);
  const InstDesc& I = *D.I;
  const int m = I.m, rows = 2 * D.e, tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int q0 = 64 * blockIdx.x, j0 = 64 * blockIdx.y;
  if (q0 >= rows || j0 >= m) return;
  const int cur = I.st->cur;
  const double* ens = (const double*)I.ens;
  const size_t slot = (size_t)I.n_act * m;
  auto row_ptr = [&](int q) {  // ensemble row of the domain's state row q
    const int inst = q < D.e ? cur : (cur ^ 1);
    const int act = I.est_act[D.est_off + (q < D.e ? q : q - D.e)];
    return ens + (size_t)inst * slot + (size_t)act * m;
  };
  {
    const int rr = tid / 4, part = tid % 4, q = q0 + rr;
    double sum = 0.0;
    if (q < rows) {
      const double* x = row_ptr(q);
      for (int j = part; j < m; j += 4) sum += x[j];
    }
    sum = group_sum<4>(sum);
    if (part == 0) xb[rr] = sum / (double)m;
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
  for (int k0 = 0; k0 < m; k0 += 32) {
    for (int idx = tid; idx < 64 * 32; idx += 256) {
      const int rr = idx / 32, kk = idx % 32, q = q0 + rr, k = k0 + kk;
      Xs[rr][kk] = (q < rows && k < m) ? row_ptr(q)[k] - xb[rr] : 0.0;
    }
    for (int idx = tid; idx < 32 * 64; idx += 256) {
      const int kk = idx / 64, cc = idx % 64, k = k0 + kk, j = j0 + cc;
      Ts[kk][cc] = (k < m && j < m) ? D.A[(size_t)k * kBigM + j] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 32; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) a[x] = Xs[ty + 16 * x][kk];
#pragma unroll
      for (int y = 0; y < 4; ++y) b[y] = Ts[kk][tx + 16 * y];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
    }
    __syncthreads();
  }
  double* Z = (double*)I.Z + (size_t)2 * D.est_off * m;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int rr = ty + 16 * x, q = q0 + rr, j = j0 + tx + 16 * y;
      if (q < rows && j < m) Z[(size_t)q * m + j] = xb[rr] + acc[x][y];
    }
}

// ----------------------------------------------------------------------------
// The allocation-free frame (letkf_step_noalloc): callers that cannot
// allocate device memory run a frame with its per-frame scratch in this
// file-scope array instead of the instance workspace.  Each GPU holds its own
// copy (kScratchBytes) until the process ends, shared by every such call on
// that GPU.  Host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (scratch_address), never through its name.
// ----------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, unsigned char** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static unsigned char* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the current device's copy
    if (e != hipSuccess) return e;
    addr[device] = (unsigned char*)p;
  }
  *out = addr[device];
  return hipSuccess;
}

// One workgroup: word copies of the instance descriptor and of the class's
// batch entry, then the pointers moved into the array.  Everything the frame
// kernels read of the header is written here (the work counter is zeroed by
// the slope kernel); the other classes' entries are never read.
__global__ __launch_bounds__(256) void k_noalloc_setup(const InstDesc* __restrict__ src,
                                                       const BatchHdr* __restrict__ src_hdr, unsigned char* sp,
                                                       NoallocLayout lay, const double* y, double* pred, int cls) {
  InstDesc* d = (InstDesc*)(sp + lay.desc);
  BatchHdr* h = (BatchHdr*)(sp + lay.hdr);
  static_assert(sizeof(InstDesc) % 4 == 0 && sizeof(ClassBatch) % 4 == 0, "word copies");
  for (int i = threadIdx.x; i < (int)(sizeof(InstDesc) / 4); i += blockDim.x)
    ((uint32_t*)d)[i] = ((const uint32_t*)src)[i];
  for (int i = threadIdx.x; i < (int)(sizeof(ClassBatch) / 4); i += blockDim.x)
    ((uint32_t*)&h->cls[cls])[i] = ((const uint32_t*)&src_hdr->cls[cls])[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    d->Yp = sp + lay.Yp;
    d->d = (double*)(sp + lay.d);
    d->Z = sp + lay.Z;
    d->Ascr = lay.Ascr ? (double*)(sp + lay.Ascr) : nullptr;
    h->yptr[0] = y;
    h->amean = (double*)(sp + lay.amean);
    h->pmean = pred;
    h->out_off[0] = 0;
    h->check_y = 0;
    h->bad[0] = 0;
  }
}

void launch_noalloc_setup(const InstDesc* src, const BatchHdr* src_hdr, unsigned char* sp, const NoallocLayout& lay,
                          const double* y, double* pred, int cls, hipStream_t s) {
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, s, src, src_hdr, sp, lay, y, pred, cls);
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
// Row and item kernels loop grid-stride, so their grids are capped: a launch
// never needs more than this many workgroups to cover its work.
constexpr int kRowGridCap = 4096;
constexpr int kItemGridCap = 2048;

template <typename T, int MP>
static void launch_rows_t(int mode, int rows, const InstDesc* tab, BatchHdr* hdr, int cls,
                          hipStream_t s) {
  const int grid = min((rows + 256 / MP - 1) / (256 / MP), kRowGridCap);
  if (grid <= 0) return;
  if (mode == 0) hipLaunchKernelGGL((k_rows<T, MP, 0>), dim3(grid), dim3(256), 0, s, tab, hdr, cls);
  if (mode == 1) hipLaunchKernelGGL((k_rows<T, MP, 1>), dim3(grid), dim3(256), 0, s, tab, hdr, cls);
  if (mode == 2) hipLaunchKernelGGL((k_rows<T, MP, 2>), dim3(grid), dim3(256), 0, s, tab, hdr, cls);
  if (mode != 0) hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, tab, hdr, cls);
}

template <typename T, int MP>
static void launch_slopes_t(int rows, const InstDesc* tab, BatchHdr* hdr, int cls, hipStream_t s) {
  const int grid = min((rows + 256 / MP - 1) / (256 / MP), kRowGridCap);
  if (grid > 0) hipLaunchKernelGGL((k_slopes<T, MP>), dim3(grid), dim3(256), 0, s, tab, hdr, cls);
}

#define LETKF_DISPATCH(FN, cls, ...)                                          \
  do {                                                                        \
    const int prec_ = (cls) / 4, sz_ = (cls) % 4;                             \
    if ((cls) == kBigClass) {                                                 \
      FN<double, 256>(__VA_ARGS__);                                           \
    } else if (prec_ == 0) {                                                  \
      if (sz_ == 0) FN<double, 16>(__VA_ARGS__);                              \
      else if (sz_ == 1) FN<double, 32>(__VA_ARGS__);                         \
      else if (sz_ == 2) FN<double, 64>(__VA_ARGS__);                         \
      else FN<double, 128>(__VA_ARGS__);                                      \
    } else {                                                                  \
      if (sz_ == 0) FN<float, 16>(__VA_ARGS__);                               \
      else if (sz_ == 1) FN<float, 32>(__VA_ARGS__);                          \
      else if (sz_ == 2) FN<float, 64>(__VA_ARGS__);                          \
      else FN<float, 128>(__VA_ARGS__);                                       \
    }                                                                         \
  } while (0)

// The analysis kernel of a class (P = precision path, M = padded size).
#define LETKF_ANA_KERNEL(cls, FN)                                   \
  do {                                                              \
    const int prec_ = (cls) / 4, sz_ = (cls) % 4;                   \
    if (prec_ == 0) {                                               \
      if (sz_ == 0) FN((k_analysis<0, 16>));                        \
      else if (sz_ == 1) FN((k_analysis<0, 32>));                   \
      else if (sz_ == 2) FN((k_analysis<0, 64>));                   \
      else FN((k_analysis<0, 128>));                                \
    } else if (prec_ == 1) {                                        \
      if (sz_ == 0) FN((k_analysis<1, 16>));                        \
      else if (sz_ == 1) FN((k_analysis<1, 32>));                   \
      else if (sz_ == 2) FN((k_analysis<1, 64>));                   \
      else FN((k_analysis<1, 128>));                                \
    } else if (prec_ == 2) {                                        \
      if (sz_ == 0) FN((k_analysis<2, 16>));                        \
      else if (sz_ == 1) FN((k_analysis<2, 32>));                   \
      else if (sz_ == 2) FN((k_analysis<2, 64>));                   \
      else FN((k_analysis<2, 128>));                                \
    } else {                                                        \
      if (sz_ == 0) FN((k_analysis<3, 16>));                        \
      else if (sz_ == 1) FN((k_analysis<3, 32>));                   \
      else if (sz_ == 2) FN((k_analysis<3, 64>));                   \
      else FN((k_analysis<3, 128>));                                \
    }                                                               \
  } while (0)

void launch_slopes(int cls, int rows, const InstDesc* tab, BatchHdr* hdr, hipStream_t s) {
  LETKF_DISPATCH(launch_slopes_t, cls, rows, tab, hdr, cls, s);
}
void launch_pistons(int cls, int items, const InstDesc* tab, BatchHdr* hdr, hipStream_t s) {
  const int grid = min(items, kItemGridCap);
  if (grid <= 0) return;
  if (cls / 4 == 0 || cls == kBigClass) hipLaunchKernelGGL(k_piston_rhs<double>, dim3(grid), dim3(256), 0, s, tab, hdr, cls);
  else hipLaunchKernelGGL(k_piston_rhs<float>, dim3(grid), dim3(256), 0, s, tab, hdr, cls);
  hipLaunchKernelGGL(k_piston_solve, dim3(grid), dim3(256), 0, s, tab, hdr, cls);
}

void launch_rows(int cls, int mode, int rows, const InstDesc* tab, BatchHdr* hdr, hipStream_t s) {
  LETKF_DISPATCH(launch_rows_t, cls, mode, rows, tab, hdr, cls, s);
}

void launch_big_analysis(int items, int rows_max, int m_max, const InstDesc* tab, BatchHdr* hdr, hipStream_t s) {
  if (items <= 0) return;
  const int cls = kBigClass, nb = 2 * ((m_max + 31) / 32);
  hipLaunchKernelGGL(k_big_gram, dim3(10, items), dim3(256), 0, s, tab, hdr, cls);
  hipLaunchKernelGGL(k_big_chol, dim3(items), dim3(64 * kBigCholWaves), 0, s, tab, hdr, cls);
  for (int sw = 0; sw < kBigMaxSweeps; ++sw) {
    for (int r = 0; r < nb - 1; ++r)
      hipLaunchKernelGGL(k_big_round, dim3(nb / 2, items), dim3(256), 0, s, tab, hdr, cls, nb, r);
    hipLaunchKernelGGL(k_big_sweep, dim3((items + 63) / 64), dim3(64), 0, s, tab, hdr, cls);
  }
  hipLaunchKernelGGL(k_big_eig, dim3(items), dim3(256), 0, s, tab, hdr, cls);
  hipLaunchKernelGGL(k_big_T, dim3(16, items), dim3(256), 0, s, tab, hdr, cls);
  hipLaunchKernelGGL(k_big_update, dim3((rows_max + 63) / 64, (m_max + 63) / 64, items), dim3(256), 0, s, tab, hdr,
                     cls);
}

void launch_analysis(int cls, int grid, const InstDesc* tab, BatchHdr* hdr, hipStream_t s, int fair) {
  if (grid <= 0 || cls == kBigClass) return;  // the m > 128 class runs launch_big_analysis
#define LETKF_LAUNCH_ANA(K) hipLaunchKernelGGL(K, dim3(grid), dim3(256), 0, s, tab, hdr, cls, fair)
  LETKF_ANA_KERNEL(cls, LETKF_LAUNCH_ANA);
#undef LETKF_LAUNCH_ANA
}

int analysis_blocks_per_cu(int cls) {
  if (cls == kBigClass) return 1;
  int n = 0;
  hipError_t e = hipSuccess;
#define LETKF_OCC(K) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, K, 256, 0)
  LETKF_ANA_KERNEL(cls, LETKF_OCC);
#undef LETKF_OCC
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace letkf
