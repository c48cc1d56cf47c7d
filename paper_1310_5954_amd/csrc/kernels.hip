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

// Sum of v over the MP lanes of a member row (MP <= 64: one wavefront segment;
// MP = 128: two wavefronts combined through LDS).  Every thread participates.
template <int MP>
__device__ __forceinline__ double row_sum(double v, double* red) {
  constexpr int W = MP < 64 ? MP : 64;
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
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
// a3: slope perturbations and innovation of every slope row of the class.
// ----------------------------------------------------------------------------
template <typename T, int MP>
__global__ __launch_bounds__(256) void k_slopes(const InstDesc* __restrict__ tab,
                                                BatchHdr* __restrict__ hdr, int cls) {
  constexpr int RPB = 256 / MP;
  __shared__ double red[4];
  const ClassBatch& cb = hdr->cls[cls];
  if (blockIdx.x == 0 && (int)threadIdx.x < cb.n) tab[cb.inst[threadIdx.x]].st->unconverged = 0;
  const int j = threadIdx.x % MP;
  const int g = blockIdx.x * RPB + threadIdx.x / MP;
  const int total = cb.slope_off[cb.n];
  const bool active = g < total;
  const int b = find_entry(cb.slope_off, cb.n, active ? g : 0);
  const InstDesc& I = tab[cb.inst[b]];
  const int m = I.m;
  const int o = g - cb.slope_off[b];
  double v = 0.0;
  if (active && j < m) {
    const T* ens = (const T*)I.ens + (size_t)I.st->cur * I.n_act * m;
    for (int k = I.d_rowptr[o]; k < I.d_rowptr[o + 1]; ++k)
      v += I.d_val[k] * ld(ens + (size_t)I.d_col[k] * m + j);
  }
  const double ybar = row_sum<MP>(v, red) / (double)m;
  if (active) {
    if (j < m) st((T*)I.Yp + (size_t)o * m + j, v - ybar);
    if (j == 0) I.d[o] = hdr->y[hdr->y_off[cb.ent[b]] + o] - ybar;
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
  const int g = blockIdx.x * RPB + threadIdx.x / MP;
  const int total = cb.act_off[cb.n];
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
  const bool live = active && j < m;
  double vk = 0.0, vkm1 = 0.0;
  if (live) {
    if (MODE == 1) {
      vk = ld(e_cur + (size_t)a * m + j);
      vkm1 = ld(e_prev + (size_t)a * m + j);
    } else {
      const T* Z = (const T*)I.Z;
      for (int q = I.mptr[a]; q < I.mptr[a + 1]; ++q) {
        const double w = I.mw[q];
        vk += w * ld(Z + (size_t)I.mrow[2 * q] * m + j);
        vkm1 += w * ld(Z + (size_t)I.mrow[2 * q + 1] * m + j);
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
    if (active && j == 0) hdr->amean[hdr->out_off[ent] + a] = s / (double)m;
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
    if (active && j == 0) hdr->pmean[hdr->out_off[ent] + a] = s / (double)m;
    // the last block to finish advances every instance of the class
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      const unsigned prev = atomicAdd(&cb.done, 1u);
      if (prev == gridDim.x - 1) {
        __threadfence();
        for (int e = 0; e < cb.n; ++e) {
          InstState* S = tab[cb.inst[e]].st;
          S->cur ^= 1;
          S->frame += 1;
        }
        cb.done = 0;
        __threadfence();
      }
    }
  }
}

// ----------------------------------------------------------------------------
// a4-a8: per-domain analysis, one 256-thread workgroup per domain.
// ----------------------------------------------------------------------------
template <int M> struct AnaCfg {
  static constexpr int NT = 256;
  static constexpr int LDB = M + 2;                // column stride of the m x m matrix in LDS
  static constexpr int KC = M <= 64 ? 32 : 8;      // rows per staged chunk
  static constexpr int TM = M / 16;                // 16 x 16 thread grid, TM x TM tile per thread
  static constexpr int TPP = (2 * NT / M) < M ? (2 * NT / M) : M;  // threads per Jacobi pair
  static constexpr int ACTIVE = (M / 2) * TPP;
  static constexpr int RPT = M / TPP;              // rows per thread in a Jacobi step
  static constexpr int MAX_SWEEPS = 40;
};

template <typename T, int M>
__global__ __launch_bounds__(256) void k_analysis(const InstDesc* __restrict__ tab,
                                                  BatchHdr* __restrict__ hdr, int cls) {
  using C = AnaCfg<M>;
  constexpr int NT = C::NT, LDB = C::LDB, KC = C::KC, TM = C::TM, TPP = C::TPP;
  __shared__ double Bm[M * LDB];
  __shared__ double Xc[KC * M];
  __shared__ double rc[KC], dc[KC];
  __shared__ double bvec[M], nrm[M], lam[M], zv[M], wbar[M];
  __shared__ int s_rot;

  const ClassBatch& cb = hdr->cls[cls];
  const int item = blockIdx.x;
  if (item >= cb.dom_off[cb.n]) return;
  const int eb = find_entry(cb.dom_off, cb.n, item);
  const InstDesc& I = tab[cb.inst[eb]];
  const int l = I.order[item - cb.dom_off[eb]];
  const int est_off = I.dom[4 * l], e = I.dom[4 * l + 1];
  const int obs_off = I.dom[4 * l + 2], s = I.dom[4 * l + 3];
  const int m = I.m;
  const int cur = I.st->cur;
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;

  // ---- a4/a5: gather Y'_O in chunks; C = Y'^T diag(r) Y', b = Y'^T diag(r) d
  double acc[TM][TM];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TM; ++y) acc[x][y] = 0.0;
  double bacc = 0.0;
  const T* Yp = (const T*)I.Yp;
  const int nobs = 2 * s;
  for (int q0 = 0; q0 < nobs; q0 += KC) {
    const int kc = min(KC, nobs - q0);
    for (int idx = tid; idx < KC * M; idx += NT) {
      const int qq = idx / M, j = idx % M;
      double v = 0.0;
      if (qq < kc && j < m) v = ld(Yp + (size_t)I.obs_row[2 * obs_off + q0 + qq] * m + j);
      Xc[idx] = v;
    }
    if (tid < KC) {
      double r = 0.0, dd = 0.0;
      if (tid < kc) {
        r = I.obs_r[2 * obs_off + q0 + tid];
        dd = I.d[I.obs_row[2 * obs_off + q0 + tid]];
      }
      rc[tid] = r;
      dc[tid] = dd;
    }
    __syncthreads();
    for (int qq = 0; qq < kc; ++qq) {
      const double r = rc[qq];
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
      for (int qq = 0; qq < kc; ++qq) bacc += rc[qq] * dc[qq] * Xc[qq * M + tid];
    __syncthreads();
  }
  double* dbg = I.dbg ? I.dbg + (size_t)l * (2 * m * m + m) : nullptr;
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TM; ++y) {
      const int i = ti + 16 * x, j = tj + 16 * y;
      double v = acc[x][y];
      if (dbg && i < m && j < m) dbg[i * m + j] = v;
      if (i >= m || j >= m) v = (i == j) ? 1.0 : 0.0;       // padded members: identity block
      else if (i == j) v += I.a_diag;                       // A = (m-1)/rho I + C
      Bm[j * LDB + i] = v;
    }
  if (tid < M) bvec[tid] = tid < m ? bacc : 0.0;
  __syncthreads();

  // ---- a6: one-sided (Hestenes) Jacobi on B = A.  Column pairs (i, i^k) for
  // k = 1..M-1 form M-1 perfect matchings that cover every pair once per sweep.
  // At convergence the columns of B = A V are lambda_i u_i (A is SPD).
  const double tol = (double)M * 1.1102230246251565e-16;
  int sweeps = 0;
  for (; sweeps < C::MAX_SWEEPS;) {
    if (tid < M) {
      double ss = 0.0;
      for (int r = 0; r < M; ++r) { const double v = Bm[tid * LDB + r]; ss += v * v; }
      nrm[tid] = ss;
    }
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int k = 1; k < M; ++k) {
      if (tid < C::ACTIVE) {
        const int q = tid / TPP, sub = tid % TPP;
        const int h = 31 - __clz(k);
        const int i = ((q >> h) << (h + 1)) | (q & ((1 << h) - 1));
        const int jj = i ^ k;
        double* bi = Bm + i * LDB;
        double* bj = Bm + jj * LDB;
        double xi[C::RPT], xj[C::RPT];
        double gsum = 0.0;
#pragma unroll
        for (int t = 0; t < C::RPT; ++t) {
          xi[t] = bi[sub + t * TPP];
          xj[t] = bj[sub + t * TPP];
          gsum += xi[t] * xj[t];
        }
#pragma unroll
        for (int off = TPP / 2; off > 0; off >>= 1) gsum += __shfl_xor(gsum, off, 64);
        const double al = nrm[i], be = nrm[jj];
        if (fabs(gsum) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * gsum);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double sn = c * t;
#pragma unroll
          for (int u = 0; u < C::RPT; ++u) {
            bi[sub + u * TPP] = c * xi[u] - sn * xj[u];
            bj[sub + u * TPP] = sn * xi[u] + c * xj[u];
          }
          if (sub == 0) {
            nrm[i] = al - t * gsum;
            nrm[jj] = be + t * gsum;
            s_rot = 1;
          }
        }
      }
      __syncthreads();
    }
    ++sweeps;
    const int any = s_rot;
    __syncthreads();
    if (!any) break;
  }

  // ---- a7: lambda, U, wbar = U Lambda^-1 U^T b, W = U sqrt((m-1)/Lambda) U^T
  if (tid < M) {
    double ss = 0.0;
    for (int r = 0; r < M; ++r) { const double v = Bm[tid * LDB + r]; ss += v * v; }
    lam[tid] = sqrt(ss);
  }
  __syncthreads();
  for (int idx = tid; idx < M * M; idx += NT) {
    const int c = idx / M, r = idx % M;
    Bm[c * LDB + r] /= lam[c];
  }
  __syncthreads();
  if (tid < M) {
    double t = 0.0;
    for (int r = 0; r < M; ++r) t += Bm[tid * LDB + r] * bvec[r];
    zv[tid] = tid < m ? t / lam[tid] : 0.0;
    nrm[tid] = tid < m ? sqrt((double)(m - 1) / lam[tid]) : 0.0;
  }
  __syncthreads();
  if (tid < M) {
    double w = 0.0;
    for (int c = 0; c < m; ++c) w += Bm[c * LDB + tid] * zv[c];
    wbar[tid] = tid < m ? w : 0.0;
  }
  double tacc[TM][TM];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TM; ++y) tacc[x][y] = 0.0;
  for (int c = 0; c < m; ++c) {
    const double sc = nrm[c];
    double ui[TM], uj[TM];
#pragma unroll
    for (int x = 0; x < TM; ++x) {
      ui[x] = Bm[c * LDB + ti + 16 * x] * sc;
      uj[x] = Bm[c * LDB + tj + 16 * x];
    }
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TM; ++y) tacc[x][y] += ui[x] * uj[y];
  }
  __syncthreads();
  // T = W + wbar 1^T, stored row-major (row = ensemble index contracted in the update)
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TM; ++y) {
      const int i = ti + 16 * x, j = tj + 16 * y;
      const double v = (i < m && j < m) ? tacc[x][y] + wbar[i] : 0.0;
      Bm[i * LDB + j] = v;
      if (dbg && i < m && j < m) dbg[m * m + m + i * m + j] = v;
    }
  if (dbg && tid < m) dbg[m * m + tid] = lam[tid];
  if (tid == 0) {
    if (I.dbg_sweeps) I.dbg_sweeps[l] = sweeps;
    if (sweeps >= C::MAX_SWEEPS) atomicAdd(&I.st->unconverged, 1);
    atomicAdd(&I.st->sweeps, (unsigned long long)sweeps);
    atomicAdd(&I.st->solves, 1ull);
  }
  __syncthreads();

  // ---- a8: Z = xbar 1^T + X' T for the domain's state rows (both instants)
  const T* ens = (const T*)I.ens;
  const size_t slot = (size_t)I.n_act * m;
  T* Z = (T*)I.Z + (size_t)2 * est_off * m;
  for (int q0 = 0; q0 < 2 * e; q0 += KC) {
    const int kc = min(KC, 2 * e - q0);
    for (int idx = tid; idx < KC * M; idx += NT) {
      const int qq = idx / M, j = idx % M;
      double v = 0.0;
      if (qq < kc && j < m) {
        const int q = q0 + qq;
        const int inst = q < e ? cur : (cur ^ 1);
        const int act = I.est_act[est_off + (q < e ? q : q - e)];
        v = ld(ens + (size_t)inst * slot + (size_t)act * m + j);
      }
      Xc[idx] = v;
    }
    __syncthreads();
    if (tid < KC) {
      double sm = 0.0;
      for (int j = 0; j < m; ++j) sm += Xc[tid * M + j];
      rc[tid] = sm / (double)m;
    }
    __syncthreads();
    for (int idx = tid; idx < kc * M; idx += NT) {
      const int qq = idx / M, j = idx % M;
      if (j < m) {
        const double xb = rc[qq];
        double z = 0.0;
        for (int k = 0; k < m; ++k) z += (Xc[qq * M + k] - xb) * Bm[k * LDB + j];
        st(Z + (size_t)(q0 + qq) * m + j, xb + z);
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
template <typename T, int MP>
static void launch_rows_t(int mode, int rows, const InstDesc* tab, BatchHdr* hdr, int cls,
                          hipStream_t s) {
  const int grid = (rows + 256 / MP - 1) / (256 / MP);
  if (grid <= 0) return;
  if (mode == 0) hipLaunchKernelGGL((k_rows<T, MP, 0>), dim3(grid), dim3(256), 0, s, tab, hdr, cls);
  if (mode == 1) hipLaunchKernelGGL((k_rows<T, MP, 1>), dim3(grid), dim3(256), 0, s, tab, hdr, cls);
  if (mode == 2) hipLaunchKernelGGL((k_rows<T, MP, 2>), dim3(grid), dim3(256), 0, s, tab, hdr, cls);
}

template <typename T, int MP>
static void launch_slopes_t(int rows, const InstDesc* tab, BatchHdr* hdr, int cls, hipStream_t s) {
  const int grid = (rows + 256 / MP - 1) / (256 / MP);
  if (grid > 0) hipLaunchKernelGGL((k_slopes<T, MP>), dim3(grid), dim3(256), 0, s, tab, hdr, cls);
}

template <typename T, int M>
static void launch_analysis_t(int items, const InstDesc* tab, BatchHdr* hdr, int cls, hipStream_t s) {
  if (items > 0) hipLaunchKernelGGL((k_analysis<T, M>), dim3(items), dim3(256), 0, s, tab, hdr, cls);
}

#define LETKF_DISPATCH(FN, cls, ...)                                          \
  do {                                                                        \
    const int prec_ = (cls) / 4, sz_ = (cls) % 4;                             \
    if (prec_ == 0) {                                                         \
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

void launch_slopes(int cls, int rows, const InstDesc* tab, BatchHdr* hdr, hipStream_t s) {
  LETKF_DISPATCH(launch_slopes_t, cls, rows, tab, hdr, cls, s);
}
void launch_rows(int cls, int mode, int rows, const InstDesc* tab, BatchHdr* hdr, hipStream_t s) {
  LETKF_DISPATCH(launch_rows_t, cls, mode, rows, tab, hdr, cls, s);
}
void launch_analysis(int cls, int items, const InstDesc* tab, BatchHdr* hdr, hipStream_t s) {
  LETKF_DISPATCH(launch_analysis_t, cls, items, tab, hdr, cls, s);
}

}  // namespace letkf
