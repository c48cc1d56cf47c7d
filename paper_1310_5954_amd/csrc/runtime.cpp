// C ABI of the single-instance path: validation, workspace layout, upload,
// and the per-frame launch sequence (slopes -> analysis -> merge/forecast).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

namespace letkf {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return LETKF_EDEVICE;
}

static bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

int validate(const letkf_dims* dims, const letkf_model* model, const letkf_domain_map* map,
             int precision, uint32_t flags, Problem& P) {
  if (!dims || !model || !map) return fail(LETKF_EINVAL, "null dims/model/map");
  if (dims->n_act < 1 || dims->n_sub < 1) return fail(LETKF_EINVAL, "n_act and n_sub must be >= 1");
  if (dims->m < 2 || dims->m > 256) return fail(LETKF_EINVAL, "m must be in [2, 256]");
  if (dims->m > 128 && precision != LETKF_FP64) return fail(LETKF_EINVAL, "m > 128 needs LETKF_FP64");
  if (dims->m > 128 && (flags & LETKF_FLAG_PISTONS))
    return fail(LETKF_EINVAL, "LETKF_FLAG_PISTONS needs m <= 128");
  if (precision != LETKF_FP64 && precision != LETKF_FP32 && precision != LETKF_BF16)
    return fail(LETKF_EINVAL, "unknown precision");
  if (flags & ~(LETKF_FLAG_DEBUG | LETKF_FLAG_PISTONS | LETKF_FLAG_GRAPH | LETKF_FLAG_FP32_ROTATIONS))
    return fail(LETKF_EINVAL, "unknown flags");
  if ((flags & LETKF_FLAG_FP32_ROTATIONS) && precision != LETKF_BF16)
    return fail(LETKF_EINVAL, "LETKF_FLAG_FP32_ROTATIONS needs LETKF_BF16");
  P.n_act = dims->n_act;
  P.n_sub = dims->n_sub;
  P.m = dims->m;
  P.prec = precision;
  P.flags = flags;
  const int n_act = P.n_act, p = 2 * P.n_sub;
  if (!model->a1 || !model->a2 || !model->r_inv || !model->d_rowptr ||
      (model->d_nnz > 0 && (!model->d_col || !model->d_val)))
    return fail(LETKF_EINVAL, "null model array");
  if (!finite_all(model->a1, n_act) || !finite_all(model->a2, n_act))
    return fail(LETKF_EINVAL, "non-finite AR coefficients");
  if (!std::isfinite(model->sigma_v) || model->sigma_v < 0) return fail(LETKF_EINVAL, "sigma_v must be finite and >= 0");
  if (!std::isfinite(model->inflation) || model->inflation <= 0) return fail(LETKF_EINVAL, "inflation must be > 0");
  if (model->obs_instant != 0 && model->obs_instant != 1) return fail(LETKF_EINVAL, "obs_instant must be 0 or 1");
  for (int i = 0; i < p; ++i)
    if (!std::isfinite(model->r_inv[i]) || model->r_inv[i] < 0) return fail(LETKF_EINVAL, "r_inv must be finite and >= 0");
  if (model->d_nnz < 0) return fail(LETKF_EINVAL, "d_nnz < 0");
  if (model->d_rowptr[0] != 0 || model->d_rowptr[p] != model->d_nnz)
    return fail(LETKF_EINVAL, "D rowptr must start at 0 and end at d_nnz");
  for (int i = 0; i < p; ++i)
    if (model->d_rowptr[i + 1] < model->d_rowptr[i]) return fail(LETKF_EINVAL, "D rowptr not monotone");
  for (int k = 0; k < model->d_nnz; ++k) {
    if (model->d_col[k] < 0 || model->d_col[k] >= n_act) return fail(LETKF_EINVAL, "D column out of range");
    if (!std::isfinite(model->d_val[k])) return fail(LETKF_EINVAL, "non-finite D value");
  }
  P.sigma_v = model->sigma_v;
  P.inflation = model->inflation;
  P.seed = model->seed;
  P.obs_instant = model->obs_instant;
  P.nnz = model->d_nnz;
  P.a1.assign(model->a1, model->a1 + n_act);
  P.a2.assign(model->a2, model->a2 + n_act);
  P.r_inv.assign(model->r_inv, model->r_inv + p);
  P.d_rowptr.assign(model->d_rowptr, model->d_rowptr + p + 1);
  P.d_col.assign(model->d_col, model->d_col + P.nnz);
  P.d_val.assign(model->d_val, model->d_val + P.nnz);

  const int L = map->n_domains;
  if (L < 1) return fail(LETKF_EINVAL, "n_domains must be >= 1");
  if (!map->est_ptr || !map->est_act || !map->est_w || !map->obs_ptr ||
      (map->obs_ptr && map->obs_ptr[L] > 0 && (!map->obs_sub || !map->obs_taper)))
    return fail(LETKF_EINVAL, "null domain-map array");
  if (map->est_ptr[0] != 0 || map->obs_ptr[0] != 0) return fail(LETKF_EINVAL, "map CSR must start at 0");
  std::vector<double> wsum(n_act, 0.0);
  for (int l = 0; l < L; ++l) {
    const int e = map->est_ptr[l + 1] - map->est_ptr[l];
    const int s = map->obs_ptr[l + 1] - map->obs_ptr[l];
    if (e < 1) return fail(LETKF_EINVAL, "domain " + std::to_string(l) + " has no actuator");
    if (s < 0) return fail(LETKF_EINVAL, "obs_ptr not monotone");
    for (int q = map->est_ptr[l]; q < map->est_ptr[l + 1]; ++q) {
      const int a = map->est_act[q];
      if (a < 0 || a >= n_act) return fail(LETKF_EINVAL, "est_act out of range");
      if (!std::isfinite(map->est_w[q]) || map->est_w[q] < 0) return fail(LETKF_EINVAL, "bad merge weight");
      wsum[a] += map->est_w[q];
    }
    for (int q = map->obs_ptr[l]; q < map->obs_ptr[l + 1]; ++q) {
      if (map->obs_sub[q] < 0 || map->obs_sub[q] >= P.n_sub) return fail(LETKF_EINVAL, "obs_sub out of range");
      const double t = map->obs_taper[q];
      if (!(t >= 0.0 && t <= 1.0)) return fail(LETKF_EINVAL, "taper must be in [0, 1]");
    }
  }
  for (int a = 0; a < n_act; ++a)
    if (std::fabs(wsum[a] - 1.0) > 1e-9)
      return fail(LETKF_EINVAL, "merge weights of actuator " + std::to_string(a) + " do not sum to 1");
  P.n_dom = L;
  P.est_ptr.assign(map->est_ptr, map->est_ptr + L + 1);
  P.obs_ptr.assign(map->obs_ptr, map->obs_ptr + L + 1);
  P.est_act.assign(map->est_act, map->est_act + P.est_ptr[L]);
  P.est_w.assign(map->est_w, map->est_w + P.est_ptr[L]);
  P.obs_sub.assign(map->obs_sub, map->obs_sub + P.obs_ptr[L]);
  P.obs_taper.assign(map->obs_taper, map->obs_taper + P.obs_ptr[L]);
  return LETKF_OK;
}

Layout make_layout(const Problem& P) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    const size_t o = off;
    off += bytes;
    return o;
  };
  const size_t es = P.esize();
  const size_t m = P.m, n_act = P.n_act, p = P.p();
  L.desc = take(sizeof(InstDesc));
  L.state = take(sizeof(InstState));
  L.hdr = take(sizeof(BatchHdr));
  L.ens = take(2 * n_act * m * es);
  L.Yp = take(p * m * es);
  L.d = take(p * 8);
  L.Z = take((size_t)P.zrows() * m * es);
  L.y = take(p * 8);
  L.amean = take(n_act * 8);
  L.pmean = take(n_act * 8);
  L.static_begin = off = (off + 255) & ~size_t(255);
  L.a1 = take(n_act * 8);
  L.a2 = take(n_act * 8);
  L.rowptr = take((p + 1) * 4);
  L.col = take((size_t)P.nnz * 4);
  L.val = take((size_t)P.nnz * 8);
  L.dom = take((size_t)P.n_dom * 16);
  L.order = take((size_t)P.n_dom * 4);
  L.est = take((size_t)P.sum_e() * 4);
  L.obs_row = take((size_t)2 * P.sum_s() * 4);
  L.obs_r = take((size_t)2 * P.sum_s() * 8);
  L.obs_sr = take((size_t)2 * P.sum_s() * 8);
  L.mptr = take((n_act + 1) * 4);
  L.mrow = take((size_t)2 * P.sum_e() * 4);
  L.mw = take((size_t)P.sum_e() * 8);
  L.mdom = take((size_t)P.sum_e() * 4);
  L.pist_op = L.pist_ptr = L.pist_row = L.pist_coef = 0;
  if (P.flags & LETKF_FLAG_PISTONS) {
    L.pist_op = take((size_t)P.n_dom * P.n_dom * 8);
    const size_t terms = P.piston_terms();
    L.pist_ptr = take((size_t)(P.n_dom + 1) * 4);
    L.pist_row = take(2 * terms * 4);
    L.pist_coef = take(terms * 8);
  }
  L.static_end = off;
  if (P.flags & LETKF_FLAG_PISTONS) {
    L.pist_r = take((size_t)P.n_dom * 2 * m * 8);
    L.pist_c = take((size_t)P.n_dom * 2 * m * 8);
  } else {
    L.pist_r = L.pist_c = 0;
  }
  L.bigA = L.bigB = L.bigv = L.bigf = 0;
  if (padded_members(P.m) > 128) {
    const size_t mm = 256 * 256;
    L.bigA = take((size_t)P.n_dom * mm * 8);
    L.bigB = take((size_t)P.n_dom * mm * 8);
    L.bigv = take((size_t)P.n_dom * 5 * 256 * 8);
    L.bigf = take((size_t)P.n_dom * 4 * 4);
  }
  L.dom_sweeps = take((size_t)P.n_dom * 4);
  {
    const size_t M = padded_members(P.m);
    L.Ascr = (P.prec == LETKF_FP64 && M <= 128) ? take((size_t)P.n_dom * tri_size(P.m) * 8) : 0;
  }
  if (P.flags & LETKF_FLAG_DEBUG) {
    L.dbg = take((size_t)P.n_dom * (2 * m * m + m + kDbgTail) * 8);
    L.dbg_sweeps = take((size_t)P.n_dom * 4);
  } else {
    L.dbg = L.dbg_sweeps = 0;
  }
  L.total = (off + 255) & ~size_t(255);
  return L;
}

template <typename T>
static void put(std::vector<char>& blob, size_t base, size_t off, const T* src, size_t n) {
  if (n) std::memcpy(blob.data() + (off - base), src, n * sizeof(T));
}

// Piston operator G (n_dom x n_dom): c = G r turns the overlap mismatches
// r_l = sum over actuators j of l of (sum of the covering domains' rows at j
// minus k_j times l's own row) into the least-squares pistons.  The normal
// equations of  min sum_j sum_{l != l' covering j} (Z_l + c_l - Z_l' - c_l')^2
// have the overlap-graph Laplacian Lap (Lap_ll = pairs through l, Lap_ll' = -
// shared actuators); G = (I - 1 w^T / sum w) Lap^+ with w_l the sum of domain
// l's merge weights.  Lap^+ per connected component of size n_c > 1:
// (Lap_c + 11^T / n_c)^-1 - 11^T / n_c (Cholesky of an SPD matrix); zero on
// isolated domains.  Dense O(n_dom^3) on the host, once per instance.
static std::vector<double> piston_operator(const Problem& P, const std::vector<int32_t>& mptr,
                                           const std::vector<int32_t>& mdom) {
  const int n = P.n_dom;
  std::vector<double> lap((size_t)n * n, 0.0);
  for (int a = 0; a < P.n_act; ++a)
    for (int x = mptr[a]; x < mptr[a + 1]; ++x)
      for (int y = mptr[a]; y < mptr[a + 1]; ++y) {
        if (x == y) continue;
        const int dx = mdom[x], dy = mdom[y];
        lap[(size_t)dx * n + dx] += 1.0;
        lap[(size_t)dx * n + dy] -= 1.0;
      }
  // connected components of the overlap graph
  std::vector<int> comp(n, -1);
  int ncomp = 0;
  for (int s0 = 0; s0 < n; ++s0) {
    if (comp[s0] >= 0) continue;
    std::vector<int> stack{s0};
    comp[s0] = ncomp;
    while (!stack.empty()) {
      const int u = stack.back();
      stack.pop_back();
      for (int v = 0; v < n; ++v)
        if (comp[v] < 0 && lap[(size_t)u * n + v] != 0.0) { comp[v] = ncomp; stack.push_back(v); }
    }
    ++ncomp;
  }
  std::vector<double> pinv((size_t)n * n, 0.0);
  for (int c = 0; c < ncomp; ++c) {
    std::vector<int> idx;
    for (int v = 0; v < n; ++v)
      if (comp[v] == c) idx.push_back(v);
    const int k = (int)idx.size();
    if (k < 2) continue;
    // M = Lap_c + 11^T / k, Cholesky M = R R^T (lower R, in place)
    std::vector<double> M((size_t)k * k);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) M[(size_t)i * k + j] = lap[(size_t)idx[i] * n + idx[j]] + 1.0 / k;
    for (int j = 0; j < k; ++j) {
      double d = M[(size_t)j * k + j];
      for (int q = 0; q < j; ++q) d -= M[(size_t)j * k + q] * M[(size_t)j * k + q];
      d = std::sqrt(d);
      M[(size_t)j * k + j] = d;
      for (int i = j + 1; i < k; ++i) {
        double v = M[(size_t)i * k + j];
        for (int q = 0; q < j; ++q) v -= M[(size_t)i * k + q] * M[(size_t)j * k + q];
        M[(size_t)i * k + j] = v / d;
      }
    }
    // columns of M^-1 by forward and back substitution, minus 11^T / k
    std::vector<double> x(k);
    for (int col = 0; col < k; ++col) {
      for (int i = 0; i < k; ++i) {
        double v = (i == col) ? 1.0 : 0.0;
        for (int q = 0; q < i; ++q) v -= M[(size_t)i * k + q] * x[q];
        x[i] = v / M[(size_t)i * k + i];
      }
      for (int i = k - 1; i >= 0; --i) {
        double v = x[i];
        for (int q = i + 1; q < k; ++q) v -= M[(size_t)q * k + i] * x[q];
        x[i] = v / M[(size_t)i * k + i];
      }
      for (int i = 0; i < k; ++i) pinv[(size_t)idx[i] * n + idx[col]] = x[i] - 1.0 / k;
    }
  }
  // gauge: G = (I - 1 w^T / sum w) Lap^+
  std::vector<double> w(n, 0.0);
  for (int l = 0; l < n; ++l)
    for (int q = P.est_ptr[l]; q < P.est_ptr[l + 1]; ++q) w[l] += P.est_w[q];
  double wsum = 0.0;
  for (double v : w) wsum += v;
  std::vector<double> g(n, 0.0);  // w^T Lap^+ / sum w
  for (int l = 0; l < n; ++l)
    for (int j = 0; j < n; ++j) g[j] += w[l] * pinv[(size_t)l * n + j];
  for (int j = 0; j < n; ++j) g[j] /= wsum;
  for (int l = 0; l < n; ++l)
    for (int j = 0; j < n; ++j) pinv[(size_t)l * n + j] -= g[j];
  return pinv;
}

std::vector<int32_t> domain_order(const Problem& P, int policy) {
  const int n = P.n_dom;
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  if (policy == LETKF_ORDER_COST) {
    // largest work first: the heaviest domains start first and the light ones fill the tail
    auto cost = [&](int l) {
      return (P.est_ptr[l + 1] - P.est_ptr[l]) + (P.obs_ptr[l + 1] - P.obs_ptr[l]);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  } else if (policy == LETKF_ORDER_XCD) {
    // Workgroup b of a launch runs on XCD b % 8.  Cut the map order into 8
    // contiguous chunks and give position b the next domain of chunk b % 8
    // (of another chunk once that one is used up), so that neighbouring
    // domains, which gather overlapping rows, share an XCD's L2.
    constexpr int X = kXcds;
    std::vector<int> head(X), end(X);
    for (int x = 0; x < X; ++x) {
      head[x] = (int)((int64_t)n * x / X);
      end[x] = (int)((int64_t)n * (x + 1) / X);
    }
    for (int b = 0; b < n; ++b) {
      int x = b % X;
      while (head[x] == end[x]) x = (x + 1) % X;
      order[b] = head[x]++;
    }
  }
  return order;
}

int upload_instance(const Problem& P, const Layout& L, char* ws, const double* X0, hipStream_t stream,
                    InstDesc& D) {
  const int n_act = P.n_act, m = P.m, p = P.p();
  const size_t es = P.esize();
  // ---- static tables
  std::vector<char> blob(L.static_end - L.static_begin, 0);
  const size_t B = L.static_begin;
  put(blob, B, L.a1, P.a1.data(), n_act);
  put(blob, B, L.a2, P.a2.data(), n_act);
  put(blob, B, L.rowptr, P.d_rowptr.data(), p + 1);
  put(blob, B, L.col, P.d_col.data(), P.nnz);
  put(blob, B, L.val, P.d_val.data(), P.nnz);
  std::vector<int32_t> dom(4 * P.n_dom), order(P.n_dom);
  for (int l = 0; l < P.n_dom; ++l) {
    dom[4 * l] = P.est_ptr[l];
    dom[4 * l + 1] = P.est_ptr[l + 1] - P.est_ptr[l];
    dom[4 * l + 2] = P.obs_ptr[l];
    dom[4 * l + 3] = P.obs_ptr[l + 1] - P.obs_ptr[l];
  }
  order = domain_order(P, LETKF_ORDER_COST);
  put(blob, B, L.dom, dom.data(), dom.size());
  put(blob, B, L.order, order.data(), order.size());
  put(blob, B, L.est, P.est_act.data(), P.est_act.size());
  std::vector<int32_t> obs_row(2 * P.sum_s());
  std::vector<double> obs_r(2 * P.sum_s());
  for (int l = 0; l < P.n_dom; ++l) {
    const int o0 = P.obs_ptr[l], s = P.obs_ptr[l + 1] - o0;
    for (int q = 0; q < s; ++q) {
      const int sub = P.obs_sub[o0 + q];
      const double t = P.obs_taper[o0 + q];
      obs_row[2 * o0 + q] = sub;
      obs_row[2 * o0 + s + q] = P.n_sub + sub;
      obs_r[2 * o0 + q] = t * P.r_inv[sub];
      obs_r[2 * o0 + s + q] = t * P.r_inv[P.n_sub + sub];
    }
  }
  put(blob, B, L.obs_row, obs_row.data(), obs_row.size());
  put(blob, B, L.obs_r, obs_r.data(), obs_r.size());
  std::vector<double> obs_sr(obs_r.size());
  for (size_t o = 0; o < obs_r.size(); ++o) obs_sr[o] = std::sqrt(obs_r[o]);
  put(blob, B, L.obs_sr, obs_sr.data(), obs_sr.size());
  // merge CSR: for each actuator, the (Z row of phi_k, Z row of phi_{k-1}, weight) of every covering domain
  std::vector<int32_t> mptr(n_act + 1, 0);
  for (int q = 0; q < P.sum_e(); ++q) mptr[P.est_act[q] + 1]++;
  for (int a = 0; a < n_act; ++a) mptr[a + 1] += mptr[a];
  std::vector<int32_t> fill(mptr.begin(), mptr.end() - 1), mrow(2 * P.sum_e()), mdom(P.sum_e());
  std::vector<double> mw(P.sum_e());
  for (int l = 0; l < P.n_dom; ++l) {
    const int e0 = P.est_ptr[l], e = P.est_ptr[l + 1] - e0;
    for (int q = 0; q < e; ++q) {
      const int a = P.est_act[e0 + q];
      const int k = fill[a]++;
      mrow[2 * k] = 2 * e0 + q;
      mrow[2 * k + 1] = 2 * e0 + e + q;
      mw[k] = P.est_w[e0 + q];
      mdom[k] = l;
    }
  }
  put(blob, B, L.mptr, mptr.data(), mptr.size());
  put(blob, B, L.mrow, mrow.data(), mrow.size());
  put(blob, B, L.mw, mw.data(), mw.size());
  put(blob, B, L.mdom, mdom.data(), mdom.size());
  if (P.flags & LETKF_FLAG_PISTONS) {
    const std::vector<double> G = piston_operator(P, mptr, mdom);
    put(blob, B, L.pist_op, G.data(), G.size());
    // mismatch terms of each domain: for every actuator j of the domain, the
    // rows of all domains covering j with coefficient 1, the domain's own
    // row with 1 - k_j (k_j = domains covering j)
    std::vector<int32_t> pptr(P.n_dom + 1, 0), prow;
    std::vector<double> pcoef;
    for (int l = 0; l < P.n_dom; ++l) {
      for (int q = P.est_ptr[l]; q < P.est_ptr[l + 1]; ++q) {
        const int a = P.est_act[q];
        const int k = mptr[a + 1] - mptr[a];
        for (int x = mptr[a]; x < mptr[a + 1]; ++x) {
          prow.push_back(mrow[2 * x]);
          prow.push_back(mrow[2 * x + 1]);
          pcoef.push_back(mdom[x] == l ? 1.0 - k : 1.0);
        }
      }
      pptr[l + 1] = (int32_t)pcoef.size();
    }
    put(blob, B, L.pist_ptr, pptr.data(), pptr.size());
    put(blob, B, L.pist_row, prow.data(), prow.size());
    put(blob, B, L.pist_coef, pcoef.data(), pcoef.size());
  }

  // ---- descriptor
  std::memset(&D, 0, sizeof(D));
  D.n_act = n_act; D.n_sub = P.n_sub; D.m = m; D.n_dom = P.n_dom;
  D.prec = P.prec; D.flags = (int32_t)P.flags; D.zrows = P.zrows(); D.nnz = P.nnz;
  D.obs_inst = P.obs_instant;
  D.sigma_v = P.sigma_v;
  D.a_diag = (double)(m - 1) / P.inflation;
  D.seed = P.seed;
  D.ens = ws + L.ens; D.Yp = ws + L.Yp; D.d = (double*)(ws + L.d); D.Z = ws + L.Z;
  D.a1 = (const double*)(ws + L.a1); D.a2 = (const double*)(ws + L.a2);
  D.d_rowptr = (const int32_t*)(ws + L.rowptr); D.d_col = (const int32_t*)(ws + L.col);
  D.d_val = (const double*)(ws + L.val);
  D.dom = (const int32_t*)(ws + L.dom); D.order = (const int32_t*)(ws + L.order);
  D.est_act = (const int32_t*)(ws + L.est);
  D.obs_row = (const int32_t*)(ws + L.obs_row); D.obs_r = (const double*)(ws + L.obs_r);
  D.obs_sr = (const double*)(ws + L.obs_sr);
  D.mptr = (const int32_t*)(ws + L.mptr); D.mrow = (const int32_t*)(ws + L.mrow);
  D.mw = (const double*)(ws + L.mw);
  D.mdom = (const int32_t*)(ws + L.mdom);
  if (P.flags & LETKF_FLAG_PISTONS) {
    D.pist_op = (const double*)(ws + L.pist_op);
    D.pist_ptr = (const int32_t*)(ws + L.pist_ptr);
    D.pist_row = (const int32_t*)(ws + L.pist_row);
    D.pist_coef = (const double*)(ws + L.pist_coef);
    D.pist_r = (double*)(ws + L.pist_r);
    D.pist_c = (double*)(ws + L.pist_c);
  }
  if (L.bigA) {
    D.bigA = (double*)(ws + L.bigA);
    D.bigB = (double*)(ws + L.bigB);
    D.bigv = (double*)(ws + L.bigv);
    D.bigf = (int32_t*)(ws + L.bigf);
  }
  D.dom_sweeps = (uint32_t*)(ws + L.dom_sweeps);
  D.Ascr = L.Ascr ? (double*)(ws + L.Ascr) : nullptr;
  D.dbg = L.dbg ? (double*)(ws + L.dbg) : nullptr;
  D.dbg_sweeps = L.dbg_sweeps ? (int32_t*)(ws + L.dbg_sweeps) : nullptr;
  D.st = (InstState*)(ws + L.state);

  InstState S{};
  S.cur = 0;
  S.frame = 0;
  // single-entry batch header of the plain path
  BatchHdr H;
  std::memset(&H, 0, sizeof(H));
  H.yptr[0] = (const double*)(ws + L.y);
  H.amean = (double*)(ws + L.amean);
  H.pmean = (double*)(ws + L.pmean);
  const int cls = P.cls();
  ClassBatch& cb = H.cls[cls];
  cb.n = 1;
  cb.inst[0] = 0;
  cb.ent[0] = 0;
  cb.act_off[1] = n_act;
  cb.slope_off[1] = p;
  cb.dom_off[1] = P.n_dom;

  // ensemble: slot 0 = phi_k (rows 0..n_act-1 of X0), slot 1 = phi_{k-1}
  std::vector<char> ens(2 * (size_t)n_act * m * es);
  if (es == 8) std::memcpy(ens.data(), X0, ens.size());
  else {
    float* f = (float*)ens.data();
    for (size_t i = 0; i < 2 * (size_t)n_act * m; ++i) f[i] = (float)X0[i];
  }
  LETKF_HIP(hipMemcpyAsync(ws + L.static_begin, blob.data(), blob.size(), hipMemcpyHostToDevice, stream));
  LETKF_HIP(hipMemcpyAsync(ws + L.desc, &D, sizeof(D), hipMemcpyHostToDevice, stream));
  LETKF_HIP(hipMemcpyAsync(ws + L.state, &S, sizeof(S), hipMemcpyHostToDevice, stream));
  LETKF_HIP(hipMemcpyAsync(ws + L.hdr, &H, sizeof(H), hipMemcpyHostToDevice, stream));
  LETKF_HIP(hipMemcpyAsync(ws + L.ens, ens.data(), ens.size(), hipMemcpyHostToDevice, stream));
  LETKF_HIP(hipMemsetAsync(ws + L.dom_sweeps, 0, sizeof(uint32_t) * P.n_dom, stream));
  if (L.dbg) LETKF_HIP(hipMemsetAsync(ws + L.dbg, 0, L.total - L.dbg, stream));
  // slopes read before the first frame is staged (letkf_autotune) are zeros, not stale memory
  LETKF_HIP(hipMemsetAsync(ws + L.y, 0, sizeof(double) * P.p(), stream));
  LETKF_HIP(hipStreamSynchronize(stream));
  return LETKF_OK;
}

}  // namespace letkf

using namespace letkf;

static int check_handle(letkf_handle* h) {
  if (!h) return fail(LETKF_EINVAL, "null handle");
  if (hipSetDevice(h->device) != hipSuccess) return fail(LETKF_EDEVICE, "hipSetDevice failed");
  return LETKF_OK;
}

// Plain-path launches: not for instances driven by a server.
static int check_plain(letkf_handle* h) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->server) return fail(LETKF_ESTATE, "instance belongs to a server: use letkf_submit_frame");
  return LETKF_OK;
}

// Stream for state access: the caller's, or the server's once the instance is idle.
static int access_stream(letkf_handle* h, void* stream, hipStream_t* out) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->server) return server_idle_stream(h, out);
  *out = (hipStream_t)stream;
  return LETKF_OK;
}

static InstDesc* dev_desc(letkf_handle* h) { return (InstDesc*)(h->ws + h->L.desc); }

static constexpr size_t kTimerQuads = 1024;

static int flush_timer(letkf_handle* h) {
  for (size_t q = 0; q < h->ev_used; ++q) {
    hipEvent_t* e = &h->ev[4 * q];
    LETKF_HIP(hipEventSynchronize(e[3]));
    for (int k = 0; k < 3; ++k) {
      float ms = 0.f;
      LETKF_HIP(hipEventElapsedTime(&ms, e[k], e[k + 1]));
      h->ms_acc[k] += ms;
    }
  }
  h->ev_used = 0;
  return LETKF_OK;
}

// Records event `k` (0..3) of the current timed call on stream s.
static int mark(letkf_handle* h, int k, hipStream_t s) {
  if (!h->timing) return LETKF_OK;
  if (k == 0 && h->ev_used == kTimerQuads) {
    int rc = flush_timer(h);
    if (rc) return rc;
  }
  LETKF_HIP(hipEventRecord(h->ev[4 * h->ev_used + k], s));
  if (k == 3) {
    ++h->ev_used;
    ++h->timed_calls;
  }
  return LETKF_OK;
}
static BatchHdr* dev_hdr(letkf_handle* h) { return (BatchHdr*)(h->ws + h->L.hdr); }

// The domain analysis of the plain path: the persistent kernel with the
// tuned grid, or the launch sequence of the m > 128 class.
static void launch_domain_analysis(letkf_handle* h, hipStream_t s) {
  if (h->cls == letkf::kBigClass)
    letkf::launch_big_analysis(h->P.n_dom, h->max_rows, h->P.m, dev_desc(h), dev_hdr(h), s);
  else
    letkf::launch_analysis(h->cls, h->ana_grid, dev_desc(h), dev_hdr(h), s, letkf::analysis_fair_grid(h->ana_grid, h->num_cu));
}

namespace letkf {

// The per-XCD order with the domains of each XCD re-placed among its CUs by
// their measured cost.  With one workgroup per domain and every workgroup
// resident at once, workgroup b runs on XCD b % 8 and shares its CU with
// b +- num_cu (the dispatcher fills the CUs of an XCD breadth first; the
// workgroup indices that ran alone were recorded on the 84x84 map).  A
// domain's time grows by about 15 % of the other's while it shares a CU, so
// the domains that take the most sweeps go where they run alone (or with the
// cheapest company): greedy over decreasing cost, each to the CU of its XCD
// whose estimated finish, max + 0.15 x (sum - max) of its domains' costs,
// stays lowest, on a tie the CU that will hold the fewest domains (so the
// costliest take the CUs nobody shares).  With more domains than workgroups
// resident at once (`resident`), the workgroups claim the later domains as
// they finish: then longest first (decreasing cost) balances the tail.
// cost[l]: domain l's cost in Jacobi-sweep units.
std::vector<int32_t> balanced_order(const Problem& P, const std::vector<double>& cost, int num_cu, int resident) {
  const int n = P.n_dom;
  if (n > resident) {
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    return order;
  }
  std::vector<int32_t> order = domain_order(P, LETKF_ORDER_XCD);
  if (num_cu < kXcds || num_cu % kXcds) return order;
  constexpr double kShare = 0.15;
  for (int x = 0; x < kXcds; ++x) {
    // the CUs this XCD's positions fall on (position b: CU b % num_cu), their positions and domains
    std::vector<std::vector<int>> cu_pos;
    std::vector<int> slot_of(num_cu, -1);
    std::vector<int32_t> doms;
    for (int b = x; b < n; b += kXcds) {
      int& sl = slot_of[b % num_cu];
      if (sl < 0) {
        sl = (int)cu_pos.size();
        cu_pos.emplace_back();
      }
      cu_pos[sl].push_back(b);
      doms.push_back(order[b]);
    }
    std::stable_sort(doms.begin(), doms.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    const int ncu = (int)cu_pos.size();
    std::vector<double> mx(ncu, 0.0), sum(ncu, 0.0);
    std::vector<int> used(ncu, 0);
    for (int32_t l : doms) {
      int best = -1;
      double best_est = 0.0;
      for (int c = 0; c < ncu; ++c) {
        if (used[c] == (int)cu_pos[c].size()) continue;
        const double m2 = std::max(mx[c], cost[l]), s2 = sum[c] + cost[l];
        const double est = m2 + kShare * (s2 - m2);
        if (best < 0 || est < best_est - 1e-12 ||
            (est <= best_est + 1e-12 && cu_pos[c].size() < cu_pos[best].size())) {
          best = c;
          best_est = est;
        }
      }
      order[cu_pos[best][used[best]++]] = l;
      mx[best] = std::max(mx[best], cost[l]);
      sum[best] += cost[l];
    }
  }
  return order;
}

int upload_order(letkf_handle* h, int policy, hipStream_t s, std::vector<int32_t>* used) {
  std::vector<int32_t> order;
  if (policy == LETKF_ORDER_BALANCED) {
    // cost of a domain: its sweeps summed over the analyses so far, plus the
    // rest of its analysis, about 3.5 sweeps' worth each time
    const int n = h->P.n_dom;
    std::vector<uint32_t> sw(n);
    InstState st{};
    LETKF_HIP(hipMemcpyAsync(sw.data(), h->ws + h->L.dom_sweeps, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s));
    LETKF_HIP(hipMemcpyAsync(&st, h->ws + h->L.state, sizeof(st), hipMemcpyDeviceToHost, s));
    LETKF_HIP(hipStreamSynchronize(s));
    const double analyses = n > 0 ? (double)st.solves / n : 0.0;
    std::vector<double> cost(n);
    for (int l = 0; l < n; ++l) cost[l] = sw[l] + 3.5 * analyses;
    int num_cu = 0;
    LETKF_HIP(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, h->device));
    order = balanced_order(h->P, cost, num_cu, analysis_blocks_per_cu(h->cls) * num_cu);
  } else {
    order = domain_order(h->P, policy);
  }
  if (used) *used = order;
  return upload_order_vec(h, order, policy, s);
}

int upload_order_vec(letkf_handle* h, const std::vector<int32_t>& order, int policy, hipStream_t s) {
  // every domain exactly once: the analysis launch maps work items through it
  std::vector<char> seen(order.size(), 0);
  if ((int)order.size() != h->P.n_dom) return fail(LETKF_ESTATE, "internal: domain order of the wrong length");
  for (int32_t l : order) {
    if (l < 0 || l >= (int32_t)order.size() || seen[l]) return fail(LETKF_ESTATE, "internal: domain order is not a permutation");
    seen[l] = 1;
  }
  LETKF_HIP(hipMemcpyAsync(h->ws + h->L.order, order.data(), sizeof(int32_t) * order.size(),
                           hipMemcpyHostToDevice, s));
  LETKF_HIP(hipStreamSynchronize(s));  // `order` is a local
  h->order = policy;
  return LETKF_OK;
}

// Candidates: domain order {by decreasing cost, map order, map order in
// per-XCD chunks, and with `balanced` the per-XCD chunks placed by measured
// cost} x grid
// {ceil(k num_cu / 2), k = 1 .. 2 x (analysis workgroups per CU)} plus one
// workgroup per item, each grid capped at the item count.  Every candidate is timed with HIP events over
// `reps` analysis launches after one warm-up launch; each launch follows a
// slope launch (which zeroes the work counter).  The analysis only rewrites
// its own outputs (slope perturbations, per-domain rows, debug readback), so
// the runs are repeatable; the instances' states (ring slot, frame and sweep
// counters) are saved before and restored after.  The per-XCD order keeps
// neighbouring domains, which share observation and state rows, in one XCD's
// L2 and so reads less from HBM (about half, measured on the 84x84 map): the
// best candidate of the per-XCD orders is kept unless another order's is
// faster by more than 2 %.  The balanced order is placed by the sweeps of the
// domains so far, the tuning launches included (which all analyse the current
// frame, so its timing here favours it somewhat); the per-domain sweep sums
// are restored afterwards like the states.  max_grid > 0 caps the grids
// (candidates and default).  `balanced` is set for the plain path, whose
// launches take the progress-ordered issue priorities where
// analysis_fair_grid allows, and its candidates are timed the same way.
int tune_class(int cls, const InstDesc* tab, BatchHdr* hdr, int slope_rows, int items,
               const std::vector<letkf_handle*>& insts, int num_cu, int reps, bool balanced, int max_grid,
               hipStream_t s, letkf_tuning* res, int* grid_out) {
  if (items <= 0 || insts.empty()) return fail(LETKF_EINVAL, "nothing to tune");
  reps = std::max(1, std::min(reps, 100));
  const int bpc = analysis_blocks_per_cu(cls);
  std::vector<int> grids;
  for (int k = 1; k <= 2 * bpc; ++k) grids.push_back(std::min(items, (k * num_cu + 1) / 2));
  grids.push_back(std::min(items, 65535));  // one workgroup per item: the hardware dispatcher balances
  if (max_grid > 0)
    for (int& g : grids) g = std::min(g, max_grid);
  std::sort(grids.begin(), grids.end());
  grids.erase(std::unique(grids.begin(), grids.end()), grids.end());
  const int def_grid = std::min(items, max_grid > 0 ? std::min(bpc * num_cu, max_grid) : bpc * num_cu);

  std::vector<InstState> saved(insts.size());
  std::vector<std::vector<uint32_t>> saved_sw(insts.size());
  for (size_t i = 0; i < insts.size(); ++i) {
    LETKF_HIP(hipMemcpyAsync(&saved[i], insts[i]->ws + insts[i]->L.state, sizeof(InstState), hipMemcpyDeviceToHost, s));
    saved_sw[i].resize(insts[i]->P.n_dom);
    LETKF_HIP(hipMemcpyAsync(saved_sw[i].data(), insts[i]->ws + insts[i]->L.dom_sweeps,
                             sizeof(uint32_t) * saved_sw[i].size(), hipMemcpyDeviceToHost, s));
  }
  LETKF_HIP(hipStreamSynchronize(s));

  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LETKF_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(LETKF_EDEVICE, "hipEventCreate");
  auto time_one = [&](int grid, float* us) -> int {
    float total = 0.f;
    for (int r = 0; r <= reps; ++r) {
      launch_slopes(cls, slope_rows, tab, hdr, s);
      LETKF_HIP(hipEventRecord(e0, s));
      launch_analysis(cls, grid, tab, hdr, s, balanced ? analysis_fair_grid(grid, num_cu) : 0);
      LETKF_HIP(hipEventRecord(e1, s));
      LETKF_HIP(hipGetLastError());
      LETKF_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      LETKF_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (r > 0) total += ms;  // r = 0 is the warm-up
    }
    *us = 1e3f * total / (float)reps;
    return LETKF_OK;
  };
  float best_us = 0.f, def_us = 0.f, xcd_us = 0.f;
  int best_grid = def_grid, best_order = LETKF_ORDER_COST, xcd_grid = 0, xcd_order = LETKF_ORDER_XCD, cand = 0;
  std::vector<int> policies = {LETKF_ORDER_COST, LETKF_ORDER_MAP, LETKF_ORDER_XCD};
  if (balanced) policies.push_back(LETKF_ORDER_BALANCED);
  std::vector<std::vector<int32_t>> bal(insts.size());  // the balanced orders as timed
  for (int policy : policies) {
    if (rc) break;
    for (size_t i = 0; i < insts.size(); ++i)
      if (!rc) rc = upload_order(insts[i], policy, s, policy == LETKF_ORDER_BALANCED ? &bal[i] : nullptr);
    for (int g : grids) {
      if (rc) break;
      float us = 0.f;
      if ((rc = time_one(g, &us))) break;
      ++cand;
      if (policy == LETKF_ORDER_COST && g == def_grid) def_us = us;
      if (cand == 1 || us < best_us) { best_us = us; best_grid = g; best_order = policy; }
      const bool local = policy == LETKF_ORDER_XCD || policy == LETKF_ORDER_BALANCED;
      if (local && (xcd_grid == 0 || us < xcd_us)) { xcd_us = us; xcd_grid = g; xcd_order = policy; }
    }
  }
  if (!rc && xcd_grid > 0 && xcd_us <= 1.02f * best_us) {
    best_us = xcd_us;
    best_grid = xcd_grid;
    best_order = xcd_order;
  }
  for (size_t i = 0; i < insts.size(); ++i) {
    if (rc) break;
    if (best_order == LETKF_ORDER_BALANCED) rc = upload_order_vec(insts[i], bal[i], best_order, s);
    else rc = upload_order(insts[i], best_order, s);
  }
  // the states and sweep sums are put back whatever happened above
  int rrc = LETKF_OK;
  for (size_t i = 0; i < insts.size(); ++i) {
    if (hipMemcpyAsync(insts[i]->ws + insts[i]->L.state, &saved[i], sizeof(InstState), hipMemcpyHostToDevice, s) !=
        hipSuccess)
      rrc = fail(LETKF_EDEVICE, "state restore");
    if (hipMemcpyAsync(insts[i]->ws + insts[i]->L.dom_sweeps, saved_sw[i].data(), sizeof(uint32_t) * saved_sw[i].size(),
                       hipMemcpyHostToDevice, s) != hipSuccess)
      rrc = fail(LETKF_EDEVICE, "sweep sums restore");
  }
  if (hipStreamSynchronize(s) != hipSuccess) rrc = fail(LETKF_EDEVICE, "hipStreamSynchronize");
  if (!rc) rc = rrc;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (res) {
    res->grid = best_grid;
    res->order = best_order;
    res->blocks_per_cu = bpc;
    res->candidates = cand;
    res->best_us = best_us;
    res->default_us = def_us;
  }
  *grid_out = best_grid;
  return LETKF_OK;
}

}  // namespace letkf

extern "C" {

int letkf_workspace_size(const letkf_dims* dims, const letkf_model* model, const letkf_domain_map* map,
                         int precision, uint32_t flags, size_t* bytes) {
  if (!bytes) return fail(LETKF_EINVAL, "null bytes");
  Problem P;
  int rc = validate(dims, model, map, precision, flags, P);
  if (rc) return rc;
  *bytes = make_layout(P).total;
  return LETKF_OK;
}

int letkf_create(const letkf_dims* dims, const letkf_model* model, const letkf_domain_map* map,
                 int precision, uint32_t flags, const double* X0, void* workspace, size_t workspace_bytes,
                 void* stream, letkf_handle** out) {
  if (!out) return fail(LETKF_EINVAL, "null out");
  *out = nullptr;
  auto* h = new letkf_handle();
  int rc = validate(dims, model, map, precision, flags, h->P);
  if (rc) { delete h; return rc; }
  if (!X0) { delete h; return fail(LETKF_EINVAL, "null X0"); }
  if (!finite_all(X0, 2 * (size_t)h->P.n_act * h->P.m)) { delete h; return fail(LETKF_ENUMERIC, "non-finite X0"); }
  h->L = make_layout(h->P);
  if (!workspace) { delete h; return fail(LETKF_EINVAL, "null workspace"); }
  if (((uintptr_t)workspace & 255) != 0) { delete h; return fail(LETKF_EINVAL, "workspace must be 256-byte aligned"); }
  if (workspace_bytes < h->L.total) {
    const size_t need = h->L.total;
    delete h;
    return fail(LETKF_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  if (hipGetDevice(&h->device) != hipSuccess) { delete h; return fail(LETKF_EDEVICE, "hipGetDevice failed"); }
  h->ws = (char*)workspace;
  h->mpad = padded_members(h->P.m);
  h->cls = h->P.cls();
  rc = upload_instance(h->P, h->L, h->ws, X0, (hipStream_t)stream, h->desc);
  if (!rc) {
    int num_cu = 0;
    if (hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || num_cu < 1)
      rc = fail(LETKF_EDEVICE, "hipDeviceGetAttribute");
    h->num_cu = num_cu;
    h->ana_grid = std::min(h->P.n_dom, analysis_blocks_per_cu(h->cls) * num_cu);
    for (int l = 0; l < h->P.n_dom; ++l)
      h->max_rows = std::max(h->max_rows, 2 * (h->P.est_ptr[l + 1] - h->P.est_ptr[l]));
  }
  if (!rc && hipHostMalloc((void**)&h->h_y, sizeof(double) * h->P.p()) != hipSuccess) rc = fail(LETKF_EDEVICE, "hipHostMalloc");
  if (!rc && hipHostMalloc((void**)&h->h_out, sizeof(double) * h->P.n_act) != hipSuccess) rc = fail(LETKF_EDEVICE, "hipHostMalloc");
  if (!rc && hipEventCreateWithFlags(&h->y_free, hipEventDisableTiming) != hipSuccess) rc = fail(LETKF_EDEVICE, "hipEventCreate");
  if (rc) { letkf_destroy(h); return rc; }
  *out = h;
  return LETKF_OK;
}

int letkf_destroy(letkf_handle* h) {
  if (!h) return LETKF_OK;
  if (h->server) return fail(LETKF_ESTATE, "instance belongs to a server: use letkf_server_remove");
  // teardown: errors here cannot be acted on, the host state goes regardless
  if (h->y_free) { (void)hipEventSynchronize(h->y_free); (void)hipEventDestroy(h->y_free); }
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph_stream) (void)hipStreamDestroy(h->graph_stream);
  if (h->h_y) (void)hipHostFree(h->h_y);
  if (h->h_out) (void)hipHostFree(h->h_out);
  delete h;
  return LETKF_OK;
}

// Stage y into the device y buffer of the handle (plain path).
static int stage_y(letkf_handle* h, const double* y, int y_on_device, hipStream_t s) {
  const size_t bytes = sizeof(double) * h->P.p();
  double* dy = (double*)(h->ws + h->L.y);
  if (!y) return fail(LETKF_EINVAL, "null y");
  if (y_on_device) {
    LETKF_HIP(hipMemcpyAsync(dy, y, bytes, hipMemcpyDeviceToDevice, s));
    return LETKF_OK;
  }
  if (!finite_all(y, h->P.p())) return fail(LETKF_ENUMERIC, "non-finite slopes");
  if (h->y_pending) LETKF_HIP(hipEventSynchronize(h->y_free));
  std::memcpy(h->h_y, y, bytes);
  LETKF_HIP(hipMemcpyAsync(dy, h->h_y, bytes, hipMemcpyHostToDevice, s));
  LETKF_HIP(hipEventRecord(h->y_free, s));
  h->y_pending = true;
  return LETKF_OK;
}

static int read_means(letkf_handle* h, size_t off, double* out, hipStream_t s) {
  LETKF_HIP(hipMemcpyAsync(h->h_out, h->ws + off, sizeof(double) * h->P.n_act, hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipStreamSynchronize(s));
  std::memcpy(out, h->h_out, sizeof(double) * h->P.n_act);
  return LETKF_OK;
}

int letkf_analyse(letkf_handle* h, const double* y, int y_on_device, double* mean_out, void* stream) {
  int rc = check_plain(h);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = stage_y(h, y, y_on_device, s))) return rc;
  if ((rc = mark(h, 0, s))) return rc;
  launch_slopes(h->cls, h->P.p(), dev_desc(h), dev_hdr(h), s);
  if ((rc = mark(h, 1, s))) return rc;
  launch_domain_analysis(h, s);
  if (h->P.flags & LETKF_FLAG_PISTONS) launch_pistons(h->cls, h->P.n_dom, dev_desc(h), dev_hdr(h), s);
  if ((rc = mark(h, 2, s))) return rc;
  launch_rows(h->cls, 0, h->P.n_act, dev_desc(h), dev_hdr(h), s);
  if ((rc = mark(h, 3, s))) return rc;
  LETKF_HIP(hipGetLastError());
  if (mean_out) return read_means(h, h->L.amean, mean_out, s);
  return LETKF_OK;
}

int letkf_forecast(letkf_handle* h, void* stream) {
  int rc = check_plain(h);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int k = 0; k < 3; ++k)
    if ((rc = mark(h, k, s))) return rc;
  launch_rows(h->cls, 1, h->P.n_act, dev_desc(h), dev_hdr(h), s);
  if ((rc = mark(h, 3, s))) return rc;
  LETKF_HIP(hipGetLastError());
  return LETKF_OK;
}

// The kernels of one frame (slopes, analysis, pistons, merge + forecast,
// state advance), all reading the frame's state from the device.
static void launch_frame(letkf_handle* h, hipStream_t s) {
  launch_slopes(h->cls, h->P.p(), dev_desc(h), dev_hdr(h), s);
  launch_domain_analysis(h, s);
  if (h->P.flags & LETKF_FLAG_PISTONS) launch_pistons(h->cls, h->P.n_dom, dev_desc(h), dev_hdr(h), s);
  launch_rows(h->cls, 2, h->P.n_act, dev_desc(h), dev_hdr(h), s);
}

// Captures launch_frame on the handle's private stream into a graph.
static int capture_frame(letkf_handle* h) {
  if (!h->graph_stream) LETKF_HIP(hipStreamCreateWithFlags(&h->graph_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  LETKF_HIP(hipStreamBeginCapture(h->graph_stream, hipStreamCaptureModeThreadLocal));
  launch_frame(h, h->graph_stream);
  const hipError_t le = hipGetLastError();
  const hipError_t ee = hipStreamEndCapture(h->graph_stream, &g);
  if (le != hipSuccess || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return fail(LETKF_EDEVICE, "stream capture of the frame failed");
  }
  const hipError_t ie = hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    h->graph_exec = nullptr;
    return fail(LETKF_EDEVICE, "hipGraphInstantiate");
  }
  return LETKF_OK;
}

int letkf_step(letkf_handle* h, const double* y, int y_on_device, double* pred_out, void* stream) {
  int rc = check_plain(h);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = stage_y(h, y, y_on_device, s))) return rc;
  if ((h->P.flags & LETKF_FLAG_GRAPH) && !h->timing) {
    if (!h->graph_exec && (rc = capture_frame(h))) return rc;
    LETKF_HIP(hipGraphLaunch(h->graph_exec, s));
    if (pred_out) return read_means(h, h->L.pmean, pred_out, s);
    return LETKF_OK;
  }
  if ((rc = mark(h, 0, s))) return rc;
  launch_slopes(h->cls, h->P.p(), dev_desc(h), dev_hdr(h), s);
  if ((rc = mark(h, 1, s))) return rc;
  launch_domain_analysis(h, s);
  if (h->P.flags & LETKF_FLAG_PISTONS) launch_pistons(h->cls, h->P.n_dom, dev_desc(h), dev_hdr(h), s);
  if ((rc = mark(h, 2, s))) return rc;
  launch_rows(h->cls, 2, h->P.n_act, dev_desc(h), dev_hdr(h), s);
  if ((rc = mark(h, 3, s))) return rc;
  LETKF_HIP(hipGetLastError());
  if (pred_out) return read_means(h, h->L.pmean, pred_out, s);
  return LETKF_OK;
}

// Offsets of the frame scratch of letkf_step_noalloc in the static array.
static NoallocLayout noalloc_layout(const Problem& P) {
  NoallocLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    const size_t o = off;
    off += bytes;
    return o;
  };
  const size_t es = P.esize(), m = P.m, p = P.p();
  L.desc = take(sizeof(InstDesc));
  L.hdr = take(sizeof(BatchHdr));
  L.Yp = take(p * m * es);
  L.d = take(p * 8);
  L.Z = take((size_t)P.zrows() * m * es);
  L.Ascr = P.prec == LETKF_FP64 ? take((size_t)P.n_dom * tri_size(P.m) * 8) : 0;
  L.amean = take((size_t)P.n_act * 8);
  L.total = (off + 255) & ~size_t(255);
  return L;
}

int letkf_step_noalloc(letkf_handle* h, const double* y_dev, double* pred_dev, void* stream) {
  int rc = check_plain(h);
  if (rc) return rc;
  if (!y_dev || !pred_dev) return fail(LETKF_EINVAL, "null y_dev or pred_dev");
  if (h->cls == kBigClass) return fail(LETKF_EINVAL, "letkf_step_noalloc needs m <= 128");
  const NoallocLayout lay = noalloc_layout(h->P);
  if (lay.total > kScratchBytes)
    return fail(LETKF_EINVAL, "frame scratch of " + std::to_string(lay.total) + " bytes exceeds the static maximum of " +
                                  std::to_string(kScratchBytes) + " bytes");
  unsigned char* sp = nullptr;
  LETKF_HIP(scratch_address(h->device, &sp));  // the current device's array (check_plain set it)
  hipStream_t s = (hipStream_t)stream;
  launch_noalloc_setup(dev_desc(h), dev_hdr(h), sp, lay, y_dev, pred_dev, h->cls, s);
  const InstDesc* tab = (const InstDesc*)(sp + lay.desc);
  BatchHdr* hdr = (BatchHdr*)(sp + lay.hdr);
  launch_slopes(h->cls, h->P.p(), tab, hdr, s);
  launch_analysis(h->cls, h->ana_grid, tab, hdr, s, analysis_fair_grid(h->ana_grid, h->num_cu));
  if (h->P.flags & LETKF_FLAG_PISTONS) launch_pistons(h->cls, h->P.n_dom, tab, hdr, s);
  launch_rows(h->cls, 2, h->P.n_act, tab, hdr, s);
  LETKF_HIP(hipGetLastError());
  return LETKF_OK;
}

int letkf_get_state(letkf_handle* h, double* X_out, uint64_t* frame_out, void* stream) {
  hipStream_t s;
  int rc = access_stream(h, stream, &s);
  if (rc) return rc;
  if (!X_out) return fail(LETKF_EINVAL, "null X_out");
  const size_t n = 2 * (size_t)h->P.n_act * h->P.m, es = h->P.esize();
  std::vector<char> buf(n * es);
  InstState S;
  LETKF_HIP(hipMemcpyAsync(buf.data(), h->ws + h->L.ens, buf.size(), hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipMemcpyAsync(&S, h->ws + h->L.state, sizeof(S), hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipStreamSynchronize(s));
  const size_t slot = (size_t)h->P.n_act * h->P.m;
  for (int part = 0; part < 2; ++part) {
    const size_t src = (size_t)(part == 0 ? S.cur : (S.cur ^ 1)) * slot;
    for (size_t i = 0; i < slot; ++i)
      X_out[part * slot + i] = es == 8 ? ((double*)buf.data())[src + i] : (double)((float*)buf.data())[src + i];
  }
  if (frame_out) *frame_out = S.frame;
  return LETKF_OK;
}

int letkf_set_state(letkf_handle* h, const double* X, uint64_t frame, void* stream) {
  hipStream_t s;
  int rc = access_stream(h, stream, &s);
  if (rc) return rc;
  if (!X) return fail(LETKF_EINVAL, "null X");
  const size_t n = 2 * (size_t)h->P.n_act * h->P.m, es = h->P.esize();
  if (!finite_all(X, n)) return fail(LETKF_ENUMERIC, "non-finite state");
  std::vector<char> buf(n * es);
  if (es == 8) std::memcpy(buf.data(), X, buf.size());
  else for (size_t i = 0; i < n; ++i) ((float*)buf.data())[i] = (float)X[i];
  InstState S{};
  S.cur = 0;
  S.frame = frame;
  LETKF_HIP(hipMemcpyAsync(h->ws + h->L.ens, buf.data(), buf.size(), hipMemcpyHostToDevice, s));
  LETKF_HIP(hipMemcpyAsync(h->ws + h->L.state, &S, sizeof(S), hipMemcpyHostToDevice, s));
  LETKF_HIP(hipStreamSynchronize(s));
  return LETKF_OK;
}

int letkf_debug_domain(letkf_handle* h, int32_t domain, double* C_out, double* lam_out, double* T_out,
                       int32_t* sweeps_out, double* cycles_out, void* stream) {
  hipStream_t s;
  int rc = access_stream(h, stream, &s);
  if (rc) return rc;
  if (!(h->P.flags & LETKF_FLAG_DEBUG)) return fail(LETKF_ESTATE, "handle created without LETKF_FLAG_DEBUG");
  if (domain < 0 || domain >= h->P.n_dom) return fail(LETKF_EINVAL, "domain out of range");
  const size_t m = h->P.m, per = 2 * m * m + m + kDbgTail;
  std::vector<double> buf(per);
  int32_t sw = 0;
  LETKF_HIP(hipMemcpyAsync(buf.data(), h->ws + h->L.dbg + domain * per * 8, per * 8, hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipMemcpyAsync(&sw, h->ws + h->L.dbg_sweeps + domain * 4, 4, hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipStreamSynchronize(s));
  if (C_out) std::memcpy(C_out, buf.data(), m * m * 8);
  if (lam_out) {
    std::vector<double> lam(buf.begin() + m * m, buf.begin() + m * m + m);
    std::sort(lam.begin(), lam.end());
    std::memcpy(lam_out, lam.data(), m * 8);
  }
  if (T_out) std::memcpy(T_out, buf.data() + m * m + m, m * m * 8);
  if (sweeps_out) *sweeps_out = sw;
  if (cycles_out)
    for (int k = 0; k < 5; ++k) cycles_out[k] = buf[2 * m * m + m + k + 1] - buf[2 * m * m + m + k];
  return LETKF_OK;
}

int letkf_debug_placement(letkf_handle* h, int32_t domain, uint32_t* hw_id_out, uint32_t* xcc_id_out,
                          int32_t* workgroup_out, double* start_clock_out, void* stream) {
  hipStream_t s;
  int rc = access_stream(h, stream, &s);
  if (rc) return rc;
  if (!(h->P.flags & LETKF_FLAG_DEBUG)) return fail(LETKF_ESTATE, "handle created without LETKF_FLAG_DEBUG");
  if (domain < 0 || domain >= h->P.n_dom) return fail(LETKF_EINVAL, "domain out of range");
  if (h->P.m > 128) return fail(LETKF_EINVAL, "placement is recorded for ensembles of at most 128 members");
  const size_t m = h->P.m, per = 2 * m * m + m + kDbgTail;
  double v[9];
  LETKF_HIP(hipMemcpyAsync(v, h->ws + h->L.dbg + (domain * per + 2 * m * m + m) * 8, sizeof(v),
                           hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipStreamSynchronize(s));
  if (hw_id_out) *hw_id_out = (uint32_t)v[6];
  if (xcc_id_out) *xcc_id_out = (uint32_t)v[7];
  if (workgroup_out) *workgroup_out = (int32_t)v[8];
  if (start_clock_out) *start_clock_out = v[0];
  return LETKF_OK;
}

int letkf_debug_substeps(letkf_handle* h, int32_t domain, double* cycles_out, void* stream) {
  hipStream_t s;
  int rc = access_stream(h, stream, &s);
  if (rc) return rc;
  if (!(h->P.flags & LETKF_FLAG_DEBUG)) return fail(LETKF_ESTATE, "handle created without LETKF_FLAG_DEBUG");
  if (domain < 0 || domain >= h->P.n_dom) return fail(LETKF_EINVAL, "domain out of range");
  if (h->P.m > 128) return fail(LETKF_EINVAL, "sub-steps are recorded for ensembles of at most 128 members");
  const size_t m = h->P.m, per = 2 * m * m + m + kDbgTail;
  double v[kDbgTail];
  LETKF_HIP(hipMemcpyAsync(v, h->ws + h->L.dbg + (domain * per + 2 * m * m + m) * 8, sizeof(v),
                           hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipStreamSynchronize(s));
  // stamps 3 (Jacobi done), 10, 11, 12, 4 (wbar/W/T done)
  if (cycles_out) {
    cycles_out[0] = v[10] - v[3];
    cycles_out[1] = v[11] - v[10];
    cycles_out[2] = v[12] - v[11];
    cycles_out[3] = v[4] - v[12];
  }
  return LETKF_OK;
}

int letkf_last_means(letkf_handle* h, double* amean_out, double* pmean_out, void* stream) {
  int rc = check_plain(h);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = sizeof(double) * h->P.n_act;
  if (amean_out) LETKF_HIP(hipMemcpyAsync(h->h_out, h->ws + h->L.amean, bytes, hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipStreamSynchronize(s));
  if (amean_out) std::memcpy(amean_out, h->h_out, bytes);
  if (pmean_out) LETKF_HIP(hipMemcpyAsync(h->h_out, h->ws + h->L.pmean, bytes, hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipStreamSynchronize(s));
  if (pmean_out) std::memcpy(pmean_out, h->h_out, bytes);
  return LETKF_OK;
}

int letkf_unconverged_domains(letkf_handle* h, int32_t* count, void* stream) {
  hipStream_t s;
  int rc = access_stream(h, stream, &s);
  if (rc) return rc;
  if (!count) return fail(LETKF_EINVAL, "null count");
  InstState S;
  LETKF_HIP(hipMemcpyAsync(&S, h->ws + h->L.state, sizeof(S), hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipStreamSynchronize(s));
  *count = S.unconverged;
  return LETKF_OK;
}

int letkf_kernel_times(letkf_handle* h, int enable, double* ms_out, uint64_t* frames_out) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (h->timing && (rc = flush_timer(h))) return rc;
  if (ms_out)
    for (int k = 0; k < 3; ++k) ms_out[k] = h->ms_acc[k];
  if (frames_out) *frames_out = h->timed_calls;
  if (enable) {
    if (h->ev.empty()) {
      h->ev.resize(4 * kTimerQuads, nullptr);
      for (auto& e : h->ev) LETKF_HIP(hipEventCreate(&e));
    }
    h->ms_acc[0] = h->ms_acc[1] = h->ms_acc[2] = 0.0;
    h->timed_calls = 0;
    h->ev_used = 0;
  }
  h->timing = enable != 0;
  return LETKF_OK;
}

int letkf_autotune(letkf_handle* h, int32_t reps, letkf_tuning* out, void* stream) {
  int rc = check_plain(h);
  if (rc) return rc;
  if (h->cls == kBigClass) return fail(LETKF_ESTATE, "the launch sequence of m > 128 has no tunable shape");
  int num_cu = 0;
  LETKF_HIP(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, h->device));
  int grid = h->ana_grid;
  if ((rc = tune_class(h->cls, dev_desc(h), dev_hdr(h), h->P.p(), h->P.n_dom, {h}, num_cu, reps, true, 0,
                       (hipStream_t)stream, out, &grid)))
    return rc;
  h->ana_grid = grid;
  if (h->graph_exec) {  // the captured frame launches the old grid
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
  }
  return LETKF_OK;
}

int letkf_set_tuning(letkf_handle* h, const letkf_tuning* t, void* stream) {
  int rc = check_plain(h);
  if (rc) return rc;
  if (h->cls == kBigClass) return fail(LETKF_ESTATE, "the launch sequence of m > 128 has no tunable shape");
  if (!t || t->grid < 1 || t->grid > 65535 || t->order < LETKF_ORDER_MAP || t->order > LETKF_ORDER_BALANCED)
    return fail(LETKF_EINVAL, "tuning: grid must be in [1, 65535] and order one of LETKF_ORDER_*");
  if ((rc = upload_order(h, t->order, (hipStream_t)stream))) return rc;
  h->ana_grid = std::min(t->grid, std::max(h->P.n_dom, 1));
  if (h->graph_exec) {
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
  }
  return LETKF_OK;
}

int letkf_sweep_stats(letkf_handle* h, uint64_t* sweeps, uint64_t* domain_solves, void* stream) {
  hipStream_t s;
  int rc = access_stream(h, stream, &s);
  if (rc) return rc;
  InstState S;
  LETKF_HIP(hipMemcpyAsync(&S, h->ws + h->L.state, sizeof(S), hipMemcpyDeviceToHost, s));
  LETKF_HIP(hipStreamSynchronize(s));
  if (sweeps) *sweeps = S.sweeps;
  if (domain_solves) *domain_solves = S.solves;
  return LETKF_OK;
}

const char* letkf_strerror(int status) {
  switch (status) {
    case LETKF_OK: return "ok";
    case LETKF_EINVAL: return "invalid argument";
    case LETKF_ENOMEM: return "not enough workspace / HBM budget";
    case LETKF_EAGAIN: return "no free slot, try again";
    case LETKF_EDEVICE: return "HIP runtime error";
    case LETKF_ENUMERIC: return "non-finite input or eigensolver failure";
    case LETKF_ESTATE: return "call not valid in this state";
    default: return "unknown status";
  }
}

const char* letkf_last_error(void) { return g_last_error.c_str(); }

#ifndef LETKF_BUILD_ID
#define LETKF_BUILD_ID "unknown"
#endif
const char* letkf_build_id(void) { return LETKF_BUILD_ID; }

}  // extern "C"
