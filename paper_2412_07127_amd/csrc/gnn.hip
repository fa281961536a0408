// Learned correction of the IC(0) factor, L_pred = L_IC + GNN(A) (Eq. 2):
// node features (supplementary Table 2), graph normalization, three
// message-passing blocks (supplementary Eqs. 7-9), the corrected factor, the
// Hutchinson loss of Eq. 5 (one Rademacher probe, normalized by ||A z||^2)
// with its gradient with respect to every parameter, and Adam.
//
// The graph: nodes are the unknowns, edges the entries of L's pattern
// (tril(A), diagonal included) in L's CSR order. An edge counts at both of
// its nodes when messages are aggregated (the diagonal once); per-node sums
// run over row i of L and row i of L^T (its column i) in ascending edge
// order, so every scatter of the method is a deterministic gather.
//
// Everything is FP64: the network is tiny (904 parameters, hidden width 8)
// and its passes are bound by memory traffic and latency, not arithmetic.
// Parameter gradients are summed per block over fixed edge (node) chunks in
// tile order, then folded over blocks in block order: deterministic.
#include <cmath>

#include "internal.hpp"

namespace icpcg {

namespace {

constexpr int kB = 256;
constexpr int ND = 9;          // node width
constexpr int NH = 8;          // hidden width
constexpr int NIN = ND + 2;    // node updater input [x, sum, mean]
constexpr int kTile = 32;      // rows per LDS tile in the gradient sums
constexpr double kGnEps = 1e-5;

constexpr int edge_in(int b) { return b == 0 ? 1 : 2; }
constexpr int edge_din(int b) { return edge_in(b) + 2 * ND; }
constexpr int edge_np(int b) { return NH * edge_din(b) + NH + NH + 1; }
constexpr int kNodeNp = NH * NIN + NH + ND * NH + ND;
// storage order: normalization (alpha, gamma, beta), edge 0, node 0, edge 1,
// node 1, edge 2
constexpr int kOffE0 = 3 * ND;
constexpr int kOffN0 = kOffE0 + edge_np(0);
constexpr int kOffE1 = kOffN0 + kNodeNp;
constexpr int kOffN1 = kOffE1 + edge_np(1);
constexpr int kOffE2 = kOffN1 + kNodeNp;
constexpr int kNumParams = kOffE2 + edge_np(2);
static_assert(kNumParams == 904, "parameter layout");
constexpr int off_edge(int b) { return b == 0 ? kOffE0 : b == 1 ? kOffE1 : kOffE2; }
constexpr int off_node(int b) { return b == 0 ? kOffN0 : kOffN1; }

unsigned grid_for(int64_t n, int per_thread = 1) {
  int64_t g = (n + (int64_t)kB * per_thread - 1) / ((int64_t)kB * per_thread);
  if (g > 65535) g = 65535;
  return (unsigned)(g < 1 ? 1 : g);
}

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

// ------------------------------------------------------------------ setup

// Row i of L must be exactly tril of row i of A (same columns, in order);
// the edge inputs are A's entries on that pattern.
__global__ void k_edge_setup(const int64_t *__restrict__ arp, const int32_t *__restrict__ aci,
                             const double *__restrict__ av, const int64_t *__restrict__ lrp,
                             const int32_t *__restrict__ lci, int64_t n, int32_t *__restrict__ erow,
                             double *__restrict__ aedge, int *bad) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const int64_t s = arp[i], m = lrp[i + 1] - lrp[i], la = arp[i + 1] - s;
    bool ok = la >= m && (la == m || aci[s + m] > i);
    for (int64_t t = 0; t < m; ++t) {
      const int64_t k = lrp[i] + t;
      if (ok && aci[s + t] != lci[k]) ok = false;
      aedge[k] = av[s + (t < la ? t : 0)];
      erow[k] = (int32_t)i;
    }
    if (!ok) __hip_atomic_fetch_or(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_deg_inc(const int64_t *__restrict__ lrp, const int64_t *__restrict__ urp, int64_t n,
                          double *__restrict__ deg) {
  for (int64_t i = gtid(); i < n; i += gstride())
    deg[i] = (double)((lrp[i + 1] - lrp[i]) + (urp[i + 1] - urp[i]) - 1);
}

// Node features (supplementary Table 2): degree; max, min, mean and variance
// of the neighbours' degrees; dominance |a_ii| / sum_j |a_ij|; decay
// max_{j != i} |a_ij| / |a_ii|; sin and cos of pi i / n.
__global__ void k_features(const int64_t *__restrict__ arp, const int32_t *__restrict__ aci,
                           const double *__restrict__ av, int64_t n, double *__restrict__ x) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const int64_t s = arp[i], e = arp[i + 1];
    double mx = 0.0, mn = 0.0, sum = 0.0, absum = 0.0, diag = 0.0, offmax = 0.0;
    int64_t cnt = 0;
    for (int64_t t = s; t < e; ++t) {
      const int64_t j = aci[t];
      const double a = fabs(av[t]);
      absum += a;
      if (j == i) {
        diag = a;
      } else {
        const double dj = (double)(arp[j + 1] - arp[j] - 1);
        mx = cnt == 0 ? dj : fmax(mx, dj);
        mn = cnt == 0 ? dj : fmin(mn, dj);
        offmax = cnt == 0 ? a : fmax(offmax, a);
        sum += dj;
        ++cnt;
      }
    }
    double mean = 0.0, var = 0.0;
    if (cnt > 0) {
      mean = sum / (double)cnt;
      for (int64_t t = s; t < e; ++t) {
        const int64_t j = aci[t];
        if (j == i) continue;
        const double dd = (double)(arp[j + 1] - arp[j] - 1) - mean;
        var += dd * dd;
      }
      var /= (double)cnt;
    }
    const double ang = (M_PI * (double)i) / (double)n;
    double *xi = x + i * ND;
    xi[0] = (double)(e - s - 1);
    xi[1] = mx;
    xi[2] = mn;
    xi[3] = mean;
    xi[4] = var;
    xi[5] = diag / absum;
    xi[6] = cnt > 0 ? offmax / diag : 0.0;
    xi[7] = sin(ang);
    xi[8] = cos(ang);
  }
}

// ------------------------------------------------------ column reductions

// partials[block * K + k] = sum over the block's rows of in[row * K + k]
// (rows split in contiguous chunks; each thread sums its strided rows, then a
// fixed tree over the block). Optional elementwise square.
template <int K, bool SQ>
__global__ __launch_bounds__(kB) void k_colsum(const double *__restrict__ in, int64_t rows, int64_t chunk,
                                               double *__restrict__ partials) {
  __shared__ double sm[K][kB];
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kB) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double v = in[r * K + k];
      acc[k] += SQ ? v * v : v;
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) sm[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int st = kB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
#pragma unroll
      for (int k = 0; k < K; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + st];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < K) partials[(int64_t)blockIdx.x * K + threadIdx.x] = sm[threadIdx.x][0];
}

// out[k] = sum over nb blocks of partials[b * K + k], in block order.
__global__ void k_fold(const double *__restrict__ partials, int nb, int K, double *__restrict__ out) {
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += partials[(int64_t)b * K + k];
    out[k] = acc;
  }
}

// ------------------------------------------------------- normalization

// d = x - alpha * mu with mu = colsum / n; writes d.
__global__ void k_gn_center(const double *__restrict__ x, const double *__restrict__ xsum, int64_t n,
                            const double *__restrict__ theta, double *__restrict__ mu, double *__restrict__ d) {
  for (int64_t t = gtid(); t < n * ND; t += gstride()) {
    const int f = (int)(t % ND);
    const double m = xsum[f] / (double)n;
    if (t < ND) mu[t] = m;
    d[t] = x[t] - theta[f] * m;
  }
}

// h0 = gamma * d / sd + beta with sd = sqrt(sum d^2 / n + eps).
__global__ void k_gn_apply(const double *__restrict__ d, const double *__restrict__ dsq, int64_t n,
                           const double *__restrict__ theta, double *__restrict__ sd, double *__restrict__ h) {
  for (int64_t t = gtid(); t < n * ND; t += gstride()) {
    const int f = (int)(t % ND);
    const double s = sqrt(dsq[f] / (double)n + kGnEps);
    if (t < ND) sd[t] = s;
    h[t] = theta[ND + f] * d[t] / s + theta[2 * ND + f];
  }
}

// --------------------------------------------------------------- forward

// Edge updater of block B: e = w2 . tanh(W1 [e_in, h_row, h_col] + b1) + b2.
template <int B>
__global__ __launch_bounds__(kB) void k_edge_fwd(const int32_t *__restrict__ erow, const int32_t *__restrict__ ecol,
                                                 int64_t nnz, const double *__restrict__ e0,
                                                 const double *__restrict__ eprev, const double *__restrict__ h,
                                                 const double *__restrict__ theta, double *__restrict__ q_out,
                                                 double *__restrict__ e_out) {
  constexpr int DIN = edge_din(B), EIN = edge_in(B);
  const double *W1 = theta + off_edge(B);
  const double *b1 = W1 + NH * DIN;
  const double *w2 = b1 + NH;
  const double b2 = w2[NH];
  for (int64_t k = gtid(); k < nnz; k += gstride()) {
    double in[DIN];
    in[0] = e0[k];
    if (EIN == 2) in[1] = eprev[k];
    const double *hr = h + (int64_t)erow[k] * ND;
    const double *hc = h + (int64_t)ecol[k] * ND;
#pragma unroll
    for (int f = 0; f < ND; ++f) {
      in[EIN + f] = hr[f];
      in[EIN + ND + f] = hc[f];
    }
    double e = 0.0;
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      double p = 0.0;
#pragma unroll
      for (int m = 0; m < DIN; ++m) p += in[m] * W1[j * DIN + m];
      const double q = tanh(p + b1[j]);
      if (q_out) q_out[k * NH + j] = q;
      e += q * w2[j];
    }
    e_out[k] = e + b2;
  }
}

// Sum of the edge values incident to node i: row i of L (ascending), then its
// column i without the diagonal (row i of L^T, diagonal first, skipped).
__device__ __forceinline__ double incident_sum(int64_t i, const int64_t *lrp, const int64_t *urp,
                                               const int32_t *upos, const double *e) {
  double sr = 0.0, sc = 0.0;
  for (int64_t k = lrp[i]; k < lrp[i + 1]; ++k) sr += e[k];
  for (int64_t t = urp[i] + 1; t < urp[i + 1]; ++t) sc += e[upos[t]];
  return sr + sc;
}

// Node updater of block B: h' = W2 tanh(W1 [h, sum, mean] + b1) + b2.
template <int B>
__global__ __launch_bounds__(kB) void k_node_fwd(const int64_t *__restrict__ lrp, const int64_t *__restrict__ urp,
                                                 const int32_t *__restrict__ upos, int64_t n,
                                                 const double *__restrict__ deg, const double *__restrict__ e,
                                                 const double *__restrict__ h, const double *__restrict__ theta,
                                                 double *__restrict__ nin_out, double *__restrict__ Q_out,
                                                 double *__restrict__ h_out) {
  const double *W1 = theta + off_node(B);
  const double *b1 = W1 + NH * NIN;
  const double *W2 = b1 + NH;
  const double *b2 = W2 + ND * NH;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    double in[NIN];
#pragma unroll
    for (int f = 0; f < ND; ++f) in[f] = h[i * ND + f];
    const double s = incident_sum(i, lrp, urp, upos, e);
    in[ND] = s;
    in[ND + 1] = s / deg[i];
    if (nin_out) {
#pragma unroll
      for (int m = 0; m < NIN; ++m) nin_out[i * NIN + m] = in[m];
    }
    double Q[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      double p = 0.0;
#pragma unroll
      for (int m = 0; m < NIN; ++m) p += in[m] * W1[j * NIN + m];
      Q[j] = tanh(p + b1[j]);
      if (Q_out) Q_out[i * NH + j] = Q[j];
    }
#pragma unroll
    for (int f = 0; f < ND; ++f) {
      double o = 0.0;
#pragma unroll
      for (int j = 0; j < NH; ++j) o += Q[j] * W2[f * NH + j];
      h_out[i * ND + f] = o + b2[f];
    }
  }
}

// Eq. 2 with a positive diagonal: off the diagonal L = L_IC + sqrt(s) g, on
// it L = L_IC exp(g / 2).
__global__ void k_assemble(const int32_t *__restrict__ erow, const int32_t *__restrict__ ecol, int64_t nnz,
                           const double *__restrict__ lic, const double *__restrict__ g, double sqrt_s,
                           double *__restrict__ L) {
  for (int64_t k = gtid(); k < nnz; k += gstride())
    L[k] = erow[k] == ecol[k] ? lic[k] * exp(g[k] / 2.0) : lic[k] + sqrt_s * g[k];
}

// ------------------------------------------------------------------ loss

// y = A z (row i in entry order).
__global__ void k_csr_mv(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const double *__restrict__ v, int64_t n, const double *__restrict__ z,
                         double *__restrict__ y) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    double acc = 0.0;
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) acc += v[t] * z[ci[t]];
    y[i] = acc;
  }
}

// y = L^T z through row i of L^T: sum over the entries of column i of L in
// ascending edge order.
__global__ void k_lt_mv(const int64_t *__restrict__ urp, const int32_t *__restrict__ uci,
                        const int32_t *__restrict__ upos, const double *__restrict__ L, int64_t n,
                        const double *__restrict__ z, double *__restrict__ y) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    double acc = 0.0;
    for (int64_t t = urp[i]; t < urp[i + 1]; ++t) acc += L[upos[t]] * z[uci[t]];
    y[i] = acc;
  }
}

// r = llz - az; rows of [r^2, az^2] for the two sums.
__global__ void k_resid(const double *__restrict__ llz, const double *__restrict__ az, int64_t n,
                        double *__restrict__ r, double *__restrict__ sq2) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const double ri = llz[i] - az[i];
    r[i] = ri;
    sq2[2 * i] = ri * ri;
    sq2[2 * i + 1] = az[i] * az[i];
  }
}

__global__ void k_loss_out(const double *__restrict__ sums, double *__restrict__ loss, int accumulate) {
  const double l = sums[0] / sums[1];
  loss[0] = accumulate ? loss[0] + l : l;
}

// d loss / d g per edge: dL = 2 / den (r_a u_b + z_a (L^T r)_b), then through
// the assembly.
__global__ void k_dout(const int32_t *__restrict__ erow, const int32_t *__restrict__ ecol, int64_t nnz,
                       const double *__restrict__ L, const double *__restrict__ r, const double *__restrict__ u,
                       const double *__restrict__ z, const double *__restrict__ ltr, const double *__restrict__ sums,
                       double sqrt_s, double *__restrict__ dout) {
  const double c = 2.0 / sums[1];
  for (int64_t k = gtid(); k < nnz; k += gstride()) {
    const int64_t a = erow[k], b = ecol[k];
    const double dL = c * (r[a] * u[b] + z[a] * ltr[b]);
    dout[k] = a == b ? dL * L[k] / 2.0 : dL * sqrt_s;
  }
}

// -------------------------------------------------------------- backward

// Edge updater of block B, per edge: dp = (de w2) (1 - q^2); d input = W1^T dp
// split into the row node's part, the column node's part and (B > 0) the
// previous block's edge value.
template <int B>
__global__ __launch_bounds__(kB) void k_edge_bwd(int64_t nnz, const double *__restrict__ de,
                                                 const double *__restrict__ q, const double *__restrict__ theta,
                                                 double *__restrict__ dp_out, double *__restrict__ dhr,
                                                 double *__restrict__ dhc, double *__restrict__ deprev) {
  constexpr int DIN = edge_din(B), EIN = edge_in(B);
  const double *W1 = theta + off_edge(B);
  const double *w2 = W1 + NH * DIN + NH;
  for (int64_t k = gtid(); k < nnz; k += gstride()) {
    double dp[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      const double qj = q[k * NH + j];
      dp[j] = de[k] * w2[j] * (1.0 - qj * qj);
      dp_out[k * NH + j] = dp[j];
    }
#pragma unroll
    for (int m = 1; m < DIN; ++m) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < NH; ++j) acc += dp[j] * W1[j * DIN + m];
      if (EIN == 2 && m == 1) deprev[k] = acc;
      else if (m < EIN + ND) dhr[k * ND + (m - EIN)] = acc;
      else dhc[k * ND + (m - EIN - ND)] = acc;
    }
  }
}

// dh_i = dh_direct_i + (row parts of the edges of row i of L, ascending)
//        + (column parts of the edges of column i of L, ascending).
__global__ void k_node_gather(const int64_t *__restrict__ lrp, const int64_t *__restrict__ urp,
                              const int32_t *__restrict__ upos, int64_t n, const double *__restrict__ direct,
                              const double *__restrict__ dhr, const double *__restrict__ dhc,
                              double *__restrict__ dh) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    double acc[ND];
#pragma unroll
    for (int f = 0; f < ND; ++f) acc[f] = direct ? direct[i * ND + f] : 0.0;
    for (int64_t k = lrp[i]; k < lrp[i + 1]; ++k) {
#pragma unroll
      for (int f = 0; f < ND; ++f) acc[f] += dhr[k * ND + f];
    }
    for (int64_t t = urp[i]; t < urp[i + 1]; ++t) {
      const int64_t k = upos[t];
#pragma unroll
      for (int f = 0; f < ND; ++f) acc[f] += dhc[k * ND + f];
    }
#pragma unroll
    for (int f = 0; f < ND; ++f) dh[i * ND + f] = acc[f];
  }
}

// Node updater of block B, per node: dP = (W2^T dh) (1 - Q^2);
// d input = W1^T dP -> direct node part and ds = d sum + d mean / deg.
template <int B>
__global__ __launch_bounds__(kB) void k_node_bwd(int64_t n, const double *__restrict__ dh,
                                                 const double *__restrict__ Q, const double *__restrict__ deg,
                                                 const double *__restrict__ theta, double *__restrict__ dP_out,
                                                 double *__restrict__ direct, double *__restrict__ ds) {
  const double *W1 = theta + off_node(B);
  const double *W2 = W1 + NH * NIN + NH;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    double dP[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int f = 0; f < ND; ++f) acc += dh[i * ND + f] * W2[f * NH + j];
      const double Qj = Q[i * NH + j];
      dP[j] = acc * (1.0 - Qj * Qj);
      dP_out[i * NH + j] = dP[j];
    }
    double din[NIN];
#pragma unroll
    for (int m = 0; m < NIN; ++m) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < NH; ++j) acc += dP[j] * W1[j * NIN + m];
      din[m] = acc;
    }
#pragma unroll
    for (int f = 0; f < ND; ++f) direct[i * ND + f] = din[f];
    ds[i] = din[ND] + din[ND + 1] / deg[i];
  }
}

// Edge value gradient of the previous block: its skip-input part plus the
// aggregation at both ends (the diagonal once).
__global__ void k_edge_de(const int32_t *__restrict__ erow, const int32_t *__restrict__ ecol, int64_t nnz,
                          const double *__restrict__ deprev, const double *__restrict__ ds,
                          double *__restrict__ de) {
  for (int64_t k = gtid(); k < nnz; k += gstride()) {
    const int64_t a = erow[k], b = ecol[k];
    de[k] = deprev[k] + ds[a] + (a == b ? 0.0 : ds[b]);
  }
}

// Parameter gradients of edge block B over a chunk of edges: tiles of kTile
// edges are staged in LDS (dp, q, de and the rebuilt input), then thread t
// sums parameter t over the tile's edges in order.
template <int B>
__global__ __launch_bounds__(kB) void k_edge_pgrad(const int32_t *__restrict__ erow,
                                                   const int32_t *__restrict__ ecol, int64_t nnz, int64_t chunk,
                                                   const double *__restrict__ e0, const double *__restrict__ eprev,
                                                   const double *__restrict__ h, const double *__restrict__ de,
                                                   const double *__restrict__ q, const double *__restrict__ dp,
                                                   double *__restrict__ partials) {
  constexpr int DIN = edge_din(B), EIN = edge_in(B), NP = edge_np(B);
  constexpr int ROW = DIN + 2 * NH + 1;
  __shared__ double tile[kTile][ROW];
  const int t = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * chunk;
  const int64_t k1 = k0 + chunk < nnz ? k0 + chunk : nnz;
  double acc = 0.0;
  for (int64_t base = k0; base < k1; base += kTile) {
    const int cnt = (int)(k1 - base < kTile ? k1 - base : kTile);
    for (int idx = t; idx < cnt * ROW; idx += kB) {
      const int e = idx / ROW, m = idx % ROW;
      const int64_t k = base + e;
      double v;
      if (m == 0) v = e0[k];
      else if (EIN == 2 && m == 1) v = eprev[k];
      else if (m < EIN + ND) v = h[(int64_t)erow[k] * ND + (m - EIN)];
      else if (m < DIN) v = h[(int64_t)ecol[k] * ND + (m - EIN - ND)];
      else if (m < DIN + NH) v = dp[k * NH + (m - DIN)];
      else if (m < DIN + 2 * NH) v = q[k * NH + (m - DIN - NH)];
      else v = de[k];
      tile[e][m] = v;
    }
    __syncthreads();
    if (t < NP) {
      for (int e = 0; e < cnt; ++e) {
        const double *row = tile[e];
        double c;
        if (t < NH * DIN) c = row[DIN + t / DIN] * row[t % DIN];              // W1[j][m]: dp_j in_m
        else if (t < NH * DIN + NH) c = row[DIN + (t - NH * DIN)];             // b1[j]: dp_j
        else if (t < NH * DIN + 2 * NH) c = row[DIN + 2 * NH] * row[DIN + NH + (t - NH * DIN - NH)];  // w2: de q_j
        else c = row[DIN + 2 * NH];                                           // b2: de
        acc += c;
      }
    }
    __syncthreads();
  }
  if (t < NP) partials[(int64_t)blockIdx.x * NP + t] = acc;
}

// Parameter gradients of node block B over a chunk of nodes (same scheme):
// W1 (dP nin), b1 (dP), W2 (dh Q), b2 (dh).
template <int B>
__global__ __launch_bounds__(kB) void k_node_pgrad(int64_t n, int64_t chunk, const double *__restrict__ nin,
                                                   const double *__restrict__ Q, const double *__restrict__ dP,
                                                   const double *__restrict__ dh, double *__restrict__ partials) {
  constexpr int ROW = NIN + NH + NH + ND;
  __shared__ double tile[kTile][ROW];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
  double acc = 0.0;
  for (int64_t base = i0; base < i1; base += kTile) {
    const int cnt = (int)(i1 - base < kTile ? i1 - base : kTile);
    for (int idx = t; idx < cnt * ROW; idx += kB) {
      const int e = idx / ROW, m = idx % ROW;
      const int64_t i = base + e;
      double v;
      if (m < NIN) v = nin[i * NIN + m];
      else if (m < NIN + NH) v = Q[i * NH + (m - NIN)];
      else if (m < NIN + 2 * NH) v = dP[i * NH + (m - NIN - NH)];
      else v = dh[i * ND + (m - NIN - 2 * NH)];
      tile[e][m] = v;
    }
    __syncthreads();
    if (t < kNodeNp) {
      for (int e = 0; e < cnt; ++e) {
        const double *row = tile[e];
        const double *rQ = row + NIN, *rdP = row + NIN + NH, *rdh = row + NIN + 2 * NH;
        double c;
        if (t < NH * NIN) c = rdP[t / NIN] * row[t % NIN];
        else if (t < NH * NIN + NH) c = rdP[t - NH * NIN];
        else if (t < NH * NIN + NH + ND * NH) {
          const int u = t - NH * NIN - NH;
          c = rdh[u / NH] * rQ[u % NH];
        } else c = rdh[t - NH * NIN - NH - ND * NH];
        acc += c;
      }
    }
    __syncthreads();
  }
  if (t < kNodeNp) partials[(int64_t)blockIdx.x * kNodeNp + t] = acc;
}

// grad[off + t] (+)= sum over blocks of partials[b * np + t], in block order.
__global__ void k_pfold(const double *__restrict__ partials, int nb, int np, double *__restrict__ grad, int accumulate) {
  for (int t = threadIdx.x; t < np; t += blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += partials[(int64_t)b * np + t];
    grad[t] = accumulate ? grad[t] + acc : acc;
  }
}

// Normalization backward, first pass: rows [dh, dh d / sd, dh gamma d].
__global__ void k_gn_bwd_rows(const double *__restrict__ dh, const double *__restrict__ d,
                              const double *__restrict__ sd, const double *__restrict__ theta, int64_t n,
                              double *__restrict__ rows) {
  for (int64_t t = gtid(); t < n * ND; t += gstride()) {
    const int64_t i = t / ND;
    const int f = (int)(t % ND);
    rows[i * 3 * ND + f] = dh[t];
    rows[i * 3 * ND + ND + f] = dh[t] * d[t] / sd[f];
    rows[i * 3 * ND + 2 * ND + f] = dh[t] * theta[ND + f] * d[t];
  }
}

// second pass: dd = dh gamma / sd + dsd d / (n sd) with dsd = -sum(dh gamma d) / sd^2.
__global__ void k_gn_bwd_dd(const double *__restrict__ dh, const double *__restrict__ d,
                            const double *__restrict__ sd, const double *__restrict__ sums3,
                            const double *__restrict__ theta, int64_t n, double *__restrict__ dd) {
  for (int64_t t = gtid(); t < n * ND; t += gstride()) {
    const int f = (int)(t % ND);
    const double dsd = sums3[2 * ND + f] * (-1.0 / (sd[f] * sd[f]));
    dd[t] = dh[t] * theta[ND + f] / sd[f] + dsd * d[t] / ((double)n * sd[f]);
  }
}

// alpha: -mu sum(dd); gamma: sum(dh d / sd); beta: sum(dh).
__global__ void k_gn_grad(const double *__restrict__ sums3, const double *__restrict__ sumdd,
                          const double *__restrict__ mu, double *__restrict__ grad, int accumulate) {
  const int f = threadIdx.x;
  if (f >= ND) return;
  const double ga = -(sumdd[f]) * mu[f], gg = sums3[ND + f], gb = sums3[f];
  grad[f] = accumulate ? grad[f] + ga : ga;
  grad[ND + f] = accumulate ? grad[ND + f] + gg : gg;
  grad[2 * ND + f] = accumulate ? grad[2 * ND + f] + gb : gb;
}

__global__ void k_adam(double *__restrict__ th, const double *__restrict__ g, double *__restrict__ m,
                       double *__restrict__ v, int64_t count, double lr, double b1, double b2, double eps,
                       double c1, double c2) {
  for (int64_t k = gtid(); k < count; k += gstride()) {
    const double mk = b1 * m[k] + (1.0 - b1) * g[k];
    const double vk = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    m[k] = mk;
    v[k] = vk;
    th[k] = th[k] - lr * (mk / c1) / (sqrt(vk / c2) + eps);
  }
}

// out = (in - sub) / div
__global__ void k_div(const double *__restrict__ in, int64_t count, double sub, double div, double *__restrict__ out) {
  for (int64_t k = gtid(); k < count; k += gstride()) out[k] = (in[k] - sub) / div;
}

}  // namespace

// ------------------------------------------------------------------ host

int gnn_num_params() { return kNumParams; }

namespace {

// Column sums of a rows x K row-major array into out[K] (device), two launches.
template <int K, bool SQ>
int colsum(const double *in, int64_t rows, DevBuf &partials, double *out, hipStream_t s) {
  int64_t nb = (rows + 4095) / 4096;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  const int64_t chunk = (rows + nb - 1) / nb;
  nb = (rows + chunk - 1) / chunk;
  if (nb < 1) nb = 1;
  if (partials.reserve((size_t)nb * K * 8)) return ICPCG_E_NOMEM;
  hipLaunchKernelGGL((k_colsum<K, SQ>), dim3((unsigned)nb), dim3(kB), 0, s, in, rows, chunk, partials.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(64), 0, s, partials.as<double>(), (int)nb, K, out);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

// Blocks and rows per block of the parameter-gradient sums.
int chunks_for(int64_t rows, int64_t *chunk) {
  int64_t nb = (rows + 2047) / 2048;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  *chunk = (rows + nb - 1) / nb;
  nb = (rows + *chunk - 1) / *chunk;
  return (int)(nb < 1 ? 1 : nb);
}

int reserve_all(icpcg_gnn *G, bool train) {
  const size_t n = (size_t)G->n, nnz = (size_t)G->nnz;
  if (G->d.reserve(n * ND * 8) || G->mu.reserve(ND * 8) || G->sd.reserve(ND * 8) || G->L.reserve(nnz * 8))
    return ICPCG_E_NOMEM;
  for (int b = 0; b < 3; ++b)
    if (G->h[b].reserve(n * ND * 8) || G->e[b].reserve(nnz * 8)) return ICPCG_E_NOMEM;
  if (!train) return ICPCG_OK;
  for (int b = 0; b < 3; ++b)
    if (G->q[b].reserve(nnz * NH * 8)) return ICPCG_E_NOMEM;
  for (int b = 0; b < 2; ++b)
    if (G->nin[b].reserve(n * NIN * 8) || G->Q[b].reserve(n * NH * 8)) return ICPCG_E_NOMEM;
  if (G->az.reserve(n * 8) || G->u.reserve(n * 8) || G->llz.reserve(n * 8) || G->r.reserve(n * 8) ||
      G->ltr.reserve(n * 8) || G->sq2.reserve(n * 16) || G->sums.reserve(64 * 8) || G->dout.reserve(nnz * 8) ||
      G->de.reserve(nnz * 8) || G->deprev.reserve(nnz * 8) || G->dhr.reserve(nnz * ND * 8) ||
      G->dhc.reserve(nnz * ND * 8) || G->dp.reserve(nnz * NH * 8) || G->dh.reserve(n * ND * 8) ||
      G->direct.reserve(n * ND * 8) || G->ds.reserve(n * 8) || G->dP.reserve(n * NH * 8) ||
      G->rows3.reserve(n * 3 * ND * 8) || G->dd.reserve(n * ND * 8))
    return ICPCG_E_NOMEM;
  return ICPCG_OK;
}

template <int B>
int edge_fwd(icpcg_gnn *G, const double *theta, bool keep, hipStream_t s) {
  const icpcg_prec *P = G->P;
  hipLaunchKernelGGL(k_edge_fwd<B>, dim3(grid_for(G->nnz)), dim3(kB), 0, s, G->erow.as<int32_t>(),
                     P->lci.as<int32_t>(), G->nnz, G->e0.as<double>(), B > 0 ? G->e[B > 0 ? B - 1 : 0].as<double>()
                                                                              : nullptr,
                     G->h[B].as<double>(), theta, keep ? G->q[B].as<double>() : nullptr, G->e[B].as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

template <int B>
int node_fwd(icpcg_gnn *G, const double *theta, bool keep, hipStream_t s) {
  const icpcg_prec *P = G->P;
  hipLaunchKernelGGL(k_node_fwd<B>, dim3(grid_for(G->n)), dim3(kB), 0, s, P->lrp.as<int64_t>(), P->urp.as<int64_t>(),
                     P->upos.as<int32_t>(), G->n, G->deg.as<double>(), G->e[B].as<double>(), G->h[B].as<double>(),
                     theta, keep ? G->nin[B].as<double>() : nullptr, keep ? G->Q[B].as<double>() : nullptr,
                     G->h[B + 1].as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

// Edge block B backward: de (this block's output gradient) -> parameter
// gradients, row / column node parts, and (B > 0) the previous edge value's.
template <int B>
int edge_bwd(icpcg_gnn *G, const double *theta, const double *de, double *grad, bool accumulate, hipStream_t s) {
  const icpcg_prec *P = G->P;
  const int64_t nnz = G->nnz;
  hipLaunchKernelGGL(k_edge_bwd<B>, dim3(grid_for(nnz)), dim3(kB), 0, s, nnz, de, G->q[B].as<double>(), theta,
                     G->dp.as<double>(), G->dhr.as<double>(), G->dhc.as<double>(), G->deprev.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  int64_t chunk = 0;
  const int nb = chunks_for(nnz, &chunk);
  constexpr int NP = edge_np(B);
  if (G->pp.reserve((size_t)nb * NP * 8)) return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_edge_pgrad<B>, dim3(nb), dim3(kB), 0, s, G->erow.as<int32_t>(), P->lci.as<int32_t>(), nnz,
                     chunk, G->e0.as<double>(), B > 0 ? G->e[B > 0 ? B - 1 : 0].as<double>() : nullptr,
                     G->h[B].as<double>(), de, G->q[B].as<double>(), G->dp.as<double>(), G->pp.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_pfold, dim3(1), dim3(kB), 0, s, G->pp.as<double>(), nb, NP, grad + off_edge(B),
                     accumulate ? 1 : 0);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int node_gather(icpcg_gnn *G, const double *direct, hipStream_t s) {
  const icpcg_prec *P = G->P;
  hipLaunchKernelGGL(k_node_gather, dim3(grid_for(G->n)), dim3(kB), 0, s, P->lrp.as<int64_t>(), P->urp.as<int64_t>(),
                     P->upos.as<int32_t>(), G->n, direct, G->dhr.as<double>(), G->dhc.as<double>(),
                     G->dh.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

// Node block B backward from dh (gradient of its output state): parameter
// gradients, the direct gradient of its input state, and the gradient of the
// previous edge values through the aggregation (into G->de).
template <int B>
int node_bwd(icpcg_gnn *G, const double *theta, double *grad, bool accumulate, hipStream_t s) {
  const icpcg_prec *P = G->P;
  const int64_t n = G->n;
  hipLaunchKernelGGL(k_node_bwd<B>, dim3(grid_for(n)), dim3(kB), 0, s, n, G->dh.as<double>(), G->Q[B].as<double>(),
                     G->deg.as<double>(), theta, G->dP.as<double>(), G->direct.as<double>(), G->ds.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  int64_t chunk = 0;
  const int nb = chunks_for(n, &chunk);
  if (G->pp.reserve((size_t)nb * kNodeNp * 8)) return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_node_pgrad<B>, dim3(nb), dim3(kB), 0, s, n, chunk, G->nin[B].as<double>(),
                     G->Q[B].as<double>(), G->dP.as<double>(), G->dh.as<double>(), G->pp.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_pfold, dim3(1), dim3(kB), 0, s, G->pp.as<double>(), nb, kNodeNp, grad + off_node(B),
                     accumulate ? 1 : 0);
  ICPCG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_edge_de, dim3(grid_for(G->nnz)), dim3(kB), 0, s, G->erow.as<int32_t>(), P->lci.as<int32_t>(),
                     G->nnz, G->deprev.as<double>(), G->ds.as<double>(), G->de.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

}  // namespace

int gnn_setup(icpcg_gnn *G, const icpcg_csr *A, const icpcg_prec *P, hipStream_t s) {
  const int64_t n = P->n, nnz = P->nnz;
  G->n = n;
  G->nnz = nnz;
  G->A = *A;
  G->P = P;
  if (G->erow.reserve(nnz * 4) || G->aedge.reserve(nnz * 8) || G->lic.reserve(nnz * 8) || G->deg.reserve(n * 8) ||
      G->x.reserve(n * ND * 8) || G->e0.reserve(nnz * 8) || G->red.reserve(64 * 8) || G->flag.reserve(8) ||
      G->tmp.reserve(nnz * 8))
    return ICPCG_E_NOMEM;
  ICPCG_HIP_TRY(hipMemsetAsync(G->flag.p, 0, 8, s));
  hipLaunchKernelGGL(k_edge_setup, dim3(grid_for(n)), dim3(kB), 0, s, A->row_ptr, A->col, (const double *)A->val,
                     P->lrp.as<int64_t>(), P->lci.as<int32_t>(), n, G->erow.as<int32_t>(), G->aedge.as<double>(),
                     G->flag.as<int>());
  ICPCG_HIP_TRY(hipGetLastError());
  int bad = 0;
  ICPCG_HIP_TRY(hipMemcpyAsync(&bad, G->flag.p, 4, hipMemcpyDeviceToHost, s));
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  if (bad) {
    set_error("gnn_create: the factor's pattern is not the lower triangle of A's");
    return ICPCG_E_INVALID;
  }
  ICPCG_HIP_TRY(hipMemcpyAsync(G->lic.p, P->lval.p, nnz * 8, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_deg_inc, dim3(grid_for(n)), dim3(kB), 0, s, P->lrp.as<int64_t>(), P->urp.as<int64_t>(), n,
                     G->deg.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_features, dim3(grid_for(n)), dim3(kB), 0, s, A->row_ptr, A->col, (const double *)A->val, n,
                     G->x.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  // input scale: population standard deviation of tril(A)'s entries (mean
  // first, then the mean square deviation)
  double *red = G->red.as<double>();
  int st;
  DevBuf part;
  if ((st = colsum<1, false>(G->aedge.as<double>(), nnz, part, red, s))) return st;
  double sum = 0.0;
  ICPCG_HIP_TRY(hipMemcpyAsync(&sum, red, 8, hipMemcpyDeviceToHost, s));
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  const double mean = sum / (double)nnz;
  hipLaunchKernelGGL(k_div, dim3(grid_for(nnz)), dim3(kB), 0, s, G->aedge.as<double>(), nnz, mean, 1.0,
                     G->tmp.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = colsum<1, true>(G->tmp.as<double>(), nnz, part, red, s))) return st;
  double ss = 0.0;
  ICPCG_HIP_TRY(hipMemcpyAsync(&ss, red, 8, hipMemcpyDeviceToHost, s));
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  G->scale = std::sqrt(ss / (double)nnz);
  if (!(G->scale > 0.0) || !std::isfinite(G->scale)) {
    set_error("gnn_create: the entries of tril(A) have no finite positive spread");
    return ICPCG_E_INVALID;
  }
  hipLaunchKernelGGL(k_div, dim3(grid_for(nnz)), dim3(kB), 0, s, G->aedge.as<double>(), nnz, 0.0, G->scale,
                     G->e0.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  G->tmp.release();
  return ICPCG_OK;
}

int gnn_inputs(const icpcg_gnn *G, double *x, double *e, hipStream_t s) {
  if (x) ICPCG_HIP_TRY(hipMemcpyAsync(x, G->x.p, (size_t)G->n * ND * 8, hipMemcpyDeviceToDevice, s));
  if (e) ICPCG_HIP_TRY(hipMemcpyAsync(e, G->e0.p, (size_t)G->nnz * 8, hipMemcpyDeviceToDevice, s));
  return ICPCG_OK;
}

int gnn_forward(icpcg_gnn *G, const double *theta, double *L_out, bool keep, hipStream_t s) {
  int st;
  if ((st = reserve_all(G, keep))) return st;
  const int64_t n = G->n;
  double *red = G->red.as<double>();  // [0, 9): column sums of x; [9, 18): of d^2
  if ((st = colsum<ND, false>(G->x.as<double>(), n, G->part, red, s))) return st;
  hipLaunchKernelGGL(k_gn_center, dim3(grid_for(n * ND)), dim3(kB), 0, s, G->x.as<double>(), red, n, theta,
                     G->mu.as<double>(), G->d.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = colsum<ND, true>(G->d.as<double>(), n, G->part, red + ND, s))) return st;
  hipLaunchKernelGGL(k_gn_apply, dim3(grid_for(n * ND)), dim3(kB), 0, s, G->d.as<double>(), red + ND, n, theta,
                     G->sd.as<double>(), G->h[0].as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = edge_fwd<0>(G, theta, keep, s)) || (st = node_fwd<0>(G, theta, keep, s)) ||
      (st = edge_fwd<1>(G, theta, keep, s)) || (st = node_fwd<1>(G, theta, keep, s)) ||
      (st = edge_fwd<2>(G, theta, keep, s)))
    return st;
  hipLaunchKernelGGL(k_assemble, dim3(grid_for(G->nnz)), dim3(kB), 0, s, G->erow.as<int32_t>(),
                     G->P->lci.as<int32_t>(), G->nnz, G->lic.as<double>(), G->e[2].as<double>(), std::sqrt(G->scale),
                     L_out ? L_out : G->L.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int gnn_loss_grad(icpcg_gnn *G, const double *theta, const double *z, double *loss, double *grad, bool accumulate,
                  hipStream_t s) {
  int st;
  if ((st = gnn_forward(G, theta, nullptr, true, s))) return st;
  const icpcg_prec *P = G->P;
  const int64_t n = G->n, nnz = G->nnz;
  const double *L = G->L.as<double>();
  const unsigned gn = grid_for(n);
  // loss of Eq. 5: r = L (L^T z) - A z, normalized by ||A z||^2
  hipLaunchKernelGGL(k_csr_mv, dim3(gn), dim3(kB), 0, s, G->A.row_ptr, G->A.col, (const double *)G->A.val, n, z,
                     G->az.as<double>());
  hipLaunchKernelGGL(k_lt_mv, dim3(gn), dim3(kB), 0, s, P->urp.as<int64_t>(), P->uci.as<int32_t>(),
                     P->upos.as<int32_t>(), L, n, z, G->u.as<double>());
  hipLaunchKernelGGL(k_csr_mv, dim3(gn), dim3(kB), 0, s, P->lrp.as<int64_t>(), P->lci.as<int32_t>(), L, n,
                     G->u.as<double>(), G->llz.as<double>());
  hipLaunchKernelGGL(k_resid, dim3(gn), dim3(kB), 0, s, G->llz.as<double>(), G->az.as<double>(), n,
                     G->r.as<double>(), G->sq2.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  double *sums = G->sums.as<double>();
  if ((st = colsum<2, false>(G->sq2.as<double>(), n, G->part, sums, s))) return st;
  hipLaunchKernelGGL(k_loss_out, dim3(1), dim3(1), 0, s, sums, loss, accumulate ? 1 : 0);
  hipLaunchKernelGGL(k_lt_mv, dim3(gn), dim3(kB), 0, s, P->urp.as<int64_t>(), P->uci.as<int32_t>(),
                     P->upos.as<int32_t>(), L, n, G->r.as<double>(), G->ltr.as<double>());
  hipLaunchKernelGGL(k_dout, dim3(grid_for(nnz)), dim3(kB), 0, s, G->erow.as<int32_t>(), P->lci.as<int32_t>(), nnz, L,
                     G->r.as<double>(), G->u.as<double>(), z, G->ltr.as<double>(), sums, std::sqrt(G->scale),
                     G->dout.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  // blocks in reverse
  if ((st = edge_bwd<2>(G, theta, G->dout.as<double>(), grad, accumulate, s))) return st;
  if ((st = node_gather(G, nullptr, s)) || (st = node_bwd<1>(G, theta, grad, accumulate, s))) return st;
  if ((st = edge_bwd<1>(G, theta, G->de.as<double>(), grad, accumulate, s))) return st;
  if ((st = node_gather(G, G->direct.as<double>(), s)) || (st = node_bwd<0>(G, theta, grad, accumulate, s)))
    return st;
  if ((st = edge_bwd<0>(G, theta, G->de.as<double>(), grad, accumulate, s))) return st;
  if ((st = node_gather(G, G->direct.as<double>(), s))) return st;
  // graph normalization (dh now holds the gradient of its output)
  hipLaunchKernelGGL(k_gn_bwd_rows, dim3(grid_for(n * ND)), dim3(kB), 0, s, G->dh.as<double>(), G->d.as<double>(),
                     G->sd.as<double>(), theta, n, G->rows3.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  double *sums3 = sums + 2;  // 27 values
  if ((st = colsum<3 * ND, false>(G->rows3.as<double>(), n, G->part, sums3, s))) return st;
  hipLaunchKernelGGL(k_gn_bwd_dd, dim3(grid_for(n * ND)), dim3(kB), 0, s, G->dh.as<double>(), G->d.as<double>(),
                     G->sd.as<double>(), sums3, theta, n, G->dd.as<double>());
  ICPCG_HIP_TRY(hipGetLastError());
  double *sumdd = sums + 2 + 3 * ND;
  if ((st = colsum<ND, false>(G->dd.as<double>(), n, G->part, sumdd, s))) return st;
  hipLaunchKernelGGL(k_gn_grad, dim3(1), dim3(64), 0, s, sums3, sumdd, G->mu.as<double>(), grad, accumulate ? 1 : 0);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

int adam_step(double *th, const double *g, double *m, double *v, int64_t count, int64_t t, double lr, double b1,
              double b2, double eps, hipStream_t s) {
  const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(count)), dim3(kB), 0, s, th, g, m, v, count, lr, b1, b2, eps, c1, c2);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

}  // namespace icpcg
