// Multicolour ordering applied as a symmetric permutation before the
// factorization: the direction the paper gives for the triangular solves
// (more parallelism in the preconditioner's layout, supplementary Additional
// Results). Nodes are the row groups of A (consecutive rows with identical
// column lists, at most 3); node v's colour is the smallest colour not used
// by its neighbours of higher (priority, id), with SplitMix64 priorities.
// Jones-Plassmann rounds compute exactly that colouring: a node is decided
// in the round after all of its higher-key neighbours are. The order sorts
// nodes by (colour, id) and keeps each node's rows together. The block
// variant colours a caller's partition of the rows (for instance mesh blocks)
// in the same rounds, with block ids as priorities, and sorts the rows by
// (colour, block, row). Also here: P A P^T and the row permutation of blocks
// of vectors.
#include <string>

#include "internal.hpp"

namespace icpcg {

namespace {

constexpr int kB = 256;
constexpr int kColourWords = 4;  // colours below 256

unsigned grid_for(int64_t n) {
  int64_t g = (n + kB - 1) / kB;
  if (g > 262144) g = 262144;
  return (unsigned)(g < 1 ? 1 : g);
}

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

// SplitMix64 (Steele, Lea and Flood): one step from state x.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Priorities: SplitMix64(seed + v), or (by_id) the reversed id, so that JP
// rounds compute sequential first fit in increasing id order.
__global__ void k_node_setup(const int32_t *__restrict__ gptr, int64_t nn, uint64_t seed, bool by_id,
                             int32_t *__restrict__ node_of, uint64_t *__restrict__ prio, int32_t *__restrict__ colour) {
  for (int64_t v = gtid(); v < nn; v += gstride()) {
    for (int32_t r = gptr[v]; r < gptr[v + 1]; ++r) node_of[r] = (int32_t)v;
    prio[v] = by_id ? ~(uint64_t)v : splitmix64(seed + (uint64_t)v);
    colour[v] = -1;
  }
}

// One Jones-Plassmann round: reads the colours of the previous round, writes
// the next; `left` counts the nodes still undecided, `over` flags a colour
// beyond the supported range.
__global__ void k_jp_round(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const int32_t *__restrict__ gptr, const int32_t *__restrict__ node_of,
                           const uint64_t *__restrict__ prio, int64_t nn, const int32_t *__restrict__ cin,
                           int32_t *__restrict__ cout, int *left, int *over) {
  for (int64_t v = gtid(); v < nn; v += gstride()) {
    const int32_t c = cin[v];
    cout[v] = c;
    if (c >= 0) continue;
    const uint64_t pv = prio[v];
    const int32_t r0 = gptr[v];
    uint64_t used[kColourWords] = {0, 0, 0, 0};
    bool ready = true;
    for (int64_t t = rp[r0]; t < rp[r0 + 1]; ++t) {
      const int32_t u = node_of[ci[t]];
      if (u == v) continue;
      const uint64_t pu = prio[u];
      if (pu < pv || (pu == pv && u < v)) continue;  // lower key: not consulted
      const int32_t cu = cin[u];
      if (cu < 0) {
        ready = false;
        break;
      }
      if (cu < 64 * kColourWords) used[cu >> 6] |= 1ull << (cu & 63);
    }
    if (!ready) {
      atomicAdd(left, 1);
      continue;
    }
    int k = 0;
    while (k < kColourWords && used[k] == ~0ull) ++k;
    if (k == kColourWords) {
      atomicOr(over, 1);
      cout[v] = 64 * kColourWords - 1;
      continue;
    }
    cout[v] = k * 64 + __builtin_ctzll(~used[k]);
  }
}

__global__ void k_node_sizes(const int32_t *__restrict__ order, const int32_t *__restrict__ gptr, int64_t nn,
                             int32_t *__restrict__ sz) {
  for (int64_t p = gtid(); p < nn; p += gstride()) sz[p] = gptr[order[p] + 1] - gptr[order[p]];
}

__global__ void k_fill_perm(const int32_t *__restrict__ order, const int32_t *__restrict__ gptr,
                            const int32_t *__restrict__ start, int64_t nn, int32_t *__restrict__ perm) {
  for (int64_t p = gtid(); p < nn; p += gstride()) {
    const int32_t v = order[p];
    for (int32_t d = 0; d < gptr[v + 1] - gptr[v]; ++d) perm[start[p] + d] = gptr[v] + d;
  }
}

__global__ void k_inverse(const int32_t *__restrict__ perm, int64_t n, uint32_t *__restrict__ inv, int *bad) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const int32_t o = perm[i];
    if (o < 0 || o >= n) {
      atomicOr(bad, 1);
      continue;
    }
    inv[o] = (uint32_t)i;
  }
}

// A permutation's inverse has every slot written exactly once.
__global__ void k_check_inverse(const int32_t *__restrict__ perm, const uint32_t *__restrict__ inv, int64_t n,
                                int *bad) {
  for (int64_t i = gtid(); i < n; i += gstride())
    if (inv[i] >= (uint64_t)n || perm[inv[i]] != i) atomicOr(bad, 1);
}

__global__ void k_new_len(const int64_t *__restrict__ rp, const int32_t *__restrict__ perm, int64_t n,
                          int64_t *__restrict__ len) {
  for (int64_t i = gtid(); i < n; i += gstride()) len[i] = rp[perm[i] + 1] - rp[perm[i]];
}

// Per stored entry: key = new column, value = entry index.
__global__ void k_entry_keys(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci, int64_t n,
                             const uint32_t *__restrict__ inv, uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                             uint32_t *__restrict__ newrow) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint32_t ni = inv[i];
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
      key[t] = inv[ci[t]];
      val[t] = (uint32_t)t;
      newrow[t] = ni;
    }
  }
}

__global__ void k_gather_u32(const uint32_t *__restrict__ src, const uint32_t *__restrict__ idx, int64_t m,
                             uint32_t *__restrict__ dst) {
  for (int64_t k = gtid(); k < m; k += gstride()) dst[k] = src[idx[k]];
}

__global__ void k_emit(const uint32_t *__restrict__ order, const int32_t *__restrict__ ci,
                       const double *__restrict__ v, const uint32_t *__restrict__ inv, int64_t m,
                       int32_t *__restrict__ oci, double *__restrict__ ov) {
  for (int64_t k = gtid(); k < m; k += gstride()) {
    const uint32_t t = order[k];
    oci[k] = (int32_t)inv[ci[t]];
    ov[k] = v[t];
  }
}

__global__ void k_permute_rows(const int32_t *__restrict__ perm, int64_t n, int64_t R, const double *__restrict__ x,
                               double *__restrict__ y, int inverse) {
  for (int64_t e = gtid(); e < n * R; e += gstride()) {
    const int64_t i = e / R, c = e % R;
    if (inverse)
      y[(int64_t)perm[i] * R + c] = x[e];
    else
      y[e] = x[(int64_t)perm[i] * R + c];
  }
}

// Block colouring: every entry (i, j) of A gives the pair (block of i, block
// of j); sorted by the first, the second ones are each block's neighbour list
// (repeats and the block itself included: the colouring round skips both).
__global__ void k_entry_blocks(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci, int64_t n,
                               const int32_t *__restrict__ blk, uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint32_t a = (uint32_t)blk[i];
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
      key[t] = a;
      val[t] = (uint32_t)blk[ci[t]];
    }
  }
}

__global__ void k_check_blocks(const int32_t *__restrict__ blk, int64_t n, int32_t nblk, int *bad) {
  for (int64_t i = gtid(); i < n; i += gstride())
    if (blk[i] < 0 || blk[i] >= nblk) atomicOr(bad, 1);
}

// After sorting the pairs by (row block, column block): keep the first of each
// run of equal pairs, and drop a block's pairs with itself.
__global__ void k_pair_keep(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b, int64_t m,
                            int32_t *__restrict__ keep) {
  for (int64_t t = gtid(); t < m; t += gstride())
    keep[t] = (a[t] != b[t] && (t == 0 || a[t] != a[t - 1] || b[t] != b[t - 1])) ? 1 : 0;
}

__global__ void k_pair_compact(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                               const int32_t *__restrict__ keep, const int32_t *__restrict__ pos, int64_t m,
                               int32_t *__restrict__ nb, unsigned long long *__restrict__ cnt) {
  for (int64_t t = gtid(); t < m; t += gstride())
    if (keep[t]) {
      nb[pos[t]] = (int32_t)b[t];
      atomicAdd(&cnt[a[t]], 1ull);
    }
}

__global__ void k_row_colour_keys(const uint32_t *__restrict__ rows, const int32_t *__restrict__ blk,
                                  const int32_t *__restrict__ colour, int64_t n, uint32_t *__restrict__ key) {
  for (int64_t p = gtid(); p < n; p += gstride()) key[p] = (uint32_t)colour[blk[rows[p]]];
}

__global__ void k_set_at(int64_t *p, int64_t i, int64_t v) { p[i] = v; }

int bits_for(int64_t maxval) {
  int b = 1;
  while (b < 32 && ((int64_t)1 << b) <= maxval) ++b;
  return b;
}

int read_int(const int *dev, hipStream_t s, int *host) {
  ICPCG_HIP_TRY(hipMemcpyAsync(host, dev, sizeof(int), hipMemcpyDeviceToHost, s));
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  return ICPCG_OK;
}

}  // namespace

// Jones-Plassmann colouring of nn nodes: node v's neighbours are the nodes
// (node_of) of the columns of row gptr[v] of (rp, ci). On return *colours
// points at ca or cb and *maxc is the largest colour.
int jp_colour(const int64_t *rp, const int32_t *ci, const int32_t *gptr, int64_t nrows, int64_t nn, uint64_t seed,
              bool by_id, DevBuf &node_of, DevBuf &ca, DevBuf &cb, int32_t **colours, int32_t *maxc,
              const char *what, hipStream_t s) {
  DevBuf prio, flags;
  if (node_of.reserve(nrows * 4) || prio.reserve(nn * 8) || ca.reserve(nn * 4) || cb.reserve(nn * 4) ||
      flags.reserve(16))
    return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_node_setup, dim3(grid_for(nn)), dim3(kB), 0, s, gptr, nn, seed, by_id,
                     node_of.as<int32_t>(), prio.as<uint64_t>(), ca.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  int *left = flags.as<int>(), *over = left + 1;
  ICPCG_HIP_TRY(hipMemsetAsync(over, 0, sizeof(int), s));
  int32_t *cin = ca.as<int32_t>(), *cout = cb.as<int32_t>();
  int st;
  // every round decides at least the undecided node of highest key
  for (int64_t round = 0;; ++round) {
    if (round > nn) {
      set_error(std::string(what) + ": colouring did not finish");
      return ICPCG_E_DEVICE;
    }
    ICPCG_HIP_TRY(hipMemsetAsync(left, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_jp_round, dim3(grid_for(nn)), dim3(kB), 0, s, rp, ci, gptr, node_of.as<int32_t>(),
                       prio.as<uint64_t>(), nn, cin, cout, left, over);
    ICPCG_HIP_TRY(hipGetLastError());
    std::swap(cin, cout);
    int h = 0;
    if ((st = read_int(left, s, &h))) return st;
    if (h == 0) break;
  }
  int ov = 0;
  if ((st = read_int(over, s, &ov))) return st;
  if (ov) {
    set_error(std::string(what) + ": the graph needs more than 256 colours");
    return ICPCG_E_INVALID;
  }
  if ((st = reduce_max_i32(cin, nn, s, maxc))) return st;
  *colours = cin;
  return ICPCG_OK;
}

int color_order(const int64_t *rp, const int32_t *ci, int64_t n, uint64_t seed, int32_t *perm, int32_t *ncolours,
                hipStream_t s) {
  DevBuf gptr, grec;
  int64_t nn = 0;
  int st = build_row_groups(rp, ci, n, kSupernodeMax, gptr, grec, &nn, s);
  if (st) return st;
  DevBuf node_of, ca, cb;
  int32_t *cin = nullptr, maxc = 0;
  if ((st = jp_colour(rp, ci, gptr.as<int32_t>(), n, nn, seed, false, node_of, ca, cb, &cin, &maxc, "color_order",
                      s)))
    return st;
  *ncolours = maxc + 1;
  // nodes by (colour, id): a stable sort of the ids on the colour
  DevBuf ids, okeys, order, sz, start;
  if (ids.reserve(nn * 4) || okeys.reserve(nn * 4) || order.reserve(nn * 4) || sz.reserve(nn * 4) ||
      start.reserve(nn * 4))
    return ICPCG_E_NOMEM;
  if ((st = fill_iota_u32(ids.as<uint32_t>(), nn, s))) return st;
  if ((st = radix_sort_pairs(reinterpret_cast<const uint32_t *>(cin), ids.as<uint32_t>(), okeys.as<uint32_t>(),
                             order.as<uint32_t>(), nn, bits_for(maxc), s)))
    return st;
  hipLaunchKernelGGL(k_node_sizes, dim3(grid_for(nn)), dim3(kB), 0, s, order.as<int32_t>(), gptr.as<int32_t>(), nn,
                     sz.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  int32_t total = 0;
  if ((st = scan_exclusive_i32(sz.as<int32_t>(), start.as<int32_t>(), nn, s, &total))) return st;
  hipLaunchKernelGGL(k_fill_perm, dim3(grid_for(nn)), dim3(kB), 0, s, order.as<int32_t>(), gptr.as<int32_t>(),
                     start.as<int32_t>(), nn, perm);
  ICPCG_HIP_TRY(hipGetLastError());
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  return ICPCG_OK;
}

// Block multicolour order: the caller partitions the rows into blocks
// (blk[i] in [0, nblk), for instance mesh blocks of nodes); blocks coupled by
// an entry of A are neighbours, block b takes the smallest colour not used by
// its neighbours of lower id (sequential first fit in id order, computed by
// JP rounds; on a block grid numbered like its nodes this is the 8-colour
// parity pattern), and the rows are ordered by (colour of their block, block,
// row).
int block_color_order(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz, const int32_t *blk, int32_t nblk,
                      int32_t *perm, int32_t *ncolours, hipStream_t s) {
  int st;
  DevBuf bad;
  if (bad.reserve(4)) return ICPCG_E_NOMEM;
  ICPCG_HIP_TRY(hipMemsetAsync(bad.p, 0, 4, s));
  hipLaunchKernelGGL(k_check_blocks, dim3(grid_for(n)), dim3(kB), 0, s, blk, n, nblk, bad.as<int>());
  ICPCG_HIP_TRY(hipGetLastError());
  int hb = 0;
  if ((st = read_int(bad.as<int>(), s, &hb))) return st;
  if (hb) {
    set_error("block_color_order: a block id is outside [0, nblk)");
    return ICPCG_E_INVALID;
  }
  // block pairs of the entries, sorted by (row block, column block): a stable
  // sort on the column block, then on the row block
  DevBuf key, val, k1, v1;
  if (key.reserve(nnz * 4) || val.reserve(nnz * 4) || k1.reserve(nnz * 4) || v1.reserve(nnz * 4))
    return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_entry_blocks, dim3(grid_for(n)), dim3(kB), 0, s, rp, ci, n, blk, key.as<uint32_t>(),
                     val.as<uint32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  const int bb = bits_for(nblk - 1);
  if ((st = radix_sort_pairs(val.as<uint32_t>(), key.as<uint32_t>(), v1.as<uint32_t>(), k1.as<uint32_t>(), nnz, bb, s)))
    return st;
  if ((st = radix_sort_pairs(k1.as<uint32_t>(), v1.as<uint32_t>(), key.as<uint32_t>(), val.as<uint32_t>(), nnz, bb, s)))
    return st;
  k1.release();
  v1.release();
  // distinct neighbours of each block (block v's list is "row" v of (qrp, nbr))
  DevBuf keep, pos, nbr, cnt, qrp;
  if (keep.reserve(nnz * 4) || pos.reserve(nnz * 4) || cnt.reserve((size_t)nblk * 8) ||
      qrp.reserve(((size_t)nblk + 1) * 8))
    return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_pair_keep, dim3(grid_for(nnz)), dim3(kB), 0, s, key.as<uint32_t>(), val.as<uint32_t>(), nnz,
                     keep.as<int32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  int32_t nedges = 0;
  if ((st = scan_exclusive_i32(keep.as<int32_t>(), pos.as<int32_t>(), nnz, s, &nedges))) return st;
  if (nbr.reserve((size_t)(nedges > 0 ? nedges : 1) * 4)) return ICPCG_E_NOMEM;
  ICPCG_HIP_TRY(hipMemsetAsync(cnt.p, 0, (size_t)nblk * 8, s));
  hipLaunchKernelGGL(k_pair_compact, dim3(grid_for(nnz)), dim3(kB), 0, s, key.as<uint32_t>(), val.as<uint32_t>(),
                     keep.as<int32_t>(), pos.as<int32_t>(), nnz, nbr.as<int32_t>(), cnt.as<unsigned long long>());
  ICPCG_HIP_TRY(hipGetLastError());
  int64_t total = 0;
  if ((st = scan_exclusive_i64(cnt.as<int64_t>(), qrp.as<int64_t>(), nblk, s, &total))) return st;
  hipLaunchKernelGGL(k_set_at, dim3(1), dim3(1), 0, s, qrp.as<int64_t>(), (int64_t)nblk, total);
  ICPCG_HIP_TRY(hipGetLastError());
  key.release();
  val.release();
  keep.release();
  pos.release();
  // colour the block graph: block v's list is "row" v of (qrp, nbr)
  DevBuf gptr, node_of, ca, cb;
  if (gptr.reserve(((size_t)nblk + 1) * 4)) return ICPCG_E_NOMEM;
  if ((st = fill_iota_u32(gptr.as<uint32_t>(), (int64_t)nblk + 1, s))) return st;
  int32_t *colour = nullptr, maxc = 0;
  if ((st = jp_colour(qrp.as<int64_t>(), nbr.as<int32_t>(), gptr.as<int32_t>(), nblk, nblk, 0, true, node_of, ca, cb,
                      &colour, &maxc, "block_color_order", s)))
    return st;
  *ncolours = maxc + 1;
  // rows by (colour, block, row): stable sorts on the block, then the colour
  DevBuf rows, rk, o1, k2, kk;
  if (rows.reserve(n * 4) || rk.reserve(n * 4) || o1.reserve(n * 4) || k2.reserve(n * 4) || kk.reserve(n * 4))
    return ICPCG_E_NOMEM;
  if ((st = fill_iota_u32(rows.as<uint32_t>(), n, s))) return st;
  if ((st = radix_sort_pairs(reinterpret_cast<const uint32_t *>(blk), rows.as<uint32_t>(), rk.as<uint32_t>(),
                             o1.as<uint32_t>(), n, bits_for(nblk - 1), s)))
    return st;
  hipLaunchKernelGGL(k_row_colour_keys, dim3(grid_for(n)), dim3(kB), 0, s, o1.as<uint32_t>(), blk, colour, n,
                     k2.as<uint32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = radix_sort_pairs(k2.as<uint32_t>(), o1.as<uint32_t>(), kk.as<uint32_t>(), reinterpret_cast<uint32_t *>(perm),
                             n, bits_for(maxc), s)))
    return st;
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  return ICPCG_OK;
}

int permute_matrix(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t nnz, const int32_t *perm,
                   int64_t *orp, int32_t *oci, double *ov, hipStream_t s) {
  DevBuf inv, len, flag;
  if (inv.reserve(n * 4) || len.reserve((n + 1) * 8) || flag.reserve(8)) return ICPCG_E_NOMEM;
  ICPCG_HIP_TRY(hipMemsetAsync(flag.p, 0, 8, s));
  int st;
  if ((st = fill_u32(inv.as<uint32_t>(), 0xFFFFFFFFu, n, s))) return st;
  hipLaunchKernelGGL(k_inverse, dim3(grid_for(n)), dim3(kB), 0, s, perm, n, inv.as<uint32_t>(), flag.as<int>());
  ICPCG_HIP_TRY(hipGetLastError());
  int bad = 0;
  if ((st = read_int(flag.as<int>(), s, &bad))) return st;
  if (!bad) {
    hipLaunchKernelGGL(k_check_inverse, dim3(grid_for(n)), dim3(kB), 0, s, perm, inv.as<uint32_t>(), n,
                       flag.as<int>());
    ICPCG_HIP_TRY(hipGetLastError());
    if ((st = read_int(flag.as<int>(), s, &bad))) return st;
  }
  if (bad) {
    set_error("permute: perm is not a permutation of 0..n-1");
    return ICPCG_E_INVALID;
  }
  hipLaunchKernelGGL(k_new_len, dim3(grid_for(n)), dim3(kB), 0, s, rp, perm, n, len.as<int64_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  int64_t total = 0;
  if ((st = scan_exclusive_i64(len.as<int64_t>(), orp, n, s, &total))) return st;
  if (total != nnz) {
    set_error("permute: row lengths do not add up to nnz");
    return ICPCG_E_INVALID;
  }
  hipLaunchKernelGGL(k_set_at, dim3(1), dim3(1), 0, s, orp, n, total);
  ICPCG_HIP_TRY(hipGetLastError());
  // entries ordered by (new row, new column): stable sorts on the column,
  // then on the row
  DevBuf k0, v0, k1, v1, nr;
  if (k0.reserve(nnz * 4) || v0.reserve(nnz * 4) || k1.reserve(nnz * 4) || v1.reserve(nnz * 4) ||
      nr.reserve(nnz * 4))
    return ICPCG_E_NOMEM;
  hipLaunchKernelGGL(k_entry_keys, dim3(grid_for(n)), dim3(kB), 0, s, rp, ci, n, inv.as<uint32_t>(),
                     k0.as<uint32_t>(), v0.as<uint32_t>(), nr.as<uint32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  const int bits = bits_for(n - 1);
  if ((st = radix_sort_pairs(k0.as<uint32_t>(), v0.as<uint32_t>(), k1.as<uint32_t>(), v1.as<uint32_t>(), nnz, bits,
                             s)))
    return st;
  hipLaunchKernelGGL(k_gather_u32, dim3(grid_for(nnz)), dim3(kB), 0, s, nr.as<uint32_t>(), v1.as<uint32_t>(), nnz,
                     k0.as<uint32_t>());
  ICPCG_HIP_TRY(hipGetLastError());
  if ((st = radix_sort_pairs(k0.as<uint32_t>(), v1.as<uint32_t>(), k1.as<uint32_t>(), v0.as<uint32_t>(), nnz, bits,
                             s)))
    return st;
  hipLaunchKernelGGL(k_emit, dim3(grid_for(nnz)), dim3(kB), 0, s, v0.as<uint32_t>(), ci, v, inv.as<uint32_t>(), nnz,
                     oci, ov);
  ICPCG_HIP_TRY(hipGetLastError());
  ICPCG_HIP_TRY(hipStreamSynchronize(s));
  return ICPCG_OK;
}

int permute_rows(const int32_t *perm, int64_t n, int64_t R, const double *x, double *y, bool inverse, hipStream_t s) {
  hipLaunchKernelGGL(k_permute_rows, dim3(grid_for(n * R)), dim3(kB), 0, s, perm, n, R, x, y, inverse ? 1 : 0);
  ICPCG_HIP_TRY(hipGetLastError());
  return ICPCG_OK;
}

}  // namespace icpcg
