// Neural bounding hierarchies (Sec. 3.3): a user-supplied tree over the
// objects of a group, each node's network a conservative bound of the union
// of the indicators below it, so that a region that meets a leaf's object is
// reported by every node on the path from the root to that leaf.
//
// A query descends the tree level by level.  Each level is one grouped
// forward over (region, node) pairs held contiguously per node, which keeps
// MFMA tiles full of one network's queries instead of letting lanes walk
// different paths.  The positive pairs are compacted into an ascending index
// list (block counts, a scan of the block totals, then each block writes its
// positives at its offset), so node p's positives are a contiguous run of
// that list, found by binary search on p's segment bounds, in the regions'
// order.  The next level is then built one thread per positive: the thread
// finds its node by binary search over the nodes' runs, reads its region
// once and copies it to every child's segment at its rank among the node's
// positives (or, at a leaf, writes the region index to the leaf's output
// segment).  The host reads the level's counts to size the next level.
#include <algorithm>
#include <cmath>
#include <vector>

#include "nb_internal.h"

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;                        // flags per thread
constexpr int kScanBlock = kScanThreads * kScanPer;  // 4096 flags per block

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
float tau_of(float eps) { return (float)std::log((0.5 - (double)eps) / (0.5 + (double)eps)); }

// Inclusive scan of one int64 per thread over the block (sh_waves holds one
// entry per wave of the block).
__device__ __forceinline__ int64_t block_inclusive(int64_t x, int64_t* sh_waves) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) sh_waves[wave] = x;
  __syncthreads();
  int64_t before = 0;
  for (int w = 0; w < wave; ++w) before += sh_waves[w];
  __syncthreads();
  return x + before;
}

// The 16 decision flags of a thread (1 for a nonzero byte), zero beyond n;
// one 16-byte load when the run is whole (h is 256-byte aligned, base a
// multiple of 16).
__device__ __forceinline__ void load_flags16(const uint8_t* __restrict__ h, int64_t n, int64_t base, int (&f)[kScanPer]) {
  if (base + kScanPer <= n) {
    const uint4 v = *reinterpret_cast<const uint4*>(h + base);
    const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) f[k] = ((w[k >> 2] >> (8 * (k & 3))) & 0xffu) != 0u;
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) f[k] = (base + k < n && h[base + k] != 0) ? 1 : 0;
  }
}

// Positive count of each 4096-flag block.
__global__ __launch_bounds__(kScanThreads) void k_flag_counts(const uint8_t* __restrict__ h, int64_t n,
                                                              int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[kScanThreads / 64];
  int f[kScanPer];
  load_flags16(h, n, (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer, f);
  int tot = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) tot += f[k];
  const int64_t incl = block_inclusive(tot, sh);
  if (threadIdx.x == kScanThreads - 1) bsum[blockIdx.x] = incl;
}

// Ascending list of the positive pairs: block b writes its positives from
// offset bpre[b] (the exclusive prefix of the block counts) on, in order.
__global__ __launch_bounds__(kScanThreads) void k_compact(const uint8_t* __restrict__ h, int64_t n,
                                                          const int64_t* __restrict__ bpre,
                                                          int32_t* __restrict__ pos_idx) {
  __shared__ int64_t sh[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int f[kScanPer];
  load_flags16(h, n, base, f);
  int tot = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) tot += f[k];
  const int64_t incl = block_inclusive(tot, sh);
  int64_t at = bpre[blockIdx.x] + incl - tot;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k)
    if (f[k]) pos_idx[at++] = (int32_t)(base + k);
}

// Exclusive prefix of the block totals in place (one block of 1024 threads,
// each summing a contiguous run of the totals first); total[0] = sum.
constexpr int kPrefixThreads = 1024;
__global__ __launch_bounds__(kPrefixThreads) void k_scan_blocks(int64_t* __restrict__ bsum, int64_t nb,
                                                                int64_t* __restrict__ total) {
  __shared__ int64_t sh[kPrefixThreads / 64];
  const int64_t per = (nb + kPrefixThreads - 1) / kPrefixThreads;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = b0 + per < nb ? b0 + per : nb;
  int64_t sum = 0;
  for (int64_t b = b0; b < b1; ++b) sum += bsum[b];
  const int64_t incl = block_inclusive(sum, sh);
  int64_t run = incl - sum;
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t x = bsum[b];
    bsum[b] = run;
    run += x;
  }
  if (threadIdx.x == kPrefixThreads - 1) total[0] = incl;
}

// Number of positive pairs with index below x: a lower bound in the
// ascending positive list of `total` entries.
__device__ __forceinline__ int64_t positives_below(int64_t x, const int32_t* __restrict__ pos_idx, int64_t total) {
  int64_t lo = 0, hi = total;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)pos_idx[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Last index c in [a, b) with off[c] <= x, for nondecreasing off with
// off[a] <= x (the segment that holds x; empty segments are skipped).
__device__ __forceinline__ int segment_of(const int64_t* __restrict__ off, int a, int b, int64_t x) {
  int lo = a, hi = b - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Per level (one block): the first positive (prank) and positive count
// (pcnt) of this level's nodes, the next level's per-node row offsets (every
// node of the group: nodes before the next level empty at 0, nodes after it
// empty at the end), the output offsets of this level's leaves, and the
// running sizes sizes[0] = rows of the next level, sizes[1] = output pairs so
// far.
__global__ __launch_bounds__(kScanThreads) void k_hier_offsets(
    int n_obj, int lvl_a, int lvl_b, int nxt_a, int nxt_b, const int64_t* __restrict__ qoff, int empty,
    const int32_t* __restrict__ pos_idx, const int64_t* __restrict__ total, const int32_t* __restrict__ parent,
    const int32_t* __restrict__ leaf_rank, int64_t* __restrict__ prank, int64_t* __restrict__ pcnt,
    int64_t* __restrict__ qoff_next, int64_t* __restrict__ out_off, int64_t* __restrict__ sizes) {
  __shared__ int64_t sh[kScanThreads / 64];
  __shared__ int64_t carry;
  const int64_t npos = empty ? 0 : total[0];
  for (int p = lvl_a + threadIdx.x; p < lvl_b; p += kScanThreads) {
    const int64_t a = empty ? 0 : positives_below(qoff[p], pos_idx, npos);
    prank[p] = a;
    pcnt[p] = empty ? 0 : positives_below(qoff[p + 1], pos_idx, npos) - a;
  }
  __syncthreads();
  auto positives = [&](int p) -> int64_t { return pcnt[p]; };
  // next level: node c gets as many rows as its parent has positives
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int c0 = nxt_a; c0 < nxt_b; c0 += kScanThreads) {
    const int c = c0 + threadIdx.x;
    const int64_t x = c < nxt_b ? positives(parent[c]) : 0;
    const int64_t incl = block_inclusive(x, sh);
    const int64_t base = carry;
    if (c < nxt_b) qoff_next[c] = base + incl - x;
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) carry = base + incl;
    __syncthreads();
  }
  const int64_t rows_next = carry;
  for (int o = threadIdx.x; o <= n_obj; o += kScanThreads) {
    if (o < nxt_a) qoff_next[o] = 0;
    if (o >= nxt_b) qoff_next[o] = rows_next;
  }
  __syncthreads();
  // this level's leaves, in node order: output segments after the ones so far
  if (threadIdx.x == 0) carry = sizes[1];
  __syncthreads();
  for (int p0 = lvl_a; p0 < lvl_b; p0 += kScanThreads) {
    const int p = p0 + threadIdx.x;
    const bool leaf = p < lvl_b && leaf_rank[p] >= 0;
    const int64_t x = leaf ? positives(p) : 0;
    const int64_t incl = block_inclusive(x, sh);
    const int64_t base = carry;
    if (leaf) out_off[leaf_rank[p]] = base + incl - x;
    __syncthreads();
    if (threadIdx.x == kScanThreads - 1) carry = base + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sizes[0] = rows_next;
    sizes[1] = carry;
  }
}

// One thread per positive pair k of this level (in the ascending positive
// list): its node p (the segment of this level's positive runs, staged in
// LDS, that holds k) and its rank r among p's positives.  The thread reads
// the pair's region once; a leaf writes the region index to its output
// segment at rank r (entries at or beyond cap are not written), an inner
// node copies the region to every child's segment at rank r, so consecutive
// positives of a node write consecutive rows of each child.
__global__ __launch_bounds__(256) void k_hier_expand(
    int in_dim, int64_t n_pos, int lvl_a, int lvl_b, const int64_t* __restrict__ prank,
    const int32_t* __restrict__ pos_idx, const int32_t* __restrict__ child_b, const int32_t* __restrict__ child_e,
    const int32_t* __restrict__ leaf_rank, const int64_t* __restrict__ qoff_next, const int64_t* __restrict__ out_off,
    const float* __restrict__ rows, const int32_t* __restrict__ qidx, float* __restrict__ rows_next,
    int32_t* __restrict__ qidx_next, int32_t* __restrict__ out, int64_t cap) {
  extern __shared__ int64_t sfirst[];   // [nl] first positive of each node of the level
  const int nl = lvl_b - lvl_a;
  for (int i = threadIdx.x; i < nl; i += blockDim.x) sfirst[i] = prank[lvl_a + i];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pos) return;
  const int i = segment_of(sfirst, 0, nl, k);
  const int p = lvl_a + i;
  const int64_t r = k - sfirst[i];
  const int64_t src = pos_idx[k];
  const int32_t qi = qidx ? qidx[src] : (int32_t)src;
  const int lr = leaf_rank[p];
  if (lr >= 0) {
    const int64_t u = out_off[lr] + r;
    if (u < cap) out[u] = qi;
    return;
  }
  float x[8];   // in_dim <= 8; unrolled so that x stays in registers
#pragma unroll
  for (int d = 0; d < 8; ++d) x[d] = d < in_dim ? rows[src * in_dim + d] : 0.0f;
  for (int c = child_b[p]; c < child_e[p]; ++c) {
    const int64_t dst = qoff_next[c] + r;
#pragma unroll
    for (int d = 0; d < 8; ++d)
      if (d < in_dim) rows_next[dst * in_dim + d] = x[d];
    qidx_next[dst] = qi;
  }
}

__global__ void k_set_i64(int64_t* __restrict__ p, int64_t v) { *p = v; }

}  // namespace

struct nb_hier {
  nb_group* g = nullptr;
  int n_nodes = 0, n_leaves = 0, device = 0;
  std::vector<int> child_b, child_e, parent, level, leaf_rank;
  std::vector<int> lvl_first;       // nodes of level l: lvl_first[l] .. lvl_first[l+1]-1
  int32_t *d_child_b = nullptr, *d_child_e = nullptr, *d_parent = nullptr, *d_leaf_rank = nullptr;
  int64_t *d_prank = nullptr, *d_pcnt = nullptr;    // per node: first positive, positive count
  // two pair buffers (rows, region index), decisions, positive list, scan, offsets
  int64_t pcap[2] = {0, 0};
  float* rows[2] = {nullptr, nullptr};
  int32_t* qidx[2] = {nullptr, nullptr};
  int64_t scap = 0;
  uint8_t* h = nullptr;
  int32_t* pos_idx = nullptr;
  int64_t* bsum = nullptr;
  int64_t* qoff[2] = {nullptr, nullptr};
  int64_t* misc = nullptr;      // [0] scan total, [1] rows of the next level, [2] output pairs so far
  std::vector<int64_t> level_pairs;   // (row, node) pairs per level of the last query
  int64_t* host_sizes = nullptr;   // pinned [3]: misc[0..2] of the last level
};

namespace {

template <class T>
nb_status hier_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return NB_OK;
  NB_HIP(hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)));
  return NB_OK;
}

template <class T>
void hier_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_pair_set(nb_hier* t, int k) {
  hier_free(t->rows[k]);
  hier_free(t->qidx[k]);
  t->pcap[k] = 0;
}

void free_scan(nb_hier* t) {
  hier_free(t->h);
  hier_free(t->pos_idx);
  hier_free(t->bsum);
  t->scap = 0;
}

int64_t grown(int64_t need) { return std::max<int64_t>(need + need / 4, 1 << 16); }

// Pair set k holds at least `need` pairs.  Called with the stream idle and
// set k unused by any pending work.
nb_status ensure_pairs(nb_hier* t, int k, int64_t need) {
  if (need <= t->pcap[k]) return NB_OK;
  free_pair_set(t, k);
  const int64_t cap = grown(need);
  NB_TRY(hier_alloc(&t->rows[k], (size_t)cap * t->g->in_dim));
  NB_TRY(hier_alloc(&t->qidx[k], (size_t)cap));
  t->pcap[k] = cap;
  return NB_OK;
}

// Decisions and scan space for `need` pairs (stream idle).
nb_status ensure_scan(nb_hier* t, int64_t need) {
  if (need <= t->scap) return NB_OK;
  free_scan(t);
  const int64_t cap = grown(need);
  NB_TRY(hier_alloc(&t->h, (size_t)cap));
  NB_TRY(hier_alloc(&t->pos_idx, (size_t)cap));
  NB_TRY(hier_alloc(&t->bsum, (size_t)(cap / kScanBlock + 2)));
  t->scap = cap;
  return NB_OK;
}

}  // namespace

extern "C" {

nb_status nb_hier_create(nb_group* g, const int32_t* child_begin_host, const int32_t* child_end_host,
                         nb_hier** out) {
  NB_REQUIRE(out && g && child_begin_host && child_end_host, "NULL argument");
  *out = nullptr;
  const int n = g->n_obj;
  // children ranges, concatenated in parent order, must be exactly 1 .. n-1
  int next = 1;
  for (int p = 0; p < n; ++p) {
    const int b = child_begin_host[p], e = child_end_host[p];
    NB_REQUIRE(e >= b, "node %d: child range [%d, %d) is reversed", p, b, e);
    if (e == b) continue;
    NB_REQUIRE(b == next && e <= n,
               "node %d: children must be the next unused nodes in breadth-first order (expected %d, got [%d, %d))",
               p, next, b, e);
    NB_REQUIRE(b > p, "node %d: a child must come after its parent", p);
    next = e;
  }
  NB_REQUIRE(next == n, "nodes %d .. %d have no parent (breadth-first order, node 0 the root)", next, n - 1);
  auto* t = new nb_hier();
  t->g = g;
  t->n_nodes = n;
  t->device = g->device;
  t->child_b.assign(child_begin_host, child_begin_host + n);
  t->child_e.assign(child_end_host, child_end_host + n);
  t->parent.assign(n, -1);
  t->level.assign(n, 0);
  t->leaf_rank.assign(n, -1);
  for (int p = 0; p < n; ++p)
    for (int c = t->child_b[p]; c < t->child_e[p]; ++c) {
      t->parent[c] = p;
      t->level[c] = t->level[p] + 1;
    }
  for (int p = 0; p < n; ++p)
    if (t->child_b[p] == t->child_e[p]) t->leaf_rank[p] = t->n_leaves++;
  const int depth = t->level[n - 1] + 1;
  t->lvl_first.assign(depth + 1, n);
  for (int p = n - 1; p >= 0; --p) t->lvl_first[t->level[p]] = p;
  nb_status st = NB_OK;
  if (st == NB_OK) st = hier_alloc(&t->d_child_b, n);
  if (st == NB_OK) st = hier_alloc(&t->d_child_e, n);
  if (st == NB_OK) st = hier_alloc(&t->d_parent, n);
  if (st == NB_OK) st = hier_alloc(&t->d_leaf_rank, n);
  if (st == NB_OK) st = hier_alloc(&t->d_prank, n);
  if (st == NB_OK) st = hier_alloc(&t->d_pcnt, n);
  if (st == NB_OK) st = hier_alloc(&t->qoff[0], (size_t)n + 1);
  if (st == NB_OK) st = hier_alloc(&t->qoff[1], (size_t)n + 1);
  if (st == NB_OK) st = hier_alloc(&t->misc, 4);
  if (st == NB_OK && hipHostMalloc(reinterpret_cast<void**>(&t->host_sizes), 3 * sizeof(int64_t)) != hipSuccess) {
    nb_set_error("hipHostMalloc of the level sizes failed");
    st = NB_ERR_OOM;
  }
  if (st == NB_OK) {
    const size_t bytes = sizeof(int32_t) * n;
    if (hipMemcpy(t->d_child_b, t->child_b.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t->d_child_e, t->child_e.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t->d_parent, t->parent.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t->d_leaf_rank, t->leaf_rank.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
      nb_set_error("hipMemcpy of the tree failed");
      st = NB_ERR_HIP;
    }
  }
  if (st != NB_OK) {
    nb_hier_destroy(t);
    return st;
  }
  *out = t;
  return NB_OK;
}

nb_status nb_hier_destroy(nb_hier* t) {
  if (!t) return NB_OK;
  free_pair_set(t, 0);
  free_pair_set(t, 1);
  free_scan(t);
  hier_free(t->d_child_b);
  hier_free(t->d_child_e);
  hier_free(t->d_parent);
  hier_free(t->d_leaf_rank);
  hier_free(t->d_prank);
  hier_free(t->d_pcnt);
  hier_free(t->qoff[0]);
  hier_free(t->qoff[1]);
  hier_free(t->misc);
  if (t->host_sizes) (void)hipHostFree(t->host_sizes);
  delete t;
  return NB_OK;
}

nb_status nb_hier_num_leaves(const nb_hier* t, int32_t* out) {
  NB_REQUIRE(t && out, "NULL argument");
  *out = t->n_leaves;
  return NB_OK;
}

nb_status nb_hier_depth(const nb_hier* t, int32_t* depth) {
  NB_REQUIRE(t && depth, "NULL argument");
  *depth = (int32_t)t->lvl_first.size() - 1;
  return NB_OK;
}

nb_status nb_hier_level_pairs(const nb_hier* t, int64_t* pairs_host) {
  NB_REQUIRE(t && pairs_host, "NULL argument");
  const int depth = (int)t->lvl_first.size() - 1;
  for (int l = 0; l < depth; ++l) pairs_host[l] = l < (int)t->level_pairs.size() ? t->level_pairs[l] : 0;
  return NB_OK;
}

nb_status nb_hier_leaf_nodes(const nb_hier* t, int32_t* nodes_host) {
  NB_REQUIRE(t && nodes_host, "NULL argument");
  for (int p = 0; p < t->n_nodes; ++p)
    if (t->leaf_rank[p] >= 0) nodes_host[t->leaf_rank[p]] = p;
  return NB_OK;
}

nb_status nb_hier_query(nb_hier* t, const float* q, int64_t n, float eps, int32_t* qidx_out, int64_t cap,
                        int64_t* leaf_off, int64_t* n_pairs_host, void* stream) {
  NB_REQUIRE(t && q && leaf_off && n_pairs_host, "NULL argument");
  NB_REQUIRE(n > 0 && n <= (int64_t)0x7FFFFFFF, "n must be in 1 .. 2^31 - 1");
  NB_REQUIRE(cap >= 0 && (cap == 0 || qidx_out), "qidx_out must hold cap >= 0 entries");
  NB_REQUIRE(eps >= 0.0f && eps < 0.5f, "eps must be in [0, 0.5)");
  int dev = -1;
  NB_HIP(hipGetDevice(&dev));
  NB_REQUIRE(dev == t->device, "the hierarchy lives on device %d, the current device is %d", t->device, dev);
  hipStream_t s = as_stream(stream);
  const float tau = tau_of(eps);
  const int in_dim = t->g->in_dim;
  const int depth = (int)t->lvl_first.size() - 1;
  t->level_pairs.assign(depth, 0);
  NB_HIP(hipStreamSynchronize(s));
  // level 0: the root over the caller's rows, region index = row
  k_set_i64<<<1, 1, 0, s>>>(t->misc + 2, 0);
  NB_LAUNCHED();
  {
    std::vector<int64_t> q0((size_t)t->n_nodes + 1, n);
    q0[0] = 0;
    NB_HIP(hipMemcpyAsync(t->qoff[0], q0.data(), sizeof(int64_t) * q0.size(), hipMemcpyHostToDevice, s));
    NB_HIP(hipStreamSynchronize(s));
  }
  const float* rows = q;
  const int32_t* qidx = nullptr;
  int64_t rows_n = n, pairs_before = 0;
  int cur = 0;   // pair set read by this level (written by the previous level)
  for (int l = 0; l < depth; ++l) {
    const int la = t->lvl_first[l], lb = t->lvl_first[l + 1];
    const int na = l + 1 < depth ? t->lvl_first[l + 1] : t->n_nodes;
    const int nbn = l + 1 < depth ? t->lvl_first[l + 2] : t->n_nodes;
    const int empty = rows_n == 0;
    t->level_pairs[l] = rows_n;
    const int64_t* qoff = t->qoff[l & 1];
    int64_t* qoff_next = t->qoff[(l + 1) & 1];
    if (!empty) {
      NB_TRY(ensure_scan(t, rows_n));   // the stream is idle: synchronised below, and before the loop
      NB_TRY(group_forward(t->g, rows, qoff, rows_n, tau, nullptr, t->h, nullptr, nullptr, s));
      const int64_t nblk = (rows_n + kScanBlock - 1) / kScanBlock;
      k_flag_counts<<<(unsigned)nblk, kScanThreads, 0, s>>>(t->h, rows_n, t->bsum);
      NB_LAUNCHED();
      k_scan_blocks<<<1, kPrefixThreads, 0, s>>>(t->bsum, nblk, t->misc);
      NB_LAUNCHED();
      k_compact<<<(unsigned)nblk, kScanThreads, 0, s>>>(t->h, rows_n, t->bsum, t->pos_idx);
      NB_LAUNCHED();
    }
    k_hier_offsets<<<1, kScanThreads, 0, s>>>(t->n_nodes, la, lb, na, nbn, qoff, empty, t->pos_idx, t->misc,
                                             t->d_parent, t->d_leaf_rank, t->d_prank, t->d_pcnt, qoff_next, leaf_off,
                                             t->misc + 1);
    NB_LAUNCHED();
    NB_HIP(hipMemcpyAsync(t->host_sizes, t->misc, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    NB_HIP(hipStreamSynchronize(s));
    const int64_t next_n = t->host_sizes[1], pairs_after = t->host_sizes[2];
    NB_REQUIRE(next_n <= (int64_t)0x7FFFFFFF, "level %d holds %lld (region, node) pairs, more than 2^31 - 1", l + 1,
               (long long)next_n);
    if (!empty) {
      const int nxt = 1 - cur;
      const int64_t n_pos = t->host_sizes[0];   // this level's positives (the scan total)
      if (next_n > 0) NB_TRY(ensure_pairs(t, nxt, next_n));   // set nxt was read by the level before: finished
      if (n_pos > 0) {
        const size_t lds = sizeof(int64_t) * (size_t)(lb - la);   // at most 4096 x 8 B
        k_hier_expand<<<(unsigned)((n_pos + 255) / 256), 256, lds, s>>>(
            in_dim, n_pos, la, lb, t->d_prank, t->pos_idx, t->d_child_b, t->d_child_e, t->d_leaf_rank, qoff_next,
            leaf_off, rows, qidx, t->rows[nxt], t->qidx[nxt], qidx_out, cap);
        NB_LAUNCHED();
      }
      NB_HIP(hipStreamSynchronize(s));
      rows = t->rows[nxt];
      qidx = t->qidx[nxt];
      cur = nxt;
    }
    pairs_before = pairs_after;
    rows_n = next_n;
  }
  const int64_t pairs = t->host_sizes[2];
  k_set_i64<<<1, 1, 0, s>>>(leaf_off + t->n_leaves, pairs);
  NB_LAUNCHED();
  *n_pairs_host = pairs;
  NB_REQUIRE(pairs <= cap, "the traversal found %lld (region, leaf) pairs, more than cap = %lld", (long long)pairs,
             (long long)cap);
  return NB_OK;
}

}  // extern "C"
