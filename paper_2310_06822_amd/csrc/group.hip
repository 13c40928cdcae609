// Many per-object bounds in one launch.
//
// The paper trains one bound per object (Sec. 3.4, "Training": no
// generalisation across objects).  A group holds n_obj bfloat16 bounds of a
// common depth and input size but their own widths (32, 64 or 128), each
// with its own voxel grid.  Queries arrive grouped by object (CSR offsets).
//
// Forward: one persistent launch.  A single-block planner lays the work out
// as tiles of 128 queries, objects ordered by decreasing width, and gives
// each workgroup a contiguous run of tiles of equal estimated cost
// (proportional to width^2 per tile); a workgroup reloads weights into LDS
// only when its run crosses into the next object, so every object's weights
// are read about once per workgroup that touches it.
#include <algorithm>
#include <numeric>
#include <vector>

#include "nb_internal.h"
#include "nb_mlp.h"
#include "nb_adam.h"
#include "nb_bf16_fwd.h"
#include "nb_voxel.h"

namespace {

// Forward tile shapes (the variants the tuner picks from): threads per
// workgroup and 16-query blocks per wave; a work item (tile) is
// threads / 64 * blocks * 16 queries of one object.
struct GroupShape {
  int threads, blocks, wg_per_cu;
};
constexpr GroupShape kGroupShapes[] = {{256, 2, 4}, {512, 2, 2}, {256, 1, 4}, {512, 1, 2},
                                       {1024, 1, 1}, {768, 1, 2}};
constexpr int kGroupVariants = sizeof(kGroupShapes) / sizeof(kGroupShapes[0]);

// Fragments of an object's forward pack held in LDS: the first layer's first
// step and the hidden layers (the second first-layer step, used for input
// dimensions above 4, is read from global memory).
__host__ __device__ inline int frags_fwd(int W, int NH) { return W / 16 + (NH - 1) * (W / 16) * (W / 32); }

// Work plan: item_off[p] = first tile of the p-th object in width order;
// wg_first[w] = first tile of workgroup w (wg_first[G] = total tiles).  One
// block of 256 threads: prefix sums over objects (tiles and cost) by a block
// scan, then every thread places its workgroup boundaries by binary search,
// cutting the tile sequence at equal shares of the total cost.
constexpr int kMaxGroup = 4096;

// Relative time of one tile by width: measured per-query forward times of
// widths 32, 64 and 128 stand about 1 : 1.3 : 2.5 (the matrix work grows as
// W^2, the per-query input, activation and output work does not).
__device__ inline double tile_cost(int W) { return (double)W * W + 8192.0; }

__global__ __launch_bounds__(256) void k_group_plan(const int64_t* __restrict__ qoff, int64_t n, int tile_q, int n_obj,
                                                    const int* __restrict__ perm, const int* __restrict__ widths,
                                                    int G, int64_t* __restrict__ item_off,
                                                    int64_t* __restrict__ wg_first) {
  __shared__ double cum[kMaxGroup + 1];   // cost of the tiles before object p (width order)
  __shared__ int64_t sitem[kMaxGroup + 1];
  __shared__ double scost[256];
  __shared__ int64_t stile[256];
  // each thread takes a contiguous segment of objects; block scan of the
  // segment sums; then every thread writes its segment's prefixes
  const int t = threadIdx.x;
  const int seg = (n_obj + 255) / 256;
  const int p0 = min(n_obj, t * seg), p1 = min(n_obj, p0 + seg);
  auto tiles_of = [&](int p) -> int64_t {
    const int o = perm[p];
    const int64_t a = qoff[o], b = qoff[o + 1];   // rows outside [0, n): no tiles
    const int64_t nq = (a >= 0 && b <= n && b > a) ? b - a : 0;
    return (nq + tile_q - 1) / tile_q;
  };
  double c_sum = 0.0;
  int64_t t_sum = 0;
  for (int p = p0; p < p1; ++p) {
    const int64_t tl = tiles_of(p);
    t_sum += tl;
    c_sum += (double)tl * tile_cost(widths[perm[p]]);
  }
  scost[t] = c_sum;
  stile[t] = t_sum;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {   // inclusive scan
    const double cv = t >= d ? scost[t - d] : 0.0;
    const int64_t tv = t >= d ? stile[t - d] : 0;
    __syncthreads();
    scost[t] += cv;
    stile[t] += tv;
    __syncthreads();
  }
  double c_acc = t > 0 ? scost[t - 1] : 0.0;
  int64_t t_acc = t > 0 ? stile[t - 1] : 0;
  for (int p = p0; p < p1; ++p) {
    cum[p] = c_acc;
    sitem[p] = t_acc;
    const int64_t tl = tiles_of(p);
    t_acc += tl;
    c_acc += (double)tl * tile_cost(widths[perm[p]]);
  }
  if (t == 255) {
    cum[n_obj] = scost[255];
    sitem[n_obj] = stile[255];
  }
  __syncthreads();
  for (int p = threadIdx.x; p <= n_obj; p += blockDim.x) item_off[p] = sitem[p];
  const double total = cum[n_obj];
  const int64_t n_tiles = sitem[n_obj];
  for (int w = threadIdx.x; w <= G; w += blockDim.x) {
    int64_t t;
    if (w == 0) {
      t = 0;
    } else if (w == G) {
      t = n_tiles;
    } else {
      // smallest t with cost(tiles [0, t)) >= target
      const double target = total * (double)w / (double)G;
      int lo = 0, hi = n_obj;   // last p with cum[p] < target (cum[0] = 0)
      if (target <= 0.0) {
        t = 0;
      } else {
        while (hi - lo > 1) {
          const int mid = (lo + hi) / 2;
          if (cum[mid] < target) lo = mid; else hi = mid;
        }
        const int o = perm[lo];
        const double cost = tile_cost(widths[o]);
        const int64_t k = (int64_t)ceil((target - cum[lo]) / cost);
        t = sitem[lo] + k;
        if (t > sitem[lo + 1]) t = sitem[lo + 1];
      }
    }
    wg_first[w] = t;
  }
}

template <int NH>
struct GroupLds {
  static constexpr size_t bytes() {
    return (size_t)frags_fwd(128, NH) * 64 * 16 + (size_t)(NH * 128 + 129) * 4;
  }
};

// Adds a wave's confusion counts for object o to counts[o] and clears them.
__device__ __forceinline__ void flush_counts(unsigned long long* __restrict__ counts, int o, unsigned (&cnt)[4]) {
  if (counts && o >= 0) {
    if ((threadIdx.x & 63) == 0)
      for (int i = 0; i < 4; ++i)
        if (cnt[i]) atomicAdd(counts + (int64_t)o * 4 + i, (unsigned long long)cnt[i]);
    cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0u;
  }
}

template <int NH, int THREADS, int NB>
__global__ __launch_bounds__(THREADS) void k_group_fwd(
    const float* __restrict__ q, const int64_t* __restrict__ qoff, int n_obj, int in_dim,
    const int* __restrict__ perm, const int* __restrict__ widths, const int64_t* __restrict__ poff,
    const int64_t* __restrict__ pkoff, const float* __restrict__ theta, const bf16x8* __restrict__ pack,
    const int64_t* __restrict__ item_off, const int64_t* __restrict__ wg_first, float tau,
    float* __restrict__ logits, uint8_t* __restrict__ hout, const uint8_t* __restrict__ g,
    unsigned long long* __restrict__ counts) {
  constexpr int TILE = THREADS / 64 * NB * 16;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  bf16x8* swt = reinterpret_cast<bf16x8*>(smem_raw);
  float* sbias = reinterpret_cast<float*>(smem_raw + (size_t)frags_fwd(128, NH) * 64 * 16);
  const int64_t s = wg_first[blockIdx.x], e = wg_first[blockIdx.x + 1];
  if (s >= e) return;
  // object (in width order) of the first tile
  int p = 0;
  {
    int lo = 0, hi = n_obj;   // last p with item_off[p] <= s
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (item_off[mid] <= s) lo = mid; else hi = mid;
    }
    p = lo;
  }
  int cur = -1, W = 0;
  const bf16x8* sext = pack;   // the current object's second first-layer step
  unsigned cnt[4] = {0u, 0u, 0u, 0u};
  const int wave = threadIdx.x >> 6, c = threadIdx.x & 15;
  // software pipeline: the next tile's inputs load while this tile computes
  float xr[NB][8];
  int64_t q0 = qoff[perm[p]] + (s - item_off[p]) * TILE + wave * (NB * 16);
  int64_t n_end = qoff[perm[p] + 1];
  load_raw<NB>(q, n_end, in_dim, q0, c, xr);
  for (int64_t it = s; it < e; ++it) {
    const int o = perm[p];
    if (o != cur) {
      flush_counts(counts, cur, cnt);
      __syncthreads();
      W = widths[o];
      const int nf = frags_fwd(W, NH);
      const bf16x8* src = pack + pkoff[o];
      sext = src + nf * 64;
      for (int i = threadIdx.x; i < nf * 64; i += THREADS) swt[i] = src[i];
      const float* th = theta + poff[o];
      for (int i = threadIdx.x; i < NH * W; i += THREADS) sbias[i] = th[nb_b_off(i / W, in_dim, W, NH) + i % W];
      for (int i = threadIdx.x; i < W + 1; i += THREADS) sbias[NH * W + i] = th[nb_w_off(NH, in_dim, W) + i];
      __syncthreads();
      cur = o;
    }
    float xn[NB][8];
    int64_t q0n = 0, n_endn = 0;
    if (it + 1 < e) {
      while (it + 1 >= item_off[p + 1]) ++p;
      const int on = perm[p];
      q0n = qoff[on] + (it + 1 - item_off[p]) * TILE + wave * (NB * 16);
      n_endn = qoff[on + 1];
      load_raw<NB>(q, n_endn, in_dim, q0n, c, xn);
    }
    if (W == 32)
      bf16_fwd_tile_x<32, NH, NB>(swt, sbias, xr, in_dim > 4, sext, n_end, q0, tau, logits, hout, g, counts, cnt);
    else if (W == 64)
      bf16_fwd_tile_x<64, NH, NB>(swt, sbias, xr, in_dim > 4, sext, n_end, q0, tau, logits, hout, g, counts, cnt);
    else
      bf16_fwd_tile_x<128, NH, NB>(swt, sbias, xr, in_dim > 4, sext, n_end, q0, tau, logits, hout, g, counts, cnt);
    if (it + 1 < e) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int j = 0; j < 8; ++j) xr[nb][j] = xn[nb][j];
      q0 = q0n;
      n_end = n_endn;
    }
  }
  flush_counts(counts, cur, cnt);
}

// Grouped exact query: every query finds its object by binary search over
// the CSR offsets and runs the voxel test on that object's grid (boxes
// through the object's count table when `table` is non-null).
__global__ void k_group_exact(int kind, const float* __restrict__ q, const int64_t* __restrict__ qoff, int n_obj,
                              int64_t n, const uint8_t* __restrict__ grids, const int64_t* __restrict__ goff,
                              const int* __restrict__ gn, const float* __restrict__ ray_t,
                              const int32_t* __restrict__ table, const int64_t* __restrict__ toff,
                              uint8_t* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i < qoff[0] || i >= qoff[n_obj]) return;
  int lo = 0, hi = n_obj;   // last o with qoff[o] <= i
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (qoff[mid] <= i) lo = mid; else hi = mid;
  }
  if (kind == 2 && table)
    g[i] = voxel_box_table_at(q + 6 * i, table + toff[lo], gn[lo]);
  else
    g[i] = nb_voxel_query(kind, q, i, grids + goff[lo], gn[lo], ray_t);
}

// Count tables (one object per blockIdx.y), built in three passes of
// running sums over lines of the (n+1)^3 table: along x from the grid's
// rows (plane x = 0 and the faces y = 0, z = 0 are zero), then along y,
// then along z.
__global__ void k_table_x(const uint8_t* __restrict__ grids, const int64_t* __restrict__ goff,
                          const int* __restrict__ gns, const int64_t* __restrict__ toff, int32_t* __restrict__ T) {
  const int o = blockIdx.y, n = gns[o];
  const int64_t m = n + 1;
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (k, j)
  if (line >= m * m) return;
  const int64_t k = line / m, j = line % m;
  int32_t* row = T + toff[o] + line * m;
  row[0] = 0;
  if (k == 0 || j == 0) {
    for (int64_t i = 1; i < m; ++i) row[i] = 0;
    return;
  }
  int32_t acc = 0;
  const uint8_t* src = grids + goff[o] + ((k - 1) * n + (j - 1)) * n;
  for (int64_t i = 1; i < m; ++i) {
    acc += src[i - 1] != 0;
    row[i] = acc;
  }
}

__global__ void k_table_yz(const int* __restrict__ gns, const int64_t* __restrict__ toff, int32_t* __restrict__ T,
                           int axis) {
  const int o = blockIdx.y;
  const int64_t m = gns[o] + 1;
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= m * m) return;
  int32_t* base = T + toff[o];
  int64_t start, stride;
  if (axis == 1) {   // along y: line = (k, i)
    start = (line / m) * m * m + line % m;
    stride = m;
  } else {           // along z: line = (j, i)
    start = line;
    stride = m * m;
  }
  int32_t acc = 0;
  for (int64_t t = 0; t < m; ++t) {
    acc += base[start + t * stride];
    base[start + t * stride] = acc;
  }
}

// Grouped pack: every element of every object's forward and transposed
// fragments; blockIdx.y is the object, x strides over its elements (forward
// pack first, then the transposed one).
__global__ void k_group_pack(const float* __restrict__ theta, const int64_t* __restrict__ poff,
                             const int64_t* __restrict__ pkoff, const int64_t* __restrict__ ptoff,
                             const int* __restrict__ widths, int in_dim, int NH, uint16_t* __restrict__ pack,
                             uint16_t* __restrict__ packT) {
  const int o = blockIdx.y;
  const int64_t nf = (pkoff[o + 1] - pkoff[o]) * 8, nt = (ptoff[o + 1] - ptoff[o]) * 8;
  const float* th = theta + poff[o];
  const int W = widths[o];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nf + nt;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nf)
      pack[pkoff[o] * 8 + e] = nb_bf16_pack_elem(th, in_dim, W, NH, e);
    else
      packT[ptoff[o] * 8 + (e - nf)] =
          nb_bf16_pack_t_elem(th, in_dim, W, NH, e - nf, nb_bf16_fused_shape(in_dim, NH, W));
  }
}

// Sum of the per-chunk partials of every parameter of every object, then one
// Adam step.  blockIdx.y is the object, one thread per parameter; the chunks
// are summed as for a single bound (eight strided partial sums, each in
// chunk order, then added in order), so a group member's update is bit for
// bit a single bound's.
__global__ __launch_bounds__(256) void k_group_reduce(const float* __restrict__ partial, int n_wg,
                                                      const int64_t* __restrict__ poff, const int* __restrict__ widths,
                                                      int in_dim, int NH, float* __restrict__ theta,
                                                      float* __restrict__ m, float* __restrict__ v, AdamArgs adam,
                                                      const float* __restrict__ lr_obj,
                                                      const uint8_t* __restrict__ active,
                                                      unsigned* __restrict__ nonfinite) {
  const int o = blockIdx.y;
  // an object outside the trained set has no partials this step; a learning
  // rate of 0 freezes it
  if (!active[o] || (lr_obj && lr_obj[o] == 0.0f)) return;
  const int64_t Po = poff[o + 1] - poff[o];
  const int64_t pl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pl >= Po) return;
  const float* base = partial + (int64_t)n_wg * poff[o] + pl;
  float part[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for (int w = 0; w < n_wg; ++w) part[w & 7] += base[(int64_t)w * Po];
  float tot = part[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) tot += part[i];
  if (!isfinite(tot)) *nonfinite = 1u;
  AdamArgs a = adam;
  if (lr_obj) a.lr = lr_obj[o];
  // a learning rate of 0 freezes the object: parameters and moments stay
  if (a.lr != 0.0f) nb_adam_update(poff[o] + pl, tot, theta, m, v, a, nb_is_weight(pl, in_dim, widths[o], NH) != 0);
}

// Per-object mean loss and confusion counts of a grouped training step.
__global__ void k_group_aux(const float* __restrict__ aux, int n_wg, int n_obj, float loss_scale,
                            const uint8_t* __restrict__ active, float* __restrict__ loss,
                            unsigned long long* __restrict__ counts) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_obj || !active[o]) return;
  float ls = 0.0f;
  unsigned long long cs[4] = {0, 0, 0, 0};
  const float* a = aux + (int64_t)o * n_wg * 8;
  for (int w = 0; w < n_wg; ++w) {
    ls += a[w * 8];
    for (int i = 0; i < 4; ++i) cs[i] += __float_as_uint(a[w * 8 + 1 + i]);
  }
  if (loss) loss[o] = ls * loss_scale;
  if (counts)
    for (int i = 0; i < 4; ++i) counts[(int64_t)o * 4 + i] = cs[i];
}

}  // namespace

// ------------------------------------------------------------------ host side

nb_status group_reduce_adam(const nb_group* gr, int n_wg, const AdamArgs& adam, const float* lr_obj, float* loss,
                            unsigned long long* counts, float loss_scale, hipStream_t s) {
  const dim3 grid((unsigned)((gr->max_obj_params + 255) / 256), (unsigned)gr->n_obj);
  k_group_reduce<<<grid, 256, 0, s>>>(gr->partial, n_wg, gr->d_poff, gr->d_widths, gr->in_dim, gr->n_hidden, gr->theta,
                                      gr->m, gr->v, adam, lr_obj, gr->d_active, gr->d_nonfinite);
  NB_LAUNCHED();
  if (loss || counts) {
    k_group_aux<<<(unsigned)((gr->n_obj + 255) / 256), 256, 0, s>>>(gr->aux, n_wg, gr->n_obj, loss_scale,
                                                                   gr->d_active, loss, counts);
    NB_LAUNCHED();
  }
  return NB_OK;
}

int group_variants() { return kGroupVariants; }

namespace {

// Workgroups of a persistent launch: as many as fit on the chip at once
// (LDS holds the widest object's weights).
int group_wgs(const GroupShape& sh, size_t lds) {
  const int fit = std::max(1, (int)((160 * 1024) / lds));
  return std::max(1, std::min(std::min(sh.wg_per_cu, fit) * nb_cu_count(), 1 << 14));
}

size_t group_lds(int NH) {
  switch (NH) {
    case 2: return GroupLds<2>::bytes();
    case 3: return GroupLds<3>::bytes();
    default: return GroupLds<4>::bytes();
  }
}

template <int NH, int THREADS, int NB>
nb_status group_fwd_launch(const nb_group* gr, const float* q, const int64_t* qoff, int G, float tau,
                           float* logits, uint8_t* h, const uint8_t* g, unsigned long long* counts, hipStream_t s) {
  const size_t lds = GroupLds<NH>::bytes();
  static bool attr[64] = {false};
  int dev = 0;
  NB_HIP(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && !attr[dev]) {
    NB_HIP(hipFuncSetAttribute((const void*)k_group_fwd<NH, THREADS, NB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
    attr[dev] = true;
  }
  k_group_fwd<NH, THREADS, NB><<<G, THREADS, lds, s>>>(
      q, qoff, gr->n_obj, gr->in_dim, gr->d_perm, gr->d_widths, gr->d_poff, gr->d_pkoff, gr->theta,
      reinterpret_cast<const bf16x8*>(gr->pack16), gr->d_item_off, gr->d_wg_first, tau, logits, h, g, counts);
  NB_LAUNCHED();
  return NB_OK;
}

template <int NH>
nb_status group_fwd_nh(const nb_group* gr, int variant, const float* q, const int64_t* qoff, int G, float tau,
                       float* logits, uint8_t* h, const uint8_t* g, unsigned long long* counts, hipStream_t s) {
  switch (variant) {
    case 0: return group_fwd_launch<NH, 256, 2>(gr, q, qoff, G, tau, logits, h, g, counts, s);
    case 1: return group_fwd_launch<NH, 512, 2>(gr, q, qoff, G, tau, logits, h, g, counts, s);
    case 2: return group_fwd_launch<NH, 256, 1>(gr, q, qoff, G, tau, logits, h, g, counts, s);
    case 3: return group_fwd_launch<NH, 512, 1>(gr, q, qoff, G, tau, logits, h, g, counts, s);
    case 4: return group_fwd_launch<NH, 1024, 1>(gr, q, qoff, G, tau, logits, h, g, counts, s);
    case 5: return group_fwd_launch<NH, 768, 1>(gr, q, qoff, G, tau, logits, h, g, counts, s);
    default: break;
  }
  nb_set_error("grouped forward variant %d out of range", variant);
  return NB_ERR_INVALID_ARG;
}

}  // namespace

nb_status group_forward(const nb_group* gr, const float* q, const int64_t* qoff, int64_t n, float tau,
                        float* logits, uint8_t* h, const uint8_t* g, unsigned long long* counts, hipStream_t s) {
  const int v = gr->variant;
  if (v < 0 || v >= kGroupVariants) {
    nb_set_error("grouped forward variant %d out of range", v);
    return NB_ERR_INVALID_ARG;
  }
  const GroupShape sh = kGroupShapes[v];
  const int G = std::min(group_wgs(sh, group_lds(gr->n_hidden)), gr->n_wg_cap);
  const int tile_q = sh.threads / 64 * sh.blocks * 16;
  if (counts) NB_TRY(launch_zero_u64(counts, 4 * gr->n_obj, s));
  k_group_plan<<<1, 256, 0, s>>>(qoff, n, tile_q, gr->n_obj, gr->d_perm, gr->d_widths, G, gr->d_item_off,
                                 gr->d_wg_first);
  NB_LAUNCHED();
  switch (gr->n_hidden) {
    case 2: return group_fwd_nh<2>(gr, v, q, qoff, G, tau, logits, h, g, counts, s);
    case 3: return group_fwd_nh<3>(gr, v, q, qoff, G, tau, logits, h, g, counts, s);
    case 4: return group_fwd_nh<4>(gr, v, q, qoff, G, tau, logits, h, g, counts, s);
    default: break;
  }
  nb_set_error("grouped forward supports 2..4 hidden layers");
  return NB_ERR_UNSUPPORTED;
}

nb_status group_exact(const nb_group* gr, int kind, const float* q, const int64_t* qoff, int64_t n, uint8_t* g,
                      hipStream_t s) {
  const bool table = gr->box_method == 1 && gr->table;
  k_group_exact<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(kind, q, qoff, gr->n_obj, n, gr->grids, gr->d_goff,
                                                           gr->d_gn, gr->ray_t, table ? gr->table : nullptr,
                                                           gr->d_toff, g);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status group_build_tables(const nb_group* gr, int max_n, hipStream_t s) {
  const int64_t lines = (int64_t)(max_n + 1) * (max_n + 1);
  const dim3 grid((unsigned)((lines + 255) / 256), (unsigned)gr->n_obj);
  k_table_x<<<grid, 256, 0, s>>>(gr->grids, gr->d_goff, gr->d_gn, gr->d_toff, gr->table);
  NB_LAUNCHED();
  k_table_yz<<<grid, 256, 0, s>>>(gr->d_gn, gr->d_toff, gr->table, 1);
  NB_LAUNCHED();
  k_table_yz<<<grid, 256, 0, s>>>(gr->d_gn, gr->d_toff, gr->table, 2);
  NB_LAUNCHED();
  return NB_OK;
}

nb_status group_pack(const nb_group* gr, hipStream_t s) {
  const dim3 grid(64, (unsigned)gr->n_obj);
  k_group_pack<<<grid, 256, 0, s>>>(gr->theta, gr->d_poff, gr->d_pkoff, gr->d_ptoff, gr->d_widths, gr->in_dim,
                                    gr->n_hidden, gr->pack16, gr->pack16t);
  NB_LAUNCHED();
  return NB_OK;
}
