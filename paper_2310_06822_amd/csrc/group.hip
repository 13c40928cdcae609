// Many per-object bounds queried and trained together.
//
// The paper trains one bound per object (Sec. 3.4, "Training": no
// generalisation across objects).  A group holds n_obj bfloat16 bounds of a
// common depth and input size but their own widths (32, 64 or 128), each
// with its own voxel grid.  Queries arrive grouped by object (CSR offsets).
//
// Forward: one persistent launch per width class, each kernel compiled for
// its width so that its registers and LDS (not the widest class's) set its
// occupancy.  A planner lays every class's work out as tiles of queries of
// one object, objects ordered by decreasing width, and gives each workgroup
// of the class an equal contiguous run of tiles; a workgroup reloads weights
// into LDS only when its run crosses into the next object, so every object's
// weights are read about once per workgroup that touches it.
#include <algorithm>
#include <numeric>
#include <vector>

#include "nb_internal.h"
#include "nb_mlp.h"
#include "nb_adam.h"
#include "nb_bf16_fwd.h"
#include "nb_voxel.h"

namespace {

// Forward tile shapes (the variants the tuner picks from, per width class):
// threads per workgroup and 16-query blocks per wave; a work item (tile) is
// threads / 64 * blocks * 16 queries of one object.  Width 128 takes at most
// two blocks per wave (four would not fit its accumulators in registers).
struct GroupShape {
  int threads, blocks;
};
constexpr GroupShape kGroupShapes[] = {{256, 2}, {512, 2}, {256, 1}, {512, 1},
                                       {1024, 1}, {768, 1}, {256, 4}, {512, 4}};
constexpr int kGroupVariants = sizeof(kGroupShapes) / sizeof(kGroupShapes[0]);
__host__ __device__ constexpr int group_blocks(int W, int blocks) { return W >= 128 && blocks > 2 ? 2 : blocks; }

// Fragments of an object's forward pack held in LDS: the pack's first
// first-layer step (unused here: the grouped kernel runs the first layer in
// float32) and the hidden layers, then the biases and output weights.
__host__ __device__ constexpr int frags_fwd(int W, int NH) { return W / 16 + (NH - 1) * (W / 16) * (W / 32); }
__host__ __device__ constexpr size_t group_lds_bytes(int W, int NH) {
  return (size_t)frags_fwd(W, NH) * 64 * 16 + (size_t)(NH * W + W + 1) * 4;
}

// The inputs of one wave's NB blocks of 16 queries that the float32 first
// layer takes from a lane: features grp and grp + 4 of query column c, as
// loaded (col_inputs masks them).  Every load reads a row of the object (its
// last row for padding queries, the last feature for features >= in_dim),
// so none is predicated; each block's row base is wave-uniform, the lane's
// offset from it 32-bit.
template <int NB>
__device__ __forceinline__ void load_cols(const float* __restrict__ q, int64_t n, int in_dim, int64_t q0, int c,
                                          int grp, float (&x)[NB][2]) {
  const int f0 = grp < in_dim ? grp : in_dim - 1, f1 = grp + 4 < in_dim ? grp + 4 : in_dim - 1;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t b0 = q0 + nb * 16;
    // rows b0 .. b0 + nv - 1 are the object's; a block wholly past its end
    // reads its last row
    const int nv = n - b0 <= 0 ? 0 : (n - b0 >= 16 ? 16 : (int)(n - b0));
    const float* base = q + (nv > 0 ? b0 : n - 1) * in_dim;
    const int r = c < nv ? c : (nv > 0 ? nv - 1 : 0);
    x[nb][0] = base[r * in_dim + f0];
    x[nb][1] = base[r * in_dim + f1];
  }
}

// The loaded inputs with features >= in_dim and queries >= n set to zero.
template <int NB>
__device__ __forceinline__ void col_inputs(const float (&raw)[NB][2], int64_t n, int in_dim, int64_t q0, int c,
                                           int grp, float (&x)[NB][2]) {
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t b0 = q0 + nb * 16;
    const int nv = n - b0 <= 0 ? 0 : (n - b0 >= 16 ? 16 : (int)(n - b0));
    x[nb][0] = c < nv && grp < in_dim ? raw[nb][0] : 0.0f;
    x[nb][1] = c < nv && grp + 4 < in_dim ? raw[nb][1] : 0.0f;
  }
}

__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One width class of a grouped forward: the objects perm[p_lo .. p_lo +
// n_obj) (all of one width), G workgroups, tiles of tile_q queries; its plan
// goes to item_off[item_base ..] and wg_first[wg_base ..].
struct ClassPlan {
  int p_lo, n_obj, G, tile_q, item_base, wg_base;
};
struct GroupPlan {
  ClassPlan c[3];
};

// Work plan, one block of 256 threads per width class (blockIdx.x):
// item_off[p] = first tile of the class's p-th object, item_off[n_obj] = the
// class's tiles; wg_first[w] = first tile of workgroup w (wg_first[G] = all
// tiles).  Every tile of a class costs the same, so the workgroups take
// equal shares of the tile sequence: a block scan of the objects' tile
// counts, then one division per workgroup boundary.
__global__ __launch_bounds__(256) void k_group_plan(const int64_t* __restrict__ qoff, int64_t n, GroupPlan plan,
                                                    const int* __restrict__ perm, int64_t* __restrict__ item_off,
                                                    int64_t* __restrict__ wg_first) {
  __shared__ int64_t stile[256];
  const ClassPlan cp = plan.c[blockIdx.x];
  const int* pm = perm + cp.p_lo;
  int64_t* io = item_off + cp.item_base;
  int64_t* wf = wg_first + cp.wg_base;
  const int t = threadIdx.x, n_obj = cp.n_obj;
  // each thread takes a contiguous segment of objects; block scan of the
  // segment sums; then every thread writes its segment's prefixes
  const int seg = (n_obj + 255) / 256;
  const int p0 = min(n_obj, t * seg), p1 = min(n_obj, p0 + seg);
  auto tiles_of = [&](int p) -> int64_t {
    const int o = pm[p];
    const int64_t a = qoff[o], b = qoff[o + 1];   // rows outside [0, n): no tiles
    const int64_t nq = (a >= 0 && b <= n && b > a) ? b - a : 0;
    return (nq + cp.tile_q - 1) / cp.tile_q;
  };
  int64_t t_sum = 0;
  for (int p = p0; p < p1; ++p) t_sum += tiles_of(p);
  stile[t] = t_sum;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {   // inclusive scan
    const int64_t tv = t >= d ? stile[t - d] : 0;
    __syncthreads();
    stile[t] += tv;
    __syncthreads();
  }
  int64_t t_acc = t > 0 ? stile[t - 1] : 0;
  for (int p = p0; p < p1; ++p) {
    io[p] = t_acc;
    t_acc += tiles_of(p);
  }
  const int64_t n_tiles = stile[255];
  if (t == 0) io[n_obj] = n_tiles;
  for (int w = t; w <= cp.G; w += 256) wf[w] = n_tiles * w / cp.G;
}

// Adds a wave's confusion counts for object o to counts[o] and clears them.
__device__ __forceinline__ void flush_counts(unsigned long long* __restrict__ counts, int o, unsigned (&cnt)[4]) {
  if (counts && o >= 0) {
    if ((threadIdx.x & 63) == 0)
      for (int i = 0; i < 4; ++i)
        if (cnt[i]) atomicAdd(counts + (int64_t)o * 4 + i, (unsigned long long)cnt[i]);
    cnt[0] = cnt[1] = cnt[2] = cnt[3] = 0u;
  }
}

// Forward + decision of one width class: a persistent workgroup runs its
// share of the class's tiles in order, reloading weights into LDS when the
// run crosses into the next object (so every object's weights are read
// about once per workgroup that touches it).  perm, item_off and wg_first
// are the class's.  The first layer runs on the float32 matrix cores
// (16x16x4: lane group g supplies features g and g + 4, so a lane loads two
// inputs and holds its slice of the first-layer weights in registers for
// the whole object); the hidden layers and the output as for single bounds.
template <int W, int NH, int THREADS, int NB>
__global__ __launch_bounds__(THREADS) void k_group_fwd(
    const float* __restrict__ q, const int64_t* __restrict__ qoff, int n_obj, int in_dim,
    const int* __restrict__ perm, const int64_t* __restrict__ poff, const int64_t* __restrict__ pkoff,
    const float* __restrict__ theta, const bf16x8* __restrict__ pack, const int64_t* __restrict__ item_off,
    const int64_t* __restrict__ wg_first, float tau, float* __restrict__ logits, uint8_t* __restrict__ hout,
    const uint8_t* __restrict__ g, unsigned long long* __restrict__ counts) {
  constexpr int TILE = THREADS / 64 * NB * 16;
  constexpr int NF = frags_fwd(W, NH), RB = W / 16;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  bf16x8* swt = reinterpret_cast<bf16x8*>(smem_raw);
  float* sbias = reinterpret_cast<float*>(smem_raw + (size_t)NF * 64 * 16);
  const int64_t s = wg_first[blockIdx.x], e = wg_first[blockIdx.x + 1];
  if (s >= e) return;
  // object (in the class's order) of the first tile
  int p = 0;
  {
    int lo = 0, hi = n_obj;   // last p with item_off[p] <= s
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (item_off[mid] <= s) lo = mid; else hi = mid;
    }
    p = lo;
  }
  int cur = -1;
  const bool wide = in_dim > 4;
  unsigned cnt[4] = {0u, 0u, 0u, 0u};
  // the wave index as a uniform value, so that tile offsets and row bases
  // stay in scalar registers
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), c = lane & 15,
            grp = lane >> 4;
  float w1[RB][2];   // first-layer weights W1[16 mo + c][grp + 4 s] of the current object
  // software pipeline: the next tile's inputs load into the other of two
  // buffers while this tile computes (two tiles per loop turn, so that no
  // copy between the buffers waits for the loads)
  auto tile = [&](int64_t it, const float (&xr)[NB][2], int64_t q0, int64_t n_end, float (&xn)[NB][2],
                  int64_t& q0n, int64_t& n_endn) {
    const int o = perm[p];
    if (o != cur) {
      flush_counts(counts, cur, cnt);
      __syncthreads();
      const bf16x8* src = pack + pkoff[o];
      for (int i = threadIdx.x; i < NF * 64; i += THREADS) swt[i] = src[i];
      const float* th = theta + poff[o];
      for (int i = threadIdx.x; i < NH * W; i += THREADS) sbias[i] = th[nb_b_off(i / W, in_dim, W, NH) + i % W];
      for (int i = threadIdx.x; i < W + 1; i += THREADS) sbias[NH * W + i] = th[nb_w_off(NH, in_dim, W) + i];
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int k = grp + 4 * t;
          w1[mo][t] = k < in_dim ? th[(int64_t)(16 * mo + c) * in_dim + k] : 0.0f;
        }
      __syncthreads();
      cur = o;
    }
    if (it + 1 < e) {
      while (it + 1 >= item_off[p + 1]) ++p;
      const int on = perm[p];
      q0n = qoff[on] + (it + 1 - item_off[p]) * TILE + wave * (NB * 16);
      n_endn = qoff[on + 1];
      load_cols<NB>(q, n_endn, in_dim, q0n, c, grp, xn);
    }
    // the loads stay ahead of this tile's work
    asm volatile("" ::: "memory");
    float x[NB][2];
    col_inputs<NB>(xr, n_end, in_dim, q0, c, grp, x);
    // query columns with a non-finite input: OR over the column's four lanes
    bool bad[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const unsigned long long m = __ballot(!isfinite(x[nb][0]) || !isfinite(x[nb][1]));
      bad[nb] = ((m | (m >> 16) | (m >> 32) | (m >> 48)) >> c) & 1ull;
    }
    floatx4 acc[NB][RB];
#pragma unroll
    for (int mo = 0; mo < RB; ++mo) {
      const floatx4 bi = *reinterpret_cast<const floatx4*>(sbias + 16 * mo + 4 * grp);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb][mo] = mfma_f32(w1[mo][0], x[nb][0], bi);
    }
    if (wide) {
#pragma unroll
      for (int mo = 0; mo < RB; ++mo)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb][mo] = mfma_f32(w1[mo][1], x[nb][1], acc[nb][mo]);
    }
    bf16_fwd_rest<W, NH, NB>(acc, bad, swt, sbias, n_end, q0, tau, logits, hout, g, counts, cnt);
  };
  float xa[NB][2], xb[NB][2];
  int64_t qa = qoff[perm[p]] + (s - item_off[p]) * TILE + wave * (NB * 16), na = qoff[perm[p] + 1];
  int64_t qb = 0, nb_end = 0;
  load_cols<NB>(q, na, in_dim, qa, c, grp, xa);
  for (int64_t it = s; it < e; it += 2) {
    tile(it, xa, qa, na, xb, qb, nb_end);
    if (it + 1 < e) tile(it + 1, xb, qb, nb_end, xa, qa, na);
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

// Arguments of one width class's forward launch.
struct ClassLaunch {
  const nb_group* gr;
  const float* q;
  const int64_t* qoff;
  float tau;
  float* logits;
  uint8_t* h;
  const uint8_t* g;
  unsigned long long* counts;
  hipStream_t s;
  ClassPlan cp;
};

// With launch false: sets the class's workgroup count (as many as are
// resident on the device at once for this kernel's registers and LDS, from
// the occupancy calculator, capped at the plan's capacity) and tile size.
// With launch true: launches the class's forward with that plan.
template <int W, int NH, int THREADS, int NB>
nb_status class_fwd(bool launch, ClassLaunch& a) {
  constexpr size_t lds = group_lds_bytes(W, NH);
  static_assert(lds <= 160 * 1024, "grouped forward LDS");
  const void* fn = reinterpret_cast<const void*>(k_group_fwd<W, NH, THREADS, NB>);
  static int resident[64] = {0};
  int dev = 0;
  NB_HIP(hipGetDevice(&dev));
  NB_REQUIRE(dev >= 0 && dev < 64, "device %d out of range", dev);
  if (!resident[dev]) {
    NB_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int per_cu = 0;
    NB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, THREADS, lds));
    resident[dev] = std::max(1, per_cu) * nb_cu_count();
  }
  if (!launch) {
    a.cp.G = std::max(1, std::min(resident[dev], a.gr->n_wg_cap));
    a.cp.tile_q = THREADS / 64 * NB * 16;
    return NB_OK;
  }
  const nb_group* gr = a.gr;
  k_group_fwd<W, NH, THREADS, NB><<<a.cp.G, THREADS, lds, a.s>>>(
      a.q, a.qoff, a.cp.n_obj, gr->in_dim, gr->d_perm + a.cp.p_lo, gr->d_poff, gr->d_pkoff, gr->theta,
      reinterpret_cast<const bf16x8*>(gr->pack16), gr->d_item_off + a.cp.item_base, gr->d_wg_first + a.cp.wg_base,
      a.tau, a.logits, a.h, a.g, a.counts);
  NB_LAUNCHED();
  return NB_OK;
}

template <int W, int NH>
nb_status class_fwd_v(int variant, bool launch, ClassLaunch& a) {
  switch (variant) {
    case 0: return class_fwd<W, NH, 256, group_blocks(W, 2)>(launch, a);
    case 1: return class_fwd<W, NH, 512, group_blocks(W, 2)>(launch, a);
    case 2: return class_fwd<W, NH, 256, 1>(launch, a);
    case 3: return class_fwd<W, NH, 512, 1>(launch, a);
    case 4: return class_fwd<W, NH, 1024, 1>(launch, a);
    case 5: return class_fwd<W, NH, 768, 1>(launch, a);
    case 6: return class_fwd<W, NH, 256, group_blocks(W, 4)>(launch, a);
    case 7: return class_fwd<W, NH, 512, group_blocks(W, 4)>(launch, a);
    default: break;
  }
  nb_set_error("grouped forward variant %d out of range", variant);
  return NB_ERR_INVALID_ARG;
}

template <int NH>
nb_status class_fwd_w(int W, int variant, bool launch, ClassLaunch& a) {
  switch (W) {
    case 32: return class_fwd_v<32, NH>(variant, launch, a);
    case 64: return class_fwd_v<64, NH>(variant, launch, a);
    case 128: return class_fwd_v<128, NH>(variant, launch, a);
    default: break;
  }
  nb_set_error("grouped forward width %d not supported", W);
  return NB_ERR_UNSUPPORTED;
}

nb_status class_fwd_any(int NH, int W, int variant, bool launch, ClassLaunch& a) {
  switch (NH) {
    case 2: return class_fwd_w<2>(W, variant, launch, a);
    case 3: return class_fwd_w<3>(W, variant, launch, a);
    case 4: return class_fwd_w<4>(W, variant, launch, a);
    default: break;
  }
  nb_set_error("grouped forward supports 2..4 hidden layers");
  return NB_ERR_UNSUPPORTED;
}

}  // namespace

// One persistent launch per width class (widths 128, 64, 32: the order of
// d_perm), each kernel compiled for its own width, so that a narrow class
// runs at the occupancy its own registers and LDS allow; one planner launch
// lays out all classes first.
nb_status group_forward(const nb_group* gr, const float* q, const int64_t* qoff, int64_t n, float tau,
                        float* logits, uint8_t* h, const uint8_t* g, unsigned long long* counts, hipStream_t s) {
  ClassLaunch a{gr, q, qoff, tau, logits, h, g, counts, s, {}};
  GroupPlan plan{};
  int nc = 0, widths[3] = {0, 0, 0}, variants[3] = {0, 0, 0};
  int p_lo = 0, item_base = 0, wg_base = 0;
  for (int c = 2; c >= 0; --c) {
    const int cnt = gr->class_all[c];
    if (cnt == 0) continue;
    const int v = gr->class_variant[c];
    if (v < 0 || v >= kGroupVariants) {
      nb_set_error("grouped forward variant %d out of range", v);
      return NB_ERR_INVALID_ARG;
    }
    a.cp = ClassPlan{p_lo, cnt, 0, 0, item_base, wg_base};
    NB_TRY(class_fwd_any(gr->n_hidden, 32 << c, v, false, a));
    plan.c[nc] = a.cp;
    widths[nc] = 32 << c;
    variants[nc] = v;
    ++nc;
    p_lo += cnt;
    item_base += cnt + 1;
    wg_base += a.cp.G + 1;
  }
  NB_REQUIRE(p_lo == gr->n_obj, "group widths must be 32, 64 or 128");
  if (counts) NB_TRY(launch_zero_u64(counts, 4 * gr->n_obj, s));
  k_group_plan<<<nc, 256, 0, s>>>(qoff, n, plan, gr->d_perm, gr->d_item_off, gr->d_wg_first);
  NB_LAUNCHED();
  for (int i = 0; i < nc; ++i) {
    a.cp = plan.c[i];
    NB_TRY(class_fwd_any(gr->n_hidden, widths[i], variants[i], true, a));
  }
  return NB_OK;
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
