// Internal declarations shared by the libnbound translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "nbound.h"

// ----------------------------------------------------------------- errors

void nb_set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

#define NB_REQUIRE(cond, ...)              \
  do {                                     \
    if (!(cond)) {                         \
      nb_set_error(__VA_ARGS__);           \
      return NB_ERR_INVALID_ARG;           \
    }                                      \
  } while (0)

#define NB_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t nb_e_ = (call);                                                           \
    if (nb_e_ != hipSuccess) {                                                           \
      nb_set_error("%s failed: %s (%d)", #call, hipGetErrorString(nb_e_), (int)nb_e_);   \
      return nb_e_ == hipErrorOutOfMemory ? NB_ERR_OOM : NB_ERR_HIP;                      \
    }                                                                                    \
  } while (0)

// Launch check: hipGetLastError after an async launch.
#define NB_LAUNCHED() NB_HIP(hipGetLastError())

#define NB_TRY(expr)                  \
  do {                                \
    nb_status nb_s_ = (expr);         \
    if (nb_s_ != NB_OK) return nb_s_; \
  } while (0)

// ------------------------------------------------------------- the handles

enum IndicatorType { IND_DISCS2D = 0, IND_VOXELS = 1, IND_METABALLS4D = 2 };

struct nb_indicator {
  int type = 0;
  int dim = 0;
  int device = 0;
  // discs: k rows (cx, cy, r); metaballs4d: a[k][3], d[k][3] = b - a, r2[k]
  int k = 0;
  float iso = 1.0f;
  float* params = nullptr;
  // voxels
  int n = 0;
  uint8_t* grid = nullptr;
  float* ray_t = nullptr;        // 256 sample parameters of the ray query
  int32_t* occupied = nullptr;        // linear indices of occupied cells (plane query)
  int64_t* occupied_count = nullptr;  // device int64: number of entries in `occupied`
  // plane query: cell centres (2i + 1)/n - 1 rounded to float, [n]; column
  // occupancy bits, [3][n][n][mask_words] (axis, then the two other axes
  // in increasing order, the higher one outer), bit b of word w = cell 64 w + b
  float* centre = nullptr;
  uint64_t* colmask = nullptr;
  int mask_words = 0;
  // the same per column of 8 x 8 cells over blocks of 8 x 8 x 8 cells:
  // [3][C][C][coarse_words], C = ceil(n / 8)
  uint64_t* coarse_mask = nullptr;
  int coarse_n = 0, coarse_words = 0;
};

struct nb_bound {
  int in_dim = 0, n_hidden = 0, width = 0, precision = 0;
  int device = 0;
  int64_t n_params = 0;
  float* theta = nullptr;    // float32 master parameters
  float* m = nullptr;        // Adam first moment
  float* v = nullptr;        // Adam second moment
  float* pack = nullptr;     // float32 weights in MFMA fragment order (NB_F32)
  int64_t pack_floats = 0;
  uint16_t* pack16 = nullptr;  // bfloat16 weight fragments (NB_BF16)
  int64_t pack16_elems = 0;
  int64_t adam_t = 0;        // Adam steps taken
  int variant = 0;           // forward kernel variant (tile shape), see nb_bound_set_variant
  // work space
  float* partial = nullptr;  // [max_wg][n_params] per-workgroup gradient partials
  float* aux = nullptr;      // [max_wg][8] per-workgroup loss / counts
  float* grad = nullptr;     // [n_params] reduced gradient
  float* batch_q = nullptr;  // training batch
  uint8_t* batch_y = nullptr;
  int64_t batch_cap = 0;
  int batch_cap_dim = 0;
  int32_t* cascade_idx = nullptr;  // positive-query index list of nb_cascade
  int64_t cascade_cap = 0;
  // early-out work space (on the second bound): gathered rows and decisions
  float* early_q = nullptr;
  uint8_t* early_h = nullptr;
  int64_t early_cap = 0;
  // bfloat16 training: transposed weight fragments, activations and gradients in HBM
  uint16_t* pack16t = nullptr;
  int64_t pack16t_elems = 0;
  uint16_t* tr_act = nullptr;      // activation slots x [padded batch][width]
  int recompute = 0;               // activation checkpoint interval (0: keep every activation)
  int train_kernel = 0;            // NB_TRAIN_AUTO (fused where it exists) or NB_TRAIN_LAYERWISE
  int activation = 0;              // NB_ACT_RELU or NB_ACT_SINE
  int tr_slots = 0;                // activation slots tr_act holds
  uint16_t* tr_grad = nullptr;     // 2 x [padded batch][width]
  int64_t tr_cap = 0;              // padded batch the two above hold
  unsigned* d_nonfinite = nullptr; // device flag: a training step met a non-finite loss or gradient
};

struct AdamArgs {
  int enabled;
  float lr, b1, b2, eps, bc1, bc2, lam1, lam2;
};

// A group of per-object bfloat16 bounds of a common depth and input size.
struct nb_group {
  int n_obj = 0, in_dim = 0, n_hidden = 0, precision = 0, device = 0;
  std::vector<int> widths;          // per object
  std::vector<int64_t> poff;        // parameter offsets [n_obj + 1]
  std::vector<int64_t> pkoff;       // forward-pack offsets, 16-byte slices [n_obj + 1]
  std::vector<int64_t> ptoff;       // transposed-pack offsets, 16-byte slices [n_obj + 1]
  std::vector<std::vector<int>> classes;   // trained object ids per width class (32, 64, 128)
  std::vector<int> class_all;              // objects per width class (work-space sizing)
  uint8_t* d_active = nullptr;             // [n_obj]: 1 for objects the training step updates
  int* d_widths = nullptr;
  int64_t* d_poff = nullptr;
  int64_t* d_pkoff = nullptr;
  int64_t* d_ptoff = nullptr;
  int* d_perm = nullptr;            // objects by decreasing width
  int* d_class = nullptr;           // concatenated class member lists
  int64_t n_params = 0, pack_elems = 0, packt_elems = 0, max_obj_params = 0;
  float* theta = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  uint16_t* pack16 = nullptr;
  uint16_t* pack16t = nullptr;
  int64_t adam_t = 0;
  // voxel grids, one per object
  uint8_t* grids = nullptr;
  int64_t* d_goff = nullptr;
  int* d_gn = nullptr;
  float* ray_t = nullptr;
  int32_t* table = nullptr;         // occupied-cell count tables, (n+1)^3 per object
  int64_t* d_toff = nullptr;
  int box_method = 1;               // 0: scan the box's cells, 1: count table
  // forward plan
  int n_wg_cap = 0;                 // most workgroups of one width class's forward launch
  int class_variant[3] = {0, 0, 0};   // grouped forward tile shape per width class (32, 64, 128)
  int64_t* d_item_off = nullptr;    // [n_obj + 3]: first tile of every object, per width class
  int64_t* d_wg_first = nullptr;    // [3 (n_wg_cap + 1)]: first tile of every workgroup, per width class
  // training work space
  int64_t tr_per_obj = 0;
  float* partial = nullptr;         // [n_wg x P_o] blocks at n_wg * poff[o]
  float* aux = nullptr;             // [n_obj][n_wg][8]
  uint16_t* tr_ws = nullptr;        // activations / gradients of every class member
  float* batch_q = nullptr;
  uint8_t* batch_y = nullptr;
  int64_t* d_qoff_train = nullptr;
  unsigned* d_nonfinite = nullptr;  // device flag: a training step met a non-finite loss or gradient
};

// ------------------------------------------------------- kernel launchers

// sampler.hip
nb_status launch_sample(int kind, int dim, uint64_t seed, uint64_t step, int64_t n, float* q,
                        hipStream_t s);

// indicators.hip
nb_status launch_query_exact(const nb_indicator* ind, int kind, const float* q, int64_t n, uint8_t* g,
                             hipStream_t s);
nb_status launch_voxelize(const float* params_dev, int k, float iso, int n, uint8_t* grid, hipStream_t s);
nb_status launch_cascade_exact(const nb_indicator* ind, int kind, const float* q, const uint8_t* h, int64_t n,
                               int32_t* idx, unsigned long long* count, uint8_t* answer, hipStream_t s);
nb_status launch_compact_positive(const uint8_t* h, int64_t n, int32_t* idx, unsigned long long* count, hipStream_t s);
// Device address (on the current device) of the allocation-free cascade's
// index list, NB_CASCADE_NOALLOC_MAX int32 entries.
constexpr int kMaxDevices = 64;
nb_status cascade_scratch(int32_t** out);
nb_status launch_collect_occupied(const uint8_t* grid, int64_t cells, int32_t* out, int64_t* count_dev,
                                  hipStream_t s);
nb_status launch_column_masks(const uint8_t* grid, int n, int words, uint64_t* mask, int coarse_n, int coarse_words,
                              uint64_t* coarse_mask, hipStream_t s);

// mlp_f32.hip
bool f32_supported(int in_dim, int n_hidden, int width);
bool f32_sine_supported(int in_dim, int n_hidden, int width);
int64_t f32_pack_floats(int in_dim, int n_hidden, int width);
nb_status f32_pack(const nb_bound* b, hipStream_t s);
// n_dev (device, nullable): evaluate only the first min(n, *n_dev) rows.
nb_status f32_forward(const nb_bound* b, const float* q, int64_t n, float tau, float* logits, uint8_t* h,
                      const uint8_t* g, unsigned long long* counts, hipStream_t s,
                      const unsigned long long* n_dev = nullptr);
// Per-workgroup partial gradients into b->partial / b->aux; returns the
// number of workgroups used through n_wg.
nb_status f32_train_partials(const nb_bound* b, const float* q, const uint8_t* y, int64_t n, float alpha,
                             float beta, float tau, int* n_wg, hipStream_t s);
int f32_max_workgroups();

// mlp_bf16.hip
bool bf16_supported(int in_dim, int n_hidden, int width);
int64_t bf16_pack_elems(int in_dim, int n_hidden, int width);
nb_status bf16_pack(const nb_bound* b, hipStream_t s);
int bf16_variants();
int bf16_variants_for(int width, int n_hidden);
nb_status bf16_forward(const nb_bound* b, const float* q, int64_t n, float tau, float* logits, uint8_t* h,
                       const uint8_t* g, unsigned long long* counts, hipStream_t s,
                       const unsigned long long* n_dev = nullptr);

// mlp_bf16_train.hip
struct BF16TrainPlan {
  int n_wg = 0;          // workgroups = batch chunks
  int64_t chunk = 0;     // queries per chunk (multiple of 64)
  int64_t padded = 0;    // n_wg * chunk
};
// Chunks of a training batch of n: at most max_wg chunks of a multiple of 64
// queries (every chunk a workgroup writing one partial gradient).
BF16TrainPlan bf16_train_plan(int64_t n, int max_wg = 256);
bool bf16_train_supported(int in_dim, int n_hidden, int width);
// mlp_bf16_fused.hip: shapes the fused training step covers
bool bf16_fused_supported(int in_dim, int n_hidden, int width);
// Whether a bfloat16 bound trains with the fused step (its transposed pack
// is then in operand order).
bool bf16_uses_fused(const nb_bound* b);
int64_t bf16_packt_elems(int n_hidden, int width);
// Activation buffers of one training pass (n_hidden - 1 without recomputation).
int bf16_act_slots(int n_hidden, int every);
nb_status bf16_pack_t(const nb_bound* b, hipStream_t s);
nb_status bf16_train_partials(const nb_bound* b, const float* q, const uint8_t* y, int64_t n, float alpha,
                              float beta, float tau, const BF16TrainPlan& plan, hipStream_t s);

nb_status bf16_group_train_class(const nb_group* gr, int width, const int* d_members, int n_members,
                                 const float* q, const uint8_t* y, int64_t per_obj, float alpha,
                                 const float* alpha_obj, float beta,
                                 float tau, const BF16TrainPlan& plan, uint16_t* act, uint16_t* grad,
                                 hipStream_t s);

// early.hip
nb_status launch_gather_rows(const float* q, int d, const int32_t* idx, const unsigned long long* count, int64_t n_max,
                             float* qc, hipStream_t s);
nb_status launch_scatter_u8(const uint8_t* hc, const int32_t* idx, const unsigned long long* count, int64_t n_max,
                            uint8_t* h, hipStream_t s);

// group.hip
int group_variants();
// Forward + decision with the group's current variant; with g and counts
// (uint64[n_obj][4], zeroed here) also per-object TP, FP, TN, FN against g.
nb_status group_forward(const nb_group* gr, const float* q, const int64_t* qoff, int64_t n, float tau,
                        float* logits, uint8_t* h, const uint8_t* g, unsigned long long* counts, hipStream_t s);
nb_status group_exact(const nb_group* gr, int kind, const float* q, const int64_t* qoff, int64_t n, uint8_t* g,
                      hipStream_t s);
nb_status group_pack(const nb_group* gr, hipStream_t s);
nb_status group_build_tables(const nb_group* gr, int max_n, hipStream_t s);
nb_status group_reduce_adam(const nb_group* gr, int n_wg, const AdamArgs& adam, const float* lr_obj, float* loss,
                            unsigned long long* counts, float loss_scale, hipStream_t s);

// optim.hip
// Reduce partials over n_wg workgroups: writes grad (if non-null), loss and
// counts (if non-null); with adam != 0 also applies one Adam step to theta,
// and with pack_f32 (float32 bounds) writes the updated weights to their
// packed fragments, so that no repack is needed after the step.
nb_status launch_reduce(const nb_bound* b, int n_wg, float* grad, float* loss, float loss_scale,
                        unsigned long long* counts, const AdamArgs& adam, hipStream_t s, bool pack_f32 = false);
nb_status launch_adam(const nb_bound* b, const float* grad, const AdamArgs& adam, hipStream_t s);
nb_status launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
// 1 for entries of theta that belong to a weight matrix (regularised), 0 for biases.
__host__ __device__ inline int nb_is_weight(int64_t p, int in_dim, int width, int n_hidden) {
  int64_t off = 0;
  for (int l = 0; l <= n_hidden; ++l) {
    const int64_t fin = l == 0 ? in_dim : width;
    const int64_t fout = l == n_hidden ? 1 : width;
    if (p < off + fin * fout) return 1;
    off += fin * fout;
    if (p < off + fout) return 0;
    off += fout;
  }
  return 0;
}
