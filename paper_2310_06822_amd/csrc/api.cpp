// extern "C" entry points of libnbound (declared and documented in nbound.h):
// argument checks, handle life cycle, and the launch sequences.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <vector>

#include "nb_internal.h"
#include "nb_mlp.h"

namespace {

thread_local char g_err[512] = "";

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

nb_status require_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    nb_set_error("no HIP device is visible");
    return NB_ERR_NO_DEVICE;
  }
  return NB_OK;
}

template <class T>
nb_status dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return NB_OK;
  NB_HIP(hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)));
  return NB_OK;
}

template <class T>
void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Logit threshold of the decision sigmoid(z) + eps >= 1/2.
float tau_of(float eps) { return (float)std::log((0.5 - (double)eps) / (0.5 + (double)eps)); }

int64_t mlp_params(int in_dim, int n_hidden, int width) {
  return (int64_t)width * in_dim + width + (int64_t)(n_hidden - 1) * ((int64_t)width * width + width) + width + 1;
}

int kind_dim(int kind, int point_dim) { return kind == NB_QUERY_POINT ? point_dim : 6; }

// Rebuild the weight fragments the forward / training kernels read.
nb_status repack(const nb_bound* b, hipStream_t s) {
  if (b->precision != NB_BF16) return f32_pack(b, s);
  NB_TRY(bf16_pack(b, s));
  return bf16_pack_t(b, s);
}

nb_status require_training(const nb_bound* b) {
  if (b->precision == NB_BF16 && !bf16_train_supported(b->in_dim, b->n_hidden, b->width)) {
    nb_set_error("training a bfloat16 bound %d x %d^%d has no kernel in this library", b->in_dim, b->width,
                 b->n_hidden);
    return NB_ERR_UNSUPPORTED;
  }
  return NB_OK;
}

void dev_free_u16(uint16_t*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Per-workgroup gradient partials for a labelled batch, either precision;
// returns the number of partials through n_wg.
nb_status train_partials(nb_bound* b, const float* q, const uint8_t* y, int64_t n, float alpha, float beta,
                         int* n_wg, hipStream_t s) {
  const float tau = tau_of(1e-5f);
  if (b->precision != NB_BF16) return f32_train_partials(b, q, y, n, alpha, beta, tau, n_wg, s);
  const BF16TrainPlan plan = bf16_train_plan(n);
  const int slots = bf16_act_slots(b->n_hidden, b->recompute);
  // the fused step keeps activations on the chip: no work space
  if (!bf16_uses_fused(b) && (b->tr_cap < plan.padded || b->tr_slots != slots)) {
    // (re)sizes the activation / gradient work space (synchronising)
    NB_HIP(hipStreamSynchronize(s));
    const int64_t cap = std::max(plan.padded, b->tr_cap);
    dev_free_u16(b->tr_act);
    dev_free_u16(b->tr_grad);
    b->tr_cap = 0;
    b->tr_slots = 0;
    const size_t per = (size_t)cap * b->width;
    NB_HIP(hipMalloc(reinterpret_cast<void**>(&b->tr_act), per * slots * sizeof(uint16_t)));
    NB_HIP(hipMalloc(reinterpret_cast<void**>(&b->tr_grad), per * 2 * sizeof(uint16_t)));
    b->tr_cap = cap;
    b->tr_slots = slots;
  }
  *n_wg = plan.n_wg;
  return bf16_train_partials(b, q, y, n, alpha, beta, tau, plan, s);
}


}  // namespace

int nb_cu_count() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cus[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cus[dev] = v;
  }
  return cus[dev];
}

void nb_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

extern "C" {

const char* nb_last_error(void) { return g_err; }

nb_status nb_version(int* major, int* minor) {
  NB_REQUIRE(major && minor, "NULL argument");
  *major = 0;
  *minor = 1;
  return NB_OK;
}

nb_status nb_device_count(int* count) {
  NB_REQUIRE(count, "count is NULL");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) n = 0;
  *count = n;
  return NB_OK;
}

// --------------------------------------------------------------- indicators

nb_status nb_indicator_discs2d(const float* discs_host, int k, nb_indicator** out) {
  NB_REQUIRE(out && discs_host, "NULL argument");
  *out = nullptr;
  NB_REQUIRE(k >= 1 && k <= 64, "k must be in 1..64");
  NB_TRY(require_device());
  auto* ind = new nb_indicator();
  ind->type = IND_DISCS2D;
  ind->dim = 2;
  ind->k = k;
  hipGetDevice(&ind->device);
  nb_status st = dev_alloc(&ind->params, (size_t)3 * k);
  if (st == NB_OK && hipMemcpy(ind->params, discs_host, sizeof(float) * 3 * k, hipMemcpyHostToDevice) != hipSuccess) {
    nb_set_error("hipMemcpy of the disc table failed");
    st = NB_ERR_HIP;
  }
  if (st != NB_OK) {
    nb_indicator_destroy(ind);
    return st;
  }
  *out = ind;
  return NB_OK;
}

nb_status nb_indicator_voxels(const uint8_t* grid, int n, nb_indicator** out) {
  NB_REQUIRE(out && grid, "NULL argument");
  *out = nullptr;
  NB_REQUIRE(n >= 2 && n <= 1024, "grid size n must be in 2..1024");
  NB_TRY(require_device());
  auto* ind = new nb_indicator();
  ind->type = IND_VOXELS;
  ind->dim = 3;
  ind->n = n;
  hipGetDevice(&ind->device);
  const int64_t cells = (int64_t)n * n * n;
  nb_status st = dev_alloc(&ind->grid, (size_t)cells);
  if (st == NB_OK) st = dev_alloc(&ind->ray_t, 256);
  if (st == NB_OK) st = dev_alloc(&ind->occupied, (size_t)cells);
  if (st == NB_OK) st = dev_alloc(&ind->occupied_count, 1);
  ind->mask_words = (n + 63) / 64;
  if (st == NB_OK) st = dev_alloc(&ind->centre, (size_t)n);
  if (st == NB_OK) st = dev_alloc(&ind->colmask, (size_t)3 * n * n * ind->mask_words);
  ind->coarse_n = (n + 7) / 8;
  ind->coarse_words = (ind->coarse_n + 63) / 64;
  if (st == NB_OK)
    st = dev_alloc(&ind->coarse_mask, (size_t)3 * ind->coarse_n * ind->coarse_n * ind->coarse_words);
  if (st == NB_OK) {
    // cell centres, computed in double and rounded once (the plane query's)
    std::vector<float> c((size_t)n);
    for (int i = 0; i < n; ++i) c[(size_t)i] = (float)((2.0 * i + 1.0) / n - 1.0);
    if (hipMemcpy(ind->centre, c.data(), sizeof(float) * n, hipMemcpyHostToDevice) != hipSuccess) {
      nb_set_error("hipMemcpy of the cell centres failed");
      st = NB_ERR_HIP;
    }
  }
  if (st == NB_OK) {
    // ray sample parameters t_j = 4 j / 255, computed in double and rounded once
    float t[256];
    for (int j = 0; j < 256; ++j) t[j] = (float)(4.0 * j / 255.0);
    if (hipMemcpy(ind->grid, grid, (size_t)cells, hipMemcpyDeviceToDevice) != hipSuccess ||
        hipMemcpy(ind->ray_t, t, sizeof(t), hipMemcpyHostToDevice) != hipSuccess) {
      nb_set_error("hipMemcpy of the voxel grid failed");
      st = NB_ERR_HIP;
    }
  }
  if (st == NB_OK) st = launch_collect_occupied(ind->grid, cells, ind->occupied, ind->occupied_count, nullptr);
  if (st == NB_OK)
    st = launch_column_masks(ind->grid, n, ind->mask_words, ind->colmask, ind->coarse_n, ind->coarse_words,
                             ind->coarse_mask, nullptr);
  if (st == NB_OK && hipDeviceSynchronize() != hipSuccess) {
    nb_set_error("building the occupied-cell list failed");
    st = NB_ERR_HIP;
  }
  if (st != NB_OK) {
    nb_indicator_destroy(ind);
    return st;
  }
  *out = ind;
  return NB_OK;
}

nb_status nb_indicator_metaballs4d(const float* a_host, const float* b_host, const float* radii_host, int k,
                                   float iso, nb_indicator** out) {
  NB_REQUIRE(out && a_host && b_host && radii_host, "NULL argument");
  *out = nullptr;
  NB_REQUIRE(k >= 1 && k <= 64, "k must be in 1..64");
  NB_TRY(require_device());
  std::vector<float> prm((size_t)7 * k);
  for (int i = 0; i < 3 * k; ++i) {
    prm[i] = a_host[i];
    prm[3 * k + i] = b_host[i] - a_host[i];  // path direction, one float32 subtraction
  }
  for (int i = 0; i < k; ++i) prm[6 * k + i] = radii_host[i];
  auto* ind = new nb_indicator();
  ind->type = IND_METABALLS4D;
  ind->dim = 4;
  ind->k = k;
  ind->iso = iso;
  hipGetDevice(&ind->device);
  nb_status st = dev_alloc(&ind->params, prm.size());
  if (st == NB_OK && hipMemcpy(ind->params, prm.data(), prm.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    nb_set_error("hipMemcpy of the metaball table failed");
    st = NB_ERR_HIP;
  }
  if (st != NB_OK) {
    nb_indicator_destroy(ind);
    return st;
  }
  *out = ind;
  return NB_OK;
}

nb_status nb_indicator_dim(const nb_indicator* ind, int* dim) {
  NB_REQUIRE(ind && dim, "NULL argument");
  *dim = ind->dim;
  return NB_OK;
}

nb_status nb_indicator_destroy(nb_indicator* ind) {
  if (!ind) return NB_OK;
  dev_free(ind->params);
  dev_free(ind->grid);
  dev_free(ind->ray_t);
  dev_free(ind->occupied);
  dev_free(ind->occupied_count);
  dev_free(ind->centre);
  dev_free(ind->colmask);
  dev_free(ind->coarse_mask);
  delete ind;
  return NB_OK;
}

nb_status nb_voxelize_metaballs(const float* centres_host, const float* radii_host, int k, float iso, int n,
                                uint8_t* grid, void* stream) {
  NB_REQUIRE(centres_host && radii_host && grid, "NULL argument");
  NB_REQUIRE(k >= 1 && k <= 64, "k must be in 1..64");
  NB_REQUIRE(n >= 2 && n <= 1024, "grid size n must be in 2..1024");
  NB_TRY(require_device());
  // Set-up call: the ball table goes through a temporary device buffer that
  // is freed after the kernel has run on `stream`.
  std::vector<float> prm((size_t)4 * k);
  std::memcpy(prm.data(), centres_host, sizeof(float) * 3 * k);
  std::memcpy(prm.data() + 3 * k, radii_host, sizeof(float) * k);
  float* prm_dev = nullptr;
  NB_TRY(dev_alloc(&prm_dev, prm.size()));
  hipStream_t s = as_stream(stream);
  nb_status st = NB_OK;
  if (hipMemcpyAsync(prm_dev, prm.data(), prm.size() * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess) {
    nb_set_error("hipMemcpyAsync of the ball table failed");
    st = NB_ERR_HIP;
  }
  if (st == NB_OK) st = launch_voxelize(prm_dev, k, iso, n, grid, s);
  if (hipStreamSynchronize(s) != hipSuccess && st == NB_OK) {
    nb_set_error("voxelisation failed");
    st = NB_ERR_HIP;
  }
  dev_free(prm_dev);
  return st;
}

// ------------------------------------------------------------------ queries

nb_status nb_query_exact(const nb_indicator* ind, int kind, const float* q, int64_t n, uint8_t* g, void* stream) {
  NB_REQUIRE(ind, "indicator is NULL");
  NB_REQUIRE(kind >= NB_QUERY_POINT && kind <= NB_QUERY_PLANE, "unknown query kind %d", kind);
  return launch_query_exact(ind, kind, q, n, g, as_stream(stream));
}

nb_status nb_sample_queries(int kind, int dim, uint64_t seed, uint64_t step, int64_t n, float* q, void* stream) {
  NB_REQUIRE(kind >= NB_QUERY_POINT && kind <= NB_QUERY_PLANE, "unknown query kind %d", kind);
  return launch_sample(kind, dim, seed, step, n, q, as_stream(stream));
}

// -------------------------------------------------------------------- bound

nb_status nb_bound_create(int in_dim, int n_hidden, int width, int precision, nb_bound** out) {
  NB_REQUIRE(out, "out is NULL");
  *out = nullptr;
  NB_REQUIRE(in_dim >= 1 && in_dim <= 8, "in_dim must be in 1..8");
  NB_REQUIRE(n_hidden >= 1 && n_hidden <= 8, "n_hidden must be in 1..8");
  NB_REQUIRE(width >= 16 && width <= 256 && width % 16 == 0, "width must be a multiple of 16 in 16..256");
  NB_REQUIRE(precision == NB_F32 || precision == NB_BF16, "unknown precision %d", precision);
  const bool ok = precision == NB_F32 ? f32_supported(in_dim, n_hidden, width) : bf16_supported(in_dim, n_hidden, width);
  if (!ok) {
    nb_set_error("no kernel for a %s bound %d x %d^%d", precision == NB_F32 ? "float32" : "bfloat16", in_dim, width,
                 n_hidden);
    return NB_ERR_UNSUPPORTED;
  }
  NB_TRY(require_device());
  auto* b = new nb_bound();
  b->in_dim = in_dim;
  b->n_hidden = n_hidden;
  b->width = width;
  b->precision = precision;
  hipGetDevice(&b->device);
  b->n_params = mlp_params(in_dim, n_hidden, width);
  b->pack_floats = precision == NB_F32 ? f32_pack_floats(in_dim, n_hidden, width) : 0;
  b->pack16_elems = precision == NB_BF16 ? bf16_pack_elems(in_dim, n_hidden, width) : 0;
  b->pack16t_elems =
      precision == NB_BF16 && bf16_train_supported(in_dim, n_hidden, width) ? bf16_packt_elems(n_hidden, width) : 0;
  const size_t P = (size_t)b->n_params;
  nb_status st = dev_alloc(&b->theta, P);
  if (st == NB_OK) st = dev_alloc(&b->m, P);
  if (st == NB_OK) st = dev_alloc(&b->v, P);
  if (st == NB_OK) st = dev_alloc(&b->grad, P);
  if (st == NB_OK) st = dev_alloc(&b->pack, (size_t)b->pack_floats);
  if (st == NB_OK) st = dev_alloc(&b->pack16, (size_t)b->pack16_elems);
  if (st == NB_OK) st = dev_alloc(&b->pack16t, (size_t)b->pack16t_elems);
  if (st == NB_OK) st = dev_alloc(&b->partial, (size_t)f32_max_workgroups() * P);
  if (st == NB_OK) st = dev_alloc(&b->aux, (size_t)f32_max_workgroups() * 8);
  if (st == NB_OK) st = dev_alloc(&b->d_nonfinite, 1);
  if (st == NB_OK) {
    if (hipMemset(b->theta, 0, P * 4) != hipSuccess || hipMemset(b->m, 0, P * 4) != hipSuccess ||
        hipMemset(b->d_nonfinite, 0, sizeof(unsigned)) != hipSuccess ||
        hipMemset(b->v, 0, P * 4) != hipSuccess ||
        (b->pack && hipMemset(b->pack, 0, (size_t)b->pack_floats * 4) != hipSuccess) ||
        (b->pack16 && hipMemset(b->pack16, 0, (size_t)b->pack16_elems * 2) != hipSuccess)) {
      nb_set_error("hipMemset of the bound state failed");
      st = NB_ERR_HIP;
    }
  }
  if (st != NB_OK) {
    nb_bound_destroy(b);
    return st;
  }
  *out = b;
  return NB_OK;
}

nb_status nb_bound_destroy(nb_bound* b) {
  if (!b) return NB_OK;
  dev_free(b->theta);
  dev_free(b->m);
  dev_free(b->v);
  dev_free(b->grad);
  dev_free(b->pack);
  dev_free(b->pack16);
  dev_free(b->pack16t);
  dev_free(b->tr_act);
  dev_free(b->tr_grad);
  dev_free(b->partial);
  dev_free(b->aux);
  dev_free(b->d_nonfinite);
  dev_free(b->batch_q);
  dev_free(b->batch_y);
  dev_free(b->cascade_idx);
  dev_free(b->early_q);
  dev_free(b->early_h);
  delete b;
  return NB_OK;
}

nb_status nb_bound_num_params(const nb_bound* b, int64_t* n_params) {
  NB_REQUIRE(b && n_params, "NULL argument");
  *n_params = b->n_params;
  return NB_OK;
}

nb_status nb_bound_shape(const nb_bound* b, int* in_dim, int* n_hidden, int* width, int* precision) {
  NB_REQUIRE(b, "bound is NULL");
  if (in_dim) *in_dim = b->in_dim;
  if (n_hidden) *n_hidden = b->n_hidden;
  if (width) *width = b->width;
  if (precision) *precision = b->precision;
  return NB_OK;
}

nb_status nb_bound_num_variants(const nb_bound* b, int* count) {
  NB_REQUIRE(b && count, "NULL argument");
  *count = b->precision == NB_BF16 ? bf16_variants_for(b->width, b->n_hidden) : 1;
  return NB_OK;
}

nb_status nb_bound_set_activation(nb_bound* b, int activation) {
  NB_REQUIRE(b, "bound is NULL");
  NB_REQUIRE(activation == NB_ACT_RELU || activation == NB_ACT_SINE, "unknown activation %d", activation);
  if (activation == NB_ACT_SINE && !(b->precision == NB_F32 && f32_sine_supported(b->in_dim, b->n_hidden, b->width))) {
    nb_set_error("sine activations run on float32 bounds of width 32 or 64 with 1..3 hidden layers");
    return NB_ERR_UNSUPPORTED;
  }
  b->activation = activation;
  return NB_OK;
}

nb_status nb_bound_set_recompute(nb_bound* b, int every) {
  NB_REQUIRE(b, "bound is NULL");
  NB_REQUIRE(every == 0 || (every >= 2 && every <= 64), "checkpoint interval must be 0 or 2..64");
  NB_REQUIRE(b->precision == NB_BF16 || every == 0, "activation recomputation applies to bfloat16 training");
  b->recompute = every;
  return NB_OK;
}

nb_status nb_bound_set_train_kernel(nb_bound* b, int kernel, void* stream) {
  NB_REQUIRE(b, "bound is NULL");
  NB_REQUIRE(kernel == NB_TRAIN_AUTO || kernel == NB_TRAIN_LAYERWISE, "unknown training kernel %d", kernel);
  NB_REQUIRE(b->precision == NB_BF16 || kernel == NB_TRAIN_AUTO, "the training kernel choice applies to bfloat16");
  if (b->train_kernel == kernel) return NB_OK;
  b->train_kernel = kernel;
  return b->precision == NB_BF16 ? bf16_pack_t(b, as_stream(stream)) : NB_OK;
}

nb_status nb_bound_set_variant(nb_bound* b, int variant) {
  NB_REQUIRE(b, "bound is NULL");
  int n = 0;
  nb_bound_num_variants(b, &n);
  NB_REQUIRE(variant >= 0 && variant < n, "variant %d out of range 0..%d", variant, n - 1);
  b->variant = variant;
  return NB_OK;
}

nb_status nb_bound_set_params(nb_bound* b, const float* theta, int64_t n_params, void* stream) {
  NB_REQUIRE(b && theta, "NULL argument");
  NB_REQUIRE(n_params == b->n_params, "bound has %lld parameters, got %lld", (long long)b->n_params,
             (long long)n_params);
  hipStream_t s = as_stream(stream);
  NB_HIP(hipMemcpyAsync(b->theta, theta, n_params * 4, hipMemcpyDeviceToDevice, s));
  NB_HIP(hipMemsetAsync(b->m, 0, n_params * 4, s));
  NB_HIP(hipMemsetAsync(b->v, 0, n_params * 4, s));
  b->adam_t = 0;
  return repack(b, s);
}

nb_status nb_bound_get_params(const nb_bound* b, float* theta, int64_t n_params, void* stream) {
  NB_REQUIRE(b && theta, "NULL argument");
  NB_REQUIRE(n_params == b->n_params, "bound has %lld parameters, got %lld", (long long)b->n_params,
             (long long)n_params);
  NB_HIP(hipMemcpyAsync(theta, b->theta, n_params * 4, hipMemcpyDeviceToDevice, as_stream(stream)));
  return NB_OK;
}

nb_status nb_bound_get_state(const nb_bound* b, float* m, float* v, int64_t n_params, int64_t* step_host,
                             void* stream) {
  NB_REQUIRE(b && m && v && step_host, "NULL argument");
  NB_REQUIRE(n_params == b->n_params, "parameter count mismatch");
  hipStream_t s = as_stream(stream);
  NB_HIP(hipMemcpyAsync(m, b->m, n_params * 4, hipMemcpyDeviceToDevice, s));
  NB_HIP(hipMemcpyAsync(v, b->v, n_params * 4, hipMemcpyDeviceToDevice, s));
  *step_host = b->adam_t;
  return NB_OK;
}

nb_status nb_bound_set_state(nb_bound* b, const float* m, const float* v, int64_t n_params, int64_t step,
                             void* stream) {
  NB_REQUIRE(b && m && v, "NULL argument");
  NB_REQUIRE(n_params == b->n_params, "parameter count mismatch");
  NB_REQUIRE(step >= 0, "step must be >= 0");
  hipStream_t s = as_stream(stream);
  NB_HIP(hipMemcpyAsync(b->m, m, n_params * 4, hipMemcpyDeviceToDevice, s));
  NB_HIP(hipMemcpyAsync(b->v, v, n_params * 4, hipMemcpyDeviceToDevice, s));
  b->adam_t = step;
  return NB_OK;
}

namespace {
// Checkpoint layout: this header, then theta, m and v (float32[n_params] each).
struct CkptHeader {
  char magic[8];
  int32_t version, in_dim, n_hidden, width, precision, activation;
  int64_t n_params, adam_t;
};
constexpr char kCkptMagic[8] = {'N', 'B', 'O', 'U', 'N', 'D', 'C', 'K'};
}  // namespace

nb_status nb_bound_save(const nb_bound* b, void* host_buf, size_t* bytes, void* stream) {
  NB_REQUIRE(b && bytes, "NULL argument");
  const size_t need = sizeof(CkptHeader) + 3 * (size_t)b->n_params * 4;
  if (!host_buf) {
    *bytes = need;
    return NB_OK;
  }
  NB_REQUIRE(*bytes >= need, "checkpoint needs %zu bytes, buffer has %zu", need, *bytes);
  CkptHeader h{};
  memcpy(h.magic, kCkptMagic, 8);
  h.version = 1;
  h.in_dim = b->in_dim;
  h.n_hidden = b->n_hidden;
  h.width = b->width;
  h.precision = b->precision;
  h.activation = b->activation;
  h.n_params = b->n_params;
  h.adam_t = b->adam_t;
  hipStream_t s = as_stream(stream);
  char* out = static_cast<char*>(host_buf);
  memcpy(out, &h, sizeof h);
  float* dst = reinterpret_cast<float*>(out + sizeof h);
  NB_HIP(hipMemcpyAsync(dst, b->theta, b->n_params * 4, hipMemcpyDeviceToHost, s));
  NB_HIP(hipMemcpyAsync(dst + b->n_params, b->m, b->n_params * 4, hipMemcpyDeviceToHost, s));
  NB_HIP(hipMemcpyAsync(dst + 2 * b->n_params, b->v, b->n_params * 4, hipMemcpyDeviceToHost, s));
  NB_HIP(hipStreamSynchronize(s));
  *bytes = need;
  return NB_OK;
}

nb_status nb_bound_load(nb_bound* b, const void* host_buf, size_t bytes, void* stream) {
  NB_REQUIRE(b && host_buf, "NULL argument");
  NB_REQUIRE(bytes >= sizeof(CkptHeader), "checkpoint too short");
  CkptHeader h;
  memcpy(&h, host_buf, sizeof h);
  NB_REQUIRE(memcmp(h.magic, kCkptMagic, 8) == 0 && h.version == 1, "not a bound checkpoint (version 1)");
  NB_REQUIRE(h.in_dim == b->in_dim && h.n_hidden == b->n_hidden && h.width == b->width &&
                 h.precision == b->precision && h.activation == b->activation && h.n_params == b->n_params,
             "checkpoint of a %d x %d^%d bound (precision %d, activation %d) does not fit this %d x %d^%d bound "
             "(precision %d, activation %d)",
             h.in_dim, h.width, h.n_hidden, h.precision, h.activation, b->in_dim, b->width, b->n_hidden,
             b->precision, b->activation);
  NB_REQUIRE(h.adam_t >= 0, "negative Adam step in the checkpoint");
  NB_REQUIRE(bytes >= sizeof h + 3 * (size_t)h.n_params * 4, "checkpoint truncated");
  hipStream_t s = as_stream(stream);
  const float* src = reinterpret_cast<const float*>(static_cast<const char*>(host_buf) + sizeof h);
  NB_HIP(hipMemcpyAsync(b->theta, src, b->n_params * 4, hipMemcpyHostToDevice, s));
  NB_HIP(hipMemcpyAsync(b->m, src + b->n_params, b->n_params * 4, hipMemcpyHostToDevice, s));
  NB_HIP(hipMemcpyAsync(b->v, src + 2 * b->n_params, b->n_params * 4, hipMemcpyHostToDevice, s));
  b->adam_t = h.adam_t;
  NB_TRY(repack(b, s));
  NB_HIP(hipStreamSynchronize(s));
  return NB_OK;
}

nb_status nb_bound_forward(const nb_bound* b, const float* q, int64_t n, float eps, float* logits, uint8_t* h,
                           const uint8_t* g, uint64_t* counts, void* stream) {
  NB_REQUIRE(b && q, "NULL argument");
  NB_REQUIRE(n > 0 && n <= (int64_t(1) << 40), "n must be positive");
  NB_REQUIRE(eps >= 0.0f && eps < 0.5f, "eps must be in [0, 0.5)");
  NB_REQUIRE(logits || h || (g && counts), "nothing to compute: logits, h and (g, counts) are all NULL");
  NB_REQUIRE((g == nullptr) == (counts == nullptr), "g and counts must be given together");
  hipStream_t s = as_stream(stream);
  auto* cnt = reinterpret_cast<unsigned long long*>(counts);
  if (cnt) NB_TRY(launch_zero_u64(cnt, 4, s));
  if (b->precision == NB_BF16) return bf16_forward(b, q, n, tau_of(eps), logits, h, g, cnt, s);
  return f32_forward(b, q, n, tau_of(eps), logits, h, g, cnt, s);
}

nb_status nb_bound_loss_grad(nb_bound* b, const float* q, const uint8_t* y, int64_t n, float alpha, float beta,
                             float* grad, float* loss, uint64_t* counts, void* stream) {
  NB_REQUIRE(b && q && y && grad, "NULL argument");
  NB_REQUIRE(n > 0 && n <= (int64_t(1) << 30), "n must be in 1..2^30");
  NB_REQUIRE(std::isfinite(alpha) && std::isfinite(beta) && alpha >= 0 && beta >= 0,
             "alpha and beta must be finite and >= 0");
  NB_TRY(require_training(b));
  hipStream_t s = as_stream(stream);
  int n_wg = 0;
  NB_TRY(train_partials(b, q, y, n, alpha, beta, &n_wg, s));
  AdamArgs none{};
  return launch_reduce(b, n_wg, grad, loss, (float)(1.0 / (double)n), reinterpret_cast<unsigned long long*>(counts),
                       none, s);
}

namespace {
AdamArgs adam_args(nb_bound* b, float lr, float b1, float b2, float eps, float lam1, float lam2) {
  b->adam_t += 1;
  AdamArgs a{};
  a.enabled = 1;
  a.lr = lr;
  a.b1 = b1;
  a.b2 = b2;
  a.eps = eps;
  a.bc1 = (float)(1.0 - std::pow((double)b1, (double)b->adam_t));
  a.bc2 = (float)(1.0 - std::pow((double)b2, (double)b->adam_t));
  a.lam1 = lam1;
  a.lam2 = lam2;
  return a;
}
}  // namespace

nb_status nb_bound_adam_step(nb_bound* b, const float* grad, float lr, float beta1, float beta2, float adam_eps,
                             float lam1, float lam2, void* stream) {
  NB_REQUIRE(b && grad, "NULL argument");
  NB_REQUIRE(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && adam_eps >= 0 && lam1 >= 0 && lam2 >= 0,
             "invalid Adam constants");
  hipStream_t s = as_stream(stream);
  const AdamArgs a = adam_args(b, lr, beta1, beta2, adam_eps, lam1, lam2);
  NB_TRY(launch_adam(b, grad, a, s));
  return repack(b, s);
}

nb_status nb_bound_train_step(nb_bound* b, const nb_indicator* ind, int kind, uint64_t seed, uint64_t step,
                              int64_t batch, float alpha, float beta, float lr, float lam1, float lam2, float* loss,
                              uint64_t* counts, void* stream) {
  NB_REQUIRE(b && ind, "NULL argument");
  NB_REQUIRE(kind >= NB_QUERY_POINT && kind <= NB_QUERY_PLANE, "unknown query kind %d", kind);
  NB_REQUIRE(batch > 0 && batch <= (int64_t(1) << 30), "batch must be in 1..2^30");
  NB_REQUIRE(lr > 0 && lam1 >= 0 && lam2 >= 0, "invalid learning rate or regularisation");
  NB_REQUIRE(std::isfinite(alpha) && std::isfinite(beta) && alpha >= 0 && beta >= 0,
             "alpha and beta must be finite and >= 0");
  NB_TRY(require_training(b));
  const int d = kind_dim(kind, ind->dim);
  NB_REQUIRE(d == b->in_dim, "bound input dimension %d does not match the %d-D query", b->in_dim, d);
  hipStream_t s = as_stream(stream);
  if (b->batch_cap < batch || b->batch_cap_dim < d) {
    // grows the work space: synchronising allocation, only when the batch grows
    NB_HIP(hipStreamSynchronize(s));
    dev_free(b->batch_q);
    dev_free(b->batch_y);
    b->batch_cap = 0;
    NB_TRY(dev_alloc(&b->batch_q, (size_t)batch * d));
    NB_TRY(dev_alloc(&b->batch_y, (size_t)batch));
    b->batch_cap = batch;
    b->batch_cap_dim = d;
  }
  NB_TRY(launch_sample(kind, ind->dim, seed, step, batch, b->batch_q, s));
  NB_TRY(launch_query_exact(ind, kind, b->batch_q, batch, b->batch_y, s));
  int n_wg = 0;
  NB_TRY(train_partials(b, b->batch_q, b->batch_y, batch, alpha, beta, &n_wg, s));
  const AdamArgs a = adam_args(b, lr, 0.9f, 0.999f, 1e-8f, lam1, lam2);
  const bool fused = b->precision == NB_F32;   // the reduction writes the float32 fragments itself
  NB_TRY(launch_reduce(b, n_wg, nullptr, loss, (float)(1.0 / (double)batch),
                       reinterpret_cast<unsigned long long*>(counts), a, s, fused));
  return fused ? NB_OK : repack(b, s);
}

namespace {
nb_status bound_forward(const nb_bound* b, const float* q, int64_t n, float tau, float* logits, uint8_t* h,
                        const uint8_t* g, unsigned long long* counts, hipStream_t s,
                        const unsigned long long* n_dev = nullptr) {
  if (b->precision == NB_BF16) return bf16_forward(b, q, n, tau, logits, h, g, counts, s, n_dev);
  return f32_forward(b, q, n, tau, logits, h, g, counts, s, n_dev);
}
}  // namespace

nb_status nb_early_out(const nb_bound* first, nb_bound* second, const float* q, int64_t n, float eps, uint8_t* h,
                       uint64_t* n_second, void* stream) {
  NB_REQUIRE(first && second && q && h && n_second, "NULL argument");
  NB_REQUIRE(first != second, "the two bounds must differ");
  NB_REQUIRE(first->in_dim == second->in_dim, "the bounds take %d and %d inputs", first->in_dim, second->in_dim);
  NB_REQUIRE(n > 0 && n <= (int64_t)0x7FFFFFFF, "n must be in 1..2^31-1");
  NB_REQUIRE(eps >= 0.0f && eps < 0.5f, "eps must be in [0, 0.5)");
  hipStream_t s = as_stream(stream);
  if (second->cascade_cap < n || second->early_cap < n) {
    // grows the work space (synchronising)
    NB_HIP(hipStreamSynchronize(s));
    dev_free(second->cascade_idx);
    dev_free(second->early_q);
    dev_free(second->early_h);
    second->cascade_cap = 0;
    second->early_cap = 0;
    NB_TRY(dev_alloc(&second->cascade_idx, (size_t)n));
    NB_TRY(dev_alloc(&second->early_q, (size_t)n * second->in_dim));
    NB_TRY(dev_alloc(&second->early_h, (size_t)n));
    second->cascade_cap = n;
    second->early_cap = n;
  }
  auto* cnt = reinterpret_cast<unsigned long long*>(n_second);
  const float tau = tau_of(eps);
  NB_TRY(launch_zero_u64(cnt, 1, s));
  NB_TRY(bound_forward(first, q, n, tau, nullptr, h, nullptr, nullptr, s));
  NB_TRY(launch_compact_positive(h, n, second->cascade_idx, cnt, s));
  NB_TRY(launch_gather_rows(q, second->in_dim, second->cascade_idx, cnt, n, second->early_q, s));
  NB_TRY(bound_forward(second, second->early_q, n, tau, nullptr, second->early_h, nullptr, nullptr, s, cnt));
  return launch_scatter_u8(second->early_h, second->cascade_idx, cnt, n, h, s);
}

nb_status nb_cascade(nb_bound* b, const nb_indicator* ind, int kind, const float* q, int64_t n, float eps,
                     uint8_t* answer, uint64_t* n_exact, void* stream) {
  NB_REQUIRE(b && ind && q && answer && n_exact, "NULL argument");
  NB_REQUIRE(kind >= NB_QUERY_POINT && kind <= NB_QUERY_PLANE, "unknown query kind %d", kind);
  NB_REQUIRE(n > 0 && n <= (int64_t)0x7FFFFFFF, "n must be in 1..2^31-1");
  NB_REQUIRE(eps >= 0.0f && eps < 0.5f, "eps must be in [0, 0.5)");
  NB_REQUIRE(kind_dim(kind, ind->dim) == b->in_dim, "bound input dimension %d does not match the query", b->in_dim);
  hipStream_t s = as_stream(stream);
  if (b->cascade_cap < n) {
    NB_HIP(hipStreamSynchronize(s));
    dev_free(b->cascade_idx);
    b->cascade_cap = 0;
    NB_TRY(dev_alloc(&b->cascade_idx, (size_t)n));
    b->cascade_cap = n;
  }
  auto* cnt = reinterpret_cast<unsigned long long*>(n_exact);
  NB_TRY(launch_zero_u64(cnt, 1, s));
  const float tau = tau_of(eps);
  if (b->precision == NB_BF16)
    NB_TRY(bf16_forward(b, q, n, tau, nullptr, answer, nullptr, nullptr, s));
  else
    NB_TRY(f32_forward(b, q, n, tau, nullptr, answer, nullptr, nullptr, s));
  return launch_cascade_exact(ind, kind, q, answer, n, b->cascade_idx, cnt, answer, s);
}

nb_status nb_cascade_noalloc(nb_bound* b, const nb_indicator* ind, int kind, const float* q, int64_t n, float eps,
                             uint8_t* answer, uint64_t* n_exact, void* stream) {
  NB_REQUIRE(b && ind && q && answer && n_exact, "NULL argument");
  NB_REQUIRE(kind >= NB_QUERY_POINT && kind <= NB_QUERY_PLANE, "unknown query kind %d", kind);
  NB_REQUIRE(n > 0 && n <= (int64_t)NB_CASCADE_NOALLOC_MAX, "n must be in 1..%d", NB_CASCADE_NOALLOC_MAX);
  NB_REQUIRE(eps >= 0.0f && eps < 0.5f, "eps must be in [0, 0.5)");
  NB_REQUIRE(kind_dim(kind, ind->dim) == b->in_dim, "bound input dimension %d does not match the query", b->in_dim);
  hipStream_t s = as_stream(stream);
  int32_t* idx = nullptr;
  NB_TRY(cascade_scratch(&idx));
  auto* cnt = reinterpret_cast<unsigned long long*>(n_exact);
  NB_TRY(launch_zero_u64(cnt, 1, s));
  const float tau = tau_of(eps);
  if (b->precision == NB_BF16)
    NB_TRY(bf16_forward(b, q, n, tau, nullptr, answer, nullptr, nullptr, s));
  else
    NB_TRY(f32_forward(b, q, n, tau, nullptr, answer, nullptr, nullptr, s));
  return launch_cascade_exact(ind, kind, q, answer, n, idx, cnt, answer, s);
}

nb_status nb_bound_sync(nb_bound* b, void* stream) {
  NB_REQUIRE(b, "bound is NULL");
  NB_HIP(hipStreamSynchronize(as_stream(stream)));
  unsigned flag = 0;
  NB_HIP(hipMemcpy(&flag, b->d_nonfinite, sizeof(flag), hipMemcpyDeviceToHost));
  if (flag) {
    NB_HIP(hipMemset(b->d_nonfinite, 0, sizeof(unsigned)));
    nb_set_error("a training step since the last check met a non-finite loss or gradient");
    return NB_ERR_NONFINITE;
  }
  return NB_OK;
}

}  // extern "C"
