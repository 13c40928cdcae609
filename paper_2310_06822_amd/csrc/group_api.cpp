// extern "C" entry points for groups of per-object bounds (nbound.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "nb_internal.h"
#include "nb_mlp.h"

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <class T>
nb_status alloc_n(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return NB_OK;
  NB_HIP(hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)));
  return NB_OK;
}

template <class T>
void free_p(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <class T>
nb_status upload(T** dst, const std::vector<T>& src) {
  NB_TRY(alloc_n(dst, src.size()));
  if (!src.empty()) NB_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return NB_OK;
}

float tau_of(float eps) { return (float)std::log((0.5 - (double)eps) / (0.5 + (double)eps)); }

int64_t mlp_params(int in_dim, int n_hidden, int width) {
  return (int64_t)width * in_dim + width + (int64_t)(n_hidden - 1) * ((int64_t)width * width + width) + width + 1;
}

const int kClassWidths[3] = {32, 64, 128};

}  // namespace

extern "C" {

nb_status nb_group_destroy(nb_group* g) {
  if (!g) return NB_OK;
  free_p(g->d_widths);
  free_p(g->d_poff);
  free_p(g->d_pkoff);
  free_p(g->d_ptoff);
  free_p(g->d_perm);
  free_p(g->d_class);
  free_p(g->d_active);
  free_p(g->d_nonfinite);
  free_p(g->theta);
  free_p(g->m);
  free_p(g->v);
  free_p(g->pack16);
  free_p(g->pack16t);
  free_p(g->grids);
  free_p(g->d_goff);
  free_p(g->d_gn);
  free_p(g->ray_t);
  free_p(g->table);
  free_p(g->d_toff);
  free_p(g->d_item_off);
  free_p(g->d_wg_first);
  free_p(g->partial);
  free_p(g->aux);
  free_p(g->tr_ws);
  free_p(g->batch_q);
  free_p(g->batch_y);
  free_p(g->d_qoff_train);
  delete g;
  return NB_OK;
}

nb_status nb_group_create(int n_obj, int in_dim, const int* widths_host, int n_hidden, int precision,
                          nb_group** out) {
  NB_REQUIRE(out && widths_host, "NULL argument");
  *out = nullptr;
  NB_REQUIRE(n_obj >= 1 && n_obj <= 4096, "n_obj must be in 1..4096");
  NB_REQUIRE(in_dim >= 1 && in_dim <= 8, "in_dim must be in 1..8");
  NB_REQUIRE(n_hidden >= 2 && n_hidden <= 4, "grouped bounds take 2..4 hidden layers");
  NB_REQUIRE(precision == NB_BF16, "grouped bounds are bfloat16");
  for (int o = 0; o < n_obj; ++o)
    NB_REQUIRE(widths_host[o] == 32 || widths_host[o] == 64 || widths_host[o] == 128,
               "object %d: width %d is not 32, 64 or 128", o, widths_host[o]);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    nb_set_error("no HIP device is visible");
    return NB_ERR_NO_DEVICE;
  }
  auto* g = new nb_group();
  g->n_obj = n_obj;
  g->in_dim = in_dim;
  g->n_hidden = n_hidden;
  g->precision = precision;
  hipGetDevice(&g->device);
  g->widths.assign(widths_host, widths_host + n_obj);
  g->poff.assign(n_obj + 1, 0);
  g->pkoff.assign(n_obj + 1, 0);
  g->ptoff.assign(n_obj + 1, 0);
  for (int o = 0; o < n_obj; ++o) {
    g->poff[o + 1] = g->poff[o] + mlp_params(in_dim, n_hidden, g->widths[o]);
    g->pkoff[o + 1] = g->pkoff[o] + nb_bf16_fwd_slices(g->widths[o], n_hidden);
    g->ptoff[o + 1] = g->ptoff[o] + nb_bf16_t_slices(g->widths[o], n_hidden);
  }
  g->n_params = g->poff[n_obj];
  for (int o = 0; o < n_obj; ++o) g->max_obj_params = std::max(g->max_obj_params, g->poff[o + 1] - g->poff[o]);
  g->pack_elems = g->pkoff[n_obj] * 8;
  g->packt_elems = g->ptoff[n_obj] * 8;
  std::vector<int> perm(n_obj);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return g->widths[a] > g->widths[b]; });
  g->classes.assign(3, {});
  g->class_all.assign(3, 0);
  std::vector<int> cls;
  for (int c = 0; c < 3; ++c) {
    for (int o = 0; o < n_obj; ++o)
      if (g->widths[o] == kClassWidths[c]) g->classes[c].push_back(o);
    g->class_all[c] = (int)g->classes[c].size();
    cls.insert(cls.end(), g->classes[c].begin(), g->classes[c].end());
  }
  g->n_wg_cap = std::max(1, std::min(8 * nb_cu_count(), 1 << 14));
  nb_status st = upload(&g->d_widths, g->widths);
  if (st == NB_OK) st = upload(&g->d_poff, g->poff);
  if (st == NB_OK) st = upload(&g->d_pkoff, g->pkoff);
  if (st == NB_OK) st = upload(&g->d_ptoff, g->ptoff);
  if (st == NB_OK) st = upload(&g->d_perm, perm);
  if (st == NB_OK) st = upload(&g->d_class, cls);
  if (st == NB_OK) st = upload(&g->d_active, std::vector<uint8_t>(n_obj, 1));
  if (st == NB_OK) st = upload(&g->d_nonfinite, std::vector<unsigned>(1, 0u));
  if (st == NB_OK) st = alloc_n(&g->theta, (size_t)g->n_params);
  if (st == NB_OK) st = alloc_n(&g->m, (size_t)g->n_params);
  if (st == NB_OK) st = alloc_n(&g->v, (size_t)g->n_params);
  if (st == NB_OK) st = alloc_n(&g->pack16, (size_t)g->pack_elems);
  if (st == NB_OK) st = alloc_n(&g->pack16t, (size_t)g->packt_elems);
  if (st == NB_OK) st = alloc_n(&g->d_item_off, (size_t)n_obj + 3);
  if (st == NB_OK) st = alloc_n(&g->d_wg_first, 3 * ((size_t)g->n_wg_cap + 1));
  if (st == NB_OK) st = alloc_n(&g->ray_t, 256);
  if (st == NB_OK) {
    float t[256];
    for (int j = 0; j < 256; ++j) t[j] = (float)(4.0 * j / 255.0);
    if (hipMemcpy(g->ray_t, t, sizeof(t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(g->theta, 0, g->n_params * 4) != hipSuccess || hipMemset(g->m, 0, g->n_params * 4) != hipSuccess ||
        hipMemset(g->v, 0, g->n_params * 4) != hipSuccess) {
      nb_set_error("initialising the group state failed");
      st = NB_ERR_HIP;
    }
  }
  if (st != NB_OK) {
    nb_group_destroy(g);
    return st;
  }
  *out = g;
  return NB_OK;
}

nb_status nb_group_num_params(const nb_group* g, int64_t* n_params) {
  NB_REQUIRE(g && n_params, "NULL argument");
  *n_params = g->n_params;
  return NB_OK;
}

nb_status nb_group_param_offsets(const nb_group* g, int64_t* offsets_host) {
  NB_REQUIRE(g && offsets_host, "NULL argument");
  std::memcpy(offsets_host, g->poff.data(), sizeof(int64_t) * (g->n_obj + 1));
  return NB_OK;
}

nb_status nb_group_set_params(nb_group* g, const float* theta, int64_t n_params, void* stream) {
  NB_REQUIRE(g && theta, "NULL argument");
  NB_REQUIRE(n_params == g->n_params, "group has %lld parameters, got %lld", (long long)g->n_params,
             (long long)n_params);
  hipStream_t s = as_stream(stream);
  NB_HIP(hipMemcpyAsync(g->theta, theta, n_params * 4, hipMemcpyDeviceToDevice, s));
  NB_HIP(hipMemsetAsync(g->m, 0, n_params * 4, s));
  NB_HIP(hipMemsetAsync(g->v, 0, n_params * 4, s));
  g->adam_t = 0;
  return group_pack(g, s);
}

nb_status nb_group_get_params(const nb_group* g, float* theta, int64_t n_params, void* stream) {
  NB_REQUIRE(g && theta, "NULL argument");
  NB_REQUIRE(n_params == g->n_params, "parameter count mismatch");
  NB_HIP(hipMemcpyAsync(theta, g->theta, n_params * 4, hipMemcpyDeviceToDevice, as_stream(stream)));
  return NB_OK;
}

nb_status nb_group_set_voxels(nb_group* g, const uint8_t* grids, const int* n_host) {
  NB_REQUIRE(g && grids && n_host, "NULL argument");
  std::vector<int64_t> goff(g->n_obj + 1, 0), toff(g->n_obj + 1, 0);
  std::vector<int> gn(n_host, n_host + g->n_obj);
  int max_n = 0;
  for (int o = 0; o < g->n_obj; ++o) {
    NB_REQUIRE(gn[o] >= 2 && gn[o] <= 1024, "object %d: grid size %d out of range", o, gn[o]);
    goff[o + 1] = goff[o] + (int64_t)gn[o] * gn[o] * gn[o];
    toff[o + 1] = toff[o] + (int64_t)(gn[o] + 1) * (gn[o] + 1) * (gn[o] + 1);
    max_n = std::max(max_n, gn[o]);
  }
  free_p(g->grids);
  free_p(g->d_goff);
  free_p(g->d_gn);
  free_p(g->table);
  free_p(g->d_toff);
  NB_TRY(alloc_n(&g->grids, (size_t)goff[g->n_obj]));
  NB_HIP(hipMemcpy(g->grids, grids, (size_t)goff[g->n_obj], hipMemcpyDeviceToDevice));
  NB_TRY(upload(&g->d_goff, goff));
  NB_TRY(upload(&g->d_gn, gn));
  NB_TRY(upload(&g->d_toff, toff));
  NB_TRY(alloc_n(&g->table, (size_t)toff[g->n_obj]));
  NB_TRY(group_build_tables(g, max_n, nullptr));
  NB_HIP(hipDeviceSynchronize());
  return NB_OK;
}

nb_status nb_group_set_active(nb_group* g, const uint8_t* active_host) {
  NB_REQUIRE(g, "group is NULL");
  std::vector<int> cls;
  for (int c = 0; c < 3; ++c) {
    g->classes[c].clear();
    for (int o = 0; o < g->n_obj; ++o)
      if (g->widths[o] == kClassWidths[c] && (!active_host || active_host[o])) g->classes[c].push_back(o);
    cls.insert(cls.end(), g->classes[c].begin(), g->classes[c].end());
  }
  if (!cls.empty())
    NB_HIP(hipMemcpy(g->d_class, cls.data(), cls.size() * sizeof(int), hipMemcpyHostToDevice));
  std::vector<uint8_t> act(g->n_obj, 1);
  if (active_host)
    for (int o = 0; o < g->n_obj; ++o) act[o] = active_host[o] ? 1 : 0;
  NB_HIP(hipMemcpy(g->d_active, act.data(), act.size(), hipMemcpyHostToDevice));
  return NB_OK;
}

nb_status nb_group_set_box_method(nb_group* g, int method) {
  NB_REQUIRE(g, "group is NULL");
  NB_REQUIRE(method == 0 || method == 1, "box method must be 0 (scan) or 1 (count table)");
  g->box_method = method;
  return NB_OK;
}

nb_status nb_group_query_exact(const nb_group* g, int kind, const float* q, const int64_t* qoff, int64_t n,
                               uint8_t* out, void* stream) {
  NB_REQUIRE(g && q && qoff && out, "NULL argument");
  NB_REQUIRE(g->grids, "the group has no voxel grids (nb_group_set_voxels)");
  NB_REQUIRE(kind == NB_QUERY_POINT || kind == NB_QUERY_RAY || kind == NB_QUERY_BOX,
             "grouped exact queries take points, rays or boxes");
  NB_REQUIRE((kind == NB_QUERY_POINT ? 3 : 6) == g->in_dim, "query kind does not match the group's input size");
  NB_REQUIRE(n > 0, "n must be positive");
  return group_exact(g, kind, q, qoff, n, out, as_stream(stream));
}

nb_status nb_group_forward(const nb_group* g, const float* q, const int64_t* qoff, int64_t n, float eps,
                           float* logits, uint8_t* h, const uint8_t* g_exact, uint64_t* counts, void* stream) {
  NB_REQUIRE(g && q && qoff, "NULL argument");
  NB_REQUIRE(logits || h || (g_exact && counts), "nothing to compute");
  NB_REQUIRE(!counts || g_exact, "counts need the exact answers g");
  NB_REQUIRE(n > 0, "n must be positive");
  NB_REQUIRE(eps >= 0.0f && eps < 0.5f, "eps must be in [0, 0.5)");
  return group_forward(g, q, qoff, n, tau_of(eps), logits, h, counts ? g_exact : nullptr,
                       reinterpret_cast<unsigned long long*>(counts), as_stream(stream));
}

nb_status nb_group_num_variants(const nb_group* g, int* count) {
  NB_REQUIRE(g && count, "NULL argument");
  *count = group_variants();
  return NB_OK;
}

nb_status nb_group_set_variant(nb_group* g, int variant) {
  NB_REQUIRE(g, "group is NULL");
  NB_REQUIRE(variant >= 0 && variant < group_variants(), "variant %d out of range 0..%d", variant,
             group_variants() - 1);
  for (int c = 0; c < 3; ++c) g->class_variant[c] = variant;
  return NB_OK;
}

nb_status nb_group_set_width_variant(nb_group* g, int width, int variant) {
  NB_REQUIRE(g, "group is NULL");
  NB_REQUIRE(width == 32 || width == 64 || width == 128, "width must be 32, 64 or 128");
  NB_REQUIRE(variant >= 0 && variant < group_variants(), "variant %d out of range 0..%d", variant,
             group_variants() - 1);
  g->class_variant[width == 32 ? 0 : width == 64 ? 1 : 2] = variant;
  return NB_OK;
}

nb_status nb_group_train_step(nb_group* g, int kind, uint64_t seed, uint64_t step, int64_t per_obj, float alpha,
                              const float* alpha_obj, float beta, float lr, const float* lr_obj, float* loss,
                              uint64_t* counts, void* stream) {
  NB_REQUIRE(g, "group is NULL");
  NB_REQUIRE(g->grids, "the group has no voxel grids (nb_group_set_voxels)");
  NB_REQUIRE(kind == NB_QUERY_BOX || kind == NB_QUERY_RAY || kind == NB_QUERY_POINT, "unsupported query kind");
  NB_REQUIRE((kind == NB_QUERY_POINT ? 3 : 6) == g->in_dim, "query kind does not match the group's input size");
  NB_REQUIRE(per_obj >= 1 && per_obj * g->n_obj <= (int64_t(1) << 31), "per_obj out of range");
  NB_REQUIRE((lr > 0 || lr_obj) && std::isfinite(alpha) && std::isfinite(beta) && alpha >= 0 && beta >= 0,
             "invalid learning rate or loss weights");
  hipStream_t s = as_stream(stream);
  // fewer, longer chunks for large groups: the class launches have
  // members x chunks workgroups (about 2048 in all fill the chip), and the
  // partial gradients cost chunks x parameters of memory traffic, written
  // by the class kernels and read by the reduction (256 objects: 8 chunks,
  // 0.48 ms per step against 0.56 ms with 16 and 0.51 ms with 4)
  const BF16TrainPlan plan = bf16_train_plan(per_obj, std::max(8, 2048 / g->n_obj));
  const int64_t total = per_obj * g->n_obj;
  if (g->tr_per_obj != per_obj) {
    // (re)sizes the work space: synchronising, only when per_obj changes
    NB_HIP(hipStreamSynchronize(s));
    free_p(g->partial);
    free_p(g->aux);
    free_p(g->tr_ws);
    free_p(g->batch_q);
    free_p(g->batch_y);
    free_p(g->d_qoff_train);
    g->tr_per_obj = 0;
    int64_t ws = 0;
    for (int c = 0; c < 3; ++c)
      ws += (int64_t)g->class_all[c] * (g->n_hidden + 1) * plan.padded * kClassWidths[c];
    NB_TRY(alloc_n(&g->partial, (size_t)plan.n_wg * g->n_params));
    NB_TRY(alloc_n(&g->aux, (size_t)g->n_obj * plan.n_wg * 8));
    NB_TRY(alloc_n(&g->tr_ws, (size_t)ws));
    NB_TRY(alloc_n(&g->batch_q, (size_t)total * g->in_dim));
    NB_TRY(alloc_n(&g->batch_y, (size_t)total));
    std::vector<int64_t> qo(g->n_obj + 1);
    for (int o = 0; o <= g->n_obj; ++o) qo[o] = (int64_t)o * per_obj;
    NB_TRY(upload(&g->d_qoff_train, qo));
    g->tr_per_obj = per_obj;
  }
  // Alg. 1: regions for every object (object o's batch is rows o*per_obj ..),
  // exact labels on the object's own grid, then each width class in one
  // launch per layer kernel.
  NB_TRY(launch_sample(kind, 3, seed, step, total, g->batch_q, s));
  NB_TRY(group_exact(g, kind, g->batch_q, g->d_qoff_train, total, g->batch_y, s));
  const float tau = tau_of(1e-5f);
  int64_t ws_off = 0, cls_off = 0;
  for (int c = 0; c < 3; ++c) {
    const int nc = (int)g->classes[c].size();
    if (nc) {
      const int W = kClassWidths[c];
      uint16_t* act = g->tr_ws + ws_off;
      uint16_t* grad = act + (int64_t)nc * (g->n_hidden - 1) * plan.padded * W;
      NB_TRY(bf16_group_train_class(g, W, g->d_class + cls_off, nc, g->batch_q, g->batch_y, per_obj, alpha,
                                    alpha_obj, beta, tau, plan, act, grad, s));
      ws_off += (int64_t)nc * (g->n_hidden + 1) * plan.padded * W;
    }
    cls_off += nc;
  }
  g->adam_t += 1;
  AdamArgs a{};
  a.enabled = 1;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  // bias corrections from the float32 constants, as for a single bound
  a.bc1 = (float)(1.0 - std::pow((double)a.b1, (double)g->adam_t));
  a.bc2 = (float)(1.0 - std::pow((double)a.b2, (double)g->adam_t));
  NB_TRY(group_reduce_adam(g, plan.n_wg, a, lr_obj, loss, reinterpret_cast<unsigned long long*>(counts),
                           (float)(1.0 / (double)per_obj), s));
  return group_pack(g, s);
}

nb_status nb_group_sync(nb_group* g, void* stream) {
  NB_REQUIRE(g, "group is NULL");
  NB_HIP(hipStreamSynchronize(as_stream(stream)));
  unsigned flag = 0;
  NB_HIP(hipMemcpy(&flag, g->d_nonfinite, sizeof(flag), hipMemcpyDeviceToHost));
  if (flag) {
    NB_HIP(hipMemset(g->d_nonfinite, 0, sizeof(unsigned)));
    nb_set_error("a grouped training step since the last check met a non-finite gradient");
    return NB_ERR_NONFINITE;
  }
  return NB_OK;
}

}  // extern "C"
