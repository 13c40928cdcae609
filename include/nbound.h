/*
 * nbound.h -- C ABI of libnbound, a HIP (gfx950) implementation of the
 * data-parallel hot path of Neural Bounding (Liu, Fischer, Yoo, Ritschel,
 * "Neural Bounding", SIGGRAPH 2024, arXiv 2310.06822).
 *
 * The problem (Sec. 3.1, "Method"): an indicator f(x) in {0,1} is 1 inside an
 * object and on its surface; a query g(r) over a region r is 1 iff f is 1
 * somewhere in r (for points g = f).  A bound h_theta(r) in {0,1} must be 1
 * wherever g(r) = 1 and may also be 1 elsewhere (false positives).  h_theta
 * is an MLP with a sigmoid output rounded to {0,1} (Sec. 3.4,
 * "Architecture"), trained with the asymmetric weighted cross-entropy of
 * Eq. 1 by Adam (Sec. 3.4, "Training"), on regions drawn uniformly and
 * labelled by the exact query (Alg. 1).
 *
 * Conventions shared by every call
 *   - Every call returns nb_status.  NB_OK is 0.  On failure the call has
 *     enqueued no work, and nb_last_error() returns a message (per thread).
 *   - Array arguments are DEVICE pointers owned by the caller unless the
 *     argument name ends in _host.  Arrays are dense and row-major.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *     the null stream) and runs asynchronously: results are valid once the
 *     stream has been synchronised.  Only set-up calls synchronise: the
 *     *_create / *_destroy calls (which allocate or free memory),
 *     nb_voxelize_metaballs, and nb_bound_train_step / nb_cascade when their
 *     batch grows beyond every earlier one (they then enlarge work space).
 *   - Queries are float32 rows:  point [n, d] (d = 2, 3 or 4: x, y, z, t);
 *     ray [n, 6] = (origin, unit direction); box [n, 6] = (min corner,
 *     max corner); plane [n, 6] = (point p0, unit normal).  These follow the
 *     supplemental "Parameterization" paragraph.
 *   - Parameters theta are float32 in linear-layer layout: for each layer in
 *     order, W[out][in] row-major, then b[out].  A bound "in_dim x w^H"
 *     has layers in_dim -> w -> ... -> w (H hidden layers) -> 1 logit.
 *   - The decision uses the output epsilon of the supplemental "Numerics"
 *     paragraph: h = 1 iff sigmoid(z) + eps >= 1/2, evaluated as
 *     !(z < tau) with tau = ln((1/2 - eps)/(1/2 + eps)) rounded to float32.
 *     NaN logits give h = 1 (the conservative side).  A query row with a
 *     non-finite value (NaN or +-inf) cannot be bounded: every forward
 *     (single, grouped, streamed, early-out, k-DOP) gives it logit NaN and
 *     so h = 1; such rows never raise an error.
 *   - The handles (nb_indicator, nb_bound) own device memory on the device
 *     that was current when they were created; use them with that device
 *     current.  A handle may be used from one stream at a time.
 */
#ifndef NBOUND_H
#define NBOUND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nb_status;
enum {
  NB_OK = 0,
  NB_ERR_INVALID_ARG = 1, /* NULL pointer, bad size, shape or kind */
  NB_ERR_NO_DEVICE = 2,   /* no HIP device visible */
  NB_ERR_HIP = 3,         /* a HIP runtime call failed (message has the code) */
  NB_ERR_OOM = 4,         /* device allocation failed */
  NB_ERR_NONFINITE = 5,   /* a training step met a non-finite loss or gradient (see *_sync) */
  NB_ERR_UNSUPPORTED = 6  /* valid request the library has no kernel for */
};

/* Query kinds (Sec. 4.2, "Query types"). */
enum { NB_QUERY_POINT = 0, NB_QUERY_RAY = 1, NB_QUERY_BOX = 2, NB_QUERY_PLANE = 3 };

/* Arithmetic of the hidden layers. */
enum { NB_F32 = 0, NB_BF16 = 1 };

typedef struct nb_indicator nb_indicator;
typedef struct nb_bound nb_bound;

/* Message of the last failed call on this thread ("" if none).  The string
 * is owned by the library and valid until the next call on this thread. */
const char* nb_last_error(void);

/* Library version (major, minor); never fails for non-NULL pointers. */
nb_status nb_version(int* major, int* minor);

/* Number of visible HIP devices (0 is not an error here). */
nb_status nb_device_count(int* count);

/* ------------------------------------------------------------------------
 * Indicators f (Sec. 3.1).  Synthetic scenes stand in for the paper's
 * images, voxelised meshes and animations (Sec. 4.2, "Indicators").
 * ---------------------------------------------------------------------- */

/* 2-D union of discs: f(x, y) = 1 iff (x-cx)^2 + (y-cy)^2 <= r^2 for some
 * disc.  discs_host: [k, 3] rows (cx, cy, r), copied.  1 <= k <= 64. */
nb_status nb_indicator_discs2d(const float* discs_host, int k, nb_indicator** out);

/* 3-D voxel grid over [-1, 1]^3: grid is uint8[n^3] (device), x fastest,
 * index (k*n + j)*n + i, any non-zero byte is occupied; copied into the
 * handle.  The cell of a coordinate p is floor((p + 1) * (n/2)) (p = 1 maps
 * to n - 1); points outside the cube have f = 0.  n is 2..1024. */
nb_status nb_indicator_voxels(const uint8_t* grid, int n, nb_indicator** out);

/* 4-D moving metaballs: ball b moves from a_b (t = 0) to b_b (t = 1) along
 * c_b(t) = a_b + t (b_b - a_b); f(x, t) = 1 iff
 * sum_b R_b^2 / |x - c_b(t)|^2 >= iso.  Arrays [k,3], [k,3], [k] on the
 * host, copied.  1 <= k <= 64. */
nb_status nb_indicator_metaballs4d(const float* a_host, const float* b_host, const float* radii_host,
                                   int k, float iso, nb_indicator** out);

/* Dimension of the indicator's domain (2, 3 or 4). */
nb_status nb_indicator_dim(const nb_indicator* ind, int* dim);

nb_status nb_indicator_destroy(nb_indicator* ind);

/* Voxelise a 3-D metaball field: grid[(k*n + j)*n + i] = 1 iff
 * sum_b R_b^2 / |c_ijk - c_b|^2 >= iso at the cell centre
 * c_i = (2i + 1)/n - 1.  centres_host [k,3], radii_host [k]; grid is a
 * device uint8[n^3] written by the call.  1 <= k <= 64, 2 <= n <= 1024.
 * A set-up call: it synchronises `stream` before returning. */
nb_status nb_voxelize_metaballs(const float* centres_host, const float* radii_host, int k, float iso,
                                int n, uint8_t* grid, void* stream);

/* ------------------------------------------------------------------------
 * Exact query g (Sec. 3.1; Sec. 4.2: any() of the indicator over the region)
 *   point  g = f(x)                       (any indicator; d = its dimension)
 *   ray    g = max_j f(o + t_j d), t_j = 4 j / 255 for j = 0..255
 *                                          (voxel indicators)
 *   box    g = 1 iff an occupied cell meets the closed box [lo, hi]
 *                                          (voxel indicators)
 *   plane  g = 1 iff an occupied cell meets the plane through p0 with unit
 *          normal n: |n.(c - p0)| <= (|n_x| + |n_y| + |n_z|) / grid_n
 *                                          (voxel indicators)
 * q: [n, d] float32; g: uint8[n] (0/1).  All geometry is float32, one IEEE
 * operation at a time, no fused multiply-add.
 * ---------------------------------------------------------------------- */
nb_status nb_query_exact(const nb_indicator* ind, int kind, const float* q, int64_t n, uint8_t* g,
                         void* stream);

/* ------------------------------------------------------------------------
 * Region sampling for training (Alg. 1, "Uniform").  Draws n regions of the
 * given kind from Philox4x32-10 (Salmon et al., SC'11) with key = seed and
 * counter = (i, step, stream, attempt); u = (word >> 8) * 2^-24.
 *   point (dim 2, 3): 2u - 1 per coordinate; dim 4: xyz = 2u - 1, t = u
 *   ray:   origin 4u - 2 accepted inside the radius-2 ball (stream 1),
 *          direction by normalised rejection from the unit ball (stream 2)
 *   box:   centre 2u - 1 (stream 3), half extents 0.01 + 0.19u (stream 4)
 *   plane: p0 = 2u - 1 (stream 5), normal as the ray direction (stream 6)
 * q: [n, d] float32 written by the call (d = dim for points, else 6).
 * ---------------------------------------------------------------------- */
nb_status nb_sample_queries(int kind, int dim, uint64_t seed, uint64_t step, int64_t n, float* q,
                            void* stream);

/* ------------------------------------------------------------------------
 * Bound h_theta (Sec. 3.4): in_dim -> width x n_hidden (ReLU) -> 1 logit.
 * Supported: in_dim 1..8;  NB_F32: width 16, 32 or 64 with n_hidden 1..4,
 * width 80 with n_hidden 1..2;  NB_BF16: width 32 or 64 with n_hidden 1..6, width 128 with n_hidden 1..5,
 * width 256 with n_hidden 2..8 (its layers stream through LDS); training
 * needs n_hidden >= 2.  Other shapes give NB_ERR_UNSUPPORTED.
 * The handle owns float32 master parameters, Adam moments and work space.
 * Parameters start at zero; set them with nb_bound_set_params.
 * ---------------------------------------------------------------------- */
nb_status nb_bound_create(int in_dim, int n_hidden, int width, int precision, nb_bound** out);
nb_status nb_bound_destroy(nb_bound* b);
nb_status nb_bound_num_params(const nb_bound* b, int64_t* n_params);
/* Shape of the bound as created (any output pointer may be NULL). */
nb_status nb_bound_shape(const nb_bound* b, int* in_dim, int* n_hidden, int* width, int* precision);

/* Forward kernel variants (tile shapes: query blocks per wave and threads
 * per workgroup) for this bound; every variant computes the same result, so
 * a tuner may time them and keep the fastest.  Variant 0 is the default. */
nb_status nb_bound_num_variants(const nb_bound* b, int* count);
nb_status nb_bound_set_variant(nb_bound* b, int variant);

/* Activation recomputation for bfloat16 training of wide or deep bounds.
 * every = 0 (default) keeps all n_hidden - 1 hidden activations of the batch
 * for the backward pass.  every = k (2..64) keeps only the checkpoints A_0,
 * A_k, A_2k, ... and one segment of k - 1 scratch buffers; the backward
 * recomputes each segment's activations from its checkpoint with the forward
 * kernel (identical bits, so identical gradients) at the cost of about one
 * more forward pass.  Float32 bounds accept only 0. */
nb_status nb_bound_set_recompute(nb_bound* b, int every);

/* Training kernel of a bfloat16 bound (Alg. 1 steps 4-5).  NB_TRAIN_AUTO
 * (default) runs one fused kernel per step for widths 32, 64 and 128 with
 * 2..4 hidden layers and input size <= 8: forward, Eq. 1 and backward of a
 * chunk of the batch on one workgroup, activations and gradients kept on the
 * chip, and the layer-wise kernels (activations of the batch in HBM, one
 * launch per layer and pass) for every other shape.  NB_TRAIN_LAYERWISE
 * forces the layer-wise kernels.  Both compute the same gradient to within
 * float32 summation order.  Repacks the bound's transposed weight fragments
 * on `stream` (the two kernels read them in different orders). */
#define NB_TRAIN_AUTO 0
#define NB_TRAIN_LAYERWISE 1
nb_status nb_bound_set_train_kernel(nb_bound* b, int kernel, void* stream);

/* Hidden-layer activation: NB_ACT_RELU (default) or NB_ACT_SINE, the paper's
 * sinusoidal activation a = sin z (Sec. 3.4, "Architecture"; derivative
 * cos z in training).  Sine is available for float32 bounds of width 32 or
 * 64 with 1..3 hidden layers and of width 80 with 1..2 (narrower layers, such
 * as the paper's 25, 50 or 75 neurons, run exactly as zero-padded ones:
 * sin 0 = 0 and the padding gets no gradient); anything else returns
 * NB_ERR_UNSUPPORTED. */
#define NB_ACT_RELU 0
#define NB_ACT_SINE 1
nb_status nb_bound_set_activation(nb_bound* b, int activation);

/* Copy theta (device, float32[n_params]) into the bound; resets the Adam
 * moments and step count to zero. */
nb_status nb_bound_set_params(nb_bound* b, const float* theta, int64_t n_params, void* stream);
/* Copy the float32 master parameters out (device float32[n_params]). */
nb_status nb_bound_get_params(const nb_bound* b, float* theta, int64_t n_params, void* stream);

/* Optimiser state for checkpoints: m, v are device float32[n_params]; the
 * Adam step count travels through the host integer. */
nb_status nb_bound_get_state(const nb_bound* b, float* m, float* v, int64_t n_params, int64_t* step_host,
                             void* stream);
nb_status nb_bound_set_state(nb_bound* b, const float* m, const float* v, int64_t n_params, int64_t step,
                             void* stream);

/* Checkpoint and resume of a training run (the paper trains each bound for
 * 20-60 minutes, Sec. 3.4 "Training"): everything the training calls read
 * from the handle -- float32 master parameters, Adam moments m and v, the
 * Adam step count -- in one host buffer, so that training resumed from a
 * checkpoint continues bit for bit as if it had not stopped.
 * nb_bound_save: with host_buf NULL, *bytes receives the size needed;
 * otherwise *bytes (in: the buffer's size, at least that much; out: bytes
 * written) and the buffer are filled.  nb_bound_load: restores a checkpoint
 * of a bound of the same shape, precision and activation
 * (NB_ERR_INVALID_ARG otherwise, with the handle unchanged).  Layout: a
 * 48-byte header (magic "NBOUNDCK", version 1, in_dim, n_hidden, width,
 * precision, activation as int32; n_params, Adam step as int64), then theta,
 * m, v as float32[n_params] each, in host byte order.  Both synchronise
 * `stream`. */
nb_status nb_bound_save(const nb_bound* b, void* host_buf, size_t* bytes, void* stream);
nb_status nb_bound_load(nb_bound* b, const void* host_buf, size_t bytes, void* stream);

/* Forward pass and decision over n queries q [n, in_dim].
 *   logits: float32[n] or NULL;  h: uint8[n] decisions or NULL.
 *   g, counts: if both non-NULL, counts (uint64[4], device) is overwritten
 *   with (TP, FP, TN, FN) of h against the exact answers g (uint8[n]).
 * eps is the output epsilon (the paper uses 1e-5), 0 <= eps < 0.5. */
nb_status nb_bound_forward(const nb_bound* b, const float* q, int64_t n, float eps, float* logits,
                           uint8_t* h, const uint8_t* g, uint64_t* counts, void* stream);

/* Loss of Eq. 1 and its gradient on a labelled batch (q [n, in_dim],
 * y uint8[n]): L = (1/n) sum_i [alpha y_i softplus(-z_i) +
 * beta (1 - y_i) softplus(z_i)].  grad: float32[n_params] overwritten with
 * dL/dtheta; loss: float32[1] or NULL; counts: uint64[4] (TP, FP, TN, FN of
 * the decision at eps = 1e-5 against y) or NULL.  The result is
 * deterministic: the reduction order depends on n only.  A bfloat16 bound
 * keeps its activations in HBM for the backward pass ((n_hidden + 1) x n x
 * width x 2 bytes); the first call with a larger n than before synchronises
 * `stream` to enlarge that space. */
nb_status nb_bound_loss_grad(nb_bound* b, const float* q, const uint8_t* y, int64_t n, float alpha, float beta,
                             float* grad, float* loss, uint64_t* counts, void* stream);

/* One Adam step (Kingma & Ba 2014) on the master parameters with gradient
 * grad (device float32[n_params]) plus lam1 sign(W) + 2 lam2 W on weight
 * matrices (L1 + L2 regularisation, supplemental "Regularization"). */
nb_status nb_bound_adam_step(nb_bound* b, const float* grad, float lr, float beta1, float beta2, float adam_eps,
                             float lam1, float lam2, void* stream);

/* One training step of Alg. 1 on the device: sample `batch` regions of
 * `kind` (nb_sample_queries with this seed and step), label them with the
 * exact query on `ind`, evaluate loss and gradient, and take one Adam step
 * (lr, beta1 0.9, beta2 0.999, eps 1e-8).  loss: float32[1] or NULL;
 * counts: uint64[4] on the training batch, or NULL. */
nb_status nb_bound_train_step(nb_bound* b, const nb_indicator* ind, int kind, uint64_t seed, uint64_t step,
                              int64_t batch, float alpha, float beta, float lr, float lam1, float lam2,
                              float* loss, uint64_t* counts, void* stream);
/* Synchronise `stream` and report whether a training call since the last
 * check (nb_bound_train_step, nb_bound_loss_grad) met a non-finite loss or
 * gradient: NB_ERR_NONFINITE if so (the flag is then cleared; the parameters
 * updated from such a gradient are not finite either), NB_OK otherwise.  The
 * training calls themselves never synchronise to look. */
nb_status nb_bound_sync(nb_bound* b, void* stream);

/* ------------------------------------------------------------------------
 * Cascade (Sec. 1, Sec. 6 "Tightness"): the bound screens the queries and
 * only the ones it calls positive reach the exact test.
 *   answer[i] = g(q_i) if h(q_i) = 1, else 0        (uint8[n], device)
 * so answer equals g for every query iff the bound has no false negative.
 * n_exact (uint64[1], device) is overwritten with the number of exact tests
 * run (= number of positives).  The bound's input dimension must match the
 * query.  Keeps an int32[n] index list in the bound: the first call with a
 * larger n than before synchronises `stream` to enlarge it.  n < 2^31. */
nb_status nb_cascade(nb_bound* b, const nb_indicator* ind, int kind, const float* q, int64_t n, float eps,
                     uint8_t* answer, uint64_t* n_exact, void* stream);

/* nb_cascade without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops).  Same
 * arguments, result and errors as nb_cascade, except that the positives'
 * index list lives in a library-owned device array of NB_CASCADE_NOALLOC_MAX
 * int32 entries (16 MiB, one per GPU, held until the process ends) instead
 * of the bound: n above NB_CASCADE_NOALLOC_MAX gives NB_ERR_INVALID_ARG.
 * The call never synchronises and never allocates.  All calls on one GPU
 * share that array: calls whose work overlaps on one GPU (other streams,
 * other threads) race and must be ordered by the caller. */
#define NB_CASCADE_NOALLOC_MAX (1 << 22)
nb_status nb_cascade_noalloc(nb_bound* b, const nb_indicator* ind, int kind, const float* q, int64_t n, float eps,
                             uint8_t* answer, uint64_t* n_exact, void* stream);

/* Neural early-out (Sec. 3, "Neural Early-out"): the early exit is a small
 * network on the region that is trained inverse-conservatively against the
 * complement 1 - g, i.e. it may only declare a region empty where g = 0.
 * Written as a bound, that is a small conservative bound `first` (trained
 * with the usual FN-weighted loss; its negative decisions are the exits).
 * Every query is decided by `first`; the ones it reports positive are
 * gathered, decided by the larger `second`, and scattered back, so
 * h = h_first AND h_second (uint8[n], overwritten), conservative whenever
 * both are.  n_second (device uint64[1]) receives the number of queries
 * `second` evaluated.  Both bounds take the same input size; the work space
 * lives on `second` (the first call with a larger n synchronises `stream`).
 * n <= 2^31 - 1. */
nb_status nb_early_out(const nb_bound* first, nb_bound* second, const float* q, int64_t n, float eps, uint8_t* h,
                       uint64_t* n_second, void* stream);

/* ------------------------------------------------------------------------
 * k-DOP bounds trained with the asymmetric loss (Sec. 4.1, "Methods"; the
 * supplemental uses k = 4 directions): the planes of k slabs in 2-4 D.
 * Parameters (device float32[k*d + 2k + 1]): directions n_1 .. n_k (d each),
 * lower offsets lo_1 .. lo_k, upper offsets hi_1 .. hi_k, logit scale s.
 * A region's projection onto n_j is [u_j, v_j] (a point: n.x; a box [a, b]:
 * n.c -+ sum_i |n_i| e_i with c = (a+b)/2, e = (b-a)/2; a ray segment
 * o + t w, t in [0, 4]: min / max of n.o and n.(o + 4w)), and the logit is
 * z = s min_j min(hi_j - u_j, v_j - lo_j) (z >= 0 iff the region's
 * projection meets every slab, necessary for meeting the k-DOP).  The
 * decision and the loss are the network's.  Query kinds: points (d = 2, 3,
 * 4), boxes and rays (d = 3).
 * ---------------------------------------------------------------------- */
typedef struct nb_kdop nb_kdop;

nb_status nb_kdop_create(int dim, int k, nb_kdop** out);   /* k in 1..8 */
nb_status nb_kdop_destroy(nb_kdop* b);
nb_status nb_kdop_num_params(const nb_kdop* b, int64_t* n_params);
/* set resets the Adam state. */
nb_status nb_kdop_set_params(nb_kdop* b, const float* theta, int64_t n_params, void* stream);
nb_status nb_kdop_get_params(const nb_kdop* b, float* theta, int64_t n_params, void* stream);
/* logits float32[n] and/or h uint8[n]; with g and counts (uint64[4],
 * overwritten) also TP, FP, TN, FN against g. */
nb_status nb_kdop_forward(const nb_kdop* b, int kind, const float* q, int64_t n, float eps, float* logits, uint8_t* h,
                          const uint8_t* g, uint64_t* counts, void* stream);
/* One step of Alg. 1 on `batch` sampled regions labelled by `ind` (same
 * dimension): Eq. 1 with (alpha, beta), the gradient of z through the
 * arg-min slab (the first on ties, its upper side on ties), a fixed-order
 * reduction and one Adam step (lr, 0.9, 0.999, 1e-8).  loss: float32[1]
 * batch mean or NULL; counts: uint64[4] or NULL. */
nb_status nb_kdop_train_step(nb_kdop* b, const nb_indicator* ind, int kind, uint64_t seed, uint64_t step,
                             int64_t batch, float alpha, float beta, float lr, float* loss, uint64_t* counts,
                             void* stream);
/* As nb_bound_sync, for the k-DOP's training steps. */
nb_status nb_kdop_sync(nb_kdop* b, void* stream);

/* ------------------------------------------------------------------------
 * Groups of per-object bounds.  The paper fits one bound per object and does
 * not generalise across objects (Sec. 3.4, "Training"); a group holds n_obj
 * bfloat16 bounds with a common input size and depth (2..4 hidden layers)
 * but their own widths (32, 64 or 128), each with its own voxel grid, so
 * hundreds of bounds train and answer queries in a few launches.
 * Parameters are the objects' theta vectors concatenated in object order
 * (offsets from nb_group_param_offsets).  Queries are grouped by object:
 * qoff (device int64[n_obj + 1], non-decreasing) gives object o the rows
 * qoff[o] .. qoff[o+1]-1 of q.
 * ---------------------------------------------------------------------- */
typedef struct nb_group nb_group;

nb_status nb_group_create(int n_obj, int in_dim, const int* widths_host, int n_hidden, int precision,
                          nb_group** out);
nb_status nb_group_destroy(nb_group* g);
nb_status nb_group_num_params(const nb_group* g, int64_t* n_params);
/* offsets_host: int64[n_obj + 1], object o's parameters are theta[off[o] .. off[o+1]). */
nb_status nb_group_param_offsets(const nb_group* g, int64_t* offsets_host);
/* Copy all objects' parameters in (resets the Adam state) / out (device float32). */
nb_status nb_group_set_params(nb_group* g, const float* theta, int64_t n_params, void* stream);
nb_status nb_group_get_params(const nb_group* g, float* theta, int64_t n_params, void* stream);
/* Per-object voxel grids over [-1, 1]^3 (as nb_indicator_voxels), concatenated
 * in object order on the device; n_host[o] is object o's grid size.  Copied;
 * synchronises the device. */
nb_status nb_group_set_voxels(nb_group* g, const uint8_t* grids, const int* n_host);
/* How the grouped exact test answers boxes: 1 (default) through each
 * object's occupied-cell count table, (n+1)^3 int32 built by
 * nb_group_set_voxels (any occupied cell in the box's cell range <=> a
 * positive count: the same answer in constant time); 0 by scanning the
 * box's cells.  Both give identical results. */
nb_status nb_group_set_box_method(nb_group* g, int method);
/* Exact point / ray / box query of every row against its object's grid;
 * g: uint8[n] (rows outside qoff[0] .. qoff[n_obj]-1 are left untouched). */
nb_status nb_group_query_exact(const nb_group* g, int kind, const float* q, const int64_t* qoff, int64_t n,
                               uint8_t* g_out, void* stream);
/* Forward + decision (Eq. 1's logit, h = !(z < tau(eps)) as for a single
 * bound, bit for bit) of every row with its object's bound: one planner
 * launch, then one persistent launch per width class (tiles of queries of
 * one object, equal runs of tiles per workgroup, weights loaded into LDS
 * once per run).
 * logits float32[n] and/or h uint8[n]; with g_exact (uint8[n]) and counts
 * (uint64[n_obj][4], overwritten) also each object's TP, FP, TN, FN.  An
 * object whose rows qoff[o] .. qoff[o+1]-1 do not lie inside [0, n) is
 * skipped (its outputs are left as they are, its counts stay 0). */
nb_status nb_group_forward(const nb_group* g, const float* q, const int64_t* qoff, int64_t n, float eps,
                           float* logits, uint8_t* h, const uint8_t* g_exact, uint64_t* counts, void* stream);
/* Tile-shape variants of the grouped forward (threads per workgroup and
 * query blocks per wave); all give identical results.  The forward runs one
 * launch per width class, each with its own variant (default 0):
 * nb_group_set_variant sets every class's, nb_group_set_width_variant the
 * variant of the objects of one width (32, 64 or 128; NB_ERR_INVALID_ARG for
 * another width or a variant outside 0 .. count-1). */
nb_status nb_group_num_variants(const nb_group* g, int* count);
nb_status nb_group_set_variant(nb_group* g, int variant);
nb_status nb_group_set_width_variant(nb_group* g, int width, int variant);
/* One training step of Alg. 1 for every object: per_obj regions of `kind`
 * per object (nb_sample_queries with n = n_obj * per_obj; object o takes rows
 * o*per_obj ..), labelled on the object's grid, Eq. 1 with FN weight alpha
 * (or alpha_obj[o], device float32[n_obj], when alpha_obj is non-NULL) and
 * beta, one Adam step (0.9, 0.999, 1e-8) per object with learning rate lr
 * (or lr_obj[o], device float32[n_obj]; 0 freezes object o: its parameters
 * and Adam moments are left as they are, which is how an object that has
 * met its stopping rule stops training while the others go on).  loss:
 * float32[n_obj] per-object mean loss or NULL; counts: uint64[n_obj][4] or
 * NULL.  The first step with a new per_obj synchronises `stream` to size the
 * work space. */
/* Restrict training to the objects with active_host[o] != 0 (host uint8[n_obj];
 * NULL: all).  The others' networks are neither evaluated nor updated by
 * nb_group_train_step, and their loss and counts entries are not written.
 * Synchronous (uploads the member lists). */
nb_status nb_group_set_active(nb_group* g, const uint8_t* active_host);
nb_status nb_group_train_step(nb_group* g, int kind, uint64_t seed, uint64_t step, int64_t per_obj, float alpha,
                              const float* alpha_obj, float beta, float lr, const float* lr_obj, float* loss,
                              uint64_t* counts, void* stream);
/* As nb_bound_sync, for the group's training steps (any object). */
nb_status nb_group_sync(nb_group* g, void* stream);

/* ------------------------------------------------------------------------
 * Neural bounding hierarchies (Sec. 3.3).  The tree is supplied by the
 * user; its nodes are the objects of a group (node i = object i), and each
 * node's network is meant to bound, conservatively, the union of the
 * indicators of the leaves below it (a leaf bounds its own object), so
 * that a region meeting a leaf's object is positive at every node on the
 * path from the root.  Nodes are numbered breadth first with node 0 the
 * root: node p's children are the nodes child_begin[p] .. child_end[p]-1,
 * and the children ranges taken in parent order are exactly 1 .. n_obj-1
 * (empty range: p is a leaf).  Leaves are ranked in node order.
 * ------------------------------------------------------------------------ */
typedef struct nb_hier nb_hier;

/* child_begin_host, child_end_host: int32[n_obj] (copied).  The hierarchy
 * refers to g, which must outlive it; g's parameters are read at each
 * query.  NB_ERR_INVALID_ARG if the ranges do not describe such a tree. */
nb_status nb_hier_create(nb_group* g, const int32_t* child_begin_host, const int32_t* child_end_host,
                         nb_hier** out);
nb_status nb_hier_destroy(nb_hier* h);
nb_status nb_hier_num_leaves(const nb_hier* h, int32_t* n_leaves);
/* nodes_host: int32[n_leaves], the node of each leaf rank. */
nb_status nb_hier_leaf_nodes(const nb_hier* h, int32_t* nodes_host);
/* Number of tree levels (the root's level is 0). */
nb_status nb_hier_depth(const nb_hier* h, int32_t* depth);
/* pairs_host: int64[depth], the (row, node) pairs each level of the last
 * nb_hier_query evaluated (level 0: the rows; zeros before any query). */
nb_status nb_hier_level_pairs(const nb_hier* h, int64_t* pairs_host);
/* Descend the tree with every row of q (float32[n][in_dim] on the device;
 * one decision !(z < tau(eps)) per visited (row, node) pair, as the grouped
 * forward): the output holds each pair (row, leaf) whose leaf and all of
 * whose ancestors decide positive, grouped by leaf rank.  leaf_off (device
 * int64[n_leaves + 1]) receives the segments; leaf r's rows are
 * qidx_out[leaf_off[r] .. leaf_off[r+1]-1] (device int32[cap]) in increasing
 * order.  *n_pairs_host receives the number of pairs.  Work space grows
 * inside the handle as needed; the call synchronises `stream` once per tree
 * level (the host sizes each level).  If the pairs exceed cap, entries
 * beyond cap are not written and NB_ERR_INVALID_ARG is returned with
 * *n_pairs_host set, so the caller can retry with a larger buffer.  n must
 * be below 2^31, as must the pairs of every level.  The handle's work space
 * and its group are shared by every call: calls on one hierarchy must not
 * overlap (one host thread at a time). */
nb_status nb_hier_query(nb_hier* h, const float* q, int64_t n, float eps, int32_t* qidx_out, int64_t cap,
                        int64_t* leaf_off, int64_t* n_pairs_host, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NBOUND_H */
