// Shared pieces of the bfloat16 training kernels (layer-wise and fused):
// which bound a workgroup trains, bfloat16 packing, and the order in which
// activation values sit in an MFMA operand.
#pragma once

#include "nb_internal.h"
#include "nb_mlp.h"

// Which bound a workgroup trains: blockIdx.y selects a member of a list of
// same-width bounds (a group's width class); a single bound has no list.
struct TrObjs {
  const int* objs;        // member -> object id (nullptr: one bound, object 0)
  const int64_t* poff;    // parameter offset per object (nullptr: 0)
  const int64_t* pkoff;   // forward-pack offset per object, 16-byte slices
  const int64_t* ptoff;   // transposed-pack offset per object, 16-byte slices
  int64_t q_stride;       // batch rows per object
  int64_t ms_a, ms_d;     // activation / gradient workspace elements per member
  int64_t P;              // parameters of the single bound (objs == nullptr)
  const float* alpha;     // per-object FN weight of Eq. 1 (nullptr: the scalar alpha)
};

// One training pass of the fused kernel over `members` same-width bounds
// (gridDim.y), each a chunked batch of n queries (plan.n_wg chunks).
struct FusedJob {
  int in_dim = 0, NH = 0, W = 0, members = 1;
  int64_t n = 0;
  BF16TrainPlan plan;
  const float* q = nullptr;
  const uint8_t* y = nullptr;
  const float* theta = nullptr;
  const nb_bf16x8* pack = nullptr;
  const nb_bf16x8* packT = nullptr;   // operand-order transposed fragments
  float* partial = nullptr;
  float* aux = nullptr;
  float alpha = 1, beta = 1, inv_n = 1, tau = 0;
  TrObjs T{};
};

// Launches the fused training step (mlp_bf16_fused.hip).
nb_status bf16_fused_train(const FusedJob& J, hipStream_t s);

// Activation slot of each A_l (l = 0 .. NH-2) that the streamed training
// forward writes; -1: not written (recomputed by the backward).
struct StreamSlots {
  int s[8];
};

// The forward half of a training step of one 256-wide bound in one launch
// (mlp_bf16_train256.hip): the kept activation rows, D_{NH-1}, and the
// chunk partials of the output layer, loss and counts.
struct StreamJob {
  int in_dim = 0, NH = 0;
  int64_t n = 0, P = 0;
  BF16TrainPlan plan;
  const float* q = nullptr;
  const uint8_t* y = nullptr;
  const float* theta = nullptr;
  const nb_bf16x8* pack = nullptr;
  uint16_t* act = nullptr;       // slot k at act + k * act_stride
  int64_t act_stride = 0;
  StreamSlots slots{};
  uint16_t* Dout = nullptr;      // D_{NH-1}, [padded batch][256]
  float* partial = nullptr;
  float* aux = nullptr;
  float alpha = 1, beta = 1, inv_n = 1, tau = 0;
};
// One backward layer of a 256-wide bound (data and weight gradient in one
// launch, mlp_bf16_train256.hip): D_{l-1} and the chunk partials of dW_l, db_l.
struct Back256Job {
  int in_dim = 0, NH = 0, l = 0;
  int64_t P = 0;
  BF16TrainPlan plan;
  const uint16_t* Dl = nullptr;       // [padded batch][256], natural neuron order
  const uint16_t* Aprev = nullptr;    // [padded batch][256], operand order
  const nb_bf16x8* packT = nullptr;   // transposed fragments, natural K order
  uint16_t* Dprev = nullptr;
  float* partial = nullptr;
};
nb_status bf16_back256(const Back256Job& J, hipStream_t s);
// Recomputation of activation rows A_{l0} .. A_{l1} of a 256-wide bound from
// the checkpoint A_{l0-1} in one launch (mlp_bf16_train256.hip).
struct RecomputeJob {
  int in_dim = 0, NH = 0, l0 = 0, l1 = 0;
  BF16TrainPlan plan;
  const uint16_t* ain = nullptr;      // A_{l0-1}
  const nb_bf16x8* pack = nullptr;
  const float* theta = nullptr;
  uint16_t* act = nullptr;            // slot k at act + k * act_stride
  int64_t act_stride = 0;
  StreamSlots slots{};                // slot of each A_l written
};
nb_status bf16_recompute256(const RecomputeJob& J, hipStream_t s);
bool bf16_stream_forward_supported(int in_dim, int n_hidden, int width);
nb_status bf16_stream_forward(const StreamJob& J, hipStream_t s);

namespace {

typedef nb_bf16x8 bf16x8;
typedef nb_floatx4 floatx4;

struct TrObj {
  int o, member;
  int64_t poff, P;
};

__device__ __forceinline__ TrObj tr_obj(const TrObjs& T) {
  TrObj r;
  r.member = blockIdx.y;
  r.o = T.objs ? T.objs[r.member] : 0;
  r.poff = T.poff ? T.poff[r.o] : 0;
  r.P = T.poff ? T.poff[r.o + 1] - r.poff : T.P;
  return r;
}

__device__ __forceinline__ uint16_t bits_of(__bf16 v) { return __builtin_bit_cast(uint16_t, v); }
__device__ __forceinline__ __bf16 bf16_of(uint16_t v) { return __builtin_bit_cast(__bf16, v); }

// Four float32 values rounded to bfloat16 and packed for one 8-byte store.
__device__ __forceinline__ uint2 pack4(float a, float b, float c, float d) {
  return uint2{(uint32_t)bits_of((__bf16)a) | ((uint32_t)bits_of((__bf16)b) << 16),
               (uint32_t)bits_of((__bf16)c) | ((uint32_t)bits_of((__bf16)d) << 16)};
}

__device__ __forceinline__ void unpack4(uint2 u, float v[4]) {
  v[0] = (float)bf16_of((uint16_t)(u.x & 0xFFFF));
  v[1] = (float)bf16_of((uint16_t)(u.x >> 16));
  v[2] = (float)bf16_of((uint16_t)(u.y & 0xFFFF));
  v[3] = (float)bf16_of((uint16_t)(u.y >> 16));
}

// Activation rows A_l in HBM are kept in the order in which the next layer
// reads them as its B operand ("operand order"): within each 32-neuron block
// ks, position 8g + j holds neuron 4g + j for j < 4 and 16 + 4g + (j - 4) for
// j >= 4.  Lane group g of a forward K = 32 step then loads its 8 values
// with one 16-byte load at 32ks + 8g, and the lane that produced them (it
// holds rows 4g .. 4g+3 of row blocks 2ks and 2ks + 1) stores them with one
// 16-byte store.  Gradient rows D_l stay in neuron order.
__device__ __forceinline__ int act_neuron(int p) {   // neuron at position p of an activation row
  return (p & ~31) + 16 * ((p >> 2) & 1) + 4 * ((p >> 3) & 3) + (p & 3);
}
__device__ __forceinline__ int act_pos(int n) {      // position of neuron n
  return (n & ~31) + 8 * ((n >> 2) & 3) + 4 * ((n >> 4) & 1) + (n & 3);
}
__device__ __forceinline__ bf16x8 load_fwd_operand(const uint16_t* __restrict__ row, int ks, int g) {
  return *reinterpret_cast<const bf16x8*>(row + 32 * ks + 8 * g);
}
// ReLU of two row blocks' accumulators (rows 4g .. 4g+3 of blocks 2ks, 2ks + 1),
// rounded to bfloat16, as the 16 bytes at 32ks + 8g of an activation row.
__device__ __forceinline__ uint4 relu_pair(floatx4 a, floatx4 b) {
  const uint2 lo = pack4(fmaxf(a[0], 0.0f), fmaxf(a[1], 0.0f), fmaxf(a[2], 0.0f), fmaxf(a[3], 0.0f));
  const uint2 hi = pack4(fmaxf(b[0], 0.0f), fmaxf(b[1], 0.0f), fmaxf(b[2], 0.0f), fmaxf(b[3], 0.0f));
  return uint4{lo.x, lo.y, hi.x, hi.y};
}

// Raise a kernel's dynamic-LDS limit once per device.
template <class K>
nb_status allow_lds(K kernel, size_t bytes) {
  static bool done[64] = {false};
  int dev = 0;
  NB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64 || done[dev]) return NB_OK;
  NB_HIP(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done[dev] = true;
  return NB_OK;
}

}  // namespace
