// adg_mlp.h — learned ghost-trace predictor: a 2-layer MLP (2V+2 inputs, 64
// GELU hidden units, V outputs) that predicts a scaled correction to the AT
// extrapolation at each PE-boundary face node. Inference runs in BF16 on the
// matrix cores with FP32 accumulation; training (forward, backward, Adam) runs
// in FP32. Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adg_internal.h"

namespace adg {

constexpr int kTrainBlocks = 64;  // blocks per gradient launch
constexpr int kTrainChunk = 64;   // samples per block per launch
constexpr int kMaxBatch = kTrainBlocks * kTrainChunk;
constexpr int kPackBytes = 8192;  // BF16 operand tiles + FP32 biases
constexpr float kTargetClip = 64.0f;  // training targets beyond this get weight 0
// the judge statistics (accepted, judged) are kept in kStatSlots copies that
// wavefronts add to round-robin, so their atomics do not queue on one address
constexpr int kStatSlots = 256;

__host__ __device__ constexpr int mlp_nin(int V) { return 2 * V + 2; }
__host__ __device__ constexpr int mlp_nparams(int V) { return kMlpH * mlp_nin(V) + kMlpH + V * kMlpH + V; }
// one training pair: features, target, weight (floats)
__host__ __device__ constexpr int mlp_pair_floats(int V) { return mlp_nin(V) + V + 1; }

struct MlpState {
  int V = 0;
  bool has_weights = false;   // a network is set (inference on)
  bool device_newer = false;  // device master weights changed by training
  char* base = nullptr;       // scratch sub-area (device), set at bind
  float* pairs = nullptr;     // caller buffer of training pairs (device)
  int64_t max_pairs = 0, n_pairs = 0;
  int64_t adam_t = 0;
  float host_w[kMlpH * 16 + kMlpH + kMaxV * kMlpH + kMaxV];
};

// device views of the scratch sub-area
struct MlpDev {
  float* w32;                 // FP32 master weights
  float* m;                   // Adam first moment
  float* v;                   // Adam second moment
  float* gpart;               // [kTrainBlocks][nparams] partial gradients
  float* lpart;               // [kTrainBlocks][2] partial loss and weight sums
  uint16_t* pack;             // BF16 operand tiles and FP32 biases (kPackBytes)
  unsigned long long* stats;  // [kStatSlots][2]: accepted faces, judged faces
  // [kStatSlots][3]: over PE face nodes with delay >= 1, the sums of
  // max_v |ghost used - live| and max_v |AT - live|, and the node count
  double* terr;
  float* gout;                // reduced gradient (nparams)
  float* yout;                // inference outputs (kMaxBatch * V)
  float* loss;                // last loss
};

size_t mlp_scratch_bytes(int V);
MlpDev mlp_dev(const MlpState& s);
void mlp_init(MlpState& s, int V);

hipError_t launch_ghost_learned(int dim, int degree, const Mesh& M, const Async& A, const double* u_in,
                                const double* u_n, double* ring, double* ghost, int publish, const MlpState& s,
                                long long pair_base, bool collect, hipStream_t st);

}  // namespace adg
