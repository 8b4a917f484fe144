// adg_mlp.hip — learned ghost-trace predictor.
//
// The network maps, per PE-boundary face node, the K = 4 newest stored
// neighbour traces T_0..T_3 (T_0 = level n-k) and the fractional delay
// tau = k + c_m to a correction of the AT extrapolation (eq. at-flux) at that
// node. Features: the second and third backward differences of the traces,
// both divided by S = max|second| + max|third| over the variables, then
// tau/4 and the stage time c_m. The output times S is the correction (it
// estimates the live stage value minus the AT trace). The trace
// used is AT + correction when every |correction| on the face is at most the
// accept bound, and AT otherwise (AT stays the fallback and the judge).
//
// Inference: one wavefront evaluates 16 face nodes with two BF16 matrix-core
// products per 16 hidden units (v_mfma_f32_16x16x16_bf16, FP32 accumulate).
// Layer 1 is computed transposed (hidden x nodes) so that its accumulator tile
// is, lane for lane, the B operand of layer 2: no data movement between the
// layers. Training: FP32 forward/backward per sample, per-block parameter
// gradients, a deterministic cross-block reduction fused with Adam.
#include <cmath>
#include <cstring>

#include "adg_ctx.h"

namespace adg {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t mlp_scratch_bytes(int V) {
  const size_t np = (size_t)mlp_nparams(V);
  size_t s = 0;
  s = al256(s + np * 4);                         // w32
  s = al256(s + np * 4);                         // m
  s = al256(s + np * 4);                         // v
  s = al256(s + (size_t)kTrainBlocks * np * 4);  // gpart
  s = al256(s + (size_t)kTrainBlocks * 2 * 4);   // lpart
  s = al256(s + kPackBytes);                     // pack
  s = al256(s + 2 * kStatSlots * sizeof(unsigned long long));  // stats
  s = al256(s + 3 * kStatSlots * sizeof(double));              // terr
  s = al256(s + np * 4);                         // gout
  s = al256(s + (size_t)kMaxBatch * V * 4);      // yout
  s = al256(s + 4 * 4);                          // loss
  return s;
}

MlpDev mlp_dev(const MlpState& s) {
  MlpDev d{};
  const size_t np = (size_t)mlp_nparams(s.V);
  char* b = s.base;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = b + o;
    o = al256(o + bytes);
    return p;
  };
  d.w32 = reinterpret_cast<float*>(take(np * 4));
  d.m = reinterpret_cast<float*>(take(np * 4));
  d.v = reinterpret_cast<float*>(take(np * 4));
  d.gpart = reinterpret_cast<float*>(take((size_t)kTrainBlocks * np * 4));
  d.lpart = reinterpret_cast<float*>(take((size_t)kTrainBlocks * 2 * 4));
  d.pack = reinterpret_cast<uint16_t*>(take(kPackBytes));
  d.stats = reinterpret_cast<unsigned long long*>(take(2 * kStatSlots * sizeof(unsigned long long)));
  d.terr = reinterpret_cast<double*>(take(3 * kStatSlots * sizeof(double)));
  d.gout = reinterpret_cast<float*>(take(np * 4));
  d.yout = reinterpret_cast<float*>(take((size_t)kMaxBatch * s.V * 4));
  d.loss = reinterpret_cast<float*>(take(16));
  return d;
}

void mlp_init(MlpState& s, int V) {
  s.V = V;
  s.has_weights = false;
  s.device_newer = false;
  s.base = nullptr;
  std::memset(s.host_w, 0, sizeof(s.host_w));
}

// ---------------------------------------------------------------- device code

// binary32 -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

// pack area: [W1 tiles: 4 x 64 lanes x 4][W2 chunks: 4 x 64 x 4] BF16, then
// b1[64], b2[16] FP32. W1 tile t, lane l: W1[16t + l%16][4(l/16) + i];
// W2 chunk t, lane l: W2[l%16][16t + 4(l/16) + i] (zero rows o >= V).
__global__ __launch_bounds__(256) void mlp_pack_kernel(const float* __restrict__ w32, int nin, int V,
                                                       uint16_t* __restrict__ pk) {
  const float *W1 = w32, *b1 = W1 + kMlpH * nin, *W2 = b1 + kMlpH, *b2 = W2 + V * kMlpH;
  for (int idx = threadIdx.x; idx < 1024; idx += blockDim.x) {
    const int t = idx >> 8, r = idx & 255, l = r >> 2, i = r & 3;
    const int hid = 16 * t + (l & 15), in = 4 * (l >> 4) + i;
    pk[idx] = in < nin ? (uint16_t)to_bf16(W1[hid * nin + in]) : 0;
    const int o = l & 15, h2 = 16 * t + 4 * (l >> 4) + i;
    pk[1024 + idx] = o < V ? (uint16_t)to_bf16(W2[o * kMlpH + h2]) : 0;
  }
  float* fb = reinterpret_cast<float*>(pk + 2048);
  for (int h = threadIdx.x; h < kMlpH; h += blockDim.x) fb[h] = b1[h];
  for (int o = threadIdx.x; o < 16; o += blockDim.x) fb[kMlpH + o] = o < V ? b2[o] : 0.0f;
}

// Evaluate the network for the 16 nodes of one wavefront. Lane l = 16g + c
// holds features 4g..4g+3 of node c and returns outputs 4g..4g+3 of node c.
__device__ __forceinline__ f32x4 mlp_forward_wave(const uint16_t* __restrict__ pk, bf16x4 xb) {
  const int l = threadIdx.x & 63, g = l >> 4;
  const bf16x4* W1p = reinterpret_cast<const bf16x4*>(pk);
  const bf16x4* W2p = reinterpret_cast<const bf16x4*>(pk + 1024);
  const float* b1 = reinterpret_cast<const float*>(pk + 2048);
  const float* b2 = b1 + kMlpH;
  f32x4 y = {b2[4 * g], b2[4 * g + 1], b2[4 * g + 2], b2[4 * g + 3]};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 z = {b1[16 * t + 4 * g], b1[16 * t + 4 * g + 1], b1[16 * t + 4 * g + 2], b1[16 * t + 4 * g + 3]};
    z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W1p[t * 64 + l], xb, z, 0, 0, 0);
    bf16x4 h;
#pragma unroll
    for (int i = 0; i < 4; ++i) h[i] = to_bf16(gelu(z[i]));
    y = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W2p[t * 64 + l], h, y, 0, 0, 0);
  }
  return y;
}

template <int D, int P>
__device__ __forceinline__ int face_node_l(int f, int j) {
  const int a = f >> 1, s = (f & 1) ? P - 1 : 0;
  if (D == 2) return a == 0 ? s + P * j : j + P * s;
  const int j0 = j % P, j1 = j / P;
  if (a == 0) return s + P * (j0 + P * j1);
  if (a == 1) return j0 + P * (s + P * j1);
  return j0 + P * (j1 + P * s);
}

// Ghost traces with the learned correction (or, when collecting, AT ghosts
// plus training pairs). One face node per lane; a wavefront holds NFW =
// 64 / Fn whole face-sides, so the per-face judge stays inside it. The
// network runs on the matrix cores in four batches of 16 nodes, its inputs
// and outputs passing through LDS.
template <int D, int P>
__global__ __launch_bounds__(256) void ghost_learned_kernel(Mesh M, Async A, const double* __restrict__ u_in,
                                                            const double* __restrict__ u_n,
                                                            double* __restrict__ ring, double* __restrict__ ghost,
                                                            int publish, const uint16_t* __restrict__ pk,
                                                            int use_net, unsigned long long* __restrict__ stats,
                                                            double* __restrict__ terr,
                                                            float* __restrict__ pairs, long long pair_base,
                                                            int collect) {
  constexpr int V = D + 2, Fn = D == 2 ? P : P * P, Pd = Fn * P, NIN = 2 * V + 2;
  constexpr int NFW = 64 / Fn;  // face-sides per wavefront
  __shared__ float s_io[4][64][17];  // per wavefront and node: features, then outputs
  __shared__ double s_max[4][64];
  __shared__ double s_est[4][64];  // |AT4 - AT3| per node (the second judge)
  __shared__ int s_acc[4][64];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const long long fs = ((long long)blockIdx.x * 4 + w) * NFW + lane / Fn;
  const int j = lane % Fn;
  const bool valid = lane < NFW * Fn && fs < M.nfs;
  const long long total = M.nfs * V * Fn;
  int k = 0;
  double at[V], live[V], S3 = 0.0, est = 0.0;
  float x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = 0.0f;
#pragma unroll
  for (int v = 0; v < V; ++v) at[v] = live[v] = 0.0;
  if (valid) {
    int cc[3], f;
    face_side_decode(M, fs, cc, &f);
    // in a Dirichlet box the slot of a boundary face is never read: it is
    // neither published nor judged and gives no training pair
    const bool inner = !M.bc || cc[f >> 1] != ((f & 1) ? M.nc[f >> 1] - 1 : 0);
    const long long nb = neighbour(M, cc, f);
    const long long src = nb * V * Pd + face_node_l<D, P>(f ^ 1, j);
    if (publish && inner)
#pragma unroll
      for (int v = 0; v < V; ++v) ring[A.slot_n * total + (fs * V + v) * Fn + j] = u_n[src + v * Pd];
    k = inner ? delay_of(M, A, subdomain_of(M, cc), f) : 0;
#pragma unroll
    for (int v = 0; v < V; ++v) live[v] = u_in[src + v * Pd];
    if (k >= 1) {
      double T[kMlpK][V];
#pragma unroll
      for (int lv = 0; lv < kMlpK; ++lv)
#pragma unroll
        for (int v = 0; v < V; ++v) T[lv][v] = ring[ring_slot(A, k + lv) * total + (fs * V + v) * Fn + j];
      const double tau = k + A.c_m;
#pragma unroll
      for (int lv = 0; lv < kMlpK; ++lv) {  // levels <= 4 = kMlpK: fixed register indices
        if (lv < A.levels) {
          const double wl = at_weight(lv, A.levels, tau);
#pragma unroll
          for (int v = 0; v < V; ++v) at[v] += wl * T[lv][v];
        }
      }
      if (A.judge) {
        // AT over 4 levels minus AT over 3: the extrapolation's error estimate
        double d[V];
#pragma unroll
        for (int v = 0; v < V; ++v) d[v] = 0.0;
#pragma unroll
        for (int lv = 0; lv < kMlpK; ++lv) {
          const double w4 = at_weight(lv, 4, tau), w3 = lv < 3 ? at_weight(lv, 3, tau) : 0.0;
#pragma unroll
          for (int v = 0; v < V; ++v) d[v] += (w4 - w3) * T[lv][v];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) est = fabs(d[v]) > est ? fabs(d[v]) : est;
      }
      // second and third backward differences (no contraction: the features
      // are bit-reproducible), both scaled by S = max|second| + max|third|
      double d2[V], d3[V], S2 = 0.0, S3s = 0.0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        d2[v] = __dadd_rn(__dsub_rn(T[0][v], __dmul_rn(2.0, T[1][v])), T[2][v]);
        d3[v] = __dsub_rn(__dadd_rn(__dsub_rn(T[0][v], __dmul_rn(3.0, T[1][v])), __dmul_rn(3.0, T[2][v])), T[3][v]);
        S2 = fabs(d2[v]) > S2 ? fabs(d2[v]) : S2;
        S3s = fabs(d3[v]) > S3s ? fabs(d3[v]) : S3s;
      }
      const double S = __dadd_rn(__dadd_rn(S2, S3s), 1e-300);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        x[v] = (float)(d2[v] / S);
        x[V + v] = (float)(d3[v] / S);
      }
      x[2 * V] = (float)(0.25 * tau);
      x[2 * V + 1] = (float)A.c_m;
      S3 = S;
    }
  }
  float(*io)[17] = s_io[w];
#pragma unroll
  for (int q = 0; q < 16; ++q) io[lane][q] = x[q];
  __syncthreads();
  // the network on batches of 16 nodes: lane 16g + c feeds features
  // 4g..4g+3 of node 16b + c and gets back outputs 4g..4g+3 of that node,
  // stored over the same four entries it read
  {
    const int c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      bf16x4 xb;
#pragma unroll
      for (int i = 0; i < 4; ++i) xb[i] = to_bf16(io[16 * b + c][4 * g + i]);
      const f32x4 y = mlp_forward_wave(pk, xb);
#pragma unroll
      for (int i = 0; i < 4; ++i) io[16 * b + c][4 * g + i] = y[i];
    }
  }
  __syncthreads();
  double dl[V], mx = 0.0;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    dl[v] = S3 * (double)io[lane][v];
    if (!(fabs(dl[v]) <= mx)) mx = fabs(dl[v]);
  }
  s_max[w][lane] = (valid && k >= 1) ? mx : 0.0;
  s_est[w][lane] = est;
  __syncthreads();
  // per face-side judge (its first node's lane), counted per wavefront
  int acc = 0, judged = 0;
  if (valid && j == 0) {
    double mm = 0.0, me = 0.0;
#pragma unroll
    for (int q = 0; q < Fn; ++q) {
      const double v = s_max[w][lane + q];
      if (!(v <= mm)) mm = v;
      me = s_est[w][lane + q] > me ? s_est[w][lane + q] : me;
    }
    acc = use_net && (mm <= A.tol) && (!A.judge || mm <= me);
    judged = k >= 1 && use_net;
    s_acc[w][lane] = acc;
  }
  const unsigned long long mj = __ballot(judged), ma = __ballot(judged && acc);
  if (lane == 0) {
    unsigned long long* slot = stats + 2 * ((blockIdx.x * 4 + w) % kStatSlots);
    if (mj) atomicAdd(&slot[1], (unsigned long long)__popcll(mj));
    if (ma) atomicAdd(&slot[0], (unsigned long long)__popcll(ma));
  }
  __syncthreads();
  // trace errors against the live stage value (what a synchronous scheme
  // would use) at the nodes with delay >= 1: of the ghost used and of AT
  double e_used = 0.0, e_at = 0.0;
  const bool delayed = valid && k >= 1;
  if (valid) {
    const int fa = s_acc[w][lane - j];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double gv = k == 0 ? live[v] : at[v] + (fa ? dl[v] : 0.0);
      ghost[(fs * V + v) * Fn + j] = gv;
      if (delayed) {
        e_used = fmax(e_used, fabs(gv - live[v]));
        e_at = fmax(e_at, fabs(at[v] - live[v]));
      }
    }
  }
  {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      e_used += __shfl_xor(e_used, o);
      e_at += __shfl_xor(e_at, o);
    }
    const unsigned long long md = __ballot(delayed);
    if (lane == 0 && md) {
      double* slot = terr + 3 * ((blockIdx.x * 4 + w) % kStatSlots);
      atomicAdd(&slot[0], e_used);
      atomicAdd(&slot[1], e_at);
      atomicAdd(&slot[2], (double)__popcll(md));
    }
  }
  if (valid) {
    if (collect) {
      // target: live stage value minus AT, in units of S. Targets beyond
      // kTargetClip (well above the largest extrapolation coefficient the
      // delays allow) come from the neighbour's own asynchronous jumps, not
      // from the history: they get weight 0.
      float* rec = pairs + (pair_base + fs * Fn + j) * (long long)(NIN + V + 1);
      bool keep = k >= 1;
      float tg[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        tg[v] = k >= 1 ? (float)((live[v] - at[v]) / S3) : 0.0f;
        keep = keep && fabsf(tg[v]) <= kTargetClip;
      }
#pragma unroll
      for (int q = 0; q < NIN; ++q) rec[q] = x[q];
#pragma unroll
      for (int v = 0; v < V; ++v) rec[NIN + v] = keep ? tg[v] : 0.0f;
      rec[NIN + V] = keep ? 1.0f : 0.0f;
    }
  }
}

hipError_t launch_ghost_learned(int dim, int degree, const Mesh& M, const Async& A, const double* u_in,
                                const double* u_n, double* ring, double* ghost, int publish, const MlpState& s,
                                long long pair_base, bool collect, hipStream_t st) {
  const int Fn = dim == 2 ? degree + 1 : (degree + 1) * (degree + 1);
  const int nfb = 4 * (64 / Fn);  // face-sides per block
  if (M.nfs == 0) return hipSuccess;
  const unsigned nblk = (unsigned)((M.nfs + nfb - 1) / nfb);
  const MlpDev d = mlp_dev(s);
  const int use_net = s.has_weights && !collect;
#define ADG_GL_CASE(dd, p)                                                                                       \
  if (dim == dd && degree == p) {                                                                                \
    hipLaunchKernelGGL((ghost_learned_kernel<dd, p + 1>), dim3(nblk), dim3(256), 0, st, M, A, u_in, u_n, ring,   \
                       ghost, publish, d.pack, use_net, d.stats, d.terr, s.pairs, pair_base, collect ? 1 : 0);   \
    return hipGetLastError();                                                                                    \
  }
  ADG_GL_CASE(2, 1) ADG_GL_CASE(2, 2) ADG_GL_CASE(2, 3) ADG_GL_CASE(2, 4)
  ADG_GL_CASE(3, 1) ADG_GL_CASE(3, 2) ADG_GL_CASE(3, 3) ADG_GL_CASE(3, 4)
#undef ADG_GL_CASE
  return hipErrorInvalidValue;
}

// inference on stored pairs (checks of the matrix-core path)
__global__ __launch_bounds__(256) void mlp_infer_kernel(const float* __restrict__ pairs, int nin, int V,
                                                        long long first, int count, const uint16_t* __restrict__ pk,
                                                        float* __restrict__ yout) {
  const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
  const int sidx = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 + c;
  const bool valid = sidx < count;
  const float* rec = pairs + (first + (valid ? sidx : 0)) * (long long)(nin + V + 1);
  bf16x4 xb;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = 4 * g + i;
    xb[i] = to_bf16(valid && q < nin ? rec[q] : 0.0f);
  }
  const f32x4 y = mlp_forward_wave(pk, xb);
  if (valid)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * g + i < V) yout[sidx * V + 4 * g + i] = y[i];
}

// FP32 loss gradient over one block's share of a minibatch. Pair index of
// sample i of the epoch: base + (pa * i + pb) mod N (a permutation when
// gcd(pa, N) = 1). Gradients are unnormalised here (sum of w * d(residual^2)).
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ pairs, int nin, int V,
                                                       long long base, long long N, unsigned long long pa,
                                                       unsigned long long pb, long long start, int bsz,
                                                       const float* __restrict__ w32, float* __restrict__ gpart,
                                                       float* __restrict__ lpart) {
  __shared__ float s_a[kTrainChunk][kMlpH], s_dz[kTrainChunk][kMlpH], s_x[kTrainChunk][16],
      s_dy[kTrainChunk][8];
  __shared__ float s_red[2][256];
  const int np = mlp_nparams(V);
  const int tid = threadIdx.x;
  const int chunk = (bsz + gridDim.x - 1) / gridDim.x;
  const int i0 = blockIdx.x * chunk;
  int nh = bsz - i0;
  nh = nh < 0 ? 0 : (nh > chunk ? chunk : nh);
  const float *W1 = w32, *b1 = W1 + kMlpH * nin, *W2 = b1 + kMlpH, *b2 = W2 + V * kMlpH;
  float lsum = 0.0f, wsum = 0.0f;
  if (tid < kTrainChunk) {
    if (tid < nh) {
      const unsigned long long i = (unsigned long long)(start + i0 + tid);
      const long long idx = base + (long long)((pa * (i % (unsigned long long)N) + pb) % (unsigned long long)N);
      const float* rec = pairs + idx * (long long)(nin + V + 1);
      float x[16], z[kMlpH];
      for (int q = 0; q < 16; ++q) x[q] = q < nin ? rec[q] : 0.0f;
      const float wgt = rec[nin + V];
      for (int h = 0; h < kMlpH; ++h) {
        float t = b1[h];
        for (int q = 0; q < nin; ++q) t = fmaf(W1[h * nin + q], x[q], t);
        z[h] = t;
        s_a[tid][h] = gelu(t);
      }
      float dy[8];
      for (int o = 0; o < V; ++o) {
        float t = b2[o];
        for (int h = 0; h < kMlpH; ++h) t = fmaf(W2[o * kMlpH + h], s_a[tid][h], t);
        const float r = t - rec[nin + o];
        lsum += wgt * r * r;
        dy[o] = 2.0f * wgt * r;
      }
      wsum = wgt;
      for (int h = 0; h < kMlpH; ++h) {
        float dh = 0.0f;
        for (int o = 0; o < V; ++o) dh = fmaf(dy[o], W2[o * kMlpH + h], dh);
        const float zz = z[h];
        const float gd = 0.5f * (1.0f + erff(zz * 0.70710678118654752f)) +
                         zz * expf(-0.5f * zz * zz) * 0.39894228040143268f;
        s_dz[tid][h] = dh * gd;
      }
      for (int q = 0; q < 16; ++q) s_x[tid][q] = x[q];
      for (int o = 0; o < 8; ++o) s_dy[tid][o] = o < V ? dy[o] : 0.0f;
    }
  }
  __syncthreads();
  for (int p = tid; p < np; p += blockDim.x) {
    float acc = 0.0f;
    if (p < kMlpH * nin) {
      const int h = p / nin, q = p - h * nin;
      for (int s = 0; s < nh; ++s) acc = fmaf(s_dz[s][h], s_x[s][q], acc);
    } else if (p < kMlpH * nin + kMlpH) {
      const int h = p - kMlpH * nin;
      for (int s = 0; s < nh; ++s) acc += s_dz[s][h];
    } else if (p < kMlpH * nin + kMlpH + V * kMlpH) {
      const int r = p - kMlpH * nin - kMlpH, o = r / kMlpH, h = r - o * kMlpH;
      for (int s = 0; s < nh; ++s) acc = fmaf(s_dy[s][o], s_a[s][h], acc);
    } else {
      const int o = p - kMlpH * nin - kMlpH - V * kMlpH;
      for (int s = 0; s < nh; ++s) acc += s_dy[s][o];
    }
    gpart[(long long)blockIdx.x * np + p] = acc;
  }
  s_red[0][tid] = lsum;
  s_red[1][tid] = wsum;
  __syncthreads();
  for (int sft = 128; sft > 0; sft >>= 1) {
    if (tid < sft) {
      s_red[0][tid] += s_red[0][tid + sft];
      s_red[1][tid] += s_red[1][tid + sft];
    }
    __syncthreads();
  }
  if (tid == 0) {
    lpart[blockIdx.x * 2] = s_red[0][0];
    lpart[blockIdx.x * 2 + 1] = s_red[1][0];
  }
}

// normalised gradient (and optionally an Adam step): g = sum_b gpart / (V W)
__global__ __launch_bounds__(256) void mlp_reduce_adam_kernel(const float* __restrict__ gpart,
                                                              const float* __restrict__ lpart, int nblk, int np,
                                                              int V, float* __restrict__ w32, float* __restrict__ m,
                                                              float* __restrict__ vv, float* __restrict__ gout,
                                                              float* __restrict__ loss, int adam, float lr, float b1,
                                                              float b2, float eps, float c1, float c2) {
  float W = 0.0f, Ls = 0.0f;
  for (int b = 0; b < nblk; ++b) {
    Ls += lpart[2 * b];
    W += lpart[2 * b + 1];
  }
  const float inv = W > 0.0f ? 1.0f / ((float)V * W) : 0.0f;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) loss[0] = Ls * inv;
  if (p >= np) return;
  float g = 0.0f;
  for (int b = 0; b < nblk; ++b) g += gpart[(long long)b * np + p];
  g *= inv;
  if (gout) gout[p] = g;
  if (adam) {
    const float mi = b1 * m[p] + (1.0f - b1) * g;
    const float vi = b2 * vv[p] + (1.0f - b2) * g * g;
    m[p] = mi;
    vv[p] = vi;
    w32[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void mlp_zero_kernel(unsigned long long* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0ull;
}

__global__ void mlp_zero_f_kernel(float* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

}  // namespace adg

using namespace adg;

// ------------------------------------------------------------- host helpers

namespace adg {

void mlp_reset_stats(adg_ctx_s* c) {
  if (!c->bound) return;
  const MlpDev d = mlp_dev(c->mlp);
  hipLaunchKernelGGL(mlp_zero_kernel, dim3((2 * kStatSlots + 63) / 64), dim3(64), 0, c->stream, d.stats,
                     2 * kStatSlots);
  // the all-zero bit pattern is 0.0
  hipLaunchKernelGGL(mlp_zero_kernel, dim3((3 * kStatSlots + 63) / 64), dim3(64), 0, c->stream,
                     reinterpret_cast<unsigned long long*>(d.terr), 3 * kStatSlots);
}

// upload host_w as the master weights, repack, zero Adam state
adg_status mlp_upload(adg_ctx_s* c) {
  const MlpDev d = mlp_dev(c->mlp);
  const int np = mlp_nparams(c->V);
  HIP_TRY(hipMemcpyAsync(d.w32, c->mlp.host_w, sizeof(float) * np, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(mlp_zero_f_kernel, dim3((np + 255) / 256), dim3(256), 0, c->stream, d.m, np);
  hipLaunchKernelGGL(mlp_zero_f_kernel, dim3((np + 255) / 256), dim3(256), 0, c->stream, d.v, np);
  hipLaunchKernelGGL(mlp_pack_kernel, dim3(1), dim3(256), 0, c->stream, d.w32, mlp_nin(c->V), c->V, d.pack);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->mlp.adam_t = 0;
  c->mlp.device_newer = false;
  return ADG_OK;
}

adg_status mlp_on_bind(adg_ctx_s* c) {
  mlp_reset_stats(c);
  if (c->mlp.has_weights) return mlp_upload(c);
  return ADG_OK;
}

void mlp_get_host(adg_ctx_s* c, float* w) {
  if (c->mlp.device_newer && c->bound) {
    const MlpDev d = mlp_dev(c->mlp);
    if (hipMemcpyAsync(c->mlp.host_w, d.w32, sizeof(float) * mlp_nparams(c->V), hipMemcpyDeviceToHost,
                       c->stream) == hipSuccess &&
        hipStreamSynchronize(c->stream) == hipSuccess)
      c->mlp.device_newer = false;
  }
  std::memcpy(w, c->mlp.host_w, sizeof(float) * mlp_nparams(c->V));
}

adg_status mlp_set_host(adg_ctx_s* c, const float* w) {
  std::memcpy(c->mlp.host_w, w, sizeof(float) * mlp_nparams(c->V));
  c->mlp.has_weights = true;
  if (c->bound) return mlp_upload(c);
  return ADG_OK;
}

}  // namespace adg

extern "C" {

adg_status adg_predictor_nparams(adg_ctx c, int32_t* nparams) {
  if (!c || !nparams) return fail(ADG_ERR_INVALID, "null argument");
  *nparams = mlp_nparams(c->V);
  return ADG_OK;
}

adg_status adg_predictor_pair_bytes(adg_ctx c, size_t* bytes) {
  if (!c || !bytes) return fail(ADG_ERR_INVALID, "null argument");
  *bytes = sizeof(float) * mlp_pair_floats(c->V);
  return ADG_OK;
}

adg_status adg_predictor_bind(adg_ctx c, void* pairs, int64_t max_pairs) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (max_pairs < 0 || max_pairs >= (1ll << 31) || (max_pairs > 0 && !pairs))
    return fail(ADG_ERR_INVALID, "bad pair buffer (0 <= max_pairs < 2^31)");
  c->mlp.pairs = static_cast<float*>(pairs);
  c->mlp.max_pairs = max_pairs;
  c->mlp.n_pairs = 0;
  return ADG_OK;
}

adg_status adg_predictor_load_pairs(adg_ctx c, const float* host_pairs, int64_t n) {
  if (!c || (n > 0 && !host_pairs)) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (n < 0 || n > c->mlp.max_pairs) return fail(ADG_ERR_INVALID, "more pairs than the bound buffer holds");
  const size_t rb = sizeof(float) * mlp_pair_floats(c->V);
  if (n) HIP_TRY(hipMemcpyAsync(c->mlp.pairs, host_pairs, rb * n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->mlp.n_pairs = n;
  return ADG_OK;
}

adg_status adg_predictor_init(adg_ctx c, uint64_t seed) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  // Glorot/Xavier uniform (Glorot & Bengio 2010), biases zero; uniforms from
  // SplitMix64 draws of the seed
  const int V = c->V, nin = mlp_nin(V), np = mlp_nparams(V);
  float* w = c->mlp.host_w;
  std::memset(w, 0, sizeof(float) * np);
  const double a1 = std::sqrt(6.0 / (nin + kMlpH)), a2 = std::sqrt(6.0 / (kMlpH + V));
  unsigned long long idx = 0;
  auto uni = [&]() { return (double)(splitmix64(seed, idx++) >> 11) * (1.0 / 9007199254740992.0); };
  for (int i = 0; i < kMlpH * nin; ++i) w[i] = (float)((2.0 * uni() - 1.0) * a1);
  float* W2 = w + kMlpH * nin + kMlpH;
  for (int i = 0; i < V * kMlpH; ++i) W2[i] = (float)((2.0 * uni() - 1.0) * a2);
  return mlp_set_host(c, w);
}

adg_status adg_predictor_collect(adg_ctx c, int64_t n_steps, double dt, int64_t* n_pairs) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (c->as.ghost != ADG_GHOST_LEARNED)
    return fail(ADG_ERR_STATE, "collection needs the LEARNED ghost mode (its ring keeps the 4 levels)");
  if (!c->mlp.pairs) return fail(ADG_ERR_UNBOUND, "no pair buffer (adg_predictor_bind)");
  adg_status s = adg_step_impl(c, n_steps, dt, true);
  if (n_pairs) *n_pairs = c->mlp.n_pairs;
  return s;
}

static adg_status run_grad(adg_ctx c, long long base, long long N, unsigned long long pa, unsigned long long pb,
                           long long start, int bsz, int adam, float lr) {
  const MlpDev d = mlp_dev(c->mlp);
  const int V = c->V, nin = mlp_nin(V), np = mlp_nparams(V);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(kTrainBlocks), dim3(256), 0, c->stream, c->mlp.pairs, nin, V, base, N,
                     pa, pb, start, bsz, d.w32, d.gpart, d.lpart);
  float c1 = 1.0f, c2 = 1.0f;
  if (adam) {
    c->mlp.adam_t += 1;
    c1 = (float)(1.0 - std::pow(0.9, (double)c->mlp.adam_t));
    c2 = (float)(1.0 - std::pow(0.999, (double)c->mlp.adam_t));
  }
  hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((np + 255) / 256), dim3(256), 0, c->stream, d.gpart, d.lpart,
                     kTrainBlocks, np, V, d.w32, d.m, d.v, adam ? nullptr : d.gout, d.loss, adam, lr, 0.9f, 0.999f,
                     1e-8f, c1, c2);
  HIP_TRY(hipGetLastError());
  return ADG_OK;
}

static unsigned long long gcd_u(unsigned long long a, unsigned long long b) {
  while (b) {
    const unsigned long long t = a % b;
    a = b;
    b = t;
  }
  return a;
}

adg_status adg_predictor_train(adg_ctx c, int32_t epochs, int32_t batch, float lr, uint64_t seed, float* loss_out) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (epochs < 1 || batch < 1 || batch > kMaxBatch || !(lr > 0.0f))
    return fail(ADG_ERR_INVALID, "need epochs >= 1, 1 <= batch <= 4096, lr > 0");
  const long long N = c->mlp.n_pairs;
  if (N < 1) return fail(ADG_ERR_STATE, "no training pairs");
  if (!c->mlp.has_weights) {
    adg_status s = adg_predictor_init(c, seed);
    if (s != ADG_OK) return s;
  }
  unsigned long long idx = 1000;
  for (int ep = 0; ep < epochs; ++ep) {
    unsigned long long pa = N > 1 ? (splitmix64(seed, idx++) % (unsigned long long)N) : 1ull;
    while (N > 1 && (pa == 0 || gcd_u(pa, (unsigned long long)N) != 1)) pa = (pa + 1) % (unsigned long long)N;
    const unsigned long long pb = splitmix64(seed, idx++) % (unsigned long long)N;
    for (long long st = 0; st < N; st += batch) {
      const int bs = (int)std::min<long long>(batch, N - st);
      adg_status s = run_grad(c, 0, N, pa, pb, st, bs, 1, lr);
      if (s != ADG_OK) return s;
    }
  }
  const MlpDev d = mlp_dev(c->mlp);
  hipLaunchKernelGGL(mlp_pack_kernel, dim3(1), dim3(256), 0, c->stream, d.w32, mlp_nin(c->V), c->V, d.pack);
  float loss = 0.0f;
  HIP_TRY(hipMemcpyAsync(&loss, d.loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->mlp.device_newer = true;
  c->mlp.has_weights = true;
  if (loss_out) *loss_out = loss;
  return ADG_OK;
}

adg_status adg_predictor_grad(adg_ctx c, int64_t first, int64_t count, float* grad, float* loss_out) {
  if (!c || !grad) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (count < 1 || count > kMaxBatch || first < 0 || first + count > c->mlp.n_pairs)
    return fail(ADG_ERR_INVALID, "pair range out of bounds (count <= 4096)");
  if (!c->mlp.has_weights) return fail(ADG_ERR_STATE, "no weights set");
  adg_status s = run_grad(c, first, count, 1ull, 0ull, 0, (int)count, 0, 0.0f);
  if (s != ADG_OK) return s;
  const MlpDev d = mlp_dev(c->mlp);
  float loss = 0.0f;
  HIP_TRY(hipMemcpyAsync(grad, d.gout, sizeof(float) * mlp_nparams(c->V), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&loss, d.loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (loss_out) *loss_out = loss;
  return ADG_OK;
}

adg_status adg_predictor_infer(adg_ctx c, int64_t first, int64_t count, float* y) {
  if (!c || !y) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (count < 1 || count > kMaxBatch || first < 0 || first + count > c->mlp.n_pairs)
    return fail(ADG_ERR_INVALID, "pair range out of bounds (count <= 4096)");
  if (!c->mlp.has_weights) return fail(ADG_ERR_STATE, "no weights set");
  const MlpDev d = mlp_dev(c->mlp);
  const unsigned nblk = (unsigned)((count + 63) / 64);
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(nblk), dim3(256), 0, c->stream, c->mlp.pairs, mlp_nin(c->V), c->V,
                     (long long)first, (int)count, d.pack, d.yout);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(y, d.yout, sizeof(float) * c->V * count, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ADG_OK;
}

adg_status adg_predictor_get(adg_ctx c, float* w) {
  if (!c || !w) return fail(ADG_ERR_INVALID, "null argument");
  mlp_get_host(c, w);
  return ADG_OK;
}

adg_status adg_predictor_set(adg_ctx c, const float* w) {
  if (!c || !w) return fail(ADG_ERR_INVALID, "null argument");
  return mlp_set_host(c, w);
}

adg_status adg_predictor_stats(adg_ctx c, double* accept_rate, int64_t* faces_judged, double* mean_trace_err,
                               double* mean_at_err) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  unsigned long long h[2] = {0, 0};
  double te[3] = {0.0, 0.0, 0.0};
  if (c->bound) {
    const MlpDev d = mlp_dev(c->mlp);
    unsigned long long slots[2 * kStatSlots];
    double ts[3 * kStatSlots];
    HIP_TRY(hipMemcpyAsync(slots, d.stats, sizeof(slots), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(ts, d.terr, sizeof(ts), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int i = 0; i < kStatSlots; ++i) {
      h[0] += slots[2 * i];
      h[1] += slots[2 * i + 1];
      for (int q = 0; q < 3; ++q) te[q] += ts[3 * i + q];
    }
  }
  if (accept_rate) *accept_rate = h[1] ? (double)h[0] / (double)h[1] : 0.0;
  if (faces_judged) *faces_judged = (int64_t)h[1];
  if (mean_trace_err) *mean_trace_err = te[2] > 0 ? te[0] / te[2] : 0.0;
  if (mean_at_err) *mean_at_err = te[2] > 0 ? te[1] / te[2] : 0.0;
  return ADG_OK;
}

}  // extern "C"
