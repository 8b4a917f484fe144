// adg_ghost.hip — ring publish and ghost traces at PE-boundary face-sides.
//
// One thread per (face-side, variable, face node). At stage 0 of step n the
// neighbour's step-start trace is published into ring slot n mod R. The
// trace the receiving element then uses is, depending on its delay k for
// this step (Sec. 3, eq. euler-adg-compact): the neighbour's live stage value
// (k = 0), the trace k steps old (standard flux on delayed data, eq.
// delayed-flux), or the AT extrapolation of `levels` consecutive stored
// levels (eq. at-flux) with weights solving eq. at-flux-constraints at the
// stage-fractional delay tau = k + c_m (naive RK coupling, Sec. 3.2).
#include "adg_internal.h"

namespace adg {

template <int D, int P>
__device__ __forceinline__ int ghost_face_node(int f, int j) {
  const int a = f >> 1, s = (f & 1) ? P - 1 : 0;
  if (D == 2) return a == 0 ? s + P * j : j + P * s;
  const int j0 = j % P, j1 = j / P;
  if (a == 0) return s + P * (j0 + P * j1);
  if (a == 1) return j0 + P * (s + P * j1);
  return j0 + P * (j1 + P * s);
}

// AT weight of level j among nlev at fractional delay tau: Lagrange
// extrapolation to offset 0 from the level times -(tau + i)
__device__ __forceinline__ double at_weight(int j, int nlev, double tau) {
  double w = 1.0;
  for (int i = 0; i < nlev; ++i)
    if (i != j) w *= (tau + i) / (double)(i - j);
  return w;
}

template <int D, int P>
__global__ __launch_bounds__(256) void ghost_kernel(Mesh M, Async A, const double* __restrict__ u_in,
                                                    const double* __restrict__ u_n, double* __restrict__ ring,
                                                    double* __restrict__ ghost, int publish) {
  constexpr int V = D + 2, Fn = D == 2 ? P : P * P, Pd = Fn * P;
  const long long total = M.nfs * V * Fn;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int j = (int)(i % Fn);
  const long long r = i / Fn;
  const int v = (int)(r % V);
  const long long fs = r / V;
  int c[3], f;
  face_side_decode(M, fs, c, &f);
  const long long nb = neighbour(M, c, f);
  const long long src = (nb * V + v) * Pd + ghost_face_node<D, P>(f ^ 1, j);
  if (publish) ring[(A.n % A.R) * total + i] = u_n[src];
  const int k = delay_of(M, A, subdomain_of(M, c), f);
  double g;
  if (k == 0) {
    g = u_in[src];
  } else if (A.ghost == 1) {
    g = ring[((A.n - k) % A.R) * total + i];
  } else {
    const double tau = k + A.c_m;
    g = 0.0;
    for (int l = 0; l < A.levels; ++l) g += at_weight(l, A.levels, tau) * ring[((A.n - k - l) % A.R) * total + i];
  }
  ghost[i] = g;
}

hipError_t launch_ghost(int dim, int degree, const Mesh& M, const Async& A, const double* u_in, const double* u_n,
                        double* ring, double* ghost, const float* mlp, int publish, double* stats,
                        hipStream_t st) {
  (void)mlp;
  (void)stats;
  const int V = dim + 2;
  long long Fn = 1;
  for (int k = 0; k < dim - 1; ++k) Fn *= degree + 1;
  const long long total = M.nfs * V * Fn;
  if (total == 0) return hipSuccess;
  const unsigned nblk = (unsigned)((total + 255) / 256);
#define ADG_GH_CASE(d, p)                                                                                  \
  if (dim == d && degree == p) {                                                                           \
    hipLaunchKernelGGL((ghost_kernel<d, p + 1>), dim3(nblk), dim3(256), 0, st, M, A, u_in, u_n, ring, ghost, \
                       publish);                                                                           \
    return hipGetLastError();                                                                              \
  }
  ADG_GH_CASE(2, 1) ADG_GH_CASE(2, 2) ADG_GH_CASE(2, 3) ADG_GH_CASE(2, 4)
  ADG_GH_CASE(3, 1) ADG_GH_CASE(3, 2) ADG_GH_CASE(3, 3) ADG_GH_CASE(3, 4)
#undef ADG_GH_CASE
  return hipErrorInvalidValue;
}

}  // namespace adg
