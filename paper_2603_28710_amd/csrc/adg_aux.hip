// adg_aux.hip — gfx950 kernels outside the time-step hot loop: L2 projection
// of the analytic problems, error norms, integrals, relative differences,
// state checks, the wave-speed maximum, a deterministic reduction, and the
// exterior states of a Dirichlet box's boundary faces (one small launch per
// stage, before the stage kernel).
#include "adg_internal.h"

namespace adg {

namespace {

constexpr double kPi = 3.14159265358979323846;

// exact solutions (Sec. 5.1 vortex with mean flow (mu, mv): the nearest
// periodic image in a periodic box, the vortex itself in a Dirichlet box;
// density wave; constant state), conserved variables
template <int D>
__device__ void exact_state(int problem, const double* prm, const double* x, double t, double gamma,
                            const Mesh& M, double* w) {
  if (problem == 0) {
    const double x0 = prm[0], y0 = prm[1], beta = prm[2], mu = prm[3], mv = prm[4];
    const double Lx = M.hi[0] - M.lo[0], Ly = M.hi[1] - M.lo[1];
    double dx = x[0] - x0 - mu * t, dy = x[1] - y0 - mv * t;
    if (!M.bc) {
      dx -= Lx * floor(dx / Lx + 0.5);
      dy -= Ly * floor(dy / Ly + 0.5);
    }
    const double g = exp(1.0 - (dx * dx + dy * dy));
    const double u = mu - beta * g * dy / (2.0 * kPi);
    const double v = mv + beta * g * dx / (2.0 * kPi);
    const double rho = pow(1.0 - (gamma - 1.0) * beta * beta * g * g / (16.0 * gamma * kPi * kPi), 1.0 / (gamma - 1.0));
    const double p = pow(rho, gamma);
    w[0] = rho;
    w[1] = rho * u;
    w[2] = rho * v;
    if (D == 3) w[3] = 0.0;
    w[D + 1] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v);
  } else if (problem == 1) {
    double s = 0.0, u2 = 0.0;
    for (int k = 0; k < D; ++k) {
      s += x[k] - prm[1 + k] * t;
      u2 += prm[1 + k] * prm[1 + k];
    }
    const double rho = 1.0 + prm[0] * sin(2.0 * kPi * s);
    w[0] = rho;
    for (int k = 0; k < D; ++k) w[1 + k] = rho * prm[1 + k];
    w[D + 1] = prm[4] / (gamma - 1.0) + 0.5 * rho * u2;
  } else {
    double u2 = 0.0;
    w[0] = prm[0];
    for (int k = 0; k < D; ++k) {
      w[1 + k] = prm[0] * prm[1 + k];
      u2 += prm[1 + k] * prm[1 + k];
    }
    w[D + 1] = prm[4] / (gamma - 1.0) + 0.5 * prm[0] * u2;
  }
}

template <int D, int P, int Q>
struct AuxDims {
  static constexpr int V = D + 2;
  static constexpr int Pd = D == 2 ? P * P : P * P * P;
  static constexpr int Qd = D == 2 ? Q * Q : Q * Q * Q;
};

// apply the 1D operator A (NO x NI) along axis ax to one element's V tensors
// of extents ext (updated); plain loops, thread per output value
template <int D>
__device__ void aux_sweep(const double* in, double* out, const double* A, int NI, int NO, int ax, int* ext,
                          int nvec) {
  int o[3] = {ext[0], ext[1], ext[2]};
  o[ax] = NO;
  const int isz = ext[0] * ext[1] * ext[2], osz = o[0] * o[1] * o[2];
  const int istr = ax == 0 ? 1 : (ax == 1 ? ext[0] : ext[0] * ext[1]);
  for (int t = threadIdx.x; t < nvec * osz; t += blockDim.x) {
    const int v = t / osz, r = t - v * osz;
    int c[3] = {r % o[0], (r / o[0]) % o[1], r / (o[0] * o[1])};
    const int oc = c[ax];
    c[ax] = 0;
    const int base = c[0] + ext[0] * (c[1] + ext[1] * c[2]);
    double acc = 0.0;
    for (int i = 0; i < NI; ++i) acc = fma(A[oc * NI + i], in[v * isz + base + i * istr], acc);
    out[v * osz + r] = acc;
  }
  ext[ax] = NO;
}

template <int D, int P, int Q>
__global__ __launch_bounds__(kThreads) void init_kernel(Mesh M, int problem, Prm prm,
                                                   double* __restrict__ u, const double* __restrict__ tab) {
  using Dm = AuxDims<D, P, Q>;
  constexpr int V = Dm::V, Pd = Dm::Pd, Qd = Dm::Qd;
  constexpr TabOff to = tab_off(P, Q);
  __shared__ double sA[V * Qd], sB[V * Qd];
  const long long e = blockIdx.x;
  int c[3];
  elem_coords(M, e, c);
  for (int q = threadIdx.x; q < Qd; q += blockDim.x) {
    const int qi[3] = {q % Q, (q / Q) % Q, q / (Q * Q)};
    double x[3] = {0, 0, 0}, w[kMaxV], wt = 1.0;
    for (int k = 0; k < D; ++k) {
      x[k] = M.lo[k] + M.h[k] * (c[k] + 0.5 * (tab[to.XQ + qi[k]] + 1.0));
      wt *= tab[to.WQ + qi[k]];
    }
    exact_state<D>(problem, prm.v, x, 0.0, M.gamma, M, w);
    for (int v = 0; v < V; ++v) sA[v * Qd + q] = wt * w[v];
  }
  __syncthreads();
  int ext[3] = {Q, Q, D == 3 ? Q : 1};
  double *in = sA, *out = sB;
  for (int ax = 0; ax < D; ++ax) {  // (phi_i, w) = B^T-sweeps of w_q w(x_q)
    aux_sweep<D>(in, out, tab + to.BT, Q, P, ax, ext, V);
    __syncthreads();
    double* t = in;
    in = out;
    out = t;
  }
  for (int ax = 0; ax < D; ++ax) {  // M1^{-1} sweeps (|J| cancels)
    aux_sweep<D>(in, out, tab + to.MI, P, P, ax, ext, V);
    __syncthreads();
    double* t = in;
    in = out;
    out = t;
  }
  for (int i = threadIdx.x; i < V * Pd; i += blockDim.x) u[e * V * Pd + i] = in[i];
}

// what: 0 error vs exact (3 comps), 1 integrals (V), 2 diff vs ref (6),
//       3 check: non-finite, non-physical counts (2), 4 max wave speed (1)
template <int D, int P, int Q>
__global__ __launch_bounds__(kThreads) void norms_kernel(Mesh M, int what, int problem, Prm prm,
                                                    double t, const double* __restrict__ u,
                                                    const double* __restrict__ ref, const double* __restrict__ tab,
                                                    double* __restrict__ partial) {
  using Dm = AuxDims<D, P, Q>;
  constexpr int V = Dm::V, Pd = Dm::Pd, Qd = Dm::Qd;
  constexpr TabOff to = tab_off(P, Q);
  __shared__ double sA[V * Qd], sB[V * Qd];
  __shared__ double red[kThreads * 6];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const double gamma = M.gamma;
  for (long long e = blockIdx.x; e < M.E; e += gridDim.x) {
    const double* ue = u + e * V * Pd;
    if (what == 0 || what == 1) {
      for (int i = threadIdx.x; i < V * Pd; i += blockDim.x) sA[i] = ue[i];
      __syncthreads();
      int ext[3] = {P, P, D == 3 ? P : 1};
      double *in = sA, *out = sB;
      for (int ax = 0; ax < D; ++ax) {
        aux_sweep<D>(in, out, tab + to.B, P, Q, ax, ext, V);
        __syncthreads();
        double* tt = in;
        in = out;
        out = tt;
      }
      int c[3];
      elem_coords(M, e, c);
      for (int q = threadIdx.x; q < Qd; q += blockDim.x) {
        const int qi[3] = {q % Q, (q / Q) % Q, q / (Q * Q)};
        double x[3] = {0, 0, 0}, wt = M.detJ;
        for (int k = 0; k < D; ++k) {
          x[k] = M.lo[k] + M.h[k] * (c[k] + 0.5 * (tab[to.XQ + qi[k]] + 1.0));
          wt *= tab[to.WQ + qi[k]];
        }
        if (what == 1) {
          for (int v = 0; v < V; ++v) acc[v] += wt * in[v * Qd + q];
        } else {
          double w[kMaxV];
          exact_state<D>(problem, prm.v, x, t, gamma, M, w);
          double d0 = in[q] - w[0];
          acc[0] += wt * d0 * d0;
          for (int k = 0; k < D; ++k) {
            const double d = in[(1 + k) * Qd + q] - w[1 + k];
            acc[1] += wt * d * d;
          }
          const double dE = in[(D + 1) * Qd + q] - w[D + 1];
          acc[2] += wt * dE * dE;
        }
      }
      __syncthreads();
    } else {
      for (int i = threadIdx.x; i < Pd; i += blockDim.x) {
        double w[kMaxV];
        for (int v = 0; v < V; ++v) w[v] = ue[v * Pd + i];
        if (what == 2) {
          const double* re = ref + e * V * Pd;
          for (int v = 0; v < V; ++v) {
            const int g = v == 0 ? 0 : (v == D + 1 ? 2 : 1);
            const double d = w[v] - re[v * Pd + i];
            acc[g] += d * d;
            acc[3 + g] += re[v * Pd + i] * re[v * Pd + i];
          }
        } else {
          double m2 = 0.0;
          for (int k = 0; k < D; ++k) m2 += w[1 + k] * w[1 + k];
          const double p = (gamma - 1.0) * (w[D + 1] - 0.5 * m2 / w[0]);
          bool fin = true;
          for (int v = 0; v < V; ++v) fin = fin && isfinite(w[v]);
          if (what == 3) {
            acc[0] += fin ? 0.0 : 1.0;
            acc[1] += (fin && (w[0] > 0.0 && p > 0.0)) ? 0.0 : (fin ? 1.0 : 0.0);
          } else if (fin && w[0] > 0.0 && p > 0.0) {
            const double s = sqrt(m2) / w[0] + sqrt(gamma * p / w[0]);
            acc[0] = s > acc[0] ? s : acc[0];
          }
        }
      }
    }
  }
  // fixed-order tree reduction inside the block
  const int nc = 6;
  for (int k = 0; k < nc; ++k) red[k * kThreads + threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < nc; ++k) {
        const double a = red[k * kThreads + threadIdx.x], b = red[k * kThreads + threadIdx.x + s];
        red[k * kThreads + threadIdx.x] = what == 4 ? (a > b ? a : b) : a + b;
      }
    __syncthreads();
  }
  if (threadIdx.x < nc) partial[blockIdx.x * nc + threadIdx.x] = red[threadIdx.x * kThreads];
}

__global__ __launch_bounds__(kThreads) void reduce_kernel(const double* __restrict__ partial, int nblk, int ncomp, int op,
                                                     double* __restrict__ out) {
  __shared__ double red[kThreads];
  for (int k = 0; k < ncomp; ++k) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) {
      const double x = partial[b * 6 + k];
      a = op ? (x > a ? x : a) : a + x;
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        const double x = red[threadIdx.x], y = red[threadIdx.x + s];
        red[threadIdx.x] = op ? (x > y ? x : y) : x + y;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = red[0];
    __syncthreads();
  }
}

// one thread per (stage, boundary face, face node) of a Dirichlet box
// (d = 2): the exact state at the node at the stage's time, written as
// bnd[stage][face][v][j]. Face node j sits at the j-th Gauss-Lobatto node of
// the tangential axis, ascending, as the stage kernel orders a neighbour's
// face trace.
template <int P>
__global__ __launch_bounds__(kThreads) void bnd_fill_kernel(Mesh M, int problem, Prm prm, StageTimes T,
                                                       const double* __restrict__ tab, double* __restrict__ bnd) {
  constexpr int V = 4;
  constexpr TabOff to = tab_off(P, P + 1);
  const int per = M.nbf * P;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= T.n * per) return;
  const int m = i / per, r = i - m * per;
  const int bf = r / P, j = r - bf * P;
  const double t = T.t[m];
  bnd += (long long)m * M.nbf * V * P;
  int f = 0;
  for (int g = 1; g < 4; ++g)
    if (bf >= M.bnd_off[g]) f = g;
  const int a = f >> 1, b = a ^ 1, ct = bf - M.bnd_off[f];
  double x[3] = {0.0, 0.0, 0.0}, w[kMaxV];
  x[a] = (f & 1) ? M.hi[a] : M.lo[a];
  x[b] = M.lo[b] + M.h[b] * (ct + 0.5 * (tab[to.XL + j] + 1.0));
  exact_state<2>(problem, prm.v, x, t, M.gamma, M, w);
  for (int v = 0; v < V; ++v) bnd[(bf * V + v) * P + j] = w[v];
}

}  // namespace

int norms_blocks(long long E) { return (int)(E < 2048 ? E : 2048); }

hipError_t launch_init(int dim, int degree, const Mesh& M, int problem, const Prm& prm, double* u,
                       const double* tab64, hipStream_t st) {
#define ADG_INIT_CASE(d, p)                                                                                    \
  if (dim == d && degree == p) {                                                                               \
    hipLaunchKernelGGL((init_kernel<d, p + 1, p + 2>), dim3((unsigned)M.E), dim3(kThreads), 0, st, M, problem, \
                       prm, u, tab64);                                                                         \
    return hipGetLastError();                                                                                  \
  }
  ADG_INIT_CASE(2, 1) ADG_INIT_CASE(2, 2) ADG_INIT_CASE(2, 3) ADG_INIT_CASE(2, 4)
  ADG_INIT_CASE(3, 1) ADG_INIT_CASE(3, 2) ADG_INIT_CASE(3, 3) ADG_INIT_CASE(3, 4)
#undef ADG_INIT_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_norms(int dim, int degree, const Mesh& M, int what, int problem, const Prm& prm, double t,
                        const double* u, const double* ref, const double* tab64, double* partial, int nblk,
                        hipStream_t st) {
#define ADG_NORM_CASE(d, p)                                                                                 \
  if (dim == d && degree == p) {                                                                            \
    hipLaunchKernelGGL((norms_kernel<d, p + 1, p + 2>), dim3(nblk), dim3(kThreads), 0, st, M, what, problem, \
                       prm, t, u, ref, tab64, partial);                                                     \
    return hipGetLastError();                                                                               \
  }
  ADG_NORM_CASE(2, 1) ADG_NORM_CASE(2, 2) ADG_NORM_CASE(2, 3) ADG_NORM_CASE(2, 4)
  ADG_NORM_CASE(3, 1) ADG_NORM_CASE(3, 2) ADG_NORM_CASE(3, 3) ADG_NORM_CASE(3, 4)
#undef ADG_NORM_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const double* partial, int nblk, int ncomp, int op, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, st, partial, nblk, ncomp, op, out);
  return hipGetLastError();
}

hipError_t launch_bnd_fill(int degree, const Mesh& M, int problem, const Prm& prm, const StageTimes& t,
                           const double* tab64, double* bnd, hipStream_t st) {
  if (M.dim != 2 || !M.bc || M.nbf <= 0 || t.n < 1 || t.n > 3) return hipErrorInvalidValue;
  const unsigned nblk = (unsigned)((t.n * M.nbf * (degree + 1) + kThreads - 1) / kThreads);
#define ADG_BND_CASE(p)                                                                                   \
  if (degree == p) {                                                                                      \
    hipLaunchKernelGGL((bnd_fill_kernel<p + 1>), dim3(nblk), dim3(kThreads), 0, st, M, problem, prm, t, tab64, \
                       bnd);                                                                              \
    return hipGetLastError();                                                                             \
  }
  ADG_BND_CASE(1) ADG_BND_CASE(2) ADG_BND_CASE(3) ADG_BND_CASE(4)
#undef ADG_BND_CASE
  return hipErrorInvalidValue;
}

}  // namespace adg
