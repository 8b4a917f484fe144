// adg_rhs.hip — gfx950 kernels of one SSP-RK3 stage of the ADG right-hand side.
//
// rhs_stage: one workgroup owns NE consecutive elements (x fastest) and does,
// entirely in LDS/registers,
//   1. interpolation of the stage input from the P^d Gauss-Lobatto nodes to the
//      Q^d Gauss points, d sum-factorised sweeps (Sec. 2.1, eq. weakform-dealii);
//   2. the Euler flux at every Gauss point, scaled by w_q |J| 2/h_a, tested
//      against grad phi with a collocation derivative sweep per direction
//      followed by d transposed interpolation sweeps (volume term);
//   3. the numerical flux of eq. lfflux at the Q^(d-1) Gauss points of each
//      face from the element's own face nodes and the neighbour's face nodes
//      (live, or the ghost trace at PE-boundary faces), lifted back to the
//      face nodes (surface term; only face nodes see it with Gauss-Lobatto
//      nodes);
//   4. the inverse mass matrix M_e^{-1} = |J|^{-1} (M1^{-1} (x) ... (x) M1^{-1})
//      as d sweeps (eq. weakform-compact-dealii);
//   5. the Shu-Osher SSP-RK3 combine out = a u_n + b (u_in + dt k), in FP64.
// T = double (FP64 path) or float (FP32-contraction path: steps 1-4 in FP32).
//
// Interior faces are evaluated by both neighbours with one instruction
// stream on identical operands in a canonical (left, right) order, so the two
// sides receive bitwise opposite fluxes and the synchronous scheme conserves
// to summation round-off.
//
// ghost: per PE-boundary face-side node, publishes the neighbour's step-start
// trace into the ring (stage 0) and builds the trace the receiving element
// uses: live, delayed (standard flux), or the AT extrapolation of eq. at-flux
// with weights from eq. at-flux-constraints at tau = k + c_m.
#include "adg_internal.h"

namespace adg {

__device__ __forceinline__ double fmx(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmx(float a, float b, float c) { return fmaf(a, b, c); }

template <int D, int P, int Q>
struct Dims {
  static constexpr int V = D + 2;
  static constexpr int Pd = D == 2 ? P * P : P * P * P;
  static constexpr int Qd = D == 2 ? Q * Q : Q * Q * Q;
  static constexpr int Fn = Pd / P;
  static constexpr int Fq = Qd / Q;
  static constexpr int nf = 2 * D;
  static constexpr int SZP = V * Pd;
  static constexpr int SZQ = V * Qd;
  static constexpr int SZNB = V * nf * Fn;
  static constexpr int SZFL = V * nf * Fq;
};

template <typename T, int D, int P, int Q>
__host__ __device__ constexpr int rhs_elems_per_block() {
  using Dm = Dims<D, P, Q>;
  constexpr int per = (2 * Dm::SZP + 3 * Dm::SZQ) * (int)sizeof(T);
  constexpr int tabb = tab_off(P, Q).total * (int)sizeof(T);
  int ne = kThreads / Dm::Pd;
  if (ne < 1) ne = 1;
  while (ne > 1 && ne * per + tabb > 64 * 1024) --ne;
  return ne;
}

// Apply the 1D operator A (NO x NI, row-major) along axis AX of nvec tensors
// stored back to back with extents (S0, S1, S2) (S_AX == NI); the result has
// extent NO along AX. One thread per line; A is uniform across the block.
template <typename T, int NI, int NO, int S0, int S1, int S2, int AX, bool ACC>
__device__ __forceinline__ void sweep(const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ A,
                                      int nvec) {
  constexpr int O0 = AX == 0 ? NO : S0, O1 = AX == 1 ? NO : S1, O2 = AX == 2 ? NO : S2;
  constexpr int isz = S0 * S1 * S2, osz = O0 * O1 * O2, nl = isz / NI;
  constexpr int istr = AX == 0 ? 1 : (AX == 1 ? S0 : S0 * S1);
  constexpr int ostr = AX == 0 ? 1 : (AX == 1 ? O0 : O0 * O1);
  static_assert((AX == 0 ? S0 : (AX == 1 ? S1 : S2)) == NI, "extent mismatch");
  for (int t = threadIdx.x; t < nvec * nl; t += kThreads) {
    const int v = t / nl, l = t - v * nl;
    int ib, ob;
    if (AX == 0) {
      ib = l * S0;
      ob = l * O0;
    } else if (AX == 1) {
      const int i0 = l % S0, i2 = l / S0;
      ib = i0 + i2 * S0 * S1;
      ob = i0 + i2 * O0 * O1;
    } else {
      ib = l;
      ob = l;
    }
    const T* ip = in + v * isz + ib;
    T* op = out + v * osz + ob;
    T x[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) x[i] = ip[i * istr];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      T acc = A[o * NI] * x[0];
#pragma unroll
      for (int i = 1; i < NI; ++i) acc = fmx(A[o * NI + i], x[i], acc);
      if (ACC)
        op[o * ostr] += acc;
      else
        op[o * ostr] = acc;
    }
  }
}

// index of face-local node j on face f (other axes ascending, lowest fastest)
template <int D, int P>
__device__ __forceinline__ int face_node(int f, int j) {
  const int a = f >> 1, s = (f & 1) ? P - 1 : 0;
  if (D == 2) return a == 0 ? s + P * j : j + P * s;
  const int j0 = j % P, j1 = j / P;
  if (a == 0) return s + P * (j0 + P * j1);
  if (a == 1) return j0 + P * (s + P * j1);
  return j0 + P * (j1 + P * s);
}

// value at face Gauss point fq from the P^(d-1) face-node values t
template <typename T, int D, int P, int Q>
__device__ __forceinline__ T face_interp(const T* t, const T* B, int fq) {
  if (D == 2) {
    T acc = B[fq * P] * t[0];
#pragma unroll
    for (int j = 1; j < P; ++j) acc = fmx(B[fq * P + j], t[j], acc);
    return acc;
  } else {
    const int q0 = fq % Q, q1 = fq / Q;
    T acc = 0;
#pragma unroll
    for (int j1 = 0; j1 < P; ++j1) {
      T r = B[q0 * P] * t[P * j1];
#pragma unroll
      for (int j0 = 1; j0 < P; ++j0) r = fmx(B[q0 * P + j0], t[j0 + P * j1], r);
      acc = j1 == 0 ? B[q1 * P] * r : fmx(B[q1 * P + j1], r, acc);
    }
    return acc;
  }
}

template <typename T, int D>
__device__ __forceinline__ T pressure_of(const T* w, T gm1) {
  T m2 = w[1] * w[1];
#pragma unroll
  for (int k = 1; k < D; ++k) m2 = fmx(w[1 + k], w[1 + k], m2);
  return gm1 * (w[D + 1] - (T)0.5 * m2 / w[0]);
}

// n.F^ for n = +e_a with left state wl and right state wr (eq. lfflux)
template <typename T, int D>
__device__ __forceinline__ void num_flux(const T* wl, const T* wr, int a, T gamma, int kind, T* G) {
  constexpr int V = D + 2;
  const T gm1 = gamma - (T)1;
  const T pl = pressure_of<T, D>(wl, gm1), pr = pressure_of<T, D>(wr, gm1);
  const T il = (T)1 / wl[0], ir = (T)1 / wr[0];
  const T ual = wl[1 + a] * il, uar = wr[1 + a] * ir;
  T Fl[V], Fr[V];
  Fl[0] = wl[1 + a];
  Fr[0] = wr[1 + a];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    Fl[1 + k] = wl[1 + k] * ual + (k == a ? pl : (T)0);
    Fr[1 + k] = wr[1 + k] * uar + (k == a ? pr : (T)0);
  }
  Fl[D + 1] = (wl[D + 1] + pl) * ual;
  Fr[D + 1] = (wr[D + 1] + pr) * uar;
  T lam;
  const T cl2 = gamma * pl * il, cr2 = gamma * pr * ir;
  if (kind == 1) {
    const T sl = fabs(ual) + sqrt(cl2), sr = fabs(uar) + sqrt(cr2);
    lam = sl > sr ? sl : sr;
  } else {
    T ul2 = (wl[1] * il) * (wl[1] * il), ur2 = (wr[1] * ir) * (wr[1] * ir);
#pragma unroll
    for (int k = 1; k < D; ++k) {
      ul2 += (wl[1 + k] * il) * (wl[1 + k] * il);
      ur2 += (wr[1 + k] * ir) * (wr[1 + k] * ir);
    }
    const T sl = ul2 + cl2, sr = ur2 + cr2;
    lam = (T)0.5 * sqrt(sl > sr ? sl : sr);
  }
  const T hl = (T)0.5 * lam;
#pragma unroll
  for (int v = 0; v < V; ++v) G[v] = (T)0.5 * (Fl[v] + Fr[v]) + hl * (wl[v] - wr[v]);
}

// logical block index: the hardware deals consecutive blocks round-robin to
// the 8 XCDs; remap so each XCD walks a contiguous range of elements and its
// L2 holds the neighbours it reads
__device__ __forceinline__ long long xcd_block() {
  const long long nb = gridDim.x, i = blockIdx.x;
  const long long per = nb / 8, rem = nb % 8, x = i % 8, k = i / 8;
  return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

template <typename T, int D, int P, int Q, int NE>
__global__ __launch_bounds__(kThreads) void rhs_stage_kernel(Mesh M, Async A, Stage S,
                                                             const double* __restrict__ u_in, const double* u_n,
                                                             double* out, const double* __restrict__ ghost,
                                                             const T* __restrict__ tab) {
  using Dm = Dims<D, P, Q>;
  constexpr int V = Dm::V, Pd = Dm::Pd, Qd = Dm::Qd, Fn = Dm::Fn, Fq = Dm::Fq, nf = Dm::nf;
  constexpr TabOff to = tab_off(P, Q);
  static_assert(Dm::SZNB + Dm::SZFL <= 3 * Dm::SZQ, "face buffers exceed LDS plan");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sU = reinterpret_cast<T*>(smem_raw);
  T* sR = sU + NE * Dm::SZP;
  T* sW = sR + NE * Dm::SZP;
  T* sX = sW + NE * Dm::SZQ;
  T* sY = sX + NE * Dm::SZQ;
  T* sT = sY + NE * Dm::SZQ;

  const long long e0 = xcd_block() * NE;
  const int ne = (int)(M.E - e0 < NE ? M.E - e0 : NE);
  const int tid = threadIdx.x;

  for (int i = tid; i < to.total; i += kThreads) sT[i] = tab[i];
  const double* gin = u_in + e0 * Dm::SZP;
  for (int i = tid; i < ne * Dm::SZP; i += kThreads) sU[i] = (T)gin[i];
  __syncthreads();

  // 1. interpolation to the Gauss points
  if constexpr (D == 2) {
    sweep<T, P, Q, P, P, 1, 0, false>(sU, sX, tab + to.B, ne * V);
    __syncthreads();
    sweep<T, P, Q, Q, P, 1, 1, false>(sX, sW, tab + to.B, ne * V);
  } else {
    sweep<T, P, Q, P, P, P, 0, false>(sU, sX, tab + to.B, ne * V);
    __syncthreads();
    sweep<T, P, Q, Q, P, P, 1, false>(sX, sY, tab + to.B, ne * V);
    __syncthreads();
    sweep<T, P, Q, Q, Q, P, 2, false>(sY, sW, tab + to.B, ne * V);
  }
  __syncthreads();

  // 2. volume flux at the Gauss points, scaled by w_q |J| 2/h_a
  constexpr int QPT = (NE * Qd + kThreads - 1) / kThreads;
  T F[QPT][D][V];
  const T gamma = (T)M.gamma, gm1 = gamma - (T)1;
#pragma unroll
  for (int k = 0; k < QPT; ++k) {
    const int idx = tid + k * kThreads;
    if (idx < ne * Qd) {
      const int le = idx / Qd, q = idx - le * Qd;
      T w[V];
#pragma unroll
      for (int v = 0; v < V; ++v) w[v] = sW[(le * V + v) * Qd + q];
      T wq = sT[to.WQ + q % Q] * sT[to.WQ + (q / Q) % Q];
      if (D == 3) wq *= sT[to.WQ + q / (Q * Q)];
      const T p = pressure_of<T, D>(w, gm1);
      const T iv = (T)1 / w[0];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const T sc = wq * (T)(M.detJ * 2.0 / M.h[a]);
        const T ua = w[1 + a] * iv;
        F[k][a][0] = sc * w[1 + a];
#pragma unroll
        for (int c = 0; c < D; ++c) F[k][a][1 + c] = sc * (w[1 + c] * ua + (c == a ? p : (T)0));
        F[k][a][D + 1] = sc * ((w[D + 1] + p) * ua);
      }
    }
  }
  // collocation derivative (transposed) along each axis, summed into sY
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
      const int idx = tid + k * kThreads;
      if (idx < ne * Qd) {
        const int le = idx / Qd, q = idx - le * Qd;
#pragma unroll
        for (int v = 0; v < V; ++v) sX[(le * V + v) * Qd + q] = F[k][a][v];
      }
    }
    __syncthreads();
    if (D == 2) {
      if (a == 0)
        sweep<T, Q, Q, Q, Q, 1, 0, false>(sX, sY, tab + to.DT, ne * V);
      else
        sweep<T, Q, Q, Q, Q, 1, 1, true>(sX, sY, tab + to.DT, ne * V);
    } else {
      if (a == 0)
        sweep<T, Q, Q, Q, Q, Q, 0, false>(sX, sY, tab + to.DT, ne * V);
      else if (a == 1)
        sweep<T, Q, Q, Q, Q, Q, 1, true>(sX, sY, tab + to.DT, ne * V);
      else
        sweep<T, Q, Q, Q, Q, Q, 2, true>(sX, sY, tab + to.DT, ne * V);
    }
    __syncthreads();
  }
  // transposed interpolation back to the nodes: residual in sR
  if constexpr (D == 2) {
    sweep<T, Q, P, Q, Q, 1, 0, false>(sY, sX, tab + to.BT, ne * V);
    __syncthreads();
    sweep<T, Q, P, P, Q, 1, 1, false>(sX, sR, tab + to.BT, ne * V);
  } else {
    sweep<T, Q, P, Q, Q, Q, 0, false>(sY, sX, tab + to.BT, ne * V);
    __syncthreads();
    sweep<T, Q, P, P, Q, Q, 1, false>(sX, sW, tab + to.BT, ne * V);
    __syncthreads();
    sweep<T, Q, P, P, P, Q, 2, false>(sW, sR, tab + to.BT, ne * V);
  }
  __syncthreads();

  // 3. surface term. Neighbour face nodes (live or ghost) into sNB.
  T* sNB = sW;
  T* sFL = sW + NE * Dm::SZNB;
  const bool use_ghost = A.ghost != 0 && M.nfs > 0;
  for (int i = tid; i < ne * Dm::SZNB; i += kThreads) {
    const int j = i % Fn;
    const int r = i / Fn;
    const int v = r % V;
    const int r2 = r / V;
    const int f = r2 % nf, le = r2 / nf;
    int c[3];
    elem_coords(M, e0 + le, c);
    const long long fs = use_ghost ? face_side(M, c, f) : -1;
    double val;
    if (fs >= 0) {
      val = ghost[(fs * V + v) * Fn + j];
    } else {
      const long long nb = neighbour(M, c, f);
      val = u_in[(nb * V + v) * Pd + face_node<D, P>(f ^ 1, j)];
    }
    sNB[i] = (T)val;
  }
  __syncthreads();
  for (int i = tid; i < ne * nf * Fq; i += kThreads) {
    const int fq = i % Fq;
    const int r = i / Fq;
    const int f = r % nf, le = r / nf;
    const int a = f >> 1, side = f & 1;
    T wo[V], wn[V], t[Fn];
#pragma unroll
    for (int v = 0; v < V; ++v) {
#pragma unroll
      for (int j = 0; j < Fn; ++j) t[j] = sU[(le * V + v) * Pd + face_node<D, P>(f, j)];
      wo[v] = face_interp<T, D, P, Q>(t, sT + to.B, fq);
#pragma unroll
      for (int j = 0; j < Fn; ++j) t[j] = sNB[((le * nf + f) * V + v) * Fn + j];
      wn[v] = face_interp<T, D, P, Q>(t, sT + to.B, fq);
    }
    // canonical (left, right) operands, one call site for both sides
    T wl[V], wr[V], G[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      wl[v] = side ? wo[v] : wn[v];
      wr[v] = side ? wn[v] : wo[v];
    }
    num_flux<T, D>(wl, wr, a, gamma, M.flux, G);
    T ws = sT[to.WQ + fq % Q];
    if (D == 3) ws *= sT[to.WQ + fq / Q];
    ws *= (T)M.detJf[a];
    const T sg = side ? (T)1 : (T)-1;
#pragma unroll
    for (int v = 0; v < V; ++v) sFL[((le * nf + f) * V + v) * Fq + fq] = sg * (G[v] * ws);
  }
  __syncthreads();
  // lift: R_i -= sum over the faces through node i of phi_i . flux
  for (int i = tid; i < ne * Dm::SZP; i += kThreads) {
    const int node = i % Pd;
    const int r = i / Pd;
    const int v = r % V, le = r / V;
    const int nc[3] = {node % P, (node / P) % P, node / (P * P)};
    T acc = 0;
    bool any = false;
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        if (nc[a] != (side ? P - 1 : 0)) continue;
        const int f = 2 * a + side;
        const int o0 = a == 0 ? 1 : 0, o1 = a == 2 ? 1 : 2;
        const int j0 = nc[o0], j1 = D == 3 ? nc[o1] : 0;
        const T* fl = sFL + ((le * nf + f) * V + v) * Fq;
        T s = 0;
        if (D == 2) {
#pragma unroll
          for (int q = 0; q < Q; ++q) s = fmx(sT[to.B + q * P + j0], fl[q], s);
        } else {
#pragma unroll
          for (int q1 = 0; q1 < Q; ++q1) {
            T r1 = 0;
#pragma unroll
            for (int q0 = 0; q0 < Q; ++q0) r1 = fmx(sT[to.B + q0 * P + j0], fl[q0 + Q * q1], r1);
            s = fmx(sT[to.B + q1 * P + j1], r1, s);
          }
        }
        acc += s;
        any = true;
      }
    }
    if (any) sR[i] -= acc;
  }
  __syncthreads();

  // 4. inverse mass: d sweeps of M1^{-1}
  T* sK;
  if constexpr (D == 2) {
    sweep<T, P, P, P, P, 1, 0, false>(sR, sX, tab + to.MI, ne * V);
    __syncthreads();
    sweep<T, P, P, P, P, 1, 1, false>(sX, sY, tab + to.MI, ne * V);
    sK = sY;
  } else {
    sweep<T, P, P, P, P, P, 0, false>(sR, sX, tab + to.MI, ne * V);
    __syncthreads();
    sweep<T, P, P, P, P, P, 1, false>(sX, sY, tab + to.MI, ne * V);
    __syncthreads();
    sweep<T, P, P, P, P, P, 2, false>(sY, sX, tab + to.MI, ne * V);
    sK = sX;
  }
  __syncthreads();

  // 5. SSP-RK3 combine in FP64
  const double idet = 1.0 / M.detJ;
  double* gout = out + e0 * Dm::SZP;
  const double* gn = u_n + e0 * Dm::SZP;
  for (int i = tid; i < ne * Dm::SZP; i += kThreads) {
    const double k = (double)sK[i] * idet;
    const double ui = sizeof(T) == 8 ? (double)sU[i] : gin[i];
    const double y = ui + S.dt * k;
    gout[i] = S.a == 0.0 ? S.b * y : S.a * gn[i] + S.b * y;
  }
}

template <typename T, int D, int p>
static hipError_t launch_rhs_t(const Mesh& M, const Async& A, const Stage& S, const double* u_in, const double* u_n,
                               double* out, const double* ghost, const T* tab, hipStream_t st) {
  constexpr int P = p + 1, Q = p + 2;
  constexpr int NE = rhs_elems_per_block<T, D, P, Q>();
  using Dm = Dims<D, P, Q>;
  const size_t smem = (size_t)(NE * (2 * Dm::SZP + 3 * Dm::SZQ) + tab_off(P, Q).total) * sizeof(T);
  const long long nblk = (M.E + NE - 1) / NE;
  hipLaunchKernelGGL((rhs_stage_kernel<T, D, P, Q, NE>), dim3((unsigned)nblk), dim3(kThreads), smem, st, M, A, S,
                     u_in, u_n, out, ghost, tab);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_rhs_prec(int dim, int degree, const Mesh& M, const Async& A, const Stage& S,
                                  const double* u_in, const double* u_n, double* out, const double* ghost,
                                  const T* tab, hipStream_t st) {
#define ADG_RHS_CASE(d, p) \
  if (dim == d && degree == p) return launch_rhs_t<T, d, p>(M, A, S, u_in, u_n, out, ghost, tab, st);
  ADG_RHS_CASE(2, 1) ADG_RHS_CASE(2, 2) ADG_RHS_CASE(2, 3) ADG_RHS_CASE(2, 4)
  ADG_RHS_CASE(3, 1) ADG_RHS_CASE(3, 2) ADG_RHS_CASE(3, 3) ADG_RHS_CASE(3, 4)
#undef ADG_RHS_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_rhs_stage(int dim, int degree, int precision, const Mesh& M, const Async& A, const Stage& S,
                            const double* u_in, const double* u_n, double* out, const double* ghost,
                            const double* tab64, const float* tab32, hipStream_t st) {
  if (precision == 1) return launch_rhs_prec<float>(dim, degree, M, A, S, u_in, u_n, out, ghost, tab32, st);
  return launch_rhs_prec<double>(dim, degree, M, A, S, u_in, u_n, out, ghost, tab64, st);
}

// ---------------------------------------------------------------------------
// ghost traces and ring publish: one thread per (face-side, variable, node)
// ---------------------------------------------------------------------------

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
  const long long src = (nb * V + v) * Pd + face_node<D, P>(f ^ 1, j);
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
