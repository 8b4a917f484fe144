// adg_rhs.hip — the fused SSP-RK3 stage of the DG right-hand side on gfx950:
// the LDS-staged kernel (hexahedra of degree 4) and the dispatch of every
// stage launch to its kernel (quadrilaterals: adg_rhs2d.hip; hexahedra of
// degree 1 and 2: adg_rhs3d.hip; degree 3: adg_rhs3d_split.hip).
//
// One workgroup (one wavefront) owns NE consecutive elements (x fastest) and
// computes, in LDS and registers, k = M_e^{-1} L_h(u_in) for each of them
// (Sec. 2.1, eq. weakform-dealii / weakform-compact-dealii), then the
// Shu-Osher combine out = a u_n + b (u_in + dt k) in FP64.
//
//   volume:  interpolation of u_in from the P^d Gauss-Lobatto nodes to the
//            Q^d Gauss points (d sweeps with B); the Euler flux columns F_a at
//            every point, scaled by w_q 2/h_a; the transposed collocation
//            derivative along each axis, summed; then d sweeps with
//            BTM = M1^{-1} B^T, which test against the basis and apply the
//            inverse mass in one pass (|J| cancels).
//   faces:   for each axis a, both faces: the element's own face-node values
//            and the neighbour's (its live values, or the ghost trace at a
//            PE-boundary face) are interpolated to the Q^(d-1) face points,
//            the local Lax-Friedrichs flux of eq. lfflux / lfflux-lambda is
//            evaluated in canonical (left, right) order and scaled by
//            -w_f 2/h_a; d-1 sweeps with BTM lift it, and the inverse mass
//            along a turns the face trace into the column of M1^{-1} at that
//            face: k += MC_side (x) lifted flux.
//
// Both neighbours of an interior face evaluate the flux with one instruction
// stream on identical operands in the same order, so their contributions are
// bitwise opposite and the synchronous scheme conserves to round-off.
// T = double (FP64 path) or float (FP32 contractions; combine in FP64).
#include "adg_device.h"
#include "adg_internal.h"
#include "adg_tables.h"

namespace adg {

// threads per workgroup: one wavefront, so the workgroup barriers between the
// LDS sweeps cost no cross-wave waiting
constexpr int kNT3 = 64;

// the 1D operators as compile-time constants in the kernel's precision
template <typename T, int P>
struct KOps {
  static constexpr int Q = P + 1;
  T B[Q * P];    // B[q][j] = l_j(x_q)
  T DT[Q * Q];   // DT[r][q] = g_r'(x_q)
  T BTM[P * Q];  // M1^{-1} B^T
};
template <typename T, int P>
constexpr KOps<T, P> make_kops() {
  constexpr int Q = P + 1;
  const ops::Ops<P> o = ops::make_ops<P>();
  KOps<T, P> k{};
  for (int q = 0; q < Q; ++q) {
    for (int j = 0; j < P; ++j) k.B[q * P + j] = static_cast<T>(o.B[q][j]);
    for (int r = 0; r < Q; ++r) k.DT[r * Q + q] = static_cast<T>(o.D[q][r]);
  }
  for (int i = 0; i < P; ++i)
    for (int q = 0; q < Q; ++q) k.BTM[i * Q + q] = static_cast<T>(o.BTM[i][q]);
  return k;
}

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
  // faces handled per pass (both faces of an axis when the buffers fit)
  static constexpr int NS = (2 * V * 2 * (Fn + Fq) + (D == 3 ? 2 * V * 2 * Q * P : 0)) <= 2 * SZQ ? 2 : 1;
  static constexpr int TR = 2 * NS * V * Fn;  // own + neighbour face nodes
  static constexpr int TQ = 2 * NS * V * Fq;  // own + neighbour face points
  static constexpr int TM = D == 3 ? 2 * NS * V * Q * P : 0;
  static_assert(TR + TQ + TM <= 2 * SZQ, "face buffers exceed the LDS plan");
};

// per (element, face) descriptor kept in LDS: neighbour element offset, the
// face-side offset of this face in the ring (or -1), the offset of the
// face-side this face feeds in the neighbour subdomain's ring (or -1), delay
constexpr int kFaceInfoBytes = 32;

template <typename T, int D, int P, int Q>
__host__ __device__ constexpr int rhs_elems_per_block() {
  using Dm = Dims<D, P, Q>;
  constexpr int per = (2 * Dm::SZP + 2 * Dm::SZQ) * (int)sizeof(T) + Dm::nf * kFaceInfoBytes;
  constexpr int tabb = tab_off(P, Q).total * (int)sizeof(T);
  int ne = kNT3 / Dm::Pd;
  if (ne < 1) ne = 1;
  while (ne > 1 && ne * per + tabb > 64 * 1024) --ne;
  return ne;
}

template <typename T, int D, int P, int Q>
__host__ __device__ constexpr size_t rhs_smem_bytes(int NE) {
  using Dm = Dims<D, P, Q>;
  return (size_t)NE * Dm::nf * kFaceInfoBytes +
         (size_t)(NE * (2 * Dm::SZP + 2 * Dm::SZQ) + tab_off(P, Q).total) * sizeof(T);
}


// Apply the 1D operator A (NO x NI, row-major) along axis AX of nvec tensors
// stored back to back with extents (S0, S1, S2) (S_AX == NI); the result has
// extent NO along AX. One thread per line; A is uniform across the block, so
// its entries come through the scalar cache.
template <typename T, int NI, int NO, int S0, int S1, int S2, int AX, bool ACC>
__device__ __forceinline__ void sweep(const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ A,
                                      int nvec) {
  constexpr int O0 = AX == 0 ? NO : S0, O1 = AX == 1 ? NO : S1, O2 = AX == 2 ? NO : S2;
  constexpr int isz = S0 * S1 * S2, osz = O0 * O1 * O2, nl = isz / NI;
  constexpr int istr = AX == 0 ? 1 : (AX == 1 ? S0 : S0 * S1);
  constexpr int ostr = AX == 0 ? 1 : (AX == 1 ? O0 : O0 * O1);
  static_assert((AX == 0 ? S0 : (AX == 1 ? S1 : S2)) == NI, "extent mismatch");
  for (int t = threadIdx.x; t < nvec * nl; t += kNT3) {
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

// node index of face-local node j on face f (other axes ascending, lowest fastest)
template <int D, int P>
__device__ __forceinline__ int face_node(int f, int j) {
  const int a = f >> 1, s = (f & 1) ? P - 1 : 0;
  if (D == 2) return a == 0 ? s + P * j : j + P * s;
  const int j0 = j % P, j1 = j / P;
  if (a == 0) return s + P * (j0 + P * j1);
  if (a == 1) return j0 + P * (s + P * j1);
  return j0 + P * (j1 + P * s);
}

template <typename T, int D, int P, int Q, int NE>
__global__ __launch_bounds__(kNT3) void rhs_stage_kernel(Mesh M, Async A, Stage S,
                                                             const double* __restrict__ u_in, const double* u_n,
                                                             double* out, int src, double* __restrict__ ring,
                                                             const double* __restrict__ ghost,
                                                             const T* __restrict__ tab) {
  using Dm = Dims<D, P, Q>;
  constexpr int V = Dm::V, Pd = Dm::Pd, Qd = Dm::Qd, Fn = Dm::Fn, Fq = Dm::Fq, nf = Dm::nf, NS = Dm::NS;
  constexpr TabOff to = tab_off(P, Q);
  static constexpr KOps<T, P> KO = make_kops<T, P>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  long long* sNb = reinterpret_cast<long long*>(smem_raw);  // neighbour element offset
  long long* sFs = sNb + NE * nf;                           // own face-side offset, or -1
  long long* sPub = sFs + NE * nf;                          // face-side fed by this face, or -1
  int* sK = reinterpret_cast<int*>(sPub + NE * nf);         // delay of this face
  T* sU = reinterpret_cast<T*>(smem_raw + NE * nf * kFaceInfoBytes);
  T* sR = sU + NE * Dm::SZP;
  T* sB1 = sR + NE * Dm::SZP;
  T* sB2 = sB1 + NE * Dm::SZQ;
  T* sT = sB2 + NE * Dm::SZQ;

  const long long e0 = (long long)xcd_block() * NE;
  const int ne = (int)(M.E - e0 < NE ? M.E - e0 : NE);
  const int tid = threadIdx.x;
  const bool async_on = src != kSrcLive && M.nfs > 0;
  const bool flux_mode = src == kSrcFlux;
  // values per ring level: face-node traces, or face-point fluxes
  const long long ring_level = M.nfs * V * (flux_mode ? Fq : Fn);
  const bool publish = src == kSrcRing && A.stage == 0;

  // per element face: neighbour, PE face-side, delay, and the face-side it feeds
  for (int t = tid; t < ne * nf; t += kNT3) {
    const int le = t / nf, f = t - le * nf;
    const ElemPos pos = elem_pos(M, e0 + le);
    sNb[t] = neighbour_of(M, e0 + le, pos, f) * V * Pd;
    const long long fs = async_on ? face_side_at(M, pos, f) : -1;
    sFs[t] = fs >= 0 ? fs * V * (flux_mode ? Fq : Fn) : -1;
    sK[t] = fs >= 0 && (src == kSrcRing || flux_mode) ? delay_of(M, A, sub_at(M, pos.sc), f) : 0;
    sPub[t] = publish && fs >= 0 ? fed_face_side(M, pos, f) * V * Fn : -1;
  }
  for (int i = tid; i < to.total; i += kNT3) sT[i] = tab[i];
  // the stage input into LDS; u_n (and, for T = float, the FP64 input) for
  // the combine into registers now, so their latency hides behind the compute
  const double* gin = u_in + e0 * Dm::SZP;
  const double* gn = u_n + e0 * Dm::SZP;
  constexpr int CPT = (NE * Dm::SZP + kNT3 - 1) / kNT3;
  double ur[CPT], un[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int i = tid + k * kNT3;
    ur[k] = un[k] = 0.0;
    if (i < ne * Dm::SZP) {
      const double x = gin[i];
      sU[i] = (T)x;
      if (sizeof(T) == 4) ur[k] = x;
      if (S.a != 0.0 || S.lserk) un[k] = gn[i];
    }
  }
  __syncthreads();

  // stage 0 of a step: publish this block's PE-boundary traces of u^n into
  // ring slot n mod R, where the neighbouring subdomain will read them. No
  // reader of this launch touches that slot: delays >= 1 read older levels,
  // delay 0 reads the live values.
  if (publish) {
    double* slot = ring + A.slot_n * ring_level;
    for (int i = tid; i < ne * nf * Fn; i += kNT3) {
      const int j = i % Fn;
      const int t = i / Fn;
      const long long pub = sPub[t];
      if (pub < 0) continue;
      const int le = t / nf, f = t - le * nf;
      const int node = face_node<D, P>(f, j);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int q = (le * V + v) * Pd + node;
        slot[pub + v * Fn + j] = sizeof(T) == 8 ? (double)sU[q] : gin[q];
      }
    }
  }

  // ---- volume: interpolation to the Gauss points (result in sB1)
  if constexpr (D == 2) {
    sweep<T, P, Q, P, P, 1, 0, false>(sU, sB2, KO.B, NE * V);
    __syncthreads();
    sweep<T, P, Q, Q, P, 1, 1, false>(sB2, sB1, KO.B, NE * V);
  } else {
    sweep<T, P, Q, P, P, P, 0, false>(sU, sB1, KO.B, NE * V);
    __syncthreads();
    sweep<T, P, Q, Q, P, P, 1, false>(sB1, sB2, KO.B, NE * V);
    __syncthreads();
    sweep<T, P, Q, Q, Q, P, 2, false>(sB2, sB1, KO.B, NE * V);
  }
  __syncthreads();

  // Euler flux columns at the Gauss points, scaled by w_q 2/h_a (registers)
  constexpr int QPT = (NE * Qd + kNT3 - 1) / kNT3;
  T F[QPT][D][V];
  const T gamma = (T)M.gamma, gm1 = gamma - (T)1;
#pragma unroll
  for (int k = 0; k < QPT; ++k) {
    const int idx = tid + k * kNT3;
    if (idx < NE * Qd) {
      const int le = idx / Qd, q = idx - le * Qd;
      T w[V];
#pragma unroll
      for (int v = 0; v < V; ++v) w[v] = sB1[(le * V + v) * Qd + q];
      T wq = sT[to.WQ + q % Q] * sT[to.WQ + (q / Q) % Q];
      if (D == 3) wq *= sT[to.WQ + q / (Q * Q)];
      const T iv = (T)1 / w[0];
      T m2 = w[1] * w[1];
#pragma unroll
      for (int c = 1; c < D; ++c) m2 = fmx(w[1 + c], w[1 + c], m2);
      const T p = gm1 * (w[D + 1] - (T)0.5 * m2 * iv);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const T sc = wq * (T)(2.0 / M.h[a]);
        const T ua = w[1 + a] * iv;
        F[k][a][0] = sc * w[1 + a];
#pragma unroll
        for (int c = 0; c < D; ++c) F[k][a][1 + c] = sc * (w[1 + c] * ua + (c == a ? p : (T)0));
        F[k][a][D + 1] = sc * ((w[D + 1] + p) * ua);
      }
    }
  }
  __syncthreads();
  // transposed collocation derivative along each axis, summed into sB2
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
      const int idx = tid + k * kNT3;
      if (idx < NE * Qd) {
        const int le = idx / Qd, q = idx - le * Qd;
#pragma unroll
        for (int v = 0; v < V; ++v) sB1[(le * V + v) * Qd + q] = F[k][a][v];
      }
    }
    __syncthreads();
    if (D == 2) {
      if (a == 0)
        sweep<T, Q, Q, Q, Q, 1, 0, false>(sB1, sB2, KO.DT, NE * V);
      else
        sweep<T, Q, Q, Q, Q, 1, 1, true>(sB1, sB2, KO.DT, NE * V);
    } else {
      if (a == 0)
        sweep<T, Q, Q, Q, Q, Q, 0, false>(sB1, sB2, KO.DT, NE * V);
      else if (a == 1)
        sweep<T, Q, Q, Q, Q, Q, 1, true>(sB1, sB2, KO.DT, NE * V);
      else
        sweep<T, Q, Q, Q, Q, Q, 2, true>(sB1, sB2, KO.DT, NE * V);
    }
    __syncthreads();
  }
  // test functions and inverse mass in one: BTM sweeps, k_volume in sR
  if constexpr (D == 2) {
    sweep<T, Q, P, Q, Q, 1, 0, false>(sB2, sB1, KO.BTM, NE * V);
    __syncthreads();
    sweep<T, Q, P, P, Q, 1, 1, false>(sB1, sR, KO.BTM, NE * V);
  } else {
    sweep<T, Q, P, Q, Q, Q, 0, false>(sB2, sB1, KO.BTM, NE * V);
    __syncthreads();
    sweep<T, Q, P, P, Q, Q, 1, false>(sB1, sB2, KO.BTM, NE * V);
    __syncthreads();
    sweep<T, Q, P, P, P, Q, 2, false>(sB2, sR, KO.BTM, NE * V);
  }
  __syncthreads();

  // ---- faces, NS faces of one axis per pass
  // layouts: sTr [side][le][s][v][Fn], sTq [side][le][s][v][Fq],
  // sTm (3D interpolation intermediate) [side][le][s][v][Q*P]
  T* sTr = sB1;
  T* sTq = sTr + NE * Dm::TR;
  T* sTm = sTq + NE * Dm::TQ;
  constexpr int HALF_R = NE * NS * V * Fn, HALF_Q = NE * NS * V * Fq;  // start of the neighbour half
#pragma unroll 1
  for (int pass = 0; pass < nf / NS; ++pass) {
    const int a = (pass * NS) >> 1;
    const int s0 = (pass * NS) & 1;
    // gather own (side 0) and neighbour (side 1) face-node values; one item
    // per (side, element, face, node), all V variables
    for (int i = tid; i < 2 * NE * NS * Fn; i += kNT3) {
      const int j = i % Fn;
      const int r = i / Fn;
      const int ls = r % (NE * NS);  // le * NS + (s - s0)
      const int side = r / (NE * NS);
      const int le = ls / NS, s = ls - le * NS + s0;
      if (le >= ne) continue;  // past the last element
      const int f = 2 * a + s;
      T* dst = sTr + side * HALF_R + ls * V * Fn + j;
      if (side == 0) {
        const T* srcp = sU + le * V * Pd + face_node<D, P>(f, j);
#pragma unroll
        for (int v = 0; v < V; ++v) dst[v * Fn] = srcp[v * Pd];
        continue;
      }
      const int t = le * nf + f;
      const long long fs = sFs[t];
      const int k = sK[t];
      if (fs < 0 || ((src == kSrcRing || flux_mode) && k == 0)) {
        // interior face, synchronous mode, or zero delay: live stage values
        const double* g = u_in + sNb[t] + face_node<D, P>(f ^ 1, j);
#pragma unroll
        for (int v = 0; v < V; ++v) dst[v * Fn] = (T)g[v * Pd];
      } else if (flux_mode) {
        // silent step: the face uses the stored flux, no trace needed
#pragma unroll
        for (int v = 0; v < V; ++v) dst[v * Fn] = (T)0;
      } else if (src == kSrcGhost) {
        const double* g = ghost + fs + j;
#pragma unroll
        for (int v = 0; v < V; ++v) dst[v * Fn] = (T)g[v * Fn];
      } else if (A.ghost == 1) {
        // standard flux on the trace k steps old (eq. delayed-flux)
        const double* g = ring + ring_slot(A, k) * ring_level + fs + j;
#pragma unroll
        for (int v = 0; v < V; ++v) dst[v * Fn] = (T)g[v * Fn];
      } else {
        // AT extrapolation of `levels` stored levels to the stage time
        // (eq. at-flux, tau = k + c_m); weights and sums in FP64
        const double tau = k + A.c_m;
        double acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0.0;
        // at most kMaxLevels levels; past A.levels the newest is read again
        // with weight 0, so every load is issued before the first is used
#pragma unroll
        for (int l = 0; l < kMaxLevels; ++l) {
          const bool on = l < A.levels;
          const double wl = on ? at_weight(l, A.levels, tau) : 0.0;
          const double* g = ring + ring_slot(A, k + (on ? l : 0)) * ring_level + fs + j;
#pragma unroll
          for (int v = 0; v < V; ++v) acc[v] += wl * g[v * Fn];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) dst[v * Fn] = (T)acc[v];
      }
    }
    __syncthreads();
    // interpolation to the face points (both sides at once)
    if constexpr (D == 2) {
      sweep<T, P, Q, P, 1, 1, 0, false>(sTr, sTq, KO.B, 2 * NE * NS * V);
    } else {
      sweep<T, P, Q, P, P, 1, 0, false>(sTr, sTm, KO.B, 2 * NE * NS * V);
      __syncthreads();
      sweep<T, P, Q, Q, P, 1, 1, false>(sTm, sTq, KO.B, 2 * NE * NS * V);
    }
    __syncthreads();
    // numerical flux at every face point, in place of the own values
    for (int i = tid; i < NE * NS * Fq; i += kNT3) {
      const int fq = i % Fq;
      const int r = i / Fq;
      const int s = r % NS + s0, le = r / NS;
      const int base = ((le * NS + (s - s0)) * V) * Fq + fq;
      T wo[V], wn[V], wl[V], wr[V], G[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        wo[v] = sTq[base + v * Fq];
        wn[v] = sTq[HALF_Q + base + v * Fq];
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        wl[v] = s ? wo[v] : wn[v];
        wr[v] = s ? wn[v] : wo[v];
      }
      const int tf = le * nf + 2 * a + s;
      const long long ffs = flux_mode && le < ne ? sFs[tf] : -1;
      const int fkd = flux_mode && le < ne ? sK[tf] : 0;
      if (ffs >= 0 && fkd > 0) {
        // silent step of Alg. caa-std / caa-at: the stored flux, or its AT
        // extrapolation to the stage time tau = k + c_m (FP64)
        const double* fp = ring + ffs + fq;
        double acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = 0.0;
        if (A.ghost == 4) {
#pragma unroll
          for (int v = 0; v < V; ++v) acc[v] = fp[ring_slot(A, fkd) * ring_level + v * Fq];
        } else {
          const double tau = fkd + A.c_m;
          // at most kMaxLevels levels; past A.levels the newest is read again
          // with weight 0, so every load is issued before the first is used
#pragma unroll
          for (int l = 0; l < kMaxLevels; ++l) {
            const bool on = l < A.levels;
            const double w = on ? at_weight(l, A.levels, tau) : 0.0;
            const double* lp = fp + ring_slot(A, fkd + (on ? l : 0)) * ring_level;
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = fma(w, lp[v * Fq], acc[v]);
          }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) G[v] = (T)acc[v];
      } else {
        num_flux<T, D>(wl, wr, a, gamma, M.flux, G);
        // communicating step of a flux-history mode: keep the stage-0 flux
        if (ffs >= 0 && A.stage == 0) {
          double* fp = ring + A.slot_n * ring_level + ffs + fq;
#pragma unroll
          for (int v = 0; v < V; ++v) fp[v * Fq] = (double)G[v];
        }
      }
      T ws = sT[to.WQ + fq % Q];
      if (D == 3) ws *= sT[to.WQ + fq / Q];
      ws *= (T)(2.0 / M.h[a]);
      const T sg = s ? (T)-1 : (T)1;  // -(n.e_a): the face term enters with a minus sign
#pragma unroll
      for (int v = 0; v < V; ++v) sTq[base + v * Fq] = sg * (G[v] * ws);
    }
    __syncthreads();
    // lift with BTM to the face nodes (own half only), result in sTr
    if constexpr (D == 2) {
      sweep<T, Q, P, Q, 1, 1, 0, false>(sTq, sTr, KO.BTM, NE * NS * V);
    } else {
      sweep<T, Q, P, Q, Q, 1, 0, false>(sTq, sTm, KO.BTM, NE * NS * V);
      __syncthreads();
      sweep<T, Q, P, P, Q, 1, 1, false>(sTm, sTr, KO.BTM, NE * NS * V);
    }
    __syncthreads();
    // inverse mass along a: k += MC_side[i_a] * lifted(j)
    for (int i = tid; i < NE * Dm::SZP; i += kNT3) {
      const int node = i % Pd;
      const int r = i / Pd;
      const int v = r % V, le = r / V;
      const int nc[3] = {node % P, (node / P) % P, node / (P * P)};
      const int o0 = a == 0 ? 1 : 0, o1 = a == 2 ? 1 : 2;
      const int j = D == 2 ? nc[o0] : nc[o0] + P * nc[o1];
      T acc = sR[i];
#pragma unroll
      for (int ss = 0; ss < NS; ++ss) {
        const int s = ss + s0;
        acc = fmx(sT[to.MC + s * P + nc[a]], sTr[((le * NS + ss) * V + v) * Fn + j], acc);
      }
      sR[i] = acc;
    }
    __syncthreads();
  }

  // ---- the stage combine in FP64
  double* gout = out + e0 * Dm::SZP;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int i = tid + k * kNT3;
    if (i < ne * Dm::SZP) {
      if (S.lserk) {
        // LSERK: u_n holds the accumulator w (read at the start)
        gout[i] = un[k] + S.dt * S.bw * (double)sR[i];
        if (S.out2) S.out2[e0 * Dm::SZP + i] = un[k] + S.dt * S.ar * (double)sR[i];
      } else {
        const double ui = sizeof(T) == 8 ? (double)sU[i] : ur[k];
        const double y = ui + S.dt * (double)sR[i];
        gout[i] = S.a == 0.0 ? S.b * y : S.a * un[k] + S.b * y;
      }
    }
  }
}

template <typename T, int D, int p>
static hipError_t launch_rhs_t(const Mesh& M, const Async& A, const Stage& S, const double* u_in, const double* u_n,
                               double* out, int src, double* ring, const double* ghost, const T* tab,
                               hipStream_t st) {
  constexpr int P = p + 1, Q = p + 2;
  constexpr int NE = rhs_elems_per_block<T, D, P, Q>();
  const size_t smem = rhs_smem_bytes<T, D, P, Q>(NE);
  const long long nblk = (M.E + NE - 1) / NE;
  hipLaunchKernelGGL((rhs_stage_kernel<T, D, P, Q, NE>), dim3((unsigned)nblk), dim3(kNT3), smem, st, M, A, S,
                     u_in, u_n, out, src, ring, ghost, tab);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_rhs_prec(int dim, int degree, const Mesh& M, const Async& A, const Stage& S,
                                  const double* u_in, const double* u_n, double* out, int src, double* ring,
                                  const double* ghost, const T* tab, hipStream_t st) {
#define ADG_RHS_CASE(d, p) \
  if (dim == d && degree == p) return launch_rhs_t<T, d, p>(M, A, S, u_in, u_n, out, src, ring, ghost, tab, st);
  ADG_RHS_CASE(3, 4)
#undef ADG_RHS_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_rhs_stage(int dim, int degree, int precision, const Mesh& M, const Async& A, const Stage& S,
                            const double* u_in, const double* u_n, double* out, int src, double* ring,
                            const double* ghost, const double* tab64, const float* tab32, hipStream_t st) {
  if (dim == 2)
    return launch_rhs_stage_2d(degree, precision, M, A, S, u_in, u_n, out, src, ring, ghost, st);
  if (degree <= 2)
    return launch_rhs_stage_3d(degree, precision, M, A, S, u_in, u_n, out, src, ring, ghost, st);
  if (degree == 3)
    return launch_rhs_stage_3d_split(degree, precision, M, A, S, u_in, u_n, out, src, ring, ghost, st);
  if (precision == 1)
    return launch_rhs_prec<float>(dim, degree, M, A, S, u_in, u_n, out, src, ring, ghost, tab32, st);
  return launch_rhs_prec<double>(dim, degree, M, A, S, u_in, u_n, out, src, ring, ghost, tab64, st);
}

}  // namespace adg
