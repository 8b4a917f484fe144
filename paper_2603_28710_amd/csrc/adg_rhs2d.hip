// adg_rhs2d.hip — the fused SSP-RK3 stage on quadrilateral meshes (d = 2).
//
// One wavefront owns 16 consecutive elements (x fastest). Lane (e, v) keeps
// the P^2 nodal values of variable v of element e in registers and applies
// every tensor-product operator of that variable there; LDS carries only the
// exchanges that the nonlinear fluxes need (all V variables at one point).
//
//   volume: the lane interpolates its variable to the Q^2 Gauss points
//           (x, then y) and stores it in LDS. Row by row of Gauss points, it
//           then reads the full state, forms its own components F_x[v] and
//           F_y[v] of the Euler flux (eq. euler-dealii) and accumulates
//             k += (2/h_x) (GW (x) BW) F_x + (2/h_y) (BW (x) GW) F_y,
//           with BW = M1^{-1} B^T W and GW = M1^{-1} B^T D^T W: the test
//           functions, the collocation derivative on the Gauss points, the
//           Gauss weights and the inverse 1D mass as one operator each
//           (eq. weakform-dealii / weakform-compact-dealii; |J| cancels).
//   faces:  per axis, every lane interpolates its own and the neighbour's
//           face traces (live values, the delayed / AT / learned trace at a
//           PE-boundary face, or the exact exterior state at a boundary face of
//           a Dirichlet box) to the Gauss points of both faces; one lane per
//           (element, face, point) evaluates the local Lax-Friedrichs flux of
//           eq. lfflux / lfflux-lambda in canonical (left, right) order, in
//           place; every lane lifts its variable with BW and adds the column
//           of M1^{-1} at that face.
//   stage:  out = a u_n + b (u_in + dt k) in FP64 from the FP64 registers,
//           written to LDS and stored as one coalesced, streamed range.
//
// Both sides of an interior face evaluate the flux with the same instruction
// stream on identical operands, so their contributions are bitwise opposite.
// At stage 0 of a step (stale and AT modes) the kernel also publishes its
// PE-boundary traces of u^n into ring slot n mod R; readers in the same launch
// use only older slots (delay >= 1) or live values (delay 0).
// T = double (FP64 path) or float (FP32 contractions, FP64 state and combine).
#include "adg_device.h"
#include "adg_internal.h"
#include "adg_tables.h"

namespace adg {

namespace {

constexpr int kNE2 = 16;  // elements per wavefront (V = 4 lanes each)

// node index of face-local node j on face f (2D, x fastest)
template <int P>
__device__ __forceinline__ constexpr int fnode(int f, int j) {
  return (f >> 1) == 0 ? j * P + ((f & 1) ? P - 1 : 0) : ((f & 1) ? P - 1 : 0) * P + j;
}

template <int P>
__device__ __forceinline__ void load_col(const double* __restrict__ p, double* u) {
  constexpr int Pd = P * P;
  if constexpr (Pd % 2 == 0) {
    const double2* p2 = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int i = 0; i < Pd / 2; ++i) {
      const double2 x = p2[i];
      u[2 * i] = x.x;
      u[2 * i + 1] = x.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < Pd; ++i) u[i] = p[i];
  }
}

// at least two wavefronts per SIMD (at most 256 VGPRs)
template <typename T, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void rhs_stage2d_kernel(
    Mesh M, Async A, Stage S, const double* __restrict__ u_in, const double* u_n, double* out, int src,
    double* __restrict__ ring, const double* __restrict__ ghost) {
  constexpr int Q = P + 1, V = 4, NE = kNE2, Pd = P * P, Qd = Q * Q;
  constexpr ops::Ops<P> O = ops::make_ops<P>();
  // per element: the state at the Gauss points [Qd][V], later the face
  // traces [face s][side][Q][V] of one axis. The element stride is padded so
  // that the 16 elements' 16-byte reads at one offset hit distinct LDS banks
  // (stride = 4 x odd dwords)
  constexpr int PER0 = Qd * V > 16 * Q ? Qd * V : 16 * Q;
  constexpr int PER = sizeof(T) == 8 ? PER0 + (6 - PER0 % 4) % 4 : PER0 + (12 - PER0 % 8) % 8;
  // the same LDS stages the wavefront's output (FP64) in the combine
  constexpr int kXB = NE * PER * (int)sizeof(T), kDB = NE * V * Pd * 8;
  __shared__ __align__(16) unsigned char sRaw[kXB > kDB ? kXB : kDB];
  T* sX = reinterpret_cast<T*>(sRaw);
  double* sD = reinterpret_cast<double*>(sRaw);
  // flux-history modes: per (element, face of the current axis) the
  // face-side offset in the flux ring (or -1) and the delay
  __shared__ long long sFsF[NE * 2];
  __shared__ int sKdF[NE * 2];

  const int lane = threadIdx.x, le = lane >> 2, v = lane & 3;
  const long long e0 = (long long)xcd_block() * NE, e = e0 + le;
  const int ne = M.E - e0 < NE ? (int)(M.E - e0) : NE;
  const bool valid = e < M.E;
  const long long col = (valid ? e : 0) * (V * Pd) + v * Pd;  // this lane's P^2 values

  double u[Pd];
  if (valid) {
    load_col<P>(u_in + col, u);
  } else {
#pragma unroll
    for (int i = 0; i < Pd; ++i) u[i] = 0.0;
  }

  // ---- volume: interpolation to the Gauss points, x then y
  {
    T X[P][Q];
#pragma unroll
    for (int iy = 0; iy < P; ++iy)
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        T acc = (T)O.B[qx][0] * (T)u[iy * P];
#pragma unroll
        for (int ix = 1; ix < P; ++ix) acc = fmx((T)O.B[qx][ix], (T)u[iy * P + ix], acc);
        X[iy][qx] = acc;
      }
    T* dst = sX + le * PER + v;
#pragma unroll
    for (int qy = 0; qy < Q; ++qy)
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        T acc = (T)O.B[qy][0] * X[0][qx];
#pragma unroll
        for (int iy = 1; iy < P; ++iy) acc = fmx((T)O.B[qy][iy], X[iy][qx], acc);
        dst[(qy * Q + qx) * V] = acc;
      }
  }
  __syncthreads();

  // the live neighbour traces, loaded now so that their latency hides behind
  // the volume work. In FP64 all four faces: the neighbour rows one element
  // row away are then read while they are still in L2 (the FP64 kernels run
  // at the same wavefronts per SIMD either way); in FP32 the x faces only,
  // where the extra registers would cost occupancy
  const ElemPos pos = elem_pos(M, valid ? e : 0);
  constexpr int NB = sizeof(T) == 8 ? 4 : 2;
  double nbv[NB][P];
#pragma unroll
  for (int f = 0; f < NB; ++f) {
    const unsigned nb = (unsigned)neighbour_of(M, valid ? e : 0, pos, f);
    const double* gp = u_in + (size_t)nb * (V * Pd) + v * Pd;
#pragma unroll
    for (int j = 0; j < P; ++j) nbv[f][j] = gp[fnode<P>(f ^ 1, j)];
  }

  // ---- volume: flux components of this lane's variable, tested row by row
  T k[Pd];
#pragma unroll
  for (int i = 0; i < Pd; ++i) k[i] = (T)0;
  {
    const T gm1 = (T)M.gamma - (T)1;
    const T sx = (T)(2.0 / M.h[0]), sy = (T)(2.0 / M.h[1]);
    const T e1 = v == 1 ? (T)1 : (T)0, e2 = v == 2 ? (T)1 : (T)0, e3 = v == 3 ? (T)1 : (T)0;
    const T* row = sX + le * PER;
    // one Gauss row per iteration keeps the live state small; the
    // row-dependent operator entries come from a device table laid out by
    // row (one wide scalar load per row)
    const ops::RowOps<P>& OR = ops::kRowOps<P>;
#pragma unroll 1
    for (int qy = 0; qy < Q; ++qy) {
      T tx[P], ty[P];
#pragma unroll
      for (int qx = 0; qx < Q; ++qx) {
        const T* w = row + (qy * Q + qx) * V;
        const T rho = w[0], mx = w[1], my = w[2], en = w[3];
        const T wv = w[v];
        const T ir = recip(rho);
        const T ux = mx * ir, uy = my * ir;
        const T p = gm1 * (en - (T)0.5 * fmx(my, uy, mx * ux));
        const T t = fmx(p, e3, wv);
        // F_x[v] = u_x (w_v + p [v=3]) + p [v=1], F_y alike
        const T fx = fmx(ux, t, p * e1);
        const T fy = fmx(uy, t, p * e2);
#pragma unroll
        for (int i = 0; i < P; ++i) {
          if (qx == 0) {
            tx[i] = (T)O.GW[i][0] * fx;
            ty[i] = (T)O.BW[i][0] * fy;
          } else {
            tx[i] = fmx((T)O.GW[i][qx], fx, tx[i]);
            ty[i] = fmx((T)O.BW[i][qx], fy, ty[i]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < P; ++i) {
        tx[i] *= sx;
        ty[i] *= sy;
      }
#pragma unroll
      for (int iy = 0; iy < P; ++iy) {
        const T bw = (T)OR.r[qy][1][iy], gw = (T)OR.r[qy][2][iy];
#pragma unroll
        for (int ix = 0; ix < P; ++ix) k[iy * P + ix] = fmx(gw, ty[ix], fmx(bw, tx[ix], k[iy * P + ix]));
      }
    }
  }

  // ---- per-face neighbour data: element, PE face-side, delay
  const bool async_on = src != kSrcLive && M.nfs > 0;
  const bool flux_mode = src == kSrcFlux;
  const long long ring_level = M.nfs * V * (flux_mode ? Q : P);  // values per ring level
  const bool publish = src == kSrcRing && A.stage == 0;

  // u^n for the combine (SSP stages 2 and 3; the accumulator w of the LSERK
  // stages after the first), loaded at the start of the last face pass so
  // that its latency hides behind the y faces (FP64, degree <= 3: elsewhere
  // the registers would cost occupancy, and the SSP combine moves u^n into
  // LDS with direct loads instead). Only this element reads its column of
  // u_n, and it writes it only in the combine.
  constexpr bool kEarlyUn = sizeof(T) == 8 && P <= 4;
  double un[Pd];
  const bool need_un = kEarlyUn && valid && (S.lserk ? u_n != u_in : S.a != 0.0);

  // ---- faces, one axis per pass
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    if (a == 1 && need_un) load_col<P>(u_n + col, un);
    __syncthreads();  // sX is rewritten
    // own and neighbour traces of variable v at the Gauss points of both faces
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int f = 2 * a + s;
      double g[P];  // neighbour trace at the face nodes
#pragma unroll
      for (int j = 0; j < P; ++j) g[j] = 0.0;
      long long fs = -1;
      int kd = 0;
      if (valid) {
        fs = async_on ? face_side_at(M, pos, f) : -1;
        if (fs >= 0 && (src == kSrcRing || flux_mode)) kd = delay_of(M, A, sub_at(M, pos.sc), f);
        if (fs >= 0 && publish) {
          double* dst = ring + A.slot_n * ring_level + fed_face_side(M, pos, f) * V * P + v * P;
#pragma unroll
          for (int j = 0; j < P; ++j) dst[j] = u[fnode<P>(f, j)];
        }
        const int bf = bnd_face_at(M, pos, f);
        if (bf >= 0) {
          // boundary face of a Dirichlet box: the exact exterior state
          const double* gp = S.bnd + ((long long)bf * V + v) * P;
#pragma unroll
          for (int j = 0; j < P; ++j) g[j] = gp[j];
        } else if (fs < 0 || ((src == kSrcRing || flux_mode) && kd == 0)) {
          if (NB == 4 || a == 0) {
#pragma unroll
            for (int j = 0; j < P; ++j) g[j] = nbv[NB == 4 ? f : s][j];
          } else {
            const unsigned nb = (unsigned)neighbour_of(M, e, pos, f);
            const double* gp = u_in + (size_t)nb * (V * Pd) + v * Pd;
#pragma unroll
            for (int j = 0; j < P; ++j) g[j] = gp[fnode<P>(f ^ 1, j)];
          }
        } else if (flux_mode) {
          // silent step: the face uses the stored flux, no trace needed
        } else if (src == kSrcGhost) {
          const double* gp = ghost + fs * V * P + v * P;
#pragma unroll
          for (int j = 0; j < P; ++j) g[j] = gp[j];
        } else if (A.ghost == 1) {
          // standard flux on the trace kd steps old (eq. delayed-flux)
          const double* gp = ring + ring_slot(A, kd) * ring_level + fs * V * P + v * P;
#pragma unroll
          for (int j = 0; j < P; ++j) g[j] = gp[j];
        } else {
          // AT extrapolation to the stage time, tau = kd + c_m (eq. at-flux)
          const double tau = kd + A.c_m;
          // at most kMaxLevels levels; past A.levels the newest is read again
          // with weight 0, so every load is issued before the first is used
#pragma unroll
          for (int l = 0; l < kMaxLevels; ++l) {
            const bool on = l < A.levels;
            const double wl = on ? at_weight(l, A.levels, tau) : 0.0;
            const double* gp = ring + ring_slot(A, kd + (on ? l : 0)) * ring_level + fs * V * P + v * P;
#pragma unroll
            for (int j = 0; j < P; ++j) g[j] = fma(wl, gp[j], g[j]);
          }
        }
      }
      if (flux_mode && v == 0) {
        sFsF[le * 2 + s] = fs;
        sKdF[le * 2 + s] = kd;
      }
      T* dst = sX + le * PER + s * (2 * Q * V) + v;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        T o = (T)O.B[q][0] * (T)u[fnode<P>(f, 0)];
        T n = (T)O.B[q][0] * (T)g[0];
#pragma unroll
        for (int j = 1; j < P; ++j) {
          o = fmx((T)O.B[q][j], (T)u[fnode<P>(f, j)], o);
          n = fmx((T)O.B[q][j], (T)g[j], n);
        }
        dst[q * V] = o;
        dst[(Q + q) * V] = n;
      }
    }
    __syncthreads();
    // numerical flux, one lane per (element, face, point), in place of the
    // own trace, scaled by -(n.e_a) 2/h_a
    {
      const T gamma = (T)M.gamma;
      const T sc = (T)(2.0 / M.h[a]);
#pragma unroll
      for (int it = 0; it < (NE * 2 * Q + 63) / 64; ++it) {
        const int t = lane + 64 * it;
        if (t < NE * 2 * Q) {
          const int q = t % Q, s = (t / Q) & 1, el = t / (2 * Q);
          T* base = sX + el * PER + s * (2 * Q * V);
          // own trace at [q], neighbour's at [Q + q]; the +a face (s = 1)
          // has the own side on the left
          const T* pl = base + (s ? q : Q + q) * V;
          const T* pr = base + (s ? Q + q : q) * V;
          T wl[4], wr[4], G[4];
#pragma unroll
          for (int vv = 0; vv < 4; ++vv) {
            wl[vv] = pl[vv];
            wr[vv] = pr[vv];
          }
          const long long ffs = flux_mode ? sFsF[el * 2 + s] : -1;
          const int fkd = flux_mode ? sKdF[el * 2 + s] : 0;
          if (ffs >= 0 && fkd > 0) {
            // silent step of Alg. caa-std / caa-at: the stored flux, or its
            // AT extrapolation to the stage time tau = k + c_m (FP64)
            const double* fp = ring + ffs * V * Q + q;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            if (A.ghost == 4) {
#pragma unroll
              for (int vv = 0; vv < 4; ++vv) acc[vv] = fp[ring_slot(A, fkd) * ring_level + vv * Q];
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
                for (int vv = 0; vv < 4; ++vv) acc[vv] = fma(w, lp[vv * Q], acc[vv]);
              }
            }
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) G[vv] = (T)acc[vv];
          } else {
            num_flux<T, 2>(wl, wr, a, gamma, M.flux, G);
            // communicating step of a flux-history mode: keep the stage-0 flux
            if (ffs >= 0 && A.stage == 0) {
              double* fp = ring + A.slot_n * ring_level + ffs * V * Q + q;
#pragma unroll
              for (int vv = 0; vv < 4; ++vv) fp[vv * Q] = (double)G[vv];
            }
          }
          const T sg = s ? -sc : sc;
#pragma unroll
          for (int vv = 0; vv < 4; ++vv) base[q * V + vv] = sg * G[vv];
        }
      }
    }
    __syncthreads();
    // lift: t_j = sum_q BW[j][q] G_q, then k(i_a, j) += MC_s[i_a] t_j
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T* gsrc = sX + le * PER + s * (2 * Q * V) + v;
      T G[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) G[q] = gsrc[q * V];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        T tj = (T)O.BW[j][0] * G[0];
#pragma unroll
        for (int q = 1; q < Q; ++q) tj = fmx((T)O.BW[j][q], G[q], tj);
#pragma unroll
        for (int ia = 0; ia < P; ++ia) {
          const int node = a == 0 ? j * P + ia : ia * P + j;
          k[node] = fmx((T)O.MC[s][ia], tj, k[node]);
        }
      }
    }
  }

  // ---- the stage combine in FP64; each output goes through LDS (the lane
  // writes its column there) and leaves as one coalesced range
  __syncthreads();  // sX is rewritten
  double* o = sD + (le * V + v) * Pd;
  if (S.lserk) {
    // LSERK: u_n holds the accumulator w (read before either write); at the
    // first stage it is the stage input itself, already in registers
    double wv[Pd];
    if (valid) {
      if (u_n == u_in) {
#pragma unroll
        for (int i = 0; i < Pd; ++i) wv[i] = u[i];
      } else if (kEarlyUn) {
#pragma unroll
        for (int i = 0; i < Pd; ++i) wv[i] = un[i];
      } else {
        load_col<P>(u_n + col, wv);
      }
#pragma unroll
      for (int i = 0; i < Pd; ++i) o[i] = wv[i] + S.dt * S.bw * (double)k[i];
    }
    __syncthreads();
    wave_stream_out<NE * V * Pd>(out + e0 * V * Pd, sD, ne * V * Pd);
    if (S.out2) {
      __syncthreads();  // the first output has left LDS
      if (valid) {
#pragma unroll
        for (int i = 0; i < Pd; ++i) o[i] = wv[i] + S.dt * S.ar * (double)k[i];
      }
      __syncthreads();
      wave_stream_out<NE * V * Pd>(S.out2 + e0 * V * Pd, sD, ne * V * Pd);
    }
  } else {
    if (!kEarlyUn && S.a != 0.0) {
      wave_stream_in<NE * V * Pd>(sD, u_n + e0 * V * Pd, ne * V * Pd);
      __syncthreads();
    }
    if (valid) {
      if (S.a == 0.0) {
#pragma unroll
        for (int i = 0; i < Pd; ++i) o[i] = S.b * (u[i] + S.dt * (double)k[i]);
      } else if (!kEarlyUn) {
#pragma unroll
        for (int i = 0; i < Pd; ++i) o[i] = S.a * o[i] + S.b * (u[i] + S.dt * (double)k[i]);
      } else {
#pragma unroll
        for (int i = 0; i < Pd; ++i) o[i] = S.a * un[i] + S.b * (u[i] + S.dt * (double)k[i]);
      }
    }
    __syncthreads();
    wave_stream_out<NE * V * Pd>(out + e0 * V * Pd, sD, ne * V * Pd);
  }
}

template <typename T, int P>
hipError_t launch2d(const Mesh& M, const Async& A, const Stage& S, const double* u_in, const double* u_n,
                    double* out, int src, double* ring, const double* ghost, hipStream_t st) {
  const long long nblk = (M.E + kNE2 - 1) / kNE2;
  hipLaunchKernelGGL((rhs_stage2d_kernel<T, P>), dim3((unsigned)nblk), dim3(64), 0, st, M, A, S, u_in, u_n, out, src,
                     ring, ghost);
  return hipGetLastError();
}

template <typename T>
hipError_t launch2d_prec(int degree, const Mesh& M, const Async& A, const Stage& S, const double* u_in,
                         const double* u_n, double* out, int src, double* ring, const double* ghost, hipStream_t st) {
  switch (degree) {
    case 1: return launch2d<T, 2>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
    case 2: return launch2d<T, 3>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
    case 3: return launch2d<T, 4>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
    case 4: return launch2d<T, 5>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_rhs_stage_2d(int degree, int precision, const Mesh& M, const Async& A, const Stage& S,
                               const double* u_in, const double* u_n, double* out, int src, double* ring,
                               const double* ghost, hipStream_t st) {
  if (M.dim != 2) return hipErrorInvalidValue;
  if (precision == 1) return launch2d_prec<float>(degree, M, A, S, u_in, u_n, out, src, ring, ghost, st);
  return launch2d_prec<double>(degree, M, A, S, u_in, u_n, out, src, ring, ghost, st);
}

}  // namespace adg
