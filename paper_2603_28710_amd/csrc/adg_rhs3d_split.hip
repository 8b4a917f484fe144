// adg_rhs3d_split.hip — the fused SSP-RK3 stage on hexahedra of degree 3,
// with the element data in registers split over pairs of lanes.
//
// At P = 4 one lane cannot hold the 64 nodal values and 64 residuals of a
// variable (256 FP64 registers). Here the two lanes (e, v, h), h = 0, 1, of a
// pair share variable v of element e: lane h keeps the node rows iy = 2h and
// 2h + 1 for every iz (32 values and their residuals). The pair are adjacent
// lanes of one quad and exchange partial results with DPP moves. One
// wavefront owns 6 consecutive elements (x fastest); lanes 60-63 idle.
//
//   volume: one Gauss plane q_z at a time. Each lane combines its rows
//           along z and interpolates them in x, swaps them with its partner
//           (the pair then holds all four rows) and interpolates in y to the
//           Gauss rows q_y = 2r + h, which it stores. For each own Gauss row
//           it reads the full state, forms its flux components F_x[v],
//           F_y[v], F_z[v] (eq. euler-dealii) and tests them:
//             A(iy, ix) = sum_qy BW[iy][qy] sx (GW F_x)(ix) + GW[iy][qy] sy (BW F_y)(ix)
//             C(iy, ix) = sum_qy BW[iy][qy] sz (BW F_z)(ix),
//           for its own rows and, separately, the partner's; the pair then
//           swaps the partner parts, and each lane adds
//             k(iz, iy, ix) += BW[iz][qz] A(iy, ix) + GW[iz][qz] C(iy, ix)
//           (BW = M1^{-1} B^T W, GW = M1^{-1} B^T D^T W;
//           eq. weakform-dealii / weakform-compact-dealii).
//   faces:  one face at a time, the pair splitting its two sides: lane 0
//           reads the own face nodes (again, from the stage input) and
//           publishes them, lane 1 builds the neighbour trace; each
//           interpolates its side to the face's Gauss points. One lane per
//           (element, point) evaluates the LLF flux (eq. lfflux /
//           lfflux-lambda) in canonical (left, right) order; each lane lifts
//           its variable with BW along both tangential axes onto the face
//           nodes of its own rows and adds the column of M1^{-1} at that face.
//   stage:  out = a u_n + b (u_in + dt k) in FP64, written to LDS and
//           stored as one coalesced, streamed range.
//
// The ring publish (stage 0), the delay schedule, the AT extrapolation, the
// learned ghosts and the flux history follow the same rules as the other
// stage kernels. T = double (FP64) or float (FP32 contractions).
#include <type_traits>

#include "adg_device.h"
#include "adg_internal.h"
#include "adg_tables.h"

namespace adg {

namespace {

constexpr int kNES = 6;  // elements per wavefront (V = 5 pairs of lanes each)

// the value held by the other lane of this lane's pair (quad permutation
// [1, 0, 3, 2]); every lane of the wavefront must be active
__device__ __forceinline__ int pair_swap_i(int x) { return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ float pair_swap(float x) { return __int_as_float(pair_swap_i(__float_as_int(x))); }
__device__ __forceinline__ double pair_swap(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = pair_swap_i((int)(b & 0xffffffffLL));
  const int hi = pair_swap_i((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// node index (x fastest) with coordinate ia along axis a and coordinates
// (j0, j1) along the other two axes in ascending order
template <int P>
__device__ __forceinline__ constexpr int nodeS(int a, int ia, int j0, int j1) {
  return a == 0 ? ia + P * (j0 + P * j1) : (a == 1 ? j0 + P * (ia + P * j1) : j0 + P * (j1 + P * ia));
}

template <typename T, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void rhs_stage3d_split_kernel(Mesh M, Async A, Stage S,
                                                               const double* __restrict__ u_in, const double* u_n,
                                                               double* out, int src, double* __restrict__ ring,
                                                               const double* __restrict__ ghost) {
  static_assert(P == 4, "the pair split assumes four node rows");
  constexpr int Q = P + 1, V = 5, NE = kNES, Pd = P * P * P, Fn = P * P, Fq = Q * Q;
  constexpr int NR = (Q + 1) / 2;  // own Gauss rows per lane: q = 2r + h
  constexpr int NU = 2 * P * P;    // own nodal values: u[(iz * 2 + jj) * P + ix], iy = 2h + jj
  constexpr ops::Ops<P> O = ops::make_ops<P>();
  // per element: the state at the points of one Gauss plane [Fq][V] during
  // the volume, the own and neighbour traces of one face [2][Fq][V] during
  // the faces; one spare element slot for the idle lanes; the stride is
  // padded so 16-byte reads of consecutive elements spread over the banks
  constexpr int PER0 = 2 * Fq * V;
  constexpr int PER = sizeof(T) == 8 ? PER0 + (6 - PER0 % 4) % 4 : PER0 + (12 - PER0 % 8) % 8;
  // the same LDS stages the wavefront's output (FP64) in the combine
  constexpr int kXB = (NE + 1) * PER * (int)sizeof(T), kDB = NE * V * Pd * 8;
  __shared__ __align__(16) unsigned char sRaw[kXB > kDB ? kXB : kDB];
  T* sX = reinterpret_cast<T*>(sRaw);
  double* sD = reinterpret_cast<double*>(sRaw);
  __shared__ long long sFsF[NE + 1];  // flux-history modes: face-side of the current face, or -1
  __shared__ int sKdF[NE + 1];        // and its delay

  const int lane = threadIdx.x, le = lane / (2 * V), rem = lane - le * 2 * V, v = rem >> 1, h = rem & 1;
  const long long e0 = (long long)xcd_block() * NE, e = e0 + le;
  const int ne = M.E - e0 < NE ? (int)(M.E - e0) : NE;
  const bool valid = le < NE && e < M.E;
  const long long col = (valid ? e : 0) * (V * Pd) + v * Pd;  // this lane's variable
  const bool hi = h != 0;

  // own rows iy = 2h, 2h + 1 of every z-plane: 8 consecutive values per plane
  double u[NU];
#pragma unroll
  for (int iz = 0; iz < P; ++iz) {
    if (valid) {
      const double2* p2 = reinterpret_cast<const double2*>(u_in + col + iz * P * P + 2 * h * P);
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const double2 x = p2[i];
        u[iz * 2 * P + 2 * i] = x.x;
        u[iz * 2 * P + 2 * i + 1] = x.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 2 * P; ++i) u[iz * 2 * P + i] = 0.0;
    }
  }

  T k[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) k[i] = (T)0;
  T* mine = sX + le * PER;

  // ---- volume, one Gauss plane q_z at a time
  {
    const T gm1 = (T)M.gamma - (T)1;
    const T sx = (T)(2.0 / M.h[0]), sy = (T)(2.0 / M.h[1]), sz = (T)(2.0 / M.h[2]);
    const T e1 = v == 1 ? (T)1 : (T)0, e2 = v == 2 ? (T)1 : (T)0, e3 = v == 3 ? (T)1 : (T)0;
    const T e4 = v == 4 ? (T)1 : (T)0;
    const ops::RowOps<P>& OR = ops::kRowOps<P>;  // entries indexed at run time, by Gauss plane
#pragma unroll 1
    for (int qz = 0; qz < Q; ++qz) {
      if (qz) __syncthreads();  // the previous plane has been read
      // the lane-dependent weights below are selected anew in every plane
      // (an opaque copy of h), not kept in registers across the loop
      int hv = h;
      asm volatile("" : "+v"(hv));
      const bool hl = hv != 0;
      // own rows: combine along z, then interpolate along x
      T Xo[2][Q];
      {
        T bz[P];
#pragma unroll
        for (int i = 0; i < P; ++i) bz[i] = (T)OR.r[qz][0][i];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          T Z[P];
#pragma unroll
          for (int ix = 0; ix < P; ++ix) {
            T acc = bz[0] * (T)u[jj * P + ix];
#pragma unroll
            for (int iz = 1; iz < P; ++iz) acc = fmx(bz[iz], (T)u[(iz * 2 + jj) * P + ix], acc);
            Z[ix] = acc;
          }
#pragma unroll
          for (int qx = 0; qx < Q; ++qx) {
            T acc = (T)O.B[qx][0] * Z[0];
#pragma unroll
            for (int ix = 1; ix < P; ++ix) acc = fmx((T)O.B[qx][ix], Z[ix], acc);
            Xo[jj][qx] = acc;
          }
        }
      }
      // y to the own Gauss rows q_y = 2r + h from the own rows and the
      // partner's (weights chosen per lane instead of reordering the rows)
      {
        T Xp[2][Q];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
          for (int qx = 0; qx < Q; ++qx) Xp[jj][qx] = pair_swap(Xo[jj][qx]);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const int qy = 2 * r + h;
          const int r1 = 2 * r + 1 < Q ? 2 * r + 1 : 0;
          T bo[2], bp[2];  // B[q_y][iy] for the own rows iy = 2h + jj and the partner's
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            bo[jj] = hl ? (T)O.B[r1][2 + jj] : (T)O.B[2 * r][jj];
            bp[jj] = hl ? (T)O.B[r1][jj] : (T)O.B[2 * r][2 + jj];
          }
          if (qy < Q) {
#pragma unroll
            for (int qx = 0; qx < Q; ++qx) {
              const T acc = fmx(bp[1], Xp[1][qx], fmx(bp[0], Xp[0][qx], fmx(bo[1], Xo[1][qx], bo[0] * Xo[0][qx])));
              mine[(qy * Q + qx) * V + v] = acc;
            }
          }
        }
      }
      __syncthreads();
      // flux components of this lane's variable on its Gauss rows, tested
      T bwz[P], gwz[P];
#pragma unroll
      for (int iz = 0; iz < P; ++iz) {
        bwz[iz] = (T)OR.r[qz][1][iz];
        gwz[iz] = (T)OR.r[qz][2][iz];
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int qy = 2 * r + h;
        // a row past the plane (h = 1, odd Q) reads the last row and adds
        // nothing: its weights below are zero
        const T* wrow = mine + (qy < Q ? qy : Q - 1) * Q * V;
        T tx[P], ty[P], tz[P];
#pragma unroll
        for (int qx = 0; qx < Q; ++qx) {
          const T* w = wrow + qx * V;
          const T rho = w[0], mx = w[1], my = w[2], mz = w[3], en = w[4];
          const T wv = w[v];
          const T ir = recip(rho);
          const T ux = mx * ir, uy = my * ir, uz = mz * ir;
          const T p = gm1 * (en - (T)0.5 * fmx(mz, uz, fmx(my, uy, mx * ux)));
          const T t = fmx(p, e4, wv);
          // F_a[v] = u_a (w_v + p [v=4]) + p [v=1+a]
          const T fx = fmx(ux, t, p * e1), fy = fmx(uy, t, p * e2), fz = fmx(uz, t, p * e3);
#pragma unroll
          for (int i = 0; i < P; ++i) {
            if (qx == 0) {
              tx[i] = (T)O.GW[i][0] * fx;
              ty[i] = (T)O.BW[i][0] * fy;
              tz[i] = (T)O.BW[i][0] * fz;
            } else {
              tx[i] = fmx((T)O.GW[i][qx], fx, tx[i]);
              ty[i] = fmx((T)O.BW[i][qx], fy, ty[i]);
              tz[i] = fmx((T)O.BW[i][qx], fz, tz[i]);
            }
          }
        }
        // the partner's row of this round (q_y = 2r + 1 - h)
        T px[P], py[P], pz[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
          tx[i] *= sx;
          ty[i] *= sy;
          tz[i] *= sz;
          px[i] = pair_swap(tx[i]);
          py[i] = pair_swap(ty[i]);
          pz[i] = pair_swap(tz[i]);
        }
        // weights for the own node rows iy = 2h + jj of the own Gauss row
        // and of the partner's: the even row 2r belongs to lane 0, the odd
        // row 2r + 1 (if any) to lane 1
        const int r1 = 2 * r + 1 < Q ? 2 * r + 1 : 0;
        const T zr = 2 * r + 1 < Q ? (T)1 : (T)0;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const T bwo = hl ? zr * (T)O.BW[2 + jj][r1] : (T)O.BW[jj][2 * r];
          const T gwo = hl ? zr * (T)O.GW[2 + jj][r1] : (T)O.GW[jj][2 * r];
          const T bwp = hl ? (T)O.BW[2 + jj][2 * r] : zr * (T)O.BW[jj][r1];
          const T gwp = hl ? (T)O.GW[2 + jj][2 * r] : zr * (T)O.GW[jj][r1];
#pragma unroll
          for (int ix = 0; ix < P; ++ix) {
            const T ab = fmx(gwp, py[ix], fmx(bwp, px[ix], fmx(gwo, ty[ix], bwo * tx[ix])));
            const T c = fmx(bwp, pz[ix], bwo * tz[ix]);
#pragma unroll
            for (int iz = 0; iz < P; ++iz) {
              const int n = (iz * 2 + jj) * P + ix;
              k[n] = fmx(gwz[iz], c, fmx(bwz[iz], ab, k[n]));
            }
          }
        }
      }
    }
  }

  // ---- faces, one face at a time
  const ElemPos pos = elem_pos(M, valid ? e : 0);
  const bool async_on = src != kSrcLive && M.nfs > 0;
  const bool flux_mode = src == kSrcFlux;
  const long long ring_level = M.nfs * V * (flux_mode ? Fq : Fn);  // values per ring level
  const bool publish = src == kSrcRing && A.stage == 0;
  auto face_pass = [&](auto fc) {
    constexpr int f = decltype(fc)::value;
    constexpr int a = f >> 1, s = f & 1, ia = s ? P - 1 : 0;
    __syncthreads();  // sX is rewritten
    // The pair splits the two sides of the face: lane h = 0 reads the own
    // trace (the face nodes of the stage input, an L2 hit) and publishes it,
    // lane h = 1 builds the neighbour trace (live values; the delayed / AT /
    // learned trace at a PE-boundary face). Face nodes j = j0 + P j1.
    double g[Fn];
#pragma unroll
    for (int j = 0; j < Fn; ++j) g[j] = 0.0;
    long long fs = -1;
    int kd = 0;
    if (valid) {
      fs = async_on ? face_side_at(M, pos, f) : -1;
      if (fs >= 0 && (src == kSrcRing || flux_mode)) kd = delay_of(M, A, sub_at(M, pos.sc), f);
      if (h == 0) {
#pragma unroll
        for (int j = 0; j < Fn; ++j) g[j] = u_in[col + nodeS<P>(a, ia, j % P, j / P)];
        if (fs >= 0 && publish) {
          double* dst = ring + A.slot_n * ring_level + fed_face_side(M, pos, f) * V * Fn + v * Fn;
#pragma unroll
          for (int j = 0; j < Fn; ++j) dst[j] = g[j];
        }
      } else if (fs < 0 || ((src == kSrcRing || flux_mode) && kd == 0)) {
        const unsigned nb = (unsigned)neighbour_of(M, e, pos, f);
        const double* gp = u_in + (size_t)nb * (V * Pd) + v * Pd;
#pragma unroll
        for (int j = 0; j < Fn; ++j) g[j] = gp[nodeS<P>(a, P - 1 - ia, j % P, j / P)];
      } else if (flux_mode) {
        // silent step: the face uses the stored flux, no trace needed
      } else if (src == kSrcGhost) {
        const double* gp = ghost + fs * V * Fn + v * Fn;
#pragma unroll
        for (int j = 0; j < Fn; ++j) g[j] = gp[j];
      } else if (A.ghost == 1) {
        // standard flux on the trace kd steps old (eq. delayed-flux)
        const double* gp = ring + ring_slot(A, kd) * ring_level + fs * V * Fn + v * Fn;
#pragma unroll
        for (int j = 0; j < Fn; ++j) g[j] = gp[j];
      } else {
        // AT extrapolation to the stage time, tau = kd + c_m (eq. at-flux)
        const double tau = kd + A.c_m;
        if constexpr (a == 0) {
          // the x faces: at most kMaxLevels levels, past A.levels the newest
          // is read again with weight 0, so every level's loads are in
          // flight together (in the y and z passes the extra registers
          // would spill)
#pragma unroll
          for (int l = 0; l < kMaxLevels; ++l) {
            const bool on = l < A.levels;
            const double wl = on ? at_weight(l, A.levels, tau) : 0.0;
            const double* gp = ring + ring_slot(A, kd + (on ? l : 0)) * ring_level + fs * V * Fn + v * Fn;
#pragma unroll
            for (int j = 0; j < Fn; ++j) g[j] = fma(wl, gp[j], g[j]);
          }
        } else {
          for (int l = 0; l < A.levels; ++l) {
            const double wl = at_weight(l, A.levels, tau);
            const double* gp = ring + ring_slot(A, kd + l) * ring_level + fs * V * Fn + v * Fn;
#pragma unroll
            for (int j = 0; j < Fn; ++j) g[j] = fma(wl, gp[j], g[j]);
          }
        }
      }
    }
    if (flux_mode && v == 0 && h == 0) {
      sFsF[le] = fs;
      sKdF[le] = kd;
    }
    // this lane's side of the trace at the Gauss points (q0 + Q q1)
    {
      T X[P][Q];
#pragma unroll
      for (int j1 = 0; j1 < P; ++j1)
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) {
          T acc = (T)O.B[q0][0] * (T)g[j1 * P];
#pragma unroll
          for (int j0 = 1; j0 < P; ++j0) acc = fmx((T)O.B[q0][j0], (T)g[j1 * P + j0], acc);
          X[j1][q0] = acc;
        }
      T* dst = mine + h * Fq * V + v;
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) {
          T acc = (T)O.B[q1][0] * X[0][q0];
#pragma unroll
          for (int j1 = 1; j1 < P; ++j1) acc = fmx((T)O.B[q1][j1], X[j1][q0], acc);
          dst[(q1 * Q + q0) * V] = acc;
        }
    }
    __syncthreads();
    // numerical flux, one lane per (element, face point), in place of the
    // own trace, scaled by -(n.e_a) 2/h_a
    {
      const T gamma = (T)M.gamma;
      const T sc = (T)(2.0 / M.h[a]);
#pragma unroll
      for (int it = 0; it < (NE * Fq + 63) / 64; ++it) {
        const int t = lane + 64 * it;
        if (t < NE * Fq) {
          const int el = t / Fq, m = t - el * Fq;
          T* base = sX + el * PER;
          const T* pl = base + (s ? m : Fq + m) * V;  // the +a face has the own side on the left
          const T* pr = base + (s ? Fq + m : m) * V;
          T wl[V], wr[V], G[V];
#pragma unroll
          for (int vv = 0; vv < V; ++vv) {
            wl[vv] = pl[vv];
            wr[vv] = pr[vv];
          }
          const long long ffs = flux_mode ? sFsF[el] : -1;
          const int fkd = flux_mode ? sKdF[el] : 0;
          if (ffs >= 0 && fkd > 0) {
            // silent step of Alg. caa-std / caa-at: the stored flux, or its
            // AT extrapolation to the stage time tau = k + c_m (FP64)
            const double* fp = ring + ffs * V * Fq + m;
            double acc[V];
#pragma unroll
            for (int vv = 0; vv < V; ++vv) acc[vv] = 0.0;
            if (A.ghost == 4) {
#pragma unroll
              for (int vv = 0; vv < V; ++vv) acc[vv] = fp[ring_slot(A, fkd) * ring_level + vv * Fq];
            } else {
              const double tau = fkd + A.c_m;
              for (int l = 0; l < A.levels; ++l) {
                const double w = at_weight(l, A.levels, tau);
                const double* lp = fp + ring_slot(A, fkd + l) * ring_level;
#pragma unroll
                for (int vv = 0; vv < V; ++vv) acc[vv] = fma(w, lp[vv * Fq], acc[vv]);
              }
            }
#pragma unroll
            for (int vv = 0; vv < V; ++vv) G[vv] = (T)acc[vv];
          } else {
            num_flux<T, 3>(wl, wr, a, gamma, M.flux, G);
            // communicating step of a flux-history mode: keep the stage-0 flux
            if (ffs >= 0 && A.stage == 0) {
              double* fp = ring + A.slot_n * ring_level + ffs * V * Fq + m;
#pragma unroll
              for (int vv = 0; vv < V; ++vv) fp[vv * Fq] = (double)G[vv];
            }
          }
          const T sg = s ? -sc : sc;
#pragma unroll
          for (int vv = 0; vv < V; ++vv) base[m * V + vv] = sg * G[vv];
        }
      }
    }
    __syncthreads();
    // lift with BW along both tangential axes onto the own face nodes, then
    // k(i_a, j0, j1) += MC_s[i_a] * lifted(j0, j1)
    if constexpr (a == 1) {
      // the face's 16 lifted values serve both lanes' rows
      T L0[Q][P];
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        T G[Q];
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) G[q0] = mine[(q1 * Q + q0) * V + v];
#pragma unroll
        for (int j0 = 0; j0 < P; ++j0) {
          T acc = (T)O.BW[j0][0] * G[0];
#pragma unroll
          for (int q0 = 1; q0 < Q; ++q0) acc = fmx((T)O.BW[j0][q0], G[q0], acc);
          L0[q1][j0] = acc;
        }
      }
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const T mc = hi ? (T)O.MC[s][2 + jj] : (T)O.MC[s][jj];
#pragma unroll
        for (int j1 = 0; j1 < P; ++j1)
#pragma unroll
          for (int j0 = 0; j0 < P; ++j0) {
            T lf = (T)O.BW[j1][0] * L0[0][j0];
#pragma unroll
            for (int q1 = 1; q1 < Q; ++q1) lf = fmx((T)O.BW[j1][q1], L0[q1][j0], lf);
            const int n = (j1 * 2 + jj) * P + j0;  // iz = j1, iy = 2h + jj, ix = j0
            k[n] = fmx(mc, lf, k[n]);
          }
      }
    } else {
      // the axis the lane holds whole first (a = 0: q1 -> j1 = iz; a = 2:
      // q0 -> j0 = ix), then the split axis onto the own rows jj
      T L0[Q][P];  // [q along the split axis][index along the whole axis]
#pragma unroll
      for (int qs = 0; qs < Q; ++qs) {
        T G[Q];
#pragma unroll
        for (int qw = 0; qw < Q; ++qw) {
          const int m = a == 0 ? qs + Q * qw : qw + Q * qs;
          G[qw] = mine[m * V + v];
        }
#pragma unroll
        for (int jw = 0; jw < P; ++jw) {
          T acc = (T)O.BW[jw][0] * G[0];
#pragma unroll
          for (int qw = 1; qw < Q; ++qw) acc = fmx((T)O.BW[jw][qw], G[qw], acc);
          L0[qs][jw] = acc;
        }
      }
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        T bws[Q];
#pragma unroll
        for (int qs = 0; qs < Q; ++qs) bws[qs] = hi ? (T)O.BW[2 + jj][qs] : (T)O.BW[jj][qs];
#pragma unroll
        for (int jw = 0; jw < P; ++jw) {
          T lf = bws[0] * L0[0][jw];
#pragma unroll
          for (int qs = 1; qs < Q; ++qs) lf = fmx(bws[qs], L0[qs][jw], lf);
#pragma unroll
          for (int i = 0; i < P; ++i) {
            // a = 0: iz = jw, ix = i; a = 2: iz = i, ix = jw
            const int n = a == 0 ? (jw * 2 + jj) * P + i : (i * 2 + jj) * P + jw;
            k[n] = fmx((T)O.MC[s][i], lf, k[n]);
          }
        }
      }
    }
  };
  face_pass(std::integral_constant<int, 0>{});
  face_pass(std::integral_constant<int, 1>{});
  face_pass(std::integral_constant<int, 2>{});
  face_pass(std::integral_constant<int, 3>{});
  face_pass(std::integral_constant<int, 4>{});
  face_pass(std::integral_constant<int, 5>{});

  // ---- the stage combine in FP64 (the stage input read again, an L2 hit);
  // each output goes through LDS (the lane writes its rows there) and leaves
  // as one coalesced range
  __syncthreads();  // sX is rewritten
  double* od = sD + (le * V + v) * Pd + 2 * h * P;
  if (S.lserk) {
    // LSERK: u_n holds the accumulator w (read before either write)
    if (valid) {
#pragma unroll
      for (int iz = 0; iz < P; ++iz) {
        const double* un = u_n + col + iz * P * P + 2 * h * P;
#pragma unroll
        for (int i = 0; i < 2 * P; ++i) od[iz * P * P + i] = un[i] + S.dt * S.bw * (double)k[iz * 2 * P + i];
      }
    }
    __syncthreads();
    wave_stream_out<NE * V * Pd>(out + e0 * V * Pd, sD, ne * V * Pd);
    if (S.out2) {
      __syncthreads();  // the first output has left LDS
      if (valid) {
#pragma unroll
        for (int iz = 0; iz < P; ++iz) {
          const double* un = u_n + col + iz * P * P + 2 * h * P;
#pragma unroll
          for (int i = 0; i < 2 * P; ++i) od[iz * P * P + i] = un[i] + S.dt * S.ar * (double)k[iz * 2 * P + i];
        }
      }
      __syncthreads();
      wave_stream_out<NE * V * Pd>(S.out2 + e0 * V * Pd, sD, ne * V * Pd);
    }
  } else {
    if (valid) {
#pragma unroll
      for (int iz = 0; iz < P; ++iz) {
        const double* ui = u_in + col + iz * P * P + 2 * h * P;
        const double* un = u_n + col + iz * P * P + 2 * h * P;
#pragma unroll
        for (int i = 0; i < 2 * P; ++i) {
          const int n = iz * 2 * P + i;
          od[iz * P * P + i] = S.a == 0.0 ? S.b * (ui[i] + S.dt * (double)k[n])
                                          : S.a * un[i] + S.b * (ui[i] + S.dt * (double)k[n]);
        }
      }
    }
    __syncthreads();
    wave_stream_out<NE * V * Pd>(out + e0 * V * Pd, sD, ne * V * Pd);
  }
}

template <typename T>
hipError_t launch_split(const Mesh& M, const Async& A, const Stage& S, const double* u_in, const double* u_n,
                        double* out, int src, double* ring, const double* ghost, hipStream_t st) {
  const long long nblk = (M.E + kNES - 1) / kNES;
  hipLaunchKernelGGL((rhs_stage3d_split_kernel<T, 4>), dim3((unsigned)nblk), dim3(64), 0, st, M, A, S, u_in, u_n,
                     out, src, ring, ghost);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rhs_stage_3d_split(int degree, int precision, const Mesh& M, const Async& A, const Stage& S,
                                     const double* u_in, const double* u_n, double* out, int src, double* ring,
                                     const double* ghost, hipStream_t st) {
  if (M.dim != 3 || degree != 3) return hipErrorInvalidValue;
  if (precision == 1) return launch_split<float>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
  return launch_split<double>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
}

}  // namespace adg
