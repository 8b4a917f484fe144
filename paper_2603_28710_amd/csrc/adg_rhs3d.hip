// adg_rhs3d.hip — the fused SSP-RK3 stage on hexahedral meshes of degree
// 1 and 2, with the element data in registers.
//
// One wavefront owns up to 12 consecutive elements of one x row (wave_range:
// the wavefronts walk the mesh in z-bands); lane (e, v) keeps
// the P^3 nodal values of variable v of element e in registers (lanes 60-63
// idle) and applies the tensor-product operators of that variable there. LDS
// carries what the nonlinear fluxes need (all V variables at a point) and,
// at the start and in the combine, the wavefront's element data: its
// elements are one contiguous range, moved into LDS by direct global-to-LDS
// loads and out of it by coalesced 16-byte stores of the whole wavefront (a
// lane's own values lie P^3 doubles from the next lane's, so direct per-lane
// accesses would touch one cache line per lane and instruction).
//
//   volume: one Gauss plane q_z at a time. The lane combines its nodal
//           planes along z (B), interpolates the result in x and y, and
//           stores the plane's values. Once per Gauss point (three points
//           per lane) the scaled velocity s_a u_a (s_a = 2/h_a) and the
//           pressure are formed and stored beside the state. Row by row each
//           lane then forms its own scaled flux components s_a F_a[v]
//           (eq. euler-dealii; four FMAs per point) and tests them along x;
//           the y test accumulates over the plane's rows into A (x- and
//           y-derivative terms) and C (z term), and the plane's z test
//           adds them once:
//             k += (GW (x) BW (x) BW) s_x F_x + (BW (x) GW (x) BW) s_y F_y
//                + (BW (x) BW (x) GW) s_z F_z
//           (BW = M1^{-1} B^T W, GW = M1^{-1} B^T D^T W per direction;
//           eq. weakform-dealii / weakform-compact-dealii).
//   faces:  the x faces in one pass: the wavefront's elements are
//           consecutive in x, so each lane interpolates its own traces on both
//           x faces, and a face between two of its elements (same row, not a
//           PE face of an asynchronous run) gets its LLF flux once for both
//           sides; only the other x face-sides (the wavefront's two ends, PE
//           faces; at most four, else the per-face passes below) take a
//           neighbour trace. Then one pass per y and z face:
//           each lane interpolates its own and the neighbour's face traces
//           (live values; the delayed / AT / learned trace at a PE-boundary
//           face; or, in the flux-history modes, the stored flux) to the
//           face's Gauss points; one lane per (element, point) evaluates the
//           LLF flux (eq. lfflux / lfflux-lambda) in canonical (left, right)
//           order; each lane lifts its variable with BW along the two
//           tangential axes and adds the column of M1^{-1} at that face.
//   stage:  out = a u_n + b (u_in + dt k) in FP64, u_n and out through LDS.
//
// The ring publish (stage 0, stale and AT modes), the delay schedule, the AT
// extrapolation and the flux history follow the same rules as the other
// stage kernels. T = double (FP64) or float (FP32 contractions).
#include <type_traits>

#include "adg_device.h"
#include "adg_internal.h"
#include "adg_tables.h"

namespace adg {

namespace {

constexpr int kNE3 = 12;  // elements per wavefront (V = 5 lanes each)

// node index (x fastest) of the node with coordinate ia along axis a and
// coordinates (j0, j1) along the other two axes in ascending order
template <int P>
__device__ __forceinline__ constexpr int node3(int a, int ia, int j0, int j1) {
  return a == 0 ? ia + P * (j0 + P * j1) : (a == 1 ? j0 + P * (ia + P * j1) : j0 + P * (j1 + P * ia));
}

// at least two wavefronts per SIMD (at most 256 VGPRs): the LDS the degree-2
// FP64 kernel takes already limits a CU to eight wavefronts
template <typename T, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void rhs_stage3d_kernel(
    Mesh M, Async A, Stage S, const double* __restrict__ u_in, const double* u_n, double* out, int src,
    double* __restrict__ ring, const double* __restrict__ ghost) {
  constexpr int Q = P + 1, V = 5, NE = kNE3, Pd = P * P * P, Fn = P * P, Fq = Q * Q;
  constexpr ops::Ops<P> O = ops::make_ops<P>();
  const ops::RowOps<P>& OR = ops::kRowOps<P>;  // entries indexed at run time, by Gauss plane
  // per element: the state at the points of one Gauss plane [Fq][V] during
  // the volume, the own and neighbour traces of one face [2][Fq][V] during
  // the faces; one spare element slot for the idle lanes; the stride is
  // padded against LDS bank conflicts
  constexpr int PER0 = 2 * Fq * V;
  // during the volume: the plane's state [Fq][V], then from kPre the
  // scaled velocity and pressure [Fq][4] (16-byte aligned)
  constexpr int kPre = (Fq * V + 3) / 4 * 4;
  static_assert(kPre + 4 * Fq <= PER0, "volume data exceed the element's LDS block");
  // (FP64 degree 2: 164 doubles, = 4 mod 16, keeps the blocks 16-byte
  // aligned and halves the bank-conflict cycles of the 162 that the rule
  // below gives, 1750 against 3270 per wavefront; measured over 160-169.
  // Elsewhere 16-byte reads of consecutive elements spread over the banks.)
  constexpr int PER = sizeof(T) == 8 ? (P == 3 ? 164 : PER0 + (6 - PER0 % 4) % 4) : PER0 + (12 - PER0 % 8) % 8;
  static_assert(PER >= PER0, "element block too small");
  // the same LDS stages the wavefront's element data (FP64) at the start and
  // the end of the stage
  // the x pass adds kExtX outside traces [Fq][V] after the element slots
  constexpr int kExtX = 4;
  constexpr int kXB = ((NE + 1) * PER + kExtX * Fq * V) * (int)sizeof(T), kDB = NE * V * Pd * 8;
  __shared__ __align__(16) unsigned char sRaw[kXB > kDB ? kXB : kDB];
  T* sX = reinterpret_cast<T*>(sRaw);
  double* sD = reinterpret_cast<double*>(sRaw);
  __shared__ long long sFsF[NE + 1];  // flux-history modes: face-side of the current face, or -1
  __shared__ int sKdF[NE + 1];        // and its delay
  __shared__ int sItem[2 * NE + 1];   // x pass: the flux items 2 l + side, then their count

  const int lane = threadIdx.x, le = lane / V, v = lane - le * V;  // le == NE: idle lane
  long long e0;
  int ne;
  wave_range<NE>(M, xcd_block(), e0, ne);
  const long long e = e0 + le;
  const bool valid = le < ne;

  double u[Pd];
  wave_load_in<NE * V * Pd>(sD, u_in + e0 * V * Pd, ne * V * Pd);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < Pd; ++i) u[i] = valid ? sD[(le * V + v) * Pd + i] : 0.0;
  __syncthreads();

  T k[Pd];
#pragma unroll
  for (int i = 0; i < Pd; ++i) k[i] = (T)0;
  T* mine = sX + le * PER;

  // ---- volume, one Gauss plane q_z at a time
  {
    const T gm1 = (T)M.gamma - (T)1;
    const T sx = (T)(2.0 / M.h[0]), sy = (T)(2.0 / M.h[1]), sz = (T)(2.0 / M.h[2]);
    // this lane's pressure terms of the scaled flux columns s_a F_a[v]
    const T cx = v == 1 ? sx : (T)0, cy = v == 2 ? sy : (T)0, cz = v == 3 ? sz : (T)0;
    const T e4 = v == 4 ? (T)1 : (T)0;
#pragma unroll 1
    for (int qz = 0; qz < Q; ++qz) {
      if (qz) __syncthreads();  // the previous plane has been read
      T bq[P], bw[P], gw[P];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        bq[i] = (T)OR.r[qz][0][i];
        bw[i] = (T)OR.r[qz][1][i];
        gw[i] = (T)OR.r[qz][2][i];
      }
      // this lane's variable on the plane: z combination, then x, then y
      {
        T Z[P][P];
#pragma unroll
        for (int iy = 0; iy < P; ++iy)
#pragma unroll
          for (int ix = 0; ix < P; ++ix) {
            T acc = bq[0] * (T)u[iy * P + ix];
#pragma unroll
            for (int iz = 1; iz < P; ++iz) acc = fmx(bq[iz], (T)u[(iz * P + iy) * P + ix], acc);
            Z[iy][ix] = acc;
          }
        T X[P][Q];
#pragma unroll
        for (int iy = 0; iy < P; ++iy)
#pragma unroll
          for (int qx = 0; qx < Q; ++qx) {
            T acc = (T)O.B[qx][0] * Z[iy][0];
#pragma unroll
            for (int ix = 1; ix < P; ++ix) acc = fmx((T)O.B[qx][ix], Z[iy][ix], acc);
            X[iy][qx] = acc;
          }
#pragma unroll
        for (int qy = 0; qy < Q; ++qy)
#pragma unroll
          for (int qx = 0; qx < Q; ++qx) {
            T acc = (T)O.B[qy][0] * X[0][qx];
#pragma unroll
            for (int iy = 1; iy < P; ++iy) acc = fmx((T)O.B[qy][iy], X[iy][qx], acc);
            mine[(qy * Q + qx) * V + v] = acc;
          }
      }
      __syncthreads();
      // once per Gauss point (three points per lane): the scaled velocity
      // s_a u_a and the pressure (eq. euler-parameters-dealii), after the
      // point's state in the element's LDS block
#pragma unroll
      for (int it = 0; it < (NE * Fq + 63) / 64; ++it) {
        const int t = lane + 64 * it;
        if (t < NE * Fq) {
          const int el = t / Fq, m = t - el * Fq;
          const T* w = sX + el * PER + m * V;
          const T rho = w[0], mx = w[1], my = w[2], mz = w[3], en = w[4];
          const T ir = recip(rho);
          const T ux = mx * ir, uy = my * ir, uz = mz * ir;
          const T p = gm1 * (en - (T)0.5 * fmx(mz, uz, fmx(my, uy, mx * ux)));
          T* d = sX + el * PER + kPre + 4 * m;
          d[0] = sx * ux;
          d[1] = sy * uy;
          d[2] = sz * uz;
          d[3] = p;
        }
      }
      __syncthreads();
      // the scaled flux columns of this lane's variable, tested with the
      // x operators per Gauss row, then with the y operators into the
      // plane's accumulators A (x- and y-derivative terms) and C (z term)
      T A[P][P], C[P][P];
#pragma unroll
      for (int iy = 0; iy < P; ++iy)
#pragma unroll
        for (int ix = 0; ix < P; ++ix) A[iy][ix] = C[iy][ix] = (T)0;
#pragma unroll
      for (int qy = 0; qy < Q; ++qy) {
        T tx[P], ty[P], tz[P];
#pragma unroll
        for (int i = 0; i < P; ++i) tx[i] = ty[i] = tz[i] = (T)0;
#pragma unroll
        for (int qx = 0; qx < Q; ++qx) {
          const int m = qy * Q + qx;
          const T wv = mine[m * V + v];
          const T* d = mine + kPre + 4 * m;
          const T su_x = d[0], su_y = d[1], su_z = d[2], p = d[3];
          // s_a F_a[v] = s_a u_a (w_v + p [v=4]) + s_a p [v=1+a]
          const T t = fmx(p, e4, wv);
          const T fx = fmx(su_x, t, p * cx), fy = fmx(su_y, t, p * cy), fz = fmx(su_z, t, p * cz);
#pragma unroll
          for (int i = 0; i < P; ++i) {
            tx[i] = fmx((T)O.GW[i][qx], fx, tx[i]);
            ty[i] = fmx((T)O.BW[i][qx], fy, ty[i]);
            tz[i] = fmx((T)O.BW[i][qx], fz, tz[i]);
          }
        }
#pragma unroll
        for (int iy = 0; iy < P; ++iy)
#pragma unroll
          for (int ix = 0; ix < P; ++ix) {
            A[iy][ix] = fmx((T)O.GW[iy][qy], ty[ix], fmx((T)O.BW[iy][qy], tx[ix], A[iy][ix]));
            C[iy][ix] = fmx((T)O.BW[iy][qy], tz[ix], C[iy][ix]);
          }
      }
      // the z operators of this plane: k += BW_z (x) A + GW_z (x) C
#pragma unroll
      for (int iz = 0; iz < P; ++iz)
#pragma unroll
        for (int iy = 0; iy < P; ++iy)
#pragma unroll
          for (int ix = 0; ix < P; ++ix) {
            const int n = (iz * P + iy) * P + ix;
            k[n] = fmx(gw[iz], C[iy][ix], fmx(bw[iz], A[iy][ix], k[n]));
          }
    }
  }

  // ---- faces, one face at a time
  const ElemPos pos = elem_pos(M, valid ? e : 0);
  const bool async_on = src != kSrcLive && M.nfs > 0;
  const bool flux_mode = src == kSrcFlux;
  const long long ring_level = M.nfs * V * (flux_mode ? Fq : Fn);  // values per ring level
  const bool publish = src == kSrcRing && A.stage == 0;
  // the neighbour trace of variable v at the face nodes (j0 + P j1) of face
  // f: live values, the delayed / AT / learned trace at a PE-boundary face
  // (whose own trace is published at stage 0), nothing in a flux-history
  // silent step; fs and kd receive the face-side and its delay
  auto gather = [&](auto fc, auto at_together, double* g, long long& fs, int& kd) {
    constexpr int f = decltype(fc)::value;
    constexpr int a = f >> 1, s = f & 1, ia = s ? P - 1 : 0;
#pragma unroll
    for (int j = 0; j < Fn; ++j) g[j] = 0.0;
    fs = -1;
    kd = 0;
    if (valid) {
      fs = async_on ? face_side_at(M, pos, f) : -1;
      if (fs >= 0 && (src == kSrcRing || flux_mode)) kd = delay_of(M, A, sub_at(M, pos.sc), f);
      if (fs >= 0 && publish) {
        double* dst = ring + A.slot_n * ring_level + fed_face_side(M, pos, f) * V * Fn + v * Fn;
#pragma unroll
        for (int j1 = 0; j1 < P; ++j1)
#pragma unroll
          for (int j0 = 0; j0 < P; ++j0) dst[j0 + P * j1] = u[node3<P>(a, ia, j0, j1)];
      }
      if (fs < 0 || ((src == kSrcRing || flux_mode) && kd == 0)) {
        const unsigned nb = (unsigned)neighbour_of(M, e, pos, f);
        const double* gp = u_in + (size_t)nb * (V * Pd) + v * Pd;
#pragma unroll
        for (int j1 = 0; j1 < P; ++j1)
#pragma unroll
          for (int j0 = 0; j0 < P; ++j0) g[j0 + P * j1] = gp[node3<P>(a, P - 1 - ia, j0, j1)];
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
        if constexpr (decltype(at_together)::value) {
          // the x pass: at most kMaxLevels levels, past A.levels the newest
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
  };
  // face-node values x[j0 + P j1] of variable v interpolated to the Gauss
  // points (q0 + Q q1) of the face, stored at dst[(q0 + Q q1) V]
  auto interp_face = [&](const auto& x, T* dst) {
    T X[P][Q];
#pragma unroll
    for (int j1 = 0; j1 < P; ++j1)
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) {
        T o = (T)O.B[q0][0] * (T)x(0, j1);
#pragma unroll
        for (int j0 = 1; j0 < P; ++j0) o = fmx((T)O.B[q0][j0], (T)x(j0, j1), o);
        X[j1][q0] = o;
      }
#pragma unroll
    for (int q1 = 0; q1 < Q; ++q1)
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) {
        T o = (T)O.B[q1][0] * X[0][q0];
#pragma unroll
        for (int j1 = 1; j1 < P; ++j1) o = fmx((T)O.B[q1][j1], X[j1][q0], o);
        dst[(q1 * Q + q0) * V] = o;
      }
  };
  // lift of the scaled fluxes src[(q0 + Q q1) V] of face f with BW along both
  // tangential axes, then k(i_a, j0, j1) += MC_s[i_a] * lifted(j0, j1)
  auto lift_face = [&](auto fc, const T* src) {
    constexpr int f = decltype(fc)::value;
    constexpr int a = f >> 1, s = f & 1;
    T L0[Q][P];
#pragma unroll
    for (int q1 = 0; q1 < Q; ++q1) {
      T G[Q];
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) G[q0] = src[(q1 * Q + q0) * V];
#pragma unroll
      for (int j0 = 0; j0 < P; ++j0) {
        T acc = (T)O.BW[j0][0] * G[0];
#pragma unroll
        for (int q0 = 1; q0 < Q; ++q0) acc = fmx((T)O.BW[j0][q0], G[q0], acc);
        L0[q1][j0] = acc;
      }
    }
#pragma unroll
    for (int j1 = 0; j1 < P; ++j1)
#pragma unroll
      for (int j0 = 0; j0 < P; ++j0) {
        T lf = (T)O.BW[j1][0] * L0[0][j0];
#pragma unroll
        for (int q1 = 1; q1 < Q; ++q1) lf = fmx((T)O.BW[j1][q1], L0[q1][j0], lf);
#pragma unroll
        for (int i = 0; i < P; ++i) {
          const int n = node3<P>(a, i, j0, j1);
          k[n] = fmx((T)O.MC[s][i], lf, k[n]);
        }
      }
  };
  // one pass per face, with the face index a compile-time constant so that
  // every register index below is fixed
  auto face_pass = [&](auto fc) {
    constexpr int f = decltype(fc)::value;
    constexpr int a = f >> 1, s = f & 1, ia = s ? P - 1 : 0;
    __syncthreads();  // sX is rewritten
    double g[Fn];
    long long fs;
    int kd;
    gather(fc, std::false_type{}, g, fs, kd);
    if (flux_mode && v == 0) {
      sFsF[le] = fs;
      sKdF[le] = kd;
    }
    // own trace at the Gauss points first (its work covers the neighbour
    // loads), then the neighbour's
    interp_face([&](int j0, int j1) { return u[node3<P>(a, ia, j0, j1)]; }, mine + v);
    interp_face([&](int j0, int j1) { return g[j0 + P * j1]; }, mine + Fq * V + v);
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
    lift_face(fc, mine + v);
  };
  // the x faces of the wavefront's consecutive elements in one pass: each
  // lane interpolates its own traces on both x faces, a face between two
  // elements of the wavefront (same row, not a PE face of an asynchronous
  // run) takes its flux once for both sides, and only the other face-sides
  // (the wavefront's ends, PE faces) take a neighbour trace, from up to
  // kExtX outside slots; otherwise the two per-face passes
  bool x_shared = false;
  if (!flux_mode) {
    // bit l: the +x face of element l is shared with element l + 1
    const bool pr = valid && le + 1 < ne && pos.c[0] + 1 < M.nc[0] && !(async_on && face_side_at(M, pos, 1) >= 0);
    const unsigned long long bal = __ballot(v == 0 && pr);
    unsigned pair = 0;
#pragma unroll
    for (int l = 0; l < NE; ++l) pair |= (unsigned)((bal >> (V * l)) & 1ull) << l;
    // bit 2l + s: face-side (l, s) takes an outside trace
    unsigned ext = 0;
    for (int l = 0; l < ne; ++l) {
      if (l == 0 || !((pair >> (l - 1)) & 1u)) ext |= 1u << (2 * l);
      if (!((pair >> l) & 1u)) ext |= 1u << (2 * l + 1);
    }
    if (__popc(ext) <= kExtX) {
      x_shared = true;
      __syncthreads();  // sX is rewritten
      // flux items in order: (l, -x) if it takes an outside trace, (l, +x);
      // lane l writes element l's, after the l +x items and the outside -x
      // items of the elements before it
      if (lane < ne) {
        const bool mx = (ext >> (2 * lane)) & 1u;
        const int at = lane + __popc(ext & 0x55555555u & ((1u << (2 * lane)) - 1u));
        if (mx) sItem[at] = lane * 2;
        sItem[at + (mx ? 1 : 0)] = lane * 2 + 1;
      }
      if (lane == 0) sItem[2 * NE] = ne + __popc(ext & 0x55555555u);
      T* outside = sX + (NE + 1) * PER;  // kExtX traces [Fq][V]
      interp_face([&](int j0, int j1) { return u[node3<P>(0, 0, j0, j1)]; }, mine + v);
      interp_face([&](int j0, int j1) { return u[node3<P>(0, P - 1, j0, j1)]; }, mine + Fq * V + v);
      // the outside traces of the face-sides that take one, -x then +x (the
      // gather publishes the own trace of a PE face at stage 0)
      const unsigned below = le < NE ? (1u << (2 * le)) - 1u : 0u;
      if (valid && ((ext >> (2 * le)) & 1u)) {
        double g[Fn];
        long long fs;
        int kd;
        gather(std::integral_constant<int, 0>{}, std::true_type{}, g, fs, kd);
        interp_face([&](int j0, int j1) { return g[j0 + P * j1]; }, outside + __popc(ext & below) * Fq * V + v);
      }
      if (valid && ((ext >> (2 * le + 1)) & 1u)) {
        double g[Fn];
        long long fs;
        int kd;
        gather(std::integral_constant<int, 1>{}, std::true_type{}, g, fs, kd);
        interp_face([&](int j0, int j1) { return g[j0 + P * j1]; },
                    outside + __popc(ext & (below | (1u << (2 * le)))) * Fq * V + v);
      }
      __syncthreads();
      // numerical flux, one lane per (item, face point): a shared face writes
      // -s G to its left element's +x slot and +s G to its right element's -x
      // slot; an outside face-side writes to its own slot only
      {
        const T gamma = (T)M.gamma;
        const T sc = (T)(2.0 / M.h[0]);
        const int nt = sItem[2 * NE] * Fq;
#pragma unroll 1
        for (int t = lane; t < nt; t += 64) {
          const int it = sItem[t / Fq], m = t - (t / Fq) * Fq;
          const int l = it >> 1, sd = it & 1;
          T* own = sX + l * PER + (sd ? Fq * V : 0) + m * V;
          const bool shared = sd && ((pair >> l) & 1u);
          T* other = shared ? sX + (l + 1) * PER + m * V
                            : outside + __popc(ext & ((1u << it) - 1u)) * Fq * V + m * V;
          T wl[V], wr[V], G[V];
#pragma unroll
          for (int vv = 0; vv < V; ++vv) {
            wl[vv] = sd ? own[vv] : other[vv];  // canonical order: left element first
            wr[vv] = sd ? other[vv] : own[vv];
          }
          num_flux<T, 3>(wl, wr, 0, gamma, M.flux, G);
          const T sg = sd ? -sc : sc;
#pragma unroll
          for (int vv = 0; vv < V; ++vv) own[vv] = sg * G[vv];
          if (shared) {
#pragma unroll
            for (int vv = 0; vv < V; ++vv) other[vv] = sc * G[vv];
          }
        }
      }
      __syncthreads();
      lift_face(std::integral_constant<int, 0>{}, mine + v);
      lift_face(std::integral_constant<int, 1>{}, mine + Fq * V + v);
    }
  }
  if (!x_shared) {
    face_pass(std::integral_constant<int, 0>{});
    face_pass(std::integral_constant<int, 1>{});
  }
  face_pass(std::integral_constant<int, 2>{});
  face_pass(std::integral_constant<int, 3>{});
  face_pass(std::integral_constant<int, 4>{});
  face_pass(std::integral_constant<int, 5>{});

  // ---- the stage combine in FP64, through LDS (u_n may be the output)
  __syncthreads();
  if (S.lserk) {
    // LSERK: u_n holds the accumulator w; the new w to out, the next
    // stage input (if any) to out2
    wave_stream_in<NE * V * Pd>(sD, u_n + e0 * V * Pd, ne * V * Pd);
    __syncthreads();
    double wv[Pd];
#pragma unroll
    for (int i = 0; i < Pd; ++i) wv[i] = valid ? sD[(le * V + v) * Pd + i] : 0.0;
    if (valid) {
#pragma unroll
      for (int i = 0; i < Pd; ++i) sD[(le * V + v) * Pd + i] = wv[i] + S.dt * S.bw * (double)k[i];
    }
    __syncthreads();
    wave_stream_out<NE * V * Pd>(out + e0 * V * Pd, sD, ne * V * Pd);
    if (S.out2) {
      __syncthreads();
      if (valid) {
#pragma unroll
        for (int i = 0; i < Pd; ++i) sD[(le * V + v) * Pd + i] = wv[i] + S.dt * S.ar * (double)k[i];
      }
      __syncthreads();
      wave_stream_out<NE * V * Pd>(S.out2 + e0 * V * Pd, sD, ne * V * Pd);
    }
    return;
  }
  if (S.a != 0.0) wave_stream_in<NE * V * Pd>(sD, u_n + e0 * V * Pd, ne * V * Pd);
  __syncthreads();
  if (valid) {
    double* o = sD + (le * V + v) * Pd;
    if (S.a == 0.0) {
#pragma unroll
      for (int i = 0; i < Pd; ++i) o[i] = S.b * (u[i] + S.dt * (double)k[i]);
    } else {
#pragma unroll
      for (int i = 0; i < Pd; ++i) o[i] = S.a * o[i] + S.b * (u[i] + S.dt * (double)k[i]);
    }
  }
  __syncthreads();
  wave_stream_out<NE * V * Pd>(out + e0 * V * Pd, sD, ne * V * Pd);
}

template <typename T, int P>
hipError_t launch3d(const Mesh& M, const Async& A, const Stage& S, const double* u_in, const double* u_n,
                    double* out, int src, double* ring, const double* ghost, hipStream_t st) {
  const long long nblk = wave_ranges<kNE3>(M);
  hipLaunchKernelGGL((rhs_stage3d_kernel<T, P>), dim3((unsigned)nblk), dim3(64), 0, st, M, A, S, u_in, u_n, out, src,
                     ring, ghost);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rhs_stage_3d(int degree, int precision, const Mesh& M, const Async& A, const Stage& S,
                               const double* u_in, const double* u_n, double* out, int src, double* ring,
                               const double* ghost, hipStream_t st) {
  if (M.dim != 3) return hipErrorInvalidValue;
  if (degree == 1) {
    if (precision == 1) return launch3d<float, 2>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
    return launch3d<double, 2>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
  }
  if (degree == 2) {
    if (precision == 1) return launch3d<float, 3>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
    return launch3d<double, 3>(M, A, S, u_in, u_n, out, src, ring, ghost, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace adg
