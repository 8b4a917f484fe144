// adg_device.h — device helpers shared by the stage kernels: fused
// multiply-add in the kernel's precision, the reciprocal, the local
// Lax-Friedrichs flux, and the XCD-aware block order. Internal.
#pragma once
#include <hip/hip_runtime.h>

namespace adg {

__device__ __forceinline__ double fmx(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmx(float a, float b, float c) { return fmaf(a, b, c); }

// 1/x to an ulp or two: the hardware estimate refined by Newton steps (two in
// FP64, one in FP32); every use of a given operand gives the same result
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// n.F^ for n = +e_a with left state wl and right state wr (eq. lfflux,
// lambda of eq. lfflux-lambda, or the Rusanov speed for kind 1). Both sides
// of a face call it on the same operands in the same order, so their
// contributions are bitwise opposite.
template <typename T, int D>
__device__ __forceinline__ void num_flux(const T* wl, const T* wr, int a, T gamma, int kind, T* G) {
  constexpr int V = D + 2;
  const T gm1 = gamma - (T)1;
  const T il = recip(wl[0]), ir = recip(wr[0]);
  T ml2 = wl[1] * wl[1], mr2 = wr[1] * wr[1];
#pragma unroll
  for (int k = 1; k < D; ++k) {
    ml2 = fmx(wl[1 + k], wl[1 + k], ml2);
    mr2 = fmx(wr[1 + k], wr[1 + k], mr2);
  }
  const T pl = gm1 * (wl[D + 1] - (T)0.5 * ml2 * il), pr = gm1 * (wr[D + 1] - (T)0.5 * mr2 * ir);
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
  const T cl2 = gamma * pl * il, cr2 = gamma * pr * ir;
  T lam;
  if (kind == 1) {
    const T sl = fabs(ual) + sqrt(cl2), sr = fabs(uar) + sqrt(cr2);
    lam = sl > sr ? sl : sr;
  } else {
    const T sl = ml2 * il * il + cl2, sr = mr2 * ir * ir + cr2;
    lam = (T)0.5 * sqrt(sl > sr ? sl : sr);
  }
  const T hl = (T)0.5 * lam;
#pragma unroll
  for (int v = 0; v < V; ++v) G[v] = (T)0.5 * (Fl[v] + Fr[v]) + hl * (wl[v] - wr[v]);
}

// n <= NMAX consecutive doubles between global memory and LDS, by the whole
// wavefront in 16-byte pieces (both addresses 16-byte aligned), four loads in
// flight per lane before their stores: a wavefront's elements are one
// contiguous range, so staging them through LDS turns per-lane strided
// accesses into coalesced ones. NT_LD / NT_ST mark the global loads / stores
// non-temporal (streamed past L2 with low retention), for data no other
// wavefront reads in this launch, so that L2 keeps the stage input the
// neighbouring wavefronts read their face traces from.
typedef double dvec2 __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ dvec2 ld2(const dvec2* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void st2(dvec2* p, dvec2 x) {
  if constexpr (NT) __builtin_nontemporal_store(x, p);
  else *p = x;
}
template <int NMAX, bool NT_LD, bool NT_ST>
__device__ __forceinline__ void wave_copy(double* dst, const double* src, int n) {
  constexpr int IT = (NMAX / 2 + 63) / 64;
  const int lane = threadIdx.x, n2 = n >> 1;
  const dvec2* s2 = reinterpret_cast<const dvec2*>(src);
  dvec2* d2 = reinterpret_cast<dvec2*>(dst);
  // past the end a lane copies piece 0 again (the same value to the same
  // place), which keeps the loop free of branches
#pragma unroll 1
  for (int k0 = 0; k0 < IT; k0 += 4) {
    const int i0 = lane + 64 * k0, i1 = i0 + 64, i2 = i0 + 128, i3 = i0 + 192;
    const int j0 = i0 < n2 ? i0 : 0, j1 = i1 < n2 ? i1 : 0, j2 = i2 < n2 ? i2 : 0, j3 = i3 < n2 ? i3 : 0;
    const dvec2 a0 = ld2<NT_LD>(s2 + j0), a1 = ld2<NT_LD>(s2 + j1), a2 = ld2<NT_LD>(s2 + j2),
                a3 = ld2<NT_LD>(s2 + j3);
    st2<NT_ST>(d2 + j0, a0);
    st2<NT_ST>(d2 + j1, a1);
    st2<NT_ST>(d2 + j2, a2);
    st2<NT_ST>(d2 + j3, a3);
  }
  if ((n & 1) && lane == 0) dst[n - 1] = src[n - 1];
}
// the stage input: kept in L2 for the neighbours' face traces
template <int NMAX>
__device__ __forceinline__ void wave_copy_in(double* lds, const double* g, int n) {
  wave_copy<NMAX, false, false>(lds, g, n);
}
// u^n and the stage output: streamed
template <int NMAX>
__device__ __forceinline__ void wave_stream_in(double* lds, const double* g, int n) {
  wave_copy<NMAX, true, false>(lds, g, n);
}
template <int NMAX>
__device__ __forceinline__ void wave_stream_out(double* g, const double* lds, int n) {
  wave_copy<NMAX, false, true>(g, lds, n);
}

// logical block index: the hardware deals consecutive blocks round-robin to
// the 8 XCDs; remap so each XCD walks a contiguous range of elements and its
// L2 holds the neighbours it reads
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, i = blockIdx.x;
  const int per = nb / 8, rem = nb % 8, x = i % 8, k = i / 8;
  return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

}  // namespace adg
