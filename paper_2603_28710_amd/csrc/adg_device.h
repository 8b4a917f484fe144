// adg_device.h — device helpers shared by the stage kernels: fused
// multiply-add in the kernel's precision, the reciprocal, the local
// Lax-Friedrichs flux, and the XCD-aware block order. Internal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
// wavefront, four loads in flight per lane before their stores: a
// wavefront's elements are one contiguous range, so staging them through LDS
// turns per-lane strided accesses into coalesced ones. 16-byte pieces when
// both addresses are 16-byte aligned, else 8-byte pieces (a range of
// hexahedra of degree 2 starts at an odd multiple of 8 bytes in rows of odd
// length). NT_LD / NT_ST mark the global loads / stores non-temporal
// (streamed past L2 with low retention), for data no other wavefront reads
// in this launch, so that L2 keeps the stage input the neighbouring
// wavefronts read their face traces from.
typedef double dvec2 __attribute__((ext_vector_type(2)));
template <bool NT, typename X>
__device__ __forceinline__ X ldg(const X* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename X>
__device__ __forceinline__ void stg(X* p, X x) {
  if constexpr (NT) __builtin_nontemporal_store(x, p);
  else *p = x;
}
template <int NMAX, bool NT_LD, bool NT_ST, typename X>
__device__ __forceinline__ void wave_copy_pieces(X* d, const X* s, int np) {
  constexpr int IT = (NMAX * (int)sizeof(double) / (int)sizeof(X) + 63) / 64;
  const int lane = threadIdx.x;
  // past the end a lane copies piece 0 again (the same value to the same
  // place), which keeps the loop free of branches
#pragma unroll 1
  for (int k0 = 0; k0 < IT; k0 += 4) {
    const int i0 = lane + 64 * k0, i1 = i0 + 64, i2 = i0 + 128, i3 = i0 + 192;
    const int j0 = i0 < np ? i0 : 0, j1 = i1 < np ? i1 : 0, j2 = i2 < np ? i2 : 0, j3 = i3 < np ? i3 : 0;
    const X a0 = ldg<NT_LD>(s + j0), a1 = ldg<NT_LD>(s + j1), a2 = ldg<NT_LD>(s + j2), a3 = ldg<NT_LD>(s + j3);
    stg<NT_ST>(d + j0, a0);
    stg<NT_ST>(d + j1, a1);
    stg<NT_ST>(d + j2, a2);
    stg<NT_ST>(d + j3, a3);
  }
}
__device__ __forceinline__ bool aligned16(const void* a, const void* b) {
  return ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0;
}
template <int NMAX, bool NT_LD, bool NT_ST>
__device__ __forceinline__ void wave_copy(double* dst, const double* src, int n) {
  if (aligned16(dst, src)) {
    wave_copy_pieces<NMAX, NT_LD, NT_ST>(reinterpret_cast<dvec2*>(dst), reinterpret_cast<const dvec2*>(src), n >> 1);
    if ((n & 1) && threadIdx.x == 0) dst[n - 1] = src[n - 1];
  } else {
    wave_copy_pieces<NMAX, NT_LD, NT_ST>(dst, src, n);
  }
}
// n <= NMAX consecutive doubles from global memory into LDS with direct
// global-to-LDS loads: each instruction moves 16 bytes per lane, the
// wavefront's 64 pieces landing contiguously at the LDS address it names,
// so every load is in flight at once and no register holds the data. Both
// addresses 16-byte aligned (else the register copy above). The loads are
// complete when it returns (the LDS is written behind the compiler's view,
// so the wait is explicit); the caller's barrier then publishes them to the
// workgroup.
template <int NMAX, bool NT>
__device__ __forceinline__ void wave_load_lds(double* lds, const double* g, int n) {
  if (!aligned16(lds, g)) {
    wave_copy_pieces<NMAX, NT, false>(lds, g, n);
    return;
  }
  constexpr int IT = (NMAX / 2 + 63) / 64;
  const int lane = threadIdx.x, n2 = n >> 1;
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int i = lane + 64 * k;
    // a lane past the end would still write its LDS slot: masked off
    if (i < n2)
      __builtin_amdgcn_global_load_lds(
          reinterpret_cast<const void*>(g + 2 * i),
          reinterpret_cast<__attribute__((address_space(3))) void*>(reinterpret_cast<uintptr_t>(lds + 128 * k)),
          16, 0, NT ? 2 : 0);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  if ((n & 1) && lane == 0) lds[n - 1] = g[n - 1];
}
// the stage input: kept in L2 for the neighbours' face traces
template <int NMAX>
__device__ __forceinline__ void wave_load_in(double* lds, const double* g, int n) {
  wave_load_lds<NMAX, false>(lds, g, n);
}
// u^n and the stage output: streamed
template <int NMAX>
__device__ __forceinline__ void wave_stream_in(double* lds, const double* g, int n) {
  wave_load_lds<NMAX, true>(lds, g, n);
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
