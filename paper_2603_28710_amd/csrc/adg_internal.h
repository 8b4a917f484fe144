// adg_internal.h — structures shared by the host runtime and the gfx950
// kernels of the ADG right-hand side. Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adg {

constexpr int kMaxP = 5;   // nodes per direction (degree <= 4)
constexpr int kMaxQ = 6;   // Gauss points per direction
constexpr int kMaxV = 5;
constexpr int kMlpK = 4;   // past levels read by the learned predictor
constexpr int kMlpH = 64;  // hidden width
constexpr int kThreads = 256;  // block size of the set-up and diagnostic kernels

// Offsets into the per-context table (doubles; a float copy has the same
// offsets). B: interpolation nodes->Gauss [Q][P]; BT: its transpose [P][Q];
// DT: transposed collocation derivative on the Gauss points [Q][Q]
// (DT[r][q] = l'_r(x_q) of the Gauss Lagrange basis); MI: inverse 1D mass
// [P][P]; WQ: Gauss weights; XQ: Gauss points; XL/WL: GLL points/weights;
// BTM = MI * BT [P][Q] (test functions followed by the inverse mass);
// MC: the first and last columns of MI, [2][P] (inverse mass applied to the
// trace of a face at -1 / +1); BW = BTM diag(WQ) [P][Q] and
// GW = BTM DT diag(WQ) [P][Q] (the Gauss weights folded in).
struct TabOff {
  int B, BT, DT, MI, WQ, XQ, XL, WL, BTM, MC, BW, GW, total;
};
__host__ __device__ constexpr TabOff tab_off(int P, int Q) {
  return TabOff{0,
                Q * P,
                2 * Q * P,
                2 * Q * P + Q * Q,
                2 * Q * P + Q * Q + P * P,
                2 * Q * P + Q * Q + P * P + Q,
                2 * Q * P + Q * Q + P * P + 2 * Q,
                2 * Q * P + Q * Q + P * P + 2 * Q + P,
                2 * Q * P + Q * Q + P * P + 2 * Q + 2 * P,
                3 * Q * P + Q * Q + P * P + 2 * Q + 2 * P,
                3 * Q * P + Q * Q + P * P + 2 * Q + 4 * P,
                4 * Q * P + Q * Q + P * P + 2 * Q + 4 * P,
                5 * Q * P + Q * Q + P * P + 2 * Q + 4 * P};
}

// Division by a divisor d >= 1 fixed at set-up, for dividends 0 <= x < 2^31:
// with s = ceil(log2 d) and m = ceil(2^(31+s) / d) < 2^32, x / d equals
// (x m) >> (31 + s) exactly, since the rounding error of m is below d and
// x < 2^31 (the multiply-shift division of Granlund and Montgomery, 1994).
struct FastDiv {
  unsigned d, m, s;
};
inline FastDiv make_fastdiv(unsigned d) {
  unsigned s = 0;
  while ((1ull << s) < d) ++s;
  const unsigned long long num = 1ull << (31 + s);
  return FastDiv{d, (unsigned)((num + d - 1) / d), s};
}
__host__ __device__ inline unsigned fdiv(unsigned x, const FastDiv& f) {
  return (unsigned)(((unsigned long long)x * f.m) >> (31 + f.s));
}
__host__ __device__ inline unsigned fmodu(unsigned x, const FastDiv& f) { return x - fdiv(x, f) * f.d; }

// x mod d for any 64-bit x and 1 <= d <= 2^15, from x = a 2^62 + b 2^31 + c
// (b, c < 2^31) and the residues of 2^31 and 2^62: every partial sum stays
// below d^2 + 5d < 2^31.
struct FastMod64 {
  FastDiv f;
  unsigned r31, r62;
};
inline FastMod64 make_fastmod64(unsigned d) {
  const unsigned r31 = (unsigned)((1ull << 31) % d);
  return FastMod64{make_fastdiv(d), r31, (unsigned)(((unsigned long long)r31 * r31) % d)};
}
__host__ __device__ inline unsigned fmod64(unsigned long long x, const FastMod64& g) {
  const unsigned a = (unsigned)(x >> 62), b = (unsigned)((x >> 31) & 0x7fffffffu), c = (unsigned)(x & 0x7fffffffu);
  return fmodu(a * g.r62 + fmodu(b, g.f) * g.r31 + fmodu(c, g.f), g.f);
}

// Structured box (periodic, or with Dirichlet sides in 2D), block partition
// into virtual subdomains, and the arithmetic enumeration of PE-boundary
// face-sides (a face-side is a pair (receiving element, face) whose neighbour
// lies in another subdomain). The enumeration is that of the periodic box in
// either case: in a Dirichlet box the slots of the boundary faces exist but
// are never written or read.
// Face-sides are grouped by receiving subdomain, then by face direction f
// (f = 2a + side; side 0 is the -a face), then lexicographically over the
// subdomain-local coordinates of the two other axes (lowest axis fastest).
struct Mesh {
  int dim;
  int nc[3];     // elements per direction (1 beyond dim)
  int parts[3];  // subdomains per direction
  int m[3];      // elements per subdomain per direction
  int nsub;
  int fs_off[6];  // offset of direction f inside a subdomain block, -1 if no PE faces
  int fs_sub;     // face-sides per subdomain
  long long nfs;  // total face-sides
  long long E;
  double h[3], lo[3], hi[3];
  double detJ;       // prod h_k / 2
  double detJf[3];   // face Jacobian for faces normal to axis a
  double gamma;
  int flux;
  int bc;            // 0 periodic; 1 Dirichlet on every side (d = 2)
  int bnd_off[4];    // first boundary face of side f: x- and x+ by iy, y- and y+ by ix
  int nbf;           // boundary faces (0 in a periodic box)
  FastDiv dnc[2];    // division by nc[0], nc[1]
  FastDiv dm[3];     // division by m[k]
  FastDiv dparts[2]; // division by parts[0], parts[1]
  FastDiv dfs_sub;   // division by fs_sub (face-side -> subdomain)
};

// Asynchrony parameters for one stage.
struct Async {
  int ghost, delay_kind, L, levels;
  int Qh;   // history levels needed (warm-up)
  int R;    // ring depth
  unsigned long long seed;
  long long n;       // absolute step index
  long long n_rel;   // steps since the history restarted
  int stage;
  double c_m;        // stage time fraction
  double tol;        // learned accept bound
  int judge;         // 1: the correction must also stay within |AT4 - AT3| on the face
  int slot_n;        // ring slot of level n (n mod R), 0 without a ring
  FastMod64 kmod;    // the delay schedule's modulus: L+1 uniform, L caa-std, L+Qh caa-at
};

// ring slot of level n - back, for 0 <= back < R
__host__ __device__ inline int ring_slot(const Async& A, int back) {
  const int s = A.slot_n - back;
  return s < 0 ? s + A.R : s;
}

// parameters of an analytic problem, passed by value
struct Prm {
  double v[5];
};

// the times t_n + c_m dt of the n stages of one step
struct StageTimes {
  double t[3];
  int n;
};

struct Stage {
  double a, b, dt;  // SSP-RK3 (Shu-Osher): out = a u_n + b (u_in + dt k)
  // LSERK (eq. lserk-dg), when lserk != 0: u_n holds the accumulator w;
  // out = w + dt bw k (the new accumulator) and, unless out2 is null,
  // out2 = w + dt ar k (the next stage's input). out2 may be u_n itself:
  // each element reads its own w before writing.
  int lserk;
  double bw, ar;
  double* out2;
  // Dirichlet box: the exterior states of the boundary faces at this stage's
  // time, [boundary face][V][P] at the face nodes (null in a periodic box)
  const double* bnd;
};

// ---- device helpers shared by several kernels -------------------------------

__host__ __device__ inline long long elem_index(const Mesh& M, int i, int j, int k) {
  return (long long)i + (long long)M.nc[0] * ((long long)j + (long long)M.nc[1] * k);
}

// element coordinates of element index e (0 <= e < E <= 2^31)
__host__ __device__ inline void elem_coords(const Mesh& M, long long e, int* c) {
  const unsigned u = (unsigned)e;
  const unsigned r = fdiv(u, M.dnc[0]);
  c[0] = (int)(u - r * (unsigned)M.nc[0]);
  const unsigned z = fdiv(r, M.dnc[1]);
  c[1] = (int)(r - z * (unsigned)M.nc[1]);
  c[2] = (int)z;
}

// Wavefront ranges of the hexahedron stage kernels: range b is up to NE
// consecutive elements of one x row, each row cut into ceil(nx / NE) ranges.
// The ranges are numbered with z fastest inside bands of kWaveBandZ layers
// (the last band may be thinner), then y, then the band, then the range's
// position along the row. A range's y and z neighbours are then at most
// kWaveBandZ ranges away in the order an XCD walks its blocks (z neighbours
// across a band edge aside), close enough that the face traces find the
// neighbour's data, fetched by its own wavefront or by this one, still in
// that XCD's L2; in x-fastest order a z neighbour is a whole element layer
// (nx ny elements) away and is fetched again.
constexpr int kWaveBandZ = 16;
template <int NE>
__host__ __device__ inline long long wave_ranges(const Mesh& M) {
  return (long long)((M.nc[0] + NE - 1) / NE) * M.nc[1] * M.nc[2];
}
template <int NE>
__device__ __forceinline__ void wave_range(const Mesh& M, int b, long long& e0, int& ne) {
  const int nx = M.nc[0], ny = M.nc[1], nz = M.nc[2];
  const int plane = ny * nz, c = b / plane;
  int r = b - c * plane;
  const int w = nz < kWaveBandZ ? nz : kWaveBandZ, full = nz / w, band = ny * w;
  int y, z;
  if (r < full * band) {
    const int t = r / band;
    r -= t * band;
    y = r / w;
    z = t * w + (r - y * w);
  } else {
    r -= full * band;
    const int wl = nz - full * w;
    y = r / wl;
    z = full * w + (r - y * wl);
  }
  // wave-uniform: kept in scalar registers
  const long long s = (long long)c * NE + (long long)nx * (y + (long long)ny * z);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)s),
                 hi = __builtin_amdgcn_readfirstlane((unsigned)(s >> 32));
  e0 = (long long)(((unsigned long long)hi << 32) | lo);
  ne = __builtin_amdgcn_readfirstlane(nx - c * NE < NE ? nx - c * NE : NE);
}

__host__ __device__ inline int subdomain_of(const Mesh& M, const int* c) {
  return (int)(fdiv(c[0], M.dm[0]) + M.parts[0] * (fdiv(c[1], M.dm[1]) + M.parts[1] * fdiv(c[2], M.dm[2])));
}

// neighbour of element coords c across face f (periodic)
__host__ __device__ inline long long neighbour(const Mesh& M, const int* c, int f) {
  int d[3] = {c[0], c[1], c[2]};
  int a = f >> 1;
  d[a] += (f & 1) ? 1 : -1;
  if (d[a] < 0) d[a] += M.nc[a];
  if (d[a] >= M.nc[a]) d[a] -= M.nc[a];
  return elem_index(M, d[0], d[1], d[2]);
}

// face-side index of (element coords c, face f), or -1 if not a PE face
__host__ __device__ inline long long face_side(const Mesh& M, const int* c, int f) {
  int a = f >> 1;
  if (M.parts[a] < 2) return -1;
  const int l = (int)fmodu(c[a], M.dm[a]);
  if ((f & 1) ? (l != M.m[a] - 1) : (l != 0)) return -1;
  const int o0 = a == 0 ? 1 : 0;
  const int o1 = a == 2 ? 1 : 2;
  long long li = fmodu(c[o0], M.dm[o0]);
  if (M.dim == 3) li += (long long)M.m[o0] * fmodu(c[o1], M.dm[o1]);
  return (long long)subdomain_of(M, c) * M.fs_sub + M.fs_off[f] + li;
}

// An element's position: its coordinates, its coordinates inside its
// subdomain and the subdomain's coordinates; computed once per element, it
// makes the per-face queries below a few integer operations each.
struct ElemPos {
  int c[3], l[3], sc[3];
};
__host__ __device__ inline ElemPos elem_pos(const Mesh& M, long long e) {
  ElemPos p;
  elem_coords(M, e, p.c);
  for (int k = 0; k < 3; ++k) {
    p.sc[k] = (int)fdiv((unsigned)p.c[k], M.dm[k]);
    p.l[k] = p.c[k] - p.sc[k] * M.m[k];
  }
  return p;
}
__host__ __device__ inline int sub_at(const Mesh& M, const int* sc) {
  return sc[0] + M.parts[0] * (sc[1] + M.parts[1] * sc[2]);
}
// element across face f of element e (periodic)
__host__ __device__ inline long long neighbour_of(const Mesh& M, long long e, const ElemPos& p, int f) {
  const int a = f >> 1;
  const long long stride = a == 0 ? 1 : (a == 1 ? (long long)M.nc[0] : (long long)M.nc[0] * M.nc[1]);
  const long long wrap = (long long)(M.nc[a] - 1) * stride;
  if (f & 1) return p.c[a] == M.nc[a] - 1 ? e - wrap : e + stride;
  return p.c[a] == 0 ? e + wrap : e - stride;
}
// position of an element's face-sides of direction f inside the subdomain's
// block of direction f (other axes ascending, lowest fastest)
__host__ __device__ inline int face_local_index(const Mesh& M, const int* l, int a) {
  const int o0 = a == 0 ? 1 : 0, o1 = a == 2 ? 1 : 2;
  return M.dim == 3 ? l[o0] + M.m[o0] * l[o1] : l[o0];
}
// index of face f of the element at p among the boundary faces of a Dirichlet
// box, or -1
__host__ __device__ inline int bnd_face_at(const Mesh& M, const ElemPos& p, int f) {
  const int a = f >> 1;
  if (!M.bc || p.c[a] != ((f & 1) ? M.nc[a] - 1 : 0)) return -1;
  return M.bnd_off[f] + p.c[a ^ 1];
}
// face_side for the element at p: its face-side of face f, or -1 (also for a
// boundary face of a Dirichlet box)
__host__ __device__ inline long long face_side_at(const Mesh& M, const ElemPos& p, int f) {
  const int a = f >> 1;
  if (M.parts[a] < 2) return -1;
  if (M.bc && p.c[a] == ((f & 1) ? M.nc[a] - 1 : 0)) return -1;
  if ((f & 1) ? (p.l[a] != M.m[a] - 1) : (p.l[a] != 0)) return -1;
  return (long long)sub_at(M, p.sc) * M.fs_sub + M.fs_off[f] + face_local_index(M, p.l, a);
}
// the face-side fed by PE face f of the element at p: face f^1 of its
// neighbour, which lies in the adjacent subdomain at the same tangential
// position
__host__ __device__ inline long long fed_face_side(const Mesh& M, const ElemPos& p, int f) {
  const int a = f >> 1;
  int sc[3] = {p.sc[0], p.sc[1], p.sc[2]};
  sc[a] += (f & 1) ? 1 : -1;
  if (sc[a] < 0) sc[a] += M.parts[a];
  if (sc[a] >= M.parts[a]) sc[a] -= M.parts[a];
  return (long long)sub_at(M, sc) * M.fs_sub + M.fs_off[f ^ 1] + face_local_index(M, p.l, a);
}

// inverse of face_side: receiving element coords and face
// (0 <= fs < n_face_sides < 2^31)
__host__ __device__ inline void face_side_decode(const Mesh& M, long long fs, int* c, int* f_out) {
  const unsigned s = fdiv((unsigned)fs, M.dfs_sub);
  const int r = (int)((unsigned)fs - s * (unsigned)M.fs_sub);
  int f = 0;
  for (int g = 0; g < 2 * M.dim; ++g)
    if (M.fs_off[g] >= 0 && r >= M.fs_off[g]) f = g;
  const int li = r - M.fs_off[f];
  const int a = f >> 1;
  const int o0 = a == 0 ? 1 : 0;
  const int o1 = a == 2 ? 1 : 2;
  const unsigned s1 = fdiv(s, M.dparts[0]);
  int sc[3] = {(int)(s - s1 * (unsigned)M.parts[0]), (int)fmodu(s1, M.dparts[1]), (int)fdiv(s1, M.dparts[1])};
  int l[3] = {0, 0, 0};
  const unsigned lq = fdiv((unsigned)li, M.dm[o0]);
  l[o0] = li - (int)lq * M.m[o0];
  if (M.dim == 3) l[o1] = (int)lq;
  l[a] = (f & 1) ? M.m[a] - 1 : 0;
  for (int k = 0; k < 3; ++k) c[k] = sc[k] * M.m[k] + l[k];
  *f_out = f;
}

// SplitMix64 (Steele, Lea, Flood 2014): draw number `idx` of the stream with
// state `seed`, i.e. the output finaliser applied to seed + (idx+1)*gamma.
__host__ __device__ inline unsigned long long splitmix64(unsigned long long seed, unsigned long long idx) {
  unsigned long long z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// delay k for (step, receiving subdomain, face direction) after the warm-up
// clamp that keeps every level read at or after the history origin
__host__ __device__ inline int delay_of(const Mesh& M, const Async& A, int sub, int f) {
  if (A.ghost == 0) return 0;
  if (A.n_rel < A.Qh - 1) return 0;
  long long k;
  if (A.delay_kind == 0) {
    k = A.L;
  } else if (A.delay_kind == 1) {
    unsigned long long idx =
        ((unsigned long long)A.n * (unsigned long long)M.nsub + (unsigned long long)sub) * (2ull * M.dim) +
        (unsigned long long)f;
    k = fmod64(splitmix64(A.seed, idx), A.kmod);  // mod (L + 1)
  } else if (A.ghost == 1 || A.ghost == 4) {
    k = fmod64((unsigned long long)A.n, A.kmod);  // Alg. caa-std: n mod L
  } else {
    const long long r = fmod64((unsigned long long)A.n, A.kmod);  // Alg. caa-at: n mod (L + Q)
    k = r < A.Qh ? 0 : r - A.Qh + 1;
  }
  long long cap = A.n_rel - A.Qh + 1;
  return (int)(k < cap ? k : cap);
}

// the most AT levels a run may use (async.levels)
constexpr int kMaxLevels = 4;

// AT weight of stored level l (0 = newest) among nlev <= 4 levels for the
// extrapolation to the fractional delay tau (eq. at-flux): the Lagrange weight
// prod_{i != l} (tau + i) / (i - l), which solves the moment constraints of
// eq. at-flux-constraints; the integer denominators enter as reciprocals
inline constexpr double kAtInvDen[5][4] = {
    {0, 0, 0, 0}, {1, 0, 0, 0}, {1, -1, 0, 0}, {0.5, -1, 0.5, 0}, {1.0 / 6, -0.5, 0.5, -1.0 / 6}};
__host__ __device__ inline double at_weight(int l, int nlev, double tau) {
  double w = kAtInvDen[nlev][l];
  for (int i = 0; i < nlev; ++i)
    if (i != l) w *= tau + i;
  return w;
}

// ---- launchers (defined in the .hip files) ---------------------------------

// Neighbour data at PE-boundary faces inside the stage kernel:
// kSrcLive   every face reads the neighbour's live stage values (synchronous);
// kSrcRing   the kernel builds the delayed / AT trace from the ring itself and,
//            at stage 0, publishes its own boundary traces (stale and AT modes);
// kSrcGhost  PE faces read a ghost buffer built by a separate kernel (learned);
// kSrcFlux   the ring holds numerical fluxes at the face Gauss points: stored
//            at stage 0 of communicating steps (delay 0), reused (FLUX_STALE)
//            or AT-extrapolated (FLUX_AT) in silent steps (Alg. caa-std /
//            caa-at).
enum GhostSrc { kSrcLive = 0, kSrcRing = 1, kSrcGhost = 2, kSrcFlux = 3 };

hipError_t launch_rhs_stage(int dim, int degree, int precision, const Mesh& M, const Async& A, const Stage& S,
                            const double* u_in, const double* u_n, double* out, int src, double* ring,
                            const double* ghost, const double* tab64, const float* tab32, hipStream_t st);
// the d = 2 stage kernel (register-resident variables, one wavefront per 16
// elements); launch_rhs_stage forwards to it for quadrilateral meshes
hipError_t launch_rhs_stage_2d(int degree, int precision, const Mesh& M, const Async& A, const Stage& S,
                               const double* u_in, const double* u_n, double* out, int src, double* ring,
                               const double* ghost, hipStream_t st);
// the d = 3 stage kernel with register-resident element data, degree 1 and 2
// (one wavefront per 12 elements); launch_rhs_stage forwards to it
hipError_t launch_rhs_stage_3d(int degree, int precision, const Mesh& M, const Async& A, const Stage& S,
                               const double* u_in, const double* u_n, double* out, int src, double* ring,
                               const double* ghost, hipStream_t st);
// the d = 3 stage kernel for degree 3, each element variable split over a
// pair of lanes (one wavefront per 6 elements); launch_rhs_stage forwards to it
hipError_t launch_rhs_stage_3d_split(int degree, int precision, const Mesh& M, const Async& A, const Stage& S,
                                     const double* u_in, const double* u_n, double* out, int src, double* ring,
                                     const double* ghost, hipStream_t st);
hipError_t launch_init(int dim, int degree, const Mesh& M, int problem, const Prm& prm, double* u,
                       const double* tab64, hipStream_t st);
hipError_t launch_norms(int dim, int degree, const Mesh& M, int what, int problem, const Prm& prm, double t,
                        const double* u, const double* ref, const double* tab64, double* partial, int nblk,
                        hipStream_t st);
hipError_t launch_reduce(const double* partial, int nblk, int ncomp, int op, double* out, hipStream_t st);
// exterior states of the boundary faces of a Dirichlet box (d = 2) at the
// stage times of one step: bnd[stage][boundary face][V][P], the exact
// solution at the face nodes
hipError_t launch_bnd_fill(int degree, const Mesh& M, int problem, const Prm& prm, const StageTimes& t,
                           const double* tab64, double* bnd, hipStream_t st);
int norms_blocks(long long E);

}  // namespace adg
