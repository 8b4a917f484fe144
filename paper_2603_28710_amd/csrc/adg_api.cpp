// adg_api.cpp — host runtime behind include/adg.h: configuration checks, the
// 1D tables (Gauss-Lobatto nodes, Gauss rule, interpolation, collocation
// derivative, inverse mass), the box (periodic or Dirichlet) and its virtual
// subdomains, the
// SSP-RK3 stage loop with its ghost/ring launches, diagnostics and
// checkpoints. All GPU work goes to the context's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/adg.h"
#include "adg_ctx.h"
#include "adg_internal.h"
#include "adg_tables.h"

using namespace adg;

namespace adg {
thread_local std::string g_err;
}

namespace {

// ---------------------------------------------------------------- 1D tables

// copy the compile-time operators for P nodes into the run-time table layout
template <int P>
void fill_tables(double* T) {
  constexpr int Q = P + 1;
  constexpr TabOff to = tab_off(P, Q);
  constexpr const ops::Ops<P>& o = ops::kOps<P>;
  for (int q = 0; q < Q; ++q) {
    for (int j = 0; j < P; ++j) {
      T[to.B + q * P + j] = o.B[q][j];
      T[to.BT + j * Q + q] = o.B[q][j];
    }
    for (int r = 0; r < Q; ++r) T[to.DT + r * Q + q] = o.D[q][r];
    T[to.WQ + q] = o.wg[q];
    T[to.XQ + q] = o.xg[q];
  }
  for (int i = 0; i < P; ++i) {
    for (int j = 0; j < P; ++j) T[to.MI + i * P + j] = o.MI[i][j];
    T[to.XL + i] = o.xl[i];
    T[to.WL + i] = o.wl[i];
    for (int q = 0; q < Q; ++q) {
      T[to.BTM + i * Q + q] = o.BTM[i][q];
      T[to.BW + i * Q + q] = o.BW[i][q];
      T[to.GW + i * Q + q] = o.GW[i][q];
    }
    T[to.MC + i] = o.MC[0][i];
    T[to.MC + P + i] = o.MC[1][i];
  }
}

bool fill_tables(int P, double* T) {
  switch (P) {
    case 2: fill_tables<2>(T); return true;
    case 3: fill_tables<3>(T); return true;
    case 4: fill_tables<4>(T); return true;
    case 5: fill_tables<5>(T); return true;
    default: return false;
  }
}

}  // namespace

namespace {

const double kSspA[3] = {0.0, 0.75, 1.0 / 3.0};
const double kSspB[3] = {1.0, 0.25, 2.0 / 3.0};
const double kSspC[3] = {0.0, 1.0, 0.5};
// SSP-RK2 (Heun) in the same form: stages (a, b) = (0, 1), (1/2, 1/2), c = (0, 1)
const double kSsp2A[2] = {0.0, 0.5}, kSsp2B[2] = {1.0, 0.5}, kSsp2C[2] = {0.0, 1.0};
// LSERK(2,2), LSERK(3,3): a_m and b_m as printed in Table lserk-scheme
const double kLs22A[2] = {1.0, 0.0}, kLs22B[2] = {0.5, 0.5};
const double kLs33A[3] = {0.755726352, 0.386954477, 0.0}, kLs33B[3] = {0.245170287, 0.184896052, 0.569933661};

int n_stages(int integrator) { return (integrator == ADG_LSERK22 || integrator == ADG_SSPRK2) ? 2 : 3; }

// stage time fraction c_m: SSP-RK3's, or c_1 = 0, c_m = b_1 + .. + b_{m-2} +
// a_{m-1} for the low-storage schemes (their own a and b, not the table's
// rounded c column)
double stage_time(int integrator, int m) {
  if (integrator == ADG_SSPRK3) return kSspC[m];
  if (integrator == ADG_SSPRK2) return kSsp2C[m];
  const double* a = integrator == ADG_LSERK22 ? kLs22A : kLs33A;
  const double* b = integrator == ADG_LSERK22 ? kLs22B : kLs33B;
  if (m == 0) return 0.0;
  double c = a[m - 1];
  for (int j = 0; j < m - 1; ++j) c += b[j];
  return c;
}

adg_status check_async(const adg_config& c, const adg_async& a) {
  if (a.ghost < 0 || a.ghost > 5) return fail(ADG_ERR_INVALID, "async.ghost must be 0..5");
  if (a.ghost >= ADG_GHOST_FLUX_STALE && a.delay_kind != ADG_DELAY_CAA)
    return fail(ADG_ERR_INVALID, "the flux-history modes need the CAA delay schedule");
  if (a.delay_kind < 0 || a.delay_kind > 2) return fail(ADG_ERR_INVALID, "async.delay_kind must be 0..2");
  if (a.L < 0 || a.L > 16) return fail(ADG_ERR_INVALID, "async.L must be in 0..16");
  if (a.levels < 1 || a.levels > 4) return fail(ADG_ERR_INVALID, "async.levels must be in 1..4");
  if ((a.ghost == 1 || a.ghost == 4) && a.delay_kind == 2 && a.L < 1)
    return fail(ADG_ERR_INVALID, "CAA with a stale trace or flux needs L >= 1");
  if (!(a.learned_tol >= 0.0)) return fail(ADG_ERR_INVALID, "async.learned_tol must be >= 0");
  if (a.learned_judge != 0 && a.learned_judge != 1) return fail(ADG_ERR_INVALID, "async.learned_judge must be 0 or 1");
  return ADG_OK;
}

void depth_of(const adg_async& a, int& R, int& Qh) {
  switch (a.ghost) {
    case 0: R = 0; Qh = 1; break;
    case 1: R = a.L + 1; Qh = 1; break;
    case 2: R = a.L + a.levels; Qh = a.levels; break;
    case 3: Qh = a.levels > kMlpK ? a.levels : kMlpK; R = a.L + Qh; break;
    case 4: R = a.L + 1; Qh = 1; break;
    default: R = a.L + a.levels; Qh = a.levels; break;
  }
}

// values per ring level: face-node traces (trace modes) or face-point fluxes
// (flux-history modes) of every PE face-side
size_t ring_level_values(const Mesh& M, int D, int P, int ghost) {
  const int Q = P + 1;
  const size_t per = ghost >= ADG_GHOST_FLUX_STALE ? (D == 3 ? Q * Q : Q) : (D == 3 ? P * P : P);
  return (size_t)M.nfs * (D + 2) * per;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Async make_async(const adg_ctx_s* c, int stage) {
  Async A{};
  A.ghost = c->as.ghost;
  A.delay_kind = c->as.delay_kind;
  A.L = c->as.L;
  A.levels = c->as.levels;
  A.Qh = c->Qh;
  A.R = c->R;
  A.seed = c->as.seed;
  A.n = c->n;
  A.n_rel = c->n - c->hist_start;
  A.stage = stage;
  A.c_m = stage_time(c->cfg.integrator, stage);
  A.tol = c->as.learned_tol;
  A.judge = c->as.learned_judge;
  A.slot_n = c->R > 0 ? (int)(c->n % c->R) : 0;
  unsigned mod = 1;
  if (A.delay_kind == 1) mod = A.L + 1;
  if (A.delay_kind == 2) mod = (A.ghost == 1 || A.ghost == 4) ? A.L : A.L + A.Qh;
  A.kmod = make_fastmod64(mod > 0 ? mod : 1);
  return A;
}

double* scratch_d(adg_ctx_s* c, size_t off) { return reinterpret_cast<double*>(c->scratch + off); }

// an analytic problem's parameters: the caller's, or the defaults
Prm problem_params(int problem, const double* params) {
  Prm prm{};
  const double def[3][5] = {{5, 5, 5, 1, 1}, {0.2, 1, 1, 1, 1}, {1, 0.3, -0.2, 0.1, 1}};
  const int pi = (problem >= 0 && problem <= 2) ? problem : 2;
  for (int i = 0; i < 5; ++i) prm.v[i] = params ? params[i] : def[pi][i];
  return prm;
}

// a norm or integral of the mesh: per-block partial sums into `partial`
// ([nblk][6]), their reduction into `red` (ncomp values), copied to host
adg_status run_norms_into(adg_ctx_s* c, int what, int problem, const double* params, const double* u,
                          const double* ref, int ncomp, int op, double* partial, double* red, double* host_out) {
  const Prm prm = problem_params(problem, params);
  const int nblk = norms_blocks(c->mesh.E);
  HIP_TRY(launch_norms(c->D, c->p, c->mesh, what, problem, prm, c->t, u, ref, c->d_tab64, partial, nblk, c->stream));
  HIP_TRY(launch_reduce(partial, nblk, ncomp, op, red, c->stream));
  HIP_TRY(hipMemcpyAsync(host_out, red, sizeof(double) * ncomp, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ADG_OK;
}

adg_status run_norms(adg_ctx_s* c, int what, int problem, const double* params, const double* u, const double* ref,
                     int ncomp, int op, double* host_out) {
  return run_norms_into(c, what, problem, params, u, ref, ncomp, op, scratch_d(c, c->partial_off),
                        scratch_d(c, c->red_off), host_out);
}

adg_status check_state(adg_ctx_s* c) {
  double r[2];
  adg_status s = run_norms(c, 3, 0, nullptr, c->u_n, nullptr, 2, 0, r);
  if (s != ADG_OK) return s;
  if (r[0] > 0) return fail(ADG_ERR_NONFINITE, "state holds non-finite values at step " + std::to_string(c->n));
  if (r[1] > 0) return fail(ADG_ERR_NONPHYSICAL, "density or pressure <= 0 at step " + std::to_string(c->n));
  return ADG_OK;
}

}  // namespace

// ---- event timing --------------------------------------------------------
constexpr int kProfPairs = 2048;

adg_status adg::prof_fold(adg_ctx_s* c) {
  auto& P = c->prof;
  if (!P.used) return ADG_OK;
  HIP_TRY(hipEventSynchronize(P.ev[2 * (P.used - 1) + 1]));
  for (int i = 0; i < P.used; ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, P.ev[2 * i], P.ev[2 * i + 1]));
    P.ms[P.kind[i]] += ms;
    P.cnt[P.kind[i]] += 1;
  }
  P.used = 0;
  return ADG_OK;
}

adg_status adg::prof_begin(adg_ctx_s* c, int kind) {
  auto& P = c->prof;
  if (!P.on || c->n % P.every) return ADG_OK;
  if (P.used == kProfPairs) {
    adg_status s = prof_fold(c);
    if (s != ADG_OK) return s;
  }
  P.kind[P.used] = kind;
  HIP_TRY(hipEventRecord(P.ev[2 * P.used], c->stream));
  return ADG_OK;
}

adg_status adg::prof_end(adg_ctx_s* c) {
  auto& P = c->prof;
  if (!P.on || c->n % P.every) return ADG_OK;
  HIP_TRY(hipEventRecord(P.ev[2 * P.used + 1], c->stream));
  P.used += 1;
  return ADG_OK;
}

#define PROF_TRY(x)                \
  do {                             \
    adg_status _s = (x);           \
    if (_s != ADG_OK) return _s;   \
  } while (0)

// one stage m of the step: the boundary data (Dirichlet box, at m = 0), the
// learned ghost traces (learned mode or pair collection), then the fused
// stage kernel
static adg_status run_stage(adg_ctx_s* c, int m, double dt, bool learned_collect, long long pair_base) {
  // registers per stage. SSP-RK3: inputs u_n, u_a, u_b; outputs u_a, u_b,
  // u_n. SSP-RK2: u_n -> u_a, then u_a -> u_n (in place; each element reads
  // its own u^n before writing). LSERK (w the accumulator, r the stage input; no stage writes the
  // register its neighbours read):
  //   (2,2): r1 = w0 = u_n -> w1 u_a, r2 u_b;  r2 = u_b, w1 = u_a -> w2 u_n
  //   (3,3): as (2,2) at m = 0; r2 = u_b, w1 = u_a -> w2 u_n, r3 u_a (in
  //          place over w1); r3 = u_a, w2 = u_n -> w3 u_n (in place)
  const int ig = c->cfg.integrator;
  double* in[3] = {c->u_n, c->u_a, c->u_b};
  double* out[3] = {c->u_a, c->u_b, c->u_n};
  double* wreg = c->u_n;  // the operand read as u_n by the combine
  double* out2 = nullptr;
  if (ig == ADG_SSPRK2) out[1] = c->u_n;  // u1 in u_a; the second stage in place over u_n
  if (ig == ADG_LSERK22 || ig == ADG_LSERK33) {
    double* lin[3] = {c->u_n, c->u_b, c->u_a};
    double* lw[3] = {c->u_n, c->u_a, c->u_n};
    double* lout[3] = {c->u_a, c->u_n, c->u_n};
    double* lout2[3] = {c->u_b, ig == ADG_LSERK33 ? c->u_a : nullptr, nullptr};
    in[m] = lin[m];
    wreg = lw[m];
    out[m] = lout[m];
    out2 = lout2[m];
  }
  Async A = make_async(c, m);
  double* ghost = scratch_d(c, c->ghost_off);
  // stale and AT traces are built inside the stage kernel from the ring; the
  // learned predictor (and pair collection) runs as its own kernel first
  int src = kSrcLive;
  if (A.ghost != 0 && c->mesh.nfs > 0) {
    if (A.ghost >= ADG_GHOST_FLUX_STALE) {
      src = kSrcFlux;
    } else if (A.ghost == 3 || learned_collect) {
      PROF_TRY(prof_begin(c, ADG_KERNEL_GHOST));
      HIP_TRY(launch_ghost_learned(c->D, c->p, c->mesh, A, in[m], c->u_n, c->ring, ghost, m == 0, c->mlp,
                                   pair_base, learned_collect, c->stream));
      PROF_TRY(prof_end(c));
      src = kSrcGhost;
    } else {
      src = kSrcRing;
    }
  }
  Stage S{kSspA[m % 3], kSspB[m % 3], dt, 0, 0.0, 0.0, nullptr, nullptr};
  if (ig == ADG_SSPRK2) {
    S.a = kSsp2A[m];
    S.b = kSsp2B[m];
  }
  if (c->mesh.bc) {
    // the boundary data of every stage of the step, in one launch at stage 0
    double* bnd = scratch_d(c, c->bnd_off);
    if (m == 0) {
      StageTimes T{};
      T.n = n_stages(ig);
      for (int j = 0; j < T.n; ++j) T.t[j] = c->t + stage_time(ig, j) * dt;
      HIP_TRY(launch_bnd_fill(c->p, c->mesh, c->bc_problem, c->bc_prm, T, c->d_tab64, bnd, c->stream));
    }
    S.bnd = bnd + (size_t)m * c->mesh.nbf * c->V * c->P;
  }
  if (ig == ADG_LSERK22 || ig == ADG_LSERK33) {
    S.lserk = 1;
    S.bw = ig == ADG_LSERK22 ? kLs22B[m] : kLs33B[m];
    S.ar = ig == ADG_LSERK22 ? kLs22A[m] : kLs33A[m];
    S.out2 = out2;
  }
  PROF_TRY(prof_begin(c, ADG_KERNEL_RHS));
  HIP_TRY(launch_rhs_stage(c->D, c->p, c->cfg.precision, c->mesh, A, S, in[m], wreg, out[m], src, c->ring,
                           ghost, c->d_tab64, c->d_tab32, c->stream));
  PROF_TRY(prof_end(c));
  return ADG_OK;
}

adg_status adg::adg_step_impl(adg_ctx c, int64_t n_steps, double dt, bool collect) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (n_steps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return fail(ADG_ERR_INVALID, "need n_steps >= 0, dt > 0");
  if (c->as.ghost != 0 && c->mesh.nfs > 0 && c->R > 0 && !c->ring) return fail(ADG_ERR_UNBOUND, "ring not bound");
  if (c->mesh.bc && c->bc_problem < 0)
    return fail(ADG_ERR_STATE, "a Dirichlet box needs its boundary problem (adg_set_boundary or adg_init_problem)");
  const int ce = c->cfg.check_every;
  for (int64_t it = 0; it < n_steps; ++it) {
    for (int m = 0; m < n_stages(c->cfg.integrator); ++m) {
      // collection writes one pair slot per PE-boundary face node and stage
      const long long per = c->mesh.nfs * (long long)c->Fn;
      const bool col = collect && per > 0 && c->mlp.n_pairs + per <= c->mlp.max_pairs;
      adg_status s = run_stage(c, m, dt, col, col ? c->mlp.n_pairs : 0);
      if (s != ADG_OK) return s;
      if (col) c->mlp.n_pairs += per;
    }
    c->n += 1;
    c->t += dt;
    if (ce > 0 && (c->n % ce == 0 || it == n_steps - 1)) {
      adg_status s = check_state(c);
      if (s != ADG_OK) return s;
    }
  }
  return ADG_OK;
}


// ----------------------------------------------------------------- C ABI

extern "C" {

const char* adg_last_error(void) { return adg::g_err.c_str(); }

adg_status adg_create(const adg_config* cfg, const adg_async* async, void* hip_stream, adg_ctx* out) {
  if (!cfg || !async || !out) return fail(ADG_ERR_INVALID, "null argument");
  *out = nullptr;
  const adg_config& c = *cfg;
  if (c.dim != 2 && c.dim != 3) return fail(ADG_ERR_INVALID, "dim must be 2 or 3");
  if (c.degree < 1 || c.degree > 4) return fail(ADG_ERR_INVALID, "degree must be in 1..4");
  if (c.n_q != 0 && c.n_q != c.degree + 2) return fail(ADG_ERR_INVALID, "n_q must be 0 or degree+2");
  if (!(c.gamma > 1.0)) return fail(ADG_ERR_INVALID, "gamma must be > 1");
  if (c.flux != ADG_FLUX_LLF && c.flux != ADG_FLUX_RUSANOV) return fail(ADG_ERR_INVALID, "unknown flux");
  if (c.integrator != ADG_SSPRK3 && c.integrator != ADG_LSERK22 && c.integrator != ADG_LSERK33 &&
      c.integrator != ADG_SSPRK2)
    return fail(ADG_ERR_INVALID, "unknown integrator");
  if (c.precision != ADG_FP64 && c.precision != ADG_FP32_CONTRACT) return fail(ADG_ERR_INVALID, "unknown precision");
  if (c.check_every < 0) return fail(ADG_ERR_INVALID, "check_every must be >= 0");
  if (c.boundary != ADG_BC_PERIODIC && c.boundary != ADG_BC_DIRICHLET) return fail(ADG_ERR_INVALID, "unknown boundary");
  if (c.boundary == ADG_BC_DIRICHLET && c.dim != 2)
    return fail(ADG_ERR_INVALID, "Dirichlet boundaries are implemented for d = 2");
  for (int k = 0; k < c.dim; ++k) {
    if (c.cells[k] < 1 || c.parts[k] < 1) return fail(ADG_ERR_INVALID, "cells and parts must be >= 1");
    if (c.cells[k] % c.parts[k]) return fail(ADG_ERR_INVALID, "cells must be divisible by parts");
    if (!(c.hi[k] > c.lo[k])) return fail(ADG_ERR_INVALID, "hi must exceed lo");
  }
  adg_status st = check_async(c, *async);
  if (st != ADG_OK) return st;
  long long E = 1;
  for (int k = 0; k < c.dim; ++k) E *= c.cells[k];
  if (E > (1ll << 31)) return fail(ADG_ERR_INVALID, "too many elements");

  adg_ctx_s* x = new adg_ctx_s();
  x->cfg = c;
  x->as = *async;
  x->stream = reinterpret_cast<hipStream_t>(hip_stream);
  x->D = c.dim;
  x->p = c.degree;
  x->P = c.degree + 1;
  x->Q = c.degree + 2;
  x->V = c.dim + 2;
  x->Pd = x->P * x->P * (c.dim == 3 ? x->P : 1);
  x->Fn = x->Pd / x->P;

  Mesh& M = x->mesh;
  M.dim = c.dim;
  M.E = E;
  M.nsub = 1;
  M.detJ = 1.0;
  for (int k = 0; k < 3; ++k) {
    const bool on = k < c.dim;
    M.nc[k] = on ? c.cells[k] : 1;
    M.parts[k] = on ? c.parts[k] : 1;
    M.m[k] = M.nc[k] / M.parts[k];
    M.nsub *= M.parts[k];
    M.lo[k] = on ? c.lo[k] : 0.0;
    M.hi[k] = on ? c.hi[k] : 1.0;
    M.h[k] = on ? (c.hi[k] - c.lo[k]) / c.cells[k] : 2.0;
    if (on) M.detJ *= 0.5 * M.h[k];
  }
  for (int a = 0; a < 3; ++a) {
    M.detJf[a] = 1.0;
    for (int k = 0; k < c.dim; ++k)
      if (k != a) M.detJf[a] *= 0.5 * M.h[k];
  }
  M.gamma = c.gamma;
  M.flux = c.flux;
  M.bc = c.boundary == ADG_BC_DIRICHLET ? 1 : 0;
  M.bnd_off[0] = 0;
  M.bnd_off[1] = M.nc[1];
  M.bnd_off[2] = 2 * M.nc[1];
  M.bnd_off[3] = 2 * M.nc[1] + M.nc[0];
  M.nbf = M.bc ? 2 * (M.nc[0] + M.nc[1]) : 0;
  for (int k = 0; k < 2; ++k) M.dnc[k] = make_fastdiv(M.nc[k]);
  for (int k = 0; k < 3; ++k) M.dm[k] = make_fastdiv(M.m[k]);
  for (int k = 0; k < 2; ++k) M.dparts[k] = make_fastdiv(M.parts[k]);
  int off = 0;
  for (int f = 0; f < 6; ++f) {
    M.fs_off[f] = -1;
    if (f >= 2 * c.dim) continue;
    const int a = f / 2;
    if (M.parts[a] < 2) continue;
    int A = 1;
    for (int k = 0; k < c.dim; ++k)
      if (k != a) A *= M.m[k];
    M.fs_off[f] = off;
    off += A;
  }
  M.fs_sub = off;
  M.nfs = (long long)off * M.nsub;
  M.dfs_sub = make_fastdiv(off > 0 ? off : 1);
  if (M.nfs >= (1ll << 31)) {
    delete x;
    return fail(ADG_ERR_INVALID, "too many PE-boundary face-sides");
  }
  x->ndof = (size_t)E * x->V * x->Pd;
  depth_of(x->as, x->R, x->Qh);

  // 1D tables
  const int P = x->P, Q = x->Q;
  const TabOff to = tab_off(P, Q);
  x->tab64.assign(to.total, 0.0);
  if (!fill_tables(P, x->tab64.data())) {
    delete x;
    return fail(ADG_ERR_INVALID, "degree out of range");
  }
  // buffer plan
  x->ring_bytes = (size_t)x->R * ring_level_values(M, x->D, x->P, x->as.ghost) * sizeof(double);
  size_t s = 0;
  x->ghost_off = s;
  s = align256(s + (size_t)M.nfs * x->V * x->Fn * sizeof(double));
  x->partial_off = s;
  s = align256(s + 2048 * 6 * sizeof(double));
  x->red_off = s;
  s = align256(s + 16 * sizeof(double));
  x->mlp_off = s;
  s = align256(s + mlp_scratch_bytes(x->V));
  x->bnd_off = s;
  s = align256(s + (size_t)3 * M.nbf * x->V * x->P * sizeof(double));
  x->scratch_bytes = s;
  mlp_init(x->mlp, x->V);
  *out = x;
  return ADG_OK;
}

adg_status adg_destroy(adg_ctx c) {
  if (!c) return ADG_OK;
  for (auto& e : c->prof.ev) hipEventDestroy(e);
  if (c->d_tab64) {
    hipStreamSynchronize(c->stream);
    hipFree(c->d_tab64);
    hipFree(c->d_tab32);
  }
  delete c;
  return ADG_OK;
}

adg_status adg_sizes(adg_ctx c, size_t* n_dof, size_t* state_bytes, size_t* ring_bytes, size_t* scratch_bytes) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (n_dof) *n_dof = c->ndof;
  if (state_bytes) *state_bytes = c->ndof * sizeof(double);
  if (ring_bytes) *ring_bytes = c->ring_bytes;
  if (scratch_bytes) *scratch_bytes = c->scratch_bytes;
  return ADG_OK;
}

adg_status adg_bind(adg_ctx c, void* u_n, void* u_a, void* u_b, void* ring, void* scratch) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (!u_n || !u_a || !u_b || !scratch) return fail(ADG_ERR_INVALID, "state registers and scratch are required");
  if (c->ring_bytes && !ring) return fail(ADG_ERR_INVALID, "this asynchrony mode needs a ring buffer");
  void* ptrs[5] = {u_n, u_a, u_b, ring, scratch};
  for (void* p : ptrs)
    if (reinterpret_cast<uintptr_t>(p) % 256) return fail(ADG_ERR_INVALID, "buffers must be 256-byte aligned");
  if (u_n == u_a || u_n == u_b || u_a == u_b) return fail(ADG_ERR_INVALID, "state registers must be distinct");
  c->u_n = static_cast<double*>(u_n);
  c->u_a = static_cast<double*>(u_a);
  c->u_b = static_cast<double*>(u_b);
  c->ring = static_cast<double*>(ring);
  c->ring_cap = ring ? c->ring_bytes : 0;
  c->scratch = static_cast<char*>(scratch);
  if (c->device < 0) HIP_TRY(hipGetDevice(&c->device));
  if (!c->d_tab64) {
    const int nt = (int)c->tab64.size();
    std::vector<float> t32(nt);
    for (int i = 0; i < nt; ++i) t32[i] = (float)c->tab64[i];
    HIP_TRY(hipMalloc(&c->d_tab64, sizeof(double) * nt));
    HIP_TRY(hipMalloc(&c->d_tab32, sizeof(float) * nt));
    HIP_TRY(hipMemcpyAsync(c->d_tab64, c->tab64.data(), sizeof(double) * nt, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->d_tab32, t32.data(), sizeof(float) * nt, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  c->mlp.base = c->scratch + c->mlp_off;
  c->bound = true;
  return mlp_on_bind(c);
}

adg_status adg_upload(adg_ctx c, const double* host, size_t n) {
  if (!c || !host) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (n != c->ndof) return fail(ADG_ERR_INVALID, "size mismatch: expected " + std::to_string(c->ndof));
  HIP_TRY(hipMemcpyAsync(c->u_n, host, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->n = 0;
  c->hist_start = 0;
  c->t = 0.0;
  mlp_reset_stats(c);
  return ADG_OK;
}

adg_status adg_download(adg_ctx c, double* host, size_t n) {
  if (!c || !host) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (n != c->ndof) return fail(ADG_ERR_INVALID, "size mismatch: expected " + std::to_string(c->ndof));
  HIP_TRY(hipMemcpyAsync(host, c->u_n, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ADG_OK;
}

adg_status adg_init_problem(adg_ctx c, int32_t problem, const double* params) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (problem < 0 || problem > 2) return fail(ADG_ERR_INVALID, "unknown problem");
  if (problem == ADG_VORTEX && c->D != 2) return fail(ADG_ERR_INVALID, "the vortex is a 2D problem");
  const Prm prm = problem_params(problem, params);
  HIP_TRY(launch_init(c->D, c->p, c->mesh, problem, prm, c->u_n, c->d_tab64, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->bc_problem = problem;
  c->bc_prm = prm;
  c->n = 0;
  c->hist_start = 0;
  c->t = 0.0;
  mlp_reset_stats(c);
  return ADG_OK;
}

adg_status adg_set_boundary(adg_ctx c, int32_t problem, const double* params) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (problem < 0 || problem > 2) return fail(ADG_ERR_INVALID, "unknown problem");
  if (problem == ADG_VORTEX && c->D != 2) return fail(ADG_ERR_INVALID, "the vortex is a 2D problem");
  c->bc_problem = problem;
  c->bc_prm = problem_params(problem, params);
  return ADG_OK;
}

adg_status adg_set_async(adg_ctx c, const adg_async* a) {
  if (!c || !a) return fail(ADG_ERR_INVALID, "null argument");
  adg_status s = check_async(c->cfg, *a);
  if (s != ADG_OK) return s;
  int R, Qh;
  depth_of(*a, R, Qh);
  const size_t need = (size_t)R * ring_level_values(c->mesh, c->D, c->P, a->ghost) * sizeof(double);
  if (c->bound && need > c->ring_cap)
    return fail(ADG_ERR_INVALID, "ring bound at adg_bind is too small for this depth (" + std::to_string(need) +
                                     " bytes needed)");
  if (c->bound) HIP_TRY(hipStreamSynchronize(c->stream));
  c->as = *a;
  c->R = R;
  c->Qh = Qh;
  if (!c->bound) c->ring_bytes = need;
  c->hist_start = c->n;
  mlp_reset_stats(c);
  return ADG_OK;
}

adg_status adg_step(adg_ctx c, int64_t n_steps, double dt) { return adg_step_impl(c, n_steps, dt, false); }

adg_status adg_delay(adg_ctx c, int64_t n, int32_t sub, int32_t dir, int32_t* k, int64_t* n_face_sides) {
  if (!c || !k) return fail(ADG_ERR_INVALID, "null argument");
  if (sub < 0 || sub >= c->mesh.nsub || dir < 0 || dir >= 2 * c->D || n < c->hist_start)
    return fail(ADG_ERR_INVALID, "subdomain, direction or step out of range");
  const int64_t keep = c->n;
  c->n = n;
  Async A = make_async(c, 0);
  c->n = keep;
  *k = delay_of(c->mesh, A, sub, dir);
  if (n_face_sides) *n_face_sides = c->mesh.nfs;
  return ADG_OK;
}

adg_status adg_basis(adg_ctx c, double* gll_x, double* gll_w, double* gauss_x, double* gauss_w) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  const TabOff to = tab_off(c->P, c->Q);
  for (int j = 0; j < c->P; ++j) {
    if (gll_x) gll_x[j] = c->tab64[to.XL + j];
    if (gll_w) gll_w[j] = c->tab64[to.WL + j];
  }
  for (int q = 0; q < c->Q; ++q) {
    if (gauss_x) gauss_x[q] = c->tab64[to.XQ + q];
    if (gauss_w) gauss_w[q] = c->tab64[to.WQ + q];
  }
  return ADG_OK;
}

adg_status adg_profile(adg_ctx c, int32_t enable) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (enable < 0) return fail(ADG_ERR_INVALID, "enable must be >= 0");
  auto& P = c->prof;
  if (enable) {
    P.every = enable;
    if (P.ev.empty()) {
      P.ev.resize(2 * kProfPairs);
      P.kind.resize(kProfPairs);
      for (auto& e : P.ev) HIP_TRY(hipEventCreate(&e));
    }
    P.used = 0;
    P.ms[0] = P.ms[1] = 0.0;
    P.cnt[0] = P.cnt[1] = 0;
    P.on = true;
  } else {
    adg_status s = prof_fold(c);
    P.on = false;
    if (s != ADG_OK) return s;
  }
  return ADG_OK;
}

adg_status adg_profile_read(adg_ctx c, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!c || (kernel != ADG_KERNEL_RHS && kernel != ADG_KERNEL_GHOST)) return fail(ADG_ERR_INVALID, "bad argument");
  adg_status s = prof_fold(c);
  if (s != ADG_OK) return s;
  if (total_ms) *total_ms = c->prof.ms[kernel];
  if (launches) *launches = c->prof.cnt[kernel];
  return ADG_OK;
}

adg_status adg_time(adg_ctx c, int64_t* n, double* t) {
  if (!c) return fail(ADG_ERR_INVALID, "null context");
  if (n) *n = c->n;
  if (t) *t = c->t;
  return ADG_OK;
}

adg_status adg_stable_dt(adg_ctx c, double cfl, double* dt) {
  if (!c || !dt) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (!(cfl > 0.0)) return fail(ADG_ERR_INVALID, "cfl must be > 0");
  double smax = 0.0;
  adg_status s = run_norms(c, 4, 0, nullptr, c->u_n, nullptr, 1, 1, &smax);
  if (s != ADG_OK) return s;
  if (!(smax > 0.0)) return fail(ADG_ERR_NONPHYSICAL, "no finite positive wave speed in the state");
  double hmin = c->mesh.h[0];
  for (int k = 1; k < c->D; ++k) hmin = std::min(hmin, c->mesh.h[k]);
  *dt = cfl * hmin / (std::pow((double)c->p, 1.5) * smax);
  return ADG_OK;
}

adg_status adg_error_norms(adg_ctx c, int32_t problem, const double* params, double out[3]) {
  if (!c || !out) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  if (problem < 0 || problem > 2) return fail(ADG_ERR_INVALID, "unknown problem");
  double r[3];
  adg_status s = run_norms(c, 0, problem, params, c->u_n, nullptr, 3, 0, r);
  if (s != ADG_OK) return s;
  for (int i = 0; i < 3; ++i) out[i] = std::sqrt(r[i]);
  return ADG_OK;
}

adg_status adg_diff_norm(adg_ctx c, const double* host_ref, double out[3]) {
  if (!c || !host_ref || !out) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  // u_a is free between steps: stage the reference there
  HIP_TRY(hipMemcpyAsync(c->u_a, host_ref, c->ndof * sizeof(double), hipMemcpyHostToDevice, c->stream));
  double r[6];
  adg_status s = run_norms(c, 2, 0, nullptr, c->u_n, c->u_a, 6, 0, r);
  if (s != ADG_OK) return s;
  for (int g = 0; g < 3; ++g) out[g] = r[3 + g] > 0 ? std::sqrt(r[g] / r[3 + g]) : std::sqrt(r[g]);
  return ADG_OK;
}

adg_status adg_integrals(adg_ctx c, double* out) {
  if (!c || !out) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  return run_norms(c, 1, 0, nullptr, c->u_n, nullptr, c->V, 0, out);
}

}  // extern "C"

// ---- adg_integrals without the bound scratch ------------------------------
// The per-block partial sums ([2048][6] doubles, the most blocks the norm
// kernels use) and the reduced values (up to 32) live in a file-scope device
// array, one copy per GPU, held until the process ends. Host code reaches it
// only through the address hipGetSymbolAddress returns on each device.
namespace {
constexpr int kStaticPartial = 2048 * 6;
constexpr int kStaticDoubles = kStaticPartial + 32;
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
double* g_static_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) double scratch[kStaticDoubles];

namespace {
// the device address of `scratch` on device dev (the current device),
// looked up once per device
adg_status static_scratch(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ADG_ERR_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ADG_ERR_HIP, "hipGetSymbolAddress returned no address for the static scratch");
    g_static_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_static_ptr[dev];
  return ADG_OK;
}
}  // namespace

extern "C" {

adg_status adg_integrals_noalloc(adg_ctx c, double* out) {
  if (!c || !out) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != c->device)
    return fail(ADG_ERR_STATE, "adg_integrals_noalloc: make the context's device (" + std::to_string(c->device) +
                                   ") current");
  const int nblk = norms_blocks(c->mesh.E);
  if ((long long)nblk * 6 > kStaticPartial || c->V > 6)
    return fail(ADG_ERR_INVALID, "adg_integrals_noalloc: " + std::to_string(nblk) +
                                     " partial blocks exceed the static scratch of 2048");
  double* base = nullptr;
  adg_status s = static_scratch(dev, &base);
  if (s != ADG_OK) return s;
  // every partial the reduction reads and every value it returns is written
  // by this call's kernels first, so nothing needs clearing
  return run_norms_into(c, 1, 0, nullptr, c->u_n, nullptr, c->V, 0, base, base + kStaticPartial, out);
}

// checkpoint blob: header, u_n, ring, predictor weights
struct BlobHeader {
  char magic[8];
  int32_t version, dim, degree, V;
  int64_t ndof, ring_bytes, nparams;
  int64_t n, hist_start;
  double t;
  int32_t ghost, delay_kind, L, levels;
  uint64_t seed;
  int32_t boundary, bc_problem;  // the box and the problem of its boundary data (-1: none set)
  double bc_prm[5];
};

adg_status adg_save(adg_ctx c, void* host_blob, size_t* bytes) {
  if (!c || !bytes) return fail(ADG_ERR_INVALID, "null argument");
  const size_t np = (size_t)mlp_nparams(c->V);
  const size_t need = sizeof(BlobHeader) + c->ndof * sizeof(double) + c->ring_bytes + np * sizeof(float);
  if (!host_blob) {
    *bytes = need;
    return ADG_OK;
  }
  if (*bytes < need) return fail(ADG_ERR_INVALID, "blob too small");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  BlobHeader h{};
  std::memcpy(h.magic, "ADGCKPT", 8);
  h.version = 2;
  h.dim = c->D;
  h.degree = c->p;
  h.V = c->V;
  h.ndof = (int64_t)c->ndof;
  h.ring_bytes = (int64_t)c->ring_bytes;
  h.nparams = (int64_t)np;
  h.n = c->n;
  h.hist_start = c->hist_start;
  h.t = c->t;
  h.ghost = c->as.ghost;
  h.delay_kind = c->as.delay_kind;
  h.L = c->as.L;
  h.levels = c->as.levels;
  h.seed = c->as.seed;
  h.boundary = c->cfg.boundary;
  h.bc_problem = c->bc_problem;
  for (int i = 0; i < 5; ++i) h.bc_prm[i] = c->bc_prm.v[i];
  char* b = static_cast<char*>(host_blob);
  std::memcpy(b, &h, sizeof(h));
  b += sizeof(h);
  HIP_TRY(hipMemcpyAsync(b, c->u_n, c->ndof * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  b += c->ndof * sizeof(double);
  if (c->ring_bytes) HIP_TRY(hipMemcpyAsync(b, c->ring, c->ring_bytes, hipMemcpyDeviceToHost, c->stream));
  b += c->ring_bytes;
  HIP_TRY(hipStreamSynchronize(c->stream));
  mlp_get_host(c, reinterpret_cast<float*>(b));
  *bytes = need;
  return ADG_OK;
}

adg_status adg_load(adg_ctx c, const void* host_blob, size_t bytes) {
  if (!c || !host_blob) return fail(ADG_ERR_INVALID, "null argument");
  if (!c->bound) return fail(ADG_ERR_UNBOUND, "buffers not bound");
  BlobHeader h;
  if (bytes < sizeof(h)) return fail(ADG_ERR_INVALID, "blob too small");
  std::memcpy(&h, host_blob, sizeof(h));
  const size_t np = (size_t)mlp_nparams(c->V);
  if (std::memcmp(h.magic, "ADGCKPT", 8) || h.version != 2 || h.dim != c->D || h.degree != c->p ||
      h.boundary != c->cfg.boundary ||
      h.ndof != (int64_t)c->ndof || h.ring_bytes != (int64_t)c->ring_bytes || h.nparams != (int64_t)np)
    return fail(ADG_ERR_INVALID, "blob does not match this configuration");
  if (bytes < sizeof(h) + c->ndof * sizeof(double) + c->ring_bytes + np * sizeof(float))
    return fail(ADG_ERR_INVALID, "blob truncated");
  adg_async a = c->as;
  a.ghost = h.ghost;
  a.delay_kind = h.delay_kind;
  a.L = h.L;
  a.levels = h.levels;
  a.seed = h.seed;
  adg_status s = adg_set_async(c, &a);
  if (s != ADG_OK) return s;
  const char* b = static_cast<const char*>(host_blob) + sizeof(h);
  HIP_TRY(hipMemcpyAsync(c->u_n, b, c->ndof * sizeof(double), hipMemcpyHostToDevice, c->stream));
  b += c->ndof * sizeof(double);
  if (c->ring_bytes) HIP_TRY(hipMemcpyAsync(c->ring, b, c->ring_bytes, hipMemcpyHostToDevice, c->stream));
  b += c->ring_bytes;
  HIP_TRY(hipStreamSynchronize(c->stream));
  s = mlp_set_host(c, reinterpret_cast<const float*>(b));
  if (s != ADG_OK) return s;
  c->n = h.n;
  c->hist_start = h.hist_start;
  c->t = h.t;
  if (h.bc_problem >= 0) {
    c->bc_problem = h.bc_problem;
    for (int i = 0; i < 5; ++i) c->bc_prm.v[i] = h.bc_prm[i];
  }
  return ADG_OK;
}

}  // extern "C"
