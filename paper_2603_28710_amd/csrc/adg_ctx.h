// adg_ctx.h — the library context behind the opaque adg_ctx handle and the
// error helpers shared by the host-side translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/adg.h"
#include "adg_internal.h"
#include "adg_mlp.h"

namespace adg {
extern thread_local std::string g_err;
inline adg_status fail(adg_status code, const std::string& msg) {
  g_err = msg;
  return code;
}
}  // namespace adg

#define HIP_TRY(expr)                                                                                   \
  do {                                                                                                  \
    hipError_t _e = (expr);                                                                             \
    if (_e != hipSuccess) return adg::fail(ADG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)


struct adg_ctx_s {
  adg_config cfg;
  adg_async as;
  hipStream_t stream = nullptr;
  int D = 0, p = 0, P = 0, Q = 0, V = 0, Pd = 0, Fn = 0;
  adg::Mesh mesh{};
  size_t ndof = 0;
  int R = 0, Qh = 1;
  size_t ring_bytes = 0, ring_cap = 0, scratch_bytes = 0;
  size_t ghost_off = 0, partial_off = 0, red_off = 0, mlp_off = 0, bnd_off = 0;
  // Dirichlet box: the problem whose exact solution gives the boundary data
  int bc_problem = -1;
  adg::Prm bc_prm{};
  double *u_n = nullptr, *u_a = nullptr, *u_b = nullptr, *ring = nullptr;
  char* scratch = nullptr;
  bool bound = false;
  int device = -1;  // the HIP device current at the first adg_bind
  double* d_tab64 = nullptr;
  float* d_tab32 = nullptr;
  std::vector<double> tab64;
  int64_t n = 0, hist_start = 0;
  double t = 0.0;
  // learned predictor
  adg::MlpState mlp;
  // event timing of the stage kernels (adg_profile)
  struct Prof {
    bool on = false;
    int every = 1;               // record the launches of steps n with n % every == 0
    std::vector<hipEvent_t> ev;  // pairs (start, end)
    std::vector<int> kind;       // kernel id per recorded pair
    int used = 0;
    double ms[2] = {0.0, 0.0};
    int64_t cnt[2] = {0, 0};
  } prof;
};


namespace adg {
void mlp_reset_stats(adg_ctx_s* c);
void mlp_get_host(adg_ctx_s* c, float* w);
adg_status mlp_set_host(adg_ctx_s* c, const float* w);
adg_status mlp_on_bind(adg_ctx_s* c);
adg_status prof_begin(adg_ctx_s* c, int kind);
adg_status prof_end(adg_ctx_s* c);
adg_status prof_fold(adg_ctx_s* c);
adg_status adg_step_impl(adg_ctx c, int64_t n_steps, double dt, bool collect);
}
