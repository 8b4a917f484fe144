/*
 * adg_oracle.h — FP64 CPU oracle for the asynchronous DG (ADG) method with
 * asynchrony-tolerant (AT) traces on the compressible Euler equations.
 *
 * TEST INFRASTRUCTURE ONLY. This is the slow, obviously-correct reference the
 * GPU library is checked against. Only the test-suite, the smoke entry and the
 * benchmark's CPU-baseline leg may load it. It shares no code, header, table or
 * generator with the GPU library: every quantity (quadrature, basis, mass matrix,
 * flux, AT weights, delay draws, MLP) is computed here from its definition.
 *
 * Everything is dense: traces and quadrature-point values are evaluated as
 * sum_j u_j * phi_j(xi) with the full tensor-product Lagrange basis; there is no
 * sum factorisation. The mass matrix is assembled by quadrature and inverted by
 * Gauss-Jordan elimination.
 */
#ifndef ADG_ORACLE_H
#define ADG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_cfg {
  int32_t dim;          /* 2 or 3 */
  int32_t p;            /* polynomial degree N_p, 1..4 */
  int32_t nq;           /* Gauss points per direction (0 -> p+2) */
  int32_t cells[3];     /* elements per direction */
  int32_t parts[3];     /* virtual subdomains per direction (block split) */
  double lo[3], hi[3];  /* the box */
  double gamma;         /* ratio of specific heats */
  int32_t flux;         /* 0: local Lax-Friedrichs as printed (lambda with 1/2), 1: Rusanov */
  int32_t ghost;        /* 0 SYNC, 1 STALE (standard flux on old traces), 2 AT, 3 LEARNED,
                           4 FLUX_STALE (Alg. caa-std: the stored flux is reused),
                           5 FLUX_AT (Alg. caa-at: AT over stored fluxes); 4 and 5 need the
                           CAA delay schedule */
  int32_t delay_kind;   /* 0 FIXED (k=L), 1 UNIFORM {0..L}, 2 CAA schedule */
  int32_t L;            /* maximum delay */
  int32_t levels;       /* AT levels (order of the extrapolation) */
  uint64_t seed;        /* seed of the delay draws */
  double learned_tol;   /* accept bound on the learned correction (physical units) */
  int32_t integrator;   /* 0 SSP-RK3 (Shu-Osher), 1 LSERK(2,2), 2 LSERK(3,3): the two-register
                           low-storage schemes of eq. lserk-dg with Table lserk-scheme;
                           3 SSP-RK2 (Heun, Shu-Osher form) */
  int32_t bc;           /* 0 periodic box; 1 Dirichlet on every side of the box (Sec. 5.1
                           vortex): the exterior state of a boundary face is the exact
                           solution of bc_problem at the stage time, and the exact
                           solutions are not wrapped periodically */
  int32_t bc_problem;   /* ORC_* problem that supplies the boundary data */
  int32_t bc_prm_set;   /* 0: the problem's default parameters; 1: bc_prm */
  double bc_prm[5];     /* parameters, as for orc_init_problem */
  int32_t learned_judge; /* 0: accept a face's correction iff max|d| <= learned_tol; 1: also
                            iff max|d| <= max|AT over 4 levels - AT over 3 levels| on the
                            face, the extrapolation's own error estimate (reading) */
} orc_cfg;

enum { ORC_VORTEX = 0, ORC_DENSITY_WAVE = 1, ORC_CONSTANT = 2 };

/* quadrature and basis */
void orc_gauss(int n, double* x, double* w);
void orc_gll(int n, double* x, double* w);
void orc_lagrange(int n, const double* nodes, double x, double* phi, double* dphi);
/* AT weights from the moment constraints; tau = k + c_m, nlev levels */
int orc_at_weights(int nlev, double tau, double* c);
/* SplitMix64 draw number `index` of the generator seeded with `seed` */
uint64_t orc_splitmix64_draw(uint64_t seed, uint64_t index);

/* solver */
void* orc_create(const orc_cfg* cfg);
void orc_destroy(void* s);
int64_t orc_ndof(void* s);
int64_t orc_nface_sides(void* s);
void orc_set_state(void* s, const double* u);
void orc_get_state(void* s, double* u);
void orc_init_problem(void* s, int problem, const double* params);
int orc_step(void* s, int64_t nsteps, double dt);
void orc_time(void* s, int64_t* n, double* t);
void orc_rhs(void* s, const double* u, double* dudt);
void orc_stage_elements(void* s, int stage, double dt, const double* u_in, const double* u_n,
                        int64_t ne, const int64_t* elems, double* out);
void orc_error_norms(void* s, int problem, const double* params, double t, double out[3]);
void orc_integrals(void* s, double* out);
int orc_delay(void* s, int64_t n, int64_t sub, int dir);
int64_t orc_subdomain(void* s, int64_t e);
/* dt from a CFL number: a reading (the paper gives no step-size rule), so
 * parity unpinned; every parity test hands the same dt to both sides */
double orc_stable_dt(void* s, double cfl);
/* n.F^ of the configured flux for n = sigma e_a, seen from the side holding wm
 * (Sec. 2.2, eq. lfflux, lfflux-lambda) */
void orc_numerical_flux(void* s, const double* wm, const double* wp, int a, double sigma, double* out);

/* learned ghost predictor (FP64 reference forward/backward) */
int orc_mlp_nparams(int nin, int nh, int nout);
void orc_mlp_forward(const double* w, int nin, int nh, int nout, int64_t n, const double* x, double* y);
double orc_mlp_loss_grad(const double* w, int nin, int nh, int nout, int64_t n, const double* x,
                         const double* y, double* grad);
void orc_mlp_forward_bf16(const float* w, int nin, int nh, int nout, int64_t n, const double* x, double* y);
void orc_adam(double* w, double* m, double* v, const double* g, int np, double lr, double b1,
              double b2, double eps, int64_t t);
void orc_set_predictor(void* s, const float* w);
void orc_learned_stats(void* s, int64_t* accepted, int64_t* rejected);
void orc_learned_features(void* s, const double* T, double tau, double cm, double* x, double* S2);
/* test hook: record the learned mode's training pairs (see adg_oracle.c) */
void orc_record_pairs(void* s, double* buf, int64_t cap);
int64_t orc_recorded_pairs(void* s);

#ifdef __cplusplus
}
#endif
#endif
