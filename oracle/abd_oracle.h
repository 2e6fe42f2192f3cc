/*
 * Plain FP64 CPU oracle for one worker's local affine-body Newton solve
 * (Eq. 5, Sec. 4.1) -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the HIP library; both are driven from the seeded scene
 * generator.  Everything here is written for a reader to check by eye
 * against the paper and the mathematics it defers to: no blocking, no
 * fusion, no FMA contraction (built with -ffp-contract=off).
 *
 * Conventions: a body's DoFs are q = [p (3), A row-major (9)]; vertex
 * positions are x = A xbar + p; arrays are FP64, AoS ([n][3] for points,
 * [n][12] for bodies, [n][144] row-major for 12x12 blocks).
 */
#ifndef ABD_ORACLE_H
#define ABD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_E_INVALID_ARG (-1)
#define ORC_E_MESH (-2)
#define ORC_E_INFEASIBLE (-3)
#define ORC_E_NOCONV (-4)
#define ORC_E_LINESEARCH (-5)
#define ORC_E_CAPACITY (-6)

#define ORC_PT 0
#define ORC_EE 1
#define ORC_PG 2

typedef struct orc_params {
  double dt, dhat, kappa, kappa_A;
  double gravity[3];
  double newton_theta, pcg_eta;
  double ground_y;
  int32_t max_newton, max_pcg, max_ls;
  int32_t has_ground, mollify_ee;
  int32_t dense_max_dof; /* dense Cholesky when 12*dynamic bodies <= this */
} orc_params;

typedef struct orc_stats {
  int32_t newton_iters, pcg_iters_total, ls_halvings, status;
  double final_eps_N, min_alpha, min_dist, scene_scale;
  int64_t n_cand_pt, n_cand_ee, n_cand_pg, n_active;
} orc_stats;

typedef struct orc_scene orc_scene;

/* ---- scene ---- */
orc_scene* orc_create(const orc_params* p);
void orc_destroy(orc_scene* s);
const char* orc_last_error(const orc_scene* s);
/* returns the body id (>= 0) or a negative status */
int orc_add_body(orc_scene* s, const double* xbar, int32_t nv,
                 const int32_t* tris, int32_t nt, double density,
                 const double* q0, const double* qdot0, int32_t kind);
int orc_finalize(orc_scene* s);
/* sizes[0..3] = bodies, vertices, triangles, edges */
int orc_sizes(const orc_scene* s, int64_t* sizes);
/* rest data of every edge: [E][2] global vertex ids */
int orc_edges(const orc_scene* s, int32_t* out);
/* body mass matrix blocks: [B][16] (4x4) and volumes [B] */
int orc_body_mass(const orc_scene* s, double* Mhat, double* vol);
int orc_set_shared(orc_scene* s, const int32_t* ids, int32_t n,
                   const double* z, const double* u, const double* rho,
                   const int32_t* kappa_b);
int orc_set_pair_replication(orc_scene* s, int32_t mode);
/* PSD projection of pair and orthogonality Hessians (default on); off
 * exposes the exact Hessian for finite-difference pins */
int orc_set_projection(orc_scene* s, int32_t on);
int orc_begin_step(orc_scene* s);
int orc_local_solve(orc_scene* s, orc_stats* st);
int orc_end_step(orc_scene* s);
int orc_get_state(const orc_scene* s, double* q, double* qdot);
int orc_set_state(orc_scene* s, const double* q, const double* qdot);
int orc_get_qtilde(const orc_scene* s, double* qtilde);
/* prescribe step-start data directly (q^t, q-tilde, scene scale) */
int orc_set_step(orc_scene* s, const double* qt, const double* qtilde,
                 double scale);

/* ---- hooks for parity ---- */
/* x [V][3] at the given q (NULL = current q) */
int orc_vertices(const orc_scene* s, const double* q, double* x);
/* candidate pairs for the given positions (and displacements, NULL = static
 * boxes), sorted; PT/EE write 2 ints per pair, PG one */
int orc_candidates(orc_scene* s, int32_t kind, const double* x,
                   const double* dx, int32_t* out, int64_t cap,
                   int64_t* count);
/* E, g [B][12], Hdiag [B][144]; off-diagonal blocks (a<b) sorted by
 * (a,b): off_ij [n][2], Hoff [n][144] */
int orc_eval(orc_scene* s, const double* q, double* E, double* g,
             double* Hdiag, int64_t cap, int64_t* n_off, int32_t* off_ij,
             double* Hoff, int64_t* n_active);
/* Newton direction at q (solve H dq = -g) */
int orc_direction(orc_scene* s, const double* q, double* dq, int32_t* iters);
/* alpha_max = min(1, min over swept candidates of the additive-CCD TOI) */
int orc_ccd(orc_scene* s, const double* q, const double* dq,
            double* alpha_max);
/* E(q + alpha dq) - E(q) evaluated term by term */
int orc_energy_delta(orc_scene* s, const double* q, const double* dq,
                     double alpha, double* dE);
/* penetration check on positions x: counts edge-triangle crossings between
 * different bodies and reports the minimum cross-body primitive distance
 * among pairs whose boxes are within `pad` */
int orc_penetration(orc_scene* s, const double* x, double pad,
                    int64_t* n_cross, double* min_dist);

/* ---- primitives for pins ---- */
void orc_barrier(double d, double dhat, double* out3);
/* squared distance and its derivatives on the pair's 12 coordinates */
int orc_sqdist(int32_t kind, const double* x12, double* D, double* g12,
               double* H144, int32_t* dtype);
/* pair barrier energy w*m*b(d); returns 1 if active (d < dhat) */
int orc_pair_eval(int32_t kind, const double* x12, double eps_x,
                  double dhat, double w, int32_t project, double* E,
                  double* g12, double* H144, double* dist, int32_t* dtype);
/* orthogonality energy ||A A^T - I||_F^2 with gradient and Hessian */
void orc_orth(const double* A9, double* E, double* g9, double* H81,
              int32_t project);
int orc_mass_props(const double* xbar, int32_t nv, const int32_t* tris,
                   int32_t nt, double density, double* Mhat16, double* vol);
void orc_psd(int32_t n, const double* H, double* out);
void orc_eig(int32_t n, const double* H, double* w, double* V);
/* additive CCD: returns the TOI in (0, tmax], tmax if no hit */
double orc_accd(int32_t kind, const double* x12, const double* dx12,
                double s, double tmax);
/* exact first time of impact of a PT or EE pair moving as x + t dx: the
 * earliest root of the coplanarity cubic in [0, tmax] at which the
 * primitives' distance vanishes (lower end of its bisection bracket);
 * tmax when they do not touch */
double orc_exact_toi(int32_t kind, const double* x12, const double* dx12,
                     double tmax);

#ifdef __cplusplus
}
#endif
#endif
