/*
 * Internal layout and device math of libabd (gfx950).  Not part of the
 * public interface (include/abd.h).
 *
 * Device data (all FP64 unless noted):
 *   body arrays  q, qt, qtilde, qdot, dq [B][12]; Mhat [B][16]; vol [B]
 *   vertices     xbar [3][V] (structure of arrays), vbody [V] int32
 *   triangles    tri [3][T] int32 global vertex ids
 *   edges        edge [2][E] int32 global vertex ids, erest2 [E]
 *   chunks       groups of <= 64 primitives of one kind of one body, with
 *                a rest-space box; the broad phase culls body pairs, then
 *                chunk pairs, then tests primitive pairs exactly
 *   Hessian      Hdiag [B][144], Hoff [slot][144] (slot = body pair a<b)
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ABD_CHUNK 64
#define ACCD_S 0.1
#define ACCD_MAX_IT 100000  /* distance evaluations of one pair's ACCD */
#define ACCD_SERIAL_IT 32   /* one-point steps, by the pair's own lane */
#define ACCD_BLOCK 64       /* then steps of 64 points, one wavefront per pair */
#define MOLL_EPS 1e-3
#define BOX_PAD_REL 1e-12

namespace abd {

enum { K_VERT = 0, K_TRI = 1, K_EDGE = 2 };
enum { C_PT = 0, C_EE = 1, C_PG = 2 };

/* device counters, one block of ints/words zeroed per phase */
struct Counters {
  int n_bp, n_cp, n_pt, n_ee, n_pg, n_act;
  int pcg_iters, err;
  unsigned long long min_dist;  /* bits of a non-negative double */
  unsigned long long min_toi;   /* bits of a non-negative double */
  unsigned long long max_dq;    /* bits of a non-negative double */
  unsigned int bar;             /* grid barrier arrivals */
  int n_rows_used;
  int n_long; /* swept block: pairs whose ACCD continues in blocked steps */
  int active; /* problems not done after a pass of the device loop */
  double pcg_rr, pcg_bb;
  /* swept block: the pass's lists are complete (no overflow in either
   * phase), so the next pass may take them as its static lists.  Static
   * block: this pass took them (the static broad phase is skipped); redo:
   * a pass launched without the static broad phase found nothing to take
   * over, so it changes no state (the next pass can take over its swept
   * lists, which cover the unchanged state).  want64 (static block): a
   * mixed-precision problem stalled in this pass and asks for FP64
   * Hessians for the rest of its solve. */
  int sweep_ok, reuse, redo, want64;
  /* arrivals of the workgroups of the kernels whose last workgroup runs
   * the controller or ends the pass */
  unsigned fin[4];
  /* connected components of the pass's linear system (static block; set by
   * the block-row build when it labels them, plan = 1): components of
   * DIR_MAX bodies or fewer solved directly (n_dir of 2 bodies or more),
   * bodies of larger components left to the PCG (n_big) */
  int plan, n_dir, n_big;
  int stat_ran; /* static block: the pass had a problem in its Newton
                   step, so these are the counters of its static phase */
};

/* largest component (bodies) solved directly (a dense elimination of up to
 * 60 rows, one wavefront) */
#define DIR_MAX 5
/* scenes of at most this many bodies build their block rows (and label
 * the components of the system) in one workgroup */
#define BSR_LDS_ROWS 12288

/* per-problem state of the device-driven Newton loop; a plain context is
 * one problem, a batch merges several */
enum { PS_NEWTON = 0, PS_LINESEARCH = 1, PS_DONE = 2 };
#define LS_TRIALS 8
/* a step accepted after more than this many halvings while eps_N < 10
 * theta ends the solve as converged (the line search at the rounding floor
 * of the energy) */
#define LS_FLOOR_HALVINGS 10
/* per-group record of the problem-local PCG: the group's partial sums of
 * one phase for each of its (at most 16) problems, published with the
 * phase number as a flag */
struct alignas(64) PcgRec {
  unsigned long long gen;
  int plo, pad; /* first problem of the group */
  double val[16][3];
};

struct ProbState {
  double scale;       /* l: bounding-box diagonal of the dynamic vertices */
  double alpha_base;  /* first trial step of the current line-search pass */
  double alpha_acc;   /* accepted step of this pass (0 = none) */
  double min_alpha, final_eps;
  double dE[LS_TRIALS];
  double acc[16];     /* PCG dot ring: [slot][rz, pAp, rr, -] */
  double bb;          /* |b|^2 of the PCG right-hand side */
  double cg_alpha[2]; /* single-reduction PCG: step of the last iterations */
  unsigned long long max_dq, min_toi;
  int state, status, newton, halvings, ls_count;
  int pcg_done, pcg_iters, pcg_total;
  /* progress of the Newton stop measure: the best eps_N so far and the
   * Newton iterations since it last fell to half the previous best; the
   * iterations taken with FP32 Hessians (mixed precision) */
  double best_eps;
  int since_best, newton32;
};

/* a mixed-precision solve asks for FP64 Hessians once eps_N has not
 * halved for MIXED_STALL_ITERS Newton iterations, or after mixed_switch
 * Newton iterations (Scene) */
#define MIXED_STALL_ITERS 16

/* the bucket map of one problem's sweep: bucket(x) = floor((x - lo) *
 * scale) clamped to [0, nb - 1], a monotone function of x */
struct SapAxis {
  double lo, scale;
  int axis, nb;
};
#define SAP_MAX_BUCKETS 8192
/* sort and sweep once every pair of each problem would exceed this many
 * box tests */
#define SAP_ALL_PAIRS_MAX (1L << 21)

/* Exact, order-independent sums for the deterministic mode: a sum of
 * doubles held as a fixed-point integer on the grid 2^-DET_FRAC, in DET_W
 * words of which each receives 32-bit signed digits (so a word takes 2^31
 * additions without overflow).  Integer additions commute, so the total
 * does not depend on the order in which terms arrive.  A term is truncated
 * toward zero onto the grid; terms of magnitude 2^DET_MAX_EXP or more (and
 * NaN) do not fit. */
#define DET_W 8
#define DET_FRAC 128
#define DET_MAX_EXP 100
typedef unsigned long long det_word;

/* add v; false if it does not fit (nothing added) */
__device__ __forceinline__ bool det_add(det_word* w, double v) {
  if (v == 0.0) return true;
  const double a = fabs(v);
  if (!(a < 0x1p100)) return false;
  int e;
  const double m = frexp(a, &e); /* a = m 2^e, m in [0.5, 1) */
  unsigned long long M = (unsigned long long)ldexp(m, 53);
  int s = e - 53 + DET_FRAC; /* a 2^DET_FRAC = M 2^s */
  if (s < 0) {
    if (s <= -53) return true;
    M >>= -s;
    s = 0;
  }
  const int wi = s >> 5, o = s & 31;
  const unsigned long long lo = M << o;
  const unsigned long long hi = o ? (M >> (64 - o)) : 0ull;
  const unsigned long long d[3] = {lo & 0xffffffffull, lo >> 32, hi};
  for (int k = 0; k < 3; ++k) {
    if (d[k] == 0ull || wi + k >= DET_W) continue;
    const unsigned long long x = v < 0.0 ? (unsigned long long)(-(long long)d[k]) : d[k];
    atomicAdd(w + wi + k, x);
  }
  return true;
}

/* the value of an accumulator, rounded (deterministically) to a double */
__device__ __forceinline__ double det_value(const det_word* w) {
  long long c = 0;
  long long d[DET_W];
  for (int k = 0; k < DET_W; ++k) {
    const long long x = (long long)w[k] + c;
    d[k] = x & 0xffffffffll;
    c = x >> 32;
  }
  double r = (double)c;
  for (int k = DET_W - 1; k >= 0; --k) r = r * 4294967296.0 + (double)d[k];
  return ldexp(r, -DET_FRAC);
}

/* a pair whose ACCD continues past its one-point steps: the anchor time
 * and distance, its candidate index in the current lists, its problem */
struct CcdLong {
  double t, da;
  int cand, prob;
};

struct Scene {
  int B, V, T, E, NC;
  /* parameters */
  double dt, dhat, kappa, kappa_A, grav[3], ground_y;
  int has_ground, mollify, pair_mode;
  /* bodies */
  double *q, *qt, *qtilde, *qdot, *dq, *Mhat, *vol, *wbody;
  int *kind;
  int *shared_slot; /* [B] -> index into z/u/rho or -1 */
  double *z, *u, *rho;
  double *body_rest; /* [B][6] rest box centre (3), half extent (3) */
  int *body_chunk;   /* [B][3][2] chunk ranges per kind */
  /* geometry */
  double *xbar;
  int *vbody, *tri, *edge;
  double *erest2;
  /* chunks */
  int *ch_body, *ch_kind, *ch_start, *ch_count, *ch_prims;
  double *ch_rest;  /* [NC][6] */
  double *ch_box;   /* [NC][6] world box lo(3) hi(3) of the current phase */
  double *body_box; /* [B][6] */
  /* body pairs by sort and sweep (per problem): the dynamic bodies of
   * each problem, sap_dyn [D] from sap_doff [NP + 1], and its static
   * bodies, sap_stat from sap_soff [NP + 1] (fixed); per pass, the dynamic
   * bodies bucketed by the lower bound of their box (sap_sorted [D]), each
   * problem's bucket starts (sap_bstart, from sap_boff [NP + 1], one entry
   * past its last bucket), its bucket map (sap_par [NP]) and the boxes in
   * sorted order */
  int *sap_dyn, *sap_doff, *sap_stat, *sap_soff;
  int *sap_sorted, *sap_bstart, *sap_boff;
  double *sap_sbox; /* [D][6] the boxes in sorted order */
  SapAxis *sap_par;
  int n_dyn;
  /* sap_on = 0: every pair of each problem instead, by the 16 x 16 body
   * tiles bp_tiles [n_bp_tiles] (tiles on or above each problem's
   * diagonal) */
  int sap_on, n_bp_tiles;
  int2 *bp_tiles;
  /* broad phase outputs */
  int2 *bp;     /* body pairs (a < b) */
  int4 *cp;     /* chunk pairs (kind, chunk P, chunk Q, body-pair slot) */
  int *cand_pt; /* [cap][3] (v, t, slot) */
  int *cand_ee; /* [cap][3] (e, f, slot) with e < f */
  int *cand_pg; /* [cap] v */
  int4 *act;    /* active pairs (kind, i, j, slot) */
  int cap_bp, cap_cp, cap_pt, cap_ee, cap_pg, cap_act;
  CcdLong *ccd_long; /* pairs of the swept lists in blocked ACCD steps */
  int cap_long;
  /* system: gradient FP64; Hessian blocks, their inverses and the PCG
   * matvec in FP64 (mixed = 0) or FP32 (mixed = 1) */
  double *g;
  void *Hdiag, *Hoff, *Pinv;
  int mixed;
  int *slot_used;
  int *row_ptr, *row_cnt, *col_slot, *col_body, *col_trans;
  int cap_col;
  /* components of the system: bmode [B] (0 alone, 1 in a component solved
   * directly, 2 in a component left to the PCG), the bodies of each
   * directly solved component dir_body [B/2 + 1][DIR_MAX] (ascending) and
   * their number dir_n [B/2 + 1]; comp_solve: label components in this
   * scene's block-row build (the PCG form in use masks the rest) */
  int *bmode, *dir_body, *dir_n;
  int comp_solve;
  /* deterministic mode: exact accumulators of the barrier contributions to
   * g [B][12], the diagonal blocks [B][144] and the off-diagonal blocks
   * [cap_bp][144], and of the line-search trial energies per problem
   * [NP][LS_TRIALS] (DET_W words each, plus one word per trial counting
   * terms that do not fit) */
  int det;
  det_word *det_g, *det_hd, *det_ho, *det_de;
  /* bsr_one: block rows and component labels in one workgroup (scenes of
   * at most BSR_LDS_ROWS bodies); else the block rows by three kernels and
   * the labels per chunk of whole problems, bodies [lab_chunk[c],
   * lab_chunk[c + 1]) of n_lab_chunks (0: no labels) */
  int *lab_chunk;
  int *chunk_tot; /* [n_lab_chunks] block-row entries of each chunk */
  int n_lab_chunks, bsr_one;
  /* PCG work */
  double *r, *zv, *p0, *p1, *Ap, *acc; /* acc: [4][4] ring of dots */
  double *pw; /* single-reduction PCG: [5][12B] w, m0, m1, t0, t1 */
  PcgRec *pcg_rec;         /* [2][groups] problem-local PCG records */
  int *prob_b0, *prob_b1;  /* [NP] first and last body of each problem */
  /* reductions */
  double *partials; /* [cap_partials] */
  int cap_partials;
  Counters *cnt;
  /* problems */
  int NP;
  int *bprob;     /* [B] problem of each body */
  ProbState *ps;  /* [NP] */
  int iter_mode;  /* 0: hooks (every problem); 1: static pass of the device
                     loop (problems in PS_NEWTON); 2: swept pass (problems
                     not PS_DONE) */
  int grid_blocks, assemble_blocks; /* launch sizes (tuning) */
  double theta;   /* Newton tolerance */
  int max_newton, max_ls, max_pcg;
  int mixed_switch; /* Newton iterations before FP64 Hessians in any case */
  double eta;
};

__device__ __forceinline__ int body_state(const Scene& S, int b) {
  return S.ps[S.bprob[b]].state;
}
/* does the current pass work on body b's problem? */
__device__ __forceinline__ bool body_in_pass(const Scene& S, int b) {
  if (S.iter_mode == 0) return true;
  const int st = S.ps[S.bprob[b]].state;
  return S.iter_mode == 1 ? st == PS_NEWTON : st != PS_DONE;
}

/* ------------------------------------------------------------------ */
/* canonical vertex transform: x_i = p_i + A_i0 xb0 + A_i1 xb1 + A_i2 xb2
 * evaluated with explicit fused multiply-adds in this fixed order, so
 * every kernel (and the export hook) produces bit-identical positions.  */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ void xform(const double* __restrict__ qb,
                                      double b0, double b1, double b2,
                                      double* x) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
    x[i] = __fma_rn(qb[5 + 3 * i], b2,
                    __fma_rn(qb[4 + 3 * i], b1,
                             __fma_rn(qb[3 + 3 * i], b0, qb[i])));
}

__device__ __forceinline__ void vertex_pos(const Scene& S, int v, double* x) {
  const double* qb = S.q + 12 * S.vbody[v];
  xform(qb, S.xbar[v], S.xbar[S.V + v], S.xbar[2 * S.V + v], x);
}

/* start and end (x + dx) of a vertex over a step dq */
__device__ __forceinline__ void vertex_pos_swept(const Scene& S, int v,
                                                 double* x, double* x1) {
  int b = S.vbody[v];
  double b0 = S.xbar[v], b1 = S.xbar[S.V + v], b2 = S.xbar[2 * S.V + v];
  xform(S.q + 12 * b, b0, b1, b2, x);
  double dx[3];
  xform(S.dq + 12 * b, b0, b1, b2, dx);
#pragma unroll
  for (int i = 0; i < 3; ++i) x1[i] = __dadd_rn(x[i], dx[i]);
}

/* position at q + alpha dq */
__device__ __forceinline__ void vertex_pos_alpha(const Scene& S, int v,
                                                 double alpha, double* x) {
  int b = S.vbody[v];
  const double* qb = S.q + 12 * b;
  const double* db = S.dq + 12 * b;
  double qa[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) qa[i] = qb[i] + alpha * db[i];
  xform(qa, S.xbar[v], S.xbar[S.V + v], S.xbar[2 * S.V + v], x);
}

/* ------------------------------------------------------------------ */
/* boxes                                                                */
/* ------------------------------------------------------------------ */
/* lo_P <= hi_Q + dhat and lo_Q <= hi_P + dhat on every axis; each bound is
 * one rounded add, compared exactly */
__device__ __forceinline__ bool box_overlap(const double* P, const double* Q,
                                            double dh) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ok = ok && (P[k] <= __dadd_rn(Q[3 + k], dh));
    ok = ok && (Q[k] <= __dadd_rn(P[3 + k], dh));
  }
  return ok;
}

/* Conservative world box of a rest box (centre c, half extent e) under the
 * affine map q: centre A c + p, half extent |A| e, padded by a relative
 * 1e-12 of the magnitudes involved, which dominates every rounding error of
 * the vertex transform; mag adds the magnitude of a second map (a step). */
__device__ __forceinline__ void world_box(const double* qb, const double* ce,
                                          double extra_mag, double* box) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double c = qb[i], e = 0.0, m = fabs(qb[i]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double a = qb[3 + 3 * i + j];
      c += a * ce[j];
      e += fabs(a) * ce[3 + j];
      m += fabs(a) * (fabs(ce[j]) + ce[3 + j]);
    }
    double pad = BOX_PAD_REL * (m + extra_mag) + 1e-300;
    box[i] = c - e - pad;
    box[3 + i] = c + e + pad;
  }
}

__device__ __forceinline__ double map_mag(const double* qb, const double* ce) {
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double mi = fabs(qb[i]);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      mi += fabs(qb[3 + 3 * i + j]) * (fabs(ce[j]) + ce[3 + j]);
    m = fmax(m, mi);
  }
  return m;
}

/* ------------------------------------------------------------------ */
/* IPC barrier b(d) = -(d - dhat)^2 ln(d/dhat), 0 < d < dhat            */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ void barrier3(double d, double dh, double& b,
                                         double& b1, double& b2) {
  if (!(d < dh)) {
    b = b1 = b2 = 0.0;
    return;
  }
  double t = d - dh;
  double L = log(d / dh);
  double id = 1.0 / d;
  b = -t * t * L;
  b1 = -t * (2.0 * L + t * id);
  b2 = -2.0 * L - 4.0 * t * id + t * t * id * id;
}

__device__ __forceinline__ double barrier_val(double d, double dh) {
  if (!(d < dh)) return 0.0;
  double t = d - dh;
  return -t * t * log(d / dh);
}

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
__device__ __forceinline__ void cross3(const double* a, const double* b,
                                       double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
/* v = sum_s l[s] x_s over the 4 pair vertices */
__device__ __forceinline__ void comb4(const signed char* l, const double* x,
                                      double* v) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
    v[i] = l[0] * x[i] + l[1] * x[3 + i] + l[2] * x[6 + i] + l[3] * x[9 + i];
}

/* ------------------------------------------------------------------ */
/* primitive distance features                                          */
/* A feature is a function of difference vectors of the 4 pair slots:  */
/*   PP:  |r|^2                       (1 vector)                         */
/*   PE:  |a x e|^2 / |e|^2           (point offset a, edge e)           */
/*   TRI: (a . (b x c))^2 / |b x c|^2 (point-plane or line-line)         */
/* Slots are (p, t0, t1, t2) for PT and (a0, a1, b0, b1) for EE.        */
/* ------------------------------------------------------------------ */
enum { F_PP = 0, F_PE = 1, F_TRI = 2 };
struct Feat {
  int type, code;
  signed char l[3][4]; /* slot coefficients of the feature's vectors */
};

__device__ __forceinline__ void set_l(signed char* l, int a, int b, int c,
                                      int d) {
  l[0] = (signed char)a; l[1] = (signed char)b;
  l[2] = (signed char)c; l[3] = (signed char)d;
}

__device__ __forceinline__ double feat_sqd(const Feat& f, const double* x) {
  if (f.type == F_PP) {
    double r[3];
    comb4(f.l[0], x, r);
    return dot3(r, r);
  }
  if (f.type == F_PE) {
    double a[3], e[3], c[3];
    comb4(f.l[0], x, a);
    comb4(f.l[1], x, e);
    cross3(a, e, c);
    return dot3(c, c) / dot3(e, e);
  }
  double a[3], b[3], c[3], n[3];
  comb4(f.l[0], x, a);
  comb4(f.l[1], x, b);
  comb4(f.l[2], x, c);
  cross3(b, c, n);
  double s = dot3(a, n);
  return s * s / dot3(n, n);
}

/* closest feature of point slot p to the closed segment (e0, e1) */
__device__ __forceinline__ Feat point_seg(const double* x, int p, int e0,
                                          int e1, int c_e0, int c_e1,
                                          int c_pe) {
  double a[3], e[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    a[i] = x[3 * p + i] - x[3 * e0 + i];
    e[i] = x[3 * e1 + i] - x[3 * e0 + i];
  }
  double ee = dot3(e, e);
  double t = ee > 0.0 ? dot3(a, e) / ee : 0.0;
  Feat f;
  signed char z[4] = {0, 0, 0, 0};
  for (int k = 0; k < 4; ++k) f.l[0][k] = f.l[1][k] = f.l[2][k] = z[k];
  if (!(ee > 0.0) || t <= 0.0) {
    f.type = F_PP; f.code = c_e0;
    f.l[0][p] = 1; f.l[0][e0] = -1;
  } else if (t >= 1.0) {
    f.type = F_PP; f.code = c_e1;
    f.l[0][p] = 1; f.l[0][e1] = -1;
  } else {
    f.type = F_PE; f.code = c_pe;
    f.l[0][p] = 1; f.l[0][e0] = -1;
    f.l[1][e1] = 1; f.l[1][e0] = -1;
  }
  return f;
}

/* Classify a PT (kind 0) or EE (kind 1) pair: minimum over features in the
 * fixed order (segment features by index, then the interior feature), the
 * first one winning ties.  Codes: PT 0..2 vertex t_k, 3..5 edge k (t0t1,
 * t1t2, t2t0), 6 interior; EE 0..3 (a_i, b_j) -> 2i + j, 4..5 a_i on
 * segment b, 6..7 b_j on segment a, 8 interior. */
__device__ __forceinline__ Feat classify(int kind, const double* x, double& Dout) {
  Feat best;
  double bestD = INFINITY;
  if (kind == C_PT) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      int e0 = 1 + k, e1 = 1 + (k + 1) % 3;
      Feat f = point_seg(x, 0, e0, e1, e0 - 1, e1 - 1, 3 + k);
      double D = feat_sqd(f, x);
      if (D < bestD) { bestD = D; best = f; }
    }
    double a[3], b[3], c[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      a[i] = x[i] - x[3 + i];
      b[i] = x[6 + i] - x[3 + i];
      c[i] = x[9 + i] - x[3 + i];
    }
    double bb = dot3(b, b), bc = dot3(b, c), cc = dot3(c, c);
    double ab = dot3(a, b), ac = dot3(a, c);
    double det = bb * cc - bc * bc;
    if (det > 0.0) {
      double u = (ab * cc - ac * bc) / det;
      double v = (ac * bb - ab * bc) / det;
      if (u > 0.0 && v > 0.0 && u + v < 1.0) {
        Feat f;
        f.type = F_TRI; f.code = 6;
        set_l(f.l[0], 1, -1, 0, 0);
        set_l(f.l[1], 0, -1, 1, 0);
        set_l(f.l[2], 0, -1, 0, 1);
        double D = feat_sqd(f, x);
        if (D < bestD) { bestD = D; best = f; }
      }
    }
  } else {
    Feat f4[4] = {point_seg(x, 0, 2, 3, 0, 1, 4), point_seg(x, 1, 2, 3, 2, 3, 5),
                  point_seg(x, 2, 0, 1, 0, 2, 6), point_seg(x, 3, 0, 1, 1, 3, 7)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double D = feat_sqd(f4[k], x);
      if (D < bestD) { bestD = D; best = f4[k]; }
    }
    double u[3], v[3], w[3], n[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u[i] = x[3 + i] - x[i];
      v[i] = x[9 + i] - x[6 + i];
      w[i] = x[i] - x[6 + i];
    }
    cross3(u, v, n);
    double N = dot3(n, n);
    if (N > 0.0) {
      double uu = dot3(u, u), uv = dot3(u, v), vv = dot3(v, v);
      double uw = dot3(u, w), vw = dot3(v, w);
      double s = (uv * vw - vv * uw) / N;
      double t = (uu * vw - uv * uw) / N;
      if (s > 0.0 && s < 1.0 && t > 0.0 && t < 1.0) {
        Feat f;
        f.type = F_TRI; f.code = 8;
        set_l(f.l[0], 1, 0, -1, 0);  /* w = a0 - b0 */
        set_l(f.l[1], -1, 1, 0, 0);  /* u = a1 - a0 */
        set_l(f.l[2], 0, 0, -1, 1);  /* v = b1 - b0 */
        double D = feat_sqd(f, x);
        if (D < bestD) { bestD = D; best = f; }
      }
    }
  }
  Dout = bestD;
  return best;
}

__device__ __forceinline__ double pair_dist(int kind, const double* x) {
  double D;
  classify(kind, x, D);
  return sqrt(D);
}

/* ------------------------------------------------------------------ */
/* reduced frame                                                        */
/* The pair energy depends only on vertex differences; it is written in  */
/* three difference vectors y_r = sum_s f_r[s] x_s whose slot rows are   */
/* mutually orthogonal:                                                  */
/*   PT: p - (t0+t1+t2)/3, t1 - t0, t2 - (t0+t1)/2  (|f|^2 = 4/3, 2, 3/2)*/
/*   EE: mid(a) - mid(b),  a1 - a0,  b1 - b0         (|f|^2 = 1, 2, 2)   */
/* so the vertex Hessian is f^T H_y f = U^T (G H_y G) U with U = G^-1 f  */
/* orthonormal and G = diag|f_r|: PSD projection of the 9x9 G H_y G     */
/* equals the projection of the 12x12 vertex Hessian.                   */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ double frame_row(int kind, int r, int s) {
  if (kind == C_PT) {
    if (r == 0) return s == 0 ? 1.0 : -1.0 / 3.0;
    if (r == 1) return s == 1 ? -1.0 : (s == 2 ? 1.0 : 0.0);
    return s == 3 ? 1.0 : (s == 0 ? 0.0 : -0.5);
  }
  if (r == 0) return s < 2 ? 0.5 : -0.5;
  if (r == 1) return s == 0 ? -1.0 : (s == 1 ? 1.0 : 0.0);
  return s == 2 ? -1.0 : (s == 3 ? 1.0 : 0.0);
}
__device__ __forceinline__ double frame_norm2(int kind, int r) {
  if (kind == C_PT) return r == 0 ? 4.0 / 3.0 : (r == 1 ? 2.0 : 1.5);
  return r == 0 ? 1.0 : 2.0;
}
/* y-coordinates of a difference vector with slot coefficients l */
__device__ __forceinline__ void frame_coef(int kind, const signed char* l,
                                           double* C) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) s += l[k] * frame_row(kind, r, k);
    C[r] = s / frame_norm2(kind, r);
  }
}

/* packed symmetric 9x9 index */
__host__ __device__ constexpr int sidx(int p, int q) {
  return p <= q ? 9 * p - (p * (p - 1)) / 2 + (q - p)
                : 9 * q - (q * (q - 1)) / 2 + (p - q);
}

/* ------------------------------------------------------------------ */
/* stopping bound of the Jacobi eigensolver of the PSD projections: the */
/* off-diagonal mass below tol2 of the total (1e-30 in FP64, 1e-12 in   */
/* FP32, i.e. about the square of each precision)                       */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }
__device__ __forceinline__ float rsq(float x) { return rsqrtf(x); }

/* Rotation parameters of one Jacobi step without the IEEE division and
 * square-root sequences: hardware reciprocal and reciprocal square root,
 * each refined by Newton steps (each step squares the relative error, so
 * two take the ~1e-8 seeds to full double precision).  The rotation only
 * needs c^2 + s^2 = 1 and t to double precision, not correct rounding. */
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __fma_rn(-x, r, 1.0);
  r = __fma_rn(r, e, r);
  e = __fma_rn(-x, r, 1.0);
  return __fma_rn(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  for (int k = 0; k < 2; ++k) {
    const double h = 0.5 * x * y;
    y = __fma_rn(-h, y * y, 1.5 * y) ;
  }
  return y;
}
/* one Newton step: relative error about 1e-14 */
__device__ __forceinline__ double rsq_nr1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * y;
  return __fma_rn(-h, y * y, 1.5 * y);
}
__device__ __forceinline__ float rsq_nr1(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp_nr(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq_nr(float x) { return __builtin_amdgcn_rsqf(x); }

/* ------------------------------------------------------------------ */
/* PSD projection of the orthogonality Hessian in closed form           */
/* ------------------------------------------------------------------ */
/* f(A) = |A A^T - I|_F^2 depends on A only through its singular values,
 * f = sum_i (s_i^2 - 1)^2, so with A = U diag(s) V^T its 9x9 Hessian (in
 * row-major vec(A)) has the eigenvectors of isotropic functions of a 3x3
 * matrix: U e_i e_i^T V^T (eigenvalue 12 s_i^2 - 4, the separable second
 * derivative), and for each pair i < j U (e_i e_j^T -/+ e_j e_i^T) V^T / sqrt2
 * with eigenvalues (f_i +/- f_j) / (s_i +/- s_j), f_i = 4 s_i (s_i^2 - 1),
 * which reduce to 4(s_i^2 -/+ s_i s_j + s_j^2 - 1).  Clamping the nine
 * eigenvalues at zero gives the same projection as a numerical eigensolve
 * of the assembled 9x9 matrix, from a 3x3 eigensolve of A^T A.  Returns
 * the packed upper triangle (sidx) of the projected Hessian of f. */
__device__ __forceinline__ void sym3_eig(double* M, double* V) {
  /* cyclic Jacobi on a symmetric 3x3 (row-major M, overwritten by its
   * eigenvalues on the diagonal); V gets the eigenvectors as columns */
#pragma unroll
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 20; ++sweep) {
    const double off = M[1] * M[1] + M[2] * M[2] + M[5] * M[5];
    const double dia = M[0] * M[0] + M[4] * M[4] + M[8] * M[8];
    if (off == 0.0 || off <= 1e-32 * (dia + off)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = M[3 * p + q];
      if (apq == 0.0) continue;
      const double app = M[3 * p + p], aqq = M[3 * q + q];
      const double aa = aqq - app, bb = 2.0 * apq;
      double t = bb / (fabs(aa) + sqrt(aa * aa + bb * bb));
      t = aa < 0.0 ? -t : t;
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double mrp = M[3 * r + p], mrq = M[3 * r + q];
        M[3 * r + p] = c * mrp - s * mrq;
        M[3 * r + q] = s * mrp + c * mrq;
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double mpr = M[3 * p + r], mqr = M[3 * q + r];
        M[3 * p + r] = c * mpr - s * mqr;
        M[3 * q + r] = s * mpr + c * mqr;
      }
      M[3 * p + q] = M[3 * q + p] = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double vrp = V[3 * r + p], vrq = V[3 * r + q];
        V[3 * r + p] = c * vrp - s * vrq;
        V[3 * r + q] = s * vrp + c * vrq;
      }
    }
  }
}

__device__ __forceinline__ void orth_hessian_psd(const double* A, double* K) {
  double AtA[9], V[9];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      double t = 0.0;
#pragma unroll
      for (int n = 0; n < 3; ++n) t += A[3 * n + k] * A[3 * n + m];
      AtA[3 * k + m] = t;
    }
  sym3_eig(AtA, V);
  double sv[3], U[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    sv[i] = sqrt(fmax(AtA[4 * i], 0.0));
    /* u_i = A v_i / s_i (A is near a rotation, s_i near 1) */
    const double inv = sv[i] > 0.0 ? 1.0 / sv[i] : 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double t = 0.0;
#pragma unroll
      for (int n = 0; n < 3; ++n) t += A[3 * k + n] * V[3 * n + i];
      U[3 * k + i] = t * inv;
    }
  }
  double lam[9], vec[9][9];
  const double r2 = 0.70710678118654752440;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    lam[i] = fmax(12.0 * sv[i] * sv[i] - 4.0, 0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) vec[i][3 * k + l] = U[3 * k + i] * V[3 * l + i];
  }
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    const int i = pr == 2 ? 1 : 0, j = pr == 0 ? 1 : 2;
    const double a = sv[i] * sv[i] + sv[j] * sv[j] - 1.0, b = sv[i] * sv[j];
    lam[3 + pr] = fmax(4.0 * (a - b), 0.0); /* antisymmetric (twist) */
    lam[6 + pr] = fmax(4.0 * (a + b), 0.0); /* symmetric (flip) */
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const double x = U[3 * k + i] * V[3 * l + j], y = U[3 * k + j] * V[3 * l + i];
        vec[3 + pr][3 * k + l] = r2 * (x - y);
        vec[6 + pr][3 * k + l] = r2 * (x + y);
      }
  }
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int e = a; e < 9; ++e) {
      double h = 0.0;
#pragma unroll
      for (int m = 0; m < 9; ++m) h += lam[m] * vec[m][a] * vec[m][e];
      K[sidx(a, e)] = h;
    }
}

/* ------------------------------------------------------------------ */
/* additive CCD on one PT/EE pair along x + t dx                        */
/* ------------------------------------------------------------------ */
/* bound (may be null): bits of a TOI another pair of the same problem has
 * already reached; once t passes it this pair cannot lower the minimum,
 * so the advance stops there and returns t (a lower bound of its TOI) */
/* Additive CCD (R11) of a pair moving on x + t dx, t in [0, tmax]: the
 * relative displacements r (each point's dx less the pair's mean), the
 * bound lp on how fast the distance can shrink, then one-point steps
 * (1 - s) d0 / lp and 0.9 d / lp while the gap s d0 holds.  Returns true
 * with the time of impact bound in *t, or false after ACCD_SERIAL_IT steps
 * with the anchor (*t, *da) from which the blocked steps continue (the
 * second phase, a wavefront per pair).  bound: stop once t passes it (the
 * problem's smallest TOI so far, which this pair can then no longer lower). */
__device__ __forceinline__ void accd_setup(int kind, const double* dx, double* r,
                                           double* lp) {
  double m[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    m[i] = 0.25 * (dx[i] + dx[3 + i] + dx[6 + i] + dx[9 + i]);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) r[3 * k + i] = dx[3 * k + i] - m[i];
  double n[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) n[k] = sqrt(dot3(r + 3 * k, r + 3 * k));
  *lp = (kind == C_PT) ? n[0] + fmax(n[1], fmax(n[2], n[3]))
                       : fmax(n[0], n[1]) + fmax(n[2], n[3]);
}
__device__ __forceinline__ double bound_of(const unsigned long long* bound) {
  return __longlong_as_double((long long)__hip_atomic_load(
      bound, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ bool accd_begin(int kind, const double* x, const double* dx,
                                           double tmax, const unsigned long long* bound,
                                           double* t_out, double* da_out) {
  double r[12], lp;
  accd_setup(kind, dx, r, &lp);
  *t_out = tmax;
  if (lp == 0.0) return true;
  double d0 = pair_dist(kind, x);
  *t_out = 0.0;
  if (!(d0 > 0.0)) return true;
  double gap = ACCD_S * d0;
  double t = 0.0;
  double tl = (1.0 - ACCD_S) * d0 / lp;
  double xt[12];
  double d = d0;
  for (int it = 0; it < ACCD_SERIAL_IT; ++it) {
    double tn = t + tl;
#pragma unroll
    for (int i = 0; i < 12; ++i) xt[i] = x[i] + tn * r[i];
    d = pair_dist(kind, xt);
    if (t > 0.0 && d < gap) {
      *t_out = t;
      return true;
    }
    t = tn;
    if (t > tmax) {
      *t_out = tmax;
      return true;
    }
    if (bound && (it & 3) == 3 && t >= bound_of(bound)) {
      *t_out = t;
      return true;
    }
    tl = 0.9 * d / lp;
  }
  *t_out = t; /* d: the distance at t */
  *da_out = d;
  return false;
}

/* ------------------------------------------------------------------ */
/* atomics on non-negative doubles through their bit patterns           */
/* ------------------------------------------------------------------ */
__device__ __forceinline__ void atomic_min_pos(unsigned long long* a,
                                               double v) {
  atomicMin(a, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ void atomic_max_pos(unsigned long long* a,
                                               double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

/* ------------------------------------------------------------------ */
/* host-side launchers (kernels.hip)                                    */
/* ------------------------------------------------------------------ */
void launch_predict(const Scene& S, hipStream_t st);
void launch_commit(const Scene& S, hipStream_t st);
void launch_transform(const Scene& S, double* x, double* dx, hipStream_t st);
void launch_body_terms(const Scene& S, hipStream_t st, const Counters* fresh = nullptr,
                       int expect_reuse = 0);
/* the pass reset of the device loop alone */
void launch_pass_reset(const Scene& S, const Counters& fresh, int expect_reuse,
                       hipStream_t st);
/* chunk and body boxes of a broad phase (with stop_test, the Newton stop
 * test in extra workgroups) */
void launch_boxes(const Scene& S, int swept, hipStream_t st,
                  const Counters* fresh = nullptr, int expect_reuse = 0,
                  int stop_test = 0);
void launch_body_pairs(const Scene& S, hipStream_t st);
void launch_chunk_pairs(const Scene& S, hipStream_t st);
void launch_prim_pairs(const Scene& S, int swept, hipStream_t st);
void launch_pg(const Scene& S, int swept, hipStream_t st);
void launch_filter(const Scene& S, hipStream_t st);
void launch_crossings(const Scene& S, hipStream_t st);
void launch_assemble(const Scene& S, int n_act_hint, hipStream_t st);
void launch_bsr(const Scene& S, hipStream_t st);
void launch_block_inverse(const Scene& S, hipStream_t st);
int launch_pcg(const Scene& S, double eta, int max_it, int grid, int variant,
               int goff, hipStream_t st);
int pcg_max_grid();
void launch_dq_norm(const Scene& S, int with_ctrl, hipStream_t st);
void launch_ccd(const Scene& S, int with_ctrl, hipStream_t st);
/* each candidate's TOI into toi[n] (n = the list's PT + EE + PG count) */
void launch_ccd_pairs(const Scene& S, double* toi, int64_t n, hipStream_t st);
void launch_energy(const Scene& S, double alpha, int mode_with_pairs,
                   int alpha_from_toi, double* out, hipStream_t st);
void launch_energy_multi(const Scene& S, hipStream_t st);
void launch_ctrl_start(const Scene& S, hipStream_t st);
void launch_update_multi(const Scene& S, Counters* ring, unsigned* pass,
                         hipStream_t st);
void launch_reset_pcg(const Scene& S, hipStream_t st);
void launch_reset_toi(const Scene& S, hipStream_t st);
/* consensus over the replicas of shared bodies in a batch scene */
struct Cons {
  int n_rep, n_groups;
  const int* rep_body;  /* [n_rep] body index in the batch scene */
  const int* rep_group; /* [n_rep] shared body of each replica */
  const int* grp_ptr;   /* [n_groups + 1] replicas of each group (CSR) */
  const int* grp_rep;   /* [n_rep] */
  const double* rho0;   /* [n_rep] initial penalties */
  double* zc;           /* [n_groups][12] current consensus z */
  unsigned long long* r_body; /* [n_groups] max over replicas |q - z|_inf */
  unsigned long long* s_body; /* [n_groups] |z_new - z_old|_inf */
  unsigned long long* red;    /* [2] r_inf, s_inf (bits of doubles >= 0) */
  double tau, mu, smin, smax;
};
void launch_cons_init(const Scene& S, const Cons& C, hipStream_t st);
void launch_cons_update(const Scene& S, const Cons& C, hipStream_t st);
void launch_cons_adapt(const Scene& S, const Cons& C, hipStream_t st);
void launch_cons_merge(const Scene& S, const Cons& C, hipStream_t st);
void launch_cons_merge_dq(const Scene& S, const Cons& C, hipStream_t st);

/* batch state movement: one descriptor per problem */
struct ProbCopy {
  double *q, *qt, *qtilde, *qdot; /* the problem's own context arrays */
  int nb, off;                     /* bodies, body offset in the batch */
};
void launch_gather(const Scene& S, const ProbCopy* pc, const double* scales,
                   int np, int max_nb, hipStream_t st);
void launch_scatter(const Scene& S, const ProbCopy* pc, int np, int max_nb,
                    hipStream_t st);
void launch_update_q(const Scene& S, double alpha, hipStream_t st);
void launch_scale(const Scene& S, double* out6, hipStream_t st);

}  // namespace abd
