/*
 * Plain FP64 CPU oracle for one worker's local affine-body Newton solve --
 * TEST INFRASTRUCTURE ONLY (see abd_oracle.h).  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * What it computes (one local solve, Eq. 5 of Sec. 4.1):
 *
 *   E(q) = sum_b (1/kappa_b) [ 1/2 (q_b - qt_b)^T M_b (q_b - qt_b)
 *                              + h^2 kappa_A V_b ||A_b A_b^T - I||_F^2 ]
 *        + h^2 sum_c (kappa / kappa_c) m_c b(d_c)
 *        + sum_{b shared} rho_b / 2 ||q_b - z_b + u_b||^2
 *
 * with the implicit-Euler incremental potential of Eq. 1 (inertia about the
 * prediction qt = q^t + h qdot + h^2 M^-1 f_ext), the affine-body
 * orthogonality energy (the paper defers its form to ABD), the IPC log
 * barrier b(d) = -(d - dhat)^2 ln(d / dhat) on unsquared primitive distances,
 * the replication weights of Eq. 3 and the ADMM penalty of Eq. 5.  It is
 * minimised by projected Newton with a CCD-filtered backtracking line
 * search, which keeps every iterate penetration free (IPC, Sec. 2).
 *
 * Readings of points the paper leaves open are listed in the design notes;
 * the ones that shape this file:
 *  - M_b = I3 (x) Mhat_b with Mhat_b = int rho [1 xbar^T; xbar xbar xbar^T]
 *    from exact polyhedral integration;
 *  - primitive distance = exact Euclidean distance between closed point,
 *    segment and triangle primitives, taken as the minimum over features in
 *    a fixed order (first feature wins ties);
 *  - edge-edge pairs use IPC's mollifier on |e_a x e_b|^2;
 *  - pair and orthogonality Hessians are projected to PSD by clamping the
 *    eigenvalues of a cyclic-Jacobi eigendecomposition;
 *  - candidate pairs use the d-hat inflated axis-aligned box predicate with
 *    exact min/max and one rounded add per bound;
 *  - additive CCD with s = 0.1, zero thickness, alpha_max = min(1, TOI);
 *  - line search halves alpha while E(q + alpha dq) - E(q) > 0, the
 *    difference being summed term by term.
 */
#include "abd_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

namespace {

const double ACCD_S = 0.1;         /* ACCD: target gap fraction s */
const int ACCD_MAX_IT = 100000;    /* ACCD: distance evaluations cap (returns safe t) */
const int ACCD_SERIAL_IT = 32;     /* ACCD: one-point steps before blocked steps */
const int ACCD_BLOCK = 64;         /* ACCD: points per blocked step */
const int LS_FLOOR_HALVINGS = 10;  /* line search at the energy's rounding floor */
const double MOLLIFIER_EPS = 1e-3; /* eps_x = 1e-3 |ea_rest|^2 |eb_rest|^2 */

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
void sub3(const double* a, const double* b, double* c) {
  c[0] = a[0] - b[0];
  c[1] = a[1] - b[1];
  c[2] = a[2] - b[2];
}
void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
double norm3(const double* a) { return std::sqrt(dot3(a, a)); }

/* skew matrix [v]x with [v]x w = v x w, row-major 3x3 */
void skew(const double* v, double* S) {
  S[0] = 0.0;   S[1] = -v[2]; S[2] = v[1];
  S[3] = v[2];  S[4] = 0.0;   S[5] = -v[0];
  S[6] = -v[1]; S[7] = v[0];  S[8] = 0.0;
}

/* ------------------------------------------------------------------ */
/* IPC log barrier on the unsquared distance                            */
/* ------------------------------------------------------------------ */
void barrier(double d, double dh, double* b, double* b1, double* b2) {
  if (!(d < dh)) {
    *b = *b1 = *b2 = 0.0;
    return;
  }
  double t = d - dh;
  double L = std::log(d / dh);
  *b = -t * t * L;
  *b1 = -2.0 * t * L - t * t / d;
  *b2 = -2.0 * L - 4.0 * t / d + t * t / (d * d);
}

/* ------------------------------------------------------------------ */
/* scalar functions with gradient and Hessian over up to 12 variables   */
/* ------------------------------------------------------------------ */
struct Deriv {
  double f;
  double g[12];
  double H[144]; /* row-major, stride 12 */
  void zero() {
    f = 0.0;
    std::memset(g, 0, sizeof(g));
    std::memset(H, 0, sizeof(H));
  }
};

/* K(u,v) = |u x v|^2 over 6 variables (u: 0..2, v: 3..5), placed at
 * variable offsets ou, ov of the output (so it can live inside a larger
 * variable set). */
void cross_norm_sq(const double* u, const double* v, int ou, int ov,
                   Deriv& K) {
  K.zero();
  double uu = dot3(u, u), vv = dot3(v, v), uv = dot3(u, v);
  double c[3];
  cross3(u, v, c);
  K.f = dot3(c, c);
  for (int i = 0; i < 3; ++i) {
    K.g[ou + i] = 2.0 * vv * u[i] - 2.0 * uv * v[i];
    K.g[ov + i] = 2.0 * uu * v[i] - 2.0 * uv * u[i];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double dij = (i == j) ? 1.0 : 0.0;
      K.H[(ou + i) * 12 + ou + j] = 2.0 * vv * dij - 2.0 * v[i] * v[j];
      K.H[(ov + i) * 12 + ov + j] = 2.0 * uu * dij - 2.0 * u[i] * u[j];
      double huv = 4.0 * u[i] * v[j] - 2.0 * uv * dij - 2.0 * v[i] * u[j];
      K.H[(ou + i) * 12 + ov + j] = huv;
      K.H[(ov + j) * 12 + ou + i] = huv;
    }
}

/* S = (a . (b x c))^2 over 9 variables (a: 0..2, b: 3..5, c: 6..8) */
void triple_sq(const double* a, const double* b, const double* c, Deriv& S) {
  S.zero();
  double bc[3], ca[3], ab[3];
  cross3(b, c, bc);
  cross3(c, a, ca);
  cross3(a, b, ab);
  double s = dot3(a, bc);
  double gs[9];
  for (int i = 0; i < 3; ++i) {
    gs[i] = bc[i];
    gs[3 + i] = ca[i];
    gs[6 + i] = ab[i];
  }
  /* Hessian of s: blocks (a,b) = -[c]x, (a,c) = [b]x, (b,c) = -[a]x */
  double Hs[81];
  std::memset(Hs, 0, sizeof(Hs));
  double Sa[9], Sb[9], Sc[9];
  skew(a, Sa);
  skew(b, Sb);
  skew(c, Sc);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Hs[(0 + i) * 9 + 3 + j] = -Sc[i * 3 + j];
      Hs[(3 + j) * 9 + 0 + i] = -Sc[i * 3 + j];
      Hs[(0 + i) * 9 + 6 + j] = Sb[i * 3 + j];
      Hs[(6 + j) * 9 + 0 + i] = Sb[i * 3 + j];
      Hs[(3 + i) * 9 + 6 + j] = -Sa[i * 3 + j];
      Hs[(6 + j) * 9 + 3 + i] = -Sa[i * 3 + j];
    }
  S.f = s * s;
  for (int i = 0; i < 9; ++i) S.g[i] = 2.0 * s * gs[i];
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j)
      S.H[i * 12 + j] = 2.0 * gs[i] * gs[j] + 2.0 * s * Hs[i * 9 + j];
}

/* f = S / N (quotient rule) over n variables */
void quotient(const Deriv& S, const Deriv& N, int n, Deriv& f) {
  f.zero();
  double iN = 1.0 / N.f;
  f.f = S.f * iN;
  for (int i = 0; i < n; ++i) f.g[i] = S.g[i] * iN - S.f * N.g[i] * iN * iN;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double h = S.H[i * 12 + j] * iN;
      h -= (S.g[i] * N.g[j] + N.g[i] * S.g[j]) * iN * iN;
      h -= S.f * N.H[i * 12 + j] * iN * iN;
      h += 2.0 * S.f * N.g[i] * N.g[j] * iN * iN * iN;
      f.H[i * 12 + j] = h;
    }
}

/* Map a function of m difference vectors y_r = sum_s coef[r][s] x_s onto the
 * 4 vertex slots (12 coordinates) of a pair. */
void to_slots(const Deriv& y, int m, const int coef[][4], Deriv& x) {
  x.zero();
  x.f = y.f;
  for (int s = 0; s < 4; ++s)
    for (int i = 0; i < 3; ++i) {
      double v = 0.0;
      for (int r = 0; r < m; ++r) v += coef[r][s] * y.g[3 * r + i];
      x.g[3 * s + i] = v;
    }
  for (int s = 0; s < 4; ++s)
    for (int t = 0; t < 4; ++t)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double v = 0.0;
          for (int r = 0; r < m; ++r)
            for (int u = 0; u < m; ++u)
              v += coef[r][s] * coef[u][t] * y.H[(3 * r + i) * 12 + 3 * u + j];
          x.H[(3 * s + i) * 12 + 3 * t + j] = v;
        }
}

/* ------------------------------------------------------------------ */
/* primitive distances                                                  */
/* ------------------------------------------------------------------ */
/* A feature of a pair: point-point, point-edge (line), or the "triple"
 * form (point-plane for PT, line-line for EE). */
enum { F_PP = 0, F_PE = 1, F_TRIPLE = 2 };
struct Feature {
  int type;
  int s0, s1, s2; /* PP: s0,s1; PE: point s0, edge s1-s2 */
  int code;       /* distance-type code reported to callers */
};

const double* slot(const double* x12, int s) { return x12 + 3 * s; }

double sqd_pp(const double* x12, int i, int j) {
  double d[3];
  sub3(slot(x12, i), slot(x12, j), d);
  return dot3(d, d);
}
double sqd_pe(const double* x12, int p, int e0, int e1) {
  double a[3], e[3], c[3];
  sub3(slot(x12, p), slot(x12, e0), a);
  sub3(slot(x12, e1), slot(x12, e0), e);
  cross3(a, e, c);
  return dot3(c, c) / dot3(e, e);
}

/* triple-form variables for PT (plane) or EE (line-line) */
const int PT_COEF[3][4] = {{1, -1, 0, 0}, {0, -1, 1, 0}, {0, -1, 0, 1}};
const int EE_COEF[3][4] = {{1, 0, -1, 0}, {-1, 1, 0, 0}, {0, 0, -1, 1}};

void triple_vars(int kind, const double* x12, double* a, double* b,
                 double* c) {
  const int(*C)[4] = (kind == ORC_PT) ? PT_COEF : EE_COEF;
  double* out[3] = {a, b, c};
  for (int r = 0; r < 3; ++r)
    for (int i = 0; i < 3; ++i) {
      double v = 0.0;
      for (int s = 0; s < 4; ++s) v += C[r][s] * x12[3 * s + i];
      out[r][i] = v;
    }
}
double sqd_triple(int kind, const double* x12) {
  double a[3], b[3], c[3], n[3];
  triple_vars(kind, x12, a, b, c);
  cross3(b, c, n);
  double s = dot3(a, n);
  return s * s / dot3(n, n);
}

/* closest feature between point p and the closed segment e0-e1 */
Feature point_segment(const double* x12, int p, int e0, int e1, int code_pp0,
                      int code_pp1, int code_pe) {
  double a[3], e[3];
  sub3(slot(x12, p), slot(x12, e0), a);
  sub3(slot(x12, e1), slot(x12, e0), e);
  double ee = dot3(e, e);
  Feature f;
  f.s2 = -1;
  if (!(ee > 0.0)) {
    f.type = F_PP; f.s0 = p; f.s1 = e0; f.code = code_pp0;
    return f;
  }
  double t = dot3(a, e) / ee;
  if (t <= 0.0) {
    f.type = F_PP; f.s0 = p; f.s1 = e0; f.code = code_pp0;
  } else if (t >= 1.0) {
    f.type = F_PP; f.s0 = p; f.s1 = e1; f.code = code_pp1;
  } else {
    f.type = F_PE; f.s0 = p; f.s1 = e0; f.s2 = e1; f.code = code_pe;
  }
  return f;
}

double feature_sqd(int kind, const double* x12, const Feature& f) {
  if (f.type == F_PP) return sqd_pp(x12, f.s0, f.s1);
  if (f.type == F_PE) return sqd_pe(x12, f.s0, f.s1, f.s2);
  return sqd_triple(kind, x12);
}

/* Distance-type codes.
 * PT (slots p,t0,t1,t2): 0..2 point-vertex t_k, 3..5 point-edge k
 *   (edges t0t1, t1t2, t2t0), 6 point-plane interior.
 * EE (slots a0,a1,b0,b1): 0..3 point-point (a_i,b_j) -> 2i+j,
 *   4..5 a_i on segment b, 6..7 b_j on segment a, 8 line-line interior. */
Feature classify(int kind, const double* x12, double* Dout) {
  Feature best;
  double bestD = INFINITY;
  if (kind == ORC_PT) {
    const int E[3][2] = {{1, 2}, {2, 3}, {3, 1}};
    for (int k = 0; k < 3; ++k) {
      Feature f = point_segment(x12, 0, E[k][0], E[k][1], E[k][0] - 1,
                                E[k][1] - 1, 3 + k);
      double D = feature_sqd(kind, x12, f);
      if (D < bestD) { bestD = D; best = f; }
    }
    double a[3], b[3], c[3];
    sub3(slot(x12, 0), slot(x12, 1), a);
    sub3(slot(x12, 2), slot(x12, 1), b);
    sub3(slot(x12, 3), slot(x12, 1), c);
    double bb = dot3(b, b), bc = dot3(b, c), cc = dot3(c, c);
    double ab = dot3(a, b), ac = dot3(a, c);
    double det = bb * cc - bc * bc;
    if (det > 0.0) {
      double b1 = (ab * cc - ac * bc) / det;
      double b2 = (ac * bb - ab * bc) / det;
      if (b1 > 0.0 && b2 > 0.0 && b1 + b2 < 1.0) {
        Feature f;
        f.type = F_TRIPLE; f.s0 = f.s1 = f.s2 = -1; f.code = 6;
        double D = feature_sqd(kind, x12, f);
        if (D < bestD) { bestD = D; best = f; }
      }
    }
  } else {
    Feature c4[4] = {point_segment(x12, 0, 2, 3, 0, 1, 4),
                     point_segment(x12, 1, 2, 3, 2, 3, 5),
                     point_segment(x12, 2, 0, 1, 0, 2, 6),
                     point_segment(x12, 3, 0, 1, 1, 3, 7)};
    for (int k = 0; k < 4; ++k) {
      double D = feature_sqd(kind, x12, c4[k]);
      if (D < bestD) { bestD = D; best = c4[k]; }
    }
    double u[3], v[3], w[3], n[3];
    sub3(slot(x12, 1), slot(x12, 0), u);
    sub3(slot(x12, 3), slot(x12, 2), v);
    sub3(slot(x12, 0), slot(x12, 2), w);
    cross3(u, v, n);
    double N = dot3(n, n);
    if (N > 0.0) {
      double uu = dot3(u, u), uv = dot3(u, v), vv = dot3(v, v);
      double uw = dot3(u, w), vw = dot3(v, w);
      double s = (uv * vw - vv * uw) / N;
      double t = (uu * vw - uv * uw) / N;
      if (s > 0.0 && s < 1.0 && t > 0.0 && t < 1.0) {
        Feature f;
        f.type = F_TRIPLE; f.s0 = f.s1 = f.s2 = -1; f.code = 8;
        double D = feature_sqd(kind, x12, f);
        if (D < bestD) { bestD = D; best = f; }
      }
    }
  }
  *Dout = bestD;
  return best;
}

/* squared distance of the classified feature with derivatives on 12 coords */
void feature_sqd_deriv(int kind, const double* x12, const Feature& f,
                       Deriv& out) {
  if (f.type == F_PP) {
    Deriv y;
    y.zero();
    double d[3];
    sub3(slot(x12, f.s0), slot(x12, f.s1), d);
    y.f = dot3(d, d);
    for (int i = 0; i < 3; ++i) {
      y.g[i] = 2.0 * d[i];
      y.H[i * 12 + i] = 2.0;
    }
    int coef[1][4] = {{0, 0, 0, 0}};
    coef[0][f.s0] = 1;
    coef[0][f.s1] = -1;
    to_slots(y, 1, coef, out);
    return;
  }
  if (f.type == F_PE) {
    double a[3], e[3];
    sub3(slot(x12, f.s0), slot(x12, f.s1), a);
    sub3(slot(x12, f.s2), slot(x12, f.s1), e);
    Deriv K, L, D;
    cross_norm_sq(a, e, 0, 3, K);
    L.zero();
    L.f = dot3(e, e);
    for (int i = 0; i < 3; ++i) {
      L.g[3 + i] = 2.0 * e[i];
      L.H[(3 + i) * 12 + 3 + i] = 2.0;
    }
    quotient(K, L, 6, D);
    int coef[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    coef[0][f.s0] += 1;
    coef[0][f.s1] -= 1; /* a = x_p - x_e0 */
    coef[1][f.s2] += 1;
    coef[1][f.s1] -= 1; /* e = x_e1 - x_e0 */
    to_slots(D, 2, coef, out);
    return;
  }
  double a[3], b[3], c[3];
  triple_vars(kind, x12, a, b, c);
  Deriv S, N, D;
  triple_sq(a, b, c, S);
  cross_norm_sq(b, c, 3, 6, N);
  quotient(S, N, 9, D);
  to_slots(D, 3, (kind == ORC_PT) ? PT_COEF : EE_COEF, out);
}

/* ------------------------------------------------------------------ */
/* symmetric eigendecomposition (cyclic Jacobi) and PSD projection      */
/* ------------------------------------------------------------------ */
void jacobi_eig(int n, const double* Hin, double* w, double* V) {
  std::vector<double> A(Hin, Hin + n * n);
  for (int i = 0; i < n * n; ++i) V[i] = 0.0;
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  double fro = 0.0;
  for (int i = 0; i < n * n; ++i) fro += A[i] * A[i];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off <= 1e-30 * fro || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = 1.0 / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        if (theta < 0.0) t = -t;
        double c = 1.0 / std::sqrt(t * t + 1.0);
        double s = t * c;
        for (int k = 0; k < n; ++k) { /* columns p, q */
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) { /* rows p, q */
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

/* H+ = V max(lambda, 0) V^T */
void psd_project(int n, const double* H, double* out) {
  std::vector<double> w(n), V(n * n);
  jacobi_eig(n, H, w.data(), V.data());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k)
        if (w[k] > 0.0) v += V[i * n + k] * w[k] * V[j * n + k];
      out[i * n + j] = v;
    }
}

/* ------------------------------------------------------------------ */
/* pair barrier energy                                                  */
/* ------------------------------------------------------------------ */
/* E = w m(c) b(d) for a PT or EE pair on 12 coordinates; m = 1 unless EE
 * with eps_x > 0. Returns 1 if the pair is active (d < dhat). */
int pair_energy(int kind, const double* x12, double eps_x, double dh,
                double w, bool want_derivs, bool project, double* E,
                double* g12, double* H144, double* dist, int* dtype) {
  double D;
  Feature f = classify(kind, x12, &D);
  double d = std::sqrt(D);
  if (dist) *dist = d;
  if (dtype) *dtype = f.code;
  if (!(d < dh)) {
    *E = 0.0;
    if (want_derivs) {
      std::memset(g12, 0, 12 * sizeof(double));
      std::memset(H144, 0, 144 * sizeof(double));
    }
    return 0;
  }
  double b, b1, b2;
  barrier(d, dh, &b, &b1, &b2);
  /* mollifier m(c) = (2 - c/eps) c/eps for c < eps, with c = |u x v|^2 */
  double m = 1.0;
  Deriv M;
  M.zero();
  bool moll = false;
  if (kind == ORC_EE && eps_x > 0.0) {
    double u[3], v[3];
    sub3(slot(x12, 1), slot(x12, 0), u);
    sub3(slot(x12, 3), slot(x12, 2), v);
    Deriv C;
    cross_norm_sq(u, v, 0, 3, C);
    if (C.f < eps_x) {
      moll = true;
      double r = C.f / eps_x;
      m = (2.0 - r) * r;
      double m1 = 2.0 * (1.0 - r) / eps_x;
      double m2 = -2.0 / (eps_x * eps_x);
      Deriv Mc;
      Mc.zero();
      Mc.f = m;
      for (int i = 0; i < 6; ++i) Mc.g[i] = m1 * C.g[i];
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j)
          Mc.H[i * 12 + j] = m2 * C.g[i] * C.g[j] + m1 * C.H[i * 12 + j];
      const int MC[2][4] = {{-1, 1, 0, 0}, {0, 0, -1, 1}};
      to_slots(Mc, 2, MC, M);
    }
  }
  *E = w * m * b;
  if (!want_derivs) return 1;
  Deriv Dd;
  feature_sqd_deriv(kind, x12, f, Dd);
  double gd[12];
  for (int i = 0; i < 12; ++i) gd[i] = Dd.g[i] / (2.0 * d);
  double Hd[144];
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < 12; ++j)
      Hd[i * 12 + j] = Dd.H[i * 12 + j] / (2.0 * d) -
                       Dd.g[i] * Dd.g[j] / (4.0 * d * d * d);
  for (int i = 0; i < 12; ++i) {
    double gi = m * b1 * gd[i];
    if (moll) gi += b * M.g[i];
    g12[i] = w * gi;
  }
  double H[144];
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < 12; ++j) {
      double h = m * (b2 * gd[i] * gd[j] + b1 * Hd[i * 12 + j]);
      if (moll)
        h += b1 * (M.g[i] * gd[j] + gd[i] * M.g[j]) + b * M.H[i * 12 + j];
      H[i * 12 + j] = w * h;
    }
  if (project)
    psd_project(12, H, H144);
  else
    std::memcpy(H144, H, sizeof(H));
  return 1;
}

double pair_distance(int kind, const double* x12) {
  double D;
  classify(kind, x12, &D);
  return std::sqrt(D);
}

/* ------------------------------------------------------------------ */
/* orthogonality energy ||A A^T - I||_F^2                               */
/* ------------------------------------------------------------------ */
void orth_energy(const double* A, double* E, double* g9, double* H81,
                 bool project) {
  double S[9], AtA[9];
  for (int k = 0; k < 3; ++k)
    for (int m = 0; m < 3; ++m) {
      double s = 0.0, t = 0.0;
      for (int n = 0; n < 3; ++n) {
        s += A[k * 3 + n] * A[m * 3 + n];
        t += A[n * 3 + k] * A[n * 3 + m];
      }
      S[k * 3 + m] = s - ((k == m) ? 1.0 : 0.0);
      AtA[k * 3 + m] = t;
    }
  double e = 0.0;
  for (int i = 0; i < 9; ++i) e += S[i] * S[i];
  *E = e;
  if (g9)
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) {
        double v = 0.0;
        for (int m = 0; m < 3; ++m) v += S[k * 3 + m] * A[m * 3 + l];
        g9[k * 3 + l] = 4.0 * v;
      }
  if (H81) {
    double H[81];
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l)
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) {
            double v = A[k * 3 + q] * A[p * 3 + l];
            if (k == p) v += AtA[q * 3 + l];
            if (l == q) v += S[k * 3 + p];
            H[(k * 3 + l) * 9 + p * 3 + q] = 4.0 * v;
          }
    if (project)
      psd_project(9, H, H81);
    else
      std::memcpy(H81, H, sizeof(H));
  }
}

/* DoF index of coordinate i, affine basis k (k = 0: p_i, k >= 1: A_i,k-1) */
int dof(int i, int k) { return (k == 0) ? i : 3 + 3 * i + (k - 1); }

/* ------------------------------------------------------------------ */
/* mass properties by the divergence theorem                            */
/* ------------------------------------------------------------------ */
void mass_props(const double* xb, int nv, const int* tris, int nt,
                double density, double* Mhat, double* vol) {
  (void)nv;
  double V = 0.0, first[3] = {0, 0, 0}, second[9] = {0};
  for (int t = 0; t < nt; ++t) {
    const double* a = xb + 3 * tris[3 * t];
    const double* b = xb + 3 * tris[3 * t + 1];
    const double* c = xb + 3 * tris[3 * t + 2];
    double bc[3];
    cross3(b, c, bc);
    double Vt = dot3(a, bc) / 6.0; /* tet (0, a, b, c) */
    V += Vt;
    double s[3];
    for (int i = 0; i < 3; ++i) {
      s[i] = a[i] + b[i] + c[i];
      first[i] += Vt * s[i] / 4.0;
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        second[i * 3 + j] += Vt / 20.0 *
                             (a[i] * a[j] + b[i] * b[j] + c[i] * c[j] +
                              s[i] * s[j]);
  }
  *vol = V;
  Mhat[0] = density * V;
  for (int i = 0; i < 3; ++i) {
    Mhat[1 + i] = density * first[i];
    Mhat[(1 + i) * 4] = density * first[i];
    for (int j = 0; j < 3; ++j)
      Mhat[(1 + i) * 4 + 1 + j] = density * second[i * 3 + j];
  }
}

/* ------------------------------------------------------------------ */
/* dense Cholesky                                                       */
/* ------------------------------------------------------------------ */
bool cholesky(int n, std::vector<double>& A) {
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = v / d;
    }
  }
  return true;
}
void cholesky_solve(int n, const std::vector<double>& L, double* b) {
  for (int i = 0; i < n; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * b[k];
    b[i] = v / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = b[i];
    for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * b[k];
    b[i] = v / L[(size_t)i * n + i];
  }
}

/* ------------------------------------------------------------------ */
/* boxes and the candidate predicate                                    */
/* ------------------------------------------------------------------ */
struct Box {
  double lo[3], hi[3];
};
void box_empty(Box& b) {
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = INFINITY;
    b.hi[k] = -INFINITY;
  }
}
void box_add(Box& b, const double* p) {
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = std::min(b.lo[k], p[k]);
    b.hi[k] = std::max(b.hi[k], p[k]);
  }
}
void box_merge(Box& b, const Box& o) {
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = std::min(b.lo[k], o.lo[k]);
    b.hi[k] = std::max(b.hi[k], o.hi[k]);
  }
}
/* lo_P <= hi_Q + dhat and lo_Q <= hi_P + dhat on every axis */
bool overlap(const Box& P, const Box& Q, double dh) {
  for (int k = 0; k < 3; ++k) {
    if (!(P.lo[k] <= Q.hi[k] + dh)) return false;
    if (!(Q.lo[k] <= P.hi[k] + dh)) return false;
  }
  return true;
}

}  // namespace

/* ==================================================================== */
/* scene                                                                 */
/* ==================================================================== */
struct orc_body {
  int kind;
  double density;
  int v0, nv, t0, nt, e0, ne;
  double Mhat[16];
  double vol;
  double q[12], qt[12], qtilde[12], qdot[12];
  bool shared;
  double z[12], u[12], rho;
  int kappa_b;
};

struct orc_scene {
  orc_params P;
  std::vector<orc_body> B;
  std::vector<double> xbar; /* [V][3] rest coordinates */
  std::vector<int> vbody;
  std::vector<int> tri; /* [T][3] global vertex ids */
  std::vector<int> tbody;
  std::vector<int> edge; /* [E][2] global vertex ids */
  std::vector<int> ebody;
  std::vector<double> erest2; /* rest squared edge length */
  int pair_mode = 0;
  bool project = true; /* PSD projection of pair and orthogonality Hessians */
  double scale = 1.0;
  bool finalized = false;
  std::string err;
};

namespace {

int fail(orc_scene* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  return code;
}

/* x = A xbar + p, summed left to right: p_i + A_i0 xb0 + A_i1 xb1 + A_i2 xb2 */
void vertex_pos(const double* q, const double* xb, double* x) {
  for (int i = 0; i < 3; ++i)
    x[i] = q[i] + q[3 + 3 * i] * xb[0] + q[4 + 3 * i] * xb[1] +
           q[5 + 3 * i] * xb[2];
}

void positions(const orc_scene* s, const double* q /*B*12*/,
               std::vector<double>& x) {
  size_t V = s->vbody.size();
  x.resize(V * 3);
#pragma omp parallel for schedule(static)
  for (size_t v = 0; v < V; ++v)
    vertex_pos(q + 12 * s->vbody[v], &s->xbar[3 * v], &x[3 * v]);
}

void current_q(const orc_scene* s, std::vector<double>& q) {
  q.resize(12 * s->B.size());
  for (size_t b = 0; b < s->B.size(); ++b)
    std::memcpy(&q[12 * b], s->B[b].q, 12 * sizeof(double));
}

struct Cands {
  std::vector<std::pair<int, int>> pt, ee;
  std::vector<int> pg;
};

/* Candidate pairs for positions x and (optionally) end positions x1 = x+dx.
 * Body boxes cull body pairs; within a body pair, primitives of one body
 * are kept only if they pass the predicate against the other body's box
 * (sound: every primitive box lies inside its body box and rounding of
 * hi + dhat is monotone), then every remaining primitive pair is tested
 * with the predicate itself. */
void candidates(const orc_scene* s, const std::vector<double>& x,
                const double* dx, Cands& C) {
  const double dh = s->P.dhat;
  size_t V = s->vbody.size(), T = s->tbody.size(), E = s->ebody.size();
  std::vector<double> x1;
  if (dx) {
    x1.resize(3 * V);
    for (size_t i = 0; i < 3 * V; ++i) x1[i] = x[i] + dx[i];
  }
  std::vector<Box> vb(V), tb(T), eb(E);
#pragma omp parallel for schedule(static)
  for (size_t v = 0; v < V; ++v) {
    box_empty(vb[v]);
    box_add(vb[v], &x[3 * v]);
    if (dx) box_add(vb[v], &x1[3 * v]);
  }
#pragma omp parallel for schedule(static)
  for (size_t t = 0; t < T; ++t) {
    box_empty(tb[t]);
    for (int k = 0; k < 3; ++k) box_merge(tb[t], vb[s->tri[3 * t + k]]);
  }
#pragma omp parallel for schedule(static)
  for (size_t e = 0; e < E; ++e) {
    box_empty(eb[e]);
    for (int k = 0; k < 2; ++k) box_merge(eb[e], vb[s->edge[2 * e + k]]);
  }
  size_t nb = s->B.size();
  std::vector<Box> bb(nb);
  for (size_t b = 0; b < nb; ++b) {
    box_empty(bb[b]);
    const orc_body& o = s->B[b];
    for (int v = 0; v < o.nv; ++v) box_merge(bb[b], vb[o.v0 + v]);
  }
  C.pt.clear();
  C.ee.clear();
  C.pg.clear();
  /* body pairs (a, b > a): the pairs found for each a are collected on
   * their own and joined in the order of a; the lists are sorted below, so
   * the result does not depend on how the loop over a is split */
  std::vector<Cands> per_a(nb);
#pragma omp parallel for schedule(dynamic, 1)
  for (size_t a = 0; a < nb; ++a) {
    Cands& Ca = per_a[a];
    std::vector<int> L1, L2;
    for (size_t b = a + 1; b < nb; ++b) {
      const orc_body& A = s->B[a];
      const orc_body& Bb = s->B[b];
      if (A.kind != 0 && Bb.kind != 0) continue;
      if (!overlap(bb[a], bb[b], dh)) continue;
      for (int dir = 0; dir < 2; ++dir) {
        const orc_body& P = dir ? Bb : A; /* point body */
        const orc_body& Q = dir ? A : Bb; /* triangle body */
        const Box& boxP = dir ? bb[b] : bb[a];
        const Box& boxQ = dir ? bb[a] : bb[b];
        L1.clear();
        L2.clear();
        for (int v = 0; v < P.nv; ++v)
          if (overlap(vb[P.v0 + v], boxQ, dh)) L1.push_back(P.v0 + v);
        for (int t = 0; t < Q.nt; ++t)
          if (overlap(tb[Q.t0 + t], boxP, dh)) L2.push_back(Q.t0 + t);
        for (int v : L1)
          for (int t : L2)
            if (overlap(vb[v], tb[t], dh)) Ca.pt.push_back({v, t});
      }
      L1.clear();
      L2.clear();
      for (int e = 0; e < A.ne; ++e)
        if (overlap(eb[A.e0 + e], bb[b], dh)) L1.push_back(A.e0 + e);
      for (int e = 0; e < Bb.ne; ++e)
        if (overlap(eb[Bb.e0 + e], bb[a], dh)) L2.push_back(Bb.e0 + e);
      for (int e : L1)
        for (int f : L2)
          if (overlap(eb[e], eb[f], dh))
            Ca.ee.push_back({std::min(e, f), std::max(e, f)});
    }
  }
  for (const Cands& Ca : per_a) {
    C.pt.insert(C.pt.end(), Ca.pt.begin(), Ca.pt.end());
    C.ee.insert(C.ee.end(), Ca.ee.begin(), Ca.ee.end());
  }
  if (s->P.has_ground) {
    double top = s->P.ground_y + dh;
    for (size_t v = 0; v < V; ++v)
      if (s->B[s->vbody[v]].kind == 0 && vb[v].lo[1] <= top)
        C.pg.push_back((int)v);
  }
  std::sort(C.pt.begin(), C.pt.end());
  std::sort(C.ee.begin(), C.ee.end());
  std::sort(C.pg.begin(), C.pg.end());
}

/* gather the 4 vertex slots of a pair */
void pair_slots(const orc_scene* s, int kind, int i, int j, int* vid) {
  if (kind == ORC_PT) {
    vid[0] = i;
    for (int k = 0; k < 3; ++k) vid[1 + k] = s->tri[3 * j + k];
  } else {
    vid[0] = s->edge[2 * i];
    vid[1] = s->edge[2 * i + 1];
    vid[2] = s->edge[2 * j];
    vid[3] = s->edge[2 * j + 1];
  }
}

double pair_kappa_c(const orc_scene* s, const int* vid, int n) {
  if (s->pair_mode == 0) return 1.0;
  for (int k = 0; k < n; ++k) {
    const orc_body& b = s->B[s->vbody[vid[k]]];
    if (b.kind == 0 && !b.shared) return 1.0;
  }
  return 2.0;
}

double pair_eps_x(const orc_scene* s, int e, int f) {
  if (!s->P.mollify_ee) return 0.0;
  return MOLLIFIER_EPS * s->erest2[e] * s->erest2[f];
}

/* global system: E, g [B][12], Hdiag [B][144], Hoff map (a<b) */
struct System {
  double E = 0.0;
  std::vector<double> g, Hd;
  std::map<std::pair<int, int>, std::vector<double>> Ho;
  int64_t n_active = 0;
  double min_dist = INFINITY;
};

/* add a vertex-space gradient / Hessian of n slots to the body system */
void jmap(const orc_scene* s, const int* vid, int n, const double* g,
          const double* H, int stride, System& S) {
  double xh[4][4];
  int bo[4];
  for (int v = 0; v < n; ++v) {
    bo[v] = s->vbody[vid[v]];
    xh[v][0] = 1.0;
    for (int k = 0; k < 3; ++k) xh[v][1 + k] = s->xbar[3 * vid[v] + k];
  }
  for (int v = 0; v < n; ++v) {
    if (s->B[bo[v]].kind != 0) continue;
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k)
        S.g[12 * bo[v] + dof(i, k)] += g[3 * v + i] * xh[v][k];
  }
  for (int v = 0; v < n; ++v)
    for (int w = 0; w < n; ++w) {
      int bv = bo[v], bw = bo[w];
      if (s->B[bv].kind != 0 || s->B[bw].kind != 0) continue;
      if (bv > bw) continue; /* lower blocks are transposes */
      double* dst;
      if (bv == bw) {
        dst = &S.Hd[144 * bv];
      } else {
        auto& blk = S.Ho[{bv, bw}];
        if (blk.empty()) blk.assign(144, 0.0);
        dst = blk.data();
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double h = H[(3 * v + i) * stride + 3 * w + j];
          for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l)
              dst[dof(i, k) * 12 + dof(j, l)] += h * xh[v][k] * xh[w][l];
        }
    }
}

/* body terms: inertia, orthogonality (times h^2 kappa_A V), ADMM penalty */
void body_terms(const orc_scene* s, const double* q, System& S) {
  const double h2 = s->P.dt * s->P.dt;
  for (size_t b = 0; b < s->B.size(); ++b) {
    const orc_body& o = s->B[b];
    double* g = &S.g[12 * b];
    double* H = &S.Hd[144 * b];
    if (o.kind != 0) {
      for (int i = 0; i < 12; ++i) H[i * 12 + i] = 1.0; /* no DoFs */
      continue;
    }
    const double* qb = q + 12 * b;
    double wb = 1.0 / o.kappa_b;
    for (int i = 0; i < 3; ++i) {
      double d[4];
      for (int k = 0; k < 4; ++k) d[k] = qb[dof(i, k)] - o.qtilde[dof(i, k)];
      for (int k = 0; k < 4; ++k) {
        double md = 0.0;
        for (int l = 0; l < 4; ++l) md += o.Mhat[k * 4 + l] * d[l];
        S.E += wb * 0.5 * d[k] * md;
        g[dof(i, k)] += wb * md;
        for (int l = 0; l < 4; ++l)
          H[dof(i, k) * 12 + dof(i, l)] += wb * o.Mhat[k * 4 + l];
      }
    }
    double Eo, go[9], Hob[81];
    orth_energy(qb + 3, &Eo, go, Hob, s->project);
    double c = wb * h2 * s->P.kappa_A * o.vol;
    S.E += c * Eo;
    for (int i = 0; i < 9; ++i) {
      g[3 + i] += c * go[i];
      for (int j = 0; j < 9; ++j) H[(3 + i) * 12 + 3 + j] += c * Hob[i * 9 + j];
    }
    if (o.shared) {
      for (int i = 0; i < 12; ++i) {
        double r = qb[i] - o.z[i] + o.u[i];
        S.E += 0.5 * o.rho * r * r;
        g[i] += o.rho * r;
        H[i * 12 + i] += o.rho;
      }
    }
  }
}

void pair_terms(const orc_scene* s, const std::vector<double>& x,
                const Cands& C, System& S) {
  const double w0 = s->P.dt * s->P.dt * s->P.kappa;
  const double dh = s->P.dhat;
  /* each PT/EE pair's energy, gradient and projected Hessian is computed
   * on its own (in parallel in the OpenMP build), then the pairs are added
   * to the system one after another in list order */
  const size_t npt = C.pt.size(), n = npt + C.ee.size();
  struct PairOut {
    int act;
    double E, d, g12[12], H144[144];
  };
  std::vector<PairOut> out(n);
#pragma omp parallel for schedule(dynamic, 16)
  for (size_t c = 0; c < n; ++c) {
    const int kind = c < npt ? ORC_PT : ORC_EE;
    const auto& pr = c < npt ? C.pt[c] : C.ee[c - npt];
    int vid[4], dtype;
    double x12[12];
    pair_slots(s, kind, pr.first, pr.second, vid);
    for (int k = 0; k < 4; ++k)
      for (int i = 0; i < 3; ++i) x12[3 * k + i] = x[3 * vid[k] + i];
    double w = w0 / pair_kappa_c(s, vid, 4);
    double ex = kind == ORC_EE ? pair_eps_x(s, pr.first, pr.second) : 0.0;
    PairOut& o = out[c];
    o.act = pair_energy(kind, x12, ex, dh, w, true, s->project, &o.E, o.g12,
                        o.H144, &o.d, &dtype);
  }
  for (size_t c = 0; c < n; ++c) {
    const int kind = c < npt ? ORC_PT : ORC_EE;
    const auto& pr = c < npt ? C.pt[c] : C.ee[c - npt];
    const PairOut& o = out[c];
    S.min_dist = std::min(S.min_dist, o.d);
    if (!o.act) continue;
    int vid[4];
    pair_slots(s, kind, pr.first, pr.second, vid);
    S.n_active++;
    S.E += o.E;
    jmap(s, vid, 4, o.g12, o.H144, 12, S);
  }
  for (int v : C.pg) {
    double dist = x[3 * v + 1] - s->P.ground_y;
    S.min_dist = std::min(S.min_dist, dist);
    if (!(dist < dh)) continue;
    double b, b1, b2;
    barrier(dist, dh, &b, &b1, &b2);
    double w = w0 / pair_kappa_c(s, &v, 1);
    double g3[3] = {0.0, w * b1, 0.0};
    double H9[9] = {0, 0, 0, 0, w * b2, 0, 0, 0, 0};
    S.n_active++;
    S.E += w * b;
    jmap(s, &v, 1, g3, H9, 3, S);
  }
}

void assemble(orc_scene* s, const double* q, System& S, Cands* Cout) {
  size_t nb = s->B.size();
  S.g.assign(12 * nb, 0.0);
  S.Hd.assign(144 * nb, 0.0);
  S.Ho.clear();
  S.E = 0.0;
  S.n_active = 0;
  S.min_dist = INFINITY;
  std::vector<double> x;
  positions(s, q, x);
  Cands C;
  candidates(s, x, nullptr, C);
  body_terms(s, q, S);
  pair_terms(s, x, C, S);
  if (Cout) *Cout = C;
}

/* ------------------------------------------------------------------ */
/* linear solve H dq = -g over the dynamic bodies                      */
/* ------------------------------------------------------------------ */
int solve(orc_scene* s, const System& S, std::vector<double>& dq,
          int* iters) {
  size_t nb = s->B.size();
  std::vector<int> di(nb, -1);
  int nd = 0;
  for (size_t b = 0; b < nb; ++b)
    if (s->B[b].kind == 0) di[b] = nd++;
  int n = 12 * nd;
  dq.assign(12 * nb, 0.0);
  *iters = 0;
  if (n == 0) return ORC_OK;
  std::vector<double> rhs(n);
  for (size_t b = 0; b < nb; ++b)
    if (di[b] >= 0)
      for (int i = 0; i < 12; ++i) rhs[12 * di[b] + i] = -S.g[12 * b + i];
  std::vector<double> sol(n, 0.0);
  if (n <= s->P.dense_max_dof) {
    std::vector<double> A((size_t)n * n, 0.0);
    for (size_t b = 0; b < nb; ++b) {
      if (di[b] < 0) continue;
      for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j)
          A[(size_t)(12 * di[b] + i) * n + 12 * di[b] + j] = S.Hd[144 * b + 12 * i + j];
    }
    for (const auto& kv : S.Ho) {
      int a = di[kv.first.first], c = di[kv.first.second];
      for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) {
          A[(size_t)(12 * a + i) * n + 12 * c + j] = kv.second[12 * i + j];
          A[(size_t)(12 * c + j) * n + 12 * a + i] = kv.second[12 * i + j];
        }
    }
    if (!cholesky(n, A)) return fail(s, ORC_E_NOCONV, "Hessian not SPD");
    sol = rhs;
    cholesky_solve(n, A, sol.data());
    *iters = 1;
  } else {
    /* block-Jacobi preconditioned CG, zero initial guess */
    std::vector<std::vector<double>> Lb(nd);
    for (size_t b = 0; b < nb; ++b) {
      if (di[b] < 0) continue;
      Lb[di[b]].assign(S.Hd.begin() + 144 * b, S.Hd.begin() + 144 * b + 144);
      if (!cholesky(12, Lb[di[b]]))
        return fail(s, ORC_E_NOCONV, "diagonal block not SPD");
    }
    auto matvec = [&](const std::vector<double>& p, std::vector<double>& y) {
      y.assign(n, 0.0);
      for (size_t b = 0; b < nb; ++b) {
        if (di[b] < 0) continue;
        int o = 12 * di[b];
        for (int i = 0; i < 12; ++i) {
          double v = 0.0;
          for (int j = 0; j < 12; ++j) v += S.Hd[144 * b + 12 * i + j] * p[o + j];
          y[o + i] += v;
        }
      }
      for (const auto& kv : S.Ho) {
        int a = 12 * di[kv.first.first], c = 12 * di[kv.first.second];
        const double* H = kv.second.data();
        for (int i = 0; i < 12; ++i)
          for (int j = 0; j < 12; ++j) {
            y[a + i] += H[12 * i + j] * p[c + j];
            y[c + j] += H[12 * i + j] * p[a + i];
          }
      }
    };
    auto precond = [&](const std::vector<double>& r, std::vector<double>& z) {
      z = r;
      for (int d = 0; d < nd; ++d) cholesky_solve(12, Lb[d], &z[12 * d]);
    };
    auto dotn = [&](const std::vector<double>& a, const std::vector<double>& b) {
      double v = 0.0;
      for (int i = 0; i < n; ++i) v += a[i] * b[i];
      return v;
    };
    std::vector<double> r = rhs, z, p, Ap;
    double bn = std::sqrt(dotn(rhs, rhs));
    double tol = s->P.pcg_eta * bn;
    precond(r, z);
    p = z;
    double rz = dotn(r, z);
    int it = 0;
    while (it < s->P.max_pcg && std::sqrt(dotn(r, r)) > tol) {
      matvec(p, Ap);
      double alpha = rz / dotn(p, Ap);
      for (int i = 0; i < n; ++i) {
        sol[i] += alpha * p[i];
        r[i] -= alpha * Ap[i];
      }
      ++it;
      precond(r, z);
      double rz1 = dotn(r, z);
      double beta = rz1 / rz;
      rz = rz1;
      for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    *iters = it;
  }
  for (size_t b = 0; b < nb; ++b)
    if (di[b] >= 0)
      for (int i = 0; i < 12; ++i) dq[12 * b + i] = sol[12 * di[b] + i];
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* additive CCD                                                         */
/* ------------------------------------------------------------------ */
double accd(int kind, const double* x, const double* dx, double s,
            double tmax) {
  double m[3] = {0, 0, 0};
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 3; ++i) m[i] += dx[3 * k + i] / 4.0;
  double r[12];
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 3; ++i) r[3 * k + i] = dx[3 * k + i] - m[i];
  double n0 = norm3(r), n1 = norm3(r + 3), n2 = norm3(r + 6),
         n3 = norm3(r + 9);
  double lp = (kind == ORC_PT) ? n0 + std::max(n1, std::max(n2, n3))
                               : std::max(n0, n1) + std::max(n2, n3);
  if (lp == 0.0) return tmax;
  double d0 = pair_distance(kind, x);
  if (!(d0 > 0.0)) return 0.0;
  double gap = s * d0;
  double t = 0.0;
  double tl = (1.0 - s) * d0 / lp;
  double xt[12];
  double d = d0;
  int it = 0;
  for (; it < ACCD_SERIAL_IT; ++it) {
    double tn = t + tl;
    for (int i = 0; i < 12; ++i) xt[i] = x[i] + tn * r[i];
    d = pair_distance(kind, xt);
    if (t > 0.0 && d < gap) return t;
    t = tn;
    if (t > tmax) return tmax;
    tl = 0.9 * d / lp;
  }
  /* then steps of ACCD_BLOCK points t + j delta that share the step
   * length delta = 0.5 da / lp of their anchor (t, da): point j is
   * reached when it keeps the gap and every point before it keeps the
   * distance at least 0.6 da, so each accepted segment keeps
   * d >= 0.6 da - lp delta = 0.1 da > 0 along it.  A pair that slides at a
   * small distance, or closes it slowly, advances up to ACCD_BLOCK points
   * per step (each point half the one-point step) */
  double da = d;
  for (; it < ACCD_MAX_IT; it += ACCD_BLOCK) {
    const double delta = 0.5 * da / lp;
    const double keep = 0.6 * da;
    int J = 0;
    double dJ = da;
    for (int j = 1; j <= ACCD_BLOCK; ++j) {
      const double tj = t + (double)j * delta;
      for (int i = 0; i < 12; ++i) xt[i] = x[i] + tj * r[i];
      const double dj = pair_distance(kind, xt);
      if (dj < gap) break;
      J = j;
      dJ = dj;
      if (dj < keep) break;
    }
    if (J == 0) return t;
    t = t + (double)J * delta;
    if (t > tmax) return tmax;
    da = dJ;
  }
  return t;
}

/* ------------------------------------------------------------------ */
/* exact time of impact along the linear trajectory                     */
/* ------------------------------------------------------------------ */
/* Affine bodies move every vertex on a straight line over a Newton step,
 * x(t) = x + t dx.  Two primitives touch at the first t where their
 * distance is zero, and a zero distance needs the four points to be
 * coplanar, i.e. a root of the signed volume
 *     PT: f(t) = ((t1 - t0) x (t2 - t0)) . (p - t0)
 *     EE: f(t) = ((a1 - a0) x (b1 - b0)) . (b0 - a0),
 * a cubic in t.  The real roots in [0, tmax] are isolated on the monotone
 * pieces between the roots of f'(t) (a quadratic), bracketed by the sign of
 * f evaluated directly from the moved points, and bisected down to adjacent
 * doubles; a critical point where f nearly vanishes (a tangential touch) is
 * a root candidate too.  The earliest candidate at which the primitives'
 * distance is zero up to rounding (within 1e-12 of the coordinates'
 * magnitude) is the contact; the lower end of its bracket is returned.  A
 * pair whose signed volume vanishes identically (motion inside a common
 * plane) is resolved by dense sampling of the distance instead.  Returns
 * tmax when the primitives do not touch in [0, tmax]. */
struct Moving {
  const double* x;
  const double* dx;
  int kind;
  void at(double t, double* y) const {
    for (int i = 0; i < 12; ++i) y[i] = x[i] + t * dx[i];
  }
  /* (u, v, w) of the signed volume (u x v) . w for point set y */
  void uvw(const double* y, double* u, double* v, double* w) const {
    if (kind == ORC_PT) {
      sub3(y + 6, y + 3, u);
      sub3(y + 9, y + 3, v);
      sub3(y + 0, y + 3, w);
    } else {
      sub3(y + 3, y + 0, u);
      sub3(y + 9, y + 6, v);
      sub3(y + 6, y + 0, w);
    }
  }
  double volume(double t) const {
    double y[12], u[3], v[3], w[3], n[3];
    at(t, y);
    uvw(y, u, v, w);
    cross3(u, v, n);
    return dot3(n, w);
  }
  double distance(double t) const {
    double y[12];
    at(t, y);
    return pair_distance(kind, y);
  }
};

/* bisect a sign change of f on [lo, hi] down to adjacent doubles; returns
 * the lower end (f(lo) has the sign of the start or is zero) */
double bisect_root(const Moving& m, double lo, double hi, double flo) {
  if (flo == 0.0) return lo;
  for (int it = 0; it < 2000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    const double fm = m.volume(mid);
    if (fm == 0.0) return mid;
    if ((fm > 0.0) == (flo > 0.0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return lo;
}

double exact_toi(int kind, const double* x, const double* dx, double tmax) {
  Moving m{x, dx, kind};
  double mag = 0.0;
  for (int i = 0; i < 12; ++i) mag = std::max(mag, std::fabs(x[i]) + std::fabs(dx[i]));
  const double tol_d = 1e-12 * mag;
  if (m.distance(0.0) <= tol_d) return 0.0;
  /* cubic coefficients of f(t) = (u x v) . w with u = u0 + t du, ... */
  double y0[12], u0[3], v0[3], w0[3], du[3], dv[3], dw[3];
  m.at(0.0, y0);
  m.uvw(y0, u0, v0, w0);
  m.uvw(dx, du, dv, dw); /* the same differences of the displacements */
  double n00[3], n01[3], n10[3], n11[3];
  cross3(u0, v0, n00);
  cross3(u0, dv, n01);
  cross3(du, v0, n10);
  cross3(du, dv, n11);
  const double c1 = dot3(n00, dw) + dot3(n01, w0) + dot3(n10, w0);
  const double c2 = dot3(n01, dw) + dot3(n10, dw) + dot3(n11, w0);
  const double c3 = dot3(n11, dw);
  const double c0 = dot3(n00, w0);
  const double vol_scale = mag * mag * mag;
  const double tol_f = 1e-13 * vol_scale;
  if (std::fabs(c0) <= tol_f && std::fabs(c1) <= tol_f && std::fabs(c2) <= tol_f &&
      std::fabs(c3) <= tol_f) {
    /* coplanar throughout: first sampled zero distance */
    const int N = 20000;
    double prev = 0.0;
    for (int i = 1; i <= N; ++i) {
      const double t = tmax * i / N;
      if (m.distance(t) <= tol_d) return prev;
      prev = t;
    }
    return tmax;
  }
  /* split points: roots of f'(t) = c1 + 2 c2 t + 3 c3 t^2 inside (0, tmax) */
  std::vector<double> cuts = {0.0};
  {
    const double A = 3.0 * c3, Bq = 2.0 * c2, Cq = c1;
    std::vector<double> r;
    if (std::fabs(A) > 1e-300) {
      const double disc = Bq * Bq - 4.0 * A * Cq;
      if (disc >= 0.0) {
        const double sq = std::sqrt(disc);
        /* numerically stable pair of roots */
        const double qq = -0.5 * (Bq + (Bq >= 0.0 ? sq : -sq));
        if (qq != 0.0) {
          r.push_back(qq / A);
          r.push_back(Cq / qq);
        } else {
          r.push_back(0.0);
        }
      }
    } else if (std::fabs(Bq) > 1e-300) {
      r.push_back(-Cq / Bq);
    }
    std::sort(r.begin(), r.end());
    for (double t : r)
      if (t > 0.0 && t < tmax) cuts.push_back(t);
  }
  cuts.push_back(tmax);
  /* root candidates in increasing order */
  std::vector<double> cand;
  for (size_t k = 0; k + 1 < cuts.size(); ++k) {
    const double a = cuts[k], b = cuts[k + 1];
    const double fa = m.volume(a), fb = m.volume(b);
    if (k > 0 && std::fabs(fa) <= tol_f) cand.push_back(a); /* touch at a cut */
    if (fa == 0.0)
      cand.push_back(a);
    else if (fb == 0.0)
      cand.push_back(b);
    else if ((fa > 0.0) != (fb > 0.0))
      cand.push_back(bisect_root(m, a, b, fa));
  }
  std::sort(cand.begin(), cand.end());
  for (double t : cand)
    if (t >= 0.0 && t <= tmax && m.distance(t) <= tol_d) return t;
  return tmax;
}

double ccd_alpha(orc_scene* s, const std::vector<double>& x,
                 const std::vector<double>& dx, const Cands& C) {
  double amax = 1.0;
  /* a minimum: the same in any order of the pairs */
  const long npt = (long)C.pt.size(), n = npt + (long)C.ee.size();
#pragma omp parallel for schedule(dynamic, 16) reduction(min : amax)
  for (long c = 0; c < n; ++c) {
    const int kind = c < npt ? ORC_PT : ORC_EE;
    const auto& pr = c < npt ? C.pt[c] : C.ee[c - npt];
    double x12[12], d12[12];
    int vid[4];
    pair_slots(s, kind, pr.first, pr.second, vid);
    for (int k = 0; k < 4; ++k)
      for (int i = 0; i < 3; ++i) {
        x12[3 * k + i] = x[3 * vid[k] + i];
        d12[3 * k + i] = dx[3 * vid[k] + i];
      }
    amax = std::min(amax, accd(kind, x12, d12, ACCD_S, 1.0));
  }
  for (int v : C.pg) {
    double y0 = x[3 * v + 1] - s->P.ground_y;
    double dy = dx[3 * v + 1];
    if (dy < 0.0) amax = std::min(amax, (1.0 - ACCD_S) * y0 / (-dy));
  }
  return amax;
}

/* E(q + alpha dq) - E(q), term by term */
double energy_delta(orc_scene* s, const double* q, const double* dq,
                    double alpha, const std::vector<double>& x,
                    const Cands& C) {
  const double h2 = s->P.dt * s->P.dt;
  double dE = 0.0;
  size_t nb = s->B.size();
  std::vector<double> q1(12 * nb);
  for (size_t i = 0; i < 12 * nb; ++i) q1[i] = q[i] + alpha * dq[i];
  for (size_t b = 0; b < nb; ++b) {
    const orc_body& o = s->B[b];
    if (o.kind != 0) continue;
    const double* qb = q + 12 * b;
    double wb = 1.0 / o.kappa_b;
    double step[12];
    for (int i = 0; i < 12; ++i) step[i] = alpha * dq[12 * b + i];
    /* inertia: D^T M (d + D/2) per coordinate */
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 4; ++k) {
        double v = 0.0;
        for (int l = 0; l < 4; ++l)
          v += o.Mhat[k * 4 + l] *
               (qb[dof(i, l)] - o.qtilde[dof(i, l)] + 0.5 * step[dof(i, l)]);
        dE += wb * step[dof(i, k)] * v;
      }
    /* orthogonality: <dS, 2S + dS> with dS = A D^T + D A^T + D D^T */
    const double* A = qb + 3;
    const double* D = step + 3;
    double acc = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int m = 0; m < 3; ++m) {
        double S = 0.0, dS = 0.0;
        for (int n = 0; n < 3; ++n) {
          S += A[k * 3 + n] * A[m * 3 + n];
          dS += A[k * 3 + n] * D[m * 3 + n] + D[k * 3 + n] * A[m * 3 + n] +
                D[k * 3 + n] * D[m * 3 + n];
        }
        if (k == m) S -= 1.0;
        acc += dS * (2.0 * S + dS);
      }
    dE += wb * h2 * s->P.kappa_A * o.vol * acc;
    if (o.shared)
      for (int i = 0; i < 12; ++i) {
        double r = qb[i] - o.z[i] + o.u[i];
        dE += o.rho * step[i] * (r + 0.5 * step[i]);
      }
  }
  std::vector<double> x1;
  positions(s, q1.data(), x1);
  const double w0 = h2 * s->P.kappa;
  const double dh = s->P.dhat;
  /* each pair's E1 - E0 on its own (in parallel in the OpenMP build), then
   * summed in list order */
  const long npt = (long)C.pt.size(), n = npt + (long)C.ee.size();
  std::vector<double> de(n);
#pragma omp parallel for schedule(dynamic, 16)
  for (long c = 0; c < n; ++c) {
    const int kind = c < npt ? ORC_PT : ORC_EE;
    const auto& pr = c < npt ? C.pt[c] : C.ee[c - npt];
    double a12[12], b12[12], E0, E1;
    int vid[4];
    pair_slots(s, kind, pr.first, pr.second, vid);
    for (int k = 0; k < 4; ++k)
      for (int i = 0; i < 3; ++i) {
        a12[3 * k + i] = x[3 * vid[k] + i];
        b12[3 * k + i] = x1[3 * vid[k] + i];
      }
    double w = w0 / pair_kappa_c(s, vid, 4);
    double ex = kind == ORC_EE ? pair_eps_x(s, pr.first, pr.second) : 0.0;
    pair_energy(kind, a12, ex, dh, w, false, false, &E0, nullptr, nullptr,
                nullptr, nullptr);
    pair_energy(kind, b12, ex, dh, w, false, false, &E1, nullptr, nullptr,
                nullptr, nullptr);
    de[c] = E1 - E0;
  }
  for (long c = 0; c < n; ++c) dE += de[c];
  for (int v : C.pg) {
    double w = w0 / pair_kappa_c(s, &v, 1);
    double b0, b1, c0, c1, t0, t1;
    barrier(x[3 * v + 1] - s->P.ground_y, dh, &b0, &c0, &t0);
    barrier(x1[3 * v + 1] - s->P.ground_y, dh, &b1, &c1, &t1);
    dE += w * (b1 - b0);
  }
  return dE;
}

double inf_norm(const std::vector<double>& v) {
  double m = 0.0;
  for (double a : v) m = std::max(m, std::fabs(a));
  return m;
}

/* segment (p,q) crosses triangle (a,b,c) strictly */
double orient(const double* a, const double* b, const double* c,
              const double* d) {
  double u[3], v[3], w[3], n[3];
  sub3(b, a, u);
  sub3(c, a, v);
  sub3(d, a, w);
  cross3(u, v, n);
  return dot3(n, w);
}
bool seg_tri_cross(const double* p, const double* q, const double* a,
                   const double* b, const double* c) {
  double sp = orient(a, b, c, p), sq = orient(a, b, c, q);
  if (!((sp > 0 && sq < 0) || (sp < 0 && sq > 0))) return false;
  double o1 = orient(p, q, a, b), o2 = orient(p, q, b, c),
         o3 = orient(p, q, c, a);
  return (o1 > 0 && o2 > 0 && o3 > 0) || (o1 < 0 && o2 < 0 && o3 < 0);
}

}  // namespace

/* ==================================================================== */
/* C API                                                                 */
/* ==================================================================== */
extern "C" {

orc_scene* orc_create(const orc_params* p) {
  if (!p) return nullptr;
  orc_scene* s = new orc_scene();
  s->P = *p;
  return s;
}

void orc_destroy(orc_scene* s) { delete s; }

const char* orc_last_error(const orc_scene* s) {
  return s ? s->err.c_str() : "null scene";
}

int orc_add_body(orc_scene* s, const double* xbar, int32_t nv,
                 const int32_t* tris, int32_t nt, double density,
                 const double* q0, const double* qdot0, int32_t kind) {
  if (!s || s->finalized || !xbar || !tris || nv <= 0 || nt <= 0 || !q0)
    return fail(s, ORC_E_INVALID_ARG, "bad add_body arguments");
  orc_body b;
  std::memset(&b, 0, sizeof(b));
  b.kind = kind;
  b.density = density;
  b.v0 = (int)s->vbody.size();
  b.nv = nv;
  b.t0 = (int)s->tbody.size();
  b.nt = nt;
  b.kappa_b = 1;
  std::memcpy(b.q, q0, 12 * sizeof(double));
  if (qdot0 && kind == 0) std::memcpy(b.qdot, qdot0, 12 * sizeof(double));
  int id = (int)s->B.size();
  for (int v = 0; v < nv; ++v) {
    for (int k = 0; k < 3; ++k) s->xbar.push_back(xbar[3 * v + k]);
    s->vbody.push_back(id);
  }
  for (int t = 0; t < nt; ++t) {
    for (int k = 0; k < 3; ++k) {
      int v = tris[3 * t + k];
      if (v < 0 || v >= nv) return fail(s, ORC_E_MESH, "triangle index");
      s->tri.push_back(b.v0 + v);
    }
    s->tbody.push_back(id);
  }
  /* unique edges (lo, hi) of local ids, sorted lexicographically */
  std::vector<std::pair<int, int>> E;
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      int a = tris[3 * t + k], c = tris[3 * t + (k + 1) % 3];
      E.push_back({std::min(a, c), std::max(a, c)});
    }
  std::sort(E.begin(), E.end());
  E.erase(std::unique(E.begin(), E.end()), E.end());
  b.e0 = (int)s->ebody.size();
  b.ne = (int)E.size();
  for (auto& e : E) {
    s->edge.push_back(b.v0 + e.first);
    s->edge.push_back(b.v0 + e.second);
    s->ebody.push_back(id);
    double d[3];
    sub3(xbar + 3 * e.second, xbar + 3 * e.first, d);
    s->erest2.push_back(dot3(d, d));
  }
  if (kind == 0) {
    /* closed and consistently oriented: every directed edge once, and
     * its reverse once */
    std::vector<std::pair<int, int>> D;
    for (int t = 0; t < nt; ++t)
      for (int k = 0; k < 3; ++k)
        D.push_back({tris[3 * t + k], tris[3 * t + (k + 1) % 3]});
    std::sort(D.begin(), D.end());
    for (size_t i = 0; i < D.size(); ++i) {
      if (i > 0 && D[i] == D[i - 1])
        return fail(s, ORC_E_MESH, "repeated directed edge");
      if (!std::binary_search(D.begin(), D.end(),
                              std::make_pair(D[i].second, D[i].first)))
        return fail(s, ORC_E_MESH, "open or inconsistently oriented mesh");
    }
    std::vector<int> tl(tris, tris + 3 * nt);
    mass_props(xbar, nv, tl.data(), nt, density, b.Mhat, &b.vol);
    if (!(b.vol > 0.0)) return fail(s, ORC_E_MESH, "non-positive volume");
  }
  std::memcpy(b.qt, b.q, sizeof(b.q));
  std::memcpy(b.qtilde, b.q, sizeof(b.q));
  s->B.push_back(b);
  return id;
}

int orc_finalize(orc_scene* s) {
  if (!s || s->finalized) return fail(s, ORC_E_INVALID_ARG, "finalize");
  s->finalized = true;
  std::vector<double> q, x;
  current_q(s, q);
  positions(s, q.data(), x);
  int64_t nc;
  double md;
  orc_penetration(s, x.data(), s->P.dhat, &nc, &md);
  if (nc > 0 || !(md > 0.0))
    return fail(s, ORC_E_INFEASIBLE, "initial state intersects");
  return ORC_OK;
}

int orc_sizes(const orc_scene* s, int64_t* sizes) {
  sizes[0] = (int64_t)s->B.size();
  sizes[1] = (int64_t)s->vbody.size();
  sizes[2] = (int64_t)s->tbody.size();
  sizes[3] = (int64_t)s->ebody.size();
  return ORC_OK;
}

int orc_edges(const orc_scene* s, int32_t* out) {
  for (size_t i = 0; i < s->edge.size(); ++i) out[i] = s->edge[i];
  return ORC_OK;
}

int orc_body_mass(const orc_scene* s, double* Mhat, double* vol) {
  for (size_t b = 0; b < s->B.size(); ++b) {
    std::memcpy(Mhat + 16 * b, s->B[b].Mhat, 16 * sizeof(double));
    vol[b] = s->B[b].vol;
  }
  return ORC_OK;
}

int orc_set_shared(orc_scene* s, const int32_t* ids, int32_t n,
                   const double* z, const double* u, const double* rho,
                   const int32_t* kappa_b) {
  if (!s || n < 0) return fail(s, ORC_E_INVALID_ARG, "set_shared");
  for (auto& b : s->B) {
    b.shared = false;
    b.kappa_b = 1;
  }
  for (int i = 0; i < n; ++i) {
    int id = ids[i];
    if (id < 0 || id >= (int)s->B.size() || s->B[id].kind != 0)
      return fail(s, ORC_E_INVALID_ARG, "shared id");
    orc_body& b = s->B[id];
    for (int k = 0; k < 12; ++k) {
      if (!std::isfinite(z[12 * i + k]) || !std::isfinite(u[12 * i + k]))
        return fail(s, ORC_E_INVALID_ARG, "non-finite z or u");
    }
    if (!(rho[i] >= 0.0) || kappa_b[i] < 1)
      return fail(s, ORC_E_INVALID_ARG, "rho or kappa_b");
    b.shared = true;
    std::memcpy(b.z, z + 12 * i, 12 * sizeof(double));
    std::memcpy(b.u, u + 12 * i, 12 * sizeof(double));
    b.rho = rho[i];
    b.kappa_b = kappa_b[i];
  }
  return ORC_OK;
}

int orc_set_projection(orc_scene* s, int32_t on) {
  s->project = on != 0;
  return ORC_OK;
}

int orc_set_pair_replication(orc_scene* s, int32_t mode) {
  if (mode != 0 && mode != 1) return fail(s, ORC_E_INVALID_ARG, "mode");
  s->pair_mode = mode;
  return ORC_OK;
}

int orc_begin_step(orc_scene* s) {
  const double h = s->P.dt;
  Box all;
  box_empty(all);
  std::vector<double> q, x;
  current_q(s, q);
  positions(s, q.data(), x);
  for (size_t v = 0; v < s->vbody.size(); ++v)
    if (s->B[s->vbody[v]].kind == 0) box_add(all, &x[3 * v]);
  double l2 = 0.0;
  for (int k = 0; k < 3; ++k) l2 += (all.hi[k] - all.lo[k]) * (all.hi[k] - all.lo[k]);
  s->scale = std::sqrt(l2);
  for (auto& b : s->B) {
    std::memcpy(b.qt, b.q, sizeof(b.q));
    if (b.kind != 0) {
      std::memcpy(b.qtilde, b.q, sizeof(b.q));
      continue;
    }
    /* qtilde = q^t + h qdot + h^2 M^-1 f_ext; for gravity M^-1 f_ext only
     * moves the translation by g (first column of Mhat is the force). */
    for (int i = 0; i < 12; ++i) b.qtilde[i] = b.q[i] + h * b.qdot[i];
    for (int i = 0; i < 3; ++i) b.qtilde[i] += h * h * s->P.gravity[i];
  }
  return ORC_OK;
}

int orc_set_step(orc_scene* s, const double* qt, const double* qtilde,
                 double scale) {
  for (size_t b = 0; b < s->B.size(); ++b) {
    std::memcpy(s->B[b].qt, qt + 12 * b, 12 * sizeof(double));
    std::memcpy(s->B[b].qtilde, qtilde + 12 * b, 12 * sizeof(double));
  }
  s->scale = scale;
  return ORC_OK;
}

int orc_local_solve(orc_scene* s, orc_stats* st) {
  orc_stats S;
  std::memset(&S, 0, sizeof(S));
  S.min_alpha = 1.0;
  S.min_dist = INFINITY;
  S.scene_scale = s->scale;
  const double hl = s->P.dt * s->scale;
  std::vector<double> q, dq, x, dx;
  current_q(s, q);
  int status = ORC_E_NOCONV;
  for (int it = 0; it < s->P.max_newton; ++it) {
    System Sys;
    Cands Cs;
    assemble(s, q.data(), Sys, &Cs);
    S.n_cand_pt = (int64_t)Cs.pt.size();
    S.n_cand_ee = (int64_t)Cs.ee.size();
    S.n_cand_pg = (int64_t)Cs.pg.size();
    S.n_active = Sys.n_active;
    S.min_dist = Sys.min_dist;
    int pit = 0;
    int rc = solve(s, Sys, dq, &pit);
    S.pcg_iters_total += pit;
    S.newton_iters = it + 1;
    if (rc != ORC_OK) {
      status = rc;
      break;
    }
    double eps = inf_norm(dq) / hl;
    S.final_eps_N = eps;
    if (eps < s->P.newton_theta) {
      status = ORC_OK;
      break;
    }
    positions(s, q.data(), x);
    size_t V = s->vbody.size();
    dx.assign(3 * V, 0.0);
#pragma omp parallel for schedule(static)
    for (size_t v = 0; v < V; ++v) {
      const double* d = &dq[12 * s->vbody[v]];
      const double* xb = &s->xbar[3 * v];
      for (int i = 0; i < 3; ++i)
        dx[3 * v + i] = d[i] + d[3 + 3 * i] * xb[0] + d[4 + 3 * i] * xb[1] +
                        d[5 + 3 * i] * xb[2];
    }
    Cands Cw;
    candidates(s, x, dx.data(), Cw);
    double alpha = ccd_alpha(s, x, dx, Cw);
    double dE = energy_delta(s, q.data(), dq.data(), alpha, x, Cw);
    int nh = 0;
    while (dE > 0.0 && nh < s->P.max_ls) {
      alpha *= 0.5;
      ++nh;
      dE = energy_delta(s, q.data(), dq.data(), alpha, x, Cw);
    }
    S.ls_halvings += nh;
    if (dE > 0.0) {
      if (eps < 10.0 * s->P.newton_theta) {
        status = ORC_OK;
      } else {
        status = ORC_E_LINESEARCH;
        s->err = "line search exhausted";
      }
      break;
    }
    S.min_alpha = std::min(S.min_alpha, alpha);
    for (size_t i = 0; i < q.size(); ++i) q[i] += alpha * dq[i];
    /* a decrease that only a step halved more than LS_FLOOR_HALVINGS times
     * finds, with eps within 10 theta, is rounding noise of the energy
     * difference: the iterate is converged to the precision the energy
     * resolves */
    if (nh > LS_FLOOR_HALVINGS && eps < 10.0 * s->P.newton_theta) {
      status = ORC_OK;
      break;
    }
  }
  for (size_t b = 0; b < s->B.size(); ++b)
    std::memcpy(s->B[b].q, &q[12 * b], 12 * sizeof(double));
  S.status = status;
  if (status == ORC_E_NOCONV && s->err.empty()) s->err = "Newton did not converge";
  if (st) *st = S;
  return status;
}

int orc_end_step(orc_scene* s) {
  for (auto& b : s->B) {
    if (b.kind != 0) continue;
    for (int i = 0; i < 12; ++i) b.qdot[i] = (b.q[i] - b.qt[i]) / s->P.dt;
  }
  return ORC_OK;
}

int orc_get_state(const orc_scene* s, double* q, double* qdot) {
  for (size_t b = 0; b < s->B.size(); ++b) {
    if (q) std::memcpy(q + 12 * b, s->B[b].q, 12 * sizeof(double));
    if (qdot) std::memcpy(qdot + 12 * b, s->B[b].qdot, 12 * sizeof(double));
  }
  return ORC_OK;
}

int orc_set_state(orc_scene* s, const double* q, const double* qdot) {
  for (size_t b = 0; b < s->B.size(); ++b) {
    if (s->B[b].kind != 0) continue;
    if (q) std::memcpy(s->B[b].q, q + 12 * b, 12 * sizeof(double));
    if (qdot) std::memcpy(s->B[b].qdot, qdot + 12 * b, 12 * sizeof(double));
  }
  return ORC_OK;
}

int orc_get_qtilde(const orc_scene* s, double* qtilde) {
  for (size_t b = 0; b < s->B.size(); ++b)
    std::memcpy(qtilde + 12 * b, s->B[b].qtilde, 12 * sizeof(double));
  return ORC_OK;
}

int orc_vertices(const orc_scene* s, const double* q, double* x) {
  std::vector<double> qq, xx;
  if (q)
    qq.assign(q, q + 12 * s->B.size());
  else
    current_q(s, qq);
  positions(s, qq.data(), xx);
  std::memcpy(x, xx.data(), xx.size() * sizeof(double));
  return ORC_OK;
}

int orc_candidates(orc_scene* s, int32_t kind, const double* x,
                   const double* dx, int32_t* out, int64_t cap,
                   int64_t* count) {
  std::vector<double> xx(x, x + 3 * s->vbody.size());
  Cands C;
  candidates(s, xx, dx, C);
  int64_t n = 0;
  if (kind == ORC_PT || kind == ORC_EE) {
    const auto& L = kind == ORC_PT ? C.pt : C.ee;
    n = (int64_t)L.size();
    if (out && n <= cap)
      for (int64_t i = 0; i < n; ++i) {
        out[2 * i] = L[i].first;
        out[2 * i + 1] = L[i].second;
      }
  } else if (kind == ORC_PG) {
    n = (int64_t)C.pg.size();
    if (out && n <= cap)
      for (int64_t i = 0; i < n; ++i) out[i] = C.pg[i];
  } else {
    return fail(s, ORC_E_INVALID_ARG, "kind");
  }
  *count = n;
  return (out && n > cap) ? ORC_E_CAPACITY : ORC_OK;
}

int orc_eval(orc_scene* s, const double* q, double* E, double* g,
             double* Hdiag, int64_t cap, int64_t* n_off, int32_t* off_ij,
             double* Hoff, int64_t* n_active) {
  System S;
  assemble(s, q, S, nullptr);
  if (E) *E = S.E;
  if (g) std::memcpy(g, S.g.data(), S.g.size() * sizeof(double));
  if (Hdiag) std::memcpy(Hdiag, S.Hd.data(), S.Hd.size() * sizeof(double));
  if (n_active) *n_active = S.n_active;
  int64_t n = (int64_t)S.Ho.size();
  if (n_off) *n_off = n;
  if (off_ij && Hoff && n <= cap) {
    int64_t i = 0;
    for (const auto& kv : S.Ho) {
      off_ij[2 * i] = kv.first.first;
      off_ij[2 * i + 1] = kv.first.second;
      std::memcpy(Hoff + 144 * i, kv.second.data(), 144 * sizeof(double));
      ++i;
    }
  }
  return (off_ij && n > cap) ? ORC_E_CAPACITY : ORC_OK;
}

int orc_direction(orc_scene* s, const double* q, double* dq, int32_t* iters) {
  System S;
  assemble(s, q, S, nullptr);
  std::vector<double> d;
  int it = 0;
  int rc = solve(s, S, d, &it);
  std::memcpy(dq, d.data(), d.size() * sizeof(double));
  if (iters) *iters = it;
  return rc;
}

int orc_ccd(orc_scene* s, const double* q, const double* dq,
            double* alpha_max) {
  std::vector<double> x, dx;
  positions(s, q, x);
  size_t V = s->vbody.size();
  dx.assign(3 * V, 0.0);
#pragma omp parallel for schedule(static)
  for (size_t v = 0; v < V; ++v) {
    const double* d = dq + 12 * s->vbody[v];
    const double* xb = &s->xbar[3 * v];
    for (int i = 0; i < 3; ++i)
      dx[3 * v + i] = d[i] + d[3 + 3 * i] * xb[0] + d[4 + 3 * i] * xb[1] +
                      d[5 + 3 * i] * xb[2];
  }
  Cands C;
  candidates(s, x, dx.data(), C);
  *alpha_max = ccd_alpha(s, x, dx, C);
  return ORC_OK;
}

int orc_energy_delta(orc_scene* s, const double* q, const double* dq,
                     double alpha, double* dE) {
  std::vector<double> x, dx;
  positions(s, q, x);
  size_t V = s->vbody.size();
  dx.assign(3 * V, 0.0);
#pragma omp parallel for schedule(static)
  for (size_t v = 0; v < V; ++v) {
    const double* d = dq + 12 * s->vbody[v];
    const double* xb = &s->xbar[3 * v];
    for (int i = 0; i < 3; ++i)
      dx[3 * v + i] = d[i] + d[3 + 3 * i] * xb[0] + d[4 + 3 * i] * xb[1] +
                      d[5 + 3 * i] * xb[2];
  }
  Cands C;
  candidates(s, x, dx.data(), C);
  *dE = energy_delta(s, q, dq, alpha, x, C);
  return ORC_OK;
}

int orc_penetration(orc_scene* s, const double* x, double pad,
                    int64_t* n_cross, double* min_dist) {
  size_t nb = s->B.size();
  std::vector<Box> bb(nb);
  for (size_t b = 0; b < nb; ++b) {
    box_empty(bb[b]);
    const orc_body& o = s->B[b];
    for (int v = 0; v < o.nv; ++v) box_add(bb[b], x + 3 * (o.v0 + v));
  }
  int64_t nc = 0;
  double md = INFINITY;
  auto prim_box = [&](const int* ids, int n) {
    Box b;
    box_empty(b);
    for (int k = 0; k < n; ++k) box_add(b, x + 3 * ids[k]);
    return b;
  };
  /* a count and a minimum: the same in any order of the body pairs */
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nc) reduction(min : md)
  for (size_t a = 0; a < nb; ++a)
    for (size_t c = a + 1; c < nb; ++c) {
      const orc_body& A = s->B[a];
      const orc_body& C = s->B[c];
      if (A.kind != 0 && C.kind != 0) continue;
      if (!overlap(bb[a], bb[c], pad)) continue;
      for (int dir = 0; dir < 2; ++dir) {
        const orc_body& P = dir ? C : A;
        const orc_body& Q = dir ? A : C;
        const Box& boxP = dir ? bb[c] : bb[a];
        const Box& boxQ = dir ? bb[a] : bb[c];
        for (int e = 0; e < P.ne; ++e) {
          const int* ev = &s->edge[2 * (P.e0 + e)];
          Box be = prim_box(ev, 2);
          if (!overlap(be, boxQ, pad)) continue;
          for (int t = 0; t < Q.nt; ++t) {
            const int* tv = &s->tri[3 * (Q.t0 + t)];
            Box bt = prim_box(tv, 3);
            if (!overlap(be, bt, pad)) continue;
            if (seg_tri_cross(x + 3 * ev[0], x + 3 * ev[1], x + 3 * tv[0],
                              x + 3 * tv[1], x + 3 * tv[2]))
              ++nc;
          }
        }
        for (int v = 0; v < P.nv; ++v) {
          int vid[4] = {P.v0 + v, 0, 0, 0};
          Box bv = prim_box(vid, 1);
          if (!overlap(bv, boxQ, pad)) continue;
          for (int t = 0; t < Q.nt; ++t) {
            const int* tv = &s->tri[3 * (Q.t0 + t)];
            Box bt = prim_box(tv, 3);
            if (!overlap(bv, bt, pad)) continue;
            double x12[12];
            int ids[4] = {P.v0 + v, tv[0], tv[1], tv[2]};
            for (int k = 0; k < 4; ++k)
              for (int i = 0; i < 3; ++i) x12[3 * k + i] = x[3 * ids[k] + i];
            md = std::min(md, pair_distance(ORC_PT, x12));
          }
        }
        (void)boxP;
      }
      for (int e = 0; e < A.ne; ++e) {
        const int* ev = &s->edge[2 * (A.e0 + e)];
        Box be = prim_box(ev, 2);
        if (!overlap(be, bb[c], pad)) continue;
        for (int f = 0; f < C.ne; ++f) {
          const int* fv = &s->edge[2 * (C.e0 + f)];
          Box bf = prim_box(fv, 2);
          if (!overlap(be, bf, pad)) continue;
          double x12[12];
          int ids[4] = {ev[0], ev[1], fv[0], fv[1]};
          for (int k = 0; k < 4; ++k)
            for (int i = 0; i < 3; ++i) x12[3 * k + i] = x[3 * ids[k] + i];
          md = std::min(md, pair_distance(ORC_EE, x12));
        }
      }
    }
  if (s->P.has_ground)
    for (size_t v = 0; v < s->vbody.size(); ++v)
      if (s->B[s->vbody[v]].kind == 0)
        md = std::min(md, x[3 * v + 1] - s->P.ground_y);
  *n_cross = nc;
  *min_dist = md;
  return ORC_OK;
}

void orc_barrier(double d, double dhat, double* out3) {
  barrier(d, dhat, out3, out3 + 1, out3 + 2);
}

int orc_sqdist(int32_t kind, const double* x12, double* D, double* g12,
               double* H144, int32_t* dtype) {
  double Dv;
  Feature f = classify(kind, x12, &Dv);
  Deriv Dd;
  feature_sqd_deriv(kind, x12, f, Dd);
  *D = Dv;
  if (g12) std::memcpy(g12, Dd.g, 12 * sizeof(double));
  if (H144) std::memcpy(H144, Dd.H, 144 * sizeof(double));
  if (dtype) *dtype = f.code;
  return ORC_OK;
}

int orc_pair_eval(int32_t kind, const double* x12, double eps_x, double dhat,
                  double w, int32_t project, double* E, double* g12,
                  double* H144, double* dist, int32_t* dtype) {
  int dt;
  int r = pair_energy(kind, x12, eps_x, dhat, w, true, project != 0, E, g12,
                      H144, dist, &dt);
  if (dtype) *dtype = dt;
  return r;
}

void orc_orth(const double* A9, double* E, double* g9, double* H81,
              int32_t project) {
  orth_energy(A9, E, g9, H81, project != 0);
}

int orc_mass_props(const double* xbar, int32_t nv, const int32_t* tris,
                   int32_t nt, double density, double* Mhat16, double* vol) {
  std::vector<int> tl(tris, tris + 3 * nt);
  mass_props(xbar, nv, tl.data(), nt, density, Mhat16, vol);
  return ORC_OK;
}

void orc_psd(int32_t n, const double* H, double* out) { psd_project(n, H, out); }

void orc_eig(int32_t n, const double* H, double* w, double* V) {
  jacobi_eig(n, H, w, V);
}

double orc_accd(int32_t kind, const double* x12, const double* dx12,
                double s, double tmax) {
  return accd(kind, x12, dx12, s, tmax);
}

double orc_exact_toi(int32_t kind, const double* x12, const double* dx12,
                     double tmax) {
  return exact_toi(kind, x12, dx12, tmax);
}

}  // extern "C"
