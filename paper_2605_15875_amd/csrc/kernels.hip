/*
 * gfx950 kernels of the local Newton solve (Eq. 5).  One kernel family per
 * step of a Newton iteration:
 *   prediction of Eq. 1 and commit      k_predict, k_commit
 *   body terms (inertia, orthogonality,  k_body_terms
 *   ADMM penalty of Eq. 5)
 *   broad phase                          k_boxes, k_body_pairs,
 *                                        k_chunk_pairs, k_prim_pairs, k_pg
 *   barrier (narrow phase + assembly)    k_filter, k_assemble
 *   block-Jacobi PCG                     k_bsr_*, k_block_inverse, k_pcg
 *   Newton stop                          k_dq_norm
 *   CCD step bound                       k_ccd
 *   line search energy                   k_energy, k_reduce
 */
#include "abd_internal.h"

namespace abd {

static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

/* DoF index of coordinate i and affine basis k (k=0: p_i, else A_i,k-1) */
__device__ __forceinline__ int dofi(int i, int k) {
  return k == 0 ? i : 3 + 3 * i + (k - 1);
}
__device__ __forceinline__ void dof_split(int d, int& i, int& k) {
  if (d < 3) { i = d; k = 0; }
  else { i = (d - 3) / 3; k = (d - 3) % 3 + 1; }
}

/* ================================================================== */
/* S1 prediction, S11 commit, transform export                         */
/* ================================================================== */
__global__ void k_predict(Scene S) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S.B * 12) return;
  int b = t / 12, i = t % 12;
  double q = S.q[t];
  S.qt[t] = q;
  if (S.kind[b] != 0) {
    S.qtilde[t] = q;
    return;
  }
  double v = q + S.dt * S.qdot[t];
  /* M^-1 f_ext for gravity moves the translation by h^2 g */
  if (i < 3) v += S.dt * S.dt * S.grav[i];
  S.qtilde[t] = v;
}

__global__ void k_commit(Scene S) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S.B * 12) return;
  if (S.kind[t / 12] != 0) return;
  S.qdot[t] = (S.q[t] - S.qt[t]) / S.dt;
}

__global__ void k_transform(Scene S, double* x, double* dx) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= S.V) return;
  int b = S.vbody[v];
  double b0 = S.xbar[v], b1 = S.xbar[S.V + v], b2 = S.xbar[2 * S.V + v];
  double p[3];
  xform(S.q + 12 * b, b0, b1, b2, p);
  x[3 * v] = p[0]; x[3 * v + 1] = p[1]; x[3 * v + 2] = p[2];
  if (dx) {
    xform(S.dq + 12 * b, b0, b1, b2, p);
    dx[3 * v] = p[0]; dx[3 * v + 1] = p[1]; dx[3 * v + 2] = p[2];
  }
}

/* ordered-integer image of a double, so atomicMin/Max order like doubles */
__device__ __forceinline__ unsigned long long ord(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

/* bounding box of the dynamic vertices (the scene scale l) */
__global__ void k_scale(Scene S, unsigned long long* out6) {
  __shared__ double red[6][256];
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (; v < S.V; v += gridDim.x * blockDim.x) {
    if (S.kind[S.vbody[v]] != 0) continue;
    double x[3];
    vertex_pos(S, v, x);
    for (int k = 0; k < 3; ++k) {
      lo[k] = fmin(lo[k], x[k]);
      hi[k] = fmax(hi[k], x[k]);
    }
  }
  for (int k = 0; k < 3; ++k) {
    red[k][threadIdx.x] = lo[k];
    red[3 + k][threadIdx.x] = hi[k];
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + s]);
        red[3 + k][threadIdx.x] =
            fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) {
      atomicMin(out6 + k, ord(red[k][0]));
      atomicMax(out6 + 3 + k, ord(red[3 + k][0]));
    }
}

/* ================================================================== */
/* S3 + S6: body terms                                                 */
/* ================================================================== */
/* Per dynamic body: inertia 1/2 (q - qt)^T M (q - qt), orthogonality
 * h^2 kappa_A V |A A^T - I|^2 (Hessian projected to PSD), both weighted by
 * 1/kappa_b, and the ADMM penalty rho/2 |q - z + u|^2 of a shared body.
 * Writes g [B][12] and Hdiag [B][144] (static bodies: 0 and identity). */
__global__ __launch_bounds__(64) void k_body_terms(Scene S) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= S.B) return;
  double* Hd = S.Hdiag + 144 * b;
  double* g = S.g + 12 * b;
  if (S.kind[b] != 0) {
    for (int i = 0; i < 144; ++i) Hd[i] = (i % 13 == 0) ? 1.0 : 0.0;
    for (int i = 0; i < 12; ++i) g[i] = 0.0;
    return;
  }
  double q[12], dq[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    q[i] = S.q[12 * b + i];
    dq[i] = q[i] - S.qtilde[12 * b + i];
  }
  double M[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) M[i] = S.Mhat[16 * b + i];
  const double wb = S.wbody[b];
  const double c = wb * S.dt * S.dt * S.kappa_A * S.vol[b];
  const double* A = q + 3;
  double Sm[9], AtA[9];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      double s = 0.0, t = 0.0;
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        s += A[3 * k + n] * A[3 * m + n];
        t += A[3 * n + k] * A[3 * n + m];
      }
      Sm[3 * k + m] = s - (k == m ? 1.0 : 0.0);
      AtA[3 * k + m] = t;
    }
  /* orthogonality Hessian 4[d_kp (A^T A)_ql + A_kq A_pl + S_kp d_lq] */
  double K[45];
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int e = a; e < 9; ++e) {
      const int k = a / 3, l = a % 3, p = e / 3, qq = e % 3;
      double h = A[3 * k + qq] * A[3 * p + l];
      if (k == p) h += AtA[3 * qq + l];
      if (l == qq) h += Sm[3 * k + p];
      K[sidx(a, e)] = 4.0 * h;
    }
  psd9_reg(K);
  /* gradient */
  double gl[12];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < 4; ++l) v += M[4 * k + l] * dq[dofi(i, l)];
      gl[dofi(i, k)] = wb * v;
    }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) v += Sm[3 * k + m] * A[3 * m + l];
      gl[3 + 3 * k + l] += c * 4.0 * v;
    }
  const int sh = S.shared_slot[b];
  const double rho = sh >= 0 ? S.rho[sh] : 0.0;
  if (sh >= 0)
#pragma unroll
    for (int i = 0; i < 12; ++i)
      gl[i] += rho * (q[i] - S.z[12 * sh + i] + S.u[12 * sh + i]);
#pragma unroll
  for (int i = 0; i < 12; ++i) g[i] = gl[i];
  /* Hessian */
#pragma unroll
  for (int r = 0; r < 12; ++r)
#pragma unroll
    for (int cc = 0; cc < 12; ++cc) {
      const int i = r < 3 ? r : (r - 3) / 3, k = r < 3 ? 0 : (r - 3) % 3 + 1;
      const int j = cc < 3 ? cc : (cc - 3) / 3, l = cc < 3 ? 0 : (cc - 3) % 3 + 1;
      double h = (i == j) ? wb * M[4 * k + l] : 0.0;
      if (r >= 3 && cc >= 3) h += c * K[sidx(r - 3, cc - 3)];
      if (r == cc) h += rho;
      Hd[12 * r + cc] = h;
    }
}

/* ================================================================== */
/* S4 broad phase                                                      */
/* ================================================================== */
/* world boxes of every chunk and body (static: at q; swept: over the
 * step q -> q + dq) */
__global__ void k_boxes(Scene S, int swept) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  int b;
  const double* rest;
  double* out;
  if (t < S.NC) {
    b = S.ch_body[t];
    rest = S.ch_rest + 6 * t;
    out = S.ch_box + 6 * t;
  } else if (t < S.NC + S.B) {
    b = t - S.NC;
    rest = S.body_rest + 6 * b;
    out = S.body_box + 6 * b;
  } else {
    return;
  }
  double ce[6];
  for (int i = 0; i < 6; ++i) ce[i] = rest[i];
  const double* qb = S.q + 12 * b;
  double box[6];
  if (!swept || S.kind[b] != 0) {
    world_box(qb, ce, 0.0, box);
  } else {
    const double* db = S.dq + 12 * b;
    double q1[12];
    for (int i = 0; i < 12; ++i) q1[i] = qb[i] + db[i];
    double m0 = map_mag(qb, ce), m1 = map_mag(db, ce);
    double b0[6], b1[6];
    world_box(qb, ce, m1, b0);
    world_box(q1, ce, m0 + m1, b1);
    for (int k = 0; k < 3; ++k) {
      box[k] = fmin(b0[k], b1[k]);
      box[3 + k] = fmax(b0[3 + k], b1[3 + k]);
    }
  }
  for (int i = 0; i < 6; ++i) out[i] = box[i];
}

/* body pairs (a < b, not both static) whose boxes pass the predicate */
__global__ void k_body_pairs(Scene S) {
  int a = blockIdx.y * 16 + threadIdx.y;
  int b = blockIdx.x * 16 + threadIdx.x;
  if ((int)(blockIdx.x * 16 + 15) <= (int)(blockIdx.y * 16)) return;
  if (a >= S.B || b >= S.B || a >= b) return;
  if (S.kind[a] != 0 && S.kind[b] != 0) return;
  if (!box_overlap(S.body_box + 6 * a, S.body_box + 6 * b, S.dhat)) return;
  int k = atomicAdd(&S.cnt->n_bp, 1);
  if (k < S.cap_bp) S.bp[k] = make_int2(a, b);
}

/* chunk pairs of every body pair: vertex chunks x triangle chunks (both
 * directions) and edge chunks x edge chunks */
__global__ __launch_bounds__(256) void k_chunk_pairs(Scene S) {
  int nbp = min(S.cnt->n_bp, S.cap_bp);
  for (int p = blockIdx.x; p < nbp; p += gridDim.x) {
    int2 ab = S.bp[p];
    const int* ca = S.body_chunk + 6 * ab.x;
    const int* cb = S.body_chunk + 6 * ab.y;
    int nva = ca[1] - ca[0], nta = ca[3] - ca[2], nea = ca[5] - ca[4];
    int nvb = cb[1] - cb[0], ntb = cb[3] - cb[2], neb = cb[5] - cb[4];
    int n1 = nva * ntb, n2 = nvb * nta, n3 = nea * neb;
    int tot = n1 + n2 + n3;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
      int kind, P, Q;
      if (t < n1) {
        kind = C_PT; P = ca[0] + t / ntb; Q = cb[2] + t % ntb;
      } else if (t < n1 + n2) {
        int u = t - n1;
        kind = C_PT; P = cb[0] + u / nta; Q = ca[2] + u % nta;
      } else {
        int u = t - n1 - n2;
        kind = C_EE; P = ca[4] + u / neb; Q = cb[4] + u % neb;
      }
      if (!box_overlap(S.ch_box + 6 * P, S.ch_box + 6 * Q, S.dhat)) continue;
      int k = atomicAdd(&S.cnt->n_cp, 1);
      if (k < S.cap_cp) S.cp[k] = make_int4(kind, P, Q, p);
    }
  }
}

/* exact box of one primitive (static, or swept over the step) */
__device__ __forceinline__ void vert_box(const Scene& S, int v, int swept,
                                         double* box) {
  double x[3], x1[3];
  if (swept) {
    vertex_pos_swept(S, v, x, x1);
    for (int k = 0; k < 3; ++k) {
      box[k] = fmin(x[k], x1[k]);
      box[3 + k] = fmax(x[k], x1[k]);
    }
  } else {
    vertex_pos(S, v, x);
    for (int k = 0; k < 3; ++k) box[k] = box[3 + k] = x[k];
  }
}
__device__ __forceinline__ void prim_box(const Scene& S, int kind, int id,
                                         int swept, double* box) {
  if (kind == K_VERT) {
    vert_box(S, id, swept, box);
    return;
  }
  int n = kind == K_TRI ? 3 : 2;
  const int* ids = kind == K_TRI ? S.tri : S.edge;
  int stride = kind == K_TRI ? S.T : S.E;
  vert_box(S, ids[id], swept, box);
  for (int j = 1; j < n; ++j) {
    double b2[6];
    vert_box(S, ids[j * stride + id], swept, b2);
    for (int k = 0; k < 3; ++k) {
      box[k] = fmin(box[k], b2[k]);
      box[3 + k] = fmax(box[3 + k], b2[3 + k]);
    }
  }
}

/* primitive pairs of every chunk pair, one wavefront per chunk pair: the
 * second chunk's exact boxes are staged in LDS, each lane tests its own
 * primitive of the first chunk against all of them */
__global__ __launch_bounds__(256) void k_prim_pairs(Scene S, int swept) {
  __shared__ double qbox[4][ABD_CHUNK][6];
  __shared__ int qid[4][ABD_CHUNK];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int ncp = min(S.cnt->n_cp, S.cap_cp);
  for (int base = blockIdx.x * 4; base < ncp; base += gridDim.x * 4) {
    int c = base + wave;
    bool valid = c < ncp;
    int4 cp = valid ? S.cp[c] : make_int4(0, 0, 0, 0);
    int P = cp.y, Q = cp.z;
    int kindP = cp.x == C_PT ? K_VERT : K_EDGE;
    int kindQ = cp.x == C_PT ? K_TRI : K_EDGE;
    int nP = valid ? S.ch_count[P] : 0;
    int nQ = valid ? S.ch_count[Q] : 0;
    if (lane < nQ) {
      int id = S.ch_prims[S.ch_start[Q] + lane];
      qid[wave][lane] = id;
      prim_box(S, kindQ, id, swept, qbox[wave][lane]);
    }
    __syncthreads();
    if (lane < nP) {
      int id = S.ch_prims[S.ch_start[P] + lane];
      double box[6];
      prim_box(S, kindP, id, swept, box);
      for (int j = 0; j < nQ; ++j) {
        if (!box_overlap(box, qbox[wave][j], S.dhat)) continue;
        int other = qid[wave][j];
        if (cp.x == C_PT) {
          int k = atomicAdd(&S.cnt->n_pt, 1);
          if (k < S.cap_pt) {
            S.cand_pt[3 * k] = id;
            S.cand_pt[3 * k + 1] = other;
            S.cand_pt[3 * k + 2] = cp.w;
          }
        } else {
          int k = atomicAdd(&S.cnt->n_ee, 1);
          if (k < S.cap_ee) {
            S.cand_ee[3 * k] = min(id, other);
            S.cand_ee[3 * k + 1] = max(id, other);
            S.cand_ee[3 * k + 2] = cp.w;
          }
        }
      }
    }
    __syncthreads();
  }
}

/* vertex-ground candidates: vertex chunks of dynamic bodies whose box
 * reaches the ground band, then each vertex exactly */
__global__ void k_pg(Scene S, int swept) {
  const double top = __dadd_rn(S.ground_y, S.dhat);
  const int lane = threadIdx.x % 64;
  const int nw = gridDim.x * (blockDim.x / 64);
  for (int c = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; c < S.NC;
       c += nw) {
    if (S.ch_kind[c] != K_VERT || S.kind[S.ch_body[c]] != 0) continue;
    if (!(S.ch_box[6 * c + 1] <= top)) continue;
    if (lane >= S.ch_count[c]) continue;
    int v = S.ch_prims[S.ch_start[c] + lane];
    double box[6];
    vert_box(S, v, swept, box);
    if (box[1] <= top) {
      int k = atomicAdd(&S.cnt->n_pg, 1);
      if (k < S.cap_pg) S.cand_pg[k] = v;
    }
  }
}

/* ================================================================== */
/* S5 barrier: narrow phase filter and assembly                        */
/* ================================================================== */
__device__ __forceinline__ void pair_vertices(const Scene& S, int kind, int i,
                                              int j, int* vid) {
  if (kind == C_PT) {
    vid[0] = i;
    vid[1] = S.tri[j];
    vid[2] = S.tri[S.T + j];
    vid[3] = S.tri[2 * S.T + j];
  } else {
    vid[0] = S.edge[i];
    vid[1] = S.edge[S.E + i];
    vid[2] = S.edge[j];
    vid[3] = S.edge[S.E + j];
  }
}

__device__ __forceinline__ double pair_weight(const Scene& S, const int* vid,
                                              int n) {
  double w = S.dt * S.dt * S.kappa;
  if (S.pair_mode == 0) return w;
  for (int k = 0; k < n; ++k) {
    int b = S.vbody[vid[k]];
    if (S.kind[b] == 0 && S.shared_slot[b] < 0) return w;
  }
  return 0.5 * w;
}

__global__ void k_filter(Scene S) {
  const int npt = min(S.cnt->n_pt, S.cap_pt);
  const int nee = min(S.cnt->n_ee, S.cap_ee);
  const int npg = min(S.cnt->n_pg, S.cap_pg);
  const int tot = npt + nee + npg;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < tot;
       t += gridDim.x * blockDim.x) {
    int kind, i, j = 0, slot = -1;
    double d;
    if (t < npt + nee) {
      const int* c = t < npt ? S.cand_pt + 3 * t : S.cand_ee + 3 * (t - npt);
      kind = t < npt ? C_PT : C_EE;
      i = c[0]; j = c[1]; slot = c[2];
      int vid[4];
      pair_vertices(S, kind, i, j, vid);
      double x[12];
      for (int k = 0; k < 4; ++k) vertex_pos(S, vid[k], x + 3 * k);
      d = pair_dist(kind, x);
    } else {
      kind = C_PG;
      i = S.cand_pg[t - npt - nee];
      double x[3];
      vertex_pos(S, i, x);
      d = x[1] - S.ground_y;
    }
    atomic_min_pos(&S.cnt->min_dist, fmax(d, 0.0));
    if (d < S.dhat) {
      int k = atomicAdd(&S.cnt->n_act, 1);
      if (k < S.cap_act) S.act[k] = make_int4(kind, i, j, slot);
    }
  }
}

/* ---- derivatives of the squared-distance features ---- */
/* K(u,v) = |u x v|^2: gradient [6] and Hessian [6][6] */
__device__ inline void d_cross(const double* u, const double* v, double& f,
                               double* G, double* H) {
  double uu = dot3(u, u), vv = dot3(v, v), uv = dot3(u, v);
  double n[3];
  cross3(u, v, n);
  f = dot3(n, n);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    G[i] = 2.0 * (vv * u[i] - uv * v[i]);
    G[3 + i] = 2.0 * (uu * v[i] - uv * u[i]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double dij = i == j ? 1.0 : 0.0;
      H[i * 6 + j] = 2.0 * (vv * dij - v[i] * v[j]);
      H[(3 + i) * 6 + 3 + j] = 2.0 * (uu * dij - u[i] * u[j]);
      double x = 4.0 * u[i] * v[j] - 2.0 * v[i] * u[j] - 2.0 * uv * dij;
      H[i * 6 + 3 + j] = x;
      H[(3 + j) * 6 + i] = x;
    }
}

/* F = S / N on n variables, S, N with gradients and Hessians (stride n) */
template <int n>
__device__ inline void d_quot(double Sv, const double* Sg, const double* Sh,
                              double Nv, const double* Ng, const double* Nh,
                              double& F, double* G, double* H) {
  double iN = 1.0 / Nv;
  double q = Sv * iN;
  F = q;
#pragma unroll
  for (int i = 0; i < n; ++i) G[i] = (Sg[i] - q * Ng[i]) * iN;
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < n; ++j)
      H[i * n + j] = (Sh[i * n + j] - q * Nh[i * n + j] -
                      (Sg[i] * Ng[j] + Ng[i] * Sg[j]) * iN +
                      2.0 * q * Ng[i] * Ng[j] * iN) * iN;
}

/* point-edge: F = |a x e|^2 / |e|^2 over (a, e) */
__device__ inline void d_pe(const double* a, const double* e, double& F,
                            double* G, double* H) {
  double Kv, Kg[6], Kh[36];
  d_cross(a, e, Kv, Kg, Kh);
  double Ng[6] = {0, 0, 0, 2.0 * e[0], 2.0 * e[1], 2.0 * e[2]};
  double Nh[36];
#pragma unroll
  for (int i = 0; i < 36; ++i) Nh[i] = 0.0;
  Nh[3 * 6 + 3] = Nh[4 * 6 + 4] = Nh[5 * 6 + 5] = 2.0;
  d_quot<6>(Kv, Kg, Kh, dot3(e, e), Ng, Nh, F, G, H);
}

/* point-plane / line-line: F = (a . (b x c))^2 / |b x c|^2 over (a, b, c) */
__device__ inline void d_tri(const double* a, const double* b,
                             const double* c, double& F, double* G,
                             double* H) {
  double bc[3], ca[3], ab[3];
  cross3(b, c, bc);
  cross3(c, a, ca);
  cross3(a, b, ab);
  double s = dot3(a, bc);
  double gs[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gs[i] = bc[i]; gs[3 + i] = ca[i]; gs[6 + i] = ab[i];
  }
  /* S = s^2 with Hessian 2 gs gs^T + 2 s Hs; Hs blocks (a,b) = -[c]x,
   * (a,c) = [b]x, (b,c) = -[a]x (and transposes) */
  double Sh[81];
#pragma unroll
  for (int i = 0; i < 9; ++i)
#pragma unroll
    for (int j = 0; j < 9; ++j) Sh[i * 9 + j] = 2.0 * gs[i] * gs[j];
  const double* vs[3] = {a, b, c};
#pragma unroll
  for (int P = 0; P < 3; ++P)
#pragma unroll
    for (int Q = 0; Q < 3; ++Q) {
      if (P == Q) continue;
      int R = 3 - P - Q;           /* the third vector */
      double sg = ((Q - P + 3) % 3 == 1) ? -1.0 : 1.0; /* (a,b),(b,c),(c,a): - */
      const double* w = vs[R];
      /* entry (i,k) of sg*[w]x */
      double sk[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          Sh[(3 * P + i) * 9 + 3 * Q + k] += 2.0 * s * sg * sk[i * 3 + k];
    }
  double Sg[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Sg[i] = 2.0 * s * gs[i];
  double Kv, Kg[6], Kh[36];
  d_cross(b, c, Kv, Kg, Kh);
  double Ng[9], Nh[81];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    Ng[i] = i < 3 ? 0.0 : Kg[i - 3];
#pragma unroll
    for (int j = 0; j < 9; ++j)
      Nh[i * 9 + j] = (i < 3 || j < 3) ? 0.0 : Kh[(i - 3) * 6 + (j - 3)];
  }
  d_quot<9>(s * s, Sg, Sh, Kv, Ng, Nh, F, G, H);
}

/* Map derivatives over k feature vectors (frame coefficients C[k][3]) into
 * the y frame: g_y (9) and the packed 9x9 Hessian K (45). */
template <int k>
__device__ __forceinline__ void to_frame(const double (*C)[3], const double* G,
                                         const double* H, double* gy,
                                         double* K) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < k; ++j) v += C[j][r] * G[3 * j + i];
      gy[3 * r + i] = v;
    }
#pragma unroll
  for (int p = 0; p < 9; ++p)
#pragma unroll
    for (int q = p; q < 9; ++q) {
      const int r = p / 3, i = p % 3, u = q / 3, i2 = q % 3;
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < k; ++j)
#pragma unroll
        for (int l = 0; l < k; ++l)
          v += C[j][r] * C[l][u] * H[(3 * j + i) * (3 * k) + 3 * l + i2];
      K[sidx(p, q)] = v;
    }
}

/* Barrier gradient g_y and PSD-projected Hessian K (packed, reduced frame)
 * of one PT/EE pair with slot positions x; also returns the distance. */
__device__ __forceinline__ void pair_frame_derivs(const Scene& S, int kind, int ei,
                                               int ej, const double* x,
                                               double w, double* gy,
                                               double* K) {
  double D;
  Feat f = classify(kind, x, D);
  const double d = sqrt(D);
  double b, b1, b2;
  barrier3(d, S.dhat, b, b1, b2);
  double gD[9];
  if (f.type == F_PP) {
    double C[1][3], r[3], G[3], H[9];
    frame_coef(kind, f.l[0], C[0]);
    comb4(f.l[0], x, r);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      G[i] = 2.0 * r[i];
#pragma unroll
      for (int j = 0; j < 3; ++j) H[i * 3 + j] = i == j ? 2.0 : 0.0;
    }
    to_frame<1>(C, G, H, gD, K);
  } else if (f.type == F_PE) {
    double C[2][3], av[3], ev[3], F, G[6], H[36];
    frame_coef(kind, f.l[0], C[0]);
    frame_coef(kind, f.l[1], C[1]);
    comb4(f.l[0], x, av);
    comb4(f.l[1], x, ev);
    d_pe(av, ev, F, G, H);
    to_frame<2>(C, G, H, gD, K);
  } else {
    double C[3][3], av[3], bv[3], cv[3], F, G[9], H[81];
#pragma unroll
    for (int j = 0; j < 3; ++j) frame_coef(kind, f.l[j], C[j]);
    comb4(f.l[0], x, av);
    comb4(f.l[1], x, bv);
    comb4(f.l[2], x, cv);
    d_tri(av, bv, cv, F, G, H);
    to_frame<3>(C, G, H, gD, K);
  }
  /* mollifier m(c) on c = |u x v|^2 (u = y_1, v = y_2 of the EE frame) */
  double m = 1.0, m1 = 0.0, m2 = 0.0, gc[9], Hc[36];
  bool moll = false;
#pragma unroll
  for (int i = 0; i < 9; ++i) gc[i] = 0.0;
  if (kind == C_EE && S.mollify) {
    const double ex = MOLL_EPS * S.erest2[ei] * S.erest2[ej];
    double u[3], v[3], cval, G6[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u[i] = x[3 + i] - x[i];
      v[i] = x[9 + i] - x[6 + i];
    }
    d_cross(u, v, cval, G6, Hc);
    if (cval < ex) {
      moll = true;
      const double rr = cval / ex;
      m = (2.0 - rr) * rr;
      m1 = 2.0 * (1.0 - rr) / ex;
      m2 = -2.0 / (ex * ex);
#pragma unroll
      for (int i = 0; i < 6; ++i) gc[3 + i] = G6[i];
    }
  }
  const double i2d = 0.5 / d, i4d3 = 0.25 / (d * d * d);
  double gd[9], Gs[9];
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    gd[p] = gD[p] * i2d;
    Gs[p] = sqrt(frame_norm2(kind, p / 3));
    gy[p] = w * (m * b1 * gd[p] + (moll ? b * m1 * gc[p] : 0.0));
  }
#pragma unroll
  for (int p = 0; p < 9; ++p)
#pragma unroll
    for (int q = p; q < 9; ++q) {
      const double hd = K[sidx(p, q)] * i2d - gD[p] * gD[q] * i4d3;
      double h = m * (b2 * gd[p] * gd[q] + b1 * hd);
      if (moll) {
        const double hc = (p >= 3 && q >= 3) ? Hc[(p - 3) * 6 + (q - 3)] : 0.0;
        h += b1 * m1 * (gc[p] * gd[q] + gd[p] * gc[q]) +
             b * (m2 * gc[p] * gc[q] + m1 * hc);
      }
      K[sidx(p, q)] = w * h * Gs[p] * Gs[q];
    }
  psd9_reg(K);
#pragma unroll
  for (int p = 0; p < 9; ++p)
#pragma unroll
    for (int q = p; q < 9; ++q) K[sidx(p, q)] /= Gs[p] * Gs[q];
}

/* One wavefront of 64 active pairs.  Phase 1 (a lane per pair): distance
 * feature, barrier gradient and Hessian in the reduced frame with its PSD
 * projection, and the frame-to-body maps W.  Phase 2 (all lanes per pair):
 * T = H_y W_Y, then the body-space gradient and 12x12 blocks W_X^T T,
 * accumulated with FP64 atomics into g, Hdiag and Hoff. */
__global__ __launch_bounds__(64) void k_assemble(Scene S) {
  __shared__ double KL[45 * 64];
  __shared__ double GW[33 * 64]; /* rows 0..8 g_y, 9..20 W_A, 21..32 W_B */
  __shared__ double TB[216];
  __shared__ int meta[3 * 64];
  const int lane = threadIdx.x;
  const int nact = min(S.cnt->n_act, S.cap_act);
  for (int base = blockIdx.x * 64; base < nact; base += gridDim.x * 64) {
    const int t = base + lane;
    int ba = -1, bb = -1, slot = -1;
    if (t < nact) {
      const int4 a = S.act[t];
      const int kind = a.x;
      slot = a.w;
      double gy[9], K[45], Wa[12], Wb[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) Wa[i] = Wb[i] = 0.0;
      if (kind == C_PG) {
        const int v = a.y;
        double x[3];
        vertex_pos(S, v, x);
        double b, b1, b2;
        barrier3(x[1] - S.ground_y, S.dhat, b, b1, b2);
        const double w = pair_weight(S, &v, 1);
#pragma unroll
        for (int i = 0; i < 9; ++i) gy[i] = 0.0;
#pragma unroll
        for (int i = 0; i < 45; ++i) K[i] = 0.0;
        gy[1] = w * b1;
        K[sidx(1, 1)] = w * b2;
        ba = S.vbody[v];
        Wa[0] = 1.0;
        Wa[1] = S.xbar[v]; Wa[2] = S.xbar[S.V + v]; Wa[3] = S.xbar[2 * S.V + v];
      } else {
        int vid[4];
        pair_vertices(S, kind, a.y, a.z, vid);
        double x[12];
#pragma unroll
        for (int s = 0; s < 4; ++s) vertex_pos(S, vid[s], x + 3 * s);
        const double w = pair_weight(S, vid, 4);
        pair_frame_derivs(S, kind, a.y, a.z, x, w, gy, K);
        /* W_side[r][k] = sum over the side's slots s of f_r[s] xhat_s[k] */
        const int sideB0 = kind == C_PT ? 1 : 2;
        ba = S.vbody[vid[0]];
        bb = S.vbody[vid[sideB0]];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double xh[4] = {1.0, S.xbar[vid[s]], S.xbar[S.V + vid[s]],
                                S.xbar[2 * S.V + vid[s]]};
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const double fr = frame_row(kind, r, s);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              if (s < sideB0) Wa[4 * r + k] += fr * xh[k];
              else Wb[4 * r + k] += fr * xh[k];
            }
          }
        }
      }
      if (ba >= 0 && S.kind[ba] != 0) ba = -1;
      if (bb >= 0 && S.kind[bb] != 0) bb = -1;
#pragma unroll
      for (int i = 0; i < 45; ++i) KL[i * 64 + lane] = K[i];
#pragma unroll
      for (int i = 0; i < 9; ++i) GW[i * 64 + lane] = gy[i];
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        GW[(9 + i) * 64 + lane] = Wa[i];
        GW[(21 + i) * 64 + lane] = Wb[i];
      }
    }
    meta[lane] = ba;
    meta[64 + lane] = bb;
    meta[128 + lane] = slot;
    __syncthreads();
    const int npairs = min(64, nact - base);
    for (int j = 0; j < npairs; ++j) {
      const int A = meta[j], Bq = meta[64 + j], sl = meta[128 + j];
      if (A < 0 && Bq < 0) continue;
      /* T_Y[(r,i)][(i2,l)] = sum_u H[(r,i),(u,i2)] W_Y[u][l] */
      for (int e = lane; e < 216; e += 64) {
        const int Y = e / 108, f = e % 108, ri = f / 12, i2 = (f % 12) / 4,
                  l = f % 4;
        const int wo = Y ? 21 : 9;
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < 3; ++u)
          v += KL[sidx(ri, 3 * u + i2) * 64 + j] * GW[(wo + 4 * u + l) * 64 + j];
        TB[e] = v;
      }
      /* gradient */
      if (lane < 24) {
        const int side = lane / 12, dd = lane % 12;
        const int body = side ? Bq : A;
        if (body >= 0) {
          int i, k;
          dof_split(dd, i, k);
          const int wo = side ? 21 : 9;
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < 3; ++r)
            v += GW[(wo + 4 * r + k) * 64 + j] * GW[(3 * r + i) * 64 + j];
          atomicAdd(S.g + 12 * body + dd, v);
        }
      }
      __syncthreads();
      /* blocks: (A,A), (B,B), (lo,hi) = W_X^T T_Y */
      for (int blk = 0; blk < 3; ++blk) {
        int X, Y;
        double* dst;
        if (blk == 0) {
          if (A < 0) continue;
          X = 0; Y = 0; dst = S.Hdiag + 144 * A;
        } else if (blk == 1) {
          if (Bq < 0) continue;
          X = 1; Y = 1; dst = S.Hdiag + 144 * Bq;
        } else {
          if (A < 0 || Bq < 0) continue;
          if (A < Bq) { X = 0; Y = 1; } else { X = 1; Y = 0; }
          dst = S.Hoff + 144 * (size_t)sl;
          if (lane == 0) S.slot_used[sl] = 1;
        }
        const int wx = X ? 21 : 9;
        for (int e = lane; e < 144; e += 64) {
          int i, k, i2, l;
          dof_split(e / 12, i, k);
          dof_split(e % 12, i2, l);
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < 3; ++r)
            v += GW[(wx + 4 * r + k) * 64 + j] *
                 TB[Y * 108 + (3 * r + i) * 12 + i2 * 4 + l];
          atomicAdd(dst + e, v);
        }
      }
      __syncthreads();
    }
    __syncthreads();
  }
}

/* ================================================================== */
/* S7 block-Jacobi PCG                                                 */
/* ================================================================== */
/* block rows of the off-diagonal blocks that received contributions:
 * row a lists (slot, b, plain), row b lists (slot, a, transposed) */
__global__ void k_bsr_count(Scene S) {
  int nbp = min(S.cnt->n_bp, S.cap_bp);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nbp;
       p += gridDim.x * blockDim.x) {
    if (!S.slot_used[p]) continue;
    int2 ab = S.bp[p];
    atomicAdd(S.row_cnt + ab.x, 1);
    atomicAdd(S.row_cnt + ab.y, 1);
  }
}
__global__ void k_bsr_scan(Scene S) {
  /* single block exclusive scan of row_cnt into row_ptr */
  __shared__ int part[1024];
  const int n = S.B;
  const int per = (n + blockDim.x - 1) / blockDim.x;
  int lo = threadIdx.x * per, hi = min(n, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += S.row_cnt[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int i = 0; i < (int)blockDim.x; ++i) {
      int v = part[i];
      part[i] = acc;
      acc += v;
    }
    S.row_ptr[n] = acc;
    S.cnt->n_rows_used = acc;
  }
  __syncthreads();
  int acc = part[threadIdx.x];
  for (int i = lo; i < hi; ++i) {
    S.row_ptr[i] = acc;
    acc += S.row_cnt[i];
    S.row_cnt[i] = 0; /* reused as fill cursor */
  }
}
__global__ void k_bsr_fill(Scene S) {
  int nbp = min(S.cnt->n_bp, S.cap_bp);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nbp;
       p += gridDim.x * blockDim.x) {
    if (!S.slot_used[p]) continue;
    int2 ab = S.bp[p];
    int k = S.row_ptr[ab.x] + atomicAdd(S.row_cnt + ab.x, 1);
    if (k < S.cap_col) {
      S.col_slot[k] = p; S.col_body[k] = ab.y; S.col_trans[k] = 0;
    }
    k = S.row_ptr[ab.y] + atomicAdd(S.row_cnt + ab.y, 1);
    if (k < S.cap_col) {
      S.col_slot[k] = p; S.col_body[k] = ab.x; S.col_trans[k] = 1;
    }
  }
}

/* inverse of every diagonal block by Gauss-Jordan (SPD, no pivoting):
 * 16 bodies per block of 192 threads, one row per thread */
__global__ __launch_bounds__(192) void k_block_inverse(Scene S) {
  __shared__ double M[16][12][25];
  const int lb = threadIdx.x / 12, r = threadIdx.x % 12;
  const int b = blockIdx.x * 16 + lb;
  const bool act = b < S.B;
  for (int c = 0; c < 12; ++c) {
    M[lb][r][c] = act ? S.Hdiag[144 * b + 12 * r + c] : (r == c ? 1.0 : 0.0);
    M[lb][r][12 + c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < 12; ++k) {
    double piv = M[lb][k][k];
    double f = M[lb][r][k] / piv;
    double rowk[24];
    for (int c = 0; c < 24; ++c) rowk[c] = M[lb][k][c];
    __syncthreads();
    if (r != k)
      for (int c = 0; c < 24; ++c) M[lb][r][c] -= f * rowk[c];
    else
      for (int c = 0; c < 24; ++c) M[lb][r][c] = rowk[c] / piv;
    __syncthreads();
  }
  if (act)
    for (int c = 0; c < 12; ++c) S.Pinv[144 * b + 12 * r + c] = M[lb][r][12 + c];
}

/* grid-wide barrier for the cooperative PCG launch; the spin is bounded so
 * that every wave exits even if a barrier were never completed */
__device__ __forceinline__ void grid_sync(unsigned* bar, unsigned nblocks,
                                          unsigned& gen, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    gen += 1;
    __threadfence();
    atomicAdd(bar, 1u);
    unsigned target = gen * nblocks;
    long spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE,
                             __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > (1L << 26)) {
        atomicOr(err, 1);
        break;
      }
    }
    __threadfence();
  }
  __syncthreads();
}

__device__ __forceinline__ double block_sum192(double v, double* red) {
  /* sum over a 192-thread block (3 waves) */
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0] + red[1] + red[2];
  __syncthreads();
  return s;
}

/* Block-Jacobi preconditioned CG on H dq = -g with zero initial guess,
 * all iterations in one cooperative launch.  Each block owns 16 bodies
 * (192 rows) per pass of a grid-stride loop.  Per iteration: phase A
 * forms p_k = z_k + beta_k p_{k-1} on the fly and the product A p_k; phase
 * B updates dq, r and z = P^-1 r; two grid barriers.  Dots are reduced in
 * FP64 with atomics into a ring of 4 accumulator slots:
 * acc[4*j + 0] = r_j . z_j, + 1 = p_j . A p_j, + 2 = r_j . r_j. */
__global__ __launch_bounds__(192) void k_pcg(Scene S, double eta, int max_it) {
  __shared__ double rloc[16][12];
  __shared__ double red[4];
  const unsigned nblk = gridDim.x;
  unsigned gen = 0;
  const int lb = threadIdx.x / 12, row = threadIdx.x % 12;
  const int ngroups = (S.B + 15) / 16;
  double* acc = S.acc;
  /* init: x = 0, r = b = -g, z = P^-1 r, p_{-1} = 0 */
  double prz = 0.0, pbb = 0.0;
  for (int gr = blockIdx.x; gr < ngroups; gr += nblk) {
    int b = gr * 16 + lb;
    bool act = b < S.B;
    double rv = act ? -S.g[12 * b + row] : 0.0;
    if (act) {
      S.dq[12 * b + row] = 0.0;
      S.r[12 * b + row] = rv;
      S.p0[12 * b + row] = 0.0;
      S.p1[12 * b + row] = 0.0;
    }
    rloc[lb][row] = rv;
    __syncthreads();
    double z = 0.0;
    if (act)
      for (int c = 0; c < 12; ++c) z += S.Pinv[144 * b + 12 * row + c] * rloc[lb][c];
    if (act) S.zv[12 * b + row] = z;
    prz += rv * z;
    pbb += rv * rv;
    __syncthreads();
  }
  double srz = block_sum192(prz, red), sbb = block_sum192(pbb, red);
  if (threadIdx.x == 0) {
    atomicAdd(acc + 0, srz);
    atomicAdd(&S.cnt->pcg_bb, sbb);
  }
  grid_sync(&S.cnt->bar, nblk, gen, &S.cnt->err);
  const double bb = S.cnt->pcg_bb;
  int it = 0;
  if (bb > 0.0) {
    const double tol2 = eta * eta * bb;
    for (it = 0; it < max_it; ++it) {
      double* pold = (it & 1) ? S.p0 : S.p1;
      double* pnew = (it & 1) ? S.p1 : S.p0;
      const double rz = acc[4 * (it & 3) + 0];
      const double beta = it == 0 ? 0.0 : rz / acc[4 * ((it - 1) & 3) + 0];
      /* phase A: p = z + beta pold, Ap */
      double ppap = 0.0;
      for (int gr = blockIdx.x; gr < ngroups; gr += nblk) {
        int b = gr * 16 + lb;
        if (b < S.B) {
          double y = 0.0;
          const double* H = S.Hdiag + 144 * b + 12 * row;
          for (int c = 0; c < 12; ++c)
            y += H[c] * (S.zv[12 * b + c] + beta * pold[12 * b + c]);
          for (int e = S.row_ptr[b]; e < S.row_ptr[b + 1]; ++e) {
            int nb = S.col_body[e];
            const double* blk = S.Hoff + 144 * (size_t)S.col_slot[e];
            if (S.col_trans[e]) {
              for (int c = 0; c < 12; ++c)
                y += blk[12 * c + row] * (S.zv[12 * nb + c] + beta * pold[12 * nb + c]);
            } else {
              for (int c = 0; c < 12; ++c)
                y += blk[12 * row + c] * (S.zv[12 * nb + c] + beta * pold[12 * nb + c]);
            }
          }
          double pk = S.zv[12 * b + row] + beta * pold[12 * b + row];
          pnew[12 * b + row] = pk;
          S.Ap[12 * b + row] = y;
          ppap += pk * y;
        }
      }
      double s = block_sum192(ppap, red);
      if (threadIdx.x == 0) atomicAdd(acc + 4 * (it & 3) + 1, s);
      grid_sync(&S.cnt->bar, nblk, gen, &S.cnt->err);
      /* phase B */
      const double alpha = rz / acc[4 * (it & 3) + 1];
      double prz2 = 0.0, prr = 0.0;
      if (blockIdx.x == 0 && threadIdx.x < 4) acc[4 * ((it + 2) & 3) + threadIdx.x] = 0.0;
      for (int gr = blockIdx.x; gr < ngroups; gr += nblk) {
        int b = gr * 16 + lb;
        bool act = b < S.B;
        double rv = 0.0;
        if (act) {
          int o = 12 * b + row;
          S.dq[o] += alpha * pnew[o];
          rv = S.r[o] - alpha * S.Ap[o];
          S.r[o] = rv;
        }
        rloc[lb][row] = rv;
        __syncthreads();
        double z = 0.0;
        if (act) {
          for (int c = 0; c < 12; ++c) z += S.Pinv[144 * b + 12 * row + c] * rloc[lb][c];
          S.zv[12 * b + row] = z;
        }
        prz2 += rv * z;
        prr += rv * rv;
        __syncthreads();
      }
      double s1 = block_sum192(prz2, red), s2 = block_sum192(prr, red);
      if (threadIdx.x == 0) {
        atomicAdd(acc + 4 * ((it + 1) & 3) + 0, s1);
        atomicAdd(acc + 4 * ((it + 1) & 3) + 2, s2);
      }
      grid_sync(&S.cnt->bar, nblk, gen, &S.cnt->err);
      double rr = acc[4 * ((it + 1) & 3) + 2];
      if (S.cnt->err) { ++it; break; }
      if (rr <= tol2) { ++it; break; }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S.cnt->pcg_iters = it;
    S.cnt->pcg_rr = acc[4 * (it & 3) + 2];
  }
}

/* ================================================================== */
/* S8 Newton stop                                                      */
/* ================================================================== */
__global__ void k_dq_norm(Scene S) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  double v = t < 12 * S.B ? fabs(S.dq[t]) : 0.0;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  if ((threadIdx.x & 63) == 0) atomic_max_pos(&S.cnt->max_dq, v);
}

/* ================================================================== */
/* S9 CCD                                                              */
/* ================================================================== */
__global__ void k_ccd(Scene S) {
  const int npt = min(S.cnt->n_pt, S.cap_pt);
  const int nee = min(S.cnt->n_ee, S.cap_ee);
  const int npg = min(S.cnt->n_pg, S.cap_pg);
  const int tot = npt + nee + npg;
  double tmin = 1.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < tot;
       t += gridDim.x * blockDim.x) {
    if (t < npt + nee) {
      const int* c = t < npt ? S.cand_pt + 3 * t : S.cand_ee + 3 * (t - npt);
      int kind = t < npt ? C_PT : C_EE;
      int vid[4];
      pair_vertices(S, kind, c[0], c[1], vid);
      double x[12], dx[12];
      for (int k = 0; k < 4; ++k) {
        int v = vid[k], b = S.vbody[v];
        double b0 = S.xbar[v], b1 = S.xbar[S.V + v], b2 = S.xbar[2 * S.V + v];
        xform(S.q + 12 * b, b0, b1, b2, x + 3 * k);
        xform(S.dq + 12 * b, b0, b1, b2, dx + 3 * k);
      }
      tmin = fmin(tmin, accd(kind, x, dx, 1.0));
    } else {
      int v = S.cand_pg[t - npt - nee], b = S.vbody[v];
      double b0 = S.xbar[v], b1 = S.xbar[S.V + v], b2 = S.xbar[2 * S.V + v];
      double x[3], dx[3];
      xform(S.q + 12 * b, b0, b1, b2, x);
      xform(S.dq + 12 * b, b0, b1, b2, dx);
      if (dx[1] < 0.0)
        tmin = fmin(tmin, (1.0 - ACCD_S) * (x[1] - S.ground_y) / (-dx[1]));
    }
  }
  for (int o = 32; o > 0; o >>= 1) tmin = fmin(tmin, __shfl_down(tmin, o, 64));
  if ((threadIdx.x & 63) == 0) atomic_min_pos(&S.cnt->min_toi, fmax(tmin, 0.0));
}

/* ================================================================== */
/* S10 line search energy                                              */
/* ================================================================== */
/* mode 0: E(q + alpha dq) - E(q) term by term; mode 1: E(q).
 * Elements: bodies, then PT, EE, PG candidates of the current list.  Each
 * block writes one partial sum (fixed grid, so the result is
 * deterministic). */
__device__ double body_energy(const Scene& S, int b, double alpha, int mode) {
  if (S.kind[b] != 0) return 0.0;
  double q[12], st[12];
  for (int i = 0; i < 12; ++i) {
    q[i] = S.q[12 * b + i];
    st[i] = mode ? 0.0 : alpha * S.dq[12 * b + i];
  }
  const double* M = S.Mhat + 16 * b;
  const double wb = S.wbody[b];
  double e = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 4; ++k) {
      double v = 0.0;
      for (int l = 0; l < 4; ++l) {
        int dl = dofi(i, l);
        double dd = q[dl] - S.qtilde[12 * b + dl];
        v += M[4 * k + l] * (mode ? 0.5 * dd : dd + 0.5 * st[dl]);
      }
      int dk = dofi(i, k);
      e += wb * (mode ? q[dk] - S.qtilde[12 * b + dk] : st[dk]) * v;
    }
  const double* A = q + 3;
  const double* D = st + 3;
  double acc = 0.0;
  for (int k = 0; k < 3; ++k)
    for (int m = 0; m < 3; ++m) {
      double s = 0.0, ds = 0.0;
      for (int n = 0; n < 3; ++n) {
        s += A[3 * k + n] * A[3 * m + n];
        ds += A[3 * k + n] * D[3 * m + n] + D[3 * k + n] * A[3 * m + n] +
              D[3 * k + n] * D[3 * m + n];
      }
      if (k == m) s -= 1.0;
      acc += mode ? s * s : ds * (2.0 * s + ds);
    }
  e += wb * S.dt * S.dt * S.kappa_A * S.vol[b] * acc;
  int sh = S.shared_slot[b];
  if (sh >= 0) {
    double rho = S.rho[sh];
    for (int i = 0; i < 12; ++i) {
      double r = q[i] - S.z[12 * sh + i] + S.u[12 * sh + i];
      e += mode ? 0.5 * rho * r * r : rho * st[i] * (r + 0.5 * st[i]);
    }
  }
  return e;
}

__device__ double pair_energy_at(const Scene& S, int kind, int i, int j,
                                 const int* vid, const double* x) {
  double w = pair_weight(S, vid, 4);
  double D;
  classify(kind, x, D);
  double b = barrier_val(sqrt(D), S.dhat);
  if (b == 0.0) return 0.0;
  double m = 1.0;
  if (kind == C_EE && S.mollify) {
    double ex = MOLL_EPS * S.erest2[i] * S.erest2[j];
    double u[3], v[3], n[3];
    for (int k = 0; k < 3; ++k) {
      u[k] = x[3 + k] - x[k];
      v[k] = x[9 + k] - x[6 + k];
    }
    cross3(u, v, n);
    double c = dot3(n, n);
    if (c < ex) {
      double rr = c / ex;
      m = (2.0 - rr) * rr;
    }
  }
  return w * m * b;
}

__global__ __launch_bounds__(256) void k_energy(Scene S, double alpha,
                                                int mode, int with_pairs,
                                                int alpha_from_toi) {
  __shared__ double red[4];
  if (alpha_from_toi) {
    const double toi = __longlong_as_double(
        (long long)__hip_atomic_load(&S.cnt->min_toi, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT));
    alpha *= fmin(1.0, toi);
  }
  const int npt = with_pairs ? min(S.cnt->n_pt, S.cap_pt) : 0;
  const int nee = with_pairs ? min(S.cnt->n_ee, S.cap_ee) : 0;
  const int npg = with_pairs ? min(S.cnt->n_pg, S.cap_pg) : 0;
  const int tot = S.B + npt + nee + npg;
  double e = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < tot;
       t += gridDim.x * blockDim.x) {
    if (t < S.B) {
      e += body_energy(S, t, alpha, mode);
      continue;
    }
    int u = t - S.B;
    if (u < npt + nee) {
      const int* c = u < npt ? S.cand_pt + 3 * u : S.cand_ee + 3 * (u - npt);
      int kind = u < npt ? C_PT : C_EE;
      int vid[4];
      pair_vertices(S, kind, c[0], c[1], vid);
      double x0[12], x1[12];
      for (int k = 0; k < 4; ++k) {
        vertex_pos(S, vid[k], x0 + 3 * k);
        if (!mode) vertex_pos_alpha(S, vid[k], alpha, x1 + 3 * k);
      }
      double E0 = pair_energy_at(S, kind, c[0], c[1], vid, x0);
      e += mode ? E0 : pair_energy_at(S, kind, c[0], c[1], vid, x1) - E0;
    } else {
      int v = S.cand_pg[u - npt - nee];
      double x0[3], x1[3];
      vertex_pos(S, v, x0);
      double w = pair_weight(S, &v, 1);
      double E0 = w * barrier_val(x0[1] - S.ground_y, S.dhat);
      if (mode) {
        e += E0;
      } else {
        vertex_pos_alpha(S, v, alpha, x1);
        e += w * barrier_val(x1[1] - S.ground_y, S.dhat) - E0;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) e += __shfl_down(e, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0)
    S.partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_reduce(Scene S, int n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += S.partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_update_q(Scene S, double alpha) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 12 * S.B) return;
  if (S.kind[t / 12] != 0) return;
  S.q[t] += alpha * S.dq[t];
}

/* ================================================================== */
/* host launchers                                                      */
/* ================================================================== */
static const int GRID_STRIDE_BLOCKS = 1024;
static const int ENERGY_BLOCKS = 512;

void launch_predict(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_predict, dim3(cdiv(12L * S.B, 256)), dim3(256), 0, st, S);
}
void launch_commit(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_commit, dim3(cdiv(12L * S.B, 256)), dim3(256), 0, st, S);
}
void launch_transform(const Scene& S, double* x, double* dx, hipStream_t st) {
  hipLaunchKernelGGL(k_transform, dim3(cdiv(S.V, 256)), dim3(256), 0, st, S, x, dx);
}
void launch_scale(const Scene& S, double* out6, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(min(1024u, cdiv(S.V, 256))), dim3(256), 0,
                     st, S, (unsigned long long*)out6);
}
void launch_body_terms(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_body_terms, dim3(cdiv(S.B, 64)), dim3(64), 0, st, S);
}
void launch_boxes(const Scene& S, int swept, hipStream_t st) {
  hipLaunchKernelGGL(k_boxes, dim3(cdiv(S.NC + S.B, 256)), dim3(256), 0, st, S, swept);
}
void launch_body_pairs(const Scene& S, hipStream_t st) {
  unsigned g = cdiv(S.B, 16);
  hipLaunchKernelGGL(k_body_pairs, dim3(g, g), dim3(16, 16), 0, st, S);
}
void launch_chunk_pairs(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_pairs, dim3(GRID_STRIDE_BLOCKS), dim3(256), 0, st, S);
}
void launch_prim_pairs(const Scene& S, int swept, hipStream_t st) {
  hipLaunchKernelGGL(k_prim_pairs, dim3(GRID_STRIDE_BLOCKS), dim3(256), 0, st, S, swept);
}
void launch_pg(const Scene& S, int swept, hipStream_t st) {
  hipLaunchKernelGGL(k_pg, dim3(min(1024u, cdiv(S.NC, 4))), dim3(256), 0, st, S, swept);
}
void launch_filter(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_filter, dim3(GRID_STRIDE_BLOCKS), dim3(256), 0, st, S);
}
void launch_assemble(const Scene& S, int n_act_hint, hipStream_t st) {
  unsigned g = n_act_hint > 0 ? min(4096u, cdiv(n_act_hint, 64)) : 512u;
  hipLaunchKernelGGL(k_assemble, dim3(g), dim3(64), 0, st, S);
}
void launch_bsr(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_bsr_count, dim3(256), dim3(256), 0, st, S);
  hipLaunchKernelGGL(k_bsr_scan, dim3(1), dim3(1024), 0, st, S);
  hipLaunchKernelGGL(k_bsr_fill, dim3(256), dim3(256), 0, st, S);
}
void launch_block_inverse(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_block_inverse, dim3(cdiv(S.B, 16)), dim3(192), 0, st, S);
}
int pcg_max_grid() {
  int dev = 0, ncu = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_pcg, 192, 0);
  return ncu * (per > 0 ? per : 1);
}
int launch_pcg(const Scene& S, double eta, int max_it, int grid, hipStream_t st) {
  void* args[] = {(void*)&S, (void*)&eta, (void*)&max_it};
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_pcg, dim3(grid),
                                            dim3(192), args, 0, st);
  return e == hipSuccess ? 0 : -1;
}
void launch_dq_norm(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_dq_norm, dim3(cdiv(12L * S.B, 256)), dim3(256), 0, st, S);
}
void launch_ccd(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_ccd, dim3(GRID_STRIDE_BLOCKS), dim3(256), 0, st, S);
}
void launch_energy(const Scene& S, double alpha, int mode_with_pairs,
                   int alpha_from_toi, double* out, hipStream_t st) {
  int mode = mode_with_pairs & 1, with_pairs = (mode_with_pairs >> 1) & 1;
  hipLaunchKernelGGL(k_energy, dim3(ENERGY_BLOCKS), dim3(256), 0, st, S, alpha,
                     mode, with_pairs, alpha_from_toi);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, st, S, ENERGY_BLOCKS, out);
}
void launch_update_q(const Scene& S, double alpha, hipStream_t st) {
  hipLaunchKernelGGL(k_update_q, dim3(cdiv(12L * S.B, 256)), dim3(256), 0, st, S, alpha);
}

}  // namespace abd
