/*
 * gfx950 kernels of the local Newton solve (Eq. 5).  One kernel family per
 * step of a Newton iteration:
 *   prediction of Eq. 1 and commit      k_predict, k_commit
 *   body terms (inertia, orthogonality,  k_body_terms
 *   ADMM penalty of Eq. 5)
 *   broad phase                          k_boxes (chunk and body boxes),
 *                                        k_body_pairs or k_sap_sort and
 *                                        k_sap_sweep (body pairs),
 *                                        k_chunk_pairs, k_prim_pairs, k_pg
 *   barrier (narrow phase + assembly)    k_filter, k_assemble
 *   linear solve by components           k_bsr_* (block rows, component
 *                                        labels), k_block_inverse, k_direct,
 *                                        block-Jacobi PCG k_pcg_cg1
 *                                        (k_pcg_local, k_pcg, k_pcg1)
 *   Newton stop                          k_boxes (swept, stop-test
 *                                        workgroups), k_dq_norm
 *   CCD step bound                       k_ccd, k_ccd_long (blocked steps)
 *   line search energy                   k_energy_multi, k_energy, k_reduce
 *   device loop                          k_ctrl_start, k_update_multi
 */
#include <algorithm>
#include <cstddef>

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
/* start of a pass of the device loop: fresh counter blocks (the static one
 * taking over the previous pass's swept lists when they are complete),
 * per-problem transients, the block-row counts and the PCG records */
__device__ __forceinline__ void pass_reset(const Scene& S, const Counters& fresh,
                                           int expect_reuse, int t, int nth) {
  if (t == 0) {
    /* The previous pass's swept lists cover every position q + alpha dq,
     * alpha in [0, 1], of the bodies it swept: every static candidate of
     * the accepted (or unchanged) state is among them, so they serve as
     * this pass's static lists. */
    const Counters c1 = S.cnt[1];
    Counters c0 = fresh;
    if (c1.sweep_ok) {
      c0.n_bp = c1.n_bp;
      c0.n_cp = c1.n_cp;
      c0.n_pt = c1.n_pt;
      c0.n_ee = c1.n_ee;
      c0.n_pg = c1.n_pg;
      c0.reuse = 1;
    } else if (expect_reuse) {
      c0.redo = 1;
    }
    S.cnt[0] = c0;
    S.cnt[1] = fresh;
  }
  for (int q = t; q < S.NP; q += nth) {
    ProbState& P = S.ps[q];
    P.max_dq = 0;
    P.min_toi = fresh.min_toi;
    P.alpha_acc = 0.0;
    P.bb = 0.0;
    P.pcg_iters = 0;
    for (int k = 0; k < LS_TRIALS; ++k) P.dE[k] = 0.0;
    for (int k = 0; k < 16; ++k) P.acc[k] = 0.0;
    if (S.det)
      for (int k = 0; k < LS_TRIALS * (DET_W + 1); ++k)
        S.det_de[(size_t)q * LS_TRIALS * (DET_W + 1) + k] = 0ull;
  }
  for (int i = t; i <= S.B; i += nth) S.row_cnt[i] = 0;
  for (int i = t; i < 2 * ((S.B + 15) / 16); i += nth)
    S.pcg_rec[i].gen = 0ull;
}

/* Per dynamic body: inertia 1/2 (q - qt)^T M (q - qt), orthogonality
 * h^2 kappa_A V |A A^T - I|^2 (Hessian projected to PSD), both weighted by
 * 1/kappa_b, and the ADMM penalty rho/2 |q - z + u|^2 of a shared body.
 * Writes g [B][12] and Hdiag [B][144] (static bodies: 0 and identity). */
template <typename HT>
__global__ __launch_bounds__(64) void k_body_terms(Scene S, Counters fresh, int reset_mode) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  /* reset_mode (first launch of a device-loop pass): 1 the pass reset,
   * 2 the same for a pass that expects to take its lists over */
  if (reset_mode) pass_reset(S, fresh, reset_mode == 2, b, gridDim.x * 64);
  if (b >= S.B) return;
  if (!body_in_pass(S, b)) return;
  HT* Hd = (HT*)S.Hdiag + 144 * b;
  double* g = S.g + 12 * b;
  if (S.kind[b] != 0) {
    for (int i = 0; i < 144; ++i) Hd[i] = (i % 13 == 0) ? HT(1) : HT(0);
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
  double Sm[9];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      double s = 0.0;
#pragma unroll
      for (int n = 0; n < 3; ++n) s += A[3 * k + n] * A[3 * m + n];
      Sm[3 * k + m] = s - (k == m ? 1.0 : 0.0);
    }
  /* projected orthogonality Hessian, in closed form from the singular
   * values of A (equal to clamping the eigenvalues of the 9x9 Hessian
   * 4[d_kp (A^T A)_ql + A_kq A_pl + S_kp d_lq]) */
  double K[45];
  orth_hessian_psd(A, K);
  HT Kt[45];
#pragma unroll
  for (int i = 0; i < 45; ++i) Kt[i] = (HT)K[i];
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
      if (r >= 3 && cc >= 3) h += c * (double)Kt[sidx(r - 3, cc - 3)];
      if (r == cc) h += rho;
      Hd[12 * r + cc] = (HT)h;
    }
}

/* ================================================================== */
/* S4 broad phase                                                      */
/* ================================================================== */
/* world boxes of every chunk and body (static: at q; swept: over the
 * step q -> q + dq) */
__device__ __forceinline__ void chunk_or_body_box(const Scene& S, int swept, int t) {
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

/* Slot in an append-only list for each lane whose pred holds: one atomic
 * per wavefront on the list counter, lanes in lane order after it.  Every
 * lane of the wavefront must make the call. */
__device__ __forceinline__ int wave_slot(bool pred, int* counter) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return -1;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(m));
  base = __shfl(base, leader, 64);
  return pred ? base + __popcll(m & ((1ull << lane) - 1ull)) : -1;
}

/* ---- body pairs (a < b, not both static) whose boxes pass the predicate ----
 * Scenes whose problems hold few bodies test every pair of each problem:
 * one workgroup per 16 x 16 tile of a problem's body range (tiles on or
 * above the diagonal, from a fixed list). */
__global__ void k_body_pairs(Scene S) {
  if (S.cnt->reuse) return;
  const int2 tl = S.bp_tiles[blockIdx.x];
  const int a = tl.x * 16 + threadIdx.y;
  const int b = tl.y * 16 + threadIdx.x;
  bool ok = a < S.B && b < S.B && a < b;
  ok = ok && !(S.kind[a] != 0 && S.kind[b] != 0);
  ok = ok && S.bprob[a] == S.bprob[b]; /* independent problems */
  ok = ok && body_in_pass(S, a);
  ok = ok && box_overlap(S.body_box + 6 * a, S.body_box + 6 * b, S.dhat);
  const int k = wave_slot(ok, &S.cnt->n_bp);
  if (ok && k < S.cap_bp) S.bp[k] = make_int2(a, b);
}

/* Larger problems: sort and sweep per problem.
 * The dynamic bodies of a problem are bucketed by the lower bound of their
 * box along the axis on which these lower bounds spread the most (one
 * bucket per body, at most SAP_MAX_BUCKETS): a counting sort in one
 * workgroup per problem.  Each dynamic body then tests the bodies whose
 * bucket lies between the buckets of its own lower bound and of its upper
 * bound plus d-hat (one contiguous run of the sorted array), keeping those
 * after it in (lower bound, index) order, and every static body of its
 * problem.  Any overlapping pair of dynamic bodies lies in the run of the
 * one first in that order (the bucket map is monotone), so each pair is
 * found exactly once, with the box predicate of every other stage. */
__device__ __forceinline__ int wave_prefix(int n, int* total);
__device__ __forceinline__ int sap_bucket(const SapAxis& a, double x) {
  /* explicit roundings: both kernels evaluate the same monotone map */
  const double t = __dmul_rn(__dsub_rn(x, a.lo), a.scale);
  if (!(t >= 1.0)) return 0; /* also NaN */
  if (!(t < (double)a.nb)) return a.nb - 1;
  return (int)t;
}

__global__ __launch_bounds__(1024) void k_sap_sort(Scene S) {
  __shared__ int cnt[SAP_MAX_BUCKETS + 1];
  __shared__ double red[16][6];
  __shared__ int wsum[16];
  __shared__ SapAxis s_ax;
  if (S.cnt->reuse) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  for (int p = blockIdx.x; p < S.NP; p += gridDim.x) {
    const int d0 = S.sap_doff[p], nd = S.sap_doff[p + 1] - d0;
    if (nd == 0 || !body_in_pass(S, S.sap_dyn[d0])) continue;
    /* range of the lower bounds on each axis */
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      const double* bx = S.body_box + 6 * S.sap_dyn[d0 + i];
      for (int k = 0; k < 3; ++k) {
        v[k] = fmin(v[k], bx[k]);
        v[3 + k] = fmax(v[3 + k], bx[k]);
      }
    }
    for (int o = 32; o > 0; o >>= 1)
      for (int k = 0; k < 3; ++k) {
        v[k] = fmin(v[k], __shfl_xor(v[k], o, 64));
        v[3 + k] = fmax(v[3 + k], __shfl_xor(v[3 + k], o, 64));
      }
    if (lane == 0)
      for (int k = 0; k < 6; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < nw; ++w)
        for (int k = 0; k < 3; ++k) {
          v[k] = fmin(v[k], red[w][k]);
          v[3 + k] = fmax(v[3 + k], red[w][3 + k]);
        }
      int ax = 0;
      for (int k = 1; k < 3; ++k)
        if (v[3 + k] - v[k] > v[3 + ax] - v[ax]) ax = k;
      SapAxis a;
      a.axis = ax;
      a.lo = v[ax];
      a.nb = S.sap_boff[p + 1] - S.sap_boff[p] - 1;
      const double w = v[3 + ax] - v[ax];
      double sc = w > 0.0 ? (double)a.nb / w : 0.0;
      if (!(sc < 1e300)) sc = 0.0;
      a.scale = sc;
      s_ax = a;
      S.sap_par[p] = a;
    }
    __syncthreads();
    const SapAxis a = s_ax;
    for (int k = threadIdx.x; k <= a.nb; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      const double* bx = S.body_box + 6 * S.sap_dyn[d0 + i];
      atomicAdd(&cnt[sap_bucket(a, bx[a.axis])], 1);
    }
    __syncthreads();
    /* exclusive scan of the counts: a run of buckets per thread */
    const int per = (a.nb + blockDim.x - 1) / blockDim.x;
    const int lo = threadIdx.x * per, hi = min(a.nb, lo + per);
    int sum = 0;
    for (int k = lo; k < hi; ++k) sum += cnt[k];
    int tot;
    const int ex = wave_prefix(sum, &tot);
    if (lane == 0) wsum[wave] = tot;
    __syncthreads();
    int acc = ex;
    for (int w = 0; w < wave; ++w) acc += wsum[w];
    const int bo = S.sap_boff[p];
    for (int k = lo; k < hi; ++k) {
      const int c = cnt[k];
      cnt[k] = acc;
      S.sap_bstart[bo + k] = d0 + acc;
      acc += c;
    }
    if (threadIdx.x == 0) S.sap_bstart[bo + a.nb] = d0 + nd;
    __syncthreads();
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
      const int b = S.sap_dyn[d0 + i];
      const double* bx = S.body_box + 6 * b;
      const int pos = d0 + atomicAdd(&cnt[sap_bucket(a, bx[a.axis])], 1);
      S.sap_sorted[pos] = b;
      for (int k = 0; k < 6; ++k) S.sap_sbox[6L * pos + k] = bx[k];
    }
    __syncthreads(); /* cnt, red and s_ax serve the next problem */
  }
}

/* SAP_PER_WAVE sorted dynamic bodies per wavefront, in its first lanes;
 * all 64 lanes share out the tests of their runs, 64 at a time (a long
 * run, such as that of a body spanning the scene, is spread over the
 * lanes).  The boxes are read in sorted order (sap_sbox). */
#define SAP_PER_WAVE 4 /* a power of two, at most 64 */
__global__ __launch_bounds__(256) void k_sap_sweep(Scene S) {
  if (S.cnt->reuse) return;
  const int D = S.n_dyn;
  const int lane = __lane_id();
  const int waves = gridDim.x * (blockDim.x >> 6);
  for (int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
       w * SAP_PER_WAVE < D; w += waves) {
    const int t = w * SAP_PER_WAVE + lane;
    int a = 0, start = 0, ndyn = 0, nst = 0, s0 = 0, axis = 0;
    if (lane < SAP_PER_WAVE && t < D) {
      a = S.sap_sorted[t];
      if (body_in_pass(S, a)) {
        const int p = S.bprob[a];
        const SapAxis ax = S.sap_par[p];
        const double* ba = S.sap_sbox + 6L * t;
        const int k0 = sap_bucket(ax, ba[ax.axis]);
        const int k1 = sap_bucket(ax, __dadd_rn(ba[3 + ax.axis], S.dhat));
        const int bo = S.sap_boff[p];
        start = S.sap_bstart[bo + k0];
        ndyn = S.sap_bstart[bo + k1 + 1] - start;
        s0 = S.sap_soff[p];
        nst = S.sap_soff[p + 1] - s0;
        axis = ax.axis;
      }
    }
    int total;
    const int excl = wave_prefix(ndyn + nst, &total);
    for (int f0 = 0; f0 < total; f0 += 64) {
      const int f = f0 + lane;
      /* the lane whose share holds test f: the last with excl <= f */
      int o = 0;
      for (int st = SAP_PER_WAVE / 2; st > 0; st >>= 1)
        if (__shfl(excl, o + st, 64) <= f) o += st;
      const int u = f - __shfl(excl, o, 64);
      const int ao = __shfl(a, o, 64), so = __shfl(start, o, 64);
      const int ndo = __shfl(ndyn, o, 64), sso = __shfl(s0, o, 64);
      const int axo = __shfl(axis, o, 64), to = w * SAP_PER_WAVE + o;
      bool ok = false;
      int bj = 0;
      if (f < total) {
        const double* pa = S.sap_sbox + 6L * to;
        if (u < ndo) {
          bj = S.sap_sorted[so + u];
          const double* pb = S.sap_sbox + 6L * (so + u);
          const double xa = pa[axo], xb = pb[axo];
          ok = bj != ao && (xb > xa || (xb == xa && bj > ao)) &&
               box_overlap(pa, pb, S.dhat);
        } else {
          bj = S.sap_stat[sso + u - ndo];
          ok = box_overlap(pa, S.body_box + 6 * bj, S.dhat);
        }
      }
      const int k = wave_slot(ok, &S.cnt->n_bp);
      if (ok && k < S.cap_bp) S.bp[k] = make_int2(min(ao, bj), max(ao, bj));
    }
  }
}

/* chunk pairs of every body pair: vertex chunks x triangle chunks (both
 * directions) and edge chunks x edge chunks */
/* Block barrier for LDS traffic only: waits for the wavefront's own LDS
 * operations, not for its global stores (a full __syncthreads also waits
 * for every outstanding global store of the wavefront to be acknowledged).
 * Global data written before it is not ordered for the other wavefronts. */
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

/* LDS written and then read by the lanes of one wavefront */
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

/* exclusive prefix of n over the wavefront, and the wavefront's total */
__device__ __forceinline__ int wave_prefix(int n, int* total) {
  const int lane = __lane_id();
  int incl = n;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  *total = __shfl(incl, 63, 64);
  return incl - n;
}

__device__ __forceinline__ void chunk_pair_of(const int* ca, const int* cb, int n1,
                                              int n2, int ntb, int nta, int neb,
                                              int t, int& kind, int& P, int& Q) {
  if (t < n1) {
    kind = C_PT; P = ca[0] + t / ntb; Q = cb[2] + t % ntb;
  } else if (t < n1 + n2) {
    const int u = t - n1;
    kind = C_PT; P = cb[0] + u / nta; Q = ca[2] + u % nta;
  } else {
    const int u = t - n1 - n2;
    kind = C_EE; P = ca[4] + u / neb; Q = cb[4] + u % neb;
  }
}

/* chunk pairs of one body pair per workgroup pass: every test once, hits
 * staged in LDS (one global atomic per body pair), more than CP_STAGE
 * hits of one body pair appended one by one */
#define CP_STAGE 1024
__global__ __launch_bounds__(256) void k_chunk_pairs(Scene S) {
  __shared__ int4 hits[CP_STAGE];
  __shared__ int s_n, s_base;
  if (S.cnt->reuse) return;
  const int nbp = min(S.cnt->n_bp, S.cap_bp);
  for (int p = blockIdx.x; p < nbp; p += gridDim.x) {
    const int2 ab = S.bp[p];
    const int* ca = S.body_chunk + 6 * ab.x;
    const int* cb = S.body_chunk + 6 * ab.y;
    const int nva = ca[1] - ca[0], nta = ca[3] - ca[2], nea = ca[5] - ca[4];
    const int nvb = cb[1] - cb[0], ntb = cb[3] - cb[2], neb = cb[5] - cb[4];
    const int n1 = nva * ntb, n2 = nvb * nta, n3 = nea * neb;
    const int tot = n1 + n2 + n3;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
      int kind, P, Q;
      chunk_pair_of(ca, cb, n1, n2, ntb, nta, neb, t, kind, P, Q);
      if (!box_overlap(S.ch_box + 6 * P, S.ch_box + 6 * Q, S.dhat)) continue;
      const int k = atomicAdd(&s_n, 1);
      if (k < CP_STAGE) {
        hits[k] = make_int4(kind, P, Q, p);
      } else {
        const int g = atomicAdd(&S.cnt->n_cp, 1);
        if (g < S.cap_cp) S.cp[g] = make_int4(kind, P, Q, p);
      }
    }
    __syncthreads();
    const int n = min(s_n, CP_STAGE);
    if (threadIdx.x == 0) s_base = n > 0 ? atomicAdd(&S.cnt->n_cp, n) : 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int g = s_base + i;
      if (g < S.cap_cp) S.cp[g] = hits[i];
    }
    __syncthreads(); /* hits and s_n are reused by the next body pair */
  }
}

/* First kernel of a broad phase: the chunk and body boxes of the phase
 * (conservative images of the rest boxes under the bodies' maps, one
 * thread each).  The primitive tests transform their vertices themselves
 * (vert_box).  With stop_test, the workgroups from nmain on run the Newton
 * stop test of the device loop (|dq|_inf per problem, then the controller
 * in the last of them).  reset_mode as for the body terms; swept < 0: the
 * reset only. */
__device__ void newton_stop_test(const Scene& S, Counters* c0, int blk, int nblk);
__global__ void k_boxes(Scene S, int swept, Counters fresh, int reset_mode,
                        int stop_test, int nmain) {
  if (stop_test && (int)blockIdx.x >= nmain) {
    /* this scene's counters are the swept block; the static one precedes */
    newton_stop_test(S, S.cnt - 1, blockIdx.x - nmain, gridDim.x - nmain);
    return;
  }
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (reset_mode) pass_reset(S, fresh, reset_mode == 2, t, gridDim.x * blockDim.x);
  if (swept < 0) return;
  if (!S.cnt->reuse) chunk_or_body_box(S, swept, t);
}

/* exact box of one vertex of a body, static at q or swept over
 * [q, q + dq]: its positions by the canonical transform of every other
 * kernel (vertex_pos, vertex_pos_swept) from the body's qb and db */
__device__ __forceinline__ void vert_box(const Scene& S, int v, const double* qb,
                                         const double* db, int swept, double* box) {
  const double b0 = S.xbar[v], b1 = S.xbar[S.V + v], b2 = S.xbar[2 * S.V + v];
  double x[3];
  xform(qb, b0, b1, b2, x);
  if (swept) {
    double dx[3];
    xform(db, b0, b1, b2, dx);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double x1 = __dadd_rn(x[k], dx[k]);
      box[k] = fmin(x[k], x1);
      box[3 + k] = fmax(x[k], x1);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) box[k] = box[3 + k] = x[k];
  }
}
/* exact box of one primitive of a body (a chunk's primitives share it) */
__device__ __forceinline__ void prim_box(const Scene& S, int kind, int id,
                                         const double* qb, const double* db,
                                         int swept, double* box) {
  if (kind == K_VERT) {
    vert_box(S, id, qb, db, swept, box);
    return;
  }
  int n = kind == K_TRI ? 3 : 2;
  const int* ids = kind == K_TRI ? S.tri : S.edge;
  int stride = kind == K_TRI ? S.T : S.E;
  vert_box(S, ids[id], qb, db, swept, box);
  for (int j = 1; j < n; ++j) {
    double b2[6];
    vert_box(S, ids[j * stride + id], qb, db, swept, b2);
    for (int k = 0; k < 3; ++k) {
      box[k] = fmin(box[k], b2[k]);
      box[3 + k] = fmax(box[3 + k], b2[3 + k]);
    }
  }
}

/* primitive pairs of every chunk pair, one wavefront per chunk pair.  The
 * second chunk's primitives whose exact box meets the first chunk's box are
 * compacted into LDS (ballot + prefix count); each lane whose own primitive
 * meets the second chunk's box tests it against the compacted list with
 * the exact predicate.  Both culls are sound: a primitive box lies inside
 * its chunk box and the rounded bound hi + dhat is monotone in hi. */
#define PP_STAGE 256
__global__ __launch_bounds__(256) void k_prim_pairs(Scene S, int swept) {
  __shared__ double qbox[4][ABD_CHUNK][6];
  __shared__ int qid[4][ABD_CHUNK];
  __shared__ int2 hits[4][PP_STAGE];
  __shared__ int hcount[4];
  if (S.cnt->reuse) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int ncp = min(S.cnt->n_cp, S.cap_cp);
  /* every wavefront works through its own chunk pairs */
  for (int c = blockIdx.x * 4 + wave; c < ncp; c += gridDim.x * 4) {
    const int4 cp = S.cp[c];
    /* uniform over the wavefront: the chunks' data in scalar loads */
    const int P = __builtin_amdgcn_readfirstlane(cp.y);
    const int Q = __builtin_amdgcn_readfirstlane(cp.z);
    const int kindP = cp.x == C_PT ? K_VERT : K_EDGE;
    const int kindQ = cp.x == C_PT ? K_TRI : K_EDGE;
    const int nP = S.ch_count[P];
    const int nQ = S.ch_count[Q];
    /* every primitive of a chunk belongs to the chunk's body */
    const int bP = S.ch_body[P], bQ = S.ch_body[Q];
    const double *qP = S.q + 12 * bP, *dP = S.dq + 12 * bP;
    const double *qQ = S.q + 12 * bQ, *dQ = S.dq + 12 * bQ;
    /* both sides' primitives are loaded together (independent gathers) */
    bool keep = false, mine = false;
    int id = 0, pid = 0;
    double qb[6], box[6];
    if (lane < nQ) {
      id = S.ch_prims[S.ch_start[Q] + lane];
      prim_box(S, kindQ, id, qQ, dQ, swept, qb);
    }
    if (lane < nP) {
      pid = S.ch_prims[S.ch_start[P] + lane];
      prim_box(S, kindP, pid, qP, dP, swept, box);
    }
    if (lane < nQ) keep = box_overlap(qb, S.ch_box + 6 * P, S.dhat);
    if (lane < nP) mine = box_overlap(box, S.ch_box + 6 * Q, S.dhat);
    const unsigned long long m = __ballot(keep);
    const int nq = __popcll(m);
    if (nq == 0) continue; /* uniform over the wavefront */
    if (keep) {
      const int pos = __popcll(m & ((1ull << lane) - 1ull));
      qid[wave][pos] = id;
#pragma unroll
      for (int k = 0; k < 6; ++k) qbox[wave][pos][k] = qb[k];
    }
    wave_lds_sync();
    /* every test once: hits staged in LDS and appended with one global
     * atomic per chunk pair (beyond PP_STAGE hits, one by one) */
    const bool pt = cp.x == C_PT; /* uniform over the wavefront */
    int* const counter = pt ? &S.cnt->n_pt : &S.cnt->n_ee;
    const int cap = pt ? S.cap_pt : S.cap_ee;
    int* const list = pt ? S.cand_pt : S.cand_ee;
    if (lane == 0) hcount[wave] = 0;
    wave_lds_sync();
    if (mine)
      for (int j = 0; j < nq; ++j) {
        if (!box_overlap(box, qbox[wave][j], S.dhat)) continue;
        const int other = qid[wave][j];
        const int a0 = pt ? pid : min(pid, other), a1 = pt ? other : max(pid, other);
        const int h = atomicAdd(&hcount[wave], 1);
        if (h < PP_STAGE) {
          hits[wave][h] = make_int2(a0, a1);
        } else {
          const int k = atomicAdd(counter, 1);
          if (k < cap) {
            list[3 * k] = a0;
            list[3 * k + 1] = a1;
            list[3 * k + 2] = cp.w;
          }
        }
      }
    wave_lds_sync();
    const int nh = min(hcount[wave], PP_STAGE);
    if (nh > 0) {
      int base = 0;
      if (lane == 0) base = atomicAdd(counter, nh);
      base = __shfl(base, 0, 64);
      for (int i = lane; i < nh; i += 64) {
        const int k = base + i;
        if (k < cap) {
          const int2 hh = hits[wave][i];
          list[3 * k] = hh.x;
          list[3 * k + 1] = hh.y;
          list[3 * k + 2] = cp.w;
        }
      }
    }
    wave_lds_sync(); /* qbox, hits are reused by the next chunk pair */
  }
}

/* vertex-ground candidates: vertex chunks of dynamic bodies whose box
 * reaches the ground band, then each vertex exactly */
__global__ void k_pg(Scene S, int swept) {
  if (S.cnt->reuse) return;
  const double top = __dadd_rn(S.ground_y, S.dhat);
  const int lane = threadIdx.x % 64;
  const int nw = gridDim.x * (blockDim.x / 64);
  for (int c = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; c < S.NC;
       c += nw) {
    if (S.ch_kind[c] != K_VERT || S.kind[S.ch_body[c]] != 0) continue;
    if (!body_in_pass(S, S.ch_body[c])) continue;
    if (!(S.ch_box[6 * c + 1] <= top)) continue;
    bool ok = false;
    int v = 0;
    if (lane < S.ch_count[c]) {
      v = S.ch_prims[S.ch_start[c] + lane];
      const int b = S.ch_body[c];
      double box[6];
      vert_box(S, v, S.q + 12 * b, S.dq + 12 * b, swept, box);
      ok = box[1] <= top;
    }
    const int k = wave_slot(ok, &S.cnt->n_pg);
    if (ok && k < S.cap_pg) S.cand_pg[k] = v;
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

/* hoff_words: 8-byte words per off-diagonal block (144 FP64, 72 FP32) */
__global__ void k_filter(Scene S, int hoff_words) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int ran = S.iter_mode == 0;
    for (int q = 0; q < S.NP && !ran; ++q) ran = S.ps[q].state == PS_NEWTON;
    S.cnt->stat_ran = ran;
  }
  const int npt = min(S.cnt->n_pt, S.cap_pt);
  const int nee = min(S.cnt->n_ee, S.cap_ee);
  const int npg = min(S.cnt->n_pg, S.cap_pg);
  const int tot = npt + nee + npg;
  const int stride = gridDim.x * blockDim.x;
  double dmin = INFINITY;
  for (int t0 = blockIdx.x * blockDim.x; t0 < tot; t0 += stride) {
    const int t = t0 + threadIdx.x;
    int kind = C_PG, i = 0, j = 0, slot = -1;
    double d = INFINITY;
    if (t < npt + nee) {
      const int* c = t < npt ? S.cand_pt + 3 * t : S.cand_ee + 3 * (t - npt);
      kind = t < npt ? C_PT : C_EE;
      i = c[0]; j = c[1]; slot = c[2];
      int vid[4];
      pair_vertices(S, kind, i, j, vid);
      /* lists taken over from the swept phase also hold pairs of problems
       * that are not in this pass */
      if (body_in_pass(S, S.vbody[vid[0]])) {
        double x[12];
        for (int k = 0; k < 4; ++k) vertex_pos(S, vid[k], x + 3 * k);
        d = pair_dist(kind, x);
      }
    } else if (t < tot) {
      i = S.cand_pg[t - npt - nee];
      if (body_in_pass(S, S.vbody[i])) {
        double xv[3];
        vertex_pos(S, i, xv);
        d = xv[1] - S.ground_y;
      }
    }
    dmin = fmin(dmin, fmax(d, 0.0));
    const bool ok = t < tot && d < S.dhat;
    const int k = wave_slot(ok, &S.cnt->n_act);
    if (ok && k < S.cap_act) S.act[k] = make_int4(kind, i, j, slot);
  }
  /* smallest distance: reduced over the wavefront, one atomic per wave */
  for (int o = 32; o > 0; o >>= 1) dmin = fmin(dmin, __shfl_xor(dmin, o, 64));
  if (__lane_id() == 0 && dmin < INFINITY) atomic_min_pos(&S.cnt->min_dist, dmin);
  /* the same launch clears the off-diagonal blocks and used flags of the
   * current body pairs, which the assembly then adds into */
  const int nbp = min(S.cnt->n_bp, S.cap_bp);
  unsigned long long* Ho = (unsigned long long*)S.Hoff;
  const long nw = (long)hoff_words * nbp;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < nw; t += stride)
    Ho[t] = 0ull;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nbp; t += stride)
    S.slot_used[t] = 0;
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

/* Barrier gradient g_y (FP64) and the frame-scaled Hessian G H_y G (packed,
 * reduced frame, not yet projected) of one PT/EE pair with slot positions
 * x; Gs receives the frame scales |f_r|. */
__device__ __forceinline__ void pair_frame_derivs(const Scene& S, int kind, int ei,
                                               int ej, const double* x,
                                               double w, double* gy,
                                               double* K, double* Gs) {
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
  double gd[9];
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
}

/* One wavefront of 64 active pairs.  Phase 1 (a lane per pair): distance
 * feature, barrier gradient and Hessian in the reduced frame with its PSD
 * projection, and the frame-to-body maps W.  Phase 2 (all lanes per pair):
 * T = H_y W_Y, then the body-space gradient and 12x12 blocks W_X^T T,
 * accumulated with FP64 atomics into g, Hdiag and Hoff. */
#define PAIRS_PER_WG 16
/* PSD projection of a symmetric 9x9 matrix K by one-sided (Hestenes)
 * Jacobi on the shifted matrix A = K' + mu I, where K' = 2^-e K with 2^e
 * the power of two at or above the largest |K| entry (exact scaling) and
 * mu = 2 |K'|_F, so that A is symmetric positive definite with eigenvalues
 * in [|K'|_F, 3 |K'|_F].  One matrix per group of 16 lanes, lane j (< 9)
 * holding column j of A.  A sweep has nine rounds; round k pairs index a
 * with (2k - a) mod 9 (the round-robin order, index k rests), so every pair
 * of columns meets once per sweep.  The two lanes of a pair swap columns
 * (cross-lane reads, no LDS) and form, in the same order, the same dot
 * products al = a_p.a_p, be = a_q.a_q, ga = a_p.a_q and the same rotation
 * making the two columns orthogonal: t = sgn(be - al) 2ga /
 * (|be - al| + hypot(be - al, 2ga)), c = 1 / sqrt(1 + t^2), s = t c
 * (evaluated with two reciprocal square roots of one Newton step each),
 * a_p <- c a_p - s a_q, a_q <- s a_p + c a_q.  A rotation is applied while
 * ga^2 > rot2 al be; a group stops after a sweep in which every pair had
 * ga^2 <= stop2 al be, independently of the other groups of the wavefront
 * (a projection does not depend on the matrices sharing its wavefront).
 * The columns are then A's eigenvectors scaled by its eigenvalues
 * sigma_j = |a_j| (A's condition number is at most 3, so the accumulated
 * rotation is not needed), K''s eigenvalues are sigma_j - mu, and
 * K+ = 2^e sum_j max(sigma_j - mu, 0) / sigma_j^2 a_j a_j^T, whose row r
 * replaces k on lane r.  Per round: one exchange of nine values and a
 * short chain (three dot products, two reciprocal square roots). */
template <typename T> struct OsjTol;
template <> struct OsjTol<double> {
  static constexpr double rot2 = 1e-28, stop2 = 1e-22;
};
template <> struct OsjTol<float> {
  static constexpr float rot2 = 1e-12f, stop2 = 1.6e-11f;
};
template <typename T>
struct OsjX {
  T col[4][9][9]; /* the converged columns of each group */
  T w[4][9];      /* max(sigma - mu, 0) / sigma^2 */
};
__device__ __forceinline__ double scale2(double x, int e) { return ldexp(x, e); }
__device__ __forceinline__ float scale2(float x, int e) { return ldexpf(x, e); }
__device__ __forceinline__ int exp2_above(double x) {
  int e;
  (void)frexp(x, &e);
  return e;
}
__device__ __forceinline__ int exp2_above(float x) {
  int e;
  (void)frexpf(x, &e);
  return e;
}
template <typename T>
__device__ __forceinline__ void psd9_osj(OsjX<T>& X, int g, bool on, T* k) {
  constexpr T rot2 = OsjTol<T>::rot2, stop2 = OsjTol<T>::stop2;
  const int lane = __lane_id();
  const int base = lane & ~15, grp = lane >> 4;
  const bool mine = on && g < 9; /* a column of the matrix */
  /* exact power-of-two scaling by the group's largest entry */
  T mx = T(0);
#pragma unroll
  for (int m = 0; m < 9; ++m) mx = fmax(mx, mine ? fabs(k[m]) : T(0));
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 16));
  const int e = mx > T(0) ? exp2_above(mx) : 0;
  T a[9];
  T ss = T(0);
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    a[m] = mine ? scale2(k[m], -e) : T(0);
    ss += a[m] * a[m];
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 16);
  const T mu = ss > T(0) ? T(2) * (ss * rsq_nr(ss)) : T(0);
#pragma unroll
  for (int m = 0; m < 9; ++m)
    if (m == g) a[m] += mu;
  /* group-uniform: a group without a matrix, or with K = 0, is done */
  bool gdone = !on || !(mu > T(0));
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (__ballot(!gdone) == 0ull) break;
    bool big = false;
#pragma unroll 1
    for (int kr = 0; kr < 9; ++kr) {
      const int q = g < 9 ? (2 * kr + 18 - g) % 9 : g;
      T b[9];
#pragma unroll
      for (int m = 0; m < 9; ++m) b[m] = __shfl(a[m], base + q, 64);
      if (!gdone && mine && q != g) {
        const bool lo = g < q;
        /* own = a.a, oth = b.b, ga = a.b: the partner lane forms the same
         * three sums in the same order (its own is this lane's oth) */
        T own = T(0), oth = T(0), ga = T(0);
#pragma unroll
        for (int m = 0; m < 9; ++m) {
          own = fma(a[m], a[m], own);
          oth = fma(b[m], b[m], oth);
          ga = fma(a[m], b[m], ga);
        }
        const T al = lo ? own : oth, be = lo ? oth : own;
        const T g2 = ga * ga, ab = al * be;
        big = big || g2 > stop2 * ab;
        if (g2 > rot2 * ab) {
          /* with r = hypot(aa, bb) and u = |aa| + r: t = sgn(aa) bb / u,
           * 1 + t^2 = 2 r u / u^2, so c = u / sqrt(2 r u) and
           * s = sgn(aa) bb / sqrt(2 r u); one Newton step on each
           * reciprocal square root leaves c^2 + s^2 within about 1e-14 of
           * 1 (the columns' scale drifts by about that per rotation) */
          const T aa = be - al, bb = T(2) * ga;
          const T h2 = aa * aa + bb * bb;
          const T r = h2 * rsq_nr1(h2);
          const T u = fabs(aa) + r;
          const T y = rsq_nr1(T(2) * r * u);
          const T c = u * y;
          const T sn = (aa < T(0) ? -bb : bb) * y;
          /* a_p <- c a_p - s a_q on the lane of p, a_q <- c a_q + s a_p */
          const T sl = lo ? -sn : sn;
#pragma unroll
          for (int m = 0; m < 9; ++m) a[m] = fma(c, a[m], sl * b[m]);
        }
      }
    }
    const unsigned long long gm = 0xFFFFull << base;
    if ((__ballot(big) & gm) == 0ull) gdone = true;
  }
  /* K+ row by row from the converged columns */
  if (mine) {
    T s2 = T(0);
#pragma unroll
    for (int m = 0; m < 9; ++m) s2 += a[m] * a[m];
    const T sig = s2 * rsq_nr(s2);
    const T lam = sig - mu;
    X.w[grp][g] = lam > T(0) ? lam * rcp_nr(s2) : T(0);
#pragma unroll
    for (int m = 0; m < 9; ++m) X.col[grp][g][m] = a[m];
  }
  wave_lds_sync();
  if (mine) {
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 9; ++j) acc += X.w[grp][j] * X.col[grp][j][g] * X.col[grp][j][m];
      k[m] = scale2(acc, e);
    }
  }
  wave_lds_sync();
}

template <typename HT>
__global__ __launch_bounds__(64) void k_assemble(Scene S) {
  __shared__ HT KL[45 * 64];
  __shared__ double GW[33 * 64]; /* rows 0..8 g_y, 9..20 W_A, 21..32 W_B */
  __shared__ HT TB[216];
  __shared__ int meta[3 * 64];
  __shared__ OsjX<HT> JX;            /* converged Jacobi columns */
  __shared__ HT IG[9 * 64];         /* inverse frame scales of each pair */
  __shared__ unsigned char proj[64]; /* the pair's 9x9 needs the projection */
  const int lane = threadIdx.x;
  const int nact = min(S.cnt->n_act, S.cap_act);
  /* pairs per workgroup: as few as the grid allows (each pair's projection
   * is one lane's serial work, so a few pairs spread over many workgroups
   * finish soonest), at most PAIRS_PER_WG */
  const int ppw = max(1, min(PAIRS_PER_WG, (nact + (int)gridDim.x - 1) / (int)gridDim.x));
  for (int base = blockIdx.x * ppw; base < nact; base += gridDim.x * ppw) {
    const int t = base + lane;
    int ba = -1, bb = -1, slot = -1;
    proj[lane] = 0;
    if (lane < ppw && t < nact) {
      const int4 a = S.act[t];
      const int kind = a.x;
      slot = a.w;
      double gy[9], Wa[12], Wb[12];
      HT K[45];
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
        for (int i = 0; i < 45; ++i) K[i] = HT(0);
        gy[1] = w * b1;
        K[sidx(1, 1)] = (HT)(w * b2);
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
        double Kd[45], Gs[9];
        pair_frame_derivs(S, kind, a.y, a.z, x, w, gy, Kd, Gs);
#pragma unroll
        for (int i = 0; i < 45; ++i) K[i] = (HT)Kd[i];
        /* projected (and scaled back by the inverse frame scales) below,
         * by the lane groups of the workgroup */
#pragma unroll
        for (int p = 0; p < 9; ++p) IG[p * 64 + lane] = (HT)(1.0 / Gs[p]);
        proj[lane] = 1;
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
    const int npairs = min(ppw, nact - base);
    /* PSD projection of the PT/EE frame Hessians, four pairs at a time */
    for (int j0 = 0; j0 < npairs; j0 += 4) {
      const int j = j0 + lane / 16, g = lane % 16, r = g;
      const bool on = j < npairs && proj[j];
      const bool kon = on && g < 9; /* the lanes holding the matrix rows */
      HT k[9];
#pragma unroll
      for (int m = 0; m < 9; ++m) k[m] = kon ? KL[sidx(r, m) * 64 + j] : HT(0);
      __syncthreads();
      psd9_osj<HT>(JX, g, on, k);
      if (kon) {
        const HT ir = IG[r * 64 + j];
#pragma unroll
        for (int m = 0; m < 9; ++m)
          if (m >= r) KL[sidx(r, m) * 64 + j] = k[m] * (ir * IG[m * 64 + j]);
      }
      __syncthreads();
    }
    for (int j = 0; j < npairs; ++j) {
      const int A = meta[j], Bq = meta[64 + j], sl = meta[128 + j];
      if (A < 0 && Bq < 0) continue;
      /* T_Y[(r,i)][(i2,l)] = sum_u H[(r,i),(u,i2)] W_Y[u][l] */
      for (int e = lane; e < 216; e += 64) {
        const int Y = e / 108, f = e % 108, ri = f / 12, i2 = (f % 12) / 4,
                  l = f % 4;
        const int wo = Y ? 21 : 9;
        HT v = 0;
#pragma unroll
        for (int u = 0; u < 3; ++u)
          v += KL[sidx(ri, 3 * u + i2) * 64 + j] * (HT)GW[(wo + 4 * u + l) * 64 + j];
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
          if (!S.det)
            atomicAdd(S.g + 12 * body + dd, v);
          else if (!det_add(S.det_g + (size_t)(12 * body + dd) * DET_W, v))
            atomicOr(&S.cnt->err, 2);
        }
      }
      __syncthreads();
      /* blocks: (A,A), (B,B), (lo,hi) = W_X^T T_Y */
      for (int blk = 0; blk < 3; ++blk) {
        int X, Y;
        HT* dst;
        det_word* ddst;
        if (blk == 0) {
          if (A < 0) continue;
          X = 0; Y = 0; dst = (HT*)S.Hdiag + 144 * A;
          ddst = S.det_hd + (size_t)144 * DET_W * A;
        } else if (blk == 1) {
          if (Bq < 0) continue;
          X = 1; Y = 1; dst = (HT*)S.Hdiag + 144 * Bq;
          ddst = S.det_hd + (size_t)144 * DET_W * Bq;
        } else {
          if (A < 0 || Bq < 0) continue;
          if (A < Bq) { X = 0; Y = 1; } else { X = 1; Y = 0; }
          dst = (HT*)S.Hoff + 144 * (size_t)sl;
          ddst = S.det_ho + (size_t)144 * DET_W * sl;
          if (lane == 0) S.slot_used[sl] = 1;
        }
        const int wx = X ? 21 : 9;
        for (int e = lane; e < 144; e += 64) {
          int i, k, i2, l;
          dof_split(e / 12, i, k);
          dof_split(e % 12, i2, l);
          HT v = 0;
#pragma unroll
          for (int r = 0; r < 3; ++r)
            v += (HT)GW[(wx + 4 * r + k) * 64 + j] *
                 TB[Y * 108 + (3 * r + i) * 12 + i2 * 4 + l];
          if (!S.det)
            atomicAdd(dst + e, v);
          else if (!det_add(ddst + (size_t)e * DET_W, (double)v))
            atomicOr(&S.cnt->err, 2);
        }
      }
      __syncthreads();
    }
    __syncthreads();
  }
}

/* deterministic mode: the exact barrier sums rounded once and added to
 * the body terms (gradient, diagonal blocks) or stored (off-diagonal
 * blocks of the body pairs that received contributions); the
 * accumulators are cleared for the next assembly.  One thread per entry. */
template <typename HT>
__global__ void k_det_finish(Scene S) {
  const long nb = 156L * S.B;
  const long nbp = min(S.cnt->n_bp, S.cap_bp);
  const long stride = (long)gridDim.x * blockDim.x;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < nb + 144 * nbp;
       t += stride) {
    if (t < nb) {
      const int b = (int)(t / 156), e = (int)(t % 156);
      if (!body_in_pass(S, b)) continue;
      det_word* w = (e < 12 ? S.det_g + (size_t)(12 * b + e) * DET_W
                            : S.det_hd + ((size_t)144 * b + e - 12) * DET_W);
      const double v = det_value(w);
      for (int k = 0; k < DET_W; ++k) w[k] = 0ull;
      if (v == 0.0) continue;
      if (e < 12) {
        S.g[12 * b + e] += v;
      } else {
        HT* h = (HT*)S.Hdiag + 144 * b + e - 12;
        *h = (HT)((double)*h + v);
      }
    } else {
      const long u = t - nb;
      const int sl = (int)(u / 144), e = (int)(u % 144);
      if (!S.slot_used[sl]) continue;
      det_word* w = S.det_ho + ((size_t)144 * sl + e) * DET_W;
      const double v = det_value(w);
      for (int k = 0; k < DET_W; ++k) w[k] = 0ull;
      ((HT*)S.Hoff)[144 * (size_t)sl + e] = (HT)v;
    }
  }
}

/* deterministic mode: each block row's entries in ascending neighbour
 * order (the fill order depends on the order of atomics), rows
 * [r0, r1) by the calling threads */
__device__ void sort_block_rows(const Scene& S, int r0, int r1, int step) {
  for (int r = r0; r < r1; r += step) {
    const int lo = S.row_ptr[r], hi = min(S.row_ptr[r + 1], S.cap_col);
    for (int i = lo + 1; i < hi; ++i) {
      const int b = S.col_body[i], sl = S.col_slot[i], tr = S.col_trans[i];
      int j = i - 1;
      while (j >= lo && S.col_body[j] > b) {
        S.col_body[j + 1] = S.col_body[j];
        S.col_slot[j + 1] = S.col_slot[j];
        S.col_trans[j + 1] = S.col_trans[j];
        --j;
      }
      S.col_body[j + 1] = b;
      S.col_slot[j + 1] = sl;
      S.col_trans[j + 1] = tr;
    }
  }
}
__global__ void k_sort_rows(Scene S) {
  sort_block_rows(S, blockIdx.x * blockDim.x + threadIdx.x, S.B, gridDim.x * blockDim.x);
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
  /* single block (1024 threads) exclusive scan of row_cnt into row_ptr:
   * per-thread runs, then a wavefront scan and a scan of the 16 wavefront
   * totals */
  __shared__ int wsum[16];
  const int n = S.B;
  const int per = (n + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * per, hi = min(n, lo + per);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    /* the component labels that follow add their counts */
    S.cnt->n_dir = 0;
    S.cnt->n_big = 0;
    S.cnt->plan = 0;
  }
  int s = 0;
  for (int i = lo; i < hi; ++i) s += S.row_cnt[i];
  int x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    int w = lane < 16 ? wsum[lane] : 0;
    for (int o = 1; o < 16; o <<= 1) {
      const int y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (lane < 16) wsum[lane] = w;
  }
  __syncthreads();
  int acc = x - s + (wave > 0 ? wsum[wave - 1] : 0);
  if (threadIdx.x == blockDim.x - 1) {
    S.row_ptr[n] = acc + s;
    S.cnt->n_rows_used = acc + s;
  }
  for (int i = lo; i < hi; ++i) {
    S.row_ptr[i] = acc;
    acc += S.row_cnt[i];
    S.row_cnt[i] = 0; /* reused as fill cursor */
  }
}
/* Connected components of the system among the bodies [c0, c0 + n) (whole
 * problems: no used block joins them to other bodies), in one workgroup
 * with LDS arrays par [n], cnt [n + 1], cur [n / 2 + 1] and sh [4]: every
 * body starts as its own root; each round, every used block whose two
 * bodies have different roots links the larger root under the smaller (an
 * LDS atomic minimum, so links only ever point to smaller indices), then
 * every body takes its root; rounds repeat until a round links nothing.
 * Then bmode of each body (0 alone, 1 in a component of 2..DIR_MAX bodies,
 * 2 larger) and a slot per directly solved component with its bodies in
 * ascending order.  single: these are all bodies of the scene (the counts
 * are stored), else the slots and counts are added to the scene's. */
__device__ void label_components(const Scene& S, int c0, int n, int nbp, int* par,
                                 int* cnt, int* cur, int* sh, bool single) {
  int& s_changed = sh[0];
  int& s_ndir = sh[1];
  int& s_nbig = sh[2];
  int& s_base = sh[3];
  volatile int* vp = par;
  for (int i = threadIdx.x; i < n; i += blockDim.x) par[i] = i;
  __syncthreads();
  bool settled = false;
  for (int round = 0; round < 64 && !settled; ++round) {
    if (threadIdx.x == 0) s_changed = 0;
    __syncthreads();
    for (int p = threadIdx.x; p < nbp; p += blockDim.x) {
      if (!S.slot_used[p]) continue;
      const int2 ab = S.bp[p];
      if (ab.x < c0 || ab.x >= c0 + n) continue;
      int ra = ab.x - c0, rb = ab.y - c0;
      while (vp[ra] != ra) ra = vp[ra];
      while (vp[rb] != rb) rb = vp[rb];
      if (ra != rb) {
        atomicMin(&par[max(ra, rb)], min(ra, rb));
        s_changed = 1;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      int r = vp[i];
      while (vp[r] != r) r = vp[r];
      vp[i] = r;
    }
    __syncthreads();
    settled = s_changed == 0;
    __syncthreads(); /* every thread has read the flag before its reset */
  }
  if (!settled) {
    /* a graph that did not settle in the bounded rounds stays with the
     * PCG: in one workgroup for the whole scene, no plan; else its bodies
     * as one large component */
    if (single) return;
    for (int i = threadIdx.x; i < n; i += blockDim.x) S.bmode[c0 + i] = 2;
    if (threadIdx.x == 0) {
      atomicAdd(&S.cnt->n_big, n);
      S.cnt->plan = 1;
    }
    return;
  }
  /* component sizes (the fill cursors are free again) */
  for (int i = threadIdx.x; i < n; i += blockDim.x) cnt[i] = 0;
  if (threadIdx.x == 0) s_ndir = s_nbig = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&cnt[par[i]], 1);
  __syncthreads();
  int nbig = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int c = cnt[par[i]];
    const int mode = c == 1 ? 0 : (c <= DIR_MAX ? 1 : 2);
    S.bmode[c0 + i] = mode;
    nbig += mode == 2;
  }
  if (nbig) atomicAdd(&s_nbig, nbig);
  __syncthreads();
  /* a slot per directly solved component, kept (negated) at its root */
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (par[i] == i && cnt[i] >= 2 && cnt[i] <= DIR_MAX) {
      const int k = atomicAdd(&s_ndir, 1);
      cur[k] = 0;
      cnt[i] = -1 - k;
    }
  __syncthreads();
  if (threadIdx.x == 0) s_base = single ? 0 : atomicAdd(&S.cnt->n_dir, s_ndir);
  __syncthreads();
  const int base = s_base;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int c = cnt[par[i]];
    if (c < 0) {
      const int k = -1 - c;
      S.dir_body[(base + k) * DIR_MAX + atomicAdd(&cur[k], 1)] = c0 + i;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < s_ndir; k += blockDim.x) S.dir_n[base + k] = cur[k];
  if (threadIdx.x == 0) {
    if (single) {
      S.cnt->n_dir = s_ndir;
      S.cnt->n_big = s_nbig;
    } else if (s_nbig) {
      atomicAdd(&S.cnt->n_big, s_nbig);
    }
    S.cnt->plan = 1;
  }
}

/* the three steps in one workgroup when the block-row counts fit in LDS:
 * counts by LDS atomics, the same scan, then the counts become the fill
 * cursors.  With comp_solve the same workgroup then labels the connected
 * components of the system (bodies joined by a used off-diagonal block)
 * and sorts them for the linear solve: a body alone is solved with its
 * block inverse, a component of 2..DIR_MAX bodies by dense elimination,
 * a larger one by the PCG. */
#define DIR_SLOTS (BSR_LDS_ROWS / 2 + 1)
__global__ __launch_bounds__(1024) void k_bsr_small(Scene S) {
  __shared__ int cnt[BSR_LDS_ROWS + 1];
  __shared__ int par[BSR_LDS_ROWS];
  __shared__ int cur[DIR_SLOTS];
  __shared__ int sh[4];
  __shared__ int wsum[16];
  const int n = S.B;
  for (int i = threadIdx.x; i <= n; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const int nbp = min(S.cnt->n_bp, S.cap_bp);
  for (int p = threadIdx.x; p < nbp; p += blockDim.x) {
    if (!S.slot_used[p]) continue;
    const int2 ab = S.bp[p];
    atomicAdd(&cnt[ab.x], 1);
    atomicAdd(&cnt[ab.y], 1);
  }
  __syncthreads();
  const int per = (n + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * per, hi = min(n, lo + per);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int s = 0;
  for (int i = lo; i < hi; ++i) s += cnt[i];
  int x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    int w = lane < 16 ? wsum[lane] : 0;
    for (int o = 1; o < 16; o <<= 1) {
      const int y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (lane < 16) wsum[lane] = w;
  }
  __syncthreads();
  int acc = x - s + (wave > 0 ? wsum[wave - 1] : 0);
  if (threadIdx.x == blockDim.x - 1) {
    S.row_ptr[n] = acc + s;
    S.cnt->n_rows_used = acc + s;
  }
  for (int i = lo; i < hi; ++i) {
    const int c = cnt[i];
    S.row_ptr[i] = acc;
    cnt[i] = acc;
    acc += c;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < nbp; p += blockDim.x) {
    if (!S.slot_used[p]) continue;
    const int2 ab = S.bp[p];
    int k = atomicAdd(&cnt[ab.x], 1);
    if (k < S.cap_col) {
      S.col_slot[k] = p; S.col_body[k] = ab.y; S.col_trans[k] = 0;
    }
    k = atomicAdd(&cnt[ab.y], 1);
    if (k < S.cap_col) {
      S.col_slot[k] = p; S.col_body[k] = ab.x; S.col_trans[k] = 1;
    }
  }
  if (S.det) {
    __syncthreads(); /* the fill's global writes, for the sort */
    sort_block_rows(S, threadIdx.x, n, blockDim.x);
  }
  if (!S.comp_solve) return;
  label_components(S, 0, n, nbp, par, cnt, cur, sh, true);
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

/* block rows (and component labels) of scenes above one workgroup's LDS,
 * one workgroup per chunk of whole problems (bodies [lab_chunk[c],
 * lab_chunk[c + 1]), at most BSR_LDS_ROWS; no used block joins two
 * chunks).  First the counts of the chunk's rows by LDS atomics, their
 * exclusive scan into row_ptr relative to the chunk, and the chunk's
 * total; then (k_bsr_chunk_fill) the chunk's offset, the sum of the totals
 * before it, the fill through LDS cursors, and the labels. */
__device__ int block_scan_1024(int* cnt, int n, int* wsum, int* row_out, int base) {
  /* exclusive scan of cnt[0..n) by 1024 threads (runs of ceil(n/1024) per
   * thread, then the wavefront and workgroup prefix); row_out[i] = base +
   * prefix, cnt[i] = the same; returns the total (valid in every thread) */
  const int per = (n + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * per, hi = min(n, lo + per);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int s = 0;
  for (int i = lo; i < hi; ++i) s += cnt[i];
  int tot;
  const int ex = wave_prefix(s, &tot);
  if (lane == 0) wsum[wave] = tot;
  __syncthreads();
  int acc = ex, all = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wave) acc += wsum[w];
    all += wsum[w];
  }
  for (int i = lo; i < hi; ++i) {
    const int c = cnt[i];
    cnt[i] = base + acc;
    row_out[i] = base + acc;
    acc += c;
  }
  return all;
}
__global__ __launch_bounds__(1024) void k_bsr_chunk_count(Scene S) {
  __shared__ int cnt[BSR_LDS_ROWS + 1];
  __shared__ int wsum[16];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    /* the component labels that follow add their counts */
    S.cnt->n_dir = 0;
    S.cnt->n_big = 0;
    S.cnt->plan = 0;
  }
  const int c0 = S.lab_chunk[blockIdx.x], n = S.lab_chunk[blockIdx.x + 1] - c0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const int nbp = min(S.cnt->n_bp, S.cap_bp);
  for (int p = threadIdx.x; p < nbp; p += blockDim.x) {
    if (!S.slot_used[p]) continue;
    const int2 ab = S.bp[p];
    if (ab.x < c0 || ab.x >= c0 + n) continue;
    atomicAdd(&cnt[ab.x - c0], 1);
    atomicAdd(&cnt[ab.y - c0], 1);
  }
  __syncthreads();
  const int tot = block_scan_1024(cnt, n, wsum, S.row_ptr + c0, 0);
  if (threadIdx.x == 0) S.chunk_tot[blockIdx.x] = tot;
}
__global__ __launch_bounds__(1024) void k_bsr_chunk_fill(Scene S) {
  __shared__ int cnt[BSR_LDS_ROWS + 1];
  __shared__ int par[BSR_LDS_ROWS];
  __shared__ int cur[DIR_SLOTS];
  __shared__ int sh[4];
  __shared__ int s_base;
  const int c0 = S.lab_chunk[blockIdx.x], n = S.lab_chunk[blockIdx.x + 1] - c0;
  if (threadIdx.x == 0) {
    int b = 0;
    for (int c = 0; c < (int)blockIdx.x; ++c) b += S.chunk_tot[c];
    s_base = b;
    if (blockIdx.x + 1 == gridDim.x) {
      S.row_ptr[S.B] = b + S.chunk_tot[blockIdx.x];
      S.cnt->n_rows_used = b + S.chunk_tot[blockIdx.x];
    }
  }
  __syncthreads();
  const int base = s_base;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = S.row_ptr[c0 + i] + base;
    S.row_ptr[c0 + i] = r;
    cnt[i] = r; /* the fill cursor of the row */
  }
  __syncthreads();
  const int nbp = min(S.cnt->n_bp, S.cap_bp);
  for (int p = threadIdx.x; p < nbp; p += blockDim.x) {
    if (!S.slot_used[p]) continue;
    const int2 ab = S.bp[p];
    if (ab.x < c0 || ab.x >= c0 + n) continue;
    int k = atomicAdd(&cnt[ab.x - c0], 1);
    if (k < S.cap_col) {
      S.col_slot[k] = p; S.col_body[k] = ab.y; S.col_trans[k] = 0;
    }
    k = atomicAdd(&cnt[ab.y - c0], 1);
    if (k < S.cap_col) {
      S.col_slot[k] = p; S.col_body[k] = ab.x; S.col_trans[k] = 1;
    }
  }
  if (S.det) {
    __syncthreads(); /* the fill's global writes, for the sort */
    sort_block_rows(S, c0 + threadIdx.x, c0 + n, blockDim.x);
  }
  if (!S.comp_solve) return;
  __syncthreads();
  label_components(S, c0, n, nbp, par, cnt, cur, sh, false);
}

/* inverse of every diagonal block by Gauss-Jordan (SPD, no pivoting):
 * twelve lanes per body, one row (with its identity half) per lane, five
 * bodies per wavefront; the pivot row reaches the other lanes of its body
 * by cross-lane shuffles, so no barrier is needed.  A body that the
 * block-row build found alone in the system (no used off-diagonal block)
 * is solved here: dq = -H^-1 g, exactly (its block is its whole system). */
template <typename HT>
__global__ __launch_bounds__(192) void k_block_inverse(Scene S) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int slot = lane / 12, r = lane % 12;
  const int b = (blockIdx.x * 3 + wave) * 5 + slot;
  const bool act = slot < 5 && b < S.B;
  const int base = slot < 5 ? lane - r : lane; /* idle lanes read themselves */
  const HT* Hd = (const HT*)S.Hdiag;
  double row[24];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    row[c] = act ? (double)Hd[144 * b + 12 * r + c] : (r == c ? 1.0 : 0.0);
    row[12 + c] = r == c ? 1.0 : 0.0;
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    double pk[24];
    const int src = slot < 5 ? base + k : lane;
#pragma unroll
    for (int c = 0; c < 24; ++c) pk[c] = __shfl(row[c], src, 64);
    const double piv = pk[k];
    if (r == k) {
      const double inv = 1.0 / piv;
#pragma unroll
      for (int c = 0; c < 24; ++c) row[c] = pk[c] * inv;
    } else {
      const double f = row[k] / piv;
#pragma unroll
      for (int c = 0; c < 24; ++c) row[c] -= f * pk[c];
    }
  }
  if (act) {
    HT* Pi = (HT*)S.Pinv;
#pragma unroll
    for (int c = 0; c < 12; ++c) Pi[144 * b + 12 * r + c] = (HT)row[12 + c];
  }
  /* a body alone: dq = -H^-1 g (FP64 from the stored Hessian) */
  if (S.cnt->plan) {
    const bool alone = act && S.bmode[b] == 0 &&
                       (S.iter_mode == 0 || S.ps[S.bprob[b]].state == PS_NEWTON);
    const double gr = alone ? S.g[12 * b + r] : 0.0;
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const int src = slot < 5 ? base + c : lane;
      v += row[12 + c] * __shfl(gr, src, 64);
    }
    if (alone) S.dq[12 * b + r] = -v;
  }
}

/* Components of 2..DIR_MAX bodies, one wavefront each: the component's
 * system (its diagonal blocks and the used off-diagonal blocks between its
 * bodies, bodies in ascending order) is formed densely in LDS with -g as
 * an extra column, then each lane takes one row into registers and the
 * system is reduced by Gauss-Jordan elimination without pivoting (it is
 * symmetric positive definite): step k takes row k, unchanged, as the
 * pivot row (read lane by lane with readlane) and removes column k from
 * every other row; at the end dq_i = rhs_i / a_ii.  The steps are unrolled
 * for each size (12 rows per body), so every register index is static.
 * FP64 from the stored Hessian of either precision; the exact solution of
 * the component's system. */
#define DIR_WAVES 2
#define DIR_N (12 * DIR_MAX)
#define DIR_LD (DIR_N + 1)          /* row stride: n columns and the rhs */
#define DIR_NE (DIR_MAX * (DIR_MAX - 1))
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
/* n rows in lanes 0..n-1 of the wavefront, row r of A (stride DIR_LD, rhs
 * in column n); returns this lane's solution entry (lanes below n) */
template <int n>
__device__ __forceinline__ double gj_solve(const double* A, int lane) {
  double row[n + 1];
#pragma unroll
  for (int c = 0; c <= n; ++c) row[c] = lane < n ? A[lane * DIR_LD + c] : 0.0;
  double diag = 1.0;
#pragma unroll
  for (int k = 0; k < n; ++k) {
    const double ip = 1.0 / readlane_d(row[k], k);
    const double f = lane == k ? 0.0 : row[k] * ip;
    if (lane == k) diag = row[k];
#pragma unroll
    for (int c = k + 1; c <= n; ++c) row[c] = __fma_rn(-f, readlane_d(row[c], k), row[c]);
  }
  return row[n] / diag;
}
template <typename HT>
__global__ __launch_bounds__(64 * DIR_WAVES) void k_direct(Scene S) {
  __shared__ double As[DIR_WAVES][DIR_N * DIR_LD];
  __shared__ int bod[DIR_WAVES][DIR_MAX];
  __shared__ int ent[DIR_WAVES][DIR_NE][3]; /* (i * DIR_MAX + j, slot, trans) */
  __shared__ int nent[DIR_WAVES];
  if (!S.cnt->plan) return;
  const int ndir = S.cnt->n_dir;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* const A = As[wave];
  int* const bw = bod[wave];
  for (int k = blockIdx.x * DIR_WAVES + wave; k < ndir; k += gridDim.x * DIR_WAVES) {
    const int m = S.dir_n[k];
    /* the bodies in ascending order (rank = number of smaller ids) */
    const int mine = lane < m ? S.dir_body[k * DIR_MAX + lane] : 0x7fffffff;
    int rank = 0;
    for (int t = 0; t < m; ++t) rank += __shfl(mine, t, 64) < mine ? 1 : 0;
    if (lane < m) bw[rank] = mine;
    if (lane == 0) nent[wave] = 0;
    wave_lds_sync();
    /* the problem's state is read alongside the system; a problem outside
     * this pass keeps its dq */
    const bool run = S.iter_mode == 0 || S.ps[S.bprob[bw[0]]].state == PS_NEWTON;
    const int n = 12 * m;
    /* block-row entries (i, j > i) of the component, one lane per body */
    if (lane < m) {
      const int b = bw[lane];
      for (int e = S.row_ptr[b], e1 = S.row_ptr[b + 1]; e < e1; ++e) {
        const int nb = S.col_body[e];
        int j = 0;
        while (j < m && bw[j] != nb) ++j;
        if (j <= lane || j >= m) continue;
        const int q = atomicAdd(&nent[wave], 1);
        if (q < DIR_NE) {
          ent[wave][q][0] = lane * DIR_MAX + j;
          ent[wave][q][1] = S.col_slot[e];
          ent[wave][q][2] = S.col_trans[e];
        }
      }
    }
    for (int t = lane; t < n * DIR_LD; t += 64) A[t] = 0.0;
    wave_lds_sync();
    const int ne = min(nent[wave], DIR_NE);
    /* diagonal blocks, off-diagonal blocks (both triangles), -g */
    for (int t = lane; t < 144 * m; t += 64) {
      const int i = t / 144, e = t % 144, r = e / 12, c = e % 12;
      A[(12 * i + r) * DIR_LD + 12 * i + c] =
          (double)((const HT*)S.Hdiag)[144 * (size_t)bw[i] + e];
    }
    for (int t = lane; t < 144 * ne; t += 64) {
      const int q = t / 144, e = t % 144, r = e / 12, c = e % 12;
      const int i = ent[wave][q][0] / DIR_MAX, j = ent[wave][q][0] % DIR_MAX;
      const HT* blk = (const HT*)S.Hoff + 144 * (size_t)ent[wave][q][1];
      /* block (i, j): rows of body i; stored rows belong to the lower id */
      const double v = (double)(ent[wave][q][2] ? blk[12 * c + r] : blk[e]);
      A[(12 * i + r) * DIR_LD + 12 * j + c] = v;
      A[(12 * j + c) * DIR_LD + 12 * i + r] = v;
    }
    for (int t = lane; t < n; t += 64) A[t * DIR_LD + n] = -S.g[12 * bw[t / 12] + t % 12];
    wave_lds_sync();
    double x = 0.0;
    if (m == 2) x = gj_solve<24>(A, lane);
    else if (m == 3) x = gj_solve<36>(A, lane);
    else if (m == 4) x = gj_solve<48>(A, lane);
    else x = gj_solve<60>(A, lane);
    if (run && lane < n) S.dq[12 * bw[lane / 12] + lane % 12] = x;
    wave_lds_sync();
  }
}

/* grid-wide barrier for the persistent PCG launch.  The workgroup barrier
 * puts every wave's stores in L2; thread 0's agent-scope release add then
 * makes them visible device-wide, and its acquire loads (before the final
 * workgroup barrier) order the block's later reads after every arrival.
 * The spin is bounded so that every wave exits even if a barrier were
 * never completed (the host then reports a device error). */
__device__ __forceinline__ void grid_sync(unsigned* bar, unsigned nblocks,
                                          unsigned& gen, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    gen += 1;
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = gen * nblocks;
    long spins = 0;
    /* poll without acquire (an acquire load invalidates the L2 on every
     * poll), then one acquire fence */
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1L << 27)) {
        atomicOr(err, 1);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}


/* Add per-row values v[0..nv) of one 16-body group into the problem
 * accumulators dst(p) (bodies of one problem are contiguous, so a group
 * spans at most 16 problems): LDS atomics per problem, then one global
 * atomic per problem and value. */
template <int nv>
__device__ __forceinline__ void group_add(double (*gs)[4], int gr, int B,
                                          const int* bprob, int p, bool act,
                                          const double* v, ProbState* ps,
                                          const int* off) {
  const int g0 = gr * 16;
  const int plo = bprob[g0];
  const int phi = bprob[min(B, g0 + 16) - 1];
  if (threadIdx.x < 64)
    for (int k = 0; k < 4; ++k) gs[threadIdx.x & 15][k] = 0.0;
  __syncthreads();
  if (act)
#pragma unroll
    for (int k = 0; k < nv; ++k)
      if (v[k] != 0.0) atomicAdd(&gs[p - plo][k], v[k]);
  __syncthreads();
  if ((int)threadIdx.x <= phi - plo)
#pragma unroll
    for (int k = 0; k < nv; ++k) {
      double* d = (double*)((char*)(ps + plo + threadIdx.x) + off[k]);
      atomicAdd(d, gs[threadIdx.x][k]);
    }
  __syncthreads();
}

#define PCG_MAX_NP 2048
__device__ __forceinline__ double ld_acq(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      (const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

/* When every block of the persistent PCG launch owns exactly one 16-body
 * group, the group's rows of the system (diagonal blocks, block inverses
 * and up to PCG_OFF_CACHE off-diagonal blocks) stay in LDS for all
 * iterations: after each grid barrier only the vectors written by other
 * blocks have to come from memory. */
#define PCG_OFF_CACHE 24
template <typename HT>
struct PcgCache {
  HT hd[12 * 192]; /* [c][thread]: row `thread` of its body's diagonal block */
  HT pi[12 * 192]; /* the same rows of the block inverse */
  HT off[PCG_OFF_CACHE][144];
  int e0, n_off;
};
template <typename HT>
__device__ __forceinline__ bool pcg_cache_load(PcgCache<HT>& C, const Scene& S,
                                               const HT* Hd, const HT* Ho,
                                               const HT* Pi, int ngroups, int gr,
                                               bool own) {
  if (!own || gr >= ngroups) return false;
  const int lb = threadIdx.x / 12, row = threadIdx.x % 12;
  const int b = gr * 16 + lb;
  for (int c = 0; c < 12; ++c) {
    C.hd[c * 192 + threadIdx.x] = b < S.B ? Hd[144 * b + 12 * row + c] : HT(0);
    C.pi[c * 192 + threadIdx.x] = b < S.B ? Pi[144 * b + 12 * row + c] : HT(0);
  }
  const int e0 = S.row_ptr[gr * 16];
  const int n = min(S.row_ptr[min(S.B, gr * 16 + 16)] - e0, PCG_OFF_CACHE);
  for (int i = threadIdx.x; i < n * 144; i += blockDim.x)
    C.off[i / 144][i % 144] = Ho[144 * (size_t)S.col_slot[e0 + i / 144] + i % 144];
  if (threadIdx.x == 0) {
    C.e0 = e0;
    C.n_off = n;
  }
  __syncthreads();
  return true;
}

/* Block-Jacobi preconditioned CG on H dq = -g with zero initial guess,
 * every problem running its own recurrence, all iterations in one
 * persistent launch.  Each block owns 16 bodies (192 rows) per pass of a
 * grid-stride loop.  Per iteration: phase A forms p_k = z_k + beta_k
 * p_{k-1} on the fly and the product A p_k; phase B updates dq, r and
 * z = P^-1 r; two grid barriers.  Dots are reduced in FP64 into each
 * problem's ring of 4 slots, acc[4*j + 0] = r_j . z_j, + 1 = p_j . A p_j,
 * + 2 = r_j . r_j.  After each iteration every block reads the same
 * residuals and marks the same problems converged (|r| <= eta |b|), whose
 * rows then stay fixed. */
template <typename HT>
__global__ __launch_bounds__(192) void k_pcg(Scene S, double eta, int max_it) {
  const HT* __restrict__ Hd = (const HT*)S.Hdiag;
  const HT* __restrict__ Ho = (const HT*)S.Hoff;
  const HT* __restrict__ Pi = (const HT*)S.Pinv;
  __shared__ double rloc[16][12];
  __shared__ double gs[16][4];
  __shared__ unsigned char pdone[PCG_MAX_NP];
  __shared__ int any_active;
  __shared__ PcgCache<HT> cache;
  const unsigned nblk = gridDim.x;
  unsigned gen = 0;
  const int lb = threadIdx.x / 12, row = threadIdx.x % 12;
  const int ngroups = (S.B + 15) / 16;
  const int NP = S.NP;
  ProbState* ps = S.ps;
  const int OFF_ACC = (int)offsetof(ProbState, acc);
  const int OFF_BB = (int)offsetof(ProbState, bb);
  /* participating problems: every problem for the hooks, the problems in
   * the Newton state inside the device loop */
  for (int p = threadIdx.x; p < NP; p += blockDim.x)
    pdone[p] = (S.iter_mode == 0 || ps[p].state == PS_NEWTON) ? 0 : 1;
  __syncthreads();
  const bool cached = pcg_cache_load(cache, S, Hd, Ho, Pi, ngroups, (int)blockIdx.x,
                                          (int)gridDim.x >= ngroups);
  /* init: x = 0, r = b = -g, z = P^-1 r, p_{-1} = 0 */
  for (int gr = blockIdx.x; gr < ngroups; gr += nblk) {
    const int b = gr * 16 + lb;
    const int p = b < S.B ? S.bprob[b] : 0;
    const bool act = b < S.B && !pdone[p];
    const double rv = act ? -S.g[12 * b + row] : 0.0;
    if (act) {
      S.dq[12 * b + row] = 0.0;
      S.r[12 * b + row] = rv;
      S.p0[12 * b + row] = 0.0;
      S.p1[12 * b + row] = 0.0;
    }
    rloc[lb][row] = rv;
    __syncthreads();
    double z = 0.0;
    if (act) {
      HT zz = 0;
      for (int c = 0; c < 12; ++c)
        zz += (cached ? cache.pi[c * 192 + threadIdx.x] : Pi[144 * b + 12 * row + c]) *
              (HT)rloc[lb][c];
      z = (double)zz;
      S.zv[12 * b + row] = z;
    }
    const double v[2] = {rv * z, rv * rv};
    const int off[2] = {OFF_ACC + 0, OFF_BB};
    group_add<2>(gs, gr, S.B, S.bprob, p, act, v, ps, off);
  }
  grid_sync(&S.cnt->bar, nblk, gen, &S.cnt->err);
  /* problems with a zero right-hand side are done at once */
  for (int p = threadIdx.x; p < NP; p += blockDim.x)
    if (!pdone[p] && !(ld_acq(&ps[p].bb) > 0.0)) {
      pdone[p] = 1;
      if (blockIdx.x == 0) ps[p].pcg_iters = 0;
    }
  __syncthreads();
  int it = 0;
  for (it = 0; it < max_it; ++it) {
    double* pold = (it & 1) ? S.p0 : S.p1;
    double* pnew = (it & 1) ? S.p1 : S.p0;
    /* phase A: p = z + beta pold, Ap */
    for (int gr = blockIdx.x; gr < ngroups; gr += nblk) {
      const int b = gr * 16 + lb;
      const int p = b < S.B ? S.bprob[b] : 0;
      const bool act = b < S.B && !pdone[p];
      double pap = 0.0;
      if (act) {
        const double* acc = ps[p].acc;
        const double rz = ld_acq(acc + 4 * (it & 3));
        const double beta = it == 0 ? 0.0 : rz / ld_acq(acc + 4 * ((it - 1) & 3));
        /* matvec in the Hessian's precision (FP32 accumulation in the
         * mixed form); p itself stays FP64 */
        HT y = 0;
        const HT* H = Hd + 144 * b + 12 * row;
        for (int c = 0; c < 12; ++c)
          y += (cached ? cache.hd[c * 192 + threadIdx.x] : H[c]) *
               (HT)(S.zv[12 * b + c] + beta * pold[12 * b + c]);
        for (int e = S.row_ptr[b]; e < S.row_ptr[b + 1]; ++e) {
          const int nb = S.col_body[e];
          const HT* blk = (cached && e - cache.e0 < cache.n_off)
                              ? cache.off[e - cache.e0]
                              : Ho + 144 * (size_t)S.col_slot[e];
          if (S.col_trans[e]) {
            for (int c = 0; c < 12; ++c)
              y += blk[12 * c + row] *
                   (HT)(S.zv[12 * nb + c] + beta * pold[12 * nb + c]);
          } else {
            for (int c = 0; c < 12; ++c)
              y += blk[12 * row + c] *
                   (HT)(S.zv[12 * nb + c] + beta * pold[12 * nb + c]);
          }
        }
        const double pk = S.zv[12 * b + row] + beta * pold[12 * b + row];
        pnew[12 * b + row] = pk;
        S.Ap[12 * b + row] = (double)y;
        pap = pk * (double)y;
      }
      const double v[1] = {pap};
      const int off[1] = {OFF_ACC + (int)sizeof(double) * (4 * (it & 3) + 1)};
      group_add<1>(gs, gr, S.B, S.bprob, p, act, v, ps, off);
    }
    grid_sync(&S.cnt->bar, nblk, gen, &S.cnt->err);
    /* phase B */
    if (blockIdx.x == 0)
      for (int t = threadIdx.x; t < 4 * NP; t += blockDim.x)
        if ((t & 3) != 3) ps[t >> 2].acc[4 * ((it + 2) & 3) + (t & 3)] = 0.0;
    for (int gr = blockIdx.x; gr < ngroups; gr += nblk) {
      const int b = gr * 16 + lb;
      const int p = b < S.B ? S.bprob[b] : 0;
      const bool act = b < S.B && !pdone[p];
      double rv = 0.0;
      if (act) {
        const double* acc = ps[p].acc;
        const double alpha = ld_acq(acc + 4 * (it & 3)) / ld_acq(acc + 4 * (it & 3) + 1);
        const int o = 12 * b + row;
        S.dq[o] += alpha * pnew[o];
        rv = S.r[o] - alpha * S.Ap[o];
        S.r[o] = rv;
      }
      rloc[lb][row] = rv;
      __syncthreads();
      double z = 0.0;
      if (act) {
        HT zz = 0;
        for (int c = 0; c < 12; ++c)
          zz += (cached ? cache.pi[c * 192 + threadIdx.x] : Pi[144 * b + 12 * row + c]) *
                (HT)rloc[lb][c];
        z = (double)zz;
        S.zv[12 * b + row] = z;
      }
      const double v[2] = {rv * z, rv * rv};
      const int off[2] = {OFF_ACC + (int)sizeof(double) * (4 * ((it + 1) & 3) + 0),
                          OFF_ACC + (int)sizeof(double) * (4 * ((it + 1) & 3) + 2)};
      group_add<2>(gs, gr, S.B, S.bprob, p, act, v, ps, off);
    }
    grid_sync(&S.cnt->bar, nblk, gen, &S.cnt->err);
    /* the same convergence decision in every block */
    if (threadIdx.x == 0) any_active = 0;
    __syncthreads();
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
      if (pdone[p]) continue;
      const double rr = ld_acq(&ps[p].acc[4 * ((it + 1) & 3) + 2]);
      if (rr <= eta * eta * ld_acq(&ps[p].bb)) {
        pdone[p] = 1;
        if (blockIdx.x == 0) ps[p].pcg_iters = it + 1;
      } else {
        any_active = 1;
      }
    }
    __syncthreads();
    const int more = any_active;
    __syncthreads();
    if (S.cnt->err || !more) { ++it; break; }
  }
  if (blockIdx.x == 0) {
    for (int p = threadIdx.x; p < NP; p += blockDim.x)
      if (!pdone[p]) ps[p].pcg_iters = it;
    if (threadIdx.x == 0) S.cnt->pcg_iters = it;
  }
}

/* Block-Jacobi PCG with problem-local synchronisation (one block per
 * 16-body group, all blocks co-resident).  The textbook recurrences as
 * above, but no grid-wide barrier and no global atomics: at the end of each
 * phase a block writes its per-problem partial sums (summed in a fixed
 * order) into its group's record and then publishes the phase number with
 * a release store; before the next phase it waits (acquire) for the
 * records of the groups that hold its problems, and every block of a
 * problem sums the same records in the same order, so all of them take the
 * same step sizes and stop together.  Problems progress independently,
 * a block leaves when its problems have converged, and the dot products
 * are deterministic. */
template <typename HT>
__device__ __forceinline__ void pcg_publish(PcgRec* rec, int ph, int nloc,
                                            const double (*part)[3], int plo = 0) {
  __syncthreads();
  if ((int)threadIdx.x < 3 * nloc)
    rec->val[threadIdx.x / 3][threadIdx.x % 3] = part[threadIdx.x / 3][threadIdx.x % 3];
  if (threadIdx.x == 0) rec->plo = plo;
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(&rec->gen, (unsigned long long)(ph + 1), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void pcg_wait(const PcgRec* recs, int glo, int ghi,
                                         int ph, int* err, int* lerr = nullptr) {
  bool polled = false;
  for (int g = glo + (int)threadIdx.x; g <= ghi; g += blockDim.x) {
    long spins = 0;
    polled = true;
    while (__hip_atomic_load(&recs[g].gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           (unsigned long long)(ph + 1)) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1L << 27)) {
        atomicOr(err, 1);
        if (lerr) *lerr = 1;
        break;
      }
    }
  }
  /* one acquire per polling thread after its flags were seen */
  if (polled) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
}

/* wait for the records of groups glo..ghi and sum, in a fixed order, the
 * partial sums of problem pg they carry (the first wavefront polls and
 * reads, one group per lane) */
__device__ __forceinline__ void pcg_wait_sum(const PcgRec* recs, int glo, int ghi,
                                             int ph, int pg, int* err,
                                             double* out, int* lerr = nullptr) {
  if (threadIdx.x < 64) {
    double sv[3] = {0.0, 0.0, 0.0};
    for (int g = glo + (int)threadIdx.x; g <= ghi; g += 64) {
      long spins = 0;
      while (__hip_atomic_load(&recs[g].gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
             (unsigned long long)(ph + 1)) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1L << 27)) {
          atomicOr(err, 1);
          if (lerr) *lerr = 1;
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      /* the first slot is read together with the group's first problem,
       * so a group whose first problem is pg costs one round trip */
      const int slot = pg - recs[g].plo;
      double v[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) v[k] = recs[g].val[0][k];
      if (slot != 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = recs[g].val[slot][k];
#pragma unroll
      for (int k = 0; k < 3; ++k) sv[k] += v[k];
    }
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int k = 0; k < 3; ++k) sv[k] += __shfl_xor(sv[k], o, 64);
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < 3; ++k) out[k] = sv[k];
  }
  __syncthreads();
}

template <typename HT>
__global__ __launch_bounds__(192) void k_pcg_local(Scene S, double eta, int max_it,
                                                   int goff) {
  const HT* __restrict__ Hd = (const HT*)S.Hdiag;
  const HT* __restrict__ Ho = (const HT*)S.Hoff;
  const HT* __restrict__ Pi = (const HT*)S.Pinv;
  __shared__ double rloc[16][12];
  __shared__ double vrow[3][192];
  __shared__ double vbody[3][16];
  __shared__ double part[16][3];
  __shared__ double tot[16][3];
  __shared__ double rz_cur[16], rz_old[16], alpha[16], bbl[16];
  __shared__ unsigned char ldone[16];
  __shared__ int s_glo, s_ghi, s_more;
  __shared__ int e_nb[PCG_OFF_CACHE], e_tr[PCG_OFF_CACHE];
  __shared__ PcgCache<HT> cache;
  const int ngroups = (S.B + 15) / 16;
  const int gr = goff + (int)blockIdx.x;
  if (gr >= ngroups) return;
  const int lb = threadIdx.x / 12, row = threadIdx.x % 12;
  const int g0 = gr * 16, gend = min(S.B, g0 + 16);
  const int b = g0 + lb;
  const bool real = b < S.B;
  const int plo = S.bprob[g0], phi = S.bprob[gend - 1];
  const int nloc = phi - plo + 1;
  const int p = real ? S.bprob[b] : phi;
  const int j = p - plo;
  ProbState* ps = S.ps;
  PcgRec* const rec0 = S.pcg_rec;
  PcgRec* const rec1 = S.pcg_rec + ngroups;
  if ((int)threadIdx.x < nloc)
    ldone[threadIdx.x] =
        (S.iter_mode == 0 || ps[plo + threadIdx.x].state == PS_NEWTON) ? 0 : 1;
  __syncthreads();
  const bool cached = pcg_cache_load(cache, S, Hd, Ho, Pi, ngroups, gr, true);
  if (!cached) __syncthreads();
  /* the group's block-row structure does not change during the solve */
  const int e0 = S.row_ptr[g0];
  for (int i = threadIdx.x; i < PCG_OFF_CACHE && e0 + i < S.row_ptr[gend]; i += blockDim.x) {
    e_nb[i] = S.col_body[e0 + i];
    e_tr[i] = S.col_trans[e0 + i];
  }
  const int e_lo = real ? S.row_ptr[b] : 0, e_hi = real ? S.row_ptr[b + 1] : 0;
  __syncthreads();
  auto hrow = [&](int c) -> HT {
    return cached ? cache.hd[c * 192 + threadIdx.x] : Hd[144 * b + 12 * row + c];
  };
  auto prow = [&](int c) -> HT {
    return cached ? cache.pi[c * 192 + threadIdx.x] : Pi[144 * b + 12 * row + c];
  };
  auto reduce = [&](int nv, const double* v) {
    for (int k = 0; k < nv; ++k) vrow[k][threadIdx.x] = v[k];
    __syncthreads();
    if (row == 0 && lb < 16) {
      for (int k = 0; k < nv; ++k) {
        double s = 0.0;
        for (int c = 0; c < 12; ++c) s += vrow[k][12 * lb + c];
        vbody[k][lb] = s;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < nloc) {
      const int q = plo + threadIdx.x;
      const int lo = max(S.prob_b0[q], g0) - g0, hi = min(S.prob_b1[q], gend - 1) - g0;
      for (int k = 0; k < nv; ++k) {
        double s = 0.0;
        for (int c = lo; c <= hi; ++c) s += vbody[k][c];
        part[threadIdx.x][k] = s;
      }
    }
  };
  auto totals = [&](const PcgRec* recs, int nv) {
    for (int q = 0; q < nloc; ++q) {
      if (ldone[q]) continue;
      const int pg = plo + q;
      const int ga = S.prob_b0[pg] / 16, gb = S.prob_b1[pg] / 16;
      if (threadIdx.x < 64) {
        double sv[3] = {0.0, 0.0, 0.0};
        for (int g = ga + (int)threadIdx.x; g <= gb; g += 64) {
          const int slot = pg - S.bprob[16 * g];
          for (int k = 0; k < nv; ++k) sv[k] += recs[g].val[slot][k];
        }
        for (int o = 32; o > 0; o >>= 1)
          for (int k = 0; k < nv; ++k) sv[k] += __shfl_xor(sv[k], o, 64);
        if (threadIdx.x == 0)
          for (int k = 0; k < nv; ++k) tot[q][k] = sv[k];
      }
    }
    __syncthreads();
  };
  auto range = [&]() {
    if (threadIdx.x == 0) {
      int lo = -1, hi = -2;
      for (int q = 0; q < nloc; ++q)
        if (!ldone[q]) {
          if (lo < 0) lo = S.prob_b0[plo + q] / 16;
          hi = S.prob_b1[plo + q] / 16;
        }
      s_glo = lo;
      s_ghi = hi;
      s_more = lo >= 0;
    }
    __syncthreads();
  };
  range();
  if (!s_more) return;
  int ph = 0;
  /* own rows of x, r, z, p and A p stay in registers; only z and p, which
   * the neighbouring rows read, go through memory */
  double xr = 0.0, rr = 0.0, zr = 0.0, pr = 0.0, apr = 0.0;
  const int o = 12 * b + row;
  /* phase 0: x = 0, r = b = -g, z = P^-1 r, p_{-1} = 0 */
  {
    const bool act = real && !ldone[j];
    rr = act ? -S.g[o] : 0.0;
    rloc[lb][row] = rr;
    __syncthreads();
    if (act) {
      HT zz = 0;
      for (int c = 0; c < 12; ++c) zz += prow(c) * (HT)rloc[lb][c];
      zr = (double)zz;
      S.zv[o] = zr;
      S.p1[o] = 0.0;
    }
    const double v[2] = {rr * zr, rr * rr};
    reduce(2, v);
    pcg_publish<HT>(rec0 + gr, ph, nloc, part);
    pcg_wait(rec0, s_glo, s_ghi, ph, &S.cnt->err);
    totals(rec0, 2);
    if ((int)threadIdx.x < nloc && !ldone[threadIdx.x]) {
      const int q = threadIdx.x, pg = plo + q;
      rz_cur[q] = tot[q][0];
      rz_old[q] = 1.0;
      bbl[q] = tot[q][1];
      const bool first = S.prob_b0[pg] >= g0; /* this group writes the stats */
      if (first) ps[pg].bb = bbl[q];
      if (!(bbl[q] > 0.0)) {
        ldone[q] = 1;
        if (first) ps[pg].pcg_iters = 0;
      }
    }
    __syncthreads();
  }
  int it = 0;
  for (it = 0; it < max_it; ++it) {
    range();
    if (!s_more || S.cnt->err) break;
    const double* pold = (it & 1) ? S.p0 : S.p1;
    double* pnew = (it & 1) ? S.p1 : S.p0;
    /* phase A: p = z + beta pold and A p */
    ++ph;
    {
      const bool act = real && !ldone[j];
      const double beta = act && it > 0 ? rz_cur[j] / rz_old[j] : 0.0;
      if (act) pr = zr + beta * pr;
      rloc[lb][row] = pr;
      __syncthreads();
      double pap = 0.0;
      if (act) {
        HT y = 0;
        for (int c = 0; c < 12; ++c) y += hrow(c) * (HT)rloc[lb][c];
        for (int e = e_lo; e < e_hi; ++e) {
          const int le = e - e0;
          const bool in = le < PCG_OFF_CACHE;
          const int nb = in ? e_nb[le] : S.col_body[e];
          const int tr = in ? e_tr[le] : S.col_trans[e];
          const HT* blk = (cached && le < cache.n_off) ? cache.off[le]
                                                       : Ho + 144 * (size_t)S.col_slot[e];
          const int st = tr ? 12 : 1, sc = tr ? 1 : 12;
          for (int c = 0; c < 12; ++c)
            y += blk[sc * row + st * c] *
                 (HT)(S.zv[12 * nb + c] + beta * pold[12 * nb + c]);
        }
        pnew[o] = pr;
        apr = (double)y;
        pap = pr * apr;
      }
      const double v[1] = {pap};
      reduce(1, v);
      PcgRec* recs = (ph & 1) ? rec1 : rec0;
      pcg_publish<HT>(recs + gr, ph, nloc, part);
      pcg_wait(recs, s_glo, s_ghi, ph, &S.cnt->err);
      totals(recs, 1);
      if ((int)threadIdx.x < nloc && !ldone[threadIdx.x])
        alpha[threadIdx.x] = rz_cur[threadIdx.x] / tot[threadIdx.x][0];
      __syncthreads();
    }
    /* phase B: x += alpha p, r -= alpha A p, z = P^-1 r */
    ++ph;
    {
      const bool act = real && !ldone[j];
      if (act) {
        const double a = alpha[j];
        xr += a * pr;
        rr -= a * apr;
      }
      rloc[lb][row] = act ? rr : 0.0;
      __syncthreads();
      if (act) {
        HT zz = 0;
        for (int c = 0; c < 12; ++c) zz += prow(c) * (HT)rloc[lb][c];
        zr = (double)zz;
        S.zv[o] = zr;
      }
      const double v[2] = {act ? rr * zr : 0.0, act ? rr * rr : 0.0};
      reduce(2, v);
      PcgRec* recs = (ph & 1) ? rec1 : rec0;
      pcg_publish<HT>(recs + gr, ph, nloc, part);
      pcg_wait(recs, s_glo, s_ghi, ph, &S.cnt->err);
      totals(recs, 2);
      if ((int)threadIdx.x < nloc && !ldone[threadIdx.x]) {
        const int q = threadIdx.x, pg = plo + q;
        rz_old[q] = rz_cur[q];
        rz_cur[q] = tot[q][0];
        if (tot[q][1] <= eta * eta * bbl[q]) {
          ldone[q] = 1;
          if (S.prob_b0[pg] >= g0) ps[pg].pcg_iters = it + 1;
        }
      }
      __syncthreads();
    }
  }
  if ((int)threadIdx.x < nloc && !ldone[threadIdx.x] && S.prob_b0[plo + threadIdx.x] >= g0)
    ps[plo + threadIdx.x].pcg_iters = it;
  /* the direction of every problem this block took part in */
  if (real && !(S.iter_mode != 0 && ps[p].state != PS_NEWTON)) S.dq[o] = xr;
  if (threadIdx.x == 0) atomicMax(&S.cnt->pcg_iters, it);
}

/* Problem-local PCG with one exchange per iteration, in the
 * Chronopoulos-Gear form: with u = P^-1 r and w = A u, both inner products
 * gamma = r.u and delta = w.u of an iteration come from one reduction,
 *   beta_i = gamma_i / gamma_{i-1},
 *   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
 *   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
 * and u and w are recomputed exactly from the new r every iteration (no
 * further recurrences).  The product w = A u needs u of the neighbouring
 * bodies; each block forms them itself, u_nb = P_nb^-1 (r_nb - alpha(w_nb +
 * beta s_nb)), from the r, w and s the neighbours published in the previous
 * phase, so one publish-and-wait per iteration carries both the vectors and
 * the partial sums.  Vectors read by other blocks are double-buffered by
 * phase; own rows stay in registers. */
#define PCG_NB_MAX 96
/* sum over the wavefront by DPP moves of the two halves of a double: row
 * shifts by 1, 2, 4, 8 (an inclusive scan within each row of 16 lanes),
 * then the last lane of row 0 into rows 1 and 3 and the last lane of row 1
 * into rows 2 and 3; lane 63 ends with the total.  Lanes a shift reads
 * from outside the row contribute zero. */
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ void wave_sum_dpp(double& x) {
  x += dpp_move<0x111, 0xF>(x); /* row_shr:1 */
  x += dpp_move<0x112, 0xF>(x); /* row_shr:2 */
  x += dpp_move<0x114, 0xF>(x); /* row_shr:4 */
  x += dpp_move<0x118, 0xF>(x); /* row_shr:8 */
  x += dpp_move<0x142, 0xA>(x); /* row_bcast:15 into rows 1, 3 */
  x += dpp_move<0x143, 0xC>(x); /* row_bcast:31 into rows 2, 3 */
}
template <typename HT>
__global__ __launch_bounds__(192) void k_pcg_cg1(Scene S, double eta, int max_it,
                                                 int goff) {
  const HT* __restrict__ Hd = (const HT*)S.Hdiag;
  const HT* __restrict__ Ho = (const HT*)S.Hoff;
  const HT* __restrict__ Pi = (const HT*)S.Pinv;
  __shared__ double rloc[16][12];
  __shared__ double uloc[16][12];
  __shared__ double rnb[PCG_NB_MAX][12];
  __shared__ double unb[PCG_NB_MAX][12];
  __shared__ double wsum[3][16][3];
  __shared__ double part[16][3];
  __shared__ double tot[16][3];
  __shared__ double gam[16], gam_old[16], alp_old[16], bbl[16], alp[16], bet[16];
  __shared__ unsigned char ldone[16];
  __shared__ int s_glo, s_ghi, s_more, s_single;
  __shared__ int e_nb[PCG_OFF_CACHE], e_q[PCG_OFF_CACHE];
  __shared__ unsigned char e_tr[PCG_OFF_CACHE];
  /* per local problem: its bodies in this group (lo..hi), its groups
   * (ga..gb), whether this group holds its first body */
  __shared__ int q_lo[16], q_hi[16], q_ga[16], q_gb[16];
  __shared__ unsigned char q_first[16];
  __shared__ int s_err;
  __shared__ HT e_pi[PCG_OFF_CACHE][144];
  __shared__ PcgCache<HT> cache;
  const int ngroups = (S.B + 15) / 16;
  const int gr = goff + (int)blockIdx.x;
  if (gr >= ngroups) return;
  /* with labelled components only the bodies of components larger than
   * DIR_MAX are solved here (the others directly); none: nothing to do */
  const bool planned = S.cnt->plan != 0;
  if (planned && S.cnt->n_big == 0) return;
  auto in_pcg = [&](int body) { return !planned || S.bmode[body] == 2; };
  const int lb = threadIdx.x / 12, row = threadIdx.x % 12;
  const int g0 = gr * 16, gend = min(S.B, g0 + 16);
  const int b = g0 + lb;
  const bool real = b < S.B;
  const int plo = S.bprob[g0], phi = S.bprob[gend - 1];
  const int nloc = phi - plo + 1;
  const int p = real ? S.bprob[b] : phi;
  const int j = p - plo;
  ProbState* ps = S.ps;
  PcgRec* const rec0 = S.pcg_rec;
  PcgRec* const rec1 = S.pcg_rec + ngroups;
  const long n12 = 12L * S.B;
  double* const Rb[2] = {S.pw, S.pw + n12};
  double* const Wb[2] = {S.pw + 2 * n12, S.pw + 3 * n12};
  double* const Sb[2] = {S.pw + 4 * n12, S.zv};
  if ((int)threadIdx.x < nloc) {
    const int q = threadIdx.x, pg = plo + q;
    ldone[q] = (S.iter_mode == 0 || ps[pg].state == PS_NEWTON) ? 0 : 1;
    const int b0 = S.prob_b0[pg], b1 = S.prob_b1[pg];
    q_lo[q] = max(b0, g0) - g0;
    q_hi[q] = min(b1, gend - 1) - g0;
    q_ga[q] = b0 / 16;
    q_gb[q] = b1 / 16;
    q_first[q] = b0 >= g0 ? 1 : 0;
  }
  if (threadIdx.x == 0) s_err = S.cnt->err;
  __syncthreads();
  const bool cached = pcg_cache_load(cache, S, Hd, Ho, Pi, ngroups, gr, true);
  if (!cached) __syncthreads();
  const int e0 = S.row_ptr[g0], e_end = S.row_ptr[gend];
  const int e_lo = real ? S.row_ptr[b] : 0, e_hi = real ? S.row_ptr[b + 1] : 0;
  /* the neighbours of the first block-row entries: body, problem, inverse */
  const int n_ec = min(e_end - e0, PCG_OFF_CACHE);
  for (int i = threadIdx.x; i < n_ec; i += blockDim.x) {
    const int nb = S.col_body[e0 + i];
    e_nb[i] = nb;
    e_q[i] = S.bprob[nb] - plo;
    e_tr[i] = (unsigned char)S.col_trans[e0 + i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_ec * 144; i += blockDim.x)
    e_pi[i / 144][i % 144] = Pi[144 * e_nb[i / 144] + i % 144];
  __syncthreads();
  auto hrow = [&](int c) -> HT {
    return cached ? cache.hd[c * 192 + threadIdx.x] : Hd[144 * b + 12 * row + c];
  };
  auto prow = [&](int c) -> HT {
    return cached ? cache.pi[c * 192 + threadIdx.x] : Pi[144 * b + 12 * row + c];
  };
  /* the group's partial sums per local problem: a problem's rows are one
   * run of threads, so a segmented tree sum over each wavefront (a lane
   * adds the lane o above it while that lane is in its run) leaves the
   * run's sum in its first lane of the wavefront; then the (at most three)
   * wavefront sums of each problem, in wavefront order */
  const int seg_lo = real ? 12 * q_lo[j] : threadIdx.x;
  const int seg_hi = real ? 12 * q_hi[j] + 11 : threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  auto reduce = [&](const double* v) {
    double x0 = v[0], x1 = v[1], x2 = v[2];
    if (nloc == 1) {
      /* one problem in the group: plain wavefront sums by DPP (the total
       * lands in lane 63), then the three wavefronts' in order */
      wave_sum_dpp(x0);
      wave_sum_dpp(x1);
      wave_sum_dpp(x2);
      if (lane == 63) {
        wsum[wave][0][0] = x0;
        wsum[wave][0][1] = x1;
        wsum[wave][0][2] = x2;
      }
      lds_barrier();
      if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) part[0][c] = wsum[0][0][c] + wsum[1][0][c] + wsum[2][0][c];
      }
      return;
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double y0 = __shfl_down(x0, o, 64), y1 = __shfl_down(x1, o, 64),
                   y2 = __shfl_down(x2, o, 64);
      if (lane + o < 64 && (int)threadIdx.x + o <= seg_hi) {
        x0 += y0;
        x1 += y1;
        x2 += y2;
      }
    }
    if (real && (int)threadIdx.x == max(seg_lo, 64 * wave)) {
      wsum[wave][j][0] = x0;
      wsum[wave][j][1] = x1;
      wsum[wave][j][2] = x2;
    }
    lds_barrier();
    if ((int)threadIdx.x < nloc) {
      const int q = threadIdx.x;
      const int lo = 12 * q_lo[q], hi = 12 * q_hi[q] + 11;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int w = 0; w < 3; ++w)
        if (lo <= 64 * w + 63 && hi >= 64 * w) {
          s0 += wsum[w][q][0];
          s1 += wsum[w][q][1];
          s2 += wsum[w][q][2];
        }
      part[q][0] = s0;
      part[q][1] = s1;
      part[q][2] = s2;
    }
  };
  auto totals = [&](const PcgRec* recs) {
    for (int q = 0; q < nloc; ++q) {
      if (ldone[q]) continue;
      const int pg = plo + q;
      const int ga = q_ga[q], gb = q_gb[q];
      if (threadIdx.x < 64) {
        double sv[3] = {0.0, 0.0, 0.0};
        for (int g = ga + (int)threadIdx.x; g <= gb; g += 64) {
          const int slot = pg - recs[g].plo;
          for (int k = 0; k < 3; ++k) sv[k] += recs[g].val[slot][k];
        }
        for (int o = 32; o > 0; o >>= 1)
          for (int k = 0; k < 3; ++k) sv[k] += __shfl_xor(sv[k], o, 64);
        if (threadIdx.x == 0)
          for (int k = 0; k < 3; ++k) tot[q][k] = sv[k];
      }
    }
    lds_barrier();
  };
  auto range = [&]() {
    if (threadIdx.x == 0) {
      int lo = -1, hi = -2, n = 0, one = -1;
      for (int q = 0; q < nloc; ++q)
        if (!ldone[q]) {
          if (lo < 0) lo = q_ga[q];
          hi = q_gb[q];
          ++n;
          one = q;
        }
      s_glo = lo;
      s_ghi = hi;
      s_more = lo >= 0;
      s_single = n == 1 ? one : -1;
    }
    lds_barrier();
  };
  /* the same from wavefront 0 after a control step, from a ballot of the
   * problems still running (lanes below nloc) */
  auto range_w0 = [&](bool live) {
    const unsigned long long m = __ballot(live);
    if (threadIdx.x == 0) {
      if (m == 0ull) {
        s_glo = -1;
        s_ghi = -2;
        s_more = 0;
        s_single = -1;
      } else {
        const int lo = __ffsll((long long)m) - 1, hi = 63 - __clzll((long long)m);
        s_glo = q_ga[lo];
        s_ghi = q_gb[hi];
        s_more = 1;
        s_single = __popcll(m) == 1 ? lo : -1;
      }
    }
  };
  /* one phase: from the own new residual rn (registers) and the
   * neighbours' published vectors, u = P^-1 r for the own body and its
   * neighbours, w = A u, publish r, w, s and the partial sums */
  double xr = 0.0, rr = 0.0, pr = 0.0, sr = 0.0, wr = 0.0;
  const int o = 12 * b + row;
  auto phase = [&](int ph, bool init) {
    const int cur = (ph - 1) & 1, nxt = ph & 1; /* buffers read / written */
    const bool act = real && !ldone[j];
    /* r and the previous s go out first: their stores complete while the
     * block works on, and only the barrier before the publication waits
     * for them */
    if (act) {
      Rb[nxt][o] = rr;
      Sb[(ph + 1) & 1][o] = sr; /* s of the previous iteration, read next phase */
    }
    /* own body: u = P^-1 r */
    rloc[lb][row] = act ? rr : 0.0;
    lds_barrier();
    double ur = 0.0;
    if (act) {
      HT uu = 0;
      for (int c = 0; c < 12; ++c) uu += prow(c) * (HT)rloc[lb][c];
      ur = (double)uu;
    }
    uloc[lb][row] = ur;
    HT y = 0;
    lds_barrier();
    if (act)
      for (int c = 0; c < 12; ++c) y += hrow(c) * (HT)uloc[lb][c];
    /* neighbours, in chunks of PCG_NB_MAX block-row entries of the group */
    for (int c0 = e0; c0 < e_end; c0 += PCG_NB_MAX) {
      const int c1 = min(e_end, c0 + PCG_NB_MAX);
      /* r of each entry's neighbour (alpha, beta of that body's problem) */
      for (int t = threadIdx.x; t < 12 * (c1 - c0); t += blockDim.x) {
        const int le = t / 12, c = t % 12, e = c0 + le, lc = e - e0;
        const int nb = lc < n_ec ? e_nb[lc] : S.col_body[e];
        const int q = lc < n_ec ? e_q[lc] : S.bprob[nb] - plo;
        double v = 0.0;
        if (q >= 0 && q < nloc && !ldone[q]) {
          const int on = 12 * nb + c;
          v = init ? (in_pcg(nb) ? -S.g[on] : 0.0)
                   : Rb[cur][on] - alp[q] * (Wb[cur][on] + bet[q] * Sb[(ph) & 1][on]);
        }
        rnb[le][c] = v;
      }
      lds_barrier();
      for (int t = threadIdx.x; t < 12 * (c1 - c0); t += blockDim.x) {
        const int le = t / 12, rw = t % 12, e = c0 + le, lc = e - e0;
        HT uu = 0;
        const HT* P = lc < n_ec ? &e_pi[lc][12 * rw] : Pi + 144 * S.col_body[e] + 12 * rw;
        for (int c = 0; c < 12; ++c) uu += P[c] * (HT)rnb[le][c];
        unb[le][rw] = (double)uu;
      }
      lds_barrier();
      if (act)
        for (int e = max(e_lo, c0); e < min(e_hi, c1); ++e) {
          const int le = e - c0, lc = e - e0;
          const HT* blk = (cached && lc < cache.n_off) ? cache.off[lc]
                                                      : Ho + 144 * (size_t)S.col_slot[e];
          const int tr = lc < n_ec ? e_tr[lc] : S.col_trans[e];
          const int st = tr ? 12 : 1, sc = tr ? 1 : 12;
          for (int c = 0; c < 12; ++c) y += blk[sc * row + st * c] * (HT)unb[le][c];
        }
      lds_barrier();
    }
    wr = (double)y;
    if (act) Wb[nxt][o] = wr;
    const double v[3] = {act ? rr * ur : 0.0, act ? wr * ur : 0.0, act ? rr * rr : 0.0};
    reduce(v);
    PcgRec* recs = (ph & 1) ? rec1 : rec0;
    pcg_publish<HT>(recs + gr, ph, nloc, part, plo);
    if (s_single >= 0) {
      /* one running problem: wait and sum in one pass over the records */
      pcg_wait_sum(recs, s_glo, s_ghi, ph, plo + s_single, &S.cnt->err, tot[s_single],
                   &s_err);
    } else {
      pcg_wait(recs, s_glo, s_ghi, ph, &S.cnt->err, &s_err);
      totals(recs);
    }
    return ur;
  };
  range();
  if (!s_more) return;
  /* phase 0: r = b = -g, x = p = s = 0, u = P^-1 r, w = A u */
  rr = real && !ldone[j] && in_pcg(b) ? -S.g[o] : 0.0;
  double ur = phase(0, true);
  if (threadIdx.x < 64) {
    bool live = false;
    if ((int)threadIdx.x < nloc && !ldone[threadIdx.x]) {
      const int q = threadIdx.x, pg = plo + q;
      gam[q] = tot[q][0];
      bbl[q] = tot[q][2];
      const bool first = q_first[q];
      if (first) ps[pg].bb = bbl[q];
      if (!(bbl[q] > 0.0)) {
        ldone[q] = 1;
        if (first) ps[pg].pcg_iters = 0;
      } else {
        alp[q] = gam[q] / tot[q][1];
        bet[q] = 0.0;
        live = true;
      }
    }
    range_w0(live);
  }
  lds_barrier();
  int it = 0;
  for (it = 0; it < max_it; ++it) {
    if (!s_more || s_err) break;
    const bool act = real && !ldone[j];
    if (act) {
      const double a = alp[j], be = bet[j];
      pr = ur + be * pr;
      sr = wr + be * sr;
      xr += a * pr;
      rr -= a * sr;
    }
    ur = phase(it + 1, false);
    /* gamma, delta, rho of the new residual: stop, or the next step sizes
     * (wavefront 0, which also finds the groups still running) */
    if (threadIdx.x < 64) {
      bool live = false;
      if ((int)threadIdx.x < nloc && !ldone[threadIdx.x]) {
        const int q = threadIdx.x, pg = plo + q;
        if (tot[q][2] <= eta * eta * bbl[q]) {
          ldone[q] = 1;
          if (q_first[q]) ps[pg].pcg_iters = it + 1;
        } else {
          gam_old[q] = gam[q];
          alp_old[q] = alp[q];
          gam[q] = tot[q][0];
          const double be = gam[q] / gam_old[q];
          bet[q] = be;
          alp[q] = gam[q] / (tot[q][1] - be * gam[q] / alp_old[q]);
          live = true;
        }
      }
      range_w0(live);
    }
    lds_barrier();
  }
  if ((int)threadIdx.x < nloc && !ldone[threadIdx.x] && q_first[threadIdx.x])
    ps[plo + threadIdx.x].pcg_iters = it;
  if (real && in_pcg(b) && !(S.iter_mode != 0 && ps[p].state != PS_NEWTON)) S.dq[o] = xr;
  if (threadIdx.x == 0) atomicMax(&S.cnt->pcg_iters, it);
}

/* Single-reduction (pipelined) block-Jacobi PCG, the same solve with one
 * grid barrier per iteration instead of two.  It follows the
 * Chronopoulos-Gear form of CG, where s = A p and the preconditioned
 * residual u = P^-1 r are carried by recurrences, so that both inner
 * products of an iteration, gamma = r.u and delta = w.u with w = A u, come
 * from the same reduction:
 *   beta_i = gamma_i / gamma_{i-1},
 *   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
 *   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s.
 * The preconditioned vectors are carried too: m = P^-1 w is formed once
 * per iteration, t = P^-1 s = m + beta t and u_{i+1} = u_i - alpha t_i, so
 * u_{i+1} of a neighbouring body is an element-wise expression of vectors
 * written before the last barrier and the product w_{i+1} = A u_{i+1}
 * needs no second barrier.  u, m and t are double-buffered by iteration
 * parity; r, s, w, p and x are read only by their own rows. */
__device__ __forceinline__ double cg_next_u(double u, double m, double tprev,
                                            double a, double be) {
  return __fma_rn(-a, __fma_rn(be, tprev, m), u);
}

template <typename HT>
__global__ __launch_bounds__(192) void k_pcg1(Scene S, double eta, int max_it) {
  const HT* __restrict__ Hd = (const HT*)S.Hdiag;
  const HT* __restrict__ Ho = (const HT*)S.Hoff;
  const HT* __restrict__ Pi = (const HT*)S.Pinv;
  __shared__ double rloc[16][12];
  __shared__ double gs[16][4];
  __shared__ unsigned char pdone[PCG_MAX_NP];
  __shared__ int any_active;
  __shared__ PcgCache<HT> cache;
  const unsigned nblk = gridDim.x;
  unsigned gen = 0;
  const int lb = threadIdx.x / 12, row = threadIdx.x % 12;
  const int ngroups = (S.B + 15) / 16;
  const int NP = S.NP;
  const long n12 = 12L * S.B;
  double* const W = S.pw;
  double* const Mv[2] = {S.pw + n12, S.pw + 2 * n12};
  double* const Tv[2] = {S.pw + 3 * n12, S.pw + 4 * n12};
  double* const Uv[2] = {S.zv, S.p1};
  double* const P = S.p0;
  double* const Sv = S.Ap;
  ProbState* ps = S.ps;
  const int OFF_ACC = (int)offsetof(ProbState, acc);
  const int OFF_BB = (int)offsetof(ProbState, bb);
  for (int p = threadIdx.x; p < NP; p += blockDim.x)
    pdone[p] = (S.iter_mode == 0 || ps[p].state == PS_NEWTON) ? 0 : 1;
  __syncthreads();
  const bool cached = pcg_cache_load(cache, S, Hd, Ho, Pi, ngroups, (int)blockIdx.x,
                                          (int)gridDim.x >= ngroups);
  auto hrow = [&](int b, int c) -> HT {
    return cached ? cache.hd[c * 192 + threadIdx.x] : Hd[144 * b + 12 * row + c];
  };
  auto prow = [&](int b, int c) -> HT {
    return cached ? cache.pi[c * 192 + threadIdx.x] : Pi[144 * b + 12 * row + c];
  };
  auto offblk = [&](int e) -> const HT* {
    return (cached && e - cache.e0 < cache.n_off) ? cache.off[e - cache.e0]
                                                  : Ho + 144 * (size_t)S.col_slot[e];
  };
  /* phase 0a: x = 0, r = b = -g, u_0 = P^-1 r, p = s = t_{-1} = 0 */
  for (int gr = blockIdx.x; gr < ngroups; gr += nblk) {
    const int b = gr * 16 + lb;
    const int p = b < S.B ? S.bprob[b] : 0;
    const bool act = b < S.B && !pdone[p];
    const int o = 12 * b + row;
    const double rv = act ? -S.g[o] : 0.0;
    rloc[lb][row] = rv;
    __syncthreads();
    if (act) {
      HT zz = 0;
      for (int c = 0; c < 12; ++c) zz += prow(b, c) * (HT)rloc[lb][c];
      S.dq[o] = 0.0;
      S.r[o] = rv;
      P[o] = 0.0;
      Sv[o] = 0.0;
      Tv[1][o] = 0.0;
      Uv[0][o] = (double)zz;
    }
    __syncthreads();
  }
  grid_sync(&S.cnt->bar, nblk, gen, &S.cnt->err);
  /* phase 0b: w_0 = A u_0, m_0 = P^-1 w_0 and the dots of iteration 0 */
  for (int gr = blockIdx.x; gr < ngroups; gr += nblk) {
    const int b = gr * 16 + lb;
    const int p = b < S.B ? S.bprob[b] : 0;
    const bool act = b < S.B && !pdone[p];
    const int o = 12 * b + row;
    double y = 0.0, uo = 0.0, rv = 0.0;
    if (act) {
      HT acc = 0;
      for (int c = 0; c < 12; ++c) acc += hrow(b, c) * (HT)Uv[0][12 * b + c];
      for (int e = S.row_ptr[b]; e < S.row_ptr[b + 1]; ++e) {
        const int nb = S.col_body[e];
        const HT* blk = offblk(e);
        const int st = S.col_trans[e] ? 12 : 1, sc = S.col_trans[e] ? 1 : 12;
        for (int c = 0; c < 12; ++c)
          acc += blk[sc * row + st * c] * (HT)Uv[0][12 * nb + c];
      }
      y = (double)acc;
      W[o] = y;
      uo = Uv[0][o];
      rv = S.r[o];
    }
    rloc[lb][row] = y;
    __syncthreads();
    if (act) {
      HT mm = 0;
      for (int c = 0; c < 12; ++c) mm += prow(b, c) * (HT)rloc[lb][c];
      Mv[0][o] = (double)mm;
    }
    const double v[4] = {rv * uo, y * uo, rv * rv, rv * rv};
    const int off[4] = {OFF_ACC + 0, OFF_ACC + (int)sizeof(double),
                        OFF_ACC + 2 * (int)sizeof(double), OFF_BB};
    group_add<4>(gs, gr, S.B, S.bprob, p, act, v, ps, off);
  }
  grid_sync(&S.cnt->bar, nblk, gen, &S.cnt->err);
  int it = 0;
  for (it = 0;; ++it) {
    /* the same decision in every block: converged (|r_it| <= eta |b|, or
     * a zero right-hand side), out of iterations, or still running */
    if (threadIdx.x == 0) any_active = 0;
    __syncthreads();
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
      if (pdone[p]) continue;
      const double* acc = ps[p].acc + 4 * (it & 3);
      const double bb = ld_acq(&ps[p].bb);
      if (!(bb > 0.0) || ld_acq(acc + 2) <= eta * eta * bb || it >= max_it) {
        pdone[p] = 1;
        if (blockIdx.x == 0) ps[p].pcg_iters = it;
        continue;
      }
      any_active = 1;
      if (blockIdx.x == 0) {
        const double g = ld_acq(acc), d = ld_acq(acc + 1);
        double a = g / d;
        if (it > 0) {
          const double be = g / ld_acq(ps[p].acc + 4 * ((it - 1) & 3));
          a = g / (d - be * g / ld_acq(&ps[p].cg_alpha[(it - 1) & 1]));
        }
        ps[p].cg_alpha[it & 1] = a;
        /* the slot of iteration it + 2 is accumulated in the next pass */
        for (int k = 0; k < 3; ++k) ps[p].acc[4 * ((it + 2) & 3) + k] = 0.0;
      }
    }
    __syncthreads();
    const int more = any_active;
    __syncthreads();
    if (!more || S.cnt->err) break;
    const int cur = it & 1, nxt = cur ^ 1;
    for (int gr = blockIdx.x; gr < ngroups; gr += nblk) {
      const int b = gr * 16 + lb;
      const int p = b < S.B ? S.bprob[b] : 0;
      const bool act = b < S.B && !pdone[p];
      const int o = 12 * b + row;
      double y = 0.0, u1 = 0.0, rv = 0.0;
      if (act) {
        const double* acc = ps[p].acc + 4 * (it & 3);
        const double g = ld_acq(acc), d = ld_acq(acc + 1);
        double a = g / d, be = 0.0;
        if (it > 0) {
          be = g / ld_acq(ps[p].acc + 4 * ((it - 1) & 3));
          a = g / (d - be * g / ld_acq(&ps[p].cg_alpha[(it - 1) & 1]));
        }
        const double uo = Uv[cur][o], mo = Mv[cur][o], tp = Tv[nxt][o];
        const double pk = __fma_rn(be, P[o], uo);
        const double sk = __fma_rn(be, Sv[o], W[o]);
        P[o] = pk;
        Sv[o] = sk;
        Tv[cur][o] = __fma_rn(be, tp, mo);
        S.dq[o] = __fma_rn(a, pk, S.dq[o]);
        rv = __fma_rn(-a, sk, S.r[o]);
        S.r[o] = rv;
        u1 = cg_next_u(uo, mo, tp, a, be);
        Uv[nxt][o] = u1;
        /* w_{it+1} = A u_{it+1}, u of every body formed on the fly */
        HT accv = 0;
        for (int c = 0; c < 12; ++c) {
          const int oc = 12 * b + c;
          accv += hrow(b, c) * (HT)cg_next_u(Uv[cur][oc], Mv[cur][oc], Tv[nxt][oc], a, be);
        }
        for (int e = S.row_ptr[b]; e < S.row_ptr[b + 1]; ++e) {
          const int nb = S.col_body[e];
          const HT* blk = offblk(e);
          const int st = S.col_trans[e] ? 12 : 1, sc = S.col_trans[e] ? 1 : 12;
          for (int c = 0; c < 12; ++c) {
            const int oc = 12 * nb + c;
            accv += blk[sc * row + st * c] *
                    (HT)cg_next_u(Uv[cur][oc], Mv[cur][oc], Tv[nxt][oc], a, be);
          }
        }
        y = (double)accv;
        W[o] = y;
      }
      rloc[lb][row] = y;
      __syncthreads();
      if (act) {
        HT mm = 0;
        for (int c = 0; c < 12; ++c) mm += prow(b, c) * (HT)rloc[lb][c];
        Mv[nxt][o] = (double)mm;
      }
      const double v[3] = {rv * u1, y * u1, rv * rv};
      const int slot = OFF_ACC + (int)sizeof(double) * 4 * ((it + 1) & 3);
      const int off[3] = {slot, slot + (int)sizeof(double),
                          slot + 2 * (int)sizeof(double)};
      group_add<3>(gs, gr, S.B, S.bprob, p, act, v, ps, off);
    }
    grid_sync(&S.cnt->bar, nblk, gen, &S.cnt->err);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) S.cnt->pcg_iters = it;
}

/* ================================================================== */
/* S8 Newton stop                                                      */
/* ================================================================== */
/* reduce a value over the wave when every lane belongs to the same
 * problem, then one atomic per wave; otherwise one atomic per lane */
__device__ __forceinline__ bool wave_uniform(int p) {
  return __ballot(p == __shfl(p, 0, 64)) == __ballot(true);
}

__device__ __forceinline__ void ctrl_newton_check(const Scene& S, ProbState& P,
                                                  Counters& c0);
__device__ __forceinline__ bool last_workgroup(unsigned* ctr, unsigned n);
/* |dq|_inf per problem over workgroup blk of nblk (256 bodies each) into
 * the counter block c0, then the Newton stop test in the last of them */
__device__ void newton_stop_test(const Scene& S, Counters* c0, int blk, int nblk) {
  const int b = blk * blockDim.x + threadIdx.x;
  const bool act = b < S.B;
  const int p = act ? S.bprob[b] : -1;
  double v = 0.0;
  if (act)
    for (int i = 0; i < 12; ++i) v = fmax(v, fabs(S.dq[12 * b + i]));
  const bool uni = wave_uniform(p); /* inactive lanes make it non-uniform */
  if (uni) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    if ((threadIdx.x & 63) == 0) {
      atomic_max_pos(&S.ps[p].max_dq, v);
      atomic_max_pos(&c0->max_dq, v);
    }
  } else if (act) {
    atomic_max_pos(&S.ps[p].max_dq, v);
    atomic_max_pos(&c0->max_dq, v);
  }
  if (last_workgroup(&c0->fin[0], (unsigned)nblk))
    for (int q = threadIdx.x; q < S.NP; q += blockDim.x)
      ctrl_newton_check(S, S.ps[q], *c0);
}

/* |dq|_inf per problem; with_ctrl: then the Newton stop test */
__global__ void k_dq_norm(Scene S, int with_ctrl) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = b < S.B;
  const int p = act ? S.bprob[b] : -1;
  double v = 0.0;
  if (act)
    for (int i = 0; i < 12; ++i) v = fmax(v, fabs(S.dq[12 * b + i]));
  const bool uni = wave_uniform(p); /* inactive lanes make it non-uniform */
  if (uni) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    if ((threadIdx.x & 63) == 0) {
      atomic_max_pos(&S.ps[p].max_dq, v);
      atomic_max_pos(&S.cnt->max_dq, v);
    }
  } else if (act) {
    atomic_max_pos(&S.ps[p].max_dq, v);
    atomic_max_pos(&S.cnt->max_dq, v);
  }
  if (with_ctrl && last_workgroup(&S.cnt[0].fin[0], gridDim.x))
    for (int q = threadIdx.x; q < S.NP; q += blockDim.x)
      ctrl_newton_check(S, S.ps[q], S.cnt[0]);
}

/* ================================================================== */
/* S9 CCD                                                              */
/* ================================================================== */
__device__ __forceinline__ void ctrl_first_trial(ProbState& P);
/* a PT or EE candidate's points at q and their motion over dq */
__device__ __forceinline__ int candidate_geom(const Scene& S, int t, int npt, double* x,
                                              double* dx, int* prob) {
  const int* c = t < npt ? S.cand_pt + 3 * t : S.cand_ee + 3 * (t - npt);
  const int kind = t < npt ? C_PT : C_EE;
  int vid[4];
  pair_vertices(S, kind, c[0], c[1], vid);
  for (int k = 0; k < 4; ++k) {
    int v = vid[k], b = S.vbody[v];
    double b0 = S.xbar[v], b1 = S.xbar[S.V + v], b2 = S.xbar[2 * S.V + v];
    xform(S.q + 12 * b, b0, b1, b2, x + 3 * k);
    xform(S.dq + 12 * b, b0, b1, b2, dx + 3 * k);
  }
  *prob = S.bprob[S.vbody[vid[0]]];
  return kind;
}

/* TOI of candidate t of the list (PT, then EE, then PG), clamped to
 * [0, 1]; *prob receives its problem.  With use_bound the advance of a PT
 * or EE pair stops once it passes the smallest TOI its problem has reached
 * (a lower bound of the pair's TOI that cannot lower the minimum).  false:
 * the pair's ACCD continues in blocked steps from the anchor (*toi, *da) */
__device__ __forceinline__ bool candidate_toi(const Scene& S, int t, int npt, int nee,
                                              bool use_bound, int* prob, double* toi,
                                              double* da) {
  *toi = 1.0;
  if (t < npt + nee) {
    double x[12], dx[12];
    const int kind = candidate_geom(S, t, npt, x, dx, prob);
    if (!accd_begin(kind, x, dx, 1.0, use_bound ? &S.ps[*prob].min_toi : nullptr, toi, da))
      return false;
  } else {
    int v = S.cand_pg[t - npt - nee], b = S.vbody[v];
    double b0 = S.xbar[v], b1 = S.xbar[S.V + v], b2 = S.xbar[2 * S.V + v];
    double x[3], dx[3];
    xform(S.q + 12 * b, b0, b1, b2, x);
    xform(S.dq + 12 * b, b0, b1, b2, dx);
    if (dx[1] < 0.0) *toi = (1.0 - ACCD_S) * (x[1] - S.ground_y) / (-dx[1]);
    *prob = S.bprob[b];
  }
  *toi = fmax(fmin(*toi, 1.0), 0.0);
  return true;
}

/* CCD of the swept candidates, first phase: a lane per candidate takes the
 * one-point ACCD steps; a pair still advancing goes to the long list (a
 * count beyond cap_long redoes the pass with a larger list).  toi_out:
 * every candidate's own TOI (no early stop) for the hooks, else the
 * problems' minima */
__global__ __launch_bounds__(256) void k_ccd(Scene S, double* toi_out) {
  const int npt = min(S.cnt->n_pt, S.cap_pt);
  const int nee = min(S.cnt->n_ee, S.cap_ee);
  const int npg = min(S.cnt->n_pg, S.cap_pg);
  const int tot = npt + nee + npg;
  double tmin = 1.0;
  const int lane = threadIdx.x & 63;
  /* whole workgroups step through the list together, so every lane of a
   * wavefront takes part in the reductions below */
  for (int base = blockIdx.x * blockDim.x; base < tot; base += gridDim.x * blockDim.x) {
    const int t = base + threadIdx.x;
    int prob = -1;
    double toi = 1.0, da = 0.0;
    bool fin = true;
    if (t < tot) fin = candidate_toi(S, t, npt, nee, !toi_out, &prob, &toi, &da);
    const int k = wave_slot(!fin, &S.cnt->n_long);
    if (!fin) {
      if (k < S.cap_long) S.ccd_long[k] = CcdLong{toi, da, t, prob};
      toi = 1.0; /* the second phase takes the pair's TOI */
    }
    if (toi_out) {
      if (t < tot && fin) toi_out[t] = toi;
      continue;
    }
    tmin = fmin(tmin, toi);
    /* the wavefront's smallest TOI below 1 of its first such lane's problem
     * with one atomic; lanes of other problems add theirs directly */
    const int p = toi < 1.0 ? prob : -1;
    const unsigned long long m = __ballot(p >= 0);
    if (m) {
      const int first = __ffsll((unsigned long long)m) - 1;
      const int p0 = __shfl(p, first, 64);
      double v = p == p0 ? toi : 1.0;
      for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
      if (lane == first) atomic_min_pos(&S.ps[p0].min_toi, v);
      if (p >= 0 && p != p0) atomic_min_pos(&S.ps[p].min_toi, toi);
    }
  }
  for (int o = 32; o > 0; o >>= 1) tmin = fmin(tmin, __shfl_down(tmin, o, 64));
  /* waves without a TOI below 1 leave the minimum alone (its readers take
   * min(1, .)), which keeps empty waves off the shared counter */
  if ((threadIdx.x & 63) == 0 && tmin < 1.0)
    atomic_min_pos(&S.cnt->min_toi, fmax(tmin, 0.0));
}

/* CCD, second phase: one wavefront per pair of the long list.  From the
 * anchor (t, da) the lanes evaluate the points t + j delta, j = 1..64,
 * delta = 0.5 da / lp; the step goes to the last point j such that every
 * point up to j keeps the gap and every point before j keeps the distance
 * at least 0.6 da (so the distance stays above 0.6 da - lp delta = 0.1 da
 * along each segment), and the point reached is the next anchor.  A pair
 * that slides at a small distance, or closes it slowly, advances up to 64
 * half steps at once.  Then, in the last workgroup, the controller's first
 * trial step (with_ctrl). */
#define CCD_LONG_BLOCKS 64
__global__ __launch_bounds__(256) void k_ccd_long(Scene S, int with_ctrl, double* toi_out) {
  const int npt = min(S.cnt->n_pt, S.cap_pt);
  const int nl = min(S.cnt->n_long, S.cap_long);
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * (blockDim.x >> 6);
  for (int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < nl; w += nw) {
    const CcdLong L = S.ccd_long[w];
    double x[12], dx[12], r[12], lp;
    int prob;
    const int kind = candidate_geom(S, L.cand, npt, x, dx, &prob);
    accd_setup(kind, dx, r, &lp);
    const double gap = ACCD_S * pair_dist(kind, x);
    double t = L.t, da = L.da;
    for (int it = ACCD_SERIAL_IT; it < ACCD_MAX_IT; it += ACCD_BLOCK) {
      const double delta = __ddiv_rn(__dmul_rn(0.5, da), lp);
      const double keep = __dmul_rn(0.6, da);
      const double tj = __dadd_rn(t, __dmul_rn((double)(lane + 1), delta));
      double xt[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) xt[i] = __dadd_rn(x[i], __dmul_rn(tj, r[i]));
      const double d = pair_dist(kind, xt);
      const unsigned long long fg = __ballot(d < gap), fc = __ballot(d < keep);
      const int A = fg ? __ffsll((long long)fg) : ACCD_BLOCK + 1;
      const int C = fc ? __ffsll((long long)fc) : ACCD_BLOCK;
      const int J = min(A - 1, C);
      if (J == 0) break;
      const double dJ = __shfl(d, J - 1, 64);
      t = __dadd_rn(t, __dmul_rn((double)J, delta));
      if (t > 1.0) {
        t = 1.0;
        break;
      }
      da = dJ;
      if (!toi_out && t >= bound_of(&S.ps[L.prob].min_toi)) break;
    }
    const double toi = fmax(fmin(t, 1.0), 0.0);
    if (lane == 0) {
      if (toi_out) {
        toi_out[L.cand] = toi;
      } else if (toi < 1.0) {
        atomic_min_pos(&S.ps[L.prob].min_toi, toi);
        atomic_min_pos(&S.cnt->min_toi, toi);
      }
    }
  }
  if (with_ctrl && last_workgroup(&S.cnt->fin[1], gridDim.x))
    for (int q = threadIdx.x; q < S.NP; q += blockDim.x) ctrl_first_trial(S.ps[q]);
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
/* device-driven Newton loop: line search trials, controllers          */
/* ================================================================== */
/* E(q + alpha_k dq) - E(q) for alpha_k = alpha_base 2^-k, k < LS_TRIALS,
 * per problem, over the bodies and swept candidates of problems that are
 * not done.  A wave whose elements belong to one problem sums them per
 * trial and keeps running sums across its grid-stride iterations; the
 * workgroup then adds its waves' sums with one atomic per trial and
 * problem (a wave straddling problems adds its lanes directly). */
__device__ __forceinline__ bool last_workgroup(unsigned* ctr, unsigned n);
__device__ __forceinline__ void ctrl_linesearch(const Scene& S, ProbState& P,
                                                const Counters& c0,
                                                const Counters& c1);
/* a trial energy term into its problem's sum: an FP64 atomic, or exact
 * in the deterministic mode */
__device__ __forceinline__ void de_add(const Scene& S, int p, int k, double v) {
  if (!S.det) {
    atomicAdd(&S.ps[p].dE[k], v);
    return;
  }
  det_word* w = S.det_de + ((size_t)p * LS_TRIALS + k) * (DET_W + 1);
  if (!det_add(w, v)) atomicAdd(w + DET_W, 1ull);
}

__global__ __launch_bounds__(256) void k_energy_multi(Scene S) {
  const int npt = min(S.cnt->n_pt, S.cap_pt);
  const int nee = min(S.cnt->n_ee, S.cap_ee);
  const int npg = min(S.cnt->n_pg, S.cap_pg);
  const int tot = S.B + npt + nee + npg;
  /* one lane per (element, trial): eight elements per wavefront */
  const int nwaves = (tot + 7) / 8;
  /* workgroups with elements (at least one, to run the controller) */
  const unsigned nwork = max(1u, min(gridDim.x, (unsigned)((nwaves + 3) / 4)));
  if (blockIdx.x >= nwork) return;
  const int lane = threadIdx.x & 63, k = lane & (LS_TRIALS - 1);
  /* lanes k < LS_TRIALS: running sum of trial k for problem accp */
  double acc = 0.0;
  int accp = -1;
  for (int w = blockIdx.x * 4 + threadIdx.x / 64; w < nwaves; w += gridDim.x * 4) {
    const int t = w * 8 + lane / LS_TRIALS;
    double e = 0.0;
    int prob = -1;
    if (t < S.B) {
      if (S.kind[t] == 0 && S.ps[S.bprob[t]].state != PS_DONE) {
        prob = S.bprob[t];
        e = body_energy(S, t, ldexp(S.ps[prob].alpha_base, -k), 0);
      }
    } else if (t < tot) {
      const int u = t - S.B;
      if (u < npt + nee) {
        const int* c = u < npt ? S.cand_pt + 3 * u : S.cand_ee + 3 * (u - npt);
        const int kind = u < npt ? C_PT : C_EE;
        int vid[4];
        pair_vertices(S, kind, c[0], c[1], vid);
        const int pb = S.bprob[S.vbody[vid[0]]];
        if (S.ps[pb].state != PS_DONE) {
          prob = pb;
          const double a = ldexp(S.ps[prob].alpha_base, -k);
          double x0[12], x1[12];
          for (int j = 0; j < 4; ++j) {
            vertex_pos(S, vid[j], x0 + 3 * j);
            vertex_pos_alpha(S, vid[j], a, x1 + 3 * j);
          }
          e = pair_energy_at(S, kind, c[0], c[1], vid, x1) -
              pair_energy_at(S, kind, c[0], c[1], vid, x0);
        }
      } else {
        const int v = S.cand_pg[u - npt - nee];
        const int pb = S.bprob[S.vbody[v]];
        if (S.ps[pb].state != PS_DONE) {
          prob = pb;
          double x0[3], x1[3];
          vertex_pos(S, v, x0);
          vertex_pos_alpha(S, v, ldexp(S.ps[prob].alpha_base, -k), x1);
          const double wv = pair_weight(S, &v, 1);
          e = wv * barrier_val(x1[1] - S.ground_y, S.dhat) -
              wv * barrier_val(x0[1] - S.ground_y, S.dhat);
        }
      }
    }
    if (S.det) {
      /* every term on its own into the exact sum: no floating-point
       * partial sum whose grouping follows the list order */
      if (prob >= 0) de_add(S, prob, k, e);
      continue;
    }
    /* per trial: the eight elements of the wavefront summed when they
     * belong to one problem (lanes k, k + 8, ... hold trial k) */
    const bool uni = wave_uniform(prob);
    if (uni) {
      if (prob >= 0) {
        for (int o = 32; o >= LS_TRIALS; o >>= 1) e += __shfl_down(e, o, 64);
        if (lane < LS_TRIALS) {
          if (accp != prob) {
            if (accp >= 0) de_add(S, accp, k, acc);
            acc = 0.0;
            accp = prob;
          }
          acc += e;
        }
      }
    } else if (prob >= 0) {
      de_add(S, prob, k, e);
    }
  }
  /* the four waves' running sums: lanes 0..LS_TRIALS-1 of a wave share
   * accp, so lane 0 publishes it */
  __shared__ double s_acc[4][LS_TRIALS];
  __shared__ int s_accp[4];
  const int wv = threadIdx.x >> 6;
  if (lane < LS_TRIALS) s_acc[wv][lane] = acc;
  if (lane == 0) s_accp[wv] = accp;
  __syncthreads();
  if (threadIdx.x < LS_TRIALS) {
    int p = -1;
    double sum = 0.0;
    for (int i = 0; i < 4; ++i) {
      const int pi = s_accp[i];
      if (pi < 0) continue;
      if (pi != p) {
        if (p >= 0) de_add(S, p, threadIdx.x, sum);
        p = pi;
        sum = 0.0;
      }
      sum += s_acc[i][threadIdx.x];
    }
    if (p >= 0) de_add(S, p, threadIdx.x, sum);
  }
  /* then every problem's line search decision (this scene's counters are
   * the swept block; the static block precedes it) */
  if (last_workgroup(&S.cnt->fin[2], nwork)) {
    const Counters* base = S.cnt - 1;
    for (int q = threadIdx.x; q < S.NP; q += blockDim.x) {
      ProbState& P = S.ps[q];
      if (S.det)
        for (int k = 0; k < LS_TRIALS; ++k) {
          det_word* w = S.det_de + ((size_t)q * LS_TRIALS + k) * (DET_W + 1);
          P.dE[k] = w[DET_W] ? INFINITY : det_value(w);
        }
      ctrl_linesearch(S, P, base[0], base[1]);
      if (P.state != PS_DONE) atomicAdd(&S.cnt->active, 1);
    }
  }
}

__device__ __forceinline__ bool static_overflow(const Counters& c, const Scene& S) {
  return c.n_bp > S.cap_bp || c.n_cp > S.cap_cp || c.n_pt > S.cap_pt ||
         c.n_ee > S.cap_ee || c.n_pg > S.cap_pg || c.n_act > S.cap_act;
}
__device__ __forceinline__ bool swept_overflow(const Counters& c, const Scene& S) {
  return c.n_bp > S.cap_bp || c.n_cp > S.cap_cp || c.n_pt > S.cap_pt ||
         c.n_ee > S.cap_ee || c.n_pg > S.cap_pg || c.n_long > S.cap_long;
}

__device__ __forceinline__ void ctrl_linesearch(const Scene& S, ProbState& P,
                                                const Counters& c0,
                                                const Counters& c1);

/* The controller of the device loop, one problem at a time.  It runs in
 * the last workgroup of the kernel that produces its input (that
 * workgroup sees every other one's atomics):
 *   start of a solve (its own kernel): every problem to the Newton state;
 *   after the PCG (last workgroup of the |dq| reduction): Newton stop
 *     |dq|_inf / (h l) < theta;
 *   after CCD (last workgroup of k_ccd): first trial step
 *     alpha_max = min(1, TOI), or the continuation of a line search;
 *   after the trial energies (last workgroup of k_energy_multi): accept the
 *     largest trial step with E(q + alpha dq) - E(q) <= 0, else continue
 *     halving or stop. */
__global__ void k_ctrl_start(Scene S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= S.NP) return;
  ProbState& P = S.ps[p];
  P.state = PS_NEWTON;
  P.status = -4; /* not converged yet */
  P.newton = P.halvings = P.ls_count = P.pcg_total = 0;
  P.min_alpha = 1.0;
  P.final_eps = 0.0;
  P.alpha_acc = 0.0;
  P.best_eps = INFINITY;
  P.since_best = P.newton32 = 0;
}
__device__ __forceinline__ void ctrl_newton_check(const Scene& S, ProbState& P,
                                                  Counters& c0) {
  if (P.state != PS_NEWTON || static_overflow(c0, S) || c0.err || c0.redo) return;
  P.newton += 1;
  P.pcg_total += P.pcg_iters;
  if (S.mixed) P.newton32 += 1;
  const double eps = __longlong_as_double((long long)P.max_dq) / (S.dt * P.scale);
  P.final_eps = eps;
  if (!isfinite(eps)) {
    P.state = PS_DONE;
    P.status = -4;
  } else if (eps < S.theta) {
    P.state = PS_DONE;
    P.status = 0;
  } else {
    if (eps <= 0.5 * P.best_eps) {
      P.best_eps = eps;
      P.since_best = 0;
    } else {
      P.since_best += 1;
    }
    /* a mixed-precision problem that stopped making progress asks the
     * host for FP64 Hessians (all problems of the scene switch) */
    if (S.mixed && (P.since_best >= MIXED_STALL_ITERS ||
                    P.newton >= S.mixed_switch))
      c0.want64 = 1;
  }
}
__device__ __forceinline__ void ctrl_first_trial(ProbState& P) {
  if (P.state == PS_NEWTON) {
    const double toi = __longlong_as_double((long long)P.min_toi);
    P.alpha_base = fmin(1.0, toi);
    P.ls_count = 0;
  }
}

/* whether this workgroup is the last of the grid to arrive at the counter
 * (which starts the kernel at zero); the last one may read what the others
 * accumulated with device-scope atomics (and stored) before arriving.  Only
 * the first n workgroups of the grid arrive (those with work: the arrivals
 * on one address are serialised, so idle workgroups leave without one).
 * The workgroup barrier by itself does not wait for outstanding vector
 * memory operations (a workgroup-scope release waits only for LDS here),
 * so every wavefront first waits until its own atomics and stores have
 * been acknowledged (vmcnt = 0), and thread 0 then arrives with an
 * agent-scope release (one L2 write-back per workgroup, for plain stores);
 * only the last workgroup acquires. */
__device__ __forceinline__ bool last_workgroup(unsigned* ctr, unsigned n) {
  __shared__ int s_last;
  /* s_waitcnt vmcnt(0), expcnt and lgkmcnt left at their maxima */
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev + 1 == n ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return false;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

__device__ __forceinline__ void ctrl_linesearch(const Scene& S, ProbState& P,
                                                const Counters& c0,
                                                const Counters& c1) {
  if (P.state == PS_DONE) return;
  const bool fresh = P.state == PS_NEWTON && P.ls_count == 0;
  if (fresh && (static_overflow(c0, S) || c0.err || c0.redo)) return; /* pass redone */
  if (swept_overflow(c1, S) || c1.err) {
    if (fresh) P.newton -= 1; /* the Newton iteration is redone */
    return;
  }
  /* trial j of this line search is alpha_max 2^-j, j = ls_count + k */
  int k = 0;
  while (k < LS_TRIALS && !(P.dE[k] <= 0.0)) ++k;
  if (k < LS_TRIALS && P.ls_count + k <= S.max_ls) {
    const double a = P.alpha_base * ldexp(1.0, -k);
    const int nh = P.ls_count + k;
    P.alpha_acc = a;
    P.halvings += nh;
    P.ls_count = 0;
    P.min_alpha = fmin(P.min_alpha, a);
    P.state = PS_NEWTON;
    if (nh > LS_FLOOR_HALVINGS && P.final_eps < 10.0 * S.theta) {
      /* a decrease found only this deep, this close to the tolerance, is
       * the rounding floor of the energy: converged with this step */
      P.state = PS_DONE;
      P.status = 0;
    } else if (P.newton >= S.max_newton) {
      P.state = PS_DONE;
      P.status = -4;
    }
  } else {
    P.ls_count += LS_TRIALS;
    if (P.ls_count > S.max_ls) {
      P.halvings += S.max_ls;
      P.state = PS_DONE;
      P.status = P.final_eps < 10.0 * S.theta ? 0 : -5;
    } else {
      P.state = PS_LINESEARCH;
      P.alpha_base *= ldexp(1.0, -LS_TRIALS);
    }
  }
}

/* q += alpha_acc dq for the bodies of problems that accepted a step; the
 * last workgroup then ends the pass: whether its lists can be taken over,
 * and both counter blocks into the host ring slot of this pass (slot =
 * pass number mod 2, the pass number kept on the device) */
__global__ void k_update_multi(Scene S, Counters* ring, unsigned* pass) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 12 * S.B) {
    const int b = t / 12;
    if (S.kind[b] == 0) {
      const double a = S.ps[S.bprob[b]].alpha_acc;
      if (a != 0.0) S.q[t] += a * S.dq[t];
    }
  }
  if (!last_workgroup(&S.cnt[0].fin[3], gridDim.x)) return;
  if (threadIdx.x == 0) {
    const Counters& c0 = S.cnt[0];
    Counters& c1 = S.cnt[1];
    c1.sweep_ok = (!static_overflow(c0, S) && !c0.err && !swept_overflow(c1, S) &&
                   !c1.err) ? 1 : 0;
  }
  __syncthreads();
  const unsigned slot = *pass & 1u;
  const int n = (int)(2 * sizeof(Counters) / sizeof(unsigned));
  const unsigned* src = (const unsigned*)S.cnt;
  unsigned* dst = (unsigned*)(ring + 2 * slot);
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  if (threadIdx.x == 0) *pass += 1u;
}

/* fresh PCG accumulators (the hooks' direct linear solve) */
__global__ void k_reset_pcg(Scene S) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) S.cnt->bar = 0;
  for (int i = t; i < 2 * ((S.B + 15) / 16); i += gridDim.x * blockDim.x)
    S.pcg_rec[i].gen = 0ull;
  if (t < S.NP) {
    ProbState& P = S.ps[t];
    P.bb = 0.0;
    P.pcg_iters = 0;
    for (int k = 0; k < 16; ++k) P.acc[k] = 0.0;
  }
}

/* start of a pass: fresh counter blocks, per-problem transients, and the
 * block-row counts of the PCG system */

/* ================================================================== */
/* consensus step over the replicas of shared bodies                   */
/* ================================================================== */
/* Alg. 1 start of a time step: z = q-tilde (the rho-weighted mean over the
 * replicas, which agree at a step start), u = 0; clears the residual
 * reductions.  One thread per (group, dof). */
__global__ void k_cons_init(Scene S, Cons C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < C.n_groups) C.r_body[t] = C.s_body[t] = 0ull;
  if (t < 2) C.red[t] = 0ull;
  if (t >= 12 * C.n_groups) return;
  const int g = t / 12, d = t % 12;
  double num = 0.0, den = 0.0;
  for (int j = C.grp_ptr[g]; j < C.grp_ptr[g + 1]; ++j) {
    const int k = C.grp_rep[j];
    num += S.rho[k] * S.qtilde[12 * C.rep_body[k] + d];
    den += S.rho[k];
  }
  const double z = num / den;
  C.zc[12 * g + d] = z;
  for (int j = C.grp_ptr[g]; j < C.grp_ptr[g + 1]; ++j) {
    const int k = C.grp_rep[j];
    S.z[12 * k + d] = z;
    S.u[12 * k + d] = 0.0;
  }
}

/* Eq. 6 (rho-weighted mean of q + u over the replicas), Eq. 7 (u += q - z),
 * and the residuals of Eqs. 9-10 per body and overall.  The new z becomes
 * every replica's target for the next local solve.  One thread per
 * (group, dof). */
__global__ void k_cons_update(Scene S, Cons C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double rmax = 0.0, sdev = 0.0;
  int g = 0;
  const bool act = t < 12 * C.n_groups;
  if (act) {
    g = t / 12;
    const int d = t % 12;
    double num = 0.0, den = 0.0;
    for (int j = C.grp_ptr[g]; j < C.grp_ptr[g + 1]; ++j) {
      const int k = C.grp_rep[j];
      num += S.rho[k] * (S.q[12 * C.rep_body[k] + d] + S.u[12 * k + d]);
      den += S.rho[k];
    }
    const double zn = num / den;
    sdev = fabs(zn - C.zc[12 * g + d]);
    C.zc[12 * g + d] = zn;
    for (int j = C.grp_ptr[g]; j < C.grp_ptr[g + 1]; ++j) {
      const int k = C.grp_rep[j];
      const double q = S.q[12 * C.rep_body[k] + d];
      rmax = fmax(rmax, fabs(q - zn));
      S.u[12 * k + d] += q - zn;
      S.z[12 * k + d] = zn;
    }
    atomic_max_pos(&C.r_body[g], rmax);
    atomic_max_pos(&C.s_body[g], sdev);
  }
  for (int o = 32; o > 0; o >>= 1) {
    rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
    sdev = fmax(sdev, __shfl_xor(sdev, o, 64));
  }
  if (__lane_id() == 0) {
    atomic_max_pos(&C.red[0], rmax);
    atomic_max_pos(&C.red[1], sdev);
  }
}

/* Eq. 12 per replica from its body's residuals, clamped to
 * [smin, smax] x rho0; the scaled dual follows as u rho_old / rho_new.
 * Clears the residual reductions for the next update. */
__global__ void k_cons_adapt(Scene S, Cons C) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= C.n_rep) return;
  const int g = C.rep_group[k];
  const double r = __longlong_as_double((long long)C.r_body[g]);
  const double sd = __longlong_as_double((long long)C.s_body[g]);
  const double old = S.rho[k];
  double nw = old;
  if (r > C.mu * sd) nw = C.tau * old;
  else if (sd > C.mu * r) nw = old / C.tau;
  nw = fmin(fmax(nw, C.smin * C.rho0[k]), C.smax * C.rho0[k]);
  const double f = old / nw;
  for (int d = 0; d < 12; ++d) S.u[12 * k + d] *= f;
  S.rho[k] = nw;
}
__global__ void k_cons_clear(Cons C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < C.n_groups) C.r_body[t] = C.s_body[t] = 0ull;
  if (t < 2) C.red[t] = 0ull;
}

/* Sec. 4.2: the merged state puts z on every replica */
__global__ void k_cons_merge(Scene S, Cons C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 12 * C.n_rep) return;
  const int k = t / 12, d = t % 12;
  S.q[12 * C.rep_body[k] + d] = C.zc[12 * C.rep_group[k] + d];
}
/* step toward the merged state: dq = z - q on replicas, 0 elsewhere; every
 * problem's CCD minimum starts at 1 */
/* every problem's CCD minimum starts unset (+inf) */
__global__ void k_reset_toi(Scene S) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < S.NP)
    S.ps[t].min_toi = (unsigned long long)__double_as_longlong(INFINITY);
}
__global__ void k_cons_dq_zero(Scene S) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 12 * S.B) S.dq[t] = 0.0;
  if (t < S.NP) S.ps[t].min_toi = (unsigned long long)__double_as_longlong(1.0);
}
__global__ void k_cons_dq(Scene S, Cons C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 12 * C.n_rep) return;
  const int k = t / 12, d = t % 12;
  const int o = 12 * C.rep_body[k] + d;
  S.dq[o] = C.zc[12 * C.rep_group[k] + d] - S.q[o];
}

/* gather every problem's state into the batch arrays (grid.y = problem) */
__global__ void k_gather(Scene S, const ProbCopy* pc, const double* scales) {
  const ProbCopy c = pc[blockIdx.y];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) S.ps[blockIdx.y].scale = scales[blockIdx.y];
  if (t >= 12 * c.nb) return;
  const int o = 12 * c.off + t;
  S.q[o] = c.q[t];
  S.qt[o] = c.qt[t];
  S.qtilde[o] = c.qtilde[t];
  S.qdot[o] = c.qdot[t];
}
__global__ void k_scatter(Scene S, const ProbCopy* pc) {
  const ProbCopy c = pc[blockIdx.y];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 12 * c.nb) return;
  c.q[t] = S.q[12 * c.off + t];
}

/* Interpenetration check for the initial state: counts edge-triangle
 * crossings between different bodies (segment strictly crossing the
 * triangle's plane and passing strictly inside its three edges, by signed
 * volumes), over every body pair and chunk pair whose boxes meet. */
__device__ __forceinline__ double orient3(const double* a, const double* b,
                                          const double* c, const double* d) {
  double u[3], v[3], w[3], n[3];
  for (int i = 0; i < 3; ++i) {
    u[i] = b[i] - a[i];
    v[i] = c[i] - a[i];
    w[i] = d[i] - a[i];
  }
  cross3(u, v, n);
  return dot3(n, w);
}

__global__ __launch_bounds__(256) void k_crossings(Scene S) {
  const int nbp = min(S.cnt->n_bp, S.cap_bp);
  for (int p = blockIdx.x; p < nbp; p += gridDim.x) {
    const int2 ab = S.bp[p];
    for (int dir = 0; dir < 2; ++dir) {
      const int* ce = S.body_chunk + 6 * (dir ? ab.y : ab.x);
      const int* ct = S.body_chunk + 6 * (dir ? ab.x : ab.y);
      const int ne = ce[5] - ce[4], nt = ct[3] - ct[2];
      for (int t = threadIdx.x; t < ne * nt; t += blockDim.x) {
        const int E = ce[4] + t / nt, Tc = ct[2] + t % nt;
        if (!box_overlap(S.ch_box + 6 * E, S.ch_box + 6 * Tc, 0.0)) continue;
        for (int i = 0; i < S.ch_count[E]; ++i) {
          const int e = S.ch_prims[S.ch_start[E] + i];
          double p0[3], p1[3];
          vertex_pos(S, S.edge[e], p0);
          vertex_pos(S, S.edge[S.E + e], p1);
          for (int j = 0; j < S.ch_count[Tc]; ++j) {
            const int tri = S.ch_prims[S.ch_start[Tc] + j];
            double a[3], b[3], c[3];
            vertex_pos(S, S.tri[tri], a);
            vertex_pos(S, S.tri[S.T + tri], b);
            vertex_pos(S, S.tri[2 * S.T + tri], c);
            const double s0 = orient3(a, b, c, p0), s1 = orient3(a, b, c, p1);
            if (!((s0 > 0 && s1 < 0) || (s0 < 0 && s1 > 0))) continue;
            const double o1 = orient3(p0, p1, a, b), o2 = orient3(p0, p1, b, c),
                         o3 = orient3(p0, p1, c, a);
            if ((o1 > 0 && o2 > 0 && o3 > 0) || (o1 < 0 && o2 < 0 && o3 < 0))
              atomicAdd(&S.cnt->n_act, 1);
          }
        }
      }
    }
  }
}


/* ================================================================== */
/* host launchers                                                      */
/* ================================================================== */
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
void launch_body_terms(const Scene& S, hipStream_t st, const Counters* fresh,
                       int expect_reuse) {
  const Counters f = fresh ? *fresh : Counters{};
  const int mode = fresh ? (expect_reuse ? 2 : 1) : 0;
  if (S.mixed)
    hipLaunchKernelGGL(k_body_terms<float>, dim3(cdiv(S.B, 64)), dim3(64), 0, st, S, f, mode);
  else
    hipLaunchKernelGGL(k_body_terms<double>, dim3(cdiv(S.B, 64)), dim3(64), 0, st, S, f, mode);
}
void launch_pass_reset(const Scene& S, const Counters& fresh, int expect_reuse,
                       hipStream_t st) {
  const long n = std::max<long>(std::max<long>(S.B + 1, S.NP), 2L * ((S.B + 15) / 16));
  hipLaunchKernelGGL(k_boxes, dim3(cdiv(n, 256)), dim3(256), 0, st, S, -1, fresh,
                     expect_reuse ? 2 : 1, 0, 0);
}
void launch_boxes(const Scene& S, int swept, hipStream_t st,
                  const Counters* fresh, int expect_reuse, int stop_test) {
  const Counters f = fresh ? *fresh : Counters{};
  const int mode = fresh ? (expect_reuse ? 2 : 1) : 0;
  const unsigned nmain = std::max(1u, cdiv((long)S.NC + S.B, 256));
  const unsigned g = nmain + (stop_test ? cdiv(S.B, 256) : 0u);
  hipLaunchKernelGGL(k_boxes, dim3(g), dim3(256), 0, st, S, swept, f, mode, stop_test,
                     (int)nmain);
}
void launch_body_pairs(const Scene& S, hipStream_t st) {
  if (S.n_dyn == 0) return;
  if (!S.sap_on) {
    if (S.n_bp_tiles == 0) return;
    hipLaunchKernelGGL(k_body_pairs, dim3(S.n_bp_tiles), dim3(16, 16), 0, st, S);
    return;
  }
  hipLaunchKernelGGL(k_sap_sort, dim3(std::min(S.NP, 1024)), dim3(1024), 0, st, S);
  hipLaunchKernelGGL(k_sap_sweep, dim3(std::min(4096u, cdiv(S.n_dyn, 4 * SAP_PER_WAVE))),
                     dim3(256), 0, st, S);
}
void launch_chunk_pairs(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_pairs, dim3(S.grid_blocks), dim3(256), 0, st, S);
}
void launch_prim_pairs(const Scene& S, int swept, hipStream_t st) {
  hipLaunchKernelGGL(k_prim_pairs, dim3(S.grid_blocks), dim3(256), 0, st, S, swept);
}
void launch_pg(const Scene& S, int swept, hipStream_t st) {
  hipLaunchKernelGGL(k_pg, dim3(min(1024u, cdiv(S.NC, 4))), dim3(256), 0, st, S, swept);
}
void launch_filter(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_filter, dim3(S.grid_blocks), dim3(256), 0, st, S,
                     S.mixed ? 72 : 144);
}
void launch_assemble(const Scene& S, int n_act_hint, hipStream_t st) {
  unsigned g = n_act_hint > 0 ? min(4096u, cdiv(n_act_hint, PAIRS_PER_WG))
                              : (unsigned)S.assemble_blocks;
  if (S.mixed)
    hipLaunchKernelGGL(k_assemble<float>, dim3(g), dim3(64), 0, st, S);
  else
    hipLaunchKernelGGL(k_assemble<double>, dim3(g), dim3(64), 0, st, S);
  if (S.det) {
    const unsigned gd = std::min(4096u, cdiv(156L * S.B + 144L * S.cap_bp, 256));
    if (S.mixed)
      hipLaunchKernelGGL(k_det_finish<float>, dim3(gd), dim3(256), 0, st, S);
    else
      hipLaunchKernelGGL(k_det_finish<double>, dim3(gd), dim3(256), 0, st, S);
  }
}
void launch_energy_multi(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_multi, dim3(512), dim3(256), 0, st, S);
}
void launch_ctrl_start(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_ctrl_start, dim3(cdiv(S.NP, 64)), dim3(64), 0, st, S);
}
void launch_update_multi(const Scene& S, Counters* ring, unsigned* pass, hipStream_t st) {
  hipLaunchKernelGGL(k_update_multi, dim3(cdiv(12L * S.B, 256)), dim3(256), 0, st, S,
                     ring, pass);
}
void launch_gather(const Scene& S, const ProbCopy* pc, const double* scales,
                   int np, int max_nb, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(cdiv(12L * max_nb, 256), np), dim3(256), 0,
                     st, S, pc, scales);
}
void launch_scatter(const Scene& S, const ProbCopy* pc, int np, int max_nb,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3(cdiv(12L * max_nb, 256), np), dim3(256), 0,
                     st, S, pc);
}
void launch_cons_init(const Scene& S, const Cons& C, hipStream_t st) {
  hipLaunchKernelGGL(k_cons_init, dim3(cdiv(12L * C.n_groups + 2, 256)), dim3(256),
                     0, st, S, C);
}
void launch_cons_update(const Scene& S, const Cons& C, hipStream_t st) {
  hipLaunchKernelGGL(k_cons_clear, dim3(cdiv(C.n_groups + 2, 256)), dim3(256), 0,
                     st, C);
  hipLaunchKernelGGL(k_cons_update, dim3(cdiv(12L * C.n_groups, 256)), dim3(256),
                     0, st, S, C);
}
void launch_cons_adapt(const Scene& S, const Cons& C, hipStream_t st) {
  hipLaunchKernelGGL(k_cons_adapt, dim3(cdiv(C.n_rep, 256)), dim3(256), 0, st, S, C);
}
void launch_cons_merge(const Scene& S, const Cons& C, hipStream_t st) {
  hipLaunchKernelGGL(k_cons_merge, dim3(cdiv(12L * C.n_rep, 256)), dim3(256), 0,
                     st, S, C);
}
void launch_cons_merge_dq(const Scene& S, const Cons& C, hipStream_t st) {
  hipLaunchKernelGGL(k_cons_dq_zero, dim3(cdiv(12L * S.B + S.NP, 256)), dim3(256),
                     0, st, S);
  hipLaunchKernelGGL(k_cons_dq, dim3(cdiv(12L * C.n_rep, 256)), dim3(256), 0, st,
                     S, C);
}
void launch_reset_toi(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_toi, dim3(cdiv(S.NP, 256)), dim3(256), 0, st, S);
}
void launch_reset_pcg(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_pcg, dim3(cdiv(S.NP, 256)), dim3(256), 0, st, S);
}
void launch_crossings(const Scene& S, hipStream_t st) {
  hipLaunchKernelGGL(k_crossings, dim3(1024), dim3(256), 0, st, S);
}
void launch_bsr(const Scene& S, hipStream_t st) {
  if (S.bsr_one) {
    hipLaunchKernelGGL(k_bsr_small, dim3(1), dim3(1024), 0, st, S);
    return;
  }
  if (S.n_lab_chunks > 0) {
    hipLaunchKernelGGL(k_bsr_chunk_count, dim3(S.n_lab_chunks), dim3(1024), 0, st, S);
    hipLaunchKernelGGL(k_bsr_chunk_fill, dim3(S.n_lab_chunks), dim3(1024), 0, st, S);
    return;
  }
  hipLaunchKernelGGL(k_bsr_count, dim3(256), dim3(256), 0, st, S);
  hipLaunchKernelGGL(k_bsr_scan, dim3(1), dim3(1024), 0, st, S);
  hipLaunchKernelGGL(k_bsr_fill, dim3(256), dim3(256), 0, st, S);
  if (S.det) hipLaunchKernelGGL(k_sort_rows, dim3(cdiv(S.B, 256)), dim3(256), 0, st, S);
}
void launch_block_inverse(const Scene& S, hipStream_t st) {
  if (S.mixed)
    hipLaunchKernelGGL(k_block_inverse<float>, dim3(cdiv(S.B, 15)), dim3(192), 0, st, S);
  else
    hipLaunchKernelGGL(k_block_inverse<double>, dim3(cdiv(S.B, 15)), dim3(192), 0, st, S);
  /* the components solved directly (none unless the block-row build
   * labelled them) */
  if (S.comp_solve) {
    const unsigned g = std::min(256u, cdiv(S.B / 2 + 1, DIR_WAVES));
    if (S.mixed)
      hipLaunchKernelGGL(k_direct<float>, dim3(g), dim3(64 * DIR_WAVES), 0, st, S);
    else
      hipLaunchKernelGGL(k_direct<double>, dim3(g), dim3(64 * DIR_WAVES), 0, st, S);
  }
}
int pcg_max_grid() {
  int dev = 0, ncu = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  int per32 = 0;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_pcg<double>, 192, 0);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per32, (const void*)k_pcg<float>, 192, 0);
  per = std::min(per, per32);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per32, (const void*)k_pcg1<double>, 192, 0);
  per = std::min(per, per32);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per32, (const void*)k_pcg1<float>, 192, 0);
  per = std::min(per, per32);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per32, (const void*)k_pcg_local<double>, 192, 0);
  per = std::min(per, per32);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per32, (const void*)k_pcg_local<float>, 192, 0);
  per = std::min(per, per32);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per32, (const void*)k_pcg_cg1<double>, 192, 0);
  per = std::min(per, per32);
  return ncu * (per > 0 ? per : 1);
}
int launch_pcg(const Scene& S, double eta, int max_it, int grid, int variant,
               int goff, hipStream_t st) {
  void* args[] = {(void*)&S, (void*)&eta, (void*)&max_it, (void*)&goff};
  const void* fn;
  if (variant == 1)
    fn = S.mixed ? (const void*)k_pcg1<float> : (const void*)k_pcg1<double>;
  else if (variant == 2)
    fn = S.mixed ? (const void*)k_pcg_local<float> : (const void*)k_pcg_local<double>;
  else if (variant == 3)
    fn = S.mixed ? (const void*)k_pcg_cg1<float> : (const void*)k_pcg_cg1<double>;
  else
    fn = S.mixed ? (const void*)k_pcg<float> : (const void*)k_pcg<double>;
  /* the blocks wait for each other, so the grid never exceeds what the
   * device holds resident at once (pcg_max_grid); every wait is bounded
   * and reports a device error instead of hanging should blocks of the
   * grid not be resident together */
  hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(192), args, 0, st);
  return e == hipSuccess ? 0 : -1;
}
void launch_dq_norm(const Scene& S, int with_ctrl, hipStream_t st) {
  hipLaunchKernelGGL(k_dq_norm, dim3(cdiv(S.B, 256)), dim3(256), 0, st, S, with_ctrl);
}
void launch_ccd(const Scene& S, int with_ctrl, hipStream_t st) {
  hipLaunchKernelGGL(k_ccd, dim3(S.grid_blocks), dim3(256), 0, st, S, (double*)nullptr);
  hipLaunchKernelGGL(k_ccd_long, dim3(CCD_LONG_BLOCKS), dim3(256), 0, st, S, with_ctrl,
                     (double*)nullptr);
}
void launch_ccd_pairs(const Scene& S, double* toi, int64_t n, hipStream_t st) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_ccd, dim3(blocks), dim3(256), 0, st, S, toi);
  hipLaunchKernelGGL(k_ccd_long, dim3(CCD_LONG_BLOCKS), dim3(256), 0, st, S, 0, toi);
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
