/*
 * Host side of libabd: the C-ABI of include/abd.h, device memory, the
 * chunk hierarchy of the broad phase, and the Newton loop of the local
 * solve (Eq. 5):
 *
 *   repeat
 *     body terms + static broad phase + barrier assembly  -> g, H
 *     block-Jacobi PCG                                     -> dq
 *     stop if |dq|_inf / (h l) < theta                    (Eq. 8 form)
 *     swept broad phase + additive CCD                     -> alpha_max
 *     halve alpha while E(q + alpha dq) - E(q) > 0         (line search)
 *     q += alpha dq
 *
 * Two host synchronisations per iteration read back a small counter block
 * (stop test and capacities; step size and energy difference).
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "../../include/abd.h"
#include "abd_internal.h"

using namespace abd;

/* timing stages: 0 body terms, 1 broad phase, 2 barrier (filter and
 * assembly), 3 PCG, 4 CCD, 5 line search, 6 other, 7 the assembly kernel
 * alone (ABD_TIMING_ASM) */
#define ABD_STAGES 8

/* Static device scratch of the allocation-free solve
 * (abd_local_solve_static): the per-pass lists of a solve (body pairs with
 * their off-diagonal blocks and block-row columns, chunk pairs, candidate
 * and active pairs) live in this array instead of buffers of the context.
 * Every GPU the library runs on holds its own copy until the process ends.
 * Host code never passes the array's name to a kernel: the device address
 * of the current device's copy is looked up once per device with
 * hipGetSymbolAddress (scratch_ptr) and only that address is used. */
#define ABD_SCRATCH_BYTES (64u << 20)
#define ABD_SCRATCH_DEVICES 64
static __device__ __align__(256) unsigned char scratch[ABD_SCRATCH_BYTES];

namespace {

struct HBody {
  int kind;
  double density;
  int v0, nv, t0, nt, e0, ne;
  double Mhat[16];
  double vol;
  double q0[12], qd0[12];
};

struct Pending {
  int stage;
  hipEvent_t a, b;
  double bytes;
};

}  // namespace

struct abd_ctx {
  abd_params P;
  uint64_t serial = 0;            /* unique per context in the process */
  abd_batch* batch_cache = nullptr; /* merged scene of abd_batch_solve */
  std::string err;
  hipStream_t st = nullptr;
  hipStream_t side = nullptr; /* body terms run here, overlapping the
                                 broad phase (default priority) */
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool finalized = false;
  std::vector<HBody> bodies;
  std::vector<double> xbar; /* [V][3] */
  std::vector<int> vbody, tri /* [T][3] */, edge /* [E][2] */;
  std::vector<double> erest2;
  int pair_mode = 0;
  double scale = 1.0;
  /* problems of a merged batch scene (empty: one problem) */
  std::vector<int> prob_of_body;
  int np = 1;
  /* host copy of the shared-body data, and its version */
  std::vector<int> sh_ids, sh_kappa;
  std::vector<double> sh_z, sh_u, sh_rho;
  unsigned sh_version = 0;
  Scene S;
  Counters* h_cnt = nullptr; /* pinned */
  /* the last static and swept counters of a device-loop pass that ran a
   * Newton step (a pass that only continues a line search has no static
   * phase): the list sizes a solve reports */
  Counters h_last[2] = {};
  Counters* h_ring = nullptr; /* pinned [2][2]: counters of passes in flight */
  Counters* d_ring = nullptr; /* the same memory as the device sees it */
  unsigned* d_pass = nullptr; /* device pass counter (ring slot parity) */
  bool switched64 = false;    /* this solve switched to FP64 Hessians */
  bool no_alloc = false;      /* a solve in the static scratch is running */
  int device = 0;             /* HIP device of the context */
  hipEvent_t ring_ev[2] = {nullptr, nullptr};
  double* h_buf = nullptr;   /* pinned scratch, 64 doubles */
  std::vector<void*> allocs; /* device memory of our own (hipMalloc) */
  /* caller workspace: blocks are handed out 256-byte aligned from its
   * bottom, as a stack; a released block's bytes are taken back once every
   * block above it has been released too */
  struct WsBlock {
    size_t off, bytes;
    bool live;
  };
  char* ws_base = nullptr;
  size_t ws_size = 0, ws_top = 0, ws_peak = 0;
  std::vector<WsBlock> ws_blocks;
  int pcg_grid = 0;
  int n_cu = 0;
  int n_shared = 0;
  /* pass halves: [0] before the PCG launch, [1] after it, [2] the first
   * half without the static broad phase (lists taken over); whole passes
   * with the PCG launch inside: [3] full, [4] taking over (passes whose PCG
   * launch is not timed, when that launch can be captured) */
  hipGraphExec_t pass_graph[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  bool whole_ok = true;
  /* with ABD_TIMING_PCG, every pcg_sample-th pass of a solve is run in
   * halves with events around its PCG launch; the others run whole */
  int pcg_sample = 4;
  unsigned long long pass_seq = 0; /* passes launched by this context */
  bool pass_timed[2] = {false, false};
  /* whether the next PCG launch is timed with ABD_TIMING_PCG (the device
   * loop clears it for passes outside the sample) */
  bool pcg_timed_now = true;
  bool graphs_ok = true; /* capture available on this runtime */
  bool own_stream = false;
  /* direct launches by default: on the benchmark scene a replayed graph
   * per pass costs more at each graph boundary than the pass's kernel
   * launches do (the host queues passes ahead either way) */
  abd_tuning tune = {ABD_PCG_LOCAL1, 0, 2048, 2048, 0, 0, 0, ABD_BODY_PAIRS_AUTO, 0, 0};
  long bp_tests = 0; /* box tests of every pair of each problem */
  /* problem-local PCG forms: launches of consecutive 16-body groups
   * (first group, count), each holding whole problems and at most
   * pcg_grid groups; empty when a problem's groups exceed that */
  std::vector<std::pair<int, int>> pcg_ranges;
  std::vector<int> hb0, hb1; /* first and last body of each problem */
  std::vector<char> padding;  /* [B] bodies a batch adds to align problems */
  /* timing */
  int timing = 0;      /* ABD_TIMING_* */
  bool capturing = false;
  double t_ms[ABD_STAGES] = {0}, t_bytes[ABD_STAGES] = {0}, t_flops[ABD_STAGES] = {0};
  int64_t t_n[ABD_STAGES] = {0};
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

int fail(abd_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

/* device address of the scratch copy of device dev (nullptr until
 * scratch_init ran on that device) */
std::atomic<void*> g_scratch[ABD_SCRATCH_DEVICES];

/* look up the current device's scratch address once (the device must be
 * current); ABD_OK or ABD_E_DEVICE */
int scratch_init(int dev) {
  if (dev < 0 || dev >= ABD_SCRATCH_DEVICES) return ABD_E_DEVICE;
  if (g_scratch[dev].load()) return ABD_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return ABD_E_DEVICE;
  }
  g_scratch[dev].store(p);
  return ABD_OK;
}

void drop_graphs(abd_ctx* c) {
  for (auto& g : c->pass_graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

#define HIPCHK(call)                                                     \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess)                                                \
      return fail(ctx, ABD_E_DEVICE,                                     \
                  std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

/* Device memory for a context buffer: from the bound workspace if there is
 * one, else from hipMalloc (kept in ctx->allocs, freed at destroy). */
int dalloc_bytes(abd_ctx* ctx, void** p, size_t bytes) {
  bytes = std::max<size_t>(bytes, 8);
  if (ctx->ws_base) {
    const size_t off = (ctx->ws_top + 255) & ~size_t(255);
    if (off > ctx->ws_size || bytes > ctx->ws_size - off)
      return fail(ctx, ABD_E_OOM,
                  "workspace exhausted: " + std::to_string(bytes) +
                      " bytes asked for at offset " + std::to_string(off) +
                      " of a " + std::to_string(ctx->ws_size) +
                      "-byte workspace");
    ctx->ws_blocks.push_back({off, bytes, true});
    ctx->ws_top = off + bytes;
    ctx->ws_peak = std::max(ctx->ws_peak, ctx->ws_top);
    *p = ctx->ws_base + off;
    return ABD_OK;
  }
  void* q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, ABD_E_OOM, "device allocation failed");
  }
  ctx->allocs.push_back(q);
  *p = q;
  return ABD_OK;
}

template <class T>
int dalloc(abd_ctx* ctx, T** p, size_t n) {
  void* q = nullptr;
  int rc = dalloc_bytes(ctx, &q, std::max<size_t>(n, 1) * sizeof(T));
  if (rc) return rc;
  *p = (T*)q;
  return ABD_OK;
}

size_t hess_elem(const abd_ctx* ctx) {
  return ctx->S.mixed ? sizeof(float) : sizeof(double);
}
/* Hessian storage is sized for FP64 in both forms, so a mixed context can
 * repeat a solve in FP64 in the same buffers */
constexpr size_t HESS_ALLOC = sizeof(double);

template <class T>
void dfree(abd_ctx* ctx, T* p) {
  if (!p) return;
  const char* c = (const char*)p;
  if (ctx->ws_base && c >= ctx->ws_base && c < ctx->ws_base + ctx->ws_size) {
    const size_t off = size_t(c - ctx->ws_base);
    for (auto& b : ctx->ws_blocks)
      if (b.off == off) b.live = false;
    while (!ctx->ws_blocks.empty() && !ctx->ws_blocks.back().live)
      ctx->ws_blocks.pop_back();
    ctx->ws_top = ctx->ws_blocks.empty()
                      ? 0
                      : ctx->ws_blocks.back().off + ctx->ws_blocks.back().bytes;
    return;
  }
  auto it = std::find(ctx->allocs.begin(), ctx->allocs.end(), (void*)p);
  if (it != ctx->allocs.end()) ctx->allocs.erase(it);
  (void)hipFree(p);
}

template <class T>
int upload(abd_ctx* ctx, T** p, const std::vector<T>& v) {
  int rc = dalloc(ctx, p, v.size());
  if (rc) return rc;
  if (!v.empty())
    HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return ABD_OK;
}

/* ---------------- timing ---------------- */
hipEvent_t get_event(abd_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  (void)hipEventCreate(&e);
  return e;
}
struct StageTimer {
  abd_ctx* ctx;
  int stage;
  double bytes;
  hipStream_t stream;
  hipEvent_t a = nullptr;
  bool active;
  StageTimer(abd_ctx* c, int s, double b = 0.0, hipStream_t on = nullptr)
      : ctx(c), stage(s), bytes(b), stream(on ? on : c->st) {
    /* never inside a capture; the PCG-only mode times the one launch that
     * is not part of the captured graphs */
    active = !ctx->capturing &&
             (ctx->timing == ABD_TIMING_ALL ||
              (ctx->timing == ABD_TIMING_PCG && stage == 3 && ctx->pcg_timed_now) ||
              (ctx->timing == ABD_TIMING_ASM && stage == 7 && ctx->pcg_timed_now));
    if (active) {
      a = get_event(ctx);
      (void)hipEventRecord(a, stream);
    }
  }
  ~StageTimer() {
    if (active) {
      hipEvent_t b = get_event(ctx);
      (void)hipEventRecord(b, stream);
      ctx->pending.push_back({stage, a, b, bytes});
    }
  }
};
void resolve_timing(abd_ctx* ctx) {
  /* events of passes still in flight stay pending */
  std::vector<Pending> keep;
  for (auto& p : ctx->pending) {
    if (hipEventQuery(p.b) != hipSuccess) {
      (void)hipGetLastError();
      keep.push_back(p);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->t_ms[p.stage] += ms;
      ctx->t_n[p.stage] += 1;
      ctx->t_bytes[p.stage] += p.bytes;
    } else {
      (void)hipGetLastError();
    }
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.swap(keep);
}

/* ---------------- mass properties (divergence theorem) ---------------- */
void mass_props(const double* xb, const int32_t* tris, int nt, double rho,
                double* M, double* vol) {
  double V = 0.0, f[3] = {0, 0, 0}, s2[9] = {0};
  for (int t = 0; t < nt; ++t) {
    const double* a = xb + 3 * tris[3 * t];
    const double* b = xb + 3 * tris[3 * t + 1];
    const double* c = xb + 3 * tris[3 * t + 2];
    double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2],
                    b[0] * c[1] - b[1] * c[0]};
    double vt = (a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2]) / 6.0;
    V += vt;
    double s[3];
    for (int i = 0; i < 3; ++i) {
      s[i] = a[i] + b[i] + c[i];
      f[i] += vt * s[i] * 0.25;
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        s2[3 * i + j] += vt * 0.05 *
                         (a[i] * a[j] + b[i] * b[j] + c[i] * c[j] + s[i] * s[j]);
  }
  *vol = V;
  M[0] = rho * V;
  for (int i = 0; i < 3; ++i) {
    M[1 + i] = M[4 * (1 + i)] = rho * f[i];
    for (int j = 0; j < 3; ++j) M[4 * (1 + i) + 1 + j] = rho * s2[3 * i + j];
  }
}

/* ---------------- chunk hierarchy ---------------- */
struct Leaf {
  std::vector<int> ids;
};

/* Split primitive ids along the longest axis of their rest centroids until
 * at most ABD_CHUNK per leaf; leaves of static bodies keep splitting while
 * they hold more than one primitive and their box is much larger than the
 * primitives in it (large container walls get boxes of their own). */
/* Chunks of one body's primitives (one kind) by median splits of the rest
 * centroids along the longest axis.  A dynamic body's chunk holds up to one
 * wavefront of primitives.  A static body (walls, containers: few, large,
 * far-apart primitives) is split further, until each chunk's box is not
 * much emptier than its primitives: the box volume, every extent padded by
 * tau, may exceed the sum of the primitives' padded box volumes at most
 * twice.  Without that, one chunk of a container's faces has the whole
 * container as its box and meets every body inside. */
void split_leaves(std::vector<int>& ids, const std::vector<double>& cen,
                  const std::vector<double>& pbox, bool is_static, double tau,
                  std::vector<Leaf>& out) {
  if (ids.empty()) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY},
         hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double blo[3] = {INFINITY, INFINITY, INFINITY},
         bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double prim_vol = 0.0;
  for (int i : ids) {
    double v = 1.0;
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], cen[3 * i + k]);
      hi[k] = std::max(hi[k], cen[3 * i + k]);
      blo[k] = std::min(blo[k], pbox[6 * i + k]);
      bhi[k] = std::max(bhi[k], pbox[6 * i + 3 + k]);
      v *= pbox[6 * i + 3 + k] - pbox[6 * i + k] + 2.0 * tau;
    }
    prim_vol += v;
  }
  double box_vol = 1.0;
  for (int k = 0; k < 3; ++k) box_vol *= bhi[k] - blo[k] + 2.0 * tau;
  const bool small = (int)ids.size() <= ABD_CHUNK;
  if (small && (!is_static || ids.size() == 1 || box_vol <= 2.0 * prim_vol)) {
    out.push_back({ids});
    return;
  }
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (hi[k] - lo[k] > hi[ax] - lo[ax]) ax = k;
  size_t mid = ids.size() / 2;
  std::nth_element(ids.begin(), ids.begin() + mid, ids.end(),
                   [&](int a, int b) { return cen[3 * a + ax] < cen[3 * b + ax]; });
  std::vector<int> L(ids.begin(), ids.begin() + mid), R(ids.begin() + mid, ids.end());
  split_leaves(L, cen, pbox, is_static, tau, out);
  split_leaves(R, cen, pbox, is_static, tau, out);
}

/* ---------------- counters ---------------- */
Counters fresh_counters() {
  Counters c;
  std::memset(&c, 0, sizeof(c));
  double inf = INFINITY;
  std::memcpy(&c.min_dist, &inf, 8);
  std::memcpy(&c.min_toi, &inf, 8);
  return c;
}

/* the counter blocks live in one device array: [0] static phase, [1] swept
 * phase; ctx->h_cnt mirrors both in pinned memory */
int reset_counters(abd_ctx* ctx, int which = 0) {
  ctx->h_cnt[which] = fresh_counters();
  HIPCHK(hipMemcpyAsync(ctx->S.cnt + which, ctx->h_cnt + which,
                        sizeof(Counters), hipMemcpyHostToDevice, ctx->st));
  return ABD_OK;
}

int reset_both(abd_ctx* ctx) {
  ctx->h_cnt[0] = fresh_counters();
  ctx->h_cnt[1] = fresh_counters();
  HIPCHK(hipMemcpyAsync(ctx->S.cnt, ctx->h_cnt, 2 * sizeof(Counters),
                        hipMemcpyHostToDevice, ctx->st));
  return ABD_OK;
}

/* the device's error bits: 1 a bounded wait ran out, 2 a barrier term
 * too large for the deterministic mode's exact sums */
const char* device_err_text(int err) {
  if (err & 2) return "a barrier term of magnitude 2^100 or more (deterministic mode)";
  return "device barrier timed out";
}

int read_counters(abd_ctx* ctx, int which = 0, int n = 1) {
  HIPCHK(hipMemcpyAsync(ctx->h_cnt + which, ctx->S.cnt + which,
                        n * sizeof(Counters), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  resolve_timing(ctx);
  for (int i = which; i < which + n; ++i)
    if (ctx->h_cnt[i].err)
      return fail(ctx, ABD_E_DEVICE, device_err_text(ctx->h_cnt[i].err));
  return ABD_OK;
}

Scene swept_scene(const abd_ctx* ctx) {
  Scene s = ctx->S;
  s.cnt = ctx->S.cnt + 1;
  return s;
}

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, 8);
  return d;
}
unsigned long long double_to_bits(double d) {
  unsigned long long b;
  std::memcpy(&b, &d, 8);
  return b;
}

/* ---------------- capacities ---------------- */
bool over_cap(const Scene& S, const Counters& c) {
  return c.n_bp > S.cap_bp || c.n_cp > S.cap_cp || c.n_pt > S.cap_pt ||
         c.n_ee > S.cap_ee || c.n_pg > S.cap_pg || c.n_act > S.cap_act ||
         c.n_long > S.cap_long;
}
/* the list that outgrew the static scratch, as an error */
int static_overflow_error(abd_ctx* ctx) {
  const Scene& S = ctx->S;
  const char* names[7] = {"body pairs", "chunk pairs", "point-triangle candidates",
                          "edge-edge candidates", "point-ground candidates",
                          "active pairs", "pairs in blocked CCD steps"};
  const int caps[7] = {S.cap_bp, S.cap_cp, S.cap_pt, S.cap_ee, S.cap_pg, S.cap_act,
                       S.cap_long};
  for (int b = 0; b < 2; ++b) {
    const Counters& c = ctx->h_cnt[b];
    const int n[7] = {c.n_bp, c.n_cp, c.n_pt, c.n_ee, c.n_pg, c.n_act, c.n_long};
    for (int i = 0; i < 7; ++i)
      if (n[i] > caps[i])
        return fail(ctx, ABD_E_CAPACITY,
                    std::string("static scratch: ") + std::to_string(n[i]) + " " +
                        names[i] + " exceed its maximum of " + std::to_string(caps[i]));
  }
  return fail(ctx, ABD_E_CAPACITY, "static scratch: a list overflowed");
}

void drop_graphs_if(abd_ctx* ctx, const Counters& c) {
  if (over_cap(ctx->S, c)) drop_graphs(ctx);
}
int grow(abd_ctx* ctx, const Counters& c, bool* changed) {
  Scene& S = ctx->S;
  drop_graphs_if(ctx, c);
  *changed = false;
  auto need = [](int have, int n) { return n > have; };
  int rc;
  if (need(S.cap_bp, c.n_bp)) {
    dfree(ctx, S.bp);
    dfree(ctx, S.Hoff);
    dfree(ctx, S.slot_used);
    S.cap_bp = (int)std::min<long>(2L * c.n_bp + 1024, 1L << 30);
    if ((rc = dalloc(ctx, &S.bp, S.cap_bp))) return rc;
    if ((rc = dalloc_bytes(ctx, &S.Hoff, 144L * S.cap_bp * HESS_ALLOC))) return rc;
    if ((rc = dalloc(ctx, &S.slot_used, S.cap_bp))) return rc;
    if (S.det) {
      dfree(ctx, S.det_ho);
      if ((rc = dalloc(ctx, &S.det_ho, (size_t)144 * DET_W * S.cap_bp))) return rc;
      HIPCHK(hipMemset(S.det_ho, 0, sizeof(det_word) * 144 * DET_W * (size_t)S.cap_bp));
    }
    dfree(ctx, S.col_slot);
    dfree(ctx, S.col_body);
    dfree(ctx, S.col_trans);
    S.cap_col = 2 * S.cap_bp;
    if ((rc = dalloc(ctx, &S.col_slot, S.cap_col))) return rc;
    if ((rc = dalloc(ctx, &S.col_body, S.cap_col))) return rc;
    if ((rc = dalloc(ctx, &S.col_trans, S.cap_col))) return rc;
    *changed = true;
  }
  if (need(S.cap_cp, c.n_cp)) {
    dfree(ctx, S.cp);
    S.cap_cp = (int)std::min<long>(2L * c.n_cp + 1024, 1L << 30);
    if ((rc = dalloc(ctx, &S.cp, S.cap_cp))) return rc;
    *changed = true;
  }
  if (need(S.cap_pt, c.n_pt)) {
    dfree(ctx, S.cand_pt);
    S.cap_pt = (int)std::min<long>(2L * c.n_pt + 1024, 1L << 29);
    if ((rc = dalloc(ctx, &S.cand_pt, 3L * S.cap_pt))) return rc;
    *changed = true;
  }
  if (need(S.cap_ee, c.n_ee)) {
    dfree(ctx, S.cand_ee);
    S.cap_ee = (int)std::min<long>(2L * c.n_ee + 1024, 1L << 29);
    if ((rc = dalloc(ctx, &S.cand_ee, 3L * S.cap_ee))) return rc;
    *changed = true;
  }
  if (need(S.cap_pg, c.n_pg)) {
    dfree(ctx, S.cand_pg);
    S.cap_pg = (int)std::min<long>(2L * c.n_pg + 1024, 1L << 30);
    if ((rc = dalloc(ctx, &S.cand_pg, S.cap_pg))) return rc;
    *changed = true;
  }
  if (need(S.cap_act, c.n_act)) {
    dfree(ctx, S.act);
    S.cap_act = (int)std::min<long>(2L * c.n_act + 1024, 1L << 30);
    if ((rc = dalloc(ctx, &S.act, S.cap_act))) return rc;
    *changed = true;
  }
  /* the long CCD list holds every PT and EE candidate (its own overflow
   * is only possible with caller-fixed capacities) */
  if (S.cap_long < S.cap_pt + S.cap_ee || need(S.cap_long, c.n_long)) {
    dfree(ctx, S.ccd_long);
    S.cap_long = std::max(S.cap_pt + S.cap_ee, 2 * c.n_long + 1024);
    if ((rc = dalloc(ctx, &S.ccd_long, S.cap_long))) return rc;
    *changed = true;
  }
  return ABD_OK;
}

/* body pairs by sort and sweep (else every pair of each problem) */
constexpr long ALL_PAIRS_BUILD_MAX = 1L << 27;
int sap_on(const abd_ctx* ctx) {
  if (ctx->tune.body_pairs == ABD_BODY_PAIRS_ALL) return 0;
  if (ctx->tune.body_pairs == ABD_BODY_PAIRS_SWEEP) return 1;
  return ctx->bp_tests > SAP_ALL_PAIRS_MAX ? 1 : 0;
}

/* ---------------- phases ---------------- */
void broad_phase(abd_ctx* ctx, const Scene& S, int swept, int stop_test = 0) {
  StageTimer t(ctx, 1);
  launch_boxes(S, swept, ctx->st, nullptr, 0, stop_test);
  launch_body_pairs(S, ctx->st);
  launch_chunk_pairs(S, ctx->st);
  launch_prim_pairs(S, swept, ctx->st);
  if (S.has_ground) launch_pg(S, swept, ctx->st);
}

void launch_swept_s(abd_ctx* ctx, const Scene& Ssw, bool ccd, bool with_ctrl = false);

/* static phase on the stream: body terms, broad phase, barrier assembly;
 * with take_over the candidate lists are the previous pass's swept lists
 * (the filter computes the positions it needs).  fresh: the device-loop
 * pass reset, run by the first kernel on the stream */
void launch_static(abd_ctx* ctx, const Scene& S, bool take_over = false,
                   const Counters* fresh = nullptr) {
  const double body_bytes = (double)S.B * (96 * 3 + 128 + 8 + 1152 + 96);
  if (ctx->tune.overlap_body) {
    if (fresh) launch_pass_reset(S, *fresh, take_over ? 1 : 0, ctx->st);
    /* body terms (writes g, Hdiag) on the side stream, concurrent with the
     * broad phase; the assembly (which adds into g, Hdiag) waits for it */
    (void)hipEventRecord(ctx->ev_fork, ctx->st);
    (void)hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0);
    {
      StageTimer t(ctx, 0, body_bytes, ctx->side);
      launch_body_terms(S, ctx->side);
    }
    (void)hipEventRecord(ctx->ev_join, ctx->side);
  } else {
    StageTimer t(ctx, 0, body_bytes);
    launch_body_terms(S, ctx->st, fresh, take_over ? 1 : 0);
  }
  if (!take_over) broad_phase(ctx, S, 0);
  {
    StageTimer t(ctx, 2);
    launch_filter(S, ctx->st);
    if (ctx->tune.overlap_body) (void)hipStreamWaitEvent(ctx->st, ctx->ev_join, 0);
    StageTimer ta(ctx, 7);
    launch_assemble(S, 0, ctx->st);
  }
}

/* PCG form in use: the problem-local forms need one resident block per
 * 16-body group of every problem (groups of different problems that share
 * no group may run in separate launches, pcg_ranges) */
int pcg_variant(const abd_ctx* ctx, const Scene& S) {
  (void)S;
  if (ctx->P.deterministic) return ABD_PCG_LOCAL1; /* finalize checked the ranges */
  if ((ctx->tune.pcg_variant == ABD_PCG_LOCAL || ctx->tune.pcg_variant == ABD_PCG_LOCAL1) &&
      ctx->pcg_ranges.empty())
    return ABD_PCG_TWO_BARRIER;
  return ctx->tune.pcg_variant;
}

/* launches of the problem-local PCG forms: problems whose 16-body groups
 * overlap form one cluster (a group holding bodies of two problems runs
 * both), clusters are packed in order into launches of at most cap
 * groups; none if one cluster alone exceeds cap */
std::vector<std::pair<int, int>> pcg_launch_ranges(const std::vector<int>& b0,
                                                   const std::vector<int>& b1,
                                                   int cap) {
  std::vector<std::pair<int, int>> clusters, out;
  for (size_t p = 0; p < b0.size(); ++p) {
    if (b1[p] < b0[p]) continue;
    const int ga = b0[p] / 16, gb = b1[p] / 16;
    if (!clusters.empty() && ga <= clusters.back().second)
      clusters.back().second = std::max(clusters.back().second, gb);
    else
      clusters.push_back({ga, gb});
  }
  for (auto& c : clusters) {
    const int n = c.second - c.first + 1;
    if (n > cap) return {};
    if (!out.empty() && out.back().first + out.back().second == c.first &&
        out.back().second + n <= cap)
      out.back().second += n;
    else
      out.push_back({c.first, n});
  }
  return out;
}
/* launch plans that follow from the problems' body ranges and the
 * tuning: the problem-local PCG launches (pcg_ranges) and the component
 * labelling chunks (consecutive whole problems of at most label_rows
 * bodies; none if a problem is larger) */
int plan_launches(abd_ctx* ctx) {
  Scene& S = ctx->S;
  const int cap = ctx->tune.pcg_launch_groups > 0
                      ? std::min(ctx->tune.pcg_launch_groups, ctx->pcg_grid)
                      : ctx->pcg_grid;
  ctx->pcg_ranges = pcg_launch_ranges(ctx->hb0, ctx->hb1, cap);
  const int rows = ctx->tune.label_rows > 0 ? std::min(ctx->tune.label_rows, BSR_LDS_ROWS)
                                            : BSR_LDS_ROWS;
  S.bsr_one = S.B <= rows ? 1 : 0;
  std::vector<int> ch = {0};
  for (int p = 0; p < ctx->np; ++p) {
    const int b0 = ctx->hb0[p], b1 = ctx->hb1[p];
    if (b1 < b0) continue;
    if (b1 - b0 + 1 > rows) {
      ch.clear();
      break;
    }
    if (b1 + 1 - ch.back() > rows) ch.push_back(b0);
  }
  if (!ch.empty() && ch.back() < S.B) ch.push_back(S.B);
  S.n_lab_chunks = ch.size() >= 2 ? (int)ch.size() - 1 : 0;
  if (S.n_lab_chunks > 0)
    HIPCHK(hipMemcpy(S.lab_chunk, ch.data(), sizeof(int) * ch.size(), hipMemcpyHostToDevice));
  return ABD_OK;
}

/* blocks of the persistent PCG launch (at most the resident capacity) */
int pcg_blocks(const abd_ctx* ctx, const Scene& S) {
  const int ng = std::max(1, (S.B + 15) / 16);
  const int v = pcg_variant(ctx, S);
  if (v == ABD_PCG_LOCAL || v == ABD_PCG_LOCAL1) return ng;
  const int want = ctx->tune.pcg_blocks > 0 ? std::min(ctx->tune.pcg_blocks, ng) : ng;
  return std::max(1, std::min(ctx->pcg_grid, want));
}

/* the PCG of a pass on the stream: one launch, or one per range of the
 * problem-local forms */
int run_pcg(abd_ctx* ctx, const Scene& S) {
  const int v = pcg_variant(ctx, S);
  if (v == ABD_PCG_LOCAL || v == ABD_PCG_LOCAL1) {
    for (auto& r : ctx->pcg_ranges)
      if (launch_pcg(S, ctx->P.pcg_eta, ctx->P.max_pcg, r.second, v, r.first, ctx->st))
        return fail(ctx, ABD_E_DEVICE, "PCG launch failed");
    return ABD_OK;
  }
  if (launch_pcg(S, ctx->P.pcg_eta, ctx->P.max_pcg, pcg_blocks(ctx, S), v, 0, ctx->st))
    return fail(ctx, ABD_E_DEVICE, "PCG launch failed");
  return ABD_OK;
}

/* whether the block-row build labels the components of the system, so
 * that bodies alone and components of at most DIR_MAX bodies are solved
 * directly and only larger ones by the PCG (the problem-local
 * one-exchange form, which masks the others; every problem within one
 * labelling chunk) */
int comp_solve_on(const abd_ctx* ctx, const Scene& S) {
  return S.n_lab_chunks > 0 && pcg_variant(ctx, S) == ABD_PCG_LOCAL1 ? 1 : 0;
}

/* block-Jacobi PCG and the Newton stop norm on the stream */
int launch_solve(abd_ctx* ctx, const Scene& S0, bool in_loop) {
  Scene S = S0;
  S.comp_solve = comp_solve_on(ctx, S);
  {
    StageTimer t(ctx, 6);
    if (!in_loop) {
      /* the device loop's pass reset already cleared these */
      HIPCHK(hipMemsetAsync(S.row_cnt, 0, sizeof(int) * (S.B + 1), ctx->st));
      launch_reset_pcg(S, ctx->st);
    }
    launch_bsr(S, ctx->st);
    launch_block_inverse(S, ctx->st);
  }
  StageTimer t(ctx, 3);
  int rc = run_pcg(ctx, S);
  if (rc) return rc;
  launch_dq_norm(S, 0, ctx->st);
  return ABD_OK;
}

void account_pcg_bytes(abd_ctx* ctx) {
  if (!ctx->timing) return;
  const Scene& S = ctx->S;
  /* algorithmic bytes of the PCG launch: per iteration the diagonal and
   * used off-diagonal blocks once, the block inverses once and the
   * length-12B FP64 vectors read and written once each (two-barrier form:
   * z, p twice, Ap twice, r twice, dq twice less shared reads = 7 passes;
   * pipelined form: u, m, t, p, s, w, r, x read and u, m, t, p, s, w, r, x
   * written = 16 passes) */
  const double blk = 144.0 * (double)hess_elem(ctx);
  const double vec = pcg_variant(ctx, S) == ABD_PCG_PIPELINED ? 16.0 : 7.0;
  const double per = (double)(S.B + ctx->h_cnt[0].n_rows_used / 2) * blk +
                     (double)S.B * blk + vec * 12.0 * S.B * 8.0;
  ctx->t_bytes[3] += per * ctx->h_cnt[0].pcg_iters;
}

/* Algorithmic work of the barrier stage (distance filter and assembly) of
 * one pass, from the pass's static counters.  Bytes, each access counted
 * once with no cache reuse: per PT/EE candidate its 12-byte list entry and
 * four vertices (rest position 24 B and body id 4 B each), per ground
 * candidate 4 + 28 B; per active pair its 16-byte entry written and read,
 * its four vertices read again, three 12x12 blocks and two 12-gradients
 * read and written; per body pair its off-diagonal block and used flag
 * cleared.  Flops: about 100 per candidate distance and 22,300 per active
 * PT/EE pair (the distance derivatives and the 9x9 projection, about 20k,
 * and the mapping to three body blocks, about 2.3k), 30 per ground pair. */
void account_s5(abd_ctx* ctx) {
  if (ctx->timing != ABD_TIMING_ALL) return;
  const Counters& c = ctx->h_cnt[0];
  const Scene& S = ctx->S;
  const double hs = (double)hess_elem(ctx);
  const double cand = (double)std::min(c.n_pt, S.cap_pt) + std::min(c.n_ee, S.cap_ee);
  const double pg = std::min(c.n_pg, S.cap_pg);
  const double act = std::min(c.n_act, S.cap_act);
  const double nbp = std::min(c.n_bp, S.cap_bp);
  ctx->t_bytes[2] += cand * (12.0 + 4 * 28.0) + pg * 32.0 +
                     act * (2 * 16.0 + 4 * 28.0 + 3 * 144.0 * hs * 2 + 2 * 96.0 * 2) +
                     nbp * (144.0 * hs + 4.0);
  ctx->t_flops[2] += cand * 100.0 + pg * 10.0 + act * 22300.0;
}

/* Algorithmic work of the assembly kernel alone (stage 7, ABD_TIMING_ASM)
 * for one pass: per active pair its 16-byte entry and four vertices (rest
 * position 24 B and body id 4 B each) read, three 12x12 blocks and two
 * 12-gradients read and written (atomic additions), each counted once
 * with no cache reuse; 22,300 flops per active pair (the distance
 * derivatives and 9x9 projection of a PT/EE pair, about 20k, and the
 * mapping to three body blocks, about 2.3k; ground pairs need far fewer,
 * so scenes with a ground plane are overcounted). */
void account_asm(abd_ctx* ctx) {
  if (ctx->timing != ABD_TIMING_ASM) return;
  const Scene& S = ctx->S;
  const double hs = (double)hess_elem(ctx);
  const double act = std::min(ctx->h_cnt[0].n_act, S.cap_act);
  ctx->t_bytes[7] += act * (16.0 + 4 * 28.0 + 3 * 144.0 * hs * 2 + 2 * 96.0 * 2);
  ctx->t_flops[7] += act * 22300.0;
}

/* swept phase on the stream: broad phase over [q, q + dq], CCD, and the
 * energy difference at alpha_scale * min(1, TOI) */
void launch_swept(abd_ctx* ctx, bool ccd, bool energy_at_toi) {
  const Scene Ssw = swept_scene(ctx);
  if (ccd) launch_reset_toi(Ssw, ctx->st);
  launch_swept_s(ctx, Ssw, ccd);
  if (energy_at_toi) {
    StageTimer t(ctx, 5);
    launch_energy(Ssw, 1.0, 0 | (1 << 1), 1,
                  ctx->S.partials + ctx->S.cap_partials - 1, ctx->st);
  }
}

void launch_swept_s(abd_ctx* ctx, const Scene& Ssw, bool ccd, bool with_ctrl) {
  /* with the controller: the Newton stop test rides on the positions launch */
  broad_phase(ctx, Ssw, 1, with_ctrl ? 1 : 0);
  if (ccd) {
    StageTimer t(ctx, 4);
    launch_ccd(Ssw, with_ctrl ? 1 : 0, ctx->st);
  }
}

/* gradient and Hessian at the current q (static phase), counters read */
int assemble(abd_ctx* ctx) {
  for (int attempt = 0; attempt < 8; ++attempt) {
    int rc = reset_counters(ctx, 0);
    if (rc) return rc;
    launch_static(ctx, ctx->S);
    if ((rc = read_counters(ctx, 0))) return rc;
    bool changed = false;
    if ((rc = grow(ctx, ctx->h_cnt[0], &changed))) return rc;
    if (!changed) return ABD_OK;
  }
  return fail(ctx, ABD_E_OOM, "capacity growth did not settle");
}

/* PCG on the assembled system; counters read */
int linear_solve(abd_ctx* ctx, int* iters) {
  int rc = launch_solve(ctx, ctx->S, false);
  if (rc) return rc;
  if ((rc = read_counters(ctx, 0))) return rc;
  *iters = ctx->h_cnt[0].pcg_iters;
  account_pcg_bytes(ctx);
  return ABD_OK;
}

int upload_dq(abd_ctx* ctx, const double* dq) {
  HIPCHK(hipMemcpyAsync(ctx->S.dq, dq, sizeof(double) * 12 * ctx->S.B,
                        hipMemcpyHostToDevice, ctx->st));
  return ABD_OK;
}

/* swept candidates for the current dq, with capacity growth; counters read
 * (and, if energy_at_toi, the energy difference at the CCD step in
 * ctx->h_buf[0]) */
int swept_phase(abd_ctx* ctx, bool ccd, bool energy_at_toi = false) {
  for (int attempt = 0; attempt < 8; ++attempt) {
    int rc = reset_counters(ctx, 1);
    if (rc) return rc;
    launch_swept(ctx, ccd, energy_at_toi);
    if (energy_at_toi)
      HIPCHK(hipMemcpyAsync(ctx->h_buf, ctx->S.partials + ctx->S.cap_partials - 1,
                            sizeof(double), hipMemcpyDeviceToHost, ctx->st));
    if ((rc = read_counters(ctx, 1))) return rc;
    bool changed = false;
    if ((rc = grow(ctx, ctx->h_cnt[1], &changed))) return rc;
    if (!changed) return ABD_OK;
  }
  return fail(ctx, ABD_E_OOM, "capacity growth did not settle");
}

/* energy (mode 0: difference at alpha, mode 1: value) over the candidate
 * list of the given phase */
int energy(abd_ctx* ctx, int phase, double alpha, int mode, int with_pairs,
           double* out) {
  const Scene Sx = phase ? swept_scene(ctx) : ctx->S;
  {
    StageTimer t(ctx, 5);
    launch_energy(Sx, alpha, mode | (with_pairs << 1), 0,
                  ctx->S.partials + ctx->S.cap_partials - 1, ctx->st);
  }
  HIPCHK(hipMemcpyAsync(ctx->h_buf, ctx->S.partials + ctx->S.cap_partials - 1,
                        sizeof(double), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  resolve_timing(ctx);
  *out = ctx->h_buf[0];
  return ABD_OK;
}

/* swept broad phase and CCD on the stream for a given scene */

/* One pass of the device-driven Newton loop, queued without host
 * synchronisation: every problem in the Newton state assembles, solves
 * and checks |dq|; every problem not done runs the swept phase, CCD, the
 * trial energies of its line search and, on acceptance, its update. */
void pass_pre(abd_ctx* ctx, bool take_over) {
  Scene S1 = ctx->S;
  S1.iter_mode = 1;
  /* the pass reset runs in the first kernel of the static phase */
  const Counters fresh = fresh_counters();
  launch_static(ctx, S1, take_over, &fresh);
  StageTimer t(ctx, 6);
  S1.comp_solve = comp_solve_on(ctx, S1);
  launch_bsr(S1, ctx->st);
  launch_block_inverse(S1, ctx->st);
}

int pass_pcg(abd_ctx* ctx) {
  Scene S1 = ctx->S;
  S1.iter_mode = 1;
  StageTimer t(ctx, 3);
  return run_pcg(ctx, S1);
}

void pass_post(abd_ctx* ctx) {
  Scene S1 = ctx->S;
  S1.iter_mode = 1;
  Scene S2 = swept_scene(ctx);
  S2.iter_mode = 2;
  /* the controller runs in the last workgroup of the |dq| reduction (stop
   * test, part of the swept positions launch), of CCD (first trial step)
   * and of the trial energies (decision); the update's last workgroup ends
   * the pass */
  launch_swept_s(ctx, S2, true, true);
  {
    StageTimer t(ctx, 5);
    launch_energy_multi(S2, ctx->st);
  }
  launch_update_multi(S1, ctx->d_ring, ctx->d_pass, ctx->st);
}

/* capture one half of a pass into an executable graph */
bool capture(abd_ctx* ctx, int which, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(ctx->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  ctx->capturing = true;
  if (which == 1) {
    pass_post(ctx);
  } else if (which <= 2) {
    pass_pre(ctx, which == 2);
  } else {
    pass_pre(ctx, which == 4);
    if (pass_pcg(ctx)) {
      ctx->capturing = false;
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(ctx->st, &g);
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      return false;
    }
    pass_post(ctx);
  }
  ctx->capturing = false;
  hipError_t e = hipStreamEndCapture(ctx->st, &g);
  if (e != hipSuccess || !g) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    return false;
  }
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return false;
  }
  return true;
}

/* One pass of the device-driven Newton loop, queued without host
 * synchronisation: every problem in the Newton state assembles, solves
 * and checks |dq|; every problem not done runs the swept phase, CCD, the
 * trial energies of its line search and, on acceptance, its update.  The
 * parts before and after the PCG launch are replayed from
 * captured graphs when possible (not while every stage is timed,
 * and not on the legacy null stream, which cannot be captured).  With
 * take_over the first half skips the static broad phase and takes over the
 * previous pass's swept lists (a pass that finds none changes no state). */
int run_pass(abd_ctx* ctx, bool take_over, bool timed) {
  ctx->pcg_timed_now = timed;
  const bool graphs = ctx->tune.use_graphs && ctx->graphs_ok &&
                      ctx->timing != ABD_TIMING_ALL &&
                      ctx->st != nullptr;
  if (graphs && (!ctx->pass_graph[0] || !ctx->pass_graph[1] || !ctx->pass_graph[2])) {
    drop_graphs(ctx);
    if (!capture(ctx, 0, &ctx->pass_graph[0]) ||
        !capture(ctx, 1, &ctx->pass_graph[1]) ||
        !capture(ctx, 2, &ctx->pass_graph[2])) {
      drop_graphs(ctx);
      ctx->graphs_ok = false;
    } else if (ctx->whole_ok &&
               (!capture(ctx, 3, &ctx->pass_graph[3]) ||
                !capture(ctx, 4, &ctx->pass_graph[4]))) {
      /* a PCG launch that cannot be captured: halves only */
      for (int i = 3; i < 5; ++i)
        if (ctx->pass_graph[i]) {
          (void)hipGraphExecDestroy(ctx->pass_graph[i]);
          ctx->pass_graph[i] = nullptr;
        }
      ctx->whole_ok = false;
    }
  }
  /* a pass whose assembly launch is timed runs its kernels directly */
  if (timed && ctx->timing == ABD_TIMING_ASM) {
    pass_pre(ctx, take_over);
    int rc = pass_pcg(ctx);
    if (rc) return rc;
    pass_post(ctx);
    return ABD_OK;
  }
  if (graphs && ctx->graphs_ok && !timed && ctx->pass_graph[3] && ctx->pass_graph[4]) {
    HIPCHK(hipGraphLaunch(ctx->pass_graph[take_over ? 4 : 3], ctx->st));
    return ABD_OK;
  }
  if (graphs && ctx->graphs_ok) {
    HIPCHK(hipGraphLaunch(ctx->pass_graph[take_over ? 2 : 0], ctx->st));
    int rc = pass_pcg(ctx);
    if (rc) return rc;
    HIPCHK(hipGraphLaunch(ctx->pass_graph[1], ctx->st));
    return ABD_OK;
  }
  pass_pre(ctx, take_over);
  int rc = pass_pcg(ctx);
  if (rc) return rc;
  pass_post(ctx);
  return ABD_OK;
}

/* Device loop: passes until every problem is done.  The host keeps one
 * pass queued ahead of the one whose counters it checks (both counter
 * blocks are copied into a pinned ring slot at the end of every pass), so
 * the check and the next launch overlap the device's work.  A pass queued
 * after the last useful one finds every problem done and does nothing; a
 * pass queued after an overflowing one repeats it, since the controller
 * keeps the state of a pass whose lists overflowed. */
int device_solve(abd_ctx* ctx) {
  /* PCG launches outside the device loop are timed as before */
  struct TimedAgain {
    abd_ctx* c;
    ~TimedAgain() { c->pcg_timed_now = true; }
  } timed_again{ctx};
  launch_ctrl_start(ctx->S, ctx->st);
  ctx->h_last[0] = Counters{};
  ctx->h_last[1] = Counters{};
  ctx->h_last[0].min_dist = double_to_bits(INFINITY);
  const int max_pass =
      ctx->P.max_newton * (2 + (ctx->P.max_ls + LS_TRIALS) / LS_TRIALS) + 8;
  int queued = 0;
  /* the pass counter picks each pass's ring slot on the device */
  HIPCHK(hipMemsetAsync(ctx->d_pass, 0, sizeof(unsigned), ctx->st));
  /* the first pass runs the full static broad phase */
  HIPCHK(hipMemsetAsync(&ctx->S.cnt[1].sweep_ok, 0, sizeof(int), ctx->st));
  /* the first pass of the solve, and the first after the lists grew, run
   * the static broad phase; the others take over the swept lists */
  bool full = true;
  auto enqueue = [&]() -> int {
    /* the sample runs over all passes of the context, so it does not
     * favour the first passes of a solve */
    const bool timed = (ctx->timing == ABD_TIMING_PCG || ctx->timing == ABD_TIMING_ASM) &&
                       ctx->pass_seq++ % std::max(1, ctx->pcg_sample) == 0;
    ctx->pass_timed[queued & 1] = timed || ctx->timing == ABD_TIMING_ALL;
    int rc = run_pass(ctx, !full, timed); /* ends by writing its counters to the ring */
    if (rc) return rc;
    full = false;
    HIPCHK(hipEventRecord(ctx->ring_ev[queued & 1], ctx->st));
    queued += 1;
    return ABD_OK;
  };
  for (int k = 0; k < max_pass;) {
    int rc;
    while (queued < k + 2)
      if ((rc = enqueue())) return rc;
    HIPCHK(hipEventSynchronize(ctx->ring_ev[k & 1]));
    const Counters* c = ctx->h_ring + 2 * (k & 1);
    ctx->h_cnt[0] = c[0];
    ctx->h_cnt[1] = c[1];
    if (c[0].stat_ran) {
      ctx->h_last[0] = c[0];
      ctx->h_last[1] = c[1];
    }
    resolve_timing(ctx);
    if (c[0].err || c[1].err) {
      HIPCHK(hipStreamSynchronize(ctx->st));
      return fail(ctx, ABD_E_DEVICE, device_err_text(c[0].err | c[1].err));
    }
    if (over_cap(ctx->S, ctx->h_cnt[0]) || over_cap(ctx->S, ctx->h_cnt[1])) {
      /* drain, grow, and start over from the state the overflowing pass
       * left unchanged */
      HIPCHK(hipStreamSynchronize(ctx->st));
      if (ctx->no_alloc) return static_overflow_error(ctx);
      bool ch0 = false, ch1 = false;
      if ((rc = grow(ctx, ctx->h_cnt[0], &ch0))) return rc;
      if ((rc = grow(ctx, ctx->h_cnt[1], &ch1))) return rc;
      /* grown lists hold nothing to take over */
      HIPCHK(hipMemsetAsync(&ctx->S.cnt[1].sweep_ok, 0, sizeof(int), ctx->st));
      full = true;
      k = queued;
      continue;
    }
    if (ctx->pass_timed[k & 1]) {
      account_pcg_bytes(ctx);
      account_s5(ctx);
      account_asm(ctx);
    }
    if (ctx->S.mixed && ctx->h_cnt[0].want64 && ctx->h_cnt[1].active != 0) {
      /* a stalled mixed-precision problem: drain the queued pass and run
       * the rest of the solve with FP64 Hessians (same buffers, which are
       * sized for FP64); every problem keeps its state */
      HIPCHK(hipStreamSynchronize(ctx->st));
      if (!ctx->no_alloc) drop_graphs(ctx); /* no graphs run without allocation */
      ctx->S.mixed = 0;
      ctx->switched64 = true;
    }
    if (ctx->h_cnt[1].active == 0) {
      HIPCHK(hipStreamSynchronize(ctx->st));
      resolve_timing(ctx);
      return ABD_OK;
    }
    k += 1;
  }
  HIPCHK(hipStreamSynchronize(ctx->st));
  return fail(ctx, ABD_E_NOCONV, "device loop did not finish");
}

/* The local solve.  A mixed-precision solve in which a problem stops
 * making progress with FP32 Hessians (eps_N not halving for
 * MIXED_STALL_ITERS Newton iterations, or a third of the Newton cap spent)
 * continues from where it is with FP64 Hessians in the same buffers for
 * the rest of the solve; *fell_back reports the switch.  The scene is
 * mixed again for the next solve. */
int solve_with_fallback(abd_ctx* ctx, bool* fell_back) {
  Scene& S = ctx->S;
  const int mixed = S.mixed;
  ctx->switched64 = false;
  int rc = device_solve(ctx);
  *fell_back = ctx->switched64;
  if (ctx->switched64) {
    if (!ctx->no_alloc) drop_graphs(ctx);
    S.mixed = mixed;
  }
  return rc;
}

int check_ctx(abd_ctx* ctx, bool need_final) {
  if (!ctx) return ABD_E_INVALID_ARG;
  if (need_final && !ctx->finalized)
    return fail(ctx, ABD_E_INVALID_ARG, "context not finalized");
  HIPCHK(hipGetLastError());
  return ABD_OK;
}

}  // namespace

/* ==================================================================== */
/* C ABI                                                                 */
/* ==================================================================== */
extern "C" {

int abd_create(abd_ctx** out, const abd_params* p) {
  if (!out || !p) return ABD_E_INVALID_ARG;
  *out = nullptr;
  if (!(p->dt > 0) || !(p->dhat > 0) || !(p->kappa > 0) || !(p->kappa_A >= 0) ||
      p->max_newton < 1 || p->max_pcg < 1 || p->max_ls < 0 ||
      !(p->newton_theta > 0) || !(p->pcg_eta > 0) ||
      (p->precision != ABD_FP64 && p->precision != ABD_MIXED) || p->list_capacity < 0 ||
      p->mixed_switch < 0 || (p->deterministic != 0 && p->deterministic != 1))
    return ABD_E_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return ABD_E_DEVICE;
  }
  static std::atomic<uint64_t> next_serial{1};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return ABD_E_DEVICE;
  }
  /* the static scratch of this device, for abd_local_solve_static */
  if (scratch_init(dev)) return ABD_E_DEVICE;
  abd_ctx* c = new abd_ctx();
  c->serial = next_serial.fetch_add(1);
  c->device = dev;
  c->P = *p;
  std::memset(&c->S, 0, sizeof(Scene));
  *out = c;
  return ABD_OK;
}

void abd_destroy(abd_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  abd_batch_destroy(ctx->batch_cache);
  ctx->batch_cache = nullptr;
  drop_graphs(ctx);
  if (ctx->own_stream && ctx->st) (void)hipStreamDestroy(ctx->st);
  for (void* p : ctx->allocs) (void)hipFree(p);
  if (ctx->h_cnt) (void)hipHostFree(ctx->h_cnt);
  if (ctx->h_ring) (void)hipHostFree(ctx->h_ring);
  for (auto e : ctx->ring_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->h_buf) (void)hipHostFree(ctx->h_buf);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  delete ctx;
}

const char* abd_last_error(const abd_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

int abd_add_body(abd_ctx* ctx, const double* xbar, int32_t nv,
                 const int32_t* tris, int32_t nt, double density,
                 const double* q0, const double* qdot0, int32_t kind,
                 int32_t* body_id) {
  if (!ctx) return ABD_E_INVALID_ARG;
  if (ctx->finalized || !xbar || !tris || !q0 || nv <= 0 || nt <= 0 ||
      (kind != ABD_DYNAMIC && kind != ABD_STATIC) ||
      (kind == ABD_DYNAMIC && !(density > 0)))
    return fail(ctx, ABD_E_INVALID_ARG, "bad add_body arguments");
  for (int i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(xbar[i])) return fail(ctx, ABD_E_INVALID_ARG, "xbar");
  for (int i = 0; i < 12; ++i)
    if (!std::isfinite(q0[i]) || (qdot0 && !std::isfinite(qdot0[i])))
      return fail(ctx, ABD_E_INVALID_ARG, "non-finite state");
  for (int i = 0; i < 3 * nt; ++i)
    if (tris[i] < 0 || tris[i] >= nv) return fail(ctx, ABD_E_MESH, "triangle index");
  HBody b;
  std::memset(&b, 0, sizeof(b));
  b.kind = kind;
  b.density = density;
  b.v0 = (int)ctx->vbody.size();
  b.nv = nv;
  b.t0 = (int)(ctx->tri.size() / 3);
  b.nt = nt;
  std::memcpy(b.q0, q0, sizeof(b.q0));
  if (qdot0 && kind == ABD_DYNAMIC) std::memcpy(b.qd0, qdot0, sizeof(b.qd0));
  /* unique edges sorted by local (lo, hi) */
  std::vector<std::pair<int, int>> E;
  E.reserve(3 * nt);
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) {
      int a = tris[3 * t + k], c = tris[3 * t + (k + 1) % 3];
      E.push_back({std::min(a, c), std::max(a, c)});
    }
  std::sort(E.begin(), E.end());
  E.erase(std::unique(E.begin(), E.end()), E.end());
  if (kind == ABD_DYNAMIC) {
    std::vector<std::pair<int, int>> D;
    D.reserve(3 * nt);
    for (int t = 0; t < nt; ++t)
      for (int k = 0; k < 3; ++k)
        D.push_back({tris[3 * t + k], tris[3 * t + (k + 1) % 3]});
    std::sort(D.begin(), D.end());
    for (size_t i = 0; i < D.size(); ++i) {
      if (i > 0 && D[i] == D[i - 1])
        return fail(ctx, ABD_E_MESH, "repeated directed edge");
      if (!std::binary_search(D.begin(), D.end(),
                              std::make_pair(D[i].second, D[i].first)))
        return fail(ctx, ABD_E_MESH, "mesh not closed or not consistently oriented");
    }
    mass_props(xbar, tris, nt, density, b.Mhat, &b.vol);
    if (!(b.vol > 0)) return fail(ctx, ABD_E_MESH, "non-positive volume");
  }
  int id = (int)ctx->bodies.size();
  b.e0 = (int)ctx->erest2.size();
  b.ne = (int)E.size();
  for (int v = 0; v < nv; ++v) {
    for (int k = 0; k < 3; ++k) ctx->xbar.push_back(xbar[3 * v + k]);
    ctx->vbody.push_back(id);
  }
  for (int t = 0; t < 3 * nt; ++t) ctx->tri.push_back(b.v0 + tris[t]);
  for (auto& e : E) {
    ctx->edge.push_back(b.v0 + e.first);
    ctx->edge.push_back(b.v0 + e.second);
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
      double d = xbar[3 * e.second + k] - xbar[3 * e.first + k];
      s += d * d;
    }
    ctx->erest2.push_back(s);
  }
  ctx->bodies.push_back(b);
  if (body_id) *body_id = id;
  return ABD_OK;
}

int abd_finalize(abd_ctx* ctx) {
  int rc = check_ctx(ctx, false);
  if (rc) return rc;
  if (ctx->finalized || ctx->bodies.empty())
    return fail(ctx, ABD_E_INVALID_ARG, "finalize: no bodies or already final");
  Scene& S = ctx->S;
  const int B = (int)ctx->bodies.size(), V = (int)ctx->vbody.size();
  const int T = (int)(ctx->tri.size() / 3), E = (int)(ctx->edge.size() / 2);
  S.B = B; S.V = V; S.T = T; S.E = E;
  S.dt = ctx->P.dt; S.dhat = ctx->P.dhat; S.kappa = ctx->P.kappa;
  S.kappa_A = ctx->P.kappa_A;
  for (int i = 0; i < 3; ++i) S.grav[i] = ctx->P.gravity[i];
  S.ground_y = ctx->P.ground_y;
  S.has_ground = ctx->P.has_ground;
  S.mollify = ctx->P.mollify_ee;
  S.pair_mode = ctx->pair_mode;

  /* chunks per body and kind */
  std::vector<int> ch_body, ch_kind, ch_start, ch_count, ch_prims, body_chunk(6 * B);
  std::vector<double> ch_rest, body_rest(6 * B);
  const std::vector<double>& xb = ctx->xbar;
  for (int b = 0; b < B; ++b) {
    const HBody& hb = ctx->bodies[b];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int v = hb.v0; v < hb.v0 + hb.nv; ++v)
      for (int k = 0; k < 3; ++k) {
        lo[k] = std::min(lo[k], xb[3 * v + k]);
        hi[k] = std::max(hi[k], xb[3 * v + k]);
      }
    for (int k = 0; k < 3; ++k) {
      body_rest[6 * b + k] = 0.5 * (lo[k] + hi[k]);
      body_rest[6 * b + 3 + k] = 0.5 * (hi[k] - lo[k]);
    }
    for (int kind = 0; kind < 3; ++kind) {
      int first = kind == 0 ? hb.v0 : kind == 1 ? hb.t0 : hb.e0;
      int n = kind == 0 ? hb.nv : kind == 1 ? hb.nt : hb.ne;
      int nvper = kind == 0 ? 1 : kind == 1 ? 3 : 2;
      std::vector<double> cen(3 * n), pbox(6 * n);
      std::vector<int> ids(n);
      for (int i = 0; i < n; ++i) {
        ids[i] = i;
        double plo[3] = {INFINITY, INFINITY, INFINITY}, phi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int j = 0; j < nvper; ++j) {
          int v = kind == 0 ? first + i
                            : (kind == 1 ? ctx->tri[3 * (first + i) + j]
                                         : ctx->edge[2 * (first + i) + j]);
          for (int k = 0; k < 3; ++k) {
            plo[k] = std::min(plo[k], xb[3 * v + k]);
            phi[k] = std::max(phi[k], xb[3 * v + k]);
          }
        }
        for (int k = 0; k < 3; ++k) {
          cen[3 * i + k] = 0.5 * (plo[k] + phi[k]);
          pbox[6 * i + k] = plo[k];
          pbox[6 * i + 3 + k] = phi[k];
        }
      }
      std::vector<Leaf> leaves;
      split_leaves(ids, cen, pbox, hb.kind != ABD_DYNAMIC, ctx->P.dhat, leaves);
      body_chunk[6 * b + 2 * kind] = (int)ch_body.size();
      for (auto& L : leaves) {
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        ch_body.push_back(b);
        ch_kind.push_back(kind);
        ch_start.push_back((int)ch_prims.size());
        ch_count.push_back((int)L.ids.size());
        for (int i : L.ids) {
          ch_prims.push_back(first + i);
          for (int k = 0; k < 3; ++k) {
            clo[k] = std::min(clo[k], pbox[6 * i + k]);
            chi[k] = std::max(chi[k], pbox[6 * i + 3 + k]);
          }
        }
        for (int k = 0; k < 3; ++k) ch_rest.push_back(0.5 * (clo[k] + chi[k]));
        for (int k = 0; k < 3; ++k) ch_rest.push_back(0.5 * (chi[k] - clo[k]));
      }
      body_chunk[6 * b + 2 * kind + 1] = (int)ch_body.size();
    }
  }
  S.NC = (int)ch_body.size();

  /* geometry in structure-of-arrays layout */
  std::vector<double> xsoa(3L * V);
  for (int v = 0; v < V; ++v)
    for (int k = 0; k < 3; ++k) xsoa[(size_t)k * V + v] = xb[3 * v + k];
  std::vector<int> tsoa(3L * T), esoa(2L * E);
  for (int t = 0; t < T; ++t)
    for (int k = 0; k < 3; ++k) tsoa[(size_t)k * T + t] = ctx->tri[3 * t + k];
  for (int e = 0; e < E; ++e)
    for (int k = 0; k < 2; ++k) esoa[(size_t)k * E + e] = ctx->edge[2 * e + k];
  std::vector<double> q(12L * B), qd(12L * B), Mh(16L * B), vol(B), wb(B, 1.0);
  std::vector<int> kind(B), shs(B, -1);
  for (int b = 0; b < B; ++b) {
    const HBody& hb = ctx->bodies[b];
    std::memcpy(&q[12 * b], hb.q0, 96);
    std::memcpy(&qd[12 * b], hb.qd0, 96);
    std::memcpy(&Mh[16 * b], hb.Mhat, 128);
    vol[b] = hb.vol;
    kind[b] = hb.kind;
  }
  if ((rc = upload(ctx, &S.xbar, xsoa))) return rc;
  if ((rc = upload(ctx, &S.vbody, ctx->vbody))) return rc;
  if ((rc = upload(ctx, &S.tri, tsoa))) return rc;
  if ((rc = upload(ctx, &S.edge, esoa))) return rc;
  if ((rc = upload(ctx, &S.erest2, ctx->erest2))) return rc;
  if ((rc = upload(ctx, &S.q, q))) return rc;
  if ((rc = upload(ctx, &S.qt, q))) return rc;
  if ((rc = upload(ctx, &S.qtilde, q))) return rc;
  if ((rc = upload(ctx, &S.qdot, qd))) return rc;
  if ((rc = upload(ctx, &S.Mhat, Mh))) return rc;
  if ((rc = upload(ctx, &S.vol, vol))) return rc;
  if ((rc = upload(ctx, &S.wbody, wb))) return rc;
  if ((rc = upload(ctx, &S.kind, kind))) return rc;
  if ((rc = upload(ctx, &S.shared_slot, shs))) return rc;
  if ((rc = upload(ctx, &S.body_rest, body_rest))) return rc;
  if ((rc = upload(ctx, &S.body_chunk, body_chunk))) return rc;
  if ((rc = upload(ctx, &S.ch_body, ch_body))) return rc;
  if ((rc = upload(ctx, &S.ch_kind, ch_kind))) return rc;
  if ((rc = upload(ctx, &S.ch_start, ch_start))) return rc;
  if ((rc = upload(ctx, &S.ch_count, ch_count))) return rc;
  if ((rc = upload(ctx, &S.ch_prims, ch_prims))) return rc;
  if ((rc = upload(ctx, &S.ch_rest, ch_rest))) return rc;
  if ((rc = dalloc(ctx, &S.ch_box, 6L * S.NC))) return rc;
  if ((rc = dalloc(ctx, &S.body_box, 6L * B))) return rc;
  if ((rc = dalloc(ctx, &S.dq, 12L * B))) return rc;
  HIPCHK(hipMemset(S.dq, 0, sizeof(double) * 12 * B));
  if ((rc = dalloc(ctx, &S.z, 12))) return rc;
  if ((rc = dalloc(ctx, &S.u, 12))) return rc;
  if ((rc = dalloc(ctx, &S.rho, 1))) return rc;
  /* work buffers */
  S.cap_bp = std::max(4 * B, 4096);
  S.cap_cp = 1 << 16;
  S.cap_pt = S.cap_ee = S.cap_pg = S.cap_act = 1 << 16;
  if (ctx->P.list_capacity > 0) {
    const int c = (int)std::min<int64_t>(ctx->P.list_capacity, 1 << 29);
    S.cap_bp = S.cap_cp = S.cap_pt = S.cap_ee = S.cap_pg = S.cap_act = c;
  }
  S.cap_col = 2 * S.cap_bp;
  S.cap_partials = 1024;
  if ((rc = dalloc(ctx, &S.bp, S.cap_bp))) return rc;
  if ((rc = dalloc(ctx, &S.cp, S.cap_cp))) return rc;
  if ((rc = dalloc(ctx, &S.cand_pt, 3L * S.cap_pt))) return rc;
  if ((rc = dalloc(ctx, &S.cand_ee, 3L * S.cap_ee))) return rc;
  if ((rc = dalloc(ctx, &S.cand_pg, S.cap_pg))) return rc;
  if ((rc = dalloc(ctx, &S.act, S.cap_act))) return rc;
  S.cap_long = S.cap_pt + S.cap_ee;
  if ((rc = dalloc(ctx, &S.ccd_long, S.cap_long))) return rc;
  if ((rc = dalloc(ctx, &S.g, 12L * B))) return rc;
  S.mixed = ctx->P.precision == ABD_MIXED;
  if ((rc = dalloc_bytes(ctx, &S.Hdiag, 144L * B * HESS_ALLOC))) return rc;
  if ((rc = dalloc_bytes(ctx, &S.Pinv, 144L * B * HESS_ALLOC))) return rc;
  if ((rc = dalloc_bytes(ctx, &S.Hoff, 144L * S.cap_bp * HESS_ALLOC))) return rc;
  if ((rc = dalloc(ctx, &S.slot_used, S.cap_bp))) return rc;
  if ((rc = dalloc(ctx, &S.row_ptr, B + 1))) return rc;
  if ((rc = dalloc(ctx, &S.row_cnt, B + 1))) return rc;
  if ((rc = dalloc(ctx, &S.col_slot, S.cap_col))) return rc;
  if ((rc = dalloc(ctx, &S.col_body, S.cap_col))) return rc;
  if ((rc = dalloc(ctx, &S.col_trans, S.cap_col))) return rc;
  S.det = ctx->P.deterministic;
  if (S.det) {
    const size_t ng = (size_t)12 * DET_W * B, nh = (size_t)144 * DET_W * B,
                 no = (size_t)144 * DET_W * S.cap_bp;
    if ((rc = dalloc(ctx, &S.det_g, ng)) || (rc = dalloc(ctx, &S.det_hd, nh)) ||
        (rc = dalloc(ctx, &S.det_ho, no)))
      return rc;
    HIPCHK(hipMemset(S.det_g, 0, sizeof(det_word) * ng));
    HIPCHK(hipMemset(S.det_hd, 0, sizeof(det_word) * nh));
    HIPCHK(hipMemset(S.det_ho, 0, sizeof(det_word) * no));
  }
  if ((rc = dalloc(ctx, &S.bmode, B))) return rc;
  if ((rc = dalloc(ctx, &S.dir_body, (long)(B / 2 + 1) * DIR_MAX))) return rc;
  if ((rc = dalloc(ctx, &S.dir_n, B / 2 + 1))) return rc;
  if ((rc = dalloc(ctx, &S.r, 12L * B))) return rc;
  if ((rc = dalloc(ctx, &S.zv, 12L * B))) return rc;
  if ((rc = dalloc(ctx, &S.p0, 12L * B))) return rc;
  if ((rc = dalloc(ctx, &S.p1, 12L * B))) return rc;
  if ((rc = dalloc(ctx, &S.Ap, 12L * B))) return rc;
  if ((rc = dalloc(ctx, &S.acc, 16))) return rc;
  if ((rc = dalloc(ctx, &S.pw, 5 * 12L * B))) return rc;
  if ((rc = dalloc(ctx, &ctx->d_pass, 1))) return rc;
  if ((rc = dalloc(ctx, &S.pcg_rec, 2L * ((B + 15) / 16)))) return rc;
  HIPCHK(hipMemset(S.pcg_rec, 0, sizeof(PcgRec) * 2 * ((B + 15) / 16)));
  {
    std::vector<int> b0(ctx->np, B), b1(ctx->np, -1);
    for (int i = 0; i < B; ++i) {
      const int p = (int)ctx->prob_of_body.size() == B ? ctx->prob_of_body[i] : 0;
      b0[p] = std::min(b0[p], i);
      b1[p] = std::max(b1[p], i);
    }
    if ((rc = upload(ctx, &S.prob_b0, b0))) return rc;
    if ((rc = upload(ctx, &S.prob_b1, b1))) return rc;
    /* sort-and-sweep lists: each problem's dynamic and static bodies, and
     * one bucket per dynamic body (at most SAP_MAX_BUCKETS) */
    std::vector<int> dyn, doff(ctx->np + 1, 0), stat, soff(ctx->np + 1, 0),
        boff(ctx->np + 1, 0);
    for (int p = 0; p < ctx->np; ++p) {
      for (int i = b0[p]; i <= b1[p]; ++i) {
        const int pi = (int)ctx->prob_of_body.size() == B ? ctx->prob_of_body[i] : 0;
        if (pi != p) continue;
        if (kind[i] == ABD_DYNAMIC)
          dyn.push_back(i);
        else if (i >= (int)ctx->padding.size() || !ctx->padding[i])
          stat.push_back(i); /* padding bodies are far from every other */
      }
      doff[p + 1] = (int)dyn.size();
      soff[p + 1] = (int)stat.size();
      const int nd = doff[p + 1] - doff[p];
      boff[p + 1] = boff[p] + std::max(1, std::min(nd, SAP_MAX_BUCKETS)) + 1;
    }
    S.n_dyn = (int)dyn.size();
    if (dyn.empty()) dyn.push_back(0);
    if (stat.empty()) stat.push_back(0);
    if ((rc = upload(ctx, &S.sap_dyn, dyn))) return rc;
    if ((rc = upload(ctx, &S.sap_sorted, dyn))) return rc;
    if ((rc = upload(ctx, &S.sap_doff, doff))) return rc;
    if ((rc = upload(ctx, &S.sap_stat, stat))) return rc;
    if ((rc = upload(ctx, &S.sap_soff, soff))) return rc;
    if ((rc = upload(ctx, &S.sap_boff, boff))) return rc;
    if ((rc = dalloc(ctx, &S.sap_bstart, (size_t)boff[ctx->np]))) return rc;
    if ((rc = dalloc(ctx, &S.sap_par, (size_t)ctx->np))) return rc;
    if ((rc = dalloc(ctx, &S.sap_sbox, 6 * dyn.size()))) return rc;
    /* the all-pairs tiles, unless they would be very many */
    long tests = 0;
    for (int p = 0; p < ctx->np; ++p) {
      const long n = std::max(0, b1[p] - b0[p] + 1);
      tests += n * (n - 1) / 2;
    }
    ctx->bp_tests = tests;
    S.sap_on = sap_on(ctx);
    std::vector<int2> tiles;
    if (tests <= ALL_PAIRS_BUILD_MAX)
      for (int p = 0; p < ctx->np; ++p) {
        if (b1[p] < b0[p]) continue;
        for (int ta = b0[p] / 16; ta <= b1[p] / 16; ++ta)
          for (int tb = ta; tb <= b1[p] / 16; ++tb) tiles.push_back(make_int2(ta, tb));
      }
    /* problems that share a tile list it once */
    std::sort(tiles.begin(), tiles.end(), [](int2 x, int2 y) {
      return x.x != y.x ? x.x < y.x : x.y < y.y;
    });
    tiles.erase(std::unique(tiles.begin(), tiles.end(),
                            [](int2 x, int2 y) { return x.x == y.x && x.y == y.y; }),
                tiles.end());
    S.n_bp_tiles = (int)tiles.size();
    if (tiles.empty()) tiles.push_back(make_int2(0, 0));
    if ((rc = upload(ctx, &S.bp_tiles, tiles))) return rc;
  }
  S.grid_blocks = ctx->tune.grid_blocks;
  S.assemble_blocks = ctx->tune.assemble_blocks;
  if ((rc = dalloc(ctx, &S.partials, S.cap_partials))) return rc;
  if ((rc = dalloc(ctx, &S.cnt, 2))) return rc;
  S.NP = ctx->np;
  S.theta = ctx->P.newton_theta;
  S.eta = ctx->P.pcg_eta;
  S.max_newton = ctx->P.max_newton;
  S.max_ls = ctx->P.max_ls;
  S.max_pcg = ctx->P.max_pcg;
  S.mixed_switch = ctx->P.mixed_switch > 0
                       ? ctx->P.mixed_switch
                       : std::max(1, ctx->P.max_newton / 3);
  S.iter_mode = 0;
  {
    std::vector<int> bp0(B, 0);
    if ((int)ctx->prob_of_body.size() == B) bp0 = ctx->prob_of_body;
    if ((rc = upload(ctx, &S.bprob, bp0))) return rc;
    if ((rc = dalloc(ctx, &S.ps, S.NP))) return rc;
    HIPCHK(hipMemset(S.ps, 0, sizeof(ProbState) * S.NP));
    if (S.det) {
      const size_t nd = (size_t)S.NP * LS_TRIALS * (DET_W + 1);
      if ((rc = dalloc(ctx, &S.det_de, nd))) return rc;
      HIPCHK(hipMemset(S.det_de, 0, sizeof(det_word) * nd));
    }
  }
  if (hipHostMalloc((void**)&ctx->h_cnt, 2 * sizeof(Counters)) != hipSuccess ||
      hipHostMalloc((void**)&ctx->h_ring, 4 * sizeof(Counters)) != hipSuccess ||
      hipHostGetDevicePointer((void**)&ctx->d_ring, ctx->h_ring, 0) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ring_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ring_ev[1], hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&ctx->h_buf, 64 * sizeof(double)) != hipSuccess)
    return fail(ctx, ABD_E_OOM, "pinned host allocation failed");
  ctx->pcg_grid = pcg_max_grid();
  {
    ctx->hb0.assign(ctx->np, B);
    ctx->hb1.assign(ctx->np, -1);
    for (int i = 0; i < B; ++i) {
      const int p = (int)ctx->prob_of_body.size() == B ? ctx->prob_of_body[i] : 0;
      ctx->hb0[p] = std::min(ctx->hb0[p], i);
      ctx->hb1[p] = std::max(ctx->hb1[p], i);
    }
    if ((rc = dalloc(ctx, &S.lab_chunk, (size_t)ctx->np + 2))) return rc;
    if ((rc = dalloc(ctx, &S.chunk_tot, (size_t)ctx->np + 2))) return rc;
    if ((rc = plan_launches(ctx))) return rc;
    if (ctx->P.deterministic && ctx->pcg_ranges.empty())
      return fail(ctx, ABD_E_INVALID_ARG,
                  "deterministic mode: a problem has more 16-body groups than the "
                  "problem-local PCG holds resident");
  }
  {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  }
  if (!ctx->st) {
    /* a stream of the library's own (default priority): the legacy null
     * stream cannot be captured into graphs */
    HIPCHK(hipStreamCreateWithFlags(&ctx->st, hipStreamNonBlocking));
    ctx->own_stream = true;
  }
  HIPCHK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  ctx->finalized = true;
  /* initial feasibility: every candidate distance > 0 */
  if ((rc = assemble(ctx))) return rc;
  double md = bits_to_double(ctx->h_cnt[0].min_dist);
  if (!(md > 0.0)) {
    ctx->finalized = false;
    return fail(ctx, ABD_E_INFEASIBLE, "initial state has a distance <= 0");
  }
  /* and no edge of one body crosses a triangle of another (the counter
   * block's active count is reused as the crossing counter) */
  if ((rc = reset_counters(ctx, 0))) return rc;
  broad_phase(ctx, S, 0);
  launch_crossings(S, ctx->st);
  if ((rc = read_counters(ctx, 0))) return rc;
  if (ctx->h_cnt[0].n_act > 0) {
    ctx->finalized = false;
    return fail(ctx, ABD_E_INFEASIBLE, "initial state has intersecting bodies");
  }
  return ABD_OK;
}

int abd_check_penetration(abd_ctx* ctx, int64_t* n_cross, double* min_dist) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (!n_cross || !min_dist) return fail(ctx, ABD_E_INVALID_ARG, "check_penetration");
  Scene& S = ctx->S;
  S.iter_mode = 0;
  if ((rc = assemble(ctx))) return rc;
  *min_dist = bits_to_double(ctx->h_cnt[0].min_dist);
  if ((rc = reset_counters(ctx, 0))) return rc;
  broad_phase(ctx, S, 0);
  launch_crossings(S, ctx->st);
  if ((rc = read_counters(ctx, 0))) return rc;
  *n_cross = ctx->h_cnt[0].n_act;
  return ABD_OK;
}

int abd_sizes(const abd_ctx* ctx, int64_t* sizes) {
  if (!ctx || !sizes) return ABD_E_INVALID_ARG;
  sizes[0] = (int64_t)ctx->bodies.size();
  sizes[1] = (int64_t)ctx->vbody.size();
  sizes[2] = (int64_t)(ctx->tri.size() / 3);
  sizes[3] = (int64_t)(ctx->edge.size() / 2);
  return ABD_OK;
}

int abd_set_shared(abd_ctx* ctx, const int32_t* ids, int32_t n,
                   const double* z, const double* u, const double* rho,
                   const int32_t* kappa_b) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  const int B = ctx->S.B;
  if (n < 0 || (n > 0 && (!ids || !z || !u || !rho || !kappa_b)))
    return fail(ctx, ABD_E_INVALID_ARG, "set_shared arguments");
  std::vector<int> slot(B, -1);
  std::vector<double> wb(B, 1.0);
  for (int i = 0; i < n; ++i) {
    int b = ids[i];
    if (b < 0 || b >= B || ctx->bodies[b].kind != ABD_DYNAMIC || slot[b] >= 0)
      return fail(ctx, ABD_E_INVALID_ARG, "shared id");
    for (int k = 0; k < 12; ++k)
      if (!std::isfinite(z[12 * i + k]) || !std::isfinite(u[12 * i + k]))
        return fail(ctx, ABD_E_INVALID_ARG, "non-finite z or u");
    if (!(rho[i] >= 0) || !std::isfinite(rho[i]) || kappa_b[i] < 1)
      return fail(ctx, ABD_E_INVALID_ARG, "rho or kappa_b");
    slot[b] = i;
    wb[b] = 1.0 / kappa_b[i];
  }
  Scene& S = ctx->S;
  if (n > ctx->n_shared) {
    drop_graphs(ctx); /* z, u, rho move */
    dfree(ctx, S.z);
    dfree(ctx, S.u);
    dfree(ctx, S.rho);
    if ((rc = dalloc(ctx, &S.z, 12L * n))) return rc;
    if ((rc = dalloc(ctx, &S.u, 12L * n))) return rc;
    if ((rc = dalloc(ctx, &S.rho, n))) return rc;
    ctx->n_shared = n;
  }
  ctx->sh_ids.assign(ids, ids + n);
  ctx->sh_kappa.assign(kappa_b, kappa_b + n);
  ctx->sh_z.assign(z, z + 12L * n);
  ctx->sh_u.assign(u, u + 12L * n);
  ctx->sh_rho.assign(rho, rho + n);
  ctx->sh_version += 1;
  if (n > 0) {
    HIPCHK(hipMemcpy(S.z, z, sizeof(double) * 12 * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.u, u, sizeof(double) * 12 * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.rho, rho, sizeof(double) * n, hipMemcpyHostToDevice));
  }
  HIPCHK(hipMemcpy(S.shared_slot, slot.data(), sizeof(int) * B, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(S.wbody, wb.data(), sizeof(double) * B, hipMemcpyHostToDevice));
  return ABD_OK;
}

int abd_set_pair_replication(abd_ctx* ctx, int32_t mode) {
  if (!ctx) return ABD_E_INVALID_ARG;
  if (mode != ABD_PAIRS_ALL_ONE && mode != ABD_PAIRS_BY_SHARED)
    return fail(ctx, ABD_E_INVALID_ARG, "pair replication mode");
  ctx->pair_mode = mode;
  ctx->S.pair_mode = mode;
  drop_graphs(ctx);
  return ABD_OK;
}

int abd_begin_step(abd_ctx* ctx) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  const Scene& S = ctx->S;
  launch_predict(S, ctx->st);
  /* scene scale from the dynamic vertices */
  unsigned long long init[6];
  double pinf = INFINITY, ninf = -INFINITY;
  unsigned long long bp, bn;
  std::memcpy(&bp, &pinf, 8);
  std::memcpy(&bn, &ninf, 8);
  /* ordered images: +inf -> bp | sign, -inf -> ~bn */
  for (int k = 0; k < 3; ++k) {
    init[k] = bp | 0x8000000000000000ull;
    init[3 + k] = ~bn;
  }
  unsigned long long* d6 = (unsigned long long*)S.partials;
  HIPCHK(hipMemcpyAsync(d6, init, sizeof(init), hipMemcpyHostToDevice, ctx->st));
  launch_scale(S, (double*)d6, ctx->st);
  unsigned long long out[6];
  HIPCHK(hipMemcpyAsync(out, d6, sizeof(out), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  double l2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    auto dec = [](unsigned long long o) {
      unsigned long long b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
      return bits_to_double(b);
    };
    double lo = dec(out[k]), hi = dec(out[3 + k]);
    if (std::isfinite(lo) && std::isfinite(hi)) l2 += (hi - lo) * (hi - lo);
  }
  ctx->scale = l2 > 0 ? std::sqrt(l2) : 1.0;
  HIPCHK(hipMemcpy(&ctx->S.ps[0].scale, &ctx->scale, sizeof(double),
                   hipMemcpyHostToDevice));
  return ABD_OK;
}

int abd_set_step(abd_ctx* ctx, const double* qt, const double* qtilde,
                 double scale) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (!qt || !qtilde || !(scale > 0)) return fail(ctx, ABD_E_INVALID_ARG, "set_step");
  HIPCHK(hipMemcpy(ctx->S.qt, qt, sizeof(double) * 12 * ctx->S.B, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(ctx->S.qtilde, qtilde, sizeof(double) * 12 * ctx->S.B,
                   hipMemcpyHostToDevice));
  ctx->scale = scale;
  HIPCHK(hipMemcpy(&ctx->S.ps[0].scale, &ctx->scale, sizeof(double),
                   hipMemcpyHostToDevice));
  return ABD_OK;
}

int abd_local_solve(abd_ctx* ctx, abd_stats* out) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  auto t0 = std::chrono::steady_clock::now();
  abd_stats st;
  std::memset(&st, 0, sizeof(st));
  st.scene_scale = ctx->scale;
  bool fell_back = false;
  int status = solve_with_fallback(ctx, &fell_back);
  st.fp64_fallback = fell_back ? 1 : 0;
  ProbState P;
  std::memset(&P, 0, sizeof(P));
  if (hipMemcpy(&P, ctx->S.ps, sizeof(P), hipMemcpyDeviceToHost) != hipSuccess)
    status = fail(ctx, ABD_E_DEVICE, "reading the solve state failed");
  if (status == ABD_OK) {
    status = P.status;
    if (status == ABD_E_NOCONV) ctx->err = "Newton did not converge";
    if (status == ABD_E_LINESEARCH) ctx->err = "line search exhausted";
  }
  const Counters& c = ctx->h_last[0];
  st.newton_iters = P.newton;
  st.newton_fp32 = P.newton32;
  st.pcg_iters_total = P.pcg_total;
  st.ls_halvings = P.halvings;
  st.final_eps_N = P.final_eps;
  st.min_alpha = P.min_alpha;
  st.n_cand_pt = c.n_pt;
  st.n_cand_ee = c.n_ee;
  st.n_cand_pg = c.n_pg;
  st.n_active = c.n_act;
  st.n_body_pairs = c.n_bp;
  st.n_chunk_pairs = c.n_cp;
  st.n_body_pairs_swept = ctx->h_last[1].n_bp;
  st.n_chunk_pairs_swept = ctx->h_last[1].n_cp;
  st.min_dist = bits_to_double(c.min_dist);
  st.status = status;
  st.t_solve_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (out) *out = st;
  return status;
}

/* Maximum list sizes of the allocation-free solve: the static scratch
 * holds every list of a solve at these capacities (about 61 MB of the
 * 64 MiB array). */
#define ABD_STATIC_BP (32 << 10)
#define ABD_STATIC_CP (256 << 10)
#define ABD_STATIC_PT (512 << 10)
#define ABD_STATIC_EE (512 << 10)
#define ABD_STATIC_PG (256 << 10)
#define ABD_STATIC_ACT (256 << 10)
#define ABD_STATIC_LONG (16 << 10)

int abd_local_solve_static(abd_ctx* ctx, abd_stats* out) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (ctx->capturing) return fail(ctx, ABD_E_INVALID_ARG, "solve during capture");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != ctx->device)
    return fail(ctx, ABD_E_INVALID_ARG, "the context's device is not current");
  if (ctx->P.deterministic)
    return fail(ctx, ABD_E_INVALID_ARG, "the static solve has no deterministic mode");
  unsigned char* base = (unsigned char*)g_scratch[ctx->device].load();
  if (!base) return fail(ctx, ABD_E_DEVICE, "static scratch not available");
  Scene& S = ctx->S;
  /* the lists of this solve, carved from the scratch at fixed capacities */
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return (void*)p;
  };
  Scene L = S;
  L.cap_bp = ABD_STATIC_BP;
  L.cap_col = 2 * L.cap_bp;
  L.cap_cp = ABD_STATIC_CP;
  L.cap_pt = ABD_STATIC_PT;
  L.cap_ee = ABD_STATIC_EE;
  L.cap_pg = ABD_STATIC_PG;
  L.cap_act = ABD_STATIC_ACT;
  L.bp = (int2*)take(sizeof(int2) * (size_t)L.cap_bp);
  L.Hoff = take(144 * sizeof(double) * (size_t)L.cap_bp);
  L.slot_used = (int*)take(sizeof(int) * (size_t)L.cap_bp);
  L.col_slot = (int*)take(sizeof(int) * (size_t)L.cap_col);
  L.col_body = (int*)take(sizeof(int) * (size_t)L.cap_col);
  L.col_trans = (int*)take(sizeof(int) * (size_t)L.cap_col);
  L.cp = (int4*)take(sizeof(int4) * (size_t)L.cap_cp);
  L.cand_pt = (int*)take(3 * sizeof(int) * (size_t)L.cap_pt);
  L.cand_ee = (int*)take(3 * sizeof(int) * (size_t)L.cap_ee);
  L.cand_pg = (int*)take(sizeof(int) * (size_t)L.cap_pg);
  L.act = (int4*)take(sizeof(int4) * (size_t)L.cap_act);
  L.cap_long = ABD_STATIC_LONG;
  L.ccd_long = (CcdLong*)take(sizeof(CcdLong) * (size_t)L.cap_long);
  if (off > ABD_SCRATCH_BYTES)
    return fail(ctx, ABD_E_DEVICE, "static scratch layout exceeds the array");
  /* swap the context's lists for the scratch ones for this call: direct
   * launches (no graph replay, whose captured launches hold the context's
   * own lists) and no stage timing (its events are created on demand) */
  const Scene saved = S;
  const int timing = ctx->timing, graphs = ctx->tune.use_graphs;
  S = L;
  ctx->no_alloc = true;
  ctx->timing = ABD_TIMING_OFF;
  ctx->tune.use_graphs = 0;
  rc = abd_local_solve(ctx, out);
  /* back to the context's own lists: only the list fields were swapped, so
   * everything else of the scene (mixed flag, state pointers) is kept */
  S.bp = saved.bp;
  S.Hoff = saved.Hoff;
  S.slot_used = saved.slot_used;
  S.col_slot = saved.col_slot;
  S.col_body = saved.col_body;
  S.col_trans = saved.col_trans;
  S.cp = saved.cp;
  S.cand_pt = saved.cand_pt;
  S.cand_ee = saved.cand_ee;
  S.cand_pg = saved.cand_pg;
  S.act = saved.act;
  S.ccd_long = saved.ccd_long;
  S.cap_long = saved.cap_long;
  S.cap_bp = saved.cap_bp;
  S.cap_col = saved.cap_col;
  S.cap_cp = saved.cap_cp;
  S.cap_pt = saved.cap_pt;
  S.cap_ee = saved.cap_ee;
  S.cap_pg = saved.cap_pg;
  S.cap_act = saved.cap_act;
  ctx->no_alloc = false;
  ctx->timing = timing;
  ctx->tune.use_graphs = graphs;
  return rc;
}

int abd_end_step(abd_ctx* ctx) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  launch_commit(ctx->S, ctx->st);
  HIPCHK(hipStreamSynchronize(ctx->st));
  return ABD_OK;
}

int abd_get_state(const abd_ctx* cctx, double* q, double* qdot) {
  abd_ctx* ctx = const_cast<abd_ctx*>(cctx);
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(ctx->st));
  size_t n = sizeof(double) * 12 * ctx->S.B;
  if (q) HIPCHK(hipMemcpy(q, ctx->S.q, n, hipMemcpyDeviceToHost));
  if (qdot) HIPCHK(hipMemcpy(qdot, ctx->S.qdot, n, hipMemcpyDeviceToHost));
  return ABD_OK;
}

int abd_set_state(abd_ctx* ctx, const double* q, const double* qdot) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  const int B = ctx->S.B;
  std::vector<double> hq(12L * B), hqd(12L * B);
  HIPCHK(hipStreamSynchronize(ctx->st));
  HIPCHK(hipMemcpy(hq.data(), ctx->S.q, sizeof(double) * 12 * B, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(hqd.data(), ctx->S.qdot, sizeof(double) * 12 * B, hipMemcpyDeviceToHost));
  for (int b = 0; b < B; ++b) {
    if (ctx->bodies[b].kind != ABD_DYNAMIC) continue;
    for (int i = 0; i < 12; ++i) {
      if (q) {
        if (!std::isfinite(q[12 * b + i])) return fail(ctx, ABD_E_INVALID_ARG, "q");
        hq[12 * b + i] = q[12 * b + i];
      }
      if (qdot) {
        if (!std::isfinite(qdot[12 * b + i])) return fail(ctx, ABD_E_INVALID_ARG, "qdot");
        hqd[12 * b + i] = qdot[12 * b + i];
      }
    }
  }
  HIPCHK(hipMemcpy(ctx->S.q, hq.data(), sizeof(double) * 12 * B, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(ctx->S.qdot, hqd.data(), sizeof(double) * 12 * B, hipMemcpyHostToDevice));
  return ABD_OK;
}

int abd_get_qtilde(const abd_ctx* cctx, double* qtilde) {
  abd_ctx* ctx = const_cast<abd_ctx*>(cctx);
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(ctx->st));
  HIPCHK(hipMemcpy(qtilde, ctx->S.qtilde, sizeof(double) * 12 * ctx->S.B,
                   hipMemcpyDeviceToHost));
  return ABD_OK;
}

int abd_bind_workspace(abd_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return ABD_E_INVALID_ARG;
  if (ctx->finalized || ctx->ws_base)
    return fail(ctx, ABD_E_INVALID_ARG,
                "a workspace is bound once, before abd_finalize");
  if (!dev_ptr || bytes < 256)
    return fail(ctx, ABD_E_INVALID_ARG, "workspace pointer or size invalid");
  hipPointerAttribute_t at;
  int dev = -1;
  if (hipPointerGetAttributes(&at, dev_ptr) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, ABD_E_INVALID_ARG, "workspace is not device memory");
  }
  if (at.type != hipMemoryTypeDevice || at.device != dev)
    return fail(ctx, ABD_E_INVALID_ARG,
                "workspace is not device memory of the current device");
  char* b = (char*)dev_ptr;
  const size_t pad = (256 - (uintptr_t)b % 256) % 256;
  ctx->ws_base = b + pad;
  ctx->ws_size = bytes - pad;
  ctx->ws_top = ctx->ws_peak = 0;
  ctx->ws_blocks.clear();
  return ABD_OK;
}

int abd_workspace_info(const abd_ctx* ctx, int64_t* info) {
  if (!ctx || !info) return ABD_E_INVALID_ARG;
  info[0] = (int64_t)ctx->ws_size;
  info[1] = (int64_t)ctx->ws_top;
  info[2] = (int64_t)ctx->ws_peak;
  return ABD_OK;
}

int abd_balance_update(abd_balance* b, double t1, double t2, double* dp) {
  if (!b || !dp || !std::isfinite(t1) || !std::isfinite(t2) || !(t1 > 0.0) ||
      !(t2 > 0.0) || !(b->smooth > 0.0 && b->smooth <= 1.0) ||
      !std::isfinite(b->k_p) || !std::isfinite(b->k_d))
    return ABD_E_INVALID_ARG;
  if (b->frames <= 0) {
    b->tau[0] = t1;
    b->tau[1] = t2;
  } else {
    b->tau[0] = (1.0 - b->smooth) * b->tau[0] + b->smooth * t1;
    b->tau[1] = (1.0 - b->smooth) * b->tau[1] + b->smooth * t2;
  }
  const double eta = b->tau[0] / b->tau[1];
  const double T = (eta - 1.0) / (eta + 1.0); /* Eq. 13 */
  const double Tp = b->frames <= 0 ? T : b->T_prev;
  *dp = b->k_p * T + b->k_d * (T - Tp); /* Eq. 14 */
  b->T_prev = T;
  b->frames = b->frames <= 0 ? 1 : b->frames + 1;
  return ABD_OK;
}

int abd_set_stream(abd_ctx* ctx, void* hip_stream) {
  if (!ctx) return ABD_E_INVALID_ARG;
  drop_graphs(ctx);
  if (ctx->own_stream && ctx->st) {
    (void)hipStreamSynchronize(ctx->st);
    (void)hipStreamDestroy(ctx->st);
    ctx->own_stream = false;
  }
  ctx->st = (hipStream_t)hip_stream;
  return ABD_OK;
}

int abd_get_vertices(abd_ctx* ctx, const double* q, const double* dq,
                     double* x, double* dx) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  Scene& S = ctx->S;
  std::vector<double> save;
  double *dx_d = nullptr, *x_d = nullptr;
  if ((rc = dalloc(ctx, &x_d, 3L * S.V))) return rc;
  if (dq && dx && (rc = dalloc(ctx, &dx_d, 3L * S.V))) { dfree(ctx, x_d); return rc; }
  if (q) {
    save.resize(12L * S.B);
    HIPCHK(hipMemcpy(save.data(), S.q, sizeof(double) * 12 * S.B, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(S.q, q, sizeof(double) * 12 * S.B, hipMemcpyHostToDevice));
  }
  if (dq && dx) HIPCHK(hipMemcpy(S.dq, dq, sizeof(double) * 12 * S.B, hipMemcpyHostToDevice));
  launch_transform(S, x_d, dx_d, ctx->st);
  HIPCHK(hipStreamSynchronize(ctx->st));
  HIPCHK(hipMemcpy(x, x_d, sizeof(double) * 3 * S.V, hipMemcpyDeviceToHost));
  if (dx_d) HIPCHK(hipMemcpy(dx, dx_d, sizeof(double) * 3 * S.V, hipMemcpyDeviceToHost));
  if (q) HIPCHK(hipMemcpy(S.q, save.data(), sizeof(double) * 12 * S.B, hipMemcpyHostToDevice));
  dfree(ctx, x_d);
  dfree(ctx, dx_d);
  return ABD_OK;
}

int abd_export_candidates(abd_ctx* ctx, int32_t kind, const double* dq,
                          int32_t* out, int64_t cap, int64_t* count) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (kind < ABD_PT || kind > ABD_PG || !count)
    return fail(ctx, ABD_E_INVALID_ARG, "export_candidates");
  const Scene& S = ctx->S;
  if (dq) {
    if ((rc = upload_dq(ctx, dq))) return rc;
    if ((rc = swept_phase(ctx, false))) return rc;
  } else {
    for (int attempt = 0; attempt < 8; ++attempt) {
      if ((rc = reset_counters(ctx, 0))) return rc;
      broad_phase(ctx, S, 0);
      if ((rc = read_counters(ctx, 0))) return rc;
      bool changed;
      if ((rc = grow(ctx, ctx->h_cnt[0], &changed))) return rc;
      if (!changed) break;
    }
  }
  const Counters& c = ctx->h_cnt[dq ? 1 : 0];
  int n = kind == ABD_PT ? c.n_pt : kind == ABD_EE ? c.n_ee : c.n_pg;
  *count = n;
  if (!out) return ABD_OK;
  if (n > cap) return fail(ctx, ABD_E_CAPACITY, "candidate buffer too small");
  if (kind == ABD_PG) {
    std::vector<int> v(n);
    if (n) HIPCHK(hipMemcpy(v.data(), S.cand_pg, sizeof(int) * n, hipMemcpyDeviceToHost));
    std::sort(v.begin(), v.end());
    std::copy(v.begin(), v.end(), out);
  } else {
    std::vector<int> v(3L * n);
    if (n)
      HIPCHK(hipMemcpy(v.data(), kind == ABD_PT ? S.cand_pt : S.cand_ee,
                       sizeof(int) * 3 * n, hipMemcpyDeviceToHost));
    std::vector<std::pair<int, int>> pr(n);
    for (int i = 0; i < n; ++i) pr[i] = {v[3 * i], v[3 * i + 1]};
    std::sort(pr.begin(), pr.end());
    for (int i = 0; i < n; ++i) {
      out[2 * i] = pr[i].first;
      out[2 * i + 1] = pr[i].second;
    }
  }
  return ABD_OK;
}

int abd_eval(abd_ctx* ctx, const double* q, double* E, double* g,
             double* Hdiag, int64_t cap, int64_t* n_off, int32_t* off_ij,
             double* Hoff, int64_t* n_active) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  Scene& S = ctx->S;
  const int B = S.B;
  std::vector<double> save(12L * B);
  HIPCHK(hipStreamSynchronize(ctx->st));
  HIPCHK(hipMemcpy(save.data(), S.q, sizeof(double) * 12 * B, hipMemcpyDeviceToHost));
  if (q) HIPCHK(hipMemcpy(S.q, q, sizeof(double) * 12 * B, hipMemcpyHostToDevice));
  rc = assemble(ctx);
  if (!rc && E) rc = energy(ctx, 0, 0.0, 1, 1, E);
  if (!rc) {
    if (n_active) *n_active = ctx->h_cnt[0].n_act;
    if (g) HIPCHK(hipMemcpy(g, S.g, sizeof(double) * 12 * B, hipMemcpyDeviceToHost));
    if (Hdiag) {
      if (S.mixed) {
        std::vector<float> h(144L * B);
        HIPCHK(hipMemcpy(h.data(), S.Hdiag, sizeof(float) * 144 * B, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < h.size(); ++i) Hdiag[i] = h[i];
      } else {
        HIPCHK(hipMemcpy(Hdiag, S.Hdiag, sizeof(double) * 144 * B, hipMemcpyDeviceToHost));
      }
    }
    int nbp = ctx->h_cnt[0].n_bp;
    std::vector<int> used(nbp);
    std::vector<int2> bp(nbp);
    if (nbp) {
      HIPCHK(hipMemcpy(used.data(), S.slot_used, sizeof(int) * nbp, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(bp.data(), S.bp, sizeof(int2) * nbp, hipMemcpyDeviceToHost));
    }
    std::vector<std::pair<std::pair<int, int>, int>> list;
    for (int p = 0; p < nbp; ++p)
      if (used[p]) list.push_back({{bp[p].x, bp[p].y}, p});
    std::sort(list.begin(), list.end());
    if (n_off) *n_off = (int64_t)list.size();
    if (off_ij && Hoff) {
      if ((int64_t)list.size() > cap) {
        rc = fail(ctx, ABD_E_CAPACITY, "off-diagonal buffer too small");
      } else {
        for (size_t i = 0; i < list.size(); ++i) {
          off_ij[2 * i] = list[i].first.first;
          off_ij[2 * i + 1] = list[i].first.second;
          if (S.mixed) {
            float h[144];
            HIPCHK(hipMemcpy(h, (float*)S.Hoff + 144L * list[i].second,
                             sizeof(float) * 144, hipMemcpyDeviceToHost));
            for (int k = 0; k < 144; ++k) Hoff[144 * i + k] = h[k];
          } else {
            HIPCHK(hipMemcpy(Hoff + 144 * i, (double*)S.Hoff + 144L * list[i].second,
                             sizeof(double) * 144, hipMemcpyDeviceToHost));
          }
        }
      }
    }
  }
  HIPCHK(hipMemcpy(S.q, save.data(), sizeof(double) * 12 * B, hipMemcpyHostToDevice));
  return rc;
}

int abd_direction(abd_ctx* ctx, double* dq, int32_t* pcg_iters) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if ((rc = assemble(ctx))) return rc;
  int it = 0;
  if ((rc = linear_solve(ctx, &it))) return rc;
  if (pcg_iters) *pcg_iters = it;
  if (dq)
    HIPCHK(hipMemcpy(dq, ctx->S.dq, sizeof(double) * 12 * ctx->S.B, hipMemcpyDeviceToHost));
  return ABD_OK;
}

}  /* extern "C" */

namespace {
/* every swept candidate's own TOI into toi (host, n entries) in the order
 * of abd_export_candidates (PT pairs sorted, then EE pairs sorted, then PG
 * vertices sorted), staged through d_toi (device, n entries) */
int toi_in_export_order(abd_ctx* ctx, double* d_toi, int64_t npt, int64_t nee,
                        int64_t npg, double* toi) {
  const Scene& S = ctx->S;
  const int64_t n = npt + nee + npg;
  HIPCHK(hipMemsetAsync(&S.cnt[1].n_long, 0, sizeof(int), ctx->st));
  launch_ccd_pairs(swept_scene(ctx), d_toi, n, ctx->st);
  std::vector<double> t(n);
  std::vector<int> pt(3 * npt), ee(3 * nee), pg(npg);
  hipError_t e = hipStreamSynchronize(ctx->st);
  if (e == hipSuccess) e = hipMemcpy(t.data(), d_toi, sizeof(double) * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && npt)
    e = hipMemcpy(pt.data(), S.cand_pt, sizeof(int) * 3 * npt, hipMemcpyDeviceToHost);
  if (e == hipSuccess && nee)
    e = hipMemcpy(ee.data(), S.cand_ee, sizeof(int) * 3 * nee, hipMemcpyDeviceToHost);
  if (e == hipSuccess && npg)
    e = hipMemcpy(pg.data(), S.cand_pg, sizeof(int) * npg, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(ctx, ABD_E_DEVICE, std::string("ccd: ") + hipGetErrorString(e));
  int64_t o = 0;
  auto emit = [&](int64_t first, int64_t m, auto key) {
    std::vector<int64_t> idx(m);
    for (int64_t i = 0; i < m; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return key(a) < key(b); });
    for (int64_t i = 0; i < m; ++i) toi[o++] = t[first + idx[i]];
  };
  emit(0, npt, [&](int64_t i) { return std::make_pair(pt[3 * i], pt[3 * i + 1]); });
  emit(npt, nee, [&](int64_t i) { return std::make_pair(ee[3 * i], ee[3 * i + 1]); });
  emit(npt + nee, npg, [&](int64_t i) { return std::make_pair(pg[i], 0); });
  return ABD_OK;
}
}  // namespace

extern "C" {

int abd_ccd(abd_ctx* ctx, const double* dq, double* alpha_max, double* toi,
            int64_t cap, int64_t* count) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (!dq || !alpha_max || cap < 0) return fail(ctx, ABD_E_INVALID_ARG, "ccd");
  if ((rc = upload_dq(ctx, dq))) return rc;
  if ((rc = swept_phase(ctx, true))) return rc;
  *alpha_max = std::min(1.0, bits_to_double(ctx->h_cnt[1].min_toi));
  const Scene& S = ctx->S;
  const Counters& c = ctx->h_cnt[1];
  const int64_t npt = std::min(c.n_pt, S.cap_pt), nee = std::min(c.n_ee, S.cap_ee),
                npg = std::min(c.n_pg, S.cap_pg), n = npt + nee + npg;
  if (count) *count = n;
  if (!toi) return ABD_OK;
  if (n > cap) return fail(ctx, ABD_E_CAPACITY, "TOI buffer too small");
  if (n == 0) return ABD_OK;
  double* d_toi = nullptr;
  if ((rc = dalloc(ctx, &d_toi, n))) return rc;
  rc = toi_in_export_order(ctx, d_toi, npt, nee, npg, toi);
  dfree(ctx, d_toi);
  return rc;
}

int abd_energy_delta(abd_ctx* ctx, const double* dq, double alpha,
                     double* dE) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (!dq || !dE) return fail(ctx, ABD_E_INVALID_ARG, "energy_delta");
  if ((rc = upload_dq(ctx, dq))) return rc;
  if ((rc = swept_phase(ctx, false))) return rc;
  return energy(ctx, 1, alpha, 0, 1, dE);
}

}  /* extern "C" */

struct abd_batch {
  std::vector<abd_ctx*> ctxs;
  std::vector<uint64_t> key; /* serials and pair rules of the contexts */
  std::vector<int> body_off;
  std::vector<unsigned> sh_seen;
  abd_ctx* M = nullptr;
  ProbCopy* pc = nullptr;  /* device descriptors */
  double* scales = nullptr; /* device [n] */
  std::vector<double> h_scales;
  int max_nb = 0;
  bool external_shared = false; /* shared data owned by a consensus object */
};

/* every context's state and scene scale into the batch scene */
static int batch_gather(abd_batch* bt) {
  abd_ctx* ctx = bt->M;
  const int n = (int)bt->ctxs.size();
  for (int i = 0; i < n; ++i) {
    HIPCHK(hipStreamSynchronize(bt->ctxs[i]->st));
    bt->h_scales[i] = bt->ctxs[i]->scale;
  }
  HIPCHK(hipMemcpyAsync(bt->scales, bt->h_scales.data(), sizeof(double) * n,
                        hipMemcpyHostToDevice, ctx->st));
  launch_gather(ctx->S, bt->pc, bt->scales, n, bt->max_nb, ctx->st);
  return ABD_OK;
}

static std::vector<uint64_t> batch_key(abd_ctx** ctxs, int n) {
  std::vector<uint64_t> k;
  for (int i = 0; i < n; ++i) {
    k.push_back(ctxs[i]->serial);
    k.push_back((uint64_t)ctxs[i]->pair_mode);
  }
  return k;
}


extern "C" {

int abd_batch_create(abd_ctx** ctxs, int32_t n, abd_batch** out) {
  if (!ctxs || n < 1 || !out) return ABD_E_INVALID_ARG;
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !ctxs[i]->finalized) return ABD_E_INVALID_ARG;
    if (std::memcmp(&ctxs[i]->P, &ctxs[0]->P, sizeof(abd_params)) != 0 ||
        ctxs[i]->pair_mode != ctxs[0]->pair_mode)
      return fail(ctxs[i], ABD_E_INVALID_ARG, "batch: parameters differ");
  }
  abd_batch* bt = new abd_batch();
  bt->ctxs.assign(ctxs, ctxs + n);
  int rc = abd_create(&bt->M, &ctxs[0]->P);
  if (rc) { delete bt; return rc; }
  abd_ctx* M = bt->M;
  M->np = n;
  M->pair_mode = ctxs[0]->pair_mode;
  int off = 0;
  for (int i = 0; i < n; ++i) {
    abd_ctx* c = ctxs[i];
    const int B = c->S.B;
    std::vector<double> q(12L * B), qd(12L * B);
    if (hipMemcpy(q.data(), c->S.q, sizeof(double) * 12 * B, hipMemcpyDeviceToHost) ||
        hipMemcpy(qd.data(), c->S.qdot, sizeof(double) * 12 * B, hipMemcpyDeviceToHost)) {
      abd_batch_destroy(bt);
      return ABD_E_DEVICE;
    }
    bt->body_off.push_back(off);
    for (int b = 0; b < B; ++b) {
      const HBody& hb = c->bodies[b];
      std::vector<int32_t> tl(3L * hb.nt);
      for (int k = 0; k < 3 * hb.nt; ++k) tl[k] = c->tri[3L * hb.t0 + k] - hb.v0;
      int32_t id;
      rc = abd_add_body(M, &c->xbar[3L * hb.v0], hb.nv, tl.data(), hb.nt,
                        hb.density, &q[12 * b], &qd[12 * b], hb.kind, &id);
      if (rc) { abd_batch_destroy(bt); return rc; }
      M->prob_of_body.push_back(i);
    }
    off += B;
    /* pad the problem to a multiple of 16 bodies with static one-triangle
     * bodies far below the scene: no 16-body group of the merged scene then
     * holds two problems, so the problem-local PCG can run the problems in
     * several launches when their groups do not all fit at once */
    static const double tv[9] = {0, 0, 0, 1e-3, 0, 0, 0, 0, 1e-3};
    static const int32_t tt[3] = {0, 1, 2};
    const double qg[12] = {0, -1e6, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int k = 0; k < (16 - B % 16) % 16; ++k) {
      int32_t id;
      rc = abd_add_body(M, tv, 3, tt, 1, 1000.0, qg, nullptr, ABD_STATIC, &id);
      if (rc) { abd_batch_destroy(bt); return rc; }
      M->prob_of_body.push_back(i);
      M->padding.resize(M->prob_of_body.size(), 0);
      M->padding.back() = 1;
      ++off;
    }
    bt->max_nb = std::max(bt->max_nb, B);
  }
  /* the first context's tuning, with direct launches: batch passes are
   * never replayed from captured graphs */
  abd_tuning tune = ctxs[0]->tune;
  tune.use_graphs = 0;
  if ((rc = abd_finalize(M)) || (rc = abd_set_tuning(M, &tune))) {
    abd_batch_destroy(bt);
    return rc;
  }
  std::vector<ProbCopy> pc(n);
  for (int i = 0; i < n; ++i)
    pc[i] = {ctxs[i]->S.q, ctxs[i]->S.qt, ctxs[i]->S.qtilde, ctxs[i]->S.qdot,
             ctxs[i]->S.B, bt->body_off[i]};
  if (hipMalloc(&bt->pc, sizeof(ProbCopy) * n) != hipSuccess ||
      hipMalloc(&bt->scales, sizeof(double) * n) != hipSuccess ||
      hipMemcpy(bt->pc, pc.data(), sizeof(ProbCopy) * n, hipMemcpyHostToDevice)) {
    abd_batch_destroy(bt);
    return ABD_E_OOM;
  }
  bt->sh_seen.assign(n, ~0u);
  bt->h_scales.assign(n, 1.0);
  bt->key = batch_key(ctxs, n);
  *out = bt;
  return ABD_OK;
}

void abd_batch_destroy(abd_batch* bt) {
  if (!bt) return;
  if (bt->pc) (void)hipFree(bt->pc);
  if (bt->scales) (void)hipFree(bt->scales);
  if (bt->M) abd_destroy(bt->M);
  delete bt;
}

int abd_batch_run(abd_batch* bt, abd_stats* out) {
  if (!bt) return ABD_E_INVALID_ARG;
  abd_ctx* M = bt->M;
  abd_ctx* ctx = M;
  const int n = (int)bt->ctxs.size();
  auto t0 = std::chrono::steady_clock::now();
  /* shared-body data: rebuilt only when a context changed it */
  bool sh_changed = false;
  for (int i = 0; i < n; ++i) sh_changed |= bt->sh_seen[i] != bt->ctxs[i]->sh_version;
  if (sh_changed && !bt->external_shared) {
    std::vector<int> ids, kb;
    std::vector<double> z, u, rho;
    for (int i = 0; i < n; ++i) {
      const abd_ctx* c = bt->ctxs[i];
      for (size_t k = 0; k < c->sh_ids.size(); ++k) ids.push_back(c->sh_ids[k] + bt->body_off[i]);
      kb.insert(kb.end(), c->sh_kappa.begin(), c->sh_kappa.end());
      z.insert(z.end(), c->sh_z.begin(), c->sh_z.end());
      u.insert(u.end(), c->sh_u.begin(), c->sh_u.end());
      rho.insert(rho.end(), c->sh_rho.begin(), c->sh_rho.end());
      bt->sh_seen[i] = c->sh_version;
    }
    int rc = abd_set_shared(M, ids.data(), (int)ids.size(), z.data(), u.data(),
                            rho.data(), kb.data());
    if (rc) return rc;
  }
  int rc0 = batch_gather(bt);
  if (rc0) return rc0;
  bool fell_back = false;
  int status = solve_with_fallback(M, &fell_back);
  launch_scatter(M->S, bt->pc, n, bt->max_nb, M->st);
  HIPCHK(hipStreamSynchronize(M->st));
  std::vector<ProbState> P(n);
  HIPCHK(hipMemcpy(P.data(), M->S.ps, sizeof(ProbState) * n, hipMemcpyDeviceToHost));
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  int first = status;
  for (int i = 0; i < n; ++i) {
    if (out) {
      abd_stats& st = out[i];
      std::memset(&st, 0, sizeof(st));
      st.newton_iters = P[i].newton;
      st.newton_fp32 = P[i].newton32;
      st.pcg_iters_total = P[i].pcg_total;
      st.ls_halvings = P[i].halvings;
      st.status = status ? status : P[i].status;
      st.final_eps_N = P[i].final_eps;
      st.min_alpha = P[i].min_alpha;
      st.scene_scale = bt->h_scales[i];
      st.min_dist = bits_to_double(M->h_last[0].min_dist);
      st.t_solve_ms = ms;
      st.fp64_fallback = fell_back ? 1 : 0;
    }
    if (first == ABD_OK && P[i].status != ABD_OK) {
      first = P[i].status;
      bt->ctxs[i]->err = "batch problem did not converge";
    }
  }
  return first;
}

int abd_batch_solve(abd_ctx** ctxs, int32_t n, abd_stats* out) {
  if (!ctxs || n < 1) return ABD_E_INVALID_ARG;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return ABD_E_INVALID_ARG;
  abd_ctx* owner = ctxs[0];
  const std::vector<uint64_t> key = batch_key(ctxs, n);
  if (!owner->batch_cache || owner->batch_cache->key != key) {
    abd_batch_destroy(owner->batch_cache);
    owner->batch_cache = nullptr;
    int rc = abd_batch_create(ctxs, n, &owner->batch_cache);
    if (rc) return rc;
  }
  return abd_batch_run(owner->batch_cache, out);
}

}  /* extern "C" */

struct abd_consensus {
  abd_batch* bt = nullptr;
  abd_admm_params ap;
  Cons C;
  std::vector<void*> allocs;
  int n_rep = 0, n_groups = 0;
  double h_red[2] = {0, 0};
};

static void cons_free(abd_consensus* c) {
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
}

template <typename T>
static int cons_upload(abd_consensus* c, const T** dst, const std::vector<T>& v) {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * std::max<size_t>(1, v.size())) != hipSuccess)
    return ABD_E_OOM;
  c->allocs.push_back(p);
  if (!v.empty() && hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice))
    return ABD_E_DEVICE;
  *dst = (const T*)p;
  return ABD_OK;
}
template <typename T>
static int cons_alloc(abd_consensus* c, T** dst, size_t n) {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * std::max<size_t>(1, n)) != hipSuccess) return ABD_E_OOM;
  c->allocs.push_back(p);
  if (hipMemset(p, 0, sizeof(T) * std::max<size_t>(1, n))) return ABD_E_DEVICE;
  *dst = (T*)p;
  return ABD_OK;
}

extern "C" {

int abd_consensus_create(abd_batch* bt, const int32_t* rep_prob,
                         const int32_t* rep_body, const int32_t* rep_group,
                         int32_t n_rep, int32_t n_groups,
                         const abd_admm_params* ap, abd_consensus** out) {
  if (!bt || !rep_prob || !rep_body || !rep_group || !ap || !out || n_rep < 1 ||
      n_groups < 1)
    return ABD_E_INVALID_ARG;
  *out = nullptr;
  abd_ctx* M = bt->M;
  const int np = (int)bt->ctxs.size();
  if (!(ap->tau > 1.0) || !(ap->mu >= 1.0) || !(ap->sigma_min > 0.0) ||
      !(ap->sigma_max >= ap->sigma_min) || ap->max_iters < 1 ||
      (!(ap->beta > 0.0) && !(ap->rho_fixed > 0.0)))
    return fail(M, ABD_E_INVALID_ARG, "admm parameters");
  std::vector<int> cnt(n_groups, 0), ids(n_rep), kb(n_rep);
  std::vector<double> rho0(n_rep), z(12L * n_rep, 0.0), u(12L * n_rep, 0.0);
  std::vector<std::pair<int, int>> seen;
  for (int k = 0; k < n_rep; ++k) {
    const int p = rep_prob[k], b = rep_body[k], g = rep_group[k];
    if (p < 0 || p >= np || g < 0 || g >= n_groups || b < 0 || b >= bt->ctxs[p]->S.B ||
        bt->ctxs[p]->bodies[b].kind != ABD_DYNAMIC)
      return fail(M, ABD_E_INVALID_ARG, "replica index");
    seen.push_back({p, g});
    cnt[g] += 1;
    ids[k] = bt->body_off[p] + b;
    const double m = bt->ctxs[p]->bodies[b].Mhat[0];
    rho0[k] = ap->beta > 0.0 ? ap->beta * m : ap->rho_fixed;
  }
  std::sort(seen.begin(), seen.end());
  if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
    return fail(M, ABD_E_INVALID_ARG, "two replicas of one body in a problem");
  for (int g = 0; g < n_groups; ++g)
    if (cnt[g] == 0) return fail(M, ABD_E_INVALID_ARG, "a shared body has no replica");
  for (int k = 0; k < n_rep; ++k) kb[k] = cnt[rep_group[k]];
  std::vector<int> ptr(n_groups + 1, 0), rep(n_rep), fill(n_groups, 0);
  for (int g = 0; g < n_groups; ++g) ptr[g + 1] = ptr[g] + cnt[g];
  for (int k = 0; k < n_rep; ++k) rep[ptr[rep_group[k]] + fill[rep_group[k]]++] = k;
  int rc = abd_set_shared(M, ids.data(), n_rep, z.data(), u.data(), rho0.data(), kb.data());
  if (rc) return rc;
  abd_consensus* c = new abd_consensus();
  c->bt = bt;
  c->ap = *ap;
  c->n_rep = n_rep;
  c->n_groups = n_groups;
  Cons& C = c->C;
  std::memset(&C, 0, sizeof(C));
  C.n_rep = n_rep;
  C.n_groups = n_groups;
  C.tau = ap->tau;
  C.mu = ap->mu;
  C.smin = ap->sigma_min;
  C.smax = ap->sigma_max;
  std::vector<int> rg(rep_group, rep_group + n_rep);
  if ((rc = cons_upload(c, &C.rep_body, ids)) || (rc = cons_upload(c, &C.rep_group, rg)) ||
      (rc = cons_upload(c, &C.grp_ptr, ptr)) || (rc = cons_upload(c, &C.grp_rep, rep)) ||
      (rc = cons_upload(c, &C.rho0, rho0)) || (rc = cons_alloc(c, &C.zc, 12L * n_groups)) ||
      (rc = cons_alloc(c, &C.r_body, n_groups)) || (rc = cons_alloc(c, &C.s_body, n_groups)) ||
      (rc = cons_alloc(c, &C.red, 2))) {
    cons_free(c);
    delete c;
    return fail(M, rc, "consensus allocation");
  }
  bt->external_shared = true;
  *out = c;
  return ABD_OK;
}

void abd_consensus_destroy(abd_consensus* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  if (c->bt) c->bt->external_shared = false;
  cons_free(c);
  delete c;
}

int abd_consensus_begin(abd_consensus* c) {
  if (!c) return ABD_E_INVALID_ARG;
  abd_ctx* ctx = c->bt->M;
  int rc = batch_gather(c->bt);
  if (rc) return rc;
  launch_cons_init(ctx->S, c->C, ctx->st);
  HIPCHK(hipStreamSynchronize(ctx->st));
  return ABD_OK;
}

static double cons_scale(abd_consensus* c) {
  if (c->ap.scale > 0.0) return c->ap.scale;
  double l = 0.0;
  for (double v : c->bt->h_scales) l = std::max(l, v);
  return l > 0.0 ? l : 1.0;
}

int abd_consensus_update(abd_consensus* c, abd_admm_report* rep) {
  if (!c) return ABD_E_INVALID_ARG;
  abd_batch* bt = c->bt;
  abd_ctx* ctx = bt->M;
  Scene& S = ctx->S;
  launch_cons_update(S, c->C, ctx->st);
  HIPCHK(hipMemcpyAsync(c->h_red, c->C.red, 2 * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->st));
  const int np = (int)bt->ctxs.size();
  std::vector<ProbState> P(np);
  double min_toi = 1.0;
  if (c->ap.merge_check) {
    /* ACCD of every problem from its q toward its merged state */
    launch_cons_merge_dq(S, c->C, ctx->st);
    int rc = swept_phase(ctx, true);
    if (rc) return rc;
  }
  HIPCHK(hipMemcpyAsync(P.data(), S.ps, sizeof(ProbState) * np, hipMemcpyDeviceToHost,
                        ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  double eps = 0.0;
  for (int p = 0; p < np; ++p) {
    eps = std::max(eps, P[p].final_eps);
    if (c->ap.merge_check)
      min_toi = std::min(min_toi, std::min(1.0, bits_to_double(P[p].min_toi)));
  }
  const double hl = ctx->P.dt * cons_scale(c);
  if (rep) {
    rep->eps_newton = eps;
    rep->r_inf = c->h_red[0] / hl;
    rep->s_inf = c->h_red[1] / hl;
    rep->min_toi = min_toi;
    rep->merge_ok = min_toi >= 1.0;
    const double th = ctx->P.newton_theta;
    rep->converged = eps < th && rep->r_inf < th && rep->s_inf < th &&
                     (!c->ap.merge_check || rep->merge_ok);
  }
  return ABD_OK;
}

int abd_consensus_adapt(abd_consensus* c) {
  if (!c) return ABD_E_INVALID_ARG;
  abd_ctx* ctx = c->bt->M;
  launch_cons_adapt(ctx->S, c->C, ctx->st);
  HIPCHK(hipStreamSynchronize(ctx->st));
  return ABD_OK;
}

int abd_consensus_merge(abd_consensus* c) {
  if (!c) return ABD_E_INVALID_ARG;
  abd_batch* bt = c->bt;
  abd_ctx* ctx = bt->M;
  launch_cons_merge(ctx->S, c->C, ctx->st);
  launch_scatter(ctx->S, bt->pc, (int)bt->ctxs.size(), bt->max_nb, ctx->st);
  HIPCHK(hipStreamSynchronize(ctx->st));
  return ABD_OK;
}

int abd_consensus_get(abd_consensus* c, double* z, double* u, double* rho) {
  if (!c) return ABD_E_INVALID_ARG;
  abd_ctx* ctx = c->bt->M;
  HIPCHK(hipStreamSynchronize(ctx->st));
  if (z) HIPCHK(hipMemcpy(z, c->C.zc, sizeof(double) * 12 * c->n_groups, hipMemcpyDeviceToHost));
  if (u) HIPCHK(hipMemcpy(u, ctx->S.u, sizeof(double) * 12 * c->n_rep, hipMemcpyDeviceToHost));
  if (rho) HIPCHK(hipMemcpy(rho, ctx->S.rho, sizeof(double) * c->n_rep, hipMemcpyDeviceToHost));
  return ABD_OK;
}

int abd_admm_step(abd_consensus* c, abd_admm_report* rep) {
  if (!c) return ABD_E_INVALID_ARG;
  abd_batch* bt = c->bt;
  const int np = (int)bt->ctxs.size();
  abd_admm_report r;
  std::memset(&r, 0, sizeof(r));
  int rc;
  for (abd_ctx* x : bt->ctxs)
    if ((rc = abd_begin_step(x))) return rc;
  if ((rc = abd_consensus_begin(c))) return rc;
  std::vector<abd_stats> st(np);
  int status = ABD_E_NOCONV;
  for (int k = 1; k <= c->ap.max_iters; ++k) {
    if (k > 1) {
      if ((rc = abd_consensus_update(c, &r))) return rc;
      if (r.converged) {
        status = ABD_OK;
        break;
      }
      if (c->ap.adapt_rho && (rc = abd_consensus_adapt(c))) return rc;
    }
    rc = abd_batch_run(bt, st.data());
    r.iters = k;
    for (int p = 0; p < np; ++p) r.newton_iters_total += st[p].newton_iters;
    if (rc) {
      if (rep) *rep = r;
      return rc;
    }
    if (k == c->ap.max_iters) {
      if ((rc = abd_consensus_update(c, &r))) return rc;
      if (r.converged) status = ABD_OK;
    }
  }
  /* merge when the consensus is safe to apply */
  if (status == ABD_OK || r.merge_ok) {
    if ((rc = abd_consensus_merge(c))) return rc;
  }
  for (abd_ctx* x : bt->ctxs)
    if ((rc = abd_end_step(x))) return rc;
  if (rep) *rep = r;
  if (status != ABD_OK) bt->M->err = "ADMM did not converge within max_iters";
  return status;
}

int abd_get_tuning(abd_ctx* ctx, abd_tuning* out) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (!out) return fail(ctx, ABD_E_INVALID_ARG, "tuning output");
  *out = ctx->tune;
  return ABD_OK;
}

int abd_set_tuning(abd_ctx* ctx, const abd_tuning* t) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  if (!t || t->pcg_variant < ABD_PCG_TWO_BARRIER || t->pcg_variant > ABD_PCG_LOCAL1 ||
      t->pcg_blocks < 0 || t->grid_blocks < 1 || t->assemble_blocks < 1 ||
      t->grid_blocks > (1 << 20) || t->assemble_blocks > (1 << 20))
    return fail(ctx, ABD_E_INVALID_ARG, "tuning values");
  if (t->pcg_coop != 0)
    return fail(ctx, ABD_E_INVALID_ARG,
                "pcg_coop is reserved and must be 0: the PCG launch is always a plain launch");
  if (t->pcg_launch_groups < 0 || t->label_rows < 0)
    return fail(ctx, ABD_E_INVALID_ARG, "pcg_launch_groups and label_rows must be >= 0");
  if (t->body_pairs < ABD_BODY_PAIRS_AUTO || t->body_pairs > ABD_BODY_PAIRS_SWEEP)
    return fail(ctx, ABD_E_INVALID_ARG, "body_pairs must be ABD_BODY_PAIRS_AUTO, _ALL or _SWEEP");
  if (t->body_pairs == ABD_BODY_PAIRS_ALL && ctx->bp_tests > ALL_PAIRS_BUILD_MAX)
    return fail(ctx, ABD_E_INVALID_ARG,
                "every-pair body tests are not set up for more than 2^27 pairs");
  drop_graphs(ctx); /* launch shapes are part of the captured graphs */
  ctx->tune = *t;
  ctx->tune.use_graphs = t->use_graphs ? 1 : 0;
  ctx->tune.overlap_body = t->overlap_body ? 1 : 0;
  ctx->S.grid_blocks = t->grid_blocks;
  ctx->S.assemble_blocks = t->assemble_blocks;
  ctx->S.sap_on = sap_on(ctx);
  return plan_launches(ctx);
}

int abd_autotune(abd_ctx* ctx, abd_tuning* out) {
  int rc = check_ctx(ctx, true);
  if (rc) return rc;
  Scene& S = ctx->S;
  const size_t nb = sizeof(double) * 12 * S.B;
  double *q0 = nullptr, *qd0 = nullptr;
  if (dalloc(ctx, &q0, 12L * S.B) || dalloc(ctx, &qd0, 12L * S.B)) {
    dfree(ctx, q0);
    return fail(ctx, ABD_E_OOM, "autotune state copy: " + ctx->err);
  }
  HIPCHK(hipMemcpyAsync(q0, S.q, nb, hipMemcpyDeviceToDevice, ctx->st));
  HIPCHK(hipMemcpyAsync(qd0, S.qdot, nb, hipMemcpyDeviceToDevice, ctx->st));
  const abd_tuning orig = ctx->tune;
  const int saved_timing = ctx->timing;
  ctx->timing = ABD_TIMING_OFF;
  /* one timed solve of the next step from the saved state; the first run
   * of a setting captures its graphs, so each setting runs twice */
  auto trial = [&](const abd_tuning& t) -> double {
    if (abd_set_tuning(ctx, &t) != ABD_OK) return INFINITY;
    double best = INFINITY;
    for (int rep = 0; rep < 2; ++rep) {
      if (hipMemcpyAsync(S.q, q0, nb, hipMemcpyDeviceToDevice, ctx->st) ||
          hipMemcpyAsync(S.qdot, qd0, nb, hipMemcpyDeviceToDevice, ctx->st))
        return INFINITY;
      if (abd_begin_step(ctx) != ABD_OK) return INFINITY;
      auto t0 = std::chrono::steady_clock::now();
      int st = device_solve(ctx);
      ProbState P[1];
      if (st == ABD_OK &&
          hipMemcpy(P, S.ps, sizeof(ProbState), hipMemcpyDeviceToHost) != hipSuccess)
        st = ABD_E_DEVICE;
      const double ms = std::chrono::duration<double, std::milli>(
                            std::chrono::steady_clock::now() - t0).count();
      if (st != ABD_OK || P[0].status != ABD_OK) return INFINITY;
      if (rep == 1) best = ms;
    }
    return best;
  };
  abd_tuning best = orig;
  double best_ms = trial(best);
  auto consider = [&](abd_tuning t) {
    const double ms = trial(t);
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  };
  const int ng = std::max(1, (S.B + 15) / 16);
  std::vector<std::pair<int, int>> tried = {{orig.pcg_variant, pcg_blocks(ctx, S)}};
  /* the pipelined form only where its attainable accuracy is not the
   * binding limit */
  std::vector<int> vars = {ABD_PCG_LOCAL, ABD_PCG_LOCAL1, ABD_PCG_TWO_BARRIER};
  if (ctx->P.pcg_eta >= 1e-6) vars.push_back(ABD_PCG_PIPELINED);
  for (int v : vars)
    for (int div : {1, 2, 4, 8}) {
      if ((v == ABD_PCG_LOCAL || v == ABD_PCG_LOCAL1) && div > 1)
        continue; /* one block per group */
      abd_tuning t = best;
      t.pcg_variant = v;
      t.pcg_blocks = std::max(1, (ng + div - 1) / div);
      const std::pair<int, int> key(v, std::min(t.pcg_blocks, ctx->pcg_grid));
      if (std::find(tried.begin(), tried.end(), key) != tried.end()) continue;
      tried.push_back(key);
      consider(t);
    }
  const abd_tuning after_pcg = best;
  for (int g : {512, 1024, 2048, 4096}) {
    abd_tuning t = after_pcg;
    t.grid_blocks = g;
    if (g != orig.grid_blocks) consider(t);
  }
  const abd_tuning after_grid = best;
  for (int g : {512, 1024, 4096}) {
    abd_tuning t = after_grid;
    t.assemble_blocks = g;
    if (g != orig.assemble_blocks) consider(t);
  }
  {
    abd_tuning t = best;
    t.overlap_body = best.overlap_body ? 0 : 1;
    consider(t);
  }
  {
    abd_tuning t = best;
    t.use_graphs = best.use_graphs ? 0 : 1;
    consider(t);
  }
  /* restore the state and keep the winner */
  (void)abd_set_tuning(ctx, &best);
  ctx->timing = saved_timing;
  HIPCHK(hipMemcpyAsync(S.q, q0, nb, hipMemcpyDeviceToDevice, ctx->st));
  HIPCHK(hipMemcpyAsync(S.qdot, qd0, nb, hipMemcpyDeviceToDevice, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  dfree(ctx, qd0);
  dfree(ctx, q0);
  if (!std::isfinite(best_ms)) return fail(ctx, ABD_E_NOCONV, "autotune: no setting solved the step");
  if (out) *out = best;
  return ABD_OK;
}

int abd_set_timing(abd_ctx* ctx, int32_t on) {
  if (!ctx) return ABD_E_INVALID_ARG;
  if (on != ABD_TIMING_OFF && on != ABD_TIMING_ALL && on != ABD_TIMING_PCG &&
      on != ABD_TIMING_ASM)
    return fail(ctx, ABD_E_INVALID_ARG, "timing mode");
  ctx->timing = on;
  return ABD_OK;
}

int abd_get_timing(abd_ctx* ctx, int32_t stage, double* ms, int64_t* launches,
                   double* bytes) {
  if (!ctx || stage < 0 || stage >= ABD_STAGES) return ABD_E_INVALID_ARG;
  (void)hipStreamSynchronize(ctx->st);
  resolve_timing(ctx);
  if (ms) *ms = ctx->t_ms[stage];
  if (launches) *launches = ctx->t_n[stage];
  if (bytes) *bytes = ctx->t_bytes[stage];
  return ABD_OK;
}

int abd_get_timing_flops(abd_ctx* ctx, int32_t stage, double* flops) {
  if (!ctx || stage < 0 || stage >= ABD_STAGES || !flops) return ABD_E_INVALID_ARG;
  (void)hipStreamSynchronize(ctx->st);
  resolve_timing(ctx);
  *flops = ctx->t_flops[stage];
  return ABD_OK;
}

int abd_reset_timing(abd_ctx* ctx) {
  if (!ctx) return ABD_E_INVALID_ARG;
  (void)hipStreamSynchronize(ctx->st);
  resolve_timing(ctx);
  for (int i = 0; i < ABD_STAGES; ++i)
    ctx->t_ms[i] = ctx->t_bytes[i] = ctx->t_flops[i] = 0.0, ctx->t_n[i] = 0;
  return ABD_OK;
}

}  // extern "C"
