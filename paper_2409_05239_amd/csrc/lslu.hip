// C ABI (include/lslu.h) and the host-side driver of one solve.
//
// A solve enqueues, on the context's stream and without host synchronisation:
//   init      r_0 = b - A x_0, pivot candidates of r_0
//   for k = 1..K (Algorithm 5), one launch per half-iteration:
//     t(k), H(k,k-1) (or beta), d_k; W(1:k-1,k); q = A^T d_k - L w and its
//       pivot candidates
//     g(k), W(k,k), l_k; H(1:k,k); u = A l_k - D h and its candidates
//   t(K+1), H(K+1,K), d_{K+1}
//   projected problems for all k                (one workgroup per k)
//   stopping rule, iterates X = x_0 + L Y, selected iterate -> x_out
// then copies the small results to pinned host memory once and waits.
// Breakdowns are detected on the device; later kernels then do nothing.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "host_ops.hpp"
#include "internal.hpp"
#include "lslu.h"

using namespace lslu;

namespace {

// A named range on the profiler's host timeline (rocprofv3 --marker-trace)
// from construction to the end of the scope; a no-op without a profiler.
// The device work a range enqueues shows in the kernel trace beside it.
struct Range {
  explicit Range(const char* name) { roctxRangePush(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

struct Layout {
  void *L = nullptr, *D = nullptr, *q = nullptr, *u = nullptr, *r0 = nullptr,
       *X = nullptr;
  double* ybuf = nullptr;  // slots of the recurrence, slots_per_launch(K) per launch
  int* flags = nullptr;    // one failure flag per launch of the recurrence
  void *TL = nullptr, *TD = nullptr;  // pivot-row triangles, basis precision
  double *grid = nullptr, *proj = nullptr;
  double *gram = nullptr, *gram_part = nullptr;  // optimal rule only
  int *rep_t = nullptr, *rep_g = nullptr, *rep_lam = nullptr;
  int* samp = nullptr;  // sampled-pivot candidate rows, (2K+1) x kMaxSampleLen
  unsigned char *mask_t = nullptr, *mask_g = nullptr;
  ArgPart* parts = nullptr;
  // result block (copied to the host in one transfer)
  unsigned char* res = nullptr;
  size_t res_bytes = 0;
  double *H = nullptr, *W = nullptr, *Y = nullptr, *lam = nullptr,
         *ghat = nullptr, *sep = nullptr, *smax = nullptr, *smin = nullptr,
         *dldl = nullptr, *psep = nullptr;  // psep: sep_t (K+1), then sep_g (K)
  unsigned long long* psep_mx = nullptr;
  int *piv_t = nullptr, *piv_g = nullptr, *own_t = nullptr, *own_g = nullptr,
      *lam_idx = nullptr, *sel = nullptr;
  DevState* st = nullptr;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Basis storage: element (i, j) at p[i * rs + j * cs].
struct Strides {
  int64_t rsL, csL, rsD, csD;
};

Strides basis_strides(bool rowmajor, int64_t m, int64_t n, int K) {
  if (rowmajor)
    return {(int64_t)align_up((size_t)K, 16), 1, (int64_t)align_up((size_t)K + 1, 16), 1};
  return {1, (int64_t)align_up((size_t)n, 64), 1, (int64_t)align_up((size_t)m, 64)};
}

// Two passes: with base == nullptr only the size is computed.  The
// projected problems' scratch has room for grid_slots grid values each.
size_t carve(unsigned char* base, int64_t m, int64_t n, int K, size_t esz,
             const Strides& bs, Layout* lay, int grid_slots = kMaxGrid) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> unsigned char* {
    off = align_up(off, 256);
    unsigned char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  Layout l;
  // the last element of a basis is at (len-1)*rs + (cols-1)*cs
  l.L = take(esz * (size_t)((n - 1) * bs.rsL + (K - 1) * bs.csL + 1));
  l.D = take(esz * (size_t)((m - 1) * bs.rsD + K * bs.csD + 1));
  l.q = take(esz * n);
  l.u = take(esz * m);
  l.r0 = take(esz * m);
  l.ybuf = reinterpret_cast<double*>(take(sizeof(double) * slots_per_launch(K) * (2 * K + 2)));
  l.flags = reinterpret_cast<int*>(take(sizeof(int) * (2 * K + 2)));
  l.X = take(esz * n * K);
  l.TL = take(esz * K * (K + 1) / 2);        // packed rows, strict lower
  l.TD = take(esz * (K + 1) * (K + 2) / 2);
  l.grid = reinterpret_cast<double*>(take(sizeof(double) * kMaxGrid));
  l.proj = reinterpret_cast<double*>(take(sizeof(double) * projected_scratch_doubles(K, grid_slots)));
  l.gram = reinterpret_cast<double*>(take(sizeof(double) * (K + 1) * (K + 1)));
  l.gram_part = reinterpret_cast<double*>(take(sizeof(double) * gram_scratch_doubles(K)));
  l.rep_t = reinterpret_cast<int*>(take(sizeof(int) * (K + 1)));
  l.rep_g = reinterpret_cast<int*>(take(sizeof(int) * K));
  l.rep_lam = reinterpret_cast<int*>(take(sizeof(int) * K));
  l.samp = reinterpret_cast<int*>(take(sizeof(int) * (2 * K + 1) * kMaxSampleLen));
  l.mask_t = take(m);
  l.mask_g = take(n);
  l.parts = reinterpret_cast<ArgPart*>(take(sizeof(ArgPart) * 2 * kMaxParts));
  l.psep_mx = reinterpret_cast<unsigned long long*>(take(sizeof(uint64_t) * (2 * K + 1)));
  // result block: doubles, then ints, then the state
  off = align_up(off, 256);
  const size_t res_start = off;
  l.H = reinterpret_cast<double*>(take(sizeof(double) * (K + 1) * K));
  l.W = reinterpret_cast<double*>(take(sizeof(double) * K * K));
  l.Y = reinterpret_cast<double*>(take(sizeof(double) * K * K));
  l.lam = reinterpret_cast<double*>(take(sizeof(double) * K));
  l.ghat = reinterpret_cast<double*>(take(sizeof(double) * K));
  l.sep = reinterpret_cast<double*>(take(sizeof(double) * K));
  l.smax = reinterpret_cast<double*>(take(sizeof(double) * K));
  l.smin = reinterpret_cast<double*>(take(sizeof(double) * K));
  l.dldl = reinterpret_cast<double*>(take(sizeof(double) * K));
  l.psep = reinterpret_cast<double*>(take(sizeof(double) * (2 * K + 1)));
  l.piv_t = reinterpret_cast<int*>(take(sizeof(int) * (K + 1)));
  l.piv_g = reinterpret_cast<int*>(take(sizeof(int) * K));
  l.own_t = reinterpret_cast<int*>(take(sizeof(int) * (K + 1)));
  l.own_g = reinterpret_cast<int*>(take(sizeof(int) * K));
  l.lam_idx = reinterpret_cast<int*>(take(sizeof(int) * K));
  l.sel = reinterpret_cast<int*>(take(sizeof(int) * 2));
  l.st = reinterpret_cast<DevState*>(take(sizeof(DevState)));
  l.res_bytes = off - res_start;
  l.res = base ? base + res_start : nullptr;
  if (lay) *lay = l;
  return align_up(off, 256);
}

}  // namespace

struct lslu_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // two more streams (default priority) and three events, made with the
  // context: the independent launches of the projected problems run side by
  // side, forked from and joined back into the context's stream
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
  std::string err;
  size_t lds_max = 0;
  // workspace
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  unsigned char* host = nullptr;  // pinned staging for the result block
  size_t host_bytes = 0;
  Layout lay;
  int64_t m = 0, n = 0;
  Strides bs{};
  bool rowmajor = false;
  int K = 0;
  size_t esz = 0;
  int grid_slots = kMaxGrid;  // grid values the projected scratch of lay holds
  // basis vectors formed by the last solve
  int last_nl = 0, last_nd = 0;
  // the last completed solve (what lslu_vjp differentiates)
  const lslu_op* last_op = nullptr;
  int last_kdone = 0;
  bool last_ok = false;
  // reverse-pass scratch (grown on demand) and a pinned word block
  unsigned char* adj = nullptr;
  size_t adj_bytes = 0;
  double* adj_host = nullptr;
  // merged-launch arguments of lslu_solve_batch, grown on demand
  unsigned char* bat = nullptr;
  size_t bat_bytes = 0;
  // device staging of lslu_solve_host (b, x_0, x_out), grown on demand and
  // reused, so that its solves keep replaying the same captured graph
  unsigned char* hio = nullptr;
  size_t hio_bytes = 0;
  // captured solve (replayed while the key matches)
  // captured solves, replayed while the key (pointers, sizes, options)
  // matches; the least recently captured is dropped beyond kGraphCache
  struct Captured {
    std::vector<double> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Captured> graphs;
  // last uploaded lambda grid and replay arrays (skipped when unchanged)
  std::vector<double> up_grid;
  std::vector<int> up_rep;
  std::vector<int> up_samp;
  // an LSLU_FLAG_ASYNC solve whose results lslu_wait has not collected yet
  bool pending = false;
  int pend_K = 0;
  lslu_result* pend_res = nullptr;
};

struct lslu_op {
  lslu_ctx* ctx = nullptr;
  DeviceOp d;
  // unique for the life of the process: captured solves are keyed by it, so
  // an operator allocated where a destroyed one lived never matches a graph
  // that baked in the destroyed operator's device arrays
  uint64_t serial = 0;
};

namespace {
std::atomic<uint64_t> g_op_serial{0};
}  // namespace

namespace {

lslu_status fail(lslu_ctx* c, lslu_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define LSLU_HIP(ctx, expr)                                                  \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail((ctx), e_ == hipErrorOutOfMemory ? LSLU_ENOMEM : LSLU_EDEVICE, \
                  std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

// Host <-> device copy ordered on the context's stream and waited for.  (A
// copy on the null stream would synchronise with every blocking stream,
// which breaks a graph being captured on another context's stream by
// another thread.)
lslu_status copy_sync(lslu_ctx* c, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  if (bytes == 0) return LSLU_OK;
  LSLU_HIP(c, hipMemcpyAsync(dst, src, bytes, kind, c->stream));
  LSLU_HIP(c, hipStreamSynchronize(c->stream));
  return LSLU_OK;
}

bool finite_all(const double* p, int64_t count) {
  for (int64_t i = 0; i < count; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

size_t prec_size(int prec) { return prec == kFP64 ? sizeof(double) : sizeof(float); }

lslu_status upload(lslu_ctx* c, void** dst, const void* src, size_t bytes) {
  LSLU_HIP(c, hipMalloc(dst, bytes > 0 ? bytes : 1));
  if (bytes) {
    const lslu_status st = copy_sync(c, *dst, src, bytes, hipMemcpyHostToDevice);
    if (st != LSLU_OK) return st;
  }
  return LSLU_OK;
}

void free_op(DeviceOp& d) {
  void* ps[] = {d.A, d.AT, d.rp, d.ci, d.val, d.rpT, d.ciT, d.valT,
                d.psf, d.psf_flip, d.psf32, d.psf32_flip, d.mb, d.mb_flip};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  d = DeviceOp{};
}

constexpr size_t kGraphCache = 64;

void destroy_captured(lslu_ctx::Captured& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

void drop_graph(lslu_ctx* c) {
  for (auto& g : c->graphs) destroy_captured(g);
  c->graphs.clear();
}

// Releases the captured solves of one operator (key entry 0 is its serial).
void drop_op_graphs(lslu_ctx* c, uint64_t serial) {
  auto& gs = c->graphs;
  for (auto it = gs.begin(); it != gs.end();) {
    if (!it->key.empty() && it->key[0] == static_cast<double>(serial)) {
      destroy_captured(*it);
      it = gs.erase(it);
    } else {
      ++it;
    }
  }
}

lslu_status ensure_ws(lslu_ctx* c, int64_t m, int64_t n, int K, size_t esz,
                      bool rowmajor) {
  const Strides bs = basis_strides(rowmajor, m, n, K);
  const size_t need = carve(nullptr, m, n, K, esz, bs, nullptr);
  if (need > c->ws_bytes) {
    drop_graph(c);
    if (c->ws) (void)hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
    void* p = nullptr;
    LSLU_HIP(c, hipMalloc(&p, need));
    c->ws = static_cast<unsigned char*>(p);
    c->ws_bytes = need;
  }
  carve(c->ws, m, n, K, esz, bs, &c->lay);
  if (c->lay.res_bytes > c->host_bytes) {
    if (c->host) (void)hipHostFree(c->host);
    c->host = nullptr;
    c->host_bytes = 0;
    void* h = nullptr;
    LSLU_HIP(c, hipHostMalloc(&h, c->lay.res_bytes, hipHostMallocDefault));
    c->host = static_cast<unsigned char*>(h);
    c->host_bytes = c->lay.res_bytes;
  }
  c->m = m;
  c->n = n;
  c->K = K;
  c->bs = bs;
  c->rowmajor = rowmajor;
  c->esz = esz;
  return LSLU_OK;
}

// Events of a timed (LSLU_FLAG_TIMING) solve, recorded on the solve's stream.
struct PhaseEvents {
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  int launches = 0;
  bool on = false;
  void mark(int i, hipStream_t s) {
    if (on) (void)hipEventRecord(ev[i], s);
  }
};

// One half-iteration launch as planned for a merged (batched) launch.
template <typename T>
struct PlannedHalf {
  HalfArgs<T> a;
  int tr;
  int ncons;
};

// part 0: the whole solve on stream s (default: the context's stream);
// part 1: the set-up kernels, with the half-iteration launches planned into
// rec instead of launched; part 2: everything after the recurrence.
template <typename T>
void enqueue_solve(lslu_ctx* c, const DeviceOp& op, const T* b, const T* x0,
                   const lslu_opts* o, T* x_out, T* X, bool replay_t,
                   bool replay_g, bool replay_lam, PhaseEvents* pe,
                   hipStream_t s_in = nullptr, int part = 0,
                   std::vector<PlannedHalf<T>>* rec = nullptr) {
  const hipStream_t s = s_in ? s_in : c->stream;
  const Layout& l = c->lay;
  const int K = c->K;
  const int64_t m = c->m, n = c->n;
  const Strides bs = c->bs;
  T* Lb = static_cast<T*>(l.L);
  T* Db = static_cast<T*>(l.D);
  T* q = static_cast<T*>(l.q);
  T* u = static_cast<T*>(l.u);
  DevState* st = l.st;
  const size_t lds = c->lds_max;

  if (part != 2) {
  Range r_rec("lslu: set-up and recurrence (enqueue)");
  launch_state_reset(st, l.psep, 2 * K + 1, s);
  launch_fill<unsigned char>(l.mask_t, 0, m, s);
  launch_fill<unsigned char>(l.mask_g, 0, n, s);
  launch_fill<int>(l.piv_t, -1, K + 1, s);
  launch_fill<int>(l.piv_g, -1, K, s);
  launch_fill<int>(l.own_t, -1, K + 1, s);
  launch_fill<int>(l.own_g, -1, K, s);
  launch_fill<int>(l.flags, 0, 2 * K + 2, s);
  launch_fill<uint64_t>(reinterpret_cast<uint64_t*>(l.ybuf), kSlotEmpty,
                        slots_per_launch(K) * (2 * K + 2), s);
  launch_fill<double>(l.H, 0.0, (int64_t)(K + 1) * K, s);
  launch_fill<double>(l.W, 0.0, (int64_t)K * K, s);
  launch_fill<double>(l.Y, 0.0, (int64_t)K * K, s);
  T* TL = static_cast<T*>(l.TL);
  T* TD = static_cast<T*>(l.TD);
  launch_fill<T>(TL, T(0), (int64_t)K * (K + 1) / 2, s);
  launch_fill<T>(TD, T(0), (int64_t)(K + 1) * (K + 2) / 2, s);
  auto packed = [](int j) { return (int64_t)j * (j - 1) / 2; };
  auto Hcol = [&](int k) { return l.H + (int64_t)(k - 1) * (K + 1); };  // H(:,k)
  auto Wcol = [&](int k) { return l.W + (int64_t)(k - 1) * K; };        // W(:,k)

  // r_0 = b - A x_0 (or b) and its pivot candidates.
  const T* r0 = b;
  if (x0) {
    op_apply(op, 0, x0, l.r0, nullptr, s);
    launch_sub<T>(b, static_cast<const T*>(l.r0), static_cast<T*>(l.r0), m, s);
    r0 = static_cast<const T*>(l.r0);
  }
  ArgPart* parts[2] = {l.parts, l.parts + kMaxParts};
  int cur = 0;  // parts[cur] holds the candidates of the last pass
  int nparts = launch_argmax_parts<T>(r0, m, parts[cur], st, s);
  int launch = 0;
  pe->mark(0, s);

  // The d-side search that a launch resolves: r_0 (k = 0) or the d side of
  // iteration k, giving t(k+1).
  auto d_job = [&](int k) {
    PivotJob j{};
    j.side = k == 0 ? 2 : 1;
    j.k = k;
    j.eligible = (k == 0 || k < m) ? 1 : 0;
    j.piv_pos = k;
    j.piv_val = k == 0 ? &st->beta : Hcol(k) + k;
    j.piv_list = l.piv_t;
    j.own_list = l.own_t;
    j.mask = l.mask_t;
    j.replay = replay_t ? l.rep_t : nullptr;
    j.st = st;
    return j;
  };
  auto set_prev_d = [&](HalfArgs<T>& a, int k, const T* vec) {
    // resolves t(k+1): d_{k+1} into column k of D, row k of T_D
    a.up = vec;
    a.lenp = m;
    a.parts_in = parts[cur];
    a.nparts_in = nparts;
    a.job = d_job(k);
    a.dstp = Db + (int64_t)k * bs.csD;
    a.dstp_stride = bs.rsD;
    a.basisp = Db;
    a.rsp = bs.rsD;
    a.csp = bs.csD;
    a.nbp = k;
    a.Trowp = k > 0 ? TD + packed(k) : nullptr;
  };
  const bool sampled = o->sample_rows != nullptr;
  auto run = [&](HalfArgs<T>& a, int tr) {
    // launch i resolves pivot search i (r_0, then q and u of each iteration)
    a.job.sample = sampled ? l.samp + (int64_t)launch * kMaxSampleLen : nullptr;
    a.job.sample_s = sampled ? o->sample_s : 0;
    a.job.sample_len = sampled ? o->sample_len : 0;
    a.entries = l.ybuf + slots_per_launch(K) * launch;
    a.cslot = a.entries + (K + 1);
    a.pslot = reinterpret_cast<uint64_t*>(a.entries + 2 * (K + 1));
    a.fail = l.flags + launch++;
    a.parts_out = parts[cur ^ 1];
    if (rec) {
      nparts = plan_half<T>(a, op, tr, lds);
      rec->push_back(PlannedHalf<T>{a, tr, nparts});
    } else {
      nparts = launch_half<T>(a, op, tr, lds, s);
    }
    cur ^= 1;
  };

  for (int k = 1; k <= K; ++k) {
    // t(k), d_k; then q = A^T d_k - L w with w = W(1:k-1,k).
    HalfArgs<T> al{};
    set_prev_d(al, k - 1, k == 1 ? r0 : u);
    al.rows = n;
    al.basis = Lb;
    al.rs = bs.rsL;
    al.cs = bs.csL;
    al.nb = k - 1;
    al.piv = l.piv_g;
    al.Tp = TL;
    al.coef = Wcol(k);
    al.mask = l.mask_g;
    al.out = q;
    run(al, 1);
    // g(k), W(k,k), l_k; then u = A l_k - D h with h = H(1:k,k).
    HalfArgs<T> ad{};
    ad.up = q;
    ad.lenp = n;
    ad.parts_in = parts[cur];
    ad.nparts_in = nparts;
    ad.job.side = 0;
    ad.job.k = k;
    ad.job.eligible = (k <= n) ? 1 : 0;
    ad.job.piv_pos = k - 1;
    ad.job.piv_val = Wcol(k) + (k - 1);
    ad.job.piv_list = l.piv_g;
    ad.job.own_list = l.own_g;
    ad.job.mask = l.mask_g;
    ad.job.replay = replay_g ? l.rep_g : nullptr;
    ad.job.st = st;
    ad.dstp = Lb + (int64_t)(k - 1) * bs.csL;
    ad.dstp_stride = bs.rsL;
    ad.basisp = Lb;
    ad.rsp = bs.rsL;
    ad.csp = bs.csL;
    ad.nbp = k - 1;
    ad.Trowp = TL + packed(k - 1);
    ad.rows = m;
    ad.basis = Db;
    ad.rs = bs.rsD;
    ad.cs = bs.csD;
    ad.nb = k;
    ad.piv = l.piv_t;
    ad.Tp = TD;
    ad.coef = Hcol(k);
    ad.mask = l.mask_t;
    ad.out = u;
    run(ad, 0);
  }
  // t(K+1), H(K+1,K), d_{K+1}.
  HalfArgs<T> af{};
  set_prev_d(af, K, u);
  af.rows = 0;
  af.nb = 0;
  af.piv = l.piv_g;
  af.Tp = TL;
  af.coef = l.ybuf;
  af.mask = l.mask_g;
  af.basis = Lb;
  af.out = q;
  run(af, 1);
  pe->launches = launch;
  pe->mark(1, s);
  }
  if (part == 1) return;

  if (o->flags & LSLU_FLAG_PIVOT_SEP)
    launch_pivot_sep<T>(Lb, bs.rsL, bs.csL, n, Db, bs.rsD, bs.csD, m, l.piv_t, l.piv_g,
                        o->sample_rows ? l.samp : nullptr, o->sample_s, K, st, l.psep_mx,
                        l.psep, l.psep + (K + 1), s);

  ProjParams pp{};
  pp.K = K;
  pp.m = static_cast<int>(std::min<int64_t>(m, INT32_MAX));
  pp.n = static_cast<int>(std::min<int64_t>(n, INT32_MAX));
  pp.reg = o->reg;
  pp.lambda = o->lambda;
  pp.n_grid = o->n_grid;
  pp.grid_relative = o->grid_relative;
  pp.omega = o->omega;
  pp.grid = l.grid;
  pp.replay_lambda = replay_lam ? l.rep_lam : nullptr;
  pp.grid_slots = c->grid_slots;
  const bool grad = (o->flags & LSLU_FLAG_GRAD_LAMBDA) != 0;
  if (o->reg == LSLU_REG_OPTIMAL || grad) {
    launch_gram<T>(Lb, bs.rsL, bs.csL, n, K, static_cast<const T*>(o->x_true_dev), x0, st,
                   l.gram_part, l.gram, s);
    pp.gram = l.gram;
  }
  pp.dldl = grad ? l.dldl : nullptr;
  {
    Range r_proj("lslu: projected problems (enqueue)");
    // fork onto the side streams, one launch group each, then join
    const hipStream_t ss[3] = {s, c->side[0], c->side[1]};
    (void)hipEventRecord(c->fork, s);
    for (int i = 0; i < 2; ++i) (void)hipStreamWaitEvent(c->side[i], c->fork, 0);
    launch_projected(l.H, st, 0.0, pp, l.Y, l.lam, l.lam_idx, l.ghat, l.sep,
                     l.smax, l.smin, l.proj, c->lds_max, ss, 3);
    for (int i = 0; i < 2; ++i) {
      (void)hipEventRecord(c->join[i], c->side[i]);
      (void)hipStreamWaitEvent(s, c->join[i], 0);
    }
  }
  pe->mark(2, s);
  Range r_asm("lslu: stopping rule and assembly (enqueue)");
  const double tol = o->stop_tol > 0.0 ? o->stop_tol : 1e-6;
  launch_stopping(l.ghat, st, tol, o->early_stop ? 1 : 0, l.sel, s);
  if (o->flags & LSLU_FLAG_FINAL_ONLY) {
    launch_assemble_final<T>(Lb, bs.rsL, bs.csL, n, l.Y, K, x0, x_out, l.sel, s);
  } else {
    launch_assemble<T>(Lb, bs.rsL, bs.csL, n, l.Y, K, x0, X, st, s);
    launch_select_x<T>(X, n, x0, x_out, st, l.sel, s);
  }
  pe->mark(3, s);
}

lslu_status validate_opts(lslu_ctx* c, const lslu_op* op, const lslu_opts* o) {
  const int64_t m = op->d.m, n = op->d.n;
  if (o->maxiter < 1 || o->maxiter > kMaxIter)
    return fail(c, LSLU_EINVAL, "maxiter must be in [1, 256]");
  if ((int64_t)o->maxiter > std::min(m, n) + 1)
    return fail(c, LSLU_EINVAL, "maxiter must not exceed min(m, n) + 1");
  if (o->reg < LSLU_REG_NONE || o->reg > LSLU_REG_OPTIMAL)
    return fail(c, LSLU_EINVAL, "unknown regularisation rule");
  if (o->reg == LSLU_REG_OPTIMAL && !o->x_true_dev)
    return fail(c, LSLU_EINVAL, "LSLU_REG_OPTIMAL needs x_true_dev");
  if ((o->flags & LSLU_FLAG_GRAD_LAMBDA) && !o->x_true_dev)
    return fail(c, LSLU_EINVAL, "LSLU_FLAG_GRAD_LAMBDA needs x_true_dev");
  if ((o->flags & LSLU_FLAG_FINAL_ONLY) && o->X_dev)
    return fail(c, LSLU_EINVAL, "LSLU_FLAG_FINAL_ONLY forms no iterates for X_dev");
  if (o->reg == LSLU_REG_FIXED && !(std::isfinite(o->lambda) && o->lambda >= 0.0))
    return fail(c, LSLU_EINVAL, "lambda must be finite and >= 0");
  if (o->reg == LSLU_REG_WGCV || o->reg == LSLU_REG_GCV || o->reg == LSLU_REG_OPTIMAL) {
    if (!o->lambda_grid || o->n_grid < 1 || o->n_grid > kMaxGrid)
      return fail(c, LSLU_EINVAL, "a lambda grid of 1..256 values is required");
    for (int i = 0; i < o->n_grid; ++i) {
      const double g = o->lambda_grid[i];
      if (!std::isfinite(g) || g <= 0.0)
        return fail(c, LSLU_EINVAL, "lambda grid values must be finite and > 0");
      if (i > 0 && !(g > o->lambda_grid[i - 1]))
        return fail(c, LSLU_EINVAL, "lambda grid must be strictly ascending");
    }
  }
  auto check_piv = [&](const int32_t* p, int count, int64_t lim,
                       const char* what) -> lslu_status {
    std::vector<char> seen(static_cast<size_t>(lim), 0);
    for (int i = 0; i < count; ++i) {
      if (p[i] < 0 || p[i] >= lim)
        return fail(c, LSLU_EINVAL, std::string(what) + ": pivot out of range");
      if (seen[p[i]])
        return fail(c, LSLU_EINVAL, std::string(what) + ": repeated pivot");
      seen[p[i]] = 1;
    }
    return LSLU_OK;
  };
  const int K = o->maxiter;
  if (o->sample_rows) {
    if (o->sample_s < 1 || o->sample_len < 1 || o->sample_len > kMaxSampleLen)
      return fail(c, LSLU_EINVAL, "sample_s must be >= 1 and sample_len in [1, 512]");
    for (int i = 0; i < 2 * K + 1; ++i) {
      const int64_t len = (i % 2 == 0) ? m : n;
      for (int e = 0; e < o->sample_len; ++e) {
        const int32_t r = o->sample_rows[(int64_t)i * o->sample_len + e];
        if (r < -1 || r >= len)
          return fail(c, LSLU_EINVAL, "sample_rows: row out of range");
      }
    }
  }
  if (o->replay_piv_t) {
    lslu_status st = check_piv(o->replay_piv_t, (int)std::min<int64_t>(K + 1, m), m,
                               "replay_piv_t");
    if (st != LSLU_OK) return st;
  }
  if (o->replay_piv_g) {
    lslu_status st = check_piv(o->replay_piv_g, (int)std::min<int64_t>(K, n), n,
                               "replay_piv_g");
    if (st != LSLU_OK) return st;
  }
  if (o->replay_lambda_idx) {
    for (int i = 0; i < K; ++i)
      if (o->replay_lambda_idx[i] >= o->n_grid)
        return fail(c, LSLU_EINVAL, "replay_lambda_idx out of range");
  }
  return LSLU_OK;
}

template <typename T>
void copy_out(T* dst, const T* src, size_t count) {
  if (dst) std::memcpy(dst, src, sizeof(T) * count);
}

// The PSF tile shape (output rows per lane) that runs one A and one A^T
// product fastest on this device, by HIP events on the context's stream:
// each candidate is warmed up, then timed over a few product pairs.  Every
// candidate sums each output in the same order, so the choice changes
// timing only.
lslu_status tune_psf(lslu_ctx* c, lslu_op* op, int* chosen) {
  const int64_t n = op->d.n;
  const size_t esz = prec_size(op->d.prec);
  void *x = nullptr, *y = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Free {
    void **x, **y;
    hipEvent_t *e0, *e1;
    ~Free() {
      if (*x) (void)hipFree(*x);
      if (*y) (void)hipFree(*y);
      if (*e0) (void)hipEventDestroy(*e0);
      if (*e1) (void)hipEventDestroy(*e1);
    }
  } guard{&x, &y, &e0, &e1};
  LSLU_HIP(c, hipMalloc(&x, esz * n));
  LSLU_HIP(c, hipMalloc(&y, esz * n));
  LSLU_HIP(c, hipEventCreate(&e0));
  LSLU_HIP(c, hipEventCreate(&e1));
  const hipStream_t s = c->stream;
  if (esz == sizeof(double))
    launch_fill<double>(static_cast<double*>(x), 1.0, n, s);
  else
    launch_fill<float>(static_cast<float*>(x), 1.0f, n, s);
  const int saved = op->d.psf_r;
  constexpr int kShapes[3] = {2, 4, 8};
  for (int r : kShapes) {  // warm-up: each shape's kernels loaded and run once
    op->d.psf_r = r;
    for (int i = 0; i < 2; ++i) op_apply(op->d, i & 1, x, y, nullptr, s);
  }
  // The fastest of five timings per shape, the shapes interleaved within each
  // round so that a slow stretch of the device (clocks, a profiler's
  // per-dispatch work) does not fall on one shape alone.
  float fastest[3] = {0.f, 0.f, 0.f};
  for (int trial = 0; trial < 5; ++trial) {
    for (int k = 0; k < 3; ++k) {
      op->d.psf_r = kShapes[k];
      LSLU_HIP(c, hipEventRecord(e0, s));
      for (int i = 0; i < 4; ++i) op_apply(op->d, i & 1, x, y, nullptr, s);
      LSLU_HIP(c, hipEventRecord(e1, s));
      LSLU_HIP(c, hipEventSynchronize(e1));
      float ms = 0.f;
      LSLU_HIP(c, hipEventElapsedTime(&ms, e0, e1));
      if (trial == 0 || ms < fastest[k]) fastest[k] = ms;
    }
  }
  int pick = kShapes[0];
  float best = fastest[0];
  for (int k = 1; k < 3; ++k)
    if (fastest[k] < best) {
      best = fastest[k];
      pick = kShapes[k];
    }
  op->d.psf_r = saved;
  LSLU_HIP(c, hipGetLastError());
  *chosen = pick;
  return LSLU_OK;
}

}  // namespace

// ------------------------------------------------- no-allocation solves ---
// The device workspace of lslu_solve_static: one fixed array in the memory
// of each GPU the library runs on (placed when the code object is loaded,
// held until the process ends), shared by every such call on that GPU.
// Host code reaches it only through the address hipGetSymbolAddress gives
// for the device, looked up once per device at context creation and kept in
// g_scratch_ptr; the array's name in host code is a host-side stand-in, not
// a device address.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// With `device` current: the device address of the static scratch, looked
// up once per device.
void init_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_tried[device]) return;
  g_scratch_tried[device] = true;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = (e == hipSuccess) ? p : nullptr;
}

void* static_scratch(int device, hipError_t* err) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  *err = g_scratch_tried[device] ? g_scratch_err[device] : hipErrorNotInitialized;
  return g_scratch_ptr[device];
}

// The part of a context's state that describes its workspace; swapped for
// the duration of a static solve and restored on every exit.
struct GeomSwap {
  lslu_ctx* c;
  Layout lay;
  int64_t m, n;
  Strides bs;
  bool rowmajor;
  int K;
  size_t esz;
  int grid_slots;
  explicit GeomSwap(lslu_ctx* ctx)
      : c(ctx), lay(ctx->lay), m(ctx->m), n(ctx->n), bs(ctx->bs), rowmajor(ctx->rowmajor),
        K(ctx->K), esz(ctx->esz), grid_slots(ctx->grid_slots) {}
  ~GeomSwap() {
    c->lay = lay;
    c->m = m;
    c->n = n;
    c->bs = bs;
    c->rowmajor = rowmajor;
    c->K = K;
    c->esz = esz;
    c->grid_slots = grid_slots;
  }
};
}  // namespace

// =========================================================================
extern "C" {

int lslu_abi_version(void) { return LSLU_ABI_VERSION; }

const char* lslu_status_name(int s) {
  switch (s) {
    case LSLU_OK: return "LSLU_OK";
    case LSLU_BREAKDOWN_Q: return "LSLU_BREAKDOWN_Q";
    case LSLU_BREAKDOWN_U: return "LSLU_BREAKDOWN_U";
    case LSLU_ZERO_RHS: return "LSLU_ZERO_RHS";
    case LSLU_EINVAL: return "LSLU_EINVAL";
    case LSLU_ENOMEM: return "LSLU_ENOMEM";
    case LSLU_EDEVICE: return "LSLU_EDEVICE";
    case LSLU_ENONFINITE: return "LSLU_ENONFINITE";
    case LSLU_EUNSUPPORTED: return "LSLU_EUNSUPPORTED";
    default: return "LSLU_UNKNOWN";
  }
}

const char* lslu_last_error(const lslu_ctx* ctx) {
  if (!ctx) return "no context (lslu_create failed or was not called)";
  return ctx->err.c_str();
}

lslu_status lslu_create(int device, void* hip_stream, lslu_ctx** out) {
  if (!out) return LSLU_EINVAL;
  *out = nullptr;
  try {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return LSLU_EDEVICE;
    if (device < 0 || device >= count) return LSLU_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return LSLU_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LSLU_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return LSLU_EDEVICE;
    lslu_ctx* c = new lslu_ctx();
    c->device = device;
    c->lds_max = prop.sharedMemPerBlock;
    recurrence_init_attributes(c->lds_max);
    projected_init_attributes(c->lds_max);
    init_static_scratch(device);
    if (hip_stream) {
      c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return LSLU_EDEVICE;
      }
      c->own_stream = true;
    }
    bool ok = true;
    for (int i = 0; i < 2; ++i) {
      ok = ok && hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking) == hipSuccess;
      ok = ok && hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      lslu_destroy(c);
      return LSLU_EDEVICE;
    }
    *out = c;
    return LSLU_OK;
  } catch (const std::bad_alloc&) {
    return LSLU_ENOMEM;
  } catch (...) {
    return LSLU_EDEVICE;
  }
}

lslu_status lslu_destroy(lslu_ctx* c) {
  if (!c) return LSLU_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (c->ws) (void)hipFree(c->ws);
  if (c->adj) (void)hipFree(c->adj);
  if (c->hio) (void)hipFree(c->hio);
  if (c->bat) (void)hipFree(c->bat);
  if (c->host) (void)hipHostFree(c->host);
  if (c->adj_host) (void)hipHostFree(c->adj_host);
  for (int i = 0; i < 2; ++i) {
    if (c->side[i]) (void)hipStreamSynchronize(c->side[i]);
    if (c->side[i]) (void)hipStreamDestroy(c->side[i]);
    if (c->join[i]) (void)hipEventDestroy(c->join[i]);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return LSLU_OK;
}

lslu_status lslu_op_dense(lslu_ctx* c, int64_t m, int64_t n, const double* A,
                          int32_t prec, lslu_op** out) {
  if (!c) return LSLU_EINVAL;
  if (!out || !A) return fail(c, LSLU_EINVAL, "NULL argument");
  *out = nullptr;
  if (m < 1 || n < 1) return fail(c, LSLU_EINVAL, "m and n must be >= 1");
  if (prec < LSLU_FP64 || prec > LSLU_FP8OP) return fail(c, LSLU_EINVAL, "bad precision");
  if (m > INT32_MAX || n > INT32_MAX) return fail(c, LSLU_EINVAL, "size too large");
  try {
    Range r_call("lslu_op_dense");
    if (!finite_all(A, m * n)) return fail(c, LSLU_ENONFINITE, "A has NaN/Inf");
    LSLU_HIP(c, hipSetDevice(c->device));
    std::vector<double> AT(static_cast<size_t>(m * n));
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < n; ++j) AT[j * m + i] = A[i * n + j];
    lslu_op* op = new lslu_op();
    op->serial = ++g_op_serial;
    op->ctx = c;
    op->d.kind = 0;
    op->d.prec = prec;
    op->d.m = m;
    op->d.n = n;
    auto va = convert_values(A, m * n, prec);
    auto vt = convert_values(AT.data(), m * n, prec);
    lslu_status st = upload(c, &op->d.A, va.data(), va.size());
    if (st == LSLU_OK) st = upload(c, &op->d.AT, vt.data(), vt.size());
    if (st != LSLU_OK) {
      free_op(op->d);
      delete op;
      return st;
    }
    *out = op;
    return LSLU_OK;
  } catch (const std::bad_alloc&) {
    return fail(c, LSLU_ENOMEM, "host allocation failed");
  }
}

lslu_status lslu_op_csr(lslu_ctx* c, int64_t m, int64_t n, int64_t nnz,
                        const int64_t* indptr, const int32_t* indices,
                        const double* data, int32_t prec, lslu_op** out) {
  if (!c) return LSLU_EINVAL;
  if (!out || !indptr || (nnz > 0 && (!indices || !data)))
    return fail(c, LSLU_EINVAL, "NULL argument");
  *out = nullptr;
  if (m < 1 || n < 1 || nnz < 0) return fail(c, LSLU_EINVAL, "bad shape");
  if (m > INT32_MAX - 1 || n > INT32_MAX - 1 || nnz > INT32_MAX - 1)
    return fail(c, LSLU_EINVAL, "sizes must be < 2^31");
  if (prec < LSLU_FP64 || prec > LSLU_FP8OP) return fail(c, LSLU_EINVAL, "bad precision");
  try {
    Range r_call("lslu_op_csr");
    if (const char* bad = csr_check(m, n, nnz, indptr, indices))
      return fail(c, LSLU_EINVAL, bad);
    if (!finite_all(data, nnz)) return fail(c, LSLU_ENONFINITE, "data has NaN/Inf");
    LSLU_HIP(c, hipSetDevice(c->device));
    std::vector<int> rp(m + 1), rpT, ciT;
    std::vector<double> valT;
    for (int64_t r = 0; r <= m; ++r) rp[r] = static_cast<int>(indptr[r]);
    csr_transpose(m, n, nnz, indptr, indices, data, rpT, ciT, valT);
    lslu_op* op = new lslu_op();
    op->serial = ++g_op_serial;
    op->ctx = c;
    op->d.kind = 1;
    op->d.prec = prec;
    op->d.m = m;
    op->d.n = n;
    op->d.nnz = nnz;
    // Index and value arrays carry kCsrPad zero entries past nnz: the
    // products read rows in aligned chunks of 4 entries.
    std::vector<int> cpad(indices, indices + nnz);
    cpad.resize(nnz + kCsrPad, 0);
    ciT.resize(nnz + kCsrPad, 0);
    std::vector<double> dpad(data, data + nnz);
    dpad.resize(nnz + kCsrPad, 0.0);
    valT.resize(nnz + kCsrPad, 0.0);
    auto va = convert_values(dpad.data(), nnz + kCsrPad, prec);
    auto vt = convert_values(valT.data(), nnz + kCsrPad, prec);
    // column indices in 16 bits when every one fits (A's are < n, A^T's < m)
    auto upload_idx = [&](void** dst, const std::vector<int>& idx, bool narrow) -> lslu_status {
      if (!narrow) return upload(c, dst, idx.data(), sizeof(int) * idx.size());
      const std::vector<uint16_t> v16 = narrow_indices(idx);
      return upload(c, dst, v16.data(), sizeof(uint16_t) * v16.size());
    };
    const bool n16 = n <= 65536, m16 = m <= 65536;
    op->d.idx16 = (n16 ? 1 : 0) | (m16 ? 2 : 0);
    lslu_status st = upload(c, reinterpret_cast<void**>(&op->d.rp), rp.data(), sizeof(int) * (m + 1));
    if (st == LSLU_OK) st = upload_idx(&op->d.ci, cpad, n16);
    if (st == LSLU_OK) st = upload(c, &op->d.val, va.data(), va.size());
    if (st == LSLU_OK) st = upload(c, reinterpret_cast<void**>(&op->d.rpT), rpT.data(), sizeof(int) * (n + 1));
    if (st == LSLU_OK) st = upload_idx(&op->d.ciT, ciT, m16);
    if (st == LSLU_OK) st = upload(c, &op->d.valT, vt.data(), vt.size());
    if (st != LSLU_OK) {
      free_op(op->d);
      delete op;
      return st;
    }
    *out = op;
    return LSLU_OK;
  } catch (const std::bad_alloc&) {
    return fail(c, LSLU_ENOMEM, "host allocation failed");
  }
}

lslu_status lslu_op_psf(lslu_ctx* c, int64_t rows, int64_t cols, int32_t ph,
                        int32_t pw, const double* psf, int32_t prec,
                        lslu_op** out) {
  if (!c) return LSLU_EINVAL;
  if (!out || !psf) return fail(c, LSLU_EINVAL, "NULL argument");
  *out = nullptr;
  if (rows < 1 || cols < 1 || rows * cols > INT32_MAX)
    return fail(c, LSLU_EINVAL, "bad image shape");
  if (ph < 1 || pw < 1 || ph % 2 == 0 || pw % 2 == 0 || ph > 31 || pw > 31)
    return fail(c, LSLU_EINVAL, "PSF sizes must be odd and <= 31");
  if (prec < LSLU_FP64 || prec > LSLU_FP8OP) return fail(c, LSLU_EINVAL, "bad precision");
  if (!finite_all(psf, (int64_t)ph * pw)) return fail(c, LSLU_ENONFINITE, "PSF has NaN/Inf");
  try {
    Range r_call("lslu_op_psf");
    LSLU_HIP(c, hipSetDevice(c->device));
    const int np = ph * pw;
    std::vector<double> p(psf, psf + np), pf(np);
    // FP32: the weights are float values (held in double, the type the FP32
    // products sum in), as the dense and CSR operators store theirs.
    if (prec == kFP32)
      for (double& w : p) w = static_cast<double>(static_cast<float>(w));
    for (int a = 0; a < ph; ++a)
      for (int b = 0; b < pw; ++b) pf[a * pw + b] = p[(ph - 1 - a) * pw + (pw - 1 - b)];
    // float copies of the weights in the 16-bit operator formats
    std::vector<float> p32(np), pf32(np);
    for (int i = 0; i < np; ++i) {
      if (prec == kFP16) {
        p32[i] = f16_to_f32(f64_to_f16(p[i]));
        pf32[i] = f16_to_f32(f64_to_f16(pf[i]));
      } else if (prec == kFP8) {
        p32[i] = fp8_to_f32(f64_to_fp8(p[i]));
        pf32[i] = fp8_to_f32(f64_to_fp8(pf[i]));
      } else {
        p32[i] = bf16_to_f32(f32_to_bf16(static_cast<float>(p[i])));
        pf32[i] = bf16_to_f32(f32_to_bf16(static_cast<float>(pf[i])));
      }
    }
    lslu_op* op = new lslu_op();
    op->serial = ++g_op_serial;
    op->ctx = c;
    op->d.kind = 2;
    op->d.prec = prec;
    op->d.m = rows * cols;
    op->d.n = rows * cols;
    op->d.rows = rows;
    op->d.cols = cols;
    op->d.ph = ph;
    op->d.pw = pw;
    lslu_status st = upload(c, reinterpret_cast<void**>(&op->d.psf), p.data(), sizeof(double) * np);
    if (st == LSLU_OK) st = upload(c, reinterpret_cast<void**>(&op->d.psf_flip), pf.data(), sizeof(double) * np);
    if (st == LSLU_OK) st = upload(c, reinterpret_cast<void**>(&op->d.psf32), p32.data(), sizeof(float) * np);
    if (st == LSLU_OK) st = upload(c, reinterpret_cast<void**>(&op->d.psf32_flip), pf32.data(), sizeof(float) * np);
    if (st == LSLU_OK && (prec == kBF16 || prec == kFP16 || prec == kFP8)) {
      const auto mb = psf_mfma_rows(p, ph, pw, prec);
      const auto mbf = psf_mfma_rows(pf, ph, pw, prec);
      st = upload(c, reinterpret_cast<void**>(&op->d.mb), mb.data(), sizeof(uint64_t) * mb.size());
      if (st == LSLU_OK)
        st = upload(c, reinterpret_cast<void**>(&op->d.mb_flip), mbf.data(),
                    sizeof(uint64_t) * mbf.size());
    }
    int r = 0;
    if (st == LSLU_OK) st = tune_psf(c, op, &r);
    if (st != LSLU_OK) {
      free_op(op->d);
      delete op;
      return st;
    }
    op->d.psf_r = r;
    *out = op;
    return LSLU_OK;
  } catch (const std::bad_alloc&) {
    return fail(c, LSLU_ENOMEM, "host allocation failed");
  }
}


lslu_status lslu_op_tile(lslu_ctx* c, lslu_op* op, int32_t rows_per_lane, int32_t* chosen) {
  if (!c) return LSLU_EINVAL;
  if (!op) return fail(c, LSLU_EINVAL, "NULL argument");
  if (op->ctx != c) return fail(c, LSLU_EINVAL, "operator belongs to another context");
  if (op->d.kind != 2) return fail(c, LSLU_EUNSUPPORTED, "only PSF operators have a tile shape");
  if (c->pending)
    return fail(c, LSLU_EINVAL, "an asynchronous solve is pending on this context (lslu_wait)");
  if (rows_per_lane != 0 && rows_per_lane != 2 && rows_per_lane != 4 && rows_per_lane != 8)
    return fail(c, LSLU_EINVAL, "rows_per_lane must be 0 (measure), 2, 4 or 8");
  try {
    Range r_call("lslu_op_tile");
    LSLU_HIP(c, hipSetDevice(c->device));
    int r = rows_per_lane;
    if (r == 0) {
      lslu_status st = tune_psf(c, op, &r);
      if (st != LSLU_OK) return st;
    }
    if (r != op->d.psf_r) drop_op_graphs(c, op->serial);  // captured with the old shape
    op->d.psf_r = r;
    if (chosen) *chosen = r;
    return LSLU_OK;
  } catch (const std::bad_alloc&) {
    return fail(c, LSLU_ENOMEM, "host allocation failed");
  }
}

lslu_status lslu_op_apply(lslu_ctx* c, const lslu_op* op, int32_t transpose,
                          const void* x, void* y) {
  if (!c) return LSLU_EINVAL;
  if (!op || !x || !y) return fail(c, LSLU_EINVAL, "NULL argument");
  if (op->ctx != c) return fail(c, LSLU_EINVAL, "operator belongs to another context");
  LSLU_HIP(c, hipSetDevice(c->device));
  op_apply(op->d, transpose ? 1 : 0, x, y, nullptr, c->stream);
  LSLU_HIP(c, hipGetLastError());
  return LSLU_OK;
}

lslu_status lslu_op_info(const lslu_op* op, int64_t* m, int64_t* n, int32_t* prec) {
  if (!op) return LSLU_EINVAL;
  if (m) *m = op->d.m;
  if (n) *n = op->d.n;
  if (prec) *prec = op->d.prec;
  return LSLU_OK;
}

lslu_status lslu_op_destroy(lslu_op* op) {
  if (!op) return LSLU_OK;
  if (op->ctx) {
    (void)hipSetDevice(op->ctx->device);
    if (op->ctx->stream) (void)hipStreamSynchronize(op->ctx->stream);
    if (op->ctx->last_op == op) {
      op->ctx->last_op = nullptr;
      op->ctx->last_ok = false;
    }
    drop_op_graphs(op->ctx, op->serial);
  }
  free_op(op->d);
  delete op;
  return LSLU_OK;
}

// Waits for the solve's stream and unpacks the result block copied to
// pinned host memory (same layout as on the device) into res.
static lslu_status complete_solve(lslu_ctx* c, int K, lslu_result* res,
                                  const PhaseEvents* pe_in) {
  const hipStream_t s = c->stream;
  const Layout& l = c->lay;
  {
    Range r_wait("lslu: wait for the solve");
    LSLU_HIP(c, hipStreamSynchronize(s));
  }
  PhaseEvents none;
  const PhaseEvents& pe = pe_in ? *pe_in : none;
    // Unpack the result block (same layout as on the device).
    auto hp = [&](const void* dev) {
      return c->host + (static_cast<const unsigned char*>(dev) - l.res);
    };
    const DevState* st = reinterpret_cast<const DevState*>(hp(l.st));
    const int* sel = reinterpret_cast<const int*>(hp(l.sel));
    c->last_nl = st->n_l;
    c->last_nd = st->n_d;
    if (st->spin_timeouts != 0)
      return fail(c, LSLU_EDEVICE, "a wait inside the recurrence ran out (device fault)");
    c->last_kdone = st->k_done;
    c->last_ok = st->status >= 0;
    float t_rec = 0.f, t_proj = 0.f, t_asm = 0.f;
    if (pe.on) {
      LSLU_HIP(c, hipEventElapsedTime(&t_rec, pe.ev[0], pe.ev[1]));
      LSLU_HIP(c, hipEventElapsedTime(&t_proj, pe.ev[1], pe.ev[2]));
      LSLU_HIP(c, hipEventElapsedTime(&t_asm, pe.ev[2], pe.ev[3]));
    }
    const lslu_status status = static_cast<lslu_status>(st->status);
    if (res) {
      res->status = status;
      res->k_done = st->k_done;
      res->k_stop = sel[0];
      res->n_l = st->n_l;
      res->n_d = st->n_d;
      res->beta = st->beta;
      res->piv_t_mismatch = st->mismatch_t;
      res->piv_g_mismatch = st->mismatch_g;
      copy_out(res->piv_t, reinterpret_cast<const int32_t*>(hp(l.piv_t)), K + 1);
      copy_out(res->piv_g, reinterpret_cast<const int32_t*>(hp(l.piv_g)), K);
      copy_out(res->own_piv_t, reinterpret_cast<const int32_t*>(hp(l.own_t)), K + 1);
      copy_out(res->own_piv_g, reinterpret_cast<const int32_t*>(hp(l.own_g)), K);
      copy_out(res->H, reinterpret_cast<const double*>(hp(l.H)), (size_t)(K + 1) * K);
      copy_out(res->W, reinterpret_cast<const double*>(hp(l.W)), (size_t)K * K);
      copy_out(res->Y, reinterpret_cast<const double*>(hp(l.Y)), (size_t)K * K);
      copy_out(res->lambda_k, reinterpret_cast<const double*>(hp(l.lam)), K);
      copy_out(res->lambda_idx, reinterpret_cast<const int32_t*>(hp(l.lam_idx)), K);
      copy_out(res->ghat, reinterpret_cast<const double*>(hp(l.ghat)), K);
      copy_out(res->sep_lambda, reinterpret_cast<const double*>(hp(l.sep)), K);
      copy_out(res->sigma_max, reinterpret_cast<const double*>(hp(l.smax)), K);
      copy_out(res->sigma_min, reinterpret_cast<const double*>(hp(l.smin)), K);
      copy_out(res->dloss_dlambda, reinterpret_cast<const double*>(hp(l.dldl)), K);
      copy_out(res->sep_t, reinterpret_cast<const double*>(hp(l.psep)), K + 1);
      copy_out(res->sep_g, reinterpret_cast<const double*>(hp(l.psep)) + (K + 1), K);
      res->t_recurrence_ms = t_rec;
      res->n_recurrence_launches = pe.on ? pe.launches : 0;
      res->t_projected_ms = t_proj;
      res->t_assemble_ms = t_asm;
    }
    return status;
}

lslu_status lslu_solve(lslu_ctx* c, const lslu_op* op, const void* b,
                       const void* x0, const lslu_opts* o, void* x_out,
                       lslu_result* res) {
  if (!c) return LSLU_EINVAL;
  if (!op || !b || !o || !x_out) return fail(c, LSLU_EINVAL, "NULL argument");
  if (op->ctx != c) return fail(c, LSLU_EINVAL, "operator belongs to another context");
  if (c->pending)
    return fail(c, LSLU_EINVAL, "an asynchronous solve is pending on this context (lslu_wait)");
  if ((o->flags & LSLU_FLAG_ASYNC) && (o->flags & LSLU_FLAG_TIMING))
    return fail(c, LSLU_EINVAL, "LSLU_FLAG_TIMING needs a synchronous solve");
  try {
    Range r_call("lslu_solve");
    lslu_status vs = validate_opts(c, op, o);
    if (vs != LSLU_OK) return vs;
    c->last_ok = false;
    c->last_op = op;
    LSLU_HIP(c, hipSetDevice(c->device));
    const int K = o->maxiter;
    const size_t esz = prec_size(op->d.prec);
    lslu_status ws = ensure_ws(c, op->d.m, op->d.n, K, esz, op->d.kind != 2);
    if (ws != LSLU_OK) return ws;
    const Layout& l = c->lay;
    const hipStream_t s = c->stream;
    const bool rt = o->replay_piv_t != nullptr, rg = o->replay_piv_g != nullptr,
               rl = o->replay_lambda_idx != nullptr;
    // Small host inputs: uploaded only when they changed (pageable copies
    // synchronise with the host).
    {
      std::vector<double> grid;
      if (o->reg == LSLU_REG_WGCV || o->reg == LSLU_REG_GCV || o->reg == LSLU_REG_OPTIMAL)
        grid.assign(o->lambda_grid, o->lambda_grid + o->n_grid);
      // the cached copy is tied to the device buffer, which moves with the
      // workspace layout
      grid.push_back(static_cast<double>(reinterpret_cast<uintptr_t>(l.grid)));
      if (grid.size() > 1 && grid != c->up_grid) {
        LSLU_HIP(c, hipMemcpyAsync(l.grid, grid.data(), sizeof(double) * (grid.size() - 1),
                                   hipMemcpyHostToDevice, s));
        LSLU_HIP(c, hipStreamSynchronize(s));
      }
      c->up_grid = grid;
      std::vector<int> rep(3 * (K + 1) + 2, -1);
      const uintptr_t rp = reinterpret_cast<uintptr_t>(l.rep_t);
      rep[3 * (K + 1)] = static_cast<int>(rp & 0x7fffffff);
      rep[3 * (K + 1) + 1] = static_cast<int>((rp >> 31) & 0x7fffffff);
      for (int i = 0; rt && i < std::min<int64_t>(K + 1, op->d.m); ++i) rep[i] = o->replay_piv_t[i];
      for (int i = 0; rg && i < std::min<int64_t>(K, op->d.n); ++i) rep[(K + 1) + i] = o->replay_piv_g[i];
      for (int i = 0; rl && i < K; ++i) rep[2 * (K + 1) + i] = o->replay_lambda_idx[i];
      if ((rt || rg || rl) && rep != c->up_rep) {
        LSLU_HIP(c, hipMemcpyAsync(l.rep_t, rep.data(), sizeof(int) * (K + 1),
                                   hipMemcpyHostToDevice, s));
        LSLU_HIP(c, hipMemcpyAsync(l.rep_g, rep.data() + (K + 1), sizeof(int) * K,
                                   hipMemcpyHostToDevice, s));
        LSLU_HIP(c, hipMemcpyAsync(l.rep_lam, rep.data() + 2 * (K + 1), sizeof(int) * K,
                                   hipMemcpyHostToDevice, s));
        LSLU_HIP(c, hipStreamSynchronize(s));
        c->up_rep = rep;
      }
      if (o->sample_rows) {
        // rows of kMaxSampleLen on the device; the key also ties the cached
        // copy to the buffer's address
        std::vector<int> sm((size_t)(2 * K + 1) * kMaxSampleLen + 2, -1);
        for (int i = 0; i < 2 * K + 1; ++i)
          std::memcpy(sm.data() + (size_t)i * kMaxSampleLen,
                      o->sample_rows + (int64_t)i * o->sample_len, sizeof(int) * o->sample_len);
        const uintptr_t sp = reinterpret_cast<uintptr_t>(l.samp);
        sm[sm.size() - 2] = static_cast<int>(sp & 0x7fffffff);
        sm[sm.size() - 1] = static_cast<int>((sp >> 31) & 0x7fffffff);
        if (sm != c->up_samp) {
          LSLU_HIP(c, hipMemcpyAsync(l.samp, sm.data(), sizeof(int) * (sm.size() - 2),
                                     hipMemcpyHostToDevice, s));
          LSLU_HIP(c, hipStreamSynchronize(s));
          c->up_samp = sm;
        }
      }
    }
    void* X = o->X_dev ? o->X_dev : l.X;
    PhaseEvents pe;
    auto enqueue = [&]() {
      if (esz == sizeof(double))
        enqueue_solve<double>(c, op->d, static_cast<const double*>(b),
                              static_cast<const double*>(x0), o,
                              static_cast<double*>(x_out), static_cast<double*>(X),
                              rt, rg, rl, &pe);
      else
        enqueue_solve<float>(c, op->d, static_cast<const float*>(b),
                             static_cast<const float*>(x0), o,
                             static_cast<float*>(x_out), static_cast<float*>(X),
                             rt, rg, rl, &pe);
    };
    struct EventsGuard {
      PhaseEvents& p;
      ~EventsGuard() {
        for (auto& e : p.ev)
          if (e) (void)hipEventDestroy(e);
      }
    } guard{pe};
    if (o->flags & LSLU_FLAG_TIMING) {
      for (auto& e : pe.ev) LSLU_HIP(c, hipEventCreate(&e));
      pe.on = true;
      enqueue();
    } else if (o->flags & LSLU_FLAG_EAGER) {
      enqueue();
    } else {
      // Everything the captured kernels bake in: pointers, sizes, options.
      std::vector<double> key = {
          (double)op->serial, (double)(uintptr_t)b, (double)(uintptr_t)x0,
          (double)(uintptr_t)x_out, (double)(uintptr_t)X, (double)(uintptr_t)c->ws,
          (double)op->d.kind, (double)op->d.prec, (double)op->d.m, (double)op->d.n,
          (double)K, (double)o->reg, o->lambda, (double)o->n_grid,
          (double)o->grid_relative, o->omega, o->stop_tol, (double)o->early_stop,
          (double)rt, (double)rg, (double)rl, (double)(uintptr_t)o->x_true_dev,
          (double)(o->sample_rows != nullptr), (double)o->sample_s, (double)o->sample_len,
          (double)(o->flags & LSLU_FLAG_GRAD_LAMBDA),
          (double)(o->flags & LSLU_FLAG_FINAL_ONLY),
          (double)(o->flags & LSLU_FLAG_PIVOT_SEP)};
      hipGraphExec_t exec = nullptr;
      for (auto& g : c->graphs)
        if (g.key == key) exec = g.exec;
      if (!exec) {
        if (c->graphs.size() >= kGraphCache) {
          destroy_captured(c->graphs.front());
          c->graphs.erase(c->graphs.begin());
        }
        Range r_cap("lslu_solve: graph capture");
        LSLU_HIP(c, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
        enqueue();
        lslu_ctx::Captured cap;
        cap.key = key;
        const hipError_t ce = hipStreamEndCapture(s, &cap.graph);
        if (ce != hipSuccess || !cap.graph)
          return fail(c, LSLU_EDEVICE, std::string("graph capture failed: ") +
                                           hipGetErrorString(ce));
        const hipError_t ie = hipGraphInstantiate(&cap.exec, cap.graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
          destroy_captured(cap);
          return fail(c, LSLU_EDEVICE, std::string("graph instantiation failed: ") +
                                           hipGetErrorString(ie));
        }
        exec = cap.exec;
        c->graphs.push_back(std::move(cap));
      }
      Range r_launch("lslu_solve: graph launch");
      LSLU_HIP(c, hipGraphLaunch(exec, s));
    }
    LSLU_HIP(c, hipGetLastError());
    LSLU_HIP(c, hipMemcpyAsync(c->host, l.res, l.res_bytes, hipMemcpyDeviceToHost, s));
    if (o->flags & LSLU_FLAG_ASYNC) {
      c->pending = true;
      c->pend_K = K;
      c->pend_res = res;
      return LSLU_OK;
    }
    return complete_solve(c, K, res, &pe);
  } catch (const std::bad_alloc&) {
    return fail(c, LSLU_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(c, LSLU_EDEVICE, "unexpected exception");
  }
}

lslu_status lslu_solve_static(lslu_ctx* c, const lslu_op* op, const void* b,
                              const void* x0, const lslu_opts* o, void* x_out,
                              lslu_result* res) {
  if (!c) return LSLU_EINVAL;
  if (!op || !b || !o || !x_out) return fail(c, LSLU_EINVAL, "NULL argument");
  if (op->ctx != c) return fail(c, LSLU_EINVAL, "operator belongs to another context");
  if (c->pending)
    return fail(c, LSLU_EINVAL, "an asynchronous solve is pending on this context (lslu_wait)");
  if (o->flags & (LSLU_FLAG_ASYNC | LSLU_FLAG_TIMING))
    return fail(c, LSLU_EINVAL, "lslu_solve_static is synchronous: no ASYNC or TIMING flag");
  try {
    const lslu_status vs = validate_opts(c, op, o);
    if (vs != LSLU_OK) return vs;
    LSLU_HIP(c, hipSetDevice(c->device));
    hipError_t serr = hipSuccess;
    unsigned char* base = static_cast<unsigned char*>(static_scratch(c->device, &serr));
    if (!base)
      return fail(c, LSLU_EDEVICE, std::string("no static scratch on this device: ") +
                                       hipGetErrorString(serr));
    const int K = o->maxiter;
    const int64_t m = op->d.m, n = op->d.n;
    const size_t esz = prec_size(op->d.prec);
    const bool rowmajor = op->d.kind != 2;
    const Strides bs = basis_strides(rowmajor, m, n, K);
    const bool grid_rule =
        o->reg == LSLU_REG_WGCV || o->reg == LSLU_REG_GCV || o->reg == LSLU_REG_OPTIMAL;
    const int G = grid_rule ? std::max(o->n_grid, 1) : 1;
    const size_t need = carve(nullptr, m, n, K, esz, bs, nullptr, G);
    if (need > kStaticScratchBytes)
      return fail(c, LSLU_EINVAL,
                  "this solve needs " + std::to_string(need >> 20) +
                      " MiB of device workspace; lslu_solve_static has " +
                      std::to_string(kStaticScratchBytes >> 20) + " MiB (use lslu_solve)");
    Layout lay;
    carve(base, m, n, K, esz, bs, &lay, G);
    const hipStream_t s = c->stream;
    // Small host inputs, copied straight from the caller's arrays.
    if (grid_rule)
      LSLU_HIP(c, hipMemcpyAsync(lay.grid, o->lambda_grid, sizeof(double) * o->n_grid,
                                 hipMemcpyHostToDevice, s));
    const bool rt = o->replay_piv_t != nullptr, rg = o->replay_piv_g != nullptr,
               rl = o->replay_lambda_idx != nullptr;
    if (rt) {
      launch_fill<int>(lay.rep_t, -1, K + 1, s);
      LSLU_HIP(c, hipMemcpyAsync(lay.rep_t, o->replay_piv_t,
                                 sizeof(int) * std::min<int64_t>(K + 1, m),
                                 hipMemcpyHostToDevice, s));
    }
    if (rg) {
      launch_fill<int>(lay.rep_g, -1, K, s);
      LSLU_HIP(c, hipMemcpyAsync(lay.rep_g, o->replay_piv_g,
                                 sizeof(int) * std::min<int64_t>(K, n),
                                 hipMemcpyHostToDevice, s));
    }
    if (rl)
      LSLU_HIP(c, hipMemcpyAsync(lay.rep_lam, o->replay_lambda_idx, sizeof(int) * K,
                                 hipMemcpyHostToDevice, s));
    if (o->sample_rows)
      LSLU_HIP(c, hipMemcpy2DAsync(lay.samp, sizeof(int) * kMaxSampleLen, o->sample_rows,
                                   sizeof(int) * o->sample_len, sizeof(int) * o->sample_len,
                                   2 * K + 1, hipMemcpyHostToDevice, s));
    void* X = o->X_dev ? o->X_dev : lay.X;
    {
      // The solve, its kernels enqueued directly, on the static workspace:
      // the context describes that workspace for the call and its own again
      // afterwards.
      GeomSwap keep(c);
      c->lay = lay;
      c->m = m;
      c->n = n;
      c->bs = bs;
      c->rowmajor = rowmajor;
      c->K = K;
      c->esz = esz;
      c->grid_slots = G;
      PhaseEvents pe;
      if (esz == sizeof(double))
        enqueue_solve<double>(c, op->d, static_cast<const double*>(b),
                              static_cast<const double*>(x0), o, static_cast<double*>(x_out),
                              static_cast<double*>(X), rt, rg, rl, &pe);
      else
        enqueue_solve<float>(c, op->d, static_cast<const float*>(b),
                             static_cast<const float*>(x0), o, static_cast<float*>(x_out),
                             static_cast<float*>(X), rt, rg, rl, &pe);
    }
    LSLU_HIP(c, hipGetLastError());
    // Results straight into the caller's arrays (and two host words here).
    DevState st{};
    int sel[2] = {0, 0};
    LSLU_HIP(c, hipMemcpyAsync(&st, lay.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    LSLU_HIP(c, hipMemcpyAsync(sel, lay.sel, sizeof(sel), hipMemcpyDeviceToHost, s));
    if (res) {
      auto get = [&](void* dst, const void* src, size_t bytes) -> lslu_status {
        if (dst) LSLU_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
        return LSLU_OK;
      };
      const size_t dK = sizeof(double) * K, iK = sizeof(int32_t) * K;
      const lslu_status gs[] = {
          get(res->piv_t, lay.piv_t, iK + sizeof(int32_t)), get(res->piv_g, lay.piv_g, iK),
          get(res->own_piv_t, lay.own_t, iK + sizeof(int32_t)), get(res->own_piv_g, lay.own_g, iK),
          get(res->H, lay.H, dK * (K + 1)), get(res->W, lay.W, dK * K), get(res->Y, lay.Y, dK * K),
          get(res->lambda_k, lay.lam, dK), get(res->lambda_idx, lay.lam_idx, iK),
          get(res->ghat, lay.ghat, dK), get(res->sep_lambda, lay.sep, dK),
          get(res->sigma_max, lay.smax, dK), get(res->sigma_min, lay.smin, dK),
          get(res->dloss_dlambda, lay.dldl, dK),
          get(res->sep_t, lay.psep, dK + sizeof(double)),
          get(res->sep_g, lay.psep + (K + 1), dK)};
      for (lslu_status g : gs)
        if (g != LSLU_OK) return g;
    }
    LSLU_HIP(c, hipStreamSynchronize(s));
    // The reverse pass and lslu_get_basis read the context's own workspace,
    // which this solve did not use.
    c->last_ok = false;
    c->last_op = nullptr;
    c->last_nl = 0;
    c->last_nd = 0;
    if (st.spin_timeouts != 0)
      return fail(c, LSLU_EDEVICE, "a wait inside the recurrence ran out (device fault)");
    const lslu_status status = static_cast<lslu_status>(st.status);
    if (res) {
      res->status = status;
      res->k_done = st.k_done;
      res->k_stop = sel[0];
      res->n_l = st.n_l;
      res->n_d = st.n_d;
      res->beta = st.beta;
      res->piv_t_mismatch = st.mismatch_t;
      res->piv_g_mismatch = st.mismatch_g;
      res->t_recurrence_ms = 0.0;
      res->n_recurrence_launches = 0;
      res->t_projected_ms = 0.0;
      res->t_assemble_ms = 0.0;
    }
    return status;
  } catch (const std::bad_alloc&) {
    return fail(c, LSLU_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(c, LSLU_EDEVICE, "unexpected exception");
  }
}

lslu_status lslu_solve_host(lslu_ctx* c, const lslu_op* op, const double* b,
                            const double* x0, const lslu_opts* o, double* x_out,
                            lslu_result* res) {
  if (!c) return LSLU_EINVAL;
  if (!op || !b || !o || !x_out) return fail(c, LSLU_EINVAL, "NULL argument");
  if (op->ctx != c) return fail(c, LSLU_EINVAL, "operator belongs to another context");
  if (o->flags & LSLU_FLAG_ASYNC)
    return fail(c, LSLU_EINVAL, "lslu_solve_host is synchronous (no LSLU_FLAG_ASYNC)");
  const int64_t m = op->d.m, n = op->d.n;
  if (!finite_all(b, m) || (x0 && !finite_all(x0, n)))
    return fail(c, LSLU_ENONFINITE, "b or x0 has NaN/Inf");
  try {
    Range r_call("lslu_solve_host");
    LSLU_HIP(c, hipSetDevice(c->device));
    const bool dbl = op->d.prec == kFP64;
    const size_t esz = dbl ? sizeof(double) : sizeof(float);
    const size_t ob = align_up(esz * m, 256), ox = align_up(esz * n, 256);
    const size_t need = ob + 2 * ox;
    if (need > c->hio_bytes) {
      if (c->hio) LSLU_HIP(c, hipFree(c->hio));
      c->hio = nullptr;
      c->hio_bytes = 0;
      LSLU_HIP(c, hipMalloc(&c->hio, need));
      c->hio_bytes = need;
    }
    unsigned char* bd = c->hio;
    unsigned char* x0d = c->hio + ob;
    unsigned char* xd = c->hio + ob + ox;
    // working precision: FP64, or each value rounded to float
    auto put = [&](void* dst, const double* src, int64_t len) -> lslu_status {
      if (dbl) {
        return copy_sync(c, dst, src, sizeof(double) * len, hipMemcpyHostToDevice);
      } else {
        std::vector<float> t(static_cast<size_t>(len));
        for (int64_t i = 0; i < len; ++i) t[i] = static_cast<float>(src[i]);
        return copy_sync(c, dst, t.data(), sizeof(float) * len, hipMemcpyHostToDevice);
      }
      return LSLU_OK;
    };
    LSLU_HIP(c, hipStreamSynchronize(c->stream));
    lslu_status st = put(bd, b, m);
    if (st == LSLU_OK && x0) st = put(x0d, x0, n);
    if (st != LSLU_OK) return st;
    const lslu_status ss = lslu_solve(c, op, bd, x0 ? x0d : nullptr, o, xd, res);
    if (ss < 0) return ss;
    if (dbl) {
      const lslu_status cs = copy_sync(c, x_out, xd, sizeof(double) * n, hipMemcpyDeviceToHost);
      if (cs != LSLU_OK) return cs;
    } else {
      std::vector<float> t(static_cast<size_t>(n));
      const lslu_status cs = copy_sync(c, t.data(), xd, sizeof(float) * n, hipMemcpyDeviceToHost);
      if (cs != LSLU_OK) return cs;
      for (int64_t i = 0; i < n; ++i) x_out[i] = t[i];
    }
    return ss;
  } catch (const std::bad_alloc&) {
    return fail(c, LSLU_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(c, LSLU_EDEVICE, "unexpected exception");
  }
}

lslu_status lslu_solve_batch(int32_t count, lslu_ctx* const* ctxs, const lslu_op* const* ops,
                             const void* const* b, const lslu_opts* o, void* const* x_out,
                             lslu_result* const* res) {
  if (count < 1 || !ctxs || !ctxs[0]) return LSLU_EINVAL;
  lslu_ctx* c0 = ctxs[0];
  if (!ops || !b || !o || !x_out) return fail(c0, LSLU_EINVAL, "NULL argument");
  if (o->flags & (LSLU_FLAG_ASYNC | LSLU_FLAG_TIMING | LSLU_FLAG_GRAD_LAMBDA))
    return fail(c0, LSLU_EINVAL, "batched solves take no ASYNC, TIMING or GRAD_LAMBDA flag");
  if (o->reg == LSLU_REG_OPTIMAL || o->x_true_dev || o->X_dev || o->sample_rows ||
      o->replay_piv_t || o->replay_piv_g || o->replay_lambda_idx)
    return fail(c0, LSLU_EINVAL,
                "batched solves take no per-problem device arrays in opts (x_true_dev, X_dev), "
                "sampled pivots or replays");
  for (int i = 0; i < count; ++i) {
    lslu_ctx* c = ctxs[i];
    if (!c || !ops[i] || !b[i] || !x_out[i]) return fail(c0, LSLU_EINVAL, "NULL argument");
    if (ops[i]->ctx != c) return fail(c0, LSLU_EINVAL, "operator belongs to another context");
    if (c->device != c0->device) return fail(c0, LSLU_EINVAL, "contexts on different devices");
    if (c->pending) return fail(c0, LSLU_EINVAL, "an asynchronous solve is pending");
    if (ops[i]->d.kind == 2 || ops[i]->d.kind != ops[0]->d.kind || ops[i]->d.prec != ops[0]->d.prec)
      return fail(c0, LSLU_EINVAL,
                  "a batch needs dense or CSR operators of one kind and one precision");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(c0, LSLU_EINVAL, "each problem needs its own context");
    const lslu_status vs = validate_opts(c, ops[i], o);
    if (vs != LSLU_OK) return fail(c0, vs, "problem " + std::to_string(i) + ": " + c->err);
  }
  try {
    Range r_call("lslu_solve_batch");
    LSLU_HIP(c0, hipSetDevice(c0->device));
    const int K = o->maxiter;
    const int P = count;
    const size_t esz = prec_size(ops[0]->d.prec);
    const hipStream_t s = c0->stream;
    std::vector<double> grid;
    if (o->reg == LSLU_REG_WGCV || o->reg == LSLU_REG_GCV)
      grid.assign(o->lambda_grid, o->lambda_grid + o->n_grid);
    for (int i = 0; i < P; ++i) {
      lslu_ctx* c = ctxs[i];
      const lslu_status ws = ensure_ws(c, ops[i]->d.m, ops[i]->d.n, K, esz, true);
      if (ws != LSLU_OK) return fail(c0, ws, c->err);
      LSLU_HIP(c0, hipStreamSynchronize(c->stream));  // nothing else uses the workspace
      if (!grid.empty())
      {
        const lslu_status cs = copy_sync(c, c->lay.grid, grid.data(),
                                         sizeof(double) * grid.size(), hipMemcpyHostToDevice);
        if (cs != LSLU_OK) return fail(c0, cs, c->err);
      }
      c->up_grid.clear();  // the single-solve upload cache no longer describes it
      c->last_ok = false;
      c->last_op = ops[i];
    }
    auto run = [&](auto tag) -> lslu_status {
      using T = decltype(tag);
      std::vector<std::vector<PlannedHalf<T>>> plans(P);
      PhaseEvents none;
      for (int i = 0; i < P; ++i)
        enqueue_solve<T>(ctxs[i], ops[i]->d, static_cast<const T*>(b[i]), nullptr, o,
                         static_cast<T*>(x_out[i]), static_cast<T*>(ctxs[i]->lay.X), false,
                         false, false, &none, s, 1, &plans[i]);
      const size_t nh = plans[0].size();
      for (int i = 1; i < P; ++i)
        if (plans[i].size() != nh) return fail(c0, LSLU_EDEVICE, "inconsistent batch plan");
      // Size classes: the problems sorted by rows, split into up to
      // kBatchStreams groups of consecutive sizes.  Each group's merged
      // launches go to the stream of its first problem's context, so the
      // groups run side by side and a group waits only for its own largest
      // problem at each launch.
      constexpr int kBatchStreams = 4;
      std::vector<int> order(P);
      for (int i = 0; i < P; ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return ops[x]->d.m < ops[y]->d.m;
      });
      const int G = std::min(kBatchStreams, P);
      std::vector<std::vector<int>> groups(G);
      for (int g = 0; g < G; ++g)
        for (int q = g * P / G; q < (g + 1) * P / G; ++q) groups[g].push_back(order[q]);
      // device copies per group: every launch's argument blocks, the row
      // access of each operator in both directions, and the block offsets
      const size_t opb = row_op_bytes(ops[0]->d);
      struct Seg {
        size_t args, ops, first;
      };
      std::vector<Seg> seg(G);
      size_t total = 0;
      for (int g = 0; g < G; ++g) {
        const size_t pg = groups[g].size();
        seg[g].args = align_up(total, 256);
        seg[g].ops = align_up(seg[g].args + sizeof(HalfArgs<T>) * nh * pg, 256);
        seg[g].first = align_up(seg[g].ops + 2 * opb * pg, 256);
        total = seg[g].first + sizeof(int) * nh * (pg + 1);
      }
      std::vector<unsigned char> hb(total, 0);
      std::vector<std::vector<int>> blocks(G, std::vector<int>(nh));
      for (int g = 0; g < G; ++g) {
        const int pg = static_cast<int>(groups[g].size());
        for (size_t h = 0; h < nh; ++h) {
          int* first = reinterpret_cast<int*>(hb.data() + seg[g].first) + h * (pg + 1);
          int off = 0;
          for (int q = 0; q < pg; ++q) {
            const PlannedHalf<T>& ph = plans[groups[g][q]][h];
            if (ph.tr != plans[0][h].tr) return fail(c0, LSLU_EDEVICE, "inconsistent batch plan");
            std::memcpy(hb.data() + seg[g].args + sizeof(HalfArgs<T>) * (h * pg + q), &ph.a,
                        sizeof(HalfArgs<T>));
            first[q] = off;
            off += ph.a.nlead + ph.ncons;
          }
          first[pg] = off;
          blocks[g][h] = off;
        }
        for (int tr = 0; tr < 2; ++tr)
          for (int q = 0; q < pg; ++q)
            row_op_write(ops[groups[g][q]]->d, tr, hb.data() + seg[g].ops + opb * (tr * pg + q));
      }
      if (total > c0->bat_bytes) {
        if (c0->bat) LSLU_HIP(c0, hipFree(c0->bat));
        c0->bat = nullptr;
        c0->bat_bytes = 0;
        LSLU_HIP(c0, hipMalloc(&c0->bat, total));
        c0->bat_bytes = total;
      }
      {
        const lslu_status cs = copy_sync(c0, c0->bat, hb.data(), total, hipMemcpyHostToDevice);
        if (cs != LSLU_OK) return cs;
      }
      // events: set-up done (on s), and each group's recurrence done
      std::vector<hipEvent_t> evs(G + 1, nullptr);
      struct EvGuard {
        std::vector<hipEvent_t>& e;
        ~EvGuard() {
          for (auto x : e)
            if (x) (void)hipEventDestroy(x);
        }
      } evg{evs};
      for (auto& e : evs) LSLU_HIP(c0, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      LSLU_HIP(c0, hipEventRecord(evs[G], s));
      std::vector<hipStream_t> gs(G);
      for (int g = 0; g < G; ++g) {
        gs[g] = ctxs[groups[g][0]]->stream;
        LSLU_HIP(c0, hipStreamWaitEvent(gs[g], evs[G], 0));
      }
      for (size_t h = 0; h < nh; ++h) {
        const int tr = plans[0][h].tr;
        for (int g = 0; g < G; ++g) {
          const int pg = static_cast<int>(groups[g].size());
          const int lead = groups[g][0];
          launch_half_batch<T>(plans[lead][h].a, ops[lead]->d, tr, c0->lds_max,
                               reinterpret_cast<const HalfArgs<T>*>(c0->bat + seg[g].args) + h * pg,
                               c0->bat + seg[g].ops + opb * tr * pg,
                               reinterpret_cast<const int*>(c0->bat + seg[g].first) + h * (pg + 1),
                               pg, blocks[g][h], gs[g]);
        }
      }
      std::vector<int> group_of(P);
      for (int g = 0; g < G; ++g) {
        LSLU_HIP(c0, hipEventRecord(evs[g], gs[g]));
        for (int i : groups[g]) group_of[i] = g;
      }
      // The projected problems and the assembly of each problem on its own
      // context's stream, after its group's recurrence.
      for (int i = 0; i < P; ++i) {
        lslu_ctx* c = ctxs[i];
        LSLU_HIP(c0, hipStreamWaitEvent(c->stream, evs[group_of[i]], 0));
        enqueue_solve<T>(c, ops[i]->d, static_cast<const T*>(b[i]), nullptr, o,
                         static_cast<T*>(x_out[i]), static_cast<T*>(c->lay.X), false, false,
                         false, &none, c->stream, 2, nullptr);
        LSLU_HIP(c0, hipMemcpyAsync(c->host, c->lay.res, c->lay.res_bytes,
                                    hipMemcpyDeviceToHost, c->stream));
      }
      LSLU_HIP(c0, hipGetLastError());
      for (int i = 0; i < P; ++i) LSLU_HIP(c0, hipStreamSynchronize(ctxs[i]->stream));
      return LSLU_OK;
    };
    const lslu_status rs = esz == sizeof(double) ? run(double{}) : run(float{});
    if (rs != LSLU_OK) return rs;
    lslu_status worst = LSLU_OK;
    for (int i = 0; i < P; ++i) {
      const lslu_status st = complete_solve(ctxs[i], K, res ? res[i] : nullptr, nullptr);
      if (st < 0 && worst >= 0) {
        worst = st;
        c0->err = "problem " + std::to_string(i) + ": " + ctxs[i]->err;
      }
    }
    return worst;
  } catch (const std::bad_alloc&) {
    return fail(c0, LSLU_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(c0, LSLU_EDEVICE, "unexpected exception");
  }
}

lslu_status lslu_wait(lslu_ctx* c) {
  if (!c) return LSLU_EINVAL;
  if (!c->pending) return LSLU_OK;
  try {
    LSLU_HIP(c, hipSetDevice(c->device));
    c->pending = false;
    return complete_solve(c, c->pend_K, c->pend_res, nullptr);
  } catch (...) {
    return fail(c, LSLU_EDEVICE, "unexpected exception");
  }
}

lslu_status lslu_vjp(lslu_ctx* c, const lslu_op* op, int32_t k, const void* xbar,
                     void* bbar, double* lambda_bar) {
  if (!c) return LSLU_EINVAL;
  if (!op || !xbar || !bbar) return fail(c, LSLU_EINVAL, "NULL argument");
  if (op->ctx != c) return fail(c, LSLU_EINVAL, "operator belongs to another context");
  if (c->pending)
    return fail(c, LSLU_EINVAL, "an asynchronous solve is pending on this context (lslu_wait)");
  if (!c->last_ok || c->last_op != op)
    return fail(c, LSLU_EINVAL, "no completed solve with this operator on the context");
  if (k < 1 || k > c->last_kdone)
    return fail(c, LSLU_EINVAL, "k must be in [1, k_done] of the last solve");
  try {
    Range r_call("lslu_vjp");
    LSLU_HIP(c, hipSetDevice(c->device));
    const int K = c->K;
    const int64_t m = c->m, n = c->n;
    const size_t esz = c->esz;
    const int64_t ldl = (int64_t)align_up((size_t)n, 64), ldd = (int64_t)align_up((size_t)m, 64);
    // scratch: two passes, sizes then pointers
    VjpArgs a{};
    auto carve_adj = [&](unsigned char* base) {
      size_t off = 0;
      auto take = [&](size_t bytes) -> unsigned char* {
        off = align_up(off, 256);
        unsigned char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
      };
      a.Lbar = take(esz * ldl * K);
      a.Dbar = take(esz * ldd * (K + 1));
      a.um = take(esz * m);
      a.un = take(esz * n);
      a.pm = take(esz * m);
      a.pn = take(esz * n);
      a.part = reinterpret_cast<double*>(take(sizeof(double) * adjoint_part_doubles(K, std::max(m, n))));
      a.M = reinterpret_cast<double*>(take(sizeof(double) * K * K));
      a.Hbar = reinterpret_cast<double*>(take(sizeof(double) * (K + 1) * K));
      a.corr = reinterpret_cast<double*>(take(sizeof(double) * (K + 2)));
      a.scal = reinterpret_cast<double*>(take(sizeof(double) * 4));
      a.fail = reinterpret_cast<int*>(take(sizeof(int)));
      a.inv_t = reinterpret_cast<int*>(take(sizeof(int) * m));
      a.inv_g = reinterpret_cast<int*>(take(sizeof(int) * n));
      return align_up(off, 256);
    };
    const size_t need = carve_adj(nullptr);
    if (need > c->adj_bytes) {
      if (c->adj) LSLU_HIP(c, hipFree(c->adj));
      c->adj = nullptr;
      c->adj_bytes = 0;
      LSLU_HIP(c, hipMalloc(&c->adj, need));
      c->adj_bytes = need;
    }
    if (!c->adj_host) LSLU_HIP(c, hipHostMalloc(&c->adj_host, 64));
    carve_adj(c->adj);
    const Layout& l = c->lay;
    a.op = &op->d;
    a.m = m;
    a.n = n;
    a.K = K;
    a.k = k;
    a.n_l = c->last_nl;
    a.n_d = c->last_nd;
    a.L = l.L;
    a.D = l.D;
    a.TL = l.TL;
    a.TD = l.TD;
    a.rsL = c->bs.rsL;
    a.csL = c->bs.csL;
    a.rsD = c->bs.rsD;
    a.csD = c->bs.csD;
    a.H = l.H;
    a.W = l.W;
    a.Y = l.Y;
    a.lam = l.lam;
    a.piv_t = l.piv_t;
    a.piv_g = l.piv_g;
    a.st = l.st;
    a.xbar = xbar;
    a.bbar = bbar;
    a.ldl = ldl;
    a.ldd = ldd;
    const hipStream_t s = c->stream;
    if (esz == sizeof(double))
      run_vjp<double>(a, s);
    else
      run_vjp<float>(a, s);
    LSLU_HIP(c, hipGetLastError());
    LSLU_HIP(c, hipMemcpyAsync(c->adj_host, a.scal, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    LSLU_HIP(c, hipMemcpyAsync(c->adj_host + 2, a.fail, sizeof(int), hipMemcpyDeviceToHost, s));
    LSLU_HIP(c, hipStreamSynchronize(s));
    int bad = 0;
    std::memcpy(&bad, c->adj_host + 2, sizeof(int));
    if (bad)
      return fail(c, LSLU_EINVAL,
                  "H_k^T H_k + lambda_k^2 I is singular: the derivative is not defined");
    if (lambda_bar) *lambda_bar = c->adj_host[1];
    return LSLU_OK;
  } catch (const std::bad_alloc&) {
    return fail(c, LSLU_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(c, LSLU_EDEVICE, "unexpected exception");
  }
}

lslu_status lslu_get_basis(lslu_ctx* c, int32_t which, int32_t count, void* dst) {
  if (!c) return LSLU_EINVAL;
  if (!dst) return fail(c, LSLU_EINVAL, "NULL argument");
  if (c->pending)
    return fail(c, LSLU_EINVAL, "an asynchronous solve is pending on this context (lslu_wait)");
  const int have = which == 0 ? c->last_nl : c->last_nd;
  if (which < 0 || which > 1 || count < 0 || count > have)
    return fail(c, LSLU_EINVAL, "count exceeds the basis of the last solve");
  if (count == 0) return LSLU_OK;
  LSLU_HIP(c, hipSetDevice(c->device));
  const int64_t len = which == 0 ? c->n : c->m;
  const int64_t rs = which == 0 ? c->bs.rsL : c->bs.rsD;
  const int64_t cs = which == 0 ? c->bs.csL : c->bs.csD;
  const void* src = which == 0 ? c->lay.L : c->lay.D;
  if (c->esz == sizeof(double))
    launch_basis_copy<double>(static_cast<const double*>(src), rs, cs, len, count,
                              static_cast<double*>(dst), c->stream);
  else
    launch_basis_copy<float>(static_cast<const float*>(src), rs, cs, len, count,
                             static_cast<float*>(dst), c->stream);
  LSLU_HIP(c, hipGetLastError());
  return LSLU_OK;
}

}  // extern "C"
