// One half-iteration of the pivoted rectangular Hessenberg process
// (Algorithm 4; the basis part of Algorithm 5) in one launch.
//
// The l side at iteration k (the d side mirrors it with A, D and t): the
// previous launch left u, the unnormalised d-side vector (zero at t(1..k-1)),
// and its per-block pivot candidates.
//   block 0           t(k) = the row of the largest |u| among the candidates
//                     (smallest row among equals), the breakdown test,
//                     H(k,k-1) (or beta at k = 1) and the new triangle row
//                     (d_1..d_{k-1})(t(k)); publishes (t(k), H(k,k-1)).  Then
//                     solves T_L w = (A^T d_k)(g(1..k-1)) by forward
//                     substitution and publishes w = W(1:k-1,k).
//   blocks 1..nlead-1 (A^T d_k)(g(j)), one wavefront per j.
//   other blocks      their rows of q0 = A^T d_k, d_k = u / H(k,k-1) into its
//                     basis column (IEEE division: exactly 1 at t(k)), then
//                     q = q0 - L_{k-1} w, q = 0 at g(1..k-1), and per block the
//                     largest remaining |q|.
// w equals the values the sequential loop of Algorithm 5 reads at g(j): l_i is
// 1 at g(i) and 0 at g(j), j < i.  The forward substitution gives each row j
// its subtractions in increasing i, as that loop does; floating-point
// contraction is disabled there so each step rounds like a multiply then a
// subtract.
//
// Products read the normalised vector as they gather it: each input is u(c)
// divided by the pivot value with the value of IEEE division (Normaliser), the
// same value the normalised basis column holds, so products and exact
// cancellations are those of the normalised vector.  The products therefore start once the pivot is
// published; the triangular solve of block 0 overlaps them.
//
// Synchronisation inside the launch: the pivot-entry blocks and the
// consumers wait only for block 0; block 0 publishes the pivot before it
// waits for anything, and then waits only for the pivot-entry blocks, which
// follow it directly (blocks 1..nlead-1, a few dozen at most).  Workgroups
// are dispatched in order, so block 0 and its entry blocks are resident
// before any consumer, and every wait ends whatever else occupies the
// device.  Everything published inside a launch (the pivot, its value, the
// pivot entries, the coefficients) goes through slots that hold a sentinel
// until written once; a waiter polls the slot itself, so no flag has to order
// other memory and nobody fences.  Every load a product needs that does not
// depend on the pivot (indices, values and the gathered entries of the
// unnormalised vector) is issued before the wait.  Every wait is bounded: a
// wait that runs out counts a device error and the launch finishes.  Results
// do not depend on timing or on the launch configuration.
#pragma once

#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "device_common.hpp"

namespace lslu {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kCoefPerLane = 16;  // coefficients per lane of the elimination
constexpr int kPartsPerThread = kMaxParts / kThreads;  // 16
constexpr int kStage = 8;
constexpr int kEntryStage = 8;   // staged terms per lane of a pivot-entry row
constexpr int kRowStage = 8;     // staged terms per lane of a consumer's first row
constexpr int kNormBatch = 8;
constexpr int kNormStage = 2;  // entries of the normalisation share loaded before the pivot
constexpr int kSpinLimit = 1 << 20;
constexpr int kTriB = 32;  // rows of a diagonal block of the triangular solve
constexpr uint64_t kSentinel = kSlotEmpty;
constexpr size_t kTriLdsMax = 32 * 1024;
static_assert(sizeof(ArgPart) == 16, "candidates are read as 16-byte vectors");

__host__ __device__ inline int64_t packed_row(int j) { return (int64_t)j * (j - 1) / 2; }

// ------------------------------------------------------------------ slots --
// Slots are written once per launch with device-coherent stores and polled
// with device-coherent loads (they bypass the non-coherent caches, so no
// fence is needed on either side: a device-scope fence writes back and
// invalidates the whole L2 of the XCD).
__device__ inline void store_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t load_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t load_u64(const double* p) {
  return load_u64(reinterpret_cast<const uint64_t*>(p));
}

__device__ inline int load_i(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t dbits(double v) { return __builtin_bit_cast(uint64_t, v); }

// Block-wide bounded wait for the pivot of the previous half.  Returns true
// with its row and value when one was found, false on breakdown or when the
// bound ran out (counted as a device error).
template <typename T>
__device__ inline bool wait_pivot(const HalfArgs<T>& a, DevState* st, int& pick,
                                  double& val) {
  __shared__ uint64_t sv, sp;
  if (threadIdx.x == 0) {
    uint64_t v = kSentinel, p = kSentinel;
    for (int it = 0; it < kSpinLimit; ++it) {
      v = load_u64(a.pslot);
      p = load_u64(a.pslot + 1);
      if (v != kSentinel && p != kSentinel) break;
      __builtin_amdgcn_s_sleep(1);
    }
    if (v == kSentinel || p == kSentinel) {
      atomicAdd(&st->spin_timeouts, 1);
      p = 0;  // state 0: stop
    }
    sv = v;
    sp = p;
  }
  __syncthreads();
  const uint64_t p = sp;
  pick = static_cast<int>(static_cast<uint32_t>(p));
  val = __builtin_bit_cast(double, sv);
  return (p >> 32) == 1;
}

// ------------------------------------------------------- triangular solve --
// T g = g in place for the nb x nb unit lower triangular T packed by rows
// (row j at offset j(j-1)/2 holds T(j, 0..j-1)), in 32-row blocks:
// wavefront 0 keeps its lanes' rows of the diagonal block in registers (zero
// above the diagonal) and runs the dependent chain with w_i broadcast by
// readlane; the workgroup then updates the rows below.
template <typename T>
__device__ __attribute__((always_inline)) inline void trisolve_inplace(
    double* g, int nb, const T* __restrict__ tp) {
#pragma clang fp contract(off)
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  for (int b0 = 0; b0 < nb; b0 += kTriB) {
    const int bs = min(kTriB, nb - b0);
    if (w == 0) {
      const int j = b0 + lane;
      const bool act = lane < bs;
      const T* row = tp + packed_row(act ? j : b0) + b0;  // T(j, b0 + i) = row[i]
      T tr[kTriB];
#pragma unroll
      for (int i = 0; i < kTriB; ++i) tr[i] = (act && i < lane) ? row[i] : T(0);
      double gl = act ? g[j] : 0.0;
#pragma unroll
      for (int i = 0; i < kTriB; ++i) {
        const double wi = readlane_d(gl, i);
        gl = gl - static_cast<double>(tr[i]) * wi;  // tr[i] == 0 unless i < lane
      }
      if (act) g[j] = gl;
    }
    __syncthreads();
    for (int j = b0 + bs + tid; j < nb; j += kThreads) {
      const T* row = tp + packed_row(j) + b0;
      double gj = g[j];
      int i = 0;
      for (; i + 8 <= bs; i += 8) {
        double tv[8], wv8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          tv[u] = static_cast<double>(row[i + u]);
          wv8[u] = g[b0 + i + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) gj = gj - tv[u] * wv8[u];
      }
      for (; i < bs; ++i) gj = gj - static_cast<double>(row[i]) * g[b0 + i];
      g[j] = gj;
    }
    __syncthreads();
  }
}

// T g = g in place for 2 <= nb <= 64 S (S <= 4) by one wavefront, the unit lower
// triangular T packed by rows in LDS: row j lives in lane j % 64, slot
// j / 64; step i broadcasts w_i = g_i by readlane and every later row
// subtracts T(j,i) w_i, so each row sees the sequential order.  The entries
// of the next 8 steps are loaded ahead (indices clamped into the triangle;
// rows not updated by a step keep their value), so no step waits on LDS.
// Rows of slot s are final once steps 0 .. 64 (s + 1) - 1 have run; each
// slot's values are then stored to pub (the coefficient slots), so
// consumers can start on the first coefficients while later ones are solved.
template <typename T, int S>
__device__ __attribute__((always_inline)) inline void trisolve_wave(double* g, int nb,
                                                                    const T* __restrict__ tp,
                                                                    uint64_t* pub) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & (kWave - 1);
  if (threadIdx.x < kWave) {
    const int64_t P = packed_row(nb);
    double gr[S];
    int64_t base[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = lane + kWave * s;
      gr[s] = j < nb ? g[j] : 0.0;
      base[s] = j < nb ? packed_row(j) : 0;
    }
#pragma unroll
    for (int s0 = 0; s0 < S; ++s0) {
      const int ib = kWave * s0, ie = min(nb, kWave * (s0 + 1));
      for (int i0 = ib; i0 < ie; i0 += 8) {
        T t[S][8];
#pragma unroll
        for (int s = s0; s < S; ++s)
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int64_t q = base[s] + i0 + u;
            t[s][u] = tp[q < P ? q : P - 1];
          }
        // No early exit: a step past the last row (i >= nb) changes no row
        // (j > i fails for every j < nb), and i - ib stays below 64 (i0 - ib
        // is a multiple of 8 below ie - ib <= 64), so all 8 steps run
        // unconditionally and the loads above are issued together instead
        // of one before each step.
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          const double wi = readlane_d(gr[s0], i - ib);
#pragma unroll
          for (int s = s0; s < S; ++s) {
            const int j = lane + kWave * s;
            const double nv = gr[s] - static_cast<double>(t[s][u]) * wi;
            gr[s] = (j > i && j < nb) ? nv : gr[s];
          }
        }
      }
      const int j = lane + kWave * s0;
      if (j < nb) store_u64(pub + j, dbits(gr[s0]));
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = lane + kWave * s;
      if (j < nb) g[j] = gr[s];
    }
  }
  __syncthreads();
}

// Sampled pivot search (the variant of Section 2.2): among the first
// sample_s listed rows that are not earlier pivots, the entry of largest
// magnitude (ties: smallest row), as a signed key; 0 when all are 0.  One
// wavefront: every listed row, its eligibility and its value are loaded
// first (kMaxSampleLen / 64 per lane), then the rank of each listed row among
// the eligible ones is a ballot prefix count in list order.  The result is
// returned to every thread of the block (one barrier).
template <typename T>
__device__ inline void sampled_search(const HalfArgs<T>& a, double& key, int& idx) {
  __shared__ double s_key;
  __shared__ int s_idx;
  static_assert(kMaxSampleLen % kWave == 0, "sample lists fill whole wavefront rows");
  constexpr int kPer = kMaxSampleLen / kWave;
  const PivotJob& job = a.job;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  if (tid < kWave) {
    int row[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int li = u * kWave + lane;
      row[u] = li < job.sample_len ? job.sample[li] : -1;
    }
    unsigned char mk[kPer];
    T v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int r = row[u] >= 0 ? row[u] : 0;
      mk[u] = job.mask[r];
      v[u] = a.up[r];
    }
    double bk = 0.0;
    int bi = INT_MAX, base = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const bool elig = row[u] >= 0 && mk[u] == 0;
      const uint64_t bal = __ballot(elig);
      const int below = __popcll(bal & ((1ull << lane) - 1ull));
      const double vv = static_cast<double>(v[u]);
      if (elig && base + below < job.sample_s && better(vv, row[u], bk, bi)) {
        bk = vv;
        bi = row[u];
      }
      base += __popcll(bal);
    }
    wave_argmax(bk, bi);
    if (lane == 0) {
      s_key = bk;
      s_idx = bi;
    }
  }
  __syncthreads();
  key = s_key;
  idx = s_idx;
}

// ------------------------------------------------------------ block 0 -----
template <typename T, bool kTriLds>
__device__ void lead(const HalfArgs<T>& a, DevState* st, unsigned char* lds) {
  __shared__ double g[kMaxIter + 1];
  __shared__ int all_in;
  const int tid = threadIdx.x;
  const int nb = a.rows > 0 ? a.nb : 0;
  // The triangle's first pass and the candidates are loaded before either is
  // used.
  T tbuf[kStage];
  const int64_t P = (kTriLds && nb > 1) ? packed_row(nb) : 0;
#pragma unroll
  for (int u = 0; u < kStage; ++u) {
    const int64_t p = (int64_t)u * kThreads + tid;
    tbuf[u] = (p < P) ? a.Tp[p] : T(0);
  }
  double key = 0.0;
  int idx = INT_MAX;
  const PivotJob& job = a.job;
  // A sampled search decides alone unless its entries are all 0; then (and
  // always without a sample) the block candidates of the previous launch are
  // reduced: the full search.
  if (job.sample) sampled_search(a, key, idx);
  if (!(fabs(key) > 0.0)) {
    key = 0.0;
    idx = INT_MAX;
    constexpr int kHalf = kPartsPerThread / 2;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int4 raw[kHalf];
#pragma unroll
      for (int u = 0; u < kHalf; ++u) {
        const int i = tid + (h * kHalf + u) * kThreads;
        raw[u] = (i < a.nparts_in) ? reinterpret_cast<const int4*>(a.parts_in)[i]
                                   : make_int4(0, 0, INT_MAX, 0);
      }
#pragma unroll
      for (int u = 0; u < kHalf; ++u) {
        const double k2 = __builtin_bit_cast(
            double, (static_cast<uint64_t>(static_cast<uint32_t>(raw[u].y)) << 32) |
                        static_cast<uint32_t>(raw[u].x));
        if (better(k2, raw[u].z, key, idx)) {
          key = k2;
          idx = raw[u].z;
        }
      }
    }
    block_argmax<kThreads>(key, idx);
  }
  const int own = (job.eligible && fabs(key) > 0.0) ? idx : -1;
  const int pick = job.replay ? (job.eligible ? job.replay[job.piv_pos] : -1) : own;
  // The winning candidate carries the pivot value; a replayed pivot is read.
  const double val = pick < 0 ? 0.0
                     : (job.replay ? static_cast<double>(a.up[pick]) : key);
  const bool brk = (pick < 0 || val == 0.0);
  if (tid == 0) {
    store_u64(a.pslot, dbits(brk ? 0.0 : val));
    store_u64(a.pslot + 1, static_cast<uint32_t>(pick) | (static_cast<uint64_t>(brk ? 2 : 1) << 32));
    if (job.own_list) job.own_list[job.piv_pos] = own;
    if (job.replay && pick != own) {
      if (job.side == 0) st->mismatch_g += 1; else st->mismatch_t += 1;
    }
    if (brk) {
      // Breakdown: no eligible nonzero entry (Algorithm 4, "else break").
      st->stopped = 1;
      if (job.side == 2) {
        st->status = kZeroRHS;
        st->k_done = 0;
      } else if (job.side == 0) {
        st->status = kBreakQ;  // x stays x_{k-1}
      } else {
        *job.piv_val = 0.0;    // H(k+1,k) = 0; x_k is still formed
        st->status = kBreakU;
        st->k_done = job.k;
      }
    } else {
      *job.piv_val = val;
      job.piv_list[job.piv_pos] = pick;
      job.mask[pick] = 1;
      if (job.side == 2) {
        st->beta = val;
        st->n_d = 1;
      } else if (job.side == 0) {
        st->n_l = job.k;
      } else {
        st->n_d = job.k + 1;
        st->k_done = job.k;
      }
    }
  }
  if (brk) return;
  if (a.Trowp) {  // needed by later launches only
    for (int j = tid; j < a.nbp; j += kThreads)
      a.Trowp[j] = a.basisp[(int64_t)pick * a.rsp + (int64_t)j * a.csp];
  }
  if (nb == 0) return;
  if constexpr (kTriLds) {
    T* lt = reinterpret_cast<T*>(lds);
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int64_t p = (int64_t)u * kThreads + tid;
      if (p < P) lt[p] = tbuf[u];
    }
    for (int64_t p0 = (int64_t)kThreads * kStage; p0 < P; p0 += (int64_t)kThreads * kStage) {
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int64_t p = p0 + (int64_t)u * kThreads + tid;
        tbuf[u] = (p < P) ? a.Tp[p] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int64_t p = p0 + (int64_t)u * kThreads + tid;
        if (p < P) lt[p] = tbuf[u];
      }
    }
  }
  // The pivot entries of the product, written once by blocks 1..nlead-1.
  bool got = true;
  for (int j = tid; j < nb; j += kThreads) {
    uint64_t bits = kSentinel;
    for (int it = 0; it < kSpinLimit; ++it) {
      bits = load_u64(a.entries + j);
      if (bits != kSentinel) break;
      __builtin_amdgcn_s_sleep(1);
    }
    if (bits == kSentinel) got = false;
    g[j] = __builtin_bit_cast(double, bits);
  }
  if (tid == 0) all_in = 1;
  __syncthreads();
  if (!got) all_in = 0;
  __syncthreads();
  if (!all_in) {
    if (tid == 0) {
      atomicAdd(&st->spin_timeouts, 1);
      __hip_atomic_store(a.fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  uint64_t* cs = reinterpret_cast<uint64_t*>(a.cslot);
  bool published = false;  // the solve stored the slots itself
  if constexpr (kTriLds) {
    const T* lt = reinterpret_cast<const T*>(lds);
    published = nb >= 2 && nb <= 4 * kWave;
    if (nb >= 2 && nb <= kWave)
      trisolve_wave<T, 1>(g, nb, lt, cs);
    else if (nb > kWave && nb <= 2 * kWave)
      trisolve_wave<T, 2>(g, nb, lt, cs);
    else if (nb > 2 * kWave && nb <= 3 * kWave)
      trisolve_wave<T, 3>(g, nb, lt, cs);
    else if (nb > 3 * kWave && nb <= 4 * kWave)
      trisolve_wave<T, 4>(g, nb, lt, cs);
    else
      trisolve_inplace<T>(g, nb, lt);
  } else {
    trisolve_inplace<T>(g, nb, a.Tp);
  }
  for (int j = tid; j < nb; j += kThreads) {
    if (!published) store_u64(cs + j, dbits(g[j]));
    a.coef[j] = g[j];
  }
}

// ------------------------------------------------- pivot-entry blocks -----
// bid: this block's index within its solve's blocks (1..nlead-1).
template <typename T, class RowOp>
__device__ void pivot_entries(const HalfArgs<T>& a, const RowOp& op, DevState* st, int bid) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int jr = (bid - 1) * kWaves + w;
  const bool act = jr < a.nb;
  if constexpr (is_psf_pixels<RowOp>::value) {
    // A PSF entry has at most 31 x 31 terms, 16 per lane: the weights and the
    // unnormalised inputs of all of them are loaded before the wait (clamped
    // in-bounds addresses, terms outside the image or the PSF masked), and
    // each lane sums its terms t = lane, lane + 64, ... in increasing t, as
    // the row policy's partial sum does.
    using Acc = typename RowOp::Acc;
    constexpr int kTaps = 16;
    T u[kTaps];
    Acc wv[kTaps];
    bool in[kTaps];
    if (act) {
      const int64_t pix = a.piv[jr];
      const int i = static_cast<int>(pix / op.cols);
      const int j = static_cast<int>(pix - (int64_t)i * op.cols);
      const int np = op.ph * op.pw, ch = op.ph / 2, cw = op.pw / 2;
#pragma unroll
      for (int q = 0; q < kTaps; ++q) {
        const int t = lane + q * kWave;
        const int aa = t / op.pw, bb = t - aa * op.pw;
        const int gi = i + aa - ch, gj = j + bb - cw;
        in[q] = t < np && gi >= 0 && gi < op.rows && gj >= 0 && gj < op.cols;
        u[q] = a.up[in[q] ? (int64_t)gi * op.cols + gj : 0];
        wv[q] = op.wt[t < np ? t : 0];
      }
    }
    int pick;
    double val;
    if (!wait_pivot(a, st, pick, val)) return;
    if (!act) return;
    const Normaliser<T> nz(static_cast<T>(val));
    Acc acc = 0;
#pragma unroll
    for (int q = 0; q < kTaps; ++q)
      if (in[q]) acc = fma(wv[q], static_cast<Acc>(in_val<RowOp::kInMode>(nz(u[q]))), acc);
    acc = group_sum<kWave>(acc);
    if (lane == 0)
      store_u64(reinterpret_cast<uint64_t*>(a.entries) + jr,
                dbits(static_cast<double>(static_cast<T>(acc))));
    return;
  }
  RowStage<typename RowOp::Val, T, kEntryStage> sg;
  if (act) op.template stage<kWave, kEntryStage>(a.piv[jr], lane, a.up, sg);
  int pick;
  double val;
  if (!wait_pivot(a, st, pick, val)) return;
  if (!act) return;
  const Normaliser<T> nz(static_cast<T>(val));
  auto xf = [&](int64_t c) -> T { return nz(a.up[c]); };
  typename RowOp::Acc acc = op.template finish<kWave, kEntryStage>(sg, nz, xf);
  acc = group_sum<kWave>(acc);
  if (lane == 0)
    store_u64(reinterpret_cast<uint64_t*>(a.entries) + jr,
              dbits(static_cast<double>(static_cast<T>(acc))));
}

// Normalise this block's share of the previous vector into its basis column:
// entries i = cb * 256 + tid + u * ncons * 256.  The first kNormStage of a
// thread's entries are loaded before the pivot is known (stage), the rest
// after it.
template <typename T>
struct NormStage {
  T v[kNormStage];
};

template <typename T>
__device__ inline void normalise_stage(const HalfArgs<T>& a, int cb, int ncons, NormStage<T>& s) {
  const int64_t step = (int64_t)ncons * kThreads;
  const int64_t i0 = (int64_t)cb * kThreads + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kNormStage; ++u) {
    const int64_t i = i0 + u * step;
    s.v[u] = (i < a.lenp) ? a.up[i] : T(0);
  }
}

template <typename T>
__device__ inline void normalise_share(const HalfArgs<T>& a, int cb, int ncons,
                                       int pick, const Normaliser<T>& nz,
                                       const NormStage<T>& s) {
  const int64_t step = (int64_t)ncons * kThreads;
  const int64_t i0 = (int64_t)cb * kThreads + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kNormStage; ++u) {
    const int64_t i = i0 + u * step;
    if (i < a.lenp) a.dstp[i * a.dstp_stride] = (i == pick) ? T(1) : nz(s.v[u]);
  }
  for (int64_t j0 = i0 + kNormStage * step; j0 < a.lenp; j0 += step * kNormStage) {
    T vv[kNormStage];
#pragma unroll
    for (int u = 0; u < kNormStage; ++u) {
      const int64_t i = j0 + u * step;
      vv[u] = (i < a.lenp) ? a.up[i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kNormStage; ++u) {
      const int64_t i = j0 + u * step;
      if (i < a.lenp) a.dstp[i * a.dstp_stride] = (i == pick) ? T(1) : nz(vv[u]);
    }
  }
}

__device__ inline void write_part(ArgPart* parts, int b, double key, int idx) {
  parts[b].key = key;
  parts[b].idx = idx;
}

// Waits for the coefficients and stages them in LDS (wavefront 0 polls all
// nb slots at once); false when the launch is to end (block 0 could not form
// them, or the bound ran out).
template <typename T>
__device__ inline bool fetch_coef(const HalfArgs<T>& a, DevState* st, double* cf) {
  __shared__ int ok_s;
  const int nb = a.nb;
  if (nb == 0) return true;
  if (threadIdx.x < kWave) {
    constexpr int kPer = kMaxIter / kWave;
    const int lane = threadIdx.x;
    const uint64_t* cs = reinterpret_cast<const uint64_t*>(a.cslot);
    uint64_t bits[kPer];
    bool ok = false, failed = false;
    for (int it = 0; it < kSpinLimit; ++it) {
      bool miss = false;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int j = lane + u * kWave;
        bits[u] = j < nb ? load_u64(cs + j) : 0;
        miss = miss || (j < nb && bits[u] == kSentinel);
      }
      if (__ballot(miss) == 0) {
        ok = true;
        break;
      }
      if (load_i(a.fail) != 0) {
        failed = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int j = lane + u * kWave;
      if (j < nb) cf[j] = __builtin_bit_cast(double, bits[u]);
    }
    if (lane == 0) {
      ok_s = ok ? 1 : 0;
      if (!ok && !failed) atomicAdd(&st->spin_timeouts, 1);
    }
  }
  __syncthreads();
  return ok_s != 0;
}

// Waits until coefficients 0 .. need - 1 are published and stages every
// coefficient of the published prefix in LDS (wavefront 0 polls); avail
// (block-uniform) becomes the prefix length, at least need.  Called again
// with a larger need when the elimination reaches past avail.  False when
// the launch is to end, as fetch_coef.
template <typename T>
__device__ inline bool fetch_coef_prefix(const HalfArgs<T>& a, DevState* st, double* cf,
                                         int need, int& avail) {
  __shared__ int ok_s, avail_s;
  const int nb = a.nb;
  if (threadIdx.x < kWave) {
    constexpr int kPer = kMaxIter / kWave;
    const int lane = threadIdx.x;
    const uint64_t* cs = reinterpret_cast<const uint64_t*>(a.cslot);
    uint64_t bits[kPer];
    bool ok = false, failed = false;
    int have = avail;
    for (int it = 0; it < kSpinLimit; ++it) {
      // the published prefix: the first slot still empty, or nb
      int first = nb;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int j = lane + u * kWave;
        bits[u] = (j >= have && j < nb) ? load_u64(cs + j) : 0;
        const uint64_t empty = __ballot(j >= have && j < nb && bits[u] == kSentinel);
        if (empty != 0 && first == nb) first = u * kWave + __builtin_ctzll(empty);
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int j = lane + u * kWave;
        if (j >= have && j < first) cf[j] = __builtin_bit_cast(double, bits[u]);
      }
      have = first;
      if (have >= need) {
        ok = true;
        break;
      }
      if (load_i(a.fail) != 0) {
        failed = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) {
      ok_s = ok ? 1 : 0;
      avail_s = have;
      if (!ok && !failed) atomicAdd(&st->spin_timeouts, 1);
    }
  }
  __syncthreads();
  avail = avail_s;
  const bool ok = ok_s != 0;
  __syncthreads();  // avail_s and ok_s are rewritten by the next call
  return ok;
}

// --------------------------------------------------- row consumer blocks --
// G lanes per row, 256 / G rows per block.  Persistent over rows
// r = (cb + i ncons) * (256 / G) + group: the loads of the first row's first
// terms before the pivot is known, then every product (the first kept in a
// register, the others parked in out[r]), the elimination inputs of the first
// row, one wait for the coefficients, then the elimination.  A waiting block
// therefore never holds resources that undispatched work needs.
template <int G, typename T>
__device__ inline void load_basis_row(const HalfArgs<T>& a, int64_t r, int sub,
                                      T (&bv)[kCoefPerLane]) {
  const T* brow = a.basis + r * a.rs;
#pragma unroll
  for (int u = 0; u < kCoefPerLane; ++u) {
    const int j = sub + u * G;
    bv[u] = (j < a.nb) ? brow[(int64_t)j * a.cs] : T(0);
  }
}

template <int G, typename T, class RowOp>
__device__ void consume_rows(const HalfArgs<T>& a, const RowOp& op, DevState* st,
                             int cb, int ncons) {
  using Acc = typename RowOp::Acc;
  constexpr int kRows = kThreads / G;  // rows per block and pass
  static_assert(G * kCoefPerLane >= kMaxIter, "one pass over the coefficients");
  __shared__ double cf[kMaxIter];
  __shared__ double sk[kRows];
  __shared__ int si[kRows];
  const int tid = threadIdx.x, sub = tid % G, rl = tid / G;
  const int nb = a.nb;
  const int64_t stride = (int64_t)ncons * kRows;
  const int64_t r0 = (int64_t)cb * kRows + rl;
  const bool has0 = r0 < a.rows;
  // 16-, 8-bit dense rows on the matrix cores: the block's 16 rows of each
  // pass as one row group (its 4 wavefronts take every 4th column block, the
  // 4 partial sums added in wavefront order)
  bool mf = false;
  if constexpr (DenseMfma<RowOp>::value) mf = G == 16 && dense_mfma_fits<RowOp::kInMode>(op.cols);
  RowStage<typename RowOp::Val, T, kRowStage> sg;
  if (has0 && !mf) op.template stage<G, kRowStage>(r0, sub, a.up, sg);
  NormStage<T> ns;
  normalise_stage(a, cb, ncons, ns);
  int pick;
  double val;
  if (!wait_pivot(a, st, pick, val)) return;
  const Normaliser<T> nz(static_cast<T>(val));
  normalise_share(a, cb, ncons, pick, nz, ns);
  auto xf = [&](int64_t c) -> T { return nz(a.up[c]); };
  T q_first = T(0);
  if (mf) {
    if constexpr (DenseMfma<RowOp>::value) {
      constexpr int kB = RowOp::kInMode;
      static_assert(kRows == 16, "one row group per pass");
      __shared__ typename PsfMfma<kB>::E xs[kDenseMfmaMaxCols];
      __shared__ float part[kWaves][16];
      __shared__ float first[16];
      dense_mfma_stage_x<kB>(xf, op.cols, xs, kThreads);
      __syncthreads();
      const int w = tid / kWave, lane = tid & (kWave - 1);
      for (int64_t rb = (int64_t)cb * kRows; rb < a.rows; rb += stride) {
        const mfma_f4 acc = dense_mfma_rows16<kB>(op.a, a.rows, op.cols, rb, xs, w, kWaves);
        if ((lane & 15) == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) part[w][4 * (lane >> 4) + r] = acc[r];
        }
        __syncthreads();
        if (tid < 16) {
          float v = part[0][tid];
#pragma unroll
          for (int i = 1; i < kWaves; ++i) v += part[i][tid];
          if (rb + tid < a.rows) {
            if (rb == (int64_t)cb * kRows)
              first[tid] = v;
            else
              a.out[rb + tid] = static_cast<T>(v);
          }
        }
        __syncthreads();
      }
      if (has0) q_first = static_cast<T>(first[rl]);
    }
  } else {
    if (has0) {
      Acc acc = op.template finish<G, kRowStage>(sg, nz, xf);
      q_first = static_cast<T>(group_sum<G>(acc));
    }
    for (int64_t r = r0 + stride; r < a.rows; r += stride) {
      Acc acc = op.template partial<G>(r, sub, xf);
      acc = group_sum<G>(acc);
      if (sub == 0) a.out[r] = static_cast<T>(acc);
    }
  }
  if (a.rows == 0) return;
  // Elimination inputs of the first row, loaded before the coefficients.
  T bv0[kCoefPerLane];
  bool piv0 = true;
  if (has0) {
    piv0 = a.mask[r0] != 0;
    load_basis_row<G>(a, r0, sub, bv0);
  }
  if (!fetch_coef(a, st, cf)) return;
  double key = 0.0;
  int idx = INT_MAX;
  for (int64_t r = r0; r < a.rows; r += stride) {
    const bool first = r == r0;
    const bool piv = first ? piv0 : a.mask[r] != 0;
    T bv[kCoefPerLane];
    if (first) {
#pragma unroll
      for (int u = 0; u < kCoefPerLane; ++u) bv[u] = bv0[u];
    } else {
      load_basis_row<G>(a, r, sub, bv);
    }
    double e = 0.0;
#pragma unroll
    for (int u = 0; u < kCoefPerLane; ++u) {
      const int j = sub + u * G;
      if (j < nb) e = fma(cf[j], static_cast<double>(bv[u]), e);
    }
    e = group_sum<G>(e);
    if (sub == 0) {
      const double q0 = static_cast<double>(first ? q_first : a.out[r]);
      const T o = piv ? T(0) : static_cast<T>(q0 - e);
      a.out[r] = o;
      const double k2 = piv ? 0.0 : static_cast<double>(o);
      if (better(k2, (int)r, key, idx)) {
        key = k2;
        idx = (int)r;
      }
    }
  }
  if (sub == 0) {
    sk[rl] = key;
    si[rl] = idx;
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 1; i < kRows; ++i)
      if (better(sk[i], si[i], key, idx)) {
        key = sk[i];
        idx = si[i];
      }
    write_part(a.parts_out, cb, key, idx);
  }
}

// Occupancy floor: 5 wavefronts per SIMD for FP32 vectors (1280 resident
// blocks, so the 1024 row groups of a 16384-row side run in one pass), 4 for
// FP64.
template <typename T>
constexpr int half_min_waves() { return sizeof(T) == 4 ? 5 : 4; }

template <typename T, class RowOp, bool kTriLds, int G>
__global__ __launch_bounds__(kThreads, half_min_waves<T>()) void k_half_rows(HalfArgs<T> a, RowOp op) {
  extern __shared__ unsigned char lds[];
  DevState* st = a.job.st;
  if (st->stopped) return;
  if (blockIdx.x == 0)
    lead<T, kTriLds>(a, st, lds);
  else if ((int)blockIdx.x < a.nlead)
    pivot_entries<T, RowOp>(a, op, st, blockIdx.x);
  else
    consume_rows<G, T, RowOp>(a, op, st, blockIdx.x - a.nlead, gridDim.x - a.nlead);
}

// --------------------------------------------------- PSF consumer blocks --
// The tile of the normalised input: each staged entry is u divided by the
// pivot value, then (BF16 mode) rounded to bfloat16.
template <typename T, typename Acc, int PH, int kIn, int R>
__device__ inline void psf_tile_norm(const T* __restrict__ u, const Normaliser<T>& nz, int rows,
                                     int cols, const Acc* __restrict__ Wt, int pw,
                                     int i0, int j0, Acc* tile, Acc (&acc)[R]) {
  const int ch = PH / 2, cw = pw / 2;
  const int TR = psf_th<R>() + PH - 1, TC = kPsfTW + pw - 1;
  for (int e = threadIdx.x; e < TR * TC; e += kThreads) {
    const int tr = e / TC, tc = e - tr * TC;
    const int gi = i0 - ch + tr, gj = j0 - cw + tc;
    Acc v = 0;
    if (gi >= 0 && gi < rows && gj >= 0 && gj < cols)
      v = static_cast<Acc>(in_val<kIn>(nz(u[(int64_t)gi * cols + gj])));
    tile[e] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int r0 = (threadIdx.x / kWave) * R;
#pragma unroll
  for (int p = 0; p < R; ++p) acc[p] = 0;
  for (int b = 0; b < pw; ++b) {
    Acc s[R + PH - 1];
#pragma unroll
    for (int q = 0; q < R + PH - 1; ++q) s[q] = tile[(r0 + q) * TC + lane + b];
#pragma unroll
    for (int aa = 0; aa < PH; ++aa) {
      const Acc wv = Wt[aa * pw + b];
#pragma unroll
      for (int p = 0; p < R; ++p) acc[p] = fma(wv, s[p + aa], acc[p]);
    }
  }
  __syncthreads();  // the tile may be restaged next
}

// Persistent over tiles cb, cb + ncons, ...: products first (parked in out),
// then the coefficients, then the elimination.  In the 16- and 8-bit modes
// the products run on the matrix cores (psf_tile_mfma; mb: the operand
// blocks), in 16-row blocks, with lanes mapped to outputs as the instruction
// lays them out.
template <typename T, typename Acc, int PH, int kIn, int R>
__device__ void consume_tiles(const HalfArgs<T>& a, const Acc* __restrict__ Wt,
                              const uint64_t* __restrict__ mb, int rows, int cols, int pw,
                              DevState* st, int cb, int ncons, unsigned char* lds) {
  __shared__ double cf[kMaxIter];
  constexpr bool kMfma = psf_on_mfma<kIn>();
  Acc* tile = reinterpret_cast<Acc*>(lds);
  const int lane = threadIdx.x & (kWave - 1);
  constexpr int TH = psf_th<R>();
  const int r0 = (threadIdx.x / kWave) * R;
  const int tiles_x = (cols + kPsfTW - 1) / kPsfTW;
  const int ntiles = a.rows > 0 ? tiles_x * ((rows + TH - 1) / TH) : 0;
  const int nb = a.nb;
  constexpr int kRB = kMfma ? TH / 16 : 1;
  MfmaTileIn<PH, kRB> first_in;  // the first tile's raw inputs (matrix-core modes)
  if constexpr (kMfma) {
    // the operand blocks and the first tile's unnormalised inputs do not
    // depend on the pivot
    if (ntiles > 0) psf_mfma_stage_b<kIn, PH>(mb, reinterpret_cast<uint64_t*>(lds));
    if (cb < ntiles)
      psf_tile_mfma_load<PH, kRB>(a.up, rows, cols, (cb / tiles_x) * TH, (cb % tiles_x) * kPsfTW,
                                  first_in);
  }
  NormStage<T> ns;
  normalise_stage(a, cb, ncons, ns);
  int pick;
  double val;
  if (!wait_pivot(a, st, pick, val)) return;
  const Normaliser<T> nz(static_cast<T>(val));
  normalise_share(a, cb, ncons, pick, nz, ns);
  for (int t = cb; t < ntiles; t += ncons) {
    const int i0 = (t / tiles_x) * TH, j0 = (t % tiles_x) * kPsfTW;
    if constexpr (kMfma) {
      static_assert(TH % 16 == 0, "matrix-core tiles are 16-row blocks");
      constexpr int RB = TH / 16;
      mfma_f4 acc[RB];
      const auto cvt = [nz](float v) { return static_cast<float>(in_val<kIn>(nz(v))); };
      const uint64_t* bl = reinterpret_cast<const uint64_t*>(lds);
      unsigned char* tl = lds + sizeof(uint64_t) * psf_mfma_b_words<kIn, PH>();
      if (t == cb)  // block-uniform
        psf_tile_mfma_from<kIn, PH, RB>(first_in, cvt, bl, tl, acc);
      else
        psf_tile_mfma<kIn, PH, RB>(a.up, cvt, rows, cols, i0, j0, bl, tl, acc);
      const int w = threadIdx.x / kWave;
      const int gj = j0 + 16 * w + (lane & 15);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = i0 + 16 * rb + 4 * (lane >> 4) + r;
          if (gi < rows && gj < cols) a.out[(int64_t)gi * cols + gj] = static_cast<T>(acc[rb][r]);
        }
    } else {
      Acc acc[R];
      psf_tile_norm<T, Acc, PH, kIn, R>(a.up, nz, rows, cols, Wt, pw, i0, j0, tile, acc);
      const int gj = j0 + lane;
#pragma unroll
      for (int p = 0; p < R; ++p) {
        const int gi = i0 + r0 + p;
        if (gi < rows && gj < cols) a.out[(int64_t)gi * cols + gj] = static_cast<T>(acc[p]);
      }
    }
  }
  if (a.rows == 0) return;
  // The coefficients arrive in 64-slot chunks (the lead publishes each as
  // its triangular solve finishes it): the first tile's elimination starts
  // on the first chunk and waits for a later one only where it reaches it.
  int avail = 0;
  if (nb > 0 && !fetch_coef_prefix(a, st, cf, min(nb, kWave), avail)) return;
  double best = 0.0;
  int bidx = INT_MAX;
  {
    // An even row length and column stride: the elimination takes pixel
    // pairs (8- or 16-byte loads, half the load instructions), lane l
    // on columns j0 + 2 (l % 32) + {0, 1} of the rows r0 + 2p + l / 32 of
    // its wavefront; the same pixels per wavefront and the same sums per
    // pixel as the one-column mapping below.
    if ((cols & 1) == 0 && (a.cs & 1) == 0 &&
        (reinterpret_cast<uintptr_t>(a.basis) & (2 * sizeof(T) - 1)) == 0) {
      using T2 = std::conditional_t<std::is_same_v<T, float>, float2, double2>;
      __syncthreads();  // products of this block's tiles, written by other lanes
      constexpr int RP = R / 2;
      const int cp = lane & 31, hr = lane >> 5;
      for (int t = cb; t < ntiles; t += ncons) {
        const int i0 = (t / tiles_x) * TH, j0 = (t % tiles_x) * kPsfTW;
        const int gj = j0 + 2 * cp;
        int64_t pix[RP];
        bool ok[RP];
        unsigned char m0[RP], m1[RP];
#pragma unroll
        for (int p = 0; p < RP; ++p) {
          const int gi = i0 + r0 + 2 * p + hr;
          ok[p] = gi < rows && gj < cols;  // then gj + 1 < cols too (cols even)
          pix[p] = ok[p] ? (int64_t)gi * cols + gj : 0;  // even, in bounds either way
          m0[p] = a.mask[pix[p]];
          m1[p] = a.mask[pix[p] + 1];
        }
        double e0[RP], e1[RP];
#pragma unroll
        for (int p = 0; p < RP; ++p) e0[p] = e1[p] = 0.0;
        // U basis vectors per step, all their loads issued first (enough
        // loads in flight per lane to keep HBM busy); each pixel still sums
        // the vectors in increasing j
        constexpr int U = sizeof(T) == 4 ? 4 : 2;
        // Columns in chunks of 64 (ce: the chunk's end), each waited for
        // only if not yet staged; U divides 64, so j reaches every chunk end
        // but the last.
        int j = 0;
        for (int ce = min(nb, kWave);; ce = min(nb, ce + kWave)) {
          if (ce > avail && !fetch_coef_prefix(a, st, cf, ce, avail)) return;
          for (; j + U <= ce; j += U) {
            T2 bq[U][RP];
#pragma unroll
            for (int uu = 0; uu < U; ++uu) {
              const T* c0 = a.basis + (int64_t)(j + uu) * a.cs;
#pragma unroll
              for (int p = 0; p < RP; ++p) bq[uu][p] = *reinterpret_cast<const T2*>(c0 + pix[p]);
            }
#pragma unroll
            for (int uu = 0; uu < U; ++uu) {
              const double w = cf[j + uu];
#pragma unroll
              for (int p = 0; p < RP; ++p) {
                e0[p] = fma(w, static_cast<double>(bq[uu][p].x), e0[p]);
                e1[p] = fma(w, static_cast<double>(bq[uu][p].y), e1[p]);
              }
            }
          }
          if (ce == nb) break;
        }
        for (; j < nb; ++j) {  // the last chunk's remainder, already staged
          const T* c0 = a.basis + (int64_t)j * a.cs;
          T2 bq[RP];
#pragma unroll
          for (int p = 0; p < RP; ++p) bq[p] = *reinterpret_cast<const T2*>(c0 + pix[p]);
          const double w0 = cf[j];
#pragma unroll
          for (int p = 0; p < RP; ++p) {
            e0[p] = fma(w0, static_cast<double>(bq[p].x), e0[p]);
            e1[p] = fma(w0, static_cast<double>(bq[p].y), e1[p]);
          }
        }
#pragma unroll
        for (int p = 0; p < RP; ++p) {
          if (!ok[p]) continue;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int64_t q = pix[p] + h;
            const bool mk = (h ? m1[p] : m0[p]) != 0;
            const double q0 = static_cast<double>(a.out[q]);
            const T o = mk ? T(0) : static_cast<T>(q0 - (h ? e1[p] : e0[p]));
            a.out[q] = o;
            const double k2 = mk ? 0.0 : static_cast<double>(o);
            if (better(k2, (int)q, best, bidx)) {
              best = k2;
              bidx = (int)q;
            }
          }
        }
      }
      block_argmax<kThreads>(best, bidx);
      if (threadIdx.x == 0) write_part(a.parts_out, cb, best, bidx);
      return;
    }
  }
  if constexpr (kMfma) __syncthreads();  // products written by other lanes
  for (int t = cb; t < ntiles; t += ncons) {
    const int i0 = (t / tiles_x) * TH, j0 = (t % tiles_x) * kPsfTW;
    const int gj = j0 + lane;
    int64_t pix[R];
    bool ok[R];
    unsigned char mk[R];
#pragma unroll
    for (int p = 0; p < R; ++p) {
      const int gi = i0 + r0 + p;
      ok[p] = gi < rows && gj < cols;
      pix[p] = ok[p] ? (int64_t)gi * cols + gj : 0;  // in bounds either way
      mk[p] = a.mask[pix[p]];
    }
    double e[R];
#pragma unroll
    for (int p = 0; p < R; ++p) e[p] = 0.0;
    int j = 0;
    for (int ce = min(nb, kWave);; ce = min(nb, ce + kWave)) {  // as above
      if (ce > avail && !fetch_coef_prefix(a, st, cf, ce, avail)) return;
      for (; j + 2 <= ce; j += 2) {
        const T* c0 = a.basis + (int64_t)j * a.cs;
        const T* c1 = c0 + a.cs;
        T b0[R], b1[R];
#pragma unroll
        for (int p = 0; p < R; ++p) {
          b0[p] = c0[pix[p]];
          b1[p] = c1[pix[p]];
        }
        const double w0 = cf[j], w1 = cf[j + 1];
#pragma unroll
        for (int p = 0; p < R; ++p) {
          e[p] = fma(w0, static_cast<double>(b0[p]), e[p]);
          e[p] = fma(w1, static_cast<double>(b1[p]), e[p]);
        }
      }
      if (ce == nb) break;
    }
    if (j < nb) {  // the last chunk's remainder, already staged
      const T* c0 = a.basis + (int64_t)j * a.cs;
      const double w0 = cf[j];
#pragma unroll
      for (int p = 0; p < R; ++p) e[p] = fma(w0, static_cast<double>(c0[pix[p]]), e[p]);
    }
#pragma unroll
    for (int p = 0; p < R; ++p) {
      if (!ok[p]) continue;
      const double q0 = static_cast<double>(a.out[pix[p]]);
      const T o = mk[p] ? T(0) : static_cast<T>(q0 - e[p]);
      a.out[pix[p]] = o;
      const double k2 = mk[p] ? 0.0 : static_cast<double>(o);
      if (better(k2, (int)pix[p], best, bidx)) {
        best = k2;
        bidx = (int)pix[p];
      }
    }
  }
  block_argmax<kThreads>(best, bidx);
  if (threadIdx.x == 0) write_part(a.parts_out, cb, best, bidx);
}

// Occupancy floor: 3 wavefronts per SIMD, so the 512 tiles of a 1024 x 1024
// image fit beside the leading blocks and each consumer takes one tile.
template <typename T, typename Acc, int PH, int kIn, bool kTriLds, int R>
__global__ __launch_bounds__(kThreads, 3) void k_half_psf(
    HalfArgs<T> a, PsfPixels<Acc, kIn> op, const Acc* __restrict__ Wt) {
  extern __shared__ unsigned char lds[];
  DevState* st = a.job.st;
  if (st->stopped) return;
  if (blockIdx.x == 0)
    lead<T, kTriLds>(a, st, lds);
  else if ((int)blockIdx.x < a.nlead)
    pivot_entries<T, PsfPixels<Acc, kIn>>(a, op, st, blockIdx.x);
  else
    consume_tiles<T, Acc, PH, kIn, R>(a, Wt, op.mb, op.rows, op.cols, op.pw, st,
                                     blockIdx.x - a.nlead, gridDim.x - a.nlead, lds);
}

static_assert(kPsfWaves * kWave == kThreads, "PSF tiles use the launch's block size");

// ------------------------------------------------ several solves at once --
// One launch of the same half-iteration of P solves: solve p owns blocks
// first[p] .. first[p+1]-1 and runs exactly the roles of its own launch
// (lead, pivot entries, consumers) on its own workspace, so every wait is
// within one solve: its entry blocks and consumers wait for its lead, and
// its lead (after publishing the pivot) for its entry blocks, which are
// dispatched right after it and before its consumers.  Solve p's blocks
// never wait for a later solve's, so solve 0 completes whatever follows it,
// then solve 1, and so on: the merged launch needs no more residency than
// the single ones.
__device__ inline int batch_solve_of_block(const int* __restrict__ first, int P) {
  int lo = 0, hi = P - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, class RowOp, bool kTriLds, int G>
__global__ __launch_bounds__(kThreads, half_min_waves<T>()) void k_half_rows_batch(
    const HalfArgs<T>* __restrict__ args, const RowOp* __restrict__ ops,
    const int* __restrict__ first, int P) {
  extern __shared__ unsigned char lds[];
  // p is the same in every lane: loaded by value from a wave-uniform
  // address, the arguments can live in scalar registers as a kernel
  // argument would
  const int p = __builtin_amdgcn_readfirstlane(batch_solve_of_block(first, P));
  const HalfArgs<T> a = args[p];
  const RowOp op = ops[p];
  DevState* st = a.job.st;
  if (st->stopped) return;
  const int bid = (int)blockIdx.x - first[p], nblk = first[p + 1] - first[p];
  if (bid == 0)
    lead<T, kTriLds>(a, st, lds);
  else if (bid < a.nlead)
    pivot_entries<T, RowOp>(a, op, st, bid);
  else
    consume_rows<G, T, RowOp>(a, op, st, bid - a.nlead, nblk - a.nlead);
}


// ------------------------------------------------------------- launchers --
template <typename T>
size_t tri_bytes(int nb) {
  return nb > 1 ? sizeof(T) * (size_t)packed_row(nb) : 0;
}

// Blocks of `kernel` that fit on the device at once (cached per kernel, LDS
// size and device); 0 if the runtime cannot tell.
int resident_blocks(const void* kernel, size_t dyn_lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, size_t, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_tuple(kernel, dyn_lds, dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, dyn_lds) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  cache[key] = per_cu * cus;
  return per_cu * cus;
}

// Consumer blocks: enough for the work, at most kMaxParts, and (persistent)
// no more than fit beside the leading blocks.
int consumer_blocks(int64_t want, int nlead, int resident) {
  int64_t c = std::min<int64_t>(std::max<int64_t>(want, 1), kMaxParts);
  if (resident > nlead) c = std::min<int64_t>(c, resident - nlead);
  return static_cast<int>(c);
}

// Batched launches (launch_half_batch) pass the merged launch instead of s.
template <typename T, class RowOp>
struct RowsBatch {
  const HalfArgs<T>* args;
  const RowOp* ops;
  const int* first;
  int P, blocks;
};

template <typename T, class RowOp, int G>
int launch_rows_g(HalfArgs<T>& a, const RowOp& op, size_t tb, bool in_lds, hipStream_t s,
                  bool dry = false, const RowsBatch<T, RowOp>* batch = nullptr) {
  constexpr int kRows = kThreads / G;
  const int64_t want = a.rows > 0 ? (a.rows + kRows - 1) / kRows
                                  : (a.lenp + kThreads * kNormBatch - 1) / (kThreads * kNormBatch);
  auto k = in_lds ? k_half_rows<T, RowOp, true, G> : k_half_rows<T, RowOp, false, G>;
  const size_t dyn = in_lds ? tb : 0;
  const int ncons = consumer_blocks(want, a.nlead, resident_blocks((const void*)k, dyn));
  if (batch) {
    auto kb = in_lds ? k_half_rows_batch<T, RowOp, true, G> : k_half_rows_batch<T, RowOp, false, G>;
    kb<<<batch->blocks, kThreads, dyn, s>>>(batch->args, batch->ops, batch->first, batch->P);
  } else if (!dry) {
    k<<<a.nlead + ncons, kThreads, dyn, s>>>(a, op);
  }
  return ncons;
}

// 16 lanes per row.  (8 lanes per row, which makes the d side of the
// tomography one pass over the rows, measured slower: the longer per-lane
// chains of dependent loads cost more than the second pass.)
template <typename T, class RowOp>
int launch_rows(HalfArgs<T>& a, const RowOp& op, size_t lds_bytes, hipStream_t s,
                bool dry = false, const RowsBatch<T, RowOp>* batch = nullptr) {
  const int nbk = a.rows > 0 ? a.nb : 0;
  a.nlead = 1 + (nbk + kWaves - 1) / kWaves;
  const size_t tb = tri_bytes<T>(nbk);
  const bool in_lds = tb > 0 && tb <= kTriLdsMax && tb + 16 * 1024 <= lds_bytes;
  return launch_rows_g<T, RowOp, 16>(a, op, tb, in_lds, s, dry, batch);
}

template <typename T, typename Acc, int PH, int kIn, int R>
int launch_tiles_r(HalfArgs<T>& a, const PsfPixels<Acc, kIn>& op, const Acc* Wt,
                   size_t lds_bytes, hipStream_t s, bool dry = false) {
  const int ntiles = ((op.cols + kPsfTW - 1) / kPsfTW) * ((op.rows + psf_th<R>() - 1) / psf_th<R>());
  const int64_t want = a.rows > 0 ? ntiles
                                  : (a.lenp + kThreads * kNormBatch - 1) / (kThreads * kNormBatch);
  const int nbk = a.rows > 0 ? a.nb : 0;
  a.nlead = 1 + (nbk + kWaves - 1) / kWaves;
  const size_t tb = tri_bytes<T>(nbk);
  const size_t pb = psf_lds_bytes<Acc, PH, kIn, R>(op.pw);
  // float bases: a 48 KB triangle (k up to about 155) stays in LDS; its
  // size is then no larger than the other LDS users of the PSF launch
  constexpr size_t tri_max = sizeof(T) == 4 ? 48 * 1024 : kTriLdsMax;
  const bool in_lds = tb > 0 && tb <= tri_max && std::max(tb, pb) + 16 * 1024 <= lds_bytes;
  if (in_lds) {
    auto k = k_half_psf<T, Acc, PH, kIn, true, R>;
    const size_t dyn = std::max(tb, pb);
    const int ncons = consumer_blocks(want, a.nlead, resident_blocks((const void*)k, dyn));
    if (!dry) k<<<a.nlead + ncons, kThreads, dyn, s>>>(a, op, Wt);
    return ncons;
  }
  auto k = k_half_psf<T, Acc, PH, kIn, false, R>;
  const int ncons = consumer_blocks(want, a.nlead, resident_blocks((const void*)k, pb));
  if (!dry) k<<<a.nlead + ncons, kThreads, pb, s>>>(a, op, Wt);
  return ncons;
}

template <typename T, typename Acc, int PH, int kIn>
int launch_tiles(HalfArgs<T>& a, const PsfPixels<Acc, kIn>& op, const Acc* Wt, int psf_r,
                 size_t lds_bytes, hipStream_t s, bool dry = false) {
  int n = 0;
  with_psf_r(psf_r, op.rows, op.cols, [&](auto rc) {
    constexpr int R = psf_rows_used<kIn, decltype(rc)::value>();
    n = launch_tiles_r<T, Acc, PH, kIn, R>(a, op, Wt, lds_bytes, s, dry);
  });
  return n;
}

// The row access of an operator for one direction (tr: A^T), and its
// value / sum types, passed to f(row_op).
template <typename T, typename F>
void with_row_op(const DeviceOp& op, int tr, F&& f) {
  with_mode<T>(op.prec, [&](auto v, auto acc, auto bf) {
    using V = decltype(v);
    using Acc = decltype(acc);
    constexpr int kB = decltype(bf)::value;
    if (op.kind == 0) {
      f(DenseRows<V, Acc, kB>{static_cast<const V*>(tr ? op.AT : op.A), tr ? op.m : op.n});
    } else if (op.kind == 1) {
      const int* rp = tr ? op.rpT : op.rp;
      const void* ci = tr ? op.ciT : op.ci;
      const V* val = static_cast<const V*>(tr ? op.valT : op.val);
      if (op.idx16 & (tr ? 2 : 1))
        f(CsrRows<V, Acc, kB, uint16_t>{rp, static_cast<const uint16_t*>(ci), val});
      else
        f(CsrRows<V, Acc, kB, int>{rp, static_cast<const int*>(ci), val});
    } else {
      const Acc* wt;
      if constexpr (std::is_same_v<Acc, double>)
        wt = tr ? op.psf : op.psf_flip;
      else
        wt = tr ? op.psf32 : op.psf32_flip;
      f(PsfPixels<Acc, kB>{wt, static_cast<int>(op.rows), static_cast<int>(op.cols), op.ph,
                           op.pw, tr ? op.mb : op.mb_flip});
    }
  });
}

// The PSF half-iteration launch of one precision mode (Acc sums, kB input
// rounding), for the PH and tile shape of the operator; dry: plan only.
template <typename T, typename Acc, int kB>
int launch_psf_mode(HalfArgs<T>& a, const DeviceOp& op, int tr, size_t lds_bytes, hipStream_t s,
                    bool dry) {
  int n = 0;
  with_row_op<T>(op, tr, [&](auto ro) {
    using RO = decltype(ro);
    if constexpr (is_psf_pixels<RO>::value) {
      if constexpr (std::is_same_v<typename RO::Acc, Acc> && RO::kInMode == kB) {
        with_ph(op.ph, [&](auto phc) {
          constexpr int PH = decltype(phc)::value;
          n = launch_tiles<T, Acc, PH, kB>(a, ro, ro.wt, op.psf_r, lds_bytes, s, dry);
        });
      }
    }
  });
  return n;
}

}  // namespace

// PSF half-iteration launches, one translation unit per precision mode
// (recurrence_psf_<mode>.hip), so that their many kernel instantiations
// (PSF height x tile shape x triangle placement) compile in parallel.
// Return the consumer count; dry: plan only (sets a.nlead).
int launch_psf_half_fp64(HalfArgs<double>& a, const DeviceOp& op, int tr, size_t lds_bytes,
                         hipStream_t s, bool dry);
int launch_psf_half_fp32(HalfArgs<float>& a, const DeviceOp& op, int tr, size_t lds_bytes,
                         hipStream_t s, bool dry);
int launch_psf_half_bf16(HalfArgs<float>& a, const DeviceOp& op, int tr, size_t lds_bytes,
                         hipStream_t s, bool dry);
int launch_psf_half_fp16(HalfArgs<float>& a, const DeviceOp& op, int tr, size_t lds_bytes,
                         hipStream_t s, bool dry);
int launch_psf_half_fp8(HalfArgs<float>& a, const DeviceOp& op, int tr, size_t lds_bytes,
                        hipStream_t s, bool dry);

}  // namespace lslu
