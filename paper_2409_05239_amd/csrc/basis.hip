// Basis recurrence of the pivoted rectangular Hessenberg process
// (Algorithm 4; the basis part of Algorithm 5).
//
// One half-iteration (the l side at iteration k; the d side is the same with
// u = A l_k, D and the row pivots t) is, after the operator product
// q0 = A^T d_k:
//
//   1. k_gather_trisolve: read q0 at the earlier pivots g(1..k-1) and solve the
//      unit lower triangular system T_L w = q0(g) with T_L(j,i) = l_i(g(j)).
//      This gives W(1:k-1,k) exactly as the sequential loop of Algorithm 5
//      does (l_i is 1 at g(i) and 0 at g(j), j < i), with the same operation
//      order: row j receives its subtractions in increasing i.
//   2. k_eliminate_argmax: one streaming pass q = q0 - sum_j w_j l_j (the sum
//      split over the four wavefronts of a block and added in a fixed order),
//      q = 0 at earlier pivots, and per block the largest |q| over the
//      remaining rows (smallest row index among equal values).
//   3. k_pivot_normalize: every block reduces the per-block candidates to the
//      pivot (the kernel boundary makes them visible, so no device-wide fence
//      or atomic is needed), detects breakdown, and writes l_k = q / W(k,k) by
//      IEEE division (exactly 1 at the pivot); block 0 records the pivot and
//      appends the new row of T_L, (l_1..l_{k-1})(g(k)), to its packed copy.
//
// Floating-point contraction is disabled in the arithmetic that mirrors the
// sequential elimination so each step rounds like a multiply then subtract;
// results are independent of timing and of the launch configuration.
#include <climits>

#include "internal.hpp"

namespace lslu {

namespace {

__device__ inline double readlane_d(double v, int lane) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  uint32_t lo = static_cast<uint32_t>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(u)), lane));
  uint32_t hi = static_cast<uint32_t>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(u >> 32)), lane));
  return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Total order used by every pivot search: larger key first, then smaller row.
__device__ inline bool better(double ka, int ia, double kb, int ib) {
  return ka > kb || (ka == kb && ia < ib);
}

__device__ inline void wave_argmax(double& key, int& idx) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    double ok = __shfl_xor(key, off);
    int oi = __shfl_xor(idx, off);
    if (better(ok, oi, key, idx)) {
      key = ok;
      idx = oi;
    }
  }
}

// Block-wide argmax; the result is returned to every thread.
template <int BLOCK>
__device__ inline void block_argmax(double& key, int& idx) {
  __shared__ double sk[BLOCK / kWave];
  __shared__ int si[BLOCK / kWave];
  wave_argmax(key, idx);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sk[w] = key;
    si[w] = idx;
  }
  __syncthreads();
  key = sk[0];
  idx = si[0];
  for (int i = 1; i < BLOCK / kWave; ++i)
    if (better(sk[i], si[i], key, idx)) {
      key = sk[i];
      idx = si[i];
    }
  __syncthreads();
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_state_reset(DevState* st) {
  if (threadIdx.x == 0) {
    DevState z{};
    *st = z;
  }
}

template <typename T>
__global__ void k_sub(const T* __restrict__ a, const T* __restrict__ b,
                      T* __restrict__ out, int64_t len) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = static_cast<T>(static_cast<double>(a[i]) - static_cast<double>(b[i]));
}

constexpr int kUnroll = 8;
constexpr int kTile = kWave;  // rows per tile; the 4 wavefronts split the columns
constexpr int kMaxElimBlocks = 1024;
constexpr int kNormBlock = 256;
constexpr int kMaxNormBlocks = 512;

// q = v0 - sum_j coef_j basis_j over 64-row tiles.  Wavefront w of a block sums
// the j in its quarter of 0..nb-1 (in increasing j); the quarters are added in
// a fixed order.  Each block writes its best pivot candidate to parts.
template <typename T>
__global__ __launch_bounds__(kArgmaxBlock) void k_eliminate_argmax(
    const T* v0, T* out, const T* __restrict__ basis, int64_t ld, int nb,
    const double* __restrict__ coef, const unsigned char* __restrict__ mask,
    int64_t len, ArgPart* __restrict__ parts, const DevState* st) {
#pragma clang fp contract(off)
  if (st->stopped) return;
  __shared__ double part[kArgmaxBlock / kWave - 1][kTile];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int chunk = (nb + 3) / 4;
  const int j0 = min(nb, w * chunk), j1 = min(nb, j0 + chunk);
  double best = -1.0;
  int bidx = INT_MAX;
  const int64_t ntiles = (len + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r = tile * kTile + lane;
    double acc = 0.0;
    if (r < len) {
      int j = j0;
      for (; j + kUnroll <= j1; j += kUnroll) {
        T bv[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) bv[u] = basis[(int64_t)(j + u) * ld + r];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          acc = acc + coef[j + u] * static_cast<double>(bv[u]);
      }
      T bt[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        bt[u] = (j + u < j1) ? basis[(int64_t)(j + u) * ld + r] : T(0);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        if (j + u < j1) acc = acc + coef[j + u] * static_cast<double>(bt[u]);
    }
    if (w > 0) part[w - 1][lane] = acc;
    __syncthreads();
    if (w == 0 && r < len) {
      double sum = acc;
#pragma unroll
      for (int i = 0; i < kArgmaxBlock / kWave - 1; ++i) sum = sum + part[i][lane];
      const double val = static_cast<double>(v0[r]) - sum;
      const bool piv = mask[r] != 0;
      const T o = piv ? T(0) : static_cast<T>(val);
      out[r] = o;
      const double key = piv ? -1.0 : fabs(static_cast<double>(o));
      if (better(key, (int)r, best, bidx)) {
        best = key;
        bidx = (int)r;
      }
    }
    __syncthreads();
  }
  block_argmax<kArgmaxBlock>(best, bidx);
  if (threadIdx.x == 0) {
    parts[blockIdx.x].key = best;
    parts[blockIdx.x].idx = bidx;
  }
}

// Pivot choice (every block, identically), breakdown test and normalisation.
template <typename T>
__global__ __launch_bounds__(kNormBlock) void k_pivot_normalize(
    const T* __restrict__ v, T* __restrict__ dst, int64_t len,
    const ArgPart* __restrict__ parts, int nparts, PivotJob job, T* Trow,
    const T* __restrict__ basis, int64_t ld, int nb) {
  DevState* st = job.st;
  if (st->stopped) return;
  double key = -1.0;
  int idx = INT_MAX;
  for (int i = threadIdx.x; i < nparts; i += kNormBlock)
    if (better(parts[i].key, parts[i].idx, key, idx)) {
      key = parts[i].key;
      idx = parts[i].idx;
    }
  block_argmax<kNormBlock>(key, idx);
  const int own = (job.eligible && key > 0.0) ? idx : -1;
  const int pick = job.replay ? (job.eligible ? job.replay[job.piv_pos] : -1) : own;
  const double val = (pick >= 0) ? static_cast<double>(v[pick]) : 0.0;
  const bool brk = (pick < 0 || val == 0.0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
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
  for (int64_t r = blockIdx.x * (int64_t)kNormBlock + threadIdx.x; r < len;
       r += (int64_t)gridDim.x * kNormBlock)
    dst[r] = (r == pick) ? T(1) : static_cast<T>(static_cast<double>(v[r]) / val);
  if (blockIdx.x == 0 && Trow != nullptr) {  // new row of the triangle
    for (int j = threadIdx.x; j < nb; j += kNormBlock)
      Trow[j] = basis[(int64_t)j * ld + pick];
  }
}

// Forward substitution T w = g (T unit lower triangular, T(j,i) = basis_i at
// pivot j, i < j) with g gathered from v0 at the pivots.  T is stored packed
// by rows (row j at offset j(j-1)/2, entries i = 0..j-1; the unit diagonal is
// implicit), so staging it in LDS is one contiguous copy.  The system is then
// solved in 64-row blocks: wavefront 0 keeps its lanes' rows of the diagonal
// block in registers (zero above the diagonal) and runs the dependent chain
// with w_i broadcast by readlane; the workgroup then updates the rows below.
// Every row j receives its subtractions in increasing i, as in the sequential
// elimination.
constexpr int kTriThreads = 256;
constexpr int kStage = 16;  // loads in flight per thread while staging

__device__ inline int64_t packed_row(int j) { return (int64_t)j * (j - 1) / 2; }

template <typename T, bool kInLds>
__global__ __launch_bounds__(kTriThreads) void k_gather_trisolve(
    const T* __restrict__ v0, const int* __restrict__ piv, int nb,
    const T* __restrict__ Tp, double* __restrict__ coef, const DevState* st) {
#pragma clang fp contract(off)
  extern __shared__ unsigned char tri_raw[];
  __shared__ double g[kMaxIter + 1];
  const T* tp = kInLds ? reinterpret_cast<const T*>(tri_raw) : Tp;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  // Gather (indices clamped: after a breakdown the list is incomplete and the
  // result is not used) and stage the triangle, all loads of a batch in
  // flight before the LDS stores.
  const int stopped = st->stopped;
  for (int j = tid; j < nb; j += kTriThreads)
    g[j] = static_cast<double>(v0[max(piv[j], 0)]);
  if constexpr (kInLds) {
    T* lt = reinterpret_cast<T*>(tri_raw);
    const int64_t P = packed_row(nb);
    for (int64_t p0 = 0; p0 < P; p0 += (int64_t)kTriThreads * kStage) {
      T buf[kStage];
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int64_t p = p0 + (int64_t)u * kTriThreads + tid;
        buf[u] = (p < P) ? Tp[p] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int64_t p = p0 + (int64_t)u * kTriThreads + tid;
        if (p < P) lt[p] = buf[u];
      }
    }
  }
  __syncthreads();
  if (stopped) return;
  for (int b0 = 0; b0 < nb; b0 += kWave) {
    const int bs = min(kWave, nb - b0);
    if (w == 0) {
      const int j = b0 + lane;
      const T* row = tp + packed_row(j) + b0;  // T(j, b0 + i) = row[i]
      double tr[kWave];
#pragma unroll
      for (int i = 0; i < kWave; ++i)
        tr[i] = (i < lane && lane < bs) ? static_cast<double>(row[i]) : 0.0;
      double gl = (lane < bs) ? g[j] : 0.0;
#pragma unroll
      for (int i = 0; i < kWave; ++i) {
        const double wi = readlane_d(gl, i);
        gl = gl - tr[i] * wi;  // tr[i] == 0 unless i < lane
      }
      if (lane < bs) g[j] = gl;
    }
    __syncthreads();
    for (int j = b0 + bs + tid; j < nb; j += kTriThreads) {
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
  for (int j = tid; j < nb; j += kTriThreads) coef[j] = g[j];
}

inline int grid_for(int64_t len, int block, int cap) {
  int64_t g = (len + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<int>(g);
}

}  // namespace

template <typename T>
void launch_fill(T* p, T v, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  k_fill<T><<<grid_for(count, 256, 4096), 256, 0, s>>>(p, v, count);
}

void launch_state_reset(DevState* st, hipStream_t s) {
  k_state_reset<<<1, 64, 0, s>>>(st);
}

template <typename T>
void launch_sub(const T* a, const T* b, T* out, int64_t len, hipStream_t s) {
  k_sub<T><<<grid_for(len, 256, 4096), 256, 0, s>>>(a, b, out, len);
}

int elim_blocks(int64_t len) { return grid_for(len, kTile, kMaxElimBlocks); }

template <typename T>
void launch_eliminate_argmax(const T* v0, T* out, const T* basis, int64_t ld,
                             int nb, const double* coef,
                             const unsigned char* mask, int64_t len,
                             ArgPart* parts, const DevState* st,
                             hipStream_t s) {
  k_eliminate_argmax<T><<<elim_blocks(len), kArgmaxBlock, 0, s>>>(
      v0, out, basis, ld, nb, coef, mask, len, parts, st);
}

template <typename T>
void launch_pivot_normalize(const T* v, T* dst, int64_t len,
                            const ArgPart* parts, const PivotJob& job, T* Tpack,
                            const T* basis, int64_t ld, int nb, hipStream_t s) {
  // the pivot row is row nb of the packed triangle
  T* Trow = Tpack ? Tpack + (int64_t)nb * (nb - 1) / 2 : nullptr;
  k_pivot_normalize<T><<<grid_for(len, kNormBlock, kMaxNormBlocks), kNormBlock,
                         0, s>>>(v, dst, len, parts, elim_blocks(len), job,
                                 Trow, basis, ld, nb);
}

template <typename T>
void launch_gather_trisolve(const T* v0, const int* piv, int nb, const T* Tp,
                            double* coef, const DevState* st, size_t lds_bytes,
                            hipStream_t s) {
  if (nb <= 0) return;
  const size_t need = sizeof(T) * (size_t)nb * (nb - 1) / 2;
  if (need + 8 * 1024 <= lds_bytes)
    k_gather_trisolve<T, true><<<1, kTriThreads, need, s>>>(v0, piv, nb, Tp, coef, st);
  else
    k_gather_trisolve<T, false><<<1, kTriThreads, 0, s>>>(v0, piv, nb, Tp, coef, st);
}

void basis_init_attributes(size_t lds_bytes) {
  if (lds_bytes <= 8 * 1024) return;
  const int dyn = static_cast<int>(lds_bytes - 8 * 1024);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_gather_trisolve<double, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_gather_trisolve<float, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

#define LSLU_INST(T)                                                          \
  template void launch_fill<T>(T*, T, int64_t, hipStream_t);                  \
  template void launch_sub<T>(const T*, const T*, T*, int64_t, hipStream_t);  \
  template void launch_eliminate_argmax<T>(                                   \
      const T*, T*, const T*, int64_t, int, const double*,                    \
      const unsigned char*, int64_t, ArgPart*, const DevState*, hipStream_t); \
  template void launch_pivot_normalize<T>(const T*, T*, int64_t,              \
                                          const ArgPart*, const PivotJob&,    \
                                          T*, const T*, int64_t, int,         \
                                          hipStream_t);                       \
  template void launch_gather_trisolve<T>(const T*, const int*, int,          \
                                          const T*, double*, const DevState*, \
                                          size_t, hipStream_t);
LSLU_INST(double)
LSLU_INST(float)
template void launch_fill<unsigned char>(unsigned char*, unsigned char, int64_t,
                                         hipStream_t);
template void launch_fill<int>(int*, int, int64_t, hipStream_t);
#undef LSLU_INST

}  // namespace lslu
