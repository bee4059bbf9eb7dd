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
//   2. k_eliminate_argmax: one streaming pass q = q0 - sum_j w_j l_j (again in
//      increasing j), q = 0 at earlier pivots, and the search for the largest
//      |q| over the remaining rows (smallest row index among equal values).
//      The last block to finish picks the pivot and detects breakdown.
//   3. k_normalize: l_k = q / W(k,k) by IEEE division (exactly 1 at the pivot)
//      and the new row of T_L, (l_1..l_{k-1})(g(k)), gathered from the basis.
//
// Floating-point contraction is disabled in the arithmetic that mirrors the
// sequential elimination so each step rounds like a multiply then subtract.
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

// Block-wide argmax; the result is valid in thread 0.
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
  if (threadIdx.x == 0) {
    for (int i = 1; i < BLOCK / kWave; ++i)
      if (better(sk[i], si[i], key, idx)) {
        key = sk[i];
        idx = si[i];
      }
  }
  __syncthreads();
}

template <typename T>
__device__ void finalize_pivot(const PivotJob& job, double key, int idx,
                               const T* out) {
  DevState* st = job.st;
  st->ticket[job.side] = 0u;  // ready for the next search on this side
  const int own = (job.eligible && key > 0.0) ? idx : -1;
  int pick = own;
  if (job.replay) {
    pick = job.eligible ? job.replay[job.piv_pos] : -1;
    if (pick != own) {
      if (job.side == 0) st->mismatch_g += 1; else st->mismatch_t += 1;
    }
  }
  if (job.own_list) job.own_list[job.piv_pos] = own;
  const double val = (pick >= 0) ? static_cast<double>(out[pick]) : 0.0;
  if (pick < 0 || val == 0.0) {
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
    return;
  }
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

template <typename T>
__global__ __launch_bounds__(kArgmaxBlock) void k_eliminate_argmax(
    const T* v0, T* out, const T* __restrict__ basis, int64_t ld,
    int nb, const double* __restrict__ coef,
    const unsigned char* __restrict__ mask, int64_t len,
    ArgPart* __restrict__ parts, PivotJob job) {
#pragma clang fp contract(off)
  if (job.st->stopped) return;
  double best = -1.0;
  int bidx = INT_MAX;
  const int64_t stride = (int64_t)gridDim.x * kArgmaxBlock;
  for (int64_t r = blockIdx.x * (int64_t)kArgmaxBlock + threadIdx.x; r < len;
       r += stride) {
    double acc = static_cast<double>(v0[r]);
    int j = 0;
    for (; j + kUnroll <= nb; j += kUnroll) {
      T bv[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) bv[u] = basis[(int64_t)(j + u) * ld + r];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        acc = acc - coef[j + u] * static_cast<double>(bv[u]);
    }
    for (; j < nb; ++j)
      acc = acc - coef[j] * static_cast<double>(basis[(int64_t)j * ld + r]);
    const bool piv = mask[r] != 0;
    const T o = piv ? T(0) : static_cast<T>(acc);
    out[r] = o;
    const double key = piv ? -1.0 : fabs(static_cast<double>(o));
    if (better(key, (int)r, best, bidx)) {
      best = key;
      bidx = (int)r;
    }
  }
  block_argmax<kArgmaxBlock>(best, bidx);
  __shared__ bool am_last;
  if (threadIdx.x == 0) {
    parts[blockIdx.x].key = best;
    parts[blockIdx.x].idx = bidx;
    __threadfence();
    const unsigned t = atomicAdd(&job.st->ticket[job.side], 1u);
    am_last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  best = -1.0;
  bidx = INT_MAX;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += kArgmaxBlock) {
    const double k2 = parts[i].key;
    const int i2 = parts[i].idx;
    if (better(k2, i2, best, bidx)) {
      best = k2;
      bidx = i2;
    }
  }
  block_argmax<kArgmaxBlock>(best, bidx);
  if (threadIdx.x == 0) finalize_pivot<T>(job, best, bidx, out);
}

template <typename T>
__global__ void k_normalize(const T* __restrict__ v, T* __restrict__ dst,
                           int64_t len, PivotJob job, double* Trow, int ldT,
                           const T* __restrict__ basis, int64_t ld, int nb) {
  if (job.st->stopped) return;
  const double pv = *job.piv_val;
  const int pr = job.piv_list[job.piv_pos];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < len;
       r += (int64_t)gridDim.x * blockDim.x)
    dst[r] = (r == pr) ? T(1) : static_cast<T>(static_cast<double>(v[r]) / pv);
  if (blockIdx.x == 0 && Trow != nullptr) {
    for (int j = threadIdx.x; j < nb; j += blockDim.x)
      Trow[(int64_t)j * ldT] = static_cast<double>(basis[(int64_t)j * ld + pr]);
    if (threadIdx.x == 0) Trow[(int64_t)nb * ldT] = 1.0;
  }
}

// One wavefront: lane l owns rows l, l+64, l+128, l+192 of the triangle.
template <typename T>
__global__ __launch_bounds__(kWave) void k_gather_trisolve(
    const T* __restrict__ v0, const int* __restrict__ piv, int nb,
    const double* __restrict__ Tm, int ldT, double* __restrict__ coef,
    const DevState* st) {
#pragma clang fp contract(off)
  if (st->stopped) return;
  const int lane = threadIdx.x;
  double g[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int j = lane + s * kWave;
    g[s] = (j < nb) ? static_cast<double>(v0[piv[j]]) : 0.0;
  }
  for (int i = 0; i < nb; ++i) {
    const int si = i >> 6;  // uniform
    double gi = g[0];
    if (si == 1) gi = g[1];
    if (si == 2) gi = g[2];
    if (si == 3) gi = g[3];
    const double wi = readlane_d(gi, i & (kWave - 1));
    const double* col = Tm + (int64_t)i * ldT;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int j = lane + s * kWave;
      if (j > i && j < nb) g[s] = g[s] - col[j] * wi;
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int j = lane + s * kWave;
    if (j < nb) coef[j] = g[s];
  }
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

template <typename T>
void launch_eliminate_argmax(const T* v0, T* out, const T* basis, int64_t ld,
                             int nb, const double* coef,
                             const unsigned char* mask, int64_t len,
                             ArgPart* parts, const PivotJob& job,
                             hipStream_t s) {
  const int grid = grid_for(len, kArgmaxBlock, kMaxArgmaxBlocks);
  k_eliminate_argmax<T><<<grid, kArgmaxBlock, 0, s>>>(
      v0, out, basis, ld, nb, coef, mask, len, parts, job);
}

template <typename T>
void launch_normalize(const T* v, T* dst, int64_t len, const PivotJob& job,
                      double* Trow, int ldT, const T* basis, int64_t ld, int nb,
                      hipStream_t s) {
  k_normalize<T><<<grid_for(len, 256, 4096), 256, 0, s>>>(
      v, dst, len, job, Trow, ldT, basis, ld, nb);
}

template <typename T>
void launch_gather_trisolve(const T* v0, const int* piv, int nb,
                            const double* Tm, int ldT, double* coef,
                            const DevState* st, hipStream_t s) {
  if (nb <= 0) return;
  k_gather_trisolve<T><<<1, kWave, 0, s>>>(v0, piv, nb, Tm, ldT, coef, st);
}

#define LSLU_INST(T)                                                         \
  template void launch_fill<T>(T*, T, int64_t, hipStream_t);                 \
  template void launch_sub<T>(const T*, const T*, T*, int64_t, hipStream_t); \
  template void launch_eliminate_argmax<T>(                                  \
      const T*, T*, const T*, int64_t, int, const double*,                   \
      const unsigned char*, int64_t, ArgPart*, const PivotJob&, hipStream_t); \
  template void launch_normalize<T>(const T*, T*, int64_t, const PivotJob&,  \
                                    double*, int, const T*, int64_t, int,    \
                                    hipStream_t);                            \
  template void launch_gather_trisolve<T>(const T*, const int*, int,         \
                                          const double*, int, double*,       \
                                          const DevState*, hipStream_t);
LSLU_INST(double)
LSLU_INST(float)
template void launch_fill<unsigned char>(unsigned char*, unsigned char, int64_t,
                                         hipStream_t);
template void launch_fill<int>(int*, int, int64_t, hipStream_t);
#undef LSLU_INST

}  // namespace lslu
