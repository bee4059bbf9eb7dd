// Small helpers of the basis recurrence: fills, the state reset, r_0 = b - A
// x_0, the pivot candidates of r_0 (the first search of Algorithm 4) and the
// copy of basis vectors to a caller's buffer.
#include "device_common.hpp"

namespace lslu {

namespace {

template <typename T>
__global__ void k_fill(T* p, T v, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Also sets the nan_count pivot separations to NaN ("no search made").
__global__ void k_state_reset(DevState* st, double* nan_fill, int nan_count) {
  if (threadIdx.x == 0) {
    DevState z{};
    *st = z;
  }
  for (int i = threadIdx.x; i < nan_count; i += blockDim.x) nan_fill[i] = __builtin_nan("");
}

template <typename T>
__global__ void k_sub(const T* __restrict__ a, const T* __restrict__ b,
                      T* __restrict__ out, int64_t len) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = static_cast<T>(static_cast<double>(a[i]) - static_cast<double>(b[i]));
}

constexpr int kArgBlock = 256;
constexpr int kMaxArgBlocks = 1024;

// Per-block entry of largest |v| (smallest index among equals), as the
// signed value and its index.
template <typename T>
__global__ __launch_bounds__(kArgBlock) void k_argmax_parts(
    const T* __restrict__ v, int64_t len, ArgPart* __restrict__ parts,
    const DevState* st) {
  if (st->stopped) return;
  double best = 0.0;
  int bidx = INT_MAX;
  for (int64_t i = blockIdx.x * (int64_t)kArgBlock + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * kArgBlock) {
    const double key = static_cast<double>(v[i]);
    if (better(key, (int)i, best, bidx)) {
      best = key;
      bidx = (int)i;
    }
  }
  block_argmax<kArgBlock>(best, bidx);
  if (threadIdx.x == 0) {
    parts[blockIdx.x].key = best;
    parts[blockIdx.x].idx = bidx;
  }
}

template <typename T>
__global__ void k_basis_copy(const T* __restrict__ src, int64_t rs, int64_t cs,
                             int64_t len, T* __restrict__ dst) {
  const int j = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[(int64_t)j * len + i] = src[i * rs + (int64_t)j * cs];
}

constexpr int kSepBlock = 256;
constexpr int kSepChunks = 64;  // blocks per searched vector

// Pivot separations (Algorithm 4's infinity-norm search, how far each choice
// is from a tie): search i produced the normalised vector d_1, l_1, d_2, l_2,
// ... (i even: d_{i/2+1} with pivot t(i/2+1); i odd: l_{(i+1)/2} with pivot
// g((i+1)/2)), whose pivot entry is 1, earlier pivots' entries 0 and the
// others the candidates divided by the pivot value.  So a2/a1 is the largest
// |entry| off the pivot row.  For a sampled search the candidates are the
// first sample_s listed rows that are not earlier pivots (one occurrence of
// the pivot row left out), unless the pivot is not among them: then the
// search fell back to the full one.  The maximum goes into mx[i] as the bit
// pattern of a non-negative double (ordered as the doubles).
template <typename T>
__global__ __launch_bounds__(kSepBlock) void k_pivot_sep_max(
    const T* __restrict__ L, int64_t rsL, int64_t csL, int64_t n,
    const T* __restrict__ D, int64_t rsD, int64_t csD, int64_t m,
    const int* __restrict__ piv_t, const int* __restrict__ piv_g,
    const int* __restrict__ samp, int sample_s, const DevState* __restrict__ st,
    unsigned long long* __restrict__ mx) {
  const int i = blockIdx.y;
  const bool lside = (i & 1) != 0;
  const int k = lside ? (i + 1) / 2 : i / 2;
  if (lside ? k > st->n_l : k + 1 > st->n_d) return;  // no such vector
  const T* v = lside ? L + (int64_t)(k - 1) * csL : D + (int64_t)k * csD;
  const int64_t rs = lside ? rsL : rsD, len = lside ? n : m;
  const int p = lside ? piv_g[k - 1] : piv_t[k];
  const int* earlier = lside ? piv_g : piv_t;
  const int nearlier = lside ? k - 1 : k;
  __shared__ int sel[kMaxSampleLen];
  __shared__ unsigned char ok[kMaxSampleLen];
  __shared__ int nsel, psel;
  __shared__ double red[kSepBlock / 64];
  double a = 0.0;
  bool full = true;
  if (samp) {
    const int* row = samp + (int64_t)i * kMaxSampleLen;
    for (int e = threadIdx.x; e < kMaxSampleLen; e += kSepBlock) {
      const int r = row[e];
      bool use = r >= 0;
      for (int q = 0; use && q < nearlier; ++q) use = earlier[q] != r;
      ok[e] = use ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int cnt = 0, pp = -1;
      for (int e = 0; e < kMaxSampleLen && cnt < sample_s; ++e) {
        if (!ok[e]) continue;
        if (row[e] == p && pp < 0) pp = cnt;
        sel[cnt++] = row[e];
      }
      nsel = cnt;
      psel = pp;
    }
    __syncthreads();
    if (psel >= 0) {
      full = false;
      if (blockIdx.x == 0)
        for (int e = threadIdx.x; e < nsel; e += kSepBlock)
          if (e != psel) a = fmax(a, fabs(static_cast<double>(v[(int64_t)sel[e] * rs])));
    }
  }
  if (full)
    for (int64_t j = blockIdx.x * (int64_t)kSepBlock + threadIdx.x; j < len;
         j += (int64_t)gridDim.x * kSepBlock)
      if (j != p) a = fmax(a, fabs(static_cast<double>(v[j * rs])));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kSepBlock / 64; ++w) a = fmax(a, red[w]);
    if (a > 0.0) atomicMax(mx + i, static_cast<unsigned long long>(__double_as_longlong(a)));
  }
}

// sep_t[k] (search 2k) and sep_g[k-1] (search 2k-1) = 1 - mx; NaN where no
// vector was formed.
__global__ void k_pivot_sep_final(const unsigned long long* __restrict__ mx, int K,
                                  const DevState* __restrict__ st, double* __restrict__ sep_t,
                                  double* __restrict__ sep_g) {
  for (int i = threadIdx.x; i < 2 * K + 1; i += blockDim.x) {
    const bool lside = (i & 1) != 0;
    const int k = lside ? (i + 1) / 2 : i / 2;
    const bool formed = lside ? k <= st->n_l : k + 1 <= st->n_d;
    const double s = formed ? 1.0 - __longlong_as_double(static_cast<long long>(mx[i]))
                            : __builtin_nan("");
    if (lside)
      sep_g[k - 1] = s;
    else
      sep_t[k] = s;
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

void launch_state_reset(DevState* st, double* nan_fill, int nan_count, hipStream_t s) {
  k_state_reset<<<1, 256, 0, s>>>(st, nan_fill, nan_count);
}

template <typename T>
void launch_sub(const T* a, const T* b, T* out, int64_t len, hipStream_t s) {
  k_sub<T><<<grid_for(len, 256, 4096), 256, 0, s>>>(a, b, out, len);
}

template <typename T>
int launch_argmax_parts(const T* v, int64_t len, ArgPart* parts,
                        const DevState* st, hipStream_t s) {
  const int g = grid_for(len, kArgBlock, kMaxArgBlocks);
  k_argmax_parts<T><<<g, kArgBlock, 0, s>>>(v, len, parts, st);
  return g;
}

template <typename T>
void launch_basis_copy(const T* src, int64_t rs, int64_t cs, int64_t len,
                       int count, T* dst, hipStream_t s) {
  if (count <= 0 || len <= 0) return;
  dim3 grid(grid_for(len, 256, 1024), count);
  k_basis_copy<T><<<grid, 256, 0, s>>>(src, rs, cs, len, dst);
}

template <typename T>
void launch_pivot_sep(const T* L, int64_t rsL, int64_t csL, int64_t n, const T* D,
                      int64_t rsD, int64_t csD, int64_t m, const int* piv_t,
                      const int* piv_g, const int* samp, int sample_s, int K,
                      const DevState* st, unsigned long long* mx, double* sep_t,
                      double* sep_g, hipStream_t s) {
  launch_fill<uint64_t>(reinterpret_cast<uint64_t*>(mx), 0, 2 * K + 1, s);
  const int64_t len = n > m ? n : m;
  dim3 grid(grid_for(len, kSepBlock, kSepChunks), 2 * K + 1);
  k_pivot_sep_max<T><<<grid, kSepBlock, 0, s>>>(L, rsL, csL, n, D, rsD, csD, m, piv_t, piv_g,
                                                samp, sample_s, st, mx);
  k_pivot_sep_final<<<1, 256, 0, s>>>(mx, K, st, sep_t, sep_g);
}

#define LSLU_INST(T)                                                          \
  template void launch_fill<T>(T*, T, int64_t, hipStream_t);                  \
  template void launch_sub<T>(const T*, const T*, T*, int64_t, hipStream_t);  \
  template int launch_argmax_parts<T>(const T*, int64_t, ArgPart*,            \
                                      const DevState*, hipStream_t);          \
  template void launch_basis_copy<T>(const T*, int64_t, int64_t, int64_t,     \
                                     int, T*, hipStream_t);                   \
  template void launch_pivot_sep<T>(const T*, int64_t, int64_t, int64_t,      \
                                    const T*, int64_t, int64_t, int64_t,      \
                                    const int*, const int*, const int*, int,  \
                                    int, const DevState*, unsigned long long*,\
                                    double*, double*, hipStream_t);
LSLU_INST(double)
LSLU_INST(float)
template void launch_fill<unsigned char>(unsigned char*, unsigned char, int64_t,
                                         hipStream_t);
template void launch_fill<int>(int*, int, int64_t, hipStream_t);
template void launch_fill<uint64_t>(uint64_t*, uint64_t, int64_t, hipStream_t);
#undef LSLU_INST

}  // namespace lslu
