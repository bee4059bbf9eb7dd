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

#define LSLU_INST(T)                                                          \
  template void launch_fill<T>(T*, T, int64_t, hipStream_t);                  \
  template void launch_sub<T>(const T*, const T*, T*, int64_t, hipStream_t);  \
  template int launch_argmax_parts<T>(const T*, int64_t, ArgPart*,            \
                                      const DevState*, hipStream_t);          \
  template void launch_basis_copy<T>(const T*, int64_t, int64_t, int64_t,     \
                                     int, T*, hipStream_t);
LSLU_INST(double)
LSLU_INST(float)
template void launch_fill<unsigned char>(unsigned char*, unsigned char, int64_t,
                                         hipStream_t);
template void launch_fill<int>(int*, int, int64_t, hipStream_t);
template void launch_fill<uint64_t>(uint64_t*, uint64_t, int64_t, hipStream_t);
#undef LSLU_INST

}  // namespace lslu
