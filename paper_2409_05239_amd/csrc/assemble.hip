// Iterates x_k = x_0 + L_k y_k (Algorithm 5, last step of the loop), for all
// k = 1..k_done at once: X = x_0 1^T + L Y with Y upper triangular (column k-1
// of Y holds y_k).  Each thread owns one row of L and a block of kChunk
// consecutive iterates; y entries are wave-uniform.  Sums run over j in
// increasing order in FP64.
//
// Also here: the stopping rule (eq. tol) evaluated on the device, and the copy
// of the selected iterate into the caller's output vector.
#include "internal.hpp"

namespace lslu {

namespace {

constexpr int kChunk = 32;
constexpr int kAsmBlock = 256;

template <typename T>
__global__ __launch_bounds__(kAsmBlock) void k_assemble(
    const T* __restrict__ L, int64_t rs, int64_t cs, int64_t n, const double* __restrict__ Y,
    int K, const T* __restrict__ x0, T* __restrict__ X,
    const DevState* __restrict__ st) {
  const int kd = st->k_done;
  const int k0 = blockIdx.y * kChunk;  // iterates k0+1 .. k0+kChunk
  if (k0 >= kd) return;
  const int64_t r = (int64_t)blockIdx.x * kAsmBlock + threadIdx.x;
  if (r >= n) return;
  const int kc = min(kChunk, kd - k0);
  double acc[kChunk];
#pragma unroll
  for (int c = 0; c < kChunk; ++c) acc[c] = 0.0;
  const int jmax = k0 + kc;  // y_{k0+kc} has k0+kc entries
  for (int j = 0; j < jmax; ++j) {
    const double l = static_cast<double>(L[r * rs + (int64_t)j * cs]);
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      // y_{k0+c+1} has entries j = 0 .. k0+c
      if (c < kc && j <= k0 + c) acc[c] = fma(l, Y[(int64_t)(k0 + c) * K + j], acc[c]);
    }
  }
  const double xb = x0 ? static_cast<double>(x0[r]) : 0.0;
#pragma unroll
  for (int c = 0; c < kChunk; ++c)
    if (c < kc) X[(int64_t)(k0 + c) * n + r] = static_cast<T>(xb + acc[c]);
}

// k_sel: iterate to return (0 = x_0).
__global__ void k_stopping(const double* __restrict__ ghat, const DevState* st,
                           double tol, int early, int* out /* [k_stop, k_sel] */) {
  if (threadIdx.x != 0) return;
  const int kd = st->k_done;
  int ks = kd;
  if (kd >= 2 && ghat[0] != 0.0) {
    for (int k = 2; k <= kd; ++k) {
      if (fabs(ghat[k - 1] - ghat[k - 2]) / ghat[0] < tol) {
        ks = k - 1;
        break;
      }
    }
  }
  out[0] = ks;
  out[1] = early ? ks : kd;
}

template <typename T>
__global__ void k_select_x(const T* __restrict__ X, int64_t n,
                           const T* __restrict__ x0, T* __restrict__ x_out,
                           const int* __restrict__ sel) {
  const int ks = sel[1];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x)
    x_out[r] = ks > 0 ? X[(int64_t)(ks - 1) * n + r] : (x0 ? x0[r] : T(0));
}

}  // namespace

template <typename T>
void launch_assemble(const T* L, int64_t rs, int64_t cs, int64_t n,
                     const double* Y, int K, const T* x0, T* X,
                     const DevState* st, hipStream_t s) {
  dim3 grid((unsigned)((n + kAsmBlock - 1) / kAsmBlock),
            (unsigned)((K + kChunk - 1) / kChunk));
  k_assemble<T><<<grid, kAsmBlock, 0, s>>>(L, rs, cs, n, Y, K, x0, X, st);
}

void launch_stopping(const double* ghat, const DevState* st, double tol,
                     int early, int* out, hipStream_t s) {
  k_stopping<<<1, 64, 0, s>>>(ghat, st, tol, early, out);
}

template <typename T>
void launch_select_x(const T* X, int64_t n, const T* x0, T* x_out,
                     const DevState*, const int* k_sel, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  k_select_x<T><<<(unsigned)g, 256, 0, s>>>(X, n, x0, x_out, k_sel);
}

template void launch_assemble<double>(const double*, int64_t, int64_t, int64_t,
                                      const double*, int, const double*,
                                      double*, const DevState*, hipStream_t);
template void launch_assemble<float>(const float*, int64_t, int64_t, int64_t,
                                     const double*, int, const float*, float*,
                                     const DevState*, hipStream_t);
template void launch_select_x<double>(const double*, int64_t, const double*,
                                      double*, const DevState*, const int*,
                                      hipStream_t);
template void launch_select_x<float>(const float*, int64_t, const float*,
                                     float*, const DevState*, const int*,
                                     hipStream_t);

}  // namespace lslu
