// Iterates x_k = x_0 + L_k y_k (Algorithm 5, last step of the loop), for all
// k = 1..k_done at once: X = x_0 1^T + L Y with Y upper triangular (column k-1
// of Y holds y_k).  A register-tiled product: a block owns 64 rows of L and
// 64 iterates; chunks of 16 columns of L (staged with loads along the
// basis's contiguous direction) and the matching 16 x 64 block of Y go
// through LDS; each thread accumulates a 4 x 4 tile.  Every x_k(r) sums its
// terms over j in increasing order in FP64, so the result does not depend on
// the tiling.  Columns of L beyond k_done are never read.
//
// Also here: the stopping rule (eq. tol) evaluated on the device, and the copy
// of the selected iterate into the caller's output vector.
#include "internal.hpp"

namespace lslu {

namespace {

constexpr int kAR = 64;   // rows of L per block
constexpr int kAC = 64;   // iterates per block
constexpr int kAJ = 16;   // columns of L per chunk
constexpr int kAsmBlock = 256;

template <typename T>
__global__ __launch_bounds__(kAsmBlock) void k_assemble(
    const T* __restrict__ L, int64_t rs, int64_t cs, int64_t n, const double* __restrict__ Y,
    int K, const T* __restrict__ x0, T* __restrict__ X,
    const DevState* __restrict__ st) {
  __shared__ double sl[kAJ][kAR + 1];
  __shared__ double sy[kAJ][kAC + 1];
  const int kd = st->k_done;
  const int k0 = blockIdx.y * kAC;  // iterates k0+1 .. k0+kAC
  if (k0 >= kd) return;
  const int64_t r0 = (int64_t)blockIdx.x * kAR;
  const int tid = threadIdx.x;
  const int tr = (tid % (kAR / 4)) * 4;  // 4 consecutive rows
  const int tc = (tid / (kAR / 4)) * 4;  // 4 consecutive iterates
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  // y_k has entries j < k, so this block needs j < min(k0 + kAC, k_done)
  const int jmax = min(k0 + kAC, kd);
  for (int j0 = 0; j0 < jmax; j0 += kAJ) {
    for (int e = tid; e < kAJ * kAR; e += kAsmBlock) {
      int jj, rr;
      if (rs == 1) {  // columns contiguous: consecutive threads along rows
        rr = e % kAR;
        jj = e / kAR;
      } else {        // rows contiguous: consecutive threads along columns
        jj = e % kAJ;
        rr = e / kAJ;
      }
      const int64_t r = r0 + rr;
      const int j = j0 + jj;
      sl[jj][rr] = (r < n && j < jmax) ? static_cast<double>(L[r * rs + (int64_t)j * cs]) : 0.0;
    }
    for (int e = tid; e < kAJ * kAC; e += kAsmBlock) {
      const int jj = e % kAJ, cc = e / kAJ;  // column k0+cc of Y is y_{k0+cc+1}
      const int j = j0 + jj, k = k0 + cc;
      sy[jj][cc] = (j < jmax && k < kd) ? Y[(int64_t)k * K + j] : 0.0;
    }
    __syncthreads();
    const int jn = min(kAJ, jmax - j0);
    for (int jj = 0; jj < jn; ++jj) {
      double lv[4], yv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) lv[a] = sl[jj][tr + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) yv[b] = sy[jj][tc + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(lv[a], yv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int k = k0 + tc + b;
    if (k >= kd) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t r = r0 + tr + a;
      if (r < n) {
        const double xb = x0 ? static_cast<double>(x0[r]) : 0.0;
        X[(int64_t)k * n + r] = static_cast<T>(xb + acc[a][b]);
      }
    }
  }
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
  dim3 grid((unsigned)((n + kAR - 1) / kAR), (unsigned)((K + kAC - 1) / kAC));
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
