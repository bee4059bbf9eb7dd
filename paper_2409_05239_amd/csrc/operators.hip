// Operator products A v and A^T w: the only place the method touches A
// (Section 1: matrix-free; Algorithm 5 uses one product with A and one with
// A^T per iteration).
//
// Precision modes (template parameters V = stored operator value, T = vector
// type, Acc = summation type):
//   FP64:   V = double,   T = double, Acc = double
//   FP32:   V = float,    T = float,  Acc = double
//   BF16OP: V = bfloat16, T = float,  Acc = float, input entries rounded to
//           bfloat16 before the product (bf16 x bf16 is exact in float)
//
// Dense and CSR products are row-parallel (one wavefront per output row, a
// fixed lane-stride partial sum and a fixed xor-butterfly reduction), so the
// result does not depend on the launch.  A^T is stored explicitly for both, so
// the adjoint is also a row product with no atomics.
//
// The PSF product is a correlation with either the PSF (A^T) or the PSF
// rotated by 180 degrees (A).  A 32 x 64 output tile and its halo are staged
// in LDS; each lane owns one output column and 8 consecutive output rows, walks
// the PSF column by column, keeps a vertical strip of 8 + ph - 1 inputs in
// registers and reads each weight as a wave-uniform (scalar) operand.
#include "internal.hpp"

namespace lslu {

namespace {

struct Bf16Tag {};

template <typename V>
struct ValTraits;
template <>
struct ValTraits<double> {
  using S = double;
  __device__ static double get(double v) { return v; }
};
template <>
struct ValTraits<float> {
  using S = float;
  __device__ static float get(float v) { return v; }
};
template <>
struct ValTraits<uint16_t> {
  __device__ static float get(uint16_t v) { return bf16_to_f32(v); }
};

// Vector input as seen by the product.
template <typename T, bool kBf16>
__device__ inline auto in_val(T v) {
  if constexpr (kBf16)
    return bf16_to_f32(f32_to_bf16(static_cast<float>(v)));
  else
    return v;
}

template <typename Acc>
__device__ inline Acc wave_sum(Acc v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

constexpr int kRowsPerBlock = 4;  // wavefronts per block, one row each

template <typename V, typename T, typename Acc, bool kBf16>
__global__ __launch_bounds__(kRowsPerBlock * kWave) void k_dense_rows(
    const V* __restrict__ A, int64_t rows, int64_t cols, const T* __restrict__ x,
    T* __restrict__ y, const int* stop) {
  if (stop && *stop) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
  if (r >= rows) return;
  const V* a = A + r * cols;
  Acc acc = 0;
  for (int64_t c = lane; c < cols; c += kWave)
    acc = fma(static_cast<Acc>(ValTraits<V>::get(a[c])),
              static_cast<Acc>(in_val<T, kBf16>(x[c])), acc);
  acc = wave_sum(acc);
  if (lane == 0) y[r] = static_cast<T>(acc);
}

template <typename V, typename T, typename Acc, bool kBf16>
__global__ __launch_bounds__(kRowsPerBlock * kWave) void k_csr_rows(
    const int* __restrict__ rp, const int* __restrict__ ci,
    const V* __restrict__ val, int64_t rows, const T* __restrict__ x,
    T* __restrict__ y, const int* stop) {
  if (stop && *stop) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
  if (r >= rows) return;
  const int beg = rp[r], end = rp[r + 1];
  Acc acc = 0;
  for (int p = beg + lane; p < end; p += kWave)
    acc = fma(static_cast<Acc>(ValTraits<V>::get(val[p])),
              static_cast<Acc>(in_val<T, kBf16>(x[ci[p]])), acc);
  acc = wave_sum(acc);
  if (lane == 0) y[r] = static_cast<T>(acc);
}

// ------------------------------------------------------------------ PSF ----
constexpr int kPsfTW = 64;          // tile width = lanes of a wavefront
constexpr int kPsfR = 8;            // output rows per lane
constexpr int kPsfWaves = 4;        // wavefronts per block
constexpr int kPsfTH = kPsfR * kPsfWaves;  // tile height

// y[i,j] = sum_{a,b} Wt[a,b] * x[i + a - PH/2, j + b - pw/2]  (zero outside)
template <typename T, typename Acc, int PH, bool kBf16>
__global__ __launch_bounds__(kPsfWaves * kWave) void k_psf_corr(
    const T* __restrict__ x, T* __restrict__ y, int rows, int cols,
    const Acc* __restrict__ Wt, int pw, const int* stop) {
  if (stop && *stop) return;
  extern __shared__ unsigned char smem_raw[];
  Acc* tile = reinterpret_cast<Acc*>(smem_raw);
  const int ch = PH / 2, cw = pw / 2;
  const int TR = kPsfTH + PH - 1;
  const int TC = kPsfTW + pw - 1;
  const int i0 = blockIdx.y * kPsfTH, j0 = blockIdx.x * kPsfTW;
  for (int e = threadIdx.x; e < TR * TC; e += blockDim.x) {
    const int tr = e / TC, tc = e - tr * TC;
    const int gi = i0 - ch + tr, gj = j0 - cw + tc;
    Acc v = 0;
    if (gi >= 0 && gi < rows && gj >= 0 && gj < cols)
      v = static_cast<Acc>(in_val<T, kBf16>(x[(int64_t)gi * cols + gj]));
    tile[e] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int r0 = w * kPsfR;  // first output row of this lane (tile-local)
  Acc acc[kPsfR];
#pragma unroll
  for (int p = 0; p < kPsfR; ++p) acc[p] = 0;
  for (int b = 0; b < pw; ++b) {
    Acc s[kPsfR + PH - 1];
#pragma unroll
    for (int q = 0; q < kPsfR + PH - 1; ++q) s[q] = tile[(r0 + q) * TC + lane + b];
#pragma unroll
    for (int a = 0; a < PH; ++a) {
      const Acc wv = Wt[a * pw + b];
#pragma unroll
      for (int p = 0; p < kPsfR; ++p) acc[p] = fma(wv, s[p + a], acc[p]);
    }
  }
  const int gj = j0 + lane;
  if (gj < cols) {
#pragma unroll
    for (int p = 0; p < kPsfR; ++p) {
      const int gi = i0 + r0 + p;
      if (gi < rows) y[(int64_t)gi * cols + gj] = static_cast<T>(acc[p]);
    }
  }
}

template <typename T, typename Acc, bool kBf16, int PH>
void psf_launch_ph(const T* x, T* y, int rows, int cols, const Acc* Wt, int pw,
                   const int* stop, hipStream_t s) {
  dim3 grid((cols + kPsfTW - 1) / kPsfTW, (rows + kPsfTH - 1) / kPsfTH);
  const size_t lds = sizeof(Acc) * (kPsfTH + PH - 1) * (kPsfTW + pw - 1);
  k_psf_corr<T, Acc, PH, kBf16><<<grid, kPsfWaves * kWave, lds, s>>>(
      x, y, rows, cols, Wt, pw, stop);
}

template <typename T, typename Acc, bool kBf16>
void psf_launch(const T* x, T* y, int rows, int cols, const Acc* Wt, int ph,
                int pw, const int* stop, hipStream_t s) {
  switch (ph) {
#define LSLU_PH(P) \
  case P: psf_launch_ph<T, Acc, kBf16, P>(x, y, rows, cols, Wt, pw, stop, s); break;
    LSLU_PH(1) LSLU_PH(3) LSLU_PH(5) LSLU_PH(7) LSLU_PH(9) LSLU_PH(11)
    LSLU_PH(13) LSLU_PH(15) LSLU_PH(17) LSLU_PH(19) LSLU_PH(21) LSLU_PH(23)
    LSLU_PH(25) LSLU_PH(27) LSLU_PH(29) LSLU_PH(31)
#undef LSLU_PH
    default: break;  // rejected at operator creation
  }
}

inline int row_grid(int64_t rows) {
  return static_cast<int>((rows + kRowsPerBlock - 1) / kRowsPerBlock);
}

template <typename V, typename T, typename Acc, bool kBf16>
void dense_apply(const DeviceOp& op, int tr, const void* x, void* y,
                 const int* stop, hipStream_t s) {
  const int64_t rows = tr ? op.n : op.m, cols = tr ? op.m : op.n;
  const V* A = static_cast<const V*>(tr ? op.AT : op.A);
  k_dense_rows<V, T, Acc, kBf16><<<row_grid(rows), kRowsPerBlock * kWave, 0, s>>>(
      A, rows, cols, static_cast<const T*>(x), static_cast<T*>(y), stop);
}

template <typename V, typename T, typename Acc, bool kBf16>
void csr_apply(const DeviceOp& op, int tr, const void* x, void* y,
               const int* stop, hipStream_t s) {
  const int64_t rows = tr ? op.n : op.m;
  k_csr_rows<V, T, Acc, kBf16><<<row_grid(rows), kRowsPerBlock * kWave, 0, s>>>(
      tr ? op.rpT : op.rp, tr ? op.ciT : op.ci,
      static_cast<const V*>(tr ? op.valT : op.val), rows,
      static_cast<const T*>(x), static_cast<T*>(y), stop);
}

}  // namespace

void op_apply(const DeviceOp& op, int tr, const void* x, void* y,
              const int* stop, hipStream_t s) {
  if (op.kind == 0) {
    if (op.prec == kFP64) dense_apply<double, double, double, false>(op, tr, x, y, stop, s);
    else if (op.prec == kFP32) dense_apply<float, float, double, false>(op, tr, x, y, stop, s);
    else dense_apply<uint16_t, float, float, true>(op, tr, x, y, stop, s);
  } else if (op.kind == 1) {
    if (op.prec == kFP64) csr_apply<double, double, double, false>(op, tr, x, y, stop, s);
    else if (op.prec == kFP32) csr_apply<float, float, double, false>(op, tr, x, y, stop, s);
    else csr_apply<uint16_t, float, float, true>(op, tr, x, y, stop, s);
  } else {
    const int rows = static_cast<int>(op.rows), cols = static_cast<int>(op.cols);
    if (op.prec == kFP64)
      psf_launch<double, double, false>(static_cast<const double*>(x),
                                        static_cast<double*>(y), rows, cols,
                                        tr ? op.psf : op.psf_flip, op.ph, op.pw,
                                        stop, s);
    else if (op.prec == kFP32)
      psf_launch<float, double, false>(static_cast<const float*>(x),
                                       static_cast<float*>(y), rows, cols,
                                       tr ? op.psf : op.psf_flip, op.ph, op.pw,
                                       stop, s);
    else
      psf_launch<float, float, true>(static_cast<const float*>(x),
                                     static_cast<float*>(y), rows, cols,
                                     tr ? op.psf32 : op.psf32_flip, op.ph, op.pw,
                                     stop, s);
  }
}

}  // namespace lslu
