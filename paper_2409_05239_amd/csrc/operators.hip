// Operator products A v and A^T w -- the only place the method touches A
// (Section 1: matrix-free; Algorithm 5 uses one product with A and one with
// A^T per iteration).  This file holds the standalone product (the residual
// r_0 = b - A x_0 and the lslu_op_apply entry point); inside the iteration
// the product is fused with the elimination that follows it
// (recurrence.hip).
//
// Precision modes (V = stored operator value, T = vector type, Acc = sum):
//   FP64:   V = double,   T = double, Acc = double
//   FP32:   V = float,    T = float,  Acc = double
//   BF16OP: V = bfloat16, T = float,  Acc = float, input entries rounded to
//           bfloat16 before the product (bf16 x bf16 is exact in float)
//   FP16OP, FP8OP: as BF16OP with IEEE binary16, 8-bit E4M3 values
// In the last three modes the PSF product and the dense product (row
// length a multiple of 16 or 32, up to 4096) run on the matrix cores
// (psf_tile_mfma, dense_mfma_rows16 in device_common.hpp).
//
// Dense and CSR products are row-parallel (a group of 16 lanes per output
// row, a fixed lane-stride partial sum and a fixed xor-butterfly reduction),
// so the result does not depend on the launch.  A^T is stored explicitly for
// both, so the adjoint is also a row product with no atomics.  The PSF
// product is a correlation with either the PSF (A^T) or the PSF rotated by
// 180 degrees (A), computed by LDS-staged tiles.
#include "device_common.hpp"

namespace lslu {

namespace {

constexpr int kRowLanes = 16;
constexpr int kRowBlock = 256;
constexpr int kRowsPerBlock = kRowBlock / kRowLanes;

template <class RowOp, typename T>
__global__ __launch_bounds__(kRowBlock) void k_rows(
    RowOp op, int64_t rows, const T* __restrict__ x, T* __restrict__ y,
    const int* stop) {
  if (stop && *stop) return;
  const int sub = threadIdx.x % kRowLanes;
  const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kRowLanes;
  if (r >= rows) return;
  auto xf = [x](int64_t c) { return x[c]; };
  typename RowOp::Acc acc = op.template partial<kRowLanes>(r, sub, xf);
  acc = group_sum<kRowLanes>(acc);
  if (sub == 0) y[r] = static_cast<T>(acc);
}

// The 16- and 8-bit dense products on the matrix cores (dense_mfma_rows16):
// the input's codes in LDS, a 16-row group per wavefront.
template <typename T, int kIn>
__global__ __launch_bounds__(kRowBlock) void k_rows_dense_mfma(
    const void* __restrict__ a, int64_t rows, int64_t n, const T* __restrict__ x,
    T* __restrict__ y, const int* stop) {
  if (stop && *stop) return;
  __shared__ typename PsfMfma<kIn>::E xs[kDenseMfmaMaxCols];
  dense_mfma_stage_x<kIn>([x](int64_t c) { return x[c]; }, n, xs, kRowBlock);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t r16 = ((int64_t)blockIdx.x * (kRowBlock / kWave) + threadIdx.x / kWave) * 16;
  if (r16 >= rows) return;
  const mfma_f4 acc = dense_mfma_rows16<kIn>(a, rows, n, r16, xs, 0, 1);
  if ((lane & 15) == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r16 + 4 * (lane >> 4) + r;
      if (row < rows) y[row] = static_cast<T>(acc[r]);
    }
  }
}

template <typename T, typename Acc, int PH, int kIn, int R>
__global__ __launch_bounds__(kPsfWaves * kWave) void k_psf_corr(
    const T* __restrict__ x, T* __restrict__ y, int rows, int cols,
    const Acc* __restrict__ Wt, int pw, const int* stop) {
  if (stop && *stop) return;
  extern __shared__ unsigned char smem_raw[];
  Acc* tile = reinterpret_cast<Acc*>(smem_raw);
  const int i0 = blockIdx.y * psf_th<R>(), j0 = blockIdx.x * kPsfTW;
  Acc acc[R];
  psf_tile<T, Acc, PH, kIn, R>(x, rows, cols, Wt, pw, i0, j0, tile, acc);
  const int lane = threadIdx.x & (kWave - 1);
  const int r0 = (threadIdx.x / kWave) * R;
  const int gj = j0 + lane;
  if (gj < cols) {
#pragma unroll
    for (int p = 0; p < R; ++p) {
      const int gi = i0 + r0 + p;
      if (gi < rows) y[(int64_t)gi * cols + gj] = static_cast<T>(acc[p]);
    }
  }
}

// The same product on the matrix cores (the 16- and 8-bit modes): a
// 16 RB x 64 tile per block, its operand blocks and input tile in LDS.
template <typename T, int PH, int kIn, int R>
__global__ __launch_bounds__(kPsfWaves * kWave) void k_psf_corr_mfma(
    const T* __restrict__ x, T* __restrict__ y, int rows, int cols,
    const uint64_t* __restrict__ mb, int pw, const int* stop) {
  if (stop && *stop) return;
  extern __shared__ unsigned char smem_raw[];
  constexpr int RB = psf_th<R>() / 16;
  uint64_t* bl = reinterpret_cast<uint64_t*>(smem_raw);
  unsigned char* tile = smem_raw + sizeof(uint64_t) * psf_mfma_b_words<kIn, PH>();
  psf_mfma_stage_b<kIn, PH>(mb, bl);
  const int i0 = blockIdx.y * psf_th<R>(), j0 = blockIdx.x * kPsfTW;
  mfma_f4 acc[RB];
  psf_tile_mfma<kIn, PH, RB>(x, [](float v) { return static_cast<float>(in_val<kIn>(v)); }, rows,
                             cols, i0, j0, bl, tile, acc);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int gj = j0 + 16 * w + (lane & 15);
  if (gj < cols) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + 16 * rb + 4 * (lane >> 4) + r;
        if (gi < rows) y[(int64_t)gi * cols + gj] = static_cast<T>(acc[rb][r]);
      }
  }
}

template <typename Acc>
const Acc* psf_weights(const DeviceOp& op, int tr) {
  if constexpr (std::is_same_v<Acc, double>)
    return tr ? op.psf : op.psf_flip;
  else
    return tr ? op.psf32 : op.psf32_flip;
}

template <typename T>
void apply_t(const DeviceOp& op, int tr, const T* x, T* y, const int* stop,
             hipStream_t s) {
  with_mode<T>(op.prec, [&](auto v, auto acc, auto bf) {
    using V = decltype(v);
    using Acc = decltype(acc);
    constexpr int kB = decltype(bf)::value;
    const int64_t rows = tr ? op.n : op.m;
    const int grid = static_cast<int>((rows + kRowsPerBlock - 1) / kRowsPerBlock);
    if (op.kind == 0) {
      DenseRows<V, Acc, kB> ro{static_cast<const V*>(tr ? op.AT : op.A), tr ? op.m : op.n};
      if constexpr (DenseMfma<decltype(ro)>::value) {
        if (dense_mfma_fits<kB>(ro.cols)) {
          const int g16 = static_cast<int>((rows + 63) / 64);
          k_rows_dense_mfma<T, kB><<<g16, kRowBlock, 0, s>>>(ro.a, rows, ro.cols, x, y, stop);
          return;
        }
      }
      k_rows<<<grid, kRowBlock, 0, s>>>(ro, rows, x, y, stop);
    } else if (op.kind == 1) {
      const int* rp = tr ? op.rpT : op.rp;
      const void* ci = tr ? op.ciT : op.ci;
      const V* val = static_cast<const V*>(tr ? op.valT : op.val);
      if (op.idx16 & (tr ? 2 : 1)) {
        CsrRows<V, Acc, kB, uint16_t> ro{rp, static_cast<const uint16_t*>(ci), val};
        k_rows<<<grid, kRowBlock, 0, s>>>(ro, rows, x, y, stop);
      } else {
        CsrRows<V, Acc, kB, int> ro{rp, static_cast<const int*>(ci), val};
        k_rows<<<grid, kRowBlock, 0, s>>>(ro, rows, x, y, stop);
      }
    } else {
      const int R = static_cast<int>(op.rows), C = static_cast<int>(op.cols);
      with_ph(op.ph, [&](auto phc) {
        constexpr int PH = decltype(phc)::value;
        with_psf_r(op.psf_r, R, C, [&](auto rc) {
          constexpr int PR = psf_rows_used<kB, decltype(rc)::value>();
          dim3 g((C + kPsfTW - 1) / kPsfTW, (R + psf_th<PR>() - 1) / psf_th<PR>());
          const size_t lds = psf_lds_bytes<Acc, PH, kB, PR>(op.pw);
          if constexpr (psf_on_mfma<kB>())
            k_psf_corr_mfma<T, PH, kB, PR><<<g, kPsfWaves * kWave, lds, s>>>(
                x, y, R, C, tr ? op.mb : op.mb_flip, op.pw, stop);
          else
            k_psf_corr<T, Acc, PH, kB, PR><<<g, kPsfWaves * kWave, lds, s>>>(
                x, y, R, C, psf_weights<Acc>(op, tr), op.pw, stop);
        });
      });
    }
  });
}

}  // namespace

void op_apply(const DeviceOp& op, int tr, const void* x, void* y,
              const int* stop, hipStream_t s) {
  if (op.prec == kFP64)
    apply_t<double>(op, tr, static_cast<const double*>(x), static_cast<double*>(y), stop, s);
  else
    apply_t<float>(op, tr, static_cast<const float*>(x), static_cast<float*>(y), stop, s);
}

}  // namespace lslu
