// One half-iteration of the pivoted rectangular Hessenberg process: the
// launch dispatch and the entry points the solve driver calls.  The kernels
// and their launch helpers are in recurrence_impl.hpp; the PSF launches of
// each precision mode are in recurrence_psf_<mode>.hip.
#include <cstring>

#include "recurrence_impl.hpp"

namespace lslu {

namespace {

// The PSF launch of the operator's precision mode.
template <typename T>
int launch_psf_half(HalfArgs<T>& a, const DeviceOp& op, int tr, size_t lds_bytes, hipStream_t s,
                    bool dry) {
  if constexpr (std::is_same_v<T, double>) {
    return launch_psf_half_fp64(a, op, tr, lds_bytes, s, dry);
  } else {
    switch (op.prec) {
      case kFP32: return launch_psf_half_fp32(a, op, tr, lds_bytes, s, dry);
      case kBF16: return launch_psf_half_bf16(a, op, tr, lds_bytes, s, dry);
      case kFP16: return launch_psf_half_fp16(a, op, tr, lds_bytes, s, dry);
      default: return launch_psf_half_fp8(a, op, tr, lds_bytes, s, dry);
    }
  }
}

// mode 0: launch; 1: plan only (sets a.nlead, returns the consumer count);
// 2: the merged launch of a batch (a and op stand for every solve of it;
// merged launches are built for the row operators only).
template <typename T>
int half_dispatch(HalfArgs<T>& a, const DeviceOp& op, int tr, size_t lds_bytes, hipStream_t s,
                  int mode, const void* bargs, const void* bops, const int* bfirst, int P,
                  int blocks) {
  if (op.kind == 2) return launch_psf_half<T>(a, op, tr, lds_bytes, s, mode != 0);
  int nparts = 0;
  with_row_op<T>(op, tr, [&](auto ro) {
    using RO = decltype(ro);
    if constexpr (!is_psf_pixels<RO>::value) {
      RowsBatch<T, RO> b{static_cast<const HalfArgs<T>*>(bargs), static_cast<const RO*>(bops),
                         bfirst, P, blocks};
      nparts = launch_rows<T, RO>(a, ro, lds_bytes, s, mode == 1, mode == 2 ? &b : nullptr);
    }
  });
  return nparts;
}

}  // namespace

template <typename T>
int launch_half(HalfArgs<T>& a, const DeviceOp& op, int tr, size_t lds_bytes,
                hipStream_t s) {
  return half_dispatch<T>(a, op, tr, lds_bytes, s, 0, nullptr, nullptr, nullptr, 0, 0);
}

template <typename T>
int plan_half(HalfArgs<T>& a, const DeviceOp& op, int tr, size_t lds_bytes) {
  return half_dispatch<T>(a, op, tr, lds_bytes, nullptr, 1, nullptr, nullptr, nullptr, 0, 0);
}

size_t row_op_bytes(const DeviceOp& op) {
  size_t n = 0;
  if (op.prec == kFP64)
    with_row_op<double>(op, 0, [&](auto ro) { n = sizeof(ro); });
  else
    with_row_op<float>(op, 0, [&](auto ro) { n = sizeof(ro); });
  return n;
}

void row_op_write(const DeviceOp& op, int tr, void* dst) {
  if (op.prec == kFP64)
    with_row_op<double>(op, tr, [&](auto ro) { std::memcpy(dst, &ro, sizeof(ro)); });
  else
    with_row_op<float>(op, tr, [&](auto ro) { std::memcpy(dst, &ro, sizeof(ro)); });
}

template <typename T>
void launch_half_batch(HalfArgs<T>& a0, const DeviceOp& op0, int tr, size_t lds_bytes,
                       const HalfArgs<T>* dargs, const void* dops, const int* dfirst, int P,
                       int blocks, hipStream_t s) {
  (void)half_dispatch<T>(a0, op0, tr, lds_bytes, s, 2, dargs, dops, dfirst, P, blocks);
}

void recurrence_init_attributes(size_t lds_bytes) {
  // Dynamic LDS stays below 64 KB (triangle up to 32 KB, PSF tile up to
  // 46.6 KB), within the default limit.
  (void)lds_bytes;
}

template int launch_half<double>(HalfArgs<double>&, const DeviceOp&, int, size_t, hipStream_t);
template int launch_half<float>(HalfArgs<float>&, const DeviceOp&, int, size_t, hipStream_t);
template int plan_half<double>(HalfArgs<double>&, const DeviceOp&, int, size_t);
template int plan_half<float>(HalfArgs<float>&, const DeviceOp&, int, size_t);
template void launch_half_batch<double>(HalfArgs<double>&, const DeviceOp&, int, size_t,
                                        const HalfArgs<double>*, const void*, const int*, int,
                                        int, hipStream_t);
template void launch_half_batch<float>(HalfArgs<float>&, const DeviceOp&, int, size_t,
                                       const HalfArgs<float>*, const void*, const int*, int,
                                       int, hipStream_t);

}  // namespace lslu
