// PSF half-iteration launches of the FP64 operator mode (see
// recurrence_impl.hpp): vectors in double, sums in double.
#include "recurrence_impl.hpp"

namespace lslu {

int launch_psf_half_fp64(HalfArgs<double>& a, const DeviceOp& op, int tr, size_t lds_bytes,
                        hipStream_t s, bool dry) {
  return launch_psf_mode<double, double, kInNone>(a, op, tr, lds_bytes, s, dry);
}

}  // namespace lslu
