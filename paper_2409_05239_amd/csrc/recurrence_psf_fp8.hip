// PSF half-iteration launches of the FP8 operator mode (see
// recurrence_impl.hpp): vectors in float, sums in float.
#include "recurrence_impl.hpp"

namespace lslu {

int launch_psf_half_fp8(HalfArgs<float>& a, const DeviceOp& op, int tr, size_t lds_bytes,
                        hipStream_t s, bool dry) {
  return launch_psf_mode<float, float, kInFp8>(a, op, tr, lds_bytes, s, dry);
}

}  // namespace lslu
