// Host-side preparation of operators: the CSR checks, the CSR of A^T, the
// 16-bit column indices, the stored value formats and the PSF weights in the
// layout of the matrix-core products.  Plain host code on caller arrays (no
// device calls), so it also builds into the sanitizer checks of the host code.
#pragma once

#include <cstdint>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace lslu {

// nullptr when (indptr, indices) describe an m x n CSR matrix with nnz
// entries: indptr[0] = 0, indptr[m] = nnz, indptr nondecreasing, every
// column index in [0, n) and strictly increasing within its row; else the
// reason.  Reads indptr[0..m] and indices[0..nnz-1] only: each row's bounds
// are checked against nnz before its indices are read.
inline const char* csr_check(int64_t m, int64_t n, int64_t nnz, const int64_t* indptr,
                             const int32_t* indices) {
  if (indptr[0] != 0 || indptr[m] != nnz)
    return "indptr[0] must be 0 and indptr[m] must be nnz";
  for (int64_t r = 0; r < m; ++r) {
    if (indptr[r + 1] < indptr[r]) return "indptr decreases";
    if (indptr[r + 1] > nnz) return "indptr exceeds nnz";
    for (int64_t p = indptr[r]; p < indptr[r + 1]; ++p) {
      if (indices[p] < 0 || indices[p] >= n) return "column index out of range";
      if (p > indptr[r] && indices[p] <= indices[p - 1])
        return "column indices not strictly increasing";
    }
  }
  return nullptr;
}

// A^T in CSR (for a matrix that passed csr_check): count per column, prefix
// sum, scatter in row order, so the column indices of A^T (rows of A) come
// out increasing.  rpT has n + 1 entries, ciT and valT nnz.
inline void csr_transpose(int64_t m, int64_t n, int64_t nnz, const int64_t* indptr,
                          const int32_t* indices, const double* data, std::vector<int>& rpT,
                          std::vector<int>& ciT, std::vector<double>& valT) {
  rpT.assign(n + 1, 0);
  ciT.assign(nnz, 0);
  valT.assign(nnz, 0.0);
  for (int64_t p = 0; p < nnz; ++p) rpT[indices[p] + 1] += 1;
  for (int64_t j = 0; j < n; ++j) rpT[j + 1] += rpT[j];
  std::vector<int> fillp(rpT.begin(), rpT.end() - 1);
  for (int64_t r = 0; r < m; ++r)
    for (int64_t p = indptr[r]; p < indptr[r + 1]; ++p) {
      const int dst = fillp[indices[p]]++;
      ciT[dst] = static_cast<int>(r);
      valT[dst] = data[p];
    }
}

// Column indices in 16 bits; the caller checked that every one is < 65536.
inline std::vector<uint16_t> narrow_indices(const std::vector<int>& idx) {
  return std::vector<uint16_t>(idx.begin(), idx.end());
}

// Host doubles in the operator's stored value type (bytes).
inline std::vector<unsigned char> convert_values(const double* v, int64_t count, int prec) {
  std::vector<unsigned char> out;
  if (prec == kFP64) {
    out.resize(sizeof(double) * count);
    if (count > 0) std::memcpy(out.data(), v, out.size());
  } else if (prec == kFP32) {
    out.resize(sizeof(float) * count);
    float* o = reinterpret_cast<float*>(out.data());
    for (int64_t i = 0; i < count; ++i) o[i] = static_cast<float>(v[i]);
  } else if (prec == kBF16) {
    out.resize(sizeof(uint16_t) * count);
    uint16_t* o = reinterpret_cast<uint16_t*>(out.data());
    for (int64_t i = 0; i < count; ++i) o[i] = f32_to_bf16(static_cast<float>(v[i]));
  } else if (prec == kFP8) {  // E4M3, rounded once from the given double
    out.resize(count);
    for (int64_t i = 0; i < count; ++i) out[i] = f64_to_fp8(v[i]);
  } else {  // binary16, rounded once from the given double
    out.resize(sizeof(uint16_t) * count);
    uint16_t* o = reinterpret_cast<uint16_t*>(out.data());
    for (int64_t i = 0; i < count; ++i) o[i] = f64_to_f16(v[i]);
  }
  return out;
}

// The correlation weights w (ph x pw, row-major) of one direction in the
// form the matrix-core PSF product reads them (device_common.hpp,
// psf_tile_mfma), in the operator's 16- or 8-bit format: for each PSF row a,
// kPer copies s = 0..kPer-1 of the row, each RL codes long, copy s shifted
// left by s codes: code j of copy s is w(a, j + s - 16 - dsh), 0 outside the
// PSF, with dsh = 16 - pw / 2 (the staged tile starts 16 columns left of the
// output tile).  kPer = 4, RL = 76 for bfloat16 and binary16; kPer = 8,
// RL = 80 for E4M3.  Returned as 8-byte words.  w holds ph * pw values,
// 1 <= pw <= 31 (odd).
inline std::vector<uint64_t> psf_mfma_rows(const std::vector<double>& w, int ph, int pw,
                                           int prec) {
  const bool f8 = prec == kFP8;
  const int kPer = f8 ? 8 : 4, RL = f8 ? 80 : 76, esz = f8 ? 1 : 2;
  const int dsh = 16 - pw / 2;
  std::vector<unsigned char> bytes(static_cast<size_t>(ph) * kPer * RL * esz, 0);
  for (int a = 0; a < ph; ++a)
    for (int sft = 0; sft < kPer; ++sft)
      for (int j = 0; j < RL; ++j) {
        const int idx = j + sft - 16 - dsh;
        if (idx < 0 || idx >= pw) continue;
        const double v = w[static_cast<size_t>(a) * pw + idx];
        const size_t at = ((static_cast<size_t>(a) * kPer + sft) * RL + j) * esz;
        if (prec == kBF16) {
          const uint16_t c = f32_to_bf16(static_cast<float>(v));
          std::memcpy(&bytes[at], &c, 2);
        } else if (prec == kFP16) {
          const uint16_t c = f64_to_f16(v);
          std::memcpy(&bytes[at], &c, 2);
        } else {
          bytes[at] = f64_to_fp8(v);
        }
      }
  std::vector<uint64_t> out(bytes.size() / 8);
  std::memcpy(out.data(), bytes.data(), bytes.size());
  return out;
}

}  // namespace lslu
