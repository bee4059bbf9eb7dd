// Device helpers shared by the operator and recurrence kernels: value access
// per precision mode, fixed-order reductions, the pivot order, and row access
// to the operator (one row of A or A^T for dense and CSR, one pixel of the PSF
// correlation) summed by an aligned group of G lanes.
#pragma once

#include <climits>
#include <type_traits>

#include "internal.hpp"

namespace lslu {

// ----------------------------------------------------------- value access --
template <typename V>
struct ValTraits;
template <>
struct ValTraits<double> {
  __device__ static double get(double v) { return v; }
};
template <>
struct ValTraits<float> {
  __device__ static float get(float v) { return v; }
};
template <>
struct ValTraits<uint16_t> {
  __device__ static float get(uint16_t v) { return bf16_to_f32(v); }
};
// E4M3: (8 + m) 2^(e - 10), subnormals m 2^-9 (exact in float).
__device__ inline float fp8_decode(uint8_t b) {
  const int e = (b >> 3) & 15, m = b & 7;
  const float v = (e == 0) ? __builtin_ldexpf(static_cast<float>(m), -9)
                           : __builtin_ldexpf(static_cast<float>(8 + m), e - 10);
  const float r = (e == 15 && m == 7) ? __builtin_nanf("") : v;
  return (b & 0x80) ? -r : r;
}
// The nearest E4M3 value of a float, ties to even, saturated to +-448.
__device__ inline float fp8_round(float x) {
  const float a = __builtin_fabsf(x);
  int e2 = 0;
  (void)__builtin_frexpf(a, &e2);
  const int e = (e2 - 1 > -6) ? e2 - 1 : -6;
  float r = __builtin_ldexpf(__builtin_rintf(__builtin_ldexpf(a, 3 - e)), e - 3);
  r = (r > 448.0f) ? 448.0f : r;
  return (a != a) ? x : __builtin_copysignf(r, x);
}
template <>
struct ValTraits<Fp8> {
  __device__ static float get(Fp8 v) { return fp8_decode(v.bits); }
};
template <>
struct ValTraits<Half> {
  __device__ static float get(Half v) {
    return static_cast<float>(__builtin_bit_cast(_Float16, v.bits));
  }
};

// The nearest binary16 value of a float (ties to even).  The float is pinned
// in a register first: the compiler folds a float -> half conversion of a
// value just rounded from double into one rounding from the double, which
// differs at the float values that lie halfway between binary16 values.
__device__ inline float fp16_round(float f) {
  __asm__("" : "+v"(f));
  return static_cast<float>(static_cast<_Float16>(f));
}

// Input rounding of the operator modes (kIn: kInNone, kInBf16, kInFp16, kInFp8):
// in the 16-bit operator modes a product's input entries are rounded to the
// operator's format, so every term is a product of two 16-bit numbers, exact
// in float.
template <int kIn, typename T>
__device__ inline auto in_val(T v) {
  if constexpr (kIn == kInBf16)
    return bf16_to_f32(f32_to_bf16(static_cast<float>(v)));
  else if constexpr (kIn == kInFp8)
    return fp8_round(static_cast<float>(v));
  else if constexpr (kIn == kInFp16)
    return fp16_round(static_cast<float>(v));
  else
    return v;
}

// ------------------------------------------------------------ normaliser --
// x / v with the value of IEEE division, for many x and one v.  FP32: the
// product x * RN(1/v) formed in FP64 has relative error at most 2^-52, while
// a quotient of two 24-bit numbers lies at least 2^-49 (relative) from every
// FP32 rounding midpoint and is never exactly on one; rounding the FP64
// product to FP32 therefore gives RN(x/v) exactly, with one multiply instead
// of a division sequence.  FP64: IEEE division.
template <typename T>
struct Normaliser;
template <>
struct Normaliser<float> {
  float v;
  double r;
  __device__ explicit Normaliser(float pivot) : v(pivot), r(1.0 / static_cast<double>(pivot)) {}
  __device__ float operator()(float x) const {
    return static_cast<float>(static_cast<double>(x) * r);
  }
};
template <>
struct Normaliser<double> {
  double v;
  __device__ explicit Normaliser(double pivot) : v(pivot) {}
  __device__ double operator()(double x) const { return x / v; }
};

// ------------------------------------------------------------ reductions --
// Lane exchanges through DPP (data-parallel primitives: VALU moves, no LDS
// round trip).  `dpp<CTRL>(v)` returns v of the lane that CTRL names.
template <int CTRL>
__device__ inline float dpp(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(u)), CTRL,
                                             0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(u >> 32)),
                                             CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                        static_cast<uint32_t>(lo));
}

template <typename Acc>
__device__ inline Acc readlane_any(Acc v, int lane);
template <>
__device__ inline float readlane_any(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Sum over the G lanes of an aligned lane group (G = 4, 8, 16, 32, 64), every
// lane of the group gets the same sum.  Within 16 lanes: pairs (quad_perm
// [1,0,3,2]), quads ([2,3,0,1]), half rows (row_half_mirror), rows
// (row_mirror); each step adds two equal-ranked partial sums, so all lanes
// hold bitwise the same value and the order never depends on timing.  Rows of
// 16 are then added through readlane in a fixed order.
template <int G, typename Acc>
__device__ inline Acc group_sum(Acc v) {
  static_assert(G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "group size");
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  if constexpr (G >= 8) v += dpp<0x141>(v);
  if constexpr (G >= 16) v += dpp<0x140>(v);
  if constexpr (G >= 32) {
    const Acc r0 = readlane_any(v, 0), r1 = readlane_any(v, 16);
    const Acc r2 = readlane_any(v, 32), r3 = readlane_any(v, 48);
    if constexpr (G == 64) {
      v = (r0 + r1) + (r2 + r3);
    } else {
      v = ((threadIdx.x & (kWave - 1)) < 32) ? r0 + r1 : r2 + r3;
    }
  }
  return v;
}

__device__ inline double readlane_d(double v, int lane) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  uint32_t lo = static_cast<uint32_t>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(u)), lane));
  uint32_t hi = static_cast<uint32_t>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(u >> 32)), lane));
  return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}
template <>
__device__ inline double readlane_any(double v, int lane) { return readlane_d(v, lane); }

// Total order of every pivot search over signed keys: larger |v| first, then
// the smaller row (ties go to the smallest index).  Ineligible rows carry key
// 0, so they never win over a nonzero entry and a search whose winner has key
// 0 has found no pivot.
__device__ inline bool better(double ka, int ia, double kb, int ib) {
  const double a = fabs(ka), b = fabs(kb);
  return a > b || (a == b && ia < ib);
}

__device__ inline void wave_argmax(double& key, int& idx) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    double ok = __shfl_xor(key, off);
    int oi = __shfl_xor(idx, off);
    if (better(ok, oi, key, idx)) {
      key = ok;
      idx = oi;
    }
  }
}

// Block-wide argmax; the result is returned to every thread.
template <int BLOCK>
__device__ inline void block_argmax(double& key, int& idx) {
  __shared__ double sk[BLOCK / kWave];
  __shared__ int si[BLOCK / kWave];
  wave_argmax(key, idx);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sk[w] = key;
    si[w] = idx;
  }
  __syncthreads();
  key = sk[0];
  idx = si[0];
  for (int i = 1; i < BLOCK / kWave; ++i)
    if (better(sk[i], si[i], key, idx)) {
      key = sk[i];
      idx = si[i];
    }
  __syncthreads();
}

// ------------------------------------------------------- operator rows ----
// Operands of the first NP terms of a lane's share of one row: the operator
// values and the entries of the not yet normalised input that they multiply.
// Loading them needs no pivot, so a launch issues these loads before the
// pivot is known; finish() normalises the staged inputs (x / pivot value,
// the values the normalised vector holds) and adds the terms in the order
// partial() would.
template <typename V, typename T, int NP>
struct RowStage {
  V v[NP];
  T x[NP];
  int64_t row;   // the row (dense, PSF) or its first entry position (CSR)
  int64_t next;  // where the terms after the staged ones start
  int64_t end;
};

// Each policy sums its row over the lanes sub, sub+G, ... of a group of G
// lanes with x(c) supplied by a functor; group_sum<G> completes the sum.

// Row r of a row-major dense matrix with `cols` columns.
template <typename V, typename AccT, int kIn>
struct DenseRows {
  using Acc = AccT;
  using Val = V;
  static constexpr int kInMode = kIn;
  const V* a;
  int64_t cols;
  template <int G, typename XF>
  __device__ Acc rest(int64_t r, int64_t c0, XF xf, Acc acc) const {
    const V* row = a + r * cols;
#pragma unroll 4
    for (int64_t c = c0; c < cols; c += G)
      acc = fma(static_cast<Acc>(ValTraits<V>::get(row[c])),
                static_cast<Acc>(in_val<kIn>(xf(c))), acc);
    return acc;
  }
  template <int G, typename XF>
  __device__ Acc partial(int64_t r, int sub, XF xf) const {
    return rest<G>(r, sub, xf, Acc(0));
  }
  // The first NP terms of the lane: columns sub, sub+G, ...
  template <int G, int NP, typename T>
  __device__ void stage(int64_t r, int sub, const T* __restrict__ u,
                        RowStage<V, T, NP>& s) const {
    const V* row = a + r * cols;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int64_t c = sub + (int64_t)k * G;
      s.v[k] = c < cols ? row[c] : V(0);
      s.x[k] = c < cols ? u[c] : T(0);
    }
    s.row = r;
    s.next = sub + (int64_t)NP * G;
    s.end = cols;
  }
  template <int G, int NP, typename T, typename NZ, typename XF>
  __device__ Acc finish(const RowStage<V, T, NP>& s, const NZ& nz, XF xf) const {
    Acc acc = 0;
#pragma unroll
    for (int k = 0; k < NP; ++k)
      if (s.next - (int64_t)(NP - k) * G < s.end)
        acc = fma(static_cast<Acc>(ValTraits<V>::get(s.v[k])),
                  static_cast<Acc>(in_val<kIn>(nz(s.x[k]))), acc);
    return rest<G>(s.row, s.next, xf, acc);
  }
};

// Four consecutive operator values from a position that is a multiple of 4
// (16-byte loads for float, two for double, one 8-byte load for bfloat16).
template <typename V>
struct Quad;
template <>
struct Quad<float> {
  __device__ static void load(const float* p, float (&v)[4]) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
};
template <>
struct Quad<double> {
  __device__ static void load(const double* p, double (&v)[4]) {
    const double2 a = reinterpret_cast<const double2*>(p)[0];
    const double2 b = reinterpret_cast<const double2*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
};
template <>
struct Quad<uint16_t> {
  __device__ static void load(const uint16_t* p, uint16_t (&v)[4]) {
    const uint2 q = *reinterpret_cast<const uint2*>(p);
    v[0] = static_cast<uint16_t>(q.x & 0xffffu); v[1] = static_cast<uint16_t>(q.x >> 16);
    v[2] = static_cast<uint16_t>(q.y & 0xffffu); v[3] = static_cast<uint16_t>(q.y >> 16);
  }
};

template <>
struct Quad<Fp8> {
  __device__ static void load(const Fp8* p, Fp8 (&v)[4]) {
    const uint32_t q = *reinterpret_cast<const uint32_t*>(p);
    v[0].bits = static_cast<uint8_t>(q & 0xffu); v[1].bits = static_cast<uint8_t>((q >> 8) & 0xffu);
    v[2].bits = static_cast<uint8_t>((q >> 16) & 0xffu); v[3].bits = static_cast<uint8_t>(q >> 24);
  }
};

template <>
struct Quad<Half> {
  __device__ static void load(const Half* p, Half (&v)[4]) {
    const uint2 q = *reinterpret_cast<const uint2*>(p);
    v[0].bits = static_cast<uint16_t>(q.x & 0xffffu); v[1].bits = static_cast<uint16_t>(q.x >> 16);
    v[2].bits = static_cast<uint16_t>(q.y & 0xffffu); v[3].bits = static_cast<uint16_t>(q.y >> 16);
  }
};

// Four column indices from a position that is a multiple of 4 (one 16-byte
// load of int32, one 8-byte load of uint16).
template <typename I>
struct Idx4;
template <>
struct Idx4<int> {
  __device__ static void load(const int* p, int (&c)[4]) {
    const int4 c4 = *reinterpret_cast<const int4*>(p);
    c[0] = c4.x; c[1] = c4.y; c[2] = c4.z; c[3] = c4.w;
  }
};
template <>
struct Idx4<uint16_t> {
  __device__ static void load(const uint16_t* p, int (&c)[4]) {
    const uint2 q = *reinterpret_cast<const uint2*>(p);
    c[0] = static_cast<int>(q.x & 0xffffu); c[1] = static_cast<int>(q.x >> 16);
    c[2] = static_cast<int>(q.y & 0xffffu); c[3] = static_cast<int>(q.y >> 16);
  }
};

// Row r of a CSR matrix (int32 row pointers; int32 or uint16 column indices;
// index and value arrays 16-byte aligned and readable 3 entries past nnz).  The row is
// read in aligned chunks of 4 entries: lane `sub` of a group of G takes the
// chunks that start at (beg & ~3) + 4 sub + 4 G i, with one vector load for
// the indices and one for the values per chunk, then the gathers of its
// entries inside [beg, end), kChunks chunks per batch so a row costs few
// dependent round trips.  Each lane adds its entries in chunk order.
template <typename V, typename AccT, int kIn, typename I = int>
struct CsrRows {
  using Acc = AccT;
  using Val = V;
  static constexpr int kChunks = 2;
  const int* rp;
  const I* ci;
  const V* val;
  // Chunks q, q + 4G, ... below end (entries outside [beg, end) skipped).
  template <int G, typename XF>
  __device__ Acc rest(int q, int beg, int end, XF xf, Acc acc) const {
    using X = decltype(xf(0));
    for (; q < end; q += kChunks * 4 * G) {
      int c[kChunks][4];
      V v[kChunks][4];
#pragma unroll
      for (int h = 0; h < kChunks; ++h) {
        const int qh = q + h * 4 * G;
        if (qh < end) {
          Idx4<I>::load(ci + qh, c[h]);
          Quad<V>::load(val + qh, v[h]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            c[h][e] = 0;
            v[h][e] = V(0);
          }
        }
      }
      X x[kChunks][4];
#pragma unroll
      for (int h = 0; h < kChunks; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int pos = q + h * 4 * G + e;
          x[h][e] = (pos >= beg && pos < end) ? xf(c[h][e]) : X(0);
        }
#pragma unroll
      for (int h = 0; h < kChunks; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int pos = q + h * 4 * G + e;
          if (pos >= beg && pos < end)
            acc = fma(static_cast<Acc>(ValTraits<V>::get(v[h][e])),
                      static_cast<Acc>(in_val<kIn>(x[h][e])), acc);
        }
    }
    return acc;
  }
  template <int G, typename XF>
  __device__ Acc partial(int64_t r, int sub, XF xf) const {
    const int beg = rp[r], end = rp[r + 1];
    return rest<G>((beg & ~3) + 4 * sub, beg, end, xf, Acc(0));
  }
  // The lane's first NP entries (NP / 4 chunks): values and the raw input
  // entries they multiply.
  template <int G, int NP, typename T>
  __device__ void stage(int64_t r, int sub, const T* __restrict__ u,
                        RowStage<V, T, NP>& s) const {
    static_assert(NP % 4 == 0, "whole chunks");
    constexpr int NC = NP / 4;
    const int beg = rp[r], end = rp[r + 1];
    const int q = (beg & ~3) + 4 * sub;
    int c[NP];
#pragma unroll
    for (int h = 0; h < NC; ++h) {
      const int qh = q + h * 4 * G;
      V vv[4];
      if (qh < end) {
        int cc[4];
        Idx4<I>::load(ci + qh, cc);
#pragma unroll
        for (int e = 0; e < 4; ++e) c[4 * h + e] = cc[e];
        Quad<V>::load(val + qh, vv);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          c[4 * h + e] = 0;
          vv[e] = V(0);
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) s.v[4 * h + e] = vv[e];
    }
#pragma unroll
    for (int h = 0; h < NC; ++h)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int pos = q + h * 4 * G + e;
        s.x[4 * h + e] = (pos >= beg && pos < end) ? u[c[4 * h + e]] : T(0);
      }
    s.row = beg;
    s.next = q;
    s.end = end;
  }
  template <int G, int NP, typename T, typename NZ, typename XF>
  __device__ Acc finish(const RowStage<V, T, NP>& s, const NZ& nz, XF xf) const {
    constexpr int NC = NP / 4;
    const int beg = static_cast<int>(s.row), end = static_cast<int>(s.end);
    const int q = static_cast<int>(s.next);
    Acc acc = 0;
#pragma unroll
    for (int h = 0; h < NC; ++h)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int pos = q + h * 4 * G + e;
        if (pos >= beg && pos < end)
          acc = fma(static_cast<Acc>(ValTraits<V>::get(s.v[4 * h + e])),
                    static_cast<Acc>(in_val<kIn>(nz(s.x[4 * h + e]))), acc);
      }
    return rest<G>(q + NC * 4 * G, beg, end, xf, acc);
  }
};

// Pixel `pix` of the zero-boundary correlation with weights wt (ph x pw):
// y(i,j) = sum_{a,b} wt(a,b) x(i + a - ph/2, j + b - pw/2).
template <typename AccT, int kIn>
struct PsfPixels {
  using Acc = AccT;
  using Val = AccT;
  static constexpr int kInMode = kIn;
  const Acc* wt;
  int rows, cols, ph, pw;
  // The same weights as the matrix-core product reads them (padded rows,
  // psf_mfma_rows on the host), in the 16- and 8-bit modes; nullptr otherwise.
  const uint64_t* mb = nullptr;
  template <int G, typename XF>
  __device__ Acc partial(int64_t pix, int sub, XF xf) const {
    const int i = static_cast<int>(pix / cols);
    const int j = static_cast<int>(pix - (int64_t)i * cols);
    const int ch = ph / 2, cw = pw / 2;
    Acc acc = 0;
    for (int t = sub; t < ph * pw; t += G) {
      const int a = t / pw, b = t - a * pw;
      const int gi = i + a - ch, gj = j + b - cw;
      if (gi >= 0 && gi < rows && gj >= 0 && gj < cols)
        acc = fma(wt[t], static_cast<Acc>(in_val<kIn>(xf((int64_t)gi * cols + gj))),
                  acc);
    }
    return acc;
  }
  // Nothing is staged: the terms need the pivot value only through x.
  template <int G, int NP, typename T>
  __device__ void stage(int64_t pix, int sub, const T* __restrict__, RowStage<Acc, T, NP>& s) const {
    s.row = pix;
    s.next = sub;
  }
  template <int G, int NP, typename T, typename NZ, typename XF>
  __device__ Acc finish(const RowStage<Acc, T, NP>& s, const NZ&, XF xf) const {
    return partial<G>(s.row, static_cast<int>(s.next), xf);
  }
};

template <typename RO>
struct is_psf_pixels : std::false_type {};
template <typename AccT, int kIn>
struct is_psf_pixels<PsfPixels<AccT, kIn>> : std::true_type {};

// --------------------------------------------------------------- PSF tile --
// An R*4 x 64 output tile and its halo are staged in LDS; each lane owns one
// output column and R consecutive output rows, walks the PSF column by column,
// keeps a vertical strip of R + ph - 1 inputs in registers and reads each
// weight as a wave-uniform (scalar) operand.  R = 8 reuses each staged input
// most; R = 2 makes four times as many tiles, which keeps more of the chip
// busy on small images (psf_rows_per_lane); an operator can also carry a
// choice measured on the device (lslu_op_tile).
constexpr int kPsfTW = 64;          // tile width = lanes of a wavefront
constexpr int kPsfWaves = 4;        // wavefronts per block
template <int R>
__host__ __device__ constexpr int psf_th() { return R * kPsfWaves; }  // tile height

// ---------------------------------------------------- PSF on the MFMA ----
// In the 16- and 8-bit operator modes every product term is a product of two
// numbers of the format, exact in float, and the terms are summed in float:
// what the matrix cores compute.  For one filter row a, the correlation along
// an image row is a banded (Toeplitz) matrix product,
//     y[i, j] += sum_c x[i + a, c] W(a, c - j)   (W zero outside 0..pw-1),
// so a 16 x 16 block of outputs (rows i, columns j) is
// sum_a sum_t X(a, t) B(a, t), with X(a, t) the 16 x kK window of the staged
// tile at row offset a and column offset kK t.  The tile starts 16 columns
// left of the output tile (a 16-byte boundary, so it is staged with 16-byte
// loads), dsh = 16 - pw/2 columns left of the first input a correlation
// needs, so B(a, t)[k][n] = W(a, kK t + k - n - dsh).  In the lane layout of
// the instruction, lane l holds row l % 16, columns kPer (l / 16) + e
// (e = 0..kPer-1) of X as one 8-byte word, B[kPer (l / 16) + e][l % 16]
// likewise, and gets rows 4 (l / 16) + r (r = 0..3), column l % 16 of the
// float result.  Lane l's word of B(a, t) is the run of kPer codes
// W(a, o - 16 - dsh + e) with o = kK t + kPer (l / 16) - l % 16 + 16: the
// operator keeps each PSF row padded with zeros (psf_mfma_rows) in kPer
// copies, copy s shifted left by s codes, so that the run starts at an
// 8-byte boundary of copy o mod kPer.  All kNT blocks t are summed for every
// PSF width (blocks outside the band multiply zeros).  Row lengths are padded
// so that the 16 lanes of a row group hit distinct LDS banks.
typedef short mfma_s4 __attribute__((ext_vector_type(4)));
typedef _Float16 mfma_h4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <int kIn>
struct PsfMfma;
template <>
struct PsfMfma<kInBf16> {
  using E = uint16_t;
  static constexpr int kK = 16, kPer = 4, kNT = 3;
  // v is a bfloat16 value held in a float: its upper 16 bits
  __device__ static E enc(float v) { return static_cast<E>(__builtin_bit_cast(uint32_t, v) >> 16); }
  __device__ static mfma_f4 mma(uint64_t a, uint64_t b, mfma_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(mfma_s4, a),
                                                     __builtin_bit_cast(mfma_s4, b), c, 0, 0, 0);
  }
};
template <>
struct PsfMfma<kInFp16> {
  using E = uint16_t;
  static constexpr int kK = 16, kPer = 4, kNT = 3;
  __device__ static E enc(float v) {
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(v));  // exact: v is binary16
  }
  __device__ static mfma_f4 mma(uint64_t a, uint64_t b, mfma_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(mfma_h4, a),
                                                 __builtin_bit_cast(mfma_h4, b), c, 0, 0, 0);
  }
};
template <>
struct PsfMfma<kInFp8> {
  using E = uint8_t;
  static constexpr int kK = 32, kPer = 8, kNT = 2;
  // v is an E4M3 value held in a float (|v| <= 448): its 8-bit code
  __device__ static E enc(float v) {
    const float a = __builtin_fabsf(v);
    const uint8_t sign = __builtin_signbitf(v) ? 0x80 : 0;
    if (a == 0.0f) return sign;
    if (a < 0x1p-6f) return sign | static_cast<uint8_t>(a * 0x1p9f);  // subnormal m 2^-9
    int e2 = 0;
    (void)__builtin_frexpf(a, &e2);
    const int e = e2 - 1;  // a in [2^e, 2^(e+1)), e >= -6
    const int m = static_cast<int>(__builtin_ldexpf(a, 3 - e)) - 8;
    return sign | static_cast<uint8_t>(((e + 7) << 3) | m);
  }
  __device__ static mfma_f4 mma(uint64_t a, uint64_t b, mfma_f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(static_cast<long>(a), static_cast<long>(b),
                                                      c, 0, 0, 0);
  }
};

template <int kIn>
constexpr bool psf_on_mfma() {
  return kIn == kInBf16 || kIn == kInFp16 || kIn == kInFp8;
}
// Tile shape in the MFMA modes: 8 output rows per lane (two 16-row blocks
// per 32 x 64 tile) whatever shape the operator was given: the shapes only
// trade staging reuse against parallelism for the vector-unit products.
template <int kIn, int R>
constexpr int psf_rows_used() {
  return psf_on_mfma<kIn>() ? 8 : R;
}
// Codes per row of the staged tile in the MFMA modes: the windows of the
// last 16-column block reach column 48 + kK kNT - 1 (95, 111); padded to a
// row of 4 x (odd) 4-byte words.
template <int kIn>
constexpr int psf_mfma_cols() {
  return PsfMfma<kIn>::kK == 16 ? 104 : 112;
}
// Codes staged from the image per tile row (24 16-byte loads of floats);
// the rest of the row is zero.
constexpr int kPsfMfmaStaged = 96;
// Codes of one padded PSF row copy: the runs reach o + kPer - 1 with
// o <= kK (kNT - 1) + 3 kPer + 16 (63, 79); padded for the LDS banks.
template <int kIn>
constexpr int psf_mfma_row() {
  return PsfMfma<kIn>::kK == 16 ? 76 : 80;
}
// 8-byte words of the padded rows of a PSF with PH rows (kPer copies each).
template <int kIn, int PH>
constexpr int psf_mfma_b_words() {
  return PH * PsfMfma<kIn>::kPer * psf_mfma_row<kIn>() * (int)sizeof(typename PsfMfma<kIn>::E) / 8;
}

template <typename Acc, int PH, int kIn, int R>
__host__ __device__ constexpr size_t psf_lds_bytes(int pw) {
  if constexpr (psf_on_mfma<kIn>()) {
    // padded rows, then the tile
    return sizeof(uint64_t) * psf_mfma_b_words<kIn, PH>() +
           sizeof(typename PsfMfma<kIn>::E) * (psf_th<R>() + PH - 1) * psf_mfma_cols<kIn>();
  } else {
    return sizeof(Acc) * (psf_th<R>() + PH - 1) * (kPsfTW + pw - 1);
  }
}

// ------------------------------------------- dense rows on the matrix cores --
// The 16-, 8-bit dense operators (stored values are the format's codes) on
// the matrix cores: 16 rows r16 .. r16+15 of the row-major m x n matrix times
// an input vector held as codes in LDS.  The rows are the A operand (lane l:
// row l % 16, the kPer codes from column kK t + kPer (l / 16), one 8-byte
// load); the input is column 0 of the B operand (lanes l % 16 == 0), the
// other 15 columns zero, so lanes with l % 16 == 0 get rows 4 (l / 16) + r of
// the product in element r.  A wave sums the column blocks t = t0, t0 + dt,
// ... in increasing t.  Only 1/16 of each instruction's columns is used: the
// product of one vector has no reuse, and the matrix cores take the codes
// as they are stored (no conversion per element).  Needs n a multiple of kK
// (rows then start at 8-byte boundaries); rows past m are read clamped and
// their results are not used.
template <typename RO>
struct DenseMfma : std::false_type {};
template <int kIn>
struct DenseMfmaVal;
template <>
struct DenseMfmaVal<kInBf16> { using V = uint16_t; };
template <>
struct DenseMfmaVal<kInFp16> { using V = Half; };
template <>
struct DenseMfmaVal<kInFp8> { using V = Fp8; };
template <typename V, int kIn>
struct DenseMfma<DenseRows<V, float, kIn>>
    : std::integral_constant<bool, psf_on_mfma<kIn>() &&
                                       std::is_same_v<V, typename DenseMfmaVal<kIn>::V>> {};

// Largest row length the matrix-core dense product takes (its input codes
// sit in LDS).
constexpr int kDenseMfmaMaxCols = 4096;

template <int kIn>
__host__ __device__ constexpr bool dense_mfma_fits(int64_t n) {
  return n > 0 && n <= kDenseMfmaMaxCols && n % PsfMfma<kIn>::kK == 0;
}

// Codes of the input x(c) (rounded to the format) for c < n, by the block's
// threads; the caller synchronises before use.
template <int kIn, typename XF>
__device__ inline void dense_mfma_stage_x(XF xf, int64_t n, typename PsfMfma<kIn>::E* xs,
                                          int nthreads) {
  for (int64_t c = threadIdx.x; c < n; c += nthreads)
    xs[c] = PsfMfma<kIn>::enc(static_cast<float>(in_val<kIn>(xf(c))));
}

template <int kIn>
__device__ inline mfma_f4 dense_mfma_rows16(const void* a, int64_t m, int64_t n, int64_t r16,
                                            const typename PsfMfma<kIn>::E* xs, int t0, int dt) {
  using M = PsfMfma<kIn>;
  using E = typename M::E;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t row = r16 + (lane & 15) < m ? r16 + (lane & 15) : m - 1;
  const E* arow = static_cast<const E*>(a) + row * n + M::kPer * (lane >> 4);
  const E* xl = xs + M::kPer * (lane >> 4);
  const bool bcol = (lane & 15) == 0;
  mfma_f4 acc = {0.f, 0.f, 0.f, 0.f};
  const int nt = static_cast<int>(n / M::kK);
  for (int t = t0; t < nt; t += dt) {
    const uint64_t aw = *reinterpret_cast<const uint64_t*>(arow + (int64_t)M::kK * t);
    const uint64_t bw = bcol ? *reinterpret_cast<const uint64_t*>(xl + M::kK * t) : 0ull;
    acc = M::mma(aw, bw, acc);
  }
  return acc;
}

// Copies the padded PSF rows into LDS (all threads of the block; every load
// is issued before the stores).
template <int kIn, int PH>
__device__ inline void psf_mfma_stage_b(const uint64_t* __restrict__ mb, uint64_t* bl) {
  constexpr int N = psf_mfma_b_words<kIn, PH>(), PER = (N + kPsfWaves * kWave - 1) / (kPsfWaves * kWave);
  uint64_t v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = threadIdx.x + u * kPsfWaves * kWave;
    v[u] = i < N ? mb[i] : 0;
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = threadIdx.x + u * kPsfWaves * kWave;
    if (i < N) bl[i] = v[u];
  }
}

// The outputs of the 16 RB x 64 tile at (i0, j0) on the matrix cores: wave w
// computes the 16-column block w of every 16-row block rb into acc[rb]
// (lane l: rows 16 rb + 4 (l / 16) + r, column 16 w + l % 16).  The product's
// input at pixel p is cvt(u[p]), rounded to the format; bl holds the padded
// PSF rows (psf_mfma_stage_b).  Every output is summed in the same order
// (a, then t) whatever RB.  Ends with a barrier (the tile may be restaged
// next).
// The raw (unnormalised) inputs of a thread's share of a matrix-core tile's
// staged rows: they do not depend on the pivot, so a consumer loads its first
// tile's before it waits (psf_tile_mfma_load), and converts them once the
// pivot is known (psf_tile_mfma_from).
template <int PH, int RB>
struct MfmaTileIn {
  static constexpr int kTR = 16 * RB + PH - 1;
  static constexpr int kQ = kPsfMfmaStaged / 4;  // 16-byte loads per row
  static constexpr int kPer = (kTR * kQ + kPsfWaves * kWave - 1) / (kPsfWaves * kWave);
  float4 v[kPer];
};

// Columns j0 - 16 + 4 g .. + 3 come as one 16-byte load when they are in the
// image (all or none of them when the row length is a multiple of 4); every
// load of the share is issued before any value is used.
template <int PH, int RB>
__device__ inline void psf_tile_mfma_load(const float* __restrict__ u, int rows, int cols, int i0,
                                          int j0, MfmaTileIn<PH, RB>& in) {
  using In = MfmaTileIn<PH, RB>;
  constexpr int NT = kPsfWaves * kWave, Q = In::kQ, TR = In::kTR;
  const int ch = PH / 2;
  const bool vec = (cols & 3) == 0 && (reinterpret_cast<uintptr_t>(u) & 15) == 0;
#pragma unroll
  for (int p = 0; p < In::kPer; ++p) {
    const int e = threadIdx.x + p * NT;
    const int tr = e / Q, g = e - tr * Q;
    const int gi = i0 - ch + tr, gj = j0 - 16 + 4 * g;
    in.v[p] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (e < TR * Q && gi >= 0 && gi < rows) {
      const float* src = u + (int64_t)gi * cols;
      if (vec) {
        if (gj >= 0 && gj < cols) in.v[p] = *reinterpret_cast<const float4*>(src + gj);
      } else {
        if (gj >= 0 && gj < cols) in.v[p].x = src[gj];
        if (gj + 1 >= 0 && gj + 1 < cols) in.v[p].y = src[gj + 1];
        if (gj + 2 >= 0 && gj + 2 < cols) in.v[p].z = src[gj + 2];
        if (gj + 3 >= 0 && gj + 3 < cols) in.v[p].w = src[gj + 3];
      }
    }
  }
}

template <int kIn, int PH, int RB, typename CVT>
__device__ inline void psf_tile_mfma_from(const MfmaTileIn<PH, RB>& in, CVT cvt,
                                          const uint64_t* __restrict__ bl,
                                          unsigned char* tile_raw, mfma_f4 (&acc)[RB]) {
  using M = PsfMfma<kIn>;
  using E = typename M::E;
  using In = MfmaTileIn<PH, RB>;
  constexpr int TCM = psf_mfma_cols<kIn>();
  constexpr int TR = In::kTR;
  constexpr int NT = kPsfWaves * kWave;
  constexpr int Q = In::kQ;
  constexpr int PER = In::kPer;
  E* tile = reinterpret_cast<E*>(tile_raw);
  {
    const float4* v = in.v;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = threadIdx.x + p * NT;
      if (e < TR * Q) {
        const int tr = e / Q, g = e - tr * Q;
        E* d = tile + tr * TCM + 4 * g;  // 4 codes: 8 (or 4) aligned bytes
        const uint64_t c0 = M::enc(cvt(v[p].x)), c1 = M::enc(cvt(v[p].y)),
                       c2 = M::enc(cvt(v[p].z)), c3 = M::enc(cvt(v[p].w));
        constexpr int sh = 8 * sizeof(E);
        const uint64_t word = c0 | (c1 << sh) | (c2 << (2 * sh)) | (c3 << (3 * sh));
        if constexpr (sizeof(E) == 2)
          *reinterpret_cast<uint64_t*>(d) = word;
        else
          *reinterpret_cast<uint32_t*>(d) = static_cast<uint32_t>(word);
      }
    }
    // columns past the staged ones, read by the last windows: zero
    if constexpr (TCM > kPsfMfmaStaged && sizeof(E) == 1) {
      for (int e = threadIdx.x; e < TR * (TCM - kPsfMfmaStaged) / 4; e += NT) {
        const int per_row = (TCM - kPsfMfmaStaged) / 4;
        const int tr = e / per_row, g = e - tr * per_row;
        *reinterpret_cast<uint32_t*>(tile + tr * TCM + kPsfMfmaStaged + 4 * g) = 0u;
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb] = mfma_f4{0.f, 0.f, 0.f, 0.f};
  const E* base = tile + (lane & 15) * TCM + 16 * w + M::kPer * (lane >> 4);
  // lane's operand run of B(a, t) starts at code o = kK t + o0 of its row
  constexpr int RL = psf_mfma_row<kIn>();
  const int o0 = M::kPer * (lane >> 4) - (lane & 15) + 16;
  const E* rows_b = reinterpret_cast<const E*>(bl);
  for (int a = 0; a < PH; ++a) {
#pragma unroll
    for (int t = 0; t < M::kNT; ++t) {
      const int o = M::kK * t + o0;
      const int sft = o & (M::kPer - 1);
      const uint64_t b = *reinterpret_cast<const uint64_t*>(
          rows_b + (a * M::kPer + sft) * RL + (o - sft));
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const uint64_t x = *reinterpret_cast<const uint64_t*>(base + (16 * rb + a) * TCM +
                                                              M::kK * t);
        acc[rb] = M::mma(x, b, acc[rb]);
      }
    }
  }
  __syncthreads();
}

template <int kIn, int PH, int RB, typename CVT>
__device__ inline void psf_tile_mfma(const float* __restrict__ u, CVT cvt, int rows, int cols,
                                     int i0, int j0, const uint64_t* __restrict__ bl,
                                     unsigned char* tile_raw, mfma_f4 (&acc)[RB]) {
  MfmaTileIn<PH, RB> in;
  psf_tile_mfma_load<PH, RB>(u, rows, cols, i0, j0, in);
  psf_tile_mfma_from<kIn, PH, RB>(in, cvt, bl, tile_raw, acc);
}

// Output rows per lane for a rows x cols image: 8 when that still gives at
// least two tiles per compute unit (512 tiles), else 2.
inline int psf_rows_per_lane(int64_t rows, int64_t cols) {
  const int64_t t8 = ((cols + kPsfTW - 1) / kPsfTW) * ((rows + psf_th<8>() - 1) / psf_th<8>());
  return t8 >= 512 ? 8 : 2;
}

// Calls f(std::integral_constant<int, R>) for R = r (2, 4 or 8; the
// operator's tuned choice), or psf_rows_per_lane(rows, cols) when r is 0.
template <typename F>
void with_psf_r(int r, int64_t rows, int64_t cols, F&& f) {
  switch (r ? r : psf_rows_per_lane(rows, cols)) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
  }
}

// acc[p] = y[i0 + r0 + p, j0 + lane] for the tile at (i0, j0), with
// y[i,j] = sum_{a,b} Wt[a,b] * x[i + a - PH/2, j + b - pw/2]  (zero outside),
// r0 = R * wavefront.  Ends with the tile still in LDS (no trailing barrier).
template <typename T, typename Acc, int PH, int kIn, int R>
__device__ inline void psf_tile(const T* __restrict__ x, int rows, int cols,
                                const Acc* __restrict__ Wt, int pw, int i0,
                                int j0, Acc* tile, Acc (&acc)[R]) {
  const int ch = PH / 2, cw = pw / 2;
  const int TR = psf_th<R>() + PH - 1;
  const int TC = kPsfTW + pw - 1;
  for (int e = threadIdx.x; e < TR * TC; e += blockDim.x) {
    const int tr = e / TC, tc = e - tr * TC;
    const int gi = i0 - ch + tr, gj = j0 - cw + tc;
    Acc v = 0;
    if (gi >= 0 && gi < rows && gj >= 0 && gj < cols)
      v = static_cast<Acc>(in_val<kIn>(x[(int64_t)gi * cols + gj]));
    tile[e] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int r0 = (threadIdx.x / kWave) * R;
#pragma unroll
  for (int p = 0; p < R; ++p) acc[p] = 0;
  for (int b = 0; b < pw; ++b) {
    Acc s[R + PH - 1];
#pragma unroll
    for (int q = 0; q < R + PH - 1; ++q) s[q] = tile[(r0 + q) * TC + lane + b];
#pragma unroll
    for (int a = 0; a < PH; ++a) {
      const Acc wv = Wt[a * pw + b];
#pragma unroll
      for (int p = 0; p < R; ++p) acc[p] = fma(wv, s[p + a], acc[p]);
    }
  }
}

// Calls f(std::integral_constant<int, PH>) for the PSF height (odd 1..31,
// checked when the operator is created).
template <typename F>
void with_ph(int ph, F&& f) {
  switch (ph) {
#define LSLU_PH(P) \
  case P: f(std::integral_constant<int, P>{}); break;
    LSLU_PH(1) LSLU_PH(3) LSLU_PH(5) LSLU_PH(7) LSLU_PH(9) LSLU_PH(11)
    LSLU_PH(13) LSLU_PH(15) LSLU_PH(17) LSLU_PH(19) LSLU_PH(21) LSLU_PH(23)
    LSLU_PH(25) LSLU_PH(27) LSLU_PH(29) LSLU_PH(31)
#undef LSLU_PH
    default: break;
  }
}

// Calls f(V{}, Acc{}, bf16 flag) for the operator's precision mode with the
// vector type T.
template <typename T, typename F>
void with_mode(int prec, F&& f) {
  if constexpr (std::is_same_v<T, double>) {
    if (prec == kFP64) f(double{}, double{}, std::integral_constant<int, kInNone>{});
  } else {
    if (prec == kFP32) f(float{}, double{}, std::integral_constant<int, kInNone>{});
    else if (prec == kBF16) f(uint16_t{}, float{}, std::integral_constant<int, kInBf16>{});
    else if (prec == kFP16) f(Half{}, float{}, std::integral_constant<int, kInFp16>{});
    else if (prec == kFP8) f(Fp8{}, float{}, std::integral_constant<int, kInFp8>{});
  }
}

}  // namespace lslu
