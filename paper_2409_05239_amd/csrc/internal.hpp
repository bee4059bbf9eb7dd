// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

namespace lslu {

constexpr int kWave = 64;
constexpr int kMaxIter = 256;   // largest maxiter accepted
constexpr int kMaxGrid = 256;   // largest lambda grid accepted
constexpr int kArgmaxBlock = 256;
constexpr int kMaxParts = 4096;  // pivot candidates per streaming pass
// Pivot-entry slots hold this NaN bit pattern until written; no product of
// finite values produces it.
constexpr uint64_t kSlotEmpty = 0x7ff4dead0000beefull;

enum Prec : int { kFP64 = 0, kFP32 = 1, kBF16 = 2, kFP16 = 3, kFP8 = 4 };
// Input rounding of a product (the 16- and 8-bit operator modes).
enum InMode : int { kInNone = 0, kInBf16 = 1, kInFp16 = 2, kInFp8 = 3 };
// An IEEE binary16 operator value (its bits).
struct Half {
  uint16_t bits;
  __host__ __device__ constexpr Half(int z = 0) : bits(static_cast<uint16_t>(z)) {}
};
// An 8-bit E4M3 operator value (its bits): 1 sign, 4 exponent bits with bias
// 7, 3 fraction bits, no infinities, 0x7f / 0xff the NaNs, largest finite
// 448, subnormals 2^-9 m.
struct Fp8 {
  uint8_t bits;
  __host__ __device__ constexpr Fp8(int z = 0) : bits(static_cast<uint8_t>(z)) {}
};
enum Reg : int { kNone = 0, kFixed = 1, kWGCV = 2, kGCV = 3, kOptimal = 4 };
enum Status : int {
  kOK = 0, kBreakQ = 1, kBreakU = 2, kZeroRHS = 3,
  kEInval = -1, kENoMem = -2, kEDevice = -3, kENonFinite = -4, kEUnsupported = -5
};

// Device-resident state of one solve.  `stopped` is read by every kernel of the
// iteration so that work enqueued after a breakdown does nothing.
struct DevState {
  int stopped;      // nonzero once the process has stopped
  int status;       // Status of the process
  int n_l;          // basis vectors l_j formed
  int n_d;          // basis vectors d_j formed
  int k_done;       // iterates x_k that exist (x_1..x_{k_done})
  int mismatch_t;   // replay: own pivot choice differed (d side)
  int mismatch_g;   // replay: own pivot choice differed (l side)
  int ticket;       // half-iteration: pivot-entry blocks finished (reset by block 0)
  double beta;      // r_0(t(1))
  int spin_timeouts;  // waits that hit their bound (an error; never expected)
};

// Zero entries past nnz in the device CSR index and value arrays.
constexpr int64_t kCsrPad = 4;

// One candidate of the pivot search: the signed value v at row idx (key; 0
// for a row that may not be a pivot).  Candidates are ordered by |key|, then
// by the smaller row, so the winner's key is the pivot value itself.
struct ArgPart {
  double key;
  int idx;
  int pad;
};

// How the pivot of one search is recorded.
struct PivotJob {
  int side;              // 0: l side (W(k,k)), 1: d side (H(k+1,k)), 2: r_0 (beta)
  int k;                 // iteration (1-based); 0 for r_0
  int eligible;          // host-side guard of the search (k <= n, k < m)
  int piv_pos;           // position in the pivot list to fill
  double* piv_val;       // where the pivot value goes (W, H or beta)
  int* piv_list;         // pivot list (device)
  int* own_list;         // own choices (device)
  unsigned char* mask;   // "is a pivot" flag per row
  const int* replay;     // replay pivot list (device) or nullptr
  const int* sample;     // candidate rows of a sampled search (device) or nullptr
  int sample_s, sample_len;
  DevState* st;
};
// Longest candidate list of a sampled pivot search.
constexpr int kMaxSampleLen = 512;

// ---------------------------------------------------------------- bf16 ----
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return static_cast<uint16_t>(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(h) << 16);
}

// ---------------------------------------------------------------- fp16 ----
// IEEE binary16 (1 sign, 5 exponent bits with bias 15, 10 fraction bits) on
// the host: a double rounded once to nearest, ties to even (overflow to
// infinity, gradual underflow to the subnormals 2^-24 * m), and back.
inline uint16_t f64_to_f16(double d) {
  if (std::isnan(d)) return 0x7e00;
  const uint16_t sign = std::signbit(d) ? 0x8000 : 0;
  const double a = std::fabs(d);
  if (a >= 65520.0) return sign | 0x7c00;        // at or beyond the rounding
                                                   // boundary of 65504
  if (a < 0x1p-14) {                               // subnormal (or zero)
    const double m = std::nearbyint(a * 0x1p24);   // exact scaling, RNE
    return sign | static_cast<uint16_t>(m);        // m == 1024: smallest normal
  }
  int e2 = 0;
  (void)std::frexp(a, &e2);                        // a = f 2^e2, f in [0.5, 1)
  int e = e2 - 1;                                  // a in [2^e, 2^(e+1))
  double m = std::nearbyint((std::ldexp(a, -e) - 1.0) * 1024.0);
  if (m == 1024.0) {
    m = 0.0;
    ++e;
  }
  if (e > 15) return sign | 0x7c00;
  return sign | static_cast<uint16_t>((e + 15) << 10) | static_cast<uint16_t>(m);
}
inline float f16_to_f32(uint16_t h) {
  const int e = (h >> 10) & 0x1f, m = h & 0x3ff;
  const float sign = (h & 0x8000) ? -1.0f : 1.0f;
  if (e == 0) return sign * std::ldexp(static_cast<float>(m), -24);
  if (e == 31) return m ? NAN : sign * INFINITY;
  return sign * std::ldexp(1.0f + static_cast<float>(m) / 1024.0f, e - 15);
}

// ----------------------------------------------------------------- fp8 ----
// E4M3 on the host: a double rounded once to the nearest E4M3 value, ties to
// even, magnitudes beyond 448 saturated to 448 (NaN stays NaN), and back.
inline double fp8_round_host(double d) {
  if (std::isnan(d)) return d;
  const double a = std::fabs(d);
  int e2 = 0;
  (void)std::frexp(a, &e2);                              // a in [2^(e2-1), 2^e2)
  const int e = std::max(e2 - 1, -6);                     // subnormal spacing 2^-9
  double r = std::ldexp(std::nearbyint(std::ldexp(a, 3 - e)), e - 3);  // exact scaling, RNE
  if (r > 448.0) r = 448.0;
  return std::copysign(r, d);
}
inline uint8_t f64_to_fp8(double d) {
  if (std::isnan(d)) return 0x7f;
  const double r = fp8_round_host(d);
  const uint8_t sign = std::signbit(d) ? 0x80 : 0;
  const double a = std::fabs(r);
  if (a == 0.0) return sign;
  if (a < 0x1p-6) return sign | static_cast<uint8_t>(std::ldexp(a, 9));  // subnormal m
  int e2 = 0;
  (void)std::frexp(a, &e2);
  const int e = e2 - 1;                                   // a in [2^e, 2^(e+1)), e >= -6
  const int m = static_cast<int>(std::ldexp(a, 3 - e)) - 8;
  return sign | static_cast<uint8_t>(((e + 7) << 3) | m);
}
inline float fp8_to_f32(uint8_t b) {
  const int e = (b >> 3) & 15, m = b & 7;
  const float sign = (b & 0x80) ? -1.0f : 1.0f;
  if (e == 15 && m == 7) return NAN;
  if (e == 0) return sign * std::ldexp(static_cast<float>(m), -9);
  return sign * std::ldexp(static_cast<float>(8 + m), e - 10);
}

// ------------------------------------------------------------- launchers ---
// A basis is stored with element (i, j) (row i of basis vector j) at
// p[i * rs + j * cs]: column-major (rs = 1) for the PSF operator, whose kernels
// map lanes to consecutive pixels, row-major (cs = 1) for dense and CSR, whose
// kernels give each row to one wavefront.

// Operators (operators.hip).
struct DeviceOp {
  int kind;         // 0 dense, 1 csr, 2 psf
  int prec;
  int64_t m, n;
  // dense: A (m x n) and AT (n x m), row-major, value type of prec
  void* A = nullptr;
  void* AT = nullptr;
  // csr: column indices as int32, or as uint16 when they all fit (idx16 bit
  // 0: ci, bit 1: ciT), which cuts the bytes an entry streams by 2
  int* rp = nullptr;  void* ci = nullptr;  void* val = nullptr;
  int* rpT = nullptr; void* ciT = nullptr; void* valT = nullptr;
  int idx16 = 0;
  int64_t nnz = 0;
  // psf
  int64_t rows = 0, cols = 0;
  int ph = 0, pw = 0;
  int psf_r = 0;  // output rows per lane of the PSF tiles (2, 4, 8); 0: by size
  double* psf = nullptr;       // correlation weights for A^T (as given)
  double* psf_flip = nullptr;  // correlation weights for A (rotated 180)
  float* psf32 = nullptr;
  float* psf32_flip = nullptr;
  // 16- and 8-bit modes: the weights as the matrix-core product reads them
  // (for A^T and for A; psf_mfma_rows)
  uint64_t* mb = nullptr;
  uint64_t* mb_flip = nullptr;
};
// y = A x (transpose 0) or A^T x (transpose 1).  `stop` may be nullptr.
void op_apply(const DeviceOp& op, int transpose, const void* x, void* y,
              const int* stop, hipStream_t s);

// One half-iteration of the recurrence in one launch (recurrence.hip).
//   block 0            resolves the pivot of the previous half from its
//                      candidates (breakdown test, bookkeeping, triangle row)
//                      and publishes it; then solves the triangular system for
//                      this half's coefficients and publishes them;
//   blocks 1..nlead-1  form the pivot entries of this half's product (one
//                      wavefront per earlier pivot of this side);
//   other blocks       form their rows of the product from the unnormalised
//                      previous vector, normalise their slice of it into its
//                      basis column once the pivot is published, and subtract
//                      the earlier basis vectors once the coefficients are,
//                      writing per-block pivot candidates.
// Entry blocks and consumers wait only for block 0, which publishes the
// pivot before waiting for the entry blocks (dispatched right after it and
// before any consumer); every wait is bounded.  Everything published inside a
// launch goes through slots that hold kSlotEmpty until written once, so a
// waiter reads the value itself and no flag orders other memory.
//
// Slots of one launch (slots_per_launch(K) doubles):
//   [0, K+1)       pivot entries of the product      (blocks 1.. -> block 0)
//   [K+1, 2K+2)    coefficients                      (block 0 -> consumers)
//   2K+2, 2K+3     pivot value; row | state << 32    (block 0 -> all), state
//                  1 = pivot found, 2 = breakdown (the launch ends)
__host__ __device__ inline int64_t slots_per_launch(int K) { return 2 * (int64_t)K + 4; }

template <typename T>
struct HalfArgs {
  // previous half: its unnormalised vector and pivot candidates
  const T* up;
  int64_t lenp;
  const ArgPart* parts_in;
  int nparts_in;
  PivotJob job;
  T* dstp;                 // its basis column: element i at dstp[i * dstp_stride]
  int64_t dstp_stride;
  const T* basisp;         // its side's basis (for the new triangle row)
  int64_t rsp, csp;
  int nbp;                 // earlier vectors of that side
  T* Trowp;                // packed triangle row destination, or nullptr
  // this half: out = op x - basis[:, :nb] coef, x = up / pivot value
  int64_t rows;            // 0: only the pivot of the previous half
  const T* basis;
  int64_t rs, cs;
  int nb;                  // coefficients to form (earlier vectors of this side)
  const int* piv;          // this side's pivots (rows of the pivot entries)
  const T* Tp;             // this side's packed triangle
  double* coef;            // coefficient destination (a column of W or H)
  double* entries;         // this launch's slots (layout above)
  double* cslot;
  uint64_t* pslot;
  int* fail;               // set by block 0 when it cannot publish coefficients
  const unsigned char* mask;
  T* out;
  ArgPart* parts_out;
  int nlead;               // blocks 0..nlead-1 lead; set by launch_half
};
// Returns the number of candidates written to parts_out.
template <typename T>
int launch_half(HalfArgs<T>& a, const DeviceOp& op, int transpose,
                size_t lds_bytes, hipStream_t s);
// The launch launch_half would make, without making it: sets a.nlead and
// returns its consumer count (the candidates it writes).
template <typename T>
int plan_half(HalfArgs<T>& a, const DeviceOp& op, int transpose, size_t lds_bytes);
// Row access of an operator as the batched kernels read it (device copies,
// one per solve): its size, and the bytes for one direction.
size_t row_op_bytes(const DeviceOp& op);
void row_op_write(const DeviceOp& op, int transpose, void* dst);
// One merged launch of the same half-iteration of P planned solves: dargs
// (P HalfArgs), dops (P row accesses), dfirst (P + 1 block offsets, the
// last = blocks) on the device.  a0 and op0 (any of the solves) select the
// kernel; the solves must share the operator kind (dense or CSR) and
// precision.
template <typename T>
void launch_half_batch(HalfArgs<T>& a0, const DeviceOp& op0, int transpose, size_t lds_bytes,
                       const HalfArgs<T>* dargs, const void* dops, const int* dfirst, int P,
                       int blocks, hipStream_t s);
void recurrence_init_attributes(size_t lds_bytes);

// Basis recurrence helpers (basis.hip).
template <typename T>
void launch_fill(T* p, T v, int64_t count, hipStream_t s);
void launch_state_reset(DevState* st, double* nan_fill, int nan_count, hipStream_t s);
// Pivot separations of the 2K+1 searches of a finished recurrence (basis.hip);
// mx: 2K+1 words of scratch; samp: the sampled candidate rows or NULL.
template <typename T>
void launch_pivot_sep(const T* L, int64_t rsL, int64_t csL, int64_t n, const T* D,
                      int64_t rsD, int64_t csD, int64_t m, const int* piv_t,
                      const int* piv_g, const int* samp, int sample_s, int K,
                      const DevState* st, unsigned long long* mx, double* sep_t,
                      double* sep_g, hipStream_t s);
template <typename T>
void launch_sub(const T* a, const T* b, T* out, int64_t len, hipStream_t s);
// Pivot candidates of v (no mask); returns the number of parts.
template <typename T>
int launch_argmax_parts(const T* v, int64_t len, ArgPart* parts,
                        const DevState* st, hipStream_t s);
// dst[j * len + i] = basis(i, j), j < count.
template <typename T>
void launch_basis_copy(const T* src, int64_t rs, int64_t cs, int64_t len,
                       int count, T* dst, hipStream_t s);

// Projected problem (projected.hip).
struct ProjParams {
  int K;           // leading dimension data: H is (K+1) x K, Y is K x K
  int m, n;
  int reg;
  double lambda;
  int n_grid;
  int grid_relative;
  double omega;    // <= 0: (k+1)/m
  const double* grid;         // device
  const int* replay_lambda;   // device or nullptr
  int grid_slots;      // grid values the scratch holds per problem (>= n_grid)
  const double* gram;  // OPTIMAL, gradient: (K+1) x (K+1) Gram matrix of [L, x_true - x_0]
  double* dldl;        // nullptr, or K entries: d/dlambda ||x_k(lambda) - x_true||^2 at lambda_k
};
// The K problems go out in up to kProjGroups launches (consecutive k with
// the same LDS placement), launch g on streams[g % nstreams]; the caller
// orders the streams around the call.
constexpr int kProjGroups = 4;
void launch_projected(const double* H, const DevState* st, double beta_unused,
                      const ProjParams& p, double* Y, double* lam,
                      int* lam_idx, double* ghat, double* sep, double* smax,
                      double* smin, double* scratch, size_t lds_bytes,
                      const hipStream_t* streams, int nstreams);
// Scratch doubles of launch_projected for K problems with room for
// grid_slots grid values each.
size_t projected_scratch_doubles(int K, int grid_slots = kMaxGrid);

// One-time kernel attributes (dynamic LDS limits), set at context creation so
// that no attribute call happens while a solve is being captured.
void projected_init_attributes(size_t lds_bytes);

// Gram matrix of [L_K, x_true - x_0] for the optimal rule (gram.hip):
// G ((K+1) x (K+1), FP64) from the first n_l columns of L (the others count
// as zero); scratch holds gram_scratch_doubles(K) doubles.
constexpr int kGramChunks = 32;
size_t gram_scratch_doubles(int K);
template <typename T>
void launch_gram(const T* L, int64_t rs, int64_t cs, int64_t n, int K,
                 const T* x_true, const T* x0, const DevState* st,
                 double* scratch, double* G, hipStream_t s);

// Iterate assembly (assemble.hip).
template <typename T>
void launch_assemble(const T* L, int64_t rs, int64_t cs, int64_t n,
                     const double* Y, int K, const T* x0, T* X,
                     const DevState* st, hipStream_t s);
// Only x_{k_sel} (k_sel[1], set by launch_stopping): x_out = x_0 + L y_{k_sel}.
template <typename T>
void launch_assemble_final(const T* L, int64_t rs, int64_t cs, int64_t n,
                           const double* Y, int K, const T* x0, T* x_out,
                           const int* k_sel, hipStream_t s);
template <typename T>
void launch_select_x(const T* X, int64_t n, const T* x0, T* x_out,
                     const DevState* st, const int* k_sel, hipStream_t s);
void launch_stopping(const double* ghat, const DevState* st, double tol,
                     int early, int* out, hipStream_t s);

// Reverse pass of a finished solve (adjoint.hip): bbar = (d x_k/d b)^T xbar
// and lambda_bar = xbar^T d x_k/d lambda with the pivots held fixed.  The
// forward arrays are those of the solve (device, as it left them); the
// adjoint arrays are scratch in the working precision (column-major, leading
// dimensions ldl >= n and ldd >= m) and FP64.
struct VjpArgs {
  const DeviceOp* op;
  int64_t m, n;
  int K, k, n_l, n_d;
  const void *L, *D;  // bases l_1..l_{n_l}, d_1..d_{n_d}
  int64_t rsL, csL, rsD, csD;
  const void *TL, *TD;  // packed pivot-row triangles of the solve (wp)
  const double *H, *W, *Y, *lam;  // (K+1) x K, K x K, K x K, K
  const int *piv_t, *piv_g;
  const DevState* st;
  const void* xbar;  // n entries
  void* bbar;        // m entries (out)
  void *Lbar, *Dbar;  // n x K (ldl), m x (K+1) (ldd)
  int64_t ldl, ldd;
  void *um, *un, *pm, *pn;  // m, n, m, n entries
  double* part;   // adjoint_part_doubles(K, max(m, n))
  double* M;      // K x K
  double* Hbar;   // (K+1) x K, leading dimension K+1
  double* corr;   // K+2
  double* scal;   // 4: betabar, lambda_bar, 1/pivot
  int *inv_t, *inv_g;  // m and n: pivot position of each row, or -1
  int* fail;      // 1 when H^T H + lambda^2 I is not positive definite
};
size_t adjoint_part_doubles(int K, int64_t maxlen);
template <typename T>
int run_vjp(const VjpArgs& a, hipStream_t s);

}  // namespace lslu
