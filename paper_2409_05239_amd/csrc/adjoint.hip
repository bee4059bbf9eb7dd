// Reverse pass of a finished solve: the vector-Jacobian product
//     bbar = (d x_k / d b)^T xbar,   lambda_bar = xbar^T d x_k / d lambda
// with the pivots of the solve held fixed (the recurrence of Algorithm 5 is
// then a smooth map of b) and x_0 held fixed.
//
// Forward pieces and their adjoints.  Each half-iteration of Algorithm 5 has
// the same shape: v_0 = (product), then for j = 1..p a coefficient read at
// the j-th pivot row, c_j = v_{j-1}(piv_j), and v_j = v_{j-1} - c_j b_j; then
// the new vector b_{p+1} = v_p / v_p(piv_{p+1}).  (d-side of iteration k:
// p = k, c = H(1:k, k), pivot entry H(k+1, k), b = d.  l-side: p = k - 1,
// c = W(1:k-1, k), pivot entry W(k, k), b = l.  Start: p = 0, pivot entry
// beta, b_1 = d_1 = r_0 / beta.)  Given the adjoint bbar_{p+1} of the new
// vector and direct adjoints cbar_j of the coefficients and pivbar of the
// pivot entry:
//     s = bbar_{p+1} . b_{p+1},  vt = bbar_{p+1} / piv,
//     corr_{p+1} = pivbar - s / piv,
//     corr_j = cbar_j - (bbar_{p+1} . b_j) / piv - sum_{i > j} corr_i b_j(piv_i)
//                                                  (j = p..1),
//     vbar_0 = vt + sum_i corr_i e_{piv_i}          (input of the adjoint product)
//     bbar_j -= c_j (vt + sum_{i > j} corr_i e_{piv_i})   (j = 1..p).
// The projected problem (eq. TSP): y = M^{-1} H^T beta e_1 with
// M = H^T H + lambda^2 I, so with z = M^{-1} ybar
//     Hbar = (beta e_1 - H y) z^T - H z y^T,  betabar = (H z)_1,
//     lambda_bar = -2 lambda z^T y,
// and x_k = x_0 + L_k y gives Lbar = xbar y^T, ybar = L_k^T xbar.
//
// The basis stays resident in HBM from the forward solve (it is needed for
// x_k anyway), and so do the entries of the basis at the pivot rows (the
// packed triangles the recurrence keeps), so nothing is recomputed.  Dot
// products are summed in FP64 by fixed row chunks and reduced in a fixed
// order: the result does not depend on the launch.
#include "device_common.hpp"

namespace lslu {

namespace {

constexpr int kAT = 256;          // threads per block
constexpr int kDotCols = 8;       // basis columns per block of the dot products
constexpr int kDotRowsPerThread = 8;
constexpr int64_t kDotChunk = (int64_t)kDotRowsPerThread * kAT;  // rows per block
constexpr int kTriCap = 8256;     // triangle entries staged in LDS (p <= 128)

__host__ __device__ inline int64_t tri_row(int i) { return (int64_t)i * (i - 1) / 2; }

int dot_chunks(int64_t len) { return static_cast<int>((len + kDotChunk - 1) / kDotChunk); }

// part[c * ncol + j] = sum over the rows of chunk c (blockIdx.x, kDotChunk
// rows) of (v1 + v2)(r) * B(r, j), for the kDotCols columns j of blockIdx.y:
// each thread reads the vector once for all of them, its rows' loads issued
// together.
template <typename T>
__global__ __launch_bounds__(kAT) void k_dots(const T* __restrict__ B, int64_t rs,
                                             int64_t cs, int64_t len, int ncol,
                                             const T* __restrict__ v1,
                                             const T* __restrict__ v2,
                                             double* __restrict__ part) {
  __shared__ double red[kAT / kWave][kDotCols];
  const int c0 = blockIdx.y * kDotCols;
  const int nc = (ncol - c0 < kDotCols) ? ncol - c0 : kDotCols;
  const int64_t r0 = (int64_t)blockIdx.x * kDotChunk;
  double acc[kDotCols];
#pragma unroll
  for (int c = 0; c < kDotCols; ++c) acc[c] = 0.0;
  // all loads of the thread first (rows beyond len and columns beyond nc
  // read as 0), then the sums, row by row in order
  double vv[kDotRowsPerThread];
  T bb[kDotRowsPerThread][kDotCols];
#pragma unroll
  for (int u = 0; u < kDotRowsPerThread; ++u) {
    const int64_t r = r0 + threadIdx.x + (int64_t)u * kAT;
    const bool in = r < len;
    vv[u] = in ? static_cast<double>(v1[r]) + (v2 ? static_cast<double>(v2[r]) : 0.0) : 0.0;
    const T* row = B + (in ? r : 0) * rs + (int64_t)c0 * cs;
#pragma unroll
    for (int c = 0; c < kDotCols; ++c) bb[u][c] = (in && c < nc) ? row[(int64_t)c * cs] : T(0);
  }
#pragma unroll
  for (int u = 0; u < kDotRowsPerThread; ++u)
#pragma unroll
    for (int c = 0; c < kDotCols; ++c) acc[c] = fma(vv[u], static_cast<double>(bb[u][c]), acc[c]);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < kDotCols; ++c) {
    const double t = group_sum<kWave>(acc[c]);
    if (lane == 0) red[w][c] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < nc) {
    double t = 0.0;
    for (int i = 0; i < kAT / kWave; ++i) t += red[i][threadIdx.x];
    part[(size_t)blockIdx.x * ncol + c0 + threadIdx.x] = t;
  }
}

// Adjoint of the projected problem of iteration k (one block, FP64).
// scal[0] = betabar, scal[1] = lambda_bar; *fail = 1 if M is not positive
// definite (then the derivative is not defined).
__global__ __launch_bounds__(kAT) void k_adj_projected(
    const double* __restrict__ H, int ldh, int k, const double* __restrict__ y,
    const double* __restrict__ lam_p, const DevState* __restrict__ st,
    const double* __restrict__ part, int nchunks, double* __restrict__ M,
    double* __restrict__ Hbar, double* __restrict__ scal, int* __restrict__ fail) {
  __shared__ double zb[kMaxIter], hy[kMaxIter + 1], hz[kMaxIter + 1], ys[kMaxIter];
  __shared__ double red[kAT / kWave];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const double lam = *lam_p;
  if (tid == 0) s_bad = 0;
  for (int j = tid; j < k; j += kAT) {
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * k + j];
    zb[j] = s;  // ybar, overwritten by z
    ys[j] = y[j];
  }
  // M = H^T H + lambda^2 I (H upper Hessenberg: column j has rows 0..j+1)
  for (int idx = tid; idx < k * k; idx += kAT) {
    const int i = idx / k, j = idx - i * k;
    const int rmax = (i < j ? i : j) + 1;
    double s = (i == j) ? lam * lam : 0.0;
    for (int r = 0; r <= rmax; ++r) s = fma(H[(size_t)i * ldh + r], H[(size_t)j * ldh + r], s);
    M[idx] = s;
  }
  __syncthreads();
  // Cholesky M = R^T R (lower factor stored in the lower triangle)
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const double d = M[(size_t)j * k + j];
      if (!(d > 0.0)) s_bad = 1;
      M[(size_t)j * k + j] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double djj = M[(size_t)j * k + j];
    for (int i = j + 1 + tid; i < k; i += kAT) M[(size_t)i * k + j] /= djj;
    __syncthreads();
    const int rem = k - j - 1;
    for (int idx = tid; idx < rem * rem; idx += kAT) {
      const int a = j + 1 + idx / rem, b = j + 1 + idx % rem;
      if (b <= a) M[(size_t)a * k + b] -= M[(size_t)a * k + j] * M[(size_t)b * k + j];
    }
    __syncthreads();
  }
  // z = M^{-1} ybar: forward then backward substitution, one column at a time
  for (int j = 0; j < k; ++j) {
    if (tid == 0) zb[j] /= M[(size_t)j * k + j];
    __syncthreads();
    for (int i = j + 1 + tid; i < k; i += kAT) zb[i] -= M[(size_t)i * k + j] * zb[j];
    __syncthreads();
  }
  for (int j = k - 1; j >= 0; --j) {
    if (tid == 0) zb[j] /= M[(size_t)j * k + j];
    __syncthreads();
    for (int i = tid; i < j; i += kAT) zb[i] -= M[(size_t)j * k + i] * zb[j];
    __syncthreads();
  }
  // H y and H z
  for (int r = tid; r <= k; r += kAT) {
    double a = 0.0, b = 0.0;
    for (int j = (r > 0 ? r - 1 : 0); j < k; ++j) {
      a = fma(H[(size_t)j * ldh + r], ys[j], a);
      b = fma(H[(size_t)j * ldh + r], zb[j], b);
    }
    hy[r] = a;
    hz[r] = b;
  }
  __syncthreads();
  const double beta = st->beta;
  for (int idx = tid; idx < (k + 1) * k; idx += kAT) {
    const int j = idx / (k + 1), r = idx - j * (k + 1);
    const double res = (r == 0 ? beta : 0.0) - hy[r];
    Hbar[(size_t)j * ldh + r] = res * zb[j] - hz[r] * ys[j];
  }
  double p = 0.0;
  for (int j = tid; j < k; j += kAT) p = fma(zb[j], ys[j], p);
  p = group_sum<kWave>(p);
  if ((tid & (kWave - 1)) == 0) red[tid / kWave] = p;
  __syncthreads();
  if (tid == 0) {
    double zy = 0.0;
    for (int i = 0; i < kAT / kWave; ++i) zy += red[i];
    scal[0] = hz[0];
    scal[1] = -2.0 * lam * zy;
    *fail = s_bad;
  }
}

struct SideArgs {
  const double* part;  // dots of bbar_{p+1} with b_1..b_{p+1} (nchunks x (p+1))
  int nchunks;
  int p;
  int has_next;            // b_{p+1} exists (else vt = 0 and no corr_{p+1})
  const double* pivval;    // pivot entry of b_{p+1}
  const double* pivbar;    // its direct adjoint, or nullptr
  const double* cbar;      // direct adjoints of c_1..c_p, or nullptr
  const void* Tp;          // packed rows: row i holds b_j(piv_i), j < i (wp)
  double* alpha;           // out: 1 / pivval (0 without b_{p+1})
  double* corr;            // out: corr_1..corr_{p+1}
};

// The coefficient adjoints of one half-iteration.  All threads reduce the
// partial dot products (a fixed split of the chunks, added in a fixed
// order) and stage the triangle (tri, tri_cap entries of LDS; rows beyond it
// are read from memory); then one wavefront runs the triangular recurrence
// for corr_j, one pivot row per step: lane l holds j = l, l + 64, ..., and
// corr_i, final once the rows below i are folded in, is broadcast from its
// lane by readlane.  Writes corr_0..corr_p and 1/pivot, and ends with a
// barrier.  red: 4 rows of red_ld doubles of LDS.
template <typename T>
__device__ void side_solve(const SideArgs& a, double* tri, int64_t tri_cap, double* red,
                           int red_ld, double* corr, double* alpha_out) {
  const int tid = threadIdx.x, p = a.p;
  const int ncol = a.has_next ? p + 1 : 0;
  const T* Tp = static_cast<const T*>(a.Tp);
  const int64_t ntri = tri_row(p + 1);  // rows 0..p
  const bool in_lds = ntri <= tri_cap;
  if (in_lds)
    for (int64_t e = tid; e < ntri; e += kAT) tri[e] = static_cast<double>(Tp[e]);
  const int nsplit = ncol <= 64 ? 4 : (ncol <= 128 ? 2 : 1);
  if (ncol > 0) {
    const int span = kAT / nsplit, part_i = tid / span;
    for (int j = tid % span; j < ncol; j += span) {
      double t = 0.0;
      for (int c = part_i; c < a.nchunks; c += nsplit) t += a.part[(size_t)c * ncol + j];
      red[part_i * red_ld + j] = t;
    }
  }
  __syncthreads();
  if (tid < kWave) {
    const int lane = tid;
    auto dot = [&](int j) {
      double t = 0.0;
      for (int i = 0; i < nsplit; ++i) t += red[i * red_ld + j];
      return t;
    };
    double alpha = 0.0, cp = 0.0;
    if (a.has_next) {
      alpha = 1.0 / *a.pivval;
      cp = (a.pivbar ? *a.pivbar : 0.0) - dot(p) * alpha;
    }
    constexpr int kQ = kMaxIter / kWave;
    double acc[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int j = lane + q * kWave;
      acc[q] = 0.0;
      if (j < p) acc[q] = (a.cbar ? a.cbar[j] : 0.0) - (a.has_next ? dot(j) * alpha : 0.0);
    }
    for (int i = p; i >= 1; --i) {
      double ci = cp;
      if (i < p) {
        double src = acc[0];
#pragma unroll
        for (int q = 1; q < kQ; ++q)
          if (q == (i >> 6)) src = acc[q];
        ci = readlane_d(src, i & (kWave - 1));
      }
      if ((i < p || a.has_next) && ci != 0.0) {
        const int64_t row = tri_row(i);
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const int j = lane + q * kWave;
          if (j < i) {
            const double t = in_lds ? tri[row + j] : static_cast<double>(Tp[row + j]);
            acc[q] = fma(-ci, t, acc[q]);
          }
        }
      }
    }
    if (lane == 0) {
      *alpha_out = alpha;
      corr[p] = cp;
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int j = lane + q * kWave;
      if (j < p) corr[j] = acc[q];
    }
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kAT) void k_adj_side(SideArgs a) {
  __shared__ double tri[kTriCap];
  __shared__ double red[4 * (kMaxIter + 2)];
  side_solve<T>(a, tri, kTriCap, red, kMaxIter + 2, a.corr, a.alpha);
}

// Streaming part of one half-iteration, with the pivot-row terms folded in:
//     out(r)     = vt(r) + corr_i                 (r = piv_i, i <= top)
//     Bbar(r, j) -= c_j (vt(r) + [j < i] corr_i)  (j < p)
// with vt = alpha (v1 + v2) and inv[r] the pivot position of row r (-1 if
// none; positions above top carry no term in this half-iteration).
template <typename T>
__global__ __launch_bounds__(kAT) void k_adj_update(
    int64_t len, int p, int top, const double* __restrict__ alpha_p,
    const T* __restrict__ v1, const T* __restrict__ v2, const double* __restrict__ coef,
    const double* __restrict__ corr, const int* __restrict__ inv, T* __restrict__ Bbar,
    int64_t ldb, T* __restrict__ out) {
  __shared__ double sc[kMaxIter], scr[kMaxIter + 2];
  for (int j = threadIdx.x; j < p; j += kAT) sc[j] = coef[j];
  for (int j = threadIdx.x; j <= top; j += kAT) scr[j] = corr[j];
  __syncthreads();
  const double alpha = *alpha_p;
  for (int64_t r = (int64_t)blockIdx.x * kAT + threadIdx.x; r < len;
       r += (int64_t)gridDim.x * kAT) {
    double v = 0.0;
    if (v1) v = static_cast<double>(v1[r]);
    if (v2) v += static_cast<double>(v2[r]);
    const double vt = alpha * v;
    const int pi = inv[r];
    const double cr = (pi >= 0 && pi <= top) ? scr[pi] : 0.0;
    out[r] = static_cast<T>(vt + cr);
    // eight columns at a time: their loads are issued together before the
    // stores (stores to Bbar could otherwise alias the next column's load)
    constexpr int kU = 8;
    for (int j0 = 0; j0 < p; j0 += kU) {
      T old[kU];
#pragma unroll
      for (int q = 0; q < kU; ++q)
        if (j0 + q < p) old[q] = Bbar[(int64_t)(j0 + q) * ldb + r];
#pragma unroll
      for (int q = 0; q < kU; ++q) {
        const int j = j0 + q;
        if (j < p) {
          const double u = (j < pi) ? vt + cr : vt;
          Bbar[(int64_t)j * ldb + r] = static_cast<T>(fma(-sc[j], u, static_cast<double>(old[q])));
        }
      }
    }
  }
}

// k_adj_side and k_adj_update in one launch for small p: every block forms
// the coefficient adjoints itself (the same sums in the same order, so all
// blocks hold bitwise the same values) and then streams its rows; no block
// waits for another.  Dynamic LDS: fused_lds_doubles(p).
__host__ __device__ inline int64_t fused_lds_doubles(int p) {
  return tri_row(p + 1) + 4 * (int64_t)(p + 2) + (p + 2) + p;
}
constexpr int kFusedMaxP = 64;

template <typename T>
__global__ __launch_bounds__(kAT) void k_adj_side_update(
    SideArgs a, int64_t len, int top, const T* __restrict__ v1, const T* __restrict__ v2,
    const double* __restrict__ coef, const int* __restrict__ inv, T* __restrict__ Bbar,
    int64_t ldb, T* __restrict__ out) {
  extern __shared__ double dyn[];
  __shared__ double s_alpha;
  const int p = a.p;
  double* tri = dyn;
  double* red = tri + tri_row(p + 1);
  double* scr = red + 4 * (p + 2);
  double* sc = scr + (p + 2);
  for (int j = threadIdx.x; j < p; j += kAT) sc[j] = coef[j];
  side_solve<T>(a, tri, tri_row(p + 1), red, p + 2, scr, &s_alpha);
  const double alpha = s_alpha;
  for (int64_t r = (int64_t)blockIdx.x * kAT + threadIdx.x; r < len;
       r += (int64_t)gridDim.x * kAT) {
    double v = 0.0;
    if (v1) v = static_cast<double>(v1[r]);
    if (v2) v += static_cast<double>(v2[r]);
    const double vt = alpha * v;
    const int pi = inv[r];
    const double cr = (pi >= 0 && pi <= top) ? scr[pi] : 0.0;
    out[r] = static_cast<T>(vt + cr);
    constexpr int kU = 8;
    for (int j0 = 0; j0 < p; j0 += kU) {
      T old[kU];
#pragma unroll
      for (int q = 0; q < kU; ++q)
        if (j0 + q < p) old[q] = Bbar[(int64_t)(j0 + q) * ldb + r];
#pragma unroll
      for (int q = 0; q < kU; ++q) {
        const int j = j0 + q;
        if (j < p) {
          const double u = (j < pi) ? vt + cr : vt;
          Bbar[(int64_t)j * ldb + r] = static_cast<T>(fma(-sc[j], u, static_cast<double>(old[q])));
        }
      }
    }
  }
}

// inv[piv[i]] = i for the count pivots of a side (inv cleared to -1 first).
__global__ void k_inv(const int* __restrict__ piv, int count, int* __restrict__ inv) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    inv[piv[i]] = i;
}

// Lbar(:, j) = xbar y_j for j < k.
template <typename T>
__global__ __launch_bounds__(kAT) void k_adj_init_l(int64_t n, int k, const T* __restrict__ xbar,
                                                   const double* __restrict__ y,
                                                   T* __restrict__ Lbar, int64_t ldl) {
  for (int64_t r = (int64_t)blockIdx.x * kAT + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * kAT) {
    const double xb = static_cast<double>(xbar[r]);
    for (int j = 0; j < k; ++j) Lbar[(int64_t)j * ldl + r] = static_cast<T>(xb * y[j]);
  }
}


int stream_grid(int64_t len) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((len + kAT - 1) / kAT, 4096)));
}

}  // namespace

size_t adjoint_part_doubles(int K, int64_t maxlen) {
  return (size_t)dot_chunks(maxlen) * (K + 2);
}

template <typename T>
int run_vjp(const VjpArgs& v, hipStream_t s) {
  const int k = v.k, K = v.K;
  const T* L = static_cast<const T*>(v.L);
  const T* D = static_cast<const T*>(v.D);
  T* Lbar = static_cast<T*>(v.Lbar);
  T* Dbar = static_cast<T*>(v.Dbar);
  T* um = static_cast<T*>(v.um);
  T* un = static_cast<T*>(v.un);
  T* pm = static_cast<T*>(v.pm);
  T* pn = static_cast<T*>(v.pn);
  const int ldh = K + 1;
  auto dots = [&](const T* B, int64_t rs, int64_t cs, int64_t len, int ncol, const T* v1,
                  const T* v2) {
    const int ch = dot_chunks(len);
    dim3 grid(ch, (ncol + kDotCols - 1) / kDotCols);
    k_dots<T><<<grid, kAT, 0, s>>>(B, rs, cs, len, ncol, v1, v2, v.part);
    return ch;
  };

  // the coefficient adjoints, then the streaming update of one half-iteration
  auto side_update = [&](const SideArgs& a, int64_t len, int top, const T* v1, const T* v2,
                         const double* coef, const int* inv, T* Bbar, int64_t ldb, T* out) {
    if (a.p <= kFusedMaxP) {
      k_adj_side_update<T><<<stream_grid(len), kAT, sizeof(double) * fused_lds_doubles(a.p), s>>>(
          a, len, top, v1, v2, coef, inv, Bbar, ldb, out);
    } else {
      k_adj_side<T><<<1, kAT, 0, s>>>(a);
      k_adj_update<T><<<stream_grid(len), kAT, 0, s>>>(len, a.p, top, a.alpha, v1, v2, coef,
                                                       a.corr, inv, Bbar, ldb, out);
    }
  };

  launch_fill<T>(Dbar, T(0), v.ldd * (int64_t)(K + 1), s);
  launch_fill<int>(v.inv_t, -1, v.m, s);
  launch_fill<int>(v.inv_g, -1, v.n, s);
  k_inv<<<1, kAT, 0, s>>>(v.piv_t, v.n_d, v.inv_t);
  k_inv<<<1, kAT, 0, s>>>(v.piv_g, v.n_l, v.inv_g);
  k_adj_init_l<T><<<stream_grid(v.n), kAT, 0, s>>>(v.n, k, static_cast<const T*>(v.xbar),
                                                   v.Y + (size_t)(k - 1) * K, Lbar, v.ldl);
  int nch = dots(L, v.rsL, v.csL, v.n, k, static_cast<const T*>(v.xbar), nullptr);
  k_adj_projected<<<1, kAT, 0, s>>>(v.H, ldh, k, v.Y + (size_t)(k - 1) * K, v.lam + (k - 1),
                                    v.st, v.part, nch, v.M, v.Hbar, v.scal, v.fail);
  const T* pm_in = nullptr;  // A qbar_0 of the l-side just reversed (adds to dbar)
  for (int kk = k; kk >= 1; --kk) {
    // d-side of iteration kk: b = d, p = kk, c = H(1:kk, kk), pivot H(kk+1, kk)
    {
      SideArgs a{};
      a.p = kk;
      a.has_next = (kk + 1 <= v.n_d) ? 1 : 0;
      const T* v1 = Dbar + (int64_t)kk * v.ldd;
      a.nchunks = a.has_next ? dots(D, v.rsD, v.csD, v.m, kk + 1, v1, pm_in) : 0;
      a.part = v.part;
      a.pivval = v.H + (size_t)(kk - 1) * ldh + kk;
      a.pivbar = v.Hbar + (size_t)(kk - 1) * ldh + kk;
      a.cbar = v.Hbar + (size_t)(kk - 1) * ldh;
      a.Tp = v.TD;
      a.alpha = v.scal + 2;
      a.corr = v.corr;
      side_update(a, v.m, a.has_next ? kk : kk - 1, v1, pm_in, v.H + (size_t)(kk - 1) * ldh,
                  v.inv_t, Dbar, v.ldd, um);
      op_apply(*v.op, 1, um, pn, nullptr, s);
    }
    // l-side of iteration kk: b = l, p = kk - 1, c = W(1:kk-1, kk), pivot W(kk, kk)
    {
      SideArgs a{};
      a.p = kk - 1;
      a.has_next = 1;
      const T* v1 = Lbar + (int64_t)(kk - 1) * v.ldl;
      a.nchunks = dots(L, v.rsL, v.csL, v.n, kk, v1, pn);
      a.part = v.part;
      a.pivval = v.W + (size_t)(kk - 1) * K + (kk - 1);
      a.pivbar = nullptr;
      a.cbar = nullptr;
      a.Tp = v.TL;
      a.alpha = v.scal + 2;
      a.corr = v.corr;
      side_update(a, v.n, kk - 1, v1, pn, v.W + (size_t)(kk - 1) * K, v.inv_g, Lbar, v.ldl, un);
      op_apply(*v.op, 0, un, pm, nullptr, s);
      pm_in = pm;
    }
  }
  // start: d_1 = r_0 / beta, r_0 = b - A x_0
  {
    SideArgs a{};
    a.p = 0;
    a.has_next = 1;
    const T* v1 = Dbar;
    a.nchunks = dots(D, v.rsD, v.csD, v.m, 1, v1, pm_in);
    a.part = v.part;
    a.pivval = &v.st->beta;
    a.pivbar = v.scal;  // betabar
    a.cbar = nullptr;
    a.Tp = v.TD;
    a.alpha = v.scal + 2;
    a.corr = v.corr;
    side_update(a, v.m, 0, v1, pm_in, nullptr, v.inv_t, Dbar, v.ldd, static_cast<T*>(v.bbar));
  }
  return 0;
}

template int run_vjp<double>(const VjpArgs&, hipStream_t);
template int run_vjp<float>(const VjpArgs&, hipStream_t);

}  // namespace lslu
