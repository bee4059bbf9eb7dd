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
// x_k anyway), so nothing is recomputed.  Dot products are summed in FP64 by
// fixed row chunks and reduced in a fixed order: the result does not depend
// on the launch.
#include "device_common.hpp"

namespace lslu {

namespace {

constexpr int kAT = 256;          // threads per block
constexpr int kDotMaxChunks = 256;

int dot_chunks(int64_t len) {
  const int64_t c = (len + 1023) / 1024;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(kDotMaxChunks, c)));
}

// part[c * ncol + j] = sum over the rows of chunk c of (v1 + v2)(r) * B(r, j).
template <typename T>
__global__ __launch_bounds__(kAT) void k_dots(const T* __restrict__ B, int64_t rs,
                                             int64_t cs, int64_t len, int ncol,
                                             const T* __restrict__ v1,
                                             const T* __restrict__ v2, int64_t chunk,
                                             double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = (r0 + chunk < len) ? r0 + chunk : len;
  double* out = part + (size_t)blockIdx.x * ncol;
  auto vec = [&](int64_t r) {
    double v = static_cast<double>(v1[r]);
    if (v2) v += static_cast<double>(v2[r]);
    return v;
  };
  if (cs == 1) {
    // rows contiguous: one thread per column, rows in order
    for (int j = threadIdx.x; j < ncol; j += kAT) {
      double acc = 0.0;
      for (int64_t r = r0; r < r1; ++r) acc = fma(vec(r), static_cast<double>(B[r * rs + j]), acc);
      out[j] = acc;
    }
  } else {
    // columns contiguous: one wavefront per column, lanes along the rows
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int j = w; j < ncol; j += kAT / kWave) {
      double acc = 0.0;
      for (int64_t r = r0 + lane; r < r1; r += kWave)
        acc = fma(vec(r), static_cast<double>(B[r * rs + (int64_t)j * cs]), acc);
      acc = group_sum<kWave>(acc);
      if (lane == 0) out[j] = acc;
    }
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
  const int* piv;          // pivot rows piv_1..piv_{p+1}
  const void* B;           // basis b_1..b_{p+1}, working precision
  int64_t rs, cs;
  double* alpha;           // out: 1 / pivval (0 without b_{p+1})
  double* corr;            // out: corr_1..corr_{p+1}
};

// The coefficient adjoints of one half-iteration (one block): the triangular
// recurrence for corr_j, column by column (the entries b_j(piv_i), i > j, of
// one pivot row are read together).
template <typename T>
__global__ __launch_bounds__(kAT) void k_adj_side(SideArgs a) {
  __shared__ double sc[kMaxIter + 2];
  __shared__ double s_alpha;
  const int tid = threadIdx.x, p = a.p;
  const int ncol = a.has_next ? p + 1 : 0;
  const T* B = static_cast<const T*>(a.B);
  if (tid == 0) {
    double s = 0.0;
    if (a.has_next) {
      for (int c = 0; c < a.nchunks; ++c) s += a.part[(size_t)c * ncol + p];
      const double piv = *a.pivval;
      s_alpha = 1.0 / piv;
      sc[p] = (a.pivbar ? *a.pivbar : 0.0) - s / piv;
    } else {
      s_alpha = 0.0;
      sc[p] = 0.0;
    }
  }
  __syncthreads();
  const double alpha = s_alpha;
  // acc_j for j = tid, tid + kAT (p <= kMaxIter = 2 kAT at most)
  double acc[2] = {0.0, 0.0};
  for (int q = 0; q < 2; ++q) {
    const int j = tid + q * kAT;
    if (j >= p) continue;
    double d = 0.0;
    if (a.has_next)
      for (int c = 0; c < a.nchunks; ++c) d += a.part[(size_t)c * ncol + j];
    acc[q] = (a.cbar ? a.cbar[j] : 0.0) - d * alpha;
  }
  for (int i = p; i >= 1; --i) {
    // corr_i (index i) is final: fold it into every j < i
    const double ci = sc[i];
    if (i < p || a.has_next) {
      const int64_t row = a.piv[i];
      for (int q = 0; q < 2; ++q) {
        const int j = tid + q * kAT;
        if (j < i && ci != 0.0)
          acc[q] = fma(-ci, static_cast<double>(B[row * a.rs + (int64_t)j * a.cs]), acc[q]);
      }
    }
    if (tid == ((i - 1) & (kAT - 1))) sc[i - 1] = acc[(i - 1) / kAT];
    __syncthreads();
  }
  if (tid == 0) *a.alpha = alpha;
  for (int i = tid; i <= p; i += kAT) a.corr[i] = sc[i];
}

// vt = alpha (v1 + v2) into out; Bbar(:, j) -= c_j vt for j < p.
template <typename T>
__global__ __launch_bounds__(kAT) void k_adj_update(int64_t len, int p,
                                                   const double* __restrict__ alpha_p,
                                                   const T* __restrict__ v1,
                                                   const T* __restrict__ v2,
                                                   const double* __restrict__ coef,
                                                   T* __restrict__ Bbar, int64_t ldb,
                                                   T* __restrict__ out) {
  __shared__ double sc[kMaxIter];
  for (int j = threadIdx.x; j < p; j += kAT) sc[j] = coef[j];
  __syncthreads();
  const double alpha = *alpha_p;
  for (int64_t r = (int64_t)blockIdx.x * kAT + threadIdx.x; r < len;
       r += (int64_t)gridDim.x * kAT) {
    double v = 0.0;
    if (v1) v = static_cast<double>(v1[r]);
    if (v2) v += static_cast<double>(v2[r]);
    const double vt = alpha * v;
    out[r] = static_cast<T>(vt);
    for (int j = 0; j < p; ++j) {
      T* e = Bbar + (int64_t)j * ldb + r;
      *e = static_cast<T>(fma(-sc[j], vt, static_cast<double>(*e)));
    }
  }
}

// The pivot-row terms: out(piv_i) += corr_i and Bbar(piv_i, j) -= c_j corr_i
// for j < i (distinct entries, no conflicts).
template <typename T>
__global__ __launch_bounds__(kAT) void k_adj_points(int p, int has_next,
                                                   const double* __restrict__ corr,
                                                   const int* __restrict__ piv,
                                                   const double* __restrict__ coef,
                                                   T* __restrict__ Bbar, int64_t ldb,
                                                   T* __restrict__ out) {
  const int top = has_next ? p : p - 1;  // largest i with a pivot row
  for (int i = threadIdx.x; i <= top; i += kAT) {
    const int64_t row = piv[i];
    out[row] = static_cast<T>(static_cast<double>(out[row]) + corr[i]);
  }
  for (int idx = threadIdx.x; idx < (top + 1) * p; idx += kAT) {
    const int i = idx / p, j = idx - i * p;
    if (j >= i) continue;
    T* e = Bbar + (int64_t)j * ldb + piv[i];
    *e = static_cast<T>(fma(-coef[j], corr[i], static_cast<double>(*e)));
  }
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

size_t adjoint_part_doubles(int K) { return (size_t)kDotMaxChunks * (K + 2); }

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
    const int64_t chunk = (len + ch - 1) / ch;
    k_dots<T><<<ch, kAT, 0, s>>>(B, rs, cs, len, ncol, v1, v2, chunk, v.part);
    return ch;
  };

  launch_fill<T>(Dbar, T(0), v.ldd * (int64_t)(K + 1), s);
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
      a.piv = v.piv_t;
      a.B = D;
      a.rs = v.rsD;
      a.cs = v.csD;
      a.alpha = v.scal + 2;
      a.corr = v.corr;
      k_adj_side<T><<<1, kAT, 0, s>>>(a);
      const double* coef = v.H + (size_t)(kk - 1) * ldh;
      k_adj_update<T><<<stream_grid(v.m), kAT, 0, s>>>(v.m, kk, v.scal + 2, v1, pm_in, coef,
                                                       Dbar, v.ldd, um);
      k_adj_points<T><<<1, kAT, 0, s>>>(kk, a.has_next, v.corr, v.piv_t, coef, Dbar, v.ldd, um);
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
      a.piv = v.piv_g;
      a.B = L;
      a.rs = v.rsL;
      a.cs = v.csL;
      a.alpha = v.scal + 2;
      a.corr = v.corr;
      k_adj_side<T><<<1, kAT, 0, s>>>(a);
      const double* coef = v.W + (size_t)(kk - 1) * K;
      k_adj_update<T><<<stream_grid(v.n), kAT, 0, s>>>(v.n, kk - 1, v.scal + 2, v1, pn, coef,
                                                       Lbar, v.ldl, un);
      k_adj_points<T><<<1, kAT, 0, s>>>(kk - 1, 1, v.corr, v.piv_g, coef, Lbar, v.ldl, un);
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
    a.piv = v.piv_t;
    a.B = D;
    a.rs = v.rsD;
    a.cs = v.csD;
    a.alpha = v.scal + 2;
    a.corr = v.corr;
    k_adj_side<T><<<1, kAT, 0, s>>>(a);
    T* bbar = static_cast<T*>(v.bbar);
    k_adj_update<T><<<stream_grid(v.m), kAT, 0, s>>>(v.m, 0, v.scal + 2, v1, pm_in, nullptr,
                                                     Dbar, v.ldd, bbar);
    k_adj_points<T><<<1, kAT, 0, s>>>(0, 1, v.corr, v.piv_t, nullptr, Dbar, v.ldd, bbar);
  }
  return 0;
}

template int run_vjp<double>(const VjpArgs&, hipStream_t);
template int run_vjp<float>(const VjpArgs&, hipStream_t);

}  // namespace lslu
