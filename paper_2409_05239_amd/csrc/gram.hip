// The Gram matrix of C = [L_K, e] in FP64 (e = x_true - x_0), for the optimal
// parameter rule (eq. lambda, a diagnostic that needs the true solution):
// for a coefficient vector y of iteration k,
//     ||x_0 + L_k y - x_true||^2 = y^T G_k y - 2 y^T h_k + ||e||^2
// with G = L^T L and h = L^T e, the leading blocks of C^T C.  The projected
// problem then prices every grid value in O(k^2) instead of a pass over L.
// This is the only place the library forms inner products of basis vectors;
// the recurrence itself never does.
//
// Deterministic: the rows are split into fixed chunks, each (16 x 16 tile,
// chunk) pair sums its rows in order, and the chunks are added in order.
#include "device_common.hpp"

namespace lslu {

namespace {

constexpr int kGT = 16;               // tile edge
constexpr int kGThreads = kGT * kGT;  // one thread per tile entry
constexpr int kGRows = 64;            // rows staged per step

template <typename T>
__device__ inline double gram_col(const T* L, int64_t rs, int64_t cs, int nl,
                                  int K, const T* xt, const T* x0, int64_t r,
                                  int j) {
  if (j < nl) return static_cast<double>(L[r * rs + (int64_t)j * cs]);
  if (j == K) {
    const double t = static_cast<double>(xt[r]);
    return x0 ? t - static_cast<double>(x0[r]) : t;
  }
  return 0.0;  // columns not formed by this solve
}

// blockIdx.x: upper-triangular tile pair (ti <= tj); blockIdx.y: row chunk.
template <typename T>
__global__ __launch_bounds__(kGThreads) void k_gram_partial(
    const T* __restrict__ L, int64_t rs, int64_t cs, int64_t n, int K,
    const T* __restrict__ xt, const T* __restrict__ x0, int64_t chunk,
    const DevState* __restrict__ st, double* __restrict__ part) {
  __shared__ double si[kGRows][kGT + 1], sj[kGRows][kGT + 1];
  const int nt = (K + 1 + kGT - 1) / kGT;
  int p = blockIdx.x, ti = 0;
  while (p >= nt - ti) {
    p -= nt - ti;
    ++ti;
  }
  const int tj = ti + p;
  const int nl = st->n_l;
  const int tid = threadIdx.x, a = tid / kGT, b = tid % kGT;
  const int64_t r_begin = (int64_t)blockIdx.y * chunk;
  const int64_t r_end = (r_begin + chunk < n) ? r_begin + chunk : n;
  double acc = 0.0;
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGRows) {
    for (int e = tid; e < kGRows * kGT; e += kGThreads) {
      // consecutive threads along the contiguous direction of the basis
      int rr, cc;
      if (rs == 1) {
        rr = e % kGRows;
        cc = e / kGRows;
      } else {
        rr = e / kGT;
        cc = e % kGT;
      }
      const int64_t r = r0 + rr;
      const bool in = r < r_end;
      si[rr][cc] = in ? gram_col(L, rs, cs, nl, K, xt, x0, r, ti * kGT + cc) : 0.0;
      sj[rr][cc] = in ? gram_col(L, rs, cs, nl, K, xt, x0, r, tj * kGT + cc) : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < kGRows; ++r) acc = fma(si[r][a], sj[r][b], acc);
    __syncthreads();
  }
  const int i = ti * kGT + a, j = tj * kGT + b;
  if (i <= K && j <= K) part[((size_t)blockIdx.y * (K + 1) + i) * (K + 1) + j] = acc;
}

__global__ void k_gram_reduce(const double* __restrict__ part, int nchunks, int K,
                              double* __restrict__ G) {
  const int N = K + 1;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N * N;
       idx += gridDim.x * blockDim.x) {
    const int i = idx / N, j = idx - i * N;
    if (i > j) continue;  // the tile pairs hold i's tile <= j's tile
    // the entry lives in the partial of tile pair (i/16, j/16); within a
    // diagonal tile both (i,j) and (j,i) were computed, take i <= j
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[((size_t)c * N + i) * N + j];
    G[(size_t)i * N + j] = s;
    G[(size_t)j * N + i] = s;
  }
}

}  // namespace

size_t gram_scratch_doubles(int K) {
  return (size_t)(kGramChunks + 1) * (K + 1) * (K + 1);
}

template <typename T>
void launch_gram(const T* L, int64_t rs, int64_t cs, int64_t n, int K,
                 const T* x_true, const T* x0, const DevState* st,
                 double* scratch, double* G, hipStream_t s) {
  const int nt = (K + 1 + kGT - 1) / kGT;
  const int pairs = nt * (nt + 1) / 2;
  int64_t chunk = (n + kGramChunks - 1) / kGramChunks;
  chunk = (chunk + kGRows - 1) / kGRows * kGRows;
  const int nchunks = static_cast<int>((n + chunk - 1) / chunk);
  dim3 grid(pairs, nchunks);
  k_gram_partial<T><<<grid, kGThreads, 0, s>>>(L, rs, cs, n, K, x_true, x0, chunk,
                                               st, scratch);
  const int N = K + 1;
  k_gram_reduce<<<(N * N + 255) / 256, 256, 0, s>>>(scratch, nchunks, K, G);
}

template void launch_gram<double>(const double*, int64_t, int64_t, int64_t, int,
                                  const double*, const double*, const DevState*,
                                  double*, double*, hipStream_t);
template void launch_gram<float>(const float*, int64_t, int64_t, int64_t, int,
                                 const float*, const float*, const DevState*,
                                 double*, double*, hipStream_t);

}  // namespace lslu
