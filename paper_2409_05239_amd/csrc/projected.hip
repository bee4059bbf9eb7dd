// The projected problem of Hybrid LSLU, in FP64 on the device.
//
// For each iteration k (one workgroup per k, all k in one launch: the basis
// does not depend on lambda, so these solves are independent of each other
// and of the recurrence):
//
//   * SVD of H_{k+1,k} = U Sigma V^T by one-sided Jacobi applied to the
//     columns of M = H^T (k rows, k+1 columns): right rotations J make the
//     columns of M J orthogonal, so J = U and the columns of M J are
//     sigma_i v_i (one of them vanishes).  Only the first row of J is kept:
//     c = U^T e_1 (Section 3.2.1, eq. gcv2).
//   * lambda_k by the chosen rule on the grid: weighted GCV with omega =
//     (k+1)/m, GCV (omega = 1), a fixed value or none (Section 3.2.1);
//   * y_k = beta sum_i sigma_i c_i / (sigma_i^2 + lambda^2) v_i (eq. TSP
//     solved through the SVD, Section 3.2.1 eq. 4);
//   * Ghat(k) (eq. stop2).
//
// Jacobi pairs follow a round-robin tournament; each wavefront rotates one
// disjoint pair at a time.  Everything is in a fixed order, so results do not
// depend on timing.
#include <cfloat>
#include <climits>

#include "internal.hpp"

namespace lslu {

namespace {

constexpr int kProjThreads = 256;
constexpr int kProjWaves = kProjThreads / kWave;
constexpr int kMaxSweeps = 40;

// Doubles of working storage per projected problem (sized for k = K).
__host__ __device__ inline size_t proj_per_k(int K) {
  return (size_t)K * (K + 1) + 2 * (size_t)(K + 1) + 2 * kMaxGrid + K;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Round-robin (circle method) pairing of Np (even) players, round r.
__device__ inline void rr_pair(int Np, int r, int i, int& a, int& b) {
  auto pos = [&](int x) { return x == 0 ? 0 : ((x - 1 + r) % (Np - 1)) + 1; };
  a = pos(i);
  b = pos(Np - 1 - i);
}

__global__ __launch_bounds__(kProjThreads) void k_projected(
    const double* __restrict__ H, const DevState* __restrict__ st,
    ProjParams p, double* __restrict__ Y, double* __restrict__ lam_out,
    int* __restrict__ lam_idx_out, double* __restrict__ ghat_out,
    double* __restrict__ sep_out, double* __restrict__ smax_out,
    double* __restrict__ smin_out, double* __restrict__ scratch, int use_lds) {
  extern __shared__ double lds[];
  const int k = blockIdx.x + 1;
  if (k > st->k_done) return;
  const double beta = st->beta;
  const int K = p.K;
  const int N = k + 1;        // columns of M
  const int Np = N + (N & 1); // padded to even
  double* base = use_lds ? lds : scratch + (size_t)(k - 1) * proj_per_k(K);
  double* M = base;                 // k x N, column c = row c of H
  double* f = M + (size_t)k * N;    // first row of J (length N)
  double* nrm = f + N;              // column norms (length N)
  double* gv = nrm + N;             // grid values of the rule (kMaxGrid)
  double* glam = gv + kMaxGrid;     // grid lambdas (kMaxGrid)
  double* ybuf = glam + kMaxGrid;   // y (length k)
  __shared__ int s_rot;
  __shared__ int s_order[kMaxIter + 2];
  __shared__ double s_lam;
  __shared__ int s_lidx;
  __shared__ double s_sep;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  for (int e = tid; e < k * N; e += kProjThreads) {
    const int c = e / k, r = e - c * k;  // M(r, c) = H(c, r)
    M[e] = H[(size_t)r * (K + 1) + c];
  }
  for (int c = tid; c < N; c += kProjThreads) f[c] = (c == 0) ? 1.0 : 0.0;
  __syncthreads();

  const double tol = DBL_EPSILON * sqrt((double)k);
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int r = 0; r < Np - 1; ++r) {
      for (int pi = wv; pi < Np / 2; pi += kProjWaves) {
        int a, b;
        rr_pair(Np, r, pi, a, b);
        if (a >= N || b >= N) continue;
        double* ca = M + (size_t)a * k;
        double* cb = M + (size_t)b * k;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < k; i += kWave) {
          const double x = ca[i], y = cb[i];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
        al = wave_sum_d(al);
        be = wave_sum_d(be);
        ga = wave_sum_d(ga);
        if (ga == 0.0 || al == 0.0 || be == 0.0) continue;
        if (fabs(ga) <= tol * sqrt(al) * sqrt(be)) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t);
        const double sn = cs * t;
        for (int i = lane; i < k; i += kWave) {
          const double x = ca[i], y = cb[i];
          ca[i] = cs * x - sn * y;
          cb[i] = sn * x + cs * y;
        }
        if (lane == 0) {
          const double x = f[a], y = f[b];
          f[a] = cs * x - sn * y;
          f[b] = sn * x + cs * y;
          s_rot = 1;
        }
      }
      __syncthreads();
    }
    const int rot = s_rot;
    __syncthreads();
    if (!rot) break;
  }

  // Column norms, then order the columns by decreasing norm (ties: column).
  for (int c = wv; c < N; c += kProjWaves) {
    const double* cc = M + (size_t)c * k;
    double s = 0.0;
    for (int i = lane; i < k; i += kWave) s = fma(cc[i], cc[i], s);
    s = wave_sum_d(s);
    if (lane == 0) nrm[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = tid; c < N; c += kProjThreads) {
    int rank = 0;
    const double v = nrm[c];
    for (int c2 = 0; c2 < N; ++c2) {
      const double v2 = nrm[c2];
      rank += (v2 > v) || (v2 == v && c2 < c);
    }
    s_order[rank] = c;
  }
  __syncthreads();
  const double sig1 = nrm[s_order[0]];
  const double cnull = f[s_order[k]];  // c_{k+1}

  // Parameter choice on the grid.
  const int reg = p.reg;
  if (reg == kWGCV || reg == kGCV) {
    const double omega =
        (reg == kGCV) ? 1.0 : (p.omega > 0.0 ? p.omega : (double)(k + 1) / p.m);
    for (int g = tid; g < p.n_grid; g += kProjThreads) {
      const double lam = p.grid_relative ? p.grid[g] * sig1 : p.grid[g];
      const double l2 = lam * lam;
      double num = 0.0, den = 0.0;
      for (int i = 0; i < k; ++i) {
        const int c = s_order[i];
        const double s2 = nrm[c] * nrm[c];
        const double fi = l2 / (s2 + l2);
        const double t = fi * f[c];
        num += t * t;
        den += ((1.0 - omega) * s2 + l2) / (s2 + l2);
      }
      num = (double)k * beta * beta * (num + cnull * cnull);
      den = 1.0 + den;
      gv[g] = num / (den * den);
      glam[g] = lam;
    }
    __syncthreads();
    if (tid == 0) {
      int bi = 0;
      for (int g = 1; g < p.n_grid; ++g)
        if (gv[g] < gv[bi]) bi = g;
      double g2 = INFINITY;
      for (int g = 0; g < p.n_grid; ++g)
        if (g != bi && gv[g] < g2) g2 = gv[g];
      double sep = INFINITY;
      if (p.n_grid > 1) sep = gv[bi] > 0.0 ? (g2 - gv[bi]) / gv[bi] : (g2 > 0.0 ? INFINITY : 0.0);
      int use = bi;
      if (p.replay_lambda && p.replay_lambda[k - 1] >= 0) use = p.replay_lambda[k - 1];
      s_lam = glam[use];
      s_lidx = use;
      s_sep = sep;
    }
  } else if (tid == 0) {
    s_lam = (reg == kFixed) ? p.lambda : 0.0;
    s_lidx = -1;
    s_sep = INFINITY;
  }
  __syncthreads();
  const double lam = s_lam;
  const double l2 = lam * lam;

  // y_k = beta * sum_i c_i/(sigma_i^2 + lambda^2) * (sigma_i v_i).
  for (int r = tid; r < k; r += kProjThreads) {
    double acc = 0.0;
    for (int i = 0; i < k; ++i) {
      const int c = s_order[i];
      const double s2 = nrm[c] * nrm[c];
      const double den = s2 + l2;
      if (den > 0.0) acc += (f[c] / den) * M[(size_t)c * k + r];
    }
    ybuf[r] = beta * acc;
  }
  __syncthreads();
  for (int r = tid; r < K; r += kProjThreads)
    Y[(size_t)(k - 1) * K + r] = (r < k) ? ybuf[r] : 0.0;
  if (tid == 0) {
    double num = 0.0, den = 0.0;
    for (int i = 0; i < k; ++i) {
      const int c = s_order[i];
      const double s2 = nrm[c] * nrm[c];
      const double fi = (s2 + l2 > 0.0) ? l2 / (s2 + l2) : 0.0;
      num += (fi * f[c]) * (fi * f[c]);
      den += fi;
    }
    num = (double)p.n * beta * beta * (num + cnull * cnull);
    den = (double)(p.m - k) + den;
    ghat_out[k - 1] = (den == 0.0) ? NAN : num / (den * den);
    lam_out[k - 1] = lam;
    lam_idx_out[k - 1] = s_lidx;
    sep_out[k - 1] = s_sep;
    smax_out[k - 1] = sig1;
    smin_out[k - 1] = nrm[s_order[k - 1]];
  }
}

}  // namespace

// Per-k scratch when the working set does not fit in LDS: k*(k+1) + 2(k+1)
// + 2*kMaxGrid + k doubles, bounded by the K case, times K problems.
size_t projected_scratch_doubles(int K) { return proj_per_k(K) * (size_t)K; }

void launch_projected(const double* H, const DevState* st, double,
                      const ProjParams& p, double* Y, double* lam, int* lam_idx,
                      double* ghat, double* sep, double* smax, double* smin,
                      double* scratch, size_t lds_bytes, hipStream_t s) {
  const size_t per = proj_per_k(p.K) * sizeof(double);
  const int use_lds = (lds_bytes > 0 && per <= lds_bytes) ? 1 : 0;
  k_projected<<<p.K, kProjThreads, use_lds ? per : 0, s>>>(
      H, st, p, Y, lam, lam_idx, ghat, sep, smax, smin, scratch, use_lds);
}

}  // namespace lslu
