// The projected problem of Hybrid LSLU, in FP64 on the device.
//
// For every iteration k (one workgroup per k, all k in one launch: the basis
// does not depend on lambda, so the K projected problems are independent of
// each other and of the recurrence) this kernel computes lambda_k, y_k and
// Ghat(k) for the (k+1) x k Hessenberg matrix H = H_{k+1,k} and beta.
//
//  1. Householder bidiagonalisation H = P [B; 0] Q^T with B upper bidiagonal
//     (diagonal d, superdiagonal e), g = P^T beta e_1 (k+1 entries).  The
//     right reflectors are kept for the back-transformation y = Q z.
//  2. The parameter rules use the residual/trace forms that define them
//     (Section 3.2.1, eq. gcv1 and eq. wgcv_projected1; eq. stop1 for Ghat):
//        ||(I - H H_lam^+) beta e_1||^2 = ||g_1:k - B z_lam||^2 + g_{k+1}^2
//        trace(H H_lam^+)               = k - lam^2 trace((B^T B + lam^2 I)^-1)
//     with z_lam = argmin ||g_1:k - B z||^2 + lam^2 ||z||^2 computed by Elden's
//     O(k) Givens elimination of [B; lam I] into an upper bidiagonal R, and
//     trace((B^T B + lam^2 I)^-1) = ||R^-1||_F^2 from a recurrence of positive
//     terms.  One thread per grid value of lambda.
//  3. sigma_1 (for the relative grid and reports) and sigma_min by parallel
//     multisection of Sturm counts of B^T B (both searches side by side).
//  4. y_k = Q z_{lambda_k}.
// In exact arithmetic these equal the SVD expressions of Section 3.2.1
// (eq. gcv2, the SVD form of weighted GCV, eq. stop2 and the filtered SVD
// solution for y).
#include <algorithm>
#include <cfloat>
#include <climits>

#include "device_common.hpp"

namespace lslu {

namespace {

constexpr int kPT = 1024;           // threads per projected problem
constexpr int kSP = 512;            // of which run the eigenvalue-count searches
constexpr int kBL = 8;              // lanes per column (row) of a reflector update
constexpr int kSectRounds = 9;      // multisection rounds (8 bits each)
size_t g_static_lds = 32 * 1024;  // static LDS of k_projected, read at init

// Working matrix A ((k+1) x k, leading dimension k+1).
__host__ __device__ inline size_t proj_a_doubles(int k) { return (size_t)(k + 1) * k; }
// Global scratch per problem: A (when not in LDS) and 3 vectors for each of
// G grid values.
__host__ __device__ inline size_t proj_scratch_per_k(int K, int G) {
  return proj_a_doubles(K) + (size_t)3 * K * G;
}

__device__ inline double wave_sum_d(double v) { return group_sum<kWave>(v); }

// Number of eigenvalues of the tridiagonal T = B^T B (diagonal a, squared
// off-diagonal b2) below x, from the signs of its LDL^T pivots.  The
// quotient b2 / q is b2 times 1/q from the hardware reciprocal refined by two
// Newton steps (a few ulps, as the count's usual error analysis allows, at
// about half the latency of a correctly rounded division).
__device__ inline int sturm_count(const double* a, const double* b2, int k,
                                  double x, double pivmin) {
  double q = a[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < k; ++i) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(fma(-q, r, 1.0), r, r);
    r = fma(fma(-q, r, 1.0), r, r);
    q = (a[i] - x) - b2[i - 1] * r;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// Elden: Givens rotations reduce [B; lam I] with right-hand side [g; 0] to an
// upper bidiagonal R (diagonal rho, superdiagonal f) with right-hand side q.
// Each step eliminates the damping entry against row i of B, then merges the
// fill it leaves in column i+1 into the next damping row.  Returns
// trace((B^T B + lam^2 I)^-1) = ||R^-1||_F^2 (0 when lam == 0).
__device__ inline double elden_forward(const double* d, const double* e,
                                       const double* g, int k, double lam,
                                       double* rho, double* f, double* q) {
  double mu = lam, h = 0.0, S = 1.0, tr = 0.0, fprev = 0.0, rprev = 1.0;
  for (int i = 0; i < k; ++i) {
    const double di = d[i];
    const double ei = (i + 1 < k) ? e[i] : 0.0;
    double c = 1.0, s = 0.0, r = di;
    if (mu != 0.0) {
      r = sqrt(di * di + mu * mu);
      c = di / r;
      s = mu / r;
    }
    const double fi = c * ei;
    rho[i] = r;
    f[i] = fi;
    q[i] = c * g[i] + s * h;
    const double hp = c * h - s * g[i];
    if (lam != 0.0) {
      if (i > 0) {
        const double a = fprev / rprev;
        S = 1.0 + a * a * S;
      }
      tr += S / (r * r);
    }
    fprev = fi;
    rprev = r;
    if (i + 1 < k) {
      const double fill = -s * ei;
      const double mup = sqrt(lam * lam + fill * fill);
      if (mup != 0.0) {
        h = (fill / mup) * hp;
        mu = mup;
      } else {
        h = 0.0;
        mu = 0.0;
      }
    }
  }
  return tr;
}

// Back substitution R z = q; returns ||g - B z||^2 (z stored when non-null).
// Rows go in blocks of 8 whose operands are all loaded first (the factors may
// sit in global scratch: one round trip per block, not per row).
__device__ inline double elden_backward(const double* d, const double* e,
                                        const double* g, int k,
                                        const double* rho, const double* f,
                                        const double* q, double* z) {
  constexpr int kB = 8;
  double znext = 0.0, mis = 0.0;
  for (int hi = k - 1; hi >= 0; hi -= kB) {
    double qb[kB], fb[kB], rb[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int i = hi - u;
      const int ic = i >= 0 ? i : 0;
      qb[u] = q[ic];
      fb[u] = f[ic];
      rb[u] = rho[ic];
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int i = hi - u;
      if (i < 0) break;
      double zi, ri;
      if (i + 1 < k) {
        zi = (qb[u] - fb[u] * znext) / rb[u];
        ri = g[i] - d[i] * zi - e[i] * znext;
      } else {
        zi = qb[u] / rb[u];
        ri = g[i] - d[i] * zi;
      }
      mis += ri * ri;
      if (z) z[i] = zi;
      znext = zi;
    }
  }
  return mis;
}

// y = Q z in place, by one wavefront: the right reflectors j = k-3..0 with
// vectors [1 at j+1; A(j, j+2:k-1)] and factors taur[j].
template <typename COL>
__device__ inline void apply_q(COL colp, const double* taur, int k, double* z, int lane) {
  for (int j = k - 3; j >= 0; --j) {
    const double tau = taur[j];
    if (tau == 0.0) continue;
    double w = 0.0;
    for (int c = j + 1 + lane; c < k; c += kWave) {
      const double u = (c == j + 1) ? 1.0 : colp(c)[j];
      w = fma(u, z[c], w);
    }
    w = wave_sum_d(w) * tau;
    for (int c = j + 1 + lane; c < k; c += kWave) {
      const double u = (c == j + 1) ? 1.0 : colp(c)[j];
      z[c] = fma(-w, u, z[c]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Dynamic LDS: [A when a_in_lds][per-grid-value Elden scratch when l_in_lds],
// sized for the largest k of the launch (k_last).  a_split (with a_in_lds
// false): A's first cs columns live in the problem's global scratch and the
// others in LDS (a_room bytes), cs as small as the room allows.  Column c is
// last changed by step c of the bidiagonalisation, so the global columns
// are only touched in the first cs steps (and by y = Q z at the end).
template <bool a_in_lds, bool l_in_lds, bool a_split>
__global__ __launch_bounds__(kPT) void k_projected(
    const double* __restrict__ H, const DevState* __restrict__ st,
    ProjParams p, int k_first, int k_last, double* __restrict__ Y,
    double* __restrict__ lam_out, int* __restrict__ lam_idx_out,
    double* __restrict__ ghat_out, double* __restrict__ sep_out,
    double* __restrict__ smax_out, double* __restrict__ smin_out,
    double* __restrict__ scratch, size_t a_room) {
  extern __shared__ double lds_a[];
  __shared__ double g[kMaxIter + 1], vb[kMaxIter + 1], taur[kMaxIter];
  __shared__ double d[kMaxIter], e[kMaxIter], ta[kMaxIter], tb[kMaxIter];
  __shared__ double zy[kMaxIter], gv[kMaxGrid];
  __shared__ double s_tau, s_sig1, s_lam, s_sep;
  __shared__ int s_lidx;

  const int k = k_first + blockIdx.x;
  if (k > st->k_done) return;
  const int K = p.K;
  const double beta = st->beta;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int lda = k + 1;
  double* blk = scratch + (size_t)(k - 1) * proj_scratch_per_k(K, p.grid_slots);
  double* A;
  if constexpr (a_in_lds) A = lds_a; else A = blk;
  int cs = 0;  // a_split: columns 0..cs-1 in global scratch
  if constexpr (a_split) {
    const int lds_cols = static_cast<int>(a_room / (sizeof(double) * (size_t)lda));
    cs = k > lds_cols ? k - lds_cols : 0;
  }
  // column c of the working matrix
  auto colp = [&](int c) -> double* {
    if constexpr (a_split)
      return c < cs ? blk + (size_t)c * lda : lds_a + (size_t)(c - cs) * lda;
    else
      return A + (size_t)c * lda;
  };
  double* lamscr;  // 3*K doubles per grid value
  if constexpr (l_in_lds)
    lamscr = lds_a + (a_in_lds ? proj_a_doubles(k_last) : 0);
  else
    lamscr = blk + proj_a_doubles(K);

  // 1. Load H (column-major, leading dimension K+1) into A; g = beta e_1.
  for (int idx = tid; idx < (k + 1) * k; idx += kPT) {
    const int c = idx / (k + 1), r = idx - c * (k + 1);
    colp(c)[r] = H[(size_t)c * (K + 1) + r];
  }
  for (int r = tid; r <= k; r += kPT) g[r] = (r == 0) ? beta : 0.0;
  __syncthreads();

  // 2. Householder bidiagonalisation (upper bidiagonal B).
  for (int j = 0; j < k; ++j) {
    // Left reflector annihilating A(j+1:k, j).
    if (wv == 0) {
      double s2 = 0.0;
      for (int r = j + 1 + lane; r <= k; r += kWave) {
        const double x = colp(j)[r];
        s2 = fma(x, x, s2);
      }
      s2 = wave_sum_d(s2);
      const double alpha = colp(j)[j];
      double tau = 0.0, bet = alpha, scal = 0.0;
      if (s2 != 0.0) {
        bet = -copysign(sqrt(alpha * alpha + s2), alpha);
        tau = (bet - alpha) / bet;
        scal = 1.0 / (alpha - bet);
      }
      for (int r = j + 1 + lane; r <= k; r += kWave)
        vb[r - j] = colp(j)[r] * scal;
      if (lane == 0) {
        vb[0] = 1.0;
        s_tau = tau;
        colp(j)[j] = bet;
      }
    }
    __syncthreads();
    {
      // kBL lanes per column: each sums its rows j + li, j + li + kBL, ...,
      // the group adds the partial sums (fixed DPP order), then updates them.
      const double tau = s_tau;
      const int ncol = k - 1 - j;  // columns j+1..k-1, then g
      if (tau != 0.0) {
        const int li = tid % kBL;
        for (int t = tid / kBL; t <= ncol; t += kPT / kBL) {
          double* col = (t < ncol) ? colp(j + 1 + t) : g;
          double d = 0.0;
          for (int r = j + li; r <= k; r += kBL) d = fma(vb[r - j], col[r], d);
          const double w = tau * group_sum<kBL>(d);
          for (int r = j + li; r <= k; r += kBL) col[r] = fma(-w, vb[r - j], col[r]);
        }
      }
    }
    __syncthreads();
    if (j + 2 >= k) continue;  // at most one entry right of the diagonal
    // Right reflector annihilating A(j, j+2:k-1).
    if (wv == 0) {
      double s2 = 0.0;
      for (int c = j + 2 + lane; c < k; c += kWave) {
        const double x = colp(c)[j];
        s2 = fma(x, x, s2);
      }
      s2 = wave_sum_d(s2);
      const double alpha = colp(j + 1)[j];
      double tau = 0.0, bet = alpha, scal = 0.0;
      if (s2 != 0.0) {
        bet = -copysign(sqrt(alpha * alpha + s2), alpha);
        tau = (bet - alpha) / bet;
        scal = 1.0 / (alpha - bet);
      }
      for (int c = j + 2 + lane; c < k; c += kWave) {
        double* cc = colp(c);
        const double v = cc[j] * scal;
        vb[c - j - 1] = v;
        cc[j] = v;  // kept for y = Q z
      }
      if (lane == 0) {
        vb[0] = 1.0;
        s_tau = tau;
        taur[j] = tau;
        colp(j + 1)[j] = bet;
      }
    }
    __syncthreads();
    {
      const double tau = s_tau;
      const int nrow = k - j;  // rows j+1..k
      const int nc = k - 1 - j;
      if (tau != 0.0) {
        const int li = tid % kBL;
        for (int t = tid / kBL; t < nrow; t += kPT / kBL) {
          const int r = j + 1 + t;
          double d = 0.0;  // row r over columns j+1 .. k-1
          for (int c = li; c < nc; c += kBL) d = fma(vb[c], colp(j + 1 + c)[r], d);
          const double w = tau * group_sum<kBL>(d);
          for (int c = li; c < nc; c += kBL) {
            double* cp = colp(j + 1 + c) + r;
            *cp = fma(-w, vb[c], *cp);
          }
        }
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < k; i += kPT) {
    d[i] = colp(i)[i];
    e[i] = (i + 1 < k) ? colp(i + 1)[i] : 0.0;
  }
  __syncthreads();
  for (int i = tid; i < k; i += kPT) {  // T = B^T B
    ta[i] = d[i] * d[i] + (i > 0 ? e[i - 1] * e[i - 1] : 0.0);
    tb[i] = (i + 1 < k) ? d[i] * e[i] : 0.0;
  }
  __syncthreads();
  const double gk1 = g[k];  // = +-beta c_{k+1}

  // 3. sigma_1^2 and sigma_min^2 by multisection of the eigenvalue count,
  // both at once: the first kSP / 2 threads bracket the first x with count k
  // (the largest eigenvalue), the next kSP / 2 the first x with count 1 (the
  // smallest), kSP / 2 + 1 intervals per round each (more threads would
  // only share the vector units the counts are bound by).
  double pivmin = DBL_MIN, gers = 0.0;
  for (int i = 0; i < k; ++i) {
    const double bl = i > 0 ? fabs(tb[i - 1]) : 0.0, br = fabs(tb[i]);
    gers = fmax(gers, ta[i] + bl + br);
    pivmin = fmax(pivmin, DBL_MIN * tb[i] * tb[i]);
  }
  __syncthreads();  // every thread has read tb: square it in place
  for (int i = tid; i < k; i += kPT) tb[i] = tb[i] * tb[i];
  {
    constexpr int kHP = kSP / 2;
    __shared__ double s_lo2[2], s_hi2[2];
    __shared__ int s_first2[2];
    const int which = tid < kSP ? tid / kHP : 0, ht = tid - which * kHP;
    const int target = which == 0 ? k : 1;
    if (tid < 2) {
      s_lo2[tid] = 0.0;
      s_hi2[tid] = gers * (1.0 + 4.0 * DBL_EPSILON) + pivmin;
    }
    __syncthreads();
    for (int rd = 0; rd < kSectRounds; ++rd) {
      const double lo = s_lo2[which], hi = s_hi2[which];
      const double step = (hi - lo) / (double)(kHP + 1);
      const int cnt = tid < kSP ? sturm_count(ta, tb, k, lo + step * (ht + 1), pivmin) : 0;
      if (tid < 2) s_first2[tid] = kHP;
      __syncthreads();
      // the first point whose count reaches the target brackets it (the last
      // interval when none does); a minimum, so the choice is deterministic
      if (tid < kSP && cnt >= target) atomicMin(&s_first2[which], ht);
      __syncthreads();
      if (tid < 2) {
        const int t = s_first2[tid];
        const double l0 = s_lo2[tid], h0 = s_hi2[tid];
        const double st2 = (h0 - l0) / (double)(kHP + 1);
        s_lo2[tid] = (t == 0) ? l0 : l0 + st2 * t;
        s_hi2[tid] = (t == kHP) ? h0 : l0 + st2 * (t + 1);
      }
      __syncthreads();
    }
    if (tid == 0) {
      const double v1 = sqrt(0.5 * (s_lo2[0] + s_hi2[0]));
      smax_out[k - 1] = v1;
      s_sig1 = v1;
      smin_out[k - 1] = sqrt(0.5 * (s_lo2[1] + s_hi2[1]));
    }
    __syncthreads();
  }
  const double sig1 = s_sig1;

  // 4. Parameter choice on the grid: one thread per grid value.
  const int reg = p.reg;
  if (reg == kWGCV || reg == kGCV) {
    const double omega =
        (reg == kGCV) ? 1.0 : (p.omega > 0.0 ? p.omega : (double)(k + 1) / p.m);
    for (int gi = tid; gi < p.n_grid; gi += kPT) {
      const double lam = p.grid_relative ? p.grid[gi] * sig1 : p.grid[gi];
      double* rho = lamscr + (size_t)gi * 3 * K;
      double* ff = rho + K;
      double* qq = ff + K;
      const double tr = elden_forward(d, e, g, k, lam, rho, ff, qq);
      const double mis = elden_backward(d, e, g, k, rho, ff, qq, qq);  // z over q
      ta[gi] = mis;  // kept for the chosen value (T is no longer needed)
      tb[gi] = tr;
      const double num = (double)k * (mis + gk1 * gk1);
      // trace(I - omega H H_lam^+) = (k+1) - omega (k - lam^2 tr)
      const double den = (double)(k + 1) - omega * ((double)k - lam * lam * tr);
      gv[gi] = num / (den * den);
    }
    __syncthreads();
    if (tid == 0) {
      int bi = 0;
      for (int gi = 1; gi < p.n_grid; ++gi)
        if (gv[gi] < gv[bi]) bi = gi;
      double g2 = INFINITY;
      for (int gi = 0; gi < p.n_grid; ++gi)
        if (gi != bi && gv[gi] < g2) g2 = gv[gi];
      double sep = INFINITY;
      if (p.n_grid > 1)
        sep = gv[bi] > 0.0 ? (g2 - gv[bi]) / gv[bi] : (g2 > 0.0 ? INFINITY : 0.0);
      int use = bi;
      if (p.replay_lambda && p.replay_lambda[k - 1] >= 0) use = p.replay_lambda[k - 1];
      s_lam = p.grid_relative ? p.grid[use] * sig1 : p.grid[use];
      s_lidx = use;
      s_sep = sep;
    }
  } else if (reg == kOptimal) {
    // z_lam for every grid value (one thread each, z over q in its slot),
    // then y_lam = Q z_lam and ||x_0 + L_k y_lam - x_true|| from the Gram
    // matrix of [L, x_true - x_0] (one wavefront per grid value).
    for (int gi = tid; gi < p.n_grid; gi += kPT) {
      const double lam = p.grid_relative ? p.grid[gi] * sig1 : p.grid[gi];
      double* rho = lamscr + (size_t)gi * 3 * K;
      double* ff = rho + K;
      double* qq = ff + K;
      elden_forward(d, e, g, k, lam, rho, ff, qq);
      elden_backward(d, e, g, k, rho, ff, qq, qq);
    }
    __syncthreads();
    const int ldg = K + 1;
    const double e0 = p.gram[(size_t)K * ldg + K];
    for (int gi = wv; gi < p.n_grid; gi += kPT / kWave) {
      double* y = lamscr + (size_t)gi * 3 * K + 2 * K;
      apply_q(colp, taur, k, y, lane);
      // y^T G y - 2 y^T h, h = G(0:k-1, K)
      double part = 0.0;
      for (int i = lane; i < k; i += kWave) {
        const double* Gi = p.gram + (size_t)i * ldg;
        double t = 0.0;
        for (int j = 0; j < k; ++j) t = fma(Gi[j], y[j], t);
        part = fma(y[i], t - 2.0 * Gi[K], part);
      }
      part = wave_sum_d(part);
      if (lane == 0) gv[gi] = sqrt(fmax(part + e0, 0.0));
    }
    __syncthreads();
    if (tid == 0) {
      int bi = 0;
      for (int gi = 1; gi < p.n_grid; ++gi)
        if (gv[gi] < gv[bi]) bi = gi;
      double g2 = INFINITY;
      for (int gi = 0; gi < p.n_grid; ++gi)
        if (gi != bi && gv[gi] < g2) g2 = gv[gi];
      double sep = INFINITY;
      if (p.n_grid > 1)
        sep = gv[bi] > 0.0 ? (g2 - gv[bi]) / gv[bi] : (g2 > 0.0 ? INFINITY : 0.0);
      int use = bi;
      if (p.replay_lambda && p.replay_lambda[k - 1] >= 0) use = p.replay_lambda[k - 1];
      s_lam = p.grid_relative ? p.grid[use] * sig1 : p.grid[use];
      s_lidx = use;
      s_sep = sep;
    }
  } else if (tid == 0) {
    s_lam = (reg == kFixed) ? p.lambda : 0.0;
    s_lidx = -1;
    s_sep = INFINITY;
  }
  __syncthreads();

  // 5. z for lambda_k and Ghat(k) (thread 0), then y = Q z (wavefront 0).
  // On a grid (GCV, weighted GCV) they were formed for the chosen value
  // already: its slot holds z and the factor R, ta/tb its residual and trace.
  const bool on_grid = reg == kWGCV || reg == kGCV;
  double* slot = lamscr + (size_t)(on_grid ? s_lidx : 0) * 3 * K;
  if (on_grid) {
    for (int i = tid; i < k; i += kPT) zy[i] = slot[2 * K + i];
    __syncthreads();
  }
  if (tid == 0) {
    const double lam = s_lam;
    double* rho = slot;
    double* ff = rho + K;
    double* qq = ff + K;
    double tr, mis;
    if (on_grid) {
      tr = tb[s_lidx];
      mis = ta[s_lidx];
    } else {
      tr = elden_forward(d, e, g, k, lam, rho, ff, qq);
      mis = elden_backward(d, e, g, k, rho, ff, qq, zy);
    }
    const double num = (double)p.n * (mis + gk1 * gk1);
    const double den = (double)(p.m - k) + lam * lam * tr;
    ghat_out[k - 1] = (den == 0.0) ? NAN : num / (den * den);
    lam_out[k - 1] = lam;
    lam_idx_out[k - 1] = s_lidx;
    sep_out[k - 1] = s_sep;
    if (p.dldl) {
      // dy/dlambda = -2 lambda (H^T H + lambda^2 I)^-1 y = -2 lambda Q w with
      // R^T R w = z: B^T B + lambda^2 I = R^T R for Elden's factor R (upper
      // bidiagonal: diagonal rho, superdiagonal ff); w overwrites qq.
      double* w = qq;
      if (lam == 0.0) {
        for (int i = 0; i < k; ++i) w[i] = 0.0;
      } else {
        for (int i = 0; i < k; ++i)  // R^T t = z
          w[i] = (zy[i] - (i > 0 ? ff[i - 1] * w[i - 1] : 0.0)) / rho[i];
        for (int i = k - 1; i >= 0; --i)  // R w = t
          w[i] = (w[i] - (i + 1 < k ? ff[i] * w[i + 1] : 0.0)) / rho[i];
        for (int i = 0; i < k; ++i) w[i] *= -2.0 * lam;
      }
    }
  }
  __syncthreads();
  double* dy = slot + 2 * K;  // -2 lambda Q w, when asked for
  if (wv == 0) {
    apply_q(colp, taur, k, zy, lane);
    if (p.dldl) apply_q(colp, taur, k, dy, lane);
  }
  __syncthreads();
  for (int r = tid; r < K; r += kPT)
    Y[(size_t)(k - 1) * K + r] = (r < k) ? zy[r] : 0.0;
  if (p.dldl) {
    // d/dlambda ||x_0 + L_k y - x_true||^2 = 2 (y^T G dy - h^T dy), G and h
    // the leading blocks of the Gram matrix of [L, x_true - x_0]
    const int ldg = K + 1;
    double part = 0.0;
    for (int i = tid; i < k; i += kPT) {
      const double* Gi = p.gram + (size_t)i * ldg;
      double t = 0.0;
      for (int j = 0; j < k; ++j) t = fma(Gi[j], dy[j], t);
      part = fma(zy[i], t, part);
      part = fma(-Gi[K], dy[i], part);
    }
    part = wave_sum_d(part);
    if (lane == 0) gv[wv] = part;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (int i = 0; i < kPT / kWave; ++i) tot += gv[i];
      p.dldl[k - 1] = 2.0 * tot;
    }
  }
}

}  // namespace

size_t projected_scratch_doubles(int K, int grid_slots) {
  return proj_scratch_per_k(K, grid_slots) * (size_t)K;
}

namespace {
// every variant launched by launch_projected
const void* const kProjKernels[] = {
    reinterpret_cast<const void*>(k_projected<true, true, false>),
    reinterpret_cast<const void*>(k_projected<true, false, false>),
    reinterpret_cast<const void*>(k_projected<false, false, true>)};
}  // namespace

void projected_init_attributes(size_t lds_bytes) {
  hipFuncAttributes fa{};
  size_t st = 0;
  for (const void* k : kProjKernels)
    if (hipFuncGetAttributes(&fa, k) == hipSuccess) st = std::max(st, fa.sharedSizeBytes);
  if (st > 0) g_static_lds = st;
  if (lds_bytes <= g_static_lds) return;
  const int dyn = static_cast<int>(lds_bytes - g_static_lds);
  for (const void* k : kProjKernels)
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

void launch_projected(const double* H, const DevState* st, double,
                      const ProjParams& p, double* Y, double* lam, int* lam_idx,
                      double* ghat, double* sep, double* smax, double* smin,
                      double* scratch, size_t lds_bytes, const hipStream_t* streams,
                      int nstreams) {
  // Each problem keeps its working matrix and its per-grid-value Elden
  // scratch (3 K doubles per grid value, indexed with stride K) in LDS when
  // both fit (placement 3), else the matrix in LDS and the Elden scratch in
  // its slice of global scratch (1), else as many of the matrix's last
  // columns as fit in LDS and the rest in global scratch (4).  Consecutive k
  // with the same placement share one launch sized for the largest of them.
  const size_t room = lds_bytes > g_static_lds ? lds_bytes - g_static_lds : 0;
  const int G = (p.reg == kWGCV || p.reg == kGCV || p.reg == kOptimal)
                    ? std::max(p.n_grid, 1) : 1;
  const size_t lam_bytes = sizeof(double) * 3 * (size_t)p.K * G;
  auto place = [&](int k) {
    const size_t a = proj_a_doubles(k) * sizeof(double);
    if (a + lam_bytes <= room) return 3;
    if (a <= room) return 1;
    return 4;
  };
  int k0 = 1, group = 0;
  while (k0 <= p.K) {
    const int pl = place(k0);
    int k1 = k0;
    while (k1 + 1 <= p.K && place(k1 + 1) == pl) ++k1;
    // the groups are independent (disjoint k, outputs and scratch slices)
    const hipStream_t s = streams[group++ % nstreams];
    const int nblk = k1 - k0 + 1;
    if (pl == 3) {
      const size_t dyn = proj_a_doubles(k1) * sizeof(double) + lam_bytes;
      k_projected<true, true, false><<<nblk, kPT, dyn, s>>>(H, st, p, k0, k1, Y, lam, lam_idx,
                                                            ghat, sep, smax, smin, scratch, 0);
    } else if (pl == 1) {
      const size_t dyn = proj_a_doubles(k1) * sizeof(double);
      k_projected<true, false, false><<<nblk, kPT, dyn, s>>>(H, st, p, k0, k1, Y, lam, lam_idx,
                                                             ghat, sep, smax, smin, scratch, 0);
    } else {
      k_projected<false, false, true><<<nblk, kPT, room, s>>>(H, st, p, k0, k1, Y, lam, lam_idx,
                                                              ghat, sep, smax, smin, scratch,
                                                              room);
    }
    k0 = k1 + 1;
  }
}

}  // namespace lslu
