// Iterates x_k = x_0 + L_k y_k (Algorithm 5, last step of the loop), for all
// k = 1..k_done at once: X = x_0 1^T + L Y with Y upper triangular (column k-1
// of Y holds y_k).  A dense FP64 contraction, so it runs on the matrix cores
// (v_mfma_f64_16x16x4).  Persistent: one block of 12 waves per CU stages,
// once, the part of Y its column group needs into LDS (4 x 16 operand blocks
// in the matrix core's lane order, read conflict-free), then every wave walks
// its own 16-row tiles of L with no further barrier: a step takes 4 columns
// of L (read straight from the basis one phase of 16 columns ahead of their
// use, so the wave's memory waits are on loads issued long before) and the
// matching Y blocks of up to 10 tiles of 16 iterates from LDS.  Y is
// triangular, so a tile of iterates k0+1..k0+16 stops taking part after
// column k0+15 of L: about half the products of the full GEMM are skipped,
// and only the nonzero blocks are staged.  Iterates beyond the first column
// group (up to 160) form further groups, sized so that their blocks of Y fit
// in LDS.  Per x_k(r) the sum over j runs in increasing blocks of 4 (inside
// a block the matrix core's order), in FP64; iterates beyond k_done are never
// written and columns of L beyond k_done never reach the result.
//
// Also here: the stopping rule (eq. tol) evaluated on the device, the copy of
// the selected iterate into the caller's output vector, and the final-only
// variant that forms that one iterate without the others.
#include "internal.hpp"

namespace lslu {

namespace {

typedef double dmfma4 __attribute__((ext_vector_type(4)));

// waves per block: 3 per SIMD
template <typename T>
constexpr int asm_waves() { return 12; }
constexpr int kCT = 10;          // at most this many 16-iterate tiles per column group
constexpr int kAsmMaxGroups = 8;
constexpr int kAsmMaxPhases = kMaxIter / 16;
// Y blocks in LDS: 256 doubles (4 steps x 64 lanes) per (phase, tile) pair,
// plus room for kCT more that the reads of tiles that take no part touch
constexpr int kAsmLdsPairs = 62;

// Column groups of iterate tiles: group g covers tiles c0[g] .. c0[g]+nt[g]-1
// (iterates 16 c0 + 1 .. 16 (c0 + nt)).
struct AsmGroups {
  int count;
  int c0[kAsmMaxGroups];
  int nt[kAsmMaxGroups];
};

// (phase, tile) pairs of a group in LDS: phase p (columns 16p .. 16p+15 of
// L) involves the tiles c >= max(0, p - c0) of the group.
__host__ __device__ inline int asm_active(int p, int c0, int nt) {
  const int lo = p - c0 > 0 ? p - c0 : 0;
  return nt - lo > 0 ? nt - lo : 0;
}

template <typename T>
__device__ inline void store4(T* p, const double* v, bool vec) {
  if constexpr (sizeof(T) == 4) {
    if (vec) {
      *reinterpret_cast<float4*>(p) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
      return;
    }
  } else {
    if (vec) {
      reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
      reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
      return;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) p[r] = static_cast<T>(v[r]);
}

template <typename T>
__global__ __launch_bounds__(64 * asm_waves<T>()) void k_assemble(
    const T* __restrict__ L, int64_t rs, int64_t cs, int64_t n, const double* __restrict__ Y,
    int K, AsmGroups groups, int blocks_per_group, bool vec, const T* __restrict__ x0,
    T* __restrict__ X, const DevState* __restrict__ st) {
  __shared__ double sy[(kAsmLdsPairs + kCT) * 256];
  __shared__ int s_off[kAsmMaxPhases + 1];
  const int kd = st->k_done;
  const int g = blockIdx.x / blocks_per_group;
  const int blk = blockIdx.x % blocks_per_group;
  const int c0 = groups.c0[g], nt = groups.nt[g];
  if (16 * c0 >= kd) return;
  const int cend = min(nt, (kd - 16 * c0 + 15) / 16);   // tiles holding iterates <= k_done
  const int jmax = min(16 * (c0 + cend), kd);           // columns of L this group needs
  const int nph = (jmax + 15) / 16;                     // phases of 16 columns
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  if (threadIdx.x == 0) {
    int o = 0;
    for (int p = 0; p < nph; ++p) {
      s_off[p] = o;
      o += 256 * asm_active(p, c0, nt);
    }
    s_off[nph] = o;
  }
  __syncthreads();
  // Stage the Y blocks: element (lane', step s4, tile c) of phase p is
  // Y(16p + 4 s4 + lk', 16(c0+c) + li'), zero off the triangle and beyond
  // k_done, at s_off[p] + ((c - clo) 4 + s4) 64 + lane'.  Consecutive threads
  // write consecutive doubles (no bank conflicts; the reads of Y are
  // scattered, once per block).
  for (int p = 0; p < nph; ++p) {
    const int act = asm_active(p, c0, nt);
    const int clo = nt - act;
    for (int e = threadIdx.x; e < 256 * act; e += 64 * asm_waves<T>()) {
      const int ln = e % 64, s4 = (e / 64) % 4, c = clo + e / 256;
      const int j = 16 * p + 4 * s4 + (ln >> 4), k = 16 * (c0 + c) + (ln & 15);
      const double v = (j < jmax && j <= k && k < kd) ? Y[(int64_t)k * K + j] : 0.0;
      sy[s_off[p] + e] = v;
    }
  }
  __syncthreads();

  // This wave's row tiles: w, w + wstride, ...
  const int64_t nrw = (n + 15) / 16;
  const int64_t wstride = (int64_t)blocks_per_group * asm_waves<T>();
  int64_t w = (int64_t)blk * asm_waves<T>() + (threadIdx.x >> 6);
  if (w >= nrw) return;
  dmfma4 acc[kCT];
#pragma unroll
  for (int c = 0; c < kCT; ++c) acc[c] = dmfma4{0.0, 0.0, 0.0, 0.0};
  // The 4 columns of L of step s of phase p of the wave's 16-row tile wt
  // (this lane's column 16p + 4s + lk), loaded one phase ahead of their use
  // into the registers the step has just used, and kept in the basis's own
  // type until used (a conversion right after the load would wait for it
  // there).  Row i of the product's tile is row 4 (i % 4) + i / 4 of the 16:
  // the product returns its row i in lane group i % 4, element i / 4, so
  // every lane ends up with 4 consecutive rows of the result.  The loads are
  // unconditional: indices are clamped into range, and a clamped row lands
  // in a row of the result that is not stored, a clamped column meets a zero
  // of Y.  Entries of L are finite.
  auto load_step = [&](int64_t wt, int p, int s4, T& a) {
    const int64_t r = min(wt * 16 + 4 * (li & 3) + (li >> 2), n - 1);
    const int64_t jc = min(16 * p + 4 * s4 + lk, jmax - 1);
    a = L[r * rs + jc * cs];
  };
  // tile c holds iterates 16(c0+c)+1..16(c0+c)+16, whose y has entries
  // j < 16(c0+c+1): in phase p only tiles c >= p - c0 take part
  // Phase p with the columns in a; each step's registers then take the same
  // step of phase np of tile nw.
  auto compute_ph = [&](int p, T (&a)[4], int64_t nw, int np) {
    const int clo = nt - asm_active(p, c0, nt);
    // tile c's block of step s4 sits at base + (4 c + s4) 64 (offsets known
    // at compile time); tiles that take no part read other blocks
    const double* base = sy + (s_off[p] - 256 * clo) + lane;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      // all reads first
      double b[kCT];
#pragma unroll
      for (int c = 0; c < kCT; ++c) b[c] = base[(4 * c + s4) * 64];
      const double av = static_cast<double>(a[s4]);
      load_step(nw, np, s4, a[s4]);
#pragma unroll
      for (int c = 0; c < kCT; ++c) {
        if (c < clo || c >= cend) continue;
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[c], acc[c], 0, 0, 0);
      }
    }
  };
  // lane holds rows 4 lk .. 4 lk + 3 of the tile, iterate 16(c0+c) + li
  auto store_tile = [&](int64_t wt) {
    const int64_t r = wt * 16 + 4 * lk;
    if (r < n) {
      double xb[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        xb[e] = (x0 && r + e < n) ? static_cast<double>(x0[r + e]) : 0.0;
      const bool full = r + 3 < n;
#pragma unroll
      for (int c = 0; c < kCT; ++c) {
        const int k = 16 * (c0 + c) + li;
        if (c >= cend || k >= kd) continue;
        double v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = xb[e] + acc[c][e];
        T* p = X + (int64_t)k * n + r;
        if (full) {
          store4<T>(p, v, vec);
        } else {
          for (int e = 0; r + e < n; ++e) p[e] = static_cast<T>(v[e]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kCT; ++c) acc[c] = dmfma4{0.0, 0.0, 0.0, 0.0};
  };
  // (tile, phase) positions in the order this wave works through them
  auto next = [&](int64_t& wt, int& p) {
    if (++p == nph) {
      p = 0;
      wt += wstride;
    }
  };
  T a[4];
  int64_t cw = w, fw = w;
  int cp = 0, fp = 0;
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) load_step(fw, fp, s4, a[s4]);
  next(fw, fp);
  while (cw < nrw) {
    compute_ph(cp, a, fw, fp);
    next(fw, fp);
    if (cp == nph - 1) store_tile(cw);
    next(cw, cp);
  }
}

constexpr int kFinalBlock = 256;

template <typename T>
__global__ __launch_bounds__(kFinalBlock) void k_assemble_final(
    const T* __restrict__ L, int64_t rs, int64_t cs, int64_t n, const double* __restrict__ Y,
    int K, const T* __restrict__ x0, T* __restrict__ x_out, const int* __restrict__ sel) {
  __shared__ double y[kMaxIter];
  const int ks = sel[1];
  for (int j = threadIdx.x; j < ks; j += blockDim.x) y[j] = Y[(int64_t)(ks - 1) * K + j];
  __syncthreads();
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    const T* lr = L + r * rs;
    for (int j = 0; j < ks; ++j) acc = fma(static_cast<double>(lr[(int64_t)j * cs]), y[j], acc);
    x_out[r] = static_cast<T>((x0 ? static_cast<double>(x0[r]) : 0.0) + acc);
  }
}

// k_sel: iterate to return (0 = x_0).
__global__ void k_stopping(const double* __restrict__ ghat, const DevState* st,
                           double tol, int early, int* out /* [k_stop, k_sel] */) {
  if (threadIdx.x != 0) return;
  const int kd = st->k_done;
  int ks = kd;
  if (kd >= 2 && ghat[0] != 0.0) {
    for (int k = 2; k <= kd; ++k) {
      if (fabs(ghat[k - 1] - ghat[k - 2]) / ghat[0] < tol) {
        ks = k - 1;
        break;
      }
    }
  }
  out[0] = ks;
  out[1] = early ? ks : kd;
}

template <typename T>
__global__ void k_select_x(const T* __restrict__ X, int64_t n,
                           const T* __restrict__ x0, T* __restrict__ x_out,
                           const int* __restrict__ sel) {
  const int ks = sel[1];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x)
    x_out[r] = ks > 0 ? X[(int64_t)(ks - 1) * n + r] : (x0 ? x0[r] : T(0));
}

}  // namespace

template <typename T>
void launch_assemble(const T* L, int64_t rs, int64_t cs, int64_t n,
                     const double* Y, int K, const T* x0, T* X,
                     const DevState* st, hipStream_t s) {
  // Column groups: as many tiles as fit (at most kCT), each group's nonzero
  // Y blocks within the LDS array (tiles of a later group take part in all
  // of the earlier groups' phases too).
  AsmGroups gr{};
  const int tiles = (K + 15) / 16;
  for (int c0 = 0; c0 < tiles;) {
    int nt = 1;
    auto pairs = [&](int t) {
      int sum = 0;
      for (int p = 0; p < c0 + t; ++p) sum += asm_active(p, c0, t);
      return sum;
    };
    while (nt < kCT && c0 + nt < tiles && pairs(nt + 1) <= kAsmLdsPairs) ++nt;
    gr.c0[gr.count] = c0;
    gr.nt[gr.count] = nt;
    ++gr.count;
    c0 += nt;
  }
  // one block per CU and group: the grid covers the device once per group
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t nrw = (n + 15) / 16;
  const int bpg = (int)std::max<int64_t>(
      1, std::min<int64_t>(cus, (nrw + asm_waves<T>() - 1) / asm_waves<T>()));
  // 4-element stores when every column of X starts 16-byte aligned
  const bool vec = (n & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
  k_assemble<T><<<(unsigned)(bpg * gr.count), 64 * asm_waves<T>(), 0, s>>>(
      L, rs, cs, n, Y, K, gr, bpg, vec, x0, X, st);
}

template <typename T>
void launch_assemble_final(const T* L, int64_t rs, int64_t cs, int64_t n,
                           const double* Y, int K, const T* x0, T* x_out,
                           const int* k_sel, hipStream_t s) {
  int64_t g = (n + kFinalBlock - 1) / kFinalBlock;
  if (g > 8192) g = 8192;
  k_assemble_final<T><<<(unsigned)g, kFinalBlock, 0, s>>>(L, rs, cs, n, Y, K, x0, x_out, k_sel);
}

void launch_stopping(const double* ghat, const DevState* st, double tol,
                     int early, int* out, hipStream_t s) {
  k_stopping<<<1, 64, 0, s>>>(ghat, st, tol, early, out);
}

template <typename T>
void launch_select_x(const T* X, int64_t n, const T* x0, T* x_out,
                     const DevState*, const int* k_sel, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  k_select_x<T><<<(unsigned)g, 256, 0, s>>>(X, n, x0, x_out, k_sel);
}

template void launch_assemble<double>(const double*, int64_t, int64_t, int64_t,
                                      const double*, int, const double*,
                                      double*, const DevState*, hipStream_t);
template void launch_assemble<float>(const float*, int64_t, int64_t, int64_t,
                                     const double*, int, const float*, float*,
                                     const DevState*, hipStream_t);
template void launch_assemble_final<double>(const double*, int64_t, int64_t, int64_t,
                                            const double*, int, const double*,
                                            double*, const int*, hipStream_t);
template void launch_assemble_final<float>(const float*, int64_t, int64_t, int64_t,
                                           const double*, int, const float*, float*,
                                           const int*, hipStream_t);
template void launch_select_x<double>(const double*, int64_t, const double*,
                                      double*, const DevState*, const int*,
                                      hipStream_t);
template void launch_select_x<float>(const float*, int64_t, const float*,
                                     float*, const DevState*, const int*,
                                     hipStream_t);

}  // namespace lslu
