// Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
// operator preparation the library runs on caller arrays (host_ops.hpp) on
// random and malformed inputs, each result checked against a direct
// computation.  Built with g++ by test_host_sanitize.py; exits nonzero on the
// first mismatch (a sanitizer finding aborts the program).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "host_ops.hpp"

using namespace lslu;

static int g_checks = 0;

static void expect(bool ok, const std::string& what) {
  ++g_checks;
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what.c_str());
    std::exit(1);
  }
}

// Exactly sized copies, so that any read past an array's end is reported.
template <typename T>
static T* heap_copy(const std::vector<T>& v) {
  T* p = static_cast<T*>(std::malloc(sizeof(T) * (v.empty() ? 1 : v.size())));
  if (!v.empty()) std::memcpy(p, v.data(), sizeof(T) * v.size());
  return p;
}

static void csr_random(std::mt19937_64& rng) {
  std::uniform_int_distribution<int> dim(1, 40);
  const int m = dim(rng), n = dim(rng);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  const double dens = u(rng);
  std::vector<int64_t> ip(m + 1, 0);
  std::vector<int32_t> ix;
  std::vector<double> dv;
  std::vector<double> dense(static_cast<size_t>(m) * n, 0.0);
  for (int r = 0; r < m; ++r) {
    for (int c = 0; c < n; ++c)
      if (u(rng) < dens) {
        ix.push_back(c);
        const double v = u(rng) - 0.5;
        dv.push_back(v);
        dense[static_cast<size_t>(r) * n + c] = v;
      }
    ip[r + 1] = static_cast<int64_t>(ix.size());
  }
  const int64_t nnz = static_cast<int64_t>(ix.size());
  int64_t* pip = heap_copy(ip);
  int32_t* pix = heap_copy(ix);
  double* pdv = heap_copy(dv);
  expect(csr_check(m, n, nnz, pip, pix) == nullptr, "valid random CSR accepted");
  std::vector<int> rpT, ciT;
  std::vector<double> valT;
  csr_transpose(m, n, nnz, pip, pix, pdv, rpT, ciT, valT);
  expect(static_cast<int>(rpT.size()) == n + 1 && rpT[n] == nnz, "A^T row pointers");
  for (int c = 0; c < n; ++c) {
    int k = rpT[c];
    for (int r = 0; r < m; ++r) {
      const double v = dense[static_cast<size_t>(r) * n + c];
      bool stored = false;
      for (int64_t p = ip[r]; p < ip[r + 1]; ++p) stored = stored || ix[p] == c;
      if (!stored) continue;
      expect(k < rpT[c + 1] && ciT[k] == r && valT[k] == v, "A^T entry (row order, value)");
      ++k;
    }
    expect(k == rpT[c + 1], "A^T row length");
  }
  if (n <= 65536) {
    std::vector<int> wide(ix.begin(), ix.end());
    const std::vector<uint16_t> nar = narrow_indices(wide);
    for (size_t i = 0; i < nar.size(); ++i) expect(nar[i] == wide[i], "16-bit index");
  }
  std::free(pip);
  std::free(pix);
  std::free(pdv);
}

static void csr_malformed() {
  struct Case {
    int64_t m, n, nnz;
    std::vector<int64_t> ip;
    std::vector<int32_t> ix;
    const char* reason;
  };
  const std::vector<Case> cases = {
      // a row whose end lies beyond nnz, before a later row would fail
      {2, 10, 5, {0, 100, 5}, {0, 1, 2, 3, 4}, "indptr exceeds nnz"},
      {3, 10, 3, {0, 2, 1, 3}, {0, 1, 2}, "indptr decreases"},
      {2, 10, 3, {1, 2, 3}, {0, 1, 2}, "indptr[0] must be 0 and indptr[m] must be nnz"},
      {2, 10, 3, {0, 2, 4}, {0, 1, 2}, "indptr[0] must be 0 and indptr[m] must be nnz"},
      {1, 4, 2, {0, 2}, {0, 4}, "column index out of range"},
      {1, 4, 2, {0, 2}, {-1, 2}, "column index out of range"},
      {1, 4, 2, {0, 2}, {2, 2}, "column indices not strictly increasing"},
      {1, 4, 2, {0, 2}, {3, 1}, "column indices not strictly increasing"},
  };
  for (const Case& c : cases) {
    int64_t* pip = heap_copy(c.ip);
    int32_t* pix = heap_copy(c.ix);
    const char* got = csr_check(c.m, c.n, c.nnz, pip, pix);
    expect(got && std::string(got) == c.reason, std::string("malformed CSR: ") + c.reason);
    std::free(pip);
    std::free(pix);
  }
  // no entries at all: indices are never read
  const std::vector<int64_t> ip0 = {0, 0, 0};
  int64_t* pip = heap_copy(ip0);
  expect(csr_check(2, 3, 0, pip, nullptr) == nullptr, "empty CSR accepted");
  std::vector<int> rpT, ciT;
  std::vector<double> valT;
  csr_transpose(2, 3, 0, pip, nullptr, nullptr, rpT, ciT, valT);
  expect(rpT.size() == 4 && rpT[3] == 0 && ciT.empty(), "empty A^T");
  std::free(pip);
}

// binary16 value of a code, from its definition.
static double f16_value(uint16_t h) {
  const int e = (h >> 10) & 31, f = h & 1023;
  const double s = (h & 0x8000) ? -1.0 : 1.0;
  if (e == 0) return s * std::ldexp(static_cast<double>(f), -24);
  return s * std::ldexp(1024.0 + f, e - 25);
}

static void conversions(std::mt19937_64& rng) {
  // binary16: the code is the nearest finite value (ties to an even code),
  // found by scanning every positive finite code
  std::uniform_real_distribution<double> ex(-26.0, 16.5);
  std::uniform_real_distribution<double> fr(1.0, 2.0);
  std::vector<double> xs = {0.0, 0x1p-25, 0x1p-24, 1.5 * 0x1p-24, 0x1p-14, 65504.0, 65519.0,
                            1.0, 1.0 + 0x1p-11, 1.0 + 3 * 0x1p-11, 2047.5, 2048.0 + 1.0};
  for (int i = 0; i < 4000; ++i) xs.push_back(fr(rng) * std::exp2(ex(rng)));
  for (double x : xs) {
    const std::vector<unsigned char> b = convert_values(&x, 1, kFP16);
    uint16_t h;
    std::memcpy(&h, b.data(), 2);
    uint16_t best = 0;
    double bd = INFINITY;
    for (uint16_t c = 0; c < 0x7c00; ++c) {
      const double d = std::fabs(f16_value(c) - x);
      if (d < bd || (d == bd && (c & 1) == 0)) {
        bd = d;
        best = c;
      }
    }
    if (x >= 65520.0)
      expect(h == 0x7c00, "binary16 overflow to infinity");
    else
      expect(h == best, "binary16 rounding of " + std::to_string(x));
    const double neg = -x;
    const std::vector<unsigned char> bn = convert_values(&neg, 1, kFP16);
    uint16_t hn;
    std::memcpy(&hn, bn.data(), 2);
    expect(hn == (h | 0x8000), "binary16 sign");
  }
  const double specials[] = {NAN, INFINITY, -INFINITY, 1e300, -1e300, 1e-300, -0.0};
  for (int prec = kFP64; prec <= kFP8; ++prec) {
    const std::vector<unsigned char> out = convert_values(specials, 7, prec);
    const size_t esz = prec == kFP64 ? 8 : prec == kFP32 ? 4 : prec == kFP8 ? 1 : 2;
    expect(out.size() == 7 * esz, "converted size");
  }
  // bfloat16 keeps the top 16 bits of the nearest float (ties to even)
  for (int i = 0; i < 4000; ++i) {
    const double x = fr(rng) * std::exp2(ex(rng)) * (i & 1 ? -1.0 : 1.0);
    const std::vector<unsigned char> b = convert_values(&x, 1, kBF16);
    uint16_t h;
    std::memcpy(&h, b.data(), 2);
    const float f = static_cast<float>(x);
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t lo = u & 0xffffu, hi = u >> 16;
    const uint32_t want = lo > 0x8000u || (lo == 0x8000u && (hi & 1u)) ? hi + 1 : hi;
    expect(h == want, "bfloat16 rounding");
  }
  // E4M3 (finite, largest 448): the code's value is within half a step
  for (int i = 0; i < 4000; ++i) {
    const double x = fr(rng) * std::exp2(std::uniform_real_distribution<double>(-10.0, 8.7)(rng));
    const std::vector<unsigned char> b = convert_values(&x, 1, kFP8);
    const int e = (b[0] >> 3) & 15, mnt = b[0] & 7;
    const double v = e == 0 ? std::ldexp(static_cast<double>(mnt), -9)
                            : std::ldexp(8.0 + mnt, e - 10);
    const double step = e == 0 ? 0x1p-9 : std::ldexp(1.0, e - 10);
    expect(std::fabs(v - std::min(x, 448.0)) <= 0.5 * step, "E4M3 rounding");
  }
}

static void psf_rows() {
  for (int prec : {kBF16, kFP16, kFP8})
    for (int ph = 1; ph <= 31; ph += 2)
      for (int pw = 1; pw <= 31; pw += 2) {
        std::vector<double> w(static_cast<size_t>(ph) * pw);
        for (size_t i = 0; i < w.size(); ++i) w[i] = 1.0 + 0.125 * static_cast<double>(i % 7);
        const std::vector<uint64_t> words = psf_mfma_rows(w, ph, pw, prec);
        const bool f8 = prec == kFP8;
        const int kPer = f8 ? 8 : 4, RL = f8 ? 80 : 76, esz = f8 ? 1 : 2;
        expect(words.size() * 8 == static_cast<size_t>(ph) * kPer * RL * esz, "PSF rows size");
        const unsigned char* bytes = reinterpret_cast<const unsigned char*>(words.data());
        const int dsh = 16 - pw / 2;
        int nonzero = 0;
        for (int a = 0; a < ph; ++a)
          for (int s = 0; s < kPer; ++s)
            for (int j = 0; j < RL; ++j) {
              const size_t at = ((static_cast<size_t>(a) * kPer + s) * RL + j) * esz;
              const bool any = bytes[at] != 0 || (esz == 2 && bytes[at + 1] != 0);
              const int idx = j + s - 16 - dsh;
              const bool inside = idx >= 0 && idx < pw;
              expect(any == inside, "PSF code placement");
              nonzero += any;
            }
        expect(nonzero == ph * pw * kPer, "every weight in every shifted copy");
      }
}

int main() {
  std::mt19937_64 rng(20240905);
  for (int i = 0; i < 300; ++i) csr_random(rng);
  csr_malformed();
  conversions(rng);
  psf_rows();
  std::printf("host checks ok: %d\n", g_checks);
  return 0;
}
