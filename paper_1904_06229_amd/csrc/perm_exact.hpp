// Exact integer products for the 0/1 walks (kern_int01.hip, and the exact
// variant of the mixed-radix walk in kern_mixed.hip).
//
// Row sums are small integers held in FP64 registers.  Rows are multiplied
// in groups of k = int01_group_rows(N) rows (|row sum| <= N, N^k < 2^50), so
// every group product G is an exact FP64 integer.  Group products are
// combined with error-free transformations: TwoProduct (h = G1*G2,
// l = fma(G1, G2, -h), G1*G2 = h + l exactly) and an exact split at 2^51
// (q = h + 1.5*2^103 rounds h to a multiple of 2^51; then h - (q - 1.5*2^103)
// is exact, and the bit pattern of q minus that of 1.5*2^103 is h's high part
// as an integer).  The product is carried as integer limbs of weight 1, 2^51,
// 2^102 held in doubles, and the limbs land in three 64-bit integer bins
// through their bit patterns: for |y| <= 2^51, bits(y + 1.5*2^52) -
// bits(1.5*2^52) = y.  Terms entered with opposite signs cancel the constant
// offsets; otherwise product_offsets() gives them.  The bins fold into a
// 128-bit sum (wrapping); they must be folded before about 2^10 products
// have entered, so that the weight-1 and weight-2^51 bins cannot wrap.
#pragma once

#include "perm_device.hpp"
#include "perm_internal.hpp"

namespace perm {
namespace exact {

constexpr double kC51 = 15845632502852867518708790067200.0;  // 1.5 * 2^103
constexpr double kM52 = 6755399441055744.0;                  // 1.5 * 2^52
constexpr double kInv51 = 1.0 / 2251799813685248.0;          // 2^-51
// 1.5 * 2^103 + 1.5 * 2^52: its bits span 2^103 .. 2^51, 53 bits, so the sum
// is exact.
constexpr double kC51M52 = kC51 + kM52;
static_assert(kC51M52 - kC51 == kM52, "1.5*2^103 + 1.5*2^52 must be exact");

// Low limb of an exact product, with the bin offset: for h = fl(x*g) with
// |h| < 2^102, l = x*g - h and q = fl(h + 1.5*2^103), returns
// (h - (q - 1.5*2^103)) + l + 1.5*2^52 exactly, whose bit pattern minus that
// of 1.5*2^52 is the product modulo 2^51 in [-2^51, 2^51].  One subtraction
// fewer than forming the remainder first: 1.5*2^103 + 1.5*2^52 - q equals
// 1.5*2^52 - (q - 1.5*2^103), a multiple of 2^51 below 2^103 (exact), and the
// two additions stay exact integers in (2^52, 2^53) because |h - (q -
// 1.5*2^103)| <= 2^50 and |l| <= 2^49.
__device__ __forceinline__ double low_limb(double h, double l, double q) {
  return (h + (kC51M52 - q)) + l;
}

__device__ __forceinline__ uint64_t bits(double x) { return (uint64_t)__double_as_longlong(x); }

struct Bins {
  uint64_t b0, b1, b2;  // weights 1, 2^51, 2^102 (two's complement, wrapping)
};

template <bool ADD>
__device__ __forceinline__ void bin_put(uint64_t& bin, uint64_t v) {
  if constexpr (ADD)
    bin += v;
  else
    bin -= v;
}

// Exact product of K factors G[0..K-1] (|G| < 2^50, the last may be < 2^51),
// entered into the bins with sign ADD ? + : -.  The entered bit patterns carry
// constant offsets (bits of 1.5*2^103 or of 1.5*2^52; see product_offsets).
template <int K, bool ADD>
__device__ __forceinline__ void product_bins(const double (&G)[K], Bins& B) {
  if constexpr (K == 1) {
    bin_put<ADD>(B.b0, bits(G[0] + kM52));
  } else {
    // X = G0 * G1 as limbs (X0 weight 1, X1 weight 2^51; X2 weight 2^102).
    double X0, X1, X2 = 0.0;
    {
      const double h = G[0] * G[1];
      const double l = fma(G[0], G[1], -h);
      const double q = h + kC51;
      if constexpr (K == 2) {
        bin_put<ADD>(B.b1, bits(q));
        bin_put<ADD>(B.b0, bits(low_limb(h, l, q)));
        return;
      }
      const double hr = q - kC51;
      X0 = (h - hr) + l;
      X1 = hr * kInv51;
    }
    // Middle factors: X <- X * G mod 2^153, limbs renormalised below 2^51.
#pragma unroll
    for (int g = 2; g + 1 < K; ++g) {
      double h[3], l[3], y[3], H[3];
      const double x[3] = {X0, X1, X2};
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        h[m] = x[m] * G[g];
        l[m] = fma(x[m], G[g], -h[m]);
        const double q = h[m] + kC51;
        const double hr = q - kC51;
        y[m] = (h[m] - hr) + l[m];
        H[m] = hr * kInv51;
      }
      double Y1 = y[1] + H[0];
      double Y2 = y[2] + H[1];
      {
        const double q = Y1 + kC51;
        const double hr = q - kC51;
        Y1 = Y1 - hr;
        Y2 = Y2 + hr * kInv51;
      }
      {
        const double q = Y2 + kC51;
        Y2 = Y2 - (q - kC51);  // keep Y2 modulo 2^51
      }
      X0 = y[0];
      X1 = Y1;
      X2 = Y2;
    }
    // Last factor: products of the limbs go straight into the bins.
    const double Gl = G[K - 1];
    {
      const double h = X0 * Gl;
      const double l = fma(X0, Gl, -h);
      const double q = h + kC51;
      bin_put<ADD>(B.b0, bits(low_limb(h, l, q)));
      bin_put<ADD>(B.b1, bits(q));
    }
    {
      const double h = X1 * Gl;
      const double l = fma(X1, Gl, -h);
      const double q = h + kC51;
      bin_put<ADD>(B.b1, bits(low_limb(h, l, q)));
      bin_put<ADD>(B.b2, bits(q));
    }
    if constexpr (K >= 4) {
      const double h = X2 * Gl;
      const double l = fma(X2, Gl, -h);
      bin_put<ADD>(B.b2, bits(low_limb(h, l, h + kC51)));
    }
  }
}

// Product of rows [lo, hi) (exact when its bound is below 2^53).
template <int N, int LO, int HI>
__device__ __forceinline__ double rows_prod(const double (&r)[N]) {
  double p = r[LO];
#pragma unroll
  for (int i = LO + 1; i < HI; ++i) p *= r[i];
  return p;
}

// Exact product of all row sums, in groups of int01_group_rows(N) rows.
template <int N, bool ADD>
__device__ __forceinline__ void term_bins(const double (&r)[N], Bins& B) {
  constexpr int k = int01_group_rows(N);
  constexpr int K = (N + k - 1) / k;
  double G[K];
#pragma unroll
  for (int g = 0; g < K; ++g) {
    double p = r[g * k];
#pragma unroll
    for (int i = g * k + 1; i < (g + 1) * k && i < N; ++i) p *= r[i];
    G[g] = p;
  }
  product_bins<K, ADD>(G, B);
}

// Offsets carried by one product_bins<K> call (per bin).
template <int K>
__device__ __forceinline__ Bins product_offsets() {
  const uint64_t c = bits(kC51), m = bits(kM52);
  if constexpr (K == 1) return Bins{m, 0, 0};
  if constexpr (K == 2) return Bins{m, c, 0};
  if constexpr (K == 3) return Bins{m, c + m, c};
  return Bins{m, c + m, c + m};
}

template <int N>
__device__ __forceinline__ Bins term_offsets() {
  constexpr int k = int01_group_rows(N);
  return product_offsets<(N + k - 1) / k>();
}

__device__ __forceinline__ u128 fold(const Bins& B) {
  const unsigned __int128 v0 = (unsigned __int128)(__int128)(int64_t)B.b0;
  const unsigned __int128 v1 = (unsigned __int128)(__int128)(int64_t)B.b1;
  const unsigned __int128 v2 = (unsigned __int128)(__int128)(int64_t)B.b2;
  const unsigned __int128 s = v0 + (v1 << 51) + (v2 << 102);
  return u128{(uint64_t)s, (uint64_t)(s >> 64)};
}

}  // namespace exact
}  // namespace perm
