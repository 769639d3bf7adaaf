// In-LDS batched complex FFT with compile-time length and several points per thread, used by
// the FP32 x and y passes and by the FP32 wall-normal DCT of the Cahn-Hilliard pair.
//
// A line of length M = 2^LOGM is transformed by a Stockham autosort sequence (natural order in
// and out): a first stage of radix 2^LR0, then stages of radix P = 2^LP. Each thread owns P
// points of one line in every stage: it always reads elements q + i T (T = M / P threads per
// line, i < P), forms the P / R radix-R butterflies j = q + c T (c < P / R) whose inputs these
// are, and writes their outputs to (j - k) R + k + u Ns (k = j mod Ns, Ns the product of the
// earlier radices). Since Ns divides T, all butterflies of a thread share k and so their
// twiddles. Every line sits in LDS at a stride of LS elements, element e at pad(e) = e +
// (e >> 4): the strided writes of the first stages then fall on distinct banks, and every
// offset of a thread's reads and writes from its own base is a compile-time constant, since
// base + offset never carries out of the low four bits (all strides, counts and radices are
// powers of two and q < T; checked exhaustively for every supported length), so the LDS
// accesses take immediate offsets. Twiddles tw[t] = exp(-2 pi i t / M), t < M, staged in LDS by the caller;
// the inverse uses their conjugates. Unnormalised.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace drpf {

template <int LOGM, int LPMAX>
struct FftPlan {
  static constexpr int M = 1 << LOGM;
  static constexpr int LP = LOGM < LPMAX ? LOGM : LPMAX;
  static constexpr int P = 1 << LP;  // points per thread
  static constexpr int LT = LOGM - LP;
  static constexpr int T = 1 << LT;  // threads per line
  // first stage radix 2^LR0 (the remainder), then radix P
  static constexpr int LR0 = LOGM <= LP ? LOGM : (LOGM % LP == 0 ? LP : LOGM % LP);
  static constexpr int NST = LOGM <= LP ? 1 : 1 + (LOGM - LR0) / LP;
  // one pad slot per 16 elements; lines at an odd stride start on different banks
  __host__ __device__ static constexpr int pad(int e) { return e + (e >> 4); }
  static constexpr int LS = M + (M >> 4) + 1;
};

// a * exp(-+ 2 pi i e / 16) (forward: minus), e a constant once unrolled; quarter turns exact
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot16(cx<T> a, int e) {
  constexpr double C[4] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};
  e &= 15;
  if (e == 0) return a;
  if (e == 8) return mk<T>(-a.re, -a.im);
  if (e == 4) return INV ? mul_i(a) : mul_mi(a);
  if (e == 12) return INV ? mul_mi(a) : mul_i(a);
  // cos and sin of 2 pi e / 16 from the first quadrant
  const int qd = e >> 2, r = e & 3;
  const double c0 = C[r], s0 = r == 0 ? 0.0 : C[4 - r];
  double c, s;
  if (qd == 0) { c = c0; s = s0; }
  else if (qd == 1) { c = -s0; s = c0; }
  else if (qd == 2) { c = -c0; s = -s0; }
  else { c = s0; s = -c0; }
  const T cc = (T)c, ss = INV ? (T)s : (T)-s;
  return mk<T>(a.re * cc - a.im * ss, a.re * ss + a.im * cc);
}

// In-register DFT of R = 2^LR points (R <= 16), natural order in and out
template <typename T, bool INV, int LR>
__device__ __forceinline__ void dft_reg(cx<T>* x) {
  if constexpr (LR == 1) {
    const cx<T> a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  } else if constexpr (LR == 2) {
    const cx<T> a = x[0] + x[2], b = x[0] - x[2], c = x[1] + x[3], d = x[1] - x[3];
    const cx<T> jd = INV ? mul_i(d) : mul_mi(d);
    x[0] = a + c;
    x[1] = b + jd;
    x[2] = a - c;
    x[3] = b - jd;
  } else {
    // R = R1 R2 with R2 = 2 (R = 8) or 4 (R = 16): n = R2 n1 + n2, k = k1 + R1 k2;
    // DFT_R1 over n1 for each n2, twiddle w_R^(n2 k1), DFT_R2 over n2 for each k1
    constexpr int L2 = LR == 3 ? 1 : 2, L1 = LR - L2;
    constexpr int R1 = 1 << L1, R2 = 1 << L2;
    cx<T> y[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = x[R2 * n1 + n2];
      dft_reg<T, INV, L1>(y[n2]);
#pragma unroll
      for (int k1 = 1; k1 < R1; ++k1) y[n2][k1] = rot16<T, INV>(y[n2][k1], n2 * k1 * (16 >> LR));
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      cx<T> z[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) z[n2] = y[n2][k1];
      dft_reg<T, INV, L2>(z);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) x[k1 + R1 * k2] = z[k2];
    }
  }
}

// One Stockham stage S of the plan on this thread's line (base `line`, thread q of the line).
// Every thread of the block calls it (two barriers); inactive threads only take part in them.
template <typename T, bool INV, int LOGM, int LPMAX, int S>
__device__ __forceinline__ void fft16_stage(cx<T>* line, int q, bool active, const cx<T>* __restrict__ tw) {
  using F = FftPlan<LOGM, LPMAX>;
  constexpr int LR = S == 0 ? F::LR0 : F::LP, R = 1 << LR;
  constexpr int LNS = S == 0 ? 0 : F::LR0 + F::LP * (S - 1), NS = 1 << LNS;
  constexpr int B = F::P / R;  // butterflies per thread
  cx<T> v[F::P];
  if (active) {
    const cx<T>* rb = line + F::pad(q);
#pragma unroll
    for (int i = 0; i < F::P; ++i) v[i] = rb[F::pad(i * F::T)];
  }
  __syncthreads();
  if (active) {
    const int k = q & (NS - 1);
    if constexpr (NS > 1) {
      // input r of each butterfly times exp(-+ 2 pi i r k / (R Ns)) = tw[r k M / (R Ns)]
      const int t1 = k << (LOGM - LR - LNS);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cx<T> w0 = tw[r * t1];
        const cx<T> w = INV ? conj(w0) : w0;
#pragma unroll
        for (int c = 0; c < B; ++c) v[c + r * B] = v[c + r * B] * w;
      }
    }
#pragma unroll
    for (int c = 0; c < B; ++c) {
      cx<T> x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = v[c + r * B];
      dft_reg<T, INV, LR>(x);
#pragma unroll
      for (int u = 0; u < R; ++u) v[c + u * B] = x[u];
    }
    cx<T>* wb = line + F::pad(((q - k) << LR) + k);
#pragma unroll
    for (int c = 0; c < B; ++c)
#pragma unroll
      for (int u = 0; u < R; ++u) wb[F::pad(c * F::T * R + u * NS)] = v[c + u * B];
  }
  __syncthreads();
}

// The whole transform of this thread's line; ends with a barrier.
template <typename T, bool INV, int LOGM, int LPMAX, int S = 0>
__device__ __forceinline__ void fft16(cx<T>* line, int q, bool active, const cx<T>* __restrict__ tw) {
  fft16_stage<T, INV, LOGM, LPMAX, S>(line, q, active, tw);
  if constexpr (S + 1 < FftPlan<LOGM, LPMAX>::NST) fft16<T, INV, LOGM, LPMAX, S + 1>(line, q, active, tw);
}

// Points per thread (log2) of the FP32 passes: 8 points (4 KB of LDS per wavefront) measured
// faster than 4 (more LDS round trips and barriers) and than 16 (half the resident waves)
template <typename T>
constexpr int fft_lp() {
  static_assert(sizeof(T) == 4, "the compile-time FFT form serves the FP32 passes");
  return 3;
}

// Run f(std::integral_constant<int, L>) for L = logm in [1, 11]
template <typename Fn>
hipError_t with_logm(int logm, Fn&& f) {
  switch (logm) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    case 11: f(std::integral_constant<int, 11>{}); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace drpf
