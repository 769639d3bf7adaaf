// In-LDS batched complex FFT with the length and the stage strides at run time: the FP64 x
// and y passes and wall-normal DCT (at 16 bytes per point this form, with consecutive lanes on
// consecutive LDS words in every stage, measured faster than the compile-time form of
// lds_fft16.hpp), and the fused x-y passes of a whole layer in both precisions.
#pragma once

#include "common.hpp"

namespace drpf {

// In-LDS complex FFT of `nlines` lines of length M = 2^logM (M >= 1). Two layouts:
//   LF (line-fast, column tiles): element n of line b at buf[(n << lnl) + b], nlines = 2^lnl;
//       consecutive lanes take consecutive lines, so a wavefront touches consecutive LDS words;
//   otherwise (row tiles): element n of line b at buf[(b << logM) + n]; consecutive lanes
//       take consecutive butterfly sets of one line; lnl is unused and nlines any count.
// Thread t < nlines * max(M/4, 1) owns one butterfly set q of one line b. Every thread of the
// block must call this (barriers). Twiddles tw[t] = exp(-2 pi i t / M); the inverse uses their
// conjugates. All index arithmetic is shifts and masks (every extent is a power of two).
template <typename T, bool INV, bool LF>
__device__ __forceinline__ void lds_fft(cx<T>* buf, int M, int logM, int nlines, int lnl,
                                        const cx<T>* __restrict__ tw) {
  const int lq = logM >= 2 ? logM - 2 : 0;
  const int quarter = 1 << lq;
  const int t = threadIdx.x;
  const bool active = t < (nlines << lq);
  int b = 0, q = 0;
  if (active) {
    if (LF) {
      q = t >> lnl;
      b = t & ((1 << lnl) - 1);
    } else {
      b = t >> lq;
      q = t & (quarter - 1);
    }
  }
  // LDS index of element n of this thread's line
  auto at = [&](int n) -> cx<T>& { return LF ? buf[(n << lnl) + b] : buf[(b << logM) + n]; };
  int lNs = 0;
  if (logM & 1) {
    // radix-2 stage (Ns = 1, unit twiddles): butterflies j = q and q + M/4 of M/2
    const int half = M >> 1;
    cx<T> v[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = q + (h << lq);
      if (active && j < half) {
        v[2 * h] = at(j);
        v[2 * h + 1] = at(j + half);
      }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = q + (h << lq);
      if (active && j < half) {
        at(2 * j) = v[2 * h] + v[2 * h + 1];
        at(2 * j + 1) = v[2 * h] - v[2 * h + 1];
      }
    }
    __syncthreads();
    lNs = 1;
  }
  for (; lNs < logM; lNs += 2) {
    const int Ns = 1 << lNs;
    const int j = q;
    const int k = j & (Ns - 1);
    cx<T> v[4];
    if (active) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = at(j + (r << lq));
    }
    __syncthreads();
    if (active) {
      // twiddle index r k M / (4 Ns)
      const int w1 = k << (logM - lNs - 2);
      cx<T> w[3] = {tw[w1], tw[2 * w1], tw[3 * w1]};
#pragma unroll
      for (int r = 1; r < 4; ++r) v[r] = v[r] * (INV ? conj(w[r - 1]) : w[r - 1]);
      const cx<T> a = v[0] + v[2], bb = v[0] - v[2], c = v[1] + v[3], d = v[1] - v[3];
      const cx<T> jd = INV ? mul_i(d) : mul_mi(d);
      const int base = ((j - k) << 2) + k;
      at(base) = a + c;
      at(base + Ns) = bb + jd;
      at(base + 2 * Ns) = a - c;
      at(base + 3 * Ns) = bb - jd;
    }
    __syncthreads();
  }
}

// The same transform with REP butterfly sets per thread: set s = threadIdx.x + r blockDim.x,
// r < REP, of the nlines * max(M/4, 1) sets (line and set numbered as in lds_fft). For
// batches that need more sets than a block has threads (a whole coarse layer in one block).
// With XL, one more line of the same length, contiguous at xl, is transformed in the same
// stages (its sets on threads 0 .. max(M/4, 1) - 1), sharing their barriers.
template <typename T, bool INV, bool LF, int REP, bool XL = false>
__device__ __forceinline__ void lds_fft_rep(cx<T>* buf, int M, int logM, int nlines, int lnl,
                                            const cx<T>* __restrict__ tw, cx<T>* xl = nullptr) {
  constexpr int NS = REP + (XL ? 1 : 0);
  const int lq = logM >= 2 ? logM - 2 : 0;
  const int quarter = 1 << lq;
  const int nsets = nlines << lq;
  int bs[NS], qs[NS];
  bool act[NS];
#pragma unroll
  for (int r = 0; r < REP; ++r) {
    const int s = threadIdx.x + r * blockDim.x;
    act[r] = s < nsets;
    qs[r] = LF ? s >> lnl : s & (quarter - 1);
    bs[r] = LF ? s & ((1 << lnl) - 1) : s >> lq;
  }
  if (XL) {
    act[NS - 1] = (int)threadIdx.x < quarter;
    qs[NS - 1] = threadIdx.x;
    bs[NS - 1] = 0;
  }
  auto at = [&](int r, int n) -> cx<T>& {
    if (XL && r == NS - 1) return xl[n];
    return LF ? buf[(n << lnl) + bs[r]] : buf[(bs[r] << logM) + n];
  };
  int lNs = 0;
  if (logM & 1) {
    const int half = M >> 1;
    cx<T> v[NS][4];
#pragma unroll
    for (int r = 0; r < NS; ++r)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = qs[r] + (h << lq);
        if (act[r] && j < half) {
          v[r][2 * h] = at(r, j);
          v[r][2 * h + 1] = at(r, j + half);
        }
      }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NS; ++r)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = qs[r] + (h << lq);
        if (act[r] && j < half) {
          at(r, 2 * j) = v[r][2 * h] + v[r][2 * h + 1];
          at(r, 2 * j + 1) = v[r][2 * h] - v[r][2 * h + 1];
        }
      }
    __syncthreads();
    lNs = 1;
  }
  for (; lNs < logM; lNs += 2) {
    const int Ns = 1 << lNs;
    cx<T> v[NS][4];
#pragma unroll
    for (int r = 0; r < NS; ++r)
      if (act[r]) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) v[r][rr] = at(r, qs[r] + (rr << lq));
      }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      if (act[r]) {
        const int j = qs[r];
        const int k = j & (Ns - 1);
        const int w1 = k << (logM - lNs - 2);
        const cx<T> w[3] = {tw[w1], tw[2 * w1], tw[3 * w1]};
#pragma unroll
        for (int rr = 1; rr < 4; ++rr) v[r][rr] = v[r][rr] * (INV ? conj(w[rr - 1]) : w[rr - 1]);
        const cx<T> a = v[r][0] + v[r][2], bb = v[r][0] - v[r][2], c = v[r][1] + v[r][3],
                    d = v[r][1] - v[r][3];
        const cx<T> jd = INV ? mul_i(d) : mul_mi(d);
        const int base = ((j - k) << 2) + k;
        at(r, base) = a + c;
        at(r, base + Ns) = bb + jd;
        at(r, base + 2 * Ns) = a - c;
        at(r, base + 3 * Ns) = bb - jd;
      }
    }
    __syncthreads();
  }
}

}  // namespace drpf
