// In-LDS batched complex FFT shared by the transform passes (x, y and the wall-normal DCT).
#pragma once

#include "common.hpp"

namespace drpf {

// In-LDS complex FFT of `nlines` lines of length M (power of two, M >= 2). Element n of
// line b lives at buf[b * bs + n * es]. Thread t < nlines * max(M/4, 1) owns one butterfly
// set q of one line b: with LF (line-fast, for column tiles with es = nlines) consecutive
// lanes take consecutive lines, so a wavefront touches consecutive LDS words; otherwise
// consecutive lanes take consecutive q of one line (row tiles with es = 1). Every thread of
// the block must call this (barriers). Twiddles tw[t] = exp(-2 pi i t / M); the inverse
// uses their conjugates.
template <typename T, bool INV, bool LF>
__device__ __forceinline__ void lds_fft(cx<T>* buf, int M, int logM, int nlines, int bs, int es,
                        const cx<T>* __restrict__ tw) {
  const int quarter = M >= 4 ? (M >> 2) : 1;
  const int t = threadIdx.x;
  const bool active = t < nlines * quarter;
  int b = 0, q = 0;
  if (active) {
    if (LF) {
      q = t / nlines;
      b = t - q * nlines;
    } else {
      b = t / quarter;
      q = t - b * quarter;
    }
  }
  cx<T>* line = buf + b * bs;
  int Ns = 1;
  if (logM & 1) {
    // radix-2 stage (Ns = 1, unit twiddles): butterflies j = q and q + M/4 of M/2
    const int half = M >> 1;
    cx<T> v[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = q + h * quarter;
      if (active && j < half) {
        v[2 * h] = line[j * es];
        v[2 * h + 1] = line[(j + half) * es];
      }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = q + h * quarter;
      if (active && j < half) {
        line[(2 * j) * es] = v[2 * h] + v[2 * h + 1];
        line[(2 * j + 1) * es] = v[2 * h] - v[2 * h + 1];
      }
    }
    __syncthreads();
    Ns = 2;
  }
  for (; Ns < M; Ns <<= 2) {
    const int j = q;
    const int k = j & (Ns - 1);
    cx<T> v[4];
    if (active) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = line[(j + r * quarter) * es];
    }
    __syncthreads();
    if (active) {
      const int step = M / (Ns * 4);
#pragma unroll
      for (int r = 1; r < 4; ++r) {
        cx<T> w = tw[r * k * step];
        if (INV) w = conj(w);
        v[r] = v[r] * w;
      }
      const cx<T> a = v[0] + v[2], bb = v[0] - v[2], c = v[1] + v[3], d = v[1] - v[3];
      const cx<T> jd = INV ? mul_i(d) : mul_mi(d);
      const int base = (j - k) * 4 + k;
      line[base * es] = a + c;
      line[(base + Ns) * es] = bb + jd;
      line[(base + 2 * Ns) * es] = a - c;
      line[(base + 3 * Ns) * es] = bb - jd;
    }
    __syncthreads();
  }
}

}  // namespace drpf
